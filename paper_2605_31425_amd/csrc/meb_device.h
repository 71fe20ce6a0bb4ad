// Device-side building blocks of libmeb.so shared by its translation units:
// wave-level helpers, the second-order-cone projection of one ball, the
// evaluation pass body and its template-instance visitor.
//
// Layout: centers C (m x d, row-major), radii R (m), multipliers U (m) and
// V (m x d).  A V row is meaningful only where U != 0: multipliers lie in the
// second-order cone, so u_i = 0 forces v_i = 0, and the evaluation reads a V
// row only for u_i != 0.  This keeps the bytes of one pass at
// m (d + 2) s + nnz(u) d s instead of 2 m (d + 1) s.
//
// Work mapping of the evaluation pass: a group of G lanes (G a power of two,
// 1..64) owns one ball; lane gl of the group owns elements
// (j G + gl) VEC + q, q < VEC, j < nl of the row, so one wave-wide load
// instruction reads 64/G consecutive rows and stays coalesced.  Every wave
// streams its own contiguous range of balls, accumulates per-lane partial
// sums in FP64, and writes one partial record; records are reduced in a
// fixed order, so results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "meb_internal.h"

namespace meb {

constexpr int WAVE = 64;
constexpr int PASS_THREADS = 256;
constexpr int WPB = PASS_THREADS / WAVE;

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
    for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Sum across groups: combines lanes with equal (lane % G).
__device__ __forceinline__ double cross_group_sum(double v, int G) {
    for (int o = G; o < WAVE; o <<= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum_t(T v) {
    for (int o = WAVE >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max_t(T v) {
    for (int o = WAVE >> 1; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

template <typename T>
__device__ __forceinline__ T cross_group_sum_t(T v, int G) {
    for (int o = G; o < WAVE; o <<= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = WAVE >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int o = WAVE >> 1; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

template <typename T>
__device__ __forceinline__ T tsqrt(T x);
template <>
__device__ __forceinline__ double tsqrt<double>(double x) { return sqrt(x); }
template <>
__device__ __forceinline__ float tsqrt<float>(float x) { return sqrtf(x); }

// Distance of (t, s) with ||s|| = n to the second-order cone.
template <typename T>
__device__ __forceinline__ T cone_dist(T t, T n) {
    if (n <= t) return T(0);
    if (n <= -t) return tsqrt<T>(t * t + n * n);
    return (n - t) * T(0.70710678118654752440);
}

template <typename T, int VEC>
struct RowVec {
    T v[VEC];
};

template <typename T, int VEC>
__device__ __forceinline__ RowVec<T, VEC> load_vec(const T* p) {
    RowVec<T, VEC> r;
    if constexpr (VEC == 1) {
        r.v[0] = *p;
    } else {
        if constexpr (sizeof(T) == 8) {
            static_assert(VEC == 2, "FP64 rows use 16-byte loads at most");
            double2 x = *reinterpret_cast<const double2*>(p);
            r.v[0] = x.x;
            r.v[1] = x.y;
        } else if constexpr (VEC == 2) {
            float2 x = *reinterpret_cast<const float2*>(p);
            r.v[0] = x.x;
            r.v[1] = x.y;
        } else {
            float4 x = *reinterpret_cast<const float4*>(p);
            r.v[0] = x.x;
            r.v[1] = x.y;
            r.v[2] = x.z;
            r.v[3] = x.w;
        }
    }
    return r;
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec(T* p, const RowVec<T, VEC>& r) {
    if constexpr (VEC == 1) {
        *p = r.v[0];
    } else {
        if constexpr (sizeof(T) == 8) {
            *reinterpret_cast<double2*>(p) = make_double2(r.v[0], r.v[1]);
        } else if constexpr (VEC == 2) {
            *reinterpret_cast<float2*>(p) = make_float2(r.v[0], r.v[1]);
        } else {
            *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
        }
    }
}

// Per-ball projection quantities.
template <typename T>
struct BallProj {
    int cs;   // 0 interior, 1 polar, 2 other
    T n;      // ||s||
    T up;     // sigma * Pi(z)_0
    T gam;    // v+ = gam * s
    T Z;      // ||Pi(z)||^2
};

template <typename T>
__device__ __forceinline__ BallProj<T> project(T t, T nn, T sig) {
    BallProj<T> b;
    b.n = tsqrt<T>(nn);
    if (b.n <= t) {
        b.cs = 0;
        b.up = sig * t;
        b.gam = sig;
        b.Z = t * t + nn;
    } else if (b.n <= -t) {
        b.cs = 1;
        b.up = T(0);
        b.gam = T(0);
        b.Z = T(0);
    } else {
        b.cs = 2;
        T hp = T(0.5) * (t + b.n);
        b.up = sig * hp;
        b.gam = sig * hp / b.n;
        b.Z = T(2) * hp * hp;
    }
    return b;
}

// ---------------------------------------------------------------------------
// Evaluation pass
// ---------------------------------------------------------------------------

// Scalar accumulator slots of the evaluation pass (per lane, flushed to the
// per-wave FP64 record).
enum : int { A_SU = 0, A_Z1, A_NI, A_NM, A_SG, A_DM, A_RS, A_WW, A_KU, A_BYTES, A_N };

template <typename T>
struct FlushPeriod {
    static constexpr int steps = 1 << 30;  // FP64 sums: no intermediate flush
};
template <>
struct FlushPeriod<float> {
    static constexpr int steps = 64;  // FP32 partial sums cover at most 64 balls per lane
};

// The evaluation pass over one wave's contiguous range of balls.
//
// KIND 0: evaluation at y = x_base + dir (Psi trials along the segment,
//         gradient and Hessian parts, the mid list);
// KIND 1: evaluation plus the updated multipliers sigma Pi(z) and the KKT terms
//         at y (the single-evaluation entry point);
// KIND 2: multiplier update at x_j, its KKT terms, and the first evaluation of
//         the next outer iteration at sigma_{k+1}.
// TRL: Armijo trials per lane (ceil(NT / G) rounded up to 1, 3 or 9).
//
// Loads are software-pipelined: the rows (and radii, u) of the next group of
// balls are requested before the current group is processed, so each wave
// keeps two steps of loads in flight.
template <typename T, int VEC, int NLMAX, int KIND, int TRL>
__device__ __forceinline__ void pass_body(const PassArgs& a, const PassConfig& cfg, int blk) {
    extern __shared__ double lds[];
    const double* st = a.state;
    const int d = a.d;
    const int G = cfg.G;
    const int nl = cfg.nl;
    const StateLayout sl = a.sl;
    const RecLayout rl = a.rl;

    const bool have_dir = (KIND != 2) && st[S_HAVE_DIR] != 0.0;
    constexpr bool is_mult = (KIND == 2);
    constexpr bool want_kkt = (KIND != 0);

    // the evaluation point y = x_base + dir and the direction, staged in LDS
    double* l_c = lds;
    double* l_dc = lds + d;
    double* l_red = lds + 2 * d;
    double part = 0.0;
    for (int k = threadIdx.x; k < d; k += PASS_THREADS) {
        double dk = have_dir ? st[sl.dir + 1 + k] : 0.0;
        l_c[k] = st[sl.xb + 1 + k] + dk;
        l_dc[k] = dk;
        part += dk * dk;
    }
    l_red[threadIdx.x] = part;
    __syncthreads();
    for (int o = PASS_THREADS / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) l_red[threadIdx.x] += l_red[threadIdx.x + o];
        __syncthreads();
    }
    const T dc2 = (T)l_red[0];
    const double dirr_d = have_dir ? st[sl.dir] : 0.0;
    const T r1 = (T)(st[sl.xb] + dirr_d);
    const T dirr = (T)dirr_d;
    const double sig_a_d = st[S_SIGMA];
    const double sig_b_d = st[S_SIGMA_NEXT];
    const T sig_a = (T)sig_a_d;
    const T inv_a = (T)(1.0 / sig_a_d);
    const T sig_b = (T)sig_b_d;
    const T inv_b = (T)(1.0 / sig_b_d);

    const T* C = static_cast<const T*>(a.C);
    const T* R = static_cast<const T*>(a.R);
    const T* U = static_cast<const T*>(a.U);
    const T* V = static_cast<const T*>(a.V);
    T* Uo = static_cast<T*>(a.Uout);
    T* Vo = static_cast<T*>(a.Vout);

    const int lane = lane_id();
    const int wid = threadIdx.x / WAVE;
    const int64_t gw = (int64_t)blk * WPB + wid;
    const int gi = lane / G;
    const int gl = lane % G;
    const int bpw = WAVE / G;
    const bool leader = (gl == 0);
    const int64_t wbeg = gw * cfg.bw;
    const int64_t wend = min(a.m, wbeg + cfg.bw);
    const T es_bytes = (T)sizeof(T);

    // per-lane owned elements; y and dir in the working precision in LDS
    // (read per use: they would cost 4 registers per owned element)
    T* l_cT = reinterpret_cast<T*>(l_red + PASS_THREADS);
    T* l_dT = l_cT + d;
    for (int k = threadIdx.x; k < d; k += PASS_THREADS) {
        l_cT[k] = (T)l_c[k];
        l_dT[k] = (T)l_dc[k];
    }
    __syncthreads();
    int base[NLMAX];
    bool own[NLMAX];
#pragma unroll
    for (int j = 0; j < NLMAX; ++j) {
        base[j] = (j * G + gl) * VEC;
        own[j] = (j < nl) && (base[j] < d);
    }

    // the wave's record doubles as the FP64 accumulator of the flushes
    double* rec = a.rec + gw * rl.len;
    for (int e = lane; e < rl.len; e += WAVE) rec[e] = 0.0;

    T sacc[A_N];
    T tacc[TRL];
    T tam[TRL];  // 1 - eta of this lane's trials
#pragma unroll
    for (int r = 0; r < TRL; ++r) {
        const int l = r * G + gl;
        tam[r] = (l < NT) ? T(1) - (T)a.etas[l] : T(1);
    }
    T vsv[NLMAX][VEC], vsw[NLMAX][VEC], vkv[NLMAX][VEC];
    T mx_p = 0, mx_d = 0, mx_c = 0;
    auto zero_acc = [&]() {
#pragma unroll
        for (int k = 0; k < A_N; ++k) sacc[k] = T(0);
#pragma unroll
        for (int k = 0; k < TRL; ++k) tacc[k] = T(0);
#pragma unroll
        for (int j = 0; j < NLMAX; ++j)
#pragma unroll
            for (int q = 0; q < VEC; ++q) vsv[j][q] = vsw[j][q] = vkv[j][q] = T(0);
    };
    auto flush = [&]() {
        T sred[A_N];
#pragma unroll
        for (int k = 0; k < A_N; ++k) sred[k] = wave_sum_t<T>(sacc[k]);
        if (lane == 0) {
            rec[rl.su] += (double)sred[A_SU];
            rec[rl.z1] += (double)sred[A_Z1];
            rec[rl.ni] += (double)sred[A_NI];
            rec[rl.nm] += (double)sred[A_NM];
            rec[rl.sg] += (double)sred[A_SG];
            rec[rl.dm] += (double)sred[A_DM];
            rec[rl.rs] += (double)sred[A_RS];
            rec[rl.ww] += (double)sred[A_WW];
            rec[rl.ku] += (double)sred[A_KU];
            rec[rl.bytes] += (double)sred[A_BYTES];
        }
        if (have_dir) {
#pragma unroll
            for (int r = 0; r < TRL; ++r) {
                const T v = cross_group_sum_t<T>(tacc[r], G);
                const int l = r * G + lane;
                if (lane < G && l < NT) rec[rl.trial + l] += (double)v;
            }
        }
#pragma unroll
        for (int j = 0; j < NLMAX; ++j) {
            if (j >= nl) break;
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const T a1 = cross_group_sum_t<T>(vsv[j][q], G);
                const T a2 = cross_group_sum_t<T>(vsw[j][q], G);
                T a3 = T(0);
                if constexpr (want_kkt) a3 = cross_group_sum_t<T>(vkv[j][q], G);
                if (lane < G && own[j]) {
                    rec[rl.sv + base[j] + q] += (double)a1;
                    rec[rl.sw + base[j] + q] += (double)a2;
                    if constexpr (want_kkt) rec[rl.kv + base[j] + q] += (double)a3;
                }
            }
        }
        zero_acc();
    };
    zero_acc();

    int32_t mid_count = 0;
    int32_t* mid_idx = a.want_mid ? a.mid_idx + gw * cfg.bw : nullptr;
    double* mid_coef = a.want_mid ? a.mid_coef + gw * cfg.bw : nullptr;

    // loads of one group of balls (one ball per lane group)
    RowVec<T, VEC> cur[NLMAX], nxt[NLMAX];
    T r_cur = 0, u_cur = 0, r_nxt = 0, u_nxt = 0;
    auto load_step = [&](int64_t b0, RowVec<T, VEC> (&buf)[NLMAX], T& rr, T& uu) {
        const int64_t i = b0 + gi;
        const bool act = i < wend;
        rr = (R && act) ? R[i] : T(0);
        uu = (U && act) ? U[i] : T(0);
#pragma unroll
        for (int j = 0; j < NLMAX; ++j) {
            if (act && own[j]) {
                buf[j] = load_vec<T, VEC>(C + i * d + base[j]);
            } else {
#pragma unroll
                for (int q = 0; q < VEC; ++q) buf[j].v[q] = T(0);
            }
        }
    };

    const int64_t chunk = (int64_t)bpw * FlushPeriod<T>::steps;
    for (int64_t c0 = wbeg; c0 < wend; c0 += chunk) {
        const int64_t c1 = min(wend, c0 + chunk);
        load_step(c0, cur, r_cur, u_cur);
        for (int64_t b0 = c0; b0 < c1; b0 += bpw) {
            if (b0 + bpw < c1) load_step(b0 + bpw, nxt, r_nxt, u_nxt);
            const int64_t i = b0 + gi;
            const bool active = i < wend;
            const T ri = r_cur;
            const T ui = u_cur;
            const bool hasv = V && (ui != T(0));
            T s[NLMAX][VEC], vv[NLMAX][VEC];
            T nn = 0, q = 0, ee = 0, es = 0;
#pragma unroll
            for (int j = 0; j < NLMAX; ++j) {
                const bool ok = active && own[j];
                RowVec<T, VEC> vr, cy, dy;
#pragma unroll
                for (int qq = 0; qq < VEC; ++qq) vr.v[qq] = cy.v[qq] = dy.v[qq] = T(0);
                if (ok && hasv) vr = load_vec<T, VEC>(V + i * d + base[j]);
                if (own[j]) {
                    cy = load_vec<T, VEC>(l_cT + base[j]);
                    if (have_dir) dy = load_vec<T, VEC>(l_dT + base[j]);
                }
#pragma unroll
                for (int qq = 0; qq < VEC; ++qq) {
                    const T ek = ok ? cur[j].v[qq] - cy.v[qq] : T(0);
                    if constexpr (is_mult) cur[j].v[qq] = ek;  // keep c_i - y for the next subproblem
                    vv[j][qq] = vr.v[qq];
                    s[j][qq] = ek + vr.v[qq] * inv_a;
                    nn += s[j][qq] * s[j][qq];
                    if constexpr (KIND != 2) {
                        if (have_dir) q += s[j][qq] * dy.v[qq];
                    }
                    if constexpr (want_kkt) {
                        ee += ek * ek;
                        es += ek * s[j][qq];
                    }
                }
            }
            nn = group_sum<T>(nn, G);
            if (have_dir) q = group_sum<T>(q, G);
            if constexpr (want_kkt) {
                ee = group_sum<T>(ee, G);
                es = group_sum<T>(es, G);
            }
            if (leader && active)
                sacc[A_BYTES] += es_bytes * (T)(d + (R ? 1 : 0) + (U ? 1 : 0) + (hasv ? d : 0));
            const T t = ri - r1 + ui * inv_a;
            BallProj<T> pa = project<T>(t, nn, sig_a);
            if (!active) pa.cs = 1, pa.up = T(0), pa.gam = T(0), pa.Z = T(0);

            T te = t, nne = nn, ue = ui;
            BallProj<T> pe = pa;
            T sig_e = sig_a;

            if constexpr (want_kkt) {
                // updated multipliers w+ = sigma Pi(z) at y and the KKT terms there
                const T un = pa.up;
                const bool wrow = Vo && (un != T(0) || a.dense_vout);
                if (leader && active) {
                    sacc[A_KU] += un;
                    const T tp = r1 - ri;
                    mx_p = fmax(mx_p, cone_dist<T>(tp, tsqrt<T>(ee)));
                    mx_d = fmax(mx_d, cone_dist<T>(un, pa.gam * pa.n));
                    mx_c = fmax(mx_c, fabs(tp * un - pa.gam * es));
                    if (Uo) Uo[i] = un;
                    sacc[A_BYTES] += (Uo ? es_bytes : T(0)) + (wrow ? es_bytes * (T)d : T(0));
                }
#pragma unroll
                for (int j = 0; j < NLMAX; ++j) {
                    RowVec<T, VEC> vn;
#pragma unroll
                    for (int qq = 0; qq < VEC; ++qq) {
                        vn.v[qq] = pa.gam * s[j][qq];
                        vkv[j][qq] += vn.v[qq];
                    }
                    if (active && own[j] && wrow) store_vec<T, VEC>(Vo + i * d + base[j], vn);
                    if constexpr (is_mult) {
#pragma unroll
                        for (int qq = 0; qq < VEC; ++qq) vv[j][qq] = vn.v[qq];
                    }
                }
                if constexpr (is_mult) {
                    // the first evaluation of the next subproblem: w+ and sigma_{k+1}
                    ue = un;
                    sig_e = sig_b;
                    te = ri - r1 + un * inv_b;
                    T n2 = 0;
#pragma unroll
                    for (int j = 0; j < NLMAX; ++j)
#pragma unroll
                        for (int qq = 0; qq < VEC; ++qq) {
                            s[j][qq] = cur[j].v[qq] + vv[j][qq] * inv_b;
                            n2 += s[j][qq] * s[j][qq];
                        }
                    nne = group_sum<T>(n2, G);
                    pe = project<T>(te, nne, sig_b);
                    if (!active) pe.cs = 1, pe.up = T(0), pe.gam = T(0), pe.Z = T(0);
                }
            }

            // ---- evaluation sums at (y, multipliers in use, sigma_e)
            if (leader && active) {
                sacc[A_SU] += pe.up;
                sacc[A_Z1] += pe.Z;
                const T du = pe.up - ue;
                sacc[A_DM] += du * du;
                sacc[A_WW] += ue * ue;
                if (pe.cs != 1) sacc[A_RS] += fabs(te) + pe.n;
                if (pe.cs == 0) sacc[A_NI] += T(1);
                if (pe.cs == 2) {
                    sacc[A_NM] += T(1);
                    sacc[A_SG] += pe.gam;
                }
            }
            // a polar ball with zero multipliers contributes nothing elementwise
            const bool quiet = (pe.cs == 1) && (ue == T(0));
            if (!quiet) {
                const T inv_n = (pe.cs == 2) ? T(1) / pe.n : T(0);
                T dmb = 0, wwb = 0;
#pragma unroll
                for (int j = 0; j < NLMAX; ++j)
#pragma unroll
                    for (int qq = 0; qq < VEC; ++qq) {
                        const T vp = pe.gam * s[j][qq];
                        const T dvk = vp - vv[j][qq];
                        vsv[j][qq] += vp;
                        vsw[j][qq] += s[j][qq] * inv_n;
                        dmb += dvk * dvk;
                        wwb += vv[j][qq] * vv[j][qq];
                    }
                sacc[A_DM] += dmb;
                sacc[A_WW] += wwb;
            }
            // Armijo trials along x_base + eta dir: lane gl takes trials gl, gl + G, ...
            if (have_dir && active) {
#pragma unroll
                for (int r = 0; r < TRL; ++r) {
                    const T am = tam[r];
                    const T tl = te + am * dirr;
                    T n2 = nne + T(2) * am * q + am * am * dc2;
                    n2 = n2 > T(0) ? n2 : T(0);
                    if (r * G + gl < NT) tacc[r] += project<T>(tl, n2, sig_e).Z;
                }
            }
            // mid list of the rank-one Hessian part: coef_i = -sigma t_i / (2 n_i^3)
            if (a.want_mid) {
                const bool is_mid = active && pe.cs == 2;
                const unsigned long long bal = __ballot(is_mid && leader);
                if (is_mid && leader) {
                    const unsigned long long lower = bal & ((1ull << lane) - 1ull);
                    const int pos = mid_count + __popcll(lower);
                    mid_idx[pos] = (int32_t)i;
                    const double nd = (double)pe.n;
                    mid_coef[pos] = -(double)sig_e * (double)te / (2.0 * nd * nd * nd);
                }
                mid_count += __popcll(bal);
            }
#pragma unroll
            for (int j = 0; j < NLMAX; ++j) cur[j] = nxt[j];
            r_cur = r_nxt;
            u_cur = u_nxt;
        }
        flush();
    }
    const T mp = wave_max_t<T>(mx_p), md = wave_max_t<T>(mx_d), mc = wave_max_t<T>(mx_c);
    if (lane == 0) {
        rec[rl.kmax + 0] = (double)mp;
        rec[rl.kmax + 1] = (double)md;
        rec[rl.kmax + 2] = (double)mc;
        if (a.mid_cnt) a.mid_cnt[gw] = mid_count;
    }
    // combine the block's wave records into the first one, in wave order
    __syncthreads();
    double* r0 = a.rec + (int64_t)blk * WPB * rl.len;
    for (int e = threadIdx.x; e < rl.len; e += PASS_THREADS) {
        const bool ismax = e >= rl.kmax && e < rl.kmax + 3;
        double v = r0[e];
#pragma unroll
        for (int w = 1; w < WPB; ++w) {
            const double x = r0[w * rl.len + e];
            v = ismax ? fmax(v, x) : v + x;
        }
        r0[e] = v;
    }
}

// The pass kernel: the solver's evaluation or multiplier update, as the device
// state's mode says (nothing when the run is done); with force_mode =
// PM_EVAL, a single evaluation (with the updated multipliers and KKT terms
// when want_kkt is set).
template <typename T, int VEC, int NLMAX, int TRL>
__device__ __forceinline__ void pass_dispatch(const PassArgs& a, const PassConfig& cfg, int blk) {
    const int mode = a.force_mode >= 0 ? a.force_mode : (int)a.state[S_MODE];
    if (mode == PM_EVAL) {
        if (a.want_kkt)
            pass_body<T, VEC, NLMAX, 1, TRL>(a, cfg, blk);
        else
            pass_body<T, VEC, NLMAX, 0, TRL>(a, cfg, blk);
    } else if (mode == PM_MULT) {
        pass_body<T, VEC, NLMAX, 2, TRL>(a, cfg, blk);
    }
}

template <typename T, int VEC, int NLMAX, int TRL>
__global__ __launch_bounds__(PASS_THREADS) void pass_kernel(PassArgs a, PassConfig cfg) {
    pass_dispatch<T, VEC, NLMAX, TRL>(a, cfg, blockIdx.x);
}

// Several instances in one launch (a tick of the multi-instance server): the
// flat block index is split by the list's ascending block offsets, and each
// instance runs exactly the blocks, arithmetic and reduction order it would
// run alone.
__device__ __forceinline__ int tick_find(const TickList& L, int b) {
    int lo = 0, hi = L.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.off[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename T, int VEC, int NLMAX, int TRL>
__global__ __launch_bounds__(PASS_THREADS) void pass_batch_kernel(const BatchItem* tab, TickList L) {
    const int k = tick_find(L, blockIdx.x);
    const BatchItem& it = tab[L.slot[k]];
    pass_dispatch<T, VEC, NLMAX, TRL>(it.pa, it.pc, blockIdx.x - L.off[k]);
}

// Kernels that take more than 64 KiB of dynamic LDS opt in to the size.
static hipError_t ensure_dynamic_lds(const void* fn, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T>
static size_t pass_lds_bytes(int d) {
    return sizeof(double) * (2 * (size_t)d + PASS_THREADS) + sizeof(T) * (2 * (size_t)d + 4);
}

// The template instance of the pass for (dtype, config): visits
// f.go<T, VEC, NLMAX, TRL>().  Valid (vec, nlmax) pairs: G < 64 implies
// nl <= ceil(8 / vec); G = 64 (one ball per wave) uses the larger nlmax, with
// one Armijo trial per lane; narrower groups take ceil(NT / G) trials per
// lane, rounded up to 3 or 9.
template <typename T, int VEC, int NLMAX, class F>
static hipError_t visit_trl(const PassConfig& cfg, F& f) {
    if (cfg.G >= 16) return f.template go<T, VEC, NLMAX, 1>();
    if (cfg.G >= 4) return f.template go<T, VEC, NLMAX, 3>();
    return f.template go<T, VEC, NLMAX, 9>();
}

template <typename T, int VEC, class F>
static hipError_t visit_vec(const PassConfig& cfg, F& f) {
    if (cfg.G < 64) {
        if constexpr (VEC == 4) return visit_trl<T, VEC, 2>(cfg, f);
        if constexpr (VEC == 2) {
            if (cfg.nlmax == 2) return visit_trl<T, VEC, 2>(cfg, f);
            return visit_trl<T, VEC, 4>(cfg, f);
        }
        if (cfg.nlmax == 2) return visit_trl<T, VEC, 2>(cfg, f);
        if (cfg.nlmax == 4) return visit_trl<T, VEC, 4>(cfg, f);
        return visit_trl<T, VEC, 8>(cfg, f);
    }
    if (cfg.nlmax <= 2) return f.template go<T, VEC, 2, 1>();
    if (cfg.nlmax == 4) return f.template go<T, VEC, 4, 1>();
    if (cfg.nlmax == 8) return f.template go<T, VEC, 8, 1>();
    return f.template go<T, VEC, 16, 1>();
}

template <class F>
static hipError_t visit_pass(int dtype, const PassConfig& cfg, F& f) {
    if (dtype == 0) {
        if (cfg.vec == 2) return visit_vec<double, 2>(cfg, f);
        return visit_vec<double, 1>(cfg, f);
    }
    if (cfg.vec == 4) return visit_vec<float, 4>(cfg, f);
    if (cfg.vec == 2) return visit_vec<float, 2>(cfg, f);
    return visit_vec<float, 1>(cfg, f);
}

}  // namespace meb
