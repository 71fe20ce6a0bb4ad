// HIP kernels of libmeb.so for gfx950 (MI355X): the proximal augmented
// Lagrangian evaluation pass of ripALM for the minimum enclosing ball of
// balls, its deterministic reductions, the rank-one Hessian contraction, the
// device-side control step (Armijo decision, relative stopping test,
// multiplier bookkeeping, FP64 Cholesky solve), the screening and
// feasibility scans, and the precision-preparation and gather kernels.
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
            double2 x = *reinterpret_cast<const double2*>(p);
            r.v[0] = x.x;
            r.v[1] = x.y;
        } else {
            float2 x = *reinterpret_cast<const float2*>(p);
            r.v[0] = x.x;
            r.v[1] = x.y;
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
        } else {
            *reinterpret_cast<float2*>(p) = make_float2(r.v[0], r.v[1]);
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
    static constexpr int steps = 32;  // FP32 partial sums cover at most 32 balls per lane
};

// KIND 0: evaluation (Psi trials, gradient, Hessian parts) -- runs when the
//         state's mode is PM_EVAL;
// KIND 1: evaluation plus the updated multipliers and KKT terms at the same
//         point (the single-evaluation entry point);
// KIND 2: multiplier update at x_j, KKT terms, and the first evaluation of the
//         next outer iteration -- runs when the mode is PM_MULT.
// TRL: Armijo trials per lane (ceil(NT / G) rounded up to 1, 3 or 9).
template <typename T, int VEC, int NLMAX, int KIND, int TRL>
__device__ __forceinline__ void pass_body(const PassArgs& a, const PassConfig& cfg) {
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
    const int64_t gw = (int64_t)blockIdx.x * WPB + wid;
    const int gi = lane / G;
    const int gl = lane % G;
    const int bpw = WAVE / G;
    const bool leader = (gl == 0);
    const int64_t wbeg = gw * cfg.bw;
    const int64_t wend = min(a.m, wbeg + cfg.bw);
    const T es_bytes = (T)sizeof(T);

    // per-lane constants: the owned elements of y and of dir
    int base[NLMAX];
    bool own[NLMAX];
    T cv[NLMAX][VEC], dv[NLMAX][VEC];
#pragma unroll
    for (int j = 0; j < NLMAX; ++j) {
        base[j] = (j * G + gl) * VEC;
        own[j] = (j < nl) && (base[j] < d);
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            cv[j][q] = own[j] ? (T)l_c[base[j] + q] : T(0);
            dv[j][q] = own[j] ? (T)l_dc[base[j] + q] : T(0);
        }
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
        // scalars: wave sums; trials and vectors: sums across groups
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

    const int64_t chunk = (int64_t)bpw * FlushPeriod<T>::steps;
    for (int64_t c0 = wbeg; c0 < wend; c0 += chunk) {
    const int64_t c1 = min(wend, c0 + chunk);
    for (int64_t b0 = c0; b0 < c1; b0 += bpw) {
        const int64_t i = b0 + gi;
        const bool active = i < wend;
        const T ri = (R && active) ? R[i] : T(0);
        const T ui = (U && active) ? U[i] : T(0);
        const bool hasv = V && (ui != T(0));
        T s[NLMAX][VEC], vv[NLMAX][VEC], e[NLMAX][VEC];
        T nn = 0, q = 0, ee = 0, es = 0;
#pragma unroll
        for (int j = 0; j < NLMAX; ++j) {
            const bool ok = active && own[j];
            RowVec<T, VEC> cr, vr;
#pragma unroll
            for (int qq = 0; qq < VEC; ++qq) cr.v[qq] = vr.v[qq] = T(0);
            if (ok) {
                cr = load_vec<T, VEC>(C + i * d + base[j]);
                if (hasv) vr = load_vec<T, VEC>(V + i * d + base[j]);
            }
#pragma unroll
            for (int qq = 0; qq < VEC; ++qq) {
                const T ek = ok ? cr.v[qq] - cv[j][qq] : T(0);
                if constexpr (is_mult) e[j][qq] = ek;
                vv[j][qq] = vr.v[qq];
                s[j][qq] = ek + vr.v[qq] * inv_a;
                nn += s[j][qq] * s[j][qq];
                if constexpr (KIND != 2) {
                    if (have_dir) q += s[j][qq] * dv[j][qq];
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
                        s[j][qq] = e[j][qq] + vv[j][qq] * inv_b;
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
    double* r0 = a.rec + (int64_t)blockIdx.x * WPB * rl.len;
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

// The solver's pass: evaluation or multiplier update, as the device state says.
template <typename T, int VEC, int NLMAX, int TRL>
__global__ __launch_bounds__(PASS_THREADS) void pass_kernel(PassArgs a, PassConfig cfg) {
    const int mode = (int)a.state[S_MODE];
    if (mode == PM_EVAL)
        pass_body<T, VEC, NLMAX, 0, TRL>(a, cfg);
    else if (mode == PM_MULT)
        pass_body<T, VEC, NLMAX, 2, TRL>(a, cfg);
}

// A single evaluation (KIND 0) or evaluation with the updated multipliers and
// KKT terms (KIND 1), independent of the state's mode.
template <typename T, int VEC, int NLMAX, int KIND, int TRL>
__global__ __launch_bounds__(PASS_THREADS) void pass_eval_kernel(PassArgs a, PassConfig cfg) {
    pass_body<T, VEC, NLMAX, KIND, TRL>(a, cfg);
}

PassConfig choose_pass_config(int64_t m, int d, int dtype, int num_cu) {
    PassConfig c;
    c.vec = (d % 2 == 0) ? 2 : 1;
    // up to 4 loads (4 VEC elements) per lane when a ball has fewer than 64
    // lanes: enough work per lane to amortize the cross-lane reduction of
    // each ball, few enough to keep registers low.  Longer rows use 64 lanes
    // and 8 or 16 loads.
    const int per_lane_target = 4;
    int need = (d + c.vec * per_lane_target - 1) / (c.vec * per_lane_target);
    int G = 1;
    while (G < need && G < 64) G <<= 1;
    c.G = G;
    c.nl = (d + G * c.vec - 1) / (G * c.vec);
    c.nlmax = c.nl <= 4 ? 4 : (c.nl <= 8 ? 8 : 16);
    c.waves_per_block = WPB;
    const int bpw = WAVE / G;
    // enough waves to fill the machine, each streaming a contiguous range
    int64_t max_waves = (int64_t)num_cu * 8;
    int64_t steps = (m + bpw - 1) / bpw;
    int64_t waves = steps < max_waves ? steps : max_waves;
    if (waves < 1) waves = 1;
    int64_t steps_per_wave = (steps + waves - 1) / waves;
    c.bw = steps_per_wave * bpw;
    waves = (m + c.bw - 1) / c.bw;
    c.blocks = (int)((waves + WPB - 1) / WPB);
    c.nwaves = c.blocks * WPB;
    (void)dtype;
    return c;
}

// kind 0 / 1: pass_eval_kernel; kind 3: the solver's pass_kernel
template <typename T, int VEC, int NLMAX, int KIND, int TRL>
static hipError_t launch_pass_t(const PassArgs& a, const PassConfig& cfg, hipStream_t s) {
    size_t lds = sizeof(double) * (2 * (size_t)a.d + PASS_THREADS);
    if constexpr (KIND == 3)
        hipLaunchKernelGGL((pass_kernel<T, VEC, NLMAX, TRL>), dim3(cfg.blocks), dim3(PASS_THREADS), lds, s, a, cfg);
    else
        hipLaunchKernelGGL((pass_eval_kernel<T, VEC, NLMAX, KIND, TRL>), dim3(cfg.blocks), dim3(PASS_THREADS), lds, s,
                           a, cfg);
    return hipGetLastError();
}

// kernels that evaluate Armijo trials need one trial slot per G lanes
template <typename T, int VEC, int KIND>
static hipError_t launch_pass_small(const PassArgs& a, const PassConfig& cfg, hipStream_t s) {
    if (cfg.G >= 16) return launch_pass_t<T, VEC, 4, KIND, 1>(a, cfg, s);
    if (cfg.G >= 4) return launch_pass_t<T, VEC, 4, KIND, 3>(a, cfg, s);
    return launch_pass_t<T, VEC, 4, KIND, 9>(a, cfg, s);
}

template <typename T, int KIND>
static hipError_t launch_pass_K(const PassArgs& a, const PassConfig& cfg, hipStream_t s) {
    // nlmax 8 and 16 are used only with G = 64 lanes per ball
    if (cfg.vec == 2) {
        if (cfg.nlmax == 4) return launch_pass_small<T, 2, KIND>(a, cfg, s);
        if (cfg.nlmax == 8) return launch_pass_t<T, 2, 8, KIND, 1>(a, cfg, s);
        return launch_pass_t<T, 2, 16, KIND, 1>(a, cfg, s);
    }
    if (cfg.nlmax == 4) return launch_pass_small<T, 1, KIND>(a, cfg, s);
    if (cfg.nlmax == 8) return launch_pass_t<T, 1, 8, KIND, 1>(a, cfg, s);
    return launch_pass_t<T, 1, 16, KIND, 1>(a, cfg, s);
}

template <typename T>
static hipError_t launch_pass_T(const PassArgs& a, const PassConfig& cfg, int kind, hipStream_t s) {
    if (kind == 0) return launch_pass_K<T, 0>(a, cfg, s);
    if (kind == 1) return launch_pass_K<T, 1>(a, cfg, s);
    return launch_pass_K<T, 3>(a, cfg, s);
}

hipError_t launch_pass(const PassArgs& a, const PassConfig& cfg, int kind, hipStream_t s) {
    if (a.dtype == 0) return launch_pass_T<double>(a, cfg, kind, s);
    return launch_pass_T<float>(a, cfg, kind, s);
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of per-wave records: out[e] = sum_w rec[w][e]
// (maximum for the three KKT maxima).  Two stages: slices of records, then
// the slices; both in ascending order.
// ---------------------------------------------------------------------------

constexpr int RED_SLICE = 32;

// Stage 1: block (x, y) sums entries [64 x, 64 x + 64) over the records of
// slice y; its four waves take records w = 4 k + wave, then combine in wave
// order.  Records are `stride` doubles apart.
__global__ __launch_bounds__(256) void reduce_stage1(const double* rec, int nrec, int len, int64_t stride, int max_lo,
                                                     int max_hi, double* part) {
    __shared__ double sp[4][64];
    const int e = blockIdx.x * 64 + (threadIdx.x & 63);
    const int sub = threadIdx.x >> 6;
    const int per = (nrec + gridDim.y - 1) / gridDim.y;
    const int w0 = blockIdx.y * per, w1 = min(nrec, w0 + per);
    const bool ismax = (e >= max_lo && e < max_hi);
    double acc = 0.0;
    if (e < len) {
        for (int w = w0 + sub; w < w1; w += 4) {
            const double v = rec[(int64_t)w * stride + e];
            acc = ismax ? fmax(acc, v) : acc + v;
        }
    }
    sp[sub][threadIdx.x & 63] = acc;
    __syncthreads();
    if (threadIdx.x < 64 && e < len) {
        double v = sp[0][threadIdx.x];
        for (int k = 1; k < 4; ++k) v = ismax ? fmax(v, sp[k][threadIdx.x]) : v + sp[k][threadIdx.x];
        part[(size_t)blockIdx.y * len + e] = v;
    }
}

__global__ __launch_bounds__(256) void reduce_stage2(const double* part, int nslice, int len, int max_lo, int max_hi,
                                                     double* out) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= len) return;
    const bool ismax = (e >= max_lo && e < max_hi);
    double acc = 0.0;
    for (int w = 0; w < nslice; ++w) {
        const double v = part[(size_t)w * len + e];
        acc = ismax ? fmax(acc, v) : acc + v;
    }
    out[e] = acc;
}

hipError_t launch_reduce_records(const double* rec, int nrec, int len, int64_t stride, double* out, hipStream_t s) {
    // `out` must have room for (RED_SLICE + 1) * len doubles: the slice
    // partials live after the result.  The three maxima sit at a fixed
    // offset ahead of the d-dependent vector parts of the record.
    const RecLayout rl = RecLayout::make(0);
    const int max_lo = rl.kmax, max_hi = rl.kmax + 3;
    int nslice = (nrec + 15) / 16;
    if (nslice > RED_SLICE) nslice = RED_SLICE;
    if (nslice < 1) nslice = 1;
    double* part = out + len;
    dim3 g1((len + 63) / 64, nslice);
    hipLaunchKernelGGL(reduce_stage1, g1, dim3(256), 0, s, rec, nrec, len, stride, max_lo, max_hi, part);
    hipLaunchKernelGGL(reduce_stage2, dim3((len + 255) / 256), dim3(256), 0, s, part, nslice, len, max_lo, max_hi,
                       out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rank-one Hessian contraction  sum_{i in mid} coef_i s_i s_i^T  (FP64
// accumulation), tiled T x T over the upper triangle of d x d, split over
// the wave segments of the mid list.  s_i is recomputed from C and V
// exactly as the pass computed it.
// ---------------------------------------------------------------------------

constexpr int SYRK_T = 32;
constexpr int SYRK_KB = 32;     // mid balls staged per step
constexpr int SYRK_KSPLIT = 8;  // blocks along the mid list per tile pair

int syrk_tile() { return SYRK_T; }

int syrk_ksplit(int d) {
    (void)d;
    return SYRK_KSPLIT;
}

// Per-wave mid counts -> exclusive offsets and total, then the copy into one
// list.  Skipped when the run is done.
__global__ __launch_bounds__(1024) void mid_scan_kernel(const int32_t* cnt, int nw, int64_t* offs, int64_t* total,
                                                        const double* st) {
    __shared__ int64_t sc[1024];
    if ((int)st[S_MODE] == PM_DONE) return;
    const int t = threadIdx.x;
    const int per = (nw + 1023) / 1024;
    const int w0 = t * per, w1 = min(nw, w0 + per);
    int64_t c = 0;
    for (int w = w0; w < w1; ++w) c += cnt[w];
    sc[t] = c;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t v = t >= o ? sc[t - o] : 0;
        __syncthreads();
        sc[t] += v;
        __syncthreads();
    }
    int64_t run = t > 0 ? sc[t - 1] : 0;
    for (int w = w0; w < w1; ++w) {
        offs[w] = run;
        run += cnt[w];
    }
    if (t == 1023) *total = sc[1023];
}

__global__ __launch_bounds__(256) void mid_copy_kernel(const int32_t* cnt, int nw, int64_t bw, const int32_t* si,
                                                       const double* sc, const int64_t* offs, int32_t* oi,
                                                       double* oc, const double* st) {
    if ((int)st[S_MODE] == PM_DONE) return;
    const int lane = lane_id();
    const int64_t w = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (w >= nw) return;
    const int64_t n = cnt[w], off = offs[w];
    for (int64_t k = lane; k < n; k += WAVE) {
        oi[off + k] = si[w * bw + k];
        oc[off + k] = sc[w * bw + k];
    }
}

hipError_t launch_mid_compact(const int32_t* mid_cnt, int nwaves, int64_t bw, const int32_t* seg_idx,
                              const double* seg_coef, int64_t* offs, int64_t* total, int32_t* out_idx,
                              double* out_coef, const double* state, hipStream_t s) {
    hipLaunchKernelGGL(mid_scan_kernel, dim3(1), dim3(1024), 0, s, mid_cnt, nwaves, offs, total, state);
    hipLaunchKernelGGL(mid_copy_kernel, dim3((nwaves + 3) / 4), dim3(256), 0, s, mid_cnt, nwaves, bw, seg_idx,
                       seg_coef, offs, out_idx, out_coef, state);
    return hipGetLastError();
}

// Rank-one Hessian part  sum_{i in mid} coef_i s_i s_i^T  with FP64
// accumulation over the compacted mid list, tiled T x T over the upper
// triangle of the d x d block; blockIdx.y splits the list evenly.  s_i is
// recomputed from C and V exactly as the pass computed it.  In a line-search
// pass with more than skip_k rows the contraction is skipped (block 0 sets
// S_HSKIP) and the control step re-evaluates if it needs this H.
template <typename T>
__global__ __launch_bounds__(256) void syrk_kernel(SyrkArgs a) {
    __shared__ double sI[SYRK_KB][SYRK_T + 1];
    __shared__ double sJ[SYRK_KB][SYRK_T + 1];
    __shared__ double cf[SYRK_KB];
    __shared__ int32_t ix[SYRK_KB];
    double* st = a.state;
    const int mode = (int)st[S_MODE];
    if (mode == PM_DONE) return;
    const int d = a.d;
    const StateLayout sl = a.sl;
    const bool have_dir = (mode == PM_EVAL) && st[S_HAVE_DIR] != 0.0;
    const int64_t K = *a.list_total;
    const bool skip = have_dir && (double)K > a.skip_k;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) st[S_HSKIP] = skip ? 1.0 : 0.0;
    if (skip) return;
    const double sig = (mode == PM_MULT) ? st[S_SIGMA_NEXT] : st[S_SIGMA];
    const T inv = (T)(1.0 / sig);
    int p = blockIdx.x, I = 0;
    while (p >= a.ntile - I) {
        p -= a.ntile - I;
        ++I;
    }
    const int J = I + p;
    const int64_t per = (K + a.ksplit - 1) / a.ksplit;
    const int64_t k0 = (int64_t)blockIdx.y * per, k1 = min(K, k0 + per);
    const T* C = static_cast<const T*>(a.C);
    const T* V = static_cast<const T*>(a.V);
    const T* U = static_cast<const T*>(a.U);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[2][2] = {{0, 0}, {0, 0}};
    for (int64_t kb = k0; kb < k1; kb += SYRK_KB) {
        const int nk = (int)min((int64_t)SYRK_KB, k1 - kb);
        __syncthreads();
        if (threadIdx.x < SYRK_KB) {
            ix[threadIdx.x] = threadIdx.x < nk ? a.list_idx[kb + threadIdx.x] : 0;
            cf[threadIdx.x] = threadIdx.x < nk ? a.list_coef[kb + threadIdx.x] : 0.0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < SYRK_KB * SYRK_T * 2; e += 256) {
            const int which = e / (SYRK_KB * SYRK_T);
            const int r = (e / SYRK_T) % SYRK_KB;
            const int cc = e % SYRK_T;
            const int col = (which ? J : I) * SYRK_T + cc;
            double v = 0.0;
            if (r < nk && col < d) {
                const int64_t i = ix[r];
                const T ck = (T)(st[sl.xb + 1 + col] + (have_dir ? st[sl.dir + 1 + col] : 0.0));
                const T ek = C[i * d + col] - ck;
                const T vk = (V && U && U[i] != T(0)) ? V[i * d + col] : T(0);
                v = (double)(ek + vk * inv);
            }
            if (which)
                sJ[r][cc] = v;
            else
                sI[r][cc] = v;
        }
        __syncthreads();
        for (int r = 0; r < nk; ++r) {
            const double c = cf[r];
            const double a0 = sI[r][ty], a1 = sI[r][ty + 16];
            const double b0 = sJ[r][tx] * c, b1 = sJ[r][tx + 16] * c;
            acc[0][0] += a0 * b0;
            acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0;
            acc[1][1] += a1 * b1;
        }
    }
    const int npairs = gridDim.x;
    double* out = a.out + ((size_t)blockIdx.y * npairs + blockIdx.x) * SYRK_T * SYRK_T;
    out[ty * SYRK_T + tx] = acc[0][0];
    out[ty * SYRK_T + tx + 16] = acc[0][1];
    out[(ty + 16) * SYRK_T + tx] = acc[1][0];
    out[(ty + 16) * SYRK_T + tx + 16] = acc[1][1];
}

hipError_t launch_syrk(const SyrkArgs& a, hipStream_t s) {
    const int pairs = a.ntile * (a.ntile + 1) / 2;
    dim3 grid(pairs, a.ksplit);
    if (a.dtype == 0)
        hipLaunchKernelGGL(syrk_kernel<double>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(syrk_kernel<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Hessian assembly from the reduced record and the contraction blocks:
//   H_rr = tau/sigma + sigma N_I + sigma/2 N_mid
//   H_rc = sigma/2 sum_mid w_i
//   H_cc = (tau/sigma + sigma N_I + sum_mid gamma_i) I + sum_mid coef_i s_i s_i^T
// (the per-case generalized Jacobian of the cone projection, Section 4).
// ---------------------------------------------------------------------------

__device__ void assemble_H(int d, const RecLayout& rl, const double* red, const double* syrk, int ksplit, int ntile,
                           int have_syrk, double sigma, double tau, double* H) {
    const int n1 = d + 1;
    const double base = tau / sigma + sigma * red[rl.ni];
    const int npairs = ntile * (ntile + 1) / 2;
    for (int e = threadIdx.x; e < n1 * n1; e += blockDim.x) {
        const int a = e / n1, b = e % n1;
        double v;
        if (a == 0 && b == 0) {
            v = base + 0.5 * sigma * red[rl.nm];
        } else if (a == 0 || b == 0) {
            const int k = (a == 0 ? b : a) - 1;
            v = 0.5 * sigma * red[rl.sw + k];
        } else {
            const int k = a - 1, l = b - 1;
            v = (k == l) ? base + red[rl.sg] : 0.0;
            if (have_syrk) {
                int kk = k, ll = l;
                if (kk / SYRK_T > ll / SYRK_T) {
                    const int t = kk;
                    kk = ll;
                    ll = t;
                }
                const int I = kk / SYRK_T, J = ll / SYRK_T;
                // pair index of (I, J) in the row-major upper triangle
                const int pidx = I * ntile - I * (I - 1) / 2 + (J - I);
                const int ia = kk % SYRK_T, ib = ll % SYRK_T;
                double sacc = 0.0;
                for (int ks = 0; ks < ksplit; ++ks)
                    sacc += syrk[((size_t)ks * npairs + pidx) * SYRK_T * SYRK_T + ia * SYRK_T + ib];
                v += sacc;
            }
        }
        H[e] = v;
    }
}

// Parallel assembly of H into the state (one thread per entry).  Runs after
// the contraction and before the control step; it is a no-op when the run is
// done.  The control step reads H only when it takes a Newton step.
__global__ __launch_bounds__(256) void assemble_kernel(double* st, StateLayout sl, RecLayout rl, const double* red,
                                                       const double* syrk, int ksplit, int ntile, int have_syrk) {
    const int mode = (int)st[S_MODE];
    if (mode == PM_DONE) return;
    if (have_syrk && st[S_HSKIP] != 0.0) return;
    const double sigma = (mode == PM_MULT) ? st[S_SIGMA_NEXT] : st[S_SIGMA];
    const double tau = st[S_TAU];
    const int d = sl.n1 - 1, n1 = sl.n1;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n1 * n1) return;
    const int a = e / n1, b = e % n1;
    const double base = tau / sigma + sigma * red[rl.ni];
    double v;
    if (a == 0 && b == 0) {
        v = base + 0.5 * sigma * red[rl.nm];
    } else if (a == 0 || b == 0) {
        v = 0.5 * sigma * red[rl.sw + (a == 0 ? b : a) - 1];
    } else {
        const int k = a - 1, l = b - 1;
        v = (k == l) ? base + red[rl.sg] : 0.0;
        if (have_syrk) {
            int kk = k, ll = l;
            if (kk / SYRK_T > ll / SYRK_T) {
                const int t = kk;
                kk = ll;
                ll = t;
            }
            const int I = kk / SYRK_T, J = ll / SYRK_T;
            const int npairs = ntile * (ntile + 1) / 2;
            const int pidx = I * ntile - I * (I - 1) / 2 + (J - I);
            const int ia = kk % SYRK_T, ib = ll % SYRK_T;
            double sacc = 0.0;
            for (int ks = 0; ks < ksplit; ++ks)
                sacc += syrk[((size_t)ks * npairs + pidx) * SYRK_T * SYRK_T + ia * SYRK_T + ib];
            v += sacc;
        }
    }
    st[sl.H + e] = v;
}

hipError_t launch_assemble(double* state, StateLayout sl, RecLayout rl, const double* red, const double* syrk,
                           int ksplit, int ntile, int have_syrk, hipStream_t s) {
    const int n = sl.n1 * sl.n1;
    hipLaunchKernelGGL(assemble_kernel, dim3((n + 255) / 256), dim3(256), 0, s, state, sl, rl, red, syrk, ksplit,
                       ntile, have_syrk);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cholesky solve of H y = b in one workgroup (FP64).  The matrix is held in
// LDS when it fits (n <= 143 on gfx950), otherwise it is factorized in
// place in global memory.
// ---------------------------------------------------------------------------

// Cholesky factorization M = L L^T in place (lower triangle, row-major n x n,
// M in LDS or global memory), blocked right-looking with panels of CB
// columns: wave 0 factors the CB x CB diagonal block (lanes own rows, no
// block barrier), all threads then solve the panel below it row by row, and
// update the trailing lower triangle in a 2-D thread layout.  Three block
// barriers per panel instead of two per column.  rdiag receives 1 / L_jj.
// Then the two triangular solves for b by wave 0 alone: lane l owns rows l,
// l + 64, ...; each step broadcasts the new unknown with a lane shuffle.
// Returns -1 if a pivot is not positive.
constexpr int CB = 16;

template <int MAXR>
__device__ int chol_solve_block(int n, double* M, double* b, double* rdiag) {
    __shared__ int bad;
    const int tid = threadIdx.x, nth = blockDim.x;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j0 = 0; j0 < n; j0 += CB) {
        const int nb = min(CB, n - j0);
        // (a) diagonal block by wave 0: lane r < nb owns row j0 + r
        if (tid < WAVE) {
            const int r = tid;
            for (int c = 0; c < nb; ++c) {
                const int jc = j0 + c;
                double ajj = M[jc * n + jc];
                // every lane reads the pivot after the owner's last update:
                // the wave executes in lockstep, LDS/global order within a wave
                const bool ok = ajj > 0.0;
                if (!ok) {
                    if (r == 0) bad = 1;
                    break;
                }
                const double ljj = sqrt(ajj);
                const double rl = 1.0 / ljj;
                if (r == c) {
                    M[jc * n + jc] = ljj;
                    rdiag[jc] = rl;
                }
                if (r > c && r < nb) M[(j0 + r) * n + jc] *= rl;
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (r > c && r < nb) {
                    const double lrc = M[(j0 + r) * n + jc];
                    for (int k = c + 1; k <= r; ++k) M[(j0 + r) * n + j0 + k] -= lrc * M[(j0 + k) * n + jc];
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
        }
        __syncthreads();
        if (bad) return -1;
        // (b) panel below: row i solves L_ib L_bb^T = A_ib (forward in the block)
        for (int i = j0 + nb + tid; i < n; i += nth) {
            for (int c = 0; c < nb; ++c) {
                double v = M[i * n + j0 + c];
                for (int k = 0; k < c; ++k) v -= M[i * n + j0 + k] * M[(j0 + c) * n + j0 + k];
                M[i * n + j0 + c] = v * rdiag[j0 + c];
            }
        }
        __syncthreads();
        // (c) trailing lower triangle: A_ik -= sum_c L_ic L_kc
        const int rem = n - j0 - nb;
        if (rem > 0) {
            const int tx = tid & 31, ty = tid >> 5, nty = nth >> 5;
            for (int ii = ty; ii < rem; ii += nty) {
                const int i = j0 + nb + ii;
                double li[CB];
#pragma unroll
                for (int c = 0; c < CB; ++c) li[c] = c < nb ? M[i * n + j0 + c] : 0.0;
                for (int kk = tx; kk <= ii; kk += 32) {
                    const int k = j0 + nb + kk;
                    double acc = 0.0;
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        if (c < nb) acc += li[c] * M[k * n + j0 + c];
                    M[i * n + k] -= acc;
                }
            }
        }
        __syncthreads();
    }
    if (tid < WAVE) {
        const int lane = tid;
        double bv[MAXR];
#pragma unroll
        for (int r = 0; r < MAXR; ++r) {
            const int row = lane + r * WAVE;
            bv[r] = row < n ? b[row] : 0.0;
        }
        // forward: L y = b
        for (int j = 0; j < n; ++j) {
            const int owner = j & (WAVE - 1), slot = j / WAVE;
            double mine = 0.0;
#pragma unroll
            for (int r = 0; r < MAXR; ++r)
                if (r == slot) mine = bv[r];
            const double yj = __shfl(mine * rdiag[j], owner, WAVE);
#pragma unroll
            for (int r = 0; r < MAXR; ++r) {
                const int row = lane + r * WAVE;
                if (row == j) bv[r] = yj;
                else if (row > j && row < n) bv[r] -= M[row * n + j] * yj;
            }
        }
        // backward: L^T x = y
        for (int i = n - 1; i >= 0; --i) {
            const int owner = i & (WAVE - 1), slot = i / WAVE;
            double mine = 0.0;
#pragma unroll
            for (int r = 0; r < MAXR; ++r)
                if (r == slot) mine = bv[r];
            const double xi = __shfl(mine * rdiag[i], owner, WAVE);
#pragma unroll
            for (int r = 0; r < MAXR; ++r) {
                const int row = lane + r * WAVE;
                if (row == i) bv[r] = xi;
                else if (row < i) bv[r] -= M[i * n + row] * xi;
            }
        }
#pragma unroll
        for (int r = 0; r < MAXR; ++r) {
            const int row = lane + r * WAVE;
            if (row < n) b[row] = bv[r];
        }
    }
    __syncthreads();
    return 0;
}

// Solve with n above the register budget of the wave-level solves: the
// triangular solves by the whole block, column oriented.
__device__ int chol_solve_block_large(int n, double* M, double* b, double* vec) {
    __shared__ int bad;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int tx = tid & 31, ty = tid >> 5, nty = nth >> 5;
    if (tid == 0) bad = 0;
    for (int e = tid; e < n; e += nth) vec[e] = b[e];
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double ajj = M[j * n + j];
        if (!(ajj > 0.0)) {
            if (tid == 0) bad = 1;
            __syncthreads();
            break;
        }
        const double ljj = sqrt(ajj);
        for (int i = j + 1 + tid; i < n; i += nth) M[i * n + j] /= ljj;
        __syncthreads();
        if (tid == 0) M[j * n + j] = ljj;
        for (int ii = j + 1 + ty; ii < n; ii += nty) {
            const double lij = M[ii * n + j];
            for (int kk = j + 1 + tx; kk <= ii; kk += 32) M[ii * n + kk] -= lij * M[kk * n + j];
        }
        __syncthreads();
    }
    if (bad) return -1;
    for (int j = 0; j < n; ++j) {
        const double yj = vec[j] / M[j * n + j];
        __syncthreads();
        if (tid == 0) vec[j] = yj;
        for (int i = j + 1 + tid; i < n; i += nth) vec[i] -= M[i * n + j] * yj;
        __syncthreads();
    }
    for (int i = n - 1; i >= 0; --i) {
        const double xi = vec[i] / M[i * n + i];
        __syncthreads();
        if (tid == 0) vec[i] = xi;
        for (int k = tid; k < i; k += nth) vec[k] -= M[i * n + k] * xi;
        __syncthreads();
    }
    for (int e = tid; e < n; e += nth) b[e] = vec[e];
    __syncthreads();
    return 0;
}

// n <= 192: wave-level triangular solves with 3 rows per lane
constexpr int CHOL_WAVE_MAX_N = 192;

// vec: scratch of at least n doubles (LDS preferred)
__device__ int chol_solve_any(int n, double* M, double* b, double* vec) {
    if (n <= CHOL_WAVE_MAX_N) return chol_solve_block<3>(n, M, b, vec);
    return chol_solve_block_large(n, M, b, vec);
}

// Kernels that take more than 64 KiB of dynamic LDS opt in once per size.
static hipError_t ensure_dynamic_lds(const void* fn, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

constexpr int CHOL_LDS_MAX_N = 140;  // 140^2 doubles + vectors < 160 KiB
constexpr int CTRL_THREADS = 1024;
// the control kernel also keeps CTRL_THREADS doubles of scratch in LDS
constexpr int CTRL_CHOL_LDS_MAX_N = 136;

__global__ __launch_bounds__(CTRL_THREADS) void chol_solve_kernel(int n, double* A, double* b, int* info) {
    extern __shared__ double sm[];
    int rc;
    if (n <= CHOL_LDS_MAX_N) {
        double* M = sm + n;
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[e] = A[e];
        __syncthreads();
        rc = chol_solve_any(n, M, b, sm);
    } else {
        rc = chol_solve_any(n, A, b, sm);
    }
    if (threadIdx.x == 0) *info = rc;
}

hipError_t launch_chol_solve(int n, double* A, double* b, int* info, hipStream_t s) {
    size_t lds = sizeof(double) * (size_t)(n <= CHOL_LDS_MAX_N ? n * n + n : n);
    hipError_t ea = ensure_dynamic_lds((const void*)chol_solve_kernel, lds);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL(chol_solve_kernel, dim3(1), dim3(CTRL_THREADS), lds, s, n, A, b, info);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Control step of the device-resident ripALM / semismooth-Newton loop.
// One workgroup.  Reads the reduced record of the pass that just ran and
// decides what the next pass computes (see the state machine in the host
// solver).  Writes S_MODE = PM_DONE when the run ends.
// ---------------------------------------------------------------------------

__device__ double block_sum(double v, double* scratch) {
    __syncthreads();
    scratch[threadIdx.x] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) scratch[threadIdx.x] += scratch[threadIdx.x + o];
        __syncthreads();
    }
    const double r = scratch[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(CTRL_THREADS) void control_kernel(double* st, StateLayout sl, RecLayout rl,
                                                               const double* red, int* flag) {
    extern __shared__ double sm[];
    double* scratch = sm;                                        // max(CTRL_THREADS, n1)
    double* lmat = sm + (CTRL_THREADS > sl.n1 ? CTRL_THREADS : sl.n1);  // Cholesky matrix when it fits
    __shared__ int s_next;                   // 0 = continue to EVAL_AT_BASE, 1 = return
    __shared__ double s_eta;
    const int mode = (int)st[S_MODE];
    if (mode == PM_DONE) return;
    const int n1 = sl.n1, d = n1 - 1;
    const double L = st[S_L];
    const double sigma = st[S_SIGMA];
    const double tau = st[S_TAU];
    const double eps = st[S_EPS];
    double* xb = st + sl.xb;
    double* dir = st + sl.dir;
    double* xbar = st + sl.xbar;
    double* ab = st + sl.ab;
    double* gb = st + sl.gb;
    double* H = st + sl.H;
    if (threadIdx.x == 0) s_next = 0;
    __syncthreads();

    if (threadIdx.x == 0) {
        st[S_NPASS] += 1.0;
        st[S_BYTES] += red[rl.bytes];
        st[S_SUMK] += red[rl.nm];
        st[S_MAXK] = fmax(st[S_MAXK], red[rl.nm]);
        if (st[S_VERBOSE] >= 2.0)
            printf("[meb] pass %d mode %d K %.0f NI %.0f have_dir %d\n", (int)st[S_NPASS], mode, red[rl.nm],
                   red[rl.ni], (int)st[S_HAVE_DIR]);
    }

    if (mode == PM_MULT) {
        // KKT_max at x_j with the updated multipliers (Section 5), lengths / L
        double pv = 0.0;
        for (int k = threadIdx.x; k < d; k += blockDim.x) pv += red[rl.kv + k] * red[rl.kv + k];
        const double nsv = sqrt(block_sum(pv, scratch));
        if (threadIdx.x == 0) {
            const double p0 = fabs(1.0 - red[rl.ku]);
            const double p2 = red[rl.kmax + 0] / L, p3 = red[rl.kmax + 1], p4 = red[rl.kmax + 2] / L;
            const double kkt = fmax(fmax(fmax(p0, nsv), fmax(p2, p3)), p4);
            st[S_KKT] = kkt;
            st[S_KKT_P0] = p0;
            st[S_KKT_P1] = nsv;
            st[S_KKT_P2] = p2;
            st[S_KKT_P3] = p3;
            st[S_KKT_P4] = p4;
            st[S_K] += 1.0;
            int done = 0;
            if (kkt <= st[S_TOL]) {
                st[S_STATUS] = 1.0;
                done = 1;
            } else {
                if (kkt < 0.5 * st[S_BEST_KKT]) {
                    st[S_BEST_KKT] = kkt;
                    st[S_STALL] = 0.0;
                } else {
                    st[S_STALL] += 1.0;
                }
                if (st[S_K] >= st[S_MAX_OUTER] || st[S_STALL] >= st[S_STALL_OUTER]) {
                    st[S_STATUS] = 2.0;
                    done = 1;
                }
            }
            if (done) {
                st[S_MODE] = (double)PM_DONE;
                s_next = 1;
            }
        }
        __syncthreads();
        // auxiliary update (alpha, beta) <- (alpha, beta) - sigma_k g^{k+1}  (Algorithm 1)
        // in units normalized by L the update reads ab -= (sigma L) g; in raw
        // units that is ab -= sigma L^2 g
        for (int k = threadIdx.x; k < n1; k += blockDim.x) ab[k] -= sigma * L * L * gb[k];
        __syncthreads();
        if (s_next) {
            if (threadIdx.x == 0 && flag) *flag = 1;
            return;
        }
        // next outer iteration: sigma, proximal center
        for (int k = threadIdx.x; k < n1; k += blockDim.x) xbar[k] = xb[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            const double sn = st[S_SIGMA_NEXT];
            st[S_SIGMA] = sn;
            st[S_SIGMA_NEXT] = fmin(sn * st[S_GROWTH], st[S_SIGMA_MAX]);
            st[S_J] = 0.0;
            st[S_HAVE_DIR] = 0.0;
        }
        __syncthreads();
        // fall through: the record's evaluation part is at (x_j, w+, sigma_{k+1})
    } else if (st[S_HAVE_DIR] != 0.0) {
        // single-pass Armijo decision along x_base + eta dir
        const double sg = sigma;
        double pdd = 0.0, pdx = 0.0, pxx = 0.0;
        for (int k = threadIdx.x; k < n1; k += blockDim.x) {
            const double dx = xb[k] - xbar[k];
            pdd += dir[k] * dir[k];
            pdx += dir[k] * dx;
            pxx += dx * dx;
        }
        const double dd = block_sum(pdd, scratch);
        const double dxd = block_sum(pdx, scratch);
        const double xx = block_sum(pxx, scratch);
        if (threadIdx.x == 0) {
            const double z0 = red[rl.trial + NT - 1];
            const double psi0 = xb[0] + 0.5 * sg * z0 - red[rl.ww] / (2.0 * sg) + tau / (2.0 * sg) * xx;
            const double gd = st[S_GD];
            const double allow = 8.0 * eps * (fabs(psi0) + 1.0);
            int acc = -1;
            for (int l = 0; l < NT - 1; ++l) {
                const double eta = solver_eta(l);
                const double dpsi = eta * dir[0] + 0.5 * sg * (red[rl.trial + l] - z0) +
                                    tau / (2.0 * sg) * (2.0 * eta * dxd + eta * eta * dd);
                if (dpsi <= 1e-4 * eta * gd + allow) {
                    acc = l;
                    break;
                }
            }
            if (acc == 0 && st[S_HSKIP] != 0.0) {
                // full step, but its Hessian contraction was skipped:
                // move there and evaluate again
                s_next = 2;
                s_eta = 1.0;
                st[S_HAVE_DIR] = 0.0;
            } else if (acc == 0) {
                s_next = 0;  // full step: record is at x_base + dir
                st[S_PSI] = psi0;
            } else {
                double eta;
                if (acc > 0) {
                    eta = solver_eta(acc);
                    st[S_HAVE_DIR] = 0.0;
                } else {
                    eta = solver_eta(NT - 2);
                    st[S_LSH] += (double)(NT - 2);
                    if (st[S_LSH] >= st[S_MAX_LS]) {
                        st[S_HAVE_DIR] = 0.0;  // take the smallest step
                    } else {
                        st[S_GD] = gd * eta;  // retry along the shorter direction
                    }
                }
                s_eta = eta;
                s_next = (acc > 0 || st[S_HAVE_DIR] == 0.0) ? 2 : 3;
            }
        }
        __syncthreads();
        if (s_next == 0) {
            for (int k = threadIdx.x; k < n1; k += blockDim.x) xb[k] += dir[k];
            __syncthreads();
            if (threadIdx.x == 0) st[S_HAVE_DIR] = 0.0;
        } else {
            const double eta = s_eta;
            if (s_next == 2) {
                for (int k = threadIdx.x; k < n1; k += blockDim.x) xb[k] += eta * dir[k];
            } else {
                for (int k = threadIdx.x; k < n1; k += blockDim.x) dir[k] *= eta;
            }
            if (threadIdx.x == 0 && flag) *flag = 1;
            return;  // next pass re-evaluates at x_base (mode EVAL)
        }
        __syncthreads();
    }

    // ---- evaluated at x_j = xb: gradient, stopping test, Newton step
    double pgg = 0.0, pag = 0.0, pxx = 0.0;
    for (int k = threadIdx.x; k < n1; k += blockDim.x) {
        const double dx = xb[k] - xbar[k];
        const double sv = (k == 0) ? red[rl.su] : red[rl.sv + k - 1];
        const double g = (k == 0 ? 1.0 : 0.0) - sv + (tau / st[S_SIGMA]) * dx;
        gb[k] = g;
        pgg += g * g;
        pag += (ab[k] - xb[k]) * g;
        pxx += dx * dx;
    }
    const double gg = block_sum(pgg, scratch);
    const double ag = block_sum(pag, scratch);
    const double xx = block_sum(pxx, scratch);
    const double sgm = st[S_SIGMA];
    if (threadIdx.x == 0) {
        st[S_J] += 1.0;
        st[S_NINNER] += 1.0;
        // relative-type stopping test of Algorithm 1 in normalized units
        const double sN = sgm * L, tN = tau * L * L;
        const double lhs = 2.0 * sN * fabs(ag / L) + sN * sN * gg;
        const double rhs = st[S_RHO] * (red[rl.dm] + tN * xx / (L * L));
        const double floor_g = 8.0 * eps * (1.0 + sgm * red[rl.rs]);
        const bool stop = (lhs <= rhs) || (sqrt(gg) <= floor_g) || (st[S_J] >= st[S_MAX_INNER]);
        if (stop) {
            st[S_MODE] = (double)PM_MULT;
            st[S_HAVE_DIR] = 0.0;
            s_next = 1;
        } else {
            s_next = 0;
        }
    }
    __syncthreads();
    if (s_next) {
        if (threadIdx.x == 0 && flag) *flag = 1;
        return;
    }
    // Newton direction: H dir = -g, H assembled by assemble_kernel
    for (int k = threadIdx.x; k < n1; k += blockDim.x) dir[k] = -gb[k];
    int rc;
    if (n1 <= CTRL_CHOL_LDS_MAX_N) {
        for (int e = threadIdx.x; e < n1 * n1; e += blockDim.x) lmat[e] = H[e];
        __syncthreads();
        rc = chol_solve_any(n1, lmat, dir, scratch);
    } else {
        __syncthreads();
        rc = chol_solve_any(n1, H, dir, scratch);
    }
    if (rc != 0) {
        if (threadIdx.x == 0) {
            st[S_STATUS] = -1.0;
            st[S_MODE] = (double)PM_DONE;
            if (flag) *flag = 1;
        }
        return;
    }
    double pgd = 0.0;
    for (int k = threadIdx.x; k < n1; k += blockDim.x) pgd += gb[k] * dir[k];
    const double gd = block_sum(pgd, scratch);
    if (threadIdx.x == 0) {
        st[S_GD] = gd;
        st[S_HAVE_DIR] = 1.0;
        st[S_LSH] = 0.0;
        st[S_MODE] = (double)PM_EVAL;
        if (flag) *flag = 1;
    }
}

hipError_t launch_control(double* state, StateLayout sl, RecLayout rl, const double* red, int* flag, hipStream_t s) {
    const int n1 = sl.n1;
    size_t lds = sizeof(double) * (size_t)(CTRL_THREADS > n1 ? CTRL_THREADS : n1);
    if (n1 <= CTRL_CHOL_LDS_MAX_N) lds += sizeof(double) * (size_t)(n1 * n1 + n1);
    hipError_t ea = ensure_dynamic_lds((const void*)control_kernel, lds);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL(control_kernel, dim3(1), dim3(CTRL_THREADS), lds, s, state, sl, rl, red, flag);
    return hipGetLastError();
}

// g and H of a single evaluation (meb_al_eval).
__global__ __launch_bounds__(CTRL_THREADS) void eval_assemble_kernel(RecLayout rl, const double* red,
                                                                     const double* syrk, int ksplit, int ntile,
                                                                     int have_syrk, double sigma, double tau, int d,
                                                                     const double* y, const double* xbar,
                                                                     double* out_g, double* out_H) {
    const int n1 = d + 1;
    if (out_g) {
        for (int k = threadIdx.x; k < n1; k += blockDim.x) {
            const double sv = (k == 0) ? red[rl.su] : red[rl.sv + k - 1];
            out_g[k] = (k == 0 ? 1.0 : 0.0) - sv + (tau / sigma) * (y[k] - xbar[k]);
        }
    }
    if (out_H) assemble_H(d, rl, red, syrk, ksplit, ntile, have_syrk, sigma, tau, out_H);
}

hipError_t launch_eval_assemble(const double* state, StateLayout sl, RecLayout rl, const double* red,
                                const double* syrk_out, int ksplit, int tile, int ntile, int have_syrk, double sigma,
                                double tau, const double* y, const double* xbar, double* out_g, double* out_H,
                                hipStream_t s) {
    (void)state;
    (void)sl;
    (void)tile;
    hipLaunchKernelGGL(eval_assemble_kernel, dim3(1), dim3(CTRL_THREADS), 0, s, rl, red, syrk_out, ksplit, ntile,
                       have_syrk, sigma, tau, rl.d, y, xbar, out_g, out_H);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streaming scans over all balls in FP64 arithmetic: the feasibility check
// (reach_i = r_i + ||c - c_i|| against r), the screening slack, and the
// FP32 preparation.  G lanes per row as in the evaluation pass; each wave
// streams a contiguous range and writes its hits, in ascending order, into
// its own segment; a single-block scan then computes segment offsets and the
// global maximum, and a copy kernel concatenates the segments.
// ---------------------------------------------------------------------------

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_WPB = SCAN_THREADS / WAVE;

ScanCfg scan_config(int64_t m, int d, int num_cu) {
    ScanCfg c;
    c.vec = (d % 2 == 0) ? 2 : 1;
    int need = (d + c.vec * 4 - 1) / (c.vec * 4);
    int G = 1;
    while (G < need && G < 64) G <<= 1;
    c.G = G;
    c.nl = (d + G * c.vec - 1) / (G * c.vec);
    const int bpw = WAVE / G;
    int64_t steps = (m + bpw - 1) / bpw;
    int64_t maxw = (int64_t)num_cu * 8;
    int64_t w = steps < maxw ? steps : maxw;
    if (w < 1) w = 1;
    c.bw = ((steps + w - 1) / w) * bpw;
    int64_t waves = (m + c.bw - 1) / c.bw;
    c.blocks = (int)((waves + SCAN_WPB - 1) / SCAN_WPB);
    c.nwaves = c.blocks * SCAN_WPB;
    return c;
}

// MODE 0: feasibility (hit: reach - r > thr; keeps max reach - r and argmax)
// MODE 1: screening (value r - r_i - ||c - c_i||; hit: value <= thr)
// MODE 2: FP32 preparation (writes float(c_i - x) and float(r_i); keeps max)
template <typename T, int VEC, int MODE>
__global__ __launch_bounds__(SCAN_THREADS) void scan_kernel(const T* C, const T* R, int64_t m, int d,
                                                            const double* xdev, double r, double thr,
                                                            double* slack, float* C32, float* R32, ScanCfg cfg,
                                                            double* wmax, int64_t* warg, int64_t* wcnt,
                                                            int64_t* seg) {
    extern __shared__ double lx[];
    for (int k = threadIdx.x; k < d; k += SCAN_THREADS) lx[k] = xdev ? xdev[k] : 0.0;
    __syncthreads();
    const int G = cfg.G, nl = cfg.nl;
    const int lane = lane_id(), wid = threadIdx.x / WAVE;
    const int64_t gw = (int64_t)blockIdx.x * SCAN_WPB + wid;
    const int gi = lane / G, gl = lane % G, bpw = WAVE / G;
    const int64_t wbeg = gw * cfg.bw, wend = min(m, wbeg + cfg.bw);
    double best = -INFINITY;
    int64_t barg = INT64_MAX;
    int64_t count = 0;
    for (int64_t b0 = wbeg; b0 < wend; b0 += bpw) {
        const int64_t i = b0 + gi;
        const bool act = i < wend;
        double acc = 0.0;
        for (int j = 0; j < nl; ++j) {
            const int base = (j * G + gl) * VEC;
            if (act && base < d) {
                const RowVec<T, VEC> cr = load_vec<T, VEC>(C + i * d + base);
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    const double e = (double)cr.v[q] - lx[base + q];
                    acc += e * e;
                    if (MODE == 2) C32[i * d + base + q] = (float)e;
                }
            }
        }
        const double dist = sqrt(group_sum<double>(acc, G));
        const double ri = (R && act) ? (double)R[i] : 0.0;
        double val;
        bool hit;
        if (MODE == 1) {
            val = r - ri - dist;
            hit = act && val <= thr;
            if (slack && act && gl == 0) slack[i] = val;
        } else {
            val = ri + dist - r;
            hit = (MODE == 0) && act && val > thr;
            if (MODE == 2 && R32 && act && gl == 0) R32[i] = (float)ri;
            if (act && (val > best || (val == best && i < barg))) {
                best = val;
                barg = i;
            }
        }
        if (MODE != 2) {
            const unsigned long long bal = __ballot(hit && gl == 0);
            if (hit && gl == 0) seg[wbeg + count + __popcll(bal & ((1ull << lane) - 1ull))] = i;
            count += __popcll(bal);
        }
    }
    if (MODE != 1) {
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            const double ov = __shfl_xor(best, o, WAVE);
            const int64_t oa = __shfl_xor(barg, o, WAVE);
            if (ov > best || (ov == best && oa < barg)) {
                best = ov;
                barg = oa;
            }
        }
    }
    if (lane == 0) {
        if (wmax) wmax[gw] = best;
        if (warg) warg[gw] = barg;
        if (wcnt) wcnt[gw] = count;
    }
}

// Exclusive prefix of the per-wave counts (into offs), the total, and the
// maximum with the smallest index on ties.  One block of 1024 threads.
__global__ __launch_bounds__(1024) void scan_finalize(const int64_t* wcnt, const double* wmax, const int64_t* warg,
                                                      int nw, int64_t* offs, int64_t* total, double* out_max,
                                                      int64_t* out_arg) {
    __shared__ int64_t sc[1024];
    __shared__ double sm[1024];
    __shared__ int64_t sa[1024];
    const int t = threadIdx.x;
    const int per = (nw + 1023) / 1024;
    const int w0 = t * per, w1 = min(nw, w0 + per);
    int64_t c = 0;
    double bm = -INFINITY;
    int64_t ba = INT64_MAX;
    for (int w = w0; w < w1; ++w) {
        if (wcnt) c += wcnt[w];
        if (wmax && (wmax[w] > bm || (wmax[w] == bm && warg[w] < ba))) {
            bm = wmax[w];
            ba = warg[w];
        }
    }
    sc[t] = c;
    sm[t] = bm;
    sa[t] = ba;
    __syncthreads();
    // inclusive Hillis-Steele scan of the per-thread counts
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t v = t >= o ? sc[t - o] : 0;
        __syncthreads();
        sc[t] += v;
        __syncthreads();
    }
    if (wcnt) {
        int64_t run = t > 0 ? sc[t - 1] : 0;
        for (int w = w0; w < w1; ++w) {
            offs[w] = run;
            run += wcnt[w];
        }
        if (t == 1023 && total) *total = sc[1023];
    }
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o && (sm[t + o] > sm[t] || (sm[t + o] == sm[t] && sa[t + o] < sa[t]))) {
            sm[t] = sm[t + o];
            sa[t] = sa[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (out_max) *out_max = sm[0];
        if (out_arg) *out_arg = sa[0];
    }
}

// Concatenation of the wave segments (one wave per segment).
__global__ __launch_bounds__(256) void scan_copy(const int64_t* seg, const int64_t* wcnt, const int64_t* offs,
                                                 int nw, int64_t bw, int64_t* out, int64_t cap) {
    const int lane = lane_id();
    const int64_t w = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (w >= nw) return;
    const int64_t cnt = wcnt[w], off = offs[w];
    for (int64_t k = lane; k < cnt; k += WAVE) {
        const int64_t pos = off + k;
        if (pos < cap) out[pos] = seg[w * bw + k];
    }
}

template <int MODE>
static hipError_t launch_scan_t(const void* C, const void* R, int64_t m, int d, int dtype, const double* x,
                                double r, double thr, double* slack, float* C32, float* R32, const ScanCfg& c,
                                double* wmax, int64_t* warg, int64_t* wcnt, int64_t* seg, hipStream_t s) {
    const size_t lds = sizeof(double) * d;
    if (dtype == 0) {
        if (c.vec == 2)
            hipLaunchKernelGGL((scan_kernel<double, 2, MODE>), dim3(c.blocks), dim3(SCAN_THREADS), lds, s,
                               (const double*)C, (const double*)R, m, d, x, r, thr, slack, C32, R32, c, wmax, warg,
                               wcnt, seg);
        else
            hipLaunchKernelGGL((scan_kernel<double, 1, MODE>), dim3(c.blocks), dim3(SCAN_THREADS), lds, s,
                               (const double*)C, (const double*)R, m, d, x, r, thr, slack, C32, R32, c, wmax, warg,
                               wcnt, seg);
    } else {
        if (c.vec == 2)
            hipLaunchKernelGGL((scan_kernel<float, 2, MODE>), dim3(c.blocks), dim3(SCAN_THREADS), lds, s,
                               (const float*)C, (const float*)R, m, d, x, r, thr, slack, C32, R32, c, wmax, warg,
                               wcnt, seg);
        else
            hipLaunchKernelGGL((scan_kernel<float, 1, MODE>), dim3(c.blocks), dim3(SCAN_THREADS), lds, s,
                               (const float*)C, (const float*)R, m, d, x, r, thr, slack, C32, R32, c, wmax, warg,
                               wcnt, seg);
    }
    return hipGetLastError();
}

hipError_t launch_scan(int mode, const void* C, const void* R, int64_t m, int d, int dtype, const double* x,
                       double r, double thr, double* slack, float* C32, float* R32, const ScanCfg& c, double* wmax,
                       int64_t* warg, int64_t* wcnt, int64_t* seg, hipStream_t s) {
    if (mode == 0) return launch_scan_t<0>(C, R, m, d, dtype, x, r, thr, slack, C32, R32, c, wmax, warg, wcnt, seg, s);
    if (mode == 1) return launch_scan_t<1>(C, R, m, d, dtype, x, r, thr, slack, C32, R32, c, wmax, warg, wcnt, seg, s);
    return launch_scan_t<2>(C, R, m, d, 0, x, r, thr, slack, C32, R32, c, wmax, warg, wcnt, seg, s);
}

hipError_t launch_scan_finalize(const int64_t* wcnt, const double* wmax, const int64_t* warg, int nw, int64_t* offs,
                                int64_t* total, double* out_max, int64_t* out_arg, hipStream_t s) {
    hipLaunchKernelGGL(scan_finalize, dim3(1), dim3(1024), 0, s, wcnt, wmax, warg, nw, offs, total, out_max,
                       out_arg);
    return hipGetLastError();
}

hipError_t launch_scan_copy(const int64_t* seg, const int64_t* wcnt, const int64_t* offs, int nw, int64_t bw,
                            int64_t* out, int64_t cap, hipStream_t s) {
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(scan_copy, dim3((nw + 3) / 4), dim3(256), 0, s, seg, wcnt, offs, nw, bw, out, cap);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gather of retained rows into a compact FP64 problem (and its warm-start
// multipliers), and scatter of the reduced multipliers back to full size.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(const T* C, const T* R, const T* U, const T* V,
                                                     const int64_t* idx, int64_t n, int d, double* Co, double* Ro,
                                                     double* Uo, double* Vo) {
    const int64_t row = (int64_t)blockIdx.x;
    if (row >= n) return;
    const int64_t i = idx[row];
    const T ui = U ? U[i] : T(0);
    for (int k = threadIdx.x; k < d; k += 256) {
        if (Co) Co[row * d + k] = (double)C[i * d + k];
        if (Vo) Vo[row * d + k] = (V && ui != T(0)) ? (double)V[i * d + k] : 0.0;
    }
    if (threadIdx.x == 0) {
        if (Ro) Ro[row] = R ? (double)R[i] : 0.0;
        if (Uo) Uo[row] = (double)ui;
    }
}

hipError_t launch_gather(const void* C, const void* R, const void* U, const void* V, int src_dtype,
                         const int64_t* idx, int64_t n, int d, double* C_out, double* R_out, double* U_out,
                         double* V_out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (src_dtype == 0)
        hipLaunchKernelGGL(gather_kernel<double>, dim3((unsigned)n), dim3(256), 0, s, (const double*)C,
                           (const double*)R, (const double*)U, (const double*)V, idx, n, d, C_out, R_out, U_out,
                           V_out);
    else
        hipLaunchKernelGGL(gather_kernel<float>, dim3((unsigned)n), dim3(256), 0, s, (const float*)C, (const float*)R,
                           (const float*)U, (const float*)V, idx, n, d, C_out, R_out, U_out, V_out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void scatter_kernel(const double* Ur, const double* Vr, const int64_t* idx,
                                                      int64_t n, int d, double* Uo, double* Vo) {
    const int64_t row = blockIdx.x;
    if (row >= n) return;
    const int64_t i = idx[row];
    const double u = Ur[row];
    if (threadIdx.x == 0 && Uo) Uo[i] = u;
    if (Vo)
        for (int k = threadIdx.x; k < d; k += 256) Vo[i * d + k] = (u != 0.0) ? Vr[row * d + k] : 0.0;
}

hipError_t launch_scatter_mult(const double* Ured, const double* Vred, const int64_t* idx, int64_t n, int d,
                               double* U_out, double* V_out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)n), dim3(256), 0, s, Ured, Vred, idx, n, d, U_out, V_out);
    return hipGetLastError();
}

// Dense FP64 copy of multipliers whose V rows are meaningful only where U != 0.
template <typename T>
__global__ __launch_bounds__(256) void dense_mult_kernel(const T* U, const T* V, int64_t m, int d, double* Uo,
                                                         double* Vo) {
    const int64_t total = m * (int64_t)d;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / d;
        const T u = U[i];
        if (Vo) Vo[e] = (u != T(0)) ? (double)V[e] : 0.0;
        if (Uo && (e % d) == 0) Uo[i] = (double)u;
    }
}

hipError_t launch_dense_mult(const void* U, const void* V, int dtype, int64_t m, int d, double* U_out, double* V_out,
                             hipStream_t s) {
    const int64_t total = m * (int64_t)d;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (dtype == 0)
        hipLaunchKernelGGL(dense_mult_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, (const double*)U,
                           (const double*)V, m, d, U_out, V_out);
    else
        hipLaunchKernelGGL(dense_mult_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, (const float*)U,
                           (const float*)V, m, d, U_out, V_out);
    return hipGetLastError();
}

__global__ void fill_f64_kernel(double* p, double v, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) p[e] = v;
}

hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

__global__ void fill_zero_kernel(uint32_t* p, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) p[e] = 0u;
}

hipError_t launch_fill_bytes_zero(void* p, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, n);
    return hipGetLastError();
}

}  // namespace meb
