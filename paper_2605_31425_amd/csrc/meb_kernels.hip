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

template <typename T, int VEC, int NLMAX>
__global__ __launch_bounds__(PASS_THREADS) void pass_kernel(PassArgs a, PassConfig cfg) {
    extern __shared__ double lds[];
    const double* st = a.state;
    const int mode = a.force_mode >= 0 ? a.force_mode : (int)st[S_MODE];
    if (mode == PM_DONE) return;
    const int d = a.d;
    const int G = cfg.G;
    const int nl = cfg.nl;
    const StateLayout sl = a.sl;
    const RecLayout rl = a.rl;

    const bool have_dir = (mode == PM_EVAL) && st[S_HAVE_DIR] != 0.0;
    const bool is_mult = (mode == PM_MULT);
    const bool want_kkt = is_mult || a.want_kkt;

    // Current point y = x_base + dir and the direction, in LDS (FP64).
    double* l_c = lds;
    double* l_dc = lds + d;
    double* l_red = lds + 2 * d;  // PASS_THREADS doubles
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

    // per-lane accumulators (FP64)
    double acc_su = 0, acc_z1 = 0, acc_ni = 0, acc_nm = 0, acc_sg = 0, acc_dm = 0, acc_rs = 0, acc_ww = 0, acc_ku = 0;
    double mx_p = 0, mx_d = 0, mx_c = 0;
    double tacc[NT];
#pragma unroll
    for (int r = 0; r < NT; ++r) tacc[r] = 0.0;
    double sv[NLMAX][VEC], sw[NLMAX][VEC], kv[NLMAX][VEC];
#pragma unroll
    for (int j = 0; j < NLMAX; ++j)
#pragma unroll
        for (int q = 0; q < VEC; ++q) sv[j][q] = sw[j][q] = kv[j][q] = 0.0;

    int32_t mid_count = 0;
    int32_t* mid_idx = a.mid_idx ? a.mid_idx + gw * cfg.bw : nullptr;
    double* mid_coef = a.mid_idx ? a.mid_coef + gw * cfg.bw : nullptr;

    for (int64_t b0 = wbeg; b0 < wend; b0 += bpw) {
        const int64_t i = b0 + gi;
        const bool active = i < wend;
        const T ri = (R && active) ? R[i] : T(0);
        const T ui = (U && active) ? U[i] : T(0);
        const bool hasv = V && (ui != T(0));
        T e[NLMAX][VEC], vv[NLMAX][VEC], s[NLMAX][VEC];
        T nn = 0, q = 0, ee = 0, es = 0;
#pragma unroll
        for (int j = 0; j < NLMAX; ++j) {
            const int base = (j * G + gl) * VEC;
            const bool ok = active && (j < nl) && (base < d);
            RowVec<T, VEC> cr, vr;
#pragma unroll
            for (int qq = 0; qq < VEC; ++qq) cr.v[qq] = vr.v[qq] = T(0);
            if (ok) {
                cr = load_vec<T, VEC>(C + i * d + base);
                if (hasv) vr = load_vec<T, VEC>(V + i * d + base);
            }
#pragma unroll
            for (int qq = 0; qq < VEC; ++qq) {
                const T ck = ok ? (T)l_c[base + qq] : T(0);
                e[j][qq] = ok ? cr.v[qq] - ck : T(0);
                vv[j][qq] = vr.v[qq];
                s[j][qq] = e[j][qq] + vr.v[qq] * inv_a;
                nn += s[j][qq] * s[j][qq];
                if (have_dir) q += s[j][qq] * (ok ? (T)l_dc[base + qq] : T(0));
                if (want_kkt) {
                    ee += e[j][qq] * e[j][qq];
                    es += e[j][qq] * s[j][qq];
                }
            }
        }
        nn = group_sum<T>(nn, G);
        if (have_dir) q = group_sum<T>(q, G);
        if (want_kkt) {
            ee = group_sum<T>(ee, G);
            es = group_sum<T>(es, G);
        }
        const T t = ri - r1 + ui * inv_a;
        BallProj<T> pa = project<T>(t, nn, sig_a);
        if (!active) pa.cs = 1, pa.up = T(0), pa.gam = T(0), pa.Z = T(0);

        // Quantities that the evaluation accumulates: point z, multipliers in use.
        T te = t, nne = nn, ue = ui;
        BallProj<T> pe = pa;
        T sig_e = sig_a;

        if (want_kkt) {
            // updated multipliers w+ = sigma Pi(z) at y and the KKT terms there
            const T un = pa.up;
            if (leader && active) {
                acc_ku += (double)un;
                const T tp = r1 - ri;
                mx_p = fmax(mx_p, (double)cone_dist<T>(tp, tsqrt<T>(ee)));
                mx_d = fmax(mx_d, (double)cone_dist<T>(un, pa.gam * pa.n));
                mx_c = fmax(mx_c, fabs((double)(tp * un - pa.gam * es)));
                if (Uo) Uo[i] = un;
            }
#pragma unroll
            for (int j = 0; j < NLMAX; ++j) {
                const int base = (j * G + gl) * VEC;
                const bool ok = active && (j < nl) && (base < d);
                RowVec<T, VEC> vn;
#pragma unroll
                for (int qq = 0; qq < VEC; ++qq) {
                    vn.v[qq] = pa.gam * s[j][qq];
                    kv[j][qq] += (double)vn.v[qq];
                }
                if (ok && Vo && (un != T(0) || a.dense_vout)) store_vec<T, VEC>(Vo + i * d + base, vn);
                if (is_mult) {
                    // the next subproblem uses w+ and sigma_{k+1}
#pragma unroll
                    for (int qq = 0; qq < VEC; ++qq) vv[j][qq] = vn.v[qq];
                }
            }
            if (is_mult) {
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

        // ---- evaluation accumulators at (y, multipliers ue/vv, sigma sig_e)
        if (leader && active) {
            acc_su += (double)pe.up;
            acc_z1 += (double)pe.Z;
            const double du = (double)pe.up - (double)ue;
            acc_dm += du * du;
            acc_ww += (double)ue * (double)ue;
            if (pe.cs != 1) acc_rs += fabs((double)te) + (double)pe.n;
            if (pe.cs == 0) acc_ni += 1.0;
            if (pe.cs == 2) {
                acc_nm += 1.0;
                acc_sg += (double)pe.gam;
            }
        }
        const T inv_n = (pe.cs == 2) ? T(1) / pe.n : T(0);
#pragma unroll
        for (int j = 0; j < NLMAX; ++j)
#pragma unroll
            for (int qq = 0; qq < VEC; ++qq) {
                const double sk = (double)s[j][qq];
                const double vk = (double)vv[j][qq];
                const double vp = (double)(pe.gam * s[j][qq]);
                sv[j][qq] += vp;
                sw[j][qq] += (double)(s[j][qq] * inv_n);
                acc_dm += (vp - vk) * (vp - vk);
                acc_ww += vk * vk;
                (void)sk;
            }
        // Armijo trials along the segment x_base + eta dir: lane gl takes
        // trials gl, gl + G, ...
        if (active) {
#pragma unroll
            for (int r = 0; r < NT; ++r) {
                const int l = r * G + gl;
                if (r * G >= NT) break;
                if (l < NT) {
                    T Zl;
                    if (have_dir) {
                        const T am = T(1) - (T)a.etas[l];
                        const T tl = te + am * dirr;
                        T n2 = nne + T(2) * am * q + am * am * dc2;
                        n2 = n2 > T(0) ? n2 : T(0);
                        Zl = project<T>(tl, n2, sig_e).Z;
                    } else {
                        Zl = pe.Z;
                    }
                    tacc[r] += (double)Zl;
                }
            }
        }
        // mid list for the rank-one Hessian contraction:
        // coef_i = -sigma t_i / (2 n_i^3) multiplies s_i s_i^T
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

    // ---- wave-level reduction and the per-wave record
    double* rec = a.rec + gw * rl.len;
    acc_su = wave_sum(acc_su);
    acc_z1 = wave_sum(acc_z1);
    acc_ni = wave_sum(acc_ni);
    acc_nm = wave_sum(acc_nm);
    acc_sg = wave_sum(acc_sg);
    acc_dm = wave_sum(acc_dm);
    acc_rs = wave_sum(acc_rs);
    acc_ww = wave_sum(acc_ww);
    acc_ku = wave_sum(acc_ku);
    mx_p = wave_max(mx_p);
    mx_d = wave_max(mx_d);
    mx_c = wave_max(mx_c);
#pragma unroll
    for (int r = 0; r < NT; ++r) tacc[r] = cross_group_sum(tacc[r], G);
#pragma unroll
    for (int j = 0; j < NLMAX; ++j)
#pragma unroll
        for (int qq = 0; qq < VEC; ++qq) {
            sv[j][qq] = cross_group_sum(sv[j][qq], G);
            sw[j][qq] = cross_group_sum(sw[j][qq], G);
            kv[j][qq] = cross_group_sum(kv[j][qq], G);
        }
    if (lane == 0) {
        rec[rl.su] = acc_su;
        rec[rl.z1] = acc_z1;
        rec[rl.ni] = acc_ni;
        rec[rl.nm] = acc_nm;
        rec[rl.sg] = acc_sg;
        rec[rl.dm] = acc_dm;
        rec[rl.rs] = acc_rs;
        rec[rl.ww] = acc_ww;
        rec[rl.ku] = acc_ku;
        rec[rl.kmax + 0] = mx_p;
        rec[rl.kmax + 1] = mx_d;
        rec[rl.kmax + 2] = mx_c;
        if (a.mid_cnt) a.mid_cnt[gw] = mid_count;
    }
    if (lane < G) {
#pragma unroll
        for (int r = 0; r < NT; ++r) {
            const int l = r * G + lane;
            if (r * G >= NT) break;
            if (l < NT) rec[rl.trial + l] = tacc[r];
        }
#pragma unroll
        for (int j = 0; j < NLMAX; ++j) {
            const int base = (j * G + lane) * VEC;
            if (j < nl && base < d) {
#pragma unroll
                for (int qq = 0; qq < VEC; ++qq) {
                    rec[rl.sv + base + qq] = sv[j][qq];
                    rec[rl.sw + base + qq] = sw[j][qq];
                    rec[rl.kv + base + qq] = kv[j][qq];
                }
            }
        }
    }
}

PassConfig choose_pass_config(int64_t m, int d, int dtype, int num_cu) {
    PassConfig c;
    c.vec = (d % 2 == 0) ? 2 : 1;
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

template <typename T, int VEC, int NLMAX>
static hipError_t launch_pass_t(const PassArgs& a, const PassConfig& cfg, hipStream_t s) {
    size_t lds = sizeof(double) * (2 * (size_t)a.d + PASS_THREADS);
    hipLaunchKernelGGL((pass_kernel<T, VEC, NLMAX>), dim3(cfg.blocks), dim3(PASS_THREADS), lds, s, a, cfg);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_pass_T(const PassArgs& a, const PassConfig& cfg, hipStream_t s) {
    if (cfg.vec == 2) {
        if (cfg.nlmax == 4) return launch_pass_t<T, 2, 4>(a, cfg, s);
        if (cfg.nlmax == 8) return launch_pass_t<T, 2, 8>(a, cfg, s);
        return launch_pass_t<T, 2, 16>(a, cfg, s);
    }
    if (cfg.nlmax == 4) return launch_pass_t<T, 1, 4>(a, cfg, s);
    if (cfg.nlmax == 8) return launch_pass_t<T, 1, 8>(a, cfg, s);
    return launch_pass_t<T, 1, 16>(a, cfg, s);
}

hipError_t launch_pass(const PassArgs& a, const PassConfig& cfg, hipStream_t s) {
    if (a.dtype == 0) return launch_pass_T<double>(a, cfg, s);
    return launch_pass_T<float>(a, cfg, s);
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of per-wave records: out[e] = sum_w rec[w][e]
// (maximum for the three KKT maxima).  Two stages: slices of records, then
// the slices; both in ascending order.
// ---------------------------------------------------------------------------

constexpr int RED_SLICE = 32;

__global__ __launch_bounds__(256) void reduce_stage1(const double* rec, int nrec, int len, int max_lo, int max_hi,
                                                     double* part) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int sl = blockIdx.y;
    const int per = (nrec + gridDim.y - 1) / gridDim.y;
    const int w0 = sl * per, w1 = min(nrec, w0 + per);
    if (e >= len) return;
    const bool ismax = (e >= max_lo && e < max_hi);
    double acc = ismax ? 0.0 : 0.0;
    for (int w = w0; w < w1; ++w) {
        const double v = rec[(size_t)w * len + e];
        acc = ismax ? fmax(acc, v) : acc + v;
    }
    part[(size_t)sl * len + e] = acc;
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

hipError_t launch_reduce_records(const double* rec, int nrec, int len, double* out, hipStream_t s) {
    // `out` must have room for (RED_SLICE + 1) * len doubles: the slice
    // partials live after the result.  The three maxima sit at a fixed
    // offset ahead of the d-dependent vector parts of the record.
    const RecLayout rl = RecLayout::make(0);
    const int max_lo = rl.kmax, max_hi = rl.kmax + 3;
    int nslice = nrec < RED_SLICE ? nrec : RED_SLICE;
    double* part = out + len;
    dim3 g1((len + 255) / 256, nslice);
    hipLaunchKernelGGL(reduce_stage1, g1, dim3(256), 0, s, rec, nrec, len, max_lo, max_hi, part);
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
constexpr int SYRK_KB = 32;  // mid balls staged per step

int syrk_tile() { return SYRK_T; }

int syrk_ksplit(int d, int nwaves) {
    int nt = (d + SYRK_T - 1) / SYRK_T;
    int pairs = nt * (nt + 1) / 2;
    int ks = 512 / pairs;
    if (ks < 1) ks = 1;
    if (ks > nwaves) ks = nwaves;
    return ks;
}

template <typename T>
__global__ __launch_bounds__(256) void syrk_kernel(SyrkArgs a) {
    __shared__ double sI[SYRK_KB][SYRK_T + 1];
    __shared__ double sJ[SYRK_KB][SYRK_T + 1];
    __shared__ double cf[SYRK_KB];
    __shared__ int32_t ix[SYRK_KB];
    const double* st = a.state;
    const int mode = (int)st[S_MODE];
    if (mode == PM_DONE) return;
    const int d = a.d;
    const StateLayout sl = a.sl;
    const bool have_dir = (mode == PM_EVAL) && st[S_HAVE_DIR] != 0.0;
    const double sig = (mode == PM_MULT) ? st[S_SIGMA_NEXT] : st[S_SIGMA];
    const T inv = (T)(1.0 / sig);
    // tile pair from blockIdx.x (upper triangle, row-major)
    int p = blockIdx.x, I = 0;
    while (p >= a.ntile - I) {
        p -= a.ntile - I;
        ++I;
    }
    const int J = I + p;
    const int ks = blockIdx.y;
    const int per = (a.nwaves + a.ksplit - 1) / a.ksplit;
    const int w0 = ks * per, w1 = min(a.nwaves, w0 + per);
    const T* C = static_cast<const T*>(a.C);
    const T* V = static_cast<const T*>(a.V);
    const T* U = static_cast<const T*>(a.U);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[2][2] = {{0, 0}, {0, 0}};
    for (int w = w0; w < w1; ++w) {
        const int cnt = a.mid_cnt[w];
        const int32_t* idx = a.mid_idx + (int64_t)w * a.bw;
        const double* coef = a.mid_coef + (int64_t)w * a.bw;
        for (int k0 = 0; k0 < cnt; k0 += SYRK_KB) {
            const int nk = min(SYRK_KB, cnt - k0);
            __syncthreads();
            if (threadIdx.x < SYRK_KB) {
                ix[threadIdx.x] = threadIdx.x < nk ? idx[k0 + threadIdx.x] : 0;
                cf[threadIdx.x] = threadIdx.x < nk ? coef[k0 + threadIdx.x] : 0.0;
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
    }
    const int npairs = gridDim.x;
    double* out = a.out + ((size_t)ks * npairs + blockIdx.x) * SYRK_T * SYRK_T;
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

// ---------------------------------------------------------------------------
// Cholesky solve of H y = b in one workgroup (FP64).  The matrix is held in
// LDS when it fits (n <= 143 on gfx950), otherwise it is factorized in
// place in global memory.
// ---------------------------------------------------------------------------

template <bool IN_LDS>
__device__ int chol_solve_block(int n, double* A, double* b, double* lds_mat, double* lds_vec) {
    double* M = IN_LDS ? lds_mat : A;
    if (IN_LDS) {
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[e] = A[e];
    }
    for (int e = threadIdx.x; e < n; e += blockDim.x) lds_vec[e] = b[e];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    // right-looking factorization, lower triangle: M = L L^T
    for (int j = 0; j < n; ++j) {
        const double ajj = M[j * n + j];
        if (!(ajj > 0.0)) {
            if (threadIdx.x == 0) bad = 1;
            __syncthreads();
            break;
        }
        const double ljj = sqrt(ajj);
        __syncthreads();
        for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) M[i * n + j] /= ljj;
        __syncthreads();
        if (threadIdx.x == 0) M[j * n + j] = ljj;
        // trailing update of the lower triangle
        const int rem = n - j - 1;
        for (int e = threadIdx.x; e < rem * rem; e += blockDim.x) {
            const int ii = j + 1 + e / rem, kk = j + 1 + e % rem;
            if (kk <= ii) M[ii * n + kk] -= M[ii * n + j] * M[kk * n + j];
        }
        __syncthreads();
    }
    if (bad) return -1;
    // forward: L y = b (column oriented)
    for (int j = 0; j < n; ++j) {
        __syncthreads();
        const double yj = lds_vec[j] / M[j * n + j];
        __syncthreads();
        if (threadIdx.x == 0) lds_vec[j] = yj;
        for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) lds_vec[i] -= M[i * n + j] * yj;
    }
    __syncthreads();
    // backward: L^T x = y (row i of L^T is column i of L)
    for (int i = n - 1; i >= 0; --i) {
        __syncthreads();
        const double xi = lds_vec[i] / M[i * n + i];
        __syncthreads();
        if (threadIdx.x == 0) lds_vec[i] = xi;
        for (int k = threadIdx.x; k < i; k += blockDim.x) lds_vec[k] -= M[i * n + k] * xi;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += blockDim.x) b[e] = lds_vec[e];
    __syncthreads();
    return 0;
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
    if (n <= CHOL_LDS_MAX_N)
        rc = chol_solve_block<true>(n, A, b, sm + n, sm);
    else
        rc = chol_solve_block<false>(n, A, b, nullptr, sm);
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
                                                               const double* red, const double* syrk, int ksplit,
                                                               int ntile, int have_syrk, int* flag) {
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

    if (threadIdx.x == 0) st[S_NPASS] += 1.0;

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
        for (int k = threadIdx.x; k < n1; k += blockDim.x) ab[k] -= sigma * gb[k];
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
            if (acc == 0) {
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
    // Newton direction: H dir = -g
    if (n1 <= CTRL_CHOL_LDS_MAX_N) {
        assemble_H(d, rl, red, syrk, ksplit, ntile, have_syrk, sgm, tau, lmat);
        for (int k = threadIdx.x; k < n1; k += blockDim.x) dir[k] = -gb[k];
        __syncthreads();
        double* vec = lmat + n1 * n1;
        // factorize from LDS directly
        int rc = chol_solve_block<false>(n1, lmat, dir, nullptr, vec);
        if (rc != 0) {
            if (threadIdx.x == 0) {
                st[S_STATUS] = -1.0;
                st[S_MODE] = (double)PM_DONE;
                if (flag) *flag = 1;
            }
            return;
        }
    } else {
        assemble_H(d, rl, red, syrk, ksplit, ntile, have_syrk, sgm, tau, H);
        for (int k = threadIdx.x; k < n1; k += blockDim.x) dir[k] = -gb[k];
        __syncthreads();
        int rc = chol_solve_block<false>(n1, H, dir, nullptr, scratch);
        if (rc != 0) {
            if (threadIdx.x == 0) {
                st[S_STATUS] = -1.0;
                st[S_MODE] = (double)PM_DONE;
                if (flag) *flag = 1;
            }
            return;
        }
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

hipError_t launch_control(double* state, StateLayout sl, RecLayout rl, const double* red, const double* syrk_out,
                          int ksplit, int tile, int ntile, int have_syrk, int* flag, hipStream_t s) {
    (void)tile;
    const int n1 = sl.n1;
    size_t lds = sizeof(double) * (size_t)(CTRL_THREADS > n1 ? CTRL_THREADS : n1);
    if (n1 <= CTRL_CHOL_LDS_MAX_N) lds += sizeof(double) * (size_t)(n1 * n1 + n1);
    hipError_t ea = ensure_dynamic_lds((const void*)control_kernel, lds);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL(control_kernel, dim3(1), dim3(CTRL_THREADS), lds, s, state, sl, rl, red, syrk_out, ksplit,
                       ntile, have_syrk, flag);
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
// Feasibility check and screening scans (FP64 arithmetic).  One wave per
// row for simplicity of the exact distance; each block covers a contiguous
// range and writes its local violator / keep list in ascending order into
// its own segment, so the final lists are deterministic.
// ---------------------------------------------------------------------------

constexpr int SCAN_THREADS = 256;

template <typename T>
__device__ __forceinline__ double row_dist(const T* row, const double* c, int d, int G, int gl) {
    double acc = 0.0;
    for (int k = gl; k < d; k += G) {
        const double e = c[k] - (double)row[k];
        acc += e * e;
    }
    return sqrt(group_sum<double>(acc, G));
}

template <typename T, bool SCREEN>
__global__ __launch_bounds__(SCAN_THREADS) void scan_kernel(const T* C, const T* R, int64_t m, int d,
                                                            const double* cdev, double r, double thr,
                                                            double* slack, double* blk_max, int64_t* blk_arg,
                                                            int64_t* blk_cnt, int64_t* seg_idx, int64_t per_block,
                                                            int G) {
    extern __shared__ double lc[];
    __shared__ int s_cnt[SCAN_THREADS / WAVE];
    __shared__ double s_max[SCAN_THREADS / WAVE];
    __shared__ int64_t s_arg[SCAN_THREADS / WAVE];
    for (int k = threadIdx.x; k < d; k += SCAN_THREADS) lc[k] = cdev[k];
    __syncthreads();
    const int lane = lane_id(), wid = threadIdx.x / WAVE;
    const int gi = lane / G, gl = lane % G, bpw = WAVE / G;
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = min(m, b0 + per_block);
    int64_t base_out = b0;
    int64_t count = 0;
    double best = -INFINITY;
    int64_t barg = INT64_MAX;
    const int step = SCAN_THREADS / G;  // balls per block step
    for (int64_t s0 = b0; s0 < b1; s0 += step) {
        const int64_t i = s0 + wid * bpw + gi;
        const bool act = i < b1;
        double val = 0.0;
        bool hit = false;
        if (act) {
            const double dist = row_dist<T>(C + i * d, lc, d, G, gl);
            const double ri = R ? (double)R[i] : 0.0;
            if (SCREEN) {
                val = r - ri - dist;
                hit = val <= thr;
                if (slack && gl == 0) slack[i] = val;
            } else {
                val = ri + dist - r;
                hit = val > thr;
            }
        }
        if (!SCREEN && act && gl == 0) {
            if (val > best || (val == best && i < barg)) {
                best = val;
                barg = i;
            }
        }
        // ordered compaction within the block step: waves in order, lanes in order
        const unsigned long long bal = __ballot(hit && act && gl == 0);
        if (lane == 0) s_cnt[wid] = __popcll(bal);
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wid; ++w) off += s_cnt[w];
        int tot = 0;
        for (int w = 0; w < SCAN_THREADS / WAVE; ++w) tot += s_cnt[w];
        if (hit && act && gl == 0) {
            const int pos = off + __popcll(bal & ((1ull << lane) - 1ull));
            seg_idx[base_out + count + pos] = i;
        }
        count += tot;
        __syncthreads();
    }
    if (!SCREEN) {
        // block max with smallest index on ties
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            const double ov = __shfl_xor(best, o, WAVE);
            const int64_t oa = __shfl_xor(barg, o, WAVE);
            if (ov > best || (ov == best && oa < barg)) {
                best = ov;
                barg = oa;
            }
        }
        if (lane == 0) {
            s_max[wid] = best;
            s_arg[wid] = barg;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double bm = s_max[0];
            int64_t ba = s_arg[0];
            for (int w = 1; w < SCAN_THREADS / WAVE; ++w)
                if (s_max[w] > bm || (s_max[w] == bm && s_arg[w] < ba)) {
                    bm = s_max[w];
                    ba = s_arg[w];
                }
            blk_max[blockIdx.x] = bm;
            blk_arg[blockIdx.x] = ba;
        }
    }
    if (threadIdx.x == 0) blk_cnt[blockIdx.x] = count;
}

static int scan_group(int d) {
    int G = 1;
    while (G < d && G < 64) G <<= 1;
    return G;
}

hipError_t launch_feasible(const void* C, const void* R, int64_t m, int d, int dtype, const double* c, double r,
                           double eps, double* blk_max, int64_t* blk_arg, int64_t* blk_cnt, int64_t* seg_idx,
                           int nblocks, int64_t per_block, hipStream_t s) {
    const int G = scan_group(d);
    size_t lds = sizeof(double) * d;
    if (dtype == 0)
        hipLaunchKernelGGL((scan_kernel<double, false>), dim3(nblocks), dim3(SCAN_THREADS), lds, s,
                           (const double*)C, (const double*)R, m, d, c, r, eps, nullptr, blk_max, blk_arg, blk_cnt,
                           seg_idx, per_block, G);
    else
        hipLaunchKernelGGL((scan_kernel<float, false>), dim3(nblocks), dim3(SCAN_THREADS), lds, s,
                           (const float*)C, (const float*)R, m, d, c, r, eps, nullptr, blk_max, blk_arg, blk_cnt,
                           seg_idx, per_block, G);
    return hipGetLastError();
}

hipError_t launch_screen(const void* C, const void* R, int64_t m, int d, int dtype, const double* c, double r,
                         double tol, double* slack, int64_t* blk_cnt, int64_t* seg_idx, int nblocks,
                         int64_t per_block, hipStream_t s) {
    const int G = scan_group(d);
    size_t lds = sizeof(double) * d;
    if (dtype == 0)
        hipLaunchKernelGGL((scan_kernel<double, true>), dim3(nblocks), dim3(SCAN_THREADS), lds, s,
                           (const double*)C, (const double*)R, m, d, c, r, tol, slack, nullptr, nullptr, blk_cnt,
                           seg_idx, per_block, G);
    else
        hipLaunchKernelGGL((scan_kernel<float, true>), dim3(nblocks), dim3(SCAN_THREADS), lds, s, (const float*)C,
                           (const float*)R, m, d, c, r, tol, slack, nullptr, nullptr, blk_cnt, seg_idx, per_block,
                           G);
    return hipGetLastError();
}

// Concatenates the per-block segments in block order.  One block per
// segment; each computes its output offset from the counts before it.
__global__ __launch_bounds__(256) void compact_kernel(const int64_t* seg_idx, const int64_t* blk_cnt, int nblocks,
                                                      int64_t per_block, int64_t* out, int64_t cap,
                                                      int64_t* total) {
    __shared__ int64_t s_off;
    const int b = blockIdx.x;
    if (threadIdx.x == 0) {
        int64_t off = 0;
        for (int k = 0; k < b; ++k) off += blk_cnt[k];
        s_off = off;
        if (b == nblocks - 1 && total) *total = off + blk_cnt[b];
    }
    __syncthreads();
    const int64_t off = s_off, cnt = blk_cnt[b];
    for (int64_t k = threadIdx.x; k < cnt; k += 256) {
        const int64_t pos = off + k;
        if (pos < cap) out[pos] = seg_idx[(int64_t)b * per_block + k];
    }
}

hipError_t launch_compact(const int64_t* seg_idx, const int64_t* blk_cnt, int nblocks, int64_t per_block,
                          int64_t* out, int64_t cap, int64_t* total_dev, hipStream_t s) {
    hipLaunchKernelGGL(compact_kernel, dim3(nblocks), dim3(256), 0, s, seg_idx, blk_cnt, nblocks, per_block, out, cap,
                       total_dev);
    return hipGetLastError();
}

__global__ void max_reduce_kernel(const double* bm, const int64_t* ba, int n, double* out_max, int64_t* out_arg) {
    if (threadIdx.x != 0) return;
    double b = -INFINITY;
    int64_t a = INT64_MAX;
    for (int k = 0; k < n; ++k)
        if (bm[k] > b || (bm[k] == b && ba[k] < a)) {
            b = bm[k];
            a = ba[k];
        }
    *out_max = b;
    *out_arg = a;
}

hipError_t launch_max_reduce(const double* blk_max, const int64_t* blk_arg, int nblocks, double* out_max,
                             int64_t* out_arg, hipStream_t s) {
    hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(64), 0, s, blk_max, blk_arg, nblocks, out_max, out_arg);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Precision preparation: C32 = float(C - origin), R32 = float(R), and the
// block maxima of ||c_i - origin|| + r_i in FP64.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(SCAN_THREADS) void prepare_kernel(const double* C, const double* R, int64_t m, int d,
                                                               const double* origin, float* C32, float* R32,
                                                               double* blk_max, int64_t per_block, int G) {
    extern __shared__ double lo[];
    __shared__ double s_max[SCAN_THREADS / WAVE];
    for (int k = threadIdx.x; k < d; k += SCAN_THREADS) lo[k] = origin ? origin[k] : 0.0;
    __syncthreads();
    const int lane = lane_id(), wid = threadIdx.x / WAVE;
    const int gi = lane / G, gl = lane % G, bpw = WAVE / G;
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = min(m, b0 + per_block);
    double best = 0.0;
    const int step = SCAN_THREADS / G;
    for (int64_t s0 = b0; s0 < b1; s0 += step) {
        const int64_t i = s0 + wid * bpw + gi;
        if (i < b1) {
            double acc = 0.0;
            for (int k = gl; k < d; k += G) {
                const double e = C[i * d + k] - lo[k];
                C32[i * d + k] = (float)e;
                acc += e * e;
            }
            const double dist = sqrt(group_sum<double>(acc, G));
            const double ri = R ? R[i] : 0.0;
            if (R && gl == 0) R32[i] = (float)ri;
            best = fmax(best, dist + ri);
        }
    }
    best = wave_max(best);
    if (lane == 0) s_max[wid] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = s_max[0];
        for (int w = 1; w < SCAN_THREADS / WAVE; ++w) b = fmax(b, s_max[w]);
        blk_max[blockIdx.x] = b;
    }
}

hipError_t launch_prepare_f32(const double* C, const double* R, int64_t m, int d, const double* origin, float* C32,
                              float* R32, double* blk_max, int nblocks, int64_t per_block, hipStream_t s) {
    const int G = scan_group(d);
    hipLaunchKernelGGL(prepare_kernel, dim3(nblocks), dim3(SCAN_THREADS), sizeof(double) * d, s, C, R, m, d, origin,
                       C32, R32, blk_max, per_block, G);
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
