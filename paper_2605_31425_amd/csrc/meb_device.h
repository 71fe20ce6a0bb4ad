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

// Cross-lane moves through the DPP modifier of a VALU instruction (no LDS
// round trip).  Patterns used: quad_perm [1,0,3,2] (lane ^ 1), quad_perm
// [2,3,0,1] (lane ^ 2), row_half_mirror (lane i <- 7 - i within 8 lanes) and
// row_mirror (lane i <- 15 - i within 16 lanes); every source lane stays in
// its row, so all lanes are valid.
constexpr int DPP_XOR1 = 0xB1;
constexpr int DPP_XOR2 = 0x4E;
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// lane ^ 16 within each half of the wave (ds_swizzle, bit mode)
__device__ __forceinline__ float swz_xor16(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}
__device__ __forceinline__ double swz_xor16(double v) {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
    return __hiloint2double(hi, lo);
}

// Sum over each aligned group of G lanes (G a power of two, wave-uniform),
// returned in every lane of the group.  Each step adds a lane's partner
// value, so all lanes of a group end with bitwise the same sum.
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
    if (G >= 2) v += dpp_move<DPP_XOR1>(v);
    if (G >= 4) v += dpp_move<DPP_XOR2>(v);
    if (G >= 8) v += dpp_move<DPP_HALF_MIRROR>(v);
    if (G >= 16) v += dpp_move<DPP_MIRROR>(v);
    if (G >= 32) v += swz_xor16(v);
    if (G >= 64) v += __shfl_xor(v, 32, WAVE);
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

// LDS of the pass: y and dir in FP64 (2d), a block reduction buffer, y and
// dir in the working precision (2d + 4), then per wave a flush scratch of
// WAVE x FLW values.  FLW = NLMAX * VEC when a wave can hold several groups
// (that needs at most 8 elements per lane), else 0.
template <int VEC, int NLMAX>
__host__ __device__ constexpr int pass_flush_width() {
    return NLMAX * VEC <= 8 ? NLMAX * VEC : 0;
}
template <typename T>
__host__ __device__ inline size_t pass_lds_head(int d) {  // in doubles
    return 2 * (size_t)d + PASS_THREADS + (sizeof(T) * (2 * (size_t)d + 4) + 7) / 8;
}
template <typename T, int VEC, int NLMAX>
__host__ __device__ inline size_t pass_lds_bytes(int d) {
    return sizeof(double) * pass_lds_head<T>(d) + sizeof(T) * (size_t)WPB * WAVE * pass_flush_width<VEC, NLMAX>();
}

// Loads and stores of data that other blocks (possibly on other XCDs, with
// their own L2) read within the same kernel: agent-scope relaxed atomics,
// i.e. write-through stores and coherent loads, so no cache flush or
// invalidation is needed.  A block publishes its data before it counts its
// arrival: the barrier waits for its stores to complete.
__device__ __forceinline__ void st_shared_dev(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_shared_dev(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int arrive(int* counter) {
    return __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum (maximum for the three KKT maxima) of n consecutive records of len
// doubles, `stride` apart, in index order, into out (written with coherent
// stores when `shared_out`).  Loads are issued in batches of sixteen before
// they are combined.
__device__ __forceinline__ void sum_records(const double* src, int n, int len, int64_t stride, int kmax,
                                            double* out, bool shared_out) {
    for (int e = threadIdx.x; e < len; e += blockDim.x) {
        const bool ismax = e >= kmax && e < kmax + 3;
        double v = ld_shared_dev(src + e);
        for (int k0 = 1; k0 < n; k0 += 16) {
            double x[16];
#pragma unroll
            for (int q = 0; q < 16; ++q)
                x[q] = (k0 + q < n) ? ld_shared_dev(src + (int64_t)(k0 + q) * stride + e) : 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (k0 + q < n) v = ismax ? fmax(v, x[q]) : v + x[q];
        }
        if (shared_out)
            st_shared_dev(out + e, v);
        else
            out[e] = v;
    }
}

// In-kernel reduction of the nrec block records (each published with
// coherent stores): the last block of each group of RED_GROUP blocks to
// arrive sums its group, then the last group sums the groups, always in
// index order, so the result does not depend on which block arrives last.
// Arrival counters are reset by the block that consumes them.
__device__ __forceinline__ void reduce_block_records(const double* rec, int nrec, const RecLayout& rl,
                                                     int64_t stride, double* red, int* sync, int blk) {
    __shared__ int s_last;
    const int len = rl.len;
    const int ng = (nrec + RED_GROUP - 1) / RED_GROUP;
    const int g = blk / RED_GROUP;
    const int gb = g * RED_GROUP, gn = min(RED_GROUP, nrec - gb);
    __syncthreads();
    if (threadIdx.x == 0) s_last = arrive(&sync[g]) == gn - 1;
    __syncthreads();
    if (!s_last) return;
    double* gp = (ng == 1) ? red : red + (size_t)(1 + g) * len;
    sum_records(rec + (int64_t)gb * stride, gn, len, stride, rl.kmax, gp, ng > 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        sync[g] = 0;
        s_last = (ng > 1) ? (arrive(&sync[SYNC_TOP]) == ng - 1) : 0;
    }
    __syncthreads();
    if (!s_last) return;
    sum_records(red + len, ng, len, len, rl.kmax, red, false);
    if (threadIdx.x == 0) sync[SYNC_TOP] = 0;
}

// Loads of one ball by one lane: its share of the row, the radius and u.
template <typename T, int VEC, int NLMAX>
struct BallLoad {
    RowVec<T, VEC> c[NLMAX];
    T r, u;
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
// Phase 1 streams the wave's balls.  With e = c_i - y and v = v_i (zero
// unless u_i != 0), everything a ball contributes to the scalar sums follows
// from five dot products, ||e||^2, <e, v>, ||v||^2, <e, dir>, <v, dir>
// (s = e + v / sigma, so ||s||^2 and <s, dir> are their combinations), so
// phase 1 keeps no per-element state beyond the row being read.  Balls whose
// vector parts are non-zero -- not polar at the evaluation point, or with an
// updated multiplier -- are appended to the wave's active list with the
// coefficients (a, b) of each part a e + b v.  Phase 2 reads those rows again
// (few, except in the first passes of a run) and accumulates the vector sums
// and writes the updated V rows.
//
// Every lane of a ball's group computes the ball's scalars redundantly (the
// group sums leave the same value in all of them); the group leader's copy
// is the one that reaches the record.  Lanes that own no part of a load read
// a valid address of the same row and discard it.  Phase-1 loads are
// software-pipelined two groups deep (the loop body is unrolled over two
// load buffers).
template <typename T, int VEC, int NLMAX, int KIND, int TRL>
__device__ __forceinline__ void pass_body(const PassArgs& a, const PassConfig& cfg, int blk) {
    extern __shared__ double lds[];
    const double* st = a.state;
    const int d = a.d;
    const int G = cfg.G;
    const int nl = cfg.nl;
    const RecLayout rl = a.rl;
    const StateLayout sl = a.sl;

    constexpr bool is_mult = (KIND == 2);
    constexpr bool want_kkt = (KIND != 0);
    const bool have_dir = (KIND != 2) && st[S_HAVE_DIR] != 0.0;

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
    // wave-uniform: keeps the wave's offsets and pointers in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int64_t gw = (int64_t)blk * WPB + wid;
    const int gi = lane / G;
    const int gl = lane % G;
    const int bpw = WAVE / G;
    const bool leader = (gl == 0);
    const int64_t wbeg = gw * cfg.bw;
    const int64_t wend = min(a.m, wbeg + cfg.bw);
    const T es_bytes = (T)sizeof(T);
    const T row_bytes = es_bytes * (T)(d + (R ? 1 : 0) + (U ? 1 : 0));

    // y and dir in the working precision, read from LDS per use
    T* l_cT = reinterpret_cast<T*>(l_red + PASS_THREADS);
    T* l_dT = l_cT + d;
    constexpr int FLW = pass_flush_width<VEC, NLMAX>();
    T* l_fl = reinterpret_cast<T*>(lds + pass_lds_head<T>(d)) + wid * WAVE * FLW;
    for (int k = threadIdx.x; k < d; k += PASS_THREADS) {
        l_cT[k] = (T)l_c[k];
        l_dT[k] = (T)l_dc[k];
    }
    __syncthreads();
    int col[NLMAX];
    bool own[NLMAX];
#pragma unroll
    for (int j = 0; j < NLMAX; ++j) {
        const int b = (j * G + gl) * VEC;
        own[j] = (j < nl) && (b < d);
        col[j] = own[j] ? b : 0;
    }

    // the wave's record doubles as the FP64 accumulator of the flushes
    double* rec = a.rec + gw * rl.len;
    for (int e = lane; e < rl.len; e += WAVE) rec[e] = 0.0;

    // ------------------------------------------------------------------
    // phase 1
    // ------------------------------------------------------------------
    T sacc[A_N];  // per-ball scalars, the same in every lane of a group
    T tacc[TRL];
    T tam[TRL];  // 1 - eta of this lane's trials
    bool tok[TRL];
#pragma unroll
    for (int r = 0; r < TRL; ++r) {
        const int l = r * G + gl;
        tok[r] = l < NT;
        tam[r] = tok[r] ? T(1) - (T)a.etas[l] : T(1);
    }
    T mx_p = 0, mx_d = 0, mx_c = 0;
    auto zero_scalars = [&]() {
#pragma unroll
        for (int k = 0; k < A_N; ++k) sacc[k] = T(0);
#pragma unroll
        for (int k = 0; k < TRL; ++k) tacc[k] = T(0);
    };
    auto flush_scalars = [&]() {
        T sred[A_N];
#pragma unroll
        for (int k = 0; k < A_N; ++k) sred[k] = group_sum<T>(leader ? sacc[k] : T(0), WAVE);
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
        zero_scalars();
    };
    zero_scalars();

    int32_t mid_count = 0, act_count = 0;
    int32_t* mid_idx = a.want_mid ? a.mid_idx + gw * cfg.bw : nullptr;
    double* mid_coef = a.want_mid ? a.mid_coef + gw * cfg.bw : nullptr;
    int32_t* act_idx = a.act_idx + gw * cfg.bw;
    T* act_coef = static_cast<T*>(a.act_coef) + gw * cfg.bw * ACT_NC;

    // rows of the group's ball; past the wave's end, its last ball again
    auto load = [&](int64_t b0, BallLoad<T, VEC, NLMAX>& L) {
        int64_t i = b0 + gi;
        i = i < wend ? i : wend - 1;
        L.r = R ? R[i] : T(0);
        L.u = U ? U[i] : T(0);
#pragma unroll
        for (int j = 0; j < NLMAX; ++j) L.c[j] = load_vec<T, VEC>(C + i * d + col[j]);
    };

    auto process = [&](int64_t b0, BallLoad<T, VEC, NLMAX>& L) {
        const int64_t i = b0 + gi;
        const bool active = i < wend;
        const T ri = L.r;
        const T ui = active ? L.u : T(0);
        const bool hasv = V && (ui != T(0));
        // dot products of e = c_i - y and v with each other and with dir
        T ee = 0, ed = 0, ev = 0, vv = 0, vd = 0;
#pragma unroll
        for (int j = 0; j < NLMAX; ++j) {
            const RowVec<T, VEC> cy = load_vec<T, VEC>(l_cT + col[j]);
            RowVec<T, VEC> dy{};
            if (KIND != 2 && have_dir) dy = load_vec<T, VEC>(l_dT + col[j]);
#pragma unroll
            for (int qq = 0; qq < VEC; ++qq) {
                const T ek = own[j] ? L.c[j].v[qq] - cy.v[qq] : T(0);
                ee += ek * ek;
                if (KIND != 2 && have_dir) ed += ek * dy.v[qq];
                L.c[j].v[qq] = ek;
            }
        }
        if (hasv) {
#pragma unroll
            for (int j = 0; j < NLMAX; ++j) {
                const RowVec<T, VEC> vr = load_vec<T, VEC>(V + i * d + col[j]);
                RowVec<T, VEC> dy{};
                if (KIND != 2 && have_dir) dy = load_vec<T, VEC>(l_dT + col[j]);
#pragma unroll
                for (int qq = 0; qq < VEC; ++qq) {
                    const T vk = own[j] ? vr.v[qq] : T(0);
                    ev += L.c[j].v[qq] * vk;
                    vv += vk * vk;
                    if (KIND != 2 && have_dir) vd += vk * dy.v[qq];
                }
            }
        }
        ee = group_sum<T>(ee, G);
        if (KIND != 2 && have_dir) ed = group_sum<T>(ed, G);
        if (__any(hasv)) {
            ev = group_sum<T>(ev, G);
            vv = group_sum<T>(vv, G);
            if (KIND != 2 && have_dir) vd = group_sum<T>(vd, G);
        }
        sacc[A_BYTES] += active ? row_bytes + (hasv ? es_bytes * (T)d : T(0)) : T(0);

        // the ball at (y, w, sigma_a): s = e + v / sigma_a
        const T t = ri - r1 + ui * inv_a;
        const T nn = ee + inv_a * (T(2) * ev + inv_a * vv);
        BallProj<T> pa = project<T>(t, nn, sig_a);
        if (!active) pa.cs = 1, pa.up = T(0), pa.gam = T(0), pa.Z = T(0);

        // evaluation point of the sums: s_e = ca e + cb v, multipliers in use
        // (ue, wa e + wb v)
        T te = t, nne = nn, ue = ui, sig_e = sig_a;
        T ca = T(1), cb = inv_a, wa = T(0), wb = T(1), wwv = vv;
        BallProj<T> pe = pa;
        T un = T(0), ga = T(0);
        if constexpr (want_kkt) {
            // updated multipliers w+ = sigma Pi(z) = (up, gam s) and the KKT terms
            un = pa.up;
            ga = pa.gam;
            if (active) {
                sacc[A_KU] += un;
                const T tp = r1 - ri;
                const T es = ee + inv_a * ev;
                mx_p = fmax(mx_p, cone_dist<T>(tp, tsqrt<T>(ee)));
                mx_d = fmax(mx_d, cone_dist<T>(un, pa.gam * pa.n));
                mx_c = fmax(mx_c, fabs(tp * un - pa.gam * es));
                if (Uo && leader) Uo[i] = un;
                sacc[A_BYTES] += (Uo ? es_bytes : T(0)) + ((Vo && un != T(0)) ? es_bytes * (T)d : T(0));
            }
            if constexpr (is_mult) {
                // the first evaluation of the next subproblem: w+ and sigma_{k+1};
                // s' = e + gam s / sigma_b = (1 + gam / sigma_b) e + gam / (sigma_a sigma_b) v
                ca = T(1) + ga * inv_b;
                cb = ga * inv_a * inv_b;
                wa = ga;
                wb = ga * inv_a;
                wwv = ga * ga * nn;
                ue = un;
                sig_e = sig_b;
                te = ri - r1 + un * inv_b;
                nne = ca * ca * ee + cb * (T(2) * ca * ev + cb * vv);
                pe = project<T>(te, nne, sig_b);
                if (!active) pe.cs = 1, pe.up = T(0), pe.gam = T(0), pe.Z = T(0);
            }
        }

        // ---- evaluation sums at (y, multipliers in use, sigma_e)
        {
            sacc[A_SU] += pe.up;
            sacc[A_Z1] += pe.Z;
            const T du = pe.up - ue;
            // ||gam_e s_e - w_v||^2 with gam_e s_e - w_v = A e + B v
            const T Ac = pe.gam * ca - wa, Bc = pe.gam * cb - wb;
            const T dv2 = Ac * Ac * ee + Bc * (T(2) * Ac * ev + Bc * vv);
            sacc[A_DM] += du * du + (active ? dv2 : T(0));
            sacc[A_WW] += ue * ue + (active ? wwv : T(0));
            sacc[A_RS] += (pe.cs != 1) ? fabs(te) + pe.n : T(0);
            sacc[A_NI] += (pe.cs == 0) ? T(1) : T(0);
            sacc[A_NM] += (pe.cs == 2) ? T(1) : T(0);
            sacc[A_SG] += (pe.cs == 2) ? pe.gam : T(0);
        }
        // Armijo trials along x_base + eta dir: lane gl takes trials gl, gl + G, ...
        if (KIND != 2 && have_dir) {
            const T q = ed + inv_a * vd;  // <s, dir>
#pragma unroll
            for (int r = 0; r < TRL; ++r) {
                const T am = tam[r];
                const T tl = te + am * dirr;
                T n2 = nne + T(2) * am * q + am * am * dc2;
                n2 = n2 > T(0) ? n2 : T(0);
                const T z = project<T>(tl, n2, sig_e).Z;
                tacc[r] += (active && tok[r]) ? z : T(0);
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
        // active list: balls with non-zero vector parts
        {
            const bool wrt = want_kkt && Vo && un != T(0);
            const bool is_act = active && (pe.cs != 1 || (want_kkt && un != T(0)));
            const unsigned long long bal = __ballot(is_act && leader);
            if (is_act && leader) {
                const unsigned long long lower = bal & ((1ull << lane) - 1ull);
                const int pos = act_count + __popcll(lower);
                act_idx[pos] = (int32_t)i;
                T* cf = act_coef + (size_t)pos * ACT_NC;
                const T inv_n = (pe.cs == 2) ? T(1) / pe.n : T(0);
                cf[0] = pe.gam * ca;
                cf[1] = pe.gam * cb;
                cf[2] = inv_n * ca;
                cf[3] = inv_n * cb;
                cf[4] = ga;
                cf[5] = ga * inv_a;
                cf[6] = (T)((hasv ? 1 : 0) | (wrt ? 2 : 0));
            }
            act_count += __popcll(bal);
        }
    };

    BallLoad<T, VEC, NLMAX> LA, LB;
    const int64_t chunk = (int64_t)bpw * FlushPeriod<T>::steps;
    for (int64_t c0 = wbeg; c0 < wend; c0 += chunk) {
        const int64_t c1 = min(wend, c0 + chunk);
        load(c0, LA);
        for (int64_t b0 = c0; b0 < c1; b0 += 2 * bpw) {
            const bool more = b0 + bpw < c1;
            if (more) load(b0 + bpw, LB);
            process(b0, LA);
            if (!more) break;
            if (b0 + 2 * bpw < c1) load(b0 + 2 * bpw, LA);
            process(b0 + bpw, LB);
        }
        flush_scalars();
    }
    {
        const T mp = wave_max_t<T>(mx_p), md = wave_max_t<T>(mx_d), mc = wave_max_t<T>(mx_c);
        if (lane == 0) {
            rec[rl.kmax + 0] = (double)mp;
            rec[rl.kmax + 1] = (double)md;
            rec[rl.kmax + 2] = (double)mc;
            if (a.mid_cnt) a.mid_cnt[gw] = mid_count;
        }
    }

    // ------------------------------------------------------------------
    // phase 2: vector parts of the active list (written above by this wave)
    // ------------------------------------------------------------------
    if (act_count > 0) {
        __threadfence_block();
        T vsv[NLMAX][VEC], vsw[NLMAX][VEC], vkv[NLMAX][VEC];
        auto zero_vec = [&]() {
#pragma unroll
            for (int j = 0; j < NLMAX; ++j)
#pragma unroll
                for (int q = 0; q < VEC; ++q) vsv[j][q] = vsw[j][q] = vkv[j][q] = T(0);
        };
        // sum over the groups of lanes with equal gl (through the wave's LDS
        // scratch when a wave holds several groups; program order within the
        // wave orders the LDS writes before the reads)
        auto flush_vec = [&](T (&A)[NLMAX][VEC], int off) {
            if (G < WAVE && FLW > 0) {
#pragma unroll
                for (int j = 0; j < NLMAX; ++j)
#pragma unroll
                    for (int q = 0; q < VEC; ++q) l_fl[(j * VEC + q) * WAVE + lane] = A[j][q];
                if (lane < G) {
#pragma unroll
                    for (int j = 0; j < NLMAX; ++j) {
                        if (!own[j]) continue;
#pragma unroll
                        for (int q = 0; q < VEC; ++q) {
                            T v = T(0);
                            for (int g = 0; g < bpw; ++g) v += l_fl[(j * VEC + q) * WAVE + g * G + lane];
                            rec[off + col[j] + q] += (double)v;
                        }
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < NLMAX; ++j)
                    if (own[j])
#pragma unroll
                        for (int q = 0; q < VEC; ++q) rec[off + col[j] + q] += (double)A[j][q];
            }
        };
        zero_vec();
        constexpr int FS = FlushPeriod<T>::steps;
        for (int k0 = 0; k0 < act_count; k0 += bpw) {
            const int k = k0 + gi;
            const bool ok = k < act_count;
            const int kk = ok ? k : act_count - 1;
            const int64_t i = act_idx[kk];
            const T* cf = act_coef + (size_t)kk * ACT_NC;
            const T a1 = cf[0], b1 = cf[1], a2 = cf[2], b2 = cf[3];
            const int flags = ok ? (int)cf[6] : 0;
            RowVec<T, VEC> er[NLMAX], vr[NLMAX];
#pragma unroll
            for (int j = 0; j < NLMAX; ++j) {
                er[j] = load_vec<T, VEC>(C + i * d + col[j]);
                const RowVec<T, VEC> cy = load_vec<T, VEC>(l_cT + col[j]);
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    er[j].v[q] = (ok && own[j]) ? er[j].v[q] - cy.v[q] : T(0);
                    vr[j].v[q] = T(0);
                }
            }
            if (flags & 1) {
#pragma unroll
                for (int j = 0; j < NLMAX; ++j)
                    if (own[j]) vr[j] = load_vec<T, VEC>(V + i * d + col[j]);
            }
#pragma unroll
            for (int j = 0; j < NLMAX; ++j)
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    vsv[j][q] += a1 * er[j].v[q] + b1 * vr[j].v[q];
                    vsw[j][q] += a2 * er[j].v[q] + b2 * vr[j].v[q];
                }
            if constexpr (want_kkt) {
                const T a3 = cf[4], b3 = cf[5];
#pragma unroll
                for (int j = 0; j < NLMAX; ++j) {
                    RowVec<T, VEC> vn;
#pragma unroll
                    for (int q = 0; q < VEC; ++q) {
                        vn.v[q] = a3 * er[j].v[q] + b3 * vr[j].v[q];
                        vkv[j][q] += vn.v[q];
                    }
                    if ((flags & 2) && own[j]) store_vec<T, VEC>(Vo + i * d + col[j], vn);
                }
            }
            if ((k0 / bpw + 1) % FS == 0 || k0 + bpw >= act_count) {
                flush_vec(vsv, rl.sv);
                flush_vec(vsw, rl.sw);
                if constexpr (want_kkt) flush_vec(vkv, rl.kv);
                zero_vec();
            }
        }
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
        st_shared_dev(r0 + e, v);
    }
    reduce_block_records(a.rec, cfg.blocks, rl, (int64_t)WPB * rl.len, a.red, a.sync, blk);
}

// The pass kernel: the solver's evaluation or multiplier update, as the device
// state's mode says (nothing when the run is done); with force_mode =
// PM_EVAL, a single evaluation (with the updated multipliers and KKT terms
// when want_kkt is set).
template <typename T, int VEC, int NLMAX, int TRL>
__device__ __forceinline__ void pass_dispatch(const PassArgs& a, const PassConfig& cfg, int blk) {
    const int mode = (int)a.state[S_MODE];
    if (mode == PM_EVAL)
        pass_body<T, VEC, NLMAX, 0, TRL>(a, cfg, blk);
    else if (mode == PM_MULT)
        pass_body<T, VEC, NLMAX, 2, TRL>(a, cfg, blk);
}

template <typename T, int VEC, int NLMAX, int TRL>
__global__ __launch_bounds__(PASS_THREADS) void pass_kernel(PassArgs a, PassConfig cfg) {
    pass_dispatch<T, VEC, NLMAX, TRL>(a, cfg, blockIdx.x);
}

// A single evaluation (meb_al_eval), independent of the state's mode; with
// want_kkt also the updated multipliers and the KKT terms.
template <typename T, int VEC, int NLMAX, int TRL>
__global__ __launch_bounds__(PASS_THREADS) void pass_eval_kernel(PassArgs a, PassConfig cfg) {
    if (a.want_kkt)
        pass_body<T, VEC, NLMAX, 1, TRL>(a, cfg, blockIdx.x);
    else
        pass_body<T, VEC, NLMAX, 0, TRL>(a, cfg, blockIdx.x);
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
