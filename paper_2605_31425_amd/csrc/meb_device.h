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
// instruction reads 64/G consecutive rows and stays coalesced; the scalar
// work per ball then runs one ball per lane (see pass_body).  Every wave
// streams its own contiguous range of balls, accumulates per-lane partial
// sums (working precision, flushed periodically into FP64), and writes one
// partial record; records are reduced in a fixed order, so results are
// bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "meb_internal.h"

namespace meb {

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
// returned in every lane of the group.  Each step adds the value of a
// partner lane that is paired with it symmetrically, so all lanes of a group
// end with bitwise the same sum.  The steps run from the widest down, as a
// switch on log2 G that falls through: scalar branches only.
// log2 G, wave-uniform (folded when G is a compile-time constant)
__device__ __forceinline__ int group_lg(int G) {
    return __builtin_constant_p(G) ? 31 - __builtin_clz(G) : __builtin_amdgcn_readfirstlane(31 - __builtin_clz(G));
}

template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
    const int lg = group_lg(G);
    switch (lg) {
        case 6:
            v += __shfl_xor(v, 32, WAVE);
            [[fallthrough]];
        case 5:
            v += swz_xor16(v);
            [[fallthrough]];
        case 4:
            v += dpp_move<DPP_MIRROR>(v);
            [[fallthrough]];
        case 3:
            v += dpp_move<DPP_HALF_MIRROR>(v);
            [[fallthrough]];
        case 2:
            v += dpp_move<DPP_XOR2>(v);
            [[fallthrough]];
        case 1:
            v += dpp_move<DPP_XOR1>(v);
            [[fallthrough]];
        default:
            break;
    }
    return v;
}

// group_sum of N values at once (one switch for all of them)
template <typename T, int N>
__device__ __forceinline__ void group_sum_n(T (&v)[N], int G) {
    const int lg = group_lg(G);
    switch (lg) {
        case 6:
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] += __shfl_xor(v[k], 32, WAVE);
            [[fallthrough]];
        case 5:
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] += swz_xor16(v[k]);
            [[fallthrough]];
        case 4:
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] += dpp_move<DPP_MIRROR>(v[k]);
            [[fallthrough]];
        case 3:
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] += dpp_move<DPP_HALF_MIRROR>(v[k]);
            [[fallthrough]];
        case 2:
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] += dpp_move<DPP_XOR2>(v[k]);
            [[fallthrough]];
        case 1:
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] += dpp_move<DPP_XOR1>(v[k]);
            [[fallthrough]];
        default:
            break;
    }
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

// ---------------------------------------------------------------------------
// Streaming rows into LDS (global_load_lds): each wave keeps a ring of
// cfg.stages blocks of DMA_BLK bytes of its contiguous row range in flight.
// The copies do not pass through registers, so many bytes stay in flight per
// wave at any register count.  Completion is tracked by vmcnt, in issue order
// among loads.  LDS accesses that may run while copies are in flight are
// written as inline assembly: the compiler would otherwise make each of them
// wait for every copy in flight.
// ---------------------------------------------------------------------------
constexpr int DMA_BLK = 2048;                 // bytes per ring block
// A block is copied by DMA_BLK / (64 x width) instructions: 16-byte copies
// (global_load_lds_dwordx4, gfx950) for instances whose row loads are 16
// bytes wide (FP32 rows with d % 4 == 0, FP64 rows with d even: every wave's
// byte range then starts 16-byte aligned), dword copies otherwise.
template <typename T, int VEC>
__host__ __device__ constexpr int dma_width() {
    return VEC * (int)sizeof(T) == 16 ? 16 : 4;
}
template <typename T, int VEC>
__host__ __device__ constexpr int dma_loads() {
    return DMA_BLK / (WAVE * dma_width<T, VEC>());
}
// rows of four parts per lane are read two steps per round
#ifndef PASS_ROUND2_NL4
#define PASS_ROUND2_NL4 1
#endif
constexpr int DMA_MIN_STAGES = 4;  // blocks per ring: the layout's minimum
// and maximum.  A wave's outstanding vector-memory operations are counted in
// six bits (at most 63), and the waits above count every copy in flight:
// with dword copies four blocks of eight copies plus the radii and
// multipliers of the next batch stay below that (eight blocks would not);
// with 16-byte copies sixteen blocks of two copies do.
constexpr int DMA_MAX_STAGES_DWORD = 4;
constexpr int DMA_MAX_STAGES_B128 = 16;
static_assert(DMA_MAX_STAGES_DWORD * (DMA_BLK / 256) + 4 <= 63, "dword copies in flight fit the counter");
static_assert(DMA_MAX_STAGES_B128 * (DMA_BLK / 1024) + 4 <= 63, "16-byte copies in flight fit the counter");
// one LDS-DMA copy of W bytes per lane (W a literal for the builtin)
template <int W>
__device__ __forceinline__ void dma_copy(const void* src, void* dst) {
    if constexpr (W == 16)
        __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
    else
        __builtin_amdgcn_global_load_lds(src, dst, 4, 0, 0);
}
__host__ __device__ constexpr int dma_max_stages(int row_load_bytes) {
    return row_load_bytes == 16 ? DMA_MAX_STAGES_B128 : DMA_MAX_STAGES_DWORD;
}

// LDS byte address of a pointer into shared memory
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char*)p;
}

// wait until at most N vector-memory operations of this wave are in flight
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt holds 6 bits");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x70 | 0xF00);
}

// wait for a copy that has at least `after` vector-memory loads of this wave
// issued after it (loads complete in issue order).  The count waited for is
// `after` rounded down to one of the steps below (waiting for more loads
// than needed is always safe).
__device__ __forceinline__ void wait_vm_after(int64_t after) {
    if (after >= 32) {
        if (after >= 63)
            wait_vm<63>();
        else if (after >= 48)
            wait_vm<48>();
        else if (after >= 40)
            wait_vm<40>();
        else
            wait_vm<32>();
    } else if (after >= 16) {
        if (after >= 28)
            wait_vm<28>();
        else if (after >= 24)
            wait_vm<24>();
        else if (after >= 20)
            wait_vm<20>();
        else
            wait_vm<16>();
    } else if (after >= 8) {
        if (after >= 14)
            wait_vm<14>();
        else if (after >= 12)
            wait_vm<12>();
        else if (after >= 10)
            wait_vm<10>();
        else
            wait_vm<8>();
    } else if (after >= 4) {
        if (after >= 6)
            wait_vm<6>();
        else
            wait_vm<4>();
    } else if (after >= 2) {
        wait_vm<2>();
    } else {
        wait_vm<0>();
    }
}

template <int BYTES>
struct LdsWord;
template <>
struct LdsWord<4> {
    typedef uint32_t type;
};
template <>
struct LdsWord<8> {
    typedef uint32_t type __attribute__((ext_vector_type(2)));
};
template <>
struct LdsWord<16> {
    typedef uint32_t type __attribute__((ext_vector_type(4)));
};

// two LDS reads of BYTES each, issued back to back, then one wait
template <int BYTES>
__device__ __forceinline__ void lds_read2(uint32_t a0, uint32_t a1, typename LdsWord<BYTES>::type& v0,
                                          typename LdsWord<BYTES>::type& v1) {
    if constexpr (BYTES == 4)
        asm volatile("ds_read_b32 %0, %2\n\tds_read_b32 %1, %3\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(v0), "=&v"(v1)
                     : "v"(a0), "v"(a1)
                     : "memory");
    else if constexpr (BYTES == 8)
        asm volatile("ds_read_b64 %0, %2\n\tds_read_b64 %1, %3\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(v0), "=&v"(v1)
                     : "v"(a0), "v"(a1)
                     : "memory");
    else
        asm volatile("ds_read_b128 %0, %2\n\tds_read_b128 %1, %3\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(v0), "=&v"(v1)
                     : "v"(a0), "v"(a1)
                     : "memory");
}

// eight LDS reads of BYTES each, then one wait
template <int BYTES>
__device__ __forceinline__ void lds_read8(const uint32_t (&a)[8], typename LdsWord<BYTES>::type (&v)[8]) {
#define MEB_LDS_READ8(OP)                                                                                  \
    asm volatile(OP " %0, %8\n\t" OP " %1, %9\n\t" OP " %2, %10\n\t" OP " %3, %11\n\t" OP " %4, %12\n\t" OP \
                 " %5, %13\n\t" OP " %6, %14\n\t" OP " %7, %15\n\ts_waitcnt lgkmcnt(0)"                        \
                 : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5]), "=&v"(v[6]),       \
                   "=&v"(v[7])                                                                                  \
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]), "v"(a[6]), "v"(a[7])          \
                 : "memory")
    if constexpr (BYTES == 4)
        MEB_LDS_READ8("ds_read_b32");
    else if constexpr (BYTES == 8)
        MEB_LDS_READ8("ds_read_b64");
    else
        MEB_LDS_READ8("ds_read_b128");
#undef MEB_LDS_READ8
}

// four LDS reads of BYTES each, then one wait
template <int BYTES>
__device__ __forceinline__ void lds_read4w(const uint32_t (&a)[4], typename LdsWord<BYTES>::type (&v)[4]) {
#define MEB_LDS_READ4W(OP)                                                                                 \
    asm volatile(OP " %0, %4\n\t" OP " %1, %5\n\t" OP " %2, %6\n\t" OP " %3, %7\n\ts_waitcnt lgkmcnt(0)"      \
                 : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3])                                          \
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3])                                                  \
                 : "memory")
    if constexpr (BYTES == 4)
        MEB_LDS_READ4W("ds_read_b32");
    else if constexpr (BYTES == 8)
        MEB_LDS_READ4W("ds_read_b64");
    else
        MEB_LDS_READ4W("ds_read_b128");
#undef MEB_LDS_READ4W
}

// four LDS reads of one T each, then one wait
template <typename T>
__device__ __forceinline__ void lds_read4(const uint32_t (&a)[4], T (&v)[4]) {
#define MEB_LDS_READ4(OP)                                                                                  \
    asm volatile(OP " %0, %4\n\t" OP " %1, %5\n\t" OP " %2, %6\n\t" OP " %3, %7\n\ts_waitcnt lgkmcnt(0)"      \
                 : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3])                                          \
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3])                                                  \
                 : "memory")
    if constexpr (sizeof(T) == 4)
        MEB_LDS_READ4("ds_read_b32");
    else
        MEB_LDS_READ4("ds_read_b64");
#undef MEB_LDS_READ4
}

template <typename T>
__device__ __forceinline__ void lds_store1(uint32_t a, T v) {
    if constexpr (sizeof(T) == 4)
        asm volatile("ds_write_b32 %0, %1" : : "v"(a), "v"(v) : "memory");
    else
        asm volatile("ds_write_b64 %0, %1" : : "v"(a), "v"(v) : "memory");
}

template <typename T>
__device__ __forceinline__ T lds_load1(uint32_t a) {
    T v;
    if constexpr (sizeof(T) == 4)
        asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(a) : "memory");
    else
        asm volatile("ds_read_b64 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(a) : "memory");
    return v;
}

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

// Square root in the projections of the evaluation pass: FP64 correctly
// rounded; FP32 (the screening precision) the hardware instruction, within
// about one ulp.
template <typename T>
__device__ __forceinline__ T psqrt(T x) {
    if constexpr (sizeof(T) == 8)
        return sqrt(x);
    else
        return __builtin_amdgcn_sqrtf(x);
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
    b.n = psqrt<T>(nn);
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

// LDS of the pass, in order: y and dir in FP64 (2d), a block reduction
// buffer, y and dir in the working precision (2d + 4); per wave the batch
// slots (BAT_N group sums of WAVE balls); one region that phase 1 uses for
// the waves' row rings (instances with NLMAX <= 4, which can stream rows
// through LDS) and phase 2 for the waves' flush scratch of WAVE x FLW values
// (FLW = NLMAX * VEC when a wave can hold several groups, which needs at most
// 16 elements per lane, else 0); then, with rings, per wave the radii and
// multipliers of two batches.
constexpr int BAT_N = 6;
template <int VEC, int NLMAX>
__host__ __device__ constexpr int pass_flush_width() {
    return NLMAX * VEC <= 16 ? NLMAX * VEC : 0;
}
__host__ __device__ constexpr bool pass_ring_capable(int nlmax) { return nlmax <= 4; }
template <typename T>
__host__ __device__ inline size_t pass_lds_head(int d) {  // in doubles, even (16-byte multiple)
    return (2 * (size_t)d + PASS_THREADS + (sizeof(T) * (2 * (size_t)d + 4) + 7) / 8 + 1) & ~(size_t)1;
}
template <typename T>
__host__ __device__ inline size_t pass_lds_bat_offset(int d) {  // bytes
    return sizeof(double) * pass_lds_head<T>(d);
}
template <typename T, int VEC, int NLMAX>
__host__ __device__ inline size_t pass_lds_ring_offset(int d) {  // bytes; also the flush scratch
    return pass_lds_bat_offset<T>(d) + sizeof(T) * (size_t)WPB * WAVE * BAT_N;
}
template <typename T, int VEC, int NLMAX>
__host__ __device__ inline size_t pass_lds_ur_offset(int d, int stages) {
    const size_t flush = sizeof(T) * (size_t)WPB * WAVE * pass_flush_width<VEC, NLMAX>();
    const size_t ring = pass_ring_capable(NLMAX) ? (size_t)WPB * stages * DMA_BLK : 0;
    static_assert(!pass_ring_capable(NLMAX) ||
                      sizeof(T) * WAVE * pass_flush_width<VEC, NLMAX>() <= DMA_MIN_STAGES * DMA_BLK,
                  "a wave's flush scratch fits its ring");
    return pass_lds_ring_offset<T, VEC, NLMAX>(d) + (ring > flush ? ring : flush);
}
// and 16 zero bytes, read by lanes that own no part of a row
template <typename T, int VEC, int NLMAX>
__host__ __device__ inline size_t pass_lds_zero_offset(int d, int stages) {
    return pass_lds_ur_offset<T, VEC, NLMAX>(d, stages) +
           (pass_ring_capable(NLMAX) ? (size_t)WPB * 4 * WAVE * sizeof(T) : 0);
}
template <typename T, int VEC, int NLMAX>
__host__ __device__ inline size_t pass_lds_bytes(int d, int stages) {
    return pass_lds_zero_offset<T, VEC, NLMAX>(d, stages) + (pass_ring_capable(NLMAX) ? 16 : 0);
}

// Loads and stores of data that other blocks (possibly on other XCDs, with
// their own L2) read within the same kernel: agent-scope relaxed atomics,
// i.e. write-through stores and coherent loads, so no cache flush or
// invalidation is needed.
//
// Ordering of a publication (a block stores its partials, then counts its
// arrival; the block that arrives last reads every partial):
//  1. every wave of the publishing block waits until its own coherent stores
//     have completed (published(): vmcnt(0); the workgroup barrier alone
//     does not wait for outstanding stores, and the compiler emits no wait
//     for relaxed atomics before it);
//  2. a workgroup barrier, then one thread counts the arrival with an
//     agent-scope atomic add: it is issued only after all of the block's
//     stores are visible at agent scope;
//  3. the block that sees the count complete reads with coherent loads,
//     issued after the counter's value returned and a barrier, so every
//     partial it reads was complete before that count was made.
// No L2 write-back or invalidation is involved: the partials never sit in a
// non-coherent cache.
__device__ __forceinline__ void st_shared_dev(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_shared_dev(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int arrive(int* counter) {
    return __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// this wave's stores (and loads) have completed
__device__ __forceinline__ void published() { wait_vm<0>(); }

// Sum (maximum for the three KKT maxima) of n consecutive records of len
// doubles, `stride` apart, in index order, into out (written with coherent
// stores when `shared_out`).  Loads are issued in batches of sixteen before
// they are combined.
__device__ __forceinline__ void sum_records(const double* src, int n, int len, int64_t stride, int kmax,
                                            double* out, bool shared_out) {
    // two elements per thread at a time, and all loads of a batch of
    // RED_GROUP records issued before the first is used (indices past n read
    // record n - 1 and are not added): a group costs one memory round trip
    // for records of up to two elements per thread
    for (int e0 = threadIdx.x; e0 < len; e0 += 2 * blockDim.x) {
        const int e1 = e0 + blockDim.x;
        const int e1c = e1 < len ? e1 : e0;
        const bool max0 = e0 >= kmax && e0 < kmax + 3, max1 = e1 >= kmax && e1 < kmax + 3;
        double v0 = 0.0, v1 = 0.0;
        for (int k0 = 0; k0 < n; k0 += RED_GROUP) {
            double x0[RED_GROUP], x1[RED_GROUP];
#pragma unroll
            for (int q = 0; q < RED_GROUP; ++q) {
                const int k = k0 + q < n ? k0 + q : n - 1;
                x0[q] = ld_shared_dev(src + (int64_t)k * stride + e0);
                x1[q] = ld_shared_dev(src + (int64_t)k * stride + e1c);
            }
#pragma unroll
            for (int q = 0; q < RED_GROUP; ++q) {
                if (k0 + q < n) {
                    v0 = (k0 + q == 0) ? x0[q] : (max0 ? fmax(v0, x0[q]) : v0 + x0[q]);
                    v1 = (k0 + q == 0) ? x1[q] : (max1 ? fmax(v1, x1[q]) : v1 + x1[q]);
                }
            }
        }
        if (shared_out) {
            st_shared_dev(out + e0, v0);
            if (e1 < len) st_shared_dev(out + e1, v1);
        } else {
            out[e0] = v0;
            if (e1 < len) out[e1] = v1;
        }
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
    published();
    __syncthreads();
    if (threadIdx.x == 0) s_last = arrive(&sync[g]) == gn - 1;
    __syncthreads();
    if (!s_last) return;
    double* gp = (ng == 1) ? red : red + (size_t)(1 + g) * len;
    sum_records(rec + (int64_t)gb * stride, gn, len, stride, rl.kmax, gp, ng > 1);
    published();
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
    T u;
};

// The evaluation pass over one wave's contiguous range of balls.
//
// KIND 0: evaluation at y = x_base + dir (Psi trials along the segment,
//         gradient and Hessian parts, the mid list);
// KIND 1: evaluation plus the updated multipliers sigma Pi(z) and the KKT terms
//         at y (the single-evaluation entry point);
// KIND 2: multiplier update at x_j, its KKT terms, and the first evaluation of
//         the next outer iteration at sigma_{k+1}.
// TRL: the group width G when the instance is specialized for one (8, 32:
//      G is then a compile-time constant), else a tag of its class of widths
//      (1, 3, 9) and G comes from the configuration.
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
// Phase 1 works in batches of WAVE balls.  The dot products of a ball are
// spread over its group of G lanes and group-summed; the group leader puts
// them in the ball's batch slot in LDS.  After a batch, lane l takes ball l
// of the batch for everything per ball -- projections, the scalar sums, the
// Armijo trials, the list entries -- so that scalar work runs on all 64
// lanes instead of once per group.  Lanes that own no part of a load read a
// valid address of the same row and discard it.  Phase-1 loads are
// software-pipelined two steps deep (the loop body is unrolled over two load
// buffers).
template <typename T, int VEC, int NLMAX, int KIND, int TRL>
__device__ __forceinline__ void pass_body(const PassArgs& a, const PassConfig& cfg, int blk) {
    extern __shared__ __align__(16) double lds[];
    const double* st = a.state;
    const int d = a.d;
    const int G = (TRL == 8 || TRL == 32) ? TRL : cfg.G;
    const int nl = cfg.nl;
    const RecLayout rl = a.rl;
    const StateLayout sl = a.sl;

    constexpr bool is_mult = (KIND == 2);
    constexpr bool want_kkt = (KIND != 0);
    // every state value the pass needs is loaded before any is used (one
    // memory round trip; the direction is read even when there is none and
    // then ignored)
    const double hd_raw = st[S_HAVE_DIR];
    const double dir0_raw = st[sl.dir];
    const double xb0 = st[sl.xb];
    const double sig_a_d = st[S_SIGMA];
    const double sig_b_d = st[S_SIGMA_NEXT];
    constexpr int KQ = (MEB_MAX_D + PASS_THREADS - 1) / PASS_THREADS;
    const int nq = (d + PASS_THREADS - 1) / PASS_THREADS;  // uniform
    double dk_raw[KQ], xk_raw[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
        if (q < nq) {
            const int k = threadIdx.x + q * PASS_THREADS;
            const int kc = k < d ? k : d - 1;
            dk_raw[q] = st[sl.dir + 1 + kc];
            xk_raw[q] = st[sl.xb + 1 + kc];
        }
    }
    const bool have_dir = (KIND != 2) && hd_raw != 0.0;

    // the evaluation point y = x_base + dir and the direction, staged in LDS
    double* l_c = lds;
    double* l_dc = lds + d;
    double* l_red = lds + 2 * d;
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
        const int k = threadIdx.x + q * PASS_THREADS;
        if (q < nq && k < d) {
            const double dk = have_dir ? dk_raw[q] : 0.0;
            l_c[k] = xk_raw[q] + dk;
            l_dc[k] = dk;
            part += dk * dk;
        }
    }
    if constexpr (pass_ring_capable(NLMAX)) {
        if (threadIdx.x < 4)
            reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(lds) +
                                        pass_lds_zero_offset<T, VEC, NLMAX>(d, cfg.stages))[threadIdx.x] = 0u;
    }
    // ||dir||^2: each wave sums its lanes, then the WPB wave sums in order
    part = wave_sum_t<double>(part);
    if ((threadIdx.x & (WAVE - 1)) == 0) l_red[threadIdx.x / WAVE] = part;
    __syncthreads();
    double dsum = 0.0;
#pragma unroll
    for (int w = 0; w < WPB; ++w) dsum += l_red[w];
    const T dc2 = (T)dsum;
    const double dirr_d = have_dir ? dir0_raw : 0.0;
    const T r1 = (T)(xb0 + dirr_d);
    const T dirr = (T)dirr_d;
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
    // a wave's flush scratch lies inside its own ring (used after its copies)
    T* l_fl = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(lds) + pass_lds_ring_offset<T, VEC, NLMAX>(d) +
                                   (size_t)wid * (pass_ring_capable(NLMAX) ? cfg.stages * DMA_BLK : WAVE * FLW * sizeof(T)));
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
    // (a) dot products: a step covers bpw balls, one per group of G lanes,
    //     and the group sums go to the wave's batch slots in LDS;
    // (b) every S = WAVE / bpw steps (a batch of WAVE balls), each lane takes
    //     one ball of the batch for the scalar part: projections, sums,
    //     Armijo trials, the mid and active lists.
    // Rows reach the dot products either through the wave's LDS ring
    // (cfg.dma: rows short enough that a step fits a ring block) or through
    // registers, two steps deep.
    const int S = WAVE / bpw;
    T* l_bat = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(lds) + pass_lds_bat_offset<T>(d)) +
               wid * (BAT_N * WAVE);
    const uint32_t bat_addr = lds_addr(l_bat);
    T sacc[A_N];  // this lane's balls' scalar sums
    T tacc[NT];   // this lane's balls' Armijo trial sums
    T mx_p = 0, mx_d = 0, mx_c = 0;
    auto zero_scalars = [&]() {
#pragma unroll
        for (int k = 0; k < A_N; ++k) sacc[k] = T(0);
#pragma unroll
        for (int k = 0; k < NT; ++k) tacc[k] = T(0);
    };
    auto flush_scalars = [&]() {
        T sred[A_N];
#pragma unroll
        for (int k = 0; k < A_N; ++k) sred[k] = group_sum<T>(sacc[k], WAVE);
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
            for (int l = 0; l < NT; ++l) {
                const T v = group_sum<T>(tacc[l], WAVE);
                if (lane == 0) rec[rl.trial + l] += (double)v;
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

    // y and dir in the lane's columns (zero in parts the lane does not own;
    // the row values there are zero too).  Instances that stream rows
    // through LDS read them from LDS at every step (the zero slot where the
    // lane owns no part), which keeps 2 NLMAX VEC registers free across the
    // scalar part; the others keep them in registers.
    constexpr bool YLDS = pass_ring_capable(NLMAX);
    RowVec<T, VEC> cyv[YLDS ? 1 : NLMAX], dyv[YLDS ? 1 : NLMAX];
    uint32_t ya[YLDS ? NLMAX : 1], da[YLDS ? NLMAX : 1];
    if constexpr (YLDS) {
        const uint32_t zero_slot =
            lds_addr(reinterpret_cast<unsigned char*>(lds) + pass_lds_zero_offset<T, VEC, NLMAX>(d, cfg.stages));
#pragma unroll
        for (int j = 0; j < NLMAX; ++j) {
            ya[j] = own[j] ? lds_addr(l_cT + col[j]) : zero_slot;
            da[j] = own[j] ? lds_addr(l_dT + col[j]) : zero_slot;
        }
    } else {
#pragma unroll
        for (int j = 0; j < NLMAX; ++j) {
            cyv[j] = load_vec<T, VEC>(l_cT + col[j]);
            dyv[j] = load_vec<T, VEC>(l_dT + col[j]);
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                cyv[j].v[q] = own[j] ? cyv[j].v[q] : T(0);
                dyv[j].v[q] = own[j] ? dyv[j].v[q] : T(0);
            }
        }
    }

    // (a) the five dot products of the groups' balls of steps s .. s + NB - 1
    // (rows in c, zero where the lane owns no part; multipliers in u), into
    // the balls' batch slots.  NB steps share one set of group sums.
    auto dots = [&](int64_t s, auto& c, auto& u) {
        constexpr int NB = sizeof(u) / sizeof(u[0]);
        RowVec<T, VEC> cy[NLMAX], dy[NLMAX];
        if constexpr (YLDS) {
            typedef typename LdsWord<VEC * sizeof(T)>::type W;
            if constexpr (NLMAX == 4) {
                const uint32_t ad[8] = {ya[0], ya[1], ya[2], ya[3], da[0], da[1], da[2], da[3]};
                W w[8];
                lds_read8<VEC * sizeof(T)>(ad, w);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    __builtin_memcpy(&cy[j], &w[j], sizeof(cy[j]));
                    __builtin_memcpy(&dy[j], &w[4 + j], sizeof(dy[j]));
                }
            } else {
                static_assert(NLMAX == 2, "ring instances have two or four parts per row");
                const uint32_t ad[4] = {ya[0], ya[1], da[0], da[1]};
                W w[4];
                lds_read4w<VEC * sizeof(T)>(ad, w);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    __builtin_memcpy(&cy[j], &w[j], sizeof(cy[j]));
                    __builtin_memcpy(&dy[j], &w[2 + j], sizeof(dy[j]));
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < NLMAX; ++j) {
                cy[j] = cyv[j];
                dy[j] = dyv[j];
            }
        }
        T g[2 * NB];  // ||e||^2, <e, dir> per step
        bool hv[NB];
        bool anyv = false;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int64_t i = wbeg + (s + t) * bpw + gi;
            const T ui = i < wend ? u[t] : T(0);
            hv[t] = V && (ui != T(0));
            anyv = anyv || hv[t];
            T ee = 0, ed = 0;
#pragma unroll
            for (int j = 0; j < NLMAX; ++j) {
#pragma unroll
                for (int qq = 0; qq < VEC; ++qq) {
                    const T ek = c[t][j].v[qq] - cy[j].v[qq];
                    ee += ek * ek;
                    if (KIND != 2 && have_dir) ed += ek * dy[j].v[qq];
                    c[t][j].v[qq] = ek;
                }
            }
            g[2 * t] = ee;
            g[2 * t + 1] = ed;
        }
        group_sum_n<T, 2 * NB>(g, G);
        // <e, v>, ||v||^2, <v, dir>, ||s||^2 per step, s = e + v / sigma_a formed
        // element by element (expanding ||s||^2 from the other products would
        // cancel when v / sigma_a is close to -e)
        T gv[4 * NB];
#pragma unroll
        for (int k = 0; k < 4 * NB; ++k) gv[k] = T(0);
        if (__any(anyv)) {
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                if (hv[t]) {
                    const int64_t i = wbeg + (s + t) * bpw + gi;
#pragma unroll
                    for (int j = 0; j < NLMAX; ++j) {
                        const RowVec<T, VEC> vr = load_vec<T, VEC>(V + i * d + col[j]);
#pragma unroll
                        for (int qq = 0; qq < VEC; ++qq) {
                            const T vk = own[j] ? vr.v[qq] : T(0);
                            const T sk = c[t][j].v[qq] + vk * inv_a;
                            gv[4 * t] += c[t][j].v[qq] * vk;
                            gv[4 * t + 1] += vk * vk;
                            if (KIND != 2 && have_dir) gv[4 * t + 2] += vk * dy[j].v[qq];
                            gv[4 * t + 3] += sk * sk;
                        }
                    }
                }
            }
            group_sum_n<T, 4 * NB>(gv, G);
        }
        if (leader) {
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                const uint32_t sa = bat_addr + (uint32_t)(((int)((s + t) % S) * bpw + gi) * (int)sizeof(T));
                lds_store1<T>(sa + 0 * WAVE * sizeof(T), g[2 * t]);
                lds_store1<T>(sa + 1 * WAVE * sizeof(T), g[2 * t + 1]);
                lds_store1<T>(sa + 2 * WAVE * sizeof(T), gv[4 * t]);
                lds_store1<T>(sa + 3 * WAVE * sizeof(T), gv[4 * t + 1]);
                lds_store1<T>(sa + 4 * WAVE * sizeof(T), gv[4 * t + 2]);
                lds_store1<T>(sa + 5 * WAVE * sizeof(T), gv[4 * t + 3]);
            }
        }
    };

    // (b) the scalar part of ball b0 + lane, with its radius and multiplier
    auto scalars = [&](int64_t b0, T ri, T ui_in) {
        const int64_t i = b0 + lane;
        const bool active = i < wend;
        const uint32_t la = bat_addr + (uint32_t)(lane * (int)sizeof(T));
        const T ee = lds_load1<T>(la + 0 * WAVE * sizeof(T));
        const T ed = lds_load1<T>(la + 1 * WAVE * sizeof(T));
        const T ev = lds_load1<T>(la + 2 * WAVE * sizeof(T));
        const T vv = lds_load1<T>(la + 3 * WAVE * sizeof(T));
        const T vd = lds_load1<T>(la + 4 * WAVE * sizeof(T));
        const T ssd = lds_load1<T>(la + 5 * WAVE * sizeof(T));
        const T ui = active ? ui_in : T(0);
        const bool hasv = V && (ui != T(0));
        sacc[A_BYTES] += active ? row_bytes + (hasv ? es_bytes * (T)d : T(0)) : T(0);

        // the ball at (y, w, sigma_a): s = e + v / sigma_a
        const T t = ri - r1 + ui * inv_a;
        const T nn = hasv ? ssd : ee;  // ||s||^2, formed element by element
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
                if (Uo) Uo[i] = un;
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
                // ||e + k s||^2 with k = gam / sigma_b; rounding can take the
                // expansion below zero when k s is close to -e
                const T kq = ga * inv_b;
                nne = ee + kq * (T(2) * (ee + inv_a * ev) + kq * nn);
                nne = nne > T(0) ? nne : T(0);
                pe = project<T>(te, nne, sig_b);
                if (!active) pe.cs = 1, pe.up = T(0), pe.gam = T(0), pe.Z = T(0);
            }
        }

        // ---- evaluation sums at (y, multipliers in use, sigma_e)
        {
            sacc[A_SU] += pe.up;
            sacc[A_Z1] += pe.Z;
            const T du = pe.up - ue;
            // ||gam_e s_e - w_v||^2: balls on the active list (below) add it in
            // phase 2, element by element; for the others gam_e = 0 and it is
            // ||v||^2 in an evaluation, 0 in a multiplier update (w+ = 0 there)
            const bool listed = pe.cs != 1 || (want_kkt && un != T(0));
            const T dv2 = (KIND != 2) ? vv : T(0);
            sacc[A_DM] += du * du + ((active && !listed) ? dv2 : T(0));
            sacc[A_WW] += ue * ue + (active ? wwv : T(0));
            sacc[A_RS] += (pe.cs != 1) ? fabs(te) + pe.n : T(0);
            sacc[A_NI] += (pe.cs == 0) ? T(1) : T(0);
            sacc[A_NM] += (pe.cs == 2) ? T(1) : T(0);
            sacc[A_SG] += (pe.cs == 2) ? pe.gam : T(0);
        }
        // Armijo trials along x_base + eta dir
        if (KIND != 2 && have_dir) {
            const T q = ed + inv_a * vd;  // <s, dir>
#pragma unroll
            for (int l = 0; l < NT; ++l) {
                const T am = T(1) - (T)a.etas[l];  // 1 - eta
                const T tl = te + am * dirr;
                T n2 = nne + T(2) * am * q + am * am * dc2;
                n2 = n2 > T(0) ? n2 : T(0);
                const T z = project<T>(tl, n2, sig_e).Z;
                tacc[l] += active ? z : T(0);
            }
        }
        // mid list of the rank-one Hessian part: coef_i = -sigma t_i / (2 n_i^3)
        if (a.want_mid) {
            const bool is_mid = active && pe.cs == 2;
            const unsigned long long bal = __ballot(is_mid);
            if (is_mid) {
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
            const unsigned long long bal = __ballot(is_act);
            if (is_act) {
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

    const int64_t nsteps = (wend - wbeg + bpw - 1) / bpw;
    const int64_t nbatch = (nsteps + S - 1) / S;
    // radius and multiplier of ball b0 + lane (clamped to the range)
    auto fetch_ur = [&](int64_t b0, T& r, T& u) {
        int64_t i = b0 + lane;
        i = i < wend ? i : wend - 1;
        r = R ? R[i] : T(0);
        u = U ? U[i] : T(0);
    };
    int nbat = 0;  // batches since the last flush
    auto after_batch = [&](int64_t bb) {
        if (++nbat == FlushPeriod<T>::steps || bb + 1 == nbatch) {
            flush_scalars();
            nbat = 0;
        }
    };
    bool done = false;
    if constexpr (pass_ring_capable(NLMAX)) {
        if (cfg.dma) {
            // rows through the LDS ring: stream bytes [S0, S0 + SB) of C.  The
            // radii and multipliers of each batch are copied the same way, one
            // batch ahead.  nld counts this wave's copies (one load each).
            // Offsets within the wave's range fit 32 bits (the host checks).
            const int rowB = d * (int)sizeof(T);
            const int64_t S0 = wbeg * (int64_t)rowB, total = a.m * (int64_t)rowB;
            const int SB = (int)(wend - wbeg) * rowB;
            const int nblk = (SB + DMA_BLK - 1) / DMA_BLK;
            const int stages = cfg.stages, ring_bytes = stages * DMA_BLK;  // power-of-two ring
            unsigned char* ring = reinterpret_cast<unsigned char*>(lds) + pass_lds_ring_offset<T, VEC, NLMAX>(d) +
                                  (size_t)wid * ring_bytes;
            const uint32_t ring_addr = lds_addr(ring);
            unsigned char* ur = reinterpret_cast<unsigned char*>(lds) + pass_lds_ur_offset<T, VEC, NLMAX>(d, stages) +
                                (size_t)wid * 4 * WAVE * sizeof(T);  // [parity][U, R][WAVE]
            const uint32_t ur_addr = lds_addr(ur);
            const uint32_t zero_addr =
                lds_addr(reinterpret_cast<unsigned char*>(lds) + pass_lds_zero_offset<T, VEC, NLMAX>(d, stages));
            const char* Cb = static_cast<const char*>(a.C) + S0;
            constexpr int DW = dma_width<T, VEC>();  // bytes per lane and copy
            constexpr int DL = dma_loads<T, VEC>();  // copies per block
            constexpr int DSTEP = DW * WAVE;          // bytes per copy
            const int64_t Clim = total - DW - S0;     // last DW-byte word of C, relative to S0
            int issued = 0, landed = -1, nld = 0;
            auto issue = [&]() {
                const int k = issued++;
                unsigned char* dst = ring + (k & (stages - 1)) * DMA_BLK;
                const char* bk = Cb + (int64_t)k * DMA_BLK;  // wave-uniform
                if ((int64_t)k * DMA_BLK + DMA_BLK - DW <= Clim) {
#pragma unroll
                    for (int q = 0; q < DL; ++q)
                        dma_copy<DW>(bk + q * DSTEP + lane * DW, dst + q * DSTEP);
                } else {  // the block passes the end of C: clamp to its last word
#pragma unroll
                    for (int q = 0; q < DL; ++q) {
                        int64_t o = (int64_t)k * DMA_BLK + q * DSTEP + lane * DW;
                        o = o <= Clim ? o : Clim;
                        dma_copy<DW>(Cb + o, dst + q * DSTEP);
                    }
                }
                nld += DL;
            };
            // relative bytes [0, end) in LDS: every block up to the one holding
            // byte end - 1 has landed
            auto ensure = [&](int end) {
                const int need = (end - 1) / DMA_BLK;
                if (landed < need) {
                    landed = need;
                    wait_vm_after((issued - 1 - landed) * DL);
                }
            };
            // relative bytes below `done_to` are consumed: refill their blocks
            auto refill = [&](int done_to) {
                const int top = min(nblk, done_to / DMA_BLK + stages);
                while (issued < top) issue();
            };
            // radii and multipliers of balls b0 .. b0 + WAVE - 1 into slot par
            auto issue_ur = [&](int64_t b0, int par) {
                const char* srcs[2] = {static_cast<const char*>(a.U), static_cast<const char*>(a.R)};
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    if (!srcs[k]) continue;
                    unsigned char* dst = ur + (size_t)(par * 2 + k) * WAVE * sizeof(T);
#pragma unroll
                    for (int q = 0; q < (int)sizeof(T) / 4; ++q) {
                        int64_t o = b0 * (int64_t)sizeof(T) + q * 256 + lane * 4;
                        const int64_t lim = a.m * (int64_t)sizeof(T) - 4;
                        o = o <= lim ? o : lim;
                        __builtin_amdgcn_global_load_lds(srcs[k] + o, dst + q * 256, 4, 0, 0);
                        ++nld;
                    }
                }
            };
            refill(0);
            issue_ur(wbeg, 0);
            int ur_mark = nld;  // copies issued up to the current batch's radii and multipliers
            const int nsteps32 = (int)nsteps;
            for (int bb = 0; bb < (int)nbatch; ++bb) {
                const int par = bb & 1;
                wait_vm_after(nld - ur_mark);
                int ur_next = 0;
                if (bb + 1 < (int)nbatch) {
                    issue_ur(wbeg + (int64_t)(bb + 1) * WAVE, par ^ 1);
                    ur_next = nld;
                }
                const uint32_t u_addr = ur_addr + (uint32_t)((par * 2 + 0) * WAVE * sizeof(T));
                const uint32_t r_addr = ur_addr + (uint32_t)((par * 2 + 1) * WAVE * sizeof(T));
                const int s0 = bb * S, s1 = min(nsteps32, s0 + S);
                const int nrange = (int)(wend - wbeg);
                // ring address of part j of the group's ball of step s
                auto row_addr = [&](int s, int j) -> uint32_t {
                    int il = s * bpw + gi;
                    il = il < nrange ? il : nrange - 1;
                    return own[j] ? ring_addr + (uint32_t)((il * rowB + col[j] * (int)sizeof(T)) & (ring_bytes - 1))
                                  : zero_addr;
                };
                auto u_addr_of = [&](int s) -> uint32_t {
                    return u_addr + (uint32_t)(((s - s0) * bpw + gi) * (int)sizeof(T));
                };
                // a round of NB steps: one wait, one read of all rows, one set of
                // group sums.  Its rows must fit the ring with a block to
                // spare: NB * bpw * rowB <= (stages - 1) * DMA_BLK.
                auto round = [&](int s, auto nb_tag) {
                    constexpr int NB = decltype(nb_tag)::value;
                    const int end = min(SB, (s + NB) * bpw * rowB);
                    ensure(end);
                    RowVec<T, VEC> c[NB][NLMAX];
                    T u[NB];
                    static_assert(NB == 1 || NLMAX == 2 || (NLMAX == 4 && NB == 2),
                                  "rounds of several steps read eight parts at most");
                    if constexpr (NB == 2 && NLMAX == 4) {
                        uint32_t ra[8];
#pragma unroll
                        for (int t = 0; t < 2; ++t)
#pragma unroll
                            for (int j = 0; j < 4; ++j) ra[4 * t + j] = row_addr(s + t, j);
                        typename LdsWord<VEC * sizeof(T)>::type w[8];
                        lds_read8<VEC * sizeof(T)>(ra, w);
#pragma unroll
                        for (int t = 0; t < 2; ++t)
#pragma unroll
                            for (int j = 0; j < 4; ++j) __builtin_memcpy(&c[t][j], &w[4 * t + j], sizeof(c[t][j]));
                        u[0] = U ? lds_load1<T>(u_addr_of(s)) : T(0);
                        u[1] = U ? lds_load1<T>(u_addr_of(s + 1)) : T(0);
                    } else if constexpr (NB == 4) {
                        uint32_t ra[8];
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            ra[2 * t] = row_addr(s + t, 0);
                            ra[2 * t + 1] = row_addr(s + t, 1);
                        }
                        typename LdsWord<VEC * sizeof(T)>::type w[8];
                        lds_read8<VEC * sizeof(T)>(ra, w);
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            __builtin_memcpy(&c[t][0], &w[2 * t], sizeof(c[t][0]));
                            __builtin_memcpy(&c[t][1], &w[2 * t + 1], sizeof(c[t][1]));
                        }
                        for (int t = 0; t < 4; ++t) u[t] = T(0);
                        if (U) {
                            const uint32_t ua[4] = {u_addr_of(s), u_addr_of(s + 1), u_addr_of(s + 2), u_addr_of(s + 3)};
                            lds_read4<T>(ua, u);
                        }
                    } else if constexpr (NB == 2) {
                        const uint32_t ra[4] = {row_addr(s, 0), row_addr(s, 1), row_addr(s + 1, 0), row_addr(s + 1, 1)};
                        typename LdsWord<VEC * sizeof(T)>::type w[4];
                        lds_read4w<VEC * sizeof(T)>(ra, w);
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            __builtin_memcpy(&c[t][0], &w[2 * t], sizeof(c[t][0]));
                            __builtin_memcpy(&c[t][1], &w[2 * t + 1], sizeof(c[t][1]));
                        }
                        u[0] = U ? lds_load1<T>(u_addr_of(s)) : T(0);
                        u[1] = U ? lds_load1<T>(u_addr_of(s + 1)) : T(0);
                    } else if constexpr (NLMAX == 2) {
                        typename LdsWord<VEC * sizeof(T)>::type w0, w1;
                        lds_read2<VEC * sizeof(T)>(row_addr(s, 0), row_addr(s, 1), w0, w1);
                        __builtin_memcpy(&c[0][0], &w0, sizeof(c[0][0]));
                        __builtin_memcpy(&c[0][1], &w1, sizeof(c[0][1]));
                        u[0] = U ? lds_load1<T>(u_addr_of(s)) : T(0);
                    } else {
                        const uint32_t ra[4] = {row_addr(s, 0), row_addr(s, 1), row_addr(s, 2), row_addr(s, 3)};
                        typename LdsWord<VEC * sizeof(T)>::type w[4];
                        lds_read4w<VEC * sizeof(T)>(ra, w);
#pragma unroll
                        for (int j = 0; j < 4; ++j) __builtin_memcpy(&c[0][j], &w[j], sizeof(c[0][j]));
                        u[0] = U ? lds_load1<T>(u_addr_of(s)) : T(0);
                    }
                    dots(s, c, u);
                    refill(end);
                };
                const int step_bytes = bpw * rowB;
                int s = s0;
                if constexpr (NLMAX == 2) {
                    if ((S & 3) == 0 && 4 * step_bytes <= (stages - 1) * DMA_BLK) {
                        for (; s + 4 <= s1; s += 4) round(s, std::integral_constant<int, 4>());
                    } else if ((S & 1) == 0 && 2 * step_bytes <= (stages - 1) * DMA_BLK) {
                        for (; s + 2 <= s1; s += 2) round(s, std::integral_constant<int, 2>());
                    }
                } else if constexpr (NLMAX == 4 && PASS_ROUND2_NL4) {
                    if ((S & 1) == 0 && 2 * step_bytes <= (stages - 1) * DMA_BLK) {
                        for (; s + 2 <= s1; s += 2) round(s, std::integral_constant<int, 2>());
                    }
                }
                for (; s < s1; ++s) round(s, std::integral_constant<int, 1>());
                const T rb = R ? lds_load1<T>(r_addr + (uint32_t)(lane * (int)sizeof(T))) : T(0);
                const T ub = U ? lds_load1<T>(u_addr + (uint32_t)(lane * (int)sizeof(T))) : T(0);
                scalars(wbeg + (int64_t)bb * WAVE, rb, ub);
                after_batch(bb);
                if (bb + 1 < (int)nbatch) ur_mark = ur_next;
            }
            wait_vm<0>();  // no copy may land after the wave moves on
            done = true;
        }
    }
    if (!done) {
        // rows of the group's ball of step s; past the wave's end, its last
        // ball again
        auto load = [&](int64_t s, BallLoad<T, VEC, NLMAX>& L) {
            int64_t i = wbeg + s * bpw + gi;
            i = i < wend ? i : wend - 1;
            L.u = U ? U[i] : T(0);
#pragma unroll
            for (int j = 0; j < NLMAX; ++j) L.c[j] = load_vec<T, VEC>(C + i * d + col[j]);
        };
        // zero the parts of a row the lane does not own
        auto own_only = [&](BallLoad<T, VEC, NLMAX>& L) -> BallLoad<T, VEC, NLMAX>& {
#pragma unroll
            for (int j = 0; j < NLMAX; ++j)
#pragma unroll
                for (int q = 0; q < VEC; ++q) L.c[j].v[q] = own[j] ? L.c[j].v[q] : T(0);
            return L;
        };
        auto step1 = [&](int64_t s, BallLoad<T, VEC, NLMAX>& L) {
            RowVec<T, VEC> c[1][NLMAX];
            own_only(L);
#pragma unroll
            for (int j = 0; j < NLMAX; ++j) c[0][j] = L.c[j];
            T u[1] = {L.u};
            dots(s, c, u);
        };
        BallLoad<T, VEC, NLMAX> LA, LB;
        if (nsteps > 0) load(0, LA);
        for (int64_t bb = 0; bb < nbatch; ++bb) {
            const int64_t s0 = bb * S, s1 = min(nsteps, s0 + S);
            for (int64_t s = s0; s < s1; s += 2) {
                if (s + 1 < s1) load(s + 1, LB);
                step1(s, LA);
                if (s + 1 >= s1) break;
                if (s + 2 < nsteps) load(s + 2, LA);
                step1(s + 1, LB);
            }
            if (((s1 - s0) & 1) && s1 < nsteps) load(s1, LA);
            T rb, ub;
            fetch_ur(wbeg + bb * WAVE, rb, ub);
            scalars(wbeg + bb * WAVE, rb, ub);
            after_batch(bb);
        }
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
        T dmv = T(0);  // this lane's part of sum ||gam_e s_e - w_v||^2 over the list
        auto zero_vec = [&]() {
            dmv = T(0);
#pragma unroll
            for (int j = 0; j < NLMAX; ++j)
#pragma unroll
                for (int q = 0; q < VEC; ++q) vsv[j][q] = vsw[j][q] = vkv[j][q] = T(0);
        };
        // sum over the groups of lanes with equal gl (through the wave's LDS
        // scratch when a wave holds several groups).  The wave's LDS accesses
        // complete in issue order; the compiler barriers keep that order in
        // the code, since a lane reads what other lanes wrote (addresses the
        // compiler may see as disjoint from the lane's own writes when G is a
        // compile-time constant).
        auto flush_vec = [&](T (&A)[NLMAX][VEC], int off) {
            if (G < WAVE && FLW > 0) {
                asm volatile("" ::: "memory");  // earlier reads of the scratch stay before these writes
#pragma unroll
                for (int j = 0; j < NLMAX; ++j)
#pragma unroll
                    for (int q = 0; q < VEC; ++q) l_fl[(j * VEC + q) * WAVE + lane] = A[j][q];
                asm volatile("" ::: "memory");  // the writes stay before the reads
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
            // the multiplier in use is (wa e + wb v): (0, 1) in an evaluation,
            // the updated one in a multiplier update
            const T wa = (KIND == 2) ? cf[4] : T(0), wb = (KIND == 2) ? cf[5] : T(1);
            const T da = a1 - wa, db = b1 - wb;
#pragma unroll
            for (int j = 0; j < NLMAX; ++j)
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    vsv[j][q] += a1 * er[j].v[q] + b1 * vr[j].v[q];
                    vsw[j][q] += a2 * er[j].v[q] + b2 * vr[j].v[q];
                    const T dk = da * er[j].v[q] + db * vr[j].v[q];
                    dmv += dk * dk;
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
                const T dms = wave_sum_t<T>(dmv);
                if (lane == 0) rec[rl.dm] += (double)dms;
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

// LDS of one compute unit (gfx950)
constexpr size_t LDS_PER_CU = 160 * 1024;

// Kernels that take more than 64 KiB of dynamic LDS opt in to the size.
// Sizes above a compute unit's LDS are refused here, before the runtime
// would record an error that a later hipGetLastError would report.
static hipError_t ensure_dynamic_lds(const void* fn, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    if (bytes > LDS_PER_CU) return hipErrorInvalidValue;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}


// The template instance of the pass for (dtype, config): visits
// f.go<T, VEC, NLMAX, TRL>().  G < 64 implies nl <= ceil(16 / vec) (FP32;
// 8 / vec for FP64); G = 64 (one ball per wave) uses the larger nlmax.  TRL
// tags instances by group width; the group shapes of rows of about a hundred
// elements (FP32: 8 lanes of four 4-wide parts, FP64: 32 lanes of two 2-wide
// parts) have instances of their own with G fixed at compile time, used when
// cfg.spec allows.
template <typename T, int VEC, int NLMAX, class F>
static hipError_t visit_trl(const PassConfig& cfg, F& f) {
    if constexpr (std::is_same<T, float>::value && VEC == 4 && NLMAX == 4)
        if (cfg.spec && cfg.G == 8) return f.template go<T, VEC, NLMAX, 8>();
    if constexpr (std::is_same<T, double>::value && VEC == 2 && NLMAX == 2)
        if (cfg.spec && cfg.G == 32) return f.template go<T, VEC, NLMAX, 32>();
    if (cfg.G >= 16) return f.template go<T, VEC, NLMAX, 1>();
    if (cfg.G >= 4) return f.template go<T, VEC, NLMAX, 3>();
    return f.template go<T, VEC, NLMAX, 9>();
}

template <typename T, int VEC, class F>
static hipError_t visit_vec(const PassConfig& cfg, F& f) {
    if (cfg.G < 64) {
        if (cfg.nlmax == 2) return visit_trl<T, VEC, 2>(cfg, f);
        if (cfg.nlmax == 4) return visit_trl<T, VEC, 4>(cfg, f);
        if constexpr (VEC == 4) return visit_trl<T, VEC, 4>(cfg, f);
        if constexpr (VEC == 2) return visit_trl<T, VEC, 8>(cfg, f);
        if (cfg.nlmax == 8) return visit_trl<T, VEC, 8>(cfg, f);
        return visit_trl<T, VEC, 16>(cfg, f);
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
