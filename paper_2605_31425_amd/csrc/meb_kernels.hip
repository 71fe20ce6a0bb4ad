// HIP kernels of libmeb.so for gfx950 (MI355X), apart from the evaluation
// pass: the deterministic reductions of the pass records, the rank-one
// Hessian contraction, the device-side control step of ripALM (Armijo
// decision, relative stopping test, multiplier bookkeeping, FP64 Cholesky
// solve), the screening and feasibility scans, the precision-preparation
// and gather kernels, and the multi-instance step of the server.
#include <algorithm>

#include "meb_device.h"

namespace meb {

// ---------------------------------------------------------------------------
// Rank-one Hessian contraction  sum_{i in mid} coef_i s_i s_i^T  (FP64
// accumulation), tiled T x T over the upper triangle of d x d and split
// over the pass's wave segments of the mid list (no compaction: block y of
// a tile pair walks the mid entries of waves [y W / S, (y + 1) W / S)).
// s_i is recomputed from C and V exactly as the pass computed it.  The last
// of the S blocks of a tile pair to finish sums their partial tiles in
// order and writes the tile of H (Section 4):
//   H_rr = tau/sigma + sigma N_I + sigma/2 N_mid
//   H_rc = sigma/2 sum_mid s_i / ||s_i||
//   H_cc = (tau/sigma + sigma N_I + sum_mid gamma_i) I + sum_mid coef_i s_i s_i^T
// (tile pair 0 also writes the r row and column).
// ---------------------------------------------------------------------------

constexpr int SYRK_KB = 32;     // mid balls staged per step
constexpr int SYRK_SEGS = 1024; // most wave segments one block walks
// Blocks along the mid list per tile pair: the launch provides up to
// SyrkArgs::ksplit of them (enough for about SYRK_BLOCKS blocks in all when
// d is small), and each pass uses one per SYRK_ROWS mid rows, at least
// SYRK_KSPLIT_MIN; the others return at once.  (More blocks for short lists
// -- about 256 in all -- made the benchmark's contractions slower: 12 -> 17 us.)
constexpr int SYRK_KSPLIT_MIN = 8;
constexpr int SYRK_KSPLIT_MAX = 1024;
constexpr int SYRK_BLOCKS = 2048;
constexpr int SYRK_ROWS = 1024;
constexpr int SYRK_MT = 64;     // tile width of the matrix-core contraction
// row stride (elements) of its staged rows: k padded by 16 bytes
template <int MI>
__host__ __device__ constexpr int syrk_ldk() {
    return SYRK_KB + (MI == 0 ? 2 : (MI == 1 ? 4 : 8));
}

int syrk_ksplit(int64_t m, int d, int nwaves) {
    const int64_t nt = (d + 31) / 32;  // pairs of the 32-wide tiling (the 64-wide one has fewer)
    const int64_t pairs = nt * (nt + 1) / 2;
    int64_t ks = std::max<int64_t>(1, SYRK_BLOCKS / pairs);
    ks = std::min<int64_t>(ks, (m + SYRK_ROWS - 1) / SYRK_ROWS);
    ks = std::min<int64_t>(ks, nwaves);
    ks = std::max<int64_t>(ks, SYRK_KSPLIT_MIN);
    return (int)std::min<int64_t>(ks, SYRK_KSPLIT_MAX);
}

// LDS of one contraction block (both arithmetics carve it)
constexpr size_t SYRK_SMEM = 44 * 1024;

// Per-block context: the tile pair, this block's share of the mid list (the
// exclusive prefix of its wave segments' counts in LDS) and the penalty.
struct SyrkCtx {
    int I, J;       // tile row / column (I <= J)
    int ks;         // blocks along the mid list in this pass
    int w0, nseg;   // this block's wave segments
    int total;      // mid entries in them
    double sig;
    bool have_dir;
};

// Returns false when the contraction is skipped or the run is done.
__device__ __forceinline__ bool syrk_prologue(const SyrkArgs& a, int bx, int by, int32_t* pref, SyrkCtx& c) {
    __shared__ int wtot[256 / WAVE];
    double* st = a.state;
    const int mode = (int)st[S_MODE];
    if (mode != PM_EVAL && mode != PM_MULT) return false;  // done, or a Newton system being re-solved
    const RecLayout rl = a.rl;
    const double* red = a.red;
    c.have_dir = (mode == PM_EVAL) && st[S_HAVE_DIR] != 0.0;
    const double K = red[rl.nm];
    // skipped: in a line-search pass with many rows, and while the
    // first-order inner solver runs (no Newton system)
    const bool skip = (c.have_dir && K > a.skip_k) || (mode == PM_EVAL && st[S_FO_ON] != 0.0);
    if (bx == 0 && by == 0 && threadIdx.x == 0) st[S_HSKIP] = skip ? 1.0 : 0.0;
    if (skip) return false;
    // every block derives the same split from K
    const double want = ceil(K / (double)SYRK_ROWS);
    c.ks = want >= (double)a.ksplit ? a.ksplit : max((int)want, SYRK_KSPLIT_MIN);
    if (by >= c.ks) return false;
    c.sig = (mode == PM_MULT) ? st[S_SIGMA_NEXT] : st[S_SIGMA];
    int p = bx, I = 0;
    while (p >= a.ntile - I) {
        p -= a.ntile - I;
        ++I;
    }
    c.I = I;
    c.J = I + p;
    const int per = (a.nwaves + c.ks - 1) / c.ks;
    c.w0 = by * per;
    const int w1 = min(a.nwaves, c.w0 + per);
    c.nseg = max(0, w1 - c.w0);
    // exclusive prefix of the segment counts: each thread sums a run of
    // four, the runs are scanned within each wave by shuffles and across the
    // four waves through LDS, then each run is written out
    const int q0 = threadIdx.x * 4;
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    int cnt[4], t = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        cnt[u] = (q0 + u < c.nseg) ? a.mid_cnt[c.w0 + q0 + u] : 0;
        t += cnt[u];
    }
    int inc = t;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const int y = __shfl_up(inc, o, WAVE);
        if (lane >= o) inc += y;
    }
    if (lane == WAVE - 1) wtot[wv] = inc;
    __syncthreads();
    int before = 0;
    for (int q = 0; q < wv; ++q) before += wtot[q];
    int run = before + inc - t;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (q0 + u <= c.nseg) pref[q0 + u] = run;
        run += cnt[u];
    }
    // with 4 * 256 segments the closing entry lies past the last run
    if (threadIdx.x == blockDim.x - 1 && c.nseg == 4 * (int)blockDim.x) pref[c.nseg] = run;
    __syncthreads();
    c.total = pref[c.nseg];
    return true;
}

// mid entry e of this block's segments: ball index and coefficient
__device__ __forceinline__ void syrk_entry(const SyrkArgs& a, const SyrkCtx& c, const int32_t* pref, int e,
                                           int32_t& id, double& cf) {
    int lo = 0, hi = c.nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pref[mid] <= e)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int64_t pos = (int64_t)(c.w0 + lo) * a.bw + (e - pref[lo]);
    id = a.mid_idx[pos];
    cf = a.mid_coef[pos];
}

// s_i(col) = (c_i - y)(col) + v_i(col) / sigma, in the working precision,
// exactly as the pass formed it
template <typename T>
__device__ __forceinline__ T syrk_s(const SyrkArgs& a, const T* C, const T* U, const T* V, int64_t i, int col, T yc,
                                    T inv) {
    const T ek = C[i * a.d + col] - yc;
    const T vk = (V && U && U[i] != T(0)) ? V[i * a.d + col] : T(0);
    return ek + vk * inv;
}

// The last of the c.ks blocks of a tile pair sums their partial tiles in
// order and writes its part of H (tile pair 0 also the r row and column).
__device__ __forceinline__ void syrk_finish(const SyrkArgs& a, const SyrkCtx& c, int bx, int npairs) {
    __shared__ int s_last;
    const int T = a.tile;
    published();
    __syncthreads();
    if (threadIdx.x == 0) s_last = arrive(&a.sync[SYNC_SYRK + bx]) == c.ks - 1;
    __syncthreads();
    if (!s_last) return;
    double* st = a.state;
    const RecLayout rl = a.rl;
    const double* red = a.red;
    const int d = a.d;
    const double tau = st[S_TAU];
    const double base = tau / c.sig + c.sig * red[rl.ni];
    const int n1 = d + 1;
    double* H = st + a.sl.H;
    // only the entries of the tile that lie inside d x d
    const int rows = min(T, d - c.I * T), cols = min(T, d - c.J * T);
    const size_t stride = (size_t)npairs * T * T;
    for (int e2 = threadIdx.x; e2 < rows * cols; e2 += blockDim.x) {
        const int r = e2 / cols, cc = e2 % cols;
        const int k = c.I * T + r, l = c.J * T + cc;
        const double* src = a.out + (size_t)bx * T * T + r * T + cc;
        double v = 0.0;
        // the partial tiles' loads in flight together: 8 at a time for the
        // usual split, 32 for long lists (past c.ks: the last one again, not
        // added)
        if (c.ks <= 8) {
            double part[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) part[u] = ld_shared_dev(src + (size_t)(u < c.ks ? u : c.ks - 1) * stride);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (u < c.ks) v += part[u];
        } else {
            for (int ks = 0; ks < c.ks; ks += 32) {
                double part[32];
#pragma unroll
                for (int u = 0; u < 32; ++u) {
                    const int k = ks + u < c.ks ? ks + u : c.ks - 1;
                    part[u] = ld_shared_dev(src + (size_t)k * stride);
                }
#pragma unroll
                for (int u = 0; u < 32; ++u)
                    if (ks + u < c.ks) v += part[u];
            }
        }
        if (k == l) v += base + red[rl.sg];
        H[(1 + k) * n1 + 1 + l] = v;
        if (c.I != c.J) H[(1 + l) * n1 + 1 + k] = v;
    }
    if (bx == 0) {
        for (int k = threadIdx.x; k < n1; k += blockDim.x) {
            if (k == 0) {
                H[0] = base + 0.5 * c.sig * red[rl.nm];
            } else {
                const double v = 0.5 * c.sig * red[rl.sw + k - 1];
                H[k] = v;
                H[k * n1] = v;
            }
        }
    }
    if (threadIdx.x == 0) a.sync[SYNC_SYRK + bx] = 0;
}

// ---------------------------------------------------------------------------
// Rank-one Hessian contraction  sum_{i in mid} coef_i s_i s_i^T, tiled over
// the upper triangle of d x d and split over the pass's wave segments of the
// mid list (no compaction: block y of a tile pair walks the mid entries of
// waves [y W / S, (y + 1) W / S)).  s_i is recomputed from C and V exactly as
// the pass computed it.  The last of the S blocks of a tile pair to finish
// sums their partial tiles in order and writes the tile of H (Section 4):
//   H_rr = tau/sigma + sigma N_I + sigma/2 N_mid
//   H_rc = sigma/2 sum_mid s_i / ||s_i||
//   H_cc = (tau/sigma + sigma N_I + sum_mid gamma_i) I + sum_mid coef_i s_i s_i^T
// Two arithmetics: FP64 FMAs from LDS (32 x 32 tiles, 2 x 2 outputs per
// thread), or matrix cores (64 x 64 tiles, a 32 x 32 quadrant per wave) with
// FP64, FP32 or BF16 inputs (FP32 accumulation for the latter two within a
// block's share of the list; the shares are summed in FP64).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void syrk_vec_body(const SyrkArgs& a, int bx, int by, int npairs, unsigned char* smem) {
    constexpr int TT = 32;
    static_assert(2 * SYRK_KB * (TT + 1) * 8 + SYRK_KB * 12 + 4 * (SYRK_SEGS + 1) <= SYRK_SMEM,
                  "staging fits the block's LDS");
    typedef double Row[TT + 1];
    Row* sI = reinterpret_cast<Row*>(smem);
    Row* sJ = sI + SYRK_KB;
    double* cf = reinterpret_cast<double*>(sJ + SYRK_KB);
    int32_t* ix = reinterpret_cast<int32_t*>(cf + SYRK_KB);
    int32_t* pref = ix + SYRK_KB;
    SyrkCtx c;
    if (!syrk_prologue(a, bx, by, pref, c)) return;
    const double* st = a.state;
    const StateLayout sl = a.sl;
    const int d = a.d;
    const T inv = (T)(1.0 / c.sig);
    const T* C = static_cast<const T*>(a.C);
    const T* V = static_cast<const T*>(a.V);
    const T* U = static_cast<const T*>(a.U);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[2][2] = {{0, 0}, {0, 0}};
    for (int kb = 0; kb < c.total; kb += SYRK_KB) {
        const int nk = min(SYRK_KB, c.total - kb);
        __syncthreads();
        if (threadIdx.x < SYRK_KB) {
            int32_t id = 0;
            double cv = 0.0;
            if (threadIdx.x < nk) syrk_entry(a, c, pref, kb + threadIdx.x, id, cv);
            ix[threadIdx.x] = id;
            cf[threadIdx.x] = cv;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < SYRK_KB * TT * 2; e += 256) {
            const int which = e / (SYRK_KB * TT);
            const int r = (e / TT) % SYRK_KB;
            const int cc = e % TT;
            const int col = (which ? c.J : c.I) * TT + cc;
            double v = 0.0;
            if (r < nk && col < d) {
                const T yc = (T)(st[sl.xb + 1 + col] + (c.have_dir ? st[sl.dir + 1 + col] : 0.0));
                v = (double)syrk_s<T>(a, C, U, V, ix[r], col, yc, inv);
            }
            if (which)
                sJ[r][cc] = v;
            else
                sI[r][cc] = v;
        }
        __syncthreads();
        for (int r = 0; r < nk; ++r) {
            const double cr = cf[r];
            const double a0 = sI[r][ty], a1 = sI[r][ty + 16];
            const double b0 = sJ[r][tx] * cr, b1 = sJ[r][tx + 16] * cr;
            acc[0][0] += a0 * b0;
            acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0;
            acc[1][1] += a1 * b1;
        }
    }
    double* out = a.out + ((size_t)by * npairs + bx) * TT * TT;
    st_shared_dev(out + ty * TT + tx, acc[0][0]);
    st_shared_dev(out + ty * TT + tx + 16, acc[0][1]);
    st_shared_dev(out + (ty + 16) * TT + tx, acc[1][0]);
    st_shared_dev(out + (ty + 16) * TT + tx + 16, acc[1][1]);
    syrk_finish(a, c, bx, npairs);
}

typedef double syrk_d4 __attribute__((ext_vector_type(4)));
typedef float syrk_f4 __attribute__((ext_vector_type(4)));
typedef __bf16 syrk_bf8 __attribute__((ext_vector_type(8)));

// Matrix-core operand types: MI = 0 FP64, 1 FP32, 2 BF16
template <int MI>
struct SyrkMM;
template <>
struct SyrkMM<0> {
    typedef double in_t;
    typedef syrk_d4 acc_t;
};
template <>
struct SyrkMM<1> {
    typedef float in_t;
    typedef syrk_f4 acc_t;
};
template <>
struct SyrkMM<2> {
    typedef __bf16 in_t;
    typedef syrk_f4 acc_t;
};

// One 16 x 16 block product over the SYRK_KB staged k of a chunk.  Staged
// rows are k-contiguous: sA[row * LDK + k], sB[col * LDK + k].  Operand lane
// layouts (16 x 16 x 4 FP64 / FP32: lane l supplies A(row l % 16, k l / 16)
// and B(k l / 16, col l % 16); 16 x 16 x 32 BF16: A(row l % 16, k 8 (l / 16)
// .. + 7) and B alike); k within a chunk is split among the four lane groups
// so each lane reads contiguous k.
template <int MI, int LDK>
__device__ __forceinline__ typename SyrkMM<MI>::acc_t syrk_mm_block(const typename SyrkMM<MI>::in_t* sA,
                                                                     const typename SyrkMM<MI>::in_t* sB,
                                                                     typename SyrkMM<MI>::acc_t acc) {
    const int lane = lane_id(), g = lane / 16, l16 = lane % 16;
    const typename SyrkMM<MI>::in_t* pa = sA + l16 * LDK + g * (SYRK_KB / 4);
    const typename SyrkMM<MI>::in_t* pb = sB + l16 * LDK + g * (SYRK_KB / 4);
    if constexpr (MI == 0) {
#pragma unroll
        for (int s2 = 0; s2 < SYRK_KB / 4; ++s2) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[s2], pb[s2], acc, 0, 0, 0);
    } else if constexpr (MI == 1) {
#pragma unroll
        for (int s2 = 0; s2 < SYRK_KB / 4; ++s2) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[s2], pb[s2], acc, 0, 0, 0);
    } else {
        static_assert(SYRK_KB == 32, "one BF16 block product covers 32 k");
        const syrk_bf8 va = *reinterpret_cast<const syrk_bf8*>(pa);
        const syrk_bf8 vb = *reinterpret_cast<const syrk_bf8*>(pb);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, acc, 0, 0, 0);
    }
    return acc;
}

template <typename T, int MI>
__device__ __forceinline__ void syrk_mm_body(const SyrkArgs& a, int bx, int by, int npairs, unsigned char* smem) {
    typedef typename SyrkMM<MI>::in_t IT;
    typedef typename SyrkMM<MI>::acc_t AT;
    constexpr int TT = SYRK_MT;
    constexpr int LDK = syrk_ldk<MI>();
    static_assert(2 * TT * LDK * sizeof(IT) + 2 * TT * sizeof(T) + SYRK_KB * 12 + 4 * (SYRK_SEGS + 1) <= SYRK_SMEM,
                  "staging fits the block's LDS");
    IT* sA = reinterpret_cast<IT*>(smem);          // tile I columns x k
    IT* sB = sA + TT * LDK;                        // tile J columns x k, times coef
    T* yI = reinterpret_cast<T*>(sB + TT * LDK);   // y on the tile's columns
    T* yJ = yI + TT;
    double* cf = reinterpret_cast<double*>(yJ + TT);
    int32_t* ix = reinterpret_cast<int32_t*>(cf + SYRK_KB);
    int32_t* pref = ix + SYRK_KB;
    SyrkCtx c;
    if (!syrk_prologue(a, bx, by, pref, c)) return;
    const double* st = a.state;
    const StateLayout sl = a.sl;
    const int d = a.d;
    const T inv = (T)(1.0 / c.sig);
    const T* C = static_cast<const T*>(a.C);
    const T* V = static_cast<const T*>(a.V);
    const T* U = static_cast<const T*>(a.U);
    for (int e = threadIdx.x; e < 2 * TT; e += blockDim.x) {
        const int col = (e < TT ? c.I : c.J) * TT + (e % TT);
        const T y = col < d ? (T)(st[sl.xb + 1 + col] + (c.have_dir ? st[sl.dir + 1 + col] : 0.0)) : T(0);
        if (e < TT)
            yI[e] = y;
        else
            yJ[e - TT] = y;
    }
    const int w = threadIdx.x / WAVE;
    const int qi = w >> 1, qj = w & 1;  // this wave's 32 x 32 quadrant
    AT acc[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[p][q][e] = 0;
    for (int kb = 0; kb < c.total; kb += SYRK_KB) {
        const int nk = min(SYRK_KB, c.total - kb);
        __syncthreads();
        if (threadIdx.x < SYRK_KB) {
            int32_t id = 0;
            double cv = 0.0;
            if (threadIdx.x < nk) syrk_entry(a, c, pref, kb + threadIdx.x, id, cv);
            ix[threadIdx.x] = id;
            cf[threadIdx.x] = cv;
        }
        __syncthreads();
        // stage s on the two tiles' columns: thread -> (k, column), columns
        // fastest so that the row reads coalesce
        for (int e = threadIdx.x; e < SYRK_KB * 2 * TT; e += blockDim.x) {
            const int k = e / (2 * TT), cc = e % (2 * TT);
            const bool isJ = cc >= TT;
            const int cl = isJ ? cc - TT : cc;
            const int col = (isJ ? c.J : c.I) * TT + cl;
            T v = T(0);
            if (k < nk && col < d) {
                v = syrk_s<T>(a, C, U, V, ix[k], col, isJ ? yJ[cl] : yI[cl], inv);
                if (isJ) v = (T)((double)v * cf[k]);
            }
            (isJ ? sB : sA)[cl * LDK + k] = (IT)v;
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
                acc[p][q] = syrk_mm_block<MI, LDK>(sA + (qi * 32 + 16 * p) * LDK, sB + (qj * 32 + 16 * q) * LDK,
                                                    acc[p][q]);
    }
    // partial tile: result slot e of lane l of block (p, q) is column l % 16
    // and row 4 e + l / 16 (FP64) or 4 (l / 16) + e (FP32, BF16) of that
    // 16 x 16 block
    double* out = a.out + ((size_t)by * npairs + bx) * TT * TT;
    const int lane = lane_id(), g = lane / 16, l16 = lane % 16;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rr = (MI == 0) ? 4 * e + g : 4 * g + e;
                const int r = qi * 32 + 16 * p + rr, cl = qj * 32 + 16 * q + l16;
                st_shared_dev(out + r * TT + cl, (double)acc[p][q][e]);
            }
    syrk_finish(a, c, bx, npairs);
}

template <typename T>
__device__ __forceinline__ void syrk_dispatch(const SyrkArgs& a, int bx, int by, int npairs, unsigned char* smem) {
    if (a.mm == SYRK_MFMA_F64)
        syrk_mm_body<T, 0>(a, bx, by, npairs, smem);
    else if (a.mm == SYRK_MFMA_F32)
        syrk_mm_body<T, 1>(a, bx, by, npairs, smem);
    else if (a.mm == SYRK_MFMA_BF16)
        syrk_mm_body<T, 2>(a, bx, by, npairs, smem);
    else
        syrk_vec_body<T>(a, bx, by, npairs, smem);
}

template <typename T>
__global__ __launch_bounds__(256) void syrk_kernel(SyrkArgs a) {
    __shared__ __align__(16) unsigned char smem[SYRK_SMEM];
    syrk_dispatch<T>(a, blockIdx.x, blockIdx.y, gridDim.x, smem);
}

hipError_t launch_syrk(const SyrkArgs& a, hipStream_t s) {
    const int pairs = a.ntile * (a.ntile + 1) / 2;
    if ((a.nwaves + SYRK_KSPLIT_MIN - 1) / SYRK_KSPLIT_MIN > SYRK_SEGS || a.ksplit < SYRK_KSPLIT_MIN ||
        a.ksplit > SYRK_KSPLIT_MAX || pairs > SYNC_LEN - SYNC_SYRK)
        return hipErrorInvalidValue;
    if (a.tile != syrk_tile_of(a.mm)) return hipErrorInvalidValue;
    dim3 grid(pairs, a.ksplit);
    if (a.dtype == 0)
        hipLaunchKernelGGL(syrk_kernel<double>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(syrk_kernel<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// g of a single evaluation (meb_al_eval), and a copy of the H the
// contraction assembled in the state.
__global__ __launch_bounds__(256) void eval_outputs_kernel(const double* st, StateLayout sl, RecLayout rl,
                                                           const double* red, double sigma, double tau, int d,
                                                           const double* y, const double* xbar, double* out_g,
                                                           double* out_H) {
    const int n1 = d + 1;
    for (int k = threadIdx.x + blockIdx.x * blockDim.x; k < n1 * n1; k += blockDim.x * gridDim.x) {
        if (out_H) out_H[k] = st[sl.H + k];
        if (out_g && k < n1) {
            const double sv = (k == 0) ? red[rl.su] : red[rl.sv + k - 1];
            out_g[k] = (k == 0 ? 1.0 : 0.0) - sv + (tau / sigma) * (y[k] - xbar[k]);
        }
    }
}

hipError_t launch_eval_outputs(const double* state, StateLayout sl, RecLayout rl, const double* red, double sigma,
                               double tau, const double* y, const double* xbar, double* out_g, double* out_H,
                               hipStream_t s) {
    const int n1 = sl.n1;
    const int blocks = (n1 * n1 + 255) / 256;
    hipLaunchKernelGGL(eval_outputs_kernel, dim3(blocks), dim3(256), 0, s, state, sl, rl, red, sigma, tau, n1 - 1, y,
                       xbar, out_g, out_H);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cholesky solve of H y = b in one workgroup (FP64).  The matrix is held in
// LDS when it fits (n <= 143 on gfx950), otherwise it is factorized in
// place in global memory.
// ---------------------------------------------------------------------------

// Cholesky solve of M y = b for SPD M (row-major, leading dimension ld >= n,
// in LDS), blocked right-looking with CB-column panels.  The sequential parts
// -- each CB x CB diagonal block and the triangular sub-solves -- run in the
// registers of wave 0 (lane r holds row r of the block) and broadcast with
// readlane instead of round trips through LDS; the panel below a block and
// the trailing update use every thread, with three block barriers per panel.
// Pivots use a reciprocal square root refined by two Newton steps instead of
// an IEEE divide and square root.  rd receives 1 / L_jj.  Returns -1 if a
// pivot is not positive.
constexpr int CB = 16;

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// 1 / sqrt(x) to double precision for x > 0: the hardware estimate
// (relative error about 2^-24) refined by one third-order step,
// y (1 + e / 2 + 3 e^2 / 8) with e = 1 - x y^2.
__device__ __forceinline__ double rsqrt_f64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

__device__ __forceinline__ int chol_solve_lds(int n, int ld, double* M, double* b, double* rd) {
    __shared__ int bad;
    const int tid = threadIdx.x, nth = blockDim.x;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j0 = 0; j0 < n; j0 += CB) {
        const int nb = min(CB, n - j0);
        if (tid < WAVE) {
            const int r = tid;
            double a[CB];
#pragma unroll
            for (int k = 0; k < CB; ++k) a[k] = (r < nb && k <= r) ? M[(j0 + r) * ld + j0 + k] : 0.0;
            int fail = 0;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                if (c < nb && !fail) {
                    const double piv = readlane_f64(a[c], c);
                    if (!(piv > 0.0)) {
                        fail = 1;
                    } else {
                        const double il = rsqrt_f64(piv);
                        if (r == c) a[c] = piv * il;
                        if (r > c) a[c] *= il;
                        if (r == 0) rd[j0 + c] = il;
#pragma unroll
                        for (int k = c + 1; k < CB; ++k) {
                            const double lkc = readlane_f64(a[c], k);
                            if (r >= k) a[k] -= a[c] * lkc;
                        }
                    }
                }
            }
            if (fail && r == 0) bad = 1;
            if (r < nb) {
#pragma unroll
                for (int k = 0; k < CB; ++k)
                    if (k <= r) M[(j0 + r) * ld + j0 + k] = a[k];
            }
        }
        __syncthreads();
        if (bad) return -1;
        // panel below the block: L_ib = A_ib L_bb^-T, one row per thread
        for (int i = j0 + nb + tid; i < n; i += nth) {
            double v[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) v[c] = c < nb ? M[i * ld + j0 + c] : 0.0;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                if (c < nb) {
                    double sacc = v[c];
#pragma unroll
                    for (int k = 0; k < c; ++k) sacc -= v[k] * M[(j0 + c) * ld + j0 + k];
                    v[c] = sacc * rd[j0 + c];
                }
            }
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c < nb) M[i * ld + j0 + c] = v[c];
        }
        __syncthreads();
        // trailing lower triangle
        const int rem = n - j0 - nb;
        if (rem > 0) {
            const int tx = tid & 15, ty = tid >> 4, nty = nth >> 4;
            for (int ii = ty; ii < rem; ii += nty) {
                const int i = j0 + nb + ii;
                double li[CB];
#pragma unroll
                for (int c = 0; c < CB; ++c) li[c] = c < nb ? M[i * ld + j0 + c] : 0.0;
                for (int kk = tx; kk <= ii; kk += 16) {
                    const int k = j0 + nb + kk;
                    double acc = 0.0;
#pragma unroll
                    for (int c = 0; c < CB; ++c) acc += li[c] * M[k * ld + j0 + c];
                    M[i * ld + k] -= acc;
                }
            }
        }
        __syncthreads();
    }
    // forward L y = b: block solves in registers of wave 0, then the update
    for (int j0 = 0; j0 < n; j0 += CB) {
        const int nb = min(CB, n - j0);
        if (tid < WAVE) {
            const int r = tid;
            double y = r < nb ? b[j0 + r] : 0.0;
            double lrow[CB];
#pragma unroll
            for (int k = 0; k < CB; ++k) lrow[k] = (r < nb && k < r) ? M[(j0 + r) * ld + j0 + k] : 0.0;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                if (c < nb) {
                    const double yc = readlane_f64(y * rd[j0 + c], c);
                    if (r == c)
                        y = yc;
                    else if (r > c)
                        y -= lrow[c] * yc;
                }
            }
            if (r < nb) b[j0 + r] = y;
        }
        __syncthreads();
        for (int i = j0 + nb + tid; i < n; i += nth) {
            double sacc = b[i];
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c < nb) sacc -= M[i * ld + j0 + c] * b[j0 + c];
            b[i] = sacc;
        }
        __syncthreads();
    }
    // backward L^T x = y from the last block
    const int nblk = (n + CB - 1) / CB;
    for (int bi = nblk - 1; bi >= 0; --bi) {
        const int j0 = bi * CB;
        const int nb = min(CB, n - j0);
        if (tid < WAVE) {
            const int r = tid;
            double x = r < nb ? b[j0 + r] : 0.0;
            double lcol[CB];
#pragma unroll
            for (int k = 0; k < CB; ++k) lcol[k] = (r < nb && k > r && k < nb) ? M[(j0 + k) * ld + j0 + r] : 0.0;
#pragma unroll
            for (int c = CB - 1; c >= 0; --c) {
                if (c < nb) {
                    const double xc = readlane_f64(x * rd[j0 + c], c);
                    if (r == c)
                        x = xc;
                    else if (r < c)
                        x -= lcol[c] * xc;
                }
            }
            if (r < nb) b[j0 + r] = x;
        }
        __syncthreads();
        for (int i = tid; i < j0; i += nth) {
            double sacc = b[i];
#pragma unroll
            for (int c = 0; c < CB; ++c)
                if (c < nb) sacc -= M[(j0 + c) * ld + i] * b[j0 + c];
            b[i] = sacc;
        }
        __syncthreads();
    }
    return 0;
}

// Solve of H x = b (H symmetric positive definite) by an LDL^T
// factorization with the matrix in registers, for n + 1 <= 128 (two rows per
// lane) and 16 waves.  Right-looking, in panels of RCH_B columns; wave p
// owns panel p.  A panel's owner factors it in its own registers -- pivots
// and the multipliers of the panel's later columns are broadcast with
// readlane, no LDS round trip and no block barrier -- and writes the unit
// lower columns of L and the pivots D to LDS (L row-major, ldr columns).
// After one block barrier every later panel takes the rank-RCH_B update
// A(:, c) -= L(:, k) D_k L(c, k) from that copy: per-lane loads of L's rows
// and uniform-address loads of the multipliers L(c, k).  A panel thus costs
// one barrier, and the critical path is the next owner's update and
// factorization; that wave runs at raised priority meanwhile.
//
// The right-hand side rides along as row n: factoring [H b; b^T *] leaves
// l = D^-1 L^-1 b in row n of L, and x solves the unit triangular system
// L^T x = l, which wave 0 does four rows at a time.  The last panel is
// padded to RCH_B columns; entries of L above the diagonal are stored as 0,
// and no result reads the padding.  A pivot that is not positive sets a
// flag: the factorization still runs its fixed sequence of barriers and
// the solve returns -1.
constexpr int RCH_B = 8;        // panel width
constexpr int RCH_WAVES = 16;   // waves of the calling block
constexpr int RCH_MAX_N = 127;  // n + 1 rows in two halves of 64 lanes

__host__ __device__ inline int rch_ldr(int n) { return (n + RCH_B - 1) / RCH_B * RCH_B + 2; }
// doubles of LDS: L with the right-hand-side row, then D (padded)
__host__ __device__ inline size_t rch_lds_doubles(int n) {
    return (size_t)(n + 1) * rch_ldr(n) + (n + RCH_B - 1) / RCH_B * RCH_B;
}
__host__ __device__ inline bool rch_fits(int n, int threads) {
    return n >= 1 && n <= RCH_MAX_N && threads == RCH_WAVES * WAVE;
}

// 1 / x to double precision for x > 0: the hardware estimate refined by one
// third-order step, y (1 + e + e^2) with e = 1 - x y.
__device__ __forceinline__ double rcp_f64(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, fma(e, e, e), y);
}

// Factor one panel held as a[j][h] = A(64 h + lane, c0 + j).  LOW: the
// panel's columns lie below 64, so pivots sit in half 0 and both halves
// carry rows below the diagonal; otherwise only half 1 does.  Columns at or
// past n are padding.  Leaves the unit lower columns of L in a, lane j of
// the wave receives the pivot D of the panel's column j, and the pivot
// failure flag is returned.
//
// Latency: a readlane round trip costs several dependent FP64 operations,
// so each column broadcasts all its entries in the panel's rows at once,
// unscaled, and the later columns are updated with the unscaled column
// times r / D; the column is scaled afterwards, off the path to the next
// pivot.
template <bool LOW>
__device__ __forceinline__ bool rch_factor(double (&a)[RCH_B][2], int c0, int n, double* d_lane) {
    const int lane = lane_id();
    bool bad = false;
    double dv = 0.0;
#pragma unroll
    for (int j = 0; j < RCH_B; ++j) {
        const int c = c0 + j;
        double r[RCH_B];
#pragma unroll
        for (int j2 = j; j2 < RCH_B; ++j2)
            r[j2] = LOW ? readlane_f64(a[j][0], c0 + j2) : readlane_f64(a[j][1], c0 + j2 - 64);
        bad |= (c < n) && !(r[j] > 0.0);
        const double piv = c < n ? r[j] : 1.0;
        const double id = rcp_f64(piv);
#pragma unroll
        for (int j2 = j + 1; j2 < RCH_B; ++j2) {
            const double m = r[j2] * id;
            if (LOW) a[j2][0] -= a[j][0] * m;
            a[j2][1] -= a[j][1] * m;
        }
        if (LOW) a[j][0] *= id;
        a[j][1] *= id;
        dv = lane == j ? piv : dv;
    }
    *d_lane = dv;
    return bad;
}

// Write a factored panel to L (rows 0..n; entries above the diagonal as 0).
template <bool LOW>
__device__ __forceinline__ void rch_store(const double (&a)[RCH_B][2], int c0, int n, double* Lr, int ldr) {
    const int lane = lane_id();
#pragma unroll
    for (int h = LOW ? 0 : 1; h < 2; ++h) {
        const int row = 64 * h + lane;
        if (row <= n) {
#pragma unroll
            for (int j = 0; j < RCH_B; j += 2) {
                const double v0 = row >= c0 + j ? a[j][h] : 0.0;
                const double v1 = row >= c0 + j + 1 ? a[j + 1][h] : 0.0;
                *reinterpret_cast<double2*>(Lr + (size_t)row * ldr + c0 + j) = make_double2(v0, v1);
            }
        }
    }
}

// Rank-RCH_B update of the panel at c0q by the factored panel at c0p.  Rows
// past n read row n and columns past n are padding: both only produce values
// that are never read.
template <bool LOWQ>
__device__ __forceinline__ void rch_update(double (&a)[RCH_B][2], int c0q, int c0p, int n, const double* Lr,
                                           int ldr, const double* D) {
    const int lane = lane_id();
    double dp[RCH_B];
#pragma unroll
    for (int j = 0; j < RCH_B; j += 2) {
        const double2 v = *reinterpret_cast<const double2*>(D + c0p + j);
        dp[j] = v.x;
        dp[j + 1] = v.y;
    }
    double lp[2][RCH_B];  // L(row, k) D_k
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int row = 64 * h + lane;
        const int rr = row <= n ? row : n;
#pragma unroll
        for (int j = 0; j < RCH_B; j += 2) {
            double2 v = make_double2(0.0, 0.0);
            if (LOWQ || h == 1) v = *reinterpret_cast<const double2*>(Lr + (size_t)rr * ldr + c0p + j);
            lp[h][j] = v.x * dp[j];
            lp[h][j + 1] = v.y * dp[j + 1];
        }
    }
#pragma unroll
    for (int jq = 0; jq < RCH_B; ++jq) {
        const int rq = c0q + jq <= n ? c0q + jq : n;  // the column's own row
        const double* lrow = Lr + (size_t)rq * ldr + c0p;
        double l[RCH_B];
#pragma unroll
        for (int j = 0; j < RCH_B; j += 2) {
            const double2 v = *reinterpret_cast<const double2*>(lrow + j);
            l[j] = v.x;
            l[j + 1] = v.y;
        }
#pragma unroll
        for (int j = 0; j < RCH_B; ++j) {
            if (LOWQ) a[jq][0] -= lp[0][j] * l[j];
            a[jq][1] -= lp[1][j] * l[j];
        }
    }
}

// H: n x n symmetric, row-major, full (global or LDS); b: n entries, read
// before x (n entries) is written, so they may alias.  Lr: LDS of
// rch_lds_doubles(n), 16-byte aligned.  Requires rch_fits(n, blockDim.x).
__device__ __forceinline__ int chol_solve_regs(int n, const double* H, const double* b, double* x, double* Lr) {
    __shared__ int s_bad;
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int np = (n + RCH_B - 1) / RCH_B;
    const int ldr = rch_ldr(n);
    double* D = Lr + (size_t)(n + 1) * ldr;
    const int c0 = w * RCH_B;
    double a[RCH_B][2];
#pragma unroll
    for (int j = 0; j < RCH_B; ++j) {
        // masks multiply the loaded values, so that no load is sunk into a
        // branch of its own
        const int c = c0 + j;
        const int cc = c < n ? c : 0;
        const double bc = b[cc];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = 64 * h + lane;
            const double hv = H[(size_t)cc * n + (row < n ? row : 0)];
            const double mh = (c < n && row < n) ? 1.0 : 0.0;
            const double mb = (c < n && row == n) ? 1.0 : 0.0;
            a[j][h] = hv * mh + bc * mb;
        }
    }
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    for (int p = 0; p < np; ++p) {
        if (w == p) {
            double dl;
            bool bad;
            if (c0 < 64) {
                bad = rch_factor<true>(a, c0, n, &dl);
                rch_store<true>(a, c0, n, Lr, ldr);
            } else {
                bad = rch_factor<false>(a, c0, n, &dl);
                rch_store<false>(a, c0, n, Lr, ldr);
            }
            if (lane < RCH_B) D[c0 + lane] = dl;
            if (bad && lane == 0) s_bad = 1;
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
        if (w > p && w < np) {
            if (w == p + 1) __builtin_amdgcn_s_setprio(2);
            if (c0 < 64)
                rch_update<true>(a, c0, p * RCH_B, n, Lr, ldr, D);
            else
                rch_update<false>(a, c0, p * RCH_B, n, Lr, ldr, D);
        }
    }
    if (s_bad) return -1;
    // L^T x = l (l in row n, L unit lower), by wave 0: x_k = w_k, then
    // w_j -= L_kj x_k for j < k (lane j holds w_j), one row at a time from the
    // bottom; the dependent chain per row is one broadcast and one FMA.  Rows
    // are read in blocks of eight aligned to 8 (one LDS round trip per block,
    // the rows needed first issued first); a block lies wholly above or below
    // row 64, so each block knows whether the upper half takes updates.  L
    // above the diagonal is 0 (the diagonal itself only changes w_k after x_k
    // has been taken), so no lane needs a mask; lanes past n only compute
    // values that are never read.
    if (w == 0) {
        const double* yr = Lr + (size_t)n * ldr;
        double z0 = lane < n ? yr[lane] : 0.0;
        double z1 = lane + 64 < n ? yr[64 + lane] : 0.0;
        double x0 = 0.0, x1 = 0.0;
        const int i0 = lane < ldr ? lane : 0;  // stays inside a row of L for small n
        for (int kb = (n - 1) & ~7; kb >= 0; kb -= 8) {
            double l0[8], l1[8];
            if (kb >= 64) {
#pragma unroll
                for (int u = 7; u >= 0; --u) {
                    const int kr = kb + u < n ? kb + u : n - 1;
                    const double* row = Lr + (size_t)kr * ldr;
                    l0[u] = row[i0];
                    l1[u] = row[64 + lane];  // n > 64: inside L
                }
#pragma unroll
                for (int u = 7; u >= 0; --u) {
                    const int k = kb + u;
                    if (k < n) {
                        const double xk = readlane_f64(z1, k - 64);
                        x1 = lane + 64 == k ? xk : x1;
                        z0 -= l0[u] * xk;
                        z1 -= l1[u] * xk;
                    }
                }
            } else {
#pragma unroll
                for (int u = 7; u >= 0; --u) {
                    const int kr = kb + u < n ? kb + u : n - 1;
                    l0[u] = Lr[(size_t)kr * ldr + i0];
                }
#pragma unroll
                for (int u = 7; u >= 0; --u) {
                    const int k = kb + u;
                    if (k < n) {
                        const double xk = readlane_f64(z0, k);
                        x0 = lane == k ? xk : x0;
                        z0 -= l0[u] * xk;
                    }
                }
            }
        }
        if (lane < n) x[lane] = x0;
        if (lane + 64 < n) x[64 + lane] = x1;
    }
    __syncthreads();
    return 0;
}

// leading dimension of the LDS copy: odd, so that consecutive rows fall in
// different LDS banks
__host__ __device__ inline int chol_ld(int n) { return n | 1; }

// ---------------------------------------------------------------------------
// Blocked Cholesky solve for n above what LDS holds, the matrix in global
// memory (where it stays in L2).  Right-looking in panels of BCH_NB columns:
//   1. one wave factors the diagonal block in registers (lane r holds row
//      r); the right-hand side rides along as one more row (lane BCH_NB), so
//      the forward substitution L y = b happens inside the factorization;
//   2. every row below the block solves x L_D^T = a by substitution against
//      L_D in LDS, stores the panel row and subtracts the row's share of the
//      forward substitution from its entry of b;
//   3. the trailing lower triangle takes the rank-BCH_NB update
//      A_ij -= sum_k L_ik L_jk in 32 x 32 tiles, one tile per wave at a time,
//      on FP64 matrix cores (16 x 16 x 4 blocks).
// Then the back substitution L^T x = y runs block by block from the bottom.
// Only the lower triangle is written; the upper triangle keeps A (the
// breakdown guard restores the lower triangle from it).  Two drivers: one
// workgroup of 8 waves (chol_solve_blocked), or one launch per phase across
// many workgroups (the mchol kernels below) for the largest systems.
// ---------------------------------------------------------------------------
constexpr int BCH_NB = MCHOL_NB;
constexpr int BCH_LD = BCH_NB + 2;  // LDS row stride of L_D (doubles, 16-byte rows)
__host__ __device__ constexpr int bch_lds_doubles() { return BCH_NB * BCH_LD + BCH_NB; }

typedef double bch_d4 __attribute__((ext_vector_type(4)));

// FP64 16 x 16 x 4 block product: lane l supplies A(row l % 16, k l / 16) and
// B(k l / 16, col l % 16); result slot q of lane l is D(row 4 q + l / 16,
// col l % 16) (the FP32 and BF16 forms place row 4 (l / 16) + q there).
__device__ __forceinline__ bch_d4 mfma_f64_16x16x4(double a, double b, bch_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Step 1 for the block at kb (nb columns), by one whole wave: lane r < nb
// loads row r of the block from M, lane BCH_NB the right-hand side bsrc[0,
// nb).  On return a[] holds this lane's row of L_D (zero above the
// diagonal), or y_D on the right-hand-side lane; L_D is also in lrow
// (row-major, BCH_LD stride) and 1 / L_D(j, j) in dinv.  Returns true (on
// every lane) if a pivot was not positive.
template <bool ALLSTEPS>
__device__ __forceinline__ bool bch_diag(int n, int kb, int nb, const double* M, const double* bsrc, double* lrow,
                                         double* dinv, double (&a)[BCH_NB]) {
    const int lane = lane_id();
    const bool is_row = lane < nb;
    const bool is_rhs = lane == BCH_NB;
    // every lane loads from a valid address (its row, the right-hand side, or
    // row 0 of the block) and keeps what it needs: loads under a condition
    // would be issued one at a time
    const double* src = is_rhs ? bsrc : M + (size_t)(kb + (is_row ? lane : 0)) * n + kb;
#pragma unroll
    for (int c = 0; c < BCH_NB; ++c) {
        const double v = src[c < nb ? c : nb - 1];
        a[c] = ((is_row & (c <= lane)) | (is_rhs & (c < nb))) ? v : 0.0;
    }
    // ALLSTEPS: every step runs (no branch on nb), so that each step's LDS
    // reads are issued together; a guarded read is issued and waited for on
    // its own.  Steps j >= nb find a zero pivot on a lane that holds no row,
    // count it as no failure and change nothing that is used: rows of lrow
    // beyond nb stay zero, dinv beyond nb is one.  Without ALLSTEPS the steps
    // and reads beyond nb are skipped (fewer registers where the factorization
    // shares a kernel with other phases).
    bool bad = false;
    double dv = 0.0;
#pragma unroll
    for (int j = 0; j < BCH_NB; ++j) {
        if (!ALLSTEPS && j >= nb) continue;
        const double piv = readlane_f64(a[j], j);
        bad = bad || ((j < nb) & !(piv > 0.0));
        const double inv = rsqrt_f64(piv > 0.0 ? piv : 1.0);
        // column j of L: lanes below the pivot scale, the pivot lane takes
        // sqrt(piv); the rhs lane gets y_j
        a[j] = (lane == j) ? piv * inv : a[j] * inv;
        if (lane == j) dv = inv;
        // broadcast column j through LDS: lrow(r, j) = L(r, j), read back by
        // every lane of the wave
        if (lane < BCH_NB) lrow[lane * BCH_LD + j] = is_row ? a[j] : 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int c = j + 1; c < BCH_NB; ++c) {
            if (ALLSTEPS || c < nb) a[c] = fma(-a[j], lrow[c * BCH_LD + j], a[c]);
        }
    }
    if (lane < BCH_NB) {
#pragma unroll
        for (int c = 0; c < BCH_NB; ++c) {
            if (!is_row || c > lane) a[c] = 0.0;
            lrow[lane * BCH_LD + c] = a[c];
        }
        dinv[lane] = dv;
    }
    return bad;
}

// Step 2 for one row below the block, its entries already in x:
// row[0, nb) <- x with x L_D^T = row; returns the row's share
// sum_c x_c y_c of the forward substitution.
__device__ __forceinline__ double bch_row_solve(double (&x)[BCH_NB], double* row, int nb, const double* lrow,
                                                const double* dinv, const double* yd) {
    // all BCH_NB columns (x_j = 0 for j >= nb: zero rows of L_D beyond nb);
    // one batch of LDS reads per column (the scheduling barrier keeps the
    // compiler from hoisting every column's reads at once, which would spill)
#pragma unroll
    for (int j = 0; j < BCH_NB; ++j) {
        if (j < nb) {
            double sacc = x[j];
#pragma unroll
            for (int c = 0; c < j; ++c) sacc = fma(-x[c], lrow[j * BCH_LD + c], sacc);
            x[j] = sacc * dinv[j];
        }
    }
    double by = 0.0;
#pragma unroll
    for (int c = 0; c < BCH_NB; ++c) {
        const double yv = yd[c < nb ? c : nb - 1];
        by = fma(x[c], c < nb ? yv : 0.0, by);
    }
#pragma unroll
    for (int c = 0; c < BCH_NB; ++c)
        if (c < nb) row[c] = x[c];
    return by;
}

__device__ __forceinline__ double bch_row(double* row, int nb, const double* lrow, const double* dinv,
                                          const double* yd) {
    double x[BCH_NB];
#pragma unroll
    for (int c = 0; c < BCH_NB; ++c) {
        const double v = row[c < nb ? c : nb - 1];
        x[c] = c < nb ? v : 0.0;
    }
    return bch_row_solve(x, row, nb, lrow, dinv, yd);
}

// lower-triangle tile t of T x T tiles (row-major over TI >= TJ)
__device__ __forceinline__ void bch_tile_of(int t, int& TI, int& TJ) {
    TI = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while (TI * (TI + 1) / 2 > t) --TI;
    while ((TI + 1) * (TI + 2) / 2 <= t) ++TI;
    TJ = t - TI * (TI + 1) / 2;
}

// Step 3 for one 32 x 32 tile of the trailing matrix at (i0, j0), by one
// whole wave: A_ij -= sum_{k < nb} L(i, kb + k) L(j, kb + k), lower part.
__device__ __forceinline__ void bch_tile(int n, double* M, int kb, int nb, int i0, int j0) {
    const int lane = lane_id(), g = lane / 16, l16 = lane % 16;
    bch_d4 acc[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = bch_d4{0.0, 0.0, 0.0, 0.0};
    // lane group g covers k in [8 g, 8 g + 8): 8 products of 4 k each, in
    // two halves (fewer operands live at once)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double av[2][4], bv[2][4];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int ri = i0 + 16 * p + l16, rj = j0 + 16 * p + l16;
            const double* pa = M + (size_t)(ri < n ? ri : n - 1) * n + kb;
            const double* pb = M + (size_t)(rj < n ? rj : n - 1) * n + kb;
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) {
                const int k = 8 * g + 4 * h + s2;
                const int kc = k < nb ? k : nb - 1;
                const double va = pa[kc], vb = pb[kc];
                av[p][s2] = ((ri < n) & (k < nb)) ? va : 0.0;
                bv[p][s2] = ((rj < n) & (k < nb)) ? vb : 0.0;
            }
        }
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q) acc[p][q] = mfma_f64_16x16x4(av[p][s2], bv[q][s2], acc[p][q]);
    }
    // the tile's entries are loaded by every lane from a valid address and
    // written back where they belong (a load under a per-lane condition
    // would wait on its own)
    double cv[2][2][4];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = i0 + 16 * p + 4 * e + g, j = j0 + 16 * q + l16;
                cv[p][q][e] = M[(size_t)(i < n ? i : n - 1) * n + (j < n ? j : n - 1)];
            }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = i0 + 16 * p + 4 * e + g, j = j0 + 16 * q + l16;
                if (i < n && j <= i) M[(size_t)i * n + j] = cv[p][q][e] - acc[p][q][e];
            }
}

// Back substitution L^T x = y by one workgroup, blocks from the bottom; b
// (LDS, n) holds y on entry and x on return.
__device__ __forceinline__ void bch_back(int n, const double* M, double* b) {
    const int tid = threadIdx.x, lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int nblk = (n + BCH_NB - 1) / BCH_NB;
    for (int bk = nblk - 1; bk >= 0; --bk) {
        const int kb = bk * BCH_NB, nb = min(BCH_NB, n - kb);
        if (w == 0) {
            // lane r < nb holds column r of L_D (L(c, r), c >= r) and y_r
            double lc[BCH_NB];
#pragma unroll
            for (int c = 0; c < BCH_NB; ++c) {
                const double v = M[(size_t)(kb + (c < nb ? c : nb - 1)) * n + kb + (lane < nb ? lane : nb - 1)];
                lc[c] = ((lane < nb) & (c < nb) & (c >= lane)) ? v : 0.0;
            }
            double y = b[kb + (lane < nb ? lane : nb - 1)];
            if (lane >= nb) y = 0.0;
            // lane r's own diagonal L(r, r) is lc[r]: its reciprocal, formed
            // by every lane at once, keeps the division off the chain
            double dl = 1.0;
#pragma unroll
            for (int c = 0; c < BCH_NB; ++c)
                if (c == lane) dl = lc[c];
            const double rd = 1.0 / dl;
            double xs = 0.0;
#pragma unroll
            for (int j = BCH_NB - 1; j >= 0; --j) {
                if (j < nb) {
                    const double xj = readlane_f64(y, j) * readlane_f64(rd, j);
                    if (lane == j) xs = xj;
                    if (lane < j) y = fma(-lc[j], xj, y);
                }
            }
            if (lane < nb) b[kb + lane] = xs;
        }
        __syncthreads();
        // y_c -= sum_j L(kb + j, c) x_j for the columns left of the block
        for (int c = tid; c < kb; c += blockDim.x) {
            double acc = 0.0;
#pragma unroll 8
            for (int j = 0; j < nb; ++j) acc = fma(M[(size_t)(kb + j) * n + c], b[kb + j], acc);
            b[c] -= acc;
        }
        __syncthreads();
    }
}

// One workgroup (8 waves): M (global, n x n) factored in place, b (LDS, n)
// holds the solution on return.  lw: bch_lds_doubles() of LDS.  Returns -1 if
// a pivot is not positive.
__device__ __forceinline__ int chol_solve_blocked(int n, double* M, double* b, double* lw) {
    __shared__ int s_bad;
    double* lrow = lw;                      // L_D row-major, BCH_NB x BCH_LD
    double* dinv = lw + BCH_NB * BCH_LD;    // 1 / L_D(j, j)
    const int tid = threadIdx.x, lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int nw = blockDim.x / WAVE;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int kb = 0; kb < n; kb += BCH_NB) {
        const int nb = min(BCH_NB, n - kb);
        // ---- 1. diagonal block (wave 0); L_D to M, y_D to b
        if (w == 0) {
            double a[BCH_NB];
            const bool bad = bch_diag<false>(n, kb, nb, M, b + kb, lrow, dinv, a);
            if (lane < nb) {
#pragma unroll
                for (int c = 0; c < BCH_NB; ++c)
                    if (c <= lane) M[(size_t)(kb + lane) * n + kb + c] = a[c];
            }
            if (lane == BCH_NB) {
#pragma unroll
                for (int c = 0; c < BCH_NB; ++c)
                    if (c < nb) b[kb + c] = a[c];
            }
            if (bad && lane == 0) s_bad = 1;
        }
        __syncthreads();
        if (s_bad) return -1;
        // ---- 2. panel rows below the block and their share of L y = b
        for (int i = kb + nb + tid; i < n; i += blockDim.x) b[i] -= bch_row(M + (size_t)i * n + kb, nb, lrow, dinv, b + kb);
        __syncthreads();
        // ---- 3. trailing update, 32 x 32 tiles of the lower triangle
        const int t0 = kb + nb;
        if (t0 < n) {
            const int T = (n - t0 + 31) / 32;
            const int ntiles = T * (T + 1) / 2;
            for (int t = w; t < ntiles; t += nw) {
                int TI, TJ;
                bch_tile_of(t, TI, TJ);
                bch_tile(n, M, kb, nb, t0 + 32 * TI, t0 + 32 * TJ);
            }
        }
        __syncthreads();
    }
    bch_back(n, M, b);
    return 0;
}

// ---------------------------------------------------------------------------
// The same factorization across many workgroups: one launch per phase, so
// that the launches themselves order the phases (no grid-wide barrier):
//   panel kb  one-wave workgroups, one row below the block per lane; every
//             workgroup factors the diagonal block itself (the same
//             arithmetic on the same data, so the same L_D and y_D in each)
//             and subtracts its rows' shares of the forward substitution
//             from b; workgroup 0 keeps L_D and y_D aside (the diagonal block
//             of M is still being read by the others);
//   update kb four tiles of the trailing lower triangle per workgroup, one
//             per wave; workgroup 0 also stores L_D into the diagonal block;
//   back      one workgroup: L^T x = y.
// With `gate`, every launch does nothing unless *gate holds PM_SOLVE (the
// solver state's mode); a pivot that is not positive sets *bad to 1, after
// which the launches do nothing.
// ---------------------------------------------------------------------------
struct MChol {
    int n;
    double* M;           // n x n, row-major; lower triangle overwritten by L
    double* b;           // right-hand side, reduced by the panels' forward updates
    double* y;           // L y = b, block by block
    double* x;           // solution (may alias b or y)
    double* ld;          // BCH_NB x BCH_NB: L_D of the current panel
    double* bad;         // 0 / 1, cleared by the caller
    const double* gate;  // nullable
};

__device__ __forceinline__ bool mchol_live(const MChol& a) {
    return (!a.gate || (int)*a.gate == PM_SOLVE) && *a.bad == 0.0;
}

constexpr int MCHOL_UPDATE_WAVES = 4;

__global__ __launch_bounds__(WAVE) void mchol_panel_kernel(MChol a, int kb) {
    __shared__ double lw[bch_lds_doubles() + BCH_NB];
    if (!mchol_live(a)) return;
    double* lrow = lw;
    double* dinv = lw + BCH_NB * BCH_LD;
    double* yd = dinv + BCH_NB;
    const int n = a.n, nb = min(BCH_NB, n - kb), lane = threadIdx.x;
    // this lane's panel row, loaded before the diagonal block is factored
    // (the loads do not depend on it)
    const int i = kb + nb + blockIdx.x * WAVE + lane;
    double* row = a.M + (size_t)(i < n ? i : n - 1) * n + kb;
    double x[BCH_NB];
#pragma unroll
    for (int c = 0; c < BCH_NB; ++c) {
        const double v = row[c < nb ? c : nb - 1];
        x[c] = ((i < n) & (c < nb)) ? v : 0.0;
    }
    double r[BCH_NB];
    const bool bad = bch_diag<true>(n, kb, nb, a.M, a.b + kb, lrow, dinv, r);
    if (bad) {
        if (blockIdx.x == 0 && lane == 0) *a.bad = 1.0;
        return;
    }
    if (lane == BCH_NB) {
#pragma unroll
        for (int c = 0; c < BCH_NB; ++c) yd[c] = r[c];
    }
    if (blockIdx.x == 0) {
        if (lane < BCH_NB) {
#pragma unroll
            for (int c = 0; c < BCH_NB; ++c) a.ld[lane * BCH_NB + c] = r[c];
        }
        if (lane == BCH_NB) {
#pragma unroll
            for (int c = 0; c < BCH_NB; ++c)
                if (c < nb) a.y[kb + c] = r[c];
        }
    }
    __syncthreads();
    if (i < n) a.b[i] -= bch_row_solve(x, row, nb, lrow, dinv, yd);
}

__global__ __launch_bounds__(WAVE * MCHOL_UPDATE_WAVES) void mchol_update_kernel(MChol a, int kb) {
    if (!mchol_live(a)) return;
    const int n = a.n, nb = min(BCH_NB, n - kb);
    if (blockIdx.x == 0) {
        for (int e = threadIdx.x; e < BCH_NB * BCH_NB; e += blockDim.x) {
            const int r = e / BCH_NB, c = e % BCH_NB;
            if (r < nb && c <= r) a.M[(size_t)(kb + r) * n + kb + c] = a.ld[e];
        }
    }
    const int t0 = kb + nb;
    if (t0 >= n) return;
    const int T = (n - t0 + 31) / 32;
    const int t = blockIdx.x * MCHOL_UPDATE_WAVES + (int)__builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    if (t >= T * (T + 1) / 2) return;
    int TI, TJ;
    bch_tile_of(t, TI, TJ);
    bch_tile(n, a.M, kb, nb, t0 + 32 * TI, t0 + 32 * TJ);
}

// Back substitution L^T x = y across workgroups, one launch per diagonal
// block from the bottom (the launches order the blocks): every workgroup
// loads its threads' column-update operands L(kb + j, c), c < kb, then its
// first wave solves the diagonal block for x_D itself (the same arithmetic in
// each workgroup, so the same x_D), and each thread subtracts its column's
// share, y_c -= sum_j L(kb + j, c) x_j.  Workgroup 0 stores x_D.  y (global)
// holds the forward substitution's result on entry of the first launch.
constexpr int MCHOL_BACK_COLS = 256;  // columns (threads) per workgroup
__global__ __launch_bounds__(MCHOL_BACK_COLS) void mchol_back_kernel(MChol a, int kb) {
    __shared__ double xd[BCH_NB];
    if (!mchol_live(a)) return;
    const int n = a.n, nb = min(BCH_NB, n - kb);
    const int tid = threadIdx.x, lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int c = blockIdx.x * MCHOL_BACK_COLS + tid;
    const int cc = c < kb ? c : 0;
    double pv[BCH_NB];
#pragma unroll
    for (int j = 0; j < BCH_NB; ++j) {
        const double v = a.M[(size_t)(kb + (j < nb ? j : nb - 1)) * n + cc];
        pv[j] = ((c < kb) & (j < nb)) ? v : 0.0;
    }
    if (w == 0) {
        // lane r holds column r of L_D (L(k, r), k >= r) and y_r
        double lc[BCH_NB];
#pragma unroll
        for (int k = 0; k < BCH_NB; ++k) {
            const double v = a.M[(size_t)(kb + (k < nb ? k : nb - 1)) * n + kb + (lane < nb ? lane : nb - 1)];
            lc[k] = ((lane < nb) & (k < nb) & (k >= lane)) ? v : 0.0;
        }
        double y = a.y[kb + (lane < nb ? lane : nb - 1)];
        if (lane >= nb) y = 0.0;
        // lane r's own pivot L(r, r) is lc[r]: its reciprocal, formed by every
        // lane at once, keeps the division off the chain
        double dl = 1.0;
#pragma unroll
        for (int k = 0; k < BCH_NB; ++k)
            if (k == lane) dl = lc[k];
        const double rd = 1.0 / dl;
        double xs = 0.0;
#pragma unroll
        for (int j = BCH_NB - 1; j >= 0; --j) {
            if (j < nb) {
                const double xj = readlane_f64(y, j) * readlane_f64(rd, j);
                if (lane == j) xs = xj;
                if (lane < j) y = fma(-lc[j], xj, y);
            }
        }
        if (lane < BCH_NB) xd[lane] = lane < nb ? xs : 0.0;
        if (blockIdx.x == 0 && lane < nb) a.x[kb + lane] = xs;
    }
    __syncthreads();
    if (c < kb) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < BCH_NB; ++j) acc = fma(pv[j], xd[j], acc);
        a.y[c] -= acc;
    }
}

// the solve's outcome: 0, or -1 if a pivot was not positive
__global__ void mchol_info_kernel(MChol a, int* info) {
    if (threadIdx.x == 0) *info = *a.bad == 0.0 ? 0 : -1;
}

// the back-substitution launches of one solve
hipError_t launch_mchol_back(const MChol& a, hipStream_t s) {
    const int n = a.n;
    for (int kb = (n - 1) / BCH_NB * BCH_NB; kb >= 0; kb -= BCH_NB) {
        const int blocks = std::max(1, (kb + MCHOL_BACK_COLS - 1) / MCHOL_BACK_COLS);
        hipLaunchKernelGGL(mchol_back_kernel, dim3(blocks), dim3(MCHOL_BACK_COLS), 0, s, a, kb);
    }
    return hipGetLastError();
}

// the panel and update launches of one factorization
hipError_t launch_mchol_factor(const MChol& a, hipStream_t s) {
    const int n = a.n;
    for (int kb = 0; kb < n; kb += BCH_NB) {
        const int nb = std::min(BCH_NB, n - kb);
        const int rows = n - kb - nb;
        hipLaunchKernelGGL(mchol_panel_kernel, dim3(std::max(1, (rows + WAVE - 1) / WAVE)), dim3(WAVE), 0, s, a, kb);
        const int T = (rows + 31) / 32;
        const int tiles = T * (T + 1) / 2;
        hipLaunchKernelGGL(mchol_update_kernel,
                           dim3(std::max(1, (tiles + MCHOL_UPDATE_WAVES - 1) / MCHOL_UPDATE_WAVES)),
                           dim3(WAVE * MCHOL_UPDATE_WAVES), 0, s, a, kb);
    }
    return hipGetLastError();
}

hipError_t launch_chol_solve_mwg(int n, double* A, double* b, double* yw, double* ldw, double* badw, int* info,
                                 hipStream_t s) {
    MChol a;
    a.n = n;
    a.M = A;
    a.b = b;
    a.y = yw;
    a.x = b;
    a.ld = ldw;
    a.bad = badw;
    a.gate = nullptr;
    hipError_t e = hipMemsetAsync(badw, 0, sizeof(double), s);
    if (e != hipSuccess) return e;
    e = launch_mchol_factor(a, s);
    if (e != hipSuccess) return e;
    e = launch_mchol_back(a, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mchol_info_kernel, dim3(1), dim3(WAVE), 0, s, a, info);
    return hipGetLastError();
}

constexpr int CHOL_LDS_MAX_N = 140;  // 140 x 141 doubles + vectors < 160 KiB
constexpr int CTRL_THREADS = 1024;
// the control kernel also keeps CTRL_THREADS doubles of scratch in LDS
constexpr int CTRL_CHOL_LDS_MAX_N = 132;  // 1024 + 132 x 133 doubles < 160 KiB
constexpr int CTRL_SHIFT_TRIES = 8;       // raises of the diagonal before an inner solve gives up
// systems above what registers and LDS hold take the blocked factorization
__host__ __device__ inline bool newton_large(int n1) {
    return !(n1 >= 1 && n1 <= RCH_MAX_N) && n1 > CTRL_CHOL_LDS_MAX_N;
}
// kernel instances of the one-workgroup Newton step: the register and LDS
// factorizations, or the blocked one in global memory
enum : int { NK_SMALL = 0, NK_LARGE = 1 };
__host__ __device__ inline int newton_kind(int n1) { return newton_large(n1) ? NK_LARGE : NK_SMALL; }
// threads of each instance: the register factorization needs 16 waves; the
// blocked one keeps more values per lane than 16 waves could hold without
// spilling, and a system below MCHOL_MIN_N needs no more than eight
__host__ __device__ constexpr int newton_threads(int nk) { return nk == NK_LARGE ? 512 : CTRL_THREADS; }
// LDS scratch of the control step: two n1-vectors and the wave sums of a
// block reduction after them, and at least one double per thread
__host__ __device__ inline int ctrl_scratch_doubles(int n1) {
    return CTRL_THREADS > 2 * n1 + 64 ? CTRL_THREADS : 2 * n1 + 64;
}

// THREADS: CTRL_THREADS for the register factorization (it needs 16 waves),
// 512 for the others (more registers per lane for the blocked one)
template <int THREADS>
__global__ __launch_bounds__(THREADS) void chol_solve_kernel(int n, double* A, double* b, int* info) {
    extern __shared__ __align__(16) double sm[];
    int rc = 0;
    if constexpr (THREADS == CTRL_THREADS) {
        if (rch_fits(n, blockDim.x)) rc = chol_solve_regs(n, A, b, b, sm);
    } else if (n <= CHOL_LDS_MAX_N) {
        // LDS: rd (n), rhs (n), M (n x ld)
        const int ld = chol_ld(n);
        double* rd = sm;
        double* bv = sm + n;
        double* M = sm + 2 * n;
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[(e / n) * ld + e % n] = A[e];
        for (int e = threadIdx.x; e < n; e += blockDim.x) bv[e] = b[e];
        __syncthreads();
        rc = chol_solve_lds(n, ld, M, bv, rd);
        for (int e = threadIdx.x; e < n; e += blockDim.x) b[e] = bv[e];
    } else {
        // rhs and solution in LDS, then the blocked factorization's scratch
        double* bv = sm;
        for (int e = threadIdx.x; e < n; e += blockDim.x) bv[e] = b[e];
        __syncthreads();
        rc = chol_solve_blocked(n, A, bv, sm + n);
        for (int e = threadIdx.x; e < n; e += blockDim.x) b[e] = bv[e];
    }
    if (threadIdx.x == 0) *info = rc;
}

hipError_t launch_chol_solve(int n, double* A, double* b, int* info, hipStream_t s) {
    size_t lds = sizeof(double) * (rch_fits(n, CTRL_THREADS) ? rch_lds_doubles(n)
                                   : (size_t)(n <= CHOL_LDS_MAX_N ? (size_t)n * chol_ld(n) + 2 * n
                                                                  : (size_t)n + bch_lds_doubles()));
    if (rch_fits(n, CTRL_THREADS)) {
        hipError_t ea = ensure_dynamic_lds((const void*)chol_solve_kernel<CTRL_THREADS>, lds);
        if (ea != hipSuccess) return ea;
        hipLaunchKernelGGL(chol_solve_kernel<CTRL_THREADS>, dim3(1), dim3(CTRL_THREADS), lds, s, n, A, b, info);
    } else {
        hipError_t ea = ensure_dynamic_lds((const void*)chol_solve_kernel<512>, lds);
        if (ea != hipSuccess) return ea;
        hipLaunchKernelGGL(chol_solve_kernel<512>, dim3(1), dim3(512), lds, s, n, A, b, info);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Control step of the device-resident ripALM / semismooth-Newton loop.
// One workgroup.  Reads the reduced record of the pass that just ran and
// decides what the next pass computes (see the state machine in the host
// solver).  Writes S_MODE = PM_DONE when the run ends.
// ---------------------------------------------------------------------------

// Sums of N values over the block, returned in every thread: each wave sums
// its lanes (symmetric cross-lane steps, so every lane holds the same sum),
// then every thread adds the wave sums from LDS in wave order.  The order is
// fixed, so the result is reproducible; three barriers for all N values.
template <int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N], double* scratch) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = group_sum<double>(v[k], WAVE);
    __syncthreads();  // earlier readers of the scratch are done
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) scratch[w * N + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double t = 0.0;
        for (int q = 0; q < nw; ++q) t += scratch[q * N + k];
        v[k] = t;
    }
    __syncthreads();  // the scratch may be rewritten after this
}

__device__ __forceinline__ double block_sum(double v, double* scratch) {
    double a[1] = {v};
    block_sum_n<1>(a, scratch);
    return a[0];
}

__device__ __forceinline__ void control_body_impl(double* st, double* hs, StateLayout sl, RecLayout rl,
                                                  const double* red) {
    extern __shared__ __align__(16) double sm[];
    double* scratch = sm;  // ctrl_scratch_doubles(n1)
    __shared__ int s_next;  // 0 = continue to EVAL_AT_BASE, 1 = return
    __shared__ double s_eta;
    const int mode = (int)hs[S_MODE];
    if (mode != PM_EVAL && mode != PM_MULT) return;  // done, or a Newton system being re-solved
    const int n1 = sl.n1, d = n1 - 1;
    const double L = hs[S_L];
    const double sigma = hs[S_SIGMA];
    const double tau = hs[S_TAU];
    const double eps = hs[S_EPS];
    double* xb = st + sl.xb;
    double* dir = st + sl.dir;
    double* xbar = st + sl.xbar;
    double* ab = st + sl.ab;
    double* gb = st + sl.gb;
    double* H = st + sl.H;
    double* xprev = st + sl.tmp;  // previous iterate of the accelerated gradient method
    if (threadIdx.x == 0) s_next = 0;
    __syncthreads();
    // the run's first evaluation opens its first inner solve
    if (mode == PM_EVAL && hs[S_NPASS] == 1.0 && hs[S_FO_OUTER] > 0.0) {
        for (int k = threadIdx.x; k < n1; k += blockDim.x) xprev[k] = xb[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            hs[S_FO_ON] = 1.0;
            hs[S_FO_PHASE] = 0.0;
            hs[S_FO_T] = 1.0;
        }
        __syncthreads();
    }

    if (threadIdx.x == 0) {
        hs[S_NPASS] += 1.0;
        hs[S_BYTES] += red[rl.bytes];
        hs[S_SUMK] += red[rl.nm];
        hs[S_MAXK] = fmax(hs[S_MAXK], red[rl.nm]);
        if (hs[S_VERBOSE] >= 2.0)
            printf("[meb] pass %d mode %d K %.0f NI %.0f have_dir %d\n", (int)hs[S_NPASS], mode, red[rl.nm],
                   red[rl.ni], (int)hs[S_HAVE_DIR]);
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
            hs[S_KKT] = kkt;
            hs[S_KKT_P0] = p0;
            hs[S_KKT_P1] = nsv;
            hs[S_KKT_P2] = p2;
            hs[S_KKT_P3] = p3;
            hs[S_KKT_P4] = p4;
            hs[S_K] += 1.0;
            int done = 0;
            if (kkt <= hs[S_TOL]) {
                hs[S_STATUS] = 1.0;
                done = 1;
            } else {
                if (kkt < 0.5 * hs[S_BEST_KKT]) {
                    hs[S_BEST_KKT] = kkt;
                    hs[S_STALL] = 0.0;
                } else {
                    hs[S_STALL] += 1.0;
                }
                if (hs[S_K] >= hs[S_MAX_OUTER] || hs[S_STALL] >= hs[S_STALL_OUTER]) {
                    hs[S_STATUS] = 2.0;
                    done = 1;
                } else if (hs[S_FLOOR] != 0.0) {
                    hs[S_STATUS] = 3.0;
                    done = 1;
                }
            }
            if (done) {
                hs[S_MODE] = (double)PM_DONE;
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
            return;
        }
        // next outer iteration: sigma, proximal center, inner solver
        const bool fo = hs[S_K] < hs[S_FO_OUTER];
        for (int k = threadIdx.x; k < n1; k += blockDim.x) {
            xbar[k] = xb[k];
            if (fo) xprev[k] = xb[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const double sn = hs[S_SIGMA_NEXT];
            hs[S_SIGMA] = sn;
            hs[S_SIGMA_NEXT] = fmin(sn * hs[S_GROWTH], hs[S_SIGMA_MAX]);
            hs[S_J] = 0.0;
            hs[S_HAVE_DIR] = 0.0;
            hs[S_FO_ON] = fo ? 1.0 : 0.0;
            hs[S_FO_PHASE] = 0.0;
            hs[S_FO_T] = 1.0;
            hs[S_FO_STEP] = 0.0;  // re-estimated for the new penalty
        }
        __syncthreads();
        // fall through: the record's evaluation part is at (x_j, w+, sigma_{k+1})
    } else if (hs[S_HAVE_DIR] != 0.0 && hs[S_FO_PHASE] != 0.0) {
        // accelerated gradient method (first-order inner solver for the
        // early outer iterations, Section 4.1): the trials gave Psi at
        // y - eta s g (dir = -s g, y = x_base).  Backtracking on the step:
        // the largest eta with Psi(y + eta dir) <= Psi(y) + eta/2 <g, dir>
        // (the quadratic upper bound with constant 1 / (eta s)); then
        // x = y + eta dir, the momentum step y' = x + (t_k - 1) / t_{k+1}
        // (x - x_prev), restarted (t = 1) when <g(y), x - x_prev> > 0.
        double pdd = 0.0, pdx = 0.0, pxx = 0.0;
        for (int k = threadIdx.x; k < n1; k += blockDim.x) {
            const double dx = xb[k] - xbar[k];
            pdd += dir[k] * dir[k];
            pdx += dir[k] * dx;
            pxx += dx * dx;
        }
        double sums[3] = {pdd, pdx, pxx};
        block_sum_n<3>(sums, scratch);
        const double dd = sums[0], dxd = sums[1], xx = sums[2];
        if (threadIdx.x == 0) {
            const double sg = sigma;
            const double z0 = red[rl.trial + NT - 1];
            const double psi0 = xb[0] + 0.5 * sg * z0 - red[rl.ww] / (2.0 * sg) + tau / (2.0 * sg) * xx;
            const double gd = hs[S_GD];
            const double allow = 8.0 * eps * (fabs(psi0) + 1.0);
            int acc = -1;
            for (int l = 0; l < NT - 1; ++l) {
                const double eta = solver_eta(l);
                const double dpsi = eta * dir[0] + 0.5 * sg * (red[rl.trial + l] - z0) +
                                    tau / (2.0 * sg) * (2.0 * eta * dxd + eta * eta * dd);
                if (dpsi <= 0.5 * eta * gd + allow) {
                    acc = l;
                    break;
                }
            }
            // no trial passed: stay at y with a step shorter than every trial
            const double eta = acc >= 0 ? solver_eta(acc) : 0.0;
            // the step grows again after a full step, so it tracks the local curvature
            hs[S_FO_STEP] *= acc == 0 ? 2.0 : (acc > 0 ? eta : solver_eta(NT - 2) * 0.5);
            s_eta = eta;
            hs[S_NFO] += 1.0;
        }
        __syncthreads();
        const double eta = s_eta;
        // x = y + eta dir; <g(y), x - x_prev> decides the restart
        double prs = 0.0;
        for (int k = threadIdx.x; k < n1; k += blockDim.x) prs += gb[k] * (xb[k] + eta * dir[k] - xprev[k]);
        const double rs = block_sum(prs, scratch);
        __shared__ double s_beta;
        if (threadIdx.x == 0) {
            double t = hs[S_FO_T];
            if (rs > 0.0 || eta == 0.0) t = 1.0;  // restart
            const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
            s_beta = (t - 1.0) / tn;
            hs[S_FO_T] = tn;
            hs[S_FO_PHASE] = 0.0;
            hs[S_HAVE_DIR] = 0.0;
        }
        __syncthreads();
        const double beta = s_beta;
        for (int k = threadIdx.x; k < n1; k += blockDim.x) {
            const double xn = xb[k] + eta * dir[k];
            xb[k] = xn + beta * (xn - xprev[k]);
            xprev[k] = xn;
        }
        return;  // next pass evaluates at the momentum point
    } else if (hs[S_HAVE_DIR] != 0.0) {
        // single-pass Armijo decision along x_base + eta dir
        const double sg = sigma;
        double pdd = 0.0, pdx = 0.0, pxx = 0.0;
        for (int k = threadIdx.x; k < n1; k += blockDim.x) {
            const double dx = xb[k] - xbar[k];
            pdd += dir[k] * dir[k];
            pdx += dir[k] * dx;
            pxx += dx * dx;
        }
        double sums[3] = {pdd, pdx, pxx};
        block_sum_n<3>(sums, scratch);
        const double dd = sums[0], dxd = sums[1], xx = sums[2];
        if (threadIdx.x == 0) {
            double trl[NT];  // the trial sums, loaded together
#pragma unroll
            for (int l = 0; l < NT; ++l) trl[l] = red[rl.trial + l];
            const double z0 = trl[NT - 1];
            const double psi0 = xb[0] + 0.5 * sg * z0 - red[rl.ww] / (2.0 * sg) + tau / (2.0 * sg) * xx;
            const double gd = hs[S_GD];
            const double allow = 8.0 * eps * (fabs(psi0) + 1.0);
            int acc = -1;
            for (int l = 0; l < NT - 1; ++l) {
                const double eta = solver_eta(l);
                const double dpsi = eta * dir[0] + 0.5 * sg * (trl[l] - z0) +
                                    tau / (2.0 * sg) * (2.0 * eta * dxd + eta * eta * dd);
                if (dpsi <= 1e-4 * eta * gd + allow) {
                    acc = l;
                    break;
                }
            }
            if (hs[S_VERBOSE] >= 2.0)
                printf("[meb]   armijo acc=%d gd=%.17g psi0=%.17g dpsi1=%.17g\n", acc, gd, psi0,
                       dir[0] + 0.5 * sg * (trl[0] - z0) + tau / (2.0 * sg) * (2.0 * dxd + dd));
            if (acc == 0 && hs[S_HSKIP] != 0.0) {
                // full step, but its Hessian contraction was skipped:
                // move there and evaluate again
                s_next = 2;
                s_eta = 1.0;
                hs[S_HAVE_DIR] = 0.0;
            } else if (acc == 0) {
                s_next = 0;  // full step: record is at x_base + dir
                hs[S_PSI] = psi0;
            } else {
                double eta;
                if (acc > 0) {
                    eta = solver_eta(acc);
                    hs[S_HAVE_DIR] = 0.0;
                } else {
                    eta = solver_eta(NT - 2);
                    hs[S_LSH] += (double)(NT - 2);
                    if (hs[S_LSH] >= hs[S_MAX_LS]) {
                        hs[S_HAVE_DIR] = 0.0;  // take the smallest step
                    } else {
                        hs[S_GD] = gd * eta;  // retry along the shorter direction
                    }
                }
                s_eta = eta;
                s_next = (acc > 0 || hs[S_HAVE_DIR] == 0.0) ? 2 : 3;
            }
        }
        __syncthreads();
        if (s_next == 0) {
            for (int k = threadIdx.x; k < n1; k += blockDim.x) xb[k] += dir[k];
            __syncthreads();
            if (threadIdx.x == 0) hs[S_HAVE_DIR] = 0.0;
        } else {
            const double eta = s_eta;
            if (s_next == 2) {
                for (int k = threadIdx.x; k < n1; k += blockDim.x) xb[k] += eta * dir[k];
            } else {
                for (int k = threadIdx.x; k < n1; k += blockDim.x) dir[k] *= eta;
            }
            return;  // next pass re-evaluates at x_base (mode EVAL)
        }
        __syncthreads();
    }

    // ---- evaluated at x_j = xb: gradient, stopping test, Newton step
    double pgg = 0.0, pag = 0.0, pxx = 0.0;
    for (int k = threadIdx.x; k < n1; k += blockDim.x) {
        const double dx = xb[k] - xbar[k];
        const double sv = (k == 0) ? red[rl.su] : red[rl.sv + k - 1];
        const double g = (k == 0 ? 1.0 : 0.0) - sv + (tau / hs[S_SIGMA]) * dx;
        gb[k] = g;
        pgg += g * g;
        pag += (ab[k] - xb[k]) * g;
        pxx += dx * dx;
    }
    double sums[3] = {pgg, pag, pxx};
    block_sum_n<3>(sums, scratch);
    const double gg = sums[0], ag = sums[1], xx = sums[2];
    const double sgm = hs[S_SIGMA];
    if (threadIdx.x == 0) {
        hs[S_J] += 1.0;
        hs[S_NINNER] += 1.0;
        // relative-type stopping test of Algorithm 1 in normalized units
        const double sN = sgm * L, tN = tau * L * L;
        const double lhs = 2.0 * sN * fabs(ag / L) + sN * sN * gg;
        const double rhs = hs[S_RHO] * (red[rl.dm] + tN * xx / (L * L));
        const double floor_g = 8.0 * eps * (1.0 + sgm * red[rl.rs]);
        const bool rel = lhs <= rhs;
        const bool flo = sqrt(gg) <= floor_g;
        const bool stop = rel || flo || (hs[S_J] >= hs[S_MAX_INNER]);
        if (hs[S_VERBOSE] >= 2.0)
            printf("[meb]   eval x0=%.17g |g|=%.6e lhs=%.6e rhs=%.6e floor=%.3e dm=%.6e stop=%d\n", xb[0], sqrt(gg),
                   lhs, rhs, floor_g, red[rl.dm], (int)stop);
        if (stop) {
            hs[S_MODE] = (double)PM_MULT;
            hs[S_HAVE_DIR] = 0.0;
            // in a low-precision (screening) run, an inner solve that ends at
            // the rounding floor means the working precision is exhausted:
            // the run ends after this multiplier update
            hs[S_FLOOR] = (flo && !rel && eps > 1e-10) ? 1.0 : 0.0;
            s_next = 1;
        } else {
            s_next = 0;
        }
    }
    __syncthreads();
    if (s_next) return;
    if (hs[S_FO_ON] != 0.0) {
        // first-order step from y = x_base along -s g (its trials come next)
        if (threadIdx.x == 0 && !(hs[S_FO_STEP] > 0.0)) {
            // first step: 1 / (a curvature estimate): tau/sigma + sigma (interior + mid/2)
            hs[S_FO_STEP] = 1.0 / (tau / sgm + sgm * (red[rl.ni] + 0.5 * red[rl.nm]) + 1e-300);
        }
        __syncthreads();
        const double step = hs[S_FO_STEP];
        for (int k = threadIdx.x; k < n1; k += blockDim.x) dir[k] = -step * gb[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            hs[S_GD] = -step * gg;
            hs[S_HAVE_DIR] = 1.0;
            hs[S_FO_PHASE] = 1.0;
            hs[S_LSH] = 0.0;
            hs[S_MODE] = (double)PM_EVAL;
        }
        return;
    }
    if (hs[S_CG] != 0.0) {
        // matrix-free Newton direction: x = 0, r = -g; the CG launches follow
        const int cs = cg_stride(n1);
        for (int k = threadIdx.x; k < n1; k += blockDim.x) {
            H[k] = 0.0;
            H[cs + k] = -gb[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            hs[S_CG_IT] = 0.0;
            hs[S_CG_DONE] = 0.0;
            hs[S_MODE] = (double)PM_CG;
        }
        return;
    }
    // the Newton system H dir = -g is solved by the next kernel of the step
    if (threadIdx.x == 0) hs[S_MODE] = (double)PM_SOLVE;
}

// The control step works on a copy of the state's scalar header in LDS
// (read with one load per thread, written back at the end): the scalars are
// read and updated one after another by one thread, and in global memory each
// access would wait for the one before.
__device__ __forceinline__ void control_body(double* st, StateLayout sl, RecLayout rl, const double* red) {
    extern __shared__ __align__(16) double sm[];
    __shared__ double hs[S_NSCALAR];
    // the pass's reduced record too, after the scratch: read once, with
    // several loads per thread in flight, instead of one value at a time
    double* lred = sm + ctrl_scratch_doubles(sl.n1);
    if (threadIdx.x < S_NSCALAR) hs[threadIdx.x] = st[threadIdx.x];
    for (int e0 = 0; e0 < rl.len; e0 += 4 * (int)blockDim.x) {
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = e0 + q * blockDim.x + threadIdx.x;
            v[q] = red[e < rl.len ? e : rl.len - 1];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = e0 + q * blockDim.x + threadIdx.x;
            if (e < rl.len) lred[e] = v[q];
        }
    }
    __syncthreads();
    control_body_impl(st, hs, sl, rl, lred);
    __syncthreads();
    if (threadIdx.x < S_NSCALAR) st[threadIdx.x] = hs[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Matrix-free Newton direction (Section 4.1, large d): preconditioned
// conjugate gradients on H dir = -g with the Hessian-vector products
//   H p = tau/sigma p + sigma sum_i P_i p,
// assembled from the pass's counts and sums (interior balls: the identity;
// the third case: sigma/2 on H_rr, sigma/2 sum w_i in the r row and column,
// sum gamma_i on the diagonal) and, for the rank-one parts, from the mid list:
//   sum_mid coef_i s_i (s_i^T p_c),  s_i recomputed as the pass formed it.
// Jacobi preconditioner (diagonal of H).  One launch per CG iteration: each
// block takes its share of the mid list, and the last block to arrive sums
// the shares in block order (reproducible) and performs the CG update.  The
// vectors x, r, p and the preconditioner live in the Hessian's place of the
// state, which this solver does not use.
// ---------------------------------------------------------------------------
constexpr int CG_THREADS = 256;

// CMAX: columns per lane (d <= 64 CMAX)
template <typename T, int CMAX>
__device__ __forceinline__ void cg_body(const CgArgs& a) {
    extern __shared__ __align__(16) double csm[];
    __shared__ int s_last;
    __shared__ int32_t pref[CG_THREADS * 4 + 1];
    __shared__ int wtot[CG_THREADS / WAVE];
    double* st = a.state;
    if ((int)st[S_MODE] != PM_CG || st[S_CG_DONE] != 0.0) return;
    const int d = a.d, n1 = d + 1, cs = cg_stride(n1);
    const StateLayout sl = a.sl;
    const RecLayout rl = a.rl;
    const double* red = a.red;
    double* cx = st + sl.H;       // solution
    double* cr = cx + cs;         // residual
    double* cp = cr + cs;         // search direction
    double* cm = cp + cs;         // preconditioner (diagonal of H)
    double* ly = csm;             // y (the evaluation point), d
    double* lp = csm + d;         // p_c (or nothing in the opening pass), d
    double* lacc = csm + 2 * d;   // block sum, d
    const double sig = st[S_SIGMA];
    const T inv = (T)(1.0 / sig);
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
        ly[k] = st[sl.xb + 1 + k];
        lp[k] = cp[1 + k];
        lacc[k] = 0.0;
    }
    // this block's wave segments and the exclusive prefix of their counts
    const int per = (a.nwaves + gridDim.x - 1) / gridDim.x;
    const int w0 = blockIdx.x * per, w1 = min(a.nwaves, w0 + per);
    const int nseg = max(0, w1 - w0);
    const int lane = lane_id(), wv = threadIdx.x / WAVE;
    {
        const int q0 = threadIdx.x * 4;
        int cnt[4], t = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            cnt[u] = (q0 + u < nseg) ? a.mid_cnt[w0 + q0 + u] : 0;
            t += cnt[u];
        }
        int inc = t;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const int y = __shfl_up(inc, o, WAVE);
            if (lane >= o) inc += y;
        }
        if (lane == WAVE - 1) wtot[wv] = inc;
        __syncthreads();
        int before = 0;
        for (int q = 0; q < wv; ++q) before += wtot[q];
        int run = before + inc - t;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (q0 + u <= nseg) pref[q0 + u] = run;
            run += cnt[u];
        }
        if (threadIdx.x == blockDim.x - 1 && nseg == 4 * (int)blockDim.x) pref[nseg] = run;
        __syncthreads();
    }
    const int total = pref[nseg];
    const T* C = static_cast<const T*>(a.C);
    const T* U = static_cast<const T*>(a.U);
    const T* V = static_cast<const T*>(a.V);
    // each wave takes every fourth entry: s_i^T p over the row (first read),
    // then coef_i (s_i^T p) s_i per column (second read, from cache), or
    // coef_i s_i^2 for the preconditioner
    double acc[CMAX];
#pragma unroll
    for (int q = 0; q < CMAX; ++q) acc[q] = 0.0;
    auto s_at = [&](int64_t i, bool hv, int k) -> double {
        const T ek = C[i * d + k] - (T)ly[k];
        const T vk = hv ? V[i * d + k] : T(0);
        return (double)(ek + vk * inv);
    };
    for (int e = wv; e < total; e += CG_THREADS / WAVE) {
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pref[mid] <= e)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int64_t pos = (int64_t)(w0 + lo) * a.bw + (e - pref[lo]);
        const int64_t i = a.mid_idx[pos];
        const double cf = a.mid_coef[pos];
        const bool hv = V && U && U[i] != T(0);
        double f = cf;
        if (!a.init) {
            double dot = 0.0;
#pragma unroll
            for (int q = 0; q < CMAX; ++q) {
                const int k = q * WAVE + lane;
                if (k < d) dot += s_at(i, hv, k) * lp[k];
            }
            f = cf * wave_sum(dot);
        }
#pragma unroll
        for (int q = 0; q < CMAX; ++q) {
            const int k = q * WAVE + lane;
            if (k < d) {
                const double sk = s_at(i, hv, k);
                acc[q] += a.init ? cf * sk * sk : f * sk;
            }
        }
    }
    // block sum, waves in order
    for (int w = 0; w < CG_THREADS / WAVE; ++w) {
        if (wv == w) {
#pragma unroll
            for (int q = 0; q < CMAX; ++q) {
                const int k = q * WAVE + lane;
                if (k < d) lacc[k] += acc[q];
            }
        }
        __syncthreads();
    }
    double* part = a.part + (size_t)blockIdx.x * d;
    for (int k = threadIdx.x; k < d; k += blockDim.x) st_shared_dev(part + k, lacc[k]);
    published();
    __syncthreads();
    if (threadIdx.x == 0) s_last = arrive(&a.sync[SYNC_CG]) == (int)gridDim.x - 1;
    __syncthreads();
    if (!s_last) return;
    // the last block: the rank-one share of every block, in block order
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
        double v = 0.0;
        for (int b = 0; b < (int)gridDim.x; ++b) v += ld_shared_dev(a.part + (size_t)b * d + k);
        lacc[k] = v;
    }
    if (threadIdx.x == 0) a.sync[SYNC_CG] = 0;
    __syncthreads();
    const double tau = st[S_TAU];
    const double hrr = tau / sig + sig * red[rl.ni] + 0.5 * sig * red[rl.nm];
    const double hdg = tau / sig + sig * red[rl.ni] + red[rl.sg];
    double* lq = lacc;  // q = H p in place of the rank-one sums (index k = column k)
    __shared__ double s_q0;
    if (a.init) {
        // preconditioner, z = M^-1 r, p = z, r^T z, ||r||^2 (x = 0, r = -g set by the control step)
        double prz = 0.0, prr = 0.0;
        for (int k = threadIdx.x; k < n1; k += blockDim.x) {
            const double m = (k == 0) ? hrr : hdg + lacc[k - 1];
            cm[k] = m > 0.0 ? m : hdg;
            const double z = cr[k] / cm[k];
            cp[k] = z;
            prz += cr[k] * z;
            prr += cr[k] * cr[k];
        }
        double sums[2] = {prz, prr};
        block_sum_n<2>(sums, csm + 3 * d);
        if (threadIdx.x == 0) {
            st[S_CG_RZ] = sums[0];
            st[S_CG_B2] = sums[1];
            if (!(sums[1] > 0.0)) st[S_CG_DONE] = 1.0;
        }
        return;
    }
    // q = H p
    double ph = 0.0;
    for (int k = threadIdx.x; k < d; k += blockDim.x) ph += 0.5 * sig * red[rl.sw + k] * cp[1 + k];
    const double hrc_p = block_sum(ph, csm + 3 * d);
    if (threadIdx.x == 0) s_q0 = hrr * cp[0] + hrc_p;
    for (int k = threadIdx.x; k < d; k += blockDim.x) lq[k] = 0.5 * sig * red[rl.sw + k] * cp[0] + hdg * cp[1 + k] + lacc[k];
    __syncthreads();
    if (a.out) {  // the product alone (meb_hess_vec)
        for (int k = threadIdx.x; k < n1; k += blockDim.x) a.out[k] = (k == 0) ? s_q0 : lq[k - 1];
        return;
    }
    double ppq = 0.0;
    for (int k = threadIdx.x; k < n1; k += blockDim.x) ppq += cp[k] * (k == 0 ? s_q0 : lq[k - 1]);
    const double pq = block_sum(ppq, csm + 3 * d);
    __shared__ double s_alpha;
    __shared__ int s_stop;
    if (threadIdx.x == 0) {
        s_stop = !(pq > 0.0);  // curvature not positive: stop with the current x
        s_alpha = s_stop ? 0.0 : st[S_CG_RZ] / pq;
    }
    __syncthreads();
    const double alpha = s_alpha;
    double prr = 0.0, prz = 0.0;
    for (int k = threadIdx.x; k < n1; k += blockDim.x) {
        const double qk = (k == 0) ? s_q0 : lq[k - 1];
        cx[k] += alpha * cp[k];
        cr[k] -= alpha * qk;
        prr += cr[k] * cr[k];
        prz += cr[k] * cr[k] / cm[k];
    }
    double sums[2] = {prr, prz};
    block_sum_n<2>(sums, csm + 3 * d);
    __shared__ double s_beta;
    if (threadIdx.x == 0) {
        const double it = st[S_CG_IT] + 1.0;
        st[S_CG_IT] = it;
        st[S_NCG] += 1.0;
        const double tol = st[S_CG_TOL];
        if (s_stop || sums[0] <= tol * tol * st[S_CG_B2] || it >= st[S_CG_MAX]) {
            st[S_CG_DONE] = 1.0;
            s_beta = -1.0;
        } else {
            s_beta = sums[1] / st[S_CG_RZ];
            st[S_CG_RZ] = sums[1];
        }
    }
    __syncthreads();
    const double beta = s_beta;
    if (beta >= 0.0)
        for (int k = threadIdx.x; k < n1; k += blockDim.x) cp[k] = cr[k] / cm[k] + beta * cp[k];
}

template <typename T, int CMAX>
__global__ __launch_bounds__(CG_THREADS) void cg_kernel(CgArgs a) {
    cg_body<T, CMAX>(a);
}

template <typename T, int CMAX>
static hipError_t launch_cg_t(const CgArgs& a, hipStream_t s) {
    const size_t lds = sizeof(double) * (3 * (size_t)a.d + 3 * (CG_THREADS / WAVE) + 8);
    const hipError_t ea = ensure_dynamic_lds((const void*)cg_kernel<T, CMAX>, lds);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL((cg_kernel<T, CMAX>), dim3(CG_BLOCKS), dim3(CG_THREADS), lds, s, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_cg_c(const CgArgs& a, hipStream_t s) {
    if (a.d <= 4 * WAVE) return launch_cg_t<T, 4>(a, s);
    if (a.d <= 8 * WAVE) return launch_cg_t<T, 8>(a, s);
    if (a.d <= 16 * WAVE) return launch_cg_t<T, 16>(a, s);
    if (a.d <= 32 * WAVE) return launch_cg_t<T, 32>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_cg_iter(const CgArgs& a, hipStream_t s) {
    return a.dtype == 0 ? launch_cg_c<double>(a, s) : launch_cg_c<float>(a, s);
}

// The Newton direction from the CG solution (x, or the preconditioned
// steepest descent direction -M^-1 g if x is not a descent direction), and
// the line search that follows.
__global__ __launch_bounds__(256) void cg_finish_kernel(double* st, StateLayout sl, int* flag) {
    __shared__ double scratch[256 / WAVE * 2 + 8];
    if ((int)st[S_MODE] == PM_CG) {
        const int n1 = sl.n1, cs = cg_stride(n1);
        const double* cx = st + sl.H;
        const double* cm = cx + 3 * cs;
        const double* gb = st + sl.gb;
        double* dir = st + sl.dir;
        double p = 0.0;
        for (int k = threadIdx.x; k < n1; k += blockDim.x) p += gb[k] * cx[k];
        const double gd = block_sum(p, scratch);
        const bool desc = gd < 0.0;
        double p2 = 0.0;
        for (int k = threadIdx.x; k < n1; k += blockDim.x) {
            dir[k] = desc ? cx[k] : -gb[k] / cm[k];
            p2 += gb[k] * dir[k];
        }
        const double gd2 = block_sum(p2, scratch);
        if (threadIdx.x == 0) {
            st[S_GD] = gd2;
            st[S_HAVE_DIR] = 1.0;
            st[S_LSH] = 0.0;
            st[S_MODE] = (double)PM_EVAL;
        }
    }
    if (threadIdx.x == 0 && flag) *flag = (int)st[S_MODE];
}

hipError_t launch_cg_finish(double* state, StateLayout sl, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(cg_finish_kernel, dim3(1), dim3(256), 0, s, state, sl, flag);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Newton step of the semismooth Newton method (Algorithm 2): H dir = -g in
// FP64 with the H the contraction assembled and the g the control step left
// in the state, then the Armijo search that follows.  Its own kernel (after
// the control step, which sets PM_SOLVE when a direction is needed): the
// factorizations keep their matrices in registers, and the control logic
// beside them would force spills.
// ---------------------------------------------------------------------------
// LARGE: the instance of the blocked factorization (n > CTRL_CHOL_LDS_MAX_N);
// otherwise the register and LDS factorizations.  Separate instances keep the
// register-resident factorization free of the blocked one's register needs.
// Breakdown guard, before a factorization attempt: the raise mu of this
// attempt (0 on the first), with the lower triangle of H restored from the
// untouched upper one and the diagonal raised when the factorization is in
// place (`large`; the diagonal of the assembled H kept in hdiag before the
// first attempt), or the diagonal raised by the change of mu otherwise.
__device__ __forceinline__ double newton_shift(double* st, StateLayout sl, bool large, double* scratch) {
    const int n1 = sl.n1;
    double* H = st + sl.H;
    double* hdiag = st + sl.tmp;
    const int attempt = (int)st[S_SHIFT_TRY];
    if (large && attempt == 0) {
        for (int k = threadIdx.x; k < n1; k += blockDim.x) hdiag[k] = H[(size_t)k * n1 + k];
        __syncthreads();
    }
    double mu = 0.0;
    if (attempt > 0) {
        if (attempt == 1) {
            double ptr = 0.0;
            for (int k = threadIdx.x; k < n1; k += blockDim.x) ptr += large ? hdiag[k] : H[(size_t)k * n1 + k];
            const double tr = block_sum(ptr, scratch);
            if (threadIdx.x == 0) st[S_SHIFT_MU0] = fmax(st[S_TAU] / st[S_SIGMA], 4.0 * st[S_EPS] * fabs(tr) / n1);
            __syncthreads();
        }
        const double mu_prev = st[S_SHIFT_MU];
        mu = st[S_SHIFT_MU0] * (double)(1u << (4 * (attempt - 1)));
        if (large) {
            for (int e = threadIdx.x; e < n1 * n1; e += blockDim.x) {
                const int i = e / n1, j = e % n1;
                if (i > j) H[e] = H[(size_t)j * n1 + i];
                if (i == j) H[e] = hdiag[i] + mu;
            }
        } else {
            for (int k = threadIdx.x; k < n1; k += blockDim.x) H[(size_t)k * n1 + k] += mu - mu_prev;
        }
        __syncthreads();
    }
    return mu;
}

// After a factorization attempt: on failure (rc != 0) the next step's Newton
// launch tries the next raise, or, after the last, the inner solve ends at
// its iterate; on success dir holds the direction and the line search
// starts.
__device__ __forceinline__ void newton_finish(double* st, StateLayout sl, int rc, double mu, double* scratch) {
    const int n1 = sl.n1;
    if (rc != 0) {
        if (threadIdx.x == 0) {
            const int attempt = (int)st[S_SHIFT_TRY];
            if (attempt < CTRL_SHIFT_TRIES) {
                st[S_SHIFT_TRY] = (double)(attempt + 1);
                st[S_SHIFT_MU] = mu;
            } else {
                // no raise helped: end the inner solve here (multiplier update next)
                st[S_NBREAK] += 1.0;
                st[S_MODE] = (double)PM_MULT;
                st[S_HAVE_DIR] = 0.0;
                st[S_FLOOR] = 0.0;
                st[S_SHIFT_TRY] = 0.0;
                st[S_SHIFT_MU] = 0.0;
            }
        }
        return;
    }
    const double* dir = st + sl.dir;
    const double* gb = st + sl.gb;
    double pgd = 0.0;
    for (int k = threadIdx.x; k < n1; k += blockDim.x) pgd += gb[k] * dir[k];
    const double gd = block_sum(pgd, scratch);
    if (threadIdx.x == 0) {
        st[S_SHIFT_TRY] = 0.0;
        st[S_SHIFT_MU] = 0.0;
        if (mu > 0.0) st[S_NSHIFT] += 1.0;
        st[S_GD] = gd;
        st[S_HAVE_DIR] = 1.0;
        st[S_LSH] = 0.0;
        st[S_MODE] = (double)PM_EVAL;
    }
}

// NK: the instance (newton_kind): the register and LDS factorizations, the
// blocked factorization on a copy in LDS, or the one-workgroup blocked
// factorization in global memory (n > CTRL_CHOL_LDS_MAX_N).  Separate
// instances keep the register-resident factorization free of the blocked
// one's register needs.
//
// Newton direction: H dir = -g, H assembled by the contraction.  H is
// positive definite through its (tau/sigma) I term in exact arithmetic
// (Section 4); rounding in its assembly can still produce a pivot that is not
// positive.  Breakdown guard: the diagonal is raised by
// mu = max(tau/sigma, 4 eps mean_k H_kk), then 16 mu, 256 mu, ... (at most
// CTRL_SHIFT_TRIES raises) and the system solved again -- a shifted system
// still gives a descent direction for the line search; if no shift succeeds,
// the inner solve ends at the current iterate.  One attempt per launch: when a
// pivot is not positive, the step ends with the mode still PM_SOLVE, the next
// step's pass, contraction and control step do nothing, and its Newton launch
// tries the next raise (a loop here would keep the register-resident
// factorization's state live across attempts and spill).
template <int NK>
__device__ __forceinline__ void newton_body(double* st, StateLayout sl) {
    extern __shared__ __align__(16) double sm[];
    if ((int)st[S_MODE] != PM_SOLVE) return;
    if (newton_kind(sl.n1) != NK) return;
    constexpr bool LARGE = NK == NK_LARGE;
    double* scratch = sm;                            // ctrl_scratch_doubles(n1)
    double* lmat = sm + ctrl_scratch_doubles(sl.n1);  // Cholesky matrix when it fits
    const int n1 = sl.n1;
    double* dir = st + sl.dir;
    const double* gb = st + sl.gb;
    double* H = st + sl.H;
    // the large path factorizes H in place (lower triangle)
    const double mu = newton_shift(st, sl, LARGE, scratch + 2 * n1);
    int rc = 0;
    if constexpr (LARGE) {
        // blocked factorization in place (global memory), rhs in LDS
        double* bv = scratch;
        for (int k = threadIdx.x; k < n1; k += blockDim.x) bv[k] = -gb[k];
        __syncthreads();
        rc = chol_solve_blocked(n1, H, bv, lmat);
        for (int k = threadIdx.x; k < n1; k += blockDim.x) dir[k] = bv[k];
        __syncthreads();
    } else if (rch_fits(n1, blockDim.x)) {
        double* bv = scratch;
        for (int k = threadIdx.x; k < n1; k += blockDim.x) bv[k] = -gb[k];
        __syncthreads();
        rc = chol_solve_regs(n1, H, bv, bv, lmat);
        for (int k = threadIdx.x; k < n1; k += blockDim.x) dir[k] = bv[k];
        __syncthreads();
    } else {
        // LDS: scratch = [rd (n1) | rhs (n1)], lmat = H with an odd leading dimension
        const int ld = chol_ld(n1);
        double* rd = scratch;
        double* bv = scratch + n1;
        for (int e = threadIdx.x; e < n1 * n1; e += blockDim.x) lmat[(e / n1) * ld + e % n1] = H[e];
        for (int k = threadIdx.x; k < n1; k += blockDim.x) bv[k] = -gb[k];
        __syncthreads();
        rc = chol_solve_lds(n1, ld, lmat, bv, rd);
        for (int k = threadIdx.x; k < n1; k += blockDim.x) dir[k] = bv[k];
        __syncthreads();
    }
    newton_finish(st, sl, rc, mu, scratch);
}

// The Newton step with the multi-workgroup factorization (systems of at
// least MCHOL_MIN_N unknowns, single-instance runs): newton_pre_kernel
// (breakdown guard, b = -g in dir, the failure flag cleared), the panel and
// update launches and the back-substitution launches into dir (all gated on
// the mode), then newton_post_kernel (the bookkeeping of newton_finish).
constexpr int NEWTON_POST_THREADS = 256;

__host__ __device__ inline MChol newton_mchol(double* st, StateLayout sl) {
    MChol a;
    a.n = sl.n1;
    a.M = st + sl.H;
    a.b = st + sl.dir;
    a.y = st + sl.yv;
    a.x = st + sl.dir;
    a.ld = st + sl.ldiag;
    a.bad = st + S_CHOL_BAD;
    a.gate = st + S_MODE;
    return a;
}

__global__ __launch_bounds__(CTRL_THREADS) void newton_pre_kernel(double* st, StateLayout sl) {
    extern __shared__ __align__(16) double sm[];
    if ((int)st[S_MODE] != PM_SOLVE) return;
    newton_shift(st, sl, true, sm);
    const int n1 = sl.n1;
    for (int k = threadIdx.x; k < n1; k += blockDim.x) st[sl.dir + k] = -st[sl.gb + k];
    if (threadIdx.x == 0) st[S_CHOL_BAD] = 0.0;
}

__global__ __launch_bounds__(NEWTON_POST_THREADS) void newton_post_kernel(double* st, StateLayout sl, int* flag) {
    __shared__ double sm[NEWTON_POST_THREADS / WAVE];
    if ((int)st[S_MODE] == PM_SOLVE) {
        const int rc = st[S_CHOL_BAD] != 0.0 ? -1 : 0;
        const int attempt = (int)st[S_SHIFT_TRY];
        const double mu = attempt > 0 ? st[S_SHIFT_MU0] * (double)(1u << (4 * (attempt - 1))) : 0.0;
        newton_finish(st, sl, rc, mu, sm);
    }
    if (threadIdx.x == 0 && flag) *flag = (int)st[S_MODE];
}

// `flag` (nullable, typically host-mapped) receives the state's mode after
// the step.
template <int NK>
__global__ __launch_bounds__(newton_threads(NK)) void newton_kernel(double* st, StateLayout sl, int* flag) {
    newton_body<NK>(st, sl);
    if (threadIdx.x == 0 && flag) *flag = (int)st[S_MODE];
}

// `flag` (nullable, typically host-mapped) receives the state's mode after
// the step, so a host can learn that the run has ended without a copy.
__global__ __launch_bounds__(CTRL_THREADS) void control_kernel(double* st, StateLayout sl, RecLayout rl,
                                                               const double* red, int* flag) {
    control_body(st, sl, rl, red);
    if (threadIdx.x == 0 && flag) *flag = (int)st[S_MODE];
}

// The control step and then the Newton step in one launch, for systems the
// one-workgroup factorizations take (newton_kind NK_SMALL): the same bodies
// as control_kernel and newton_kernel<NK_SMALL>, one after the other on the
// same workgroup of CTRL_THREADS, so a solver step pays one kernel boundary
// less.  The Newton body reads the header the control body wrote back to
// global memory after the block barrier (same workgroup: no cache
// maintenance).  Both bodies use the dynamic LDS from its start, one after
// the other.  `flag` as for newton_kernel.
__global__ __launch_bounds__(CTRL_THREADS) void control_newton_kernel(double* st, StateLayout sl, RecLayout rl,
                                                                      const double* red, int* flag) {
    control_body(st, sl, rl, red);
    __syncthreads();
    newton_body<NK_SMALL>(st, sl);
    if (threadIdx.x == 0 && flag) *flag = (int)st[S_MODE];
}

size_t control_lds_bytes(int n1) {
    return sizeof(double) * ((size_t)ctrl_scratch_doubles(n1) + (size_t)RecLayout::make(n1 - 1).len);
}

size_t newton_lds_bytes(int n1) {
    size_t lds = sizeof(double) * (size_t)ctrl_scratch_doubles(n1);
    if (newton_large(n1)) return lds + sizeof(double) * (size_t)bch_lds_doubles();
    if (rch_fits(n1, CTRL_THREADS)) return lds + sizeof(double) * rch_lds_doubles(n1);
    return lds + sizeof(double) * (size_t)n1 * chol_ld(n1);
}

hipError_t launch_newton(double* state, StateLayout sl, int* flag, hipStream_t s) {
    if (sl.n1 >= MCHOL_MIN_N) {
        hipLaunchKernelGGL(newton_pre_kernel, dim3(1), dim3(CTRL_THREADS), sizeof(double) * CTRL_THREADS, s, state,
                           sl);
        hipError_t ea = launch_mchol_factor(newton_mchol(state, sl), s);
        if (ea != hipSuccess) return ea;
        ea = launch_mchol_back(newton_mchol(state, sl), s);
        if (ea != hipSuccess) return ea;
        hipLaunchKernelGGL(newton_post_kernel, dim3(1), dim3(NEWTON_POST_THREADS), 0, s, state, sl, flag);
        return hipGetLastError();
    }
    const size_t lds = newton_lds_bytes(sl.n1);
    const int nk = newton_kind(sl.n1);
    const void* fn = nk == NK_LARGE ? (const void*)newton_kernel<NK_LARGE> : (const void*)newton_kernel<NK_SMALL>;
    hipError_t ea = ensure_dynamic_lds(fn, lds);
    if (ea != hipSuccess) return ea;
    if (nk == NK_LARGE)
        hipLaunchKernelGGL(newton_kernel<NK_LARGE>, dim3(1), dim3(newton_threads(NK_LARGE)), lds, s, state, sl, flag);
    else
        hipLaunchKernelGGL(newton_kernel<NK_SMALL>, dim3(1), dim3(CTRL_THREADS), lds, s, state, sl, flag);
    return hipGetLastError();
}

bool control_newton_fused(int n1) { return n1 < MCHOL_MIN_N && newton_kind(n1) == NK_SMALL; }

hipError_t launch_control_newton(double* state, StateLayout sl, RecLayout rl, const double* red, int* flag,
                                 hipStream_t s) {
    if (!control_newton_fused(sl.n1)) return hipErrorInvalidValue;
    const size_t lds = std::max(control_lds_bytes(sl.n1), newton_lds_bytes(sl.n1));
    hipError_t ea = ensure_dynamic_lds((const void*)control_newton_kernel, lds);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL(control_newton_kernel, dim3(1), dim3(CTRL_THREADS), lds, s, state, sl, rl, red, flag);
    return hipGetLastError();
}

hipError_t launch_control(double* state, StateLayout sl, RecLayout rl, const double* red, int* flag, hipStream_t s) {
    const size_t lds = control_lds_bytes(sl.n1);
    hipError_t ea = ensure_dynamic_lds((const void*)control_kernel, lds);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL(control_kernel, dim3(1), dim3(CTRL_THREADS), lds, s, state, sl, rl, red, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One solver step for several instances (a tick of the multi-instance
// server): the same bodies as the single-instance kernels, with each
// instance's blocks located by the tick list.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void syrk_batch_kernel(const BatchItem* tab, TickList L) {
    const int k = tick_find(L, blockIdx.x);
    const BatchItem& it = tab[L.slot[k]];
    const int b = blockIdx.x - L.off[k];
    const int npairs = it.sa.ntile * (it.sa.ntile + 1) / 2;
    __shared__ __align__(16) unsigned char smem[SYRK_SMEM];
    if (it.sa.dtype == 0)
        syrk_dispatch<double>(it.sa, b % npairs, b / npairs, npairs, smem);
    else
        syrk_dispatch<float>(it.sa, b % npairs, b / npairs, npairs, smem);
}

__global__ __launch_bounds__(CTRL_THREADS) void control_batch_kernel(const BatchItem* tab, TickList L) {
    const BatchItem& it = tab[L.slot[blockIdx.x]];
    double* st = const_cast<double*>(it.pa.state);
    control_body(st, it.pa.sl, it.pa.rl, it.pa.red);
}

template <int NK>
__global__ __launch_bounds__(newton_threads(NK)) void newton_batch_kernel(const BatchItem* tab, TickList L) {
    const BatchItem& it = tab[L.slot[blockIdx.x]];
    double* st = const_cast<double*>(it.pa.state);
    newton_body<NK>(st, it.pa.sl);
    // the flag after the item's own Newton instance
    if (threadIdx.x == 0 && it.flag && newton_kind(it.pa.sl.n1) == NK) *it.flag = (int)st[S_MODE];
}

namespace {
// fills L with the items' slots and block offsets; returns the total blocks
template <class F>
int make_list(const BatchItem* htab, const int* slots, int n, TickList& L, F&& blocks_of) {
    L.n = n;
    int off = 0;
    for (int k = 0; k < n; ++k) {
        L.slot[k] = slots[k];
        L.off[k] = off;
        off += blocks_of(htab[slots[k]]);
    }
    L.off[n] = off;
    return off;
}
}  // namespace

hipError_t launch_tick(const BatchItem* dtab, const BatchItem* htab, const int* slots, int n, hipStream_t s) {
    for (int c0 = 0; c0 < n; c0 += TICK_MAX) {
        const int cn = n - c0 < TICK_MAX ? n - c0 : TICK_MAX;
        const int* sl = slots + c0;
        TickList L;
        // evaluation passes (with their reductions), one launch per template instance
        {
            int ids[TICK_MAX];
            bool done[TICK_MAX];
            for (int k = 0; k < cn; ++k) {
                ids[k] = pass_variant(htab[sl[k]].pa.dtype, htab[sl[k]].pc);
                done[k] = false;
            }
            for (int k = 0; k < cn; ++k) {
                if (done[k]) continue;
                int grp[TICK_MAX];
                int ng = 0, max_d = 0, max_stages = 0;
                for (int q = k; q < cn; ++q)
                    if (!done[q] && ids[q] == ids[k]) {
                        grp[ng++] = sl[q];
                        done[q] = true;
                        if (htab[sl[q]].pa.d > max_d) max_d = htab[sl[q]].pa.d;
                        if (htab[sl[q]].pc.stages > max_stages) max_stages = htab[sl[q]].pc.stages;
                    }
                const int blocks = make_list(htab, grp, ng, L, [](const BatchItem& it) { return it.pc.blocks; });
                const hipError_t e = launch_pass_group(dtab, L, blocks, max_d, max_stages, htab[grp[0]].pa.dtype,
                                                       htab[grp[0]].pc, s);
                if (e != hipSuccess) return e;
            }
        }
        // contraction with the Hessian assembly
        int ws[TICK_MAX];
        int nw = 0;
        for (int k = 0; k < cn; ++k)
            if (htab[sl[k]].pa.want_mid) ws[nw++] = sl[k];
        if (nw > 0) {
            const int nb = make_list(htab, ws, nw, L, [](const BatchItem& it) {
                return it.sa.ntile * (it.sa.ntile + 1) / 2 * it.sa.ksplit;
            });
            hipLaunchKernelGGL(syrk_batch_kernel, dim3(nb), dim3(256), 0, s, dtab, L);
        }
        size_t lds = 0;
        for (int k = 0; k < cn; ++k) {
            const size_t b = control_lds_bytes(htab[sl[k]].pa.sl.n1);
            if (b > lds) lds = b;
        }
        make_list(htab, sl, cn, L, [](const BatchItem&) { return 1; });
        const hipError_t ea = ensure_dynamic_lds((const void*)control_batch_kernel, lds);
        if (ea != hipSuccess) return ea;
        hipLaunchKernelGGL(control_batch_kernel, dim3(cn), dim3(CTRL_THREADS), lds, s, dtab, L);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // the Newton solves: one launch per instance that some item needs
        // (items of the other kinds return)
        size_t nlds[2] = {0, 0};
        for (int k = 0; k < cn; ++k) {
            const int n1 = htab[sl[k]].pa.sl.n1;
            const int nk = newton_kind(n1);
            nlds[nk] = std::max(nlds[nk], newton_lds_bytes(n1));
        }
        const void* fns[2] = {(const void*)newton_batch_kernel<NK_SMALL>, (const void*)newton_batch_kernel<NK_LARGE>};
        for (int nk = 0; nk < 2; ++nk) {
            if (nlds[nk] == 0) continue;
            const hipError_t eb = ensure_dynamic_lds(fns[nk], nlds[nk]);
            if (eb != hipSuccess) return eb;
            if (nk == NK_SMALL)
                hipLaunchKernelGGL(newton_batch_kernel<NK_SMALL>, dim3(cn), dim3(CTRL_THREADS), nlds[nk], s, dtab, L);
            else
                hipLaunchKernelGGL(newton_batch_kernel<NK_LARGE>, dim3(cn), dim3(newton_threads(NK_LARGE)), nlds[nk], s,
                                   dtab, L);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
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
    (void)d;
    ScanCfg c;
    // many waves with few rows each: the scan keeps little state, so a CU
    // holds enough waves to keep HBM busy; bw is a multiple of 64 so that
    // every lane-group width divides it
    const int64_t maxw = (int64_t)num_cu * 32;
    int64_t w = (m + 63) / 64;
    if (w > maxw) w = maxw;
    if (w < 1) w = 1;
    c.bw = (((m + w - 1) / w) + 63) / 64 * 64;
    const int64_t waves = (m + c.bw - 1) / c.bw;
    c.blocks = (int)((waves + SCAN_WPB - 1) / SCAN_WPB);
    c.nwaves = c.blocks * SCAN_WPB;
    return c;
}

// Lanes per row for a scan of precision dtype: 16-byte loads where the row
// allows, about 16 bytes x 4 loads per lane.
struct ScanLanes {
    int G, vec, nl, nlmax;
};
static ScanLanes scan_lanes(int d, int dtype) {
    ScanLanes l;
    if (dtype != 0 && d % 4 == 0)
        l.vec = 4;
    else
        l.vec = (d % 2 == 0) ? 2 : 1;
    const int per_lane = (dtype == 0) ? 8 : 16;
    const int need = (d + per_lane - 1) / per_lane;
    int G = 1;
    while (G < need && G < 64) G <<= 1;
    l.G = G;
    l.nl = (d + G * l.vec - 1) / (G * l.vec);
    l.nlmax = l.nl <= 2 ? 2 : (l.nl <= 4 ? 4 : (l.nl <= 8 ? 8 : (l.nl <= 16 ? 16 : 32)));
    return l;
}

// MODE 0: feasibility (hit: reach - r > thr; keeps max reach - r and argmax)
// MODE 1: screening (value r - r_i - ||c - c_i||; hit: value <= thr)
// MODE 2: FP32 preparation (writes float(c_i - x) and float(r_i); keeps max)
// Distances are accumulated in FP64 (FP32 rows are widened exactly).  Each
// wave streams its own rows with the next group's loads issued before the
// current group is used.
// Hits go to seg: by default into the wave's own segment seg[wbeg ..]
// (concatenated afterwards by scan_copy); with a placement (pl.offs) straight
// to their final positions seg[pl.offs[wave] + k], those below pl.cap, after
// a counting pass has filled pl.offs -- and the kernel returns at once if
// *pl.gate (that pass's total) is zero.  seg may be NULL (count only).
template <typename T, int VEC, int NLMAX, int MODE>
__global__ __launch_bounds__(SCAN_THREADS) void scan_kernel(const T* C, const T* R, int64_t m, int d, int G, int nl,
                                                            const double* xdev, double r, double thr,
                                                            double* slack, float* C32, float* R32, ScanCfg cfg,
                                                            double* wmax, int64_t* warg, int64_t* wcnt,
                                                            int64_t* seg, ScanPlace pl) {
    extern __shared__ double lx[];
    if (pl.gate && *pl.gate == 0) return;
    for (int k = threadIdx.x; k < d; k += SCAN_THREADS) lx[k] = xdev ? xdev[k] : 0.0;
    __syncthreads();
    const int lane = lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int64_t gw = (int64_t)blockIdx.x * SCAN_WPB + wid;
    const int gi = lane / G, gl = lane % G, bpw = WAVE / G;
    const int64_t wbeg = gw * cfg.bw, wend = min(m, wbeg + cfg.bw);
    const int64_t obase = pl.offs ? pl.offs[gw] : wbeg;
    const int64_t ocap = pl.offs ? pl.cap : INT64_MAX;
    int col[NLMAX];
    bool own[NLMAX];
#pragma unroll
    for (int j = 0; j < NLMAX; ++j) {
        const int b = (j * G + gl) * VEC;
        own[j] = (j < nl) && (b < d);
        col[j] = own[j] ? b : 0;
    }
    double best = -INFINITY;
    int64_t barg = INT64_MAX;
    int64_t count = 0;
    struct Rows {
        RowVec<T, VEC> c[NLMAX];
        T r;
    };
    auto load = [&](int64_t b0, Rows& L) {
        int64_t i = b0 + gi;
        i = i < wend ? i : wend - 1;
        L.r = R ? R[i] : T(0);
#pragma unroll
        for (int j = 0; j < NLMAX; ++j) L.c[j] = load_vec<T, VEC>(C + i * d + col[j]);
    };
    auto process = [&](int64_t b0, const Rows& L) {
        const int64_t i = b0 + gi;
        const bool act = i < wend;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < NLMAX; ++j) {
            RowVec<float, VEC> o;
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const double e = own[j] ? (double)L.c[j].v[q] - lx[col[j] + q] : 0.0;
                acc += e * e;
                o.v[q] = (float)e;
            }
            if (MODE == 2 && C32 && act && own[j]) store_vec<float, VEC>(C32 + i * d + col[j], o);
        }
        const double dist = sqrt(group_sum<double>(acc, G));
        const double ri = act ? (double)L.r : 0.0;
        double val;
        bool hit;
        if (MODE == 1) {
            val = r - ri - dist;
            hit = act && val <= thr;
            if (slack && act && gl == 0) slack[i] = val;
        } else {
            val = ri + dist - r;
            // the preparation flags a negative radius or a non-finite value
            // (including NaN, which the maximum below would skip) as +inf
            if (MODE == 2 && !(ri >= 0.0 && val < INFINITY)) val = INFINITY;
            hit = (MODE == 0) && act && val > thr;
            if (MODE == 2 && R32 && act && gl == 0) R32[i] = (float)ri;
            if (act && (val > best || (val == best && i < barg))) {
                best = val;
                barg = i;
            }
        }
        if (MODE != 2) {
            const unsigned long long bal = __ballot(hit && gl == 0);
            if (seg && hit && gl == 0) {
                const int64_t q = obase + count + __popcll(bal & ((1ull << lane) - 1ull));
                if (q < ocap) seg[q] = i;
            }
            count += __popcll(bal);
        }
    };
    Rows A, B;
    if (wbeg < wend) load(wbeg, A);
    for (int64_t b0 = wbeg; b0 < wend; b0 += 2 * bpw) {
        const bool more = b0 + bpw < wend;
        if (more) load(b0 + bpw, B);
        process(b0, A);
        if (!more) break;
        if (b0 + 2 * bpw < wend) load(b0 + 2 * bpw, A);
        process(b0 + bpw, B);
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

template <typename T, int MODE, int VEC, int NLMAX>
static hipError_t launch_scan_v(const void* C, const void* R, int64_t m, int d, const ScanLanes& l, const double* x,
                                double r, double thr, double* slack, float* C32, float* R32, const ScanCfg& c,
                                double* wmax, int64_t* warg, int64_t* wcnt, int64_t* seg, const ScanPlace& pl,
                                hipStream_t s) {
    hipLaunchKernelGGL((scan_kernel<T, VEC, NLMAX, MODE>), dim3(c.blocks), dim3(SCAN_THREADS), sizeof(double) * d, s,
                       (const T*)C, (const T*)R, m, d, l.G, l.nl, x, r, thr, slack, C32, R32, c, wmax, warg, wcnt,
                       seg, pl);
    return hipGetLastError();
}

template <typename T, int MODE, int VEC>
static hipError_t launch_scan_n(const void* C, const void* R, int64_t m, int d, const ScanLanes& l, const double* x,
                                double r, double thr, double* slack, float* C32, float* R32, const ScanCfg& c,
                                double* wmax, int64_t* warg, int64_t* wcnt, int64_t* seg, const ScanPlace& pl,
                                hipStream_t s) {
#define MEB_SCAN_ARGS C, R, m, d, l, x, r, thr, slack, C32, R32, c, wmax, warg, wcnt, seg, pl, s
    if (l.nlmax == 2) return launch_scan_v<T, MODE, VEC, 2>(MEB_SCAN_ARGS);
    if (l.nlmax == 4) return launch_scan_v<T, MODE, VEC, 4>(MEB_SCAN_ARGS);
    if (l.nlmax == 8) return launch_scan_v<T, MODE, VEC, 8>(MEB_SCAN_ARGS);
    if (l.nlmax == 16) return launch_scan_v<T, MODE, VEC, 16>(MEB_SCAN_ARGS);
    return launch_scan_v<T, MODE, VEC, 32>(MEB_SCAN_ARGS);
}

template <int MODE>
static hipError_t launch_scan_t(const void* C, const void* R, int64_t m, int d, int dtype, const double* x,
                                double r, double thr, double* slack, float* C32, float* R32, const ScanCfg& c,
                                double* wmax, int64_t* warg, int64_t* wcnt, int64_t* seg, const ScanPlace& pl,
                                hipStream_t s) {
    const ScanLanes l = scan_lanes(d, dtype);
    if (dtype == 0) {
        if (l.vec == 2) return launch_scan_n<double, MODE, 2>(MEB_SCAN_ARGS);
        return launch_scan_n<double, MODE, 1>(MEB_SCAN_ARGS);
    }
    if constexpr (MODE == 2) return hipErrorInvalidValue;  // the preparation reads FP64
    if (l.vec == 4) return launch_scan_n<float, MODE, 4>(MEB_SCAN_ARGS);
    if (l.vec == 2) return launch_scan_n<float, MODE, 2>(MEB_SCAN_ARGS);
    return launch_scan_n<float, MODE, 1>(MEB_SCAN_ARGS);
#undef MEB_SCAN_ARGS
}

hipError_t launch_scan(int mode, const void* C, const void* R, int64_t m, int d, int dtype, const double* x,
                       double r, double thr, double* slack, float* C32, float* R32, const ScanCfg& c, double* wmax,
                       int64_t* warg, int64_t* wcnt, int64_t* seg, hipStream_t s, const ScanPlace& pl) {
    if (mode == 0)
        return launch_scan_t<0>(C, R, m, d, dtype, x, r, thr, slack, C32, R32, c, wmax, warg, wcnt, seg, pl, s);
    if (mode == 1)
        return launch_scan_t<1>(C, R, m, d, dtype, x, r, thr, slack, C32, R32, c, wmax, warg, wcnt, seg, pl, s);
    return launch_scan_t<2>(C, R, m, d, 0, x, r, thr, slack, C32, R32, c, wmax, warg, wcnt, seg, pl, s);
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

__global__ void widen_f32_kernel(const float* src, double* dst, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
        dst[e] = (double)src[e];
}

hipError_t launch_widen_f32(const float* src, double* dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(widen_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
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
