// Internal declarations shared by the host solver and the kernel launchers of
// libmeb.so.  Nothing here is part of the public C ABI (include/meb.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "meb.h"

namespace meb {

// Number of Armijo trial step sizes evaluated in one data pass.  The solver
// uses eta = 1, 1/2, ..., 2^-(NT-2), and 0 (the base point) last.
constexpr int NT = 9;

__host__ __device__ inline double solver_eta(int l) { return l == NT - 1 ? 0.0 : 1.0 / (double)(1 << l); }

// ----------------------------------------------------------------------------
// Device-resident solver state (doubles).  One ripALM run keeps its whole
// control state on the device so that the evaluation pass, the Hessian
// contraction and the control step can be enqueued back to back without a
// host round trip.  Scalar slots first, then (d+1)-vectors, then H.
// ----------------------------------------------------------------------------
enum StateSlot : int {
    S_MODE = 0,      // 0 = evaluate, 1 = multiplier update + evaluate, 2 = done
    S_SIGMA,         // current raw penalty sigma_k
    S_SIGMA_NEXT,    // raw penalty of the next outer iteration
    S_TAU,           // raw proximal weight
    S_L,             // instance scale
    S_RHO,
    S_TOL,           // normalized KKT tolerance of this run
    S_GROWTH,
    S_SIGMA_MAX,     // raw
    S_MAX_OUTER,
    S_MAX_INNER,
    S_MAX_LS,
    S_STALL_OUTER,
    S_EPS,           // unit roundoff of the working precision
    S_K,             // outer iterations done
    S_J,             // Newton iterations in the current outer iteration
    S_NINNER,        // Newton iterations in total
    S_NPASS,         // evaluation passes in total
    S_HAVE_DIR,      // 1 if dir holds a Newton direction to line-search
    S_GD,            // <g(x_base), dir>
    S_LSH,           // halvings spent on the current direction
    S_STATUS,        // 0 running, 1 converged, 2 max iterations / stall, 3 rounding floor
                     // of a low-precision run reached, -1 numeric failure
    S_KKT,           // last normalized KKT_max
    S_KKT_P0, S_KKT_P1, S_KKT_P2, S_KKT_P3, S_KKT_P4,
    S_BEST_KKT,
    S_STALL,
    S_PSI,           // Psi at the current iterate (for reporting)
    S_VERBOSE,
    S_BYTES,         // algorithmic bytes moved by the evaluation passes of this run
    S_SUMK,          // rows of the rank-one Hessian contraction, summed over passes
    S_MAXK,          // largest such row count of one pass
    S_HSKIP,         // 1 if the contraction of the last pass was skipped
    S_FLOOR,         // 1 if the last inner solve of a low-precision run stopped at the rounding floor
    S_NSHIFT,        // Newton systems solved with a raised diagonal (breakdown guard)
    S_NBREAK,        // inner solves ended because no shift made the factorization succeed
    S_FO_OUTER,      // outer iterations (from the first) whose inner solve is first-order
    S_FO_ON,         // 1 while the current inner solve is the accelerated gradient method
    S_FO_PHASE,      // 1 after a gradient step was proposed (its trial pass is next)
    S_FO_T,          // momentum sequence t_k of the accelerated gradient method
    S_FO_STEP,       // current gradient step size s (raw units)
    S_NFO,           // first-order iterations in total
    S_CG,            // 1: Newton directions by preconditioned CG with Hessian-vector products
    S_CG_MAX,        // CG iterations per Newton direction
    S_CG_TOL,        // relative residual at which CG stops
    S_CG_IT,         // CG iterations of the current direction
    S_CG_DONE,       // 1 once the current CG solve has stopped
    S_CG_RZ,         // r^T z of the current CG iteration
    S_CG_B2,         // ||b||^2 of the current system
    S_NCG,           // CG iterations in total
    S_SHIFT_TRY,     // raises of the Newton system's diagonal tried for the current direction
    S_SHIFT_MU0,     // first raise mu of the current direction
    S_SHIFT_MU,      // raise in effect
    S_CHOL_BAD,      // 1 when the multi-workgroup factorization met a pivot that is not positive
    S_NSCALAR = 64
};

constexpr int WAVE = 64;           // lanes per wavefront
constexpr int PASS_THREADS = 256;  // threads per evaluation-pass block
constexpr int WPB = PASS_THREADS / WAVE;

// panel width of the blocked Cholesky factorizations, and the system size
// from which a single-instance Newton step factors across many workgroups
constexpr int MCHOL_NB = 32;
constexpr int MCHOL_MIN_N = 320;

struct StateLayout {
    int n1;      // d + 1
    int xb;      // current inner iterate (line-search base)
    int dir;     // Newton direction (possibly scaled by the line search)
    int xbar;    // proximal center
    int ab;      // auxiliary sequence (alpha, beta)
    int gb;      // gradient at xb
    int tmp;     // previous iterate of the accelerated gradient method
    int yv;      // forward substitution L y = -g of the multi-workgroup factorization
    int ldiag;   // its current diagonal factor block (MCHOL_NB^2)
    int H;       // (d+1)^2 Hessian / Cholesky factor
    int len;
    static StateLayout make(int d) {
        StateLayout s;
        s.n1 = d + 1;
        int o = S_NSCALAR;
        auto vec = [&](int n) { int r = o; o += (n + 7) & ~7; return r; };
        s.xb = vec(s.n1);
        s.dir = vec(s.n1);
        s.xbar = vec(s.n1);
        s.ab = vec(s.n1);
        s.gb = vec(s.n1);
        s.tmp = vec(s.n1);
        s.yv = vec(s.n1);
        s.ldiag = vec(MCHOL_NB * MCHOL_NB);
        s.H = vec(s.n1 * s.n1);
        s.len = o;
        return s;
    }
};

// ----------------------------------------------------------------------------
// Per-block partial record of one evaluation pass (doubles).
// ----------------------------------------------------------------------------
struct RecLayout {
    int d;
    int trial;  // NT sums of ||Pi(z_i(eta))||^2
    int su;     // sum u+            (evaluation point)
    int z1;     // sum ||Pi(z_i)||^2 at the evaluation point
    int sv;     // d: sum v+
    int ni;     // # interior
    int nm;     // # mid
    int sg;     // sum over mid of gamma_i
    int sw;     // d: sum over mid of s_i / ||s_i||
    int dm;     // sum ||w+ - w||^2
    int rs;     // sum over non-polar of |t_i| + ||s_i||
    int ww;     // sum ||w_i||^2 of the multipliers in use
    int bytes;  // algorithmic bytes read and written by this pass
    int ku;     // sum u of the updated multipliers (KKT)
    int kv;     // d: sum v of the updated multipliers (KKT)
    int kmax;   // 3 maxima: primal cone distance, dual cone distance, |complementarity|
    int len;
    static RecLayout make(int d) {
        RecLayout r;
        r.d = d;
        int o = 0;
        r.trial = o; o += NT;
        r.su = o; o += 1;
        r.z1 = o; o += 1;
        r.ni = o; o += 1;
        r.nm = o; o += 1;
        r.sg = o; o += 1;
        r.dm = o; o += 1;
        r.rs = o; o += 1;
        r.ww = o; o += 1;
        r.bytes = o; o += 1;
        r.ku = o; o += 1;
        r.kmax = o; o += 3;
        r.sv = o; o += d;
        r.sw = o; o += d;
        r.kv = o; o += d;
        r.len = o;
        return r;
    }
};

// Coefficients of one active-list entry (working precision): the ball's
// vector parts are a e + b v with e = c_i - y and v = v_i, for the sums
// sum gamma s (sv), sum_mid s / ||s|| (sw) and the updated multiplier (kv,
// also the V row written), then a flag word (bit 0: v_i is read, bit 1: the
// V row is written).
constexpr int ACT_NC = 7;

static_assert(S_CHOL_BAD < S_NSCALAR, "state scalars fit their slots");

// Pass modes.  PM_CG: a Newton direction is being computed by conjugate
// gradients (set by the control step, cleared by the CG finish step).
// PM_SOLVE: the control step asks the Newton kernel of the step for a
// direction (cleared by it).
enum PassMode : int { PM_EVAL = 0, PM_MULT = 1, PM_DONE = 2, PM_CG = 3, PM_SOLVE = 4 };

// Arguments of the matrix-free Newton solve (conjugate gradients with
// Hessian-vector products over the mid list of the last pass).
struct CgArgs {
    const void* C;
    const void* U;
    const void* V;
    int d;
    int dtype;
    double* state;
    StateLayout sl;
    const double* red;          // reduced record of the pass
    RecLayout rl;
    const int32_t* mid_cnt;
    const int32_t* mid_idx;
    const double* mid_coef;
    int nwaves;
    int64_t bw;
    double* part;               // CG_BLOCKS x d block partial sums
    int* sync;                  // arrival counter (SYNC_CG)
    int init;                   // 1: the preconditioner pass that opens a solve
    double* out;                // non-null: write H p here (d + 1) instead of a CG update
};
constexpr int CG_BLOCKS = 512;  // blocks of a Hessian-vector product
// CG vectors, in the Hessian's place of the state (unused by this solver)
__host__ __device__ inline int cg_stride(int n1) { return (n1 + 7) & ~7; }

// Kernel configuration chosen by the host for (d, dtype).
struct PassConfig {
    int G;        // lanes per ball (power of two, 1..64)
    int vec;      // elements per lane per load (1, 2, or 4 for FP32)
    int nl;       // loads per lane per row
    int nlmax;    // compile-time bound on nl (2, 4, 8 or 16)
    int waves_per_block;
    int blocks;   // grid size
    int64_t bw;   // balls per wave (multiple of 64 / G)
    int nwaves;   // blocks * waves_per_block
    int dma;      // rows stream through the waves' LDS rings
    int stages;   // ring blocks per wave (DMA_MIN_STAGES or DMA_MAX_STAGES)
    int spec;     // the instance specialized for this group width may be used
    int fill_min, fill_max;  // resident waves of the two instances (smaller, larger)
};

PassConfig choose_pass_config(int64_t m, int d, int dtype, int num_cu);
int pass_min_steps();
constexpr int PASS_OVERSUB_DEFAULT = 1;
int pass_oversub();

// Arguments of the evaluation pass.
struct PassArgs {
    const void* C;
    const void* R;       // nullable
    const void* U;       // nullable (zero multipliers)
    const void* V;
    void* Uout;          // nullable: write updated multipliers (may alias U)
    void* Vout;
    int64_t m;
    int d;
    int dtype;
    const double* state; // device state (StateLayout)
    StateLayout sl;
    RecLayout rl;
    double* rec;         // blocks x rl.len
    int32_t* mid_idx;    // nwaves segments of bw entries
    double* mid_coef;
    int32_t* mid_cnt;    // nwaves
    int32_t* act_idx;    // nwaves segments of bw entries: balls with vector parts
    void* act_coef;      // ACT_NC working-precision coefficients per entry
    double* red;         // reduced record (len), then the group partials
    int* sync;           // arrival counters of the in-kernel reductions (zero between passes)
    int force_mode;      // -1: read S_MODE from state; else PM_EVAL / PM_MULT
    int want_kkt;        // evaluate KKT terms in PM_EVAL (meb_al_eval)
    int want_mid;        // write the mid list (Hessian contraction needed)
    double etas[NT];     // Armijo trial step sizes
};

// Arrival counters (ints) of the in-kernel reductions: SYNC_GROUPS group
// counters and one top counter for the pass, then one counter per tile pair
// of the contraction.  Each counter returns to zero after use.
constexpr int RED_GROUP = 32;      // block records summed per group
constexpr int SYNC_GROUPS = 64;    // at most RED_GROUP * SYNC_GROUPS pass blocks
constexpr int SYNC_TOP = SYNC_GROUPS;
constexpr int SYNC_SYRK = 128;     // first tile-pair counter
constexpr int SYNC_LEN = 4096;
constexpr int SYNC_CG = SYNC_LEN - 1;  // arrival counter of a Hessian-vector product

struct SyrkArgs {
    const void* C;
    const void* V;
    const void* U;
    int d;
    int dtype;
    double* state;       // block 0 writes S_HSKIP; the tile finishers write H
    StateLayout sl;
    const double* red;   // reduced record of the pass
    RecLayout rl;
    const int32_t* mid_cnt;    // per-wave mid counts of the pass
    const int32_t* mid_idx;    // per-wave segments of bw entries
    const double* mid_coef;
    int nwaves;
    int64_t bw;
    double* out;         // ksplit x pairs x T x T partial blocks
    int* sync;           // tile-pair counters (at SYNC_SYRK)
    int ksplit;          // blocks per tile pair in the launch (a pass uses a prefix of them)
    int tile;
    int ntile;           // tiles per dimension
    double skip_k;       // in a line-search pass, skip when K exceeds this
    int mm;              // arithmetic: SYRK_VEC, SYRK_MFMA_F64, SYRK_MFMA_F32, SYRK_MFMA_BF16
};
// contraction arithmetic (SyrkArgs::mm) and its tile width
enum : int { SYRK_VEC = 0, SYRK_MFMA_F64 = 1, SYRK_MFMA_F32 = 2, SYRK_MFMA_BF16 = 3 };
inline int syrk_tile_of(int mm) { return mm == SYRK_VEC ? 32 : 64; }
// partial-tile doubles an engine reserves for d (the larger of the two tilings)
inline size_t syrk_partial_doubles(int d, int ksplit) {
    size_t best = (size_t)CG_BLOCKS * d;  // the CG products' block sums share the buffer
    for (int t : {32, 64}) {
        const size_t nt = (size_t)(d + t - 1) / t;
        const size_t v = (size_t)ksplit * nt * (nt + 1) / 2 * t * t;
        if (v > best) best = v;
    }
    return best;
}

// One instance of the multi-instance step: the arguments of its pass,
// contraction and control kernels.  Lives in a device table indexed by slot;
// a tick names the slots it steps.
struct BatchItem {
    PassArgs pa;
    PassConfig pc;
    SyrkArgs sa;
    int* flag;            // nullable: the state's mode after each control step
};

// Instances of one launch and the first flat block of each (ascending);
// passed by value as a kernel argument.
constexpr int TICK_MAX = 128;
struct TickList {
    int n;
    int slot[TICK_MAX];
    int off[TICK_MAX + 1];
};

// One solver step (pass with its reduction, contraction with the Hessian
// assembly, control) for the `n` instances slots[0..n) of the device table
// `dtab`; `htab` is its host mirror (read for the launch shapes).  The pass
// takes one launch per template instance among the items; the other two
// kernels one launch per TICK_MAX items.
// The pass of a group of items that share one template instance.
hipError_t launch_pass_group(const BatchItem* dtab, const TickList& L, int blocks, int max_d, int max_stages,
                             int dtype, const PassConfig& cfg, hipStream_t s);
hipError_t launch_tick(const BatchItem* dtab, const BatchItem* htab, const int* slots, int n, hipStream_t s);
int pass_variant(int dtype, const PassConfig& cfg);
size_t control_lds_bytes(int n1);
size_t newton_lds_bytes(int n1);

// ----------------------------------------------------------------------------
// Launchers (meb_kernels.hip).  All return hipError_t of the launch.
// ----------------------------------------------------------------------------
// The evaluation pass: the solver's evaluation or multiplier update (+ KKT
// + next evaluation) as the state's mode says, nothing when the run is done;
// force_mode = PM_EVAL gives a single evaluation (want_kkt adds the updated
// multipliers and the KKT terms).  The last block to finish sums the block
// records into a.red (fixed order), so the record is complete when the
// launch is.
hipError_t launch_pass(const PassArgs& a, const PassConfig& cfg, hipStream_t s);
// the single evaluation (force_mode >= 0), called by launch_pass
hipError_t launch_pass_eval(const PassArgs& a, const PassConfig& cfg, hipStream_t s);
// The rank-one Hessian part over the pass's mid list, tiled; the last block
// of each tile pair sums the k-split partials and writes its part of H
// (with the diagonal and the r row and column from the record) into the
// state, unless the contraction is skipped.
hipError_t launch_syrk(const SyrkArgs& a, hipStream_t s);
// one conjugate-gradient iteration (or, with a.init, the opening
// preconditioner pass); nothing unless the state's mode is PM_CG and the
// solve has not stopped
hipError_t launch_cg_iter(const CgArgs& a, hipStream_t s);
// the direction from a finished CG solve; `flag` as for the control step
hipError_t launch_cg_finish(double* state, StateLayout sl, int* flag, hipStream_t s);
// the Newton solve of a step (nothing unless the control step asked for one);
// `flag` (nullable) receives the state's mode after it
hipError_t launch_newton(double* state, StateLayout sl, int* flag, hipStream_t s);
int syrk_ksplit(int64_t m, int d, int nwaves);
hipError_t launch_control(double* state, StateLayout sl, RecLayout rl, const double* red, int* flag_host_mapped,
                          hipStream_t s);
// control step and Newton step in one launch (systems of n1 unknowns for
// which control_newton_fused(n1) holds); the same effect as launch_control
// followed by launch_newton
bool control_newton_fused(int n1);
hipError_t launch_control_newton(double* state, StateLayout sl, RecLayout rl, const double* red, int* flag,
                                 hipStream_t s);
// g of a single evaluation, and a copy of the H assembled in the state
hipError_t launch_eval_outputs(const double* state, StateLayout sl, RecLayout rl, const double* red, double sigma,
                               double tau, const double* y, const double* xbar, double* out_g, double* out_H,
                               hipStream_t s);
// Partition of a scan over rows (the lanes per row are chosen per launch).
struct ScanCfg {
    int64_t bw;  // rows per wave, a multiple of 64
    int nwaves, blocks;
};
ScanCfg scan_config(int64_t m, int d, int num_cu);
// Placement of a scan's hits: with offs, hit k of wave w goes to
// seg[offs[w] + k] if below cap (offs from a counting pass), and the scan
// does nothing if *gate is zero; without, into the wave's own segment.
struct ScanPlace {
    const int64_t* offs = nullptr;
    int64_t cap = 0;
    const int64_t* gate = nullptr;
};
// mode 0: feasibility, 1: screening, 2: FP32 preparation (see meb_kernels.hip)
hipError_t launch_scan(int mode, const void* C, const void* R, int64_t m, int d, int dtype, const double* x,
                       double r, double thr, double* slack, float* C32, float* R32, const ScanCfg& c, double* wmax,
                       int64_t* warg, int64_t* wcnt, int64_t* seg, hipStream_t s, const ScanPlace& pl = ScanPlace());
hipError_t launch_scan_finalize(const int64_t* wcnt, const double* wmax, const int64_t* warg, int nw, int64_t* offs,
                                int64_t* total, double* out_max, int64_t* out_arg, hipStream_t s);
hipError_t launch_scan_copy(const int64_t* seg, const int64_t* wcnt, const int64_t* offs, int nw, int64_t bw,
                            int64_t* out, int64_t cap, hipStream_t s);
hipError_t launch_gather(const void* C, const void* R, const void* U, const void* V, int src_dtype,
                         const int64_t* idx, int64_t n, int d, double* C_out, double* R_out, double* U_out,
                         double* V_out, hipStream_t s);
hipError_t launch_scatter_mult(const double* Ured, const double* Vred, const int64_t* idx, int64_t n, int d,
                               double* U_out, double* V_out, hipStream_t s);
hipError_t launch_dense_mult(const void* U, const void* V, int dtype, int64_t m, int d, double* U_out,
                             double* V_out, hipStream_t s);
hipError_t launch_chol_solve(int n, double* A, double* b, int* info, hipStream_t s);
// the multi-workgroup factorization (n >= MCHOL_MIN_N): b (device) holds the
// solution on return; yw n, ldw MCHOL_NB^2 and badw 1 doubles of scratch
hipError_t launch_chol_solve_mwg(int n, double* A, double* b, double* yw, double* ldw, double* badw, int* info,
                                 hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);
// dst[k] = (double)src[k] (exact), k < n
hipError_t launch_widen_f32(const float* src, double* dst, int64_t n, hipStream_t s);
hipError_t launch_fill_bytes_zero(void* p, size_t bytes, hipStream_t s);

// Device-to-device copies between state slots and small vectors are done
// with hipMemcpyAsync by the host.

}  // namespace meb
