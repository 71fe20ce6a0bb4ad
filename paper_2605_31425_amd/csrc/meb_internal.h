// Internal declarations shared by the host solver and the kernel launchers of
// libmeb.so.  Nothing here is part of the public C ABI (include/meb.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

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
    S_STATUS,        // 0 running, 1 converged, 2 max iterations / stall, -1 numeric failure
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
    S_NSCALAR = 48
};

struct StateLayout {
    int n1;      // d + 1
    int xb;      // current inner iterate (line-search base)
    int dir;     // Newton direction (possibly scaled by the line search)
    int xbar;    // proximal center
    int ab;      // auxiliary sequence (alpha, beta)
    int gb;      // gradient at xb
    int tmp;     // scratch vector
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

// Pass modes.
enum PassMode : int { PM_EVAL = 0, PM_MULT = 1, PM_DONE = 2 };

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
};

PassConfig choose_pass_config(int64_t m, int d, int dtype, int num_cu);

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
    int force_mode;      // -1: read S_MODE from state; else PM_EVAL / PM_MULT
    int want_kkt;        // evaluate KKT terms in PM_EVAL (meb_al_eval)
    int want_mid;        // write the mid list (Hessian contraction needed)
    int dense_vout;      // write every V row of the update (else only u != 0 rows)
    double etas[NT];     // Armijo trial step sizes
};

struct SyrkArgs {
    const void* C;
    const void* V;
    const void* U;
    int d;
    int dtype;
    double* state;       // block 0 writes S_HSKIP
    StateLayout sl;
    const double* red;   // reduced record (its mid count)
    RecLayout rl;
    const int32_t* list_idx;   // compacted mid list (K entries)
    const double* list_coef;
    const int64_t* list_total; // K
    double* out;         // ksplit x pairs x T x T partial blocks
    int ksplit;
    int tile;
    int ntile;           // tiles per dimension
    double skip_k;       // in a line-search pass, skip when K exceeds this
};

// Concatenates the per-wave mid-list segments into one list (ascending wave
// order): offsets by a single-block scan, then a copy.
// One instance of the multi-instance step: the arguments of its pass,
// reduction, contraction, assembly and control kernels.  Lives in a device
// table indexed by slot; a tick names the slots it steps.
struct BatchItem {
    PassArgs pa;
    PassConfig pc;
    SyrkArgs sa;
    double* red;          // reduced record, then the slice partials
    int64_t* list_offs;   // per-wave offsets of the compacted mid list
    int* flag;            // nullable: the state's mode after each control step
    int ksplit, ntile;
    int use_syrk;
};

// Instances of one launch and the first flat block of each (ascending);
// passed by value as a kernel argument.
constexpr int TICK_MAX = 128;
struct TickList {
    int n;
    int slot[TICK_MAX];
    int off[TICK_MAX + 1];
};

// One solver step (pass, reduction, mid-list compaction, contraction,
// assembly, control) for the `n` instances slots[0..n) of the device table
// `dtab`; `htab` is its host mirror (read for the launch shapes).  The pass
// takes one launch per template instance among the items; every other kernel
// one launch per TICK_MAX items.
// The pass of a group of items that share one template instance.
hipError_t launch_pass_group(const BatchItem* dtab, const TickList& L, int blocks, int max_d, int dtype,
                             const PassConfig& cfg, hipStream_t s);
hipError_t launch_tick(const BatchItem* dtab, const BatchItem* htab, const int* slots, int n, hipStream_t s);
int pass_variant(int dtype, const PassConfig& cfg);
int reduce_nslice(int nrec);
size_t control_lds_bytes(int n1);

hipError_t launch_mid_compact(const int32_t* mid_cnt, int nwaves, int64_t bw, const int32_t* seg_idx,
                              const double* seg_coef, int64_t* offs, int64_t* total, int32_t* out_idx,
                              double* out_coef, const double* state, hipStream_t s);

// ----------------------------------------------------------------------------
// Launchers (meb_kernels.hip).  All return hipError_t of the launch.
// ----------------------------------------------------------------------------
// The evaluation pass: the solver's evaluation or multiplier update (+ KKT
// + next evaluation) as the state's mode says, nothing when the run is done;
// force_mode = PM_EVAL gives a single evaluation (want_kkt adds the updated
// multipliers and the KKT terms).
hipError_t launch_pass(const PassArgs& a, const PassConfig& cfg, hipStream_t s);
// the single evaluation (force_mode >= 0), called by launch_pass
hipError_t launch_pass_eval(const PassArgs& a, const PassConfig& cfg, hipStream_t s);
// Sums (maxima for the KKT maxima) of nrec records of len doubles, `stride`
// doubles apart; the pass leaves one record per block at stride
// waves_per_block * len.
hipError_t launch_reduce_records(const double* rec, int nrec, int len, int64_t stride, double* out, hipStream_t s);
hipError_t launch_syrk(const SyrkArgs& a, hipStream_t s);
int syrk_ksplit(int d);
int syrk_tile();
hipError_t launch_control(double* state, StateLayout sl, RecLayout rl, const double* red, int* flag_host_mapped,
                          hipStream_t s);
hipError_t launch_assemble(double* state, StateLayout sl, RecLayout rl, const double* red, const double* syrk,
                           int ksplit, int ntile, int have_syrk, hipStream_t s);
hipError_t launch_eval_assemble(const double* state, StateLayout sl, RecLayout rl, const double* red,
                                const double* syrk_out, int ksplit, int tile, int ntile, int have_syrk, double sigma,
                                double tau, const double* x1, const double* xbar, double* out_g, double* out_H,
                                hipStream_t s);
struct ScanCfg {
    int G, vec, nl;
    int64_t bw;  // rows per wave
    int nwaves, blocks;
};
ScanCfg scan_config(int64_t m, int d, int num_cu);
// mode 0: feasibility, 1: screening, 2: FP32 preparation (see meb_kernels.hip)
hipError_t launch_scan(int mode, const void* C, const void* R, int64_t m, int d, int dtype, const double* x,
                       double r, double thr, double* slack, float* C32, float* R32, const ScanCfg& c, double* wmax,
                       int64_t* warg, int64_t* wcnt, int64_t* seg, hipStream_t s);
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
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);
hipError_t launch_fill_bytes_zero(void* p, size_t bytes, hipStream_t s);

// Device-to-device copies between state slots and small vectors are done
// with hipMemcpyAsync by the host.

}  // namespace meb
