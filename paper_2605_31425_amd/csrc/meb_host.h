// Host-side pieces of libmeb.so shared by the C ABI (meb_api.hip) and the
// multi-instance server (meb_server.hip): workspace carving, the buffers of
// one evaluation engine, the scan helpers, and the solve as a resumable job.
//
// A solve is a sequence of phases: scale and FP32 preparation, the FP32
// screening run, screening and gather, FP64 run(s) with the full FP64
// feasibility check and reinsertion, and the radius fix-up (Section 4.2).
// Each phase enqueues its work on a stream and ends with a small readback
// into the job's pinned staging; the driver calls on_ready() once that
// readback has completed.  During a ripALM run the driver owns the stepping:
// meb_solve enqueues single-instance steps, the server batches the steps of
// many jobs into one launch per kernel.  Either way every instance runs the
// same kernels with the same launch shapes, so its results do not depend on
// the driver or on the other jobs.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/meb.h"
#include "meb_internal.h"

namespace meb {

// Sets the calling thread's last error message; returns `code`.
int fail(int code, const std::string& msg);
const char* last_error_text();

#define HIPCHK(expr)                                                                                      \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return ::meb::fail(MEB_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CHK(expr)                \
    do {                         \
        int rc_ = (expr);        \
        if (rc_ < 0) return rc_; \
    } while (0)

constexpr size_t ALIGN = 256;

inline size_t al(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

struct Arena {
    char* base;
    size_t size;
    size_t off;
    template <typename T>
    T* take(size_t n) {
        size_t o = al(off);
        off = o + al(n * sizeof(T));
        return reinterpret_cast<T*>(base + o);
    }
    bool ok() const { return off <= size; }
};

// Counting arena: computes the size of a carving without memory.
struct Sizer {
    size_t off = 0;
    template <typename T>
    T* take(size_t n) {
        off = al(off) + al(n * sizeof(T));
        return nullptr;
    }
};

int device_cus();
// shape, dtype, pointer and alignment checks shared by the entry points
int check_common(const void* C, int64_t m, int32_t d, int32_t dtype);
// contraction arithmetic (SYRK_*) of a run of precision dtype under option hess
int syrk_arith(int hess, int dtype, int d);
double now_ms();
inline size_t dtype_size(int dtype) { return dtype == MEB_F64 ? 8 : 4; }

// ---------------------------------------------------------------------------
// Evaluation engine: the buffers of the pass / reduce / contraction / control
// sequence for one instance shape.
// ---------------------------------------------------------------------------
struct Engine {
    int64_t m = 0;
    int d = 0;
    int dtype = 0;
    PassConfig pc{};
    StateLayout sl{};
    RecLayout rl{};
    int ksplit = 0;
    // capacities the carving provides: block records, mid / active list
    // entries, contraction blocks per tile pair (those of m unless raised by
    // reserve_subsets)
    int64_t rec_cap = 0, list_cap = 0;
    int ks_cap = 0;
    int mm = 0;         // contraction arithmetic (SYRK_*), chosen per run
    int cg_iters = 0;   // > 0: matrix-free Newton directions with this many CG launches per step
    double* state = nullptr;
    double* rec = nullptr;
    double* red = nullptr;
    int32_t* mid_idx = nullptr;
    double* mid_coef = nullptr;
    int32_t* mid_cnt = nullptr;
    int32_t* act_idx = nullptr;
    double* act_coef = nullptr;  // ACT_NC per entry, in the working precision
    double* syrk = nullptr;
    int* sync = nullptr;         // SYNC_LEN arrival counters, zero between kernels
    double skip_k = INFINITY;

    void setup(int64_t m_, int d_, int dtype_);
    // raise the capacities so that setup(n) for any n <= m fits the same carving
    void reserve_subsets();
    // setup(n) inside the carving of this engine (n <= its m after
    // reserve_subsets); false if it does not fit
    bool resize_within(int64_t n);
    template <typename A>
    void carve(A& a) {
        state = a.template take<double>(sl.len);
        rec = a.template take<double>((size_t)rec_cap * rl.len);
        red = a.template take<double>((size_t)(SYNC_GROUPS + 1) * rl.len);
        const size_t cap = (size_t)list_cap;
        mid_idx = a.template take<int32_t>(cap);
        mid_coef = a.template take<double>(cap);
        mid_cnt = a.template take<int32_t>(pc.nwaves);
        act_idx = a.template take<int32_t>(cap);
        act_coef = a.template take<double>(cap * ACT_NC);
        syrk = a.template take<double>(syrk_partial_doubles(d, ks_cap));
        sync = a.template take<int>(SYNC_LEN);
    }
    PassArgs args(const void* C, const void* R, void* U, void* V) const;
    SyrkArgs syrk_args(const void* C, const void* U, const void* V) const;
    CgArgs cg_args(const void* C, const void* U, const void* V, int init) const;
    // the multi-instance table entry of a run over (C, R, U, V)
    BatchItem item(const PassArgs& a, int* flag) const;
    // pass (with its reduction) + contraction (with the H assembly)
    // (+ control when `control`); with `ev0` non-null, the pass launch is
    // bracketed by the two events
    // `flag` (nullable, host-mapped) receives the state's mode after the control step
    int step(const PassArgs& a, bool control, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
             int* flag = nullptr);
    // clears the arrival counters (before the first kernel of a run)
    int reset_sync(hipStream_t s);
};

size_t engine_bytes(int64_t m, int d, int dtype);

// ---------------------------------------------------------------------------
// Scan helpers (feasibility check / screening / FP32 preparation).  The
// results of a scan are three words in `res` (device): the maximum, its
// smallest argmax and the number of listed rows.
// ---------------------------------------------------------------------------
struct ScanBufs {
    ScanCfg cfg{};
    int64_t m = 0;
    int d = 0;
    double* wmax = nullptr;
    int64_t* warg = nullptr;
    int64_t* wcnt = nullptr;
    int64_t* offs = nullptr;
    int64_t* seg = nullptr;
    double* res = nullptr;
    double* cvec = nullptr;
    void setup(int64_t m_, int d_);
    template <typename A>
    void carve(A& a) {
        wmax = a.template take<double>(cfg.nwaves);
        warg = a.template take<int64_t>(cfg.nwaves);
        wcnt = a.template take<int64_t>(cfg.nwaves);
        offs = a.template take<int64_t>(cfg.nwaves);
        seg = a.template take<int64_t>((size_t)cfg.nwaves * cfg.bw);
        res = a.template take<double>(4);
        cvec = a.template take<double>((size_t)d + 8);
    }
    double* out_max() const { return res; }
    int64_t* out_arg() const { return reinterpret_cast<int64_t*>(res + 1); }
    int64_t* total() const { return reinterpret_cast<int64_t*>(res + 2); }
};

size_t scan_bytes(int64_t m, int d);

// Enqueue-only scans; the three result words are copied into host `out`
// (pinned, 3 doubles; words 1 and 2 hold int64 bits).  c_dev is a device
// vector of d doubles.
int enq_check(const void* C, const void* R, int64_t m, int d, int dtype, double r, const double* c_dev, double eps,
              ScanBufs& b, int64_t* viol_idx, int64_t viol_cap, double* out, hipStream_t s);
int enq_screen(const void* C, const void* R, int64_t m, int d, int dtype, double r, const double* c_dev, double tol,
               ScanBufs& b, int64_t* keep_idx, double* slack, double* out, hipStream_t s);
int enq_prepare(const double* C, const double* R, int64_t m, int d, const double* origin_dev, float* C32, float* R32,
                ScanBufs& b, double* out, hipStream_t s);

inline int64_t word_i64(const double* w) {
    int64_t v;
    memcpy(&v, w, 8);
    return v;
}

// ---------------------------------------------------------------------------
// meb_solve workspace
// ---------------------------------------------------------------------------
struct SolveWs {
    Engine e32, e64;  // FP32 run on all m; FP64 run (all m, or the reduced set)
    ScanBufs scan;
    float* C32 = nullptr;
    float* R32 = nullptr;
    float* U32 = nullptr;
    float* V32 = nullptr;
    double* U64 = nullptr;
    double* V64 = nullptr;
    double* Cred = nullptr;
    double* Rred = nullptr;
    int64_t* keep = nullptr;  // retained indices (device)
    int64_t* viol = nullptr;  // violated indices (device)
    double* Cin = nullptr;    // FP64 copy of FP32 input (widened exactly), else unused
    double* Rin = nullptr;
    void setup(int64_t m, int d, const meb_options* o);
    template <typename A>
    void carve(A& a, int64_t m, int d, const meb_options* o, bool has_r, int in_dtype) {
        if (in_dtype == MEB_F32) {
            Cin = a.template take<double>((size_t)m * d);
            Rin = has_r ? a.template take<double>((size_t)m) : nullptr;
        }
        e64.carve(a);
        scan.carve(a);
        U64 = a.template take<double>((size_t)m);
        V64 = a.template take<double>((size_t)m * d);
        if (o->mode == MEB_MODE_MIXED) {
            e32.carve(a);
            C32 = a.template take<float>((size_t)m * d);
            R32 = has_r ? a.template take<float>((size_t)m) : nullptr;
            U32 = a.template take<float>((size_t)m);
            V32 = a.template take<float>((size_t)m * d);
            Cred = a.template take<double>((size_t)m * d);
            Rred = a.template take<double>((size_t)m);
            keep = a.template take<int64_t>((size_t)m);
            viol = a.template take<int64_t>((size_t)m);
        }
    }
};

size_t solve_ws_bytes(int64_t m, int d, int in_dtype, const meb_options* o);

// ---------------------------------------------------------------------------
// Pinned staging of one job (doubles): readback targets and the sources of
// small uploads.  A region is rewritten only after the job has observed the
// completion of the copy that used it last.
// ---------------------------------------------------------------------------
struct JobPin {
    double* hdr = nullptr;   // S_NSCALAR scalars, then the iterate (n1): one copy
    double* x = nullptr;     // = hdr + S_NSCALAR
    double* c1 = nullptr;    // d: the first center
    double* init = nullptr;  // StateLayout(d).H doubles: initial state of a run
    double* cvec = nullptr;  // d: center uploaded for a scan
    double* scal = nullptr;  // 8: scan results and small constants
    static size_t doubles(int d) {
        const StateLayout sl = StateLayout::make(d);
        return (size_t)S_NSCALAR + 3 * ((size_t)d + 8) + (size_t)sl.H + 8 + 8;
    }
    void carve(double* base, int d) {
        const StateLayout sl = StateLayout::make(d);
        hdr = base;
        x = hdr + S_NSCALAR;
        c1 = x + d + 8;
        init = c1 + d + 8;
        cvec = init + sl.H;
        scal = cvec + d + 8;
    }
};

enum class JobPhase : int { Start, WaitPrep, Run, WaitRunEnd, WaitScreen, WaitCheck, WaitViol, Done };

struct Job {
    // request
    const void* C = nullptr;
    const void* R = nullptr;
    const void* C_in = nullptr;  // the caller's FP32 input, when widened
    const void* R_in = nullptr;
    int64_t m = 0;
    int d = 0;
    meb_options o{};
    double* U_out = nullptr;  // device, nullable (full-size multipliers)
    double* V_out = nullptr;
    // resources
    SolveWs w;
    JobPin pin;
    // progress
    JobPhase ph = JobPhase::Start;
    int run_id = 0;  // 0: FP32 screening run, 1: FP64 run
    Engine* e = nullptr;
    PassArgs pa{};
    int64_t steps = 0, max_steps = 0;
    bool forced_end = false;  // the driver ended the run at max_steps
    double run_pass_ms = 0;   // filled by a profiling driver before end_run
    int run_launches = 0;
    int last_k = -1;
    double L = 0, tau_raw = 0, sigma0_raw = 0;
    std::vector<double> c1, x1, xw, xfin;
    double sigma1 = 0, sigma_w = 0;
    bool warm1 = true;  // the screening run converged: its multipliers warm-start the refinement
    double tol_red = 0;
    int screen_tries = 0;
    int64_t n_red = 0;
    int64_t n_viol = 0;
    int rounds = 0;
    bool fixup_only = false;
    double mreach = -INFINITY;
    int64_t* viol_h = nullptr;  // pinned
    size_t viol_cap = 0;
    int64_t* keep_pin = nullptr;  // pinned
    size_t keep_cap = 0;
    std::vector<int64_t> keep_h, keep_sorted;
    meb_stats st{};
    int status = MEB_OK;
    double r_out = 0;
    double t_start = 0, t_mark = 0, t_run = 0, t_check = 0, tr_total = 0, tc_total = 0;

    Job() = default;
    Job(const Job&) = delete;
    Job& operator=(const Job&) = delete;
    ~Job();

    // Validates and carves the workspace; `pin_base` holds JobPin::doubles(d).
    // C and R are FP64, or FP32 (in_dtype), which the job first widens into the workspace.
    int init(const void* C, const void* R, int64_t m, int d, int in_dtype, const meb_options* o, void* ws,
             size_t ws_bytes, double* pin_base, double* U_out, double* V_out);
    int start(hipStream_t s);     // Start -> WaitPrep
    int on_ready(hipStream_t s);  // a Wait* phase's readback has completed
    int end_run(hipStream_t s);   // Run -> WaitRunEnd
    bool stepping() const { return ph == JobPhase::Run; }
    bool done() const { return ph == JobPhase::Done; }

  private:
    int begin_run(int id, Engine& eng, const void* Cr, const void* Rr, void* U, void* V, const double* x0,
                  double sigma_raw, double tol, double eps, hipStream_t s);
    int screen(hipStream_t s);
    int start_fp64_reduced(hipStream_t s);
    int check(hipStream_t s);
    int finish_mixed(hipStream_t s);
    void finish();
};

// Runs a job to completion on one stream with single-instance launches
// (batches of four steps between polls of the state header).
int drive_sync(Job& j, hipStream_t s);

}  // namespace meb
