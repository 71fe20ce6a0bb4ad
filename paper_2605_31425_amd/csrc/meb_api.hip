// Host side of libmeb.so: the C ABI of include/meb.h, workspace carving, and
// the drivers of plain FP64 ripALM and of the mixed-precision reduction.
//
// A ripALM run is a device-resident state machine.  The host enqueues a fixed
// sequence per Newton step -- evaluation pass, record reduction, rank-one
// Hessian contraction, control step -- and the control kernel decides on the
// device what the next pass computes (Armijo trials along the Newton
// direction, a plain re-evaluation, or the multiplier update fused with the
// first evaluation of the next outer iteration).  The host only polls the
// state's scalar header every few steps to learn when the run has ended.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <iterator>
#include <chrono>
#include <string>
#include <vector>

#include "../../include/meb.h"
#include "meb_internal.h"

using namespace meb;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(MEB_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CHK(expr)                  \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ < 0) return rc_;   \
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

int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess && p.multiProcessorCount > 0)
            cus[dev] = p.multiProcessorCount;
        else
            cus[dev] = 256;
    }
    return cus[dev];
}

// Thread-local pinned staging for small device-to-host reads.
struct Pinned {
    double* buf = nullptr;
    size_t cap = 0;
    ~Pinned() {
        if (buf) (void)hipHostFree(buf);
    }
    double* get(size_t n) {
        if (n > cap) {
            if (buf) (void)hipHostFree(buf);
            buf = nullptr;
            cap = 0;
            if (hipHostMalloc((void**)&buf, n * sizeof(double), hipHostMallocDefault) != hipSuccess) return nullptr;
            cap = n;
        }
        return buf;
    }
};
thread_local Pinned g_pin;

size_t dtype_size(int dtype) { return dtype == MEB_F64 ? 8 : 4; }

// Thread-local pool of HIP events for the optional per-pass timing.
struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipEvent_t at(size_t i) {
        while (ev.size() <= i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev.push_back(e);
        }
        return ev[i];
    }
};
thread_local EventPool g_events;

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
    int ntile = 0, ksplit = 0;
    bool use_syrk = true;
    double* state = nullptr;
    double* rec = nullptr;
    double* red = nullptr;
    int32_t* mid_idx = nullptr;
    double* mid_coef = nullptr;
    int32_t* mid_cnt = nullptr;
    double* syrk = nullptr;
    int32_t* list_idx = nullptr;
    double* list_coef = nullptr;
    int64_t* list_offs = nullptr;
    int64_t* list_total = nullptr;
    double skip_k = INFINITY;

    void setup(int64_t m_, int d_, int dtype_) {
        m = m_;
        d = d_;
        dtype = dtype_;
        pc = choose_pass_config(m, d, dtype, device_cus());
        sl = StateLayout::make(d);
        rl = RecLayout::make(d);
        ntile = (d + syrk_tile() - 1) / syrk_tile();
        ksplit = syrk_ksplit(d);
        // a line-search pass skips the contraction above this many rows
        skip_k = std::max(4096.0, 16.0 * d);
    }
    template <typename A>
    void carve(A& a) {
        state = a.template take<double>(sl.len);
        rec = a.template take<double>((size_t)pc.nwaves * rl.len);
        red = a.template take<double>((size_t)(32 + 1) * rl.len);
        const size_t cap = (size_t)pc.nwaves * (size_t)pc.bw;
        mid_idx = a.template take<int32_t>(cap);
        mid_coef = a.template take<double>(cap);
        mid_cnt = a.template take<int32_t>(pc.nwaves);
        const size_t pairs = (size_t)ntile * (ntile + 1) / 2;
        syrk = a.template take<double>((size_t)ksplit * pairs * syrk_tile() * syrk_tile());
        list_idx = a.template take<int32_t>(cap);
        list_coef = a.template take<double>(cap);
        list_offs = a.template take<int64_t>(pc.nwaves);
        list_total = a.template take<int64_t>(4);
    }
    PassArgs args(const void* C, const void* R, void* U, void* V) const {
        PassArgs a;
        memset(&a, 0, sizeof(a));
        a.C = C;
        a.R = R;
        a.U = U;
        a.V = V;
        a.Uout = U;
        a.Vout = V;
        a.m = m;
        a.d = d;
        a.dtype = dtype;
        a.state = state;
        a.sl = sl;
        a.rl = rl;
        a.rec = rec;
        a.mid_idx = mid_idx;
        a.mid_coef = mid_coef;
        a.mid_cnt = mid_cnt;
        a.force_mode = -1;
        a.want_kkt = 0;
        a.want_mid = 1;
        a.dense_vout = 0;
        for (int l = 0; l < NT; ++l) a.etas[l] = solver_eta(l);
        return a;
    }
    SyrkArgs syrk_args(const void* C, const void* U, const void* V) const {
        SyrkArgs s;
        memset(&s, 0, sizeof(s));
        s.C = C;
        s.U = U;
        s.V = V;
        s.d = d;
        s.dtype = dtype;
        s.state = state;
        s.sl = sl;
        s.red = red;
        s.rl = rl;
        s.list_idx = list_idx;
        s.list_coef = list_coef;
        s.list_total = list_total;
        s.skip_k = skip_k;
        s.out = syrk;
        s.ksplit = ksplit;
        s.tile = syrk_tile();
        s.ntile = ntile;
        return s;
    }
    // pass + reduce + contraction (+ control when `control`); with `ev0`
    // non-null, the pass launch is bracketed by the two events
    int step(const PassArgs& a, bool control, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
        if (ev0) HIPCHK(hipEventRecord(ev0, s));
        HIPCHK(launch_pass(a, pc, 3, s));
        if (ev1) HIPCHK(hipEventRecord(ev1, s));
        HIPCHK(launch_reduce_records(rec, pc.blocks, rl.len, (int64_t)pc.waves_per_block * rl.len, red, s));
        if (use_syrk && a.want_mid) {
            HIPCHK(launch_mid_compact(mid_cnt, pc.nwaves, pc.bw, mid_idx, mid_coef, list_offs, list_total, list_idx,
                                      list_coef, state, s));
            HIPCHK(launch_syrk(syrk_args(a.C, a.Uout ? a.Uout : a.U, a.Vout ? a.Vout : a.V), s));
        }
        if (control) HIPCHK(launch_assemble(state, sl, rl, red, syrk, ksplit, ntile, use_syrk ? 1 : 0, s));
        if (control) HIPCHK(launch_control(state, sl, rl, red, nullptr, s));
        return MEB_OK;
    }
};

size_t engine_bytes(int64_t m, int d, int dtype) {
    Engine e;
    e.setup(m, d, dtype);
    Sizer sz;
    e.carve(sz);
    return sz.off;
}

// ---------------------------------------------------------------------------
// Scan helpers (feasibility check / screening)
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
    double* out_max = nullptr;
    int64_t* out_arg = nullptr;
    int64_t* total = nullptr;
    double* cvec = nullptr;
    void setup(int64_t m_, int d_) {
        m = m_;
        d = d_;
        cfg = scan_config(m, d, device_cus());
    }
    template <typename A>
    void carve(A& a) {
        wmax = a.template take<double>(cfg.nwaves);
        warg = a.template take<int64_t>(cfg.nwaves);
        wcnt = a.template take<int64_t>(cfg.nwaves);
        offs = a.template take<int64_t>(cfg.nwaves);
        seg = a.template take<int64_t>((size_t)cfg.nwaves * cfg.bw);
        out_max = a.template take<double>(4);
        out_arg = a.template take<int64_t>(4);
        total = a.template take<int64_t>(4);
        cvec = a.template take<double>((size_t)d + 8);
    }
};

size_t scan_bytes(int64_t m, int d) {
    ScanBufs b;
    b.setup(m, d);
    Sizer s;
    b.carve(s);
    return s.off;
}

// max_i (r_i + ||c - c_i|| - r) with its smallest argmax, and the ascending
// list of {i : r_i + ||c - c_i|| - r > eps} (first viol_cap entries).
int run_check(const void* C, const void* R, int64_t m, int d, int dtype, double r, const double* c_host, double eps,
              ScanBufs& b, double* dmax, int64_t* argmax, int64_t* viol_idx, int64_t viol_cap, int64_t* n_viol,
              hipStream_t s) {
    HIPCHK(hipMemcpyAsync(b.cvec, c_host, sizeof(double) * d, hipMemcpyHostToDevice, s));
    HIPCHK(launch_scan(0, C, R, m, d, dtype, b.cvec, r, eps, nullptr, nullptr, nullptr, b.cfg, b.wmax, b.warg, b.wcnt,
                       b.seg, s));
    HIPCHK(launch_scan_finalize(b.wcnt, b.wmax, b.warg, b.cfg.nwaves, b.offs, b.total, b.out_max, b.out_arg, s));
    if (viol_idx && viol_cap > 0)
        HIPCHK(launch_scan_copy(b.seg, b.wcnt, b.offs, b.cfg.nwaves, b.cfg.bw, viol_idx, viol_cap, s));
    double* h = g_pin.get(3);
    if (!h) return fail(MEB_ERR_HIP, "pinned host allocation failed");
    HIPCHK(hipMemcpyAsync(h, b.out_max, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h + 1, b.out_arg, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h + 2, b.total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (dmax) *dmax = h[0];
    int64_t a, n;
    memcpy(&a, h + 1, 8);
    memcpy(&n, h + 2, 8);
    if (argmax) *argmax = a;
    if (n_viol) *n_viol = n;
    return MEB_OK;
}

int run_screen(const void* C, const void* R, int64_t m, int d, int dtype, double r, const double* c_host, double tol,
               ScanBufs& b, int64_t* keep_idx, int64_t* n_keep, double* slack, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(b.cvec, c_host, sizeof(double) * d, hipMemcpyHostToDevice, s));
    HIPCHK(launch_scan(1, C, R, m, d, dtype, b.cvec, r, tol, slack, nullptr, nullptr, b.cfg, nullptr, nullptr, b.wcnt,
                       b.seg, s));
    HIPCHK(launch_scan_finalize(b.wcnt, nullptr, nullptr, b.cfg.nwaves, b.offs, b.total, nullptr, nullptr, s));
    HIPCHK(launch_scan_copy(b.seg, b.wcnt, b.offs, b.cfg.nwaves, b.cfg.bw, keep_idx, m, s));
    double* h = g_pin.get(1);
    if (!h) return fail(MEB_ERR_HIP, "pinned host allocation failed");
    HIPCHK(hipMemcpyAsync(h, b.total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t n;
    memcpy(&n, h, 8);
    *n_keep = n;
    return MEB_OK;
}

// FP32 copy shifted by `origin` (device, d) and L = max_i ||c_i - origin|| + r_i.
int run_prepare(const double* C, const double* R, int64_t m, int d, const double* origin_dev, float* C32, float* R32,
                ScanBufs& b, double* L, hipStream_t s) {
    HIPCHK(launch_scan(2, C, R, m, d, MEB_F64, origin_dev, 0.0, 0.0, nullptr, C32, R32, b.cfg, b.wmax, b.warg,
                       nullptr, nullptr, s));
    HIPCHK(launch_scan_finalize(nullptr, b.wmax, b.warg, b.cfg.nwaves, nullptr, nullptr, b.out_max, b.out_arg, s));
    double* h = g_pin.get(1);
    if (!h) return fail(MEB_ERR_HIP, "pinned host allocation failed");
    HIPCHK(hipMemcpyAsync(h, b.out_max, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *L = h[0];
    return MEB_OK;
}

// ---------------------------------------------------------------------------
// One ripALM run on (C, R) with multipliers (U, V) in `dtype`.
// ---------------------------------------------------------------------------
struct RunParams {
    double L;
    double sigma_raw;  // first penalty of this run
    double tau_raw;
    double tol;
    double eps;
    const meb_options* o;
};

struct RunResult {
    std::vector<double> x;  // d + 1
    double sigma_end;       // raw
    int outer, inner, passes, status;
    double kkt;
    double pass_ms = 0, pass_bytes = 0;
    int launches = 0;
    double sumk = 0, maxk = 0;
};

int run_ripalm(Engine& e, const void* C, const void* R, void* U, void* V, const double* x0, const RunParams& p,
               RunResult& out, hipStream_t s) {
    const int n1 = e.d + 1;
    const meb_options* o = p.o;
    std::vector<double> h(e.sl.len, 0.0);
    h[S_MODE] = PM_EVAL;
    h[S_SIGMA] = p.sigma_raw;
    h[S_SIGMA_NEXT] = std::min(p.sigma_raw * o->sigma_growth, o->sigma_max / p.L);
    h[S_TAU] = p.tau_raw;
    h[S_L] = p.L;
    h[S_RHO] = o->rho;
    h[S_TOL] = p.tol;
    h[S_GROWTH] = o->sigma_growth;
    h[S_SIGMA_MAX] = o->sigma_max / p.L;
    h[S_MAX_OUTER] = o->max_outer;
    h[S_MAX_INNER] = o->max_inner;
    h[S_MAX_LS] = o->max_ls;
    h[S_STALL_OUTER] = o->stall_outer;
    h[S_EPS] = p.eps;
    h[S_BEST_KKT] = INFINITY;
    h[S_VERBOSE] = o->verbose;
    for (int k = 0; k < n1; ++k) {
        h[e.sl.xb + k] = x0[k];
        h[e.sl.xbar + k] = x0[k];
        h[e.sl.ab + k] = x0[k];
    }
    HIPCHK(hipMemcpyAsync(e.state, h.data(), sizeof(double) * e.sl.len, hipMemcpyHostToDevice, s));
    PassArgs a = e.args(C, R, U, V);
    double* hs = g_pin.get(S_NSCALAR);
    if (!hs) return fail(MEB_ERR_HIP, "pinned host allocation failed");
    const int batch = 4;
    const int64_t max_steps = (int64_t)o->max_outer * (o->max_inner + o->max_ls + 2) + 16;
    int64_t steps = 0;
    int last_k = -1;
    const bool prof = o->profile != 0;
    size_t nev = 0;
    for (;;) {
        for (int b = 0; b < batch; ++b) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (prof) {
                e0 = g_events.at(nev);
                e1 = g_events.at(nev + 1);
                if (!e0 || !e1) return fail(MEB_ERR_HIP, "hipEventCreate failed");
                nev += 2;
            }
            CHK(e.step(a, true, s, e0, e1));
        }
        steps += batch;
        HIPCHK(hipMemcpyAsync(hs, e.state, sizeof(double) * S_NSCALAR, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (o->verbose && (int)hs[S_K] != last_k) {
            last_k = (int)hs[S_K];
            fprintf(stderr, "[meb] k=%d sigma=%.3e kkt=%.3e passes=%d newton=%d\n", (int)hs[S_K], hs[S_SIGMA],
                    hs[S_KKT], (int)hs[S_NPASS], (int)hs[S_NINNER]);
        }
        if ((int)hs[S_MODE] == PM_DONE) break;
        if (steps > max_steps) {
            hs[S_STATUS] = 2.0;
            break;
        }
    }
    out.x.resize(n1);
    HIPCHK(hipMemcpyAsync(g_pin.get(S_NSCALAR + n1) + S_NSCALAR, e.state + e.sl.xb, sizeof(double) * n1,
                          hipMemcpyDeviceToHost, s));
    double* hh = g_pin.get(S_NSCALAR + n1);
    HIPCHK(hipMemcpyAsync(hh, e.state, sizeof(double) * S_NSCALAR, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int k = 0; k < n1; ++k) out.x[k] = hh[S_NSCALAR + k];
    out.sigma_end = hh[S_SIGMA];
    out.outer = (int)hh[S_K];
    out.inner = (int)hh[S_NINNER];
    out.passes = (int)hh[S_NPASS];
    out.kkt = hh[S_KKT];
    out.status = (int)hh[S_STATUS];
    out.pass_bytes = hh[S_BYTES];
    out.sumk = hh[S_SUMK];
    out.maxk = hh[S_MAXK];
    if (prof) {
        double ms = 0;
        for (size_t k = 0; k + 1 < nev; k += 2) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, g_events.at(k), g_events.at(k + 1)));
            ms += t;
        }
        out.pass_ms = ms;
        out.launches = (int)(nev / 2);
    }
    if (out.status < 0) return fail(MEB_ERR_NUMERIC, "Newton system not positive definite");
    for (int k = 0; k < n1; ++k)
        if (!std::isfinite(out.x[k])) return fail(MEB_ERR_NUMERIC, "non-finite iterate");
    return MEB_OK;
}

// ---------------------------------------------------------------------------
// meb_solve workspace
// ---------------------------------------------------------------------------
struct SolveWs {
    Engine e32, e64;   // FP32 run on all m; FP64 run (all m, or the reduced set)
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
    double* orig = nullptr;   // d
    void setup(int64_t m, int d, const meb_options* o) {
        e64.setup(m, d, MEB_F64);
        if (o->mode == MEB_MODE_MIXED) e32.setup(m, d, MEB_F32);
        scan.setup(m, d);
    }
    template <typename A>
    void carve(A& a, int64_t m, int d, const meb_options* o, bool has_r) {
        e64.carve(a);
        scan.carve(a);
        U64 = a.template take<double>((size_t)m);
        V64 = a.template take<double>((size_t)m * d);
        orig = a.template take<double>((size_t)d + 8);
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

int check_common(const void* C, int64_t m, int32_t d, int32_t dtype) {
    if (!C) return fail(MEB_ERR_ARG, "C is NULL");
    if (m < 1) return fail(MEB_ERR_ARG, "m must be >= 1");
    if (m > 0x7fffffffLL) return fail(MEB_ERR_ARG, "m must be < 2^31");
    if (d < 1 || d > MEB_MAX_D) return fail(MEB_ERR_ARG, "d must be in [1, MEB_MAX_D]");
    if (dtype != MEB_F64 && dtype != MEB_F32) return fail(MEB_ERR_ARG, "bad dtype");
    const size_t es = dtype_size(dtype);
    if ((uintptr_t)C % es) return fail(MEB_ERR_ARG, "C is not aligned to its element size");
    if ((d % 2 == 1) && d > 1024) return fail(MEB_ERR_UNSUPPORTED, "odd d above 1024 is not supported");
    return MEB_OK;
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int meb_default_options(meb_options* o) {
    if (!o) return fail(MEB_ERR_ARG, "opts is NULL");
    memset(o, 0, sizeof(*o));
    o->rho = 0.9;
    o->sigma0 = 1.0;
    o->sigma_growth = 5.0;
    o->sigma_max = 1e5;
    o->tau = 1.0;
    o->tol_kkt = 1e-8;
    o->tol_kkt_low = 1e-2;
    o->tol_red = 0.03;
    o->eps_feas_rel = 1e-10;
    o->max_outer = 200;
    o->max_inner = 50;
    o->max_ls = 40;
    o->max_reinsert = 20;
    o->mode = MEB_MODE_MIXED;
    o->stall_outer = 3;
    o->verbose = 0;
    o->profile = 0;
    return MEB_OK;
}

const char* meb_last_error(void) { return g_err.c_str(); }

int meb_workspace_size(int64_t m, int32_t d, int32_t dtype, const meb_options* opts, size_t* bytes) {
    if (!bytes) return fail(MEB_ERR_ARG, "bytes is NULL");
    if (m < 1 || d < 1 || d > MEB_MAX_D) return fail(MEB_ERR_ARG, "bad shape");
    if (dtype != MEB_F64 && dtype != MEB_F32) return fail(MEB_ERR_ARG, "bad dtype");
    meb_options def;
    meb_default_options(&def);
    const meb_options* o = opts ? opts : &def;
    SolveWs w;
    w.setup(m, d, o);
    Sizer s;
    w.carve(s, m, d, o, true);
    *bytes = s.off + ALIGN;
    return MEB_OK;
}

int meb_eval_workspace_size(int64_t m, int32_t d, int32_t dtype, size_t* bytes) {
    if (!bytes) return fail(MEB_ERR_ARG, "bytes is NULL");
    if (m < 1 || d < 1 || d > MEB_MAX_D) return fail(MEB_ERR_ARG, "bad shape");
    if (dtype != MEB_F64 && dtype != MEB_F32) return fail(MEB_ERR_ARG, "bad dtype");
    size_t a = engine_bytes(m, d, dtype) + al(sizeof(double) * (2 * (size_t)d + 8));
    size_t b = scan_bytes(m, d);
    *bytes = std::max(a, b) + ALIGN;
    return MEB_OK;
}

int meb_al_eval(const void* C, const void* R, const void* U, const void* V, int64_t m, int32_t d, int32_t dtype,
                const double* x, const double* xbar, double sigma, double tau, const double* dir, int32_t n_eta,
                const double* etas, uint32_t want, double* psi, double* psi_trial, double* g, double* H, void* U_new,
                void* V_new, double* dmult, double* kkt, void* ws, size_t ws_bytes, void* stream) {
    CHK(check_common(C, m, d, dtype));
    if (!x || !xbar) return fail(MEB_ERR_ARG, "x and xbar are required");
    if (!(sigma > 0) || !(tau > 0)) return fail(MEB_ERR_ARG, "sigma and tau must be positive");
    if (n_eta < 0 || n_eta > NT || (n_eta > 0 && (!etas || !psi_trial)))
        return fail(MEB_ERR_ARG, "n_eta must be in [0, 9] with etas and psi_trial given");
    if ((want & MEB_WANT_MULT) && (!U_new || !V_new)) return fail(MEB_ERR_ARG, "MULT needs U_new and V_new");
    if ((U == nullptr) != (V == nullptr)) return fail(MEB_ERR_ARG, "U and V must both be given or both NULL");
    size_t need;
    CHK(meb_eval_workspace_size(m, d, dtype, &need));
    if (!ws || ws_bytes < need) return fail(MEB_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int n1 = d + 1;
    Engine e;
    e.setup(m, d, dtype);
    Arena ar{(char*)ws, ws_bytes, 0};
    e.carve(ar);
    double* ybuf = ar.take<double>(2 * (size_t)n1 + 8);
    std::vector<double> h(e.sl.len, 0.0);
    h[S_MODE] = PM_EVAL;
    h[S_SIGMA] = sigma;
    h[S_SIGMA_NEXT] = sigma;
    h[S_TAU] = tau;
    h[S_HAVE_DIR] = dir ? 1.0 : 0.0;
    std::vector<double> y(n1);
    for (int k = 0; k < n1; ++k) {
        h[e.sl.xb + k] = x[k];
        h[e.sl.dir + k] = dir ? dir[k] : 0.0;
        h[e.sl.xbar + k] = xbar[k];
        y[k] = x[k] + (dir ? dir[k] : 0.0);
    }
    HIPCHK(hipMemcpyAsync(e.state, h.data(), sizeof(double) * e.sl.len, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ybuf, y.data(), sizeof(double) * n1, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ybuf + n1, xbar, sizeof(double) * n1, hipMemcpyHostToDevice, s));
    PassArgs a = e.args(C, R, const_cast<void*>(U), const_cast<void*>(V));
    a.force_mode = PM_EVAL;
    a.want_kkt = (want & (MEB_WANT_KKT | MEB_WANT_MULT)) ? 1 : 0;
    a.Uout = (want & MEB_WANT_MULT) ? U_new : nullptr;
    a.Vout = (want & MEB_WANT_MULT) ? V_new : nullptr;
    a.dense_vout = 1;
    a.want_mid = (want & MEB_WANT_HESS) ? 1 : 0;
    for (int l = 0; l < NT; ++l) a.etas[l] = (l < n_eta) ? etas[l] : 0.0;
    HIPCHK(launch_pass(a, e.pc, a.want_kkt ? 1 : 0, s));
    HIPCHK(launch_reduce_records(e.rec, e.pc.blocks, e.rl.len, (int64_t)e.pc.waves_per_block * e.rl.len, e.red, s));
    if (want & MEB_WANT_HESS) {
        HIPCHK(launch_mid_compact(e.mid_cnt, e.pc.nwaves, e.pc.bw, e.mid_idx, e.mid_coef, e.list_offs, e.list_total,
                                  e.list_idx, e.list_coef, e.state, s));
        SyrkArgs sa = e.syrk_args(C, U, V);
        sa.skip_k = INFINITY;
        HIPCHK(launch_syrk(sa, s));
    }
    // g and H into the tail of the state buffer (free in this call)
    double* gdev = e.state + e.sl.gb;
    double* Hdev = e.state + e.sl.H;
    if (want & (MEB_WANT_GRAD | MEB_WANT_HESS))
        HIPCHK(launch_eval_assemble(e.state, e.sl, e.rl, e.red, e.syrk, e.ksplit, syrk_tile(), e.ntile,
                                    (want & MEB_WANT_HESS) ? 1 : 0, sigma, tau, ybuf, ybuf + n1,
                                    (want & MEB_WANT_GRAD) ? gdev : nullptr, (want & MEB_WANT_HESS) ? Hdev : nullptr,
                                    s));
    std::vector<double> rh(e.rl.len);
    HIPCHK(hipMemcpyAsync(rh.data(), e.red, sizeof(double) * e.rl.len, hipMemcpyDeviceToHost, s));
    if ((want & MEB_WANT_GRAD) && g) HIPCHK(hipMemcpyAsync(g, gdev, sizeof(double) * n1, hipMemcpyDeviceToHost, s));
    if ((want & MEB_WANT_HESS) && H)
        HIPCHK(hipMemcpyAsync(H, Hdev, sizeof(double) * n1 * n1, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const RecLayout& rl = e.rl;
    auto prox = [&](double eta) {
        double acc = 0.0;
        for (int k = 0; k < n1; ++k) {
            const double v = x[k] + eta * (dir ? dir[k] : 0.0) - xbar[k];
            acc += v * v;
        }
        return acc;
    };
    if ((want & MEB_WANT_PSI) && psi)
        *psi = y[0] + 0.5 * sigma * rh[rl.z1] - rh[rl.ww] / (2.0 * sigma) + tau / (2.0 * sigma) * prox(1.0);
    if ((want & MEB_WANT_PSI) && psi_trial)
        for (int l = 0; l < n_eta; ++l)
            psi_trial[l] = x[0] + etas[l] * (dir ? dir[0] : 0.0) + 0.5 * sigma * rh[rl.trial + l] -
                           rh[rl.ww] / (2.0 * sigma) + tau / (2.0 * sigma) * prox(etas[l]);
    if ((want & MEB_WANT_DMULT) && dmult) *dmult = rh[rl.dm];
    if ((want & MEB_WANT_KKT) && kkt) {
        double nv = 0.0;
        for (int k = 0; k < d; ++k) nv += rh[rl.kv + k] * rh[rl.kv + k];
        kkt[0] = fabs(1.0 - rh[rl.ku]);
        kkt[1] = sqrt(nv);
        kkt[2] = rh[rl.kmax + 0];
        kkt[3] = rh[rl.kmax + 1];
        kkt[4] = rh[rl.kmax + 2];
    }
    return MEB_OK;
}

int meb_screen(const void* C, const void* R, int64_t m, int32_t d, int32_t dtype, double r_hat, const double* c_hat,
               double tol_red, int64_t* keep_idx, int64_t* n_keep, double* slack, void* ws, size_t ws_bytes,
               void* stream) {
    CHK(check_common(C, m, d, dtype));
    if (!c_hat || !keep_idx || !n_keep) return fail(MEB_ERR_ARG, "c_hat, keep_idx and n_keep are required");
    size_t need;
    CHK(meb_eval_workspace_size(m, d, dtype, &need));
    if (!ws || ws_bytes < need) return fail(MEB_ERR_WORKSPACE, "workspace too small");
    ScanBufs b;
    b.setup(m, d);
    Arena ar{(char*)ws, ws_bytes, 0};
    b.carve(ar);
    return run_screen(C, R, m, d, dtype, r_hat, c_hat, tol_red, b, keep_idx, n_keep, slack, (hipStream_t)stream);
}

int meb_check_feasible(const void* C, const void* R, int64_t m, int32_t d, int32_t dtype, double r, const double* c,
                       double eps, double* delta_max, int64_t* argmax, int64_t* viol_idx, int64_t viol_cap,
                       int64_t* n_viol, void* ws, size_t ws_bytes, void* stream) {
    CHK(check_common(C, m, d, dtype));
    if (!c) return fail(MEB_ERR_ARG, "c is required");
    if (viol_cap > 0 && !viol_idx) return fail(MEB_ERR_ARG, "viol_idx is NULL with viol_cap > 0");
    size_t need;
    CHK(meb_eval_workspace_size(m, d, dtype, &need));
    if (!ws || ws_bytes < need) return fail(MEB_ERR_WORKSPACE, "workspace too small");
    ScanBufs b;
    b.setup(m, d);
    Arena ar{(char*)ws, ws_bytes, 0};
    b.carve(ar);
    return run_check(C, R, m, d, dtype, r, c, eps, b, delta_max, argmax, viol_cap > 0 ? viol_idx : nullptr, viol_cap,
                     n_viol, (hipStream_t)stream);
}

int meb_prepare_f32(const double* C, const double* R, int64_t m, int32_t d, const double* origin, float* C32,
                    float* R32, double* L_out, void* ws, size_t ws_bytes, void* stream) {
    CHK(check_common(C, m, d, MEB_F64));
    if (!C32 || (R && !R32)) return fail(MEB_ERR_ARG, "C32 (and R32 when R is given) are required");
    size_t need;
    CHK(meb_eval_workspace_size(m, d, MEB_F64, &need));
    if (!ws || ws_bytes < need) return fail(MEB_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    ScanBufs b;
    b.setup(m, d);
    Arena ar{(char*)ws, ws_bytes, 0};
    b.carve(ar);
    if (origin) HIPCHK(hipMemcpyAsync(b.cvec, origin, sizeof(double) * d, hipMemcpyHostToDevice, s));
    else HIPCHK(launch_fill_f64(b.cvec, 0.0, d, s));
    double L = 0.0;
    CHK(run_prepare(C, R, m, d, b.cvec, C32, R32, b, &L, s));
    if (L_out) *L_out = L;
    return MEB_OK;
}

int meb_chol_workspace_size(int32_t n, size_t* bytes) {
    if (n < 1 || n > MEB_MAX_D + 1 || !bytes) return fail(MEB_ERR_ARG, "bad size");
    *bytes = al(sizeof(double) * (size_t)n * n) + al(sizeof(int) * 4) + ALIGN;
    return MEB_OK;
}

int meb_chol_solve(int32_t n, const double* H, const double* b, double* y, void* ws, size_t ws_bytes, void* stream) {
    size_t need;
    CHK(meb_chol_workspace_size(n, &need));
    if (!H || !b || !y) return fail(MEB_ERR_ARG, "H, b and y are required");
    if (!ws || ws_bytes < need) return fail(MEB_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    Arena ar{(char*)ws, ws_bytes, 0};
    double* A = ar.take<double>((size_t)n * n);
    int* info = ar.take<int>(4);
    HIPCHK(hipMemcpyAsync(A, H, sizeof(double) * n * n, hipMemcpyDeviceToDevice, s));
    if (y != b) HIPCHK(hipMemcpyAsync(y, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_chol_solve(n, A, y, info, s));
    int hinfo = 0;
    HIPCHK(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hinfo != 0) return fail(MEB_ERR_NUMERIC, "matrix is not positive definite");
    return MEB_OK;
}

int meb_solve(const void* C, const void* R, int64_t m, int32_t d, int32_t dtype, const meb_options* opts, void* ws,
              size_t ws_bytes, double* r_out, double* c_out, double* U_out, double* V_out, meb_stats* stats,
              void* stream) {
    const double t_start = now_ms();
    CHK(check_common(C, m, d, dtype));
    if (!r_out || !c_out) return fail(MEB_ERR_ARG, "r_out and c_out are required");
    meb_options def;
    meb_default_options(&def);
    const meb_options* o = opts ? opts : &def;
    if (!(o->rho >= 0 && o->rho < 1)) return fail(MEB_ERR_ARG, "rho must be in [0, 1)");
    if (!(o->sigma0 > 0) || !(o->tau > 0) || !(o->sigma_growth >= 1) || !(o->sigma_max >= o->sigma0))
        return fail(MEB_ERR_ARG, "bad sigma / tau options");
    if (o->mode != MEB_MODE_FP64 && o->mode != MEB_MODE_MIXED) return fail(MEB_ERR_ARG, "bad mode");
    if (dtype != MEB_F64) return fail(MEB_ERR_ARG, "meb_solve needs FP64 input");
    size_t need;
    CHK(meb_workspace_size(m, d, dtype, o, &need));
    if (!ws || ws_bytes < need) return fail(MEB_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int n1 = d + 1;
    meb_stats st;
    memset(&st, 0, sizeof(st));
    SolveWs w;
    w.setup(m, d, o);
    Arena ar{(char*)ws, ws_bytes, 0};
    w.carve(ar, m, d, o, R != nullptr);

    // origin c_1 and scale L = max_i ||c_i - c_1|| + r_i
    std::vector<double> c1(d);
    HIPCHK(hipMemcpyAsync(c1.data(), C, sizeof(double) * d, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double L = 0.0;
    double t0 = now_ms();
    if (o->mode == MEB_MODE_MIXED) {
        HIPCHK(hipMemcpyAsync(w.orig, c1.data(), sizeof(double) * d, hipMemcpyHostToDevice, s));
        CHK(run_prepare((const double*)C, (const double*)R, m, d, w.orig, w.C32, w.R32, w.scan, &L, s));
    } else {
        double dm;
        int64_t am, nv;
        CHK(run_check(C, R, m, d, dtype, 0.0, c1.data(), INFINITY, w.scan, &dm, &am, nullptr, 0, &nv, s));
        L = dm;
    }
    st.L = L;
    if (!std::isfinite(L)) return fail(MEB_ERR_NUMERIC, "non-finite input");
    std::vector<double> xfin(n1);
    double mreach_mixed = -INFINITY;  // max reach at xfin, when the mixed path already computed it
    int status = MEB_OK;
    if (!(L > 0)) {
        // every ball is the point c_1
        xfin[0] = 0.0;
        for (int k = 0; k < d; ++k) xfin[1 + k] = c1[k];
        if (U_out) HIPCHK(launch_fill_f64(U_out, 0.0, m, s));
        if (V_out) HIPCHK(launch_fill_f64(V_out, 0.0, m * (int64_t)d, s));
        if (U_out) {
            const double one = 1.0;
            HIPCHK(hipMemcpyAsync(U_out, &one, sizeof(double), hipMemcpyHostToDevice, s));
        }
        HIPCHK(hipStreamSynchronize(s));
        *r_out = 0.0;
        memcpy(c_out, c1.data(), sizeof(double) * d);
        st.ms_total = now_ms() - t_start;
        if (stats) *stats = st;
        return MEB_OK;
    }
    const double tau_raw = o->tau / (L * L);
    const double sigma0_raw = o->sigma0 / L;

    if (o->mode == MEB_MODE_FP64) {
        HIPCHK(launch_fill_f64(w.U64, 0.0, m, s));
        std::vector<double> x0(n1);
        x0[0] = L;
        for (int k = 0; k < d; ++k) x0[1 + k] = c1[k];
        RunParams p{L, sigma0_raw, tau_raw, o->tol_kkt, 2.220446049250313e-16, o};
        RunResult rr;
        const double tr = now_ms();
        CHK(run_ripalm(w.e64, C, R, w.U64, w.V64, x0.data(), p, rr, s));
        st.ms_phase[2] = now_ms() - tr;
        st.outer[1] = rr.outer;
        st.inner[1] = rr.inner;
        st.passes[1] = rr.passes;
        st.kkt[1] = rr.kkt;
        st.pass_ms[1] = rr.pass_ms;
        st.pass_bytes[1] = rr.pass_bytes;
        st.pass_launches[1] = rr.launches;
        st.mid_rows[1] = rr.sumk;
        st.mid_rows_max[1] = rr.maxk;
        st.n_red = m;
        if (rr.status != 1) status = MEB_WARN_MAXITER;
        xfin = rr.x;
        if (U_out || V_out) HIPCHK(launch_dense_mult(w.U64, w.V64, MEB_F64, m, d, U_out, V_out, s));
    } else {
        // ---- phase 1: FP32 run on all m balls, shifted by c_1
        HIPCHK(launch_fill_bytes_zero(w.U32, sizeof(float) * (size_t)m, s));
        std::vector<double> x0(n1, 0.0);
        x0[0] = L;
        RunParams p1{L, sigma0_raw, tau_raw, o->tol_kkt_low, 5.9604644775390625e-08, o};
        RunResult r1;
        CHK(run_ripalm(w.e32, w.C32, R ? (const void*)w.R32 : nullptr, w.U32, w.V32, x0.data(), p1, r1, s));
        st.ms_phase[0] = now_ms() - t0;
        st.outer[0] = r1.outer;
        st.inner[0] = r1.inner;
        st.passes[0] = r1.passes;
        st.kkt[0] = r1.kkt;
        st.pass_ms[0] = r1.pass_ms;
        st.pass_bytes[0] = r1.pass_bytes;
        st.pass_launches[0] = r1.launches;
        st.mid_rows[0] = r1.sumk;
        st.mid_rows_max[0] = r1.maxk;
        // ---- screening on the FP32 copy (FP64 arithmetic), tol_red in units of L
        const double ts = now_ms();
        std::vector<double> chat_s(d);  // shifted coordinates
        for (int k = 0; k < d; ++k) chat_s[k] = r1.x[1 + k];
        double tol_red = o->tol_red * L;
        int64_t n_red = 0;
        for (int tries = 0; tries < 8; ++tries) {
            CHK(run_screen(w.C32, R ? (const void*)w.R32 : nullptr, m, d, MEB_F32, r1.x[0], chat_s.data(), tol_red,
                           w.scan, w.keep, &n_red, nullptr, s));
            if (n_red > 0) break;
            tol_red = tol_red < 0 ? 0.0 : std::max(4.0 * tol_red, 1e-6 * L);
        }
        if (n_red == 0) return fail(MEB_ERR_NUMERIC, "screening retained no ball");
        // gather retained rows (FP64 data) and the FP32 multipliers as warm start
        HIPCHK(launch_gather(C, R, nullptr, nullptr, MEB_F64, w.keep, n_red, d, w.Cred, R ? w.Rred : nullptr,
                             nullptr, nullptr, s));
        HIPCHK(launch_gather(nullptr, nullptr, w.U32, w.V32, MEB_F32, w.keep, n_red, d, nullptr, nullptr, w.U64,
                             w.V64, s));
        st.ms_phase[1] = now_ms() - ts;
        // ---- phase 2: FP64 run(s) on the retained set, with reinsertion
        std::vector<double> xw(n1);
        xw[0] = r1.x[0];
        for (int k = 0; k < d; ++k) xw[1 + k] = c1[k] + r1.x[1 + k];
        double sigma_w = r1.sigma_end;
        double mreach_final = INFINITY;
        std::vector<int64_t> keep_h;   // retained indices in device order
        std::vector<int64_t> keep_sorted;
        int rounds = 0;
        double tr_total = 0, tc_total = 0;
        for (;;) {
            // the FP64 engine was carved for m balls; re-carve it for the
            // reduced size inside the same region (the carving grows with m)
            Engine& e = w.e64;
            char* region = (char*)e.state;
            const size_t region_bytes = engine_bytes(m, d, MEB_F64);
            if (engine_bytes(n_red, d, MEB_F64) > region_bytes)
                return fail(MEB_ERR_WORKSPACE, "reduced engine does not fit");
            e.setup(n_red, d, MEB_F64);
            {
                Arena sub{region, region_bytes, 0};
                e.carve(sub);
            }
            RunParams p2{L, sigma_w, tau_raw, o->tol_kkt, 2.220446049250313e-16, o};
            RunResult r2;
            const double tr = now_ms();
            CHK(run_ripalm(e, w.Cred, R ? (const void*)w.Rred : nullptr, w.U64, w.V64, xw.data(), p2, r2, s));
            tr_total += now_ms() - tr;
            st.outer[1] += r2.outer;
            st.inner[1] += r2.inner;
            st.passes[1] += r2.passes;
            st.kkt[1] = r2.kkt;
            st.pass_ms[1] += r2.pass_ms;
            st.pass_bytes[1] += r2.pass_bytes;
            st.pass_launches[1] += r2.launches;
            st.mid_rows[1] += r2.sumk;
            st.mid_rows_max[1] = std::max(st.mid_rows_max[1], r2.maxk);
            if (r2.status != 1) status = MEB_WARN_MAXITER;
            xw = r2.x;
            sigma_w = r2.sigma_end;
            // full FP64 check: reach_i = r_i + ||c - c_i||; violated if reach_i - rbar > eps
            const double tc = now_ms();
            const double eps_feas = o->eps_feas_rel * (1.0 + xw[0]);
            double mreach;
            int64_t am, nv;
            CHK(run_check(C, R, m, d, MEB_F64, 0.0, xw.data() + 1, xw[0] + eps_feas, w.scan, &mreach, &am, w.viol, m,
                          &nv, s));
            tc_total += now_ms() - tc;
            st.delta_max = mreach - xw[0];
            mreach_final = mreach;
            if (nv == 0 || rounds >= o->max_reinsert) break;
            // new violators not yet retained
            std::vector<int64_t> vh(nv);
            HIPCHK(hipMemcpyAsync(vh.data(), w.viol, sizeof(int64_t) * nv, hipMemcpyDeviceToHost, s));
            if (keep_h.empty()) {
                keep_h.resize(n_red);
                HIPCHK(hipMemcpyAsync(keep_h.data(), w.keep, sizeof(int64_t) * n_red, hipMemcpyDeviceToHost, s));
            }
            HIPCHK(hipStreamSynchronize(s));
            if (keep_sorted.empty()) keep_sorted = keep_h;  // screening output is ascending
            std::vector<int64_t> add;
            std::set_difference(vh.begin(), vh.end(), keep_sorted.begin(), keep_sorted.end(), std::back_inserter(add));
            if (add.empty()) break;
            rounds++;
            // append the new balls at the end of the reduced problem (zero multipliers)
            HIPCHK(hipMemcpyAsync(w.viol, add.data(), sizeof(int64_t) * add.size(), hipMemcpyHostToDevice, s));
            const int64_t na = (int64_t)add.size();
            HIPCHK(launch_gather(C, R, nullptr, nullptr, MEB_F64, w.viol, na, d, w.Cred + (size_t)n_red * d,
                                 R ? w.Rred + n_red : nullptr, nullptr, nullptr, s));
            HIPCHK(launch_fill_f64(w.U64 + n_red, 0.0, na, s));
            std::vector<int64_t> merged;
            merged.reserve(keep_h.size() + add.size());
            merged.insert(merged.end(), keep_h.begin(), keep_h.end());
            merged.insert(merged.end(), add.begin(), add.end());
            keep_h.swap(merged);
            {
                std::vector<int64_t> ms;
                ms.reserve(keep_sorted.size() + add.size());
                std::merge(keep_sorted.begin(), keep_sorted.end(), add.begin(), add.end(), std::back_inserter(ms));
                keep_sorted.swap(ms);
            }
            HIPCHK(hipMemcpyAsync(w.keep, keep_h.data(), sizeof(int64_t) * keep_h.size(), hipMemcpyHostToDevice, s));
            n_red += na;
        }
        st.ms_phase[2] = tr_total;
        st.ms_phase[3] = tc_total;
        st.reinsert_rounds = rounds;
        st.n_red = n_red;
        xfin = xw;
        mreach_mixed = mreach_final;
        if (U_out || V_out) {
            if (U_out) HIPCHK(launch_fill_f64(U_out, 0.0, m, s));
            if (V_out) HIPCHK(launch_fill_f64(V_out, 0.0, m * (int64_t)d, s));
            HIPCHK(launch_scatter_mult(w.U64, w.V64, w.keep, n_red, d, U_out, V_out, s));
        }
    }
    // fix-up: the returned radius encloses every ball (FP64 check over all m;
    // the mixed path's last full check already holds it for this center)
    double mreach = mreach_mixed;
    if (!(mreach > -INFINITY)) {
        int64_t am, nv;
        const double tcf = now_ms();
        CHK(run_check(C, R, m, d, dtype, 0.0, xfin.data() + 1, INFINITY, w.scan, &mreach, &am, nullptr, 0, &nv, s));
        st.ms_phase[3] += now_ms() - tcf;
    }
    st.rbar = xfin[0];
    st.delta_max = mreach - xfin[0];
    *r_out = std::max(xfin[0], mreach);
    memcpy(c_out, xfin.data() + 1, sizeof(double) * d);
    HIPCHK(hipStreamSynchronize(s));
    st.status = status;
    st.ms_total = now_ms() - t_start;
    if (stats) *stats = st;
    return status;
}

}  // extern "C"
