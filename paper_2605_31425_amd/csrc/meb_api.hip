// Host side of libmeb.so: the C ABI of include/meb.h, workspace carving, the
// scan helpers, and the solve as a resumable job with its synchronous driver.
//
// A ripALM run is a device-resident state machine.  The host enqueues a fixed
// sequence per Newton step -- evaluation pass, record reduction, rank-one
// Hessian contraction, assembly, control step -- and the control kernel
// decides on the device what the next pass computes (Armijo trials along the
// Newton direction, a plain re-evaluation, or the multiplier update fused with
// the first evaluation of the next outer iteration).  The host only polls the
// state's scalar header every few steps to learn when the run has ended.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <iterator>
#include <string>
#include <vector>

#include "meb_host.h"

namespace meb {

namespace {
thread_local std::string g_err;
}  // namespace

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

const char* last_error_text() { return g_err.c_str(); }

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

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------
void Engine::setup(int64_t m_, int d_, int dtype_) {
    m = m_;
    d = d_;
    dtype = dtype_;
    pc = choose_pass_config(m, d, dtype, device_cus());
    sl = StateLayout::make(d);
    rl = RecLayout::make(d);
    ksplit = syrk_ksplit(m, d, pc.nwaves);
    rec_cap = pc.nwaves;
    list_cap = (int64_t)pc.nwaves * pc.bw;
    ks_cap = ksplit;
    mm = SYRK_VEC;
    // a line-search pass skips the contraction above this many rows
    skip_k = std::max(4096.0, 16.0 * d);
}

// For n <= m the configuration takes one step per wave while n fits the
// resident waves, and more steps per wave beyond (fewer waves than at the
// threshold), so the wave count peaks at the larger instance's resident
// waves; a wave's range is bw(n) <= bw at the smaller instance's resident
// waves, and the lists hold at most n + WPB bw(n) entries.
void Engine::reserve_subsets() {
    const int64_t bpw = WAVE / pc.G;
    const int64_t wmax = ((int64_t)pc.fill_max + WPB - 1) / WPB * WPB;
    rec_cap = std::max<int64_t>(rec_cap, wmax);
    const int64_t steps = (m + bpw - 1) / bpw;
    const int64_t fmin = std::max(1, pc.fill_min);
    const int64_t bw_max = std::max<int64_t>((steps + fmin - 1) / fmin, pass_min_steps()) * bpw;
    list_cap = std::max<int64_t>(list_cap, m + (int64_t)WPB * bw_max);
    ks_cap = std::max(ks_cap, syrk_ksplit(m, d, (int)rec_cap));
}

bool Engine::resize_within(int64_t n) {
    const int64_t rc = rec_cap, lc = list_cap;
    const int kc = ks_cap;
    setup(n, d, dtype);
    if (rec_cap > rc || list_cap > lc || ksplit > kc) return false;
    rec_cap = rc;
    list_cap = lc;
    ks_cap = kc;
    return true;
}

PassArgs Engine::args(const void* C, const void* R, void* U, void* V) const {
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
    a.act_idx = act_idx;
    a.act_coef = act_coef;
    a.red = red;
    a.sync = sync;
    a.force_mode = -1;
    a.want_kkt = 0;
    a.want_mid = 1;
    for (int l = 0; l < NT; ++l) a.etas[l] = solver_eta(l);
    return a;
}

SyrkArgs Engine::syrk_args(const void* C, const void* U, const void* V) const {
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
    s.mid_cnt = mid_cnt;
    s.mid_idx = mid_idx;
    s.mid_coef = mid_coef;
    s.nwaves = pc.nwaves;
    s.bw = pc.bw;
    s.skip_k = skip_k;
    s.out = syrk;
    s.sync = sync;
    s.ksplit = ksplit;
    s.mm = mm;
    s.tile = syrk_tile_of(mm);
    s.ntile = (d + s.tile - 1) / s.tile;
    return s;
}

BatchItem Engine::item(const PassArgs& a, int* flag) const {
    BatchItem it;
    memset(&it, 0, sizeof(it));
    it.pa = a;
    it.pc = pc;
    it.sa = syrk_args(a.C, a.Uout ? a.Uout : a.U, a.Vout ? a.Vout : a.V);
    it.flag = flag;
    return it;
}

CgArgs Engine::cg_args(const void* C, const void* U, const void* V, int init) const {
    CgArgs c;
    memset(&c, 0, sizeof(c));
    c.C = C;
    c.U = U;
    c.V = V;
    c.d = d;
    c.dtype = dtype;
    c.state = state;
    c.sl = sl;
    c.red = red;
    c.rl = rl;
    c.mid_cnt = mid_cnt;
    c.mid_idx = mid_idx;
    c.mid_coef = mid_coef;
    c.nwaves = pc.nwaves;
    c.bw = pc.bw;
    c.part = syrk;
    c.sync = sync;
    c.init = init;
    return c;
}

int Engine::step(const PassArgs& a, bool control, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, int* flag) {
    if (ev0) HIPCHK(hipEventRecord(ev0, s));
    HIPCHK(launch_pass(a, pc, s));
    if (ev1) HIPCHK(hipEventRecord(ev1, s));
    const void* U = a.Uout ? a.Uout : a.U;
    const void* V = a.Vout ? a.Vout : a.V;
    if (cg_iters > 0 && control) {
        // matrix-free Newton directions: no assembled H; the control step
        // opens a CG solve when a Newton direction is needed, the CG launches
        // do nothing otherwise
        HIPCHK(launch_control(state, sl, rl, red, nullptr, s));
        HIPCHK(launch_cg_iter(cg_args(a.C, U, V, 1), s));
        const CgArgs it = cg_args(a.C, U, V, 0);
        for (int k = 0; k < cg_iters; ++k) HIPCHK(launch_cg_iter(it, s));
        HIPCHK(launch_cg_finish(state, sl, flag, s));
        return MEB_OK;
    }
    if (a.want_mid) HIPCHK(launch_syrk(syrk_args(a.C, U, V), s));
    if (control && control_newton_fused(sl.n1)) {
        HIPCHK(launch_control_newton(state, sl, rl, red, flag, s));
    } else if (control) {
        HIPCHK(launch_control(state, sl, rl, red, nullptr, s));
        HIPCHK(launch_newton(state, sl, flag, s));
    }
    return MEB_OK;
}

int Engine::reset_sync(hipStream_t s) {
    HIPCHK(launch_fill_bytes_zero(sync, sizeof(int) * SYNC_LEN, s));
    return MEB_OK;
}

size_t engine_bytes(int64_t m, int d, int dtype) {
    Engine e;
    e.setup(m, d, dtype);
    Sizer sz;
    e.carve(sz);
    return sz.off;
}

// ---------------------------------------------------------------------------
// Scans
// ---------------------------------------------------------------------------
void ScanBufs::setup(int64_t m_, int d_) {
    m = m_;
    d = d_;
    cfg = scan_config(m, d, device_cus());
}

size_t scan_bytes(int64_t m, int d) {
    ScanBufs b;
    b.setup(m, d);
    Sizer s;
    b.carve(s);
    return s.off;
}

// max_i (r_i + ||c - c_i|| - r) with its smallest argmax, and the ascending
// list of {i : r_i + ||c - c_i|| - r > eps} (first viol_cap entries).
int enq_check(const void* C, const void* R, int64_t m, int d, int dtype, double r, const double* c_dev, double eps,
              ScanBufs& b, int64_t* viol_idx, int64_t viol_cap, double* out, hipStream_t s) {
    HIPCHK(launch_scan(0, C, R, m, d, dtype, c_dev, r, eps, nullptr, nullptr, nullptr, b.cfg, b.wmax, b.warg, b.wcnt,
                       b.seg, s));
    HIPCHK(launch_scan_finalize(b.wcnt, b.wmax, b.warg, b.cfg.nwaves, b.offs, b.total(), b.out_max(), b.out_arg(), s));
    if (viol_idx && viol_cap > 0)
        HIPCHK(launch_scan_copy(b.seg, b.wcnt, b.offs, b.cfg.nwaves, b.cfg.bw, viol_idx, viol_cap, s));
    HIPCHK(hipMemcpyAsync(out, b.res, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    return MEB_OK;
}

// I_red = {i : r - r_i - ||c - c_i|| <= tol}, ascending.
int enq_screen(const void* C, const void* R, int64_t m, int d, int dtype, double r, const double* c_dev, double tol,
               ScanBufs& b, int64_t* keep_idx, double* slack, double* out, hipStream_t s) {
    HIPCHK(launch_scan(1, C, R, m, d, dtype, c_dev, r, tol, slack, nullptr, nullptr, b.cfg, nullptr, nullptr, b.wcnt,
                       b.seg, s));
    HIPCHK(launch_scan_finalize(b.wcnt, nullptr, nullptr, b.cfg.nwaves, b.offs, b.total(), nullptr, nullptr, s));
    HIPCHK(launch_scan_copy(b.seg, b.wcnt, b.offs, b.cfg.nwaves, b.cfg.bw, keep_idx, m, s));
    HIPCHK(hipMemcpyAsync(out, b.res, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    return MEB_OK;
}

// FP32 copy shifted by `origin` (device, d) and L = max_i ||c_i - origin|| + r_i.
int enq_prepare(const double* C, const double* R, int64_t m, int d, const double* origin_dev, float* C32, float* R32,
                ScanBufs& b, double* out, hipStream_t s) {
    HIPCHK(launch_scan(2, C, R, m, d, MEB_F64, origin_dev, 0.0, 0.0, nullptr, C32, R32, b.cfg, b.wmax, b.warg,
                       nullptr, nullptr, s));
    HIPCHK(launch_scan_finalize(nullptr, b.wmax, b.warg, b.cfg.nwaves, nullptr, nullptr, b.out_max(), b.out_arg(), s));
    HIPCHK(hipMemcpyAsync(out, b.res, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    return MEB_OK;
}

// ---------------------------------------------------------------------------
// Solve workspace
// ---------------------------------------------------------------------------
void SolveWs::setup(int64_t m, int d, const meb_options* o) {
    e64.setup(m, d, MEB_F64);
    if (o->mode == MEB_MODE_MIXED) {
        e32.setup(m, d, MEB_F32);
        e64.reserve_subsets();  // the FP64 run then takes the reduced set
    }
    scan.setup(m, d);
}

size_t solve_ws_bytes(int64_t m, int d, int in_dtype, const meb_options* o) {
    SolveWs w;
    w.setup(m, d, o);
    Sizer s;
    w.carve(s, m, d, o, true, in_dtype);
    return s.off + ALIGN;
}

namespace {

// Thread-local pinned staging for the synchronous entry points.
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

// Thread-local pool of HIP events for the optional per-pass timing.  They
// are read only after the stream has been synchronized, so they skip the
// system-scope fence (cache writeback and invalidation) that a default
// event performs when it is recorded, which would add a gap around every
// timed launch.
struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipEvent_t at(size_t i) {
        while (ev.size() <= i) {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
            ev.push_back(e);
        }
        return ev[i];
    }
};
thread_local EventPool g_events;

// Pinned headers and completion events of the two step batches that the
// synchronous driver keeps in flight, and the host-mapped mode word that
// every control step writes (read instead of a header copy unless the
// driver prints progress).
struct PollSlots {
    double* buf = nullptr;
    double* hdr[2] = {nullptr, nullptr};
    int* mode = nullptr;   // host view of the mode word (mapped, coherent)
    int* dmode = nullptr;  // its device address
    hipEvent_t ev[2] = {nullptr, nullptr};
    ~PollSlots() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
        if (buf) (void)hipHostFree(buf);
        if (mode) (void)hipHostFree(mode);
    }
    int init() {
        if (buf) return MEB_OK;
        for (auto& e : ev)
            if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIPCHK(hipHostMalloc((void**)&mode, sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
        HIPCHK(hipHostGetDevicePointer((void**)&dmode, mode, 0));
        HIPCHK(hipHostMalloc((void**)&buf, 2 * S_NSCALAR * sizeof(double), hipHostMallocDefault));
        hdr[0] = buf;
        hdr[1] = buf + S_NSCALAR;
        return MEB_OK;
    }
};
thread_local PollSlots g_poll;

// grows a pinned int64 buffer (contents are not kept)
int grow_pinned(int64_t*& p, size_t& cap, size_t n) {
    if (n <= cap) return MEB_OK;
    if (p) HIPCHK(hipHostFree(p));
    p = nullptr;
    cap = 0;
    HIPCHK(hipHostMalloc((void**)&p, std::max<size_t>(n, 16) * sizeof(int64_t), hipHostMallocDefault));
    cap = std::max<size_t>(n, 16);
    return MEB_OK;
}

// synchronous wrappers of the scans for the public entry points
int run_check(const void* C, const void* R, int64_t m, int d, int dtype, double r, const double* c_host, double eps,
              ScanBufs& b, double* dmax, int64_t* argmax, int64_t* viol_idx, int64_t viol_cap, int64_t* n_viol,
              hipStream_t s) {
    double* h = g_pin.get((size_t)d + 8);
    if (!h) return fail(MEB_ERR_HIP, "pinned host allocation failed");
    memcpy(h + 8, c_host, sizeof(double) * d);
    HIPCHK(hipMemcpyAsync(b.cvec, h + 8, sizeof(double) * d, hipMemcpyHostToDevice, s));
    CHK(enq_check(C, R, m, d, dtype, r, b.cvec, eps, b, viol_idx, viol_cap, h, s));
    HIPCHK(hipStreamSynchronize(s));
    if (dmax) *dmax = h[0];
    if (argmax) *argmax = word_i64(h + 1);
    if (n_viol) *n_viol = word_i64(h + 2);
    return MEB_OK;
}

int run_screen(const void* C, const void* R, int64_t m, int d, int dtype, double r, const double* c_host, double tol,
               ScanBufs& b, int64_t* keep_idx, int64_t* n_keep, double* slack, hipStream_t s) {
    double* h = g_pin.get((size_t)d + 8);
    if (!h) return fail(MEB_ERR_HIP, "pinned host allocation failed");
    memcpy(h + 8, c_host, sizeof(double) * d);
    HIPCHK(hipMemcpyAsync(b.cvec, h + 8, sizeof(double) * d, hipMemcpyHostToDevice, s));
    CHK(enq_screen(C, R, m, d, dtype, r, b.cvec, tol, b, keep_idx, slack, h, s));
    HIPCHK(hipStreamSynchronize(s));
    *n_keep = word_i64(h + 2);
    return MEB_OK;
}

}  // namespace

// Arithmetic of the Hessian contraction for a run of precision dtype.
int syrk_arith(int hess, int dtype, int d) {
    if (dtype == MEB_F64) {
        if (hess == MEB_HESS_F64) return SYRK_VEC;
        if (hess == MEB_HESS_MFMA_F64) return SYRK_MFMA_F64;
        return d >= 128 ? SYRK_MFMA_F64 : SYRK_VEC;  // AUTO (and the FP32-run choices)
    }
    switch (hess) {
        case MEB_HESS_MFMA_F32:
            return SYRK_MFMA_F32;
        case MEB_HESS_MFMA_BF16:
            return SYRK_MFMA_BF16;
        case MEB_HESS_AUTO:
            return d >= 256 ? SYRK_MFMA_BF16 : SYRK_VEC;
        default:
            return SYRK_VEC;
    }
}

// ---------------------------------------------------------------------------
// Job
// ---------------------------------------------------------------------------
constexpr double EPS64 = 2.220446049250313e-16;
constexpr double START_MARGIN = 0x1p-10;  // relative margin of the starting radius above L
constexpr double EPS32 = 5.9604644775390625e-08;

Job::~Job() {
    if (viol_h) (void)hipHostFree(viol_h);
    if (keep_pin) (void)hipHostFree(keep_pin);
}

int Job::init(const void* C_, const void* R_, int64_t m_, int d_, int in_dtype, const meb_options* o_, void* ws,
              size_t ws_bytes, double* pin_base, double* U_out_, double* V_out_) {
    C = C_;
    R = R_;
    m = m_;
    d = d_;
    o = *o_;
    U_out = U_out_;
    V_out = V_out_;
    w.setup(m, d, &o);
    Arena ar{(char*)ws, ws_bytes, 0};
    w.carve(ar, m, d, &o, R != nullptr, in_dtype);
    if (!ar.ok()) return fail(MEB_ERR_WORKSPACE, "workspace too small");
    if (in_dtype == MEB_F32) {
        // every phase reads the FP64 copy that start() writes
        C_in = C;
        R_in = R;
        C = w.Cin;
        R = R ? (const void*)w.Rin : nullptr;
    }
    pin.carve(pin_base, d);
    memset(&st, 0, sizeof(st));
    ph = JobPhase::Start;
    t_start = now_ms();
    return MEB_OK;
}

int Job::start(hipStream_t s) {
    // scale L = max_i ||c_i - c_1|| + r_i around the first center (read on
    // the device from row 0), and in mixed mode the shifted FP32 copy
    t_mark = now_ms();
    if (C_in) {
        HIPCHK(launch_widen_f32(static_cast<const float*>(C_in), w.Cin, m * (int64_t)d, s));
        if (R_in) HIPCHK(launch_widen_f32(static_cast<const float*>(R_in), w.Rin, m, s));
    }
    const double* c1_dev = static_cast<const double*>(C);
    // the preparation pass also flags a negative radius or a non-finite value
    // (the scale comes back as +inf); the FP32 copy only in mixed mode
    const bool mixed = o.mode == MEB_MODE_MIXED;
    CHK(enq_prepare((const double*)C, (const double*)R, m, d, c1_dev, mixed ? w.C32 : nullptr,
                    mixed ? w.R32 : nullptr, w.scan, pin.scal, s));
    HIPCHK(hipMemcpyAsync(pin.c1, C, sizeof(double) * d, hipMemcpyDeviceToHost, s));
    ph = JobPhase::WaitPrep;
    return MEB_OK;
}

int Job::begin_run(int id, Engine& eng, const void* Cr, const void* Rr, void* U, void* V, const double* x0,
                   double sigma_raw, double tol, double eps, hipStream_t s) {
    const int n1 = d + 1;
    eng.mm = syrk_arith(o.hess, eng.dtype, d);
    const StateLayout& sl = eng.sl;
    double* h = pin.init;
    memset(h, 0, sizeof(double) * sl.H);
    h[S_MODE] = PM_EVAL;
    h[S_SIGMA] = sigma_raw;
    h[S_SIGMA_NEXT] = std::min(sigma_raw * o.sigma_growth, o.sigma_max / L);
    h[S_TAU] = tau_raw;
    h[S_L] = L;
    h[S_RHO] = o.rho;
    h[S_TOL] = tol;
    h[S_GROWTH] = o.sigma_growth;
    h[S_SIGMA_MAX] = o.sigma_max / L;
    h[S_MAX_OUTER] = o.max_outer;
    h[S_MAX_INNER] = o.max_inner;
    h[S_MAX_LS] = o.max_ls;
    h[S_STALL_OUTER] = o.stall_outer;
    h[S_EPS] = eps;
    h[S_BEST_KKT] = INFINITY;
    h[S_VERBOSE] = o.verbose;
    // first-order inner solves in the early outer iterations of ripALM: the
    // plain FP64 run, or the mixed path's screening run (its FP64 run is a
    // warm-started continuation near the solution)
    h[S_FO_OUTER] = (o.mode == MEB_MODE_FP64 || id == 0) ? o.first_order_outer : 0;
    h[S_CG] = o.newton == MEB_NEWTON_CG ? 1.0 : 0.0;
    h[S_CG_MAX] = o.cg_max_iter;
    h[S_CG_TOL] = o.cg_tol;
    eng.cg_iters = o.newton == MEB_NEWTON_CG ? o.cg_max_iter : 0;
    for (int k = 0; k < n1; ++k) {
        h[sl.xb + k] = x0[k];
        h[sl.xbar + k] = x0[k];
        h[sl.ab + k] = x0[k];
    }
    // H is assembled before any Newton step reads it
    HIPCHK(hipMemcpyAsync(eng.state, h, sizeof(double) * sl.H, hipMemcpyHostToDevice, s));
    CHK(eng.reset_sync(s));
    pa = eng.args(Cr, Rr, U, V);
    e = &eng;
    run_id = id;
    steps = 0;
    max_steps = (int64_t)o.max_outer * (o.max_inner + o.max_ls + 2) + 16;
    forced_end = false;
    run_pass_ms = 0;
    run_launches = 0;
    last_k = -1;
    t_run = now_ms();
    ph = JobPhase::Run;
    return MEB_OK;
}

int Job::end_run(hipStream_t s) {
    // the scalar header and the iterate are contiguous in the state
    HIPCHK(hipMemcpyAsync(pin.hdr, e->state, sizeof(double) * (S_NSCALAR + d + 1), hipMemcpyDeviceToHost, s));
    ph = JobPhase::WaitRunEnd;
    return MEB_OK;
}

int Job::screen(hipStream_t s) {
    // FP32 copy, FP64 arithmetic; coordinates shifted by c_1
    for (int k = 0; k < d; ++k) pin.cvec[k] = x1[1 + k];
    HIPCHK(hipMemcpyAsync(w.scan.cvec, pin.cvec, sizeof(double) * d, hipMemcpyHostToDevice, s));
    CHK(enq_screen(w.C32, R ? (const void*)w.R32 : nullptr, m, d, MEB_F32, x1[0], w.scan.cvec, tol_red, w.scan, w.keep,
                   nullptr, pin.scal, s));
    ph = JobPhase::WaitScreen;
    return MEB_OK;
}

int Job::start_fp64_reduced(hipStream_t s) {
    // the FP64 engine was carved for m balls; re-carve it for the reduced
    // size inside the same region (the carving grows with m)
    Engine& eng = w.e64;
    char* region = (char*)eng.state;
    Sizer full;
    eng.carve(full);
    if (!eng.resize_within(n_red)) return fail(MEB_ERR_WORKSPACE, "reduced engine does not fit");
    Arena sub{region, full.off, 0};
    eng.carve(sub);
    return begin_run(1, eng, w.Cred, R ? (const void*)w.Rred : nullptr, w.U64, w.V64, xw.data(), sigma_w, o.tol_kkt,
                     EPS64, s);
}

int Job::check(hipStream_t s) {
    // full FP64 check: reach_i = r_i + ||c - c_i||; violated if reach_i - rbar > eps
    t_check = now_ms();
    const double eps_feas = o.eps_feas_rel * (1.0 + xw[0]);
    for (int k = 0; k < d; ++k) pin.cvec[k] = xw[1 + k];
    HIPCHK(hipMemcpyAsync(w.scan.cvec, pin.cvec, sizeof(double) * d, hipMemcpyHostToDevice, s));
    CHK(enq_check(C, R, m, d, MEB_F64, 0.0, w.scan.cvec, xw[0] + eps_feas, w.scan, w.viol, m, pin.scal, s));
    ph = JobPhase::WaitCheck;
    return MEB_OK;
}

int Job::finish_mixed(hipStream_t s) {
    st.ms_phase[2] = tr_total;
    st.ms_phase[3] = tc_total;
    st.reinsert_rounds = rounds;
    st.n_red = n_red;
    xfin = xw;
    if (U_out || V_out) {
        if (U_out) HIPCHK(launch_fill_f64(U_out, 0.0, m, s));
        if (V_out) HIPCHK(launch_fill_f64(V_out, 0.0, m * (int64_t)d, s));
        HIPCHK(launch_scatter_mult(w.U64, w.V64, w.keep, n_red, d, U_out, V_out, s));
    }
    finish();
    return MEB_OK;
}

void Job::finish() {
    // fix-up: the returned radius encloses every ball
    st.rbar = xfin[0];
    st.delta_max = mreach - xfin[0];
    r_out = std::max(xfin[0], mreach);
    st.status = status;
    ph = JobPhase::Done;
}

int Job::on_ready(hipStream_t s) {
    const int n1 = d + 1;
    switch (ph) {
        case JobPhase::WaitPrep: {
            L = pin.scal[0];
            c1.assign(pin.c1, pin.c1 + d);
            st.L = L;
            if (!std::isfinite(L)) return fail(MEB_ERR_ARG, "input holds a negative radius or a non-finite value");
            if (!(L > 0)) {
                // every ball is the point c_1
                xfin.assign(n1, 0.0);
                for (int k = 0; k < d; ++k) xfin[1 + k] = c1[k];
                mreach = 0.0;
                if (U_out) HIPCHK(launch_fill_f64(U_out, 0.0, m, s));
                if (V_out) HIPCHK(launch_fill_f64(V_out, 0.0, m * (int64_t)d, s));
                if (U_out) {
                    pin.scal[7] = 1.0;
                    HIPCHK(hipMemcpyAsync(U_out, pin.scal + 7, sizeof(double), hipMemcpyHostToDevice, s));
                }
                finish();
                return MEB_OK;
            }
            tau_raw = o.tau / (L * L);
            sigma0_raw = o.sigma0 / L;
            // start a little above L: at (L, c_1) the ball attaining L sits
            // exactly on the boundary between the polar and the third
            // projection case, where rounding would pick the Jacobian
            std::vector<double> x0(n1, 0.0);
            x0[0] = L * (1.0 + START_MARGIN);
            if (o.mode == MEB_MODE_FP64) {
                HIPCHK(launch_fill_f64(w.U64, 0.0, m, s));
                for (int k = 0; k < d; ++k) x0[1 + k] = c1[k];
                return begin_run(1, w.e64, C, R, w.U64, w.V64, x0.data(), sigma0_raw, o.tol_kkt, EPS64, s);
            }
            // FP32 run on all m balls, shifted by c_1
            HIPCHK(launch_fill_bytes_zero(w.U32, sizeof(float) * (size_t)m, s));
            return begin_run(0, w.e32, w.C32, R ? (const void*)w.R32 : nullptr, w.U32, w.V32, x0.data(), sigma0_raw,
                             o.tol_kkt_low, EPS32, s);
        }
        case JobPhase::WaitRunEnd: {
            const double* hh = pin.hdr;
            std::vector<double> x(pin.x, pin.x + n1);
            int rstatus = (int)hh[S_STATUS];
            if (forced_end && (int)hh[S_MODE] != PM_DONE) rstatus = 2;
            const int r = run_id;
            if (r == 0) {
                st.outer[0] = (int)hh[S_K];
                st.inner[0] = (int)hh[S_NINNER];
                st.passes[0] = (int)hh[S_NPASS];
                st.kkt[0] = hh[S_KKT];
                st.pass_ms[0] = run_pass_ms;
                st.pass_bytes[0] = hh[S_BYTES];
                st.pass_launches[0] = run_launches;
                st.mid_rows[0] = hh[S_SUMK];
                st.mid_rows_max[0] = hh[S_MAXK];
                st.newton_shifted[0] = (int)hh[S_NSHIFT];
                st.inner_breaks[0] = (int)hh[S_NBREAK];
                st.first_order_steps[0] = (int)hh[S_NFO];
                st.cg_iterations[0] = (int)hh[S_NCG];
            } else {
                st.outer[1] += (int)hh[S_K];
                st.inner[1] += (int)hh[S_NINNER];
                st.passes[1] += (int)hh[S_NPASS];
                st.kkt[1] = hh[S_KKT];
                st.pass_ms[1] += run_pass_ms;
                st.pass_bytes[1] += hh[S_BYTES];
                st.pass_launches[1] += run_launches;
                st.mid_rows[1] += hh[S_SUMK];
                st.mid_rows_max[1] = std::max(st.mid_rows_max[1], hh[S_MAXK]);
                st.newton_shifted[1] += (int)hh[S_NSHIFT];
                st.inner_breaks[1] += (int)hh[S_NBREAK];
                st.first_order_steps[1] += (int)hh[S_NFO];
                st.cg_iterations[1] += (int)hh[S_NCG];
            }
            if (rstatus < 0) return fail(MEB_ERR_NUMERIC, "numeric failure in the solver run");
            for (int k = 0; k < n1; ++k)
                if (!std::isfinite(x[k])) return fail(MEB_ERR_NUMERIC, "non-finite iterate");
            if (r == 0) {
                x1 = x;
                sigma1 = hh[S_SIGMA];
                warm1 = rstatus == 1;
                st.ms_phase[0] = now_ms() - t_mark;
                t_mark = now_ms();
                tol_red = o.tol_red * L;
                screen_tries = 0;
                return screen(s);
            }
            if (rstatus != 1) status = MEB_WARN_MAXITER;
            if (o.mode == MEB_MODE_FP64) {
                st.ms_phase[2] = now_ms() - t_run;
                st.n_red = m;
                xfin = x;
                if (U_out || V_out) HIPCHK(launch_dense_mult(w.U64, w.V64, MEB_F64, m, d, U_out, V_out, s));
                fixup_only = true;
                t_check = now_ms();
                for (int k = 0; k < d; ++k) pin.cvec[k] = xfin[1 + k];
                HIPCHK(hipMemcpyAsync(w.scan.cvec, pin.cvec, sizeof(double) * d, hipMemcpyHostToDevice, s));
                CHK(enq_check(C, R, m, d, MEB_F64, 0.0, w.scan.cvec, INFINITY, w.scan, nullptr, 0, pin.scal, s));
                ph = JobPhase::WaitCheck;
                return MEB_OK;
            }
            tr_total += now_ms() - t_run;
            xw = x;
            sigma_w = hh[S_SIGMA];
            return check(s);
        }
        case JobPhase::WaitScreen: {
            n_red = word_i64(pin.scal + 2);
            if (n_red == 0) {
                if (++screen_tries >= 8) return fail(MEB_ERR_NUMERIC, "screening retained no ball");
                tol_red = tol_red < 0 ? 0.0 : std::max(4.0 * tol_red, 1e-6 * L);
                return screen(s);
            }
            // gather retained rows (FP64 data) and, when the screening run
            // converged, its multipliers and penalty as warm start; a run that
            // stopped at the FP32 rounding floor or its iteration limit hands
            // over only its point (multipliers zero, sigma_0)
            HIPCHK(launch_gather(C, R, nullptr, nullptr, MEB_F64, w.keep, n_red, d, w.Cred, R ? w.Rred : nullptr,
                                 nullptr, nullptr, s));
            if (warm1) {
                HIPCHK(launch_gather(nullptr, nullptr, w.U32, w.V32, MEB_F32, w.keep, n_red, d, nullptr, nullptr,
                                     w.U64, w.V64, s));
            } else {
                HIPCHK(launch_fill_bytes_zero(w.U64, sizeof(double) * (size_t)n_red, s));
                HIPCHK(launch_fill_bytes_zero(w.V64, sizeof(double) * (size_t)n_red * d, s));
            }
            st.ms_phase[1] = now_ms() - t_mark;
            xw.assign(n1, 0.0);
            xw[0] = x1[0];
            for (int k = 0; k < d; ++k) xw[1 + k] = c1[k] + x1[1 + k];
            sigma_w = warm1 ? sigma1 : sigma0_raw;
            rounds = 0;
            keep_h.clear();
            keep_sorted.clear();
            return start_fp64_reduced(s);
        }
        case JobPhase::WaitCheck: {
            const double mr = pin.scal[0];
            if (fixup_only) {
                mreach = mr;
                st.ms_phase[3] += now_ms() - t_check;
                finish();
                return MEB_OK;
            }
            tc_total += now_ms() - t_check;
            n_viol = word_i64(pin.scal + 2);
            st.delta_max = mr - xw[0];
            mreach = mr;
            if (n_viol == 0 || rounds >= o.max_reinsert) return finish_mixed(s);
            // new violators not yet retained: bring both lists to the host
            CHK(grow_pinned(viol_h, viol_cap, (size_t)n_viol));
            HIPCHK(hipMemcpyAsync(viol_h, w.viol, sizeof(int64_t) * n_viol, hipMemcpyDeviceToHost, s));
            if (keep_h.empty()) {
                CHK(grow_pinned(keep_pin, keep_cap, (size_t)n_red));
                HIPCHK(hipMemcpyAsync(keep_pin, w.keep, sizeof(int64_t) * n_red, hipMemcpyDeviceToHost, s));
            }
            ph = JobPhase::WaitViol;
            return MEB_OK;
        }
        case JobPhase::WaitViol: {
            if (keep_h.empty()) {
                keep_h.assign(keep_pin, keep_pin + n_red);
                keep_sorted = keep_h;  // screening output is ascending
            }
            std::vector<int64_t> add;
            std::set_difference(viol_h, viol_h + n_viol, keep_sorted.begin(), keep_sorted.end(),
                                std::back_inserter(add));
            if (add.empty()) return finish_mixed(s);
            rounds++;
            // append the new balls at the end of the reduced problem (zero multipliers)
            const int64_t na = (int64_t)add.size();
            memcpy(viol_h, add.data(), sizeof(int64_t) * na);
            HIPCHK(hipMemcpyAsync(w.viol, viol_h, sizeof(int64_t) * na, hipMemcpyHostToDevice, s));
            HIPCHK(launch_gather(C, R, nullptr, nullptr, MEB_F64, w.viol, na, d, w.Cred + (size_t)n_red * d,
                                 R ? w.Rred + n_red : nullptr, nullptr, nullptr, s));
            HIPCHK(launch_fill_f64(w.U64 + n_red, 0.0, na, s));
            keep_h.insert(keep_h.end(), add.begin(), add.end());
            {
                std::vector<int64_t> ms;
                ms.reserve(keep_sorted.size() + add.size());
                std::merge(keep_sorted.begin(), keep_sorted.end(), add.begin(), add.end(), std::back_inserter(ms));
                keep_sorted.swap(ms);
            }
            CHK(grow_pinned(keep_pin, keep_cap, keep_h.size()));
            memcpy(keep_pin, keep_h.data(), sizeof(int64_t) * keep_h.size());
            HIPCHK(hipMemcpyAsync(w.keep, keep_pin, sizeof(int64_t) * keep_h.size(), hipMemcpyHostToDevice, s));
            n_red += na;
            return start_fp64_reduced(s);
        }
        default:
            return fail(MEB_ERR_ARG, "job is not waiting for a readback");
    }
}

// Solver steps per enqueued batch (two batches in flight).  The steps
// queued behind the one that ends a run still launch and return at once
// (≈ 4 us per kernel), and up to one and a half batches of them delay what
// follows the run; batches of two keep the device fed with less of that
// tail than four (the d = 1000 workload 51.1 -> 49.7 ms, the others
// unchanged), single steps starve the small instances.  A step of many
// launches (the factorization across workgroups, conjugate gradients) is
// long enough for single steps, and its queued copies cost the most.
// Tuning override MEB_STEP_BATCH, 1 to 8.
int step_batch(const Engine& e) {
    static const int v = [] {
        const char* s = getenv("MEB_STEP_BATCH");
        const int k = s ? atoi(s) : 0;
        return k >= 1 && k <= 8 ? k : 0;
    }();
    if (v) return v;
    return (e.sl.n1 >= MCHOL_MIN_N || e.cg_iters > 0) ? 1 : 2;
}

int drive_sync(Job& j, hipStream_t s) {
    CHK(j.start(s));
    const bool prof = j.o.profile != 0;
    size_t nev = 0;
    PollSlots& ps = g_poll;
    CHK(ps.init());
    int inflight = 0, head = 0;  // batches enqueued whose header is unread; the oldest one's slot
    while (!j.done()) {
        if (j.stepping()) {
            // Two batches in flight: the next batch is enqueued before the
            // older one's end is observed, so the device does not wait for
            // the host between batches.  Steps enqueued after the run has
            // ended leave the state unchanged.  The end is read from the mode
            // word the control steps write to host memory (a later step's
            // value at worst, which only reports the end earlier); with
            // progress printing, from a copy of the state header.
            const bool copy_hdr = j.o.verbose != 0;
            if (inflight == 0) *reinterpret_cast<volatile int*>(ps.mode) = PM_EVAL;
            while (inflight < 2) {
                const int batch = step_batch(*j.e);
                for (int b = 0; b < batch; ++b) {
                    hipEvent_t e0 = nullptr, e1 = nullptr;
                    if (prof) {
                        e0 = g_events.at(nev);
                        e1 = g_events.at(nev + 1);
                        if (!e0 || !e1) return fail(MEB_ERR_HIP, "hipEventCreate failed");
                        nev += 2;
                    }
                    CHK(j.e->step(j.pa, true, s, e0, e1, copy_hdr ? nullptr : ps.dmode));
                }
                j.steps += batch;
                const int slot = (head + inflight) & 1;
                if (copy_hdr)
                    HIPCHK(hipMemcpyAsync(ps.hdr[slot], j.e->state, sizeof(double) * S_NSCALAR, hipMemcpyDeviceToHost,
                                          s));
                HIPCHK(hipEventRecord(ps.ev[slot], s));
                ++inflight;
            }
            HIPCHK(hipEventSynchronize(ps.ev[head]));
            const double* hs = ps.hdr[head];
            head ^= 1;
            --inflight;
            if (copy_hdr && (int)hs[S_K] != j.last_k) {
                j.last_k = (int)hs[S_K];
                fprintf(stderr, "[meb] k=%d sigma=%.3e kkt=%.3e passes=%d newton=%d\n", (int)hs[S_K], hs[S_SIGMA],
                        hs[S_KKT], (int)hs[S_NPASS], (int)hs[S_NINNER]);
            }
            const int mode_now = copy_hdr ? (int)hs[S_MODE] : *reinterpret_cast<volatile int*>(ps.mode);
            const bool ended = mode_now == PM_DONE;
            if (ended || j.steps > j.max_steps) {
                if (prof) {
                    HIPCHK(hipStreamSynchronize(s));  // the newer batch's events too
                    double ms = 0;
                    for (size_t k = 0; k + 1 < nev; k += 2) {
                        float t = 0.f;
                        HIPCHK(hipEventElapsedTime(&t, g_events.at(k), g_events.at(k + 1)));
                        ms += t;
                    }
                    j.run_pass_ms = ms;
                    j.run_launches = (int)(nev / 2);
                    nev = 0;
                }
                j.forced_end = !ended;
                CHK(j.end_run(s));
                inflight = 0;  // the newer batch's header is not read (the run is over)
                head = 0;
            }
        } else {
            HIPCHK(hipStreamSynchronize(s));
            CHK(j.on_ready(s));
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    return MEB_OK;
}

int check_common(const void* C, int64_t m, int32_t d, int32_t dtype) {
    if (!C) return fail(MEB_ERR_ARG, "C is NULL");
    if (m < 1) return fail(MEB_ERR_ARG, "m must be >= 1");
    if (m > 0x7fffffffLL) return fail(MEB_ERR_ARG, "m must be < 2^31");
    if (d < 1 || d > MEB_MAX_D) return fail(MEB_ERR_ARG, "d must be in [1, MEB_MAX_D]");
    if (dtype != MEB_F64 && dtype != MEB_F32) return fail(MEB_ERR_ARG, "bad dtype");
    // rows are read with 16-byte loads and 16-byte LDS copies where d allows
    if ((uintptr_t)C % 16) return fail(MEB_ERR_ARG, "C is not 16-byte aligned");
    if ((d % 2 == 1) && d > 1024) return fail(MEB_ERR_UNSUPPORTED, "odd d above 1024 is not supported");
    return MEB_OK;
}

int check_solve_options(const meb_options* o) {
    if (!(o->rho >= 0 && o->rho < 1)) return fail(MEB_ERR_ARG, "rho must be in [0, 1)");
    if (!(o->sigma0 > 0) || !(o->tau > 0) || !(o->sigma_growth >= 1) || !(o->sigma_max >= o->sigma0))
        return fail(MEB_ERR_ARG, "bad sigma / tau options");
    if (o->mode != MEB_MODE_FP64 && o->mode != MEB_MODE_MIXED) return fail(MEB_ERR_ARG, "bad mode");
    if (o->hess < MEB_HESS_AUTO || o->hess > MEB_HESS_MFMA_BF16) return fail(MEB_ERR_ARG, "bad hess");
    if (o->first_order_outer < 0) return fail(MEB_ERR_ARG, "first_order_outer must be >= 0");
    if (o->newton != MEB_NEWTON_DENSE && o->newton != MEB_NEWTON_CG) return fail(MEB_ERR_ARG, "bad newton");
    if (o->newton == MEB_NEWTON_CG && (o->cg_max_iter < 1 || o->cg_max_iter > 1000 || !(o->cg_tol > 0)))
        return fail(MEB_ERR_ARG, "cg_max_iter must be in [1, 1000] and cg_tol > 0");
    return MEB_OK;
}

}  // namespace meb

using namespace meb;

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
    o->tol_kkt = 1e-9;
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
    o->hess = MEB_HESS_AUTO;
    o->newton = MEB_NEWTON_DENSE;
    o->cg_max_iter = 20;
    o->cg_tol = 1e-2;
    return MEB_OK;
}

const char* meb_last_error(void) { return last_error_text(); }

#ifndef MEB_SOURCE_HASH
#define MEB_SOURCE_HASH "unknown"
#endif
const char* meb_source_hash(void) { return MEB_SOURCE_HASH; }

int meb_workspace_size(int64_t m, int32_t d, int32_t dtype, const meb_options* opts, size_t* bytes) {
    if (!bytes) return fail(MEB_ERR_ARG, "bytes is NULL");
    if (m < 1 || d < 1 || d > MEB_MAX_D) return fail(MEB_ERR_ARG, "bad shape");
    if (dtype != MEB_F64 && dtype != MEB_F32) return fail(MEB_ERR_ARG, "bad dtype");
    meb_options def;
    meb_default_options(&def);
    *bytes = solve_ws_bytes(m, d, dtype, opts ? opts : &def);
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
    if ((uintptr_t)V % 16 || (uintptr_t)V_new % 16) return fail(MEB_ERR_ARG, "V and V_new must be 16-byte aligned");
    const size_t es = dtype_size(dtype);
    if ((uintptr_t)R % es || (uintptr_t)U % es || (uintptr_t)U_new % es)
        return fail(MEB_ERR_ARG, "R, U and U_new must be aligned to their element size");
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
    a.want_mid = (want & MEB_WANT_HESS) ? 1 : 0;
    for (int l = 0; l < NT; ++l) a.etas[l] = (l < n_eta) ? etas[l] : 0.0;
    // the pass writes the V rows of non-zero updated multipliers only
    if (want & MEB_WANT_MULT) HIPCHK(launch_fill_bytes_zero(V_new, dtype_size(dtype) * (size_t)m * d, s));
    CHK(e.reset_sync(s));
    HIPCHK(launch_pass(a, e.pc, s));
    if (want & MEB_WANT_HESS) {
        // the contraction assembles H into the state, in the arithmetic that
        // bits 8..10 of want select (MEB_HESS_*, AUTO when zero)
        e.mm = syrk_arith((int)((want >> 8) & 7u), dtype, d);
        SyrkArgs sa = e.syrk_args(C, U, V);
        sa.skip_k = INFINITY;
        HIPCHK(launch_syrk(sa, s));
    }
    double* gdev = e.state + e.sl.gb;
    double* Hdev = e.state + e.sl.H;
    if (want & MEB_WANT_GRAD)
        HIPCHK(launch_eval_outputs(e.state, e.sl, e.rl, e.red, sigma, tau, ybuf, ybuf + n1, gdev, nullptr, s));
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

int meb_hess_vec(const void* C, const void* R, const void* U, const void* V, int64_t m, int32_t d, int32_t dtype,
                 const double* x, double sigma, double tau, const double* q, double* Hq, void* ws, size_t ws_bytes,
                 void* stream) {
    CHK(check_common(C, m, d, dtype));
    if (!x || !q || !Hq) return fail(MEB_ERR_ARG, "x, q and Hq are required");
    if (!(sigma > 0) || !(tau > 0)) return fail(MEB_ERR_ARG, "sigma and tau must be positive");
    if ((U == nullptr) != (V == nullptr)) return fail(MEB_ERR_ARG, "U and V must both be given or both NULL");
    if ((uintptr_t)V % 16) return fail(MEB_ERR_ARG, "V must be 16-byte aligned");
    size_t need;
    CHK(meb_eval_workspace_size(m, d, dtype, &need));
    if (!ws || ws_bytes < need) return fail(MEB_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int n1 = d + 1;
    Engine e;
    e.setup(m, d, dtype);
    Arena ar{(char*)ws, ws_bytes, 0};
    e.carve(ar);
    double* out = ar.take<double>(2 * (size_t)n1 + 8);
    // the state: the evaluation point, and q where the CG search direction lives
    std::vector<double> h(e.sl.len, 0.0);
    h[S_MODE] = PM_CG;
    h[S_SIGMA] = sigma;
    h[S_SIGMA_NEXT] = sigma;
    h[S_TAU] = tau;
    for (int k = 0; k < n1; ++k) h[e.sl.xb + k] = x[k];
    const int cs = cg_stride(n1);
    for (int k = 0; k < n1; ++k) h[e.sl.H + 2 * cs + k] = q[k];
    HIPCHK(hipMemcpyAsync(e.state, h.data(), sizeof(double) * e.sl.len, hipMemcpyHostToDevice, s));
    PassArgs a = e.args(C, R, const_cast<void*>(U), const_cast<void*>(V));
    a.force_mode = PM_EVAL;
    a.want_kkt = 0;
    a.Uout = nullptr;
    a.Vout = nullptr;
    a.want_mid = 1;
    CHK(e.reset_sync(s));
    HIPCHK(launch_pass(a, e.pc, s));
    CgArgs c = e.cg_args(C, U, V, 0);
    c.out = out;
    HIPCHK(launch_cg_iter(c, s));
    HIPCHK(hipMemcpyAsync(Hq, out, sizeof(double) * n1, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
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
    double* h = g_pin.get((size_t)d + 8);
    if (!h) return fail(MEB_ERR_HIP, "pinned host allocation failed");
    if (origin) {
        memcpy(h + 8, origin, sizeof(double) * d);
        HIPCHK(hipMemcpyAsync(b.cvec, h + 8, sizeof(double) * d, hipMemcpyHostToDevice, s));
    } else {
        HIPCHK(launch_fill_f64(b.cvec, 0.0, d, s));
    }
    CHK(enq_prepare(C, R, m, d, b.cvec, C32, R32, b, h, s));
    HIPCHK(hipStreamSynchronize(s));
    if (L_out) *L_out = h[0];
    return MEB_OK;
}

int meb_chol_workspace_size(int32_t n, size_t* bytes) {
    if (n < 1 || n > MEB_MAX_D + 1 || !bytes) return fail(MEB_ERR_ARG, "bad size");
    *bytes = al(sizeof(double) * (size_t)n * n) + al(sizeof(int) * 4) + al(sizeof(double) * (size_t)n) +
             al(sizeof(double) * MCHOL_NB * MCHOL_NB) + al(sizeof(double)) + ALIGN;
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
    if (n >= MCHOL_MIN_N) {
        double* yw = ar.take<double>(n);
        double* ldw = ar.take<double>(MCHOL_NB * MCHOL_NB);
        double* badw = ar.take<double>(1);
        HIPCHK(launch_chol_solve_mwg(n, A, y, yw, ldw, badw, info, s));
    } else {
        HIPCHK(launch_chol_solve(n, A, y, info, s));
    }
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
    CHK(check_solve_options(o));
    size_t need;
    CHK(meb_workspace_size(m, d, dtype, o, &need));
    if (!ws || ws_bytes < need) return fail(MEB_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    double* pin = g_pin.get(JobPin::doubles(d));
    if (!pin) return fail(MEB_ERR_HIP, "pinned host allocation failed");
    Job j;
    CHK(j.init(C, R, m, d, dtype, o, ws, ws_bytes, pin, U_out, V_out));
    CHK(drive_sync(j, s));
    *r_out = j.r_out;
    memcpy(c_out, j.xfin.data() + 1, sizeof(double) * d);
    j.st.ms_total = now_ms() - t_start;
    if (stats) *stats = j.st;
    return j.status;
}

}  // extern "C"
