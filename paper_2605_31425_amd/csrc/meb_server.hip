// Multi-instance MEB server of libmeb.so: continuous batching of many
// minimum-enclosing-ball solves on one GPU.
//
// Requests are admitted in arrival order (FIFO) when a slot is free and
// their workspace fits in the caller's device pool (first fit, 256-byte
// granules).  An engine thread owns one HIP stream and runs every admitted
// request as a resumable job (the mixed-precision solve of meb_solve).  Each
// loop of the engine
//   1. admits queued requests and starts their first phase;
//   2. advances jobs whose last readback has completed (screening, gather,
//      feasibility check, reinsertion, the start of their next ripALM run);
//   3. enqueues one tick: a single solver step for every job that is inside
//      a ripALM run, batched into one launch per kernel (one per template
//      instance of the evaluation pass), so many small instances share each
//      launch and instances of different sizes overlap on the device;
//   4. retires ticks two behind the newest, reading each job's run-ended
//      flag (written by the control step into pinned host memory).
// Every instance runs the kernels, launch shapes and reduction order it runs
// alone, so its result does not depend on what else is in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "meb_host.h"

namespace meb {

int check_solve_options(const meb_options* o);

// ---------------------------------------------------------------------------
// First-fit allocator over [0, size) in ALIGN granules.
// ---------------------------------------------------------------------------
struct FirstFit {
    std::map<size_t, size_t> free_;  // offset -> length, non-adjacent
    size_t size = 0;
    size_t used = 0;
    size_t peak = 0;
    void reset(size_t n) {
        size = n & ~(ALIGN - 1);
        free_.clear();
        if (size) free_[0] = size;
        used = peak = 0;
    }
    static size_t round(size_t b) { return al(b ? b : 1); }
    bool alloc(size_t bytes, size_t* off) {
        const size_t b = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= b) {
                *off = it->first;
                const size_t rest = it->second - b;
                const size_t roff = it->first + b;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                used += b;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        size_t b = round(bytes);
        size_t o = off;
        used -= b;
        auto nx = free_.lower_bound(o);
        if (nx != free_.end() && o + b == nx->first) {
            b += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == o) {
                o = pv->first;
                b += pv->second;
                free_.erase(pv);
            }
        }
        free_[o] = b;
    }
};

// ---------------------------------------------------------------------------
// Admission: FIFO over (id, bytes), limited by the pool and the slot count.
// The head of the queue blocks the ones behind it, so no request starves.
// ---------------------------------------------------------------------------
struct Admission {
    FirstFit pool;
    int max_active = 0;
    int active = 0;
    std::deque<std::pair<int64_t, size_t>> q;
    void reset(size_t pool_bytes, int slots) {
        pool.reset(pool_bytes);
        max_active = slots;
        active = 0;
        q.clear();
    }
    bool fits_ever(size_t bytes) const { return FirstFit::round(bytes) <= pool.size; }
    void push(int64_t id, size_t bytes) { q.emplace_back(id, bytes); }
    // admits the head if a slot is free and its bytes fit
    bool admit(int64_t* id, size_t* off, size_t* bytes) {
        if (q.empty() || active >= max_active) return false;
        if (!pool.alloc(q.front().second, off)) return false;
        *id = q.front().first;
        *bytes = q.front().second;
        q.pop_front();
        ++active;
        return true;
    }
    void retire(size_t off, size_t bytes) {
        pool.release(off, bytes);
        --active;
    }
};

namespace {

constexpr int TICKS_IN_FLIGHT = 2;

struct Request {
    int64_t ticket;
    int64_t tag;
    const void* C;
    const void* R;
    int64_t m;
    int32_t d;
    double* c_out;
    size_t bytes;
    double t_submit;
};

struct Slot {
    bool used = false;
    Request req{};
    size_t off = 0;
    double t_admit = 0;
    std::unique_ptr<Job> job;
    hipEvent_t ev = nullptr;  // completion of the job's last readback
    uint64_t ev_seq = 0;      // enqueue order of that event
    bool waiting = false;
    bool in_run = false;  // its table entry is stepped by ticks
    int lane = 0;         // the lane (stream) its work runs on
    int err = 0;
    std::string msg;
};

struct Tick {
    hipEvent_t ev = nullptr;
    std::vector<int> slots;
};

}  // namespace

}  // namespace meb

using namespace meb;

// Requests run in one of two lanes, each with its own stream and its own
// ticks: a tick steps every job of its lane that is inside a ripALM run, so
// its duration is set by the lane's largest pass.  Small requests (m d below
// LANE_SPLIT elements) do not wait for the passes of large ones.
constexpr int NLANES = 2;
constexpr double LANE_SPLIT = 8e6;

struct meb_server {
    int dev = 0;
    hipStream_t ls[NLANES] = {nullptr, nullptr};
    char* pool = nullptr;
    size_t pool_bytes = 0;
    char* pool_jobs = nullptr;  // after the item table
    meb_options o{};
    int max_active = 0;
    int max_d = 0;
    Admission adm;
    std::vector<Slot> slots;
    BatchItem* dtab = nullptr;  // device item table (in the pool)
    BatchItem* htab = nullptr;  // pinned host mirror: upload sources
    int* hflag = nullptr;       // pinned, device-mapped run-ended flags
    int* dflag = nullptr;
    double* pinslab = nullptr;  // per-slot job staging
    size_t pin_stride = 0;
    std::deque<Tick> ticks[NLANES];
    std::vector<hipEvent_t> tick_events;
    int64_t lane_ticks[NLANES] = {0, 0};
    uint64_t seq = 0;
    int64_t n_ticks = 0;
    double tick_items = 0;
    // shared with the API threads
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> incoming;
    std::deque<meb_server_result> done;
    std::map<int64_t, Request> pending;  // queued, not yet admitted
    int64_t next_ticket = 1;
    int64_t n_submitted = 0, n_completed = 0, n_failed = 0;
    int n_queued = 0, n_active = 0;
    size_t pool_used = 0, pool_peak = 0;
    bool stop = false;
    std::thread th;
    std::string fatal;

    ~meb_server();
    void loop();
    int admit_locked(std::vector<int>& started);
    int start_slot(int k);
    int advance(int k);
    int upload_item(int k);
    void complete(int k, int rc);
    int tick(int lane);
    int retire_tick(int lane);
    hipStream_t stream_of(int k) const { return ls[slots[k].lane]; }
};

meb_server::~meb_server() {
    for (auto& sl : slots)
        if (sl.ev) (void)hipEventDestroy(sl.ev);
    for (auto e : tick_events) (void)hipEventDestroy(e);
    if (htab) (void)hipHostFree(htab);
    if (hflag) (void)hipHostFree(hflag);
    if (pinslab) (void)hipHostFree(pinslab);
    for (auto st : ls)
        if (st) (void)hipStreamDestroy(st);
}

// Admits what fits; returns the slots started.  Called with `mu` held.
int meb_server::admit_locked(std::vector<int>& started) {
    while (!incoming.empty()) {
        const Request& r = incoming.front();
        pending[r.ticket] = r;
        adm.push(r.ticket, r.bytes);
        incoming.pop_front();
    }
    for (;;) {
        int k = -1;
        for (int i = 0; i < max_active; ++i)
            if (!slots[i].used) {
                k = i;
                break;
            }
        if (k < 0) break;
        int64_t id;
        size_t off, bytes;
        if (!adm.admit(&id, &off, &bytes)) break;
        Slot& sl = slots[k];
        sl.used = true;
        sl.req = pending[id];
        pending.erase(id);
        sl.off = off;
        sl.lane = (double)sl.req.m * sl.req.d >= LANE_SPLIT ? 1 : 0;
        sl.t_admit = now_ms();
        sl.waiting = false;
        sl.in_run = false;
        sl.err = 0;
        sl.msg.clear();
        started.push_back(k);
    }
    n_queued = (int)adm.q.size();
    n_active = adm.active;
    pool_used = adm.pool.used;
    pool_peak = adm.pool.peak;
    return MEB_OK;
}

int meb_server::start_slot(int k) {
    Slot& sl = slots[k];
    sl.job.reset(new Job());
    CHK(sl.job->init(sl.req.C, sl.req.R, sl.req.m, sl.req.d, MEB_F64, &o, pool_jobs + sl.off, sl.req.bytes,
                     pinslab + (size_t)k * pin_stride, nullptr, nullptr));
    hipStream_t s = stream_of(k);
    CHK(sl.job->start(s));
    HIPCHK(hipEventRecord(sl.ev, s));
    sl.ev_seq = ++seq;
    sl.waiting = true;
    return MEB_OK;
}

// Writes the slot's table entry for its current run and uploads it (the
// pinned source is rewritten only at the job's next run, after this copy).
int meb_server::upload_item(int k) {
    Slot& sl = slots[k];
    Job& j = *sl.job;
    htab[k] = j.e->item(j.pa, dflag + k);
    hflag[k] = PM_EVAL;
    HIPCHK(hipMemcpyAsync(dtab + k, htab + k, sizeof(BatchItem), hipMemcpyHostToDevice, stream_of(k)));
    sl.in_run = true;
    return MEB_OK;
}

// The slot's readback has completed: run the job's next phase.
int meb_server::advance(int k) {
    Slot& sl = slots[k];
    Job& j = *sl.job;
    hipStream_t s = stream_of(k);
    sl.waiting = false;
    CHK(j.on_ready(s));
    if (j.done()) return MEB_OK;
    if (j.stepping()) return upload_item(k);
    HIPCHK(hipEventRecord(sl.ev, s));
    sl.ev_seq = ++seq;
    sl.waiting = true;
    return MEB_OK;
}

void meb_server::complete(int k, int rc) {
    Slot& sl = slots[k];
    meb_server_result r;
    memset(&r, 0, sizeof(r));
    r.ticket = sl.req.ticket;
    r.tag = sl.req.tag;
    r.m = sl.req.m;
    r.d = sl.req.d;
    r.t_submit_ms = sl.req.t_submit;
    r.t_admit_ms = sl.t_admit;
    r.t_done_ms = now_ms();
    if (rc < 0) {
        r.status = rc;
        snprintf(r.message, sizeof(r.message), "%s", last_error_text());
    } else {
        Job& j = *sl.job;
        r.status = j.status;
        r.r = j.r_out;
        if (sl.req.c_out) memcpy(sl.req.c_out, j.xfin.data() + 1, sizeof(double) * sl.req.d);
        r.stats = j.st;
        r.stats.ms_total = r.t_done_ms - sl.t_admit;
    }
    sl.job.reset();
    sl.used = false;
    sl.waiting = false;
    sl.in_run = false;
    std::lock_guard<std::mutex> g(mu);
    adm.retire(sl.off, sl.req.bytes);
    n_active = adm.active;
    pool_used = adm.pool.used;
    if (rc < 0)
        ++n_failed;
    else
        ++n_completed;
    done.push_back(r);
    cv_done.notify_all();
}

// One solver step for every job of the lane inside a run.
int meb_server::tick(int lane) {
    std::vector<int> list;
    for (int k = 0; k < max_active; ++k)
        if (slots[k].used && slots[k].in_run && slots[k].lane == lane) list.push_back(k);
    if (list.empty()) return 0;
    hipStream_t s = ls[lane];
    HIPCHK(launch_tick(dtab, htab, list.data(), (int)list.size(), s));
    for (int k : list) slots[k].job->steps += 1;
    Tick t;
    // each lane cycles through events of its own (more than it keeps queued)
    t.ev = tick_events[lane * (TICKS_IN_FLIGHT + 1) + lane_ticks[lane]++ % (TICKS_IN_FLIGHT + 1)];
    HIPCHK(hipEventRecord(t.ev, s));
    t.slots.swap(list);
    tick_items += (double)t.slots.size();
    ++n_ticks;
    ticks[lane].push_back(std::move(t));
    return 1;
}

// Waits for the lane's oldest tick and ends the runs it finished.
int meb_server::retire_tick(int lane) {
    Tick t = std::move(ticks[lane].front());
    ticks[lane].pop_front();
    hipStream_t s = ls[lane];
    HIPCHK(hipEventSynchronize(t.ev));
    for (int k : t.slots) {
        Slot& sl = slots[k];
        if (!sl.used || !sl.in_run) continue;
        Job& j = *sl.job;
        const int mode = *(volatile int*)(hflag + k);
        const bool ended = mode == PM_DONE;
        if (ended || j.steps > j.max_steps) {
            j.forced_end = !ended;
            sl.in_run = false;
            int rc = j.end_run(s);
            if (rc >= 0) {
                if (hipEventRecord(sl.ev, s) != hipSuccess) rc = fail(MEB_ERR_HIP, "hipEventRecord failed");
                sl.ev_seq = ++seq;
                sl.waiting = true;
            }
            if (rc < 0) complete(k, rc);
        }
    }
    return MEB_OK;
}

void meb_server::loop() {
    if (hipSetDevice(dev) != hipSuccess) {
        std::lock_guard<std::mutex> g(mu);
        fatal = "hipSetDevice failed in the engine thread";
        stop = true;
        cv_done.notify_all();
        return;
    }
    for (;;) {
        std::vector<int> started;
        {
            std::unique_lock<std::mutex> g(mu);
            const bool idle = incoming.empty() && adm.q.empty() && adm.active == 0;
            if (idle && stop) break;
            if (idle) {
                cv_work.wait_for(g, std::chrono::milliseconds(50));
                continue;
            }
            admit_locked(started);
        }
        bool progressed = !started.empty();
        for (int k : started) {
            const int rc = start_slot(k);
            if (rc < 0) complete(k, rc);
        }
        // jobs whose readback has completed
        for (int k = 0; k < max_active; ++k) {
            Slot& sl = slots[k];
            if (!sl.used || !sl.waiting) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) continue;
            progressed = true;
            int rc = q == hipSuccess ? advance(k) : fail(MEB_ERR_HIP, hipGetErrorString(q));
            if (rc < 0 || (sl.job && sl.job->done())) complete(k, rc);
        }
        // each lane keeps TICKS_IN_FLIGHT ticks queued; a lane's oldest
        // tick is retired when it has completed, or waited for when the lane
        // is full (or idle with ticks left) and nothing else progressed
        bool bad = false;
        int full[NLANES];
        for (int lane = 0; lane < NLANES && !bad; ++lane) {
            full[lane] = 0;
            if ((int)ticks[lane].size() < TICKS_IN_FLIGHT) {
                const int launched = tick(lane);
                if (launched < 0) {
                    bad = true;
                    break;
                }
                progressed = progressed || launched > 0;
                if (launched == 0 && !ticks[lane].empty()) full[lane] = 1;
            }
            if ((int)ticks[lane].size() >= TICKS_IN_FLIGHT) full[lane] = 1;
            while (!ticks[lane].empty() && hipEventQuery(ticks[lane].front().ev) == hipSuccess) {
                if (retire_tick(lane) < 0) {
                    bad = true;
                    break;
                }
                progressed = true;
                full[lane] = 0;
            }
        }
        if (!bad && !progressed) {
            // both lanes waiting on the device: block on the lane whose
            // oldest tick was enqueued first
            int w = -1;
            for (int lane = 0; lane < NLANES; ++lane)
                if (full[lane] && !ticks[lane].empty()) {
                    w = lane;
                    break;
                }
            if (w >= 0) {
                if (retire_tick(w) < 0) bad = true;
                progressed = true;
            }
        }
        if (bad) {
            std::lock_guard<std::mutex> g(mu);
            fatal = last_error_text();
            break;
        }
        if (!progressed) {
            // only readbacks outstanding: wait for the earliest enqueued one
            int best = -1;
            for (int k = 0; k < max_active; ++k)
                if (slots[k].used && slots[k].waiting && (best < 0 || slots[k].ev_seq < slots[best].ev_seq)) best = k;
            if (best >= 0) (void)hipEventSynchronize(slots[best].ev);
        }
    }
    // fail whatever is left (only after a fatal error)
    for (auto st : ls) (void)hipStreamSynchronize(st);
    for (int k = 0; k < max_active; ++k)
        if (slots[k].used) complete(k, fail(MEB_ERR_HIP, fatal.empty() ? "server stopped" : fatal));
    std::lock_guard<std::mutex> g(mu);
    while (!incoming.empty()) {
        meb_server_result r;
        memset(&r, 0, sizeof(r));
        r.ticket = incoming.front().ticket;
        r.tag = incoming.front().tag;
        r.status = MEB_ERR_HIP;
        snprintf(r.message, sizeof(r.message), "%s", fatal.empty() ? "server stopped" : fatal.c_str());
        done.push_back(r);
        incoming.pop_front();
        ++n_failed;
    }
    stop = true;
    cv_done.notify_all();
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int meb_server_create(void* pool, size_t pool_bytes, const meb_options* opts, int32_t max_active, int32_t max_d,
                      meb_server** out) {
    if (!out) return fail(MEB_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!pool || pool_bytes == 0) return fail(MEB_ERR_ARG, "pool is required");
    if ((uintptr_t)pool % ALIGN) return fail(MEB_ERR_ARG, "pool must be 256-byte aligned");
    if (max_active < 1 || max_active > 1024) return fail(MEB_ERR_ARG, "max_active must be in [1, 1024]");
    if (max_d < 1 || max_d > MEB_MAX_D) return fail(MEB_ERR_ARG, "max_d must be in [1, MEB_MAX_D]");
    meb_options def;
    meb_default_options(&def);
    const meb_options* o = opts ? opts : &def;
    CHK(check_solve_options(o));
    if (o->profile) return fail(MEB_ERR_ARG, "per-pass profiling is not available in the server");
    if (o->newton != MEB_NEWTON_DENSE) return fail(MEB_ERR_ARG, "the server solves Newton systems densely");
    std::unique_ptr<meb_server> sv(new meb_server());
    HIPCHK(hipGetDevice(&sv->dev));
    sv->o = *o;
    sv->max_active = max_active;
    sv->max_d = max_d;
    sv->pool = (char*)pool;
    sv->pool_bytes = pool_bytes;
    const size_t tab_bytes = al(sizeof(BatchItem) * (size_t)max_active);
    if (tab_bytes >= pool_bytes) return fail(MEB_ERR_WORKSPACE, "pool too small");
    sv->dtab = reinterpret_cast<BatchItem*>(pool);
    sv->pool_jobs = (char*)pool + tab_bytes;
    sv->adm.reset(pool_bytes - tab_bytes, max_active);
    sv->slots.resize(max_active);
    for (auto& sl : sv->slots) HIPCHK(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    sv->tick_events.resize(NLANES * (TICKS_IN_FLIGHT + 1));
    for (auto& e : sv->tick_events) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(hipHostMalloc((void**)&sv->htab, sizeof(BatchItem) * (size_t)max_active, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&sv->hflag, sizeof(int) * (size_t)max_active,
                         hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void**)&sv->dflag, sv->hflag, 0));
    sv->pin_stride = (JobPin::doubles(max_d) + 31) & ~(size_t)31;
    HIPCHK(hipHostMalloc((void**)&sv->pinslab, sizeof(double) * sv->pin_stride * (size_t)max_active,
                         hipHostMallocDefault));
    for (auto& st : sv->ls) HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    sv->th = std::thread([p = sv.get()] { p->loop(); });
    *out = sv.release();
    return MEB_OK;
}

int meb_server_submit(meb_server* sv, const void* C, const void* R, int64_t m, int32_t d, int32_t dtype, int64_t tag,
                      double* c_out, int64_t* ticket) {
    if (!sv) return fail(MEB_ERR_ARG, "server is NULL");
    CHK(check_common(C, m, d, dtype));
    if (dtype != MEB_F64) return fail(MEB_ERR_ARG, "the server needs FP64 input");
    if (d > sv->max_d) return fail(MEB_ERR_ARG, "d exceeds the server's max_d");
    const size_t bytes = solve_ws_bytes(m, d, MEB_F64, &sv->o);
    Request r;
    r.tag = tag;
    r.C = C;
    r.R = R;
    r.m = m;
    r.d = d;
    r.c_out = c_out;
    r.bytes = bytes;
    r.t_submit = now_ms();
    {
        std::lock_guard<std::mutex> g(sv->mu);
        if (sv->stop) return fail(MEB_ERR_ARG, "server is stopping");
        if (!sv->adm.fits_ever(bytes)) return fail(MEB_ERR_WORKSPACE, "request does not fit in the pool");
        r.ticket = sv->next_ticket++;
        sv->incoming.push_back(r);
        ++sv->n_submitted;
        ++sv->n_queued;
    }
    sv->cv_work.notify_one();
    if (ticket) *ticket = r.ticket;
    return MEB_OK;
}

int meb_server_poll(meb_server* sv, meb_server_result* out, int32_t cap, int32_t wait_ms, int32_t* n_out) {
    if (!sv || !n_out || (cap > 0 && !out)) return fail(MEB_ERR_ARG, "bad arguments");
    *n_out = 0;
    std::unique_lock<std::mutex> g(sv->mu);
    if (sv->done.empty() && wait_ms > 0 && !sv->stop)
        sv->cv_done.wait_for(g, std::chrono::milliseconds(wait_ms), [sv] { return !sv->done.empty() || sv->stop; });
    int n = 0;
    while (n < cap && !sv->done.empty()) {
        out[n++] = sv->done.front();
        sv->done.pop_front();
    }
    *n_out = n;
    return MEB_OK;
}

int meb_server_info(meb_server* sv, meb_server_stats* info) {
    if (!sv || !info) return fail(MEB_ERR_ARG, "bad arguments");
    std::lock_guard<std::mutex> g(sv->mu);
    memset(info, 0, sizeof(*info));
    info->submitted = sv->n_submitted;
    info->completed = sv->n_completed;
    info->failed = sv->n_failed;
    info->queued = (int32_t)(sv->incoming.size() + sv->adm.q.size());
    info->active = sv->adm.active;
    info->pool_used = sv->pool_used;
    info->pool_peak = sv->pool_peak;
    info->pool_capacity = sv->adm.pool.size;
    info->ticks = sv->n_ticks;
    info->mean_tick_items = sv->n_ticks ? sv->tick_items / (double)sv->n_ticks : 0.0;
    if (!sv->fatal.empty()) snprintf(info->message, sizeof(info->message), "%s", sv->fatal.c_str());
    return MEB_OK;
}

int meb_server_destroy(meb_server* sv) {
    if (!sv) return MEB_OK;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->th.joinable()) sv->th.join();
    delete sv;
    return MEB_OK;
}

// Discrete-event run of the admission policy with a simulated clock and
// caller-given service times, for testing it without a GPU.
int meb_sched_simulate(int32_t n, const double* arrival, const double* service, const uint64_t* bytes,
                       uint64_t pool_bytes, int32_t max_active, double* t_admit, double* t_done, uint64_t* offset) {
    if (n < 0 || max_active < 1 || (n > 0 && (!arrival || !service || !bytes || !t_admit || !t_done || !offset)))
        return fail(MEB_ERR_ARG, "bad arguments");
    for (int i = 1; i < n; ++i)
        if (arrival[i] < arrival[i - 1]) return fail(MEB_ERR_ARG, "arrivals must be non-decreasing");
    Admission adm;
    adm.reset(pool_bytes, max_active);
    for (int i = 0; i < n; ++i)
        if (!adm.fits_ever(bytes[i])) return fail(MEB_ERR_WORKSPACE, "a request does not fit in the pool");
    // running: (done time, id)
    std::multimap<double, int> running;
    int next = 0;
    double now = 0.0;
    int finished = 0;
    while (finished < n) {
        // next event: an arrival or a completion, completions first on ties
        const double ta = next < n ? arrival[next] : INFINITY;
        const double td = running.empty() ? INFINITY : running.begin()->first;
        if (td <= ta) {
            now = td;
            while (!running.empty() && running.begin()->first == now) {
                const int id = running.begin()->second;
                running.erase(running.begin());
                adm.retire(offset[id], bytes[id]);
                ++finished;
            }
        } else {
            now = ta;
            while (next < n && arrival[next] == now) {
                adm.push(next, bytes[next]);
                ++next;
            }
        }
        int64_t id;
        size_t off, b;
        while (adm.admit(&id, &off, &b)) {
            t_admit[id] = now;
            offset[id] = off;
            t_done[id] = now + service[id];
            running.emplace(t_done[id], (int)id);
        }
    }
    return MEB_OK;
}

}  // extern "C"
