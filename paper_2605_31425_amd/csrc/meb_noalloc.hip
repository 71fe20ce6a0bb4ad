// meb_check_feasible_noalloc: the a-posteriori feasibility check with its
// scratch in a fixed device array of this library instead of a caller
// workspace, for callers that cannot allocate device memory.
//
// The array `scratch` below is a __device__ symbol: in host code its name is
// only a stand-in for the symbol, not a device address.  Its address on each
// device is looked up once (hipGetSymbolAddress, with that device current)
// and cached; kernels receive that address.
#include <mutex>

#include "meb_host.h"

namespace meb {
namespace {

// Layout of the scratch (bytes, each part 256-byte aligned):
//   cvec  MEB_MAX_D + 8 doubles    the center c
//   res   4 doubles                max, argmax, count (finalize output)
//   wmax, warg, wcnt, offs         NOALLOC_WAVES entries of 8 bytes each
constexpr int NOALLOC_WAVES = 16384;
constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t OFF_CVEC = 0;
constexpr size_t OFF_RES = al256(OFF_CVEC + sizeof(double) * (MEB_MAX_D + 8));
constexpr size_t OFF_WMAX = al256(OFF_RES + sizeof(double) * 4);
constexpr size_t OFF_WARG = al256(OFF_WMAX + sizeof(double) * NOALLOC_WAVES);
constexpr size_t OFF_WCNT = al256(OFF_WARG + sizeof(int64_t) * NOALLOC_WAVES);
constexpr size_t OFF_OFFS = al256(OFF_WCNT + sizeof(int64_t) * NOALLOC_WAVES);
constexpr size_t NOALLOC_BYTES = al256(OFF_OFFS + sizeof(int64_t) * NOALLOC_WAVES);  // about 540 KB

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
char* g_ptr[MAX_DEVICES] = {};

}  // namespace
}  // namespace meb

// one copy per device, kept until the process ends
static __device__ __align__(256) unsigned char scratch[meb::NOALLOC_BYTES];

namespace meb {
namespace {

// device address of `scratch` on the current device (looked up once)
int scratch_ptr(char** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(MEB_ERR_UNSUPPORTED, "device index beyond the library's table");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MEB_ERR_HIP, "scratch symbol has no device address");
        g_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_ptr[dev];
    return MEB_OK;
}

}  // namespace
}  // namespace meb

using namespace meb;

extern "C" int meb_check_feasible_noalloc(const void* C, const void* R, int64_t m, int32_t d, int32_t dtype, double r,
                                          const double* c, double eps, double* delta_max, int64_t* argmax,
                                          int64_t* viol_idx, int64_t viol_cap, int64_t* n_viol, void* stream) {
    CHK(check_common(C, m, d, dtype));
    if (!c) return fail(MEB_ERR_ARG, "c is required");
    if (viol_cap > 0 && !viol_idx) return fail(MEB_ERR_ARG, "viol_idx is NULL with viol_cap > 0");
    const ScanCfg cfg = scan_config(m, d, device_cus());
    if (cfg.nwaves > NOALLOC_WAVES)
        return fail(MEB_ERR_UNSUPPORTED, "the scan of this device needs more wave slots than the fixed scratch holds");
    char* base = nullptr;
    CHK(scratch_ptr(&base));
    double* cvec = reinterpret_cast<double*>(base + OFF_CVEC);
    double* res = reinterpret_cast<double*>(base + OFF_RES);
    double* wmax = reinterpret_cast<double*>(base + OFF_WMAX);
    int64_t* warg = reinterpret_cast<int64_t*>(base + OFF_WARG);
    int64_t* wcnt = reinterpret_cast<int64_t*>(base + OFF_WCNT);
    int64_t* offs = reinterpret_cast<int64_t*>(base + OFF_OFFS);
    int64_t* total = reinterpret_cast<int64_t*>(res + 2);
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(cvec, c, sizeof(double) * d, hipMemcpyHostToDevice, s));
    // pass 1 counts the violated balls of each wave (and the maximum);
    // every wave writes its slots, so nothing needs clearing
    HIPCHK(launch_scan(0, C, R, m, d, dtype, cvec, r, eps, nullptr, nullptr, nullptr, cfg, wmax, warg, wcnt, nullptr,
                       s));
    HIPCHK(launch_scan_finalize(wcnt, wmax, warg, cfg.nwaves, offs, total, res, reinterpret_cast<int64_t*>(res + 1),
                                s));
    // pass 2 (skipped on the device when pass 1 found none) writes each
    // violated index to its final position; the same FP64 arithmetic makes
    // the same decisions as pass 1
    if (viol_cap > 0) {
        ScanPlace pl;
        pl.offs = offs;
        pl.cap = viol_cap;
        pl.gate = total;
        HIPCHK(launch_scan(0, C, R, m, d, dtype, cvec, r, eps, nullptr, nullptr, nullptr, cfg, nullptr, nullptr, nullptr,
                           viol_idx, s, pl));
    }
    double h[3];
    HIPCHK(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (delta_max) *delta_max = h[0];
    if (argmax) memcpy(argmax, &h[1], sizeof(int64_t));
    if (n_viol) memcpy(n_viol, &h[2], sizeof(int64_t));
    return MEB_OK;
}
