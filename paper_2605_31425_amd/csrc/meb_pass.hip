// The evaluation pass of ripALM (single-instance launches): the kernel
// instances for every (precision, load width, loads per lane, trials per
// lane) and the launch configuration for a shape.
#include "meb_device.h"

namespace meb {

PassConfig choose_pass_config(int64_t m, int d, int dtype, int num_cu) {
    PassConfig c;
    // 16-byte loads where the row length allows; about 8 elements per lane
    // (G lanes per ball), 64 lanes for long rows
    if (dtype != 0 && d % 4 == 0)
        c.vec = 4;
    else
        c.vec = (d % 2 == 0) ? 2 : 1;
    const int per_lane = (dtype == 0) ? 4 : 8;  // elements per lane
    int need = (d + per_lane - 1) / per_lane;
    int G = 1;
    while (G < need && G < 64) G <<= 1;
    c.G = G;
    c.nl = (d + G * c.vec - 1) / (G * c.vec);
    c.nlmax = c.nl <= 2 ? 2 : (c.nl <= 4 ? 4 : (c.nl <= 8 ? 8 : 16));
    c.waves_per_block = WPB;
    const int bpw = WAVE / G;
    // enough waves to fill the machine, each streaming a contiguous range
    int64_t max_waves = (int64_t)num_cu * 16;
    int64_t steps = (m + bpw - 1) / bpw;
    int64_t waves = steps < max_waves ? steps : max_waves;
    if (waves < 1) waves = 1;
    int64_t steps_per_wave = (steps + waves - 1) / waves;
    c.bw = steps_per_wave * bpw;
    waves = (m + c.bw - 1) / c.bw;
    c.blocks = (int)((waves + WPB - 1) / WPB);
    c.nwaves = c.blocks * WPB;
    return c;
}

struct SingleLaunch {
    const PassArgs& a;
    const PassConfig& cfg;
    hipStream_t s;
    template <typename T, int VEC, int NLMAX, int TRL>
    hipError_t go() {
        const size_t lds = pass_lds_bytes<T, VEC, NLMAX>(a.d);
        const hipError_t ea = ensure_dynamic_lds((const void*)pass_kernel<T, VEC, NLMAX, TRL>, lds);
        if (ea != hipSuccess) return ea;
        hipLaunchKernelGGL((pass_kernel<T, VEC, NLMAX, TRL>), dim3(cfg.blocks), dim3(PASS_THREADS), lds, s, a, cfg);
        return hipGetLastError();
    }
};

// identifies the template instance (instances of one id share a launch)
struct VariantId {
    int id = -1;
    template <typename T, int VEC, int NLMAX, int TRL>
    hipError_t go() {
        id = (sizeof(T) == 8 ? 100000 : 0) + VEC * 1000 + NLMAX * 10 + TRL;
        return hipSuccess;
    }
};

hipError_t launch_pass(const PassArgs& a, const PassConfig& cfg, hipStream_t s) {
    if (a.force_mode >= 0) return launch_pass_eval(a, cfg, s);
    SingleLaunch f{a, cfg, s};
    return visit_pass(a.dtype, cfg, f);
}

int pass_variant(int dtype, const PassConfig& cfg) {
    VariantId f;
    (void)visit_pass(dtype, cfg, f);
    return f.id;
}

}  // namespace meb
