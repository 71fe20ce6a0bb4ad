// The single-evaluation pass of meb_al_eval (the per-kernel parity
// surface): one launch over all balls, independent of any solver state.
#include "meb_device.h"

namespace meb {

struct EvalLaunch {
    const PassArgs& a;
    const PassConfig& cfg;
    hipStream_t s;
    template <typename T, int VEC, int NLMAX, int TRL>
    hipError_t go() {
        const size_t lds = pass_lds_bytes<T, VEC, NLMAX>(a.d, cfg.stages);
        const hipError_t ea = ensure_dynamic_lds((const void*)pass_eval_kernel<T, VEC, NLMAX, TRL>, lds);
        if (ea != hipSuccess) return ea;
        hipLaunchKernelGGL((pass_eval_kernel<T, VEC, NLMAX, TRL>), dim3(cfg.blocks), dim3(PASS_THREADS), lds, s, a,
                           cfg);
        return hipGetLastError();
    }
};

hipError_t launch_pass_eval(const PassArgs& a, const PassConfig& cfg, hipStream_t s) {
    EvalLaunch f{a, cfg, s};
    return visit_pass(a.dtype, cfg, f);
}

}  // namespace meb
