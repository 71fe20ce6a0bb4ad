// The evaluation pass for several instances in one launch (a tick of the
// multi-instance server): one launch per template instance among them.
#include "meb_device.h"

namespace meb {

struct BatchPassLaunch {
    const BatchItem* tab;
    const TickList& L;
    int blocks;
    int max_d;
    int max_stages;
    hipStream_t s;
    template <typename T, int VEC, int NLMAX, int TRL>
    hipError_t go() {
        const size_t lds = pass_lds_bytes<T, VEC, NLMAX>(max_d, max_stages);
        const hipError_t ea = ensure_dynamic_lds((const void*)pass_batch_kernel<T, VEC, NLMAX, TRL>, lds);
        if (ea != hipSuccess) return ea;
        hipLaunchKernelGGL((pass_batch_kernel<T, VEC, NLMAX, TRL>), dim3(blocks), dim3(PASS_THREADS), lds, s, tab, L);
        return hipGetLastError();
    }
};

hipError_t launch_pass_group(const BatchItem* dtab, const TickList& L, int blocks, int max_d, int max_stages,
                             int dtype, const PassConfig& cfg, hipStream_t s) {
    BatchPassLaunch f{dtab, L, blocks, max_d, max_stages, s};
    return visit_pass(dtype, cfg, f);
}

}  // namespace meb
