// The evaluation pass of ripALM (single-instance launches): the kernel
// instances for every (precision, load width, loads per lane, trials per
// lane) and the launch configuration for a shape.
#include <stdlib.h>

#include "meb_device.h"

namespace meb {

int pass_blocks_per_cu(int dtype, const PassConfig& cfg, int d);

// Lane groups for rows of d elements at per_lane elements per lane.
static void group_shape(PassConfig& c, int d, int per_lane) {
    int need = (d + per_lane - 1) / per_lane;
    int G = 1;
    while (G < need && G < 64) G <<= 1;
    c.G = G;
    c.nl = (d + G * c.vec - 1) / (G * c.vec);
    c.nlmax = c.nl <= 2 ? 2 : (c.nl <= 4 ? 4 : (c.nl <= 8 ? 8 : 16));
}

// steps per wave at least (tuning override MEB_PASS_MIN_STEPS; default 1: as
// many waves as steps, up to the resident ones)
int pass_min_steps() {
    static const int v = [] {
        const char* e = getenv("MEB_PASS_MIN_STEPS");
        const int k = e ? atoi(e) : 1;
        return k >= 1 && k <= 1024 ? k : 1;
    }();
    return v;
}

// rounds of resident blocks a long pass is cut into (tuning override
// MEB_PASS_OVERSUB, 1 to 8)
int pass_oversub() {
    static const int v = [] {
        const char* e = getenv("MEB_PASS_OVERSUB");
        const int k = e ? atoi(e) : PASS_OVERSUB_DEFAULT;
        return k >= 1 && k <= 8 ? k : PASS_OVERSUB_DEFAULT;
    }();
    return v;
}

PassConfig choose_pass_config(int64_t m, int d, int dtype, int num_cu) {
    PassConfig c;
    // 16-byte loads where the row length allows
    if (dtype != 0 && d % 4 == 0)
        c.vec = 4;
    else
        c.vec = (d % 2 == 0) ? 2 : 1;
    const int esize = dtype == 0 ? 8 : 4;
    // Rows stream through the waves' LDS rings when a step's rows fit a ring
    // with a block to spare.  In FP32, wide lane groups pay more for group
    // sums and per-step overhead than they save, so groups take about 16
    // elements per lane; FP64 rows (and FP32 rows that would need more than
    // four loads per lane) take 4 (at most four loads, and a step of at most
    // 2 KiB).  Rows too long for the ring (64 lanes per ball) go through
    // registers.
    auto ring_fits = [&]() {
        return pass_ring_capable(c.nlmax) && (int64_t)(WAVE / c.G) * d * esize <= (DMA_MIN_STAGES - 1) * DMA_BLK;
    };
    group_shape(c, d, dtype == 0 ? 4 : 16);
    c.dma = ring_fits() ? 1 : 0;
    if (!c.dma) {
        group_shape(c, d, 4);
        c.dma = ring_fits() ? 1 : 0;
    }
    c.waves_per_block = WPB;
    const int bpw = WAVE / c.G;
    // enough waves to fill the machine once, each streaming a contiguous
    // range: as many as fit on a compute unit at once (for the instance the
    // configuration selects).  A deeper ring (more bytes in flight per wave),
    // where the copy counter allows one, is taken when the LDS it needs does
    // not lower that count, i.e. when registers bound the occupancy anyway.
    // ring depth forced for tuning sweeps (MEB_PASS_STAGES = 4, 8 or 16)
    static const int forced_stages = [] {
        const char* e = getenv("MEB_PASS_STAGES");
        const int v = e ? atoi(e) : 0;
        return (v == 4 || v == 8 || v == 16) ? v : 0;
    }();
    auto resident_waves = [&]() -> int64_t {
        c.stages = DMA_MIN_STAGES;
        int per_cu = pass_blocks_per_cu(dtype, c, d);
        if (c.dma && forced_stages > DMA_MIN_STAGES && forced_stages <= dma_max_stages(c.vec * esize)) {
            PassConfig deep = c;
            deep.stages = forced_stages;
            const int n = pass_blocks_per_cu(dtype, deep, d);
            if (n >= 1) {
                c.stages = forced_stages;
                per_cu = n;
            }
        } else if (c.dma) {
            // the deepest power-of-two ring the copy counter allows that
            // keeps the occupancy
            for (int st = dma_max_stages(c.vec * esize); st > DMA_MIN_STAGES; st >>= 1) {
                PassConfig deep = c;
                deep.stages = st;
                if (pass_blocks_per_cu(dtype, deep, d) >= per_cu) {
                    c.stages = st;
                    break;
                }
            }
        }
        if (per_cu < 1) per_cu = 1;
        // pass_oversub() times the resident waves: the blocks beyond one
        // round start as others finish, so compute units that stream faster
        // take more blocks (per-block records keep the sums' order fixed)
        int64_t mw = (int64_t)num_cu * per_cu * WPB * pass_oversub();
        // the in-kernel reduction takes at most RED_GROUP * SYNC_GROUPS blocks
        if (mw > (int64_t)RED_GROUP * SYNC_GROUPS * WPB) mw = (int64_t)RED_GROUP * SYNC_GROUPS * WPB;
        return mw;
    };
    const int64_t steps = (m + bpw - 1) / bpw;
    // The instances specialized for one group width run fewer instructions
    // per step.  One is taken unless it holds fewer waves per compute unit
    // than the generic instance (more registers) and the pass is long (more
    // than eight steps per wave at the generic instance's occupancy): short
    // passes are bound by the latency of their few steps, not by occupancy.
    c.spec = 0;
    const int64_t mw_generic = resident_waves();
    const int stages_generic = c.stages;
    c.spec = 1;
    int64_t max_waves = resident_waves();
    c.fill_min = (int)(max_waves < mw_generic ? max_waves : mw_generic);
    c.fill_max = (int)(max_waves < mw_generic ? mw_generic : max_waves);
    if (max_waves < mw_generic && steps > 8 * mw_generic) {
        c.spec = 0;
        c.stages = stages_generic;
        max_waves = mw_generic;
    }
    const int64_t min_steps = pass_min_steps();
    int64_t waves = (steps + min_steps - 1) / min_steps;
    if (waves > max_waves) waves = max_waves;
    if (waves < 1) waves = 1;
    int64_t steps_per_wave = (steps + waves - 1) / waves;
    c.bw = steps_per_wave * bpw;
    // the ring path keeps offsets within a wave's range in 32 bits
    if (c.bw * d * esize >= ((int64_t)1 << 30)) {
        c.dma = 0;
        c.stages = DMA_MIN_STAGES;
    }
    waves = (m + c.bw - 1) / c.bw;
    c.blocks = (int)((waves + WPB - 1) / WPB);
    c.nwaves = c.blocks * WPB;
    return c;
}

// resident blocks per compute unit of the instance a configuration uses (at
// its ring depth): a
// block puts one wave on each SIMD, so the count is bounded by the waves a
// SIMD holds at the kernel's register count (512 VGPRs per lane, granule 8),
// by LDS (160 KiB per compute unit) and by 8 waves per SIMD
struct Occupancy {
    int d;
    int stages;
    int n = 0;
    template <typename T, int VEC, int NLMAX, int TRL>
    hipError_t go() {
        const size_t lds = pass_lds_bytes<T, VEC, NLMAX>(d, stages);
        if (lds > LDS_PER_CU) {  // this ring depth does not fit at all
            n = 0;
            return hipSuccess;
        }
        const void* fn = (const void*)pass_kernel<T, VEC, NLMAX, TRL>;
        const hipError_t ea = ensure_dynamic_lds(fn, lds);
        if (ea != hipSuccess) return ea;
        hipFuncAttributes at;
        const hipError_t eb = hipFuncGetAttributes(&at, fn);
        if (eb != hipSuccess) return eb;
        const int regs = at.numRegs > 0 ? (at.numRegs + 7) / 8 * 8 : 128;
        const int by_vgpr = 512 / regs;
        const size_t per_block = lds + at.sharedSizeBytes;
        const int by_lds = per_block > 0 ? (int)(LDS_PER_CU / per_block) : 8;
        n = by_vgpr < by_lds ? by_vgpr : by_lds;
        if (n > 8) n = 8;
        return hipSuccess;
    }
};

int pass_blocks_per_cu(int dtype, const PassConfig& cfg, int d) {
    Occupancy f{d, cfg.stages};
    if (visit_pass(dtype, cfg, f) != hipSuccess) return 4;
    return f.n;
}

struct SingleLaunch {
    const PassArgs& a;
    const PassConfig& cfg;
    hipStream_t s;
    template <typename T, int VEC, int NLMAX, int TRL>
    hipError_t go() {
        const size_t lds = pass_lds_bytes<T, VEC, NLMAX>(a.d, cfg.stages);
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
        id = (sizeof(T) == 8 ? 1000000 : 0) + VEC * 10000 + NLMAX * 100 + TRL;
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
