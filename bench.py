"""Benchmark: time-to-solution of the minimum enclosing ball on one MI355X.

Workload (default): balls, m = 1,000,000, d = 100, centers uniform in
[-1, 1]^d, radii uniform in [0, 0.1], FP64 storage, seed 2 -- synthetic data
of the shape the headline metric is quoted on.  One step is one complete
meb_solve in mixed precision (FP32 preparation and screening run, FP64
refinement of the retained balls, full FP64 feasibility check with
reinsertion, radius fix-up), with the instance already resident in HBM.
The plain FP64 ripALM solve of the same instance is timed beside it.

Prints one JSON line.  `roofline` is the FP32 evaluation pass (the dominant
kernel): algorithmic bytes it reads and writes (centers, radii, multipliers;
counted on the device per launch) over its launch durations, both measured
live with HIP events on the solve's stream during the timed steps.
`cpu_baseline` runs the CPU oracle on a bounded sample of the same instance.

`serving` is the request-stream leg: requests with m log-uniform in
[1e3, 1e6], d uniform over {2, 3, 10, 50, 200}, centers N(0, I), radii
uniform in [0, 0.05], arriving as a Poisson stream, solved in mixed
precision by the multi-instance server (meb_server_*).  Request data are
windows of one device-resident bank of random numbers, so the stream needs
no host-side generation; a request is submitted at its arrival time and its
latency runs from submission to completion.  The leg first measures the
saturation throughput (every request queued at once), then replays the
stream at a fraction of it and reports p50 / p99 latency and solves/s.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "balls_1e6_d100": dict(gen="balls_uniform", args=(1000000, 100, 2),
                           desc="balls, m=1,000,000, d=100, centers U[-1,1]^d, radii U[0,0.1], FP64, seed 2"),
    "points_1e4_d10": dict(gen="points_normal", args=(10000, 10, 1),
                           desc="points, m=10,000, d=10, centers N(0,I), FP64, seed 1"),
    "points_1e7_d10": dict(gen="points_ball_sphere", args=(10000000, 10, 4),
                           desc="points, m=10,000,000, d=10, 90% in the unit ball, 10% on the sphere, seed 4"),
    "balls_2e5_d1000": dict(gen="balls_normal", args=(200000, 1000, 3),
                            desc="balls, m=200,000, d=1000, centers N(0,I), radii |N(0,0.05^2)|, seed 3"),
}


PROFILE_HBM = os.path.join(ROOT, "profiles", "pass_kernel_f32_balls_1e6_d100_hbm.md")


def measured_traffic():
    """HBM bytes per launch of the FP32 evaluation pass from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when the kernel source
    has changed since the counters were taken."""
    import hashlib
    import re
    try:
        txt = open(PROFILE_HBM).read()
    except OSError:
        return None
    m_t = re.search(r"traffic_bytes_per_launch: (\d+)", txt)
    m_h = re.search(r"source_sha256\(meb_device.h\): ([0-9a-f]+)", txt)
    if not m_t or not m_h:
        return None
    src = os.path.join(ROOT, "paper_2605_31425_amd", "csrc", "meb_device.h")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_h.group(1):
        return None
    return float(m_t.group(1))


def golden(name):
    p = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.json")
    if os.path.exists(p):
        with open(p) as f:
            return json.load(f)
    return None


def host_cpu():
    """Core count and model of the host this runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count(), len(os.sched_getaffinity(0)), model


def cpu_baseline(C, R, m_full, sample_m):
    """The oracle as it stands (plain C, one thread), on the first sample_m
    balls; time-to-solution scaled by m_full / sample_m (each pass is linear
    in m, and the iteration counts of the sample and the full instance are
    alike)."""
    import oracle
    Cs = np.ascontiguousarray(C[:sample_m])
    Rs = None if R is None else np.ascontiguousarray(R[:sample_m])
    t = time.perf_counter()
    oracle.ripalm(Cs, Rs, tol=1e-8)
    el = time.perf_counter() - t
    ncpu, naff, model = host_cpu()
    return dict(value=el * m_full / sample_m, unit="s", cores=1, kind="oracle",
                sample=f"oracle ripALM to KKT 1e-8 on the first {sample_m} balls of the same instance "
                       f"({el:.2f} s on one core), scaled by {m_full}/{sample_m}",
                host_cpus=ncpu, host_cpus_available=naff, host_cpu_model=model, sample_seconds=el)


def time_solves(meb, Cd, Rd, mode, reps, hess="auto"):
    """(ms per solve, last result) of `reps` solves after one warm-up."""
    import torch
    o = meb.options(mode=mode, hess=hess)
    meb.solve(Cd, Rd, opts=o)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        res = meb.solve(Cd, Rd, opts=o)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3 / reps, res


def other_workloads(names, log):
    """Time-to-solution of the other workloads, mixed and plain FP64, with
    their error against the oracle's stored radius."""
    import torch
    from paper_2605_31425_amd import inputs, meb
    out = {}
    for name in names:
        wl = WORKLOADS[name]
        m, d, seed = wl["args"]
        C, R = getattr(inputs, wl["gen"])(m, d, seed)
        Cd = torch.as_tensor(C, device="cuda:0")
        Rd = None if R is None else torch.as_tensor(R, device="cuda:0")
        g = golden(name)
        row = dict(workload=wl["desc"])
        for mode in ("mixed", "fp64"):
            ms, (r, c, st) = time_solves(meb, Cd, Rd, mode, 1 if m * d > 1e8 else 3)
            row[f"{mode}_ms"] = ms
            row[f"{mode}_radius_relerr_vs_oracle"] = abs(r - g["r_fixed"]) / g["r_fixed"] if g else None
            row[f"{mode}_passes"] = st["passes"]
            row[f"{mode}_newton_steps"] = st["inner"]
            row[f"{mode}_ms_phase"] = [round(x, 3) for x in st["ms_phase"]]
            row[f"{mode}_mid_rows_max"] = st["mid_rows_max"]
            if mode == "mixed":
                row["kept_for_fp64"] = st["n_red"]
                row["reinsert_rounds"] = st["reinsert_rounds"]
        row["speedup_mixed_vs_fp64"] = row["fp64_ms"] / row["mixed_ms"]
        log(f"{name}: mixed {row['mixed_ms']:.2f} ms, fp64 {row['fp64_ms']:.2f} ms")
        out[name] = row
        del Cd, Rd
        torch.cuda.empty_cache()
    return out


# Table 1 of the paper: balls kept for the FP64 run (RTX 4070 runs; context)
TABLE1 = {20: (23, 43, 82, 405, 807), 30: (28, 42, 88, 449, 899), 40: (45, 77, 155, 780, 1586),
          50: (41, 96, 182, 929, 1852)}


def paper_instances(log):
    """The paper's LCG instances (Section 5): the Figure 2 / Table 1 grid and
    the Figure 3 shapes up to d = 1000, mixed and plain FP64, with the kept
    counts beside Table 1's (not comparable one to one: the paper does not
    state its screening margin) and the error against the oracle."""
    import torch
    from paper_2605_31425_amd import inputs, meb
    p = os.path.join(ROOT, "tests", "golden", "oracle_lcg.json")
    gold = {}
    if os.path.exists(p):
        with open(p) as f:
            gold = {(e["d"], e["m"]): e["r_fixed"] for e in json.load(f)["instances"]}
    rows = []
    ms_list = (1000, 5000, 10000, 50000, 100000)
    shapes = [(d, m) for d in (20, 30, 40, 50) for m in ms_list] + [(d, m) for d in (100, 500, 1000)
                                                                     for m in (1000, 5000)]
    for d, m in shapes:
        C, R = inputs.lcg_instance(m, d)
        Cd = torch.as_tensor(C, device="cuda:0")
        Rd = torch.as_tensor(R, device="cuda:0")
        row = dict(d=d, m=m)
        for mode in ("mixed", "fp64"):
            ms, (r, c, st) = time_solves(meb, Cd, Rd, mode, 3)
            row[f"{mode}_ms"] = round(ms, 3)
            ref = gold.get((d, m))
            row[f"{mode}_relerr"] = abs(r - ref) / ref if ref else None
            if mode == "mixed":
                row["kept"] = st["n_red"]
                if d in TABLE1:
                    row["kept_paper_table1"] = TABLE1[d][ms_list.index(m)]
        rows.append(row)
    log(f"paper instances: {len(rows)} shapes, mixed total {sum(r['mixed_ms'] for r in rows):.1f} ms")
    return rows


def serving_leg(n_req, loads, seed, max_active, pool_gb, check_sample, log):
    """Saturation run, then one Poisson stream at each of `loads` x the
    saturation rate (the first load's stream is the one reported at the top
    level; every load's latencies are listed under "loads")."""
    import torch

    from paper_2605_31425_amd import inputs, meb

    reqs = inputs.serving_requests(n_req, seed)
    need = max(m * d for m, d, _ in reqs)
    mmax = max(m for m, _, _ in reqs)
    bank_n = max(need * 5 // 4, 1 << 20)
    Z, Rb = inputs.serving_bank_device(bank_n, mmax * 2, seed)
    rng = np.random.default_rng(seed + 1)
    views = []
    for m, d, _ in reqs:
        o = int(rng.integers(0, (bank_n - m * d) // 2 + 1)) * 2  # 16-byte aligned rows
        ro = int(rng.integers(0, mmax + 1))
        views.append((Z[o:o + m * d].view(m, d), Rb[ro:ro + m]))
    torch.cuda.synchronize()
    opts = meb.options(mode="mixed")

    def run(arrivals):
        srv = meb.Server(int(pool_gb * (1 << 30)), opts=opts, max_active=max_active, max_d=256)
        res = {}
        try:
            t0 = time.perf_counter()
            i = 0
            while len(res) < n_req:
                now = time.perf_counter() - t0
                while i < n_req and arrivals[i] <= now:
                    C, R = views[i]
                    srv.submit(C, R, tag=i)
                    i += 1
                wait = 0 if i < n_req else 50
                if i < n_req:
                    wait = max(0, min(2, int((arrivals[i] - (time.perf_counter() - t0)) * 1e3)))
                for r in srv.poll(wait_ms=wait, cap=1024):
                    res[r["tag"]] = r
            info = srv.info()
        finally:
            srv.close()
        bad = [r for r in res.values() if r["status"] < 0]
        if bad:
            raise RuntimeError(f"serving: {len(bad)} requests failed: {bad[0]['message']}")
        lat = np.array([res[k]["t_done_ms"] - res[k]["t_submit_ms"] for k in range(n_req)])
        t_first = min(r["t_submit_ms"] for r in res.values())
        t_last = max(r["t_done_ms"] for r in res.values())
        return res, lat, n_req / ((t_last - t_first) / 1e3), info

    _, lat_sat, thr_sat, info_sat = run(np.zeros(n_req))
    log(f"serving saturation: {thr_sat:.1f} solves/s, mean tick items {info_sat['mean_tick_items']:.1f}")
    sweep = []
    main = None
    for load in loads:
        rate = load * thr_sat
        arr = inputs.poisson_arrivals(n_req, rate, seed + 2)
        res_l, lat_l, thr_l, info_l = run(arr)
        log(f"serving stream at {rate:.1f}/s ({load} x saturation): p50 {np.percentile(lat_l, 50):.2f} ms "
            f"p99 {np.percentile(lat_l, 99):.2f} ms")
        sweep.append(dict(load_vs_saturation=load, arrival_rate_per_s=rate, solves_per_s=thr_l,
                          p50_ms=float(np.percentile(lat_l, 50)), p99_ms=float(np.percentile(lat_l, 99)),
                          mean_ms=float(lat_l.mean()), mean_requests_per_tick=info_l["mean_tick_items"]))
        if main is None or abs(load - 0.7) < abs(main[0] - 0.7):
            main = (load, rate, res_l, lat_l, thr_l, info_l)
    load, rate, res, lat, thr, info = main
    # sample: bitwise equal to meb_solve alone, and feasible in FP64
    idx = sorted(rng.choice(n_req, size=min(check_sample, n_req), replace=False).tolist())
    same, viol = True, -np.inf
    for k in idx:
        C, R = views[k]
        r, c, _ = meb.solve(C, R, opts=opts)
        same = same and (r == res[k]["r"]) and bool(np.array_equal(c, res[k]["c"]))
        dmax, _, _, _ = meb.check_feasible(C, R, res[k]["r"], res[k]["c"], np.inf, viol_cap=0)
        viol = max(viol, dmax / (1 + res[k]["r"]))
    ms = np.array([m for m, _, _ in reqs])
    return {
        "requests": n_req,
        "arrivals": "poisson",
        "arrival_rate_per_s": rate,
        "load_vs_saturation": load,
        "solves_per_s": thr,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "saturation_solves_per_s": thr_sat,
        "saturation_p50_ms": float(np.percentile(lat_sat, 50)),
        "saturation_p99_ms": float(np.percentile(lat_sat, 99)),
        "mean_requests_per_tick": info["mean_tick_items"],
        "ticks": info["ticks"],
        "pool_peak_GB": info["pool_peak"] / 1e9,
        "max_active": max_active,
        "m_range": [int(ms.min()), int(ms.max())],
        "dims": sorted(set(d for _, d, _ in reqs)),
        "sample_checked": len(idx),
        "sample_bitwise_equal_to_meb_solve": same,
        "sample_max_violation_rel": viol,
        "loads": sweep,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="balls_1e6_d100", choices=sorted(WORKLOADS))
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=250000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--serve-load", type=float, nargs="+", default=[0.5, 0.7, 0.9])
    ap.add_argument("--no-others", action="store_true", help="skip the other workloads and the paper's instances")
    ap.add_argument("--serve-max-active", type=int, default=128)
    ap.add_argument("--serve-pool-gb", type=float, default=64.0)
    ap.add_argument("--serve-check", type=int, default=8)
    ap.add_argument("--contraction-probe", action="store_true",
                    help="only run single evaluations with the Hessian contraction of 10^5 mid-case balls at d = 1000 "
                         "in each arithmetic (time the kernels with rocprofv3)")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (3 times), to scale HBM byte counters")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {a.gpus} is not supported "
              "(the path would shard the balls by rows across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch

    if a.copy_calibration > 0:
        n = int(a.copy_calibration * (1 << 30)) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)
        return

    from paper_2605_31425_amd import inputs, meb

    if a.contraction_probe:
        # balls N(0, I) in d = 1000, radii |N(0, 0.05^2)|, evaluated at c = 0 with r the median reach: about half
        # the balls lie in the third projection case, so the contraction has K ~ 10^5 rows
        m, d = 200000, 1000
        gen = torch.Generator(device="cuda:0").manual_seed(3)
        C64 = torch.randn((m, d), generator=gen, device="cuda:0", dtype=torch.float64)
        R64 = torch.randn(m, generator=gen, device="cuda:0", dtype=torch.float64).abs() * 0.05
        x = np.zeros(d + 1)
        x[0] = float((C64.norm(dim=1) + R64).median())
        res = []
        for dt, hess in [(torch.float32, "mfma_bf16"), (torch.float32, "mfma_f32"), (torch.float64, "mfma_f64"),
                         (torch.float64, "f64")]:
            C, R = C64.to(dt), R64.to(dt)
            U = torch.zeros(m, device="cuda:0", dtype=dt)
            V = torch.zeros((m, d), device="cuda:0", dtype=dt)
            want = meb.WANT_PSI | meb.WANT_GRAD | meb.WANT_HESS | (meb._HESS[hess] << 8)
            for _ in range(4):
                out = meb.al_eval(C, R, U, V, x, x.copy(), 1.0, 1.0, want=want)
            torch.cuda.synchronize()
            k_mid = int(round(2.0 * (out["H"][0, 0] - 1.0)))  # H_rr = tau/sigma + sigma N_I + sigma/2 N_mid
            res.append({"dtype": str(dt).replace("torch.", ""), "hess": hess, "mid_rows": k_mid,
                        "flop_per_contraction": float(k_mid) * d * (d + 1)})
        print(json.dumps({"contraction_probe": res}), flush=True)
        return

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    wl = WORKLOADS[a.workload]
    gen = getattr(inputs, wl["gen"])
    m, d, seed = wl["args"]
    C, R = gen(m, d, seed)
    dev = torch.device("cuda:0")
    Cd = torch.as_tensor(C, device=dev)
    Rd = None if R is None else torch.as_tensor(R, device=dev)
    opts_mixed = meb.options(mode="mixed", profile=1)
    opts_fp64 = meb.options(mode="fp64", profile=1)
    import ctypes  # noqa: E402
    nb = ctypes.c_size_t()
    meb._check(meb.lib.meb_workspace_size(m, d, meb.MEB_F64, ctypes.byref(opts_mixed), ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    for _ in range(a.warmup):
        meb.solve(Cd, Rd, opts=opts_mixed, workspace=ws)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        results.append(meb.solve(Cd, Rd, opts=opts_mixed, workspace=ws))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_mixed = (t1 - t0) * 1e3 / a.steps

    # plain FP64 ripALM on the same instance
    fp64 = []
    nb64 = ctypes.c_size_t()
    meb._check(meb.lib.meb_workspace_size(m, d, meb.MEB_F64, ctypes.byref(opts_fp64), ctypes.byref(nb64)))
    ws64 = ws if nb64.value <= ws.numel() else torch.empty(nb64.value, dtype=torch.uint8, device=dev)
    meb.solve(Cd, Rd, opts=opts_fp64, workspace=ws64)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(a.fp64_steps):
        fp64.append(meb.solve(Cd, Rd, opts=opts_fp64, workspace=ws64))
    torch.cuda.synchronize()
    ms_fp64 = (time.perf_counter() - t2) * 1e3 / max(a.fp64_steps, 1)

    # the same solves without the per-pass timing events (reported beside the
    # timed steps, whose events cost a little launch time each)
    def untimed(mode, n, wsp):
        o = meb.options(mode=mode)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            meb.solve(Cd, Rd, opts=o, workspace=wsp)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / n
    ms_mixed_plain = untimed("mixed", max(a.steps, 1), ws)
    ms_fp64_plain = untimed("fp64", max(a.fp64_steps, 1), ws64)

    r, c, st = results[-1]
    g = golden(a.workload)
    r_ref = g["r_fixed"] if g else None
    reach = np.linalg.norm(C - c, axis=1) + (0.0 if R is None else R)
    viol = float(reach.max() - r)

    # roofline of the FP32 evaluation pass over the timed steps
    p_ms = sum(s["pass_ms"][0] for _, _, s in results)
    p_bytes = sum(s["pass_bytes"][0] for _, _, s in results)
    p_launch = sum(s["pass_launches"][0] for _, _, s in results)
    achieved = (p_bytes / 1e9) / (p_ms / 1e3) if p_ms > 0 else 0.0
    f64_ms = sum(s["pass_ms"][1] for _, _, s in fp64)
    f64_bytes = sum(s["pass_bytes"][1] for _, _, s in fp64)

    out = {
        "metric": "time-to-solution at 1e-8 rel. radius (mixed vs FP64); HBM GB/s; p50/p99 latency",
        "value": ms_mixed / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_mixed,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": wl["desc"],
            "mode": "mixed: FP32 screening run to KKT 1e-2, FP64 refinement to KKT 1e-8, full FP64 check",
            "fp64_ripalm_ms": ms_fp64,
            "speedup_mixed_vs_fp64": ms_fp64 / ms_mixed,
            "mixed_ms_without_pass_events": ms_mixed_plain,
            "fp64_ms_without_pass_events": ms_fp64_plain,
            "radius": r,
            "radius_relerr_vs_oracle": (abs(r - r_ref) / r_ref) if r_ref else None,
            "fp64_radius_relerr_vs_oracle": (abs(fp64[-1][0] - r_ref) / r_ref) if (r_ref and fp64) else None,
            "max_violation": viol,
            "kept_for_fp64": st["n_red"],
            "reinsert_rounds": st["reinsert_rounds"],
            "passes": st["passes"],
            "ms_phase": st["ms_phase"],
            "fp64_pass_GBps": (f64_bytes / 1e9) / (f64_ms / 1e3) if f64_ms > 0 else None,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "pass_kernel<float> (FP32 evaluation pass over all m balls)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            # the committed counters cover the default workload only
            "traffic": measured_traffic() if a.workload == "balls_1e6_d100" else None,
            "launches": p_launch,
            "avg_launch_us": (p_ms * 1e3 / p_launch) if p_launch else None,
            "algorithmic_bytes_per_launch": (p_bytes / p_launch) if p_launch else None,
        },
    }
    del ws, ws64, Cd, Rd
    torch.cuda.empty_cache()
    if not a.no_others:
        out["other_workloads"] = other_workloads([n for n in ("points_1e4_d10", "balls_2e5_d1000", "points_1e7_d10")
                                                  if n != a.workload], log)
        out["paper_instances"] = paper_instances(log)
    if a.serve_requests > 0:
        out["serving"] = serving_leg(a.serve_requests, a.serve_load, 5, a.serve_max_active, a.serve_pool_gb,
                                     a.serve_check, log)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(C, R, m, min(a.cpu_sample, m))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
