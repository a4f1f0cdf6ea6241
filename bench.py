"""Throughput of the CPM multigrid V-cycle on one MI355X.

One step = one V(3,3) cycle of the whole hot path (smoothing, residual, restriction,
coarsest solve, prolongation on every level, plus the stopping residual) on the unit
sphere, h = 1/64, 5 levels (424,510 finest band nodes), FP64, with all inputs resident in
HBM.  value = finest-level band DOFs x cycles / second.  Also reported: time to a 1e-10
relative residual from u = 0 in FP64 and mixed precision, the roofline of the dominant
kernel (extension + smoothing pass on the finest level) and the CPU oracle's rate.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

REPO = os.path.dirname(os.path.abspath(__file__))
if REPO not in sys.path:
    sys.path.insert(0, REPO)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cycles", type=int, default=100)
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-tolerance solves")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(cfg, cycles: int):
    """The oracle as it stands (scipy CSR, one BLAS thread) on a bounded sample: `cycles`
    V-cycles of the same hierarchy (setup not timed)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import band as ob
    from oracle import vcycle as ov

    with threadpool_limits(limits=1):
        H = ob.build_hierarchy(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
        f = cfg.problem.f(H.levels[0].cp)
        p = ov.Params(c=cfg.problem.c)
        coarse = ov.CoarseSolver(H, p)
        u = np.zeros(H.levels[0].n)
        t0 = time.perf_counter()
        for _ in range(cycles):
            u = ov.vcycle(H, 0, u, f, p, coarse)
        dt = time.perf_counter() - t0
    n0 = H.levels[0].n
    return {"value": n0 * cycles / dt, "unit": "DOF*V-cycles/s", "cores": 1, "kind": "oracle",
            "sample": "%d V(3,3) cycles of the sphere h=1/64 5-level hierarchy (%d finest DOFs), "
                      "scipy CSR mat-vecs, 1 thread, setup excluded; %.2f s" % (cycles, n0, dt)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the CPM solver runs each problem on a single device "
              "(multi-GPU sharding is a design note, not an implemented path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1307_4354_amd as cpm
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = W.config_sphere(64, 5)
    s = cfg.problem.surface
    t0 = time.perf_counter()
    band = cpm.cpm_build_band(cpm.make_surface(s.kind, s.R, s.r, s.center), cfg.h0, cfg.levels, cfg.lam2)
    t_build = time.perf_counter() - t0
    sizes = band.sizes()
    n0 = sizes[0]
    _, cp = band.export(0)
    fd = torch.as_tensor(cfg.problem.f(cp)).to("cuda")
    p64 = cpm.make_params(c=cfg.problem.c, nu1=cfg.nu1, nu2=cfg.nu2, omega=cfg.omega)
    pmx = cpm.make_params(c=cfg.problem.c, nu1=cfg.nu1, nu2=cfg.nu2, omega=cfg.omega, precision=cpm.CPM_MIXED)
    nb64 = cpm.cpm_workspace_size(band, p64)
    nbmx = cpm.cpm_workspace_size(band, pmx)
    work = torch.empty(max(nb64, nbmx), dtype=torch.uint8, device="cuda")
    t0 = time.perf_counter()
    cpm.cpm_autotune(band)  # per-level launch configurations (setup, like the band build)
    t_tune = time.perf_counter() - t0
    tuning = [cpm.cpm_band_tuning(band, l) for l in range(band.levels)]
    ud = torch.zeros_like(fd)
    hist = torch.zeros(max(args.steps, args.warmup) + 8, dtype=torch.float64, device="cuda")
    per_launch = 10

    def run(p, nb, k):
        cpm.cpm_run_cycles(band, p, fd, ud, work, nb, k, min(per_launch, max(k, 1)), hist)

    # FP64 throughput: warm-up (graph capture, coarse factorization), then exactly K timed cycles
    run(p64, nb64, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(p64, nb64, args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = n0 * args.steps / dt

    # mixed-precision throughput (same cycles, float32 inner / float64 outer)
    ud.zero_()
    run(pmx, nbmx, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(pmx, nbmx, args.steps)
    torch.cuda.synchronize()
    dt_mx = time.perf_counter() - t0

    # time to 1e-10 from u = 0 (graph per cycle, one host check per cycle); first call warms up
    tt = {}
    for name, p, nb in (() if args.no_solve else (("f64", p64, nb64), ("mixed", pmx, nbmx))):
        ud.zero_()
        cpm.cpm_solve(band, p, fd, ud, work, nb, rtol=1e-10, max_cycles=80)
        ud.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = cpm.cpm_solve(band, p, fd, ud, work, nb, rtol=1e-10, max_cycles=80)
        torch.cuda.synchronize()
        tt[name] = {"seconds": time.perf_counter() - t0, "cycles": st.cycles, "relres": st.relres}

    # dominant kernel: finest-level extension + smoothing pass, timed with HIP events on the
    # band's stream.  Algorithmic bytes per node: 3 closest-point fractions (24 B), u read (8),
    # u write (8), one read of g (8) = 48 B (FP64, 3-D).
    ud.zero_()
    avg_us = cpm.cpm_time_kernel(band, p64, 0, 0, args.kernel_reps, fd, ud, work, nb64)
    alg_bytes = 48.0 * n0
    achieved = alg_bytes / (avg_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": ("k_ext_lds" if tuning[0][0] else "k_ext") + "<3,double,EXT_SMOOTH> level 0", "avg_launch_us": round(avg_us, 3),
                "alg_bytes_per_launch": int(alg_bytes)}

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)  # reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        del a, b

    line = {
        "metric": "band DOF*V-cycles/s and time to 1e-10 rel residual: FP64 vs mixed/learned",
        "value": value,
        "unit": "DOF*V-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (unit sphere, u = (x^2 - y^2) z, f = 13 u, sampled at closest points)",
        "config": {"workload": "sphere_h1/64_5levels_V(3,3)_omega2/3_fp64", "n_per_level": sizes,
                   "levels": cfg.levels, "band_radius": "sqrt(17) h", "c": cfg.problem.c},
        "mixed": {"value": n0 * args.steps / dt_mx, "ms_per_step": 1000.0 * dt_mx / args.steps, "dtype": "f32+f64"},
        "time_to_1e-10": tt,
        "band_build_s": t_build,
        "autotune_s": t_tune,
        "tuning": [{"level": l, "lds": t[0], "ext_block": t[1], "nsum_block": t[2]} for l, t in enumerate(tuning)],
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_cycles)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
