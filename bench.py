"""Throughput of the CPM multigrid V-cycle on one MI355X.

One step = one V(3,3) cycle of the whole hot path (smoothing, residual, restriction,
coarsest solve, prolongation on every level, plus the stopping residual) on the torus
R = 1, r = 0.4 at h = 1/256 (6 levels down to h = 1/8, 8,531,440 finest band nodes, a
seeded 16-mode right-hand side), FP64, with all inputs resident in HBM.
value = finest-level band DOFs x cycles / second.  Also reported: the same cycles in mixed
precision (float32 inner cycles, float64 outer refinement), time to a 1e-10 relative
residual from u = 0 (FP64, mixed, FP64 with the full-multigrid start, W-cycles), the
mixed solution's error against the float64 oracle at h = 1/64, the roofline of the
dominant kernel (the finest level's smoothing pass) and the CPU oracle's rate.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload torus256|sphere64|...]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

REPO = os.path.dirname(os.path.abspath(__file__))
if REPO not in sys.path:
    sys.path.insert(0, REPO)

HBM_PEAK_GBS = 8000.0
PER_LAUNCH = 10  # cycles per captured graph launch in the throughput runs


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cycles", type=int, default=100)
    ap.add_argument("--kernel-reps", type=int, default=100)
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-tolerance solves")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the oracle comparison at h = 1/64 and the secondary surfaces")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--workload", default="torus256",
                    choices=["torus256", "sphere64", "batched256", "learned", "torus512"],
                    help="torus256 (default, the headline line); the others are secondary measurements")
    ap.add_argument("--nprob", type=int, default=256, help="batched256: number of problems")
    ap.add_argument("--train-steps", type=int, default=3000, help="learned: Adam steps")
    return ap.parse_args()


def _build(cpm, prob, h0, levels, lam2=0.0):
    s = prob.surface
    return cpm.cpm_build_band(cpm.make_surface(s.kind, s.R, s.r, s.center), h0, levels, lam2)


def _solve(cpm, torch, band, p, fd, rtol=1e-10, max_cycles=120, repeat=True):
    """Time to rtol from u = 0 (the first call warms graphs and the coarse factorization)."""
    nb = cpm.cpm_workspace_size(band, p)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    ud = torch.zeros_like(fd)
    if repeat:
        cpm.cpm_solve(band, p, fd, ud, work, nb, rtol=rtol, max_cycles=max_cycles, raise_on_noconv=False)
        ud.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = cpm.cpm_solve(band, p, fd, ud, work, nb, rtol=rtol, max_cycles=max_cycles, raise_on_noconv=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h = st.history()
    rho = (h[-1] / h[1]) ** (1.0 / (len(h) - 2)) if len(h) > 3 else float("nan")
    worst = max((h[k + 1] / h[k] for k in range(1, len(h) - 1)), default=float("nan"))
    return ud, {"seconds": dt, "cycles": st.cycles, "relres": st.relres, "contraction": rho,
                "worst_cycle_contraction": worst, "fallback_cycle": st.fallback_cycle, "status": st.status}


def _host_info():
    """Cores, CPU model and thread environment of the host that runs the CPU baseline."""
    model = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True,
                             timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    return {"nproc": os.cpu_count(), "cpu_model": model, "thread_env": env}


# Dominant kernel of a level's smoothing pass for a tuning (cpm_band_tuning's fields): (kernel
# name as the profiler prints it, launch grid in work-items, algorithmic bytes per node,
# cpm_time_kernel selector, description).  The extension pass moves 3 closest-point fractions
# (24 B), one read of g (8), u read and write (16): 48 B per node in FP64; the fused one-pass
# sweep moves the fractions, u and E f read, u' written: 56 B; the tiled pass the fractions,
# u and f read, u' written: 48 B.
def _dominant_kernel(tuning, n0, ntiles=0, ext_slots=256):
    use_lds, ext_block, _, fused, sweep_block, sweep_lds, tiled, prefetch = tuning
    if tiled:
        return ("k_tile<double, double, 0>", ntiles * 256, 48.0, 6,
                "tiled Ruuth-Merriman sweep (f + N u in LDS, extension, Jacobi step), level 0")
    if fused:
        name = ("k_sweep_lds" if sweep_lds else "k_sweep") + "<3, double, 0>"
        blk = 256 if sweep_lds else sweep_block
        return name, -(-n0 // blk) * blk, 56.0, 5, "fused one-pass sweep E f + (E N) u (Jacobi step), level 0"
    # the LDS-staged form runs 256 lanes per workgroup over ext_slots stencil slots (a
    # template argument of its kernels)
    if use_lds:
        name = "%s<3, double, double, 0, %d>" % ("k_ext_ldsp" if prefetch else "k_ext_lds", ext_slots // 256)
        grid = -(-n0 // ext_slots) * 256
    else:
        name = "k_ext<3, double, double, 0>"
        grid = -(-n0 // ext_block) * ext_block
    return name, grid, 48.0, 0, "extension + Jacobi smoothing pass, level 0"


def _traffic_file(workload):
    return os.path.join(REPO, "profiles", "traffic_level0_sweep_%s.json" % workload)


def headline_torus256(args):
    """The headline line: FP64 V(3,3) cycles on the torus at h = 1/256, mixed beside it."""
    import numpy as np
    import torch

    import paper_1307_4354_amd as cpm
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = W.config_torus_mixed(256)
    s = cfg.problem.surface
    t0 = time.perf_counter()
    band = cpm.cpm_build_band(cpm.make_surface(s.kind, s.R, s.r, s.center), cfg.h0, cfg.levels, cfg.lam2)
    t_build = time.perf_counter() - t0
    sizes = band.sizes()
    n0 = sizes[0]
    print("band built: %s in %.1f s" % (sizes, t_build), file=sys.stderr, flush=True)
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
    K, Wm = args.steps, max(args.warmup, 1)
    hist = torch.zeros(max(K, Wm) + 8, dtype=torch.float64, device="cuda")

    def run(p, nb, k):
        cpm.cpm_run_cycles(band, p, fd, ud, work, nb, k, PER_LAUNCH, hist)

    def timed(p, nb):
        # warm-up: W cycles, then the timed run's exact launch pattern once, so that every
        # graph it launches (first launch, full launches, remainder) is captured beforehand
        ud.zero_()
        run(p, nb, Wm)
        run(p, nb, K)
        ud.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(p, nb, K)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    dt = timed(p64, nb64)
    dt_mx = timed(pmx, nbmx)
    print("cycles: f64 %.3f ms, mixed %.3f ms" % (1e3 * dt / K, 1e3 * dt_mx / K), file=sys.stderr, flush=True)

    # time to 1e-10 from u = 0 (one graph per cycle, one host check per cycle); the first
    # call of each warms its graphs
    tt, sol = {}, {}
    if not args.no_solve:
        for name, p in (("f64", p64), ("mixed", pmx),
                        ("f64_fmg_start", cpm.make_params(c=cfg.problem.c, fmg=True)),
                        ("mixed_fmg_start", cpm.make_params(c=cfg.problem.c, fmg=True, precision=cpm.CPM_MIXED)),
                        ("f64_W_cycle", cpm.make_params(c=cfg.problem.c, gamma=2))):
            sol[name], tt[name] = _solve(cpm, torch, band, p, fd, max_cycles=80)
        tt["speedup_mixed_over_f64"] = tt["f64"]["seconds"] / tt["mixed"]["seconds"]
        tt["mixed_vs_f64_max_rel_diff"] = float((sol["mixed"] - sol["f64"]).abs().max() / sol["f64"].abs().max())
        _, tt["standard_relaxation_to_increment_1e-10"] = _solve(
            cpm, torch, band, cpm.make_params(c=cfg.problem.c, smoother=cpm.CPM_SMOOTH_STANDARD), fd, max_cycles=80)
        sol.clear()

    # dominant kernel: the finest level's smoothing pass, timed with HIP events on the stream
    # it is launched on
    kname, grid0, bpn, which, what = _dominant_kernel(tuning[0], n0, ext_slots=cpm.cpm_band_ext_slots(band, 0))
    ud.zero_()
    avg_us = cpm.cpm_time_kernel(band, p64, which, 0, args.kernel_reps, fd, ud, work, nb64)
    alg_bytes = bpn * n0
    achieved = alg_bytes / (avg_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": _measured_traffic(_traffic_file("torus256"), kname, grid0),
                "kernel": "%s (%s)" % (kname, what), "grid": grid0, "avg_launch_us": round(avg_us, 3),
                "alg_bytes_per_node": bpn, "alg_bytes_per_launch": int(alg_bytes)}
    if roofline["traffic"]:
        # the counter-measured bytes over the same live launch time, beside the algorithmic rate
        tr = roofline["traffic"] / (avg_us * 1e-6) / 1e9
        roofline["traffic_rate"] = round(tr, 1)
        roofline["traffic_frac"] = round(tr / HBM_PEAK_GBS, 4)
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)  # reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        del a, b
    del work, hist
    band.free()

    line = {
        "metric": "band DOF*V-cycles/s and time to 1e-10 rel residual: FP64 vs mixed/learned",
        "value": n0 * K / dt,
        "unit": "DOF*V-cycles/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * dt / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (torus R=1, r=0.4; f = seeded mix of 16 torus Fourier modes, sampled at closest points)",
        "config": {"workload": "torus_R1_r0.4_h1/256_6levels_V(3,3)_omega2/3_fp64", "n_per_level": sizes,
                   "levels": cfg.levels, "band_radius": "sqrt(17) h", "c": cfg.problem.c,
                   "cycles_per_graph_launch": PER_LAUNCH},
        "mixed": {"value": n0 * K / dt_mx, "ms_per_step": 1000.0 * dt_mx / K, "dtype": "f32+f64",
                  "speedup_over_f64": dt / dt_mx},
        "time_to_1e-10": tt,
        "band_build_s": t_build,
        "autotune_s": t_tune,
        "tuning": [{"level": l, "lds": t[0], "ext_block": t[1], "nsum_block": t[2], "fused_sweep": t[3],
                    "sweep_block": t[4], "sweep_lds": t[5], "tiled": t[6], "ext_prefetch": t[7]}
                   for l, t in enumerate(tuning)],
        "roofline": roofline,
    }
    if not args.no_extras:
        o64 = oracle_at_64(args, cpm, torch)
        if "cpu_baseline" in o64:
            line["cpu_baseline"] = o64.pop("cpu_baseline")
        line["h1/64_oracle"] = o64
        line["extras"] = secondary_surfaces(cpm, torch)
    print(json.dumps(line), flush=True)


def oracle_at_64(args, cpm, torch):
    """The same torus and right-hand side at h = 1/64 (4 levels, 531,968 nodes): the GPU's
    mixed and FP64 solutions against the float64 oracle's, and the oracle's own V-cycle rate
    on one core (the CPU baseline)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import band as ob
    from oracle import vcycle as ov

    c64 = W.config_torus_mixed(64)
    t0 = time.perf_counter()
    H = ob.build_hierarchy(c64.problem.surface, c64.h0, c64.levels, c64.lam2)
    f = c64.problem.f(H.levels[0].cp)
    ref = ov.solve(H, f, ov.Params(c=c64.problem.c), rtol=1e-10, max_cycles=80)
    print("oracle at h=1/64: %d cycles in %.1f s" % (ref.cycles, time.perf_counter() - t0), file=sys.stderr,
          flush=True)
    band = _build(cpm, c64.problem, c64.h0, c64.levels, c64.lam2)
    fd = torch.as_tensor(f).to("cuda")
    out = {"workload": "torus_R1_r0.4_h1/64_4levels", "n": H.levels[0].n, "oracle_cycles": ref.cycles}
    for name, p in (("mixed", cpm.make_params(precision=cpm.CPM_MIXED)), ("f64", cpm.make_params())):
        ug, st = _solve(cpm, torch, band, p, fd, repeat=False)
        out[name] = {"gpu_cycles": st["cycles"], "relres": st["relres"],
                     "max_rel_diff_vs_fp64_oracle": float(np.max(np.abs(ug.cpu().numpy() - ref.u)) /
                                                          np.max(np.abs(ref.u)))}
    band.free()
    if not args.no_cpu_baseline:
        with threadpool_limits(limits=1):
            p = ov.Params(c=c64.problem.c)
            coarse = ov.CoarseSolver(H, p)
            u = np.zeros(H.levels[0].n)
            t0 = time.perf_counter()
            for _ in range(args.cpu_cycles):
                u = ov.vcycle(H, 0, u, f, p, coarse)
            dt = time.perf_counter() - t0
        n0 = H.levels[0].n
        out["cpu_baseline"] = {
            "value": n0 * args.cpu_cycles / dt, "unit": "DOF*V-cycles/s", "cores": 1, "kind": "oracle",
            "sample": "%d V(3,3) cycles of the same torus and right-hand side at h = 1/64 (4 levels, %d finest "
                      "DOFs; the oracle's cost per cycle is proportional to the DOFs), scipy CSR mat-vecs, 1 thread, "
                      "setup excluded; %.2f s" % (args.cpu_cycles, n0, dt),
            **_host_info()}
    return out


def secondary_surfaces(cpm, torch):
    """The variable-coefficient sphere example and Dziuk's level-set surface at h = 1/64."""
    import workloads as W

    out = {}
    pv = W.sphere_varcoef()
    cfg = W.config_sphere(64, 5)
    band = _build(cpm, pv, cfg.h0, cfg.levels, cfg.lam2)
    for l in range(band.levels):
        _, cpl = band.export(l)
        cpm.cpm_set_diffusion(band, l, pv.a(cpl))
    _, cp = band.export(0)
    u, r = _solve(cpm, torch, band, cpm.make_params(c=pv.c), torch.as_tensor(pv.f(cp)).to("cuda"))
    out["variable_coefficient_sphere_h1/64"] = {
        "seconds_to_1e-10": r["seconds"], "cycles": r["cycles"], "relres": r["relres"],
        "max_error_vs_exact": float(abs(u.cpu().numpy() - pv.u_exact(cp)).max())}
    band.free()
    pl = W.dziuk_x1x2()
    t0 = time.perf_counter()
    bl = _build(cpm, pl, 1.0 / 64, 4)
    t_bl = time.perf_counter() - t0
    _, cpl = bl.export(0)
    ul, rl = _solve(cpm, torch, bl, cpm.make_params(c=pl.c), torch.as_tensor(pl.f(cpl)).to("cuda"))
    out["levelset_dziuk_h1/64"] = {"n_per_level": bl.sizes(), "band_build_s": t_bl,
                                   "seconds_to_1e-10": rl["seconds"], "cycles": rl["cycles"],
                                   "contraction": rl["contraction"],
                                   "max_error_vs_exact": float(abs(ul.cpu().numpy() - pl.u_exact(cpl)).max())}
    bl.free()
    return out


def run_batched256(args):
    """256 uneven problems in one batched solve (float32 inner, float64 outer), against
    unbatched solves of a sample of them."""
    import torch

    import paper_1307_4354_amd as cpm
    import workloads as W

    items = W.batch_problems(args.nprob)
    t0 = time.perf_counter()
    # all bands at once on the host's cores (one band per thread)
    surfs = [cpm.make_surface(it.problem.surface.kind, it.problem.surface.R, it.problem.surface.r,
                              it.problem.surface.center) for it in items]
    bands = cpm.cpm_build_bands(surfs, [(it.h0, it.levels, it.lam2) for it in items])
    t_build = time.perf_counter() - t0
    print("built %d bands in %.1f s" % (len(bands), t_build), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    fs = []
    for it, b in zip(items, bands):
        _, cp = b.export(0)
        fs.append(torch.as_tensor(it.problem.f(cp)).to("cuda"))
    t_rhs = time.perf_counter() - t0
    sizes = [b.n(0) for b in bands]
    p = cpm.make_params(precision=cpm.CPM_MIXED)
    nbytes = cpm.cpm_workspace_size_batched(bands, p)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    us = [torch.zeros_like(f) for f in fs]
    cpm.cpm_solve_batched(bands, p, fs, us, work, nbytes, rtol=1e-10, max_cycles=120, raise_on_noconv=False)
    for u in us:
        u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, stats = cpm.cpm_solve_batched(bands, p, fs, us, work, nbytes, rtol=1e-10, max_cycles=120,
                                          raise_on_noconv=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dof_cycles = sum(n * st.cycles for n, st in zip(sizes, stats))
    # unbatched reference on a sample: same cycles, same iterate, time
    sample = list(range(0, len(bands), max(1, len(bands) // 8)))[:8]
    # (the unbatched solves may sweep small levels with the fused pass, which rounds
    # differently from the batched two-pass sweep: compare cycles and the iterate's difference)
    seq_t, same_cycles, max_diff = 0.0, True, 0.0
    for k in sample:
        u1, r = _solve(cpm, torch, bands[k], p, fs[k])
        seq_t += r["seconds"]
        same_cycles &= r["cycles"] == stats[k].cycles
        max_diff = max(max_diff, float((u1 - us[k]).abs().max() / us[k].abs().max()))
    sample_n = sum(sizes[k] * stats[k].cycles for k in sample)
    print(json.dumps({"metric": "batched band DOF*V-cycles/s (mixed precision, 1e-10)", "nprob": len(bands),
                      "status": status, "total_finest_dofs": sum(sizes), "min_n": min(sizes), "max_n": max(sizes),
                      "seconds": dt, "dof_cycles_per_s": dof_cycles / dt,
                      "cycles_min": min(s.cycles for s in stats), "cycles_max": max(s.cycles for s in stats),
                      "max_relres": max(s.relres for s in stats), "tile_block": stats[0].tile_block,
                      "tile_blocks_per_cu": stats[0].tile_blocks_per_cu, "band_build_s": t_build,
                      "rhs_export_and_eval_s": t_rhs, "cycles_per_graph_launch": stats[0].cycles_per_launch, "host_syncs": stats[0].host_syncs,
                      "unbatched_sample": {"problems": sample, "seconds": seq_t,
                                           "dof_cycles_per_s": sample_n / seq_t, "same_cycles_as_batched": same_cycles,
                                           "max_rel_diff_to_batched": max_diff}}),
          flush=True)


def run_learned(args):
    """Train the learned smoother on pairs from plain V-cycles (random spheres and tori), then
    compare learned vs plain FP64 solves on the unit sphere and the torus at h = 1/256."""
    import numpy as np
    import torch

    import paper_1307_4354_amd as cpm
    import workloads as W
    from paper_1307_4354_amd import learned

    rng = np.random.default_rng(W.SEED_BASE + 5)
    probs = []
    for k in range(4):
        if k % 2 == 0:
            probs.append((W.sphere_modes(float(rng.uniform(0.7, 1.3)), int(rng.integers(1 << 30))), 1 / 64, 5))
        else:
            probs.append((W.torus_modes(float(rng.uniform(0.8, 1.2)), float(rng.uniform(0.3, 0.45)),
                                        int(rng.integers(1 << 30))), 1 / 64, 4))
    t0 = time.perf_counter()
    pairs = learned.generate_pairs(probs, cycles=4)
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = learned.train(pairs, steps=args.train_steps, batch=65536, lr=1e-3, log_every=250)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    w_jac = learned._bf16_bits(learned.jacobi_init(2.0 / 3.0, 3, 0))
    out = {"metric": "learned smoother vs plain FP64 V-cycle, time to 1e-10", "pairs": int(pairs.X.shape[0]),
           "data_s": t_data, "train_s": t_train, "train_steps": args.train_steps, "loss_history": res.losses,
           "loss_jacobi_init": learned.evaluate_loss(pairs, w_jac), "loss_trained": learned.evaluate_loss(pairs, res.w_bits)}
    evals = {"sphere_h1/256_7levels": (W.sphere_l3(), 1 / 256, 7),
             "torus_R1_r0.4_h1/256_6levels": (W.config_torus_mixed(256).problem, 1 / 256, 6)}
    for name, (prob, h0, levels) in evals.items():
        band = _build(cpm, prob, h0, levels)
        cpm.cpm_autotune(band)
        _, cp = band.export(0)
        fd = torch.as_tensor(prob.f(cp)).to("cuda")
        _, plain = _solve(cpm, torch, band, cpm.make_params(), fd)
        res_e = {"n": band.n(0), "plain_f64_V33": plain}
        # the undamped plain cycle, the step the network is trained to reproduce
        _, res_e["plain_f64_V33_omega1_for_reference"] = _solve(cpm, torch, band, cpm.make_params(omega=1.0), fd)
        # fall back to Jacobi when a cycle contracts worse than plain V(3,3) ever did
        cpm.cpm_set_smoother_weights(band, res.w_bits, plain["worst_cycle_contraction"])
        p0 = cpm.make_params()
        nb = cpm.cpm_workspace_size(band, p0)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        ut = torch.zeros_like(fd)
        res_e["level0_us"] = {"jacobi_ext_smooth": cpm.cpm_time_kernel(band, p0, 0, 0, 50, fd, ut, work, nb),
                              "learned_update": cpm.cpm_time_kernel(band, p0, 4, 0, 50, fd, ut, work, nb),
                              "neighbour_sum": cpm.cpm_time_kernel(band, p0, 1, 0, 50, fd, ut, work, nb)}
        del work, ut
        for k in (0, 1, 2):
            _, lk = _solve(cpm, torch, band, cpm.make_params(smoother=cpm.CPM_SMOOTH_LEARNED, learned_sweeps=k), fd)
            tag = "learned_V33" if k == 0 else "learned_%d_sweeps" % k
            res_e[tag] = lk
            res_e["speedup_%s_over_plain_V33" % tag] = plain["seconds"] / lk["seconds"]
        out[name] = res_e
        band.free()
    print(json.dumps(out), flush=True)


def _measured_traffic(path: str, kernel: str, grid: int):
    """HBM bytes per launch of the dominant kernel from a committed FETCH_SIZE / WRITE_SIZE
    summary, or None when there is none, it is for another kernel or launch shape, or the
    kernel's sources have changed since the counters were taken."""
    from paper_1307_4354_amd import prof_summary

    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel") != kernel or t.get("grid") != grid:
        return None
    if t.get("source_sha256") != prof_summary.sources_sha256(t.get("sources", [])):
        return None
    return int(round(t["traffic_bytes"]))


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
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    {"torus256": headline_torus256, "sphere64": run_sphere64, "batched256": run_batched256,
     "learned": run_learned, "torus512": run_torus512}[args.workload](args)


def run_torus512(args):
    """The headline torus one refinement further (h = 1/512, 7 levels, 34 million finest
    nodes): FP64 and mixed cycle rates, times to 1e-10 from u = 0, and the band's device
    memory (the band's arrays go through torch's caching allocator for the count)."""
    import torch

    import paper_1307_4354_amd as cpm
    import workloads as W

    cfg = W.config_torus_mixed(512)
    s = cfg.problem.surface
    cpm.use_torch_allocator(True)
    m0 = torch.cuda.memory_allocated()
    t0 = time.perf_counter()
    band = cpm.cpm_build_band(cpm.make_surface(s.kind, s.R, s.r, s.center), cfg.h0, cfg.levels, cfg.lam2)
    t_build = time.perf_counter() - t0
    band_bytes = torch.cuda.memory_allocated() - m0
    sizes = band.sizes()
    _, cp = band.export(0)
    fd = torch.as_tensor(cfg.problem.f(cp)).to("cuda")
    t0 = time.perf_counter()
    cpm.cpm_autotune(band)
    t_tune = time.perf_counter() - t0
    out = {"metric": "band DOF*V-cycles/s, torus h=1/512 (secondary workload)", "unit": "DOF*V-cycles/s",
           "n_per_level": sizes, "band_build_s": t_build, "autotune_s": t_tune,
           "band_device_bytes": int(band_bytes)}
    for name, prec in (("f64", cpm.CPM_F64), ("mixed", cpm.CPM_MIXED)):
        p = cpm.make_params(c=cfg.problem.c, nu1=cfg.nu1, nu2=cfg.nu2, omega=cfg.omega, precision=prec)
        nb = cpm.cpm_workspace_size(band, p)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        ud = torch.zeros_like(fd)
        hist = torch.zeros(2 * PER_LAUNCH + 8, dtype=torch.float64, device="cuda")
        for _ in range(2):  # both graphs of the timed run captured
            cpm.cpm_run_cycles(band, p, fd, ud, work, nb, 2 * PER_LAUNCH, PER_LAUNCH, hist)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cpm.cpm_run_cycles(band, p, fd, ud, work, nb, 2 * PER_LAUNCH, PER_LAUNCH, hist)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / (2 * PER_LAUNCH)
        del work
        _, sol = _solve(cpm, torch, band, p, fd, max_cycles=100)
        out[name] = {"value": sizes[0] / dt, "ms_per_cycle": dt * 1e3, "time_to_1e-10": sol,
                     "workspace_bytes": int(nb)}
    band.free()
    print(json.dumps(out), flush=True)


def run_sphere64(args):
    """The unit sphere at h = 1/64 (5 levels, 424,510 nodes): cycle rates, time to 1e-10 and
    the standard relaxation on a level set whose working set fits the 256 MB last-level cache."""
    import numpy as np
    import torch

    import paper_1307_4354_amd as cpm
    import workloads as W

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
    def run(p, nb, k):
        cpm.cpm_run_cycles(band, p, fd, ud, work, nb, k, PER_LAUNCH, hist)

    # FP64 throughput: warm-up (graph capture, coarse factorization), then exactly K timed cycles
    run(p64, nb64, max(args.warmup, 1))
    run(p64, nb64, args.steps)  # the timed run's launch pattern, so its graphs are captured
    ud.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(p64, nb64, args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = n0 * args.steps / dt

    # mixed-precision throughput (same cycles, float32 inner / float64 outer)
    ud.zero_()
    run(pmx, nbmx, max(args.warmup, 1))
    run(pmx, nbmx, args.steps)
    ud.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(pmx, nbmx, args.steps)
    torch.cuda.synchronize()
    dt_mx = time.perf_counter() - t0

    # time to 1e-10 from u = 0 (graph per cycle, one host check per cycle); first call warms up
    tt = {}
    p_fmg = cpm.make_params(c=cfg.problem.c, nu1=cfg.nu1, nu2=cfg.nu2, omega=cfg.omega, fmg=True)
    p_w = cpm.make_params(c=cfg.problem.c, nu1=cfg.nu1, nu2=cfg.nu2, omega=cfg.omega, gamma=2)
    for name, p, nb in (() if args.no_solve else (("f64", p64, nb64), ("mixed", pmx, nbmx),
                                                  ("f64_fmg_start", p_fmg, nb64), ("f64_W_cycle", p_w, nb64))):
        ud.zero_()
        cpm.cpm_solve(band, p, fd, ud, work, nb, rtol=1e-10, max_cycles=80)
        ud.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = cpm.cpm_solve(band, p, fd, ud, work, nb, rtol=1e-10, max_cycles=80)
        torch.cuda.synchronize()
        tt[name] = {"seconds": time.perf_counter() - t0, "cycles": st.cycles, "relres": st.relres}

    # the standard-relaxation cycle (Jacobi on A, residual f - A(E u)): time until the
    # relative increment drops below 1e-10 (the paper's stopping test for it)
    std_res = None
    if not args.no_solve:
        pst = cpm.make_params(c=cfg.problem.c, nu1=cfg.nu1, nu2=cfg.nu2, omega=cfg.omega,
                              smoother=cpm.CPM_SMOOTH_STANDARD)
        ud.zero_()
        cpm.cpm_solve(band, pst, fd, ud, work, nb64, rtol=1e-10, max_cycles=80, raise_on_noconv=False)
        ud.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = cpm.cpm_solve(band, pst, fd, ud, work, nb64, rtol=1e-10, max_cycles=80, raise_on_noconv=False)
        torch.cuda.synchronize()
        std_res = {"seconds": time.perf_counter() - t0, "cycles": st.cycles, "final_increment": st.relres,
                   "status": st.status}

    # dominant kernel: the finest level's smoothing pass, timed with HIP events on the stream it
    # runs on
    kname, grid0, bpn, which, _ = _dominant_kernel(tuning[0], n0, ext_slots=cpm.cpm_band_ext_slots(band, 0))
    ud.zero_()
    avg_us = cpm.cpm_time_kernel(band, p64, which, 0, args.kernel_reps, fd, ud, work, nb64)
    alg_bytes = bpn * n0
    achieved = alg_bytes / (avg_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": _measured_traffic(_traffic_file("sphere64"), kname, grid0),
                "kernel": kname + " (extension + Jacobi smoothing, level 0)", "grid": grid0,
                "avg_launch_us": round(avg_us, 3), "alg_bytes_per_launch": int(alg_bytes)}

    # variable diffusion coefficient (the paper's sphere example a = cos(phi) + 1.5) on the
    # same band: cycle time, and time to 1e-10 from u = 0
    vc_res = None
    if not args.no_solve:
        pv = W.sphere_varcoef()
        for l in range(band.levels):
            _, cpl = band.export(l)
            cpm.cpm_set_diffusion(band, l, pv.a(cpl))
        fv = torch.as_tensor(pv.f(cp)).to("cuda")
        pvc = cpm.make_params(c=pv.c, nu1=cfg.nu1, nu2=cfg.nu2, omega=cfg.omega)
        ud.zero_()
        cpm.cpm_solve(band, pvc, fv, ud, work, nb64, rtol=1e-10, max_cycles=80)
        ud.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = cpm.cpm_solve(band, pvc, fv, ud, work, nb64, rtol=1e-10, max_cycles=80)
        torch.cuda.synchronize()
        t_vc = time.perf_counter() - t0
        err = float((ud.cpu().numpy() - pv.u_exact(cp)).__abs__().max())
        hist_vc = torch.zeros(64, dtype=torch.float64, device="cuda")  # >= the 50 cycles recorded
        cpm.cpm_run_cycles(band, pvc, fv, ud, work, nb64, 10, 10, hist_vc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cpm.cpm_run_cycles(band, pvc, fv, ud, work, nb64, 50, 10, hist_vc)
        torch.cuda.synchronize()
        vc_res = {"seconds_to_1e-10": t_vc, "cycles": st.cycles, "relres": st.relres,
                  "ms_per_cycle": 1000.0 * (time.perf_counter() - t0) / 50, "max_error_vs_exact": err}
        cpm.cpm_set_diffusion(band, 0, None)

    # level-set surface (Dziuk's surface, Newton closest points): band build and solve
    ls_res = None
    if not args.no_solve:
        pl = W.dziuk_x1x2()
        t0 = time.perf_counter()
        bl = _build(cpm, pl, 1.0 / 64, 4)
        t_bl = time.perf_counter() - t0
        _, cpl = bl.export(0)
        fl = torch.as_tensor(pl.f(cpl)).to("cuda")
        ul, rl = _solve(cpm, torch, bl, cpm.make_params(c=pl.c), fl)
        ls_res = {"workload": "dziuk_h1/64_4levels", "n_per_level": bl.sizes(), "band_build_s": t_bl,
                  "seconds_to_1e-10": rl["seconds"], "cycles": rl["cycles"], "contraction": rl["contraction"],
                  "max_error_vs_exact": float((ul.cpu().numpy() - pl.u_exact(cpl)).__abs__().max())}
        bl.free()

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)  # reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        del a, b

    line = {
        "metric": "band DOF*V-cycles/s, sphere h=1/64 (secondary workload)",
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
        "standard_relaxation_to_increment_1e-10": std_res,
        "variable_coefficient_sphere": vc_res,
        "levelset_surface": ls_res,
        "band_build_s": t_build,
        "autotune_s": t_tune,
        "tuning": [{"level": l, "lds": t[0], "ext_block": t[1], "nsum_block": t[2], "fused_sweep": t[3],
                    "sweep_block": t[4], "sweep_lds": t[5], "tiled": t[6], "ext_prefetch": t[7]}
                   for l, t in enumerate(tuning)],
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_cycles)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
