"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

* band and stencil index construction: bit-exact (indices, closest points)
* operator application and extension: within 1e-13 relative (FP64 rounding order only)
* V-cycle iterates: within 1e-12 relative, cycle for cycle
* mixed precision: same cycle count as the float32/float64 oracle, final iterate within
  1e-9 of the double-precision fixed point
"""
import numpy as np
import pytest

import workloads as W
from oracle import band as ob
from oracle import vcycle as ov
from oracle.mixed import solve_mixed
from tests.gpu_util import (build_gpu, dev, host, log, oracle_for, rel_inf, torch_cuda, workspace)

pytestmark = pytest.mark.gpu

BAND_CASES = [
    ("circle64", W.config_circle(64, 4)),
    ("sphere64", W.config_sphere(64, 5)),
    ("torus64", W.SolverConfig("torus64", W.torus_modes(1.0, 0.4, 7), 1 / 64, 4, W.LAM2_3D)),
    ("torus_paper16", W.SolverConfig("tp16", W.torus_paper(), 1 / 16, 3, W.LAM2_3D)),
    ("sphere_off", W.SolverConfig("so", W.sphere_modes(0.7, 3, center=(0.1, -0.2, 0.05)), 1 / 32, 3, W.LAM2_3D)),
]


@pytest.mark.parametrize("name,cfg", BAND_CASES, ids=[c[0] for c in BAND_CASES])
def test_band_construction_bitexact(name, cfg):
    log("band bit-exact: %s" % name)
    H = oracle_for(cfg)
    s = cfg.problem.surface
    band = build_gpu(s, cfg.h0, cfg.levels, cfg.lam2)
    assert band.levels == cfg.levels and band.dim == s.dim
    for l, lev in enumerate(H.levels):
        idx, cp = band.export(l)
        assert idx.shape == lev.idx.shape
        assert np.array_equal(idx.astype(np.int64), lev.idx), "band nodes differ on level %d" % l
        assert np.array_equal(cp, lev.cp), "closest points differ on level %d" % l
        runE, nbr, runP, runR = band.export_stencils(l)
        assert np.array_equal(runE, H.E[l].indices.reshape(lev.n, -1)[:, ::4])
        # Laplacian neighbours are kept for B_interp (the nodes E reads); other rows read -2
        interp = np.zeros(lev.n, bool)
        interp[np.unique(H.E[l].indices)] = True
        assert np.array_equal(nbr[interp], ob.neighbour_indices(lev)[interp])
        assert np.all(nbr[~interp] == -2)
        if l + 1 < cfg.levels:
            assert np.array_equal(runP, H.P[l].indices.reshape(lev.n, -1)[:, ::2])
        if l > 0:
            assert np.array_equal(runR, H.R[l - 1].indices.reshape(lev.n, -1)[:, ::2])


@pytest.mark.parametrize("name,cfg", BAND_CASES[:3], ids=[c[0] for c in BAND_CASES[:3]])
def test_apply_and_extend_parity(name, cfg):
    log("apply/extend parity: %s" % name)
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    c = 1.3
    for l, lev in enumerate(H.levels):
        u = W.random_vector(lev.n, 100 + l)
        ud = dev(u)
        out = torch.empty_like(ud)
        work = torch.empty_like(ud)
        cpm.cpm_apply(band, l, c, ud, out, work)
        delta = c + 2.0 * lev.dim / lev.h ** 2
        ref = delta * u - H.E[l] @ (H.N[l] @ u)
        assert rel_inf(host(out), ref) < 1e-13, (l, rel_inf(host(out), ref))
        cpm.cpm_extend(band, l, ud, out)
        assert rel_inf(host(out), H.E[l] @ u) < 1e-14
        # A 1 = c 1 (rows of M sum to zero)
        one = torch.ones_like(ud)
        cpm.cpm_apply(band, l, c, one, out, work)
        assert np.max(np.abs(host(out) - c)) < 1e-9 * delta


def _gpu_iterates(cfg, ncycles, params=None, check_sweep=None):
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    if check_sweep is not None:
        tun = [cpm.cpm_band_tuning(band, l) for l in range(band.levels - 1)]
        fused, tiled = [t[3] for t in tun], [t[6] for t in tun]
        assert all(fused) if check_sweep == "fused" else not any(fused), fused
        assert all(tiled) if check_sweep == "tile" else not any(tiled), tiled
    p = params or cpm.make_params(c=cfg.problem.c, nu1=cfg.nu1, nu2=cfg.nu2, omega=cfg.omega)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    its, rels = [], []
    for _ in range(ncycles):
        rels.append(cpm.cpm_vcycle(band, p, fd, ud, work, nbytes, want_relres=True))
        its.append(host(ud).copy())
    return H, f, its, rels


@pytest.mark.parametrize("name,cfg,ncyc", [
    ("circle64", W.config_circle(64, 4), 13),
    ("sphere32", W.config_sphere(32, 4), 23),
    ("sphere64_first4", W.config_sphere(64, 5), 4),
    ("torus32", W.SolverConfig("t32", W.torus_modes(1.0, 0.4, 7), 1 / 32, 3, W.LAM2_3D), 20),
], ids=["circle64", "sphere32", "sphere64_first4", "torus32"])
@pytest.mark.parametrize("sweep", ["split", "fused", "tile"])
def test_vcycle_iterates_match_oracle(name, cfg, ncyc, sweep, monkeypatch):
    """Every sweep form (neighbour sum + extension passes, the fused E f + (E N) u pass, the
    tiled pass that forms f + N u in LDS; pinned with CPM_SWEEP when the band is built, tiles
    built on every 3-D level) gives the oracle's iterates."""
    if sweep == "tile" and cfg.problem.surface.dim == 2:
        pytest.skip("the tiled pass is 3-D only")
    log("V-cycle iterate parity: %s (%d cycles, %s sweeps)" % (name, ncyc, sweep))
    monkeypatch.setenv("CPM_SWEEP", sweep)
    monkeypatch.setenv("CPM_TILE_MIN_NODES", "1000")
    H, f, its, rels = _gpu_iterates(cfg, ncyc, check_sweep=sweep)
    ref = ov.solve(H, f, ov.Params(c=cfg.problem.c), rtol=0.0, max_cycles=ncyc, keep_iterates=True)
    for k in range(ncyc):
        err = rel_inf(its[k], ref.iterates[k])
        assert err < 1e-12, (k, err)
        assert abs(rels[k] - ref.relres[k]) <= 1e-3 * ref.relres[k] + 1e-14, (k, rels[k], ref.relres[k])


@pytest.mark.parametrize("name,cfg", [
    ("circle64", W.config_circle(64, 4)),
    ("sphere32", W.config_sphere(32, 4)),
    ("torus_paper16", W.SolverConfig("tp16", W.torus_paper(), 1 / 16, 3, W.LAM2_3D)),
], ids=["circle64", "sphere32", "torus_paper16"])
def test_solve_matches_oracle(name, cfg):
    log("solve parity: %s" % name)
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ref = ov.solve(H, f, ov.Params(c=cfg.problem.c), rtol=1e-10, max_cycles=60)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(c=cfg.problem.c)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
    assert st.cycles == ref.cycles
    assert st.relres < 1e-10
    assert rel_inf(host(ud), ref.u) < 1e-12
    assert np.allclose(st.history(), ref.relres, rtol=1e-3, atol=1e-14)


@pytest.mark.parametrize("name,cfg", [
    ("circle64", W.config_circle(64, 4)),
    ("torus32", W.config_torus_mixed(32, 3)),
], ids=["circle64", "torus32"])
@pytest.mark.parametrize("sweep", ["split", "fused", "tile"])
def test_mixed_precision_matches_oracle(name, cfg, sweep, monkeypatch):
    if sweep == "tile" and cfg.problem.surface.dim == 2:
        pytest.skip("the tiled pass is 3-D only")
    log("mixed precision parity: %s (%s sweeps)" % (name, sweep))
    import paper_1307_4354_amd as cpm

    monkeypatch.setenv("CPM_SWEEP", sweep)
    monkeypatch.setenv("CPM_TILE_MIN_NODES", "1000")
    torch = torch_cuda()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ref64 = ov.solve(H, f, ov.Params(c=cfg.problem.c), rtol=1e-10, max_cycles=60)
    ref32 = solve_mixed(H, f, ov.Params(c=cfg.problem.c), rtol=1e-10, max_cycles=60)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(c=cfg.problem.c, precision=cpm.CPM_MIXED)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
    assert st.relres < 1e-10
    assert abs(st.cycles - ref32.cycles) <= 1
    # float32 inner arithmetic: per-cycle residuals agree to float32-level relative accuracy
    hist = st.history()
    for k in range(min(len(hist), len(ref32.relres)) - 1):
        assert abs(hist[k] - ref32.relres[k]) <= 1e-2 * ref32.relres[k], (k, hist[k], ref32.relres[k])
    assert rel_inf(host(ud), ref64.u) < 1e-9


@pytest.mark.parametrize("sweep", ["split", "fused", "tile"])
def test_graph_replays_match_eager_cycles(sweep, monkeypatch):
    """cpm_run_cycles (captured graph, replayed) gives the same iterates as eager cycles, bit
    for bit, also where its later cycles start from the residual the previous cycle left."""
    import paper_1307_4354_amd as cpm

    monkeypatch.setenv("CPM_SWEEP", sweep)
    monkeypatch.setenv("CPM_TILE_MIN_NODES", "1000")
    torch = torch_cuda()
    cfg = W.config_sphere(32, 4)
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params()
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ua = torch.zeros_like(fd)
    ref = []
    for _ in range(6):
        cpm.cpm_vcycle(band, p, fd, ua, work, nbytes)
        ref.append(host(ua).copy())
    ub = torch.zeros_like(fd)
    hist = torch.zeros(16, dtype=torch.float64, device="cuda")
    for k in range(6):
        cpm.cpm_run_cycles(band, p, fd, ub, work, nbytes, 1, 1, hist)
        torch.cuda.synchronize()
        assert np.array_equal(host(ub), ref[k]), k
        _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work between replays
    ub.zero_()
    cpm.cpm_run_cycles(band, p, fd, ub, work, nbytes, 6, 3, hist)
    assert np.array_equal(host(ub), ref[-1])
    ho = host(hist)
    assert np.all(ho[:6] > 0) and np.all(np.diff(ho[:6]) < 0)


@pytest.mark.parametrize("name,cfg", [
    ("circle128", W.config_circle(128, 5)),
    ("sphere32", W.config_sphere(32, 4)),
    ("torus32", W.config_torus_mixed(32, 3)),
], ids=["circle128", "sphere32", "torus32"])
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_fused_sweep_lds_equals_gathers(name, cfg, precision, monkeypatch):
    """The LDS-staged fused sweep does the gather form's arithmetic term for term: cycles
    with either form on every level give the same iterates, bit for bit."""
    log("fused sweep LDS vs gathers: %s %s" % (name, precision))
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    prec = cpm.CPM_F64 if precision == "f64" else cpm.CPM_MIXED
    out = {}
    fd = None
    for lds in ("1", "0"):
        monkeypatch.setenv("CPM_SWEEP", "fused")
        monkeypatch.setenv("CPM_SWEEP_LDS", lds)
        band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
        if fd is None:
            fd = dev(cfg.problem.f(band.export(0)[1]))
        tun = [cpm.cpm_band_tuning(band, l) for l in range(band.levels - 1)]
        assert all(t[3] for t in tun)
        assert all(t[5] == (lds == "1") for t in tun)
        p = cpm.make_params(c=cfg.problem.c, precision=prec)
        work, nbytes = workspace(band, p)
        ud = torch.zeros_like(fd)
        hist = torch.zeros(8, dtype=torch.float64, device="cuda")
        its = []
        for _ in range(4):
            cpm.cpm_run_cycles(band, p, fd, ud, work, nbytes, 1, 1, hist)
            its.append(host(ud).copy())
        out[lds] = its
        del work, band
    for k in range(4):
        assert np.array_equal(out["1"][k], out["0"][k]), k


@pytest.mark.parametrize("name,cfg", [
    ("sphere64", W.config_sphere(64, 5)),
    ("torus32", W.config_torus_mixed(32, 3)),
], ids=["sphere64", "torus32"])
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_tiled_sweep_equals_two_passes(name, cfg, precision, monkeypatch):
    """The tiled pass forms f + N u in LDS in the neighbour-sum pass's order and interpolates
    it in the extension pass's order: cycles with it on every level agree with the two-pass
    cycles to rounding (the same expressions; the compiler may contract them differently)."""
    log("tiled sweep vs two passes: %s %s" % (name, precision))
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    prec = cpm.CPM_F64 if precision == "f64" else cpm.CPM_MIXED
    monkeypatch.setenv("CPM_TILE_MIN_NODES", "1000")
    out = {}
    fd = None
    for form in ("tile", "split"):
        monkeypatch.setenv("CPM_SWEEP", form)
        band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
        if fd is None:
            fd = dev(cfg.problem.f(band.export(0)[1]))
        tun = [cpm.cpm_band_tuning(band, l) for l in range(band.levels - 1)]
        assert all(t[6] == (form == "tile") for t in tun)
        p = cpm.make_params(c=cfg.problem.c, precision=prec)
        work, nbytes = workspace(band, p)
        ud = torch.zeros_like(fd)
        hist = torch.zeros(8, dtype=torch.float64, device="cuda")
        its = []
        for _ in range(4):
            cpm.cpm_run_cycles(band, p, fd, ud, work, nbytes, 1, 1, hist)
            its.append(host(ud).copy())
        out[form] = its
        del work, band
    tol = 1e-13 if precision == "f64" else 1e-5
    for k in range(4):
        err = rel_inf(out["tile"][k], out["split"][k])
        log("cycle %d: rel diff %.3e (bitwise equal: %s)" % (k, err, np.array_equal(out["tile"][k], out["split"][k])))
        assert err <= tol, (k, err)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_ext_prefetch_equals_plain_lds(precision, monkeypatch):
    """The LDS-staged extension that loads each node's own data before the staging does the
    same arithmetic as the one that loads it after: cycles agree bit for bit."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_sphere(32, 4)
    prec = cpm.CPM_F64 if precision == "f64" else cpm.CPM_MIXED
    monkeypatch.setenv("CPM_SWEEP", "split")
    out = {}
    fd = None
    for pf in ("1", "0"):
        monkeypatch.setenv("CPM_EXT_PREFETCH", pf)
        band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
        if fd is None:
            fd = dev(cfg.problem.f(band.export(0)[1]))
        tun = [cpm.cpm_band_tuning(band, l) for l in range(band.levels - 1)]
        assert all(t[0] and t[7] == (pf == "1") for t in tun), tun
        p = cpm.make_params(precision=prec)
        work, nbytes = workspace(band, p)
        ud = torch.zeros_like(fd)
        hist = torch.zeros(8, dtype=torch.float64, device="cuda")
        its = []
        for _ in range(4):
            cpm.cpm_run_cycles(band, p, fd, ud, work, nbytes, 1, 1, hist)
            its.append(host(ud).copy())
        out[pf] = its
        del work, band
    for k in range(4):
        assert np.array_equal(out["1"][k], out["0"][k]), k


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_visit_order_and_workgroup_slots_leave_cycles_unchanged(precision, monkeypatch):
    """The stencil visit order (Morton blocks of 16^3 or 8^3 cells, or plain (z, y, x)), the
    number of stencil slots a staging workgroup takes per lane (1, 2, 4), the neighbour sum's
    addressing (segments of consecutive entries, or per-node lists) and the residual before restriction
    (formed at the restriction's fine nodes only, or everywhere) change only which workgroup
    handles a node, where its indices come from and which never-read entries are written,
    not the arithmetic: cycles agree bit for bit, on the torus at h = 1/64."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.SolverConfig("t64", W.torus_modes(1.0, 0.4, 11), 1 / 64, 4, W.LAM2_3D)
    prec = cpm.CPM_F64 if precision == "f64" else cpm.CPM_MIXED
    monkeypatch.setenv("CPM_SWEEP", "split")
    monkeypatch.setenv("CPM_EXT_PREFETCH", "1")
    out = {}
    fd = None
    for tag, env in (("default", {}), ("plain_order", {"CPM_MORTON_BITS": "-1"}), ("morton8", {"CPM_MORTON_BITS": "3"}),
                     ("npt2", {"CPM_EXT_NPT": "2"}), ("npt4", {"CPM_EXT_NPT": "4"}),
                     ("nsum_lists", {"CPM_NSUM_SEG": "0"}), ("resid_full", {"CPM_RESID_SUBSET": "0"})):
        for k in ("CPM_MORTON_BITS", "CPM_EXT_NPT", "CPM_NSUM_SEG", "CPM_RESID_SUBSET"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
        if fd is None:
            fd = dev(cfg.problem.f(band.export(0)[1]))
        slots = cpm.cpm_band_ext_slots(band, 0)
        assert slots == 256 * int(env.get("CPM_EXT_NPT", "1")), (tag, slots)
        subset = bool(band.flags(0) & cpm.CPM_BAND_RESID_SUBSET)
        assert subset == (tag != "resid_full"), (tag, band.flags(0))
        assert cpm.cpm_band_tuning(band, 0)[0]  # the LDS-staged extension runs
        p = cpm.make_params(precision=prec)
        work, nbytes = workspace(band, p)
        ud = torch.zeros_like(fd)
        hist = torch.zeros(8, dtype=torch.float64, device="cuda")
        its = []
        for _ in range(3):
            cpm.cpm_run_cycles(band, p, fd, ud, work, nbytes, 1, 1, hist)
            its.append(host(ud).copy())
        out[tag] = its
        log("%s: %d slots per workgroup" % (tag, slots))
        del work, band
    for tag in ("plain_order", "morton8", "npt2", "npt4", "nsum_lists", "resid_full"):
        for k in range(3):
            assert np.array_equal(out[tag][k], out["default"][k]), (tag, k)


def test_calls_run_on_the_callers_stream():
    """Cycles enqueued on a side stream are ordered with that stream's later work (no
    synchronisation in between) and give the default stream's iterates bit for bit."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_sphere(32, 4)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    fd = dev(cfg.problem.f(band.export(0)[1]))
    p = cpm.make_params()
    work, nbytes = workspace(band, p)
    hist = torch.zeros(16, dtype=torch.float64, device="cuda")
    ua = torch.zeros_like(fd)
    cpm.cpm_run_cycles(band, p, fd, ua, work, nbytes, 5, 5, hist)
    ref = host(ua).copy()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ub = torch.zeros_like(fd)
        cpm.cpm_run_cycles(band, p, fd, ub, work, nbytes, 5, 5, hist, stream=side)
        snap = ub.clone()  # runs after the cycles on the same stream
    torch.cuda.synchronize()
    assert np.array_equal(host(snap), ref)


def test_set_band_tuning():
    """cpm_set_band_tuning applies a configuration (read back by cpm_band_tuning), rejects
    one the level cannot run, and the pinned configuration still solves to the oracle."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_sphere(32, 4)
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    for l in range(band.levels - 1):
        cpm.cpm_set_band_tuning(band, l, False, 128, 512, True, 512, False)
        assert cpm.cpm_band_tuning(band, l) == (False, 128, 512, True, 512, False, False, False)
    with pytest.raises(cpm.CpmError):
        cpm.cpm_set_band_tuning(band, 0, True, 100, 256, False, 256, False)  # workgroup size
    before = cpm.cpm_band_tuning(band, 0)
    with pytest.raises(cpm.CpmError):
        cpm.cpm_set_band_tuning(band, band.levels, True, 256, 256, False, 256, False)  # no such level
    assert cpm.cpm_band_tuning(band, 0) == before
    ref = ov.solve(H, f, ov.Params(), rtol=1e-10, max_cycles=60)
    p = cpm.make_params()
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
    assert st.cycles == ref.cycles
    assert rel_inf(host(ud), ref.u) < 1e-12


def test_autotune_on_bands_that_cannot_cycle():
    """Autotuning needs no cycle: a one-level band whose single level exceeds the dense
    coarsest solve tunes its passes, and only the solve reports the size limit."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_sphere(32, 1)
    band = build_gpu(cfg.problem.surface, cfg.h0, 1, cfg.lam2)
    assert band.n(0) > 12000
    cpm.cpm_autotune(band)
    assert len(cpm.cpm_band_tuning(band, 0)) == 8
    fd = dev(cfg.problem.f(band.export(0)[1]))
    p = cpm.make_params()
    work, nbytes = workspace(band, p)
    with pytest.raises(cpm.CpmError):
        cpm.cpm_solve(band, p, fd, torch.zeros_like(fd), work, nbytes, rtol=1e-10, max_cycles=5)


def test_error_paths():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    s = W.unit_sphere()
    with pytest.raises(cpm.CpmError) as ei:
        build_gpu(s, 1 / 16, 2, 4.0)  # band radius 2h is too narrow for cubic stencils
    assert ei.value.status == cpm.CPM_E_BAND
    with pytest.raises(cpm.CpmError):
        build_gpu(W.torus(0.4, 1.0), 1 / 16, 2)  # r > R
    band = build_gpu(W.unit_circle(), 1 / 32, 3)
    p = cpm.make_params(c=-1.0)
    n = band.n(0)
    fd = torch.ones(n, dtype=torch.float64, device="cuda")
    ud = torch.zeros_like(fd)
    with pytest.raises(cpm.CpmError):
        cpm.cpm_solve(band, p, fd, ud, fd, 8, 1e-10, 10)
    p = cpm.make_params()
    work, nbytes = workspace(band, p)
    with pytest.raises(cpm.CpmError) as ei:
        cpm.cpm_solve(band, p, fd, ud, work, nbytes // 2, 1e-10, 10)
    assert ei.value.status == cpm.CPM_E_WORKSPACE
    # zero right-hand side: u = 0 immediately
    fz = torch.zeros_like(fd)
    ud.fill_(3.0)
    st = cpm.cpm_solve(band, p, fz, ud, work, nbytes, 1e-10, 10)
    assert st.relres == 0.0 and float(ud.abs().max()) == 0.0
    # not converged within the cycle budget
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, 1e-30, 2, raise_on_noconv=False)
    assert st.status == cpm.CPM_E_NOCONV and st.cycles == 2
    # a tolerance below the rounding floor of the residual: the solve stops once the residual
    # has stagnated for 8 cycles, well before the cycle budget, and says so
    ud.zero_()
    with pytest.raises(cpm.CpmError, match="stagnated") as ei:
        cpm.cpm_solve(band, p, fd, ud, work, nbytes, 1e-30, 500)
    assert ei.value.status == cpm.CPM_E_NOCONV
    ud.zero_()
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, 1e-30, 500, raise_on_noconv=False)
    hist = st.history()
    assert st.cycles < 100 and min(hist) < 1e-10, (st.cycles, min(hist))
    assert min(hist[-8:]) >= 0.99 * min(hist[:-8]), hist[-10:]
    # NaN right-hand side is reported as divergence (a NaN at a node outside every
    # interpolation stencil would never reach E f, so poison all entries)
    fd.fill_(float("nan"))
    ud.zero_()
    with pytest.raises(cpm.CpmError) as ei:
        cpm.cpm_solve(band, p, fd, ud, work, nbytes, 1e-10, 5)
    assert ei.value.status in (cpm.CPM_E_DIVERGED,)


def test_single_level_is_direct_solve():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_circle(16, 1)
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ref = ov.solve(H, f, ov.Params(), rtol=1e-12, max_cycles=2)
    band = build_gpu(cfg.problem.surface, cfg.h0, 1)
    p = cpm.make_params()
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, 1e-12, 2)
    assert st.cycles == 1
    assert rel_inf(host(ud), ref.u) < 1e-12


def test_autotuned_solve_matches_oracle():
    """The autotuner changes launch configurations only: iterates still match the oracle."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_sphere(32, 4)
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ref = ov.solve(H, f, ov.Params(), rtol=1e-10, max_cycles=60)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    cpm.cpm_autotune(band)
    for l in range(band.levels):
        lds, eb, nb, fused, sb, slds, tiled, pf = cpm.cpm_band_tuning(band, l)
        assert lds or not pf
        assert eb in (128, 256, 512) and nb in (128, 256, 512) and sb in (128, 256, 512)
        assert sb == 256 or not slds
    p = cpm.make_params()
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
    assert st.cycles == ref.cycles
    assert rel_inf(host(ud), ref.u) < 1e-12
