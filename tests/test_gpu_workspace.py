"""The workspace's contents on entry do not matter: every solve form gives the same result bit
for bit from a workspace of zero bytes and from one of 0xFF bytes (a NaN in float32 and in
float64), so no kernel reads a workspace entry before writing it."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import build_gpu, dev, host, log, torch_cuda

pytestmark = pytest.mark.gpu


def _forms(cpm):
    mx, std = cpm.CPM_MIXED, cpm.CPM_SMOOTH_STANDARD
    return [("f64", {}), ("mixed", {"precision": mx}), ("f64_fmg", {"fmg": True}),
            ("mixed_fmg", {"precision": mx, "fmg": True}), ("f64_w", {"gamma": 2}),
            ("standard", {"smoother": std})]


@pytest.mark.parametrize("sweep", ["split", "fused", "tile"])
def test_solves_ignore_workspace_contents(sweep, monkeypatch):
    import paper_1307_4354_amd as cpm

    monkeypatch.setenv("CPM_SWEEP", sweep)
    monkeypatch.setenv("CPM_TILE_MIN_NODES", "1000")
    torch = torch_cuda()
    cfg = W.SolverConfig("t32", W.torus_modes(1.0, 0.4, 5), 1 / 32, 3, W.LAM2_3D)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    fd = dev(cfg.problem.f(band.export(0)[1]))
    for name, kw in _forms(cpm):
        p = cpm.make_params(**kw)
        nbytes = cpm.cpm_workspace_size(band, p)
        work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        out = []
        for fill in (0, 255):
            work.fill_(fill)
            ud = torch.zeros_like(fd)
            st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
            out.append((host(ud).copy(), st.cycles, st.history().copy()))
        log("%s sweep, %s: %d cycles from both workspaces" % (sweep, name, out[0][1]))
        assert out[0][1] == out[1][1], name
        assert np.array_equal(out[0][0], out[1][0]), name
        assert np.array_equal(out[0][2], out[1][2]), name
        # one cycle of cpm_vcycle (double precision) as well
        if kw.get("precision", cpm.CPM_F64) == cpm.CPM_F64 and not kw.get("fmg"):
            its = []
            for fill in (0, 255):
                work.fill_(fill)
                ud = torch.zeros_like(fd)
                cpm.cpm_vcycle(band, p, fd, ud, work, nbytes)
                its.append(host(ud).copy())
            assert np.array_equal(its[0], its[1]), name


def test_batched_solve_ignores_workspace_contents():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    items = W.batch_problems(3, seed=W.SEED_BASE + 46, h_choices=(16, 32), coarse_h_inv=4)
    bands, fs = [], []
    for it in items:
        b = build_gpu(it.problem.surface, it.h0, it.levels, it.lam2)
        bands.append(b)
        fs.append(dev(it.problem.f(b.export(0)[1])))
    p = cpm.make_params(precision=cpm.CPM_MIXED)
    nbytes = cpm.cpm_workspace_size_batched(bands, p)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    res = []
    for fill in (0, 255):
        work.fill_(fill)
        us = [torch.zeros_like(f) for f in fs]
        status, stats = cpm.cpm_solve_batched(bands, p, fs, us, work, nbytes, rtol=1e-10, max_cycles=80)
        assert status == cpm.CPM_OK
        res.append(([host(u).copy() for u in us], [s.cycles for s in stats]))
    assert res[0][1] == res[1][1]
    for a, b in zip(res[0][0], res[1][0]):
        assert np.array_equal(a, b)
