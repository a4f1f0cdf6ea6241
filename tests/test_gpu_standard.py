"""The standard-relaxation V-cycle (Sec. 4.5) on the GPU against the oracle's: every
iterate within 1e-12, the same number of cycles to the paper's increment criterion, the
increments of each cycle, and the argument checks."""
import numpy as np
import pytest

import workloads as W
from oracle import standard as ostd
from tests.gpu_util import build_gpu, dev, host, log, oracle_for, rel_inf, torch_cuda, workspace

pytestmark = pytest.mark.gpu

CASES = [
    ("circle64", W.config_circle(64, 4), 12),
    ("sphere32", W.config_sphere(32, 4), 12),
    ("torus32", W.SolverConfig("t32", W.torus_modes(1.0, 0.4, 7), 1 / 32, 3, W.LAM2_3D), 10),
]


@pytest.mark.parametrize("name,cfg,ncyc", CASES, ids=[c[0] for c in CASES])
def test_standard_iterates_match_oracle(name, cfg, ncyc):
    log("standard relaxation iterates: %s (%d cycles)" % (name, ncyc))
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ref = ostd.solve(H, f, ostd.StdParams(c=cfg.problem.c), rtol=0.0, max_cycles=ncyc, keep_iterates=True)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(c=cfg.problem.c, smoother=cpm.CPM_SMOOTH_STANDARD)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    for k in range(ncyc):
        inc = cpm.cpm_vcycle(band, p, fd, ud, work, nbytes, want_relres=True)
        err = rel_inf(host(ud), ref.iterates[k])
        assert err < 1e-12, (k, err)
        # an increment is a difference of two iterates that each agree to ~1e-13 of ||u||:
        # its error is absolute in units of ||u||
        assert abs(inc - ref.increments[k]) <= 1e-11 + 1e-6 * ref.increments[k], (k, inc, ref.increments[k])


@pytest.mark.parametrize("name,cfg", [c[:2] for c in CASES[:2]], ids=[c[0] for c in CASES[:2]])
def test_standard_solve_matches_oracle(name, cfg):
    log("standard relaxation solve: %s" % name)
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ref = ostd.solve(H, f, ostd.StdParams(c=cfg.problem.c), rtol=1e-10, max_cycles=60)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(c=cfg.problem.c, smoother=cpm.CPM_SMOOTH_STANDARD)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
    assert st.cycles == ref.cycles
    assert st.relres < 1e-10
    assert rel_inf(host(ud), ref.u) < 1e-11
    hist = st.history()
    for k in range(len(hist)):
        assert abs(hist[k] - ref.increments[k]) <= 1e-11 + 1e-6 * ref.increments[k], k
    # a second solve with another c rebuilds the coarse inverse and the relaxation weights
    p2 = cpm.make_params(c=2.0, smoother=cpm.CPM_SMOOTH_STANDARD)
    ref2 = ostd.solve(H, f, ostd.StdParams(c=2.0), rtol=1e-10, max_cycles=60)
    ud.zero_()
    st2 = cpm.cpm_solve(band, p2, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
    assert st2.cycles == ref2.cycles
    assert rel_inf(host(ud), ref2.u) < 1e-11


def test_standard_rejects_mixed_precision():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_circle(32, 3)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(smoother=cpm.CPM_SMOOTH_STANDARD, precision=cpm.CPM_MIXED)
    work = torch.empty(1 << 24, dtype=torch.uint8, device="cuda")
    fd = torch.ones(band.n(0), dtype=torch.float64, device="cuda")
    ud = torch.zeros_like(fd)
    with pytest.raises(cpm.CpmError):
        cpm.cpm_solve(band, p, fd, ud, work, work.numel(), rtol=1e-10, max_cycles=5)
