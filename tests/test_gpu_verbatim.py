"""The residual of Algorithm 4.1 step 2 as printed (r = f - (cI - L) u at every node, the
coarsest level solving A_c e = f_c, progress measured by the relative increment) on the GPU
against the oracle's verbatim mode, iterate by iterate."""
import numpy as np
import pytest

import workloads as W
from oracle import vcycle as ov
from tests.gpu_util import build_gpu, dev, host, log, oracle_for, rel_inf, torch_cuda, workspace

pytestmark = pytest.mark.gpu

CASES = [("circle64", W.config_circle(64, 4), 12), ("sphere32", W.config_sphere(32, 4), 12)]


@pytest.mark.parametrize("name,cfg,ncyc", CASES, ids=[c[0] for c in CASES])
def test_verbatim_iterates_match_oracle(name, cfg, ncyc):
    log("verbatim residual parity: %s" % name)
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    pv = ov.Params(c=cfg.problem.c, residual_mode="verbatim")
    ref = ov.solve(H, f, pv, rtol=0.0, max_cycles=ncyc, keep_iterates=True)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(c=cfg.problem.c, residual_mode=cpm.CPM_RESIDUAL_VERBATIM)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    for k in range(ncyc):
        inc = cpm.cpm_vcycle(band, p, fd, ud, work, nbytes, want_relres=True)
        err = rel_inf(host(ud), ref.iterates[k])
        assert err < 1e-12, (k, err)
        # an increment is a difference of iterates that agree to 1e-12 of max |u|
        assert abs(inc - ref.increments[k]) <= 1e-6 * ref.increments[k] + 1e-11, (k, inc, ref.increments[k])


def test_verbatim_solve_stops_on_the_increment():
    """The verbatim cycle's fixed point leaves E f - A u at the discretization level (the
    residual stagnates), while the increment falls below 1e-10 in the oracle's cycle count."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_circle(64, 4)
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    pv = ov.Params(c=cfg.problem.c, residual_mode="verbatim")
    ref = ov.solve(H, f, pv, rtol=1e-10, max_cycles=60)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(c=cfg.problem.c, residual_mode=cpm.CPM_RESIDUAL_VERBATIM)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
    assert abs(st.cycles - ref.cycles) <= 1 and st.relres < 1e-10
    assert rel_inf(host(ud), ref.u) < 1e-9
    assert ref.relres[-1] > 1e-5  # E f - A u stagnates (the literal residual's fixed point)


def test_verbatim_rejects_other_modes():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_circle(64, 4)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    fd = dev(cfg.problem.f(band.export(0)[1]))
    for p in (cpm.make_params(residual_mode=cpm.CPM_RESIDUAL_VERBATIM, precision=cpm.CPM_MIXED),
              cpm.make_params(residual_mode=7)):
        work, nbytes = workspace(band, cpm.make_params(precision=cpm.CPM_MIXED))
        with pytest.raises(cpm.CpmError):
            cpm.cpm_solve(band, p, fd, torch.zeros_like(fd), work, nbytes, rtol=1e-10, max_cycles=5)
