"""W-cycles (cycle index 2) and the full-multigrid start on the GPU against the oracle: every
iterate within 1e-12 for both sweep forms and for the standard relaxation; the mixed-precision
solve from the full-multigrid start against the oracle's; argument checks."""
import numpy as np
import pytest

import workloads as W
from oracle import standard as ostd
from oracle import vcycle as ov
from tests.gpu_util import build_gpu, dev, host, log, oracle_for, rel_inf, torch_cuda, workspace

pytestmark = pytest.mark.gpu

CASES = [("circle64", W.config_circle(64, 4)), ("sphere32", W.config_sphere(32, 4))]


@pytest.mark.parametrize("name,cfg", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("sweep", ["split", "fused"])
def test_w_cycle_iterates_match_oracle(name, cfg, sweep, monkeypatch):
    log("W-cycle parity: %s (%s sweeps)" % (name, sweep))
    import paper_1307_4354_amd as cpm

    monkeypatch.setenv("CPM_SWEEP", sweep)
    torch = torch_cuda()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ref = ov.solve(H, f, ov.Params(gamma=2), rtol=0.0, max_cycles=6, keep_iterates=True)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(gamma=2)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    for k in range(6):
        rel = cpm.cpm_vcycle(band, p, fd, ud, work, nbytes, want_relres=True)
        assert rel_inf(host(ud), ref.iterates[k]) < 1e-12, k
        assert abs(rel - ref.relres[k]) <= 1e-3 * ref.relres[k] + 1e-14


@pytest.mark.parametrize("name,cfg", CASES, ids=[c[0] for c in CASES])
def test_fmg_solve_matches_oracle(name, cfg):
    log("FMG start parity: %s" % name)
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    cp = H.levels[0].cp
    f = cfg.problem.f(cp)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(fmg=True)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    for ncyc in (1, 3):
        ref = ov.solve(H, f, ov.Params(), rtol=0.0, max_cycles=ncyc, keep_iterates=True, fmg=True)
        ud = torch.zeros_like(fd)
        st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=0.0, max_cycles=ncyc, raise_on_noconv=False)
        assert st.cycles == ncyc
        assert rel_inf(host(ud), ref.iterates[-1]) < 1e-12, ncyc
    ref = ov.solve(H, f, ov.Params(), rtol=1e-10, max_cycles=60, fmg=True)
    ud = torch.zeros_like(fd)
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
    assert st.cycles == ref.cycles
    plain = cpm.cpm_solve(band, cpm.make_params(), fd, torch.zeros_like(fd), work, nbytes, rtol=1e-10, max_cycles=60)
    assert st.cycles < plain.cycles


@pytest.mark.parametrize("name,cfg", CASES, ids=[c[0] for c in CASES])
def test_mixed_fmg_solve_matches_oracle(name, cfg):
    """Mixed precision from the full-multigrid start: the float64 start (as in the float64
    solve), then float32 cycles with float64 refinement, against the oracle's mixed solve from
    its own float64 start: the start within 1e-12, cycle count within one, each cycle's
    relative residual within 1 %, the solution within 1e-9 of the float64 oracle's."""
    log("mixed FMG parity: %s" % name)
    import paper_1307_4354_amd as cpm
    from oracle import mixed as omx

    torch = torch_cuda()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    op = ov.Params()
    u0 = ov.fmg_start(H, f, op, ov.CoarseSolver(H, op))
    mx = omx.solve_mixed(H, f, op, rtol=1e-10, max_cycles=60, u0=u0)
    r64 = ov.solve(H, f, op, rtol=1e-10, max_cycles=60)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(fmg=True, precision=cpm.CPM_MIXED)
    work, nbytes = workspace(band, p)
    assert nbytes >= cpm.cpm_workspace_size(band, cpm.make_params())  # the start's float64 layout
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st0 = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=0, raise_on_noconv=False)
    assert st0.cycles == 0
    assert rel_inf(host(ud), u0) < 1e-12  # the start alone
    ud.zero_()
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
    plain = cpm.cpm_solve(band, cpm.make_params(precision=cpm.CPM_MIXED), fd, torch.zeros_like(fd), work, nbytes,
                          rtol=1e-10, max_cycles=60)
    log("%s: GPU %d cycles (oracle %d, from u = 0 %d)" % (name, st.cycles, len(mx.relres), plain.cycles))
    assert abs(st.cycles - len(mx.relres)) <= 1
    hg, ho = st.history(), mx.relres
    for j in range(min(len(hg), len(ho))):
        assert abs(hg[j] - ho[j]) <= 1e-2 * ho[j], (j, hg[j], ho[j])
    assert st.relres < 1e-10
    assert rel_inf(host(ud), r64.u) < 1e-9
    assert st.cycles < plain.cycles


def test_standard_w_cycle_matches_oracle():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_sphere(32, 4)
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ref = ostd.solve(H, f, ostd.StdParams(gamma=2), rtol=0.0, max_cycles=5, keep_iterates=True)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(smoother=cpm.CPM_SMOOTH_STANDARD, gamma=2)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    for k in range(5):
        cpm.cpm_vcycle(band, p, fd, ud, work, nbytes)
        assert rel_inf(host(ud), ref.iterates[k]) < 1e-12, k


def test_cycle_arguments_rejected():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_circle(32, 3)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    fd = torch.ones(band.n(0), dtype=torch.float64, device="cuda")
    ud = torch.zeros_like(fd)
    for p in (cpm.make_params(fmg=True, smoother=cpm.CPM_SMOOTH_STANDARD), cpm.make_params(gamma=7)):
        work, nbytes = workspace(band, cpm.make_params())
        with pytest.raises(cpm.CpmError):
            cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=3)
    # a mixed-precision solve with the full-multigrid start needs the float64 layout too
    pm = cpm.make_params(fmg=True, precision=cpm.CPM_MIXED)
    work, nbytes = workspace(band, cpm.make_params(precision=cpm.CPM_MIXED))
    assert cpm.cpm_workspace_size(band, pm) > nbytes
    with pytest.raises(cpm.CpmError) as ei:
        cpm.cpm_solve(band, pm, fd, ud, work, nbytes, rtol=1e-10, max_cycles=3)
    assert ei.value.status == cpm.CPM_E_WORKSPACE
    pb = cpm.make_params(precision=cpm.CPM_MIXED, gamma=2)
    nb = cpm.cpm_workspace_size_batched([band], pb)
    wb = torch.empty(nb, dtype=torch.uint8, device="cuda")
    with pytest.raises(cpm.CpmError):
        cpm.cpm_solve_batched([band], pb, [fd], [ud], wb, nb, rtol=1e-10, max_cycles=3)
