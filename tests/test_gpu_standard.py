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
@pytest.mark.parametrize("order", ["jacobi", "redblack"])
def test_standard_iterates_match_oracle(name, cfg, ncyc, order):
    """Jacobi sweeps, and Gauss-Seidel sweeps in red-black order (both half-sweeps in place
    on the GPU, the black one reading the new red values)."""
    log("standard relaxation iterates: %s (%d cycles, %s)" % (name, ncyc, order))
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ref = ostd.solve(H, f, ostd.StdParams(c=cfg.problem.c, smoother=order), rtol=0.0, max_cycles=ncyc,
                     keep_iterates=True)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    sm = cpm.CPM_SMOOTH_STANDARD if order == "jacobi" else cpm.CPM_SMOOTH_STANDARD_RB
    p = cpm.make_params(c=cfg.problem.c, smoother=sm)
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
@pytest.mark.parametrize("order", ["jacobi", "redblack"])
def test_standard_solve_matches_oracle(name, cfg, order):
    log("standard relaxation solve: %s (%s)" % (name, order))
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ref = ostd.solve(H, f, ostd.StdParams(c=cfg.problem.c, smoother=order), rtol=1e-10, max_cycles=60)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    sm = cpm.CPM_SMOOTH_STANDARD if order == "jacobi" else cpm.CPM_SMOOTH_STANDARD_RB
    p = cpm.make_params(c=cfg.problem.c, smoother=sm)
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


@pytest.mark.parametrize("name,cfg", [("circle64", W.config_circle(64, 4)), ("sphere32", W.config_sphere(32, 4))],
                         ids=["circle64", "sphere32"])
def test_linear_el_operator_apply_matches_oracle(name, cfg):
    """Remark 3.2's operator A = c I - (E_1 L - gamma (I - E_3)) applied matrix-free on the GPU
    against the oracle's assembled matrix (the one its Table 3.1 pin checks), every level."""
    import paper_1307_4354_amd as cpm
    from oracle import direct as od

    torch = torch_cuda()
    H = oracle_for(cfg)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    for l in range(band.levels):
        lev = H.levels[l]
        u = W.random_vector(lev.n, 40 + l)
        ref = od.assemble_A(lev, 1.0, p=1, q=3) @ u
        out = torch.empty(lev.n, dtype=torch.float64, device="cuda")
        work = torch.empty_like(out)
        cpm.cpm_apply_pq(band, l, 1, 1.0, dev(u), out, work)
        assert rel_inf(host(out), ref) < 1e-13, (l, rel_inf(host(out), ref))


@pytest.mark.parametrize("name,cfg,ncyc", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_linear_el_standard_iterates_match_oracle(name, cfg, ncyc):
    """The standard-relaxation V-cycle on Remark 3.2's operator, iterate by iterate."""
    log("standard relaxation, linear E in front of L: %s" % name)
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    ref = ostd.solve(H, f, ostd.StdParams(c=cfg.problem.c, el_degree=1), rtol=0.0, max_cycles=ncyc,
                     keep_iterates=True)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    p = cpm.make_params(c=cfg.problem.c, smoother=cpm.CPM_SMOOTH_STANDARD, el_degree=1)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    for k in range(ncyc):
        cpm.cpm_vcycle(band, p, fd, ud, work, nbytes)
        err = rel_inf(host(ud), ref.iterates[k])
        assert err < 1e-12, (k, err)


@pytest.mark.parametrize("dx,table", [(0.025, 4.76e-3), (0.0125, 1.19e-3)])
def test_linear_el_solve_reproduces_table_3_1(dx, table):
    """Table 3.1 on the GPU: the standard-relaxation V-cycle with the plain residual on Remark
    3.2's operator converges to the direct solve of A u = f; its relative error on the circle
    (20,000 surface points, cubic interpolation) is the printed one within 1 %."""
    import paper_1307_4354_amd as cpm
    from oracle import band as ob
    from oracle import direct as od
    from oracle import errors as oe

    torch = torch_cuda()
    prob = W.circle_sin12()
    H = ob.build_hierarchy(prob.surface, dx, 3, W.LAM2_2D)
    f = prob.f(H.levels[0].cp)
    u_star = od.solve_direct(H.levels[0], f, 1.0, p=1, q=3)
    band = build_gpu(prob.surface, dx, 3, W.LAM2_2D)
    p = cpm.make_params(smoother=cpm.CPM_SMOOTH_STANDARD, el_degree=1, residual_mode=cpm.CPM_RESIDUAL_VERBATIM)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-13, max_cycles=120)
    u = host(ud)
    assert rel_inf(u, u_star) < 1e-9
    e = oe.surface_error(H.levels[0], u, prob.u_exact, 20000)
    log("dx %g: %d cycles, error %.4e (Table 3.1: %.2e)" % (dx, st.cycles, e, table))
    assert abs(e - table) / table < 0.01
