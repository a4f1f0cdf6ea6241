"""Learned smoother on the GPU: the BF16-MFMA forward and backward kernels against the
float64 oracle of the network, the feature kernel against the oracle's features, one
learned V-cycle against the oracle's learned V-cycle, and a short training run."""
import numpy as np
import pytest

import workloads as W
from oracle import band as ob
from oracle import mlp as om
from oracle import vcycle as ov
from tests.gpu_util import build_gpu, dev, host, log, oracle_for, rel_inf, torch_cuda, workspace

pytestmark = pytest.mark.gpu


def _rand_weights(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return om.pack(rng.standard_normal((64, 64)) * scale, rng.standard_normal(64) * 0.1,
                   rng.standard_normal(64) * scale, 0.25)


def _bits_dev(bits):
    return dev(np.asarray(bits, dtype=np.uint16).view(np.int16))


@pytest.mark.parametrize("m", [1, 64, 1000, 70000])
def test_mlp_forward_matches_oracle(m):
    log("mlp forward m=%d" % m)
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    rng = np.random.default_rng(m)
    X = om.bf16_round(rng.uniform(-1, 1, (m, 64)).astype(np.float32))
    w = _rand_weights(7)
    y_ref, h_ref = om.forward(X, w)
    Xd = _bits_dev(om.bf16_bits(X))
    Y = torch.empty(m, dtype=torch.float32, device="cuda")
    H = torch.empty((m, 64), dtype=torch.float32, device="cuda")
    cpm.cpm_mlp_forward(m, Xd, _bits_dev(w), Y, H)
    y, h = host(Y), host(H)
    assert np.max(np.abs(y - y_ref)) <= 1e-4 * max(1.0, np.max(np.abs(y_ref)))
    assert np.max(np.abs(h - h_ref)) <= 1e-4 * max(1.0, np.max(np.abs(h_ref)))


@pytest.mark.parametrize("m", [100, 5000])
def test_mlp_backward_matches_oracle(m):
    log("mlp backward m=%d" % m)
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    rng = np.random.default_rng(10 + m)
    X = om.bf16_round(rng.uniform(-1, 1, (m, 64)).astype(np.float32))
    T = rng.standard_normal(m).astype(np.float32)
    w = _rand_weights(8)
    _, g_ref = om.loss_and_grad(X, T.astype(np.float64), w)
    Xd, Wd = _bits_dev(om.bf16_bits(X)), _bits_dev(w)
    Y = torch.empty(m, dtype=torch.float32, device="cuda")
    H = torch.empty((m, 64), dtype=torch.float32, device="cuda")
    G = torch.empty(om.N_W, dtype=torch.float32, device="cuda")
    cpm.cpm_mlp_forward(m, Xd, Wd, Y, H)
    cpm.cpm_mlp_backward(m, Xd, Wd, H, Y, dev(T), G)
    g = host(G).astype(np.float64)
    o = 64 * 64
    # dW1 is contracted on the matrix cores with dH rounded to bf16 (relative 2^-9 per term)
    assert np.linalg.norm(g[:o] - g_ref[:o]) <= 1e-2 * np.linalg.norm(g_ref[:o])
    # b1, w2, b2 are float32 sums
    assert np.max(np.abs(g[o:] - g_ref[o:])) <= 1e-4 * max(1e-6, np.max(np.abs(g_ref[o:])))


def _learned_case():
    return W.config_sphere(16, 3)


def test_features_match_oracle():
    log("smoother features")
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = _learned_case()
    H = oracle_for(cfg)
    lev = H.levels[0]
    f = cfg.problem.f(lev.cp)
    u = W.random_vector(lev.n, 5) * 0.01
    r = ov.residual(H, 0, u, f, ov.Params())
    X_ref, s_ref = om.features(lev, r)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    X = torch.empty((lev.n, 64), dtype=torch.int16, device="cuda")
    s = torch.empty(lev.n, dtype=torch.float32, device="cuda")
    work = torch.empty(2 * lev.n, dtype=torch.float64, device="cuda")
    cpm.cpm_smoother_features(band, 0, 1.0, dev(f), dev(u), X, s, work)
    Xg = om.from_bf16_bits(host(X).view(np.uint16))
    assert np.allclose(host(s), s_ref.astype(np.float32), rtol=1e-6)
    diff = Xg != X_ref.astype(np.float32)
    # identical except where a double-rounding boundary of bf16 is hit (weights computed in
    # a different but equivalent product order)
    assert diff.mean() < 1e-3
    assert np.max(np.abs(Xg - X_ref)) <= 2 ** -7


def test_learned_vcycle_matches_oracle():
    log("learned V-cycle parity")
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = _learned_case()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    w = _rand_weights(9, scale=0.05)
    ref = ov.solve(H, f, ov.Params(learned=w), rtol=0.0, max_cycles=2, keep_iterates=True)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    cpm.cpm_set_smoother_weights(band, w, 10.0)
    p = cpm.make_params(smoother=cpm.CPM_SMOOTH_LEARNED)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=0.0, max_cycles=1, raise_on_noconv=False)
    assert st.cycles == 1
    err = rel_inf(host(ud), ref.iterates[0])
    assert err < 1e-4, err


def test_learned_cycles_from_the_stopping_residual():
    """Cycles after the first take the learned update of their first sweep from the residual
    the previous cycle's stopping test computed: five graph-replayed cycles give the iterate of
    five separate one-cycle runs (where no residual is carried over) bit for bit."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = _learned_case()
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    cpm.cpm_set_smoother_weights(band, _rand_weights(9, scale=0.05), 10.0)
    fd = dev(cfg.problem.f(band.export(0)[1]))
    p = cpm.make_params(smoother=cpm.CPM_SMOOTH_LEARNED)
    work, nbytes = workspace(band, p)
    hist = torch.zeros(8, dtype=torch.float64, device="cuda")
    ua = torch.zeros_like(fd)
    for _ in range(5):
        cpm.cpm_run_cycles(band, p, fd, ua, work, nbytes, 1, 1, hist)
    ub = torch.zeros_like(fd)
    cpm.cpm_run_cycles(band, p, fd, ub, work, nbytes, 5, 5, hist)
    a, b = host(ua), host(ub)
    assert np.all(np.isfinite(a)) and np.max(np.abs(a)) > 0
    assert np.array_equal(a, b)


def test_jacobi_network_reproduces_plain_solve():
    """With the weights of the damped Jacobi network the learned solve matches the plain one."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_sphere(32, 4)
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    fd = dev(f)
    p = cpm.make_params()
    work, nbytes = workspace(band, p)
    u0 = torch.zeros_like(fd)
    plain = cpm.cpm_solve(band, p, fd, u0, work, nbytes, rtol=1e-10, max_cycles=60)
    cpm.cpm_set_smoother_weights(band, om.jacobi_weights(2.0 / 3.0, 3), 10.0)
    pl = cpm.make_params(smoother=cpm.CPM_SMOOTH_LEARNED)
    u1 = torch.zeros_like(fd)
    lst = cpm.cpm_solve(band, pl, fd, u1, work, nbytes, rtol=1e-10, max_cycles=60)
    assert abs(lst.cycles - plain.cycles) <= 1
    assert rel_inf(host(u1), host(u0)) < 1e-8


def test_fallback_trips_for_bad_network():
    """A network that diverges is replaced by Jacobi once a cycle contracts worse than the
    plain method; the solve still reaches the tolerance."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_sphere(32, 4)
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    cpm.cpm_set_smoother_weights(band, om.jacobi_weights(-3.0, 3), 0.5)
    p = cpm.make_params(smoother=cpm.CPM_SMOOTH_LEARNED)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=80)
    assert st.fallback_cycle >= 0
    assert st.relres < 1e-10


def test_training_reduces_loss_and_beats_damped_jacobi():
    """Train on pairs from plain cycles (spheres and a torus at h = 1/32), then solve a
    sphere problem that was not in the training set: the trained smoother must contract
    faster per cycle than the plain damped Jacobi cycle, without tripping the fallback."""
    log("training + gain")
    import paper_1307_4354_amd as cpm
    from paper_1307_4354_amd import learned

    torch = torch_cuda()
    probs = [(W.sphere_modes(0.9, 1), 1 / 32, 4), (W.torus_modes(1.0, 0.4, 2), 1 / 32, 3)]
    pairs = learned.generate_pairs(probs, cycles=2)
    assert pairs.X.shape[0] > 100000
    res = learned.train(pairs, steps=300, batch=16384, lr=2e-3, log_every=50)
    l0 = learned.evaluate_loss(pairs, learned._bf16_bits(learned.jacobi_init(2.0 / 3.0, 3, 0)))
    l1 = learned.evaluate_loss(pairs, res.w_bits)
    assert np.all(np.isfinite(res.losses))
    assert l1 < 0.5 * l0
    cfg = W.config_sphere(32, 4)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    _, cp = band.export(0)
    fd = dev(cfg.problem.f(cp))
    p = cpm.make_params()
    work, nbytes = workspace(band, p)
    u0 = torch.zeros_like(fd)
    plain = cpm.cpm_solve(band, p, fd, u0, work, nbytes, rtol=1e-10, max_cycles=80)
    hist = list(plain.relres_history[:plain.cycles])
    rho = max(b / a for a, b in zip(hist, hist[1:]))
    cpm.cpm_set_smoother_weights(band, res.w_bits, rho)
    u1 = torch.zeros_like(fd)
    lst = cpm.cpm_solve(band, cpm.make_params(smoother=cpm.CPM_SMOOTH_LEARNED), fd, u1, work, nbytes,
                        rtol=1e-10, max_cycles=80)
    log("plain %d cycles, learned %d cycles, fallback %d" % (plain.cycles, lst.cycles, lst.fallback_cycle))
    assert lst.fallback_cycle < 0
    assert lst.relres < 1e-10
    assert lst.cycles < plain.cycles
