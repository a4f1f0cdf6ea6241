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


def _near_jacobi_weights(seed, noise=0.02, omega=0.8):
    """A network with every weight random (scale `noise`) except two hidden units that carry
    the Jacobi step omega * x_centre: a non-trivial network whose cycle contracts."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((64, 64)) * noise
    b1 = rng.standard_normal(64) * noise
    w2 = rng.standard_normal(64) * noise
    W1[0, :] = 0.0
    W1[1, :] = 0.0
    W1[0, 13] = 1.0
    W1[1, 13] = -1.0
    b1[:2] = 0.0
    w2[0], w2[1] = omega, -omega
    return om.pack(W1, b1, w2, 0.0)


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


@pytest.mark.parametrize("m", [100, 5000, 70001])
def test_mlp_backward_matches_oracle(m):
    """The backward kernel on the oracle's forward values (H, Y rounded to float32): every
    element of dW1 against the oracle's gradient that rounds the hidden error to bfloat16 as
    the matrix cores take it, within float32 accumulation (1e-5 of the sum of the terms'
    magnitudes); b1, w2, b2 element by element to float32 accumulation."""
    log("mlp backward m=%d" % m)
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    rng = np.random.default_rng(10 + m)
    X = om.bf16_round(rng.uniform(-1, 1, (m, 64)).astype(np.float32))
    T = rng.standard_normal(m).astype(np.float32)
    w = _rand_weights(8)
    y_ref, h_ref = om.forward(X, w)
    H32, Y32 = h_ref.astype(np.float32), y_ref.astype(np.float32)
    g_ref = om.backward_bf16(X, w, H32, Y32, T)
    Xd, Wd = _bits_dev(om.bf16_bits(X)), _bits_dev(w)
    G = torch.empty(om.N_W, dtype=torch.float32, device="cuda")
    cpm.cpm_mlp_backward(m, Xd, Wd, dev(H32), dev(Y32), dev(T), G)
    g = host(G).astype(np.float64)
    o = 64 * 64
    dy = (np.float32(2.0) / np.float32(m)) * (Y32 - T)
    dh = np.abs(np.where(H32 > 0, dy[:, None] * om.unpack(w)[2].astype(np.float32)[None, :], 0.0))
    mag = dh.astype(np.float64).T @ np.abs(X.astype(np.float64))  # sum of |terms| per element
    assert np.all(np.abs(g[:o] - g_ref[:o]) <= 1e-5 * mag.ravel() + 1e-30)
    mag_b1 = dh.astype(np.float64).sum(axis=0)
    assert np.all(np.abs(g[o:o + 64] - g_ref[o:o + 64]) <= 1e-5 * mag_b1 + 1e-30)
    mag_w2 = H32.astype(np.float64).T @ np.abs(dy.astype(np.float64))
    assert np.all(np.abs(g[o + 64:o + 128] - g_ref[o + 64:o + 128]) <= 1e-5 * mag_w2 + 1e-30)
    assert abs(g[-1] - g_ref[-1]) <= 1e-5 * float(np.abs(dy).astype(np.float64).sum())


def test_mlp_loss_matches_definition():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    rng = np.random.default_rng(3)
    for m in (1, 1000, 65536):
        Y = rng.standard_normal(m).astype(np.float32)
        T = rng.standard_normal(m).astype(np.float32)
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        cpm.cpm_mlp_loss(m, dev(Y), dev(T), out)
        ref = float(np.mean((Y.astype(np.float64) - T.astype(np.float64)) ** 2))
        assert abs(float(host(out)[0]) - ref) <= 1e-12 * ref


def _learned_case():
    return W.config_sphere(16, 3)


def _features_check(cfg, level, u_seed):
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    lev = H.levels[level]
    f = cfg.problem.f(lev.cp) if level == 0 else W.random_vector(lev.n, u_seed + 1)
    u = W.random_vector(lev.n, u_seed) * 0.01
    r = ov.residual(H, level, u, f, ov.Params())
    X_ref, s_ref = om.features(lev, r)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    X = torch.empty((lev.n, 64), dtype=torch.int16, device="cuda")
    s = torch.empty(lev.n, dtype=torch.float32, device="cuda")
    work = torch.empty(2 * lev.n, dtype=torch.float64, device="cuda")
    cpm.cpm_smoother_features(band, level, 1.0, dev(f), dev(u), X, s, work)
    Xg = om.from_bf16_bits(host(X).view(np.uint16))
    assert np.allclose(host(s), s_ref.astype(np.float32), rtol=1e-6)
    ref = X_ref.astype(np.float32)
    diff = Xg != ref
    # both sides round the same float32 quotient to bfloat16; the residual itself is summed in
    # another order (rounding-level differences), which can move a value across a rounding
    # boundary: then the two differ by one bfloat16 step, and only rarely
    log("features level %d: %d of %d entries differ" % (level, int(diff.sum()), diff.size))
    assert diff.mean() < 1e-5
    ulp = np.abs(ref) * 2.0 ** -7
    assert np.all(np.abs(Xg - ref)[diff] <= ulp[diff] * (1 + 1e-6) + 1e-38)
    # training targets: the undamped step r / s in the network's units, clipped
    T = torch.empty(lev.n, dtype=torch.float32, device="cuda")
    cpm.cpm_smoother_pairs(band, level, 1.0, dev(f), dev(u), X, T, s, 16.0, work)
    safe = np.where(s_ref > 0, s_ref, 1.0)
    t_ref = np.where(s_ref > 0, np.clip(r / safe, -16.0, 16.0), 0.0).astype(np.float32)
    assert np.all(np.abs(host(T) - t_ref) <= 1e-6 * np.abs(t_ref) + 1e-30)


def test_features_match_oracle():
    log("smoother features")
    _features_check(_learned_case(), 0, 5)


def test_features_match_oracle_with_gapped_patch_rows():
    """Level 1 of the torus R = 1, r = 0.25 at h = 1/16 has patch rows whose middle node is
    outside the band while both outer ones are inside."""
    log("smoother features, gapped rows")
    _features_check(_gap_case(), 1, 6)


def _gap_case():
    return W.SolverConfig("torus_r0.25_h16", W.torus_modes(1.0, 0.25, W.SEED_BASE + 50), 1.0 / 16, 3, W.LAM2_3D)


@pytest.mark.parametrize("case", ["sphere16", "torus_gapped"])
def test_learned_vcycles_match_oracle(case):
    """Four learned V-cycles (network on levels 0 and 1) against the oracle's learned cycle,
    iterate by iterate, with a network whose every weight is non-zero and whose cycle
    contracts (a diverging cycle amplifies any rounding difference).  The network runs in
    float32 on the GPU (bf16 MFMA, float32 accumulation of 40 products per hidden unit, 64
    per output) and in float64 in the oracle on the same bf16 inputs and weights, so every
    learned update differs by about 1e-6 of its size; a cycle makes 24 of them (6 sweeps on
    each of two levels, before and after the coarse correction), and the differences add up
    until the cycle's contraction damps them: the iterates agree to 2e-4 relative (measured:
    6e-6 after one cycle, 4e-5 after two); the residual E f - A u weighs those differences by
    A's large diagonal (6/h^2), so the per-cycle residuals agree to 1e-2 relative (measured:
    1.2e-3 after three cycles)."""
    log("learned V-cycle parity %s" % case)
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = _learned_case() if case == "sphere16" else _gap_case()
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    w = _near_jacobi_weights(9)
    ref = ov.solve(H, f, ov.Params(learned=w), rtol=0.0, max_cycles=4, keep_iterates=True)
    assert ref.relres[-1] < 0.1 * ref.relres[0]
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    cpm.cpm_set_smoother_weights(band, w, 10.0)
    p = cpm.make_params(smoother=cpm.CPM_SMOOTH_LEARNED)
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    for k in range(4):
        st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=0.0, max_cycles=1, raise_on_noconv=False)
        assert st.cycles == 1 and st.fallback_cycle < 0
        err = rel_inf(host(ud), ref.iterates[k])
        log("cycle %d: rel diff %.3e, relres %.4e vs %.4e" % (k, err, st.relres, ref.relres[k]))
        assert err < 2e-4, (k, err)
        assert abs(st.relres - ref.relres[k]) <= 1e-2 * ref.relres[k]


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
