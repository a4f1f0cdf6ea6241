"""Pins of the learned-smoother network reference (CPU, no GPU)."""
import numpy as np
import pytest

import workloads as W
from oracle import band as ob
from oracle import mlp as om
from oracle import vcycle as ov


def test_bf16_rounding_matches_definition():
    x = np.array([1.0, 1.00390625, 1.005859375, -3.0e-3, 65504.0, 1e-30], dtype=np.float32)
    b = om.bf16_bits(x)
    back = om.from_bf16_bits(b)
    # nearest representable with 8 significant bits, ties to even
    assert back[0] == 1.0
    assert back[1] == 1.0  # 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even (1.0)
    assert back[2] == np.float32(1.0078125)
    assert abs(back[3] - (-3.0e-3)) <= 2 ** -8 * 3.0e-3
    assert np.all(np.abs(back - x) <= np.abs(x) * 2 ** -8 + 1e-45)


def test_jacobi_weights_reproduce_damped_jacobi():
    """The network with jacobi_weights returns omega * x_centre exactly (in bf16 arithmetic)."""
    rng = np.random.default_rng(0)
    X = om.bf16_round(rng.uniform(-1, 1, (100, om.N_IN)).astype(np.float32))
    for dim, centre in ((3, 13), (2, 4)):
        w = om.jacobi_weights(2.0 / 3.0, dim)
        y, _ = om.forward(X, w)
        omega_bf = float(om.from_bf16_bits(om.bf16_bits(np.array([2.0 / 3.0], np.float32)))[0])
        assert np.allclose(y, omega_bf * X[:, centre].astype(np.float64), rtol=1e-12, atol=1e-15)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    m = 37
    X = om.bf16_round(rng.uniform(-1, 1, (m, om.N_IN)).astype(np.float32)).astype(np.float64)
    T = rng.standard_normal(m)
    W1 = rng.standard_normal((om.N_HID, om.N_IN)) * 0.2
    b1 = rng.standard_normal(om.N_HID) * 0.1
    w2 = rng.standard_normal(om.N_HID) * 0.2
    b2 = 0.3
    loss, g = om.loss_and_grad_params(X, T, W1, b1, w2, b2)
    flat = np.concatenate([W1.ravel(), b1, w2, [b2]])
    eps = 1e-6
    for idx in rng.choice(flat.size, 40, replace=False):
        fp = flat.copy()
        fp[idx] += eps
        fm = flat.copy()
        fm[idx] -= eps

        def unpack_f(v):
            return (v[:om.N_HID * om.N_IN].reshape(om.N_HID, om.N_IN), v[om.N_HID * om.N_IN:om.N_HID * om.N_IN + om.N_HID],
                    v[om.N_HID * om.N_IN + om.N_HID:-1], v[-1])

        lp = om.loss_and_grad_params(X, T, *unpack_f(fp))[0]
        lm = om.loss_and_grad_params(X, T, *unpack_f(fm))[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, g[idx])


def test_features_layout_and_zero_residual_fixed_point():
    lev = ob.build_level(W.unit_sphere(), 1 / 8, W.LAM2_3D)
    # residual equal to the node's x index: patch entries differ by the dx offset
    r = lev.idx[:, 0].astype(np.float64) + 100.0
    X, s = om.features(lev, r)
    i = int(np.argmax(np.all(ob.neighbour_indices(lev) >= 0, axis=1)))
    x = lev.idx[i, 0] + 100.0
    patch = X[i, :27].astype(np.float64) * s[i]
    expect = np.tile([x - 1, x, x + 1], 9)
    # interior node: every patch entry present (diagonal neighbours may be absent near edges)
    present = patch != 0
    assert np.allclose(patch[present], expect[present], rtol=2 ** -8)
    assert patch[13] != 0
    # 1-D weights after the patch
    _, W1d, _ = ob.stencil(lev.cp[i:i + 1], lev.h, 3)
    assert np.allclose(X[i, 27:39], om.bf16_round(W1d.reshape(-1).astype(np.float32)))
    assert np.all(X[:, 39:] == 0)
    # zero residual -> zero update, whatever the weights
    rng = np.random.default_rng(2)
    w = om.pack(rng.standard_normal((64, 64)), rng.standard_normal(64), rng.standard_normal(64), 0.7)
    du = om.learned_update(lev, np.zeros(lev.n), 100.0, w)
    assert np.all(du == 0.0)


def test_learned_update_with_jacobi_weights_is_jacobi_step():
    cfg = W.config_sphere(16, 3)
    H = ob.build_hierarchy(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    f = cfg.problem.f(H.levels[0].cp)
    p = ov.Params()
    u = np.random.default_rng(3).standard_normal(H.levels[0].n) * 0.01
    r = ov.residual(H, 0, u, f, p)
    d0 = ov.delta(H, 0, p.c)
    du = om.learned_update(H.levels[0], r, d0, om.jacobi_weights(2.0 / 3.0, 3))
    ref = (2.0 / 3.0) / d0 * r
    assert np.max(np.abs(du - ref)) <= 2 ** -7 * np.max(np.abs(ref))


def test_backward_bf16_is_the_gradient_within_bf16_rounding():
    """The gradient with the hidden error rounded to bfloat16 differs from the exact gradient
    (itself pinned by finite differences) by at most the rounding of each term, 2^-8 of the
    sum of the terms' magnitudes; the other parameters' gradients equal it to float32 rounding."""
    rng = np.random.default_rng(4)
    m = 300
    X = om.bf16_round(rng.uniform(-1, 1, (m, om.N_IN)).astype(np.float32))
    T = rng.standard_normal(m).astype(np.float32)
    w = om.pack(rng.standard_normal((64, 64)) * 0.3, rng.standard_normal(64) * 0.1,
                rng.standard_normal(64) * 0.3, 0.25)
    y, Hh = om.forward(X, w)
    H32, Y32 = Hh.astype(np.float32), y.astype(np.float32)
    g = om.backward_bf16(X, w, H32, Y32, T)
    # exact gradient at the same (float32-rounded) forward values
    W1, b1, w2, b2 = om.unpack(w)
    dy = 2.0 * (Y32.astype(np.float64) - T.astype(np.float64)) / m
    dH = np.outer(dy, w2) * (H32 > 0)
    gW1 = dH.T @ X.astype(np.float64)
    bound = np.abs(dH).T @ np.abs(X.astype(np.float64))
    o = 64 * 64
    assert np.all(np.abs(g[:o] - gW1.ravel()) <= 2 ** -8 * bound.ravel() * (1 + 1e-6) + 1e-12)
    assert np.max(np.abs(g[o:o + 64] - dH.sum(axis=0))) <= 1e-5 * np.max(np.abs(dH.sum(axis=0)))
    # exactly representable hidden errors are not rounded: then dW1 is exact
    w2x = np.zeros(64)
    w2x[:8] = 0.5
    wx = om.pack(W1, b1, w2x, b2)
    Tx = (Y32 - np.float32(m) / np.float32(2.0) * np.float32(0.25)).astype(np.float32)  # dy = 0.25 exactly
    gx = om.backward_bf16(X, wx, H32, Y32, Tx)
    dHx = np.outer(np.full(m, 0.25), om.unpack(wx)[2]) * (H32 > 0)
    assert np.allclose(gx[:o], (dHx.T @ X.astype(np.float64)).ravel(), rtol=1e-12, atol=1e-12)
