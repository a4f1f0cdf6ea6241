"""Training driver of the learned smoother (argument marshalling around libcpm's kernels).

Training pairs come from the plain solver itself: plain V-cycles are run from u = 0 on
random problems; for every iterate the solver reaches (the start of each cycle, and the
state after pre-smoothing and coarse-grid correction, which is what the post-smoother
sees) the library writes the network features of every node (normalised residual patch
and interpolation weights) and the patch scale s.  The target is the correction of one
undamped Ruuth-Merriman step from that state, in the network's units:
t_i = r_i / s_i with r = E f - A w (the step moves w_i by r_i / delta).  It is a function
of the features the network sees, so the regression is well posed and its minimiser is
a stable smoother; the library computes these targets (cpm_smoother_pairs) and the loss
(cpm_mlp_loss).  Targets that ask one local step to do the work of several sweeps, or
to predict the total error u* - w, need information outside the 3^d residual patch; the
networks fitted to them gave V-cycles that diverge.  Forward, backward and the Adam update
all run in the library's kernels; torch only holds device memory and draws the minibatch
indices.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

from . import binding as cpm

N_IN = cpm.CPM_MLP_IN
N_W = cpm.MLP_WEIGHT_COUNT


def _torch():
    import torch

    return torch


def _bf16_bits(x: np.ndarray) -> np.ndarray:
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    return (((b + 0x7FFF + ((b >> 16) & 1)) >> 16)).astype(np.uint16)


def jacobi_init(omega: float, dim: int, seed: int, noise: float = 0.05) -> np.ndarray:
    """float32 master weights equal to the damped Jacobi network plus small random hidden
    units (so every unit starts active on part of the data)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((64, 64)) * noise
    b1 = np.full(64, 0.01)
    w2 = rng.standard_normal(64) * noise * 0.1
    centre = 13 if dim == 3 else 4
    W1[0, :] = 0.0
    W1[1, :] = 0.0
    W1[0, centre] = 1.0
    W1[1, centre] = -1.0
    b1[0] = b1[1] = 0.0
    w2[0] = omega
    w2[1] = -omega
    return np.concatenate([W1.ravel(), b1, w2, [0.0]]).astype(np.float32)


@dataclass
class Pairs:
    X: object  # torch uint16 (N x 64) on the GPU
    T: object  # torch float32 (N)


def generate_pairs(problems: Sequence[Tuple[object, float, int]], cycles: int = 4, clip: float = 16.0,
                   nu1: int = 3, omega: float = 2.0 / 3.0) -> Pairs:
    """problems: (workloads.Problem, h0, levels).  Returns features / targets of the
    finest level for every node with a non-zero residual patch, from the iterates of
    ``cycles`` plain V(nu1, nu1) cycles (two states per cycle)."""
    torch = _torch()
    Xs, Ts = [], []
    for prob, h0, levels in problems:
        s = prob.surface
        band = cpm.cpm_build_band(cpm.make_surface(s.kind, s.R, s.r, s.center), h0, levels)
        _, cp = band.export(0)
        n = band.n(0)
        f = torch.as_tensor(prob.f(cp)).to("cuda")
        p = cpm.make_params(c=prob.c, nu1=nu1, nu2=nu1, omega=omega)
        pre = cpm.make_params(c=prob.c, nu1=nu1, nu2=0, omega=omega)
        nbytes = cpm.cpm_workspace_size(band, p)
        work = torch.empty(max(nbytes, 16 * n), dtype=torch.uint8, device="cuda")
        u = torch.zeros_like(f)
        X = torch.empty((n, N_IN), dtype=torch.int16, device="cuda")
        t = torch.empty(n, dtype=torch.float32, device="cuda")
        sc = torch.empty(n, dtype=torch.float32, device="cuda")

        def add(w):
            cpm.cpm_smoother_pairs(band, 0, prob.c, f, w, X, t, sc, clip, work)
            keep = sc > 0  # nodes whose residual patch is not zero
            Xs.append(X[keep].clone())
            Ts.append(t[keep].clone())

        for _ in range(cycles):
            add(u)
            w = u.clone()
            cpm.cpm_vcycle(band, pre, f, w, work, nbytes)
            add(w)
            cpm.cpm_vcycle(band, p, f, u, work, nbytes)
        band.free()
    return Pairs(torch.cat(Xs), torch.cat(Ts))


@dataclass
class TrainResult:
    w_bits: np.ndarray
    losses: List[float]


def train(pairs: Pairs, steps: int = 2000, batch: int = 65536, lr: float = 1e-3, seed: int = 0,
          omega: float = 2.0 / 3.0, dim: int = 3, log_every: int = 100) -> TrainResult:
    """Adam on minibatches drawn uniformly from the pairs; forward, backward and the update
    run in libcpm's kernels (BF16 MFMA, float32 accumulation)."""
    torch = _torch()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    N = pairs.X.shape[0]
    w = torch.as_tensor(jacobi_init(omega, dim, seed)).to("cuda")
    m1 = torch.zeros_like(w)
    m2 = torch.zeros_like(w)
    wb = torch.as_tensor(_bf16_bits(w.cpu().numpy()).view(np.int16)).to("cuda")
    G = torch.zeros_like(w)
    Y = torch.empty(batch, dtype=torch.float32, device="cuda")
    Hh = torch.empty((batch, 64), dtype=torch.float32, device="cuda")
    loss_d = torch.zeros(1, dtype=torch.float64, device="cuda")
    losses = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, N, (batch,), device="cuda", generator=gen)
        Xb = pairs.X[idx].contiguous()
        Tb = pairs.T[idx].contiguous()
        cpm.cpm_mlp_forward(batch, Xb, wb, Y, Hh)
        cpm.cpm_mlp_backward(batch, Xb, wb, Hh, Y, Tb, G)
        cpm.cpm_mlp_adam(step, lr, w, m1, m2, G, wb)
        if step % log_every == 0 or step == 1:
            cpm.cpm_mlp_loss(batch, Y, Tb, loss_d)
            losses.append(float(loss_d.item()))
    return TrainResult(wb.cpu().numpy().view(np.uint16).copy(), losses)


def evaluate_loss(pairs: Pairs, w_bits: np.ndarray, limit: int = 1 << 20) -> float:
    torch = _torch()
    n = min(limit, pairs.X.shape[0])
    wb = torch.as_tensor(np.asarray(w_bits, dtype=np.uint16).view(np.int16)).to("cuda")
    Y = torch.empty(n, dtype=torch.float32, device="cuda")
    loss_d = torch.zeros(1, dtype=torch.float64, device="cuda")
    cpm.cpm_mlp_forward(n, pairs.X[:n].contiguous(), wb, Y, None)
    cpm.cpm_mlp_loss(n, Y, pairs.T[:n].contiguous(), loss_d)
    return float(loss_d.item())
