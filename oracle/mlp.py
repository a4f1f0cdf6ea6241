"""Reference of the learned local smoother network (not in the paper; it replaces the damped
Ruuth-Merriman Jacobi step of Sec. 4.2 on the two finest levels).

Per node i of a level with spacing h:
  r        A-space residual r = b + E(f + N u) - delta u (b = 0 on coarse levels)
  patch    r at the 3^d grid nodes i + (dx, dy[, dz]), dx fastest, 0 outside the band
  s        max |patch|; the update is 0 when s = 0 (so a zero residual is a fixed point)
  x        [patch / s, the node's 1-D cubic weights (4 per axis, x then y then z), zeros]
           padded to 64 features, rounded to bfloat16
  hidden   relu(W1 x + b1)                   (64 units, W1 is 64 x 64, row = unit)
  y        w2 . hidden + b2
  update   u_i += (s / delta) y

The Jacobi step u_i += (omega/delta) r_i is the special case y = omega * patch_centre / s,
which a network of this shape represents exactly, so the learned step is a generalisation
of the paper's smoother that keeps its scale: y depends only on the normalised patch.

Weights are bfloat16 (round to nearest even on the float32 bits); arithmetic is float32 in
the GPU kernels and float64 here, with the inputs rounded exactly as the kernels round them.
Training outcome: parity unpinned (reported as the contraction gain over Jacobi).
"""
from __future__ import annotations

import numpy as np

from .band import Level, lagrange_weights, stencil

N_IN = 64
N_HID = 64
N_W = N_HID * N_IN + N_HID + N_HID + 1


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float values to bfloat16 (nearest even), returned as float32."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    rounded = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(f), f, out)


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns (uint16) of float values (nearest even)."""
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def unpack(w_bits: np.ndarray):
    w = from_bf16_bits(w_bits).astype(np.float64)
    W1 = w[: N_HID * N_IN].reshape(N_HID, N_IN)
    o = N_HID * N_IN
    b1 = w[o:o + N_HID]
    w2 = w[o + N_HID:o + 2 * N_HID]
    b2 = w[o + 2 * N_HID]
    return W1, b1, w2, b2


def pack(W1, b1, w2, b2) -> np.ndarray:
    flat = np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(w2), [b2]]).astype(np.float32)
    return bf16_bits(flat)


def jacobi_weights(omega: float = 2.0 / 3.0, dim: int = 3) -> np.ndarray:
    """Weights for which the network reproduces the damped Jacobi step exactly:
    y = omega * x_centre via hidden units relu(x_c) - relu(-x_c)."""
    W1 = np.zeros((N_HID, N_IN))
    centre = 13 if dim == 3 else 4
    W1[0, centre] = 1.0
    W1[1, centre] = -1.0
    w2 = np.zeros(N_HID)
    w2[0] = omega
    w2[1] = -omega
    return pack(W1, np.zeros(N_HID), w2, 0.0)


def patch_offsets(dim: int) -> np.ndarray:
    r = (-1, 0, 1)
    if dim == 2:
        return np.array([(dx, dy) for dy in r for dx in r], dtype=np.int64)
    return np.array([(dx, dy, dz) for dz in r for dy in r for dx in r], dtype=np.int64)


def features(lev: Level, r: np.ndarray):
    """(X float32 bf16-rounded (n x 64), s float64 (n)) for residual r on level lev."""
    d = lev.dim
    off = patch_offsets(d)
    n = lev.n
    P = np.zeros((n, off.shape[0]))
    for q, o in enumerate(off):
        j = lev.lookup(lev.idx + o)
        ok = j >= 0
        P[ok, q] = r[j[ok]]
    s = np.max(np.abs(P), axis=1)
    X = np.zeros((n, N_IN), dtype=np.float32)
    # the normalised patch is a quantised input (bfloat16): its rounding is decided in the
    # precision the kernels take it in, float32(r) * (1 / float32(s)) in float32
    s32 = s.astype(np.float32)
    inv = np.where(s32 > 0, np.float32(1.0) / np.where(s32 > 0, s32, np.float32(1.0)), np.float32(0.0))
    X[:, :off.shape[0]] = P.astype(np.float32) * inv[:, None]
    _, W1d, _ = stencil(lev.cp, lev.h, 3)  # (n, d, 4)
    X[:, off.shape[0]:off.shape[0] + 4 * d] = W1d.reshape(n, 4 * d).astype(np.float32)
    return bf16_round(X), s


def forward_params(X: np.ndarray, W1, b1, w2, b2):
    """(y, hidden) in float64 for given (unrounded) parameters."""
    Hpre = X.astype(np.float64) @ np.asarray(W1).T + b1
    H = np.maximum(Hpre, 0.0)
    return H @ w2 + b2, H


def forward(X: np.ndarray, w_bits: np.ndarray):
    """(y, hidden) in float64 from bf16 inputs and weights."""
    return forward_params(X, *unpack(w_bits))


def loss_and_grad_params(X: np.ndarray, T: np.ndarray, W1, b1, w2, b2):
    """Mean squared loss (1/m) sum (y - t)^2 and its gradient w.r.t. (W1, b1, w2, b2),
    flattened in the packing order."""
    y, H = forward_params(X, W1, b1, w2, b2)
    m = X.shape[0]
    dy = 2.0 * (y - T) / m
    gw2 = H.T @ dy
    gb2 = dy.sum()
    dH = np.outer(dy, w2) * (H > 0)
    gW1 = dH.T @ X.astype(np.float64)
    gb1 = dH.sum(axis=0)
    loss = float(np.mean((y - T) ** 2))
    return loss, np.concatenate([gW1.ravel(), gb1, gw2, [gb2]])


def loss_and_grad(X: np.ndarray, T: np.ndarray, w_bits: np.ndarray):
    """loss_and_grad_params at the bf16 weights."""
    return loss_and_grad_params(X, T, *unpack(w_bits))


def learned_update(lev: Level, r: np.ndarray, delta: float, w_bits: np.ndarray) -> np.ndarray:
    """Correction (s/delta) y of one learned smoothing step."""
    X, s = features(lev, r)
    y, _ = forward(X, w_bits)
    return s / delta * y


def backward_bf16(X: np.ndarray, w_bits: np.ndarray, H: np.ndarray, Y: np.ndarray, T: np.ndarray):
    """Gradient of (1/m) sum (y - t)^2 given the forward pass's hidden activations H and
    outputs Y (float32), with the layer-1 weight gradient taken from bfloat16 inputs: the
    per-node output error dy = (2/m)(y - t) and the hidden error dh = dy w2 [h > 0] are formed
    in float32, dh is rounded to bfloat16 (the matrix cores' input type), and
    dW1 = sum_i dh_i x_i^T is summed exactly (float64).  b1, w2, b2 take the unrounded float32
    dh, dy.  Returns the gradient in packing order (float64)."""
    _, _, w2, _ = unpack(w_bits)
    m = X.shape[0]
    f32 = np.float32
    H32 = np.asarray(H, dtype=f32)
    dy = (f32(2.0) / f32(m)) * (np.asarray(Y, dtype=f32) - np.asarray(T, dtype=f32))
    dh = np.where(H32 > 0, dy[:, None] * w2.astype(f32)[None, :], f32(0.0)).astype(f32)
    dh_bf = bf16_round(dh).astype(np.float64)
    gW1 = dh_bf.T @ np.asarray(X, dtype=np.float64)
    gb1 = dh.astype(np.float64).sum(axis=0)
    gw2 = H32.astype(np.float64).T @ dy.astype(np.float64)
    gb2 = float(dy.astype(np.float64).sum())
    return np.concatenate([gW1.ravel(), gb1, gw2, [gb2]])
