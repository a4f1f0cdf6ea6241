"""Helpers shared by the GPU tests: build a band through the C ABI for a workload, move
seeded inputs to the device, and build the matching oracle hierarchy."""
from __future__ import annotations

import functools
import sys

import numpy as np

import workloads as W


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def surface_args(s: W.Surface):
    import paper_1307_4354_amd as cpm

    return cpm.make_surface(s.kind, s.R, s.r, s.center)


def build_gpu(s: W.Surface, h0: float, levels: int, lam2: float = 0.0):
    import paper_1307_4354_amd as cpm

    return cpm.cpm_build_band(surface_args(s), h0, levels, lam2)


def dev(x, dtype=None):
    torch = torch_cuda()
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t):
    torch_cuda().cuda.synchronize()
    return t.detach().cpu().numpy()


def workspace(band, params):
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    nbytes = cpm.cpm_workspace_size(band, params)
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda"), nbytes


@functools.lru_cache(maxsize=8)
def oracle_hierarchy(kind, R, r, center, h0, levels, lam2):
    from oracle import band as ob

    s = W.Surface(kind, R, r, center)
    return ob.build_hierarchy(s, h0, levels, lam2)


def oracle_for(cfg: W.SolverConfig):
    s = cfg.problem.surface
    return oracle_hierarchy(s.kind, s.R, s.r, tuple(s.center), cfg.h0, cfg.levels, cfg.lam2)


def rel_inf(a, b) -> float:
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
