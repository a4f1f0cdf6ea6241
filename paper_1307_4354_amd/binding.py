"""ctypes binding of libcpm.so with the C ABI's names (argument marshalling only).

Device vectors are passed as torch CUDA tensors (or raw integer device addresses);
streams as torch streams (default: torch's current stream) or raw hipStream_t integers.
Every call raises ``CpmError`` when the library returns a non-zero status.  Importing
this module fails loudly if the native library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, byref, c_char_p, c_double, c_int, c_int32, c_int64,
                    c_size_t, c_uint16, c_void_p)
from typing import Optional, Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcpm.so")

CPM_OK, CPM_E_INVALID, CPM_E_BAND, CPM_E_NOMEM, CPM_E_HIP, CPM_E_NOCONV, CPM_E_DIVERGED, CPM_E_WORKSPACE = range(8)
CPM_CIRCLE, CPM_SPHERE, CPM_TORUS, CPM_DZIUK = 0, 1, 2, 3
CPM_F64, CPM_MIXED = 0, 1
CPM_DTYPE_F64, CPM_DTYPE_F32 = 0, 1
CPM_BAND_BEYOND_REACH = 1
CPM_BAND_RESID_SUBSET = 2
CPM_RESIDUAL_CONSISTENT, CPM_RESIDUAL_VERBATIM = 0, 1
CPM_SMOOTH_JACOBI, CPM_SMOOTH_LEARNED, CPM_SMOOTH_STANDARD, CPM_SMOOTH_STANDARD_RB = 0, 1, 2, 3
CPM_MAX_HISTORY = 256
CPM_MLP_IN = 64
CPM_MLP_HIDDEN = 64
CPM_MLP_FEATURES = 39
MLP_WEIGHT_COUNT = 64 * 64 + 64 + 64 + 1


class cpm_surface(Structure):
    _fields_ = [("kind", c_int), ("center", c_double * 3), ("R", c_double), ("r", c_double)]


class cpm_grid(Structure):
    _fields_ = [("h0", c_double), ("levels", c_int), ("lam2", c_double)]


class cpm_params(Structure):
    _fields_ = [("c", c_double), ("nu1", c_int), ("nu2", c_int), ("omega", c_double),
                ("precision", c_int), ("smoother", c_int), ("learned_sweeps", c_int), ("gamma", c_int),
                ("fmg", c_int), ("residual_mode", c_int), ("el_degree", c_int)]


class cpm_stats(Structure):
    _fields_ = [("cycles", c_int), ("relres", c_double), ("relres_history", c_double * CPM_MAX_HISTORY),
                ("fallback_cycle", c_int), ("seconds", c_double), ("tile_block", c_int),
                ("tile_blocks_per_cu", c_int), ("host_syncs", c_int), ("cycles_per_launch", c_int)]

    def history(self):
        return [self.relres_history[k] for k in range(min(self.cycles, CPM_MAX_HISTORY))]


class CpmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("libcpm status %d (%s): %s" % (status, _lib.cpm_status_string(status).decode(), message))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcpm.so is not built (run paper_1307_4354_amd.build.build()); "
                          "there is no non-native fallback")
    # torch ships its own HIP runtime (soname libamdhip64.so.7).  Loading torch first makes
    # libcpm bind to that same runtime instead of a second copy from the ROCm install, so
    # torch-allocated memory and torch streams are valid handles for libcpm.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    sigs = {
        "cpm_status_string": (c_char_p, [c_int]),
        "cpm_last_error": (c_char_p, []),
        "cpm_build_band": (c_int, [POINTER(cpm_surface), POINTER(cpm_grid), vp, POINTER(vp)]),
        "cpm_band_free": (c_int, [vp]),
        "cpm_build_bands": (c_int, [c_int, POINTER(cpm_surface), POINTER(cpm_grid), vp, POINTER(vp)]),
        "cpm_band_levels": (c_int, [vp, POINTER(c_int), POINTER(c_int)]),
        "cpm_band_info": (c_int, [vp, c_int, POINTER(c_int64), POINTER(c_double), POINTER(c_int)]),
        "cpm_set_allocator": (c_int, [vp, vp, vp]),
        "cpm_band_export": (c_int, [vp, c_int, vp, vp]),
        "cpm_band_export_stencils": (c_int, [vp, c_int, vp, vp, vp, vp]),
        "cpm_workspace_size": (c_int, [vp, POINTER(cpm_params), POINTER(c_size_t)]),
        "cpm_apply": (c_int, [vp, c_int, c_int, c_double, vp, vp, vp, vp]),
        "cpm_apply_pq": (c_int, [vp, c_int, c_int, c_double, vp, vp, vp, vp]),
        "cpm_apply_static": (c_int, [vp, c_int, c_int, c_double, vp, vp, vp]),
        "cpm_extend": (c_int, [vp, c_int, vp, vp, vp]),
        "cpm_vcycle": (c_int, [vp, POINTER(cpm_params), vp, vp, vp, c_size_t, POINTER(c_double), vp]),
        "cpm_solve": (c_int, [vp, POINTER(cpm_params), vp, vp, vp, c_size_t, c_double, c_int,
                              POINTER(cpm_stats), vp]),
        "cpm_run_cycles": (c_int, [vp, POINTER(cpm_params), vp, vp, vp, c_size_t, c_int, c_int, vp, vp]),
        "cpm_time_kernel": (c_int, [vp, POINTER(cpm_params), c_int, c_int, c_int, vp, vp, vp, c_size_t,
                                    POINTER(c_double), vp]),
        "cpm_workspace_size_batched": (c_int, [c_int, POINTER(vp), POINTER(cpm_params), POINTER(c_size_t)]),
        "cpm_solve_batched": (c_int, [c_int, POINTER(vp), POINTER(cpm_params), POINTER(vp), POINTER(vp), vp,
                                      c_size_t, c_double, c_int, POINTER(cpm_stats), vp]),
        "cpm_autotune": (c_int, [vp, vp]),
        "cpm_set_band_tuning": (c_int, [vp, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int]),
        "cpm_band_tuning": (c_int, [vp, c_int, POINTER(c_int), POINTER(c_int), POINTER(c_int), POINTER(c_int),
                                    POINTER(c_int), POINTER(c_int), POINTER(c_int), POINTER(c_int), POINTER(c_int)]),
        "cpm_set_smoother_weights": (c_int, [vp, vp, c_double]),
        "cpm_set_diffusion": (c_int, [vp, c_int, vp]),
        "cpm_mlp_forward": (c_int, [c_int64, vp, vp, vp, vp, vp]),
        "cpm_mlp_backward": (c_int, [c_int64, vp, vp, vp, vp, vp, vp, vp]),
        "cpm_mlp_adam": (c_int, [c_int, ctypes.c_float, vp, vp, vp, vp, vp, vp]),
        "cpm_smoother_features": (c_int, [vp, c_int, c_double, vp, vp, vp, vp, vp, vp]),
        "cpm_smoother_pairs": (c_int, [vp, c_int, c_double, vp, vp, vp, vp, vp, c_double, vp, vp]),
        "cpm_mlp_loss": (c_int, [c_int64, vp, vp, vp, vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def exported_symbols() -> Sequence[str]:
    return [n for n in dir(_lib) if n.startswith("cpm_")]


def _check(st: int) -> None:
    if st != CPM_OK:
        raise CpmError(st, (_lib.cpm_last_error() or b"").decode())


def _ptr(x) -> Optional[int]:
    """Device address of a torch tensor (checked contiguous) or an int; None -> NULL."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    raise TypeError("expected a tensor, an int address or None")


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


_KINDS = {"circle": CPM_CIRCLE, "sphere": CPM_SPHERE, "torus": CPM_TORUS, "dziuk": CPM_DZIUK}


def make_surface(kind, R: float, r: float = 0.0, center=(0.0, 0.0, 0.0)) -> cpm_surface:
    k = _KINDS[kind] if isinstance(kind, str) else int(kind)
    c = list(center) + [0.0] * (3 - len(center))
    return cpm_surface(k, (c_double * 3)(*c[:3]), float(R), float(r))


def make_params(c: float = 1.0, nu1: int = 3, nu2: int = 3, omega: float = 2.0 / 3.0,
                precision: int = CPM_F64, smoother: int = CPM_SMOOTH_JACOBI, learned_sweeps: int = 0,
                gamma: int = 1, fmg: bool = False, residual_mode: int = 0, el_degree: int = 0) -> cpm_params:
    return cpm_params(float(c), int(nu1), int(nu2), float(omega), int(precision), int(smoother),
                      int(learned_sweeps), int(gamma), int(bool(fmg)), int(residual_mode), int(el_degree))


class Band:
    """Owning wrapper of a cpm_band handle."""

    def __init__(self, handle: int):
        self.handle = handle
        L, d = c_int(), c_int()
        _check(_lib.cpm_band_levels(handle, byref(L), byref(d)))
        self.levels = L.value
        self.dim = d.value

    def n(self, level: int = 0) -> int:
        n = c_int64()
        _check(_lib.cpm_band_info(self.handle, level, byref(n), None, None))
        return n.value

    def h(self, level: int = 0) -> float:
        h = c_double()
        _check(_lib.cpm_band_info(self.handle, level, None, byref(h), None))
        return h.value

    def flags(self, level: int = 0) -> int:
        fl = c_int()
        _check(_lib.cpm_band_info(self.handle, level, None, None, byref(fl)))
        return fl.value

    def sizes(self):
        return [self.n(l) for l in range(self.levels)]

    def export(self, level: int = 0):
        n = self.n(level)
        idx = np.empty((n, self.dim), dtype=np.int32)
        cp = np.empty((n, self.dim), dtype=np.float64)
        _check(_lib.cpm_band_export(self.handle, level, idx.ctypes.data, cp.ctypes.data))
        return idx, cp

    def export_stencils(self, level: int = 0):
        n, d = self.n(level), self.dim
        runE = np.empty((n, 4 ** (d - 1)), dtype=np.int32)
        nbr = np.empty((n, 2 * d), dtype=np.int32)
        runP = np.full((n, 2 ** (d - 1)), -1, dtype=np.int32)
        runR = np.full((n, 2 ** (d - 1)), -1, dtype=np.int32)
        _check(_lib.cpm_band_export_stencils(self.handle, level, runE.ctypes.data, nbr.ctypes.data,
                                             runP.ctypes.data, runR.ctypes.data))
        return runE, nbr, runP, runR

    def free(self):
        if self.handle:
            _lib.cpm_band_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


_ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_void_p, c_size_t)
_FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)
_allocator_keepalive = None


def cpm_set_allocator(alloc, release, ctx=None) -> None:
    """Register device allocation functions (C function pointers as ints, ctypes callbacks, or
    None for both to restore hipMalloc / hipFree) for the arrays of bands built afterwards."""
    a = ctypes.cast(alloc, c_void_p) if alloc is not None else None
    r = ctypes.cast(release, c_void_p) if release is not None else None
    _check(_lib.cpm_set_allocator(a, r, ctx))


def use_torch_allocator(enable: bool = True) -> None:
    """Back the arrays of bands built afterwards with torch's caching allocator (or restore
    hipMalloc / hipFree).  The callbacks only forward the sizes and addresses."""
    global _allocator_keepalive
    if not enable:
        cpm_set_allocator(None, None)
        _allocator_keepalive = None
        return
    import torch

    def _alloc(ctx, nbytes):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except RuntimeError:
            return None

    def _free(ctx, ptr):
        torch.cuda.caching_allocator_delete(int(ptr))

    fa, ff = _ALLOC_FN(_alloc), _FREE_FN(_free)
    _allocator_keepalive = (fa, ff)  # the library keeps the raw pointers
    cpm_set_allocator(fa, ff)


def cpm_build_band(surface: cpm_surface, h0: float, levels: int, lam2: float = 0.0, stream=None) -> Band:
    g = cpm_grid(float(h0), int(levels), float(lam2))
    out = c_void_p()
    _check(_lib.cpm_build_band(byref(surface), byref(g), _stream(stream) if stream is not None else None,
                               byref(out)))
    return Band(out.value)


def cpm_build_bands(surfaces: Sequence[cpm_surface], grids: Sequence[tuple], stream=None):
    """Build several bands at once; grids are (h0, levels, lam2) tuples."""
    n = len(surfaces)
    sa = (cpm_surface * n)(*surfaces)
    ga = (cpm_grid * n)(*[cpm_grid(float(h0), int(L), float(lam2)) for h0, L, lam2 in grids])
    out = (c_void_p * n)()
    _check(_lib.cpm_build_bands(n, sa, ga, _stream(stream) if stream is not None else None, out))
    return [Band(out[k]) for k in range(n)]


def cpm_band_free(band: Band) -> None:
    band.free()


def cpm_workspace_size(band: Band, params: cpm_params) -> int:
    b = c_size_t()
    _check(_lib.cpm_workspace_size(band.handle, byref(params), byref(b)))
    return b.value


def cpm_apply(band: Band, level: int, c: float, u, Au, work, stream=None) -> None:
    """Au = A u on one level; the vectors' element type (float64 or float32 tensors) selects
    the precision."""
    import torch

    dt = CPM_DTYPE_F32 if getattr(u, "dtype", None) == torch.float32 else CPM_DTYPE_F64
    _check(_lib.cpm_apply(band.handle, level, dt, float(c), _ptr(u), _ptr(Au), _ptr(work), _stream(stream)))


def cpm_apply_pq(band: Band, level: int, p: int, c: float, u, Au, work, stream=None) -> None:
    _check(_lib.cpm_apply_pq(band.handle, level, int(p), float(c), _ptr(u), _ptr(Au), _ptr(work), _stream(stream)))


def cpm_apply_static(band: Band, level: int, c: float, u, Au, stream=None) -> None:
    """cpm_apply without a workspace argument (the library's static scratch array)."""
    import torch

    dt = CPM_DTYPE_F32 if getattr(u, "dtype", None) == torch.float32 else CPM_DTYPE_F64
    _check(_lib.cpm_apply_static(band.handle, level, dt, float(c), _ptr(u), _ptr(Au), _stream(stream)))


def cpm_extend(band: Band, level: int, g, out, stream=None) -> None:
    _check(_lib.cpm_extend(band.handle, level, _ptr(g), _ptr(out), _stream(stream)))


def cpm_set_diffusion(band: Band, level: int, a) -> None:
    """Variable diffusion coefficient a(cp(x_i)) on one level (host float64 array of n(level)
    values, copied); a = None removes it from every level."""
    if a is None:
        _check(_lib.cpm_set_diffusion(band.handle, int(level), None))
        return
    arr = np.ascontiguousarray(a, dtype=np.float64)
    if arr.shape != (band.n(level),):
        raise ValueError("coefficient must have n(level) = %d values" % band.n(level))
    _check(_lib.cpm_set_diffusion(band.handle, int(level), arr.ctypes.data_as(c_void_p)))


def cpm_vcycle(band: Band, params: cpm_params, f, u, work, work_bytes: int, want_relres: bool = False,
               stream=None) -> Optional[float]:
    rr = c_double(0.0)
    _check(_lib.cpm_vcycle(band.handle, byref(params), _ptr(f), _ptr(u), _ptr(work), work_bytes,
                           byref(rr) if want_relres else None, _stream(stream)))
    return rr.value if want_relres else None


def cpm_solve(band: Band, params: cpm_params, f, u, work, work_bytes: int, rtol: float = 1e-10,
              max_cycles: int = 100, stream=None, raise_on_noconv: bool = True) -> cpm_stats:
    st = cpm_stats()
    status = _lib.cpm_solve(band.handle, byref(params), _ptr(f), _ptr(u), _ptr(work), work_bytes, float(rtol),
                            int(max_cycles), byref(st), _stream(stream))
    if status != CPM_OK and (raise_on_noconv or status != CPM_E_NOCONV):
        _check(status)
    st.status = status
    return st


def cpm_run_cycles(band: Band, params: cpm_params, f, u, work, work_bytes: int, cycles: int,
                   cycles_per_launch: int, relres_dev, stream=None) -> None:
    if hasattr(relres_dev, "numel") and relres_dev.numel() < cycles:
        raise ValueError("relres_dev holds %d values, %d cycles record one each" % (relres_dev.numel(), cycles))
    _check(_lib.cpm_run_cycles(band.handle, byref(params), _ptr(f), _ptr(u), _ptr(work), work_bytes, int(cycles),
                               int(cycles_per_launch), _ptr(relres_dev), _stream(stream)))


def cpm_workspace_size_batched(bands: Sequence[Band], params: cpm_params) -> int:
    arr = (c_void_p * len(bands))(*[b.handle for b in bands])
    out = c_size_t()
    _check(_lib.cpm_workspace_size_batched(len(bands), arr, byref(params), byref(out)))
    return out.value


def cpm_solve_batched(bands: Sequence[Band], params: cpm_params, fs, us, work, work_bytes: int,
                      rtol: float = 1e-10, max_cycles: int = 100, stream=None, raise_on_noconv: bool = True):
    nb = len(bands)
    arr = (c_void_p * nb)(*[b.handle for b in bands])
    fp = (c_void_p * nb)(*[_ptr(f) for f in fs])
    up = (c_void_p * nb)(*[_ptr(u) for u in us])
    stats = (cpm_stats * nb)()
    status = _lib.cpm_solve_batched(nb, arr, byref(params), fp, up, _ptr(work), work_bytes, float(rtol),
                                    int(max_cycles), stats, _stream(stream))
    if status != CPM_OK and (raise_on_noconv or status != CPM_E_NOCONV):
        _check(status)
    return status, list(stats)


def cpm_autotune(band: Band, stream=None) -> None:
    _check(_lib.cpm_autotune(band.handle, _stream(stream)))


def cpm_set_smoother_weights(band: Band, w_bf16: np.ndarray, rho_plain: float) -> None:
    w = np.ascontiguousarray(w_bf16, dtype=np.uint16)
    if w.size != MLP_WEIGHT_COUNT:
        raise ValueError("expected %d bf16 weights" % MLP_WEIGHT_COUNT)
    _check(_lib.cpm_set_smoother_weights(band.handle, w.ctypes.data, float(rho_plain)))


def cpm_mlp_forward(m: int, X, W, Y, H=None, stream=None) -> None:
    _check(_lib.cpm_mlp_forward(int(m), _ptr(X), _ptr(W), _ptr(Y), _ptr(H), _stream(stream)))


def cpm_mlp_backward(m: int, X, W, H, Y, T, G, stream=None) -> None:
    _check(_lib.cpm_mlp_backward(int(m), _ptr(X), _ptr(W), _ptr(H), _ptr(Y), _ptr(T), _ptr(G), _stream(stream)))


def cpm_smoother_features(band: Band, level: int, c: float, f, u, X, s, work, stream=None) -> None:
    _check(_lib.cpm_smoother_features(band.handle, level, float(c), _ptr(f), _ptr(u), _ptr(X), _ptr(s), _ptr(work),
                                      _stream(stream)))


def cpm_smoother_pairs(band: Band, level: int, c: float, f, u, X, T, s, clip: float, work, stream=None) -> None:
    _check(_lib.cpm_smoother_pairs(band.handle, level, float(c), _ptr(f), _ptr(u), _ptr(X), _ptr(T), _ptr(s),
                                   float(clip), _ptr(work), _stream(stream)))


def cpm_mlp_loss(m: int, Y, T, loss, stream=None) -> None:
    _check(_lib.cpm_mlp_loss(int(m), _ptr(Y), _ptr(T), _ptr(loss), _stream(stream)))


def cpm_time_kernel(band: Band, params: cpm_params, which: int, level: int, reps: int, f, u, work,
                    work_bytes: int, stream=None) -> float:
    """Average launch duration (microseconds) of one V-cycle kernel, timed with HIP events."""
    us = c_double()
    _check(_lib.cpm_time_kernel(band.handle, byref(params), int(which), int(level), int(reps), _ptr(f), _ptr(u),
                                _ptr(work), work_bytes, byref(us), _stream(stream)))
    return us.value


def cpm_mlp_adam(step: int, lr: float, w_master, m1, m2, G, w_bf16, stream=None) -> None:
    _check(_lib.cpm_mlp_adam(int(step), float(lr), _ptr(w_master), _ptr(m1), _ptr(m2), _ptr(G), _ptr(w_bf16),
                             _stream(stream)))


def cpm_set_band_tuning(band: Band, level: int, use_lds: bool, ext_block: int, nsum_block: int, fused: bool,
                        sweep_block: int, sweep_lds: bool, tiled: bool = False, ext_prefetch: bool = False) -> None:
    """Pin one level's launch configuration (the fields cpm_band_tuning reports)."""
    _check(_lib.cpm_set_band_tuning(band.handle, int(level), int(bool(use_lds)), int(ext_block), int(nsum_block),
                                    int(bool(fused)), int(sweep_block), int(bool(sweep_lds)), int(bool(tiled)),
                                    int(bool(ext_prefetch))))


def cpm_band_tuning(band: Band, level: int):
    """(use_lds, ext_block, nsum_block, fused, sweep_block, sweep_lds, tiled, ext_prefetch) of one level."""
    v = [c_int() for _ in range(9)]
    _check(_lib.cpm_band_tuning(band.handle, int(level), *[byref(x) for x in v]))
    a, b, c, d, e, g, t, pf, _ = [x.value for x in v]
    return bool(a), b, c, bool(d), e, bool(g), bool(t), bool(pf)


def cpm_band_ext_slots(band: Band, level: int) -> int:
    """Stencil slots per workgroup of the LDS-staged extension on one level (cpm_band_tuning's
    ext_slots; 0 without the staging tables)."""
    v = c_int()
    z = [None] * 8
    _check(_lib.cpm_band_tuning(band.handle, int(level), *z, byref(v)))
    return v.value
