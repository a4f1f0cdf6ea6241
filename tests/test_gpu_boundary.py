"""Calls of the C boundary beyond the solver: the reach flag of cpm_band_info, the float32
operator application, and a registered device allocator (torch's caching allocator)."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import vcycle as ov
from tests.gpu_util import build_gpu, dev, host, log, oracle_for, rel_inf, torch_cuda, workspace

pytestmark = pytest.mark.gpu


def test_band_info_flags_levels_beyond_the_reach():
    """sqrt(17) h >= reach (Sec. 2.1): the unit sphere's reach is 1, so only h = 1/4 of the
    h = 1/64 .. 1/4 hierarchy is flagged; the torus R = 1, r = 0.4 has reach 0.4, so h = 1/8 is
    flagged and h = 1/16 is not."""
    import paper_1307_4354_amd as cpm

    torch_cuda()
    cfg = W.config_sphere(64, 5)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    assert [band.flags(l) & cpm.CPM_BAND_BEYOND_REACH for l in range(5)] == [0, 0, 0, 0, 1]
    cfg = W.config_torus_mixed(32, 3)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    assert [band.flags(l) & cpm.CPM_BAND_BEYOND_REACH for l in range(3)] == [0, 0, 1]
    # the level set: its largest principal curvature is about 10.1 (radius 0.099), so
    # sqrt(17) h reaches it from h = 1/32 on (0.129) but not at h = 1/64 (0.064)
    band = build_gpu(W.dziuk_surface(), 1 / 64, 3, W.LAM2_3D)
    assert [band.flags(l) & 1 for l in range(3)] == [0, 1, 1]


@pytest.mark.parametrize("name,cfg", [("circle64", W.config_circle(64, 4)), ("sphere32", W.config_sphere(32, 4))],
                         ids=["circle64", "sphere32"])
def test_apply_float32_matches_oracle(name, cfg):
    """A u in float32 (float vectors, float arithmetic) against the oracle's float64 product:
    the relative error is float32 rounding of a 64-term interpolation of N u (scale 1/h^2)."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    H = oracle_for(cfg)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    for l in range(band.levels):
        lev = H.levels[l]
        u = W.random_vector(lev.n, 60 + l).astype(np.float32)
        delta = ov.delta(H, l, 1.0)
        u64 = u.astype(np.float64)
        ref = delta * u64 - H.E[l] @ (H.N[l] @ u64)
        ud = dev(u)
        out = torch.empty_like(ud)
        work = torch.empty_like(ud)
        cpm.cpm_apply(band, l, 1.0, ud, out, work)
        assert out.dtype == torch.float32
        err = np.max(np.abs(host(out).astype(np.float64) - ref)) / (delta * np.max(np.abs(u64)))
        assert err < 1e-5, (l, err)


def test_torch_allocator_backs_the_band():
    """With torch's caching allocator registered, a band's arrays come from it (torch's count
    of allocated bytes grows by them and returns when the band is freed) and the solve is the
    oracle's."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_sphere(32, 4)
    H = oracle_for(cfg)
    f = cfg.problem.f(H.levels[0].cp)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    cpm.use_torch_allocator(True)
    try:
        band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
        m1 = torch.cuda.memory_allocated()
        log("band arrays through torch: %d bytes" % (m1 - m0))
        assert m1 - m0 > 100 * band.n(0)  # index tables and fractions of every level
        p = cpm.make_params()
        work, nbytes = workspace(band, p)
        fd = dev(f)
        ud = torch.zeros_like(fd)
        st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
        ref = ov.solve(H, f, ov.Params(), rtol=1e-10, max_cycles=60)
        assert st.cycles == ref.cycles and rel_inf(host(ud), ref.u) < 1e-12
        del work, fd, ud
        band.free()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == m0
    finally:
        cpm.use_torch_allocator(False)
    # one function without the other is refused
    fn = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)(lambda c, n: None)
    with pytest.raises(cpm.CpmError):
        cpm.cpm_set_allocator(fn, None)
