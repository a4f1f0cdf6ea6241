"""cpm_apply_static: the operator application that allocates nothing (its work vector is a
static device array) gives cpm_apply's result bit for bit, on two calls in a row (the second
on a smaller level), in both precisions; a level too large for the static array is refused."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import build_gpu, dev, host, log, torch_cuda

pytestmark = pytest.mark.gpu


def test_apply_static_equals_apply():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_sphere(32, 4)
    band = build_gpu(cfg.problem.surface, cfg.h0, cfg.levels, cfg.lam2)
    for dtype in (torch.float64, torch.float32):
        for level in (0, 1):  # the second call on a smaller level reuses the scratch array
            n = band.n(level)
            log("apply_static level %d n %d %s" % (level, n, dtype))
            u = dev(W.random_vector(n, 31 + level)).to(dtype)
            ref = torch.empty_like(u)
            work = torch.empty_like(u)
            cpm.cpm_apply(band, level, 1.0, u, ref, work)
            out = torch.full_like(u, float("nan"))
            cpm.cpm_apply_static(band, level, 1.0, u, out)
            assert np.array_equal(host(out), host(ref)), (level, dtype)


def test_apply_static_refuses_a_level_beyond_its_scratch():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_sphere(256, 2)  # 6.8 M nodes: 54 MB of double work space > 32 MiB
    band = build_gpu(cfg.problem.surface, cfg.h0, 2, cfg.lam2)
    n = band.n(0)
    u = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(cpm.CpmError) as ei:
        cpm.cpm_apply_static(band, 0, 1.0, u, torch.empty_like(u))
    assert ei.value.status == cpm.CPM_E_WORKSPACE
    # the smaller coarse level fits
    n1 = band.n(1)
    u1 = dev(W.random_vector(n1, 5))
    ref, out, work = torch.empty_like(u1), torch.empty_like(u1), torch.empty_like(u1)
    cpm.cpm_apply(band, 1, 1.0, u1, ref, work)
    cpm.cpm_apply_static(band, 1, 1.0, u1, out)
    assert np.array_equal(host(out), host(ref))
