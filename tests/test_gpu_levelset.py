"""The level-set example (Dziuk's surface) on the GPU: the band (indices and Newton closest
points) equals the oracle's bit for bit, the V-cycle iterates match within 1e-12, and the
solve reaches 1e-10 in the oracle's number of cycles with a second-order accurate limit."""
import numpy as np
import pytest

import workloads as W
from oracle import vcycle as ov
from tests.gpu_util import build_gpu, dev, host, log, oracle_for, rel_inf, torch_cuda, workspace

pytestmark = pytest.mark.gpu

CFG = W.config_dziuk(32, 3)


def test_levelset_band_bitexact():
    log("level-set band: Dziuk h = 1/32, 3 levels")
    torch_cuda()
    H = oracle_for(CFG)
    band = build_gpu(CFG.problem.surface, CFG.h0, CFG.levels, CFG.lam2)
    for l, lev in enumerate(H.levels):
        idx, cp = band.export(l)
        assert idx.shape == lev.idx.shape
        assert np.array_equal(idx, lev.idx), l
        assert np.array_equal(cp, lev.cp), l


@pytest.mark.parametrize("sweep", ["split", "fused"])
def test_levelset_iterates_and_solve(sweep, monkeypatch):
    log("level-set V-cycle parity (%s sweeps)" % sweep)
    import paper_1307_4354_amd as cpm

    monkeypatch.setenv("CPM_SWEEP", sweep)
    torch = torch_cuda()
    H = oracle_for(CFG)
    cp = H.levels[0].cp
    f = CFG.problem.f(cp)
    ref = ov.solve(H, f, ov.Params(), rtol=1e-10, max_cycles=60, keep_iterates=True)
    band = build_gpu(CFG.problem.surface, CFG.h0, CFG.levels, CFG.lam2)
    p = cpm.make_params()
    work, nbytes = workspace(band, p)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    for k in range(6):
        cpm.cpm_vcycle(band, p, fd, ud, work, nbytes)
        assert rel_inf(host(ud), ref.iterates[k]) < 1e-12, k
    ud.zero_()
    st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
    assert st.cycles == ref.cycles
    assert rel_inf(host(ud), ref.u) < 1e-12
    assert np.max(np.abs(host(ud) - CFG.problem.u_exact(cp))) < 1.5e-3
