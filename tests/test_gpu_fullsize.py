"""Parity at the largest single-GPU size (the torus R = 1, r = 0.4 at h = 1/256, 8.5 million
band nodes, the mixed-precision workload), on outputs the oracle computes one by one:

* closest points of 4,000 sampled band nodes are the oracle's, bit for bit, and inside the
  band radius;
* the band is ordered (x fastest) and contains every node of the sampled nodes' cubic
  stencils and their axis neighbours (the containment property of Sec. 3.1);
* the extension E u of a seeded random vector, at the sampled nodes, equals the oracle's
  stencil sum to rounding, in the gather form and in the LDS-staged form the bench times
  (workgroups of 512 stencil slots, the node's own data loaded before the staging), and the
  operator A u = delta u - E(N u) does too;
* a mixed-precision solve reaches 1e-10 and agrees with the double-precision solve.
"""
import numpy as np
import pytest

import workloads as W
from oracle import band as ob
from oracle import geometry as og
from tests.gpu_util import build_gpu, dev, host, log, torch_cuda, workspace

pytestmark = pytest.mark.gpu


def test_torus256_sampled_parity():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    cfg = W.config_torus_mixed(256)
    s = cfg.problem.surface
    log("full-size parity: torus h = 1/256, %d levels" % cfg.levels)
    band = build_gpu(s, cfg.h0, cfg.levels, cfg.lam2)
    idx, cp = band.export(0)
    n = idx.shape[0]
    assert n == 8531440
    h = cfg.h0
    thr = cfg.lam2 * (h * h)
    # band order: lexicographic keys (z, y, x), strictly increasing
    lo = idx.min(axis=0) - 4
    ext = idx.max(axis=0) - lo + 5
    keys = ((idx[:, 2] - lo[2]) * ext[1] + (idx[:, 1] - lo[1])) * ext[0] + (idx[:, 0] - lo[0])
    assert np.all(np.diff(keys) > 0)

    def lookup(M):
        k = ((M[:, 2] - lo[2]) * ext[1] + (M[:, 1] - lo[1])) * ext[0] + (M[:, 0] - lo[0])
        pos = np.clip(np.searchsorted(keys, k), 0, n - 1)
        return np.where(keys[pos] == k, pos, -1)

    sel = np.random.default_rng(W.SEED_BASE + 60).choice(n, 4000, replace=False)
    cpo, d2 = og.closest_point_and_dist2(s, idx[sel].astype(np.float64) * h)
    assert np.array_equal(cpo, cp[sel])
    assert np.all(d2 <= thr)
    base, W1, _ = ob.stencil(cp[sel], h, 3)
    M = base[:, None, :] + ob.stencil_offsets(3, 3)[None, :, :]
    cols = lookup(M.reshape(-1, 3)).reshape(sel.size, -1)
    assert np.all(cols >= 0)
    for a in range(3):
        for sg in (-1, 1):
            Q = M.reshape(-1, 3).copy()
            Q[:, a] += sg
            assert np.all(lookup(Q) >= 0)
    u = W.random_vector(n, W.SEED_BASE + 61)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ref = np.sum(ob.tensor_weights(W1) * u[cols], axis=1)
    # A u at the sampled nodes: (N u) at each stencil node from its axis neighbours
    inv_h2 = 1.0 / (h * h)
    Mf = M.reshape(-1, 3)
    nu = np.zeros(Mf.shape[0])
    for a in range(3):
        for sg in (-1, 1):
            Q = Mf.copy()
            Q[:, a] += sg
            nu += u[lookup(Q)] * inv_h2
    delta = cfg.problem.c + 6.0 * inv_h2
    ref_a = delta * u[sel] - np.sum(ob.tensor_weights(W1) * nu.reshape(sel.size, -1), axis=1)
    assert cpm.cpm_band_ext_slots(band, 0) == 512  # two slots per lane on an 8.5M-node level
    assert cpm.cpm_band_ext_slots(band, 1) == 256
    tun = cpm.cpm_band_tuning(band, 0)
    wa = torch.empty(n, dtype=torch.float64, device="cuda")
    for lds, pf in ((False, False), (True, False), (True, True)):
        cpm.cpm_set_band_tuning(band, 0, lds, 256, tun[2], False, tun[4], False, False, pf)
        cpm.cpm_extend(band, 0, dev(u), out)
        got = host(out)[sel]
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(u)), (lds, pf)
        cpm.cpm_apply(band, 0, cfg.problem.c, dev(u), out, wa)
        got = host(out)[sel]
        assert np.max(np.abs(got - ref_a)) <= 1e-12 * np.max(np.abs(ref_a)), (lds, pf)
    del wa
    # solves at full size: mixed precision against double precision
    f = cfg.problem.f(cp)
    fd = dev(f)
    res = {}
    for prec in (cpm.CPM_F64, cpm.CPM_MIXED):
        p = cpm.make_params(precision=prec)
        work, nbytes = workspace(band, p)
        ud = torch.zeros_like(fd)
        st = cpm.cpm_solve(band, p, fd, ud, work, nbytes, rtol=1e-10, max_cycles=60)
        assert st.relres < 1e-10
        res[prec] = host(ud)
        del work
    diff = np.max(np.abs(res[cpm.CPM_MIXED] - res[cpm.CPM_F64])) / np.max(np.abs(res[cpm.CPM_F64]))
    assert diff < 1e-9, diff
