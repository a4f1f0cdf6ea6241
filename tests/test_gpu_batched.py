"""Batched solves: each problem of an uneven batch, solved in one batched launch sequence,
equals its own unbatched mixed-precision solve (same cycles, same iterate), and reaches the
tolerance.  The unbatched solve is itself checked against the oracle in test_gpu_parity.
The batched kernels sweep with the two passes (neighbour sum, then extension), so the
unbatched reference solves are pinned to that form (CPM_SWEEP=split) for bitwise equality."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import build_gpu, dev, host, log, torch_cuda, workspace

pytestmark = pytest.mark.gpu


def _setup(items):
    import paper_1307_4354_amd as cpm

    bands, fs = [], []
    for it in items:
        s = it.problem.surface
        b = build_gpu(s, it.h0, it.levels, it.lam2)
        _, cp = b.export(0)
        bands.append(b)
        fs.append(dev(it.problem.f(cp)))
    return bands, fs


def test_batched_equals_unbatched_mixed(monkeypatch):
    import paper_1307_4354_amd as cpm

    monkeypatch.setenv("CPM_SWEEP", "split")
    torch = torch_cuda()
    items = W.batch_problems(8, seed=W.SEED_BASE + 40, h_choices=(16, 32), coarse_h_inv=4)
    log("batched parity: %d problems, sizes %s" % (len(items), [round(1 / it.h0) for it in items]))
    bands, fs = _setup(items)
    p = cpm.make_params(precision=cpm.CPM_MIXED)
    us = [torch.zeros_like(f) for f in fs]
    nbytes = cpm.cpm_workspace_size_batched(bands, p)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    status, stats = cpm.cpm_solve_batched(bands, p, fs, us, work, nbytes, rtol=1e-10, max_cycles=80)
    assert status == cpm.CPM_OK
    for k, (b, f, u, st) in enumerate(zip(bands, fs, us, stats)):
        w, nb = workspace(b, p)
        u1 = torch.zeros_like(f)
        ref = cpm.cpm_solve(b, p, f, u1, w, nb, rtol=1e-10, max_cycles=80)
        assert st.cycles == ref.cycles, (k, st.cycles, ref.cycles)
        assert st.relres < 1e-10
        assert np.allclose(st.history(), ref.history(), rtol=1e-12, atol=0)
        a, r = host(u), host(u1)
        assert np.max(np.abs(a - r)) <= 1e-14 * np.max(np.abs(r)), k
    assert stats[0].tile_block in (128, 256, 512)


def test_batched_converged_problem_is_frozen():
    """A problem that starts at its solution does no cycle while the others run."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    items = W.batch_problems(3, seed=W.SEED_BASE + 41, h_choices=(16,), coarse_h_inv=4)
    bands, fs = _setup(items)
    p = cpm.make_params(precision=cpm.CPM_MIXED)
    fs[1].zero_()  # E f = 0: solved by u = 0 before any cycle
    us = [torch.zeros_like(f) for f in fs]
    nbytes = cpm.cpm_workspace_size_batched(bands, p)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    status, stats = cpm.cpm_solve_batched(bands, p, fs, us, work, nbytes, rtol=1e-10, max_cycles=80)
    assert status == cpm.CPM_OK
    assert stats[1].cycles == 0 and float(us[1].abs().max()) == 0.0
    assert stats[0].cycles > 5 and stats[2].cycles > 5


def test_batched_rejects_bad_arguments():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    items = W.batch_problems(2, seed=W.SEED_BASE + 42, h_choices=(16,), coarse_h_inv=4)
    bands, fs = _setup(items)
    us = [torch.zeros_like(f) for f in fs]
    p64 = cpm.make_params()
    with pytest.raises(cpm.CpmError):
        cpm.cpm_solve_batched(bands, p64, fs, us, fs[0], 8, 1e-10, 5)
    p = cpm.make_params(precision=cpm.CPM_MIXED)
    nbytes = cpm.cpm_workspace_size_batched(bands, p)
    with pytest.raises(cpm.CpmError) as ei:
        cpm.cpm_solve_batched(bands, p, fs, us, fs[0], 8, 1e-10, 5)
    assert ei.value.status == cpm.CPM_E_WORKSPACE
