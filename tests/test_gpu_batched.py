"""Batched solves: each problem of an uneven batch (spheres and tori, 3 and 4 levels) against
the oracle's mixed-precision solve of the same problem (cycle count, per-cycle residual) and
its float64 solution; each problem also equals its own unbatched mixed-precision solve.
The batched kernels sweep with the two passes (neighbour sum, then extension), so the
unbatched reference solves are pinned to that form (CPM_SWEEP=split) for bitwise equality."""
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from oracle import band as ob
from oracle import mixed as omx
from oracle import vcycle as ov
from tests.gpu_util import build_gpu, dev, host, log, rel_inf, torch_cuda, workspace

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


def _oracle_batch():
    items = W.batch_problems(6, seed=W.SEED_BASE + 43, h_choices=(16, 32), coarse_h_inv=4)
    out = []
    for k, it in enumerate(items):
        h_inv = 16 if k % 3 == 0 else 32
        out.append(dataclasses.replace(it, h0=1.0 / h_inv, levels=int(round(math.log2(h_inv / 4))) + 1))
    return out


def test_batched_matches_oracle():
    """Six problems (three spheres, three tori; h = 1/16 and 1/32, coarsened to 1/4) in one
    batched solve against the oracle: cycle count within one of the oracle's mixed-precision
    solve, each cycle's relative residual within 1 % of it (float32 inner cycles round
    differently), the final iterate within 1e-9 of the oracle's float64 solution."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    items = _oracle_batch()
    bands, fs, refs = [], [], []
    for k, it in enumerate(items):
        s = it.problem.surface
        H = ob.build_hierarchy(s, it.h0, it.levels, it.lam2)
        f = it.problem.f(H.levels[0].cp)
        mx = omx.solve_mixed(H, f, ov.Params(), rtol=1e-10, max_cycles=80)
        r64 = ov.solve(H, f, ov.Params(), rtol=1e-10, max_cycles=80)
        log("oracle problem %d: %s h=1/%d n=%s, mixed %d cycles, f64 %d cycles" % (
            k, s.kind, round(1 / it.h0), [l.n for l in H.levels], mx.cycles, r64.cycles))
        refs.append((mx, r64))
        bands.append(build_gpu(s, it.h0, it.levels, it.lam2))
        fs.append(dev(f))
    p = cpm.make_params(precision=cpm.CPM_MIXED)
    us = [torch.zeros_like(f) for f in fs]
    nbytes = cpm.cpm_workspace_size_batched(bands, p)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    status, stats = cpm.cpm_solve_batched(bands, p, fs, us, work, nbytes, rtol=1e-10, max_cycles=80)
    assert status == cpm.CPM_OK
    for k, (st, u, (mx, r64)) in enumerate(zip(stats, us, refs)):
        err = rel_inf(host(u), r64.u)
        log("problem %d: %d cycles (oracle %d), relres %.3e, rel diff to f64 oracle %.2e" % (
            k, st.cycles, mx.cycles, st.relres, err))
        assert abs(st.cycles - mx.cycles) <= 1
        hg, ho = st.history(), mx.relres
        for j in range(min(len(hg), len(ho))):
            assert abs(hg[j] - ho[j]) <= 1e-2 * ho[j], (k, j, hg[j], ho[j])
        assert st.relres < 1e-10
        assert err < 1e-9
    # one host synchronization per graph launch of several cycles
    cyc = max(st.cycles for st in stats)
    assert stats[0].cycles_per_launch > 1
    assert stats[0].host_syncs <= -(-cyc // stats[0].cycles_per_launch) + 1


def test_batched_stops_at_max_cycles():
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    items = W.batch_problems(3, seed=W.SEED_BASE + 44, h_choices=(16,), coarse_h_inv=4)
    bands, fs = _setup(items)
    p = cpm.make_params(precision=cpm.CPM_MIXED)
    us = [torch.zeros_like(f) for f in fs]
    nbytes = cpm.cpm_workspace_size_batched(bands, p)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    status, stats = cpm.cpm_solve_batched(bands, p, fs, us, work, nbytes, rtol=1e-10, max_cycles=5,
                                          raise_on_noconv=False)
    assert status == cpm.CPM_E_NOCONV
    assert all(st.cycles == 5 for st in stats)


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


def test_batched_forms_give_the_same_solve(monkeypatch):
    """The batched solve is the same bit for bit whether its workgroups stage the extension in
    LDS (256 lanes) or gather (128 lanes), and whether the residual before restriction covers
    only the restriction's fine nodes (the default) or every node (CPM_RESID_SUBSET=0): the
    restriction reads that residual at those nodes only."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    items = W.batch_problems(4, seed=W.SEED_BASE + 45, h_choices=(16, 32), coarse_h_inv=4)
    p = cpm.make_params(precision=cpm.CPM_MIXED)
    runs = {}
    for block, subset in (("256", "1"), ("256", "0"), ("128", "1")):
        monkeypatch.setenv("CPM_BATCH_BLOCK", block)
        monkeypatch.setenv("CPM_RESID_SUBSET", subset)
        bands, fs = _setup(items)
        flagged = [bool(b.flags(0) & cpm.CPM_BAND_RESID_SUBSET) for b in bands]
        assert any(flagged) if subset == "1" else not any(flagged)
        us = [torch.zeros_like(f) for f in fs]
        nbytes = cpm.cpm_workspace_size_batched(bands, p)
        work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        status, stats = cpm.cpm_solve_batched(bands, p, fs, us, work, nbytes, rtol=1e-10, max_cycles=80)
        assert status == cpm.CPM_OK
        assert stats[0].tile_block == int(block)
        log("batched block %s, residual subset %s: cycles %s" % (block, subset, [st.cycles for st in stats]))
        runs[(block, subset)] = ([host(u) for u in us], [st.history() for st in stats])
    ref_u, ref_h = runs[("256", "1")]
    for key in (("256", "0"), ("128", "1")):
        us, hs = runs[key]
        for k in range(len(items)):
            assert np.array_equal(us[k], ref_u[k]), (key, k)
            assert np.array_equal(hs[k], ref_h[k]), (key, k)


def test_batched_converged_problem_is_frozen():
    """A problem with E f = 0 gets u = 0 (from a non-zero start) and no cycle while the others
    run."""
    import paper_1307_4354_amd as cpm

    torch = torch_cuda()
    items = W.batch_problems(3, seed=W.SEED_BASE + 41, h_choices=(16,), coarse_h_inv=4)
    bands, fs = _setup(items)
    p = cpm.make_params(precision=cpm.CPM_MIXED)
    fs[1].zero_()  # E f = 0: solved by u = 0 before any cycle, whatever the start
    us = [torch.zeros_like(f) for f in fs]
    us[1].fill_(0.5)
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
