"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (batched, graph-captured, sparse boundary solve).

The oracle is too slow to solve every snapshot, so each test solves the whole
batch on the GPU and checks a seeded sample of snapshots against the oracle,
plus properties that hold for every snapshot (all converge within the
10-iteration cap; the objective sits near its chi-square expectation m - n).
"""
import math

import numpy as np
import pytest

from gpu_common import Case, assert_state_close, say
from paper_2604_23175_amd import mase

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,sample", [("c2", (0, 31, 63)), ("c3", (5, 62))])
def test_full_batch_sampled_parity(name, sample):
    say("full size", name)
    c = Case(name, 64, seed=0)
    m = c.ctx()
    iters, conv = m.mase_solve(1e-6, 10)
    assert conv.all(), iters
    vm, va = m.mase_state()
    J = m.mase_objective()
    mn = c.net.m - c.net.n
    assert np.all(np.abs(J - mn) <= 4 * math.sqrt(2 * mn)), (J.min(), J.max(), mn)
    for i in sample:
        say("  oracle snapshot", i)
        ref = c.oracle_solve(i)
        assert ref["converged"] and iters[i] == ref["iters"]
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    m.close()


def test_plain_schedule_matches_batched_c2():
    say("plain vs batched c2")
    c = Case("c2", 2, seed=1)
    res = []
    for kw in (dict(), dict(batched=False)):
        m = c.ctx(**kw)
        it, conv = m.mase_solve(1e-6, 10)
        assert conv.all()
        res.append(m.mase_state())
        m.close()
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("name", ["c2k2", "c2k64"])
def test_partition_extremes_sampled_parity(name):
    # K = 2: areas of up to 6,950 buses (assembly staged in HBM, right-hand
    # sides of the level kernels in HBM); K = 64: a 1,476-variable boundary
    # system with many independent elimination subtrees
    say("partition extreme", name)
    c = Case(name, 16, seed=4)
    m = c.ctx()
    iters, conv = m.mase_solve(1e-6, 10)
    assert conv.all(), iters
    vm, va = m.mase_state()
    for i in (0, 15):
        say("  oracle snapshot", i)
        ref = c.oracle_solve(i)
        assert ref["converged"] and iters[i] == ref["iters"]
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    m.close()


def test_stream_full_size_matches_batched_and_oracle():
    # the benchmark's stream configuration: 64 slots on the 9241-bus grid,
    # a stream longer than the slots (every snapshot bitwise equal to its
    # batched solve), sampled against the oracle
    import torch
    say("stream full size c2")
    dev = torch.device("cuda:0")
    from paper_2604_23175_amd import mase
    c = Case("c2", 96, seed=7)
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 64, slack=c.slack)
    n = c.z.shape[0]
    vm = torch.empty((n, c.g.n_bus), dtype=torch.float64, device=dev)
    va = torch.empty_like(vm)
    it, conv = m.mase_solve_stream(torch.tensor(c.z, device=dev), vm, va, None, None, 1e-6, 10)
    assert conv.all(), it
    vm, va = vm.cpu().numpy(), va.cpu().numpy()
    for i0 in (0, 64):
        idx = list(range(i0, min(n, i0 + 64)))
        pad = idx + [idx[-1]] * (64 - len(idx))
        m.mase_set_measurements(c.z[pad])
        m.mase_set_state()
        bit, bconv = m.mase_solve(1e-6, 10)
        bvm, bva = m.mase_state()
        k = len(idx)
        np.testing.assert_array_equal(it[idx], bit[:k])
        np.testing.assert_array_equal(vm[idx], bvm[:k])
        np.testing.assert_array_equal(va[idx], bva[:k])
    for i in (3, 70, 95):
        say("  oracle snapshot", i)
        ref = c.oracle_solve(i)
        assert ref["converged"] and it[i] == ref["iters"]
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    m.close()


@pytest.mark.parametrize("schedule", ["autotune", "panel16"])
def test_stream_headline_schedule_matches_oracle(schedule, tmp_path, monkeypatch):
    # the benchmark's configuration on the 9241-bus grid: 64 slots, a stream
    # of 96 snapshots, the schedule the autotuner picks (or the 16-column
    # dense-block kernel with lookahead forced), checked against the oracle
    import torch
    say("stream headline schedule c2", schedule)
    from paper_2604_23175_amd import mase
    dev = torch.device("cuda:0")
    c = Case("c2", 96, seed=9)
    if schedule == "panel16":
        monkeypatch.setenv("MASE_DENSE_PANEL", "1")
        m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 64, slack=c.slack)
        assert m.mase_info("gamma_dense_panel") == 16
    else:
        m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 64, slack=c.slack, autotune=True,
                                tune_cache=str(tmp_path / "tune.txt"))
    n = c.z.shape[0]
    vm = torch.empty((n, c.g.n_bus), dtype=torch.float64, device=dev)
    va = torch.empty_like(vm)
    it, conv = m.mase_solve_stream(torch.tensor(c.z, device=dev), vm, va, None, None, 1e-6, 10)
    say("  schedule:", {k: m.mase_info(k) for k in ("pipeline_groups", "gamma_supernodal",
                                                   "gamma_subtree_groups", "gamma_dense_panel")})
    assert conv.all(), it
    vm, va = vm.cpu().numpy(), va.cpu().numpy()
    for i in (1, 50, 94):
        say("  oracle snapshot", i)
        ref = c.oracle_solve(i)
        assert ref["converged"] and it[i] == ref["iters"], (it[i], ref["iters"])
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    m.close()


def test_dense_boundary_block_beyond_960_rows_c2():
    # The whole boundary system as one dense block (9241 buses: 481 boundary
    # buses, 962 variables, more than the 960 rows up to which the dense
    # kernels' back substitution runs right-looking) takes the left-looking
    # back substitution; its states agree with the supernodal boundary solve.
    say("dense boundary mode c2")
    c = Case("c2", 2, seed=5)
    res = []
    for gm in (mase.MASE_GAMMA_SPARSE, mase.MASE_GAMMA_DENSE):
        m = c.ctx(gamma_mode=gm)
        if gm == mase.MASE_GAMMA_DENSE:
            assert 2 * m.mase_info("gamma_tail") > 960, m.mase_info("gamma_tail")
        iters, conv = m.mase_solve(1e-8, 12)
        assert conv.all(), iters
        res.append((m.mase_state(), iters))
        m.close()
    np.testing.assert_array_equal(res[0][1], res[1][1])
    for i in range(2):
        assert_state_close(res[1][0][0][i], res[1][0][1][i], res[0][0][0][i], res[0][0][1][i], 1e-10)
