"""GPU: the stream solve that allocates nothing (mase_solve_stream_noalloc)
against the allocating stream solve (mase_solve_stream).

* on a fresh context (no iteration graph yet: kernels launched directly)
  and then on a context whose graph exists (replayed), two calls in a row,
  the second with fewer snapshots, each equal bitwise (states, iteration
  counts, flags) to mase_solve_stream on the same snapshots, and a sample
  within 1e-8 of the oracle with its iteration count;
* a stream longer than the fixed scratch array allows is rejected before
  any device work.
"""
import numpy as np
import pytest
import torch

from gpu_common import Case, assert_state_close, say
from paper_2604_23175_amd import mase

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None

pytestmark = pytest.mark.gpu


def _run(m, z, noalloc):
    n = z.shape[0]
    zd = torch.tensor(z, device=DEV)
    vm = torch.full((n, m.n_bus), -7.0, dtype=torch.float64, device=DEV)
    va = torch.full_like(vm, -7.0)
    fn = m.mase_solve_stream_noalloc if noalloc else m.mase_solve_stream
    iters, conv = fn(zd, vm, va, None, None, 1e-6, 10)
    torch.cuda.synchronize()
    return vm.cpu().numpy(), va.cpu().numpy(), iters, conv


@pytest.mark.parametrize("graph_first", [False, True])
def test_noalloc_stream_equals_stream(graph_first):
    say("no-alloc stream vs stream, graph instantiated first:", graph_first)
    c = Case("c1", 29, seed=41)
    slots = 8
    ref_ctx = mase.Mase.from_grid(c.g, c.t, c.a, c.s, slots, slack=c.slack)
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, slots, slack=c.slack)
    assert m.mase_stream_noalloc_max() == ((1 << 20) - 3 * slots - 2) // 2
    if graph_first:
        # an allocating stream call first instantiates the context's graph
        _run(m, c.z[:3], noalloc=False)
    for n_total in (29, 13):  # the second call smaller than the first
        z = c.z[:n_total]
        vm, va, it, cv = _run(m, z, noalloc=True)
        rvm, rva, rit, rcv = _run(ref_ctx, z, noalloc=False)
        np.testing.assert_array_equal(it, rit)
        np.testing.assert_array_equal(cv, rcv)
        np.testing.assert_array_equal(vm, rvm)
        np.testing.assert_array_equal(va, rva)
        assert cv.all()
        for i in (0, n_total - 1):
            ref = c.oracle_solve(i)
            assert ref["converged"] and it[i] == ref["iters"], (i, it[i], ref["iters"])
            assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    m.close()
    ref_ctx.close()


def test_noalloc_stream_rejects_oversize():
    say("no-alloc stream size limit")
    c = Case("c0", 2, seed=3)
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 4, slack=c.slack)
    cap = m.mase_stream_noalloc_max()
    assert cap == ((1 << 20) - 3 * 4 - 2) // 2
    # a zero-stride view: cap + 1 rows without cap + 1 rows of memory; the
    # call must refuse before reading any of it
    z = torch.tensor(c.z[:1], device=DEV).expand(cap + 1, -1)
    vm = torch.empty((1, m.n_bus), dtype=torch.float64, device=DEV).expand(cap + 1, -1)
    n = cap + 1
    rc = m.lib.mase_solve_stream_noalloc(m.ctx, mase._dptr(z), None, None, n, 1e-6, 10, mase._dptr(vm),
                                         mase._dptr(vm), None, None)
    assert rc == mase.MASE_ERR_ARG
    assert "exceeds" in m.lib.mase_last_error().decode()
    m.close()
