"""GPU continuous batching (mase_solve_stream) against the batched solve and the oracle.

* every snapshot of a stream longer than the slot count ends bitwise equal
  (state and iteration count) to the same snapshot solved by mase_solve in a
  batch on the same context from the same start: a snapshot's arithmetic
  does not depend on its slot or on the other snapshots in flight;
* a sample of the stream matches the oracle's centralized Gauss-Newton to
  1e-8 relative with the oracle's iteration count;
* given starting states are used; streams shorter than the slot count and
  empty streams; the iteration cap (every snapshot unconverged after
  max_iter steps, states equal to the batched solve's); an unobservable area
  drains the stream and reports MASE_ERR_NOT_POSDEF;
* the stream without graph capture equals the graph-replayed one bitwise, and
  a context that autotunes inside its first stream call reaches the oracle.
"""
import numpy as np
import pytest
import torch

from gpu_common import Case, assert_state_close, say
from paper_2604_23175_amd import mase

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None

pytestmark = pytest.mark.gpu


def batched_reference(m, z, vm0=None, va0=None, tol=1e-6, max_iter=10):
    """Each chunk of n_snap snapshots solved by mase_solve on the same context
    (the last chunk padded with copies of its last snapshot)."""
    S, n = m.n_snap, z.shape[0]
    vm = np.zeros((n, m.n_bus))
    va = np.zeros((n, m.n_bus))
    it = np.zeros(n, dtype=np.int32)
    cv = np.zeros(n, dtype=bool)
    for i0 in range(0, n, S):
        idx = list(range(i0, min(n, i0 + S)))
        pad = idx + [idx[-1]] * (S - len(idx))
        m.mase_set_measurements_dev(torch.tensor(z[pad], device=DEV))
        if vm0 is None:
            m.mase_set_state_dev(None, None)
        else:
            m.mase_set_state_dev(torch.tensor(vm0[pad], device=DEV), torch.tensor(va0[pad], device=DEV))
        iters, conv = m.mase_solve(tol, max_iter)
        v, a = m.mase_state()
        k = len(idx)
        vm[idx], va[idx], it[idx], cv[idx] = v[:k], a[:k], iters[:k], conv[:k]
    return vm, va, it, cv


def run_stream(m, z, vm0=None, va0=None, tol=1e-6, max_iter=10):
    n = z.shape[0]
    zd = torch.tensor(z, device=DEV)
    vm = torch.full((n, m.n_bus), -7.0, dtype=torch.float64, device=DEV)
    va = torch.full_like(vm, -7.0)
    v0 = None if vm0 is None else torch.tensor(vm0, device=DEV)
    a0 = None if va0 is None else torch.tensor(va0, device=DEV)
    iters, conv = m.mase_solve_stream(zd, vm, va, v0, a0, tol, max_iter)
    torch.cuda.synchronize()
    return vm.cpu().numpy(), va.cpu().numpy(), iters, conv


@pytest.mark.parametrize("name,slots,n_total", [("k5", 3, 11), ("c1", 8, 21), ("c1", 8, 8)])
def test_stream_bitwise_equal_to_batched(name, slots, n_total):
    say("stream vs batched", name, slots, n_total)
    c = Case(name, n_total, seed=31)
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, slots, slack=c.slack)
    vm, va, it, cv = run_stream(m, c.z)
    rvm, rva, rit, rcv = batched_reference(m, c.z)
    np.testing.assert_array_equal(it, rit)
    np.testing.assert_array_equal(cv, rcv)
    np.testing.assert_array_equal(vm, rvm)
    np.testing.assert_array_equal(va, rva)
    assert cv.all()
    for i in (0, n_total // 2, n_total - 1):
        ref = c.oracle_solve(i)
        assert ref["converged"] and it[i] == ref["iters"], (i, it[i], ref["iters"])
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    m.close()


def test_stream_given_starting_states():
    say("stream warm states")
    c = Case("k5", 7, seed=32)
    rng = np.random.default_rng(5)
    vm0 = c.vm_true + rng.normal(0.0, 0.01, c.vm_true.shape)
    va0 = c.va_true + rng.normal(0.0, 0.02, c.va_true.shape)
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 3, slack=c.slack)
    vm, va, it, cv = run_stream(m, c.z, vm0, va0)
    rvm, rva, rit, rcv = batched_reference(m, c.z, vm0, va0)
    np.testing.assert_array_equal(it, rit)
    np.testing.assert_array_equal(vm, rvm)
    np.testing.assert_array_equal(va, rva)
    assert cv.all()
    m.close()


def test_stream_shorter_than_slots_and_empty():
    say("stream short / empty")
    c = Case("k5", 2, seed=33)
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 5, slack=c.slack)
    vm, va, it, cv = run_stream(m, c.z)
    assert cv.all()
    for i in range(2):
        ref = c.oracle_solve(i)
        assert it[i] == ref["iters"]
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    empty = np.zeros((0, c.z.shape[1]))
    _, _, it0, cv0 = run_stream(m, empty)
    assert it0.size == 0 and cv0.size == 0
    # a later batched solve on the same context still works
    m.mase_set_measurements(np.concatenate([c.z, c.z, c.z[:1]]))
    m.mase_set_state()
    iters, conv = m.mase_solve(1e-6, 10)
    assert conv.all()
    m.close()


def test_stream_iteration_cap():
    say("stream iteration cap")
    c = Case("k5", 5, seed=34)
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 2, slack=c.slack)
    vm, va, it, cv = run_stream(m, c.z, max_iter=2)
    rvm, rva, rit, rcv = batched_reference(m, c.z, max_iter=2)
    assert not cv.any() and (it == 2).all()
    np.testing.assert_array_equal(rit, it)
    np.testing.assert_array_equal(vm, rvm)
    np.testing.assert_array_equal(va, rva)
    m.close()


def test_stream_unobservable_area_reports_not_posdef():
    say("stream not posdef")
    c = Case("k5", 4, seed=35)
    w = 1.0 / c.s ** 2
    w[c.A.meas_area == 2] = 0.0
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 3, slack=c.slack)
    m.mase_set_measurements(np.concatenate([c.z[:3]]), w)
    with pytest.raises(mase.MaseError) as e:
        run_stream(m, c.z)
    assert e.value.code == mase.MASE_ERR_NOT_POSDEF
    m.close()


def test_stream_needs_batched_schedule():
    say("stream plain rejected")
    c = Case("c0", 2, seed=36)
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 2, slack=c.slack, batched=False)
    with pytest.raises(mase.MaseError) as e:
        run_stream(m, c.z)
    assert e.value.code == mase.MASE_ERR_ARG
    m.close()


def test_stream_schedules_and_autotune(tmp_path):
    # the stream without graph capture (direct launches, one host check per
    # pass) equals the graph-replayed stream bitwise; a context that tunes
    # inside its first stream call reaches the oracle's states
    say("stream schedules / autotune")
    c = Case("c1", 11, seed=37)
    out = []
    for kw in (dict(), dict(use_graph=False)):
        m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 4, slack=c.slack, **kw)
        out.append(run_stream(m, c.z))
        m.close()
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 4, slack=c.slack, autotune=True,
                            tune_cache=str(tmp_path / "tune.txt"))
    vm, va, it, cv = run_stream(m, c.z)
    assert cv.all()
    assert (tmp_path / "tune.txt").exists()
    for i in (0, 5, 10):
        ref = c.oracle_solve(i)
        assert it[i] == ref["iters"]
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    m.close()


def test_stream_failed_snapshot_among_healthy_ones():
    # one snapshot of the stream with NaN measurements is retired as failed;
    # the others pass through the same slots and match their batched solves
    say("stream: one failing snapshot")
    c = Case("k5", 9, seed=41)
    z = c.z.copy()
    z[4, :] = np.nan
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, 3, slack=c.slack)
    n = z.shape[0]
    vm = torch.empty((n, c.g.n_bus), dtype=torch.float64, device=DEV)
    va = torch.empty_like(vm)
    with pytest.raises(mase.MaseError) as e:
        m.mase_solve_stream(torch.tensor(z, device=DEV), vm, va, None, None, 1e-6, 10)
    assert e.value.code == mase.MASE_ERR_NOT_POSDEF
    vm, va = vm.cpu().numpy(), va.cpu().numpy()
    for i in (0, 3, 5, 8):
        ref = c.oracle_solve(i)
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    m.close()


@pytest.mark.parametrize("name,slots,n_total,start", [("k5", 3, 11, False), ("c1", 8, 37, True),
                                                      ("c1", 8, 5, False)])
def test_stream_host_buffers_equal_device_stream(name, slots, n_total, start):
    # measurements uploaded chunk by chunk from pinned host memory while the
    # stream iterates, states downloaded as chunks finish: bitwise the device
    # stream's results
    say("stream with host buffers", name, slots, n_total, start)
    c = Case(name, n_total, seed=17)
    m = mase.Mase.from_grid(c.g, c.t, c.a, c.s, slots, slack=c.slack)
    vm0 = va0 = None
    if start:
        rng = np.random.default_rng(3)
        vm0 = torch.tensor(c.vm_true + rng.normal(0, 0.01, c.vm_true.shape)).pin_memory()
        va0 = torch.tensor(c.va_true + rng.normal(0, 0.01, c.va_true.shape)).pin_memory()
    zd = torch.tensor(c.z, device=DEV)
    vd = torch.empty((n_total, c.g.n_bus), dtype=torch.float64, device=DEV)
    ad = torch.empty_like(vd)
    it_d, conv_d = m.mase_solve_stream(zd, vd, ad, None if vm0 is None else vm0.to(DEV),
                                       None if va0 is None else va0.to(DEV), 1e-6, 10)
    zh = torch.tensor(c.z).pin_memory()
    vh = torch.empty((n_total, c.g.n_bus), dtype=torch.float64).pin_memory()
    ah = torch.empty_like(vh).pin_memory()
    work = torch.empty(m.mase_stream_host_work(n_total, start), dtype=torch.float64, device=DEV)
    it_h, conv_h = m.mase_solve_stream_host(zh, vh, ah, work, vm0, va0, 1e-6, 10)
    np.testing.assert_array_equal(it_h, it_d)
    np.testing.assert_array_equal(conv_h, conv_d)
    np.testing.assert_array_equal(vh.numpy(), vd.cpu().numpy())
    np.testing.assert_array_equal(ah.numpy(), ad.cpu().numpy())
    assert conv_h.all()
    ref = c.oracle_solve(n_total - 1) if not start else None
    if ref is not None:
        assert_state_close(vh.numpy()[-1], ah.numpy()[-1], ref["vm"], ref["va"], 1e-8)
    # null buffers and a workspace one double short are argument errors
    import ctypes
    P = ctypes.c_void_p
    rc = m.lib.mase_solve_stream_host(m.ctx, None, None, None, n_total, 1e-6, 10, None, None, None, None, None, 0)
    assert rc == mase.MASE_ERR_ARG
    need = m.mase_stream_host_work(n_total, start)
    rc = m.lib.mase_solve_stream_host(m.ctx, P(zh.data_ptr()), None if vm0 is None else P(vm0.data_ptr()),
                                      None if va0 is None else P(va0.data_ptr()), n_total, 1e-6, 10,
                                      P(vh.data_ptr()), P(ah.data_ptr()), None, None, P(work.data_ptr()), need - 1)
    assert rc == mase.MASE_ERR_ARG
    m.close()
