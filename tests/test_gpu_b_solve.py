"""GPU end-to-end solves against the oracle, schedules and failure handling.

* states after mase_solve match the oracle's centralized GN to 1e-8 relative
  (theta in rad, |V| in p.u.) with the same iteration counts;
* noise-free measurements return the generating state;
* the batched, graph-captured schedule, the batched schedule without the
  graph and the plain per-area/per-snapshot schedule give bitwise identical
  states (same arithmetic in the same order), and two runs are identical;
* dense and sparse factorisation of the boundary system agree;
* a zero weight equals a deleted row;
* an unobservable area reports MASE_ERR_NOT_POSDEF, max_iter = 1 reports
  MASE_NOT_CONVERGED.
"""
import numpy as np
import pytest
import torch

from gpu_common import Case, assert_state_close, say
from gridgen import synth
from oracle import network as nw
from paper_2604_23175_amd import mase

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,n_snap", [("c0", 4), ("k5", 4), ("c1", 3)])
def test_solve_matches_oracle(name, n_snap):
    say("solve", name, n_snap)
    c = Case(name, n_snap, seed=21)
    m = c.ctx()
    iters, conv = m.mase_solve(1e-6, 10)
    vm, va = m.mase_state()
    for i in range(n_snap):
        ref = c.oracle_solve(i)
        assert conv[i] and ref["converged"]
        assert iters[i] == ref["iters"], (iters[i], ref["iters"])
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    J = m.mase_objective()
    for i in range(n_snap):
        assert abs(J[i] - c.oracle_solve(i)["J"]) <= 1e-8 * J[i]
    m.close()


def test_noise_free_recovery():
    say("noise-free")
    c = Case("c1", 2, seed=2)
    c.z = np.stack([c.net.h(c.vm_true[i], c.va_true[i]) for i in range(2)])
    m = c.ctx()
    iters, conv = m.mase_solve(1e-12, 15)
    assert conv.all()
    vm, va = m.mase_state()
    np.testing.assert_allclose(vm, c.vm_true, rtol=0, atol=1e-10)
    np.testing.assert_allclose(va, c.va_true, rtol=0, atol=1e-10)
    m.close()


def test_schedules_bitwise_identical():
    say("schedules")
    c = Case("k5", 3, seed=4)
    out = []
    for kw in (dict(), dict(use_graph=False), dict(batched=False)):
        m = c.ctx(**kw)
        iters, conv = m.mase_solve(1e-6, 10)
        out.append((m.mase_state(), iters))
        m.close()
    for (vm, va), it in out[1:]:
        np.testing.assert_array_equal(vm, out[0][0][0])
        np.testing.assert_array_equal(va, out[0][0][1])
        np.testing.assert_array_equal(it, out[0][1])


@pytest.mark.parametrize("name,n_snap,groups", [("k5", 3, 3), ("c1", 8, 4), ("c1", 7, 2)])
def test_pipelined_groups_bitwise_identical(name, n_snap, groups):
    # mase_solve with snapshot groups iterating on their own streams runs the
    # same kernels per snapshot as the one-group schedule
    say("pipeline groups", name, n_snap, groups)
    c = Case(name, n_snap, seed=13)
    out = []
    for g in (1, groups):
        m = c.ctx(pipeline_groups=g)
        iters, conv = m.mase_solve(1e-8, 10)
        out.append((m.mase_state(), iters, conv))
        # a second solve from the converged state: every group stops at once
        it2, conv2 = m.mase_solve(1e-8, 10)
        assert conv2.all() and (it2 == iters).all()
        m.close()
    np.testing.assert_array_equal(out[1][0][0], out[0][0][0])
    np.testing.assert_array_equal(out[1][0][1], out[0][0][1])
    np.testing.assert_array_equal(out[1][1], out[0][1])
    np.testing.assert_array_equal(out[1][2], out[0][2])
    assert out[0][2].all()


def test_autotune_choice_cached_and_results_match(tmp_path):
    say("autotune")
    c = Case("c1", 8, seed=14)
    ref = c.ctx()
    ref.mase_solve(1e-10, 12)
    xr = ref.mase_state()
    ref.close()
    cache = tmp_path / "tune.txt"
    m = c.ctx(autotune=True, tune_cache=str(cache))
    iters, conv = m.mase_solve(1e-10, 12)
    assert conv.all()
    x = m.mase_state()
    assert_state_close(x[0], x[1], xr[0], xr[1], 1e-10)
    keys = ("pipeline_groups", "gamma_supernodal", "gamma_dense_panel", "elim_threads")
    choice = tuple(m.mase_info(k) for k in keys)
    m.close()
    lines = [ln.split() for ln in cache.read_text().splitlines() if ln.strip()]
    assert len(lines) == 1 and len(lines[0]) == 6
    panel = {0: 0, 1: 16}.get(int(lines[0][3]), int(lines[0][4]))
    assert (int(lines[0][1]), int(lines[0][2]), panel, int(lines[0][5])) == choice
    # a second context takes the cached choice without tuning again
    m2 = c.ctx(autotune=True, tune_cache=str(cache))
    m2.mase_solve(1e-10, 12)
    assert tuple(m2.mase_info(k) for k in keys) == choice
    x2 = m2.mase_state()
    np.testing.assert_array_equal(x2[0], x[0])
    np.testing.assert_array_equal(x2[1], x[1])
    m2.close()
    assert len([ln for ln in cache.read_text().splitlines() if ln.strip()]) == 1


def test_repeat_runs_bitwise_identical():
    say("determinism")
    c = Case("c1", 2, seed=8)
    m = c.ctx()
    m.mase_solve(1e-6, 10)
    a = m.mase_state()
    m.mase_set_state()
    m.mase_solve(1e-6, 10)
    b = m.mase_state()
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    m.close()


def test_dense_and_sparse_gamma_agree():
    say("gamma modes")
    c = Case("c1", 2, seed=9)
    res = []
    for gm in (mase.MASE_GAMMA_SPARSE, mase.MASE_GAMMA_DENSE):
        m = c.ctx(gamma_mode=gm)
        m.mase_solve(1e-10, 12)
        res.append(m.mase_state())
        m.close()
    assert_state_close(res[0][0], res[0][1], res[1][0], res[1][1], 1e-10)


@pytest.mark.parametrize("gm", ["sparse", "dense"])
def test_dense_block_panel_variants(gm, monkeypatch):
    # The boundary block's Cholesky uses the widest panels that fit in LDS
    # (MASE_DENSE_PANEL=2); =1 stages 16-column panels in LDS and =0 reads them
    # from HBM.  1 and 0 do the same arithmetic in the same order (bitwise
    # equal); wide panels sum the trailing updates in another order.
    say("dense panel variants", gm)
    c = Case("c1", 2, seed=11)
    mode = mase.MASE_GAMMA_SPARSE if gm == "sparse" else mase.MASE_GAMMA_DENSE
    res = []
    for flag in ("2", "1", "0"):
        monkeypatch.setenv("MASE_DENSE_PANEL", flag)
        m = c.ctx(gamma_mode=mode)
        iters, conv = m.mase_solve(1e-8, 12)
        assert conv.all()
        res.append((m.mase_state(), iters))
        m.close()
    np.testing.assert_array_equal(res[1][0][0], res[2][0][0])
    np.testing.assert_array_equal(res[1][0][1], res[2][0][1])
    np.testing.assert_array_equal(res[1][1], res[2][1])
    np.testing.assert_array_equal(res[0][1], res[1][1])
    for i in range(2):
        assert_state_close(res[0][0][0][i], res[0][0][1][i], res[1][0][0][i], res[1][0][1][i], 1e-10)


@pytest.mark.parametrize("name", ["c1", "k8"])
def test_supernodal_and_level_boundary_elimination_agree(name, monkeypatch):
    # The boundary system's sparse part runs supernodal (LDS panels, MFMA
    # updates) by default; MASE_GAMMA_SNODE=0 selects the level-scheduled
    # engine.  Different summation order, same factorisation.
    say("boundary supernodes vs levels", name)
    c = Case(name, 3, seed=12)
    res = []
    for flag in ("1", "0"):
        monkeypatch.setenv("MASE_GAMMA_SNODE", flag)
        m = c.ctx()
        iters, conv = m.mase_solve(1e-10, 12)
        assert conv.all()
        res.append((m.mase_state(), iters))
        m.close()
    assert_state_close(res[0][0][0], res[0][0][1], res[1][0][0], res[1][0][1], 1e-10)
    for i in range(c.n_snap):
        o = c.oracle_solve(i, tol=1e-10, max_iter=12)
        assert_state_close(res[0][0][0][i], res[0][0][1][i], o["vm"], o["va"], 1e-8)


def test_zero_weight_equals_deleted_row():
    say("masking")
    c = Case("k5", 1, seed=6)
    w = 1.0 / c.s ** 2
    w[c.t == synth.QT] = 0.0
    c.w = w
    m = c.ctx()
    m.mase_stage_assemble()
    keep = c.t != synth.QT
    m2 = mase.Mase.from_grid(c.g, c.t[keep], c.a[keep], c.s[keep], 1)
    m2.mase_set_measurements(c.z[:, keep])
    m2.mase_set_state()
    m2.mase_stage_assemble()
    for k in range(c.g.n_area):
        G1, b1 = m.mase_read_local_system(0, k)
        G2, b2 = m2.mase_read_local_system(0, k)
        np.testing.assert_array_equal(G1, G2)
        np.testing.assert_array_equal(b1, b2)
    m.close()
    m2.close()
    m = c.ctx()
    m.mase_solve(1e-6, 10)
    vm, va = m.mase_state()
    ref = c.oracle_solve(0)
    assert_state_close(vm[0], va[0], ref["vm"], ref["va"], 1e-8)
    m.close()


def test_device_weights_and_default_reset():
    # weights given on the device mask rows like host weights; omitting them
    # restores 1/sigma^2 (no stale mask)
    say("device weights")
    c = Case("k5", 2, seed=7)
    w = 1.0 / c.s ** 2
    w[c.t == synth.PT] = 0.0
    zd = torch.tensor(c.z, device=DEV)
    m = c.ctx()
    m.mase_set_measurements_dev(zd, torch.tensor(w, device=DEV))
    torch.cuda.synchronize()
    m.mase_set_state()
    m.mase_solve(1e-10, 12)
    masked = m.mase_state()
    m.mase_set_measurements_dev(zd)
    torch.cuda.synchronize()
    m.mase_set_state()
    m.mase_solve(1e-10, 12)
    plain = m.mase_state()
    m.close()
    ref = c.ctx()
    ref.mase_solve(1e-10, 12)
    x = ref.mase_state()
    ref.close()
    np.testing.assert_array_equal(plain[0], x[0])
    np.testing.assert_array_equal(plain[1], x[1])
    c.w = w
    for i in range(2):
        o = c.oracle_solve(i, tol=1e-10, max_iter=12)
        assert_state_close(masked[0][i], masked[1][i], o["vm"], o["va"], 1e-8)


@pytest.mark.parametrize("n_area", [1, 2])
def test_large_areas_stage_in_hbm(n_area):
    # areas of ~1400-2900 buses exceed what the assembly kernel can stage in
    # LDS, so every area stages in HBM; one area means no boundary at all
    say("large areas", n_area)
    import dataclasses
    g = synth.make_config("c1")
    g = dataclasses.replace(g, n_area=n_area,
                            bus_area=synth.partition(g.pos, g.br_from, g.br_to, n_area, "balanced"))
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    b = synth.make_batch(g, 2, 21)
    vt = b.va_true - b.va_true[:, [g.slack]]
    net = nw.from_grid(g, t, a, s)
    z = np.stack([nw.measurements(net, b.vm_true[i], vt[i], b.eps[i]) for i in range(2)])
    m = mase.Mase.from_grid(g, t, a, s, 2)
    m.mase_set_measurements(z)
    m.mase_set_state()
    iters, conv = m.mase_solve(1e-10, 12)
    assert conv.all()
    vm, va = m.mase_state()
    if n_area == 1:
        assert m.mase_info("n_gamma") == 0
    m.close()
    from oracle import wls
    for i in range(2):
        o = wls.gauss_newton(net, z[i], tol=1e-10, max_iter=12)
        assert_state_close(vm[i], va[i], o["vm"], o["va"], 1e-8)


def test_unobservable_area_reports_not_posdef():
    say("not posdef")
    c = Case("k5", 2, seed=1)
    w = 1.0 / c.s ** 2
    w[c.A.meas_area == 2] = 0.0
    c.w = w
    m = c.ctx()
    with pytest.raises(mase.MaseError) as e:
        m.mase_gn_iter()
    assert e.value.code == mase.MASE_ERR_NOT_POSDEF
    m.close()


def test_iteration_cap_reports_not_converged():
    say("not converged")
    c = Case("c0", 2, seed=1)
    m = c.ctx()
    iters, conv = m.mase_solve(1e-6, 1)
    assert not conv.any()
    assert (iters == 1).all()
    m.close()


def test_slack_on_boundary_solve():
    say("slack on boundary")
    from gpu_common import boundary_slack, grid
    c = Case("k5", 2, seed=12, slack=boundary_slack(grid("k5")))
    assert c.A.is_boundary[c.slack]
    m = c.ctx()
    m.mase_solve(1e-6, 10)
    vm, va = m.mase_state()
    for i in range(2):
        ref = c.oracle_solve(i)
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    m.close()


@pytest.mark.parametrize("name,steps", [("k5", 1), ("c1", 2)])
def test_local_steps_iterate_matches_oracle(name, steps):
    """One iteration = `steps` local steps with the boundary held (Eq. 6),
    then the condensed step (Eq. 8-11), each taken by the oracle in turn."""
    say("local-steps iterate", name, steps)
    c = Case(name, 3, seed=13)
    m = c.ctx(local_steps=steps)
    m.mase_gn_iter()
    vm, va = m.mase_state()
    for i in range(3):
        x = c.net.pack(np.ones(c.g.n_bus), np.zeros(c.g.n_bus))
        for _ in range(steps):
            rvm, rva = c.net.unpack(x)
            x = x + c.A.local_step(c.z[i], rvm, rva)
        rvm, rva = c.net.unpack(x)
        x = x + c.A.condensed_step(c.z[i], rvm, rva)
        rvm, rva = c.net.unpack(x)
        assert_state_close(vm[i], va[i], rvm, rva, 1e-8)
    m.close()


@pytest.mark.parametrize("steps", [1, 3])
def test_local_steps_solve_reaches_oracle_minimizer(steps):
    say("local-steps solve", steps)
    c = Case("c1", 3, seed=17)
    m = c.ctx(local_steps=steps)
    iters, conv = m.mase_solve(1e-8, 12)
    assert conv.all()
    vm, va = m.mase_state()
    for i in range(3):
        ref = c.oracle_solve(i, tol=1e-10, max_iter=15)
        assert ref["converged"]
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
        say("  snapshot", i, "iterations", int(iters[i]), "centralized", ref["iters"])
    m.close()


def test_local_steps_need_batched_schedule():
    say("local-steps plain schedule rejected")
    c = Case("k5", 1, seed=1)
    with pytest.raises(mase.MaseError):
        c.ctx(local_steps=1, batched=False)
    with pytest.raises(mase.MaseError):
        c.ctx(local_steps=-1)


@pytest.mark.parametrize("name", ["c1", "k8"])
def test_subtree_groups_bitwise_identical(name, monkeypatch):
    # The supernodal boundary elimination runs independent elimination
    # subtrees in separate workgroups and applies every update of the dense
    # block in supernode order afterwards, so the number of groups changes
    # nothing in the arithmetic.
    say("subtree groups", name)
    c = Case(name, 3, seed=19)
    res = []
    for cap in ("1", "64"):
        monkeypatch.setenv("MASE_SNODE_GROUPS", cap)
        m = c.ctx()
        if m.mase_info("gamma_supernodal") != 1:
            pytest.skip("boundary system not supernodal on this grid")
        groups = m.mase_info("gamma_subtree_groups")
        iters, conv = m.mase_solve(1e-8, 12)
        assert conv.all()
        res.append((groups, m.mase_state(), iters))
        m.close()
    say("  groups", res[0][0], "->", res[1][0])
    assert res[0][0] == 1 and res[1][0] >= 1
    np.testing.assert_array_equal(res[0][1][0], res[1][1][0])
    np.testing.assert_array_equal(res[0][1][1], res[1][1][1])
    np.testing.assert_array_equal(res[0][2], res[1][2])


def test_high_weight_rows_match_oracle():
    # the top of the weight range FP64 is kept for (Eq. 2, W = R^-1): every
    # 10th |V| row and every 10th active from-end flow row measured with
    # sigma = 1e-4 (w = 1e8) beside the other rows' w = 1.6e4 - 6.3e4, so the
    # weights span 1e4 - 1e8; states within 1e-8 of the oracle
    say("weights up to 1e8")
    c = Case("c1", 3, seed=31)
    t = c.t
    hi = np.concatenate([np.nonzero(t == synth.VM)[0][::10], np.nonzero(t == synth.PF)[0][::10]])
    sig = np.asarray(c.s, dtype=np.float64).copy()
    sig[hi] = 1e-4
    for i in range(c.n_snap):
        h = c.net.h(c.vm_true[i], c.va_true[i])
        c.z[i, hi] = h[hi] + sig[hi] * c.batch.eps[i, hi]
    c.w = 1.0 / sig ** 2
    assert c.w.max() / c.w.min() >= 1e4 - 1
    m = c.ctx()
    iters, conv = m.mase_solve(1e-6, 10)
    vm, va = m.mase_state()
    J = m.mase_objective()
    for i in range(c.n_snap):
        ref = c.oracle_solve(i)
        assert conv[i] and ref["converged"]
        assert iters[i] == ref["iters"], (iters[i], ref["iters"])
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
        assert abs(J[i] - ref["J"]) <= 1e-8 * ref["J"]
    m.close()


@pytest.mark.parametrize("npipe", [1, 2])
def test_failed_snapshot_leaves_the_others_solved(npipe):
    # NaN measurements in one snapshot: its state turns NaN and the next
    # iteration's factorisation meets a non-positive (NaN) pivot; that
    # snapshot is frozen and reported, every other one is solved as usual
    say("one failing snapshot, pipeline groups", npipe)
    c = Case("c1", 6, seed=33)
    c.z[2, :] = np.nan
    m = c.ctx(pipeline_groups=npipe)
    iters = np.zeros(6, dtype=np.int32)
    conv = np.zeros(6, dtype=np.int32)
    import ctypes
    rc = m.lib.mase_solve(m.ctx, 1e-6, 10, iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          conv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert rc == mase.MASE_ERR_NOT_POSDEF
    assert conv[2] == 0 and conv[[0, 1, 3, 4, 5]].all(), conv
    vm, va = m.mase_state()
    for i in (0, 1, 3, 4, 5):
        ref = c.oracle_solve(i)
        assert iters[i] == ref["iters"], (i, iters[i], ref["iters"])
        assert_state_close(vm[i], va[i], ref["vm"], ref["va"], 1e-8)
    m.close()


@pytest.mark.parametrize("name", ["c0", "k5", "c1", "c2", "c3"])
def test_lds_elimination_bitwise_equal_to_level_engine(name, monkeypatch):
    # the areas' elimination held in LDS runs the level schedule's arithmetic
    # in the same order as the level engine over HBM: identical S_b^k after
    # one condensation and identical states after a solve (c2: five areas keep
    # their Schur block in HBM; c3: three areas too large for LDS stay on the
    # level engine beside the others)
    say("LDS elimination vs level engine", name)
    c = Case(name, 2, seed=51)
    out = []
    for env in ("1", "0"):
        monkeypatch.setenv("MASE_AREA_LDS", env)
        m = c.ctx()
        n_lds = m.mase_info("area_lds")
        assert (n_lds > 0) == (env == "1"), n_lds
        m.mase_stage_assemble()
        m.mase_stage_condense()
        S = [m.mase_read_schur(1, k) for k in range(c.g.n_area)]
        m.mase_set_state()
        it, conv = m.mase_solve(1e-6, 10)
        out.append((S, m.mase_state(), it, n_lds))
        m.close()
    say("  areas in LDS:", out[0][3], "of", c.g.n_area)
    for k in range(c.g.n_area):
        np.testing.assert_array_equal(out[0][0][k][0], out[1][0][k][0])
        np.testing.assert_array_equal(out[0][0][k][1], out[1][0][k][1])
    np.testing.assert_array_equal(out[0][1][0], out[1][1][0])
    np.testing.assert_array_equal(out[0][1][1], out[1][1][1])
    np.testing.assert_array_equal(out[0][2], out[1][2])
