"""Pins for oracle.wls: centralized WLS Gauss-Newton.

* noise-free measurements: the generating state is an exact zero of the
  residual, so GN from flat start must return it (to 1e-10);
* the objective at the estimate follows its chi-square law with m - n degrees
  of freedom, as the paper's own printed objectives do (golden fixture);
* the GN step equals numpy's dense least-squares solution of the linearised
  weighted problem;
* a zero weight is the same as deleting the row (Section 4.1).
"""
import json
import math
import os

import numpy as np
import pytest

from gridgen import synth
from oracle import network as nw
from oracle import wls

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


def _setup(name, seed=0):
    g = synth.make_config(name, seed)
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    return g, nw.from_grid(g, t, a, s)


def test_paper_counts_fix_readings():
    gold = json.load(open(GOLDEN))
    c = gold["state_variable_count"]
    t, a, s = synth.measurement_set(c["n_bus"], c["n_branch"])
    net = nw.Network(c["n_bus"], [0], [1], [0.1], [0.1], [0.0], 0, t[:1], a[:1], s[:1])
    assert net.n == c["state_variables"]  # n = 2N - 1: slack angle removed
    mk = gold["masking"]
    t, _, _ = synth.measurement_set(mk["n_bus"], mk["n_branch"])
    assert int(np.sum(t == synth.PF)) == mk["removed_rows"]
    assert round(100.0 * mk["removed_rows"] / t.size, 2) == mk["removed_percent"]  # m = 3N + 4B


def test_paper_objectives_are_chi_square():
    # printed "objective" is r'Wr / 2 and the residual norm sqrt(r'Wr);
    # r'Wr then sits within 4 standard deviations of m - n.
    gold = json.load(open(GOLDEN))["converged_objectives"]["grids"]
    for gr in gold:
        rwr = gr["weighted_residual_norm"] ** 2
        assert abs(rwr - 2 * gr["objective"]) < 2 * gr["weighted_residual_norm"] * 0.005 + 1e-9
        m = 3 * gr["n_bus"] + 4 * gr["n_branch"]
        n = 2 * gr["n_bus"] - 1
        assert abs(rwr - (m - n)) < 4 * math.sqrt(2 * (m - n))


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_noise_free_recovery(name):
    g, net = _setup(name)
    z = net.h(g.vm, g.va)
    out = wls.gauss_newton(net, z, tol=1e-12, max_iter=15)
    assert out["converged"]
    np.testing.assert_allclose(out["vm"], g.vm, rtol=0, atol=1e-10)
    np.testing.assert_allclose(out["va"], g.va, rtol=0, atol=1e-10)
    assert out["J"] < 1e-16


def test_flat_start_converges_within_cap():
    g, net = _setup("c1")
    b = synth.make_batch(g, 2, seed=0)
    for s in range(2):
        z = nw.measurements(net, b.vm_true[s], b.va_true[s], b.eps[s])
        out = wls.gauss_newton(net, z, tol=1e-6, max_iter=10)
        assert out["converged"] and 2 <= out["iters"] <= 10
        m, n = net.m, net.n
        assert abs(out["J"] - (m - n)) <= 4 * math.sqrt(2 * (m - n))


def test_chi_square_mean_over_seeds():
    g, net = _setup("c0")
    m, n = net.m, net.n
    Js = []
    for seed in range(400):
        eps = np.random.default_rng(1000 + seed).standard_normal(net.m)
        z = nw.measurements(net, g.vm, g.va, eps)
        out = wls.gauss_newton(net, z, tol=1e-10, max_iter=20)
        assert out["converged"]
        Js.append(out["J"])
    mean = float(np.mean(Js))
    assert abs(mean / (m - n) - 1.0) < 0.02, (mean, m - n)


def test_gn_step_is_weighted_least_squares():
    g, net = _setup("c0")
    rng = np.random.default_rng(4)
    eps = rng.standard_normal(net.m)
    z = nw.measurements(net, g.vm, g.va, eps)
    vm = g.vm + rng.normal(0, 0.01, g.n_bus)
    va = g.va + rng.normal(0, 0.02, g.n_bus)
    dx = wls.gn_step(net, z, vm, va)
    sw = np.sqrt(1.0 / net.sigma ** 2)
    H = net.jacobian(vm, va).toarray()
    r = z - net.h(vm, va)
    ref, *_ = np.linalg.lstsq(sw[:, None] * H, sw * r, rcond=None)
    np.testing.assert_allclose(dx, ref, rtol=1e-9, atol=1e-12)


def test_zero_weight_equals_row_removed():
    g, net = _setup("c0")
    eps = np.random.default_rng(9).standard_normal(net.m)
    z = nw.measurements(net, g.vm, g.va, eps)
    w = 1.0 / net.sigma ** 2
    w[net.mtype == synth.QF] = 0.0
    keep = net.mtype != synth.QF
    net2 = nw.Network(g.n_bus, g.br_from, g.br_to, g.br_r, g.br_x, g.br_b, g.slack,
                      net.mtype[keep], net.mat[keep], net.sigma[keep])
    vm = g.vm * 1.01
    va = g.va * 0.9
    G1, b1 = wls.normal_equations(net, z, vm, va, w)
    G2, b2 = wls.normal_equations(net2, z[keep], vm, va)
    np.testing.assert_allclose(G1.toarray(), G2.toarray(), rtol=1e-14, atol=1e-9)
    np.testing.assert_allclose(b1, b2, rtol=1e-14, atol=1e-9)
    o1 = wls.gauss_newton(net, z, w=w)
    o2 = wls.gauss_newton(net2, z[keep])
    np.testing.assert_allclose(o1["vm"], o2["vm"], atol=1e-12)
    np.testing.assert_allclose(o1["va"], o2["va"], atol=1e-12)
