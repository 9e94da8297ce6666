"""Pins for oracle.network: measurement functions and Jacobian.

Each check is independent of the formulas the oracle implements:
closed forms of a lossless line, the complex-power definition S = V conj(I)
with the admittance matrix built from the incidence matrix, Kirchhoff's
current law, finite differences and the complex step.
"""
import math

import numpy as np
import pytest

from gridgen import synth
from oracle import network as nw


def two_bus(r, x, b, vm, va):
    t, a, s = synth.measurement_set(2, 1)
    net = nw.Network(2, [0], [1], [r], [x], [b], 0, t, a, s)
    return net, net.h(np.array(vm, float), np.array(va, float))


def test_lossless_line_closed_forms():
    # r = 0, b = 0: P_f = V_f V_t sin(th_ft)/x, Q_f = (V_f^2 - V_f V_t cos th_ft)/x
    vf, vt, thf, tht, x = 1.0, 0.9, 0.0, -0.1, 0.5
    net, h = two_bus(0.0, x, 0.0, [vf, vt], [thf, tht])
    d = thf - tht
    pf = vf * vt * math.sin(d) / x
    qf = (vf * vf - vf * vt * math.cos(d)) / x
    pt = -pf
    qt = (vt * vt - vf * vt * math.cos(d)) / x
    # order: VM0 VM1 P0 P1 Q0 Q1 PF QF PT QT
    expect = [vf, vt, pf, pt, qf, qt, pf, qf, pt, qt]
    np.testing.assert_allclose(h, expect, rtol=0, atol=1e-14)


def _complex_reference(net, vm, va):
    """S_bus = V conj(Y V), S_f = V_f conj(I_f) from first principles."""
    n, nb = net.n_bus, net.n_branch
    V = vm * np.exp(1j * va)
    y = 1.0 / (net.r + 1j * net.x)
    # incidence C: +1 at from, -1 at to; Y = C^T diag(y) C + diag(charging)
    C = np.zeros((nb, n))
    C[np.arange(nb), net.f] = 1.0
    C[np.arange(nb), net.t] = -1.0
    Y = C.T @ np.diag(y) @ C
    ch = np.zeros(n, complex)
    np.add.at(ch, net.f, 0.5j * net.bc)
    np.add.at(ch, net.t, 0.5j * net.bc)
    Y = Y + np.diag(ch)
    S = V * np.conj(Y @ V)
    If = (V[net.f] - V[net.t]) * y + 0.5j * net.bc * V[net.f]
    It = (V[net.t] - V[net.f]) * y + 0.5j * net.bc * V[net.t]
    Sf = V[net.f] * np.conj(If)
    St = V[net.t] * np.conj(It)
    return S, Sf, St


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_complex_power_definition(seed):
    g = synth.make_grid(30, 41, 3, seed=seed)
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    net = nw.from_grid(g, t, a, s)
    rng = np.random.default_rng(100 + seed)
    vm = rng.uniform(0.9, 1.1, g.n_bus)
    va = rng.uniform(-0.5, 0.5, g.n_bus)
    S, Sf, St = _complex_reference(net, vm, va)
    p, q = net.injections(vm, va)
    pf, qf, pt, qt = net.flows(vm, va)
    np.testing.assert_allclose(p, S.real, atol=1e-12)
    np.testing.assert_allclose(q, S.imag, atol=1e-12)
    np.testing.assert_allclose(pf, Sf.real, atol=1e-12)
    np.testing.assert_allclose(qf, Sf.imag, atol=1e-12)
    np.testing.assert_allclose(pt, St.real, atol=1e-12)
    np.testing.assert_allclose(qt, St.imag, atol=1e-12)


def test_kcl_injection_equals_sum_of_flows():
    g = synth.make_config("c1")
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    net = nw.from_grid(g, t, a, s)
    p, q = net.injections(g.vm, g.va)
    pf, qf, pt, qt = net.flows(g.vm, g.va)
    ps = np.zeros(g.n_bus)
    qs = np.zeros(g.n_bus)
    np.add.at(ps, net.f, pf)
    np.add.at(ps, net.t, pt)
    np.add.at(qs, net.f, qf)
    np.add.at(qs, net.t, qt)
    np.testing.assert_allclose(p, ps, atol=1e-11)
    np.testing.assert_allclose(q, qs, atol=1e-11)


def test_measurement_vector_layout():
    g = synth.make_config("c0")
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    assert t.size == 3 * g.n_bus + 4 * g.n_branch
    net = nw.from_grid(g, t, a, s)
    h = net.h(g.vm, g.va)
    np.testing.assert_array_equal(h[:g.n_bus], g.vm)
    assert net.n == 2 * g.n_bus - 1


@pytest.mark.parametrize("seed", [0, 3])
def test_jacobian_finite_difference(seed):
    g = synth.make_grid(30, 41, 3, seed=seed)
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    net = nw.from_grid(g, t, a, s)
    rng = np.random.default_rng(seed)
    x = net.pack(rng.uniform(0.9, 1.1, g.n_bus), rng.uniform(-0.4, 0.4, g.n_bus))
    H = net.jacobian_x(x).toarray()
    eps = 1e-6
    Hfd = np.empty_like(H)
    for j in range(net.n):
        e = np.zeros(net.n)
        e[j] = eps
        Hfd[:, j] = (net.h_x(x + e) - net.h_x(x - e)) / (2 * eps)
    np.testing.assert_allclose(H, Hfd, atol=1e-7)


@pytest.mark.parametrize("seed", [0, 5])
def test_jacobian_complex_step(seed):
    # h is analytic in x, so Im h(x + i*eps*e_j)/eps is dh/dx_j to rounding
    g = synth.make_grid(30, 41, 3, seed=seed)
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    net = nw.from_grid(g, t, a, s)
    rng = np.random.default_rng(seed + 7)
    x = net.pack(rng.uniform(0.9, 1.1, g.n_bus), rng.uniform(-0.4, 0.4, g.n_bus))
    H = net.jacobian_x(x).toarray()
    eps = 1e-30
    Hcs = np.empty_like(H)
    for j in range(net.n):
        e = np.zeros(net.n, complex)
        e[j] = 1j * eps
        Hcs[:, j] = net.h_x(x + e).imag / eps
    np.testing.assert_allclose(H, Hcs, rtol=1e-13, atol=1e-13)


def test_jacobian_structure_kept_at_flat_start():
    # structural entries stay even where a partial is numerically zero
    g = synth.make_config("c0")
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    net = nw.from_grid(g, t, a, s)
    H = net.jacobian(np.ones(g.n_bus), np.zeros(g.n_bus))
    deg = np.bincount(np.concatenate([net.f, net.t]), minlength=g.n_bus)
    row_nnz = np.diff(H.indptr)
    nonslack = lambda b: 2 - (b == net.slack)
    for i in range(net.m):
        ty, at = net.mtype[i], net.mat[i]
        if ty == nw.VM:
            assert row_nnz[i] == 1
        elif ty in (nw.PINJ, nw.QINJ):
            nb = [at] + [int(v) for v in np.concatenate([net.t[net.f == at], net.f[net.t == at]])]
            assert row_nnz[i] == sum(nonslack(b) for b in nb)
            assert len(nb) == deg[at] + 1
        else:
            e = at
            assert row_nnz[i] == nonslack(net.f[e]) + nonslack(net.t[e])
