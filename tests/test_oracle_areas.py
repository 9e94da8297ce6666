"""Pins for oracle.areas: maps, local blocks and boundary condensation.

* block elimination is exact: the condensed step (Eq. 8-11) equals the
  centralized GN step for K = 1, 2, 3 and with the slack on the boundary;
* G_ii^k, G_ib^k are slices of the centralized gain matrix and the
  E_k-assembled G_bb^k add up to its boundary block;
* maps and symbolic patterns agree with brute-force enumerations written from
  the definitions (adjacency, row supports).
"""
import numpy as np
import pytest

from gridgen import synth
from oracle import areas as oa
from oracle import network as nw
from oracle import wls


def _case(K, seed=0, slack=None, mode="plain"):
    g = synth.make_grid(30, 41, K, seed=seed, mode=mode)
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    net = nw.from_grid(g, t, a, s, slack=slack)
    A = oa.Areas(net, g.bus_area, K)
    rng = np.random.default_rng(seed + 11)
    z = nw.measurements(net, g.vm, g.va, rng.standard_normal(net.m))
    vm = g.vm + rng.normal(0, 0.02, g.n_bus)
    va = g.va + rng.normal(0, 0.05, g.n_bus)
    return g, net, A, z, vm, va


@pytest.mark.parametrize("K", [1, 2, 3])
@pytest.mark.parametrize("seed", [0, 1])
def test_condensed_step_equals_centralized(K, seed):
    g, net, A, z, vm, va = _case(K, seed)
    dx_c = wls.gn_step(net, z, vm, va)
    dx_s = A.condensed_step(z, vm, va)
    np.testing.assert_allclose(dx_s, dx_c, rtol=1e-9, atol=1e-12)


def test_condensed_step_slack_on_boundary():
    g, net, A, z, vm, va = _case(3, 0)
    bnd = np.nonzero(A.is_boundary)[0]
    g2, net2, A2, z2, vm2, va2 = _case(3, 0, slack=int(bnd[0]))
    assert A2.is_boundary[net2.slack]
    dx_c = wls.gn_step(net2, z2, vm2, va2)
    dx_s = A2.condensed_step(z2, vm2, va2)
    np.testing.assert_allclose(dx_s, dx_c, rtol=1e-9, atol=1e-12)


def test_condensed_step_with_masked_rows():
    g, net, A, z, vm, va = _case(3, 2)
    w = 1.0 / net.sigma ** 2
    w[net.mtype == synth.PT] = 0.0
    np.testing.assert_allclose(A.condensed_step(z, vm, va, w), wls.gn_step(net, z, vm, va, w),
                               rtol=1e-9, atol=1e-12)


def test_local_blocks_are_slices_of_global_gain():
    g, net, A, z, vm, va = _case(3, 0)
    Gc, bc = oa.centralized_G(net, z, vm, va)
    ng = A.gamma_vars.size
    Sbb = np.zeros((ng, ng))
    bbb = np.zeros(ng)
    for k in range(A.K):
        G, b = A.local_system(k, z, vm, va)
        ni = A.n_internal_vars[k]
        cols = A.columns(A.local_vars[k])
        ci = cols[:ni]
        np.testing.assert_allclose(G[:ni, :ni], Gc[np.ix_(ci, ci)], rtol=1e-12, atol=1e-6)
        np.testing.assert_allclose(G[:ni, ni:], Gc[np.ix_(ci, cols[ni:])], rtol=1e-12, atol=1e-6)
        np.testing.assert_allclose(b[:ni], bc[ci], rtol=1e-12, atol=1e-8)
        E = A.E[k]
        Sbb[np.ix_(E, E)] += G[ni:, ni:]
        np.add.at(bbb, E, b[ni:])
    cg = A.columns(A.gamma_vars)
    np.testing.assert_allclose(Sbb, Gc[np.ix_(cg, cg)], rtol=1e-12, atol=1e-6)
    np.testing.assert_allclose(bbb, bc[cg], rtol=1e-12, atol=1e-8)


@pytest.mark.parametrize("K,mode", [(3, "plain"), (4, "balanced"), (5, "plain")])
def test_maps_brute_force(K, mode):
    g = synth.make_grid(30, 41, K, seed=3, mode=mode)
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    net = nw.from_grid(g, t, a, s)
    A = oa.Areas(net, g.bus_area, K)
    n = g.n_bus
    adj = np.zeros((n, n), dtype=bool)
    adj[g.br_from, g.br_to] = True
    adj[g.br_to, g.br_from] = True
    ar = g.bus_area
    bnd = np.array([any(adj[u, v] and ar[v] != ar[u] for v in range(n)) for u in range(n)])
    np.testing.assert_array_equal(A.is_boundary, bnd)
    gam = []
    for b in range(n):
        if bnd[b]:
            if b != net.slack:
                gam.append(2 * b)
            gam.append(2 * b + 1)
    np.testing.assert_array_equal(A.gamma_vars, gam)
    for k in range(K):
        internal = [u for u in range(n) if ar[u] == k and not bnd[u]]
        lb = [u for u in range(n) if bnd[u] and (ar[u] == k or any(adj[u, v] and ar[v] == k for v in range(n)))]
        vi = [v for u in internal for v in ([2 * u] if u != net.slack else []) + [2 * u + 1]]
        vb = [v for u in lb for v in ([2 * u] if u != net.slack else []) + [2 * u + 1]]
        np.testing.assert_array_equal(A.local_vars[k], vi + vb)
        assert A.n_internal_vars[k] == len(vi)
        np.testing.assert_array_equal(A.E[k], [gam.index(v) for v in vb])
    for i in range(net.m):
        ty, at = net.mtype[i], net.mat[i]
        owner = ar[at] if ty in (synth.VM, synth.PINJ, synth.QINJ) else (
            ar[g.br_from[at]] if ty in (synth.PF, synth.QF) else ar[g.br_to[at]])
        assert A.meas_area[i] == owner


@pytest.mark.parametrize("K", [2, 3])
def test_pattern_brute_force(K):
    g = synth.make_grid(30, 41, K, seed=1)
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    net = nw.from_grid(g, t, a, s)
    A = oa.Areas(net, g.bus_area, K)
    n = g.n_bus
    nbrs = [set() for _ in range(n)]
    for f, tt in zip(g.br_from, g.br_to):
        nbrs[f].add(int(tt))
        nbrs[tt].add(int(f))
    for k in range(K):
        lv = A.local_vars[k].tolist()
        pos = {v: i for i, v in enumerate(lv)}
        M = np.zeros((len(lv), len(lv)), dtype=bool)
        for i in np.nonzero(A.meas_area == k)[0]:
            ty, at = net.mtype[i], net.mat[i]
            if ty == synth.VM:
                vars_ = [2 * at + 1]
            else:
                buses = ({int(at)} | nbrs[at]) if ty in (synth.PINJ, synth.QINJ) else {int(g.br_from[at]), int(g.br_to[at])}
                vars_ = [v for b in buses for v in (2 * b, 2 * b + 1) if not (v == 2 * net.slack)]
            idx = [pos[v] for v in vars_]
            M[np.ix_(idx, idx)] = True
        rp, ci = A.pattern(k)
        P = oa.dense_lower_from_csr(len(lv), rp, ci)
        np.testing.assert_array_equal(P, M)
        # and every numerically nonzero entry at a random state is in it
        rng = np.random.default_rng(k)
        z = nw.measurements(net, g.vm, g.va, rng.standard_normal(net.m))
        G, _ = A.local_system(k, z, g.vm * 1.01, g.va + 0.01)
        assert not np.any((G != 0) & ~P)


# ---- local steps with the boundary fixed (Eq. 6) ------------------------------

def _internal_columns(A):
    return np.concatenate([A.columns(A.local_vars[k][:A.n_internal_vars[k]]) for k in range(A.K)])


@pytest.mark.parametrize("K", [2, 3])
def test_local_step_is_gn_in_internal_variables(K):
    # every row that touches an internal variable of area k is owned by area k,
    # so the per-area steps are the GN step of the centralized problem in the
    # internal variables with all boundary variables held: checked against the
    # centralized Jacobian restricted to the internal columns
    g, net, A, z, vm, va = _case(K, 1)
    dx = A.local_step(z, vm, va)
    H = net.jacobian(vm, va)
    H = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    w = 1.0 / net.sigma ** 2
    r = z - net.h(vm, va)
    cols = _internal_columns(A)
    HI = H[:, cols]
    ref = np.zeros(net.n)
    ref[cols] = np.linalg.solve(HI.T @ (w[:, None] * HI), HI.T @ (w * r))
    np.testing.assert_allclose(dx, ref, rtol=1e-9, atol=1e-12)
    assert (dx[A.columns(A.gamma_vars)] == 0.0).all()


def test_local_step_single_area_is_full_gn_step():
    g, net, A, z, vm, va = _case(1, 0)
    np.testing.assert_allclose(A.local_step(z, vm, va), wls.gn_step(net, z, vm, va), rtol=1e-9, atol=1e-12)


def test_local_steps_reach_local_stationarity():
    # repeated local steps solve each area's local WLS problem: its gradient in
    # the internal variables, b_i^k = H_i^T W r, vanishes
    g, net, A, z, vm, va = _case(3, 2)
    b0 = [A.local_system(k, z, vm, va)[1][:A.n_internal_vars[k]] for k in range(A.K)]
    x = net.pack(vm, va)
    for _ in range(8):
        x = x + A.local_step(z, *net.unpack(x))
    vm2, va2 = net.unpack(x)
    for k in range(A.K):
        ni = A.n_internal_vars[k]
        b = A.local_system(k, z, vm2, va2)[1][:ni]
        assert np.linalg.norm(b) < 1e-8 * np.linalg.norm(b0[k])
    # the boundary variables never moved
    cg = A.columns(A.gamma_vars)
    np.testing.assert_array_equal(x[cg], net.pack(vm, va)[cg])
