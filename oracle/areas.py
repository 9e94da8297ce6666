"""Oracle: multi-area maps, local normal-equation blocks, Schur condensation.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 2.3 and Section 3 of the paper, written out densely:

* Boundary buses are the terminal buses of cut branches (branches whose ends
  lie in different areas).
* Area k's variables: internal variables x_i^k (theta, |V| of its buses that
  are not boundary buses) and boundary variables x_b^k.  The local boundary set
  is the area's own boundary buses plus the foreign terminal of each of its
  cut branches, so local boundary vectors of neighbouring areas overlap
  (Section 2.3).
* Measurement assignment (the paper leaves it implicit; this reading makes
  the condensation exact): |V| and injections at bus i belong to area(i); a
  from-end flow belongs to area(from); a to-end flow to area(to).
* x_Gamma stacks the variables of all boundary buses; the selector E_k picks
  area k's local boundary variables out of it (Eq. 5).
* Local blocks (Eq. 7): G^k = H_k^T W_k H_k and b^k = H_k^T W_k r_k over
  area k's rows and local variables, split into ii / ib / bb parts.
* Condensation (Eq. 8-10): S_b^k = G_bb - G_bi G_ii^-1 G_ib,
  bhat_b^k = b_b - G_bi G_ii^-1 b_i (dense numpy solves).
* Coordinator (Eq. 11): S_Gamma = sum_k E_k^T S_b^k E_k,
  bhat_Gamma = sum_k E_k^T bhat_b^k; solve S_Gamma dx_Gamma = bhat_Gamma;
  dx_b^k = E_k dx_Gamma; dx_i^k = G_ii^-1 (b_i - G_ib dx_b^k) (Eq. 8).

Canonical orders used for every export and comparison:

* global variable id of a bus b: 2*b for theta (never for the slack bus),
  2*b + 1 for |V|;
* area k's local variables: its internal buses in increasing bus id, then its
  local boundary buses in increasing bus id, each bus contributing theta
  (unless slack) then |V|;
* Gamma: boundary buses in increasing bus id, theta (unless slack) then |V|.

Pins (tests/test_oracle_areas.py): the condensed step equals the centralized step
of oracle.wls for K = 1, 2, 3 (block elimination is exact); G_ii^k and G_ib^k
are slices of the centralized G and the E_k-assembled G_bb^k add up to
G_Gamma,Gamma; on tiny grids the maps agree with a brute-force enumeration;
the symbolic pattern contains every numerically nonzero entry at random states.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .network import Network, VM, PINJ, QINJ, PF, QF, PT, QT


class Areas:
    def __init__(self, net: Network, bus_area, n_area: int):
        self.net = net
        self.area = np.asarray(bus_area, dtype=np.int64)
        self.K = int(n_area)
        f, t = net.f, net.t
        cut = self.area[f] != self.area[t]
        self.cut = cut
        bnd = np.zeros(net.n_bus, dtype=bool)
        bnd[f[cut]] = True
        bnd[t[cut]] = True
        self.is_boundary = bnd

        # measurement -> area
        ma = np.empty(net.m, dtype=np.int64)
        bus_rows = np.isin(net.mtype, (VM, PINJ, QINJ))
        ma[bus_rows] = self.area[net.mat[bus_rows]]
        fr = np.isin(net.mtype, (PF, QF))
        ma[fr] = self.area[f[net.mat[fr]]]
        tr = np.isin(net.mtype, (PT, QT))
        ma[tr] = self.area[t[net.mat[tr]]]
        self.meas_area = ma

        # Gamma
        self.gamma_buses = np.nonzero(bnd)[0]
        self.gamma_vars = self._vars_of(self.gamma_buses)
        self.gamma_index = {v: i for i, v in enumerate(self.gamma_vars.tolist())}

        self.internal_buses, self.boundary_buses = [], []
        self.local_vars, self.n_internal_vars, self.E = [], [], []
        for k in range(self.K):
            own = np.nonzero(self.area == k)[0]
            internal = own[~bnd[own]]
            lb = set(own[bnd[own]].tolist())
            ck = np.nonzero(cut & ((self.area[f] == k) | (self.area[t] == k)))[0]
            lb.update(f[ck].tolist())
            lb.update(t[ck].tolist())
            lb = np.array(sorted(lb), dtype=np.int64)
            self.internal_buses.append(internal)
            self.boundary_buses.append(lb)
            vi = self._vars_of(internal)
            vb = self._vars_of(lb)
            self.local_vars.append(np.concatenate([vi, vb]))
            self.n_internal_vars.append(vi.size)
            self.E.append(np.array([self.gamma_index[v] for v in vb.tolist()], dtype=np.int64))

    def _vars_of(self, buses):
        out = []
        for b in np.asarray(buses).tolist():
            if b != self.net.slack:
                out.append(2 * b)
            out.append(2 * b + 1)
        return np.array(out, dtype=np.int64)

    # ---- variable id <-> oracle column ------------------------------------
    def columns(self, var_ids):
        var_ids = np.asarray(var_ids, dtype=np.int64)
        bus = var_ids // 2
        is_v = (var_ids % 2) == 1
        return np.where(is_v, self.net.col_v[bus], self.net.col_th[bus])

    # ---- local blocks (Eq. 7) ----------------------------------------------
    def local_system(self, k, z, vm, va, w=None):
        """G^k (dense, canonical local order) and b^k from area k's rows only."""
        net = self.net
        W = 1.0 / net.sigma ** 2 if w is None else np.asarray(w, dtype=np.float64)
        rows = np.nonzero(self.meas_area == k)[0]
        H = net.jacobian(vm, va)[rows]
        cols = self.columns(self.local_vars[k])
        Hk = H[:, cols].toarray()
        # every nonzero of area k's rows must lie in its local variables
        Hfull = H.toarray()
        rest = np.ones(net.n, dtype=bool)
        rest[cols] = False
        assert not np.any(Hfull[:, rest]), "area rows touch non-local variables"
        r = z[rows] - net.h(vm, va)[rows]
        Wk = W[rows]
        G = Hk.T @ (Wk[:, None] * Hk)
        b = Hk.T @ (Wk * r)
        return G, b

    def condense(self, k, G, b):
        """S_b^k and bhat_b^k (Eq. 9-10)."""
        ni = self.n_internal_vars[k]
        Gii, Gib, Gbi, Gbb = G[:ni, :ni], G[:ni, ni:], G[ni:, :ni], G[ni:, ni:]
        X = np.linalg.solve(Gii, np.column_stack([Gib, b[:ni]]))
        S = Gbb - Gbi @ X[:, :-1]
        bh = b[ni:] - Gbi @ X[:, -1]
        return S, bh

    def condensed_step(self, z, vm, va, w=None, detail=False):
        """One GN step by boundary condensation (Eq. 8-11); dx in oracle column order."""
        ng = self.gamma_vars.size
        SG = np.zeros((ng, ng))
        bG = np.zeros(ng)
        systems = []
        for k in range(self.K):
            G, b = self.local_system(k, z, vm, va, w)
            S, bh = self.condense(k, G, b)
            E = self.E[k]
            SG[np.ix_(E, E)] += S
            np.add.at(bG, E, bh)
            systems.append((G, b, S, bh))
        dG = np.linalg.solve(SG, bG) if ng else np.zeros(0)
        dx = np.zeros(self.net.n)
        if ng:
            dx[self.columns(self.gamma_vars)] = dG
        for k in range(self.K):
            G, b, _, _ = systems[k]
            ni = self.n_internal_vars[k]
            dxb = dG[self.E[k]]
            dxi = np.linalg.solve(G[:ni, :ni], b[:ni] - G[:ni, ni:] @ dxb)
            dx[self.columns(self.local_vars[k][:ni])] = dxi
        if detail:
            return dx, {"systems": systems, "S_gamma": SG, "b_gamma": bG, "dx_gamma": dG}
        return dx

    # ---- symbolic structure --------------------------------------------------
    def local_step(self, z, vm, va, w=None):
        """One Gauss-Newton step of every area's local WLS problem with its
        boundary variables held as parameters (Eq. 6): in the block normal
        equations (Eq. 7) with dx_b = 0 the first block row gives
        G_ii^k dx_i^k = b_i^k.  Each internal variable belongs to one area, so
        the per-area steps combine into one vector; boundary entries stay 0.
        Oracle column order."""
        dx = np.zeros(self.net.n)
        for k in range(self.K):
            G, b = self.local_system(k, z, vm, va, w)
            ni = self.n_internal_vars[k]
            if ni:
                dx[self.columns(self.local_vars[k][:ni])] = np.linalg.solve(G[:ni, :ni], b[:ni])
        return dx

    def pattern(self, k):
        """Scalar symbolic pattern of G^k as CSR (rowptr, colidx), canonical order.

        Built from the structural nonzeros of area k's Jacobian rows (boolean
        product H_k^T H_k with all-ones values, so no cancellation).
        """
        net = self.net
        rows = np.nonzero(self.meas_area == k)[0]
        H = net.jacobian(np.ones(net.n_bus), np.zeros(net.n_bus))[rows]
        cols = self.columns(self.local_vars[k])
        Hk = H[:, cols].tocsr().astype(np.float64)
        Hk.data[:] = 1.0
        P = (Hk.T @ Hk).tocsr()
        P.sort_indices()
        return P.indptr.astype(np.int32), P.indices.astype(np.int32)


def centralized_G(net: Network, z, vm, va, w=None):
    """Dense G = H^T W H and rhs of the whole grid (oracle column order)."""
    W = 1.0 / net.sigma ** 2 if w is None else np.asarray(w, dtype=np.float64)
    H = net.jacobian(vm, va).toarray()
    r = z - net.h(vm, va)
    return H.T @ (W[:, None] * H), H.T @ (W * r)


def dense_lower_from_csr(n, rowptr, colidx):
    """Boolean dense matrix from a CSR pattern (test helper)."""
    M = np.zeros((n, n), dtype=bool)
    for i in range(n):
        M[i, colidx[rowptr[i]:rowptr[i + 1]]] = True
    return M


__all__ = ["Areas", "centralized_G", "dense_lower_from_csr", "sp"]
