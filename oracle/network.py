"""Oracle: branch model, measurement functions h(x) and analytic Jacobian H.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the paper's measurement model z = h(x) + e (Section 2.1, Eq. 1) in
the bus-branch formulation: the state stacks bus voltage angles theta and
magnitudes |V|; z holds |V|, active/reactive injections and active/reactive
branch flows; each row has a type tau(i) and parameters p_i (Eq. 4).

Branch model (the paper does not spell it out; standard pi model, no taps, no
phase shift, no bus shunts): series admittance y = 1/(r + jx) = g + j*b_s and
half of the total line charging b at each end.  Injections use the bus
admittance matrix; flows use the two-port of each branch.  Both are the
textbook formulas (Abur and Exposito, "Power System State Estimation",
Ch. 2), written with numpy so that they also accept complex states (used by
the complex-step Jacobian pin).

The slack bus angle is fixed at 0 and is not a state variable, so the state
has n = 2N - 1 entries: the paper's PEGASE-2869 count 5737 = 2*2869 - 1
(Section 5.2) fixes this reading.  Column order of H: theta of every non-slack
bus in bus order, then |V| of every bus in bus order.

Pins (tests/test_oracle_network.py): closed forms of a lossless 2-bus line
(r = 0, b = 0: P_f = V_f V_t sin(theta_ft) / x and the matching Q_f, P_t, Q_t),
the complex-power definition S = V conj(Y V) computed with complex arithmetic,
Kirchhoff's current law (injection = sum of flows leaving the bus),
finite-difference and complex-step Jacobians.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

VM, PINJ, QINJ, PF, QF, PT, QT = range(7)


class Network:
    """Grid arrays plus the measurement list (types, locations, sigmas)."""

    def __init__(self, n_bus, br_from, br_to, br_r, br_x, br_b, slack,
                 meas_type, meas_at, meas_sigma):
        self.n_bus = int(n_bus)
        self.f = np.asarray(br_from, dtype=np.int64)
        self.t = np.asarray(br_to, dtype=np.int64)
        self.r = np.asarray(br_r, dtype=np.float64)
        self.x = np.asarray(br_x, dtype=np.float64)
        self.bc = np.asarray(br_b, dtype=np.float64)
        self.slack = int(slack)
        self.mtype = np.asarray(meas_type, dtype=np.int64)
        self.mat = np.asarray(meas_at, dtype=np.int64)
        self.sigma = np.asarray(meas_sigma, dtype=np.float64)
        self.n_branch = self.f.shape[0]
        self.m = self.mtype.shape[0]
        self.n = 2 * self.n_bus - 1
        # series admittance y = 1/(r + jx)
        y = 1.0 / (self.r + 1j * self.x)
        self.g = y.real
        self.bs = y.imag
        self.Y = self._ybus()
        coo = self.Y.tocoo()
        self.yi = coo.row.astype(np.int64)
        self.yj = coo.col.astype(np.int64)
        self.yG = coo.data.real.copy()
        self.yB = coo.data.imag.copy()
        self.Gdiag = self.Y.diagonal().real.copy()
        self.Bdiag = self.Y.diagonal().imag.copy()
        # state column maps
        self.col_th = np.full(self.n_bus, -1, dtype=np.int64)
        nonslack = np.array([b for b in range(self.n_bus) if b != self.slack], dtype=np.int64)
        self.col_th[nonslack] = np.arange(self.n_bus - 1)
        self.col_v = (self.n_bus - 1) + np.arange(self.n_bus)

    def _ybus(self):
        y = 1.0 / (self.r + 1j * self.x)
        half = 0.5j * self.bc
        rows = np.concatenate([self.f, self.t, self.f, self.t])
        cols = np.concatenate([self.f, self.t, self.t, self.f])
        vals = np.concatenate([y + half, y + half, -y, -y])
        return sp.coo_matrix((vals, (rows, cols)), shape=(self.n_bus, self.n_bus)).tocsr()

    # ---- state vector helpers -------------------------------------------
    def pack(self, vm, va):
        x = np.empty(self.n, dtype=np.result_type(vm, va))
        x[self.col_th[self.col_th >= 0]] = np.delete(va, self.slack)
        x[self.col_v] = vm
        return x

    def unpack(self, x):
        va = np.zeros(self.n_bus, dtype=x.dtype)
        mask = self.col_th >= 0
        va[mask] = x[self.col_th[mask]]
        vm = x[self.col_v].copy()
        return vm, va

    # ---- measurement functions (Eq. 1, Eq. 4) ----------------------------
    def flows(self, vm, va):
        """P_f, Q_f, P_t, Q_t of every branch (pi model)."""
        f, t, g, bs, hb = self.f, self.t, self.g, self.bs, 0.5 * self.bc
        vf, vt = vm[f], vm[t]
        d = va[f] - va[t]
        c, s = np.cos(d), np.sin(d)
        pf = g * vf * vf - vf * vt * (g * c + bs * s)
        qf = -(bs + hb) * vf * vf - vf * vt * (g * s - bs * c)
        # to end: swap f and t, angle difference changes sign
        pt = g * vt * vt - vt * vf * (g * c - bs * s)
        qt = -(bs + hb) * vt * vt - vt * vf * (-g * s - bs * c)
        return pf, qf, pt, qt

    def injections(self, vm, va):
        """P_i, Q_i = V_i sum_j V_j (G_ij cos th_ij +- B_ij sin th_ij)."""
        i, j = self.yi, self.yj
        d = va[i] - va[j]
        c, s = np.cos(d), np.sin(d)
        tp = vm[i] * vm[j] * (self.yG * c + self.yB * s)
        tq = vm[i] * vm[j] * (self.yG * s - self.yB * c)
        dt = np.result_type(vm, va)
        p = np.zeros(self.n_bus, dtype=dt)
        q = np.zeros(self.n_bus, dtype=dt)
        np.add.at(p, i, tp)
        np.add.at(q, i, tq)
        return p, q

    def h(self, vm, va):
        """Measurement vector h(x) in the order of the measurement list."""
        p, q = self.injections(vm, va)
        pf, qf, pt, qt = self.flows(vm, va)
        table = [vm, p, q, pf, qf, pt, qt]
        out = np.empty(self.m, dtype=np.result_type(vm, va))
        for ty in range(7):
            sel = self.mtype == ty
            out[sel] = table[ty][self.mat[sel]]
        return out

    def h_x(self, x):
        vm, va = self.unpack(x)
        return self.h(vm, va)

    # ---- analytic Jacobian H = dh/dx (Eq. 3) -----------------------------
    def jacobian(self, vm, va):
        """Sparse H (m x n), structural entries kept even when numerically 0."""
        rows, cols, vals = [], [], []

        def put(r, c, v):
            keep = c >= 0
            rows.append(r[keep])
            cols.append(c[keep])
            vals.append(v[keep])

        p, q = self.injections(vm, va)
        f, t, g, bs, hb = self.f, self.t, self.g, self.bs, 0.5 * self.bc
        vf, vt = vm[f], vm[t]
        d = va[f] - va[t]
        c, s = np.cos(d), np.sin(d)
        # partials of every branch quantity w.r.t. (th_f, th_t, V_f, V_t)
        d_pf = (vf * vt * (g * s - bs * c), -vf * vt * (g * s - bs * c),
                2 * g * vf - vt * (g * c + bs * s), -vf * (g * c + bs * s))
        d_qf = (-vf * vt * (g * c + bs * s), vf * vt * (g * c + bs * s),
                -2 * (bs + hb) * vf - vt * (g * s - bs * c), -vf * (g * s - bs * c))
        d_pt = (-vt * vf * (-g * s - bs * c), vt * vf * (-g * s - bs * c),
                -vt * (g * c - bs * s), 2 * g * vt - vf * (g * c - bs * s))
        d_qt = (vt * vf * (g * c - bs * s), -vt * vf * (g * c - bs * s),
                -vt * (-g * s - bs * c), -2 * (bs + hb) * vt - vf * (-g * s - bs * c))
        flow_d = {PF: d_pf, QF: d_qf, PT: d_pt, QT: d_qt}

        # injections: textbook partials over the bus admittance pattern
        i, j = self.yi, self.yj
        dd = va[i] - va[j]
        cc, ss = np.cos(dd), np.sin(dd)
        off = i != j
        G, B = self.yG, self.yB
        dp_dth_j = vm[i] * vm[j] * (G * ss - B * cc)
        dp_dv_j = vm[i] * (G * cc + B * ss)
        dq_dth_j = -vm[i] * vm[j] * (G * cc + B * ss)
        dq_dv_j = vm[i] * (G * ss - B * cc)
        Gd, Bd = self.Gdiag, self.Bdiag
        dp_dth_i = -q - Bd * vm * vm
        dp_dv_i = p / vm + Gd * vm
        dq_dth_i = p - Gd * vm * vm
        dq_dv_i = q / vm - Bd * vm

        for ty in range(7):
            sel = np.nonzero(self.mtype == ty)[0]
            if sel.size == 0:
                continue
            at = self.mat[sel]
            if ty == VM:
                put(sel, self.col_v[at], np.ones(sel.size, dtype=np.result_type(vm, va)))
            elif ty in (PINJ, QINJ):
                # row of bus b: diagonal entries + one entry per off-diagonal Ybus nonzero
                if ty == PINJ:
                    dth_i, dv_i, dth_j, dv_j = dp_dth_i, dp_dv_i, dp_dth_j, dp_dv_j
                else:
                    dth_i, dv_i, dth_j, dv_j = dq_dth_i, dq_dv_i, dq_dth_j, dq_dv_j
                put(sel, self.col_th[at], dth_i[at])
                put(sel, self.col_v[at], dv_i[at])
                # map bus -> measurement rows of this type at that bus
                row_of_bus = np.full(self.n_bus, -1, dtype=np.int64)
                row_of_bus[at] = sel
                k = np.nonzero(off & (row_of_bus[i] >= 0))[0]
                rr = row_of_bus[i[k]]
                put(rr, self.col_th[j[k]], dth_j[k])
                put(rr, self.col_v[j[k]], dv_j[k])
            else:
                dth_f, dth_t, dv_f, dv_t = (a[at] for a in flow_d[ty])
                put(sel, self.col_th[f[at]], dth_f)
                put(sel, self.col_th[t[at]], dth_t)
                put(sel, self.col_v[f[at]], dv_f)
                put(sel, self.col_v[t[at]], dv_t)
        R = np.concatenate(rows)
        C = np.concatenate(cols)
        V = np.concatenate(vals)
        return sp.coo_matrix((V, (R, C)), shape=(self.m, self.n)).tocsr()

    def jacobian_x(self, x):
        vm, va = self.unpack(x)
        return self.jacobian(vm, va)


def from_grid(grid, meas_type, meas_at, meas_sigma, slack=None) -> Network:
    """Build a Network from a gridgen.Grid and a measurement list."""
    return Network(grid.n_bus, grid.br_from, grid.br_to, grid.br_r, grid.br_x, grid.br_b,
                   grid.slack if slack is None else slack, meas_type, meas_at, meas_sigma)


def measurements(net: Network, vm_true, va_true, eps):
    """z = h(x_true) + sigma * eps for one snapshot (Eq. 1); eps ~ N(0, 1)."""
    return net.h(vm_true, va_true) + net.sigma * eps
