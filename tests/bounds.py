"""Per-entry rounding-error bounds for the stage parity tests.

The GPU and the oracle compute G^k = H_k^T W_k H_k, b^k = H_k^T W_k r_k
(Eq. 7) and S_b^k = G_bb - G_bi G_ii^-1 G_ib (Eq. 9) with different formulas
and summation orders, so their results differ by rounding.  A bound relative
to a matrix's largest entry leaves its small entries unchecked (G entries of
one block span about four orders of magnitude), so these helpers bound every
entry separately:

* T_r bounds the sum of absolute values of the terms that make up h_r and
  each of its partial derivatives (pi model: every term is a product of two
  |V| and one of |g|, |b_s|, |b_c / 2|).  A computed partial then carries an
  absolute error of a few eps * T_r.
* G: |dG_ab| <= c eps M_ab with M = sum over rows touching both a and b of
  w_r T_r^2 (a partial's error times the other partial, plus the summation).
* b: |db_a| <= c eps sum_r w_r T_r (T_r + |z_r|) (the residual z - h carries
  an error of eps * T_r; |r| <= |z| + T_r).
* S_b: to first order a perturbation dG moves the Schur complement by
  dG_bb - dG_bi X - X^T dG_ib + X^T dG_ii X with X = G_ii^-1 G_ib, and the
  Cholesky elimination itself is backward stable with |dG| <= c eps |L||L^T|
  (Higham, Accuracy and Stability of Numerical Algorithms, Thm. 10.3).  The
  bound takes |dG| <= c eps (M + |L||L^T|) entrywise and pushes it through
  the first-order formula in absolute values.
The constants c cover both sides' errors; the tests print the largest ratio
error / bound seen.
"""
import numpy as np

from oracle.network import VM, PINJ, QINJ, PF, QF, PT, QT

EPS = np.finfo(np.float64).eps


def row_terms(net, vm):
    """T_r for every measurement row at the state magnitudes vm."""
    g, bs, hb = np.abs(net.g), np.abs(net.bs), 0.5 * np.abs(net.bc)
    ym = g + bs + hb
    f, t = net.f, net.t
    br = 2.0 * (vm[f] + vm[t]) ** 2 * ym          # per branch, either end
    inj = np.zeros(net.n_bus)
    np.add.at(inj, f, br)
    np.add.at(inj, t, br)
    T = np.ones(net.m)
    ty, at = net.mtype, net.mat
    isinj = (ty == PINJ) | (ty == QINJ)
    T[isinj] = inj[at[isinj]]
    isfl = ty >= PF
    T[isfl] = br[at[isfl]]
    return T


def row_buses(net, r):
    """Buses whose variables row r depends on."""
    ty, at = int(net.mtype[r]), int(net.mat[r])
    if ty == VM:
        return [at]
    if ty in (PINJ, QINJ):
        nb = list(net.t[net.f == at]) + list(net.f[net.t == at])
        return [at] + nb
    return [int(net.f[at]), int(net.t[at])]


def local_magnitudes(A, k, z, vm, w=None):
    """M_G [n_local x n_local] and M_b [n_local] of area k, canonical order."""
    net = A.net
    W = 1.0 / net.sigma ** 2 if w is None else np.asarray(w, dtype=np.float64)
    T = row_terms(net, vm)
    pos = {int(v): i for i, v in enumerate(A.local_vars[k])}
    n = len(pos)
    MG = np.zeros((n, n))
    Mb = np.zeros(n)
    for r in np.nonzero(A.meas_area == k)[0]:
        idx = []
        for b in row_buses(net, r):
            for v in (2 * b, 2 * b + 1):
                if v in pos:
                    idx.append(pos[v])
        idx = np.array(idx)
        MG[np.ix_(idx, idx)] += W[r] * T[r] ** 2
        Mb[idx] += W[r] * T[r] * (T[r] + abs(z[r]))
    return MG, Mb


def schur_bound(G, MG, ni, c_in, c_chol):
    """First-order entrywise bound on the error of S_b = G_bb - G_bi G_ii^-1 G_ib."""
    # factor of the interior block and the boundary rows below it (the
    # boundary block itself is left as the Schur complement, not factored)
    Lii = np.linalg.cholesky(G[:ni, :ni])
    Lbi = np.linalg.solve(Lii, G[:ni, ni:]).T
    L = np.vstack([Lii, Lbi])
    LL = np.abs(L) @ np.abs(L).T
    dG = c_in * EPS * MG + c_chol * EPS * LL
    X = np.abs(np.linalg.solve(G[:ni, :ni], G[:ni, ni:]))
    return dG[ni:, ni:] + dG[ni:, :ni] @ X + X.T @ dG[:ni, ni:] + X.T @ dG[:ni, :ni] @ X


def check_entries(a, ref, bound, what):
    """Every |a - ref| <= bound; returns the largest ratio."""
    err = np.abs(a - ref)
    ratio = float(np.max(err / np.maximum(bound, np.finfo(float).tiny))) if a.size else 0.0
    bad = err > bound
    assert not bad.any(), (f"{what}: {int(bad.sum())} entries over their bound, "
                           f"largest ratio {ratio:.3g}")
    return ratio
