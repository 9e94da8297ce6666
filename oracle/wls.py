"""Oracle: WLS objective and centralized Gauss-Newton.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Objective (Eq. 2): J(x) = r^T W r with r = z - h(x), W = diag(w),
  w = 1/sigma^2 unless given (w = 0 masks a row, Section 4.1).
* Gauss-Newton (Eq. 3): G dx = H^T W r with G = H^T W H, x <- x + dx, using an
  explicit sparse Jacobian and a sparse LU (scipy splu) of G.
* Stopping rule (the paper gives only the 10-iteration cap of Section 5.1):
  stop after the first step whose max |dx| < tol; the iteration count is the
  number of steps taken, including that last small one.
* Flat start: |V| = 1, theta = 0.  The slack angle is the reference and stays
  0 whatever the starting point holds there.

Pins (tests/test_oracle_wls.py): noise-free measurements give back the generating
state to 1e-10 (it is an exact zero of the residual); the objective at the
estimate sits at its chi-square expectation m - n (also what the paper's
printed objectives show, Section 5.2); the GN step equals the dense
least-squares solution of the linearised problem (numpy lstsq on W^1/2 H);
masking a row with w = 0 equals deleting it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from .network import Network


def weights(net: Network, w=None):
    return 1.0 / net.sigma ** 2 if w is None else np.asarray(w, dtype=np.float64)


def objective(net: Network, z, vm, va, w=None):
    """J = r^T W r (Eq. 2)."""
    r = z - net.h(vm, va)
    return float(np.sum(weights(net, w) * r * r))


def normal_equations(net: Network, z, vm, va, w=None):
    """G = H^T W H and rhs = H^T W r at (vm, va) (Eq. 3)."""
    W = weights(net, w)
    H = net.jacobian(vm, va)
    r = z - net.h(vm, va)
    HW = sp.diags(W) @ H
    G = (H.T @ HW).tocsc()
    rhs = H.T @ (W * r)
    return G, rhs


def gn_step(net: Network, z, vm, va, w=None):
    """One centralized GN step: returns dx (length n = 2N - 1)."""
    G, rhs = normal_equations(net, z, vm, va, w)
    return splu(G).solve(rhs)


def flat_start(net: Network):
    return np.ones(net.n_bus), np.zeros(net.n_bus)


def gauss_newton(net: Network, z, w=None, vm0=None, va0=None, tol=1e-6, max_iter=10,
                 history=False):
    """Centralized WLS Gauss-Newton from (vm0, va0) or flat start.

    Returns dict(vm, va, iters, converged, J, max_dx=[...], states=[...]).
    """
    if vm0 is None:
        vm, va = flat_start(net)
    else:
        vm, va = np.array(vm0, dtype=np.float64), np.array(va0, dtype=np.float64)
    x = net.pack(vm, va)
    steps = []
    states = []
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        vm, va = net.unpack(x)
        dx = gn_step(net, z, vm, va, w)
        x = x + dx
        m = float(np.max(np.abs(dx)))
        steps.append(m)
        if history:
            states.append(net.unpack(x))
        if m < tol:
            converged = True
            break
    vm, va = net.unpack(x)
    out = {"vm": vm, "va": va, "iters": it, "converged": converged,
           "J": objective(net, z, vm, va, w), "max_dx": steps}
    if history:
        out["states"] = states
    return out
