"""Shared set-up for the GPU parity tests: seeded inputs, oracle references."""
import sys

import numpy as np

from gridgen import synth
from oracle import areas as oa
from oracle import network as nw
from oracle import wls
from paper_2604_23175_amd import mase


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def grid(name):
    if name in synth.CONFIGS:
        return synth.make_config(name)
    if name.startswith("c2k"):
        # the 9241-bus grid re-partitioned into K areas (same buses and branches)
        import dataclasses
        k = int(name[3:])
        g = synth.make_config("c2")
        return dataclasses.replace(g, n_area=k, bus_area=synth.partition(g.pos, g.br_from, g.br_to, k, "plain"))
    if name == "k2":
        return synth.make_grid(30, 41, 2, seed=1)
    if name == "k5":
        return synth.make_grid(80, 120, 5, seed=3)
    if name == "k8":
        return synth.make_grid(400, 600, 8, seed=5)
    raise KeyError(name)


def boundary_slack(g):
    cut = g.bus_area[g.br_from] != g.bus_area[g.br_to]
    return int(np.min(np.concatenate([g.br_from[cut], g.br_to[cut]])))


class Case:
    """A grid, its oracle network/areas, a seeded batch and the measurements."""

    def __init__(self, name, n_snap, seed=0, slack=None, w=None):
        self.name = name
        self.g = grid(name)
        g = self.g
        self.slack = g.slack if slack is None else slack
        self.t, self.a, self.s = synth.measurement_set(g.n_bus, g.n_branch)
        self.net = nw.from_grid(g, self.t, self.a, self.s, slack=self.slack)
        self.A = oa.Areas(self.net, g.bus_area, g.n_area)
        self.batch = synth.make_batch(g, n_snap, seed)
        vt = self.batch.va_true - self.batch.va_true[:, [self.slack]]  # reference angle 0 at the slack
        self.va_true = vt
        self.vm_true = self.batch.vm_true
        self.z = np.stack([nw.measurements(self.net, self.vm_true[i], vt[i], self.batch.eps[i])
                           for i in range(n_snap)])
        self.w = w
        self.n_snap = n_snap

    def ctx(self, **kw):
        m = mase.Mase.from_grid(self.g, self.t, self.a, self.s, self.n_snap, slack=self.slack, **kw)
        m.mase_set_measurements(self.z, self.w)
        m.mase_set_state()
        return m

    def oracle_solve(self, i, tol=1e-6, max_iter=10, history=False):
        return wls.gauss_newton(self.net, self.z[i], w=self.w, tol=tol, max_iter=max_iter, history=history)

    def dx_by_var(self, dx_cols):
        """Oracle step (column order) -> [2 N] by global variable id."""
        out = np.zeros(2 * self.g.n_bus)
        vm_c, va_c = self.net.unpack(dx_cols)
        out[0::2] = va_c
        out[1::2] = vm_c
        return out


def assert_state_close(vm, va, vm_ref, va_ref, rel=1e-8):
    """|x - x_ref| <= rel * max(1, |x_ref|) elementwise (theta rad, |V| p.u.)."""
    for x, r in ((vm, vm_ref), (va, va_ref)):
        err = np.abs(x - r) / np.maximum(1.0, np.abs(r))
        assert float(err.max()) <= rel, float(err.max())
