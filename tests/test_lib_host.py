"""CPU-only checks of the C-ABI library (no GPU calls).

* the shared library loads and exports every function include/mase.h declares;
* host-only contexts build maps and symbolic patterns that are bit-exact
  against the oracle's independent construction (oracle.areas);
* invalid inputs are rejected with MASE_ERR_ARG.
"""
import os
import re

import numpy as np
import pytest

from gridgen import synth
from oracle import areas as oa
from oracle import network as nw
from paper_2604_23175_amd import mase

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = mase.load()
    hdr = open(os.path.join(ROOT, "include", "mase.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(mase_[a-z_]+)\s*\(", hdr))
    assert declared == set(mase.SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name


def _ctx(g, slack=None, gamma_mode=0, n_snap=2):
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    m = mase.Mase.from_grid(g, t, a, s, n_snap, slack=slack, host_only=True, gamma_mode=gamma_mode)
    net = nw.from_grid(g, t, a, s, slack=slack)
    A = oa.Areas(net, g.bus_area, g.n_area)
    return m, net, A


CASES = [
    ("c0", None), ("c1", None),
    ("k2", None), ("k4b", None), ("k5", None), ("slack_bnd", "bnd"),
    # the benchmark grids (9241 buses / 32 areas, 10000 buses / 16 areas)
    ("c2", None), ("c3", None),
]


def _grid(name):
    if name in ("c0", "c1", "c2", "c3"):
        return synth.make_config(name)
    if name == "k2":
        return synth.make_grid(30, 41, 2, seed=1)
    if name == "k4b":
        return synth.make_grid(60, 90, 4, seed=2, mode="balanced")
    if name in ("k5", "slack_bnd"):
        return synth.make_grid(80, 120, 5, seed=3)
    raise KeyError(name)


@pytest.mark.parametrize("name,slack", CASES)
def test_maps_bit_exact(name, slack):
    g = _grid(name)
    if slack == "bnd":
        cut = g.bus_area[g.br_from] != g.bus_area[g.br_to]
        slack = int(np.min(np.concatenate([g.br_from[cut], g.br_to[cut]])))
    m, net, A = _ctx(g, slack)
    np.testing.assert_array_equal(m.mase_export_map("boundary_flag"), A.is_boundary.astype(np.int32))
    np.testing.assert_array_equal(m.mase_export_map("meas_area"), A.meas_area)
    np.testing.assert_array_equal(m.mase_export_map("gamma_vars"), A.gamma_vars)
    assert m.mase_info("n_gamma") == A.gamma_vars.size
    for k in range(g.n_area):
        np.testing.assert_array_equal(m.mase_export_map("local_vars", k), A.local_vars[k])
        assert int(m.mase_export_map("n_internal", k)[0]) == A.n_internal_vars[k]
        np.testing.assert_array_equal(m.mase_export_map("E", k), A.E[k])


@pytest.mark.parametrize("name,slack", CASES[:4] + CASES[6:])
def test_patterns_bit_exact(name, slack):
    g = _grid(name)
    m, net, A = _ctx(g, slack)
    for k in range(g.n_area):
        rp, ci = m.mase_export_pattern(k)
        orp, oci = A.pattern(k)
        np.testing.assert_array_equal(rp, orp)
        np.testing.assert_array_equal(ci, oci)


def test_dense_gamma_mode_plans():
    g = synth.make_config("c1")
    m, _, _ = _ctx(g, gamma_mode=mase.MASE_GAMMA_DENSE)
    assert m.mase_info("gamma_tail") == m.mase_info("n_boundary_bus")
    m2, _, _ = _ctx(g)
    assert 0 < m2.mase_info("gamma_tail") < m2.mase_info("n_boundary_bus")
    assert m2.mase_info("flops_gamma") < m.mase_info("flops_gamma")


def _base():
    g = synth.make_config("c0")
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    return dict(n_bus=g.n_bus, br_from=g.br_from.copy(), br_to=g.br_to.copy(), br_r=g.br_r.copy(),
                br_x=g.br_x.copy(), br_b=g.br_b.copy(), slack_bus=0, n_area=g.n_area,
                bus_area=g.bus_area.copy(), meas_type=t.copy(), meas_at=a.copy(),
                meas_sigma=s.copy(), n_snap=1)


def _create(**kw):
    o = mase.mase_default_options()
    o.host_only = 1
    args = _base()
    args.update(kw)
    return mase.mase_create(opt=o, **args)


@pytest.mark.parametrize("mutate", [
    lambda a: a["br_from"].__setitem__(0, 99),
    lambda a: a["br_to"].__setitem__(0, a["br_from"][0]),
    lambda a: a["meas_sigma"].__setitem__(3, 0.0),
    lambda a: a["meas_sigma"].__setitem__(3, np.nan),
    lambda a: a["meas_at"].__setitem__(-1, 10**6),
    lambda a: a["meas_type"].__setitem__(0, 9),
    lambda a: a["bus_area"].__setitem__(0, 7),
    lambda a: a["br_x"].__setitem__(2, np.inf),
])
def test_invalid_input_rejected(mutate):
    args = _base()
    mutate(args)
    with pytest.raises(mase.MaseError) as e:
        _create(**args)
    assert e.value.code == mase.MASE_ERR_ARG


def test_area_without_internal_bus_rejected():
    args = _base()
    area = args["bus_area"].copy()
    # an area made of one boundary bus
    area[:] = 0
    area[5] = 1
    args["bus_area"] = area
    args["n_area"] = 2
    with pytest.raises(mase.MaseError) as e:
        _create(**args)
    assert "internal" in str(e.value)


def test_disconnected_area_rejected():
    g = synth.make_grid(40, 50, 2, seed=4)
    t, a, s = synth.measurement_set(g.n_bus, g.n_branch)
    area = g.bus_area.copy()
    # move a far, internal bus of area 1 into area 0
    cand = [b for b in range(g.n_bus) if area[b] == 1 and
            not np.any(area[np.concatenate([g.br_to[g.br_from == b], g.br_from[g.br_to == b]])] == 0)]
    area[cand[0]] = 0
    with pytest.raises(mase.MaseError):
        _create(n_bus=g.n_bus, br_from=g.br_from, br_to=g.br_to, br_r=g.br_r, br_x=g.br_x,
                br_b=g.br_b, n_area=2, bus_area=area, meas_type=t, meas_at=a, meas_sigma=s)


def test_host_only_context_refuses_gpu_calls():
    o = mase.mase_default_options()
    o.host_only = 1
    m = mase.Mase.__new__(mase.Mase)
    m.lib = mase.load()
    args = _base()
    m.ctx = mase.mase_create(opt=o, **args)
    m.n_snap, m.n_bus, m.n_meas = 1, args["n_bus"], args["meas_type"].size
    with pytest.raises(mase.MaseError) as e:
        m.mase_gn_iter()
    assert e.value.code == mase.MASE_ERR_NO_DEVICE
    m.close()
