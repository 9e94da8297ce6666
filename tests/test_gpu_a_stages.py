"""GPU per-stage parity against the oracle on small grids (through the C ABI).

Stage 1 (G^k, b^k), stage 2 (S_b^k, bhat_b^k), stage 3a (S_Gamma, bhat_Gamma)
and stage 4 (the full step dx) are read back in canonical order and compared
with the oracle's dense construction on the same seeded inputs.  Floating-point
sums run in a different order on the two sides.  G^k, b^k, S_b^k and S_Gamma
are held entry by entry to rounding bounds built from the magnitudes of the
terms that make up each entry (tests/bounds.py); bhat and dx, results of
solves, to a bar relative to their largest entry.
"""
import numpy as np
import pytest

import bounds
from gpu_common import Case, assert_state_close, boundary_slack, say
from oracle import wls

C_ASM = 64     # per-entry constant of the assembly bound (both sides' rounding)
C_CHOL = 64    # per-entry constant of the elimination's backward error

pytestmark = pytest.mark.gpu

RTOL_G = 1e-12    # assembly: sums of products, no cancellation-prone solves
RTOL_S = 1e-10    # condensation: cond(G_ii) ~ 1e5..1e6 amplifies rounding
RTOL_DX = 1e-9    # a step relative to its largest entry


def _close(a, b, rtol, what):
    scale = max(1.0, float(np.max(np.abs(b))))
    err = float(np.max(np.abs(a - b))) / scale if a.size else 0.0
    assert err <= rtol, f"{what}: relative error {err:.3e} > {rtol:.1e}"


def _perturbed_state(c, seed=7):
    rng = np.random.default_rng(seed)
    vm = c.vm_true + rng.normal(0, 0.01, c.vm_true.shape)
    va = c.va_true + rng.normal(0, 0.02, c.va_true.shape)
    va[:, c.slack] = 0.0
    return vm, va


CASES = [("c0", None), ("k2", None), ("k5", None), ("k5", "bnd"), ("c1", None)]


@pytest.mark.parametrize("name,slack", CASES)
@pytest.mark.parametrize("gamma_mode", [0, 1])
def test_stage_parity(name, slack, gamma_mode):
    say("stage parity", name, slack, "gamma_mode", gamma_mode)
    from gpu_common import grid
    sl = boundary_slack(grid(name)) if slack == "bnd" else None
    c = Case(name, 2, seed=3, slack=sl)
    m = c.ctx(gamma_mode=gamma_mode)
    vm, va = _perturbed_state(c)
    m.mase_set_state(vm, va)
    m.mase_stage_assemble()
    worst = {"G": 0.0, "b": 0.0, "S": 0.0, "SG": 0.0}
    mags, sbnd = {}, {}
    for s in range(2):
        for k in range(c.g.n_area):
            G, b = m.mase_read_local_system(s, k)
            Go, bo = c.A.local_system(k, c.z[s], vm[s], va[s])
            MG, Mb = bounds.local_magnitudes(c.A, k, c.z[s], vm[s])
            mags[s, k] = MG
            worst["G"] = max(worst["G"], bounds.check_entries(G, Go, C_ASM * bounds.EPS * MG, f"G^{k}"))
            worst["b"] = max(worst["b"], bounds.check_entries(b, bo, C_ASM * bounds.EPS * Mb, f"b^{k}"))
            _close(G, Go, RTOL_G, f"G^{k}")
    m.mase_stage_condense()
    for s in range(2):
        for k in range(c.g.n_area):
            S, bh = m.mase_read_schur(s, k)
            Go, bo = c.A.local_system(k, c.z[s], vm[s], va[s])
            So, bho = c.A.condense(k, Go, bo)
            ni = c.A.n_internal_vars[k]
            sbnd[s, k] = bounds.schur_bound(Go, mags[s, k], ni, C_ASM, C_CHOL)
            worst["S"] = max(worst["S"], bounds.check_entries(S, So, sbnd[s, k], f"S_b^{k}"))
            _close(bh, bho, RTOL_S, f"bhat_b^{k}")
    m.mase_stage_gamma_assemble()
    for s in range(2):
        SG, bG = m.mase_read_gamma_system(s)
        _, det = c.A.condensed_step(c.z[s], vm[s], va[s], detail=True)
        # the gather adds the areas' blocks: their bounds add the same way
        # (plus the rounding of the sums themselves)
        ng = SG.shape[0]
        BG = np.zeros((ng, ng))
        for k in range(c.g.n_area):
            E = c.A.E[k]
            BG[np.ix_(E, E)] += sbnd[s, k] + 4 * bounds.EPS * np.abs(det["systems"][k][2])
        worst["SG"] = max(worst["SG"], bounds.check_entries(SG, det["S_gamma"], BG, "S_Gamma"))
        _close(bG, det["b_gamma"], RTOL_S, "bhat_Gamma")
    say("  largest error / per-entry bound:", {k: f"{v:.3g}" for k, v in worst.items()})
    m.mase_stage_gamma_solve()
    m.mase_stage_update()
    for s in range(2):
        dx = m.mase_read_step(s)
        ref = c.dx_by_var(wls.gn_step(c.net, c.z[s], vm[s], va[s]))
        _close(dx, ref, RTOL_DX, "dx")
    vm2, va2 = m.mase_state()
    for s in range(2):
        ref = wls.gn_step(c.net, c.z[s], vm[s], va[s])
        x = c.net.pack(vm[s], va[s]) + ref
        rvm, rva = c.net.unpack(x)
        assert_state_close(vm2[s], va2[s], rvm, rva, 1e-9)
    m.close()


@pytest.mark.parametrize("name", ["c0", "k5", "c1"])
def test_iterates_match_oracle(name):
    say("iterates", name)
    c = Case(name, 3, seed=11)
    m = c.ctx()
    refs = [c.oracle_solve(i, history=True) for i in range(3)]
    for it in range(4):
        m.mase_gn_iter()
        vm, va = m.mase_state()
        for i in range(3):
            st = refs[i]["states"]
            if it < len(st):
                assert_state_close(vm[i], va[i], st[it][0], st[it][1], 1e-8)
    m.close()


def test_objective_and_measurement_functions():
    say("objective / eval_h")
    import torch
    c = Case("c1", 2, seed=5)
    m = c.ctx()
    vm, va = _perturbed_state(c)
    m.mase_set_state(vm, va)
    J = m.mase_objective()
    for s in range(2):
        Jo = wls.objective(c.net, c.z[s], vm[s], va[s])
        assert abs(J[s] - Jo) <= 1e-10 * Jo
    dvm = torch.tensor(vm, device="cuda")
    dva = torch.tensor(va, device="cuda")
    h = torch.zeros((2, c.net.m), dtype=torch.float64, device="cuda")
    m.mase_eval_h_dev(dvm, dva, h)
    torch.cuda.synchronize()
    hh = h.cpu().numpy()
    for s in range(2):
        np.testing.assert_allclose(hh[s], c.net.h(vm[s], va[s]), rtol=0, atol=1e-12)
    m.close()
