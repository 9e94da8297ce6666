"""GPU tests of the learned warm start (C ABI through the binding).

* loss and gradients of the per-area MLP (bf16 MFMA kernels, FP32
  accumulation) match oracle.mlp on the same bf16 recipe;
* one Adam step matches oracle.mlp.adam_step applied to the GPU's gradient;
* training lowers the loss;
* the warm start keeps a prediction exactly when J(pred) <= J(flat), accepted
  starts reach the same minimiser as flat start, rejected snapshots solve
  exactly as from flat start, and a corrupted network is rejected.
"""
import numpy as np
import pytest
import torch

from gpu_common import Case, say
from oracle import mlp as omlp
from paper_2604_23175_amd import mase
from paper_2604_23175_amd import warmstart as ws

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _oracle_inputs(c, M, z, vm, va, z_mean, y_mean, y_std):
    Xs, Ts = [], []
    for k in range(c.g.n_area):
        im = M.in_meas[k]
        Xs.append((z[:, im] - z_mean[im]) / c.s[im])
        ov = M.out_var[k]
        x = np.where(ov % 2 == 0, va[:, ov // 2], vm[:, ov // 2])
        Ts.append((x - y_mean[ov]) / y_std[ov])
    return Xs, Ts


def _setup(hidden, B, seed=0):
    c = Case("c0", 4, seed=seed)
    ctx = c.ctx()
    M = mase.Mlp(ctx, hidden=hidden, max_batch=8)
    rng = np.random.default_rng(seed)
    params = []
    for m, H, O in M.shapes:
        params.append({"W1": rng.normal(0, 1 / np.sqrt(m), (m, H)), "b1": rng.normal(0, 0.1, H),
                       "W2": rng.normal(0, 1 / np.sqrt(H), (H, H)), "b2": rng.normal(0, 0.1, H),
                       "W3": rng.normal(0, 1 / np.sqrt(H), (H, O)), "b3": rng.normal(0, 0.1, O)})
    flat = omlp.flatten(params).astype(np.float32)
    M.mase_mlp_set_params(flat)
    n_bus = c.g.n_bus
    z_mean = c.z.mean(0)
    y_mean = rng.normal(0, 0.1, 2 * n_bus)
    y_std = rng.uniform(0.05, 0.2, 2 * n_bus)
    M.mase_mlp_set_norm(z_mean, y_mean, y_std)
    z = c.z[rng.integers(0, 4, B)] + rng.normal(0, 0.01, (B, c.net.m))
    vm = rng.uniform(0.95, 1.05, (B, n_bus))
    va = rng.normal(-0.2, 0.1, (B, n_bus))
    return c, ctx, M, flat, (z, vm, va), (z_mean, y_mean, y_std)


@pytest.mark.parametrize("hidden,B", [(32, 5), (256, 8)])
def test_loss_and_gradients_match_oracle(hidden, B):
    say("mlp gradients", hidden, B)
    c, ctx, M, flat, (z, vm, va), (zm, ym, ys) = _setup(hidden, B)
    t = lambda a: torch.tensor(a, device=DEV, dtype=torch.float64)
    loss, g = M.mase_mlp_loss_grad(t(z), t(vm), t(va), B)
    Xs, Ts = _oracle_inputs(c, M, z, vm, va, zm, ym, ys)
    params = omlp.unflatten(flat.astype(np.float64), M.shapes)
    lo, go = omlp.loss_and_grads(params, Xs, Ts, recipe=True)
    assert abs(loss - lo) <= 1e-5 * lo, (loss, lo)
    gg = omlp.unflatten(g.astype(np.float64), M.shapes)
    for k in range(len(M.shapes)):
        for key in omlp.PARAM_ORDER:
            a, b = gg[k][key], go[k][key]
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            assert rel <= 2e-3, (k, key, rel)
    ctx.close()


def test_adam_step_matches_oracle():
    say("adam")
    c, ctx, M, flat, (z, vm, va), _ = _setup(32, 6, seed=1)
    t = lambda a: torch.tensor(a, device=DEV, dtype=torch.float64)
    _, g = M.mase_mlp_loss_grad(t(z), t(vm), t(va), 6)
    M.mase_mlp_train_step(t(z), t(vm), t(va), 6, 1e-3)
    new = M.mase_mlp_get_params()
    ref, _, _ = omlp.adam_step(flat.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, 1e-3)
    np.testing.assert_allclose(new, ref, rtol=1e-6, atol=1e-7)
    ctx.close()


def test_training_lowers_loss():
    say("training")
    c, ctx, M, flat, (z, vm, va), _ = _setup(64, 8, seed=2)
    t = lambda a: torch.tensor(a, device=DEV, dtype=torch.float64)
    zt, vt, at = t(z), t(vm), t(va)
    first = M.mase_mlp_train_step(zt, vt, at, 8, 3e-3, want_loss=True)
    for _ in range(60):
        M.mase_mlp_train_step(zt, vt, at, 8, 3e-3)
    last, _ = M.mase_mlp_loss_grad(zt, vt, at, 8, want_grad=False)
    assert last < 0.2 * first, (first, last)
    ctx.close()


def test_warm_start_acceptance_rule_and_fallback():
    """The objective test decides per snapshot; accepted starts reach the same
    minimiser; a corrupted network is rejected and the solve equals flat
    start.  The iteration counts with and without the network are printed
    (the gain it shows on this workload is recorded in the benchmark)."""
    say("warm start")
    from gridgen import synth
    g = synth.make_config("c1")
    t_, a_, s_ = synth.measurement_set(g.n_bus, g.n_branch)
    S = 32
    ctx = mase.Mase.from_grid(g, t_, a_, s_, S)
    z, vm, va, bad = ws.solved_set(ctx, g, s_, 48, 32, ws.TRAIN_SEED, DEV)
    assert bad == 0
    M = mase.Mlp(ctx, hidden=256, max_batch=256)
    norm = ws.set_normalisation(M, z, vm, va)
    ws.init_params(M, 0, ws.input_rms(M, z, norm[0], s_))
    hist = ws.train(M, z, vm, va, epochs=25, batch=256, lr=1e-3)
    assert np.isfinite(hist).all() and hist[-1] < hist[0], hist
    # held-out snapshots
    hv, ha, he = synth.make_chains(g, 1, S, ws.HELDOUT_SEED)
    ha = ha - ha[:, [g.slack]]
    zh = ws.measurements_dev(ctx, hv, ha, he, s_, DEV)
    ctx.mase_set_measurements_dev(zh)
    ctx.mase_set_state()
    J_flat = ctx.mase_objective()
    it_flat, conv_f = ctx.mase_solve(1e-6, 10)
    ctx.mase_set_state()
    ctx.mase_solve(1e-10, 15)
    x_flat = ctx.mase_state()
    pv = torch.empty((S, g.n_bus), dtype=torch.float64, device=DEV)
    pa = torch.empty_like(pv)
    M.mase_mlp_predict_dev(zh, S, pv, pa)
    torch.cuda.synchronize()
    ctx.mase_set_state(pv.cpu().numpy(), pa.cpu().numpy())
    J_pred = ctx.mase_objective()
    acc = mase.mase_warm_start(ctx, M)
    np.testing.assert_array_equal(acc, J_pred <= J_flat)
    # the objectives the decision used, and the acceptance cap on J(pred)
    jp, jf = M.mase_warm_start_objectives()
    np.testing.assert_allclose(jp, J_pred, rtol=1e-12)
    np.testing.assert_allclose(jf, J_flat, rtol=1e-12)
    cap = float(np.median(jp))
    M.mase_mlp_set_accept_cap(cap)
    np.testing.assert_array_equal(mase.mase_warm_start(ctx, M), (jp <= jf) & (jp <= cap))
    M.mase_mlp_set_accept_cap(float("-inf"))
    assert not mase.mase_warm_start(ctx, M).any()
    # a negative cap short-circuits: flat start, nothing evaluated
    assert np.isnan(M.mase_warm_start_objectives()[0]).all()
    it_neg, _ = ctx.mase_solve(1e-6, 10)
    np.testing.assert_array_equal(it_neg, it_flat)
    with pytest.raises(mase.MaseError):
        M.mase_mlp_set_accept_cap(float("nan"))
    M.mase_mlp_set_accept_cap(float("inf"))
    acc = mase.mase_warm_start(ctx, M)
    it_warm, conv_w = ctx.mase_solve(1e-6, 10)
    assert conv_f.all() and conv_w.all()
    say("  accepted", int(acc.sum()), "of", S, "| mean GN iterations flat", it_flat.mean(),
        "warm", it_warm.mean(), "| rejected snapshots identical:",
        bool(np.array_equal(it_warm[~acc], it_flat[~acc])))
    np.testing.assert_array_equal(it_warm[~acc], it_flat[~acc])
    mase.mase_warm_start(ctx, M)
    ctx.mase_solve(1e-10, 15)
    x_warm = ctx.mase_state()
    np.testing.assert_allclose(x_warm[0], x_flat[0], rtol=0, atol=1e-8)
    np.testing.assert_allclose(x_warm[1], x_flat[1], rtol=0, atol=1e-8)
    # a corrupted network: its prediction is far off and must be rejected
    p = M.mase_mlp_get_params()
    p[:] = 0.0
    o = 0
    for m, H, O in M.shapes:
        o += m * H + H + H * H + H + H * O
        p[o:o + O] = 40.0  # 40 standard deviations off in every output
        o += O
    M.mase_mlp_set_params(p)
    acc = mase.mase_warm_start(ctx, M)
    assert not acc.any()
    it_rej, _ = ctx.mase_solve(1e-6, 10)
    np.testing.assert_array_equal(it_rej, it_flat)
    M.close()
    ctx.close()
