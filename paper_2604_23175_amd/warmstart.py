"""Learned warm start: training-set generation, training loop, checkpoints.

The networks and every computation on them live in the HIP library (bf16
MFMA forward/backward and Adam kernels, include/mase.h); this module only
orchestrates: it draws seeded drift chains (gridgen), lets the library's
plain flat-start Gauss-Newton converge them to build (z, x_hat) pairs,
initialises and normalises the networks, and runs minibatch training.
PyTorch is used for device memory only.
"""
from __future__ import annotations

import numpy as np
import torch

from gridgen import synth

from . import mase

TRAIN_SEED = 10_000
HELDOUT_SEED = 20_000


def measurements_dev(ctx: mase.Mase, vm, va, eps, sigma, device):
    """z = h(x) + sigma * eps on the device for one batch of ctx.n_snap states."""
    vm_t = torch.as_tensor(vm, device=device, dtype=torch.float64).contiguous()
    va_t = torch.as_tensor(va, device=device, dtype=torch.float64).contiguous()
    h = torch.empty((ctx.n_snap, ctx.n_meas), dtype=torch.float64, device=device)
    torch.cuda.synchronize()
    ctx.mase_eval_h_dev(vm_t, va_t, h)
    torch.cuda.synchronize()
    z = h + torch.as_tensor(sigma, device=device) * torch.as_tensor(eps, device=device)
    # the library reads z on its own stream: finish torch's work first
    torch.cuda.synchronize()
    return z


def solved_set(ctx: mase.Mase, grid, sigma, n_chain, chain_len, seed, device, tol=1e-8, max_iter=15):
    """(z, vm_hat, va_hat) for n_chain drift chains of chain_len snapshots.

    Each chain starts from the grid's base state (independent seeds seed+c);
    every snapshot is converged by the plain flat-start Gauss-Newton of the
    library in batches of ctx.n_snap.  Returns device tensors [n, ...].
    """
    vm, va, eps = synth.make_chains(grid, n_chain, chain_len, seed)
    va = va - va[:, [grid.slack]]
    n, S = vm.shape[0], ctx.n_snap
    z_all = torch.empty((n, ctx.n_meas), dtype=torch.float64, device=device)
    vm_all = torch.empty((n, ctx.n_bus), dtype=torch.float64, device=device)
    va_all = torch.empty_like(vm_all)
    out_vm = torch.empty((S, ctx.n_bus), dtype=torch.float64, device=device)
    out_va = torch.empty_like(out_vm)
    n_bad = 0
    for b0 in range(0, n, S):
        idx = np.arange(b0, b0 + S) % n  # the last batch wraps around
        z = measurements_dev(ctx, vm[idx], va[idx], eps[idx], sigma, device)
        ctx.mase_set_measurements_dev(z)
        ctx.mase_set_state_dev(None, None)
        iters, conv = ctx.mase_solve(tol, max_iter)
        n_bad += int((~conv).sum())
        ctx.mase_state_dev(out_vm, out_va)
        torch.cuda.synchronize()
        keep = min(S, n - b0)
        z_all[b0:b0 + keep] = z[:keep]
        vm_all[b0:b0 + keep] = out_vm[:keep]
        va_all[b0:b0 + keep] = out_va[:keep]
    torch.cuda.synchronize()
    return z_all, vm_all, va_all, n_bad


def init_params(mlp: mase.Mlp, seed=0, in_rms=None):
    """He-normal weights (first layer divided by the area's input RMS, since
    measurements normalised by sigma spread far beyond unit scale), zero
    biases, a small output layer; in the library's parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (m, H, O) in enumerate(mlp.shapes):
        r = 1.0 if in_rms is None else max(in_rms[k], 1e-3)
        parts += [rng.normal(0, np.sqrt(2.0 / m) / r, m * H), np.zeros(H),
                  rng.normal(0, np.sqrt(2.0 / H), H * H), np.zeros(H),
                  rng.normal(0, 0.1 * np.sqrt(1.0 / H), H * O), np.zeros(O)]
    p = np.concatenate(parts).astype(np.float32)
    mlp.mase_mlp_set_params(p)
    return p


def set_normalisation(mlp: mase.Mlp, z, vm, va):
    """Normalisation from the training set, computed by the library on the
    device: z mean per measurement, per-variable mean / std of the targets.
    Returns ((z_mean, y_mean, y_std), in_rms): the statistics (host copies,
    for checkpoints) and the per-area RMS of the normalised inputs."""
    torch.cuda.synchronize()
    in_rms = mlp.mase_mlp_fit_norm(z, vm, va)
    return mlp.mase_mlp_get_norm(), [float(r) for r in in_rms]


def train(mlp: mase.Mlp, z, vm, va, epochs=30, batch=256, lr=1e-3, lr_final=1e-5, seed=0, log=None):
    """Minibatch Adam over shuffled (z, x_hat) pairs with a cosine lr decay."""
    n = z.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    steps = epochs * (n // batch)
    step = 0
    history = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(z.device)
        zs, vms, vas = z[perm].contiguous(), vm[perm].contiguous(), va[perm].contiguous()
        torch.cuda.synchronize()
        losses = []
        for b0 in range(0, n - batch + 1, batch):
            t = step / max(1, steps - 1)
            cur = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * t))
            want = (b0 == 0)
            l = mlp.mase_mlp_train_step(zs[b0:], vms[b0:], vas[b0:], batch, cur, want_loss=want)
            if want:
                losses.append(l)
            step += 1
        history.append(float(np.mean(losses)) if losses else float("nan"))
        if log:
            log(f"epoch {ep}: loss {history[-1]:.4g}")
    torch.cuda.synchronize()
    return history


def calibrate_accept_cap(ctx: mase.Mase, mlp: mase.Mlp, grid, sigma, device, n_chain=2,
                         seed=HELDOUT_SEED, tol=1e-6, max_iter=10):
    """Acceptance cap on J(pred) from held-out drift chains.

    Gauss-Newton converges from a prediction only as fast as its error allows
    at the scale of single branches; a prediction can beat flat start on J and
    still cost iterations.  For every held-out snapshot this measures the
    iterations from flat start and from the prediction (forced) and J(pred);
    sorted by J(pred), the cap is the J that ends the prefix with the largest
    total saving.  With no saving anywhere the cap is -inf (flat start
    everywhere).  Sets the cap on mlp and returns (cap, summary).
    """
    S = ctx.n_snap
    vm, va, eps = synth.make_chains(grid, n_chain, S, seed)
    va = va - va[:, [grid.slack]]
    pv = torch.empty((S, ctx.n_bus), dtype=torch.float64, device=device)
    pa = torch.empty_like(pv)
    mlp.mase_mlp_set_accept_cap(float("inf"))
    jp_all, it_flat, it_pred, conv_pred = [], [], [], []
    for b0 in range(0, vm.shape[0], S):
        idx = np.arange(b0, b0 + S)
        z = measurements_dev(ctx, vm[idx], va[idx], eps[idx], sigma, device)
        ctx.mase_set_measurements_dev(z)
        mase.mase_warm_start(ctx, mlp)
        jp, _ = mlp.mase_warm_start_objectives()
        ctx.mase_set_state_dev(None, None)
        itf, _ = ctx.mase_solve(tol, max_iter)
        mlp.mase_mlp_predict_dev(z, S, pv, pa)
        torch.cuda.synchronize()
        ctx.mase_set_state_dev(pv, pa)
        itp, cp = ctx.mase_solve(tol, max_iter)
        jp_all.append(jp)
        it_flat.append(itf)
        it_pred.append(np.where(cp, itp, max_iter + 1))
        conv_pred.append(cp)
    jp, itf, itp = np.concatenate(jp_all), np.concatenate(it_flat), np.concatenate(it_pred)
    order = np.argsort(jp, kind="stable")
    gain = np.cumsum((itf - itp)[order].astype(np.float64))
    best = int(np.argmax(gain)) if gain.size else -1
    cap = float(jp[order][best]) if best >= 0 and gain[best] > 0 else float("-inf")
    mlp.mase_mlp_set_accept_cap(cap)
    summary = {"snapshots": int(jp.size), "seed": seed, "mean_iters_flat": float(itf.mean()),
               "mean_iters_forced_prediction": float(itp.mean()),
               "forced_prediction_converged": int(np.concatenate(conv_pred).sum()),
               "j_cap": cap, "accepted_under_cap": int((jp <= cap).sum()),
               "iterations_saved": float(gain[best]) if best >= 0 and gain[best] > 0 else 0.0}
    return cap, summary


def save(path, mlp: mase.Mlp, norm):
    z_mean, y_mean, y_std = norm
    np.savez(path, params=mlp.mase_mlp_get_params(), z_mean=z_mean, y_mean=y_mean, y_std=y_std,
             hidden=mlp.hidden)


def load_into(path, mlp: mase.Mlp):
    d = np.load(path)
    mlp.mase_mlp_set_params(d["params"])
    mlp.mase_mlp_set_norm(d["z_mean"], d["y_mean"], d["y_std"])
    return d["z_mean"], d["y_mean"], d["y_std"]
