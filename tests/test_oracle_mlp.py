"""Pins for oracle.mlp (the warm-start network's FP64 reference).

* the analytic gradient of the exact (unrounded) loss matches central finite
  differences;
* the bfloat16 rounding matches torch's float32 -> bfloat16 conversion and
  hand-picked round-to-nearest-even ties;
* the first Adam step equals its closed form lr * g / (|g| + eps).
"""
import numpy as np
import pytest

from oracle import mlp


def _params(rng, shapes):
    out = []
    for m, H, O in shapes:
        out.append({"W1": rng.normal(0, 1 / np.sqrt(m), (m, H)), "b1": rng.normal(0, 0.1, H),
                    "W2": rng.normal(0, 1 / np.sqrt(H), (H, H)), "b2": rng.normal(0, 0.1, H),
                    "W3": rng.normal(0, 1 / np.sqrt(H), (H, O)), "b3": rng.normal(0, 0.1, O)})
    return out


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    shapes = [(7, 5, 4), (3, 5, 2)]
    params = _params(rng, shapes)
    B = 6
    Xs = [rng.normal(size=(B, m)) for m, _, _ in shapes]
    Ts = [rng.normal(size=(B, O)) for _, _, O in shapes]
    loss, grads = mlp.loss_and_grads(params, Xs, Ts, recipe=False)
    h = 1e-6
    for a in range(len(shapes)):
        for key in mlp.PARAM_ORDER:
            P = params[a][key]
            G = grads[a][key]
            for idx in list(np.ndindex(P.shape))[:12]:
                old = P[idx]
                P[idx] = old + h
                lp, _ = mlp.loss_and_grads(params, Xs, Ts, recipe=False)
                P[idx] = old - h
                lm, _ = mlp.loss_and_grads(params, Xs, Ts, recipe=False)
                P[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - G[idx]) <= 1e-6 * max(1.0, abs(fd)), (a, key, idx, fd, G[idx])


def test_bf16_rounding():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.normal(0, 1e-3, 5000), [0.0, -0.0, 1.0, -2.5]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)
    # ties: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 -> even (1.0);
    # 1 + 3 * 2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6 -> even (1 + 2^-6)
    assert mlp.bf16(1 + 2.0 ** -8) == 1.0
    assert mlp.bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(2)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = mlp.adam_step(th, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    np.testing.assert_allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_flatten_roundtrip():
    rng = np.random.default_rng(3)
    shapes = [(4, 3, 2), (5, 3, 6)]
    params = _params(rng, shapes)
    back = mlp.unflatten(mlp.flatten(params), shapes)
    for p, q in zip(params, back):
        for k in mlp.PARAM_ORDER:
            np.testing.assert_array_equal(p[k], q[k])
