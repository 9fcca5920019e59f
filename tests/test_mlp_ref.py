"""Pins of the FP64 learned-estimator reference (oracle/mlp_ref.py):
bfloat16 rounding and GELU against torch's CPU routines and closed forms,
backpropagation against finite differences, Adam's first step in closed form."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as M

torch = pytest.importorskip("torch")


def test_bf16_round_known_values_and_torch():
    one = 1.0
    assert M.bf16_round(np.float32(one)) == 1.0
    assert M.bf16_round(np.float32(1 + 2**-8)) == 1.0  # tie -> even mantissa
    assert M.bf16_round(np.float32(1 + 3 * 2**-8)) == 1 + 2**-6  # tie -> even (up)
    assert M.bf16_round(np.float32(1 + 2**-8 + 2**-12)) == 1 + 2**-7  # above the tie
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), ref)


def test_gelu_closed_forms_and_torch():
    assert M.gelu(0.0) == 0.0
    x = np.linspace(-6, 6, 1001)
    np.testing.assert_allclose(M.gelu(x) - M.gelu(-x), x, rtol=0, atol=1e-12)  # erf is odd
    ref = torch.nn.functional.gelu(torch.from_numpy(x), approximate="none").numpy()
    np.testing.assert_allclose(M.gelu(x), ref, rtol=1e-12, atol=1e-14)
    xt = torch.from_numpy(x).requires_grad_(True)
    torch.nn.functional.gelu(xt, approximate="none").sum().backward()
    np.testing.assert_allclose(M.gelu_grad(x), xt.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(1)
    params = M.init_params(3).astype(np.float64)
    feats = rng.uniform(0, 1, (9, M.N_IN))
    targets = rng.uniform(0, 8, 9)
    loss, grad = M.loss_and_grad(params, feats, targets)
    idx = rng.choice(M.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [M.N_PARAMS - 1, 0, M.N_HID * M.N_IN]])  # b3, W1[0,0], b1[0]
    h = 1e-6
    for i in idx:
        p1, p2 = params.copy(), params.copy()
        p1[i] += h
        p2[i] -= h
        fd = (M.loss_and_grad(p1, feats, targets)[0] - M.loss_and_grad(p2, feats, targets)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    newp, m1, m2 = M.adam_step(p, np.zeros(3), np.zeros(3), g, 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(newp, p - 0.01 * np.sign(g), rtol=1e-12)  # bias-corrected: lr * g/|g|


def test_features_layout():
    hist = np.zeros((2, 33))
    hist[0, 0], hist[0, 5] = 200, 56
    hist[1, 3] = 256
    pool = np.arange(33, dtype=np.float64)
    f = M.features(hist, pool, 256, 1 << 18)
    assert f.shape == (2, 67)
    assert f[0, 0] == 200 / 256 and f[1, 3] == 1.0
    assert np.allclose(f[:, 33:66], pool / 2**18)
    assert f[0, 66] == pytest.approx(math.log(256 / 2**18))


def test_inference_close_to_unrounded_forward():
    """With bf16-exact weights and inputs, inference differs from the fp64
    forward pass only through the bf16 rounding of the first hidden layer."""
    params = M.bf16_round(M.init_params(5)).astype(np.float32)
    rng = np.random.default_rng(2)
    feats = M.bf16_round(rng.uniform(0, 1, (50, M.N_IN)).astype(np.float32))
    y_inf = M.infer(params, feats)
    y_fwd, _ = M.forward_train(params.astype(np.float64), feats)
    assert np.max(np.abs(y_inf - y_fwd)) < 0.05 * (1 + np.max(np.abs(y_fwd)))
    assert not np.array_equal(y_inf, y_fwd)
