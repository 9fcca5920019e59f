"""FP64 reference of the learned cardinality estimator -- TEST INFRASTRUCTURE.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It is the plain definition of the learned estimator that sits
beside the HyperLogLog estimate of Alg. 5 (not part of the paper):

features of a host (67):
    hist[r] / g      for r = 0..32  -- the host's register histogram (Alg. 5)
    pool[r] / m      for r = 0..32  -- the pool's register histogram
    ln(g / m)
network:  67 -> 64 -> 64 -> 1, GELU(x) = x/2 (1 + erf(x / sqrt 2)),
          output y estimates ln(1 + n), so n_hat = exp(y) - 1 (clamped at 0).
inference precision: inputs, W1, W2, w3 and the first hidden layer rounded
    to bfloat16 (round to nearest even); biases float32; everything else here
    in float64.
training: float32 master parameters, loss mean((y - ln(1 + n))^2), Adam.

Flat parameter vector (float32, 8577 entries):
    W1 (64 x 67, row-major), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3 (1)
"""
import math

import numpy as np

N_IN, N_HID = 67, 64
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)), ("w3", (N_HID,)),
         ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(params):
    params = np.asarray(params)
    assert params.shape == (N_PARAMS,)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = params[o:o + n].reshape(shape)
        o += n
    return out


def bf16_round(x):
    """float32 -> bfloat16 (round to nearest, ties to even), returned as float64."""
    x = np.asarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    r = np.where(np.isnan(x), np.uint64(0x7FC00000), r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    x = np.asarray(x, dtype=np.float64)
    erf = np.vectorize(math.erf, otypes=[np.float64])
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    x = np.asarray(x, dtype=np.float64)
    erf = np.vectorize(math.erf, otypes=[np.float64])
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def features(host_hist, pool_hist, g, m):
    """(n, 33) host register histograms + (33,) pool histogram -> (n, 67)."""
    host_hist = np.asarray(host_hist, dtype=np.float64).reshape(-1, 33)
    pool = np.asarray(pool_hist, dtype=np.float64).reshape(33)
    n = host_hist.shape[0]
    f = np.empty((n, N_IN), dtype=np.float64)
    f[:, :33] = host_hist / g
    f[:, 33:66] = pool[None, :] / m
    f[:, 66] = math.log(g / m)
    return f


def infer(params, feats):
    """Learned estimate (n,) float64 of ln(1 + n) with the inference roundings."""
    p = unpack(np.asarray(params, dtype=np.float32))
    x = bf16_round(np.asarray(feats, dtype=np.float32))
    W1, W2, w3 = bf16_round(p["W1"]), bf16_round(p["W2"]), bf16_round(p["w3"])
    b1, b2, b3 = (p[k].astype(np.float64) for k in ("b1", "b2", "b3"))
    h1 = bf16_round(gelu(x @ W1.T + b1).astype(np.float32))
    h2 = gelu(h1 @ W2.T + b2)
    return h2 @ w3 + b3[0]


def forward_train(params, feats):
    p = unpack(np.asarray(params, dtype=np.float64))
    x = np.asarray(feats, dtype=np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(z2)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(params, feats, targets):
    """Mean squared error of y against targets and its gradient (FP64 backprop)."""
    y, (x, z1, h1, z2, h2) = forward_train(params, feats)
    t = np.asarray(targets, dtype=np.float64)
    B = len(t)
    r = y - t
    loss = float(np.mean(r * r))
    p = unpack(np.asarray(params, dtype=np.float64))
    dy = 2.0 * r / B
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, p["w3"]) * gelu_grad(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * gelu_grad(z1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    flat = np.concatenate([g[name].reshape(-1) for name, _ in SIZES])
    return loss, flat


def adam_step(params, m1, m2, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step counts from 1."""
    m1 = beta1 * m1 + (1 - beta1) * grad
    m2 = beta2 * m2 + (1 - beta2) * grad * grad
    mh = m1 / (1 - beta1**step)
    vh = m2 / (1 - beta2**step)
    return params - lr * mh / (np.sqrt(vh) + eps), m1, m2


def init_params(seed: int):
    """He-style uniform initialisation, float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SIZES:
        if name.startswith(("W", "w")):
            fan_in = shape[-1] if len(shape) > 1 else N_HID
            lim = math.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, int(np.prod(shape))))
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts).astype(np.float32)
