"""FP64 reference of the learned warm start's network (test infrastructure).

The network maps the 26 features of one observation's local problem --
residual at the start point (2), camera copy minus consensus (9), point copy
minus consensus (3), the scaled duals (9 + 3) -- to a predicted update of
the local solve (12 values): 26 -> 128 -> GELU -> 128 -> GELU -> 12.

Precision points (the same as the GPU kernels; q() is round-to-nearest-even
to bfloat16):
  forward : x = q(pad32((f - mu_in) / sd_in)), W1..W3 = q(weights),
            Z1 = x W1 + b1, H1 = q(gelu(Z1)), Z2 = H1 W2 + b2,
            H2 = q(gelu(Z2)), Y = H2 W3 + b3, delta = Y * sd_out + mu_out;
  backward: for the loss mean((Y - t)^2) over batch x 12 outputs,
            dY = 2 (Y - t) / (B 12); dW3 = H2^T q(dY), db3 = sum dY;
            dZ2 = (q(dY) W3^T) * gelu'(Z2); dW2 = H1^T q(dZ2), db2 = sum dZ2;
            dZ1 = (q(dZ2) W2^T) * gelu'(Z1); dW1 = x^T q(dZ1), db1 = sum dZ1.
GELU is the tanh form (Hendrycks & Gimpel 2016).  Adam (Kingma & Ba 2015)
with bias correction updates FP32 master weights.
"""
from __future__ import annotations

import numpy as np

N_IN, N_IN_PAD, N_HID, N_OUT, N_OUT_PAD = 26, 32, 128, 12, 16
GELU_C = np.sqrt(2.0 / np.pi)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(a)
    if nan.any():
        out[nan] = np.nan
    return out


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    u = GELU_C * (z + 0.044715 * z ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3 * 0.044715 * z * z)


def init_params(seed=0):
    """Weights ~ N(0, 1/fan_in) (zero for padded rows/columns), biases 0."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((N_IN_PAD, N_HID))
    W1[:N_IN] = rng.normal(0, 1 / np.sqrt(N_IN), (N_IN, N_HID))
    W2 = rng.normal(0, 1 / np.sqrt(N_HID), (N_HID, N_HID))
    W3 = np.zeros((N_HID, N_OUT_PAD))
    W3[:, :N_OUT] = rng.normal(0, 1 / np.sqrt(N_HID), (N_HID, N_OUT))
    return dict(W1=W1, b1=np.zeros(N_HID), W2=W2, b2=np.zeros(N_HID), W3=W3, b3=np.zeros(N_OUT_PAD))


def standardize_input(f, mu_in, sd_in):
    x = np.zeros((f.shape[0], N_IN_PAD))
    x[:, :N_IN] = (f - mu_in) / sd_in
    return x


def forward(params, x, quantize=True):
    """x: (B, 32) standardized inputs.  Returns Y (B, 16) and the cache."""
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    xq = q(x)
    W1, W2, W3 = q(params["W1"]), q(params["W2"]), q(params["W3"])
    Z1 = xq @ W1 + params["b1"]
    H1 = q(gelu(Z1))
    Z2 = H1 @ W2 + params["b2"]
    H2 = q(gelu(Z2))
    Y = H2 @ W3 + params["b3"]
    return Y, dict(xq=xq, W1=W1, W2=W2, W3=W3, Z1=Z1, H1=H1, Z2=Z2, H2=H2)


def loss(Y, t):
    """Mean squared error over the batch and the 12 outputs (padding ignored)."""
    d = Y[:, :N_OUT] - t[:, :N_OUT]
    return float(np.mean(d * d))


def backward(params, cache, Y, t, quantize=True):
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    B = Y.shape[0]
    dY = np.zeros_like(Y)
    dY[:, :N_OUT] = 2.0 * (Y[:, :N_OUT] - t[:, :N_OUT]) / (B * N_OUT)
    dYq = q(dY)
    g = {}
    g["W3"] = cache["H2"].T @ dYq
    g["b3"] = dY.sum(0)
    dZ2 = (dYq @ cache["W3"].T) * gelu_grad(cache["Z2"])
    dZ2q = q(dZ2)
    g["W2"] = cache["H1"].T @ dZ2q
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2q @ cache["W2"].T) * gelu_grad(cache["Z1"])
    dZ1q = q(dZ1)
    g["W1"] = cache["xq"].T @ dZ1q
    g["b1"] = dZ1.sum(0)
    g["W1"][N_IN:] = 0.0
    g["W3"][:, N_OUT:] = 0.0
    g["b3"][N_OUT:] = 0.0
    return g


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place (step counts from 1)."""
    for k in params:
        m[k] = beta1 * m[k] + (1 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1 - beta2) * grads[k] * grads[k]
        mh = m[k] / (1 - beta1 ** step)
        vh = v[k] / (1 - beta2 ** step)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)


# flat parameter block of the C ABI: W1 [32][128] b1 [128] W2 [128][128]
# b2 [128] W3 [128][16] b3 [16]
_FLAT = (("W1", (N_IN_PAD, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("W3", (N_HID, N_OUT_PAD)), ("b3", (N_OUT_PAD,)))


def flatten(params):
    return np.concatenate([np.asarray(params[k], np.float64).reshape(-1) for k, _ in _FLAT])


def unflatten(flat):
    out, o = {}, 0
    for k, shp in _FLAT:
        n = int(np.prod(shp))
        out[k] = np.asarray(flat[o:o + n], np.float64).reshape(shp)
        o += n
    return out
