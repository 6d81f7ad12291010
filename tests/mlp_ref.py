"""CPU FP64 reference of the contact-time bracket perceptron (checker only).

Same architecture and head as the library's model (include/stiv.h); the
bf16 rounding of weights, inputs and hidden activations is applied at the
same points as on the matrix cores, everything else is FP64.
"""
import numpy as np

N_IN, N_H, N_OUT = 18, 64, 2


def bf16(a):
    """Round FP32 values to bf16 (nearest even) and return them as float64."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = []
    for shp in ((N_IN, N_H), (N_H,), (N_H, N_H), (N_H,), (N_H, N_OUT), (N_OUT,)):
        k = int(np.prod(shp))
        out.append(p[o:o + k].reshape(shp))
        o += k
    return out


def forward(p, x, round_bf16=True):
    """Raw outputs [n,2] and the activations."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    xr = r(x)
    h1 = r(np.maximum(xr @ r(W1) + b1, 0.0))
    h2 = r(np.maximum(h1 @ r(W2) + b2, 0.0))
    o = h2 @ r(W3) + b3
    return o, (xr, h1, h2)


def head(o):
    mu = 1.0 / (1.0 + np.exp(-o[:, 0]))
    sd = np.logaddexp(0.0, o[:, 1]) + 1e-3
    return mu, sd


def loss(p, x, s, round_bf16=False):
    o, _ = forward(p, x, round_bf16)
    mu, sd = head(o)
    z = (s - mu) / sd
    return float(np.mean(0.5 * z * z + np.log(sd)))


def grad(p, x, s, round_bf16=False):
    """Gradient of the mean loss by reverse mode in FP64 (through the
    bf16-rounded forward when round_bf16, treating rounding as identity)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    o, (xr, h1, h2) = forward(p, x, round_bf16)
    n = x.shape[0]
    mu, sd = head(o)
    z = (s - mu) / sd
    d0 = -z / sd * mu * (1 - mu)
    d1 = (1.0 / sd - z * z / sd) / (1.0 + np.exp(-o[:, 1]))
    dO = np.stack([d0, d1], axis=1) / n
    gW3 = h2.T @ dO
    gb3 = dO.sum(0)
    dh2 = (dO @ r(W3).T) * (h2 > 0)
    gW2 = h1.T @ dh2
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ r(W2).T) * (h1 > 0)
    gW1 = xr.T @ dh1
    gb1 = dh1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
