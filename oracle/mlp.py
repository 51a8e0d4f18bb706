"""FP64 reference of the grid-narrowing network (oracle; test infrastructure).

Not part of the paper: a small MLP that predicts (e1, e2, ln alpha) and
their log-variances from a facet, used to centre a narrowed ellipticity grid.

  input   x: the facet's cells with -32 <= ix, iy <= 31, Vbar / (S g) (S the
          catalogue flux at the reference frequency, g the mean over the
          observation's channels of the spectral factor (nu_c / nu_ref)^beta of
          Eq. 1), clipped to [-X_CLIP, X_CLIP] (the noise of faint sources
          would otherwise reach hundreds): Re at (iy+32)*64 + ix+32, Im at
          4096 + same, 0 for empty cells  -> 8192 values, rounded to BF16
  layers  z_l = h_{l-1} W_l + b_l,  h_l = GELU(z_l) = z Phi(z)  (l = 1..3, width 512)
          y = h_3 W_4 + b_4  (6 outputs: mu = y[0:3], s = y[3:6] log-variances)
  loss    mean over samples of sum_d (s'_d + (t_d - mu_d)^2 exp(-s'_d)) / 2,
          s' = max(s, S_MIN): the predicted variance is floored at 1e-3 (a
          sample whose prediction sits below the floor passes no gradient to
          its s), which bounds the loss of confident misses

BF16 rounding (round to nearest even, from the FP32 value) is applied where
the kernels round: inputs, weights and activations before each product, and
the back-propagated gradients dY and dZ before each product.  Products and
sums are FP64 here (FP32 accumulation in the kernels).  Biases, the head and
the optimiser are unrounded.  `round_bf16=False` gives the exact FP64
network, used to check the back-propagation by finite differences.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_IN, N_HID, N_OUT, N_TGT = 8192, 512, 6, 3
S_MIN = math.log(1e-3)
X_CLIP = 4.0
SHAPES = [("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("W4", (N_HID, N_OUT)), ("b4", (N_OUT,))]


def n_params():
    return sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    out, o = {}, 0
    for k, s in SHAPES:
        n = int(np.prod(s))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(s)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[k], dtype=np.float64).reshape(-1) for k, _ in SHAPES])


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) via the FP32 value; returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def spectral_norm(freq_hz, ref_freq_hz=1.4e9, beta=-0.7):
    """g: mean over channels of the spectral factor (nu_c / nu_ref)^beta."""
    return float(np.mean((np.asarray(freq_hz, dtype=np.float64) / ref_freq_hz) ** beta))


def features(ix, iy, vbar, norm):
    """Network input of one facet (cells ix, iy, complex Vbar) divided by
    norm = S g and clipped, unrounded."""
    x = np.zeros(N_IN)
    keep = (ix >= -32) & (ix <= 31) & (iy >= -32) & (iy <= 31)
    pos = (iy[keep] + 32) * 64 + (ix[keep] + 32)
    x[pos] = np.clip(vbar.real[keep] / norm, -X_CLIP, X_CLIP)
    x[4096 + pos] = np.clip(vbar.imag[keep] / norm, -X_CLIP, X_CLIP)
    return x


def forward(x, p, round_bf16=True):
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    cache = {"x": r(x)}
    h = cache["x"]
    for l in (1, 2, 3):
        z = h @ r(p[f"W{l}"]) + p[f"b{l}"]
        cache[f"z{l}"] = z
        h = r(gelu(z))
        cache[f"h{l}"] = h
    y = h @ r(p["W4"]) + p["b4"]
    cache["y"] = y
    return y, cache


def loss(y, t):
    mu, s = y[:, :N_TGT], np.maximum(y[:, N_TGT:], S_MIN)
    return float(np.mean(np.sum(0.5 * (s + (t - mu) ** 2 * np.exp(-s)), axis=1)))


def backward(p, cache, t, round_bf16=True):
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    y = cache["y"]
    n = y.shape[0]
    mu, s_raw = y[:, :N_TGT], y[:, N_TGT:]
    s = np.maximum(s_raw, S_MIN)
    d = t - mu
    ds = np.where(s_raw < S_MIN, 0.0, 0.5 * (1.0 - d * d * np.exp(-s)))
    dy = np.concatenate([-d * np.exp(-s), ds], axis=1) / n
    g = {"b4": dy.sum(0)}
    dyr = r(dy)
    g["W4"] = cache["h3"].T @ dyr
    dh = dyr @ r(p["W4"]).T
    for l in (3, 2, 1):
        dz = dh * gelu_grad(cache[f"z{l}"])
        g[f"b{l}"] = dz.sum(0)
        dzr = r(dz)
        hin = cache["x"] if l == 1 else cache[f"h{l - 1}"]
        g[f"W{l}"] = hin.T @ dzr
        if l > 1:
            dh = dzr @ r(p[f"W{l}"]).T
    return g


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (p, m, v)."""
    pn, mn, vn = {}, {}, {}
    for k, _ in SHAPES:
        mn[k] = b1 * m[k] + (1.0 - b1) * g[k]
        vn[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k]
        mh = mn[k] / (1.0 - b1 ** step)
        vh = vn[k] / (1.0 - b2 ** step)
        pn[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return pn, mn, vn


def windows(y, nsigma=3.0, n_e=81, step=0.02, min_half=3, full_frac=1.0):
    """Inclusive e-grid boxes centred on the predicted (e1, e2): +-nsigma
    predicted standard deviations (from the floored log-variance), widened to
    at least +-min_half steps, snapped outward to the grid, clamped to
    [0, n_e-1]; a box holding more than full_frac of the n_e^2 grid points
    becomes the whole grid."""
    c = (n_e - 1) // 2
    out = np.zeros((y.shape[0], 4), dtype=np.int64)
    for i in range(y.shape[0]):
        for d in (0, 1):
            mu = y[i, d]
            sd = math.exp(0.5 * max(y[i, 3 + d], S_MIN))
            lo = math.floor((mu - nsigma * sd) / step + c)
            hi = math.ceil((mu + nsigma * sd) / step + c)
            mid = int(round(mu / step + c))
            lo = min(lo, mid - min_half)
            hi = max(hi, mid + min_half)
            out[i, 2 * d] = min(max(lo, 0), n_e - 1)
            out[i, 2 * d + 1] = min(max(hi, 0), n_e - 1)
        if (out[i, 1] - out[i, 0] + 1) * (out[i, 3] - out[i, 2] + 1) > full_frac * n_e * n_e:
            out[i] = (0, n_e - 1, 0, n_e - 1)
    return out
