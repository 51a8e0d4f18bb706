"""Pins of the network oracle: BF16 rounding, GELU, the Gaussian NLL and Adam
against PyTorch's independent CPU implementations, back-propagation against
finite differences, and hand-worked features and windows."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp


def _params(seed=0, scale=0.02):
    rng = np.random.default_rng(seed)
    p = {}
    for k, s in mlp.SHAPES:
        fan_in = s[0] if len(s) == 2 else 1
        p[k] = (rng.standard_normal(s) * (scale if len(s) == 1 else 1.0 / math.sqrt(fan_in))).astype(np.float32)
        p[k] = p[k].astype(np.float64)
    return p


def test_parameter_count_matches_library():
    from paper_2203_14071_amd import rlf
    assert mlp.n_params() == 4723206 == int(rlf.lib().rlf_mlp_num_params())
    p = _params()
    assert np.array_equal(mlp.pack(mlp.unpack(mlp.pack(p))), mlp.pack(p))


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 0.0, -0.0]])   # exact ties
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)
    assert mlp.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0          # tie to even (down)
    assert mlp.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6   # tie to even (up)


def test_gelu_and_its_derivative():
    z = np.linspace(-8, 8, 2001)
    ref = torch.nn.functional.gelu(torch.tensor(z), approximate="none").numpy()
    assert np.allclose(mlp.gelu(z), ref, rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, rtol=1e-7, atol=1e-8)


def test_gaussian_nll_matches_torch():
    rng = np.random.default_rng(2)
    y = rng.standard_normal((7, 6))
    t = rng.standard_normal((7, 3))
    ref = torch.nn.GaussianNLLLoss(full=False, eps=0.0, reduction="mean")(
        torch.tensor(y[:, :3]), torch.tensor(t), torch.tensor(np.exp(y[:, 3:]))).item()
    assert mlp.loss(y, t) == pytest.approx(3 * ref, rel=1e-12)      # torch averages over the 3 targets too


def test_backprop_against_finite_differences():
    """Exact FP64 network: analytic gradients of the batch loss equal central
    differences for sampled entries of every parameter array."""
    p = _params(3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, mlp.N_IN)) * 0.3
    t = rng.standard_normal((3, 3)) * 0.3
    y, cache = mlp.forward(x, p, round_bf16=False)
    g = mlp.backward(p, cache, t, round_bf16=False)
    h = 1e-6
    for k, s in mlp.SHAPES:
        for _ in range(4):
            idx = tuple(int(rng.integers(0, d)) for d in s)
            orig = p[k][idx]
            p[k][idx] = orig + h
            lp = mlp.loss(mlp.forward(x, p, round_bf16=False)[0], t)
            p[k][idx] = orig - h
            lm = mlp.loss(mlp.forward(x, p, round_bf16=False)[0], t)
            p[k][idx] = orig
            fd = (lp - lm) / (2 * h)
            assert g[k][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9), (k, idx)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p = {k: rng.standard_normal(s if len(s) == 1 else (3, 2)) for k, s in mlp.SHAPES}
    tp = {k: torch.tensor(v.copy(), requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    for step in range(1, 4):
        g = {k: rng.standard_normal(p[k].shape) for k in p}
        for k in p:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
        p, m, v = mlp.adam(p, g, m, v, step, 1e-2)
        for k in p:
            assert np.allclose(p[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14), (step, k)


def test_features_layout():
    ix = np.array([0, -32, 31, 40, 5])
    iy = np.array([0, -32, 31, 0, -33])
    vb = np.array([2 + 1j, 4 - 2j, 6 + 0j, 8 + 8j, 9 + 9j])
    x = mlp.features(ix, iy, vb, 2.0)
    assert x[32 * 64 + 32] == 1.0 and x[4096 + 32 * 64 + 32] == 0.5
    assert x[0] == 2.0 and x[4096] == -1.0
    assert x[63 * 64 + 63] == 3.0
    assert np.count_nonzero(x) == 5                                   # cells outside the crop are dropped


def test_windows_hand_case():
    y = np.array([[0.1, -0.3, 0.0, math.log(0.05 ** 2), math.log(0.05 ** 2), 0.0],
                  [0.79, 0.0, 0.0, math.log(1e-6), math.log(1e-6), 0.0]])
    w = mlp.windows(y, nsigma=3.0, min_half=3)
    # e1: 0.1 +- 0.15 -> grid (-0.05/0.02 + 40, 0.25/0.02 + 40) = (37.5, 52.5) -> (37, 53);
    # e2: -0.3 +- 0.15 -> (-0.45/0.02 + 40, -0.15/0.02 + 40) = (17.5, 32.5) -> (17, 33)
    assert w[0].tolist() == [37, 53, 17, 33]
    # tiny predicted variance: floored at 1e-3, sd 0.0316, +-0.0949 ->
    # e1 (74.75, 84.74) -> (74, 80 clamped); e2 (35.26, 44.74) -> (35, 45)
    assert w[1].tolist() == [74, 80, 35, 45]


def test_variance_floor_matches_torch_clamp_and_stops_the_gradient():
    rng = np.random.default_rng(6)
    y = rng.standard_normal((9, 6))
    y[:4, 3:] = mlp.S_MIN - rng.uniform(0.5, 5.0, (4, 3))         # predictions below the floor
    t = rng.standard_normal((9, 3)) * 0.1
    ref = torch.nn.GaussianNLLLoss(full=False, eps=1e-3, reduction="mean")(
        torch.tensor(y[:, :3]), torch.tensor(t), torch.tensor(np.exp(y[:, 3:]))).item()
    assert mlp.loss(y, t) == pytest.approx(3 * ref, rel=1e-12)
    # the loss no longer depends on s below the floor; above it, it does
    h = 1e-6
    for i, d in ((0, 3), (2, 5), (6, 4), (8, 3)):
        yp, ym = y.copy(), y.copy()
        yp[i, d] += h
        ym[i, d] -= h
        fd = (mlp.loss(yp, t) - mlp.loss(ym, t)) / (2 * h)
        assert (fd == 0.0) == (i < 4)
    # b4's gradient is the batch mean of dL/dy: rows below the floor add nothing to the s columns
    p = _params(8)
    x = rng.standard_normal((9, mlp.N_IN)) * 0.3
    yy, cache = mlp.forward(x, p, round_bf16=False)
    cache["y"] = y
    g = mlp.backward(p, cache, t, round_bf16=False)
    above = y[4:, 3:]
    expect = np.sum(0.5 * (1.0 - (t[4:] - y[4:, :3]) ** 2 * np.exp(-above)), axis=0) / 9
    assert np.allclose(g["b4"][3:], expect, rtol=1e-12, atol=0)


def test_spectral_norm():
    assert mlp.spectral_norm([1.4e9]) == 1.0
    assert mlp.spectral_norm([0.7e9, 1.4e9]) == pytest.approx((2 ** 0.7 + 1.0) / 2, rel=1e-15)
    assert mlp.spectral_norm([2.8e9], beta=-1.0) == pytest.approx(0.5, rel=1e-15)


def test_features_are_clipped():
    x = mlp.features(np.array([0, 1]), np.array([0, 0]), np.array([100 - 3j, -50 + 2j]), 10.0)
    assert x[32 * 64 + 32] == 4.0 and x[4096 + 32 * 64 + 32] == -0.3
    assert x[32 * 64 + 33] == -4.0 and x[4096 + 32 * 64 + 33] == 0.2


def test_windows_full_grid_above_area_fraction():
    y = np.array([[0.1, -0.3, 0.0, math.log(0.05 ** 2), math.log(0.05 ** 2), 0.0]])
    # the box (37..53) x (17..33) holds 17 * 17 = 289 points = 0.04405 of 81^2
    assert mlp.windows(y, full_frac=0.0441)[0].tolist() == [37, 53, 17, 33]
    assert mlp.windows(y, full_frac=0.0440)[0].tolist() == [0, 80, 0, 80]
    assert mlp.windows(y, full_frac=0.0)[0].tolist() == [0, 80, 0, 80]
