"""The grid-narrowing network's HIP kernels (BF16 MFMA GEMMs, epilogues,
loss, back-propagation, Adam, features, windows) against the FP64 network
oracle with BF16 rounding at the same places.

Tolerances: both sides multiply the same BF16 operands; the kernels
accumulate in FP32 (relative error ~ sqrt(K) 2^-24 per sum, K <= 8192) and
round activations / gradients to BF16 from FP32 values that differ from the
oracle's FP64 values in the last FP32 bits, which moves a small fraction of
roundings by one BF16 step (2^-8 relative).  Outputs and gradient blocks are
therefore compared in relative L2 norm (1e-3), and the fraction of elements
off by more than a few BF16 steps is bounded."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import mlp as M
from paper_2203_14071_amd import rlf, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _init(seed):
    rng = np.random.default_rng(seed)
    p = {}
    for k, s in M.SHAPES:
        if len(s) == 2:
            p[k] = rng.standard_normal(s) * math.sqrt(2.0 / s[0])
        else:
            p[k] = rng.standard_normal(s) * 0.05
        p[k] = p[k].astype(np.float32).astype(np.float64)
    return p


def _bf16_tensor(x):
    torch = G.torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16).to("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.fixture(scope="module")
def ctx():
    return rlf.Context(0)


def test_forward_matches_oracle(ctx):
    torch = G.torch_cuda()
    p = _init(7)
    rng = np.random.default_rng(8)
    n = 300                                    # ragged against 128-row tiles
    x = M.bf16(rng.standard_normal((n, M.N_IN)) * 0.2)
    net = rlf.Mlp(ctx, max_batch=128)          # forward runs in chunks of 128 rows
    net.set_state(M.pack(p))
    y = torch.empty((n, 6), dtype=torch.float32, device="cuda:0")
    net.forward(_bf16_tensor(x), y)
    ctx.sync()
    ref, _ = M.forward(x, p)
    got = y.cpu().numpy().astype(np.float64)
    assert _rel(got, ref) < 1e-3, _rel(got, ref)
    assert np.median(np.abs(got - ref)) < 1e-4 * np.median(np.abs(ref)) + 1e-6
    net.free()


@pytest.mark.parametrize("n", [200, 37])
def test_train_step_gradients_and_adam_match_oracle(ctx, n):
    """n = 200: the NT products for every weight gradient; n = 37 (not a
    multiple of 8): the strided products, and a last 5-row slice in the
    output layer's gradient sums."""
    torch = G.torch_cuda()
    p = _init(9)
    rng = np.random.default_rng(10)
    x = M.bf16(rng.standard_normal((n, M.N_IN)) * 0.2)
    t = rng.standard_normal((n, 3)) * 0.3
    net = rlf.Mlp(ctx, max_batch=256)
    net.set_state(M.pack(p))
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    tt = torch.from_numpy(t.astype(np.float32)).to("cuda:0")
    lr = 1e-3
    net.train_step(_bf16_tensor(x), tt, lr, loss)
    ctx.sync()
    st = net.get_state()
    y, cache = M.forward(x, p)
    t32 = t.astype(np.float32).astype(np.float64)
    assert loss.item() == pytest.approx(M.loss(y, t32), rel=1e-4)
    g = M.backward(p, cache, t32)
    gg = M.unpack(st["grad"])
    for k, _ in M.SHAPES:
        assert _rel(gg[k], g[k]) < 2e-3, (k, _rel(gg[k], g[k]))
    # Adam's first step moves every weight by lr * g / |g| (= +-lr up to eps)
    zero = {k: np.zeros_like(v) for k, v in p.items()}
    pn, mn, vn = M.adam(p, g, zero, zero, 1, lr)
    new = M.unpack(st["params"])
    for k, _ in M.SHAPES:
        d = np.abs(new[k] - pn[k])
        assert np.mean(d > 1e-6) < 1e-2, k           # only tiny-gradient entries may differ in sign
    assert st["step"] == 1
    net.free()


def test_windows_match_oracle(ctx):
    torch = G.torch_cuda()
    rng = np.random.default_rng(11)
    y = np.zeros((500, 6))
    y[:, :2] = rng.uniform(-0.85, 0.85, (500, 2))
    y[:, 3:5] = np.log(rng.uniform(0.005, 0.2, (500, 2)) ** 2)
    y = y.astype(np.float32).astype(np.float64)
    yd = torch.from_numpy(y.astype(np.float32)).to("cuda:0")
    w = torch.empty((500, 4), dtype=torch.int32, device="cuda:0")
    net = rlf.Mlp(ctx, max_batch=8)
    net.windows(yd, w, nsigma=3.0, min_half=3)
    ctx.sync()
    assert np.array_equal(w.cpu().numpy(), M.windows(y, 3.0, 81, 0.02, 3))
    net.windows(yd, w, nsigma=2.5, min_half=2, full_frac=0.1)
    ctx.sync()
    ref = M.windows(y, 2.5, 81, 0.02, 2, full_frac=0.1)
    assert np.array_equal(w.cpu().numpy(), ref)
    assert 0 < np.count_nonzero(ref[:, 1] - ref[:, 0] == 80) < 500
    net.free()


@pytest.mark.parametrize("freq", [None, (0.95e9, 1.05e9, 1.15e9)])
def test_features_match_oracle_facets(ctx, freq):
    """One channel at the reference frequency (g = 1) and three channels
    below it (g = mean spectral factor > 1)."""
    import dataclasses
    torch = G.torch_cuda()
    cfg = synth.CONFIGS[0]
    if freq is not None:
        cfg = dataclasses.replace(cfg, freq_hz=freq)
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, synth.rng(0, synth.STREAM_CAT))
    nz = synth.noise(cfg, synth.rng(0, synth.STREAM_NOISE), o.n_rows * o.n_chan)
    obs = G.make_obs(o, nz)
    f = ctx.facets_create(obs, cat)
    ctx.extract_facets(obs, cat, obs.vis, f)
    x = torch.empty((cat.n_src, M.N_IN), dtype=torch.bfloat16, device="cuda:0")
    net = rlf.Mlp(ctx, max_batch=8)
    net.features(f, x)
    ctx.sync()
    got = x.to(torch.float32).cpu().numpy().astype(np.float64)
    g = M.spectral_norm(o.freq_hz)
    assert (g == 1.0) == (freq is None)
    for s in range(cat.n_src):
        fac = G.oracle_facet(o, nz, cat, s)
        ref = M.bf16(M.features(fac.ix, fac.iy, fac.vbar, cat.flux_jy[s] * g))
        assert np.mean(got[s] != ref) < 1e-3, s      # BF16 ties of values equal to ~1e-12 may round apart
        assert np.max(np.abs(got[s] - ref)) <= 2 ** -7 * np.max(np.abs(ref))
    net.free()
    f.free()


def test_predict_and_train_on_facet_objects(ctx):
    """rlf_mlp_predict equals features + forward bit for bit, across chunks
    of max_batch with a ragged last chunk (10 sources, max_batch 4), and
    rlf_mlp_train_facets equals train_step on the same features (parameters,
    Adam state and loss bit for bit); a facet object larger than max_batch
    is refused for training."""
    from paper_2203_14071_amd import surrogate
    torch = G.torch_cuda()
    cfg = synth.CONFIGS[0]
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, synth.rng(0, synth.STREAM_CAT))
    nz = synth.noise(cfg, synth.rng(0, synth.STREAM_NOISE), o.n_rows * o.n_chan)
    obs = G.make_obs(o, nz)
    f = ctx.facets_create(obs, cat)
    ctx.extract_facets(obs, cat, obs.vis, f)
    n = cat.n_src
    assert n == 10
    init = surrogate.init_params(out_scale=0.1)
    x = torch.empty((n, M.N_IN), dtype=torch.bfloat16, device="cuda:0")
    small = rlf.Mlp(ctx, max_batch=4)
    small.set_state(init)
    small.features(f, x)
    y_ref = torch.empty((n, 6), dtype=torch.float32, device="cuda:0")
    y = torch.full((n, 6), float("nan"), dtype=torch.float32, device="cuda:0")
    small.forward(x, y_ref)
    small.predict(f, y)
    ctx.sync()
    assert torch.equal(y, y_ref)
    rng = np.random.default_rng(4)
    tgt = torch.from_numpy(rng.standard_normal((n, 3)).astype(np.float32) * 0.3).to("cuda:0")
    with pytest.raises(rlf.RlfError):
        small.train_facets(f, tgt, 1e-3, torch.zeros(1, dtype=torch.float64, device="cuda:0"))
    a, b = rlf.Mlp(ctx, max_batch=16), rlf.Mlp(ctx, max_batch=16)
    a.set_state(init)
    b.set_state(init)
    la = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    lb = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    for _ in range(2):
        a.train_step(x, tgt, 1e-3, la)
        b.train_facets(f, tgt, 1e-3, lb)
    ctx.sync()
    sa, sb = a.get_state(), b.get_state()
    for k in ("params", "m", "v"):
        assert np.array_equal(sa[k], sb[k]), k
    assert sa["step"] == sb["step"] == 2
    assert la.item() == lb.item()
    assert not np.array_equal(sa["params"], np.asarray(init, dtype=np.float32))
    for net in (small, a, b):
        net.free()
    f.free()


def test_training_reduces_loss_and_resumes_bit_exactly(ctx):
    torch = G.torch_cuda()
    rng = np.random.default_rng(12)
    n = 1024
    t = rng.standard_normal((n, 3)) * 0.3
    # inputs carrying the targets (a learnable map)
    proj = rng.standard_normal((3, M.N_IN)) * 0.05
    x = M.bf16(t @ proj + 0.01 * rng.standard_normal((n, M.N_IN)))
    xd = _bf16_tensor(x)
    td = torch.from_numpy(t.astype(np.float32)).to("cuda:0")
    p = _init(13)
    net = rlf.Mlp(ctx, max_batch=256)
    net.set_state(M.pack(p))
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    losses = []
    for step in range(60):
        b = (step % 4) * 256
        net.train_step(xd[b:b + 256], td[b:b + 256], 1e-3, loss)
        ctx.sync()
        losses.append(loss.item())
    assert np.mean(losses[-8:]) < np.mean(losses[:8]) - 0.5, (losses[:4], losses[-4:])
    # checkpoint after 60 steps, continue two copies for 5 steps: identical bits
    st = net.get_state()
    net2 = rlf.Mlp(ctx, max_batch=256)
    net2.set_state(st["params"], st["m"], st["v"], st["step"])
    loss2 = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    for step in range(5):
        b = (step % 4) * 256
        net.train_step(xd[b:b + 256], td[b:b + 256], 1e-3, loss)
        net2.train_step(xd[b:b + 256], td[b:b + 256], 1e-3, loss2)
        ctx.sync()
        assert loss.item() == loss2.item(), step          # the loss is summed in a fixed order
    a, c = net.get_state(), net2.get_state()
    assert np.array_equal(a["params"], c["params"]) and np.array_equal(a["m"], c["m"])
    assert a["step"] == c["step"] == 65
    net.free()
    net2.free()


def test_checkpoint_file_resumes_bit_exactly(ctx, tmp_path):
    """rlf_mlp_save / rlf_mlp_load: train, save to a file, train on; a new
    network loaded from the file and trained on the same batches ends with
    identical parameters, moments and step.  Damaged or foreign files are
    refused with RLF_EIO and leave the network's state unchanged."""
    torch = G.torch_cuda()
    rng = np.random.default_rng(21)
    n = 512
    t = rng.standard_normal((n, 3)) * 0.3
    x = M.bf16(t @ (rng.standard_normal((3, M.N_IN)) * 0.05) + 0.01 * rng.standard_normal((n, M.N_IN)))
    xd = _bf16_tensor(x)
    td = torch.from_numpy(t.astype(np.float32)).to("cuda:0")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    net = rlf.Mlp(ctx, max_batch=128)
    net.set_state(M.pack(_init(22)))
    for step in range(12):
        net.train_step(xd[(step % 4) * 128:(step % 4 + 1) * 128], td[(step % 4) * 128:(step % 4 + 1) * 128], 1e-3, loss)
    path = str(tmp_path / "net.ckpt")
    net.save(path)
    saved = net.get_state()
    assert os.path.getsize(path) == 40 + 3 * 4 * net.n_params
    assert not os.path.exists(path + ".tmp")
    for step in range(12, 19):
        net.train_step(xd[(step % 4) * 128:(step % 4 + 1) * 128], td[(step % 4) * 128:(step % 4 + 1) * 128], 1e-3, loss)
    net2 = rlf.Mlp(ctx, max_batch=128)
    net2.load(path)
    st2 = net2.get_state()
    for k in ("params", "m", "v"):
        assert np.array_equal(st2[k], saved[k]), k
    assert st2["step"] == saved["step"] == 12
    for step in range(12, 19):
        net2.train_step(xd[(step % 4) * 128:(step % 4 + 1) * 128], td[(step % 4) * 128:(step % 4 + 1) * 128], 1e-3, loss)
    a, b = net.get_state(), net2.get_state()
    for k in ("params", "m", "v"):
        assert np.array_equal(a[k], b[k]), k
    assert a["step"] == b["step"] == 19
    # damaged files: the loading network keeps its state
    raw = open(path, "rb").read()
    bad = {"truncated": raw[:-4], "flipped": raw[:1000] + bytes([raw[1000] ^ 1]) + raw[1001:],
           "magic": b"XXXXXXXX" + raw[8:], "longer": raw + b"\0", "empty": b""}
    for name, blob in bad.items():
        p = str(tmp_path / f"{name}.ckpt")
        open(p, "wb").write(blob)
        with pytest.raises(rlf.RlfError) as ei:
            net2.load(p)
        assert ei.value.code == rlf.RLF_EIO, name
    with pytest.raises(rlf.RlfError) as ei:
        net2.load(str(tmp_path / "missing.ckpt"))
    assert ei.value.code == rlf.RLF_EIO
    c = net2.get_state()
    assert np.array_equal(c["params"], b["params"]) and c["step"] == 19
    net.free()
    net2.free()


def test_variance_floor_in_the_head(ctx):
    """Log-variance outputs far below the floor: the loss is the oracle's
    floored loss and no gradient reaches the log-variance outputs."""
    torch = G.torch_cuda()
    p = _init(14)
    p["b4"][3:] = -20.0
    rng = np.random.default_rng(15)
    n = 64
    x = M.bf16(rng.standard_normal((n, M.N_IN)) * 0.2)
    t = rng.standard_normal((n, 3)) * 0.01
    net = rlf.Mlp(ctx, max_batch=64)
    net.set_state(M.pack(p))
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    net.train_step(_bf16_tensor(x), torch.from_numpy(t.astype(np.float32)).to("cuda:0"), 1e-4, loss)
    ctx.sync()
    y, cache = M.forward(x, p)
    assert np.all(y[:, 3:] < M.S_MIN - 5)
    t32 = t.astype(np.float32).astype(np.float64)
    assert loss.item() == pytest.approx(M.loss(y, t32), rel=1e-4)
    gg = M.unpack(net.get_state()["grad"])
    assert np.all(gg["b4"][3:] == 0.0) and np.all(gg["W4"][:, 3:] == 0.0)
    assert np.any(gg["b4"][:3] != 0.0)
    net.free()
