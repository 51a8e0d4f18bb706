"""The learned grid narrowing end to end: simulate training facets with the
method, train the network on the GPU with the library's kernels, then on the
10,000-source config-3 field compare the narrowed fit (windows from the
network, full-grid fallback) with the plain full-grid fit, the judge of its
error: RMS(e_window - e_full) <= 1e-3 while evaluating a fraction of the grid.
A source is refitted on the full grid when its narrowed maximum, or any
member of its 5 % set, sits on an inner window edge, or its window holds no
valid grid point."""
import numpy as np
import pytest

from paper_2203_14071_amd import rlf, surrogate, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def test_narrowed_fit_matches_full_fit_on_config3():
    torch = G.torch_cuda()
    ctx = rlf.Context(0, None, rlf.params(precision=rlf.RLF_MIXED))
    net = rlf.Mlp(ctx, max_batch=512)
    net.set_state(surrogate.init_params())
    x, tg = surrogate.training_set(ctx, net, n_total=20_000, batch_src=10_000)
    hist = surrogate.train(ctx, net, x, tg, epochs=4)
    print("training losses", [round(h, 3) for h in hist])
    assert hist[-1] < hist[0]
    del x, tg

    cfg = synth.CONFIGS[3]
    o = synth.observation(3)
    cat = synth.catalogue(cfg, synth.rng(3, synth.STREAM_CAT))
    nz = synth.noise(cfg, synth.rng(3, synth.STREAM_NOISE), o.n_rows * o.n_chan)
    obs = G.make_obs(o, nz.astype(np.complex64), mixed=True)
    ctx.model_vis(obs, cat, obs.vis, mode=rlf.RLF_MODEL_ACCUMULATE)
    catc = G.circular(cat)
    f = ctx.facets_create(obs, catc)
    ctx.extract_facets(obs, catc, None, f)
    n = cat.n_src
    full = G.fit_out_tensors(n, surface=False)
    ctx.fit_sources(f, full)
    w = surrogate.Windowed(ctx, net, n)
    nar = G.fit_out_tensors(n, surface=False)
    w.fit(f, nar)
    ctx.sync()
    a, b = G.host(full), G.host(nar)
    win = w.win.cpu().numpy()
    area = (win[:, 1] - win[:, 0] + 1) * (win[:, 3] - win[:, 2] + 1)
    ok = np.isfinite(a["e1"]) & np.isfinite(b["e1"])
    assert np.array_equal(ok, np.isfinite(a["e1"]))
    de = np.concatenate([b["e1"][ok] - a["e1"][ok], b["e2"][ok] - a["e2"][ok]])
    rms = float(np.sqrt(np.mean(de ** 2)))
    fb = float(np.mean((b["flags"] & rlf.RLF_FLAG_FALLBACK) > 0))
    print(f"narrowed fit: RMS(de) {rms:.2e}, max |de| {np.max(np.abs(de)):.2e}, fallback {fb:.3f}, "
          f"mean window {area.mean():.0f} of 6561 grid points")
    assert rms <= 1e-3
    # a lightly trained network (20k facets, 4 epochs): the narrowing must
    # still help some sources; the benchmark reports the fully trained rates
    assert fb < 0.9
    assert area.mean() < 0.6 * 6561
    f.free()
    net.free()
    ctx.close()
