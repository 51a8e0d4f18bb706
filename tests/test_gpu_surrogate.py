"""The learned grid narrowing end to end: simulate training facets with the
method, train the network on the GPU with the library's kernels, then on the
10,000-source config-3 field compare the narrowed fit (windows from the
network, full-grid fallback) with the plain full-grid fit, the reference for its
error: RMS(e_window - e_full) <= 1e-3 while evaluating a fraction of the grid.
A source is refitted on the full grid when a member of its window's 5 % set
sits on an inner window edge, its window holds no valid grid point, or a
point of the stride-4 lattice outside the window reaches that set."""
import numpy as np
import pytest

import oracle
from paper_2203_14071_amd import rlf, surrogate, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def test_narrowed_fit_matches_full_fit_on_config3():
    torch = G.torch_cuda()
    ctx = rlf.Context(0, None, rlf.params(precision=rlf.RLF_MIXED))
    net = rlf.Mlp(ctx, max_batch=512)
    net.set_state(surrogate.init_params())
    x, tg = surrogate.training_set(ctx, net, n_total=200_000, batch_src=20_000, population="config3")
    hist = surrogate.train(ctx, net, x, tg, epochs=24)
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
    w.fit(f, nar, check_stride=4)
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
    # grid points evaluated: window + lattice outside it, plus the full grid on refits
    i1, i2, _, _, valid = oracle.e_grid(81, 0.02)
    lat = valid & ((i1 - 40) % 4 == 0) & ((i2 - 40) % 4 == 0)
    evals = 0
    for k in range(n):
        inside = (i1 >= win[k, 0]) & (i1 <= win[k, 1]) & (i2 >= win[k, 2]) & (i2 <= win[k, 3])
        evals += np.count_nonzero(valid & inside) + np.count_nonzero(lat & ~inside)
    evals += np.count_nonzero(b["flags"] & rlf.RLF_FLAG_FALLBACK) * np.count_nonzero(valid)
    frac = evals / (n * np.count_nonzero(valid))
    print(f"evaluated {frac:.3f} of the full-grid points")
    assert rms <= 1e-3
    # what the network gains: a share of the sources is fitted on a narrowed
    # window that the full grid confirms, and fewer grid points are evaluated.
    # The trained network depends on the last bits of its training facets
    # (a change in the kernels' FP32 rounding gives another network), and
    # config-3 posteriors are broad, so the gain is small and moves with such
    # changes: the bounds leave room for that (current kernels: 8.4 % kept,
    # 0.978 of the points evaluated).
    kept = (area < 81 * 81) & ((b["flags"] & rlf.RLF_FLAG_FALLBACK) == 0)
    print(f"narrowed and kept: {kept.mean():.3f} of the sources")
    assert kept.mean() >= 0.05
    assert frac < 0.99
    f.free()
    net.free()
    ctx.close()
