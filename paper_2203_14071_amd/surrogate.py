"""Grid-narrowing network workflow: simulate training facets with the method
itself, train the network, and fit with narrowed ellipticity windows.

Everything numeric runs in librlf.so (rlf_extract_facets, rlf_mlp_*,
rlf_fit_sources); this module only arranges the calls and the buffers.

Training facets come from the SKA-MID-like field generator (config 1: its
array, 8 h track, one channel at 1.4 GHz and noise level), each source
isolated (the residual handed to the extraction is pure noise, so every
facet holds its own exact model plus noise: the "single source" case of
Sec. 4.1), a fresh noise realisation per batch of sources.  The source
population is config 1's (50-200 uJy, log-normal sizes) or, with
population="config3", that of the 10,000-source field (10-1000 uJy, sizes
from the size-flux relation), so that the network sees the signal-to-noise
range it is used on.

Every training facet is also fitted on the full grid, and each epoch's
targets are drawn around those fits: (e1, e2) = the full-grid estimate plus
kappa times its spread times a fresh standard normal number, with the drawn
source's ln alpha as the third target.  Under the Gaussian NLL the network's
mean then tends to the method's estimate and its variance to the posterior
spread (times kappa squared) plus its own error, which is what a window
around the estimate must cover: trained on the true shapes instead, its mean
carries the full posterior scatter (no better than the estimate) and its
windows miss.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import rlf, synth

N_IN = 8192


def init_params(seed_stream=synth.STREAM_INIT, out_scale=1e-3):
    """He-normal hidden weights, an output layer scaled by out_scale (so the
    network starts near mu = 0, log-variance 0, where the Gaussian NLL is
    well conditioned), zero biases; drawn from the config-1 init stream."""
    g = synth.rng(1, seed_stream)
    shapes = [(N_IN, 512), (512,), (512, 512), (512,), (512, 512), (512,), (512, 6), (6,)]
    parts = []
    for i, s in enumerate(shapes):
        if len(s) == 2:
            w = g.standard_normal(s) * math.sqrt(2.0 / s[0])
            if i == 6:
                w *= out_scale
            parts.append(w.astype(np.float32).reshape(-1))
        else:
            parts.append(np.zeros(s, np.float32))
    return np.concatenate(parts)


def training_population(population="config1"):
    """The config-1 generator with the source population of `population`."""
    cfg = synth.CONFIGS[1]
    if population == "config1":
        return cfg
    if population == "config3":
        c3 = synth.CONFIGS[3]
        return dataclasses.replace(cfg, flux_min_ujy=c3.flux_min_ujy, flux_max_ujy=c3.flux_max_ujy,
                                   flux_slope=c3.flux_slope, size_law=c3.size_law)
    raise ValueError(population)


@dataclasses.dataclass
class TrainingSet:
    """Device tensors of the simulated training facets: network inputs x
    (BF16 [n x 8192]); the full-grid fit of every facet, e1, e2, s1, s2
    (FP64 [n]); ln alpha of the drawn sources (FP32 [n]); the drawn true
    shapes and ln alpha (FP32 [n x 3], for reference)."""
    x: object
    e1: object
    e2: object
    s1: object
    s2: object
    ln_alpha: object
    truth: object

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def training_set(ctx: rlf.Context, net: rlf.Mlp, n_total=200_000, batch_src=20_000, device="cuda:0",
                 log=None, population="config1") -> TrainingSet:
    """Simulate n_total training facets on the config-1 coverage and fit each
    on the full grid."""
    import torch
    cfg = training_population(population)
    o = synth.observation(1)
    g = synth.rng(1, synth.STREAM_TRAIN)
    mixed = ctx.p.precision == rlf.RLF_MIXED
    cdt = torch.complex64 if mixed else torch.complex128
    wdt = torch.float32 if mixed else torch.float64
    t = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a)).to(device, dtype=dt)
    uvw = (t(o.u_m), t(o.v_m), t(o.w_m))
    wt = t(o.weight, wdt)
    f64 = dict(dtype=torch.float64, device=device)
    ts = TrainingSet(x=torch.empty((n_total, N_IN), dtype=torch.bfloat16, device=device),
                     e1=torch.empty(n_total, **f64), e2=torch.empty(n_total, **f64),
                     s1=torch.empty(n_total, **f64), s2=torch.empty(n_total, **f64),
                     ln_alpha=torch.empty(n_total, dtype=torch.float32, device=device),
                     truth=torch.empty((n_total, 3), dtype=torch.float32, device=device))
    flags = torch.empty(batch_src, dtype=torch.int32, device=device)
    for b0 in range(0, n_total, batch_src):
        nb = min(batch_src, n_total - b0)
        cat = synth.catalogue(cfg, g, nb)
        nz = synth.noise(cfg, g, o.n_rows)
        obs = rlf.Obs(*uvw, o.freq_hz, t(nz, cdt), wt)
        f = ctx.facets_create(obs, cat)
        ctx.extract_facets(obs, cat, obs.vis, f)
        net.features(f, ts.x[b0:b0 + nb])
        ctx.fit_sources(f, {"e1": ts.e1[b0:b0 + nb], "e2": ts.e2[b0:b0 + nb], "s1": ts.s1[b0:b0 + nb],
                            "s2": ts.s2[b0:b0 + nb], "flags": flags[:nb]})
        ts.ln_alpha[b0:b0 + nb] = t(np.log(cat.alpha_arcsec).astype(np.float32))
        ts.truth[b0:b0 + nb] = t(np.stack([cat.e1, cat.e2, np.log(cat.alpha_arcsec)], axis=1).astype(np.float32))
        ctx.sync()
        f.free()
        del obs
        if log:
            log(f"[surrogate] training facets {b0 + nb}/{n_total}")
    return ts


def train(ctx: rlf.Context, net: rlf.Mlp, ts: TrainingSet, epochs=96, batch=512, lr=3e-4, kappa=1.1,
          seed=0x5EED, log=None):
    """Adam over contiguous batches (the sources are drawn i.i.d.), targets
    drawn afresh each epoch around the full-grid fits (stream seed + epoch);
    the learning rate drops to lr/4 for the last quarter of the steps.
    Returns the per-epoch mean losses."""
    import torch
    n = ts.n
    steps = (n + batch - 1) // batch
    loss = torch.zeros(1, dtype=torch.float64, device=ts.x.device)
    acc = torch.zeros(1, dtype=torch.float64, device=ts.x.device)
    tg = torch.empty((n, 3), dtype=torch.float32, device=ts.x.device)
    history = []
    total = epochs * steps
    k = 0
    for ep in range(epochs):
        net.posterior_targets(ts.e1, ts.e2, ts.s1, ts.s2, ts.ln_alpha, tg, kappa, seed + ep)
        acc.zero_()
        for s in range(steps):
            b0 = s * batch
            b1 = min(n, b0 + batch)
            rate = lr if k < 0.75 * total else lr / 4
            net.train_step(ts.x[b0:b1], tg[b0:b1], rate, loss)
            acc += loss
            k += 1
        ctx.sync()
        history.append(acc.item() / steps)
        if log and (ep + 1) % 8 == 0:
            log(f"[surrogate] epoch {ep + 1}/{epochs}: mean loss {history[-1]:.4f}")
    return history


class Windowed:
    """Buffers and calls for the network-narrowed fit of one facet object."""

    def __init__(self, ctx: rlf.Context, net: rlf.Mlp, n_src, device="cuda:0"):
        import torch
        self.ctx, self.net = ctx, net
        self.x = torch.empty((n_src, N_IN), dtype=torch.bfloat16, device=device)
        self.y = torch.empty((n_src, 6), dtype=torch.float32, device=device)
        self.win = torch.empty((n_src, 4), dtype=torch.int32, device=device)

    def fit(self, facets: rlf.Facets, out: dict, nsigma=3.0, min_half=3, check_stride=4, full_frac=0.6):
        """Enqueue features -> network -> windows -> windowed fit with the
        full-grid fallback and its lattice check (no synchronisation).
        Windows above full_frac of the grid are fitted on the whole grid."""
        self.net.features(facets, self.x)
        self.net.forward(self.x, self.y)
        self.net.windows(self.y, self.win, nsigma, min_half, full_frac)
        self.ctx.fit_sources(facets, out, mode=1, window=self.win, fallback=True, check_stride=check_stride)
