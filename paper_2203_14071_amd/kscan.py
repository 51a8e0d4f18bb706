"""Facet-size tuning experiment (Sec. 4.1): fit a population of single
sources on the SKA-MID-like coverage for several facet-size factors K and
measure the multiplicative and additive biases of the linear model
e_measured - e_true = m e_true + c (per component), and the number of bad
fits.  Each fit is the full grid followed by the adaptive refinement around
the maximum (the paper's sampler; rlf_refine_sources).

Sources (stream +6 of the config-1 generator): the paper's population of
faint star-forming galaxies, 10-200 uJy with pdf ~ S^-1.6, sizes from the
size-flux relation with its scatter, ellipticity components N(0, 0.3)
with |e| < 0.8; each source alone in the field (the residual handed to the
extraction is noise, so each facet holds its own model plus noise); the
noise set so that the faintest reference source (10 uJy at its median size)
has SNR 19, the paper's figure for its realistic noise variance divided by
5.  Everything numeric runs in librlf.so; this
module arranges the calls and fits the bias lines.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import rlf, synth

STREAM_KSCAN = 6


def population(n_src=1000):
    """The scan's catalogue and noise configuration (config-1 generator)."""
    c1, c3 = synth.CONFIGS[1], synth.CONFIGS[3]
    cfg = dataclasses.replace(c1, flux_min_ujy=10.0, flux_max_ujy=200.0, flux_slope=c3.flux_slope,
                              size_law=c3.size_law, noise_sigma_jy=synth.SIGMA_KSCAN)
    cat = synth.catalogue(cfg, synth.rng(1, STREAM_KSCAN), n_src)
    return cfg, cat


def bias_line(e_true, e_meas):
    """Least-squares m, c of e_meas - e_true = m e_true + c, with standard
    errors from the residual scatter."""
    x = np.asarray(e_true, dtype=np.float64)
    d = np.asarray(e_meas, dtype=np.float64) - x
    A = np.stack([x, np.ones_like(x)], axis=1)
    coef, _, _, _ = np.linalg.lstsq(A, d, rcond=None)
    r = d - A @ coef
    dof = max(1, len(x) - 2)
    cov = np.linalg.inv(A.T @ A) * float(r @ r) / dof
    return float(coef[0]), float(coef[1]), float(math.sqrt(cov[0, 0])), float(math.sqrt(cov[1, 1]))


def run(Ks=(20, 30, 38, 50, 60, 70, 80, 100), n_src=1000, precision=rlf.RLF_FP64, device="cuda:0", log=None,
        refine=True, noise=True):
    """One row per K.  noise=False keeps the weights of the noise level but
    hands the extraction a zero residual, so every facet is its source's
    model alone: what remains of the bias then comes from the method (the
    facet model at cell centres, the prior, the thresholded estimator), not
    from the noise realisation."""
    import torch
    cfg, cat = population(n_src)
    o = synth.observation(1)
    t = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a)).to(device, dtype=dt)
    mixed = precision == rlf.RLF_MIXED
    nz = synth.noise(cfg, synth.rng(1, STREAM_KSCAN + 100), o.n_rows)
    if not noise:
        nz = np.zeros_like(nz)
    vis = t(nz, torch.complex64 if mixed else torch.complex128)
    wt = t(np.full(o.n_rows, 1.0 / cfg.noise_sigma_jy ** 2), torch.float32 if mixed else torch.float64)
    obs = rlf.Obs(t(o.u_m), t(o.v_m), t(o.w_m), o.freq_hz, vis, wt)
    rows = []
    for K in Ks:
        ctx = rlf.Context(0, torch.cuda.current_stream().cuda_stream, rlf.params(K=float(K), precision=precision))
        t0 = time.perf_counter()
        f = ctx.facets_create(obs, cat)
        ctx.extract_facets(obs, cat, obs.vis, f)           # true shapes: each facet is its own source + noise
        out = {k: torch.empty(n_src, dtype=torch.float64, device=device) for k in ("e1", "e2", "s1", "s2")}
        out["flags"] = torch.empty(n_src, dtype=torch.int32, device=device)
        out["n_above"] = torch.empty(n_src, dtype=torch.int32, device=device)
        ctx.fit_sources(f, out)
        grid_bad = int(((out["flags"] & rlf.RLF_FLAG_BAD_VAR) != 0).sum().item())
        if refine:                                            # the paper's adaptive sampling around the maximum
            ctx.refine_sources(f, out)
        ctx.sync()
        dt = time.perf_counter() - t0
        h = {k: v.cpu().numpy() for k, v in out.items()}
        cells = np.diff(f.copy()["offsets"])
        f.free()
        ctx.close()
        good = (h["flags"] & (rlf.RLF_FLAG_BAD_VAR | rlf.RLF_FLAG_EMPTY)) == 0
        m1, c1, sm1, sc1 = bias_line(cat.e1[good], h["e1"][good])
        m2, c2, sm2, sc2 = bias_line(cat.e2[good], h["e2"][good])
        row = {"K": K, "m1": round(m1, 5), "m1_err": round(sm1, 5), "m2": round(m2, 5), "m2_err": round(sm2, 5),
               "c1": round(c1, 5), "c2": round(c2, 5), "bad": int(np.sum(~good)), "bad_before_refinement": grid_bad,
               "refined": int(np.sum((h["flags"] & rlf.RLF_FLAG_REFINED) > 0)),
               "mean_cells": round(float(cells.mean()), 1), "s": round(dt, 3)}
        rows.append(row)
        if log:
            log(f"[kscan{'' if noise else ', noiseless'}] K {K}: m1 {m1:+.4f} +- {sm1:.4f}, m2 {m2:+.4f} +- {sm2:.4f}, c1 {c1:+.5f}, "
                f"c2 {c2:+.5f}, bad {row['bad']}, mean cells {row['mean_cells']}")
    return rows
