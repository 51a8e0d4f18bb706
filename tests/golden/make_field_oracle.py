"""Write tests/golden/field_oracle_cfg{1,2}.npz: the oracle's results for
every source of the 1000-source SKA-MID-like field, the workload the
benchmark times.

The field: the generator's observation, catalogue and noise for config 1
(config 2 draws the same streams); data = noise + the sky model of the true
shapes (Sec. 2.2, Eq. 1-3); one data-parallel pass with the circular initial
sky model (Sec. 2.2, 2.3): residual = data - Sky(e = 0), every source
extracted into its facet with its own circular model restored (Sec. 2.3) and
fitted over the full e-grid with flux and scale marginalised (Sec. 2.4).
Config 2 is the same field on the mixed form's inputs: the data rounded to
complex64 and the weights to float32, then widened back to FP64 exactly, so
the oracle sees what that form is given.

Only the oracle and the seeded generator are called.  The work is spread
over the host's cores: the sky model by blocks of rows (each row is computed
on its own, so the blocks' values are those of one call), the facets and fits
by source.

Stored per source (keys in the file):
  theta, n_cells, cells_sha256 (SHA-256 of the int32 arrays ix, iy, count in
  facet order), wsum_total, wz_re, wz_im (sum_c W_c Vbar_c), wv2 (sum_c W_c
  |Vbar_c|^2);
  the estimate: e1, e2, s1, s2, c12, lmax, argmax, n_above, flags;
  every grid point with ln L >= lmax + ln(0.05) - BAND: pt_offsets [n+1],
  pt_index (flat e-grid index, uint16), pt_value (ln L, f64).  These are all
  the points the estimate reads, plus those within BAND below its threshold;
  for sampled sources (sample_src) the full surface and the facet itself.

    python tests/golden/make_field_oracle.py --config 1 [--workers N]
    python tests/golden/make_field_oracle.py --config 2
"""
import argparse
import hashlib
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2203_14071_amd import synth  # noqa: E402

BAND = 0.05                  # ln L band kept below each source's 5 % threshold
ROW_BLOCK = 1 << 20
_STATE = {}


def sample_sources(cat):
    a = cat.alpha_arcsec
    pick = {int(np.argmin(a)), int(np.argmax(a)), int(np.argsort(a)[len(a) // 2]), 0, cat.n_src - 1,
            137, 321, 500, 777}
    return sorted(pick)


def _sky_block(args):
    r0, r1 = args
    o, cat, catc = _STATE["o"], _STATE["cat"], _STATE["catc"]
    sl = slice(r0, r1)
    true = oracle.sky_model(o.u_m[sl], o.v_m[sl], o.w_m[sl], o.freq_hz, cat)
    circ = oracle.sky_model(o.u_m[sl], o.v_m[sl], o.w_m[sl], o.freq_hz, catc)
    return r0, r1, true, circ


def _source(s):
    o, catc, resid, cat = _STATE["o"], _STATE["catc"], _STATE["resid"], _STATE["cat"]
    p = oracle.Params()
    theta = oracle.facet_theta(catc.alpha_arcsec[s], p.K)
    src = (catc.l[s], catc.m[s], catc.flux_jy[s], catc.alpha_arcsec[s], catc.e1[s], catc.e2[s])
    f = oracle.extract_facet(o.u_m, o.v_m, o.w_m, o.freq_hz, _STATE["weight"], resid, src, theta,
                             p.ref_freq_hz, p.beta)
    surf, est = oracle.fit_source(f, cat.flux_jy[s], p)
    h = hashlib.sha256()
    for arr in (f.ix, f.iy, f.count):
        h.update(np.ascontiguousarray(arr, dtype=np.int32).tobytes())
    wz = np.sum(f.wsum * f.vbar) if f.n_cells else 0j
    if math.isfinite(est.lmax):
        keep = np.flatnonzero(np.isfinite(surf) & (surf >= est.lmax + math.log(p.frac) - BAND))
    else:
        keep = np.zeros(0, dtype=np.int64)
    rec = dict(s=s, theta=theta, n_cells=f.n_cells, sha=np.frombuffer(h.digest(), dtype=np.uint8),
               wsum_total=float(np.sum(f.wsum)), wz=complex(wz), wv2=float(np.sum(f.wsum * np.abs(f.vbar) ** 2)),
               est=est, idx=keep.astype(np.uint16), val=surf[keep])
    if s in _STATE["sample"]:
        rec["surface"] = surf
        rec["facet"] = f
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, choices=(1, 2), default=1)
    ap.add_argument("--workers", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("--sources", type=int, default=0, help="first N sources only (0 = all; for a trial run)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    k = args.config
    cfg = synth.CONFIGS[k]
    t0 = time.time()
    o = synth.observation(k)
    cat = synth.catalogue(cfg, synth.rng(k, synth.STREAM_CAT))
    nz = synth.noise(cfg, synth.rng(k, synth.STREAM_NOISE), o.n_rows * o.n_chan)
    catc = cat.with_shape(np.zeros(cat.n_src), np.zeros(cat.n_src))
    _STATE.update(o=o, cat=cat, catc=catc)
    print(f"[golden] config {k}: {o.n_rows} rows, {cat.n_src} sources; sky model on {args.workers} workers",
          flush=True)
    blocks = [(r, min(r + ROW_BLOCK, o.n_rows)) for r in range(0, o.n_rows, ROW_BLOCK)]
    data = np.empty(o.n_rows, dtype=np.complex128)
    circ = np.empty(o.n_rows, dtype=np.complex128)
    with mp.get_context("fork").Pool(args.workers) as pool:
        for r0, r1, tr, ci in pool.imap_unordered(_sky_block, blocks):
            data[r0:r1] = nz[r0:r1] + tr
            circ[r0:r1] = ci
    weight = o.weight
    if k == 2:       # the mixed form's inputs, widened back exactly
        data = data.astype(np.complex64).astype(np.complex128)
        weight = weight.astype(np.float32).astype(np.float64)
    resid = data - circ
    del data, circ, nz
    print(f"[golden] residual ready after {time.time() - t0:.0f} s", flush=True)
    n = cat.n_src if args.sources <= 0 else min(args.sources, cat.n_src)
    sample = [s for s in sample_sources(cat) if s < n]
    _STATE.update(resid=resid, weight=weight, sample=set(sample))
    recs = [None] * n
    with mp.get_context("fork").Pool(args.workers) as pool:
        for j, rec in enumerate(pool.imap_unordered(_source, range(n))):
            recs[rec["s"]] = rec
            if (j + 1) % 50 == 0:
                print(f"[golden] {j + 1}/{n} sources after {time.time() - t0:.0f} s", flush=True)
    est = [r["est"] for r in recs]
    pt_off = np.zeros(n + 1, dtype=np.int64)
    pt_off[1:] = np.cumsum([r["idx"].size for r in recs])
    out = dict(
        config=np.int64(k), seed_config=np.int64(synth.SEED_CONFIG.get(k, k)), n_rows=np.int64(o.n_rows),
        band=np.float64(BAND),
        theta=np.array([r["theta"] for r in recs]), n_cells=np.array([r["n_cells"] for r in recs], np.int64),
        cells_sha256=np.stack([r["sha"] for r in recs]),
        wsum_total=np.array([r["wsum_total"] for r in recs]),
        wz_re=np.array([r["wz"].real for r in recs]), wz_im=np.array([r["wz"].imag for r in recs]),
        wv2=np.array([r["wv2"] for r in recs]),
        e1=np.array([e.e1 for e in est]), e2=np.array([e.e2 for e in est]),
        s1=np.array([e.s1 for e in est]), s2=np.array([e.s2 for e in est]),
        c12=np.array([e.c12 for e in est]), lmax=np.array([e.lmax for e in est]),
        argmax=np.array([e.argmax for e in est], np.int64), n_above=np.array([e.n_above for e in est], np.int64),
        flags=np.array([e.flags for e in est], np.int64),
        pt_offsets=pt_off, pt_index=np.concatenate([r["idx"] for r in recs]),
        pt_value=np.concatenate([r["val"] for r in recs]),
        sample_src=np.array(sample, np.int64),
        sample_surface=np.stack([recs[s]["surface"] for s in sample]) if sample else np.zeros((0, 81 * 81)),
    )
    for j, s in enumerate(sample):
        f = recs[s]["facet"]
        out[f"sample{j}_ix"], out[f"sample{j}_iy"], out[f"sample{j}_count"] = f.ix, f.iy, f.count
        out[f"sample{j}_wsum"], out[f"sample{j}_vbar"] = f.wsum, f.vbar
    path = args.out or os.path.join(HERE, f"field_oracle_cfg{k}.npz")
    np.savez_compressed(path, **out)
    print(f"[golden] wrote {path} ({os.path.getsize(path) / 1e6:.1f} MB) after {time.time() - t0:.0f} s "
          f"on {args.workers} workers", flush=True)


if __name__ == "__main__":
    main()
