"""Write tests/golden/cfg3_sample_oracle.npz: the oracle's facets and fits for
32 sources of the 10,000-source, 8-channel field, chosen across the range of
source sizes (and so of facet cell counts: the largest facet-size bucket
included), on the inputs the mixed form is given.

The field: the generator's observation, catalogue and noise for config 3;
the noise rounded to complex64 and the weights to float32, then widened back
exactly.  Each sampled source's facet is extracted from the noise alone with
its own true-shape model restored (Sec. 2.3), so that the facet is the
source plus noise without the other 9,999 sources' sky model, and fitted
over the full e-grid with flux and scale marginalised (Sec. 2.4).  The GPU
test builds the same facets by handing its pass the residual against the
true-shape sky (the library's own model of the data it simulated).

Sources: catalogue indices at 32 evenly spaced ranks of the scale length,
smallest and largest included.  Only the oracle and the seeded generator are
called; the sources are spread over the host's cores.

Stored per sampled source (index order of `src`): theta, n_cells,
cells_sha256 (SHA-256 of int32 ix, iy, count in facet order), wsum_total,
wz_re, wz_im; the estimate e1, e2, s1, s2, c12, lmax, argmax, n_above,
flags; and the full surface [32 x 6561] (ln L, -inf outside |e| < 1).

    python tests/golden/make_cfg3_sample_oracle.py [--workers N]
"""
import argparse
import hashlib
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2203_14071_amd import synth  # noqa: E402

N_SAMPLE = 32
_STATE = {}


def sample_sources(cat, n=N_SAMPLE):
    order = np.argsort(cat.alpha_arcsec, kind="stable")
    ranks = np.unique(np.round(np.linspace(0, cat.n_src - 1, n)).astype(np.int64))
    return [int(order[r]) for r in ranks]


def _source(s):
    o, cat, nz, weight = _STATE["o"], _STATE["cat"], _STATE["nz"], _STATE["weight"]
    p = oracle.Params()
    theta = oracle.facet_theta(cat.alpha_arcsec[s], p.K)
    src = (cat.l[s], cat.m[s], cat.flux_jy[s], cat.alpha_arcsec[s], cat.e1[s], cat.e2[s])
    f = oracle.extract_facet(o.u_m, o.v_m, o.w_m, o.freq_hz, weight, nz, src, theta, p.ref_freq_hz, p.beta)
    surf, est = oracle.fit_source(f, cat.flux_jy[s], p)
    h = hashlib.sha256()
    for arr in (f.ix, f.iy, f.count):
        h.update(np.ascontiguousarray(arr, dtype=np.int32).tobytes())
    wz = np.sum(f.wsum * f.vbar) if f.n_cells else 0j
    return dict(s=s, theta=theta, n_cells=f.n_cells, sha=np.frombuffer(h.digest(), dtype=np.uint8),
                wsum_total=float(np.sum(f.wsum)), wz=complex(wz), est=est, surface=surf)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("--out", default=os.path.join(HERE, "cfg3_sample_oracle.npz"))
    args = ap.parse_args()
    t0 = time.time()
    cfg = synth.CONFIGS[3]
    o = synth.observation(3)
    cat = synth.catalogue(cfg, synth.rng(3, synth.STREAM_CAT))
    nz = synth.noise(cfg, synth.rng(3, synth.STREAM_NOISE), o.n_rows * o.n_chan)
    nz = nz.astype(np.complex64).astype(np.complex128)
    weight = o.weight.astype(np.float32).astype(np.float64)
    src = sample_sources(cat)
    _STATE.update(o=o, cat=cat, nz=nz, weight=weight)
    print(f"[golden] config 3: {o.n_rows} rows x {o.n_chan} channels, {len(src)} sampled sources "
          f"on {args.workers} workers", flush=True)
    recs = {}
    with mp.get_context("fork").Pool(args.workers) as pool:
        for j, rec in enumerate(pool.imap_unordered(_source, src)):
            recs[rec["s"]] = rec
            print(f"[golden] {j + 1}/{len(src)} sources after {time.time() - t0:.0f} s", flush=True)
    recs = [recs[s] for s in src]
    est = [r["est"] for r in recs]
    out = dict(
        config=np.int64(3), n_rows=np.int64(o.n_rows), n_chan=np.int64(o.n_chan), src=np.array(src, np.int64),
        theta=np.array([r["theta"] for r in recs]), n_cells=np.array([r["n_cells"] for r in recs], np.int64),
        cells_sha256=np.stack([r["sha"] for r in recs]),
        wsum_total=np.array([r["wsum_total"] for r in recs]),
        wz_re=np.array([r["wz"].real for r in recs]), wz_im=np.array([r["wz"].imag for r in recs]),
        e1=np.array([e.e1 for e in est]), e2=np.array([e.e2 for e in est]),
        s1=np.array([e.s1 for e in est]), s2=np.array([e.s2 for e in est]),
        c12=np.array([e.c12 for e in est]), lmax=np.array([e.lmax for e in est]),
        argmax=np.array([e.argmax for e in est], np.int64), n_above=np.array([e.n_above for e in est], np.int64),
        flags=np.array([e.flags for e in est], np.int64),
        surface=np.stack([r["surface"] for r in recs]),
    )
    np.savez_compressed(args.out, **out)
    print(f"[golden] wrote {args.out} ({os.path.getsize(args.out) / 1e6:.1f} MB) after {time.time() - t0:.0f} s",
          flush=True)


if __name__ == "__main__":
    main()
