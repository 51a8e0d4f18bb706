"""Parity of the mixed-precision form (FP64 phase and cell index, FP32
sin/cos, profile and likelihood with block-FP64 sums; complex64 visibilities)
against the FP64 oracle on the same inputs: cells and counts bit-exact,
shapes within |de| <= 1e-4."""
import math

import numpy as np
import pytest

import oracle
from paper_2203_14071_amd import rlf, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

# FP32 arithmetic with hardware sin/cos (absolute error ~1e-6 of the term):
# per source term ~2e-6 S, so the sky model sum is within 2e-6 * sum S.
VIS_MIXED_L1 = 2e-6
VBAR_MIXED = 2e-5
E_MIXED = 1e-4


@pytest.fixture(scope="module")
def ctx():
    return rlf.Context(0, None, rlf.params(precision=rlf.RLF_MIXED))


def _mixed_inputs(o, data):
    """complex64 / f32 inputs, and the exactly upcast copies the oracle uses."""
    d32 = data.astype(np.complex64)
    o.weight = o.weight.astype(np.float32).astype(np.float64)
    return d32, d32.astype(np.complex128)


def _est_ok(h, s, variants, tol):
    for e in variants:
        if abs(h["e1"][s] - e.e1) <= tol and abs(h["e2"][s] - e.e2) <= tol:
            return True
    return False


def _check_sources(o, cat, data64, fac, h, sources, resid_scale):
    catc = G.circular(cat)
    worst_e, worst_l = 0.0, 0.0
    for s in sources:
        ref = G.oracle_facet(o, data64 - oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, catc), catc, s) \
            if resid_scale is None else G.oracle_facet(o, data64, cat, s)
        a, b = fac["offsets"][s], fac["offsets"][s + 1]
        assert b - a == ref.n_cells
        assert np.array_equal(fac["ix"][a:b], ref.ix) and np.array_equal(fac["iy"][a:b], ref.iy)
        assert np.array_equal(fac["count"][a:b], ref.count)
        scale = np.max(np.abs(data64)) if resid_scale is None else resid_scale
        assert np.max(np.abs(fac["vbar"][a:b] - ref.vbar)) <= VBAR_MIXED * (scale + cat.flux_jy[s])
        surf, est = oracle.fit_source(ref, cat.flux_jy[s])
        fin = np.isfinite(surf)
        worst_l = max(worst_l, float(np.max(np.abs(h["surface"][s][fin] - surf[fin]))))
        variants = G.oracle_estimate_variants(surf)
        # near the 5 % threshold FP32 may move points in or out: accept any flip set
        i1, i2, e1, e2, valid = oracle.e_grid(81, 0.02)
        thr = est.lmax + math.log(0.05)
        near = valid & fin & (np.abs(surf - thr) <= 0.05)
        if np.any(near):
            for shift in (+1, -1):
                s2 = surf.copy()
                s2[near] = thr + shift * 0.1
                variants.append(oracle.estimate(s2, e1, e2, valid, 81))
        assert _est_ok(h, s, variants, E_MIXED), (s, h["e1"][s], h["e2"][s], est.e1, est.e2)
        worst_e = max(worst_e, min(max(abs(h["e1"][s] - e.e1), abs(h["e2"][s] - e.e2)) for e in variants))
    return worst_e, worst_l


def test_mixed_model_vis_tiny(ctx):
    torch = G.torch_cuda()
    cfg = synth.CONFIGS[0]
    o = synth.observation(0)
    cat = synth.catalogue(cfg, synth.rng(0, synth.STREAM_CAT))
    nz = synth.noise(cfg, synth.rng(0, synth.STREAM_NOISE), o.n_rows)
    d32, d64 = _mixed_inputs(o, nz)
    obs = G.make_obs(o, d32, mixed=True)
    out = torch.empty_like(obs.vis)
    ctx.model_vis(obs, cat, out, mode=rlf.RLF_MODEL_WRITE)
    ctx.sync()
    ref = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat)
    err = np.max(np.abs(out.cpu().numpy().astype(np.complex128) - ref))
    assert err <= VIS_MIXED_L1 * np.sum(cat.flux_jy), err


def test_mixed_full_path_tiny(ctx):
    cfg = synth.CONFIGS[0]
    o = synth.observation(0)
    cat = synth.catalogue(cfg, synth.rng(0, synth.STREAM_CAT))
    nz = synth.noise(cfg, synth.rng(0, synth.STREAM_NOISE), o.n_rows)
    data = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat) + nz
    d32, d64 = _mixed_inputs(o, data)
    obs = G.make_obs(o, d32, mixed=True)
    catc = G.circular(cat)
    f = ctx.facets_create(obs, catc)
    ctx.extract_facets(obs, catc, None, f)
    out = G.fit_out_tensors(cat.n_src)
    ctx.fit_sources(f, out, want_surface=True)
    ctx.sync()
    fac, h = f.copy(), G.host(out)
    worst_e, worst_l = _check_sources(o, cat, d64, fac, h, range(cat.n_src), None)
    print(f"mixed tiny: max |de| {worst_e:.2e}, max |dl| {worst_l:.2e}")
    f.free()


def test_mixed_full_size_sampled(ctx):
    """Config 2 (the SKA-MID-like field in the mixed form): residual = noise,
    true shapes, sampled sources through the FP64 oracle."""
    cfg = synth.CONFIGS[2]
    o = synth.observation(2)
    cat = synth.catalogue(cfg, synth.rng(2, synth.STREAM_CAT))
    nz = synth.noise(cfg, synth.rng(2, synth.STREAM_NOISE), o.n_rows)
    d32, d64 = _mixed_inputs(o, nz)
    obs = G.make_obs(o, d32, mixed=True)
    f = ctx.facets_create(obs, cat)
    ctx.extract_facets(obs, cat, obs.vis, f)
    out = G.fit_out_tensors(cat.n_src)
    ctx.fit_sources(f, out, want_surface=True)
    ctx.sync()
    fac, h = f.copy(), G.host(out)
    cnt = np.add.reduceat(fac["count"], fac["offsets"][:-1])
    assert np.all(cnt == o.n_rows)
    a = cat.alpha_arcsec
    pick = sorted({int(np.argmin(a)), int(np.argmax(a)), int(np.argsort(a)[len(a) // 2]), 321})
    worst_e, worst_l = _check_sources(o, cat, d64, fac, h, pick, float(np.max(np.abs(d64))))
    print(f"mixed full size: max |de| {worst_e:.2e}, max |dl| {worst_l:.2e}")
    f.free()
