"""Parity of the mixed-precision form (FP64 phase and cell index, FP32
sin/cos, profile and likelihood with block-FP64 sums; complex64 visibilities)
against the FP64 oracle on the same inputs: cells and counts bit-exact,
shapes within |de| <= 1e-4."""
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


def _check_sources(o, cat, data64, fac, h, sources, resid_scale):
    """Facets of the given sources cell by cell, and each fit against the
    FP64 oracle on the same (rounded) inputs: ln L within the mixed form's
    error bound delta at every grid point, the 5 % set equal to the oracle's
    up to points within 2 delta of its threshold, shapes within 1e-4 (over
    the same set, and as computed when no point changed sides)."""
    catc = G.circular(cat)
    worst_e, worst_l, flips = 0.0, 0.0, 0
    ll_tol = lambda v, lmax: np.full(np.shape(v), G.mixed_delta(lmax))
    band = lambda lmax: 2 * G.mixed_delta(lmax)
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
        raw, adj, wl, fl = G.check_estimate_matched(h, s, surf, h["surface"][s], ll_tol, band, E_MIXED, est)
        worst_e, worst_l, flips = max(worst_e, raw), max(worst_l, wl), flips + fl
    return worst_e, worst_l, flips


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
    worst_e, worst_l, flips = _check_sources(o, cat, d64, fac, h, range(cat.n_src), None)
    print(f"mixed tiny: max |de| {worst_e:.2e}, max |dl| / delta {worst_l:.3f}, flips {flips}")
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
    worst_e, worst_l, flips = _check_sources(o, cat, d64, fac, h, pick, float(np.max(np.abs(d64))))
    print(f"mixed full size: max |de| {worst_e:.2e}, max |dl| / delta {worst_l:.3f}, flips {flips}")
    f.free()
