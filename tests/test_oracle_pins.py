"""Pins of the oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a brute-
force computation, a closed form, an invariant, a library routine, or a
special case.  Together they are chosen so that a plausible slip anywhere
in the oracle (a dropped factor, a wrong sign or index, a transposed
operand, a wrong reading of a threshold) fails at least one of them.
"""
import cmath
import json
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.interpolate

import oracle
from oracle.estimate import FLAG_BAD_VAR, FLAG_EDGE, FLAG_EMPTY
from paper_2203_14071_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ARC = oracle.ARCSEC


# ---------------------------------------------------------------- Eq. 1-3 (P1-P3)

@pytest.mark.parametrize("e1,e2", [(0.3, -0.15), (0.0, 0.0), (-0.2, 0.45)])
def test_p1_disk_transform_matches_pixelised_disk(e1, e2):
    """Eq. 1 shape factor, normalisation, orientation (R2) and phase sign
    (R1) against a brute-force DFT of a pixelised sheared exponential disk
    I(x) ~ exp(-|A x| / alpha) normalised to unit flux (Eq. 2)."""
    alpha_as = 1.0
    a = alpha_as * ARC
    A = np.array([[1 - e1, -e2], [-e2, 1 + e1]])
    ext = int(math.ceil(17.0 / (1.0 - math.hypot(e1, e2))))   # the major axis reaches alpha/(1-|e|)
    npx = 2 * ext * 32
    h = 2 * ext * a / npx
    x = (np.arange(npx) - npx / 2 + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="ij")
    I = np.exp(-np.hypot(A[0, 0] * X + A[0, 1] * Y, A[1, 0] * X + A[1, 1] * Y) / a)
    I /= I.sum()
    l0, m0 = 2e-5, -1e-5
    for (u, v) in [(0.05 / a, 0.0), (0.0, 0.05 / a), (0.2 / a, 0.1 / a), (-0.1 / a, 0.25 / a),
                   (0.3 / a, -0.05 / a)]:
        vb = np.sum(I * np.exp(2j * np.pi * (u * (X + l0) + v * (Y + m0))))
        vc = oracle.disk_vis(u, v, 0.0, l0, m0, 1.0, alpha_as, e1, e2)
        assert abs(vb - vc) < 1e-4, (u, v, vb, vc)


def test_p1_orientation_e1_elongates_along_l():
    """e1 > 0 stretches the image along l, so the visibility falls faster along u."""
    k = 0.3 / ARC
    fu = oracle.model.disk_profile(k, 0.0, 1.0, 0.3, 0.0)
    fv = oracle.model.disk_profile(0.0, k, 1.0, 0.3, 0.0)
    assert fu < fv


def test_p2_point_source_and_zero_spacing():
    """alpha -> 0 or k = 0 gives S * spec exactly; a source at the phase
    centre has no w dependence (Eq. 1)."""
    rng = np.random.default_rng(0)
    u, v, w = rng.normal(0, 3e4, (3, 100))
    V = oracle.disk_vis(u, v, w, 0.0, 0.0, 2.5e-4, 1e-12, 0.2, -0.1, spec=0.9)
    assert np.allclose(V, 2.5e-4 * 0.9, rtol=1e-12, atol=0)
    V0 = oracle.disk_vis(0.0, 0.0, 0.0, 0.01, -0.02, 2.5e-4, 1.7, 0.3, 0.4, spec=1.1)
    assert V0 == pytest.approx(2.5e-4 * 1.1, rel=1e-15)
    Va = oracle.disk_vis(u, v, w, 0.0, 0.0, 1.0, 1.3, 0.1, 0.2)
    Vb = oracle.disk_vis(u, v, -3 * w, 0.0, 0.0, 1.0, 1.3, 0.1, 0.2)
    assert np.array_equal(Va, Vb)


def test_p2_spectral_factor_direction():
    """(lambda_ref/lambda)^beta = (nu/nu_ref)^beta: with beta = -0.7 a lower
    frequency is brighter."""
    s = oracle.spectral_factor(np.array([0.7e9, 1.4e9, 2.8e9]), 1.4e9, -0.7)
    assert s[1] == 1.0 and s[0] == pytest.approx(2 ** 0.7) and s[2] == pytest.approx(2 ** -0.7)


def test_p3_rotation_and_conjugation_invariants():
    """Rotating a source by t rotates e by 2t (Eq. 3): V(R_t k; e e^{2it}) = V(k; e).
    V(-k, -w) = conj V(k, w); |V| <= S spec."""
    rng = np.random.default_rng(1)
    u, v, w = rng.normal(0, 4e4, (3, 200))
    e = 0.35 - 0.2j
    for t in (0.3, 1.1, -2.0):
        er = e * cmath.exp(2j * t)
        ur = math.cos(t) * u - math.sin(t) * v
        vr = math.sin(t) * u + math.cos(t) * v
        V1 = oracle.disk_vis(ur, vr, 0.0, 0.0, 0.0, 1.0, 1.2, er.real, er.imag)
        V0 = oracle.disk_vis(u, v, 0.0, 0.0, 0.0, 1.0, 1.2, e.real, e.imag)
        assert np.allclose(V1, V0, rtol=1e-12, atol=1e-15)
    Vp = oracle.disk_vis(u, v, w, 0.003, -0.002, 1.0, 1.2, 0.3, 0.1)
    Vm = oracle.disk_vis(-u, -v, -w, 0.003, -0.002, 1.0, 1.2, 0.3, 0.1)
    assert np.allclose(Vm, np.conj(Vp), rtol=1e-12, atol=1e-15)
    assert np.all(np.abs(Vp) <= 1.0 + 1e-15)


def test_eq4_scale_flux_relation():
    """Eq. 4 at S = 1 uJy and its slope in ln S."""
    assert oracle.alpha_from_flux(1e-6) == pytest.approx(math.exp(-0.93), rel=1e-14)
    r = oracle.alpha_from_flux(np.array([10e-6, 100e-6]))
    assert r[1] / r[0] == pytest.approx(10 ** 0.33, rel=1e-13)


# ---------------------------------------------------------------- sky model (P4)

def _small_field(n_src=4, seed=7):
    cfg = synth.small_config(0, n_ant=8, n_time=12, n_src=n_src)
    obs = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(seed))
    return cfg, obs, cat


def test_p4_sky_model_against_scalar_loop():
    """Sky model = sum over sources of Eq. 1, checked against a per-visibility
    scalar loop written with the math module (no numpy broadcasting)."""
    cfg, obs, cat = _small_field()
    freq = np.array([1.1e9, 1.4e9])
    sky = oracle.sky_model(obs.u_m, obs.v_m, obs.w_m, freq, cat)
    for r in (0, 5, 33, obs.n_rows - 1):
        for c, nu in enumerate(freq):
            sc = nu / 299792458.0
            u, v, w = obs.u_m[r] * sc, obs.v_m[r] * sc, obs.w_m[r] * sc
            acc = 0j
            for s in range(cat.n_src):
                e1, e2 = cat.e1[s], cat.e2[s]
                det = 1 - e1 * e1 - e2 * e2
                ku = ((1 + e1) * u + e2 * v) / det
                kv = (e2 * u + (1 - e1) * v) / det
                a = cat.alpha_arcsec[s] * math.pi / 648000
                f = 1.0 / (1 + 4 * math.pi ** 2 * a * a * (ku * ku + kv * kv)) ** 1.5
                n1 = math.sqrt(1 - cat.l[s] ** 2 - cat.m[s] ** 2) - 1
                ph = u * cat.l[s] + v * cat.m[s] + w * n1
                acc += (nu / 1.4e9) ** -0.7 * cat.flux_jy[s] * f * cmath.exp(2j * math.pi * ph)
            got = sky[r * 2 + c]
            assert abs(got - acc) <= 1e-12 * abs(acc) + 1e-20


# ---------------------------------------------------------------- extraction (P5, P6)

def _grid_bruteforce(u, v, wt, z, theta):
    cells = {}
    for k in range(u.shape[0]):
        if wt[k] <= 0:
            continue
        key = (int(round_half_even(v[k] * theta)), int(round_half_even(u[k] * theta)))
        n, W, Z = cells.get(key, (0, 0.0, 0j))
        cells[key] = (n + 1, W + wt[k], Z + wt[k] * z[k])
    return cells


def round_half_even(x):
    r = math.floor(x + 0.5)
    if r - x == 0.5 and r % 2 == 1:       # exact tie rounded up to an odd integer: go down
        r -= 1
    return r


def test_p5_extraction_identity_bruteforce():
    """(data - Sky + V_s) shifted equals data - sum_{t != s} V_t shifted; the
    facet equals a dictionary-based weighted gridding of that (Sec. 2.3)."""
    cfg, obs, cat = _small_field(n_src=4)
    rng = np.random.default_rng(3)
    freq = obs.freq_hz
    data = oracle.sky_model(obs.u_m, obs.v_m, obs.w_m, freq, cat) + \
        1e-5 * (rng.standard_normal(obs.n_rows) + 1j * rng.standard_normal(obs.n_rows))
    catc = cat.with_shape(np.zeros(cat.n_src), np.zeros(cat.n_src))
    resid = data - oracle.sky_model(obs.u_m, obs.v_m, obs.w_m, freq, catc)
    wt = obs.weight.copy()
    wt[::7] = 0.0                     # flagged visibilities are skipped
    for s in range(cat.n_src):
        others = [t for t in range(cat.n_src) if t != s]
        iso = data - oracle.sky_model(obs.u_m, obs.v_m, obs.w_m, freq, catc, sources=others)
        sc = freq[0] / 299792458.0
        u, v, w = obs.u_m * sc, obs.v_m * sc, obs.w_m * sc
        n1 = math.sqrt(1 - cat.l[s] ** 2 - cat.m[s] ** 2) - 1
        z = iso * np.exp(-2j * np.pi * (u * cat.l[s] + v * cat.m[s] + w * n1))
        theta = oracle.facet_theta(cat.alpha_arcsec[s])
        ref = _grid_bruteforce(u, v, wt, z, theta)
        f = oracle.extract_facet(obs.u_m, obs.v_m, obs.w_m, freq, wt, resid,
                                 (cat.l[s], cat.m[s], cat.flux_jy[s], cat.alpha_arcsec[s], 0.0, 0.0), theta)
        keys = sorted(ref.keys())
        assert [(int(a), int(b)) for a, b in zip(f.iy, f.ix)] == keys
        for k, key in enumerate(keys):
            n, W, Z = ref[key]
            assert f.count[k] == n
            assert f.wsum[k] == pytest.approx(W, rel=1e-14)
            assert abs(f.vbar[k] - Z / W) <= 1e-9 * abs(Z / W) + 1e-16


def test_p5_noiseless_exact_sky_gives_real_model():
    """Noiseless data with the exact sky model: each shifted visibility is
    spec * S * profile, so the facet is real and equals the weighted mean of
    the model in each cell."""
    cfg, obs, cat = _small_field(n_src=3)
    data = oracle.sky_model(obs.u_m, obs.v_m, obs.w_m, obs.freq_hz, cat)
    resid = np.zeros_like(data)
    resid += data - oracle.sky_model(obs.u_m, obs.v_m, obs.w_m, obs.freq_hz, cat)
    for s in range(cat.n_src):
        src = (cat.l[s], cat.m[s], cat.flux_jy[s], cat.alpha_arcsec[s], cat.e1[s], cat.e2[s])
        f = oracle.extract_facet(obs.u_m, obs.v_m, obs.w_m, obs.freq_hz, obs.weight, resid, src,
                                 oracle.facet_theta(cat.alpha_arcsec[s]))
        assert np.max(np.abs(f.vbar.imag)) < 1e-12 * cat.flux_jy[s]
        assert np.all(f.vbar.real > 0) and np.all(f.vbar.real <= cat.flux_jy[s] * (1 + 1e-12))


def test_p5_lone_source_at_phase_centre_is_plain_gridding():
    """l = m = 0 and zero model: the facet is plain weighted gridding of the
    data, checked with numpy's histogram2d on cell edges (k - 1/2, k + 1/2)."""
    cfg, obs, cat = _small_field(n_src=1)
    rng = np.random.default_rng(5)
    data = rng.standard_normal(obs.n_rows) + 1j * rng.standard_normal(obs.n_rows)
    theta = oracle.facet_theta(1.3)
    f = oracle.extract_facet(obs.u_m, obs.v_m, obs.w_m, obs.freq_hz, obs.weight, data,
                             (0.0, 0.0, 0.0, 1.3, 0.0, 0.0), theta)
    sc = obs.freq_hz[0] / 299792458.0
    tu, tv = obs.u_m * sc * theta, obs.v_m * sc * theta
    N = int(np.ceil(max(np.abs(tu).max(), np.abs(tv).max()))) + 1
    edges = np.arange(-N, N + 2) - 0.5
    H, _, _ = np.histogram2d(tv, tu, bins=[edges, edges])
    Hr, _, _ = np.histogram2d(tv, tu, bins=[edges, edges], weights=obs.weight * data.real)
    Hw, _, _ = np.histogram2d(tv, tu, bins=[edges, edges], weights=obs.weight)
    nz = np.argwhere(H > 0)
    assert nz.shape[0] == f.n_cells
    for k, (a, b) in enumerate(nz):        # argwhere is row-major: sorted by (iy, ix)
        assert (f.iy[k], f.ix[k]) == (a - N, b - N)
        assert f.count[k] == H[a, b]
        assert f.vbar.real[k] == pytest.approx(Hr[a, b] / Hw[a, b], rel=1e-10)


def test_p6_gridding_integers_and_symmetries():
    """sum n = #{w > 0}; sum W = sum w; (u,v) -> (-u,-v) maps cells to
    (-ix,-iy); (u,v) -> (-v,u) maps (ix,iy) -> (-iy,ix), counts unchanged."""
    cfg, obs, cat = _small_field(n_src=1)
    rng = np.random.default_rng(11)
    wt = rng.uniform(0.5, 2.0, obs.n_rows)
    wt[rng.random(obs.n_rows) < 0.1] = 0.0
    data = rng.standard_normal(obs.n_rows) + 1j * rng.standard_normal(obs.n_rows)
    theta = oracle.facet_theta(0.9)
    src = (0.0, 0.0, 0.0, 0.9, 0.0, 0.0)
    f = oracle.extract_facet(obs.u_m, obs.v_m, obs.w_m, obs.freq_hz, wt, data, src, theta)
    assert f.count.sum() == np.count_nonzero(wt > 0)
    assert f.wsum.sum() == pytest.approx(wt.sum(), rel=1e-13)
    fm = oracle.extract_facet(-obs.u_m, -obs.v_m, obs.w_m, obs.freq_hz, wt, data, src, theta)
    a = {(x, y): n for x, y, n in zip(f.ix, f.iy, f.count)}
    b = {(-x, -y): n for x, y, n in zip(fm.ix, fm.iy, fm.count)}
    assert a == b
    fr = oracle.extract_facet(-obs.v_m, obs.u_m, obs.w_m, obs.freq_hz, wt, data, src, theta)
    c = {(y, -x): n for x, y, n in zip(fr.ix, fr.iy, fr.count)}   # (ix', iy') = (-iy, ix)
    assert a == c


def test_round_half_even_at_ties():
    """Cell index of an exact half-integer follows round-half-even on both sides."""
    theta = 1.0
    u = np.array([0.5, 1.5, 2.5, -0.5, -1.5])
    f = oracle.extract_facet(u, np.zeros(5), np.zeros(5), np.array([299792458.0]), np.ones(5),
                             np.ones(5, np.complex128), (0, 0, 0, 1.0, 0, 0), theta)
    assert sorted(f.ix.tolist()) == [-2, 0, 2]
    assert [round_half_even(x) for x in u] == [0, 2, 2, 0, -2]


# ---------------------------------------------------------------- likelihood (P7, P8)

def _tiny_facet(rng, n=12, theta=None):
    theta = oracle.facet_theta(1.0) if theta is None else theta
    ix = rng.integers(-6, 7, n)
    iy = rng.integers(-6, 7, n)
    key = np.unique(np.stack([iy, ix], 1), axis=0)
    iy, ix = key[:, 0], key[:, 1]
    n = ix.shape[0]
    W = rng.uniform(1e6, 5e6, n)
    vb = rng.normal(2e-4, 5e-4, n) + 1j * rng.normal(0, 5e-4, n)
    return oracle.Facet(theta, ix, iy, np.ones(n, np.int64), W, vb, ix / theta, iy / theta)


def test_p7_flux_marginalisation_closed_form():
    """ln int exp(-chi2(S)/2) dS (numerical quadrature over S) equals
    D^2/(2Mm) - ln(Mm)/2 plus the omitted shape-free terms."""
    rng = np.random.default_rng(2)
    f = _tiny_facet(rng)
    for (e1, e2, a) in [(0.1, -0.3, 0.8), (0.0, 0.0, 1.5), (-0.5, 0.2, 2.2)]:
        prof = oracle.model.disk_profile(f.uc, f.vc, a, e1, e2)
        chi2 = lambda S: np.sum(f.wsum * np.abs(f.vbar - S * prof) ** 2)
        c0 = chi2(0.0)
        D = np.sum(f.wsum * prof * f.vbar.real)
        Mm = np.sum(f.wsum * prof * prof)
        s0, sd = D / Mm, 1 / math.sqrt(Mm)
        val, _ = scipy.integrate.quad(lambda S: math.exp(-(chi2(S) - c0) / 2 - D * D / (2 * Mm)),
                                      s0 - 12 * sd, s0 + 12 * sd, epsabs=0, epsrel=1e-12, limit=200)
        numeric = math.log(val) - c0 / 2 + D * D / (2 * Mm)
        closed = oracle.loglike_alpha(f, e1, e2, a)[0] + 0.5 * math.log(2 * math.pi) - c0 / 2
        assert numeric == pytest.approx(closed, abs=1e-8)


def test_p7_noiseless_truth_reaches_cauchy_schwarz_bound():
    """At a noiseless facet equal to S f, D^2/Mm = sum W |Vbar|^2."""
    rng = np.random.default_rng(4)
    f = _tiny_facet(rng)
    prof = oracle.model.disk_profile(f.uc, f.vc, 1.2, 0.2, 0.1)
    f.vbar = 3e-4 * prof + 0j
    l = oracle.loglike_alpha(f, 0.2, 0.1, 1.2)[0]
    Mm = np.sum(f.wsum * prof * prof)
    assert l + 0.5 * math.log(Mm) == pytest.approx(0.5 * np.sum(f.wsum * np.abs(f.vbar) ** 2), rel=1e-12)


def test_p8_spline_quadrature_weights():
    """Natural cubic spline quadrature: sum c = RMAX - RMIN; exact on linear
    integrands; equal to scipy's natural CubicSpline integral; all weights
    positive on the paper's knots."""
    x = oracle.alpha_knots(0.3, 3.5, 20)
    assert x[0] == 0.3 and x[-1] == 3.5 and np.all(np.diff(np.diff(x)) > 0)
    c = oracle.spline_quadrature_weights(x)
    assert c.sum() == pytest.approx(3.2, rel=1e-14)
    assert np.sum(c * (2.0 * x - 1.0)) == pytest.approx(3.5 ** 2 - 0.3 ** 2 - 3.2, rel=1e-13)
    assert np.all(c > 0)
    rng = np.random.default_rng(0)
    for _ in range(5):
        y = rng.normal(size=20)
        ref = scipy.interpolate.CubicSpline(x, y, bc_type="natural").integrate(0.3, 3.5)
        assert np.sum(c * y) == pytest.approx(ref, rel=1e-12, abs=1e-13)
    for n in (23, 2, 3):
        xk = oracle.alpha_knots(0.3, 3.5, n)
        assert oracle.spline_quadrature_weights(xk).sum() == pytest.approx(3.2, rel=1e-14)


def test_p8_log_normal_prior_normalised():
    """The scale prior is a normalised log-normal density with median e^mu."""
    val, _ = scipy.integrate.quad(lambda a: math.exp(oracle.log_normal_prior(a, 0.4, 0.3136)), 0, 50,
                                  points=[math.exp(0.4)], limit=200)
    assert val == pytest.approx(1.0, rel=1e-9)
    ref = scipy.stats_lognorm = __import__("scipy.stats", fromlist=["lognorm"]).lognorm(0.3136, scale=math.exp(0.4))
    assert math.exp(oracle.log_normal_prior(1.7, 0.4, 0.3136)) == pytest.approx(ref.pdf(1.7), rel=1e-12)


def test_e_grid_counts():
    """81 x 81 points at 0.02; 6,333 inside |e| < 1; centre and corner values."""
    i1, i2, e1, e2, valid = oracle.e_grid(81, 0.02)
    assert valid.sum() == 6333
    assert np.all(np.hypot(e1[valid], e2[valid]) < 1) and np.all(np.hypot(e1[~valid], e2[~valid]) >= 1 - 1e-12)
    assert e1[0] == pytest.approx(-0.8) and e2[80] == pytest.approx(0.8) and e1[40 * 81 + 40] == 0.0


# ---------------------------------------------------------------- estimator (P9)

def test_p9_estimator_on_isotropic_gaussian():
    """An isotropic Gaussian surface of width sigma >> step centred on a grid
    point: the mean is the centre and each thresholded likelihood-weighted
    standard deviation is sigma sqrt(1 - c e^-c / (1 - e^-c)), c = ln 20,
    i.e. 0.9178 sigma (an unweighted reading would give 1.224 sigma)."""
    i1, i2, e1, e2, valid = oracle.e_grid(81, 0.02)
    sig = 0.1
    c0 = (0.2, -0.1)
    surf = -((e1 - c0[0]) ** 2 + (e2 - c0[1]) ** 2) / (2 * sig ** 2)
    est = oracle.estimate(np.where(valid, surf, -np.inf), e1, e2, valid, 81)
    assert est.e1 == pytest.approx(c0[0], abs=1e-12) and est.e2 == pytest.approx(c0[1], abs=1e-12)
    c = math.log(20)
    expect = sig * math.sqrt(1 - c * math.exp(-c) / (1 - math.exp(-c)))
    assert expect == pytest.approx(0.9178 * sig, rel=1e-4)
    assert est.s1 == pytest.approx(expect, rel=0.01) and est.s2 == pytest.approx(expect, rel=0.01)
    assert abs(est.c12) < 1e-12 and est.flags == 0
    assert est.argmax == (int(round(c0[0] / 0.02)) + 40) * 81 + int(round(c0[1] / 0.02)) + 40


def test_p9_estimator_flags_and_ties():
    i1, i2, e1, e2, valid = oracle.e_grid(81, 0.02)
    # a spike: one sample above threshold -> zero variance -> bad fit
    surf = np.where(valid, -1000.0, -np.inf)
    surf[40 * 81 + 45] = 0.0
    est = oracle.estimate(surf, e1, e2, valid, 81)
    assert est.flags & FLAG_BAD_VAR and est.n_above == 1 and est.s1 == 0.0
    # maximum next to a masked point -> edge
    surf = np.where(valid, -((e1 - 0.8) ** 2 + e2 ** 2) / 0.02, -np.inf)
    assert oracle.estimate(surf, e1, e2, valid, 81).flags & FLAG_EDGE
    # equal maxima: the smallest flat index wins
    surf = np.where(valid, -10.0, -np.inf)
    surf[41 * 81 + 40] = 0.0
    surf[40 * 81 + 41] = 0.0
    assert oracle.estimate(surf, e1, e2, valid, 81).argmax == 40 * 81 + 41
    # nothing valid -> empty
    est = oracle.estimate(np.full(81 * 81, -np.inf), e1, e2, valid, 81)
    assert est.flags == FLAG_EMPTY and math.isnan(est.e1)


# ---------------------------------------------------------------- whole fit (P10, P11)

def _centre_facet(data, u_m, v_m, alpha):
    n = u_m.shape[0]
    return oracle.extract_facet(u_m, v_m, np.zeros(n), np.array([299792458.0]), np.ones(n) * 1e8,
                                data, (0.0, 0.0, 0.0, alpha, 0.0, 0.0), oracle.facet_theta(alpha))


def test_p10_fit_grid_symmetries():
    """Rotating the uv plane by 90 deg maps l(e) to l(-e); u -> -u maps e2 to
    -e2; u <-> v maps e1 to -e1.  Exact lattice symmetries, so surfaces agree
    to rounding and the estimates flip accordingly."""
    rng = np.random.default_rng(9)
    n = 3000
    um = rng.normal(0, 15000, n)
    vm = rng.normal(0, 15000, n)
    alpha = 1.1
    k = 1.0 / (2 * math.pi * alpha * ARC)
    data = 1e-3 * oracle.model.disk_profile(um, vm, alpha, 0.25, -0.15) + \
        1e-4 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    assert np.abs(um).max() > 0.5 * k
    p = oracle.Params(num_r=6)
    i1, i2, e1, e2, valid = oracle.e_grid(p.n_e, p.e_step)
    s0, est0 = oracle.fit_source(_centre_facet(data, um, vm, alpha), 1e-3, p, mu=0.0)
    idx = np.arange(81 * 81)
    I1, I2 = idx // 81, idx % 81
    cases = [((-vm, um), (80 - I1) * 81 + (80 - I2), (-1, -1)),      # 90 deg: e -> -e
             ((-um, vm), I1 * 81 + (80 - I2), (1, -1)),              # u -> -u: e2 -> -e2
             ((vm, um), (80 - I1) * 81 + I2, (-1, 1))]               # u <-> v: e1 -> -e1
    for (uu, vv), perm, (g1, g2) in cases:
        s1, est1 = oracle.fit_source(_centre_facet(data, uu, vv, alpha), 1e-3, p, mu=0.0)
        fin = np.isfinite(s0)
        assert np.array_equal(fin, np.isfinite(s1[perm]))
        assert np.allclose(s1[perm][fin], s0[fin], rtol=1e-11, atol=1e-8)
        assert est1.e1 == pytest.approx(g1 * est0.e1, abs=1e-10)
        assert est1.e2 == pytest.approx(g2 * est0.e2, abs=1e-10)


@pytest.mark.parametrize("ie1,ie2", [(55, 30), (40, 40), (22, 61)])
def test_p11_noiseless_fit_recovers_injected_point(ie1, ie2):
    """uv samples on cell centres, alpha on a knot, noiseless data and high
    weight: the surface peaks at the injected grid point and the estimate
    equals it (Sec. 2.4; reading R10 has no effect when samples sit on
    centres)."""
    p = oracle.Params(num_r=8)
    knots = oracle.alpha_knots(p.rmin, p.rmax, p.num_r)
    alpha = knots[4]
    theta = oracle.facet_theta(alpha)
    g = np.arange(-14, 15)
    IX, IY = np.meshgrid(g, g, indexing="ij")
    u = IX.reshape(-1) / theta
    v = IY.reshape(-1) / theta
    e1, e2 = (ie1 - 40) * 0.02, (ie2 - 40) * 0.02
    data = 2e-4 * oracle.model.disk_profile(u, v, alpha, e1, e2) + 0j
    n = u.shape[0]
    f = oracle.extract_facet(u, v, np.zeros(n), np.array([299792458.0]), np.full(n, 1e14), data,
                             (0.0, 0.0, 0.0, alpha, 0.0, 0.0), theta)
    assert f.n_cells == n
    surf, est = oracle.fit_source(f, 2e-4, p, mu=math.log(alpha))
    assert est.argmax == ie1 * 81 + ie2
    assert est.e1 == pytest.approx(e1, abs=1e-9) and est.e2 == pytest.approx(e2, abs=1e-9)


def test_empty_facet_fit():
    f = oracle.extract_facet(np.ones(3), np.ones(3), np.ones(3), np.array([1.4e9]), np.zeros(3),
                             np.ones(3, np.complex128), (0, 0, 1e-4, 1.0, 0, 0), oracle.facet_theta(1.0))
    surf, est = oracle.fit_source(f, 1e-4)
    assert f.n_cells == 0 and est.flags == FLAG_EMPTY and np.all(np.isneginf(surf))


# ---------------------------------------------------------------- inputs and constants

def test_paper_constants_are_oracle_defaults():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    p = oracle.Params()
    for key, attr in [("beta", "beta"), ("add", "add"), ("esp", "esp"), ("K", "K"), ("rmin_arcsec", "rmin"),
                      ("rmax_arcsec", "rmax"), ("r_std", "r_std"), ("frac_thresh", "frac"),
                      ("bad_sigma", "bad_sigma"), ("bad_sqrtdet", "bad_sqrtdet"), ("ref_freq_hz", "ref_freq_hz")]:
        assert getattr(p, attr) == g[key]["value"], key


def test_workload_matches_paper_uv_count():
    """The SKA-MID-like coverage has the paper's 9,266,880 uv points (Sec. 5)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert synth.CONFIGS[1].n_rows == g["uv_points_ska1_1000"]["value"]
    assert synth.CONFIGS[0].n_rows == 11400 and synth.CONFIGS[3].n_rows * 8 == 74135040


def test_noise_sigma_constants_match_calibration_script():
    import importlib.util
    spec = importlib.util.spec_from_file_location("mk", os.path.join(GOLDEN, "make_noise_sigma.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    stored = json.load(open(os.path.join(GOLDEN, "noise_sigma.json")))
    for k in (0, 1, 3):
        assert synth.CONFIGS[k].noise_sigma_jy == stored[str(k)]
    assert synth.SIGMA_KSCAN == stored["kscan"]
    assert mk.sigma_for(0) == pytest.approx(stored["0"], rel=1e-12)


def test_alpha_marginalisation_against_scipy_logsumexp():
    """l(e) = ln sum_k w_k L(e, alpha_k) computed stably, against scipy's
    logsumexp on the same knot log-likelihoods (values near 1e4, where a
    naive exp would overflow)."""
    from scipy.special import logsumexp
    rng = np.random.default_rng(12)
    f = _tiny_facet(rng)
    f.wsum *= 1e5
    knots = oracle.alpha_knots(0.3, 3.5, 7)
    logw = oracle.log_alpha_weights([1e-4], knots)[0]
    e1 = np.array([0.1, -0.4, 0.0])
    e2 = np.array([0.2, 0.3, 0.0])
    got = oracle.marginal_surface(f, e1, e2, knots, logw)
    L = np.stack([oracle.loglike_alpha(f, e1, e2, a) for a in knots], 0)
    assert np.max(L) > 1e3
    assert np.allclose(got, logsumexp(L + logw[:, None], axis=0), rtol=1e-14, atol=1e-10)


# ---- the narrowed fit's window rule (not in the paper) ----------------------

def _two_bumps(p, big=(20, 20), small=(55, 55), h_small=-1.0, width=3.0):
    """Synthetic ln L surface: two Gaussian bumps on the valid grid, the
    larger (height 0) at `big`, the smaller (height h_small) at `small`."""
    i1, i2, _, _, valid = oracle.e_grid(p.n_e, p.e_step)
    g = lambda c: -((i1 - c[0]) ** 2 + (i2 - c[1]) ** 2) / (2 * width ** 2)
    s = np.logaddexp(g(big), h_small + g(small))
    return np.where(valid, s, -np.inf)


def test_window_rule_hand_cases():
    p = oracle.Params()
    s = _two_bumps(p)
    # a box around the larger bump holding its whole 5 % set: trusted
    assert not oracle.window_rejected(s, (10, 30, 10, 30), 0, p)
    # the same box cut through the set: a member has a neighbour outside
    assert oracle.window_rejected(s, (20, 30, 10, 30), 0, p)
    # a box around the smaller bump: its own set is interior, trusted without
    # the lattice; with stride 4 the lattice point (20, 20) (offset -20 from
    # the centre 40 on both axes) sits at the larger bump and rejects it
    assert not oracle.window_rejected(s, (45, 65, 45, 65), 0, p)
    assert oracle.window_rejected(s, (45, 65, 45, 65), 4, p)
    # stride 3: offsets -21 and -18 on each axis bracket the bump at -20
    # (distance^2 = 1 + 1 = 2 -> ln L = -2/18): still above the threshold
    assert oracle.window_rejected(s, (45, 65, 45, 65), 3, p)
    # a bump far below the window's threshold is not a reason to refit
    s2 = _two_bumps(p, h_small=+4.0)           # the window's bump is now the larger by e^4 > 1/0.05
    assert not oracle.window_rejected(s2, (45, 65, 45, 65), 4, p)
    # a window holding no valid point (a corner beyond |e| = 1)
    assert oracle.window_rejected(s, (0, 3, 0, 3), 0, p)
    # the domain edge is not a window edge: the full grid is never rejected
    assert not oracle.window_rejected(s, (0, 80, 0, 80), 4, p)


def test_window_rule_brute_force_on_tiny_grid():
    """Against a direct reading of the rule, point by point, on a 21x21 grid
    (e_step 0.1) with random surfaces and boxes."""
    p = oracle.Params(n_e=21, e_step=0.1)
    rng = np.random.default_rng(3)
    i1, i2, _, _, valid = oracle.e_grid(p.n_e, p.e_step)
    ctr = 10
    for trial in range(300):
        s = np.where(valid, rng.normal(0, 1.5, p.n_e * p.n_e), -np.inf)
        a, b = sorted(rng.integers(0, 21, 2))
        c, d = sorted(rng.integers(0, 21, 2))
        S = int(rng.choice([0, 2, 3, 4]))
        box = lambda x, y: a <= x <= b and c <= y <= d
        ok = lambda x, y: 0 <= x < 21 and 0 <= y < 21 and (x - ctr) ** 2 + (y - ctr) ** 2 < 100
        pts = [(x, y) for x in range(21) for y in range(21) if ok(x, y) and box(x, y)]
        if not pts:
            expect = True
        else:
            thr = max(s[x * 21 + y] for x, y in pts) + math.log(0.05)
            expect = False
            for x, y in pts:
                if s[x * 21 + y] >= thr:
                    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                        if ok(x + dx, y + dy) and not box(x + dx, y + dy):
                            expect = True
            if S:
                for x in range(21):
                    for y in range(21):
                        if ok(x, y) and not box(x, y) and (x - ctr) % S == 0 and (y - ctr) % S == 0 \
                                and s[x * 21 + y] >= thr:
                            expect = True
        assert oracle.window_rejected(s, (a, b, c, d), S, p) == expect, trial


# ---- facet sizing (Sec. 2.3) and the default scale prior (Sec. 2.2 Eq. 4, Sec. 2.4)

# One arcsecond in radians, written out as a number (IAU: 1" = pi/648000 rad),
# not computed by the oracle's own expression.
RAD_PER_ARCSEC = 4.84813681109535993589914e-6


def test_facet_theta_is_K_scale_lengths_in_radians():
    """theta = K alpha with alpha converted to radians: a 1" source at K = 38
    has a field of view of 38 arcsec = 1.8423e-4 rad, i.e. a cell of
    1/theta = 5428 wavelengths.  Dropping the arcsec conversion, sizing the
    facet by another width (a FWHM) or taking another K moves these numbers
    far outside the tolerances."""
    assert oracle.facet_theta(1.0, 38.0) == pytest.approx(38 * RAD_PER_ARCSEC, rel=1e-15)
    assert oracle.facet_theta(1.0, 38.0) == pytest.approx(1.842291988216237e-4, rel=1e-13)
    assert 1.0 / oracle.facet_theta(1.0, 38.0) == pytest.approx(5428.0, abs=0.5)
    # numpy's own degree conversion as an independent route
    for a, K in ((0.3, 38.0), (1.7, 38.0), (3.5, 20.0), (2.2, 100.0)):
        assert oracle.facet_theta(a, K) == pytest.approx(K * np.deg2rad(a / 3600.0), rel=1e-14)
    # the default K is the paper's 38 (Sec. 4.1)
    assert oracle.facet_theta(1.3) == oracle.facet_theta(1.3, 38.0)


def test_facet_cells_follow_theta():
    """A visibility at u = (k + 0.4) / theta lands in cell k and one at
    (k + 0.6) / theta in cell k + 1, so the cell width in wavelengths is the
    inverse field of view of Sec. 2.3."""
    alpha = 1.25
    theta = oracle.facet_theta(alpha)
    cell = 1.0 / (38 * alpha * RAD_PER_ARCSEC)
    ks = np.array([-3, 0, 2, 7])
    u = np.concatenate([(ks + 0.4) * cell, (ks + 0.6) * cell])
    freq = np.array([oracle.C_LIGHT])                        # wavelength 1 m: metres = wavelengths
    f = oracle.extract_facet(u, np.zeros_like(u), np.zeros_like(u), freq, np.ones_like(u),
                             np.zeros(u.size, np.complex128), (0.0, 0.0, 0.0, alpha, 0.0, 0.0), theta)
    assert sorted(f.ix.tolist()) == sorted(ks.tolist() + (ks + 1).tolist())
    assert np.all(f.iy == 0) and np.all(f.count == 1)


@pytest.mark.parametrize("flux_ujy", [10.0, 50.0, 200.0, 1000.0])
def test_default_prior_median_follows_eq4(flux_ujy):
    """With no per-source median, the scale prior is log-normal with median
    e^ADD (S/uJy)^ESP (Eq. 4, written here in its power form) and width
    R_STD = 0.3136 (Sec. 2.4), times the natural-spline quadrature weights;
    against scipy's lognorm and CubicSpline.  A flux taken in Jy instead of
    uJy, ADD and ESP swapped, or the median of another relation fails."""
    from scipy.stats import lognorm
    knots = oracle.alpha_knots(0.3, 3.5, 20)
    got = oracle.log_alpha_weights([flux_ujy * 1e-6], knots)[0]
    median = math.exp(-0.93) * flux_ujy ** 0.33
    c = np.array([scipy.interpolate.CubicSpline(knots, np.eye(20)[k], bc_type="natural").integrate(0.3, 3.5)
                  for k in range(20)])
    ref = np.log(c) + lognorm(0.3136, scale=median).logpdf(knots)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
    # the prior peaks (in ln alpha) at the median: the knot nearest it carries the largest prior density x alpha
    dens = got - np.log(c) + np.log(knots)
    assert abs(math.log(knots[int(np.argmax(dens))]) - math.log(median)) <= np.max(np.diff(np.log(knots)))
