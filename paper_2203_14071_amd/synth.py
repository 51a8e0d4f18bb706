"""Seeded synthetic observations and source catalogues.

This module draws every random input the hot path and its oracle consume:
antenna layouts, Earth-rotation (u, v, w) tracks, source catalogues and
visibility noise.  It holds none of the method's arithmetic (no visibility
model, no extraction, no likelihood): the noiseless sky visibilities are made
by whoever consumes these arrays, with their own implementation of the model.

The workloads stand in for the paper's simulated SKA1-MID observation
(Sec. 4: 8 h at 60 s, one 1.4 GHz channel, 9,266,880 uv points, 1000 faint
star-forming galaxies), whose Measurement Set, antenna layout and catalogue
are not available.  Shapes and sizes follow that observation; the value
distributions are the ones stated in each config below.

Random streams use numpy's PCG64 with seed = 1000*config + stream (config 2,
the precision form of config 1, uses config 1's seeds):
  +1 antennas, +2 catalogue (positions, flux, scale, ellipticity in that
  order), +3 noise (real parts then imaginary parts), +4 training set,
  +5 network initialisation.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_LIGHT = 299792458.0            # m/s
SIDEREAL_DAY_S = 86164.0905      # s
SITE_LAT_DEG = -30.7             # SKA-MID-like site latitude (assumed)

STREAM_ANT, STREAM_CAT, STREAM_NOISE, STREAM_TRAIN, STREAM_INIT = 1, 2, 3, 4, 5


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n_ant: int
    layout: str                  # "disk" (uniform in a disk) | "exp" (radial pdf ~ exp(-r/scale))
    layout_radius_m: float       # disk radius, or maximum radius of the exp layout
    layout_scale_m: float        # exp scale (unused for "disk")
    n_time: int
    dt_s: float
    dec_deg: float
    freq_hz: tuple               # channel centres
    n_src: int
    field_deg: float             # side of the square field
    flux_min_ujy: float
    flux_max_ujy: float
    flux_slope: float            # pdf ~ S**flux_slope
    size_law: str                # "lognormal1" (ln a ~ N(ln 1", 0.3)) | "scaleflux" (size-flux median, N(0, 0.3136) scatter)
    e_sigma: float
    e_max: float
    noise_sigma_jy: float        # per real/imaginary part; weights are 1/sigma**2
    vis_dtype: str               # "c128" or "c64"

    @property
    def n_baselines(self) -> int:
        return self.n_ant * (self.n_ant - 1) // 2

    @property
    def n_rows(self) -> int:
        return self.n_baselines * self.n_time

    @property
    def n_chan(self) -> int:
        return len(self.freq_hz)


# Noise levels: sigma is chosen so that a reference source (config 0-2: 50 uJy,
# 1", circular; config 3: 10 uJy at the size-flux median, circular) reaches the
# matched-filter SNR stated for the config (20, resp. 8.5).  The numbers come
# from tests/golden/make_noise_sigma.py (which evaluates the visibility model
# with the oracle) and a test checks they still agree with that script.
_SIGMA = {0: 0.00017231271326032695, 1: 0.006789083290568159, 3: 0.011537361476379389}
# the facet-size experiment's noise on the config-1 coverage (same script)
SIGMA_KSCAN = 0.0014667958180515958

_CFG3_FREQS = tuple(962.5e6 + 25.0e6 * c for c in range(8))   # 8 x 25 MHz over 950-1150 MHz

CONFIGS = {
    0: Config("tiny", 20, "disk", 5000.0, 0.0, 60, 60.0, -30.0, (1.4e9,), 10, 0.5,
              50.0, 200.0, -1.6, "lognormal1", 0.3, 0.8, _SIGMA[0], "c128"),
    1: Config("ska_mid_1k", 197, "exp", 150000.0, 1500.0, 480, 60.0, -30.0, (1.4e9,), 1000, 1.0,
              50.0, 200.0, -1.6, "lognormal1", 0.3, 0.8, _SIGMA[1], "c128"),
    2: Config("ska_mid_1k_mixed", 197, "exp", 150000.0, 1500.0, 480, 60.0, -30.0, (1.4e9,), 1000, 1.0,
              50.0, 200.0, -1.6, "lognormal1", 0.3, 0.8, _SIGMA[1], "c64"),
    3: Config("ska_mid_10k_8ch", 197, "exp", 150000.0, 1500.0, 480, 60.0, -30.0, _CFG3_FREQS, 10000,
              math.sqrt(3.0), 10.0, 1000.0, -1.6, "scaleflux", 0.3, 0.8, _SIGMA[3], "c64"),
}

# Population size-flux relation used to draw config 3 sizes (the relation of
# Eq. 4 with its published coefficients, used here as a population model).
POP_SIZE_ADD, POP_SIZE_ESP, POP_SIZE_SCATTER = -0.93, 0.33, 0.3136
SIZE_MIN_ARCSEC, SIZE_MAX_ARCSEC = 0.3, 3.5


# Config 2 is config 1 in the mixed-precision form: it draws config 1's streams.
SEED_CONFIG = {2: 1}


def rng(cfg_index: int, stream: int) -> np.random.Generator:
    base = SEED_CONFIG.get(cfg_index, cfg_index)
    return np.random.Generator(np.random.PCG64(1000 * base + stream))


def antennas(cfg: Config, g: np.random.Generator) -> np.ndarray:
    """Antenna positions, local east/north/up in metres, shape [n_ant, 3]."""
    if cfg.layout == "disk":
        r = cfg.layout_radius_m * np.sqrt(g.random(cfg.n_ant))
    elif cfg.layout == "exp":
        # radial pdf ~ exp(-r/s) per unit radius on [0, rmax], by inverse CDF
        s, rmax = cfg.layout_scale_m, cfg.layout_radius_m
        r = -s * np.log1p(-g.random(cfg.n_ant) * (-math.expm1(-rmax / s)))
    else:
        raise ValueError(cfg.layout)
    phi = 2.0 * math.pi * g.random(cfg.n_ant)
    return np.stack([r * np.cos(phi), r * np.sin(phi), np.zeros(cfg.n_ant)], axis=1)


def uvw_tracks(cfg: Config, enu: np.ndarray):
    """Earth-rotation synthesis tracks (u, v, w) in metres.

    Rows are baseline-major with time fastest, so consecutive rows trace one
    baseline's uv arc.  Standard ENU -> equatorial XYZ -> uvw relations
    (Thompson, Moran & Swenson, ch. 4) with hour angles centred on transit.
    """
    lat = math.radians(SITE_LAT_DEG)
    dec = math.radians(cfg.dec_deg)
    e, n, up = enu[:, 0], enu[:, 1], enu[:, 2]
    x = -math.sin(lat) * n + math.cos(lat) * up
    y = e
    z = math.cos(lat) * n + math.sin(lat) * up
    i, j = np.triu_indices(cfg.n_ant, k=1)
    bx, by, bz = x[j] - x[i], y[j] - y[i], z[j] - z[i]
    ha = (np.arange(cfg.n_time) - 0.5 * (cfg.n_time - 1)) * cfg.dt_s * (2.0 * math.pi / SIDEREAL_DAY_S)
    sh, ch = np.sin(ha)[None, :], np.cos(ha)[None, :]
    bx, by, bz = bx[:, None], by[:, None], bz[:, None]
    u = sh * bx + ch * by
    v = -math.sin(dec) * ch * bx + math.sin(dec) * sh * by + math.cos(dec) * bz
    w = math.cos(dec) * ch * bx - math.cos(dec) * sh * by + math.sin(dec) * bz
    return (np.ascontiguousarray(u.reshape(-1)), np.ascontiguousarray(v.reshape(-1)),
            np.ascontiguousarray(w.reshape(-1)))


@dataclasses.dataclass
class Catalogue:
    l: np.ndarray
    m: np.ndarray
    flux_jy: np.ndarray
    alpha_arcsec: np.ndarray
    e1: np.ndarray
    e2: np.ndarray

    @property
    def n_src(self) -> int:
        return int(self.l.shape[0])

    def subset(self, idx) -> "Catalogue":
        return Catalogue(*(np.ascontiguousarray(a[idx]) for a in dataclasses.astuple(self)))

    def with_shape(self, e1, e2) -> "Catalogue":
        return Catalogue(self.l, self.m, self.flux_jy, self.alpha_arcsec,
                         np.ascontiguousarray(e1, dtype=np.float64), np.ascontiguousarray(e2, dtype=np.float64))


def catalogue(cfg: Config, g: np.random.Generator, n_src: int | None = None) -> Catalogue:
    """Sources drawn in the order positions, flux, scale, ellipticity.

    Sorted by decreasing flux, the processing order the paper asks for
    (Sec. 2.1).  Positions are direction cosines uniform over a square field.
    """
    n = cfg.n_src if n_src is None else n_src
    half = 0.5 * math.radians(cfg.field_deg)
    l = g.uniform(-half, half, n)
    m = g.uniform(-half, half, n)
    a1 = cfg.flux_slope + 1.0
    lo, hi = cfg.flux_min_ujy ** a1, cfg.flux_max_ujy ** a1
    flux_ujy = (lo + g.random(n) * (hi - lo)) ** (1.0 / a1)
    alpha = np.empty(n)
    for k in range(n):
        while True:
            if cfg.size_law == "lognormal1":
                a = math.exp(0.3 * g.standard_normal())
            else:
                a = math.exp(POP_SIZE_ADD + POP_SIZE_ESP * math.log(flux_ujy[k])
                             + POP_SIZE_SCATTER * g.standard_normal())
            if SIZE_MIN_ARCSEC <= a <= SIZE_MAX_ARCSEC:
                break
        alpha[k] = a
    e1 = np.empty(n)
    e2 = np.empty(n)
    for k in range(n):
        while True:
            a, b = cfg.e_sigma * g.standard_normal(2)
            if a * a + b * b < cfg.e_max * cfg.e_max:
                break
        e1[k], e2[k] = a, b
    order = np.argsort(-flux_ujy, kind="stable")
    return Catalogue(l[order], m[order], flux_ujy[order] * 1e-6, alpha[order], e1[order], e2[order])


def noise(cfg: Config, g: np.random.Generator, n_vis: int, sigma: float | None = None) -> np.ndarray:
    """Complex Gaussian noise, sigma per real/imaginary part (complex128)."""
    s = cfg.noise_sigma_jy if sigma is None else sigma
    re = g.standard_normal(n_vis)
    im = g.standard_normal(n_vis)
    out = np.empty(n_vis, dtype=np.complex128)
    out.real = s * re
    out.imag = s * im
    return out


@dataclasses.dataclass
class Observation:
    u_m: np.ndarray
    v_m: np.ndarray
    w_m: np.ndarray
    freq_hz: np.ndarray
    weight: np.ndarray           # [n_rows * n_chan], channel fastest

    @property
    def n_rows(self) -> int:
        return int(self.u_m.shape[0])

    @property
    def n_chan(self) -> int:
        return int(self.freq_hz.shape[0])


def observation(cfg_index: int, cfg: Config | None = None) -> Observation:
    cfg = CONFIGS[cfg_index] if cfg is None else cfg
    enu = antennas(cfg, rng(cfg_index, STREAM_ANT))
    u, v, w = uvw_tracks(cfg, enu)
    wt = np.full(u.shape[0] * cfg.n_chan, 1.0 / cfg.noise_sigma_jy ** 2)
    return Observation(u, v, w, np.asarray(cfg.freq_hz, dtype=np.float64), wt)


def small_config(base: int, n_ant: int, n_time: int, n_src: int, **kw) -> Config:
    """A reduced copy of a config (same distributions, fewer antennas/samples/sources)."""
    return dataclasses.replace(CONFIGS[base], n_ant=n_ant, n_time=n_time, n_src=n_src, **kw)
