"""The kernels' FP64 elementary functions against extended-precision
references.

exp(2 pi i phi) (the exact reduction to 1/T turn, a
T-entry table and short Taylor polynomials; T = 1024 and T = 2048) against
an extended-precision reference, over phases the sky model and the
extraction meet (a few thousand turns) and far beyond (up to 2^39 turns),
including the points half a table step from a table entry, where the
polynomials' argument and their truncation are largest.

Bound: the table entry, the polynomial value and the final FMA each round
once, by at most 2^-53 of a value at most 1 (1.1e-16 each), plus the
truncation of the series (cos to x^4: < 1.2e-18; sin to x^5 with 1024
entries: < 4.3e-22, sin to x^3 with 2048 entries: < 7.2e-17), so every
component is within 4.1e-16 of exp(2 pi i phi)."""
import ctypes
import os

import numpy as np
import pytest

from paper_2203_14071_amd import build

pytestmark = pytest.mark.gpu

TWO_PI = 2 * np.longdouble("3.14159265358979323846264338327950288")


def _phases(table):
    rng = np.random.default_rng(20260 + table)
    n = 1 << 18
    typical = rng.uniform(-5000.0, 5000.0, n)
    far = rng.integers(-(1 << 39), 1 << 39, n).astype(np.float64) + rng.uniform(-0.5, 0.5, n)
    k = rng.integers(-(1 << 20), 1 << 20, n).astype(np.float64)
    # half a table step from an entry, on either side (|d| = 1/(2T) up to rounding)
    half = (2.0 * k + rng.choice([-1.0, 1.0], n)) / (2.0 * table)
    return np.concatenate([typical, far, half, np.array([0.0, 0.25, 0.5, -0.5, 1.0 / table, -1.0 / table])])


@pytest.mark.parametrize("table", [1024, 2048])
def test_table_exp_matches_extended_precision(table):
    assert os.path.exists(build.PROBE_LIB), "probe library not built"
    lib = ctypes.CDLL(build.PROBE_LIB)
    lib.valu_probe_cis.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    phi = np.ascontiguousarray(_phases(table))
    out = np.empty((phi.size, 2))
    rc = lib.valu_probe_cis(table, phi.ctypes.data, phi.size, out.ctypes.data)
    assert rc == 0, rc
    frac = (phi - np.rint(phi)).astype(np.longdouble)   # exact: |phi| < 2^52
    ang = TWO_PI * frac
    err_c = np.abs(out[:, 0].astype(np.longdouble) - np.cos(ang)).astype(np.float64)
    err_s = np.abs(out[:, 1].astype(np.longdouble) - np.sin(ang)).astype(np.float64)
    worst = max(err_c.max(), err_s.max())
    print(f"T = {table}: max |error| {worst:.3e} (cos {err_c.max():.3e}, sin {err_s.max():.3e}) over {phi.size} phases")
    assert worst <= 4.1e-16


def test_profile_power_matches_extended_precision():
    """pow_m32_f64(x) = (2/3) x^(-3/2) from v_rsq_f64 and one correction,
    y^3 (5/3 - x y^2): with e = 1 - x y^2 the correction leaves a relative
    error of (15/8) e^2, below 2.7e-14 for |e| <= 2^-23, plus a few
    roundings; arguments 1 + s q from 1 to 2^40 (measured: 2.0e-14, so the
    instruction's error reaches about 2^-23.2 at some of these arguments,
    more than the 2^-24.2 of the probe's log-uniform sweep)."""
    assert os.path.exists(build.PROBE_LIB), "probe library not built"
    lib = ctypes.CDLL(build.PROBE_LIB)
    lib.valu_probe_pow_m32.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    rng = np.random.default_rng(3)
    x = np.ascontiguousarray(np.concatenate([np.exp2(rng.uniform(0.0, 40.0, 1 << 20)), [1.0, 2.0, 4.0, 2.0 ** 40]]))
    out = np.empty_like(x)
    assert lib.valu_probe_pow_m32(x.ctypes.data, x.size, out.ctypes.data) == 0
    xl = x.astype(np.longdouble)
    ref = (np.longdouble(2) / 3) / (xl * np.sqrt(xl))
    rel = np.abs((out.astype(np.longdouble) - ref) / ref).astype(np.float64)
    print(f"pow_m32_f64: max relative error {rel.max():.3e} over {x.size} arguments")
    assert rel.max() < 3e-14
