"""The facet-size experiment's bias estimator: least squares of
e_measured - e_true = m e_true + c on constructed data."""
import numpy as np
import pytest

from paper_2203_14071_amd import kscan


def test_bias_line_recovers_m_and_c():
    rng = np.random.default_rng(3)
    e = rng.uniform(-0.7, 0.7, 5000)
    meas = (1.0 + 0.05) * e - 0.002
    m, c, sm, sc = kscan.bias_line(e, meas)
    assert m == pytest.approx(0.05, abs=1e-12) and c == pytest.approx(-0.002, abs=1e-12)
    assert sm < 1e-12 and sc < 1e-12
    noisy = meas + 0.01 * rng.standard_normal(e.size)
    m, c, sm, sc = kscan.bias_line(e, noisy)
    assert abs(m - 0.05) < 4 * sm and abs(c + 0.002) < 4 * sc
    assert sm == pytest.approx(0.01 / (np.std(e) * np.sqrt(e.size)), rel=0.05)


def test_population_follows_the_papers_description():
    cfg, cat = kscan.population(2000)
    f = cat.flux_jy * 1e6
    assert f.min() >= 10.0 and f.max() <= 200.0
    assert np.all(np.hypot(cat.e1, cat.e2) < 0.8)
    assert cfg.noise_sigma_jy == kscan.synth.SIGMA_KSCAN
    # S^-1.6 on [10, 200]: the median is 10 * (1 + (20^-0.6 - 1) / 2)^(-1 / 0.6)
    med = 10.0 * (1 + (20.0 ** -0.6 - 1) / 2) ** (-1 / 0.6)
    assert np.median(f) == pytest.approx(med, rel=0.05)
