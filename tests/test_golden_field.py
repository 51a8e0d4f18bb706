"""The stored full-field oracle results (tests/golden/field_oracle_cfg*.npz,
written by tests/golden/make_field_oracle.py) are consistent with themselves,
with the generator's catalogue, and with the oracle as it stands: the facet
field of view of every source, the thresholded set held by the stored points,
and for sampled sources the fit recomputed from the stored facet."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2203_14071_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("k", [1, 2])
def test_field_golden_consistent_with_oracle(k):
    path = os.path.join(GOLDEN, f"field_oracle_cfg{k}.npz")
    with np.load(path) as z:
        g = {name: z[name] for name in z.files}
    cfg = synth.CONFIGS[k]
    cat = synth.catalogue(cfg, synth.rng(k, synth.STREAM_CAT))
    n = cat.n_src
    assert int(g["config"]) == k and int(g["n_rows"]) == cfg.n_rows and g["e1"].shape == (n,)
    # facet field of view, bit for bit (Sec. 2.3)
    assert np.array_equal(g["theta"], np.array([oracle.facet_theta(a) for a in cat.alpha_arcsec]))
    # every stored source: the stored points hold its whole 5 % set, its
    # maximum and argmax; the set's size is n_above
    i1, i2, e1g, e2g, valid = oracle.e_grid(81, 0.02)
    off = g["pt_offsets"]
    assert off[0] == 0 and off[-1] == g["pt_index"].size == g["pt_value"].size
    for s in range(n):
        idx = g["pt_index"][off[s]:off[s + 1]].astype(np.int64)
        val = g["pt_value"][off[s]:off[s + 1]]
        assert np.all(valid[idx])
        assert val.max() == g["lmax"][s] and idx[np.argmax(val)] == g["argmax"][s]
        assert np.count_nonzero(val >= g["lmax"][s] + math.log(0.05)) == g["n_above"][s]
        assert val.min() >= g["lmax"][s] + math.log(0.05) - float(g["band"])
        # the estimate from the stored points alone is the stored estimate
        surf = np.full(81 * 81, -np.inf)
        surf[idx] = val
        est = oracle.estimate(surf, e1g, e2g, valid, 81)
        assert (est.e1, est.e2, est.s1, est.s2, est.c12, est.flags) == \
            (g["e1"][s], g["e2"][s], g["s1"][s], g["s2"][s], g["c12"][s], g["flags"][s]), s
    # sampled sources: the stored surface is the oracle's fit of the stored facet
    for j, s in enumerate(g["sample_src"][:2]):
        s = int(s)
        th = float(g["theta"][s])
        ix, iy = g[f"sample{j}_ix"], g[f"sample{j}_iy"]
        f = oracle.Facet(th, ix, iy, g[f"sample{j}_count"], g[f"sample{j}_wsum"], g[f"sample{j}_vbar"],
                         ix / th, iy / th)
        assert f.n_cells == g["n_cells"][s]
        surf, est = oracle.fit_source(f, cat.flux_jy[s])
        assert np.array_equal(surf, g["sample_surface"][j])
        assert est.e1 == g["e1"][s] and est.e2 == g["e2"][s]


def test_config3_sample_golden_consistent_with_oracle():
    """tests/golden/cfg3_sample_oracle.npz: the sampled sources are the
    generator's by its stated rule, theta is the oracle's, and every stored
    estimate is the oracle's estimator on the stored surface."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_cfg3", os.path.join(GOLDEN, "make_cfg3_sample_oracle.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    with np.load(os.path.join(GOLDEN, "cfg3_sample_oracle.npz")) as z:
        g = {name: z[name] for name in z.files}
    cfg = synth.CONFIGS[3]
    cat = synth.catalogue(cfg, synth.rng(3, synth.STREAM_CAT))
    src = mk.sample_sources(cat)
    assert list(g["src"]) == src and len(src) == 32
    assert int(np.argmin(cat.alpha_arcsec)) in src and int(np.argmax(cat.alpha_arcsec)) in src
    assert np.array_equal(g["theta"], np.array([oracle.facet_theta(cat.alpha_arcsec[s]) for s in src]))
    i1, i2, e1g, e2g, valid = oracle.e_grid(81, 0.02)
    for j in range(len(src)):
        est = oracle.estimate(g["surface"][j], e1g, e2g, valid, 81)
        assert (est.e1, est.e2, est.s1, est.s2, est.c12, est.lmax, est.argmax, est.n_above, est.flags) == \
            (g["e1"][j], g["e2"][j], g["s1"][j], g["s2"][j], g["c12"][j], g["lmax"][j], g["argmax"][j],
             g["n_above"][j], g["flags"][j]), j
        assert np.all(np.isneginf(g["surface"][j][~valid]))
