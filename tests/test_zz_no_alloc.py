"""rlf_model_vis_noalloc (the sky model without device allocation, its tables
in a fixed library-owned device array) against rlf_model_vis: bit-identical
outputs in every mode and both forms, on two calls in a row (the second with
fewer rows, channels and sources than the first), and the size limit."""
import numpy as np
import pytest

from paper_2203_14071_amd import rlf, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _field(n_ant, n_time, n_src, freq, seed):
    import dataclasses
    cfg = synth.small_config(3, n_ant=n_ant, n_time=n_time, n_src=n_src)
    cfg = dataclasses.replace(cfg, freq_hz=freq)
    o = synth.observation(3, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(seed))
    rng = np.random.default_rng(seed + 1)
    n = o.n_rows * o.n_chan
    vis = 1e-3 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    return o, cat, vis


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_model_matches_model_vis(precision):
    torch = G.torch_cuda()
    mixed = precision == "mixed"
    ctx = rlf.Context(0, None, rlf.params(precision=rlf.RLF_MIXED if mixed else rlf.RLF_FP64))
    # first call: 3000 sources (a range of them), 3 channels; second: fewer rows, channels and sources
    cases = [(_field(40, 30, 3500, (1.0e9, 1.05e9, 1.1e9), 3), 250, 3250),
             (_field(12, 10, 40, (1.4e9,), 5), 3, 40)]
    for (o, cat, vis), b, e in cases:
        obs = G.make_obs(o, vis, mixed=mixed)
        for mode in (rlf.RLF_MODEL_WRITE, rlf.RLF_MODEL_ACCUMULATE, rlf.RLF_MODEL_RESIDUAL):
            ref = obs.vis.clone() if mode != rlf.RLF_MODEL_WRITE else torch.full_like(obs.vis, 7.0)
            got = ref.clone()
            ctx.model_vis(obs, cat, ref, mode=mode, src_begin=b, src_end=e)
            ctx.model_vis_noalloc(obs, cat, got, mode=mode, src_begin=b, src_end=e)
            ctx.sync()
            assert torch.equal(torch.view_as_real(got), torch.view_as_real(ref)), (precision, mode, e - b)
    # the scratch holds at most 4096 sources per call
    o, cat, vis = _field(8, 4, 4097, (1.4e9,), 7)
    obs = G.make_obs(o, vis, mixed=mixed)
    out = torch.empty_like(obs.vis)
    with pytest.raises(rlf.RlfError) as ei:
        ctx.model_vis_noalloc(obs, cat, out)
    assert ei.value.code == rlf.RLF_EINVAL
    ctx.model_vis_noalloc(obs, cat, out, src_begin=1, src_end=4097)      # 4096: accepted
    ctx.sync()
    ctx.close()
