"""Write tests/golden/noise_sigma.json: the per-config noise level.

sigma (per real/imaginary part, Jy) is set so that a reference source reaches
a stated matched-filter SNR = sqrt(sum_i |V_ref(k_i)|^2) / sigma on the
config's uv coverage:
  configs 0-2: 50 uJy, alpha = 1", circular, SNR 20;
  config 3:    10 uJy at the Eq. 4 median size, circular, SNR 8.5 (the
               paper's faintest SNR, Sec. 4.2);
  "kscan":     the facet-size experiment on the config-1 coverage: the same
               10 uJy reference at SNR 19 (Sec. 4.1: the realistic noise
               variance divided by 5, a minimum SNR of about 19).
The model is evaluated with the oracle only.

    python tests/golden/make_noise_sigma.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2203_14071_amd import synth  # noqa: E402

REFERENCE = {0: (50e-6, 1.0, 20.0), 1: (50e-6, 1.0, 20.0), 3: (10e-6, None, 8.5), "kscan": (10e-6, None, 19.0)}


def sigma_for(key):
    cfg_index = 1 if key == "kscan" else key
    cfg = synth.CONFIGS[cfg_index]
    enu = synth.antennas(cfg, synth.rng(cfg_index, synth.STREAM_ANT))
    u_m, v_m, w_m = synth.uvw_tracks(cfg, enu)
    flux, alpha, snr = REFERENCE[key]
    if alpha is None:
        alpha = float(oracle.alpha_from_flux(flux))
    cat = synth.Catalogue(*(np.array([x]) for x in (0.0, 0.0, flux, alpha, 0.0, 0.0)))
    v = oracle.sky_model(u_m, v_m, w_m, np.asarray(cfg.freq_hz), cat)
    return float(np.sqrt(np.sum(np.abs(v) ** 2)) / snr)


def main():
    out = {str(k): sigma_for(k) for k in REFERENCE}
    with open(os.path.join(HERE, "noise_sigma.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


if __name__ == "__main__":
    main()
