"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/rlf.h, the ctypes structures match the C layout, the
host-only entry points compute what they document, and invalid arguments
come back as status codes."""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2203_14071_amd import rlf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rlf.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|int64_t|const char \*)\s*(rlf_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = rlf.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(rlf.exported_symbols()) == names
    out = subprocess.run(["nm", "-D", "--defined-only", rlf.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, flags=re.M), n


def test_struct_layout_matches_header(tmp_path):
    """Compile a C probe against include/rlf.h with gcc and compare sizes and
    offsets with the ctypes mirrors."""
    structs = {"rlf_params": rlf.rlf_params, "rlf_obs": rlf.rlf_obs, "rlf_catalog": rlf.rlf_catalog,
               "rlf_fit_opts": rlf.rlf_fit_opts, "rlf_fit_out": rlf.rlf_fit_out}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rlf.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        s, f, v = ln.split()
        got[(s, f)] = int(v)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)


def test_params_default_are_the_papers():
    import json
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")))
    p = rlf.params()
    assert p.beta == g["beta"]["value"] and p.add == g["add"]["value"] and p.esp == g["esp"]["value"]
    assert p.K == g["K"]["value"] and p.r_std == g["r_std"]["value"]
    assert p.rmin_arcsec == g["rmin_arcsec"]["value"] and p.rmax_arcsec == g["rmax_arcsec"]["value"]
    assert p.frac_thresh == g["frac_thresh"]["value"]
    assert p.bad_sigma == g["bad_sigma"]["value"] and p.bad_sqrtdet == g["bad_sqrtdet"]["value"]
    assert p.ref_freq_hz == g["ref_freq_hz"]["value"]
    assert (p.num_r, p.n_e, p.e_step, p.precision) == (20, 81, 0.02, rlf.RLF_FP64)
    assert rlf.lib().rlf_version() >= 100


def test_alpha_from_flux_is_eq4():
    f = np.array([1e-6, 10e-6, 55e-6, 1e-3])
    a = rlf.alpha_from_flux(f)
    assert np.allclose(a, np.exp(-0.93 + 0.33 * np.log(f * 1e6)), rtol=1e-15, atol=0)
    assert a[0] == pytest.approx(math.exp(-0.93), rel=1e-15)
    with pytest.raises(rlf.RlfError):
        rlf.alpha_from_flux(np.array([1e-6, -1.0]))


def test_invalid_arguments_return_status_without_crashing():
    L = rlf.lib()
    assert L.rlf_params_default(None) == rlf.RLF_EINVAL
    assert L.rlf_model_vis(None, None, None, 0, 0, None, 0) == rlf.RLF_EINVAL
    assert L.rlf_extract_facets(None, None, None, None, None) == rlf.RLF_EINVAL
    assert L.rlf_fit_sources(None, None, None, None) == rlf.RLF_EINVAL
    assert L.rlf_facets_free(None) == rlf.RLF_OK
    assert L.rlf_destroy(None) == rlf.RLF_OK
    assert L.rlf_sync(None) == rlf.RLF_EINVAL
    h = ctypes.c_void_p()
    for bad in (dict(num_r=1), dict(num_r=33), dict(n_e=80), dict(n_e=1), dict(e_step=0.03),
                dict(rmin_arcsec=3.5), dict(K=0.0), dict(precision=7), dict(frac_thresh=0.0),
                dict(reserved=1), dict(r_std=-1.0)):
        p = rlf.params(**bad)
        assert L.rlf_create(ctypes.byref(h), 0, None, ctypes.byref(p)) == rlf.RLF_EINVAL, bad
    p = rlf.params()
    assert L.rlf_create(None, 0, None, ctypes.byref(p)) == rlf.RLF_EINVAL
    assert L.rlf_create(ctypes.byref(h), -1, None, ctypes.byref(p)) == rlf.RLF_EINVAL


def test_create_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    p = rlf.params()
    assert rlf.lib().rlf_create(ctypes.byref(h), 0, None, ctypes.byref(p)) == rlf.RLF_EDEVICE
