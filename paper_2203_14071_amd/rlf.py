"""Python binding of the C ABI in include/rlf.h (ctypes; argument marshalling only).

Every computation runs in librlf.so's HIP kernels.  PyTorch supplies device
memory (tensor data pointers) and the stream (torch's current stream by
default).  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librlf.so")

RLF_OK, RLF_EINVAL, RLF_ENOMEM, RLF_EDEVICE, RLF_ERANGE, RLF_EUNSUPPORTED, RLF_EIO = 0, -1, -2, -3, -4, -5, -6
RLF_FP64, RLF_MIXED = 0, 1
RLF_FLAG_BAD_VAR, RLF_FLAG_EMPTY, RLF_FLAG_EDGE, RLF_FLAG_FALLBACK, RLF_FLAG_REFIT, RLF_FLAG_REFINED = 1, 2, 4, 8, 16, 32
RLF_MODEL_WRITE, RLF_MODEL_ACCUMULATE, RLF_MODEL_RESIDUAL = 0, 1, 2

_c_dp = ctypes.POINTER(ctypes.c_double)
_c_ip = ctypes.POINTER(ctypes.c_int32)
_c_lp = ctypes.POINTER(ctypes.c_int64)
_c_up = ctypes.POINTER(ctypes.c_uint32)
_c_vp = ctypes.c_void_p


class rlf_params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("ref_freq_hz", ctypes.c_double), ("K", ctypes.c_double),
                ("add", ctypes.c_double), ("esp", ctypes.c_double), ("r_std", ctypes.c_double),
                ("rmin_arcsec", ctypes.c_double), ("rmax_arcsec", ctypes.c_double),
                ("num_r", ctypes.c_int32), ("n_e", ctypes.c_int32), ("e_step", ctypes.c_double),
                ("frac_thresh", ctypes.c_double), ("bad_sigma", ctypes.c_double),
                ("bad_sqrtdet", ctypes.c_double), ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class rlf_obs(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_chan", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("u_m", _c_vp), ("v_m", _c_vp), ("w_m", _c_vp), ("freq_hz_host", _c_dp),
                ("vis", _c_vp), ("weight", _c_vp)]


class rlf_catalog(ctypes.Structure):
    _fields_ = [("n_src", ctypes.c_int64), ("l", _c_dp), ("m", _c_dp), ("flux_jy", _c_dp),
                ("alpha_arcsec", _c_dp), ("e1", _c_dp), ("e2", _c_dp), ("prior_mu", _c_dp)]


class rlf_fit_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("want_surface", ctypes.c_int32), ("window", _c_vp),
                ("fallback", ctypes.c_int32), ("check_stride", ctypes.c_int32)]


class rlf_fit_out(ctypes.Structure):
    _fields_ = [("e1", _c_vp), ("e2", _c_vp), ("s1", _c_vp), ("s2", _c_vp), ("c12", _c_vp), ("lmax", _c_vp),
                ("argmax", _c_vp), ("n_above", _c_vp), ("flags", _c_vp), ("surface", _c_vp)]


_SIGNATURES = {
    "rlf_version": ([], ctypes.c_int),
    "rlf_params_default": ([ctypes.POINTER(rlf_params)], ctypes.c_int),
    "rlf_create": ([ctypes.POINTER(_c_vp), ctypes.c_int, _c_vp, ctypes.POINTER(rlf_params)], ctypes.c_int),
    "rlf_destroy": ([_c_vp], ctypes.c_int),
    "rlf_set_stream": ([_c_vp, _c_vp], ctypes.c_int),
    "rlf_sync": ([_c_vp], ctypes.c_int),
    "rlf_last_error": ([_c_vp], ctypes.c_char_p),
    "rlf_alpha_from_flux": ([_c_dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, _c_dp], ctypes.c_int),
    "rlf_model_vis": ([_c_vp, ctypes.POINTER(rlf_obs), ctypes.POINTER(rlf_catalog), ctypes.c_int64,
                       ctypes.c_int64, _c_vp, ctypes.c_int], ctypes.c_int),
    "rlf_model_vis_noalloc": ([_c_vp, ctypes.POINTER(rlf_obs), ctypes.POINTER(rlf_catalog), ctypes.c_int64,
                               ctypes.c_int64, _c_vp, ctypes.c_int], ctypes.c_int),
    "rlf_facets_create": ([_c_vp, ctypes.POINTER(rlf_obs), ctypes.POINTER(rlf_catalog), ctypes.POINTER(_c_vp)],
                          ctypes.c_int),
    "rlf_extract_facets": ([_c_vp, ctypes.POINTER(rlf_obs), ctypes.POINTER(rlf_catalog), _c_vp, _c_vp],
                           ctypes.c_int),
    "rlf_facets_info": ([_c_vp, _c_vp, _c_lp, _c_lp, _c_lp], ctypes.c_int),
    "rlf_facets_copy": ([_c_vp, _c_vp, _c_lp, _c_ip, _c_ip, _c_ip, _c_dp, _c_dp, _c_dp], ctypes.c_int),
    "rlf_facets_free": ([_c_vp], ctypes.c_int),
    "rlf_facets_set_positions": ([_c_vp, _c_vp, ctypes.c_int32, ctypes.c_double], ctypes.c_int),
    "rlf_fit_sources": ([_c_vp, _c_vp, ctypes.POINTER(rlf_fit_opts), ctypes.POINTER(rlf_fit_out)], ctypes.c_int),
    "rlf_pass_create": ([_c_vp, ctypes.POINTER(rlf_obs), ctypes.POINTER(rlf_catalog), _c_vp,
                         ctypes.POINTER(rlf_fit_opts), ctypes.POINTER(rlf_fit_out), ctypes.c_char_p,
                         ctypes.POINTER(_c_vp)], ctypes.c_int),
    "rlf_refine_sources": ([_c_vp, _c_vp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(rlf_fit_out)], ctypes.c_int),
    "rlf_fit_sequential": ([_c_vp, ctypes.POINTER(rlf_obs), ctypes.POINTER(rlf_catalog), ctypes.c_int64,
                            ctypes.c_int32, ctypes.POINTER(rlf_fit_out), _c_dp, _c_dp], ctypes.c_int),
    "rlf_pass_launch": ([_c_vp], ctypes.c_int),
    "rlf_pass_tiles": ([_c_vp, _c_ip, _c_ip], ctypes.c_int),
    "rlf_pass_free": ([_c_vp], ctypes.c_int),
    "rlf_mlp_num_params": ([], ctypes.c_int64),
    "rlf_mlp_create": ([_c_vp, ctypes.c_int64, ctypes.POINTER(_c_vp)], ctypes.c_int),
    "rlf_mlp_free": ([_c_vp], ctypes.c_int),
    "rlf_mlp_set_state": ([_c_vp, _c_vp, _c_vp, _c_vp, ctypes.c_int64], ctypes.c_int),
    "rlf_mlp_get_state": ([_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_lp], ctypes.c_int),
    "rlf_mlp_save": ([_c_vp, ctypes.c_char_p], ctypes.c_int),
    "rlf_mlp_load": ([_c_vp, ctypes.c_char_p], ctypes.c_int),
    "rlf_mlp_features": ([_c_vp, _c_vp, _c_vp], ctypes.c_int),
    "rlf_mlp_forward": ([_c_vp, _c_vp, ctypes.c_int64, _c_vp], ctypes.c_int),
    "rlf_mlp_train_step": ([_c_vp, _c_vp, _c_vp, ctypes.c_int64, ctypes.c_float, _c_vp], ctypes.c_int),
    "rlf_mlp_predict": ([_c_vp, _c_vp, _c_vp], ctypes.c_int),
    "rlf_mlp_train_facets": ([_c_vp, _c_vp, _c_vp, ctypes.c_float, _c_vp], ctypes.c_int),
    "rlf_mlp_posterior_targets": ([_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_uint64, _c_vp], ctypes.c_int),
    "rlf_mlp_windows": ([_c_vp, _c_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_double, _c_vp],
                        ctypes.c_int),
}

_lib = None


def lib():
    """The loaded librlf.so; raises if it is missing (build it with paper_2203_14071_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -m paper_2203_14071_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class RlfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rlf error {code}: {msg}")
        self.code = code


def _dp(a):
    return None if a is None else a.ctypes.data_as(_c_dp)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def params(**kw) -> rlf_params:
    p = rlf_params()
    lib().rlf_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


@dataclasses.dataclass
class Obs:
    """Device-resident observation (torch tensors on the context's device)."""
    u_m: object
    v_m: object
    w_m: object
    freq_hz: np.ndarray
    vis: object
    weight: object

    def c(self) -> rlf_obs:
        o = rlf_obs()
        o.n_rows = int(self.u_m.shape[0])
        o.n_chan = int(len(self.freq_hz))
        o.reserved = 0
        o.u_m, o.v_m, o.w_m = _ptr(self.u_m), _ptr(self.v_m), _ptr(self.w_m)
        self._freq = np.ascontiguousarray(self.freq_hz, dtype=np.float64)
        o.freq_hz_host = _dp(self._freq)
        o.vis = _ptr(self.vis)
        o.weight = _ptr(self.weight)
        return o


def catalog(cat, prior_mu=None):
    """rlf_catalog over host arrays of an object with l, m, flux_jy, alpha_arcsec, e1, e2.
    Returns (struct, keepalive)."""
    arrs = [np.ascontiguousarray(getattr(cat, k), dtype=np.float64)
            for k in ("l", "m", "flux_jy", "alpha_arcsec", "e1", "e2")]
    mu = None if prior_mu is None else np.ascontiguousarray(prior_mu, dtype=np.float64)
    c = rlf_catalog()
    c.n_src = int(arrs[0].shape[0])
    c.l, c.m, c.flux_jy, c.alpha_arcsec, c.e1, c.e2 = (_dp(a) for a in arrs)
    c.prior_mu = _dp(mu)
    return c, (arrs, mu)


class Context:
    """Owns an rlf_ctx; methods mirror the rlf_* entry points."""

    def __init__(self, device=0, stream=None, p: rlf_params | None = None):
        self.p = params() if p is None else p
        h = _c_vp()
        rc = lib().rlf_create(ctypes.byref(h), int(device), _c_vp(stream) if stream else None, ctypes.byref(self.p))
        if rc != RLF_OK:
            raise RlfError(rc, "rlf_create failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            lib().rlf_destroy(self.h)
            self.h = None

    def __del__(self):
        # at interpreter exit the HIP runtime may already be gone: leave the
        # device memory to the process teardown
        if sys is None or sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != RLF_OK:
            raise RlfError(rc, (lib().rlf_last_error(self.h) or b"").decode())
        return rc

    def set_stream(self, stream):
        return self._check(lib().rlf_set_stream(self.h, _c_vp(stream) if stream else None))

    def sync(self):
        return self._check(lib().rlf_sync(self.h))

    def model_vis(self, obs: Obs, cat, out, mode=RLF_MODEL_WRITE, src_begin=0, src_end=None, prior_mu=None):
        o = obs.c()
        c, keep = catalog(cat, prior_mu)
        end = c.n_src if src_end is None else src_end
        return self._check(lib().rlf_model_vis(self.h, ctypes.byref(o), ctypes.byref(c), int(src_begin), int(end),
                                               _ptr(out), int(mode)))

    def model_vis_noalloc(self, obs: Obs, cat, out, mode=RLF_MODEL_WRITE, src_begin=0, src_end=None):
        """rlf_model_vis_noalloc: model_vis without device allocation (at most 4096 sources per call)."""
        o = obs.c()
        c, keep = catalog(cat)
        end = c.n_src if src_end is None else src_end
        return self._check(lib().rlf_model_vis_noalloc(self.h, ctypes.byref(o), ctypes.byref(c), int(src_begin),
                                                       int(end), _ptr(out), int(mode)))

    def facets_create(self, obs: Obs, cat, prior_mu=None) -> "Facets":
        o = obs.c()
        c, keep = catalog(cat, prior_mu)
        h = _c_vp()
        self._check(lib().rlf_facets_create(self.h, ctypes.byref(o), ctypes.byref(c), ctypes.byref(h)))
        return Facets(self, h)

    def extract_facets(self, obs: Obs, cat, residual, facets: "Facets", prior_mu=None):
        o = obs.c()
        c, keep = catalog(cat, prior_mu)
        return self._check(lib().rlf_extract_facets(self.h, ctypes.byref(o), ctypes.byref(c), _ptr(residual),
                                                     facets.h))

    def fit_sources(self, facets: "Facets", out: dict, mode=0, window=None, want_surface=False, fallback=False,
                    check_stride=0):
        """out: dict of torch device tensors e1, e2, s1, s2, c12, lmax (f64), argmax, n_above (i32),
        flags (i32 viewed as u32), surface (f64) -- any may be absent except flags."""
        o, r = _fit_structs(out, mode, window, want_surface, fallback, check_stride)
        return self._check(lib().rlf_fit_sources(self.h, facets.h, ctypes.byref(o), ctypes.byref(r)))

    def set_positions(self, facets: "Facets", n_side, step_arcsec=0.0):
        """Marginalise later fits of `facets` over an n_side x n_side grid of
        position offsets at spacing step_arcsec (n_side = 1: position fixed)."""
        return self._check(lib().rlf_facets_set_positions(self.h, facets.h, int(n_side), float(step_arcsec)))

    def refine_sources(self, facets: "Facets", out: dict, np_max=30, e_res=0.003):
        """Adaptive refinement of the last full-grid fit of `facets` (in place in `out`)."""
        _, r = _fit_structs(out, 0, None, False, False)
        return self._check(lib().rlf_refine_sources(self.h, facets.h, int(np_max), float(e_res), ctypes.byref(r)))

    def fit_sequential(self, obs: Obs, cat, chunk, out: dict, refit_bad=True, prior_mu=None):
        """Sequential sky-model refinement; `out` as for fit_sources (e1, e2,
        flags required).  Returns the final model shapes (e1, e2) as numpy."""
        o = obs.c()
        c, keep = catalog(cat, prior_mu)
        _, r = _fit_structs(out, 0, None, False, False)
        e1 = np.zeros(c.n_src)
        e2 = np.zeros(c.n_src)
        self._check(lib().rlf_fit_sequential(self.h, ctypes.byref(o), ctypes.byref(c), int(chunk),
                                             1 if refit_bad else 0, ctypes.byref(r), _dp(e1), _dp(e2)))
        return e1, e2

    def pass_create(self, obs: Obs, cat, facets: "Facets", out: dict, tune_path=None, mode=0, window=None,
                    want_surface=False, fallback=False, prior_mu=None, check_stride=0) -> "Pass":
        o, r = _fit_structs(out, mode, window, want_surface, fallback, check_stride)
        ob = obs.c()
        c, keep = catalog(cat, prior_mu)
        h = _c_vp()
        tp = None if tune_path is None else os.fsencode(tune_path)
        self._check(lib().rlf_pass_create(self.h, ctypes.byref(ob), ctypes.byref(c), facets.h, ctypes.byref(o),
                                          ctypes.byref(r), tp, ctypes.byref(h)))
        return Pass(self, h)


def _fit_structs(out, mode, window, want_surface, fallback, check_stride=0):
    o = rlf_fit_opts()
    o.mode = int(mode)
    o.want_surface = 1 if want_surface else 0
    o.window = _ptr(window)
    o.fallback = 1 if fallback else 0
    o.check_stride = int(check_stride)
    r = rlf_fit_out()
    for k in ("e1", "e2", "s1", "s2", "c12", "lmax", "argmax", "n_above", "flags", "surface"):
        setattr(r, k, _ptr(out.get(k)))
    return o, r


class Pass:
    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h

    def launch(self):
        return self.ctx._check(lib().rlf_pass_launch(self.h))

    def tiles(self):
        t = (ctypes.c_int32 * 4)()
        u = (ctypes.c_int32 * 4)()
        self.ctx._check(lib().rlf_pass_tiles(self.h, t, u))
        return list(t), list(u)

    def free(self):
        if self.h:
            lib().rlf_pass_free(self.h)
            self.h = None

    def __del__(self):
        # at interpreter exit the HIP runtime may already be gone: leave the
        # device memory to the process teardown
        if sys is None or sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


class Facets:
    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h

    def free(self):
        if self.h:
            lib().rlf_facets_free(self.h)
            self.h = None

    def __del__(self):
        # at interpreter exit the HIP runtime may already be gone: leave the
        # device memory to the process teardown
        if sys is None or sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass

    def info(self):
        n_src, n_cells, n_dense = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self.ctx._check(lib().rlf_facets_info(self.ctx.h, self.h, ctypes.byref(n_src), ctypes.byref(n_cells),
                                              ctypes.byref(n_dense)))
        return n_src.value, n_cells.value, n_dense.value

    def copy(self):
        """Host copy of the last extraction: dict of numpy arrays (synchronises)."""
        n_src, n_cells, _ = self.info()
        off = np.zeros(n_src + 1, np.int64)
        ix = np.zeros(n_cells, np.int32)
        iy = np.zeros(n_cells, np.int32)
        cnt = np.zeros(n_cells, np.int32)
        ws = np.zeros(n_cells, np.float64)
        vb = np.zeros(2 * n_cells, np.float64)
        th = np.zeros(n_src, np.float64)
        self.ctx._check(lib().rlf_facets_copy(self.ctx.h, self.h, off.ctypes.data_as(_c_lp),
                                              ix.ctypes.data_as(_c_ip), iy.ctypes.data_as(_c_ip),
                                              cnt.ctypes.data_as(_c_ip), _dp(ws), _dp(vb), _dp(th)))
        return dict(offsets=off, ix=ix, iy=iy, count=cnt, wsum=ws, vbar=vb[0::2] + 1j * vb[1::2], theta=th)


def _np_ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class Mlp:
    """The grid-narrowing network (rlf_mlp_*); tensors are torch device tensors."""

    def __init__(self, ctx: Context, max_batch=512):
        self.ctx = ctx
        h = _c_vp()
        ctx._check(lib().rlf_mlp_create(ctx.h, int(max_batch), ctypes.byref(h)))
        self.h = h
        self.n_params = int(lib().rlf_mlp_num_params())

    def free(self):
        if self.h:
            lib().rlf_mlp_free(self.h)
            self.h = None

    def __del__(self):
        # at interpreter exit the HIP runtime may already be gone: leave the
        # device memory to the process teardown
        if sys is None or sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass

    def set_state(self, params, m=None, v=None, step=0):
        p = np.ascontiguousarray(params, dtype=np.float32)
        mm = None if m is None else np.ascontiguousarray(m, dtype=np.float32)
        vv = None if v is None else np.ascontiguousarray(v, dtype=np.float32)
        assert p.size == self.n_params
        self.ctx._check(lib().rlf_mlp_set_state(self.h, _np_ptr(p), _np_ptr(mm), _np_ptr(vv), int(step)))

    def get_state(self):
        out = {k: np.zeros(self.n_params, np.float32) for k in ("params", "m", "v", "grad")}
        st = ctypes.c_int64()
        self.ctx._check(lib().rlf_mlp_get_state(self.h, _np_ptr(out["params"]), _np_ptr(out["m"]),
                                                _np_ptr(out["v"]), _np_ptr(out["grad"]), ctypes.byref(st)))
        out["step"] = st.value
        return out

    def save(self, path):
        """Checkpoint (parameters, Adam moments, step) to a file (rlf_mlp_save)."""
        self.ctx._check(lib().rlf_mlp_save(self.h, os.fsencode(path)))

    def load(self, path):
        """Restore a checkpoint written by save (rlf_mlp_load)."""
        self.ctx._check(lib().rlf_mlp_load(self.h, os.fsencode(path)))

    def features(self, facets: "Facets", x):
        return self.ctx._check(lib().rlf_mlp_features(self.ctx.h, facets.h, _ptr(x)))

    def forward(self, x, y):
        return self.ctx._check(lib().rlf_mlp_forward(self.h, _ptr(x), int(x.shape[0]), _ptr(y)))

    def train_step(self, x, target, lr, loss):
        return self.ctx._check(lib().rlf_mlp_train_step(self.h, _ptr(x), _ptr(target), int(x.shape[0]),
                                                        float(lr), _ptr(loss)))

    def predict(self, facets: "Facets", y):
        """rlf_mlp_predict: the network on every source of a facet object."""
        return self.ctx._check(lib().rlf_mlp_predict(self.h, facets.h, _ptr(y)))

    def train_facets(self, facets: "Facets", target, lr, loss):
        """rlf_mlp_train_facets: one Adam step on the sources of a facet object."""
        return self.ctx._check(lib().rlf_mlp_train_facets(self.h, facets.h, _ptr(target), float(lr), _ptr(loss)))

    def posterior_targets(self, e1, e2, s1, s2, ln_alpha, target, kappa, seed):
        """rlf_mlp_posterior_targets: targets drawn around the full-grid estimates."""
        return self.ctx._check(lib().rlf_mlp_posterior_targets(self.ctx.h, _ptr(e1), _ptr(e2), _ptr(s1), _ptr(s2),
                                                               _ptr(ln_alpha), int(e1.shape[0]), float(kappa),
                                                               int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(target)))

    def windows(self, y, window, nsigma=3.0, min_half=3, full_frac=1.0):
        return self.ctx._check(lib().rlf_mlp_windows(self.ctx.h, _ptr(y), int(y.shape[0]), float(nsigma),
                                                     int(min_half), float(full_frac), _ptr(window)))


def alpha_from_flux(flux_jy, add=-0.93, esp=0.33):
    f = np.ascontiguousarray(flux_jy, dtype=np.float64)
    out = np.empty_like(f)
    rc = lib().rlf_alpha_from_flux(_dp(f), int(f.shape[0]), float(add), float(esp), _dp(out))
    if rc != RLF_OK:
        raise RlfError(rc, "rlf_alpha_from_flux")
    return out


def exported_symbols():
    return sorted(_SIGNATURES)
