// Host runtime behind the C ABI of include/rlf.h: argument validation,
// per-source and per-channel constant tables, facet sizing and buffers,
// kernel launches on the context's stream, HIP-error mapping.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "rlf_objects.h"

using namespace rlf;

namespace {

constexpr double kArcsec = M_PI / 648000.0;     // radians per arcsecond
constexpr double kC = 299792458.0;              // m/s
constexpr int kVersion = 100;                   // 0.1.0
constexpr int kMaxFacetHalf = 16383;            // side*side stays below 2^31
constexpr int kSortedPad = 64;                  // zero-weight tail of the sorted arrays
constexpr int kMaxRefineLevel = 12;             // finest refinement step e_step / 4096
// Bound on the mixed form's ln L error, delta = kRecheckRel (|ln Lmax| +
// kRecheckAbs), used to pick the points its estimator re-evaluates in FP64.
// FP32 terms summed in blocks of 32 cells into FP64 carry a relative error of
// a few ulp of the largest terms; the error measured against the FP64 form
// on the 1000-source SKA-MID-like field is at most 18 * 2^-24 |ln Lmax|, and
// 2^-16 leaves a factor 14 over it.  The offset covers the -ln(M)/2 part of
// ln L (|ln M| / 2 < 64 for any M in e^[-128, 128]).
constexpr double kRecheckRel = 1.0 / 65536.0;
constexpr double kRecheckAbs = 64.0;

}  // namespace

namespace rlf {

int fail(rlf_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(rlf_ctx *c, hipError_t e, const char *what) {
  return fail(c, RLF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace rlf

namespace {

bool is_fin(double x) { return std::isfinite(x); }

int validate_params(const rlf_params *p, std::string &why) {
  if (!p) return why = "params is NULL", RLF_EINVAL;
  if (!is_fin(p->beta) || !(p->ref_freq_hz > 0) || !is_fin(p->ref_freq_hz)) return why = "beta/ref_freq_hz", RLF_EINVAL;
  if (!(p->K > 0) || !is_fin(p->K)) return why = "K must be > 0", RLF_EINVAL;
  if (!is_fin(p->add) || !is_fin(p->esp) || !(p->r_std > 0) || !is_fin(p->r_std)) return why = "add/esp/r_std", RLF_EINVAL;
  if (!(p->rmin_arcsec > 0) || !(p->rmax_arcsec > p->rmin_arcsec) || !is_fin(p->rmax_arcsec))
    return why = "need 0 < rmin < rmax", RLF_EINVAL;
  if (p->num_r < 2 || p->num_r > kMaxKnots) return why = "num_r must be in [2, 32]", RLF_EINVAL;
  if (p->n_e < 3 || p->n_e > 255 || (p->n_e % 2) == 0) return why = "n_e must be odd, in [3, 255]", RLF_EINVAL;
  if (!(p->e_step > 0) || !is_fin(p->e_step)) return why = "e_step must be > 0", RLF_EINVAL;
  const double R = std::nearbyint(1.0 / p->e_step);
  if (R < 1 || std::fabs(R * p->e_step - 1.0) > 1e-9) return why = "1/e_step must be an integer", RLF_EINVAL;
  if (!(p->frac_thresh > 0) || !(p->frac_thresh <= 1)) return why = "frac_thresh must be in (0, 1]", RLF_EINVAL;
  if (!is_fin(p->bad_sigma) || !is_fin(p->bad_sqrtdet)) return why = "bad thresholds", RLF_EINVAL;
  if (p->precision != RLF_FP64 && p->precision != RLF_MIXED) return why = "precision", RLF_EINVAL;
  if (p->reserved != 0) return why = "reserved must be 0", RLF_EINVAL;
  return RLF_OK;
}

// Natural cubic spline through (x_k, y_k): its exact integral over
// [x_0, x_{n-1}] is linear in y; return the weights.  Second derivatives M
// solve h_{i-1} M_{i-1} + 2 (h_{i-1} + h_i) M_i + h_i M_{i+1} = 6 (d_i - d_{i-1})
// (d_i the slope on interval i, M_0 = M_{n-1} = 0, Thomas algorithm), and each
// interval contributes h (y_i + y_{i+1}) / 2 - h^3 (M_i + M_{i+1}) / 24.
std::vector<double> spline_weights(const std::vector<double> &x) {
  const int n = (int)x.size();
  std::vector<double> h(n - 1), w(n, 0.0);
  for (int i = 0; i + 1 < n; ++i) h[i] = x[i + 1] - x[i];
  for (int k = 0; k < n; ++k) {
    std::vector<double> y(n, 0.0), M(n, 0.0);
    y[k] = 1.0;
    const int m = n - 2;
    if (m > 0) {
      std::vector<double> a(m), b(m), c(m), r(m);
      for (int t = 0; t < m; ++t) {
        const int i = t + 1;
        a[t] = h[i - 1];
        b[t] = 2.0 * (h[i - 1] + h[i]);
        c[t] = h[i];
        r[t] = 6.0 * ((y[i + 1] - y[i]) / h[i] - (y[i] - y[i - 1]) / h[i - 1]);
      }
      for (int t = 1; t < m; ++t) {
        const double f = a[t] / b[t - 1];
        b[t] -= f * c[t - 1];
        r[t] -= f * r[t - 1];
      }
      M[m] = r[m - 1] / b[m - 1];
      for (int t = m - 2; t >= 0; --t) M[t + 1] = (r[t] - c[t] * M[t + 2]) / b[t];
    }
    double integral = 0.0;
    for (int i = 0; i + 1 < n; ++i)
      integral += h[i] * (y[i] + y[i + 1]) / 2.0 - h[i] * h[i] * h[i] * (M[i] + M[i + 1]) / 24.0;
    w[k] = integral;
  }
  return w;
}

int check_obs(rlf_ctx *c, const rlf_obs *o) {
  if (!o) return fail(c, RLF_EINVAL, "obs is NULL");
  if (o->n_rows <= 0) return fail(c, RLF_EINVAL, "obs.n_rows must be > 0");
  if (o->n_chan < 1 || o->n_chan > kMaxChan) return fail(c, RLF_EINVAL, "obs.n_chan must be in [1, 64]");
  if (o->reserved != 0) return fail(c, RLF_EINVAL, "obs.reserved must be 0");
  if (!o->u_m || !o->v_m || !o->w_m || !o->freq_hz_host || !o->weight)
    return fail(c, RLF_EINVAL, "obs: NULL array");
  if (o->n_rows > ((int64_t)1 << 40) / o->n_chan) return fail(c, RLF_EINVAL, "obs too large");
  for (int k = 0; k < o->n_chan; ++k)
    if (!(o->freq_hz_host[k] > 0) || !is_fin(o->freq_hz_host[k]))
      return fail(c, RLF_EINVAL, "obs.freq_hz_host must be finite and > 0");
  return RLF_OK;
}

int check_cat(rlf_ctx *c, const rlf_catalog *k, bool need_prior_flux) {
  if (!k) return fail(c, RLF_EINVAL, "catalog is NULL");
  if (k->n_src <= 0 || k->n_src > (1 << 24)) return fail(c, RLF_EINVAL, "catalog.n_src must be in [1, 2^24]");
  if (!k->l || !k->m || !k->flux_jy || !k->alpha_arcsec || !k->e1 || !k->e2)
    return fail(c, RLF_EINVAL, "catalog: NULL array");
  for (int64_t s = 0; s < k->n_src; ++s) {
    const double l = k->l[s], m = k->m[s], e1 = k->e1[s], e2 = k->e2[s];
    if (!is_fin(l) || !is_fin(m) || !(l * l + m * m < 1.0)) return fail(c, RLF_EINVAL, "catalog: need l^2+m^2 < 1");
    if (!is_fin(k->flux_jy[s]) || !(k->flux_jy[s] >= 0.0))
      return fail(c, RLF_EINVAL, "catalog: flux must be finite and >= 0");
    if (need_prior_flux && !k->prior_mu && !(k->flux_jy[s] > 0))
      return fail(c, RLF_EINVAL, "catalog: flux must be > 0 for the Eq. 4 prior (or give prior_mu)");
    if (!(k->alpha_arcsec[s] > 0) || !is_fin(k->alpha_arcsec[s])) return fail(c, RLF_EINVAL, "catalog: alpha must be finite and > 0");
    if (!is_fin(e1) || !is_fin(e2) || !(e1 * e1 + e2 * e2 < 1.0)) return fail(c, RLF_EINVAL, "catalog: need |e| < 1");
    if (k->prior_mu && !is_fin(k->prior_mu[s])) return fail(c, RLF_EINVAL, "catalog: prior_mu must be finite");
  }
  return RLF_OK;
}

SrcModel pack_source(const rlf_params &p, const rlf_catalog *k, int64_t s) {
  SrcModel r{};
  const double l = k->l[s], m = k->m[s];
  const double r2 = l * l + m * m;
  r.l = l;
  r.m = m;
  r.n1 = -r2 / (1.0 + std::sqrt(1.0 - r2));
  r.flux = k->flux_jy[s];
  const double e1 = k->e1[s], e2 = k->e2[s];
  const double det = 1.0 - e1 * e1 - e2 * e2;
  const double a11 = (1.0 + e1) / det, a12 = e2 / det, a22 = (1.0 - e1) / det;
  const double ar = k->alpha_arcsec[s] * kArcsec;
  const double cst = 4.0 * M_PI * M_PI * ar * ar;
  r.q11 = cst * (a11 * a11 + a12 * a12);
  r.q12x2 = 2.0 * cst * a12 * (a11 + a22);
  r.q22 = cst * (a12 * a12 + a22 * a22);
  r.theta = p.K * (k->alpha_arcsec[s] * kArcsec);
  return r;
}

std::vector<double> cat_key(const rlf_catalog *k) {
  std::vector<double> key;
  key.reserve((size_t)k->n_src * 6);
  const double *arr[6] = {k->l, k->m, k->flux_jy, k->alpha_arcsec, k->e1, k->e2};
  for (int a = 0; a < 6; ++a) key.insert(key.end(), arr[a], arr[a] + k->n_src);
  return key;
}

SrcMixed to_mixed(const SrcModel &m) {
  SrcMixed r{};
  r.l = m.l;
  r.m = m.m;
  r.n1 = m.n1;
  r.flux = (float)m.flux;
  r.q11 = (float)m.q11;
  r.q12x2 = (float)m.q12x2;
  r.q22 = (float)m.q22;
  r.theta = m.theta;
  return r;
}

constexpr size_t kPinnedRing = (size_t)8 << 20;   // bytes of the upload staging ring

// Device memory of rlf_model_vis_noalloc: the channel table and the source
// tables of at most kNoAllocMaxSources sources, in one file-scope array per
// device (held until the process ends).  In host code `scratch` names a host
// stand-in: the device address comes from hipGetSymbolAddress, resolved once
// per device with that device current (rlf_create) and used everywhere the
// host passes the array's memory on.
constexpr int64_t kNoAllocMaxSources = 4096;
constexpr size_t kNoAllocChanOff = 0;
constexpr size_t kNoAllocSrcOff = 1024;                                         // >= sizeof(ChanTable)
constexpr size_t kNoAllocSrc32Off = kNoAllocSrcOff + kNoAllocMaxSources * sizeof(SrcModel);
constexpr size_t kNoAllocBytes = kNoAllocSrc32Off + kNoAllocMaxSources * sizeof(SrcMixed);
static_assert(sizeof(ChanTable) <= kNoAllocSrcOff, "channel table does not fit its slot");
static_assert(kNoAllocSrcOff % 256 == 0 && kNoAllocSrc32Off % 256 == 0, "table offsets must stay aligned");

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device `device`, resolved
// on the first call for that device.
int resolve_scratch(rlf_ctx *c, int device) {
  if (device < 0 || device >= kMaxDevices) return fail(c, RLF_EUNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return RLF_OK;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_fail(c, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
  g_scratch_ptr[device] = ptr;
  return RLF_OK;
}

void *scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace

namespace rlf {

int upload_async(rlf_ctx *c, void *dst, const void *src, size_t bytes) {
  if (bytes == 0) return RLF_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCHK(c, hipStreamIsCapturing(c->stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return fail(c, RLF_EINVAL, "table upload while the stream is being captured");
  if (bytes > kPinnedRing / 4) {                      // large tables: a plain copy once the stream is idle
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return RLF_OK;
  }
  if (!c->pinned) {
    void *p = nullptr;
    HIPCHK(c, hipHostMalloc(&p, kPinnedRing, hipHostMallocDefault));
    c->pinned = static_cast<char *>(p);
    c->pinned_off = 0;
  }
  size_t off = (c->pinned_off + 255) & ~(size_t)255;
  if (off + bytes > kPinnedRing) {                    // wrap: every earlier copy must have run
    HIPCHK(c, hipStreamSynchronize(c->stream));
    off = 0;
  }
  std::memcpy(c->pinned + off, src, bytes);
  HIPCHK(c, hipMemcpyAsync(dst, c->pinned + off, bytes, hipMemcpyHostToDevice, c->stream));
  c->pinned_off = off + bytes;
  return RLF_OK;
}

}  // namespace rlf

namespace {

// Source tables of a catalogue, uploaded behind the work already queued on
// the stream (kernels still reading the old tables run first).
int upload_sources(rlf_ctx *c, const rlf_catalog *k, SrcModel *dst, SrcMixed *dst32) {
  std::vector<SrcModel> h((size_t)k->n_src);
  std::vector<SrcMixed> h32((size_t)k->n_src);
  for (int64_t s = 0; s < k->n_src; ++s) {
    h[(size_t)s] = pack_source(c->p, k, s);
    h32[(size_t)s] = to_mixed(h[(size_t)s]);
  }
  if (int e = upload_async(c, dst, h.data(), sizeof(SrcModel) * h.size())) return e;
  return upload_async(c, dst32, h32.data(), sizeof(SrcMixed) * h32.size());
}

// Device source table for rlf_model_vis, reused while the catalogue content is unchanged.
int model_table(rlf_ctx *c, const rlf_catalog *k, const SrcModel **out, const SrcMixed **out32) {
  std::vector<double> key = cat_key(k);
  ++c->tick;
  for (auto &sl : c->slot)
    if (sl.d && sl.key == key) {
      sl.used = c->tick;
      *out = sl.d;
      *out32 = sl.d32;
      return RLF_OK;
    }
  auto &sl = c->slot[0].used <= c->slot[1].used ? c->slot[0] : c->slot[1];
  if (sl.cap < k->n_src) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(sl.d);
    dfree(sl.d32);
    sl.cap = 0;
    if (int e = dalloc(c, &sl.d, k->n_src)) return e;
    if (int e = dalloc(c, &sl.d32, k->n_src)) return e;
    sl.cap = k->n_src;
  }
  sl.key.clear();
  if (int e = upload_sources(c, k, sl.d, sl.d32)) return e;
  sl.key.swap(key);
  sl.used = c->tick;
  *out = sl.d;
  *out32 = sl.d32;
  return RLF_OK;
}

void fill_chan(const rlf_ctx *c, const rlf_obs *o, ChanTable &h) {
  h = ChanTable{};
  for (int k = 0; k < o->n_chan; ++k) {
    h.scale[k] = o->freq_hz_host[k] / kC;
    h.spec[k] = std::pow(o->freq_hz_host[k] / c->p.ref_freq_hz, c->p.beta);
  }
}

int chan_table(rlf_ctx *c, const rlf_obs *o) {
  std::vector<double> key(o->freq_hz_host, o->freq_hz_host + o->n_chan);
  if (c->d_chan && key == c->chan_key) return RLF_OK;
  ChanTable h{};
  fill_chan(c, o, h);
  if (!c->d_chan)
    if (int e = dalloc(c, &c->d_chan, 1)) return e;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->d_chan, &h, sizeof(h), hipMemcpyHostToDevice));
  c->chan_key.swap(key);
  return RLF_OK;
}

int set_device(rlf_ctx *c) {
  HIPCHK(c, hipSetDevice(c->device));
  return RLF_OK;
}

void free_facets(rlf_facets *f) {
  dfree(f->d_src);
  dfree(f->d_src32);
  if (f->owns_sorted) {
    dfree(f->sv.order);
    dfree(f->sv.geo);
    dfree(f->sv.wt);
    if (f->sv.quad) (void)hipFree(f->sv.quad);
    if (f->sv.res) (void)hipFree(f->sv.res);
  }
  f->sv = Sorted{};
  dfree(f->d_geom);
  dfree(f->d_order);
  dfree(f->acc.cell);
  dfree(f->cells.offsets);
  dfree(f->cells.n_nonempty);
  dfree(f->cells.ix);
  dfree(f->cells.iy);
  dfree(f->cells.count);
  dfree(f->cells.wsum);
  dfree(f->cells.vre);
  dfree(f->cells.vim);
  dfree(f->cells.fit64);
  dfree(f->cells.fit32);
  dfree(f->d_logw);
  dfree(f->d_lsurf);
  dfree(f->d_redo);
  dfree(f->d_win);
  dfree(f->d_refine_win);
  dfree(f->d_refine_l);
  if (f->d_pos_g) (void)hipFree(f->d_pos_g);
  f->d_pos_g = nullptr;
}

int check_device_error(rlf_ctx *c) {
  uint32_t e = 0;
  HIPCHK(c, hipMemcpy(&e, c->d_err, sizeof(e), hipMemcpyDeviceToHost));
  if (e) {
    uint32_t z = 0;
    HIPCHK(c, hipMemcpy(c->d_err, &z, sizeof(z), hipMemcpyHostToDevice));
    return fail(c, RLF_ERANGE, "a visibility fell outside its facet: the observation's uvw changed after rlf_facets_create");
  }
  return RLF_OK;
}

int build_sorted(rlf_ctx *c, const rlf_obs *obs, const double mx[2], rlf_facets *f) {
  const int64_t n = obs->n_rows * obs->n_chan;
  if (n >= ((int64_t)1 << 32)) return fail(c, RLF_ERANGE, "more than 2^32 - 1 visibilities");
  if (int e = chan_table(c, obs)) return e;
  Sorted &sv = f->sv;
  sv.n_vis = n;
  const size_t esz = f->mixed ? 4 : 8;
  // the extraction reads visibilities in groups: pad every array read there,
  // with zero weight (skipped) and zero coordinates in the padding
  const int64_t np = n + kSortedPad;
  if (int e = dalloc(c, &sv.order, n)) return e;
  if (int e = dalloc(c, &sv.geo, np)) return e;
  if (int e = dalloc(c, &sv.wt, np)) return e;
  HIPCHK(c, hipMalloc(&sv.quad, 4 * esz * (size_t)np));
  HIPCHK(c, hipMalloc(&sv.res, 2 * esz * (size_t)np));
  HIPCHK(c, hipMemset(sv.geo, 0, sizeof(double4) * (size_t)np));
  HIPCHK(c, hipMemset(sv.wt, 0, sizeof(double) * (size_t)np));
  HIPCHK(c, hipMemset(sv.quad, 0, 4 * esz * (size_t)np));
  HIPCHK(c, hipMemset(sv.res, 0, 2 * esz * (size_t)np));
  double smax = 0.0;
  for (int k = 0; k < obs->n_chan; ++k) smax = std::fmax(smax, obs->freq_hz_host[k] / kC);
  const double su = mx[0] * smax, svv = mx[1] * smax;
  uint32_t *kin = nullptr, *vin = nullptr, *kout = nullptr;
  void *tmp = nullptr;
  int rc = RLF_OK;
  do {
    if ((rc = dalloc(c, &kin, n))) break;
    if ((rc = dalloc(c, &vin, n))) break;
    if ((rc = dalloc(c, &kout, n))) break;
    SortKeyArgs ka{};
    ka.u_m = obs->u_m;
    ka.v_m = obs->v_m;
    ka.n_rows = obs->n_rows;
    ka.n_chan = obs->n_chan;
    ka.chan = c->d_chan;
    ka.inv_span_u = su > 0 ? 1.0 / (2.0 * su) : 1.0;
    ka.inv_span_v = svv > 0 ? 1.0 / (2.0 * svv) : 1.0;
    ka.keys = kin;
    ka.vals = vin;
    hipError_t e = launch_sort_keys(ka, c->stream);
    size_t tmp_bytes = 0;
    if (e == hipSuccess) e = sort_pairs_u32(nullptr, tmp_bytes, kin, kout, vin, sv.order, n, c->stream);
    if (e == hipSuccess) e = hipMalloc(&tmp, tmp_bytes ? tmp_bytes : 1);
    if (e == hipSuccess) e = sort_pairs_u32(tmp, tmp_bytes, kin, kout, vin, sv.order, n, c->stream);
    if (e == hipSuccess)
      e = launch_sorted_static(sv, obs->u_m, obs->v_m, obs->w_m, obs->n_chan, c->d_chan, f->mixed, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = hip_fail(c, e, "uv sort of the visibilities");
  } while (0);
  dfree(kin);
  dfree(vin);
  dfree(kout);
  if (tmp) (void)hipFree(tmp);
  return rc;
}

}  // namespace

extern "C" {

int rlf_version(void) { return kVersion; }

int rlf_params_default(rlf_params *p) {
  if (!p) return RLF_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->beta = -0.7;
  p->ref_freq_hz = 1.4e9;
  p->K = 38.0;
  p->add = -0.93;
  p->esp = 0.33;
  p->r_std = 0.3136;
  p->rmin_arcsec = 0.3;
  p->rmax_arcsec = 3.5;
  p->num_r = 20;
  p->n_e = 81;
  p->e_step = 0.02;
  p->frac_thresh = 0.05;
  p->bad_sigma = 5e-3;
  p->bad_sqrtdet = 5e-5;
  p->precision = RLF_FP64;
  p->reserved = 0;
  return RLF_OK;
}

int rlf_create(rlf_ctx **out, int device, void *hip_stream, const rlf_params *p) {
  if (!out) return RLF_EINVAL;
  std::string why;
  if (validate_params(p, why) != RLF_OK) return RLF_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return device < 0 ? RLF_EINVAL : RLF_EDEVICE;
  }
  rlf_ctx *c = new (std::nothrow) rlf_ctx();
  if (!c) return RLF_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->p = *p;
  int rc = RLF_OK;
  do {
    if ((rc = set_device(c))) break;
    // ellipticity grid: valid points (|e| < 1 on the integers), increasing flat index
    const int R = (int)std::nearbyint(1.0 / p->e_step);
    const int ctr = (p->n_e - 1) / 2;
    c->half_r2 = R * R;
    std::vector<int32_t> ep;
    for (int i1 = 0; i1 < p->n_e; ++i1)
      for (int i2 = 0; i2 < p->n_e; ++i2)
        if ((i1 - ctr) * (i1 - ctr) + (i2 - ctr) * (i2 - ctr) < c->half_r2) ep.push_back(i1 * p->n_e + i2);
    c->n_valid = (int)ep.size();
    std::vector<int32_t> vidx((size_t)p->n_e * p->n_e, -1);
    for (size_t j = 0; j < ep.size(); ++j) vidx[(size_t)ep[j]] = (int32_t)j;
    if ((rc = dalloc(c, &c->d_epts, c->n_valid))) break;
    if ((rc = dalloc(c, &c->d_vidx, (int64_t)vidx.size()))) break;
    if (hipMemcpy(c->d_epts, ep.data(), sizeof(int32_t) * ep.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_vidx, vidx.data(), sizeof(int32_t) * vidx.size(), hipMemcpyHostToDevice) != hipSuccess) {
      rc = RLF_EDEVICE;
      break;
    }
    // knots alpha_k = rmin + (rmax - rmin) (k / (n-1))^2 and s_k = 4 pi^2 alpha_k^2
    c->knots.resize(p->num_r);
    std::vector<double> sk(p->num_r);
    for (int k = 0; k < p->num_r; ++k) {
      const double t = (double)k / (double)(p->num_r - 1);
      c->knots[k] = p->rmin_arcsec + (p->rmax_arcsec - p->rmin_arcsec) * t * t;
      const double ar = c->knots[k] * kArcsec;
      sk[k] = 4.0 * M_PI * M_PI * ar * ar;
    }
    c->ck = spline_weights(c->knots);
    if ((rc = dalloc(c, &c->d_sk, p->num_r))) break;
    if (hipMemcpy(c->d_sk, sk.data(), sizeof(double) * sk.size(), hipMemcpyHostToDevice) != hipSuccess) {
      rc = RLF_EDEVICE;
      break;
    }
    if ((rc = dalloc(c, &c->d_err, 1))) break;
    if ((rc = dalloc(c, &c->d_absmax, 2))) break;
    if (hipMemset(c->d_err, 0, sizeof(uint32_t)) != hipSuccess) {
      rc = RLF_EDEVICE;
      break;
    }
    // rlf_model_vis_noalloc: the device's scratch address and a host staging
    // buffer of the same size, made here so that the entry point allocates nothing
    if ((rc = resolve_scratch(c, device))) break;
    try {
      c->noalloc_stage.resize(kNoAllocBytes);
    } catch (...) {
      rc = RLF_ENOMEM;
      break;
    }
  } while (0);
  if (rc != RLF_OK) {
    rlf_destroy(c);
    return rc;
  }
  *out = c;
  return RLF_OK;
}

int rlf_destroy(rlf_ctx *c) {
  if (!c) return RLF_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  dfree(c->d_epts);
  dfree(c->d_vidx);
  dfree(c->d_sk);
  dfree(c->d_chan);
  dfree(c->d_err);
  dfree(c->d_absmax);
  dfree(c->d_part);
  if (c->pinned) (void)hipHostFree(c->pinned);
  c->pinned = nullptr;
  for (auto &sl : c->slot) {
    dfree(sl.d);
    dfree(sl.d32);
  }
  delete c;
  return RLF_OK;
}

int rlf_set_stream(rlf_ctx *c, void *hip_stream) {
  if (!c) return RLF_EINVAL;
  if (int e = set_device(c)) return e;
  // uploads staged for the old stream must have run before the ring is reused
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->stream = (hipStream_t)hip_stream;
  return RLF_OK;
}

int rlf_sync(rlf_ctx *c) {
  if (!c) return RLF_EINVAL;
  if (int e = set_device(c)) return e;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return check_device_error(c);
}

const char *rlf_last_error(const rlf_ctx *c) { return c ? c->err.c_str() : "context is NULL"; }

int rlf_alpha_from_flux(const double *flux, int64_t n, double add, double esp, double *alpha) {
  if (!flux || !alpha || n <= 0 || !is_fin(add) || !is_fin(esp)) return RLF_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    if (!(flux[i] > 0) || !is_fin(flux[i])) return RLF_EINVAL;
  for (int64_t i = 0; i < n; ++i) alpha[i] = std::exp(add + esp * std::log(flux[i] * 1e6));
  return RLF_OK;
}

int rlf_model_vis(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, int64_t src_begin,
                  int64_t src_end, void *out, int mode) {
  if (!c) return RLF_EINVAL;
  c->err.clear();
  if (int e = check_obs(c, obs)) return e;
  if (int e = check_cat(c, cat, false)) return e;
  if (!out) return fail(c, RLF_EINVAL, "out is NULL");
  if (mode < 0 || mode > 2) return fail(c, RLF_EINVAL, "mode");
  if (mode == RLF_MODEL_RESIDUAL && !obs->vis) return fail(c, RLF_EINVAL, "obs.vis is NULL");
  if (src_begin < 0 || src_end > cat->n_src || src_begin > src_end) return fail(c, RLF_EINVAL, "source range");
  if (int e = set_device(c)) return e;
  if (int e = chan_table(c, obs)) return e;
  const SrcModel *d_src = nullptr;
  const SrcMixed *d_src32 = nullptr;
  if (int e = model_table(c, cat, &d_src, &d_src32)) return e;
  ModelArgs a{};
  a.u_m = obs->u_m;
  a.v_m = obs->v_m;
  a.w_m = obs->w_m;
  a.n_rows = obs->n_rows;
  a.n_chan = obs->n_chan;
  a.mode = mode;
  a.chan = c->d_chan;
  a.src = d_src;
  a.src32 = d_src32;
  a.s_begin = (int32_t)src_begin;
  a.s_end = (int32_t)src_end;
  a.vis_in = obs->vis;
  a.out = out;
  hipError_t e = launch_model(a, c->p.precision == RLF_MIXED, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "model kernel launch");
  return RLF_OK;
}

int rlf_model_vis_noalloc(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, int64_t src_begin,
                          int64_t src_end, void *out, int mode) {
  if (!c) return RLF_EINVAL;
  c->err.clear();
  if (int e = check_obs(c, obs)) return e;
  if (int e = check_cat(c, cat, false)) return e;
  if (!out) return fail(c, RLF_EINVAL, "out is NULL");
  if (mode < 0 || mode > 2) return fail(c, RLF_EINVAL, "mode");
  if (mode == RLF_MODEL_RESIDUAL && !obs->vis) return fail(c, RLF_EINVAL, "obs.vis is NULL");
  if (src_begin < 0 || src_end > cat->n_src || src_begin > src_end) return fail(c, RLF_EINVAL, "source range");
  const int64_t n = src_end - src_begin;
  if (n > kNoAllocMaxSources)
    return fail(c, RLF_EINVAL, "rlf_model_vis_noalloc: at most 4096 sources per call (its fixed scratch size)");
  char *ptr = static_cast<char *>(scratch_ptr(c->device));
  if (!ptr || c->noalloc_stage.size() < kNoAllocBytes)
    return fail(c, RLF_EDEVICE, "rlf_model_vis_noalloc: scratch not resolved for this device");
  if (int e = set_device(c)) return e;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCHK(c, hipStreamIsCapturing(c->stream, &cs));
  if (cs != hipStreamCaptureStatusNone)
    return fail(c, RLF_EUNSUPPORTED, "rlf_model_vis_noalloc copies its tables from host memory: not under capture");
  // the previous call's copy and kernels on this stream read the same
  // scratch and staging memory: let them finish first
  HIPCHK(c, hipStreamSynchronize(c->stream));
  unsigned char *h = c->noalloc_stage.data();
  ChanTable ch{};
  fill_chan(c, obs, ch);
  std::memcpy(h + kNoAllocChanOff, &ch, sizeof ch);
  SrcModel *hs = reinterpret_cast<SrcModel *>(h + kNoAllocSrcOff);
  SrcMixed *hs32 = reinterpret_cast<SrcMixed *>(h + kNoAllocSrc32Off);
  for (int64_t s = 0; s < n; ++s) {
    hs[s] = pack_source(c->p, cat, src_begin + s);
    hs32[s] = to_mixed(hs[s]);
  }
  HIPCHK(c, hipMemcpyAsync(ptr + kNoAllocChanOff, h + kNoAllocChanOff, sizeof(ChanTable), hipMemcpyHostToDevice,
                           c->stream));
  if (n > 0) {
    HIPCHK(c, hipMemcpyAsync(ptr + kNoAllocSrcOff, hs, sizeof(SrcModel) * (size_t)n, hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(ptr + kNoAllocSrc32Off, hs32, sizeof(SrcMixed) * (size_t)n, hipMemcpyHostToDevice,
                             c->stream));
  }
  ModelArgs a{};
  a.u_m = obs->u_m;
  a.v_m = obs->v_m;
  a.w_m = obs->w_m;
  a.n_rows = obs->n_rows;
  a.n_chan = obs->n_chan;
  a.mode = mode;
  a.chan = reinterpret_cast<const ChanTable *>(ptr + kNoAllocChanOff);
  a.src = reinterpret_cast<const SrcModel *>(ptr + kNoAllocSrcOff);
  a.src32 = reinterpret_cast<const SrcMixed *>(ptr + kNoAllocSrc32Off);
  a.s_begin = 0;
  a.s_end = (int32_t)n;
  a.vis_in = obs->vis;
  a.out = out;
  hipError_t e = launch_model(a, c->p.precision == RLF_MIXED, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "model kernel launch");
  return RLF_OK;
}

}  // extern "C"

namespace rlf {

// Per-source facet geometry: theta = K alpha, the half-size bounding every
// rint(u theta) of the observation (largest |u|, |v| in metres `mx`), and
// each source's dense block of (2 half + 1)^2 cells.
int facet_geometry(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, const double mx[2],
                   std::vector<double> &theta, std::vector<SrcGeom> &geom, int64_t &total) {
  theta.resize((size_t)cat->n_src);
  geom.resize((size_t)cat->n_src);
  total = 0;
  for (int64_t s = 0; s < cat->n_src; ++s) {
    const double th = c->p.K * (cat->alpha_arcsec[s] * kArcsec);
    int64_t half = 0;
    for (int k = 0; k < obs->n_chan; ++k) {
      const double sc = obs->freq_hz_host[k] / kC;
      const double tu = std::nearbyint((mx[0] * sc) * th), tv = std::nearbyint((mx[1] * sc) * th);
      const double t = tu > tv ? tu : tv;
      if (!(t <= (double)kMaxFacetHalf))
        return fail(c, RLF_ERANGE, "facet half-size exceeds 16383 cells (alpha * K too large for the uv extent)");
      half = (int64_t)t > half ? (int64_t)t : half;
    }
    theta[(size_t)s] = th;
    geom[(size_t)s].base = total;
    geom[(size_t)s].half = (int32_t)half;
    geom[(size_t)s].side = (int32_t)(2 * half + 1);
    total += (2 * half + 1) * (2 * half + 1);
  }
  return RLF_OK;
}

// Scale-marginalisation weights ln(c_k) + ln p_s(alpha_k) (log-normal prior)
// [n_src * num_r].
std::vector<double> facet_logw(rlf_ctx *c, const rlf_catalog *cat) {
  const int R = c->p.num_r;
  std::vector<double> logw((size_t)cat->n_src * R);
  for (int64_t s = 0; s < cat->n_src; ++s) {
    const double mu = cat->prior_mu ? cat->prior_mu[s] : c->p.add + c->p.esp * std::log(cat->flux_jy[s] * 1e6);
    for (int k = 0; k < R; ++k) {
      const double a = c->knots[k];
      const double z = std::log(a) - mu;
      const double lp = -z * z / (2.0 * c->p.r_std * c->p.r_std) - std::log(a * c->p.r_std * std::sqrt(2.0 * M_PI));
      logw[(size_t)s * R + k] = std::log(c->ck[k]) + lp;
    }
  }
  return logw;
}

// Extraction lanes take the sources in order of cell size: cell boundaries
// (rint(u theta)) of neighbouring lanes then nearly coincide, so their cell
// changes come at nearly the same visibilities and the branches of a wave
// diverge less.
std::vector<int32_t> lane_order(const std::vector<double> &theta) {
  std::vector<int32_t> order(theta.size());
  for (size_t s = 0; s < theta.size(); ++s) order[s] = (int32_t)s;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return theta[(size_t)x] < theta[(size_t)y]; });
  return order;
}

// A facet object for `cat`; with `share`, the uv-sorted layout of `share`
// (made for the same observation) is borrowed instead of sorted again.
int create_facets(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, const rlf_facets *share,
                  rlf_facets **out) {
  if (!out) return fail(c, RLF_EINVAL, "out is NULL");
  if (int e = check_obs(c, obs)) return e;
  if (int e = check_cat(c, cat, true)) return e;
  if (int e = set_device(c)) return e;
  double mx[2] = {0.0, 0.0};
  if (share) {
    mx[0] = share->mx[0];
    mx[1] = share->mx[1];
  } else {
    // largest |u|, |v| (metres) bound every cell index
    HIPCHK(c, hipMemsetAsync(c->d_absmax, 0, 2 * sizeof(double), c->stream));
    HIPCHK(c, launch_absmax(obs->u_m, obs->n_rows, c->d_absmax, 0, c->stream));
    HIPCHK(c, launch_absmax(obs->v_m, obs->n_rows, c->d_absmax, 1, c->stream));
    HIPCHK(c, hipMemcpyAsync(mx, c->d_absmax, sizeof(mx), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!is_fin(mx[0]) || !is_fin(mx[1])) return fail(c, RLF_EINVAL, "obs: non-finite u or v");
  }

  rlf_facets *f = new (std::nothrow) rlf_facets();
  if (!f) return fail(c, RLF_ENOMEM, "host allocation");
  f->ctx = c;
  f->mx[0] = mx[0];
  f->mx[1] = mx[1];
  f->n_src = cat->n_src;
  f->mixed = c->p.precision == RLF_MIXED;
  {
    double g = 0.0;
    for (int32_t k = 0; k < obs->n_chan; ++k) g += std::pow(obs->freq_hz_host[k] / c->p.ref_freq_hz, c->p.beta);
    f->spec_norm = g / obs->n_chan;
  }
  f->alpha.assign(cat->alpha_arcsec, cat->alpha_arcsec + cat->n_src);
  int64_t total = 0;
  if (int e = facet_geometry(c, obs, cat, mx, f->theta, f->geom, total)) {
    delete f;
    return e;
  }
  f->dense_total = total;
  f->dense_cap = total;
  const std::vector<double> logw = facet_logw(c, cat);
  int rc = RLF_OK;
  do {
    if ((rc = dalloc(c, &f->d_src, f->n_src))) break;
    if ((rc = dalloc(c, &f->d_src32, f->n_src))) break;
    if ((rc = dalloc(c, &f->d_geom, f->n_src))) break;
    if ((rc = dalloc(c, &f->d_order, f->n_src))) break;
    if ((rc = dalloc(c, &f->acc.cell, total))) break;
    if ((rc = dalloc(c, &f->cells.offsets, f->n_src + 1))) break;
    if ((rc = dalloc(c, &f->cells.n_nonempty, f->n_src))) break;
    if ((rc = dalloc(c, &f->cells.ix, total))) break;
    if ((rc = dalloc(c, &f->cells.iy, total))) break;
    if ((rc = dalloc(c, &f->cells.count, total))) break;
    if ((rc = dalloc(c, &f->cells.wsum, total))) break;
    if ((rc = dalloc(c, &f->cells.vre, total))) break;
    if ((rc = dalloc(c, &f->cells.vim, total))) break;
    if (f->mixed && (rc = dalloc(c, &f->cells.fit32, total))) break;
    if ((rc = dalloc(c, &f->cells.fit64, total))) break;
    if ((rc = dalloc(c, &f->d_logw, f->n_src * c->p.num_r))) break;
    if ((rc = dalloc(c, &f->d_lsurf, f->n_src * (int64_t)c->n_valid))) break;
    if ((rc = dalloc(c, &f->d_redo, f->n_src))) break;
    if ((rc = dalloc(c, &f->d_win, f->n_src * 4))) break;
  } while (0);
  if (rc != RLF_OK) {
    free_facets(f);
    delete f;
    return rc;
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(f->d_geom, f->geom.data(), sizeof(SrcGeom) * f->geom.size(), hipMemcpyHostToDevice);
  const std::vector<int32_t> order = lane_order(f->theta);
  if (e == hipSuccess) e = hipMemcpy(f->d_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(f->d_logw, logw.data(), sizeof(double) * logw.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(f->acc.cell, 0, sizeof(double4) * (size_t)total);
  if (e == hipSuccess) e = hipMemset(f->cells.offsets, 0, sizeof(int64_t) * (size_t)(f->n_src + 1));
  if (e == hipSuccess) e = hipMemset(f->d_redo, 0, sizeof(int32_t) * (size_t)f->n_src);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_facets(f);
    delete f;
    return hip_fail(c, e, "facet buffer initialisation");
  }
  if (int r = upload_sources(c, cat, f->d_src, f->d_src32)) {
    free_facets(f);
    delete f;
    return r;
  }
  f->model_key = cat_key(cat);
  if (share) {
    if (int e = chan_table(c, obs)) {
      free_facets(f);
      delete f;
      return e;
    }
    f->sv = share->sv;
    f->owns_sorted = false;
  } else if (int r = build_sorted(c, obs, mx, f)) {
    free_facets(f);
    delete f;
    return r;
  }
  *out = f;
  return RLF_OK;
}

// Point an existing facet object at another catalogue of as many sources
// (same observation): new geometry, weights, lane order and model table;
// the dense arrays are reused while they are large enough, the uv-sorted
// layout (owned or borrowed) is kept, and positions go back to fixed.
int retarget_facets(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, rlf_facets *f) {
  if (!f || f->ctx != c) return fail(c, RLF_EINVAL, "facets is NULL or from another context");
  if (int e = check_obs(c, obs)) return e;
  if (int e = check_cat(c, cat, true)) return e;
  if (cat->n_src != f->n_src) return fail(c, RLF_EINVAL, "retarget: source count differs");
  if (int e = set_device(c)) return e;
  std::vector<double> theta;
  std::vector<SrcGeom> geom;
  int64_t total = 0;
  if (int e = facet_geometry(c, obs, cat, f->mx, theta, geom, total)) return e;
  if (total > f->dense_cap) {
    HIPCHK(c, hipStreamSynchronize(c->stream));        // queued kernels may still use the arrays
    dfree(f->acc.cell);
    dfree(f->cells.ix);
    dfree(f->cells.iy);
    dfree(f->cells.count);
    dfree(f->cells.wsum);
    dfree(f->cells.vre);
    dfree(f->cells.vim);
    dfree(f->cells.fit64);
    dfree(f->cells.fit32);
    if (f->d_pos_g) (void)hipFree(f->d_pos_g);
    f->d_pos_g = nullptr;
    f->pos_cap = 0;
    f->dense_cap = 0;
    f->dense_total = 0;
    int rc = RLF_OK;
    do {
      if ((rc = dalloc(c, &f->acc.cell, total))) break;
      if ((rc = dalloc(c, &f->cells.ix, total))) break;
      if ((rc = dalloc(c, &f->cells.iy, total))) break;
      if ((rc = dalloc(c, &f->cells.count, total))) break;
      if ((rc = dalloc(c, &f->cells.wsum, total))) break;
      if ((rc = dalloc(c, &f->cells.vre, total))) break;
      if ((rc = dalloc(c, &f->cells.vim, total))) break;
      if (f->mixed && (rc = dalloc(c, &f->cells.fit32, total))) break;
      if ((rc = dalloc(c, &f->cells.fit64, total))) break;
    } while (0);
    if (rc != RLF_OK) return rc;                       // the object stays unusable until freed
    f->dense_cap = total;
  }
  const std::vector<double> logw = facet_logw(c, cat);
  const std::vector<int32_t> order = lane_order(theta);
  // everything below is queued behind the work already on the stream
  if (int e = upload_async(c, f->d_geom, geom.data(), sizeof(SrcGeom) * geom.size())) return e;
  if (int e = upload_async(c, f->d_order, order.data(), sizeof(int32_t) * order.size())) return e;
  if (int e = upload_async(c, f->d_logw, logw.data(), sizeof(double) * logw.size())) return e;
  HIPCHK(c, hipMemsetAsync(f->acc.cell, 0, sizeof(double4) * (size_t)total, c->stream));
  HIPCHK(c, hipMemsetAsync(f->cells.offsets, 0, sizeof(int64_t) * (size_t)(f->n_src + 1), c->stream));
  HIPCHK(c, hipMemsetAsync(f->d_redo, 0, sizeof(int32_t) * (size_t)f->n_src, c->stream));
  if (int e = upload_sources(c, cat, f->d_src, f->d_src32)) return e;
  f->model_key = cat_key(cat);
  f->alpha.assign(cat->alpha_arcsec, cat->alpha_arcsec + cat->n_src);
  f->theta.swap(theta);
  f->geom.swap(geom);
  f->dense_total = total;
  f->pos_side = 1;
  f->pos_step = 0.0;
  return RLF_OK;
}

// Gather (or subtract the facet object's own catalogue from) the visibilities
// into the sorted layout, then extract and compact; `vis` NULL: the sorted
// layout already holds the residual (kept there by the caller), no gather.
int extract_facets(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, const void *vis, int subtract,
                   rlf_facets *f, const UpdateArgs *upd) {
  if (!f || f->ctx != c) return fail(c, RLF_EINVAL, "facets is NULL or from another context");
  if (int e = check_obs(c, obs)) return e;
  if (obs->n_rows * obs->n_chan != f->sv.n_vis) return fail(c, RLF_EINVAL, "observation size differs from rlf_facets_create");
  if (int e = check_cat(c, cat, false)) return e;
  if (cat->n_src != f->n_src || std::memcmp(cat->alpha_arcsec, f->alpha.data(), sizeof(double) * f->n_src) != 0)
    return fail(c, RLF_EINVAL, "catalogue sources/sizes differ from rlf_facets_create");
  if (int e = set_device(c)) return e;
  if (int e = chan_table(c, obs)) return e;
  std::vector<double> key = cat_key(cat);
  if (key != f->model_key) {
    if (int e = upload_sources(c, cat, f->d_src, f->d_src32)) return e;
    f->model_key.swap(key);
  }
  hipError_t e = hipSuccess;
  if (vis && upd) return fail(c, RLF_EINVAL, "a residual update applies to the kept sorted residual only");
  if (vis) {
    ResidualArgs ra{};
    ra.sv = f->sv;
    ra.n_chan = obs->n_chan;
    ra.n_src = (int32_t)f->n_src;
    ra.chan = c->d_chan;
    ra.src = f->d_src;
    ra.src32 = f->d_src32;
    ra.vis = vis;
    ra.weight = obs->weight;
    ra.subtract = subtract;
    e = launch_residual_sorted(ra, f->mixed, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "residual kernel launch");
  }
  ExtractArgs a{};
  a.sv = f->sv;
  a.n_chan = obs->n_chan;
  a.n_src = (int32_t)f->n_src;
  a.n_tiles = (int32_t)((f->n_src + 63) / 64);
  // chunk and n_chunks: chosen by the launcher from the device's occupancy
  a.chan = c->d_chan;
  a.src = f->d_src;
  a.src32 = f->d_src32;
  a.geom = f->d_geom;
  a.order = f->d_order;
  a.acc = f->acc;
  a.err = c->d_err;
  e = launch_extract(a, f->mixed, c->stream, upd);
  if (e != hipSuccess) return hip_fail(c, e, "extract kernel launch");
  CompactArgs ca{};
  ca.n_src = (int32_t)f->n_src;
  ca.geom = f->d_geom;
  ca.src = f->d_src;
  ca.acc = f->acc;
  ca.cells = f->cells;
  e = launch_compact(ca, f->mixed, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "compact kernel launch");
  return RLF_OK;
}

// Residual of the sky catalogue `sky` (obs.vis minus its models) into the
// sorted layout of f, with the unweighted FP64 residual in `rs` as well.
int sorted_residual(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *sky, const rlf_facets *f, double2 *rs) {
  if (int e = check_obs(c, obs)) return e;
  if (!obs->vis) return fail(c, RLF_EINVAL, "obs.vis is NULL");
  if (obs->n_rows * obs->n_chan != f->sv.n_vis) return fail(c, RLF_EINVAL, "observation size differs");
  if (int e = check_cat(c, sky, false)) return e;
  if (!f->mixed && !rs) return fail(c, RLF_EINVAL, "FP64 form needs the unweighted residual buffer");
  if (int e = set_device(c)) return e;
  if (int e = chan_table(c, obs)) return e;
  const SrcModel *d_src = nullptr;
  const SrcMixed *d_src32 = nullptr;
  if (int e = model_table(c, sky, &d_src, &d_src32)) return e;
  ResidualArgs ra{};
  ra.sv = f->sv;
  ra.n_chan = obs->n_chan;
  ra.n_src = (int32_t)sky->n_src;
  ra.chan = c->d_chan;
  ra.src = d_src;
  ra.src32 = d_src32;
  ra.vis = obs->vis;
  ra.weight = obs->weight;
  ra.subtract = 1;
  ra.rs = f->mixed ? nullptr : rs;
  hipError_t e = launch_residual_sorted(ra, f->mixed, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "residual kernel launch");
  return RLF_OK;
}

// Arguments of R += (models of old_m) - (models of new_m) on the residual
// kept in the sorted layout of f (and in rs for the FP64 form); the two
// model tables are uploaded into the context's two model slots.
int prepare_update(rlf_ctx *c, const rlf_catalog *old_m, const rlf_catalog *new_m, const rlf_facets *f,
                   double2 *rs, UpdateArgs &u) {
  if (int e = check_cat(c, old_m, false)) return e;
  if (int e = check_cat(c, new_m, false)) return e;
  if (!f->mixed && !rs) return fail(c, RLF_EINVAL, "FP64 form needs the unweighted residual buffer");
  if (int e = set_device(c)) return e;
  u = UpdateArgs{};
  // the second lookup replaces the least recently used slot, never the one
  // just returned
  if (int e = model_table(c, old_m, &u.old64, &u.old32)) return e;
  if (int e = model_table(c, new_m, &u.new64, &u.new32)) return e;
  if (u.old64 == u.new64 && cat_key(old_m) != cat_key(new_m))
    return fail(c, RLF_EINVAL, "model tables of the update share a slot");
  u.sv = f->sv;
  u.n_old = (int32_t)old_m->n_src;
  u.n_new = (int32_t)new_m->n_src;
  u.rs = f->mixed ? nullptr : rs;
  return RLF_OK;
}

int update_sorted_residual(rlf_ctx *c, const UpdateArgs &u, int mixed) {
  hipError_t e = launch_update_sorted(u, mixed, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "residual update kernel launch");
  return RLF_OK;
}

}  // namespace rlf

extern "C" {

int rlf_facets_create(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, rlf_facets **out) {
  if (!c) return RLF_EINVAL;
  c->err.clear();
  return create_facets(c, obs, cat, nullptr, out);
}

int rlf_extract_facets(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, const void *residual,
                       rlf_facets *f) {
  if (!c) return RLF_EINVAL;
  c->err.clear();
  if (!residual && (!obs || !obs->vis)) return fail(c, RLF_EINVAL, "residual and obs.vis are both NULL");
  return extract_facets(c, obs, cat, residual ? residual : obs->vis, residual ? 0 : 1, f);
}

int rlf_facets_info(rlf_ctx *c, const rlf_facets *f, int64_t *n_src, int64_t *n_cells, int64_t *n_dense) {
  if (!c) return RLF_EINVAL;
  if (!f || f->ctx != c) return fail(c, RLF_EINVAL, "facets");
  if (n_src) *n_src = f->n_src;
  if (n_dense) *n_dense = f->dense_total;
  if (n_cells) {
    if (int e = set_device(c)) return e;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(n_cells, f->cells.offsets + f->n_src, sizeof(int64_t), hipMemcpyDeviceToHost));
    return check_device_error(c);
  }
  return RLF_OK;
}

int rlf_facets_copy(rlf_ctx *c, const rlf_facets *f, int64_t *offsets, int32_t *ix, int32_t *iy,
                    int32_t *count, double *wsum, double *vbar, double *theta) {
  if (!c) return RLF_EINVAL;
  if (!f || f->ctx != c) return fail(c, RLF_EINVAL, "facets");
  if (int e = set_device(c)) return e;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (int e = check_device_error(c)) return e;
  int64_t n = 0;
  HIPCHK(c, hipMemcpy(&n, f->cells.offsets + f->n_src, sizeof(int64_t), hipMemcpyDeviceToHost));
  if (offsets) HIPCHK(c, hipMemcpy(offsets, f->cells.offsets, sizeof(int64_t) * (f->n_src + 1), hipMemcpyDeviceToHost));
  if (ix) HIPCHK(c, hipMemcpy(ix, f->cells.ix, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  if (iy) HIPCHK(c, hipMemcpy(iy, f->cells.iy, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  if (count) HIPCHK(c, hipMemcpy(count, f->cells.count, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  if (wsum) HIPCHK(c, hipMemcpy(wsum, f->cells.wsum, sizeof(double) * n, hipMemcpyDeviceToHost));
  if (vbar) {
    std::vector<double> re((size_t)n), im((size_t)n);
    HIPCHK(c, hipMemcpy(re.data(), f->cells.vre, sizeof(double) * n, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(im.data(), f->cells.vim, sizeof(double) * n, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < n; ++k) {
      vbar[2 * k] = re[(size_t)k];
      vbar[2 * k + 1] = im[(size_t)k];
    }
  }
  if (theta) std::memcpy(theta, f->theta.data(), sizeof(double) * f->n_src);
  return RLF_OK;
}

int rlf_facets_free(rlf_facets *f) {
  if (!f) return RLF_OK;
  rlf_ctx *c = f->ctx;
  if (c) {
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
  }
  free_facets(f);
  delete f;
  return RLF_OK;
}

int rlf_facets_set_positions(rlf_ctx *c, rlf_facets *f, int32_t n_side, double step_arcsec) {
  if (!c) return RLF_EINVAL;
  c->err.clear();
  if (!f || f->ctx != c) return fail(c, RLF_EINVAL, "facets is NULL or from another context");
  if (n_side != 1 && n_side != 3 && n_side != 5 && n_side != 7) return fail(c, RLF_EINVAL, "n_side: 1, 3, 5 or 7");
  if (n_side > 1 && !(step_arcsec > 0.0 && is_fin(step_arcsec)))
    return fail(c, RLF_EINVAL, "step_arcsec must be positive and finite");
  if (int e = set_device(c)) return e;
  if (n_side > 1) {
    const int64_t need = f->dense_total * (int64_t)n_side * n_side;
    if (need > f->pos_cap) {
      HIPCHK(c, hipStreamSynchronize(c->stream));        // a queued fit may still read the old rows
      if (f->d_pos_g) (void)hipFree(f->d_pos_g);
      f->d_pos_g = nullptr;
      f->pos_cap = 0;
      hipError_t e = hipMalloc(&f->d_pos_g, (size_t)need * (f->mixed ? sizeof(float) : sizeof(double)));
      if (e != hipSuccess) {
        f->d_pos_g = nullptr;
        (void)hipGetLastError();
        f->pos_side = 1;
        return fail(c, RLF_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
      }
      f->pos_cap = need;
    }
  }
  f->pos_side = n_side;
  f->pos_step = n_side > 1 ? step_arcsec * kArcsec : 0.0;
  return RLF_OK;
}

int rlf_refine_sources(rlf_ctx *c, rlf_facets *f, int32_t np_max, double e_res, rlf_fit_out *out) {
  if (!c) return RLF_EINVAL;
  c->err.clear();
  if (!f || f->ctx != c) return fail(c, RLF_EINVAL, "facets is NULL or from another context");
  if (!out || !out->flags) return fail(c, RLF_EINVAL, "out/out.flags is NULL");
  if (np_max < 1 || !(e_res > 0) || !is_fin(e_res)) return fail(c, RLF_EINVAL, "np_max >= 1 and e_res > 0");
  if (int e = set_device(c)) return e;
  int last = 0;
  while (last < kMaxRefineLevel && c->p.e_step / (double)(1 << last) > e_res) ++last;
  if (last == 0) return RLF_OK;                          // the grid is already fine enough
  if (c->p.e_step / (double)(1 << last) > e_res)
    return fail(c, RLF_EINVAL, "e_res below e_step / 2^12");
  constexpr int kSide = 64;
  if (!f->d_refine_win) {
    if (int e = dalloc(c, &f->d_refine_win, f->n_src * 5)) return e;
    if (int e = dalloc(c, &f->d_refine_l, f->n_src * (int64_t)kSide * kSide)) return e;
  }
  RefineArgs r{};
  r.n_src = (int32_t)f->n_src;
  r.last_level = last;
  r.np_max = np_max;
  r.max_side = kSide;
  r.unit = (int32_t)std::nearbyint(1.0 / c->p.e_step);
  r.n_e = c->p.n_e;
  r.n_valid = c->n_valid;
  r.e_step = c->p.e_step;
  r.log_frac = std::log(c->p.frac_thresh);
  r.bad_sigma = c->p.bad_sigma;
  r.bad_sqrtdet = c->p.bad_sqrtdet;
  r.epts = c->d_epts;
  r.lsurf = f->d_lsurf;
  r.offsets = f->cells.offsets;
  r.win = f->d_refine_win;
  r.lloc = f->d_refine_l;
  r.e1 = out->e1;
  r.e2 = out->e2;
  r.s1 = out->s1;
  r.s2 = out->s2;
  r.c12 = out->c12;
  r.lmax = out->lmax;
  r.n_above = out->n_above;
  r.flags = out->flags;
  FitArgs fa{};
  if (int e = fit_args(c, f, fa)) return e;
  HIPCHK(c, launch_refine_start(r, c->stream));
  for (int level = 1; level <= last; ++level) {
    r.level = level;
    HIPCHK(c, launch_refine_eval(fa, r, f->mixed, c->stream));
    HIPCHK(c, launch_refine_estimate(r, c->stream));
  }
  return RLF_OK;
}

int rlf_fit_sources(rlf_ctx *c, const rlf_facets *f, const rlf_fit_opts *opts, rlf_fit_out *out) {
  if (!c) return RLF_EINVAL;
  c->err.clear();
  if (!f || f->ctx != c) return fail(c, RLF_EINVAL, "facets is NULL or from another context");
  if (!out || !out->flags) return fail(c, RLF_EINVAL, "out/out.flags is NULL");
  rlf_fit_opts o{};
  if (opts) o = *opts;
  if (o.mode != 0 && o.mode != 1 && o.mode != 2) return fail(c, RLF_EINVAL, "opts.mode");
  if (o.mode == 2 && (o.check_stride < 2 || o.check_stride >= c->p.n_e))
    return fail(c, RLF_EINVAL, "lattice-seeded mode needs opts.check_stride in 2..n_e-1");
  if (o.mode != 2 && o.check_stride != 0 &&
      (o.mode != 1 || !o.fallback || o.check_stride < 2 || o.check_stride >= c->p.n_e))
    return fail(c, RLF_EINVAL, "opts.check_stride: 0, or 2..n_e-1 in windowed mode with fallback");
  if (o.mode == 1 && !o.window) return fail(c, RLF_EINVAL, "windowed mode needs opts.window");
  if (o.want_surface && !out->surface) return fail(c, RLF_EINVAL, "want_surface needs out.surface");
  if (o.mode != 0 && f->pos_side > 1)
    return fail(c, RLF_EUNSUPPORTED, "position marginalisation is implemented for the full grid only");
  if (int e = set_device(c)) return e;
  return enqueue_fit(c, f, o, *out, nullptr, 0);
}

}  // extern "C"

namespace rlf {

int fit_args(rlf_ctx *c, const rlf_facets *f, FitArgs &fa) {
  fa = FitArgs{};
  fa.n_src = (int32_t)f->n_src;
  fa.n_valid = c->n_valid;
  fa.n_e = c->p.n_e;
  fa.num_r = c->p.num_r;
  fa.e_step = c->p.e_step;
  fa.epts = c->d_epts;
  fa.valid_index = c->d_vidx;
  fa.sk = c->d_sk;
  fa.logw = f->d_logw;
  fa.offsets = f->cells.offsets;
  fa.fit64 = f->cells.fit64;
  fa.fit32 = f->cells.fit32;
  fa.lsurf = f->d_lsurf;
  fa.size_order = f->d_order;
  if (f->pos_side > 1) {
    PosPrepArgs pa{};
    pa.n_src = (int32_t)f->n_src;
    pa.n_side = f->pos_side;
    pa.n_pos = f->pos_side * f->pos_side;
    pa.step = f->pos_step;
    pa.src = f->d_src;
    pa.offsets = f->cells.offsets;
    pa.ix = f->cells.ix;
    pa.iy = f->cells.iy;
    pa.wsum = f->cells.wsum;
    pa.vre = f->cells.vre;
    pa.vim = f->cells.vim;
    pa.g64 = f->mixed ? nullptr : (double *)f->d_pos_g;
    pa.g32 = f->mixed ? (float *)f->d_pos_g : nullptr;
    HIPCHK(c, launch_pos_prep(pa, f->mixed, c->stream));
    fa.n_pos = pa.n_pos;
    fa.pos_g64 = pa.g64;
    fa.pos_g32 = pa.g32;
  }
  // few sources: split each source's cells over several waves per grid point
  // (a source alone is ~100 waves; split until ~2048 waves run), unless the
  // stream is being captured (the partial-sum buffer may have to grow)
  if (!f->mixed && f->pos_side <= 1 && c->p.num_r == 20) {
    const int64_t waves = f->n_src * (int64_t)((c->n_valid + 63) / 64);
    const int64_t parts = std::min<int64_t>(16, 2048 / std::max<int64_t>(1, waves));
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(c, hipStreamIsCapturing(c->stream, &cs));
    if (parts >= 2 && cs == hipStreamCaptureStatusNone) {
      const int64_t need = f->n_src * parts * 2 * c->p.num_r * (int64_t)c->n_valid;
      if (need > c->part_cap) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        dfree(c->d_part);
        c->part_cap = 0;
        if (int e = dalloc(c, &c->d_part, need)) return e;
        c->part_cap = need;
      }
      fa.parts = (int32_t)parts;
      fa.part_sums = c->d_part;
    }
  }
  return RLF_OK;
}

int enqueue_fit(rlf_ctx *c, const rlf_facets *f, const rlf_fit_opts &o, const rlf_fit_out &out,
                const QueueArgs *queue, int queue_blocks) {
  const bool lattice = o.mode == 2;
  const bool windowed = o.mode == 1 || lattice;
  FitArgs fa{};
  if (int e = fit_args(c, f, fa)) return e;
  if (lattice) {
    // the stride-S lattice first, then each source's window from it
    fa.check_stride = o.check_stride;
    fa.lattice_pass = 1;
    hipError_t e = f->mixed ? launch_fit_mixed(fa, c->stream) : launch_fit_f64(fa, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "lattice pass launch");
    e = launch_lattice_windows(fa, std::log(c->p.frac_thresh), f->d_win, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "lattice window launch");
    fa.lattice_pass = 2;
  }
  const bool fallback = lattice || o.fallback;
  fa.window = lattice ? f->d_win : (windowed ? o.window : nullptr);
  fa.check_stride = (windowed && fallback) ? o.check_stride : 0;
  fa.redo = nullptr;
  fa.lsurf = f->d_lsurf;
  EstimateArgs ea{};
  ea.n_src = (int32_t)f->n_src;
  ea.n_valid = c->n_valid;
  ea.n_e = c->p.n_e;
  ea.half_r2 = c->half_r2;
  ea.e_step = c->p.e_step;
  ea.log_frac = std::log(c->p.frac_thresh);
  ea.bad_sigma = c->p.bad_sigma;
  ea.bad_sqrtdet = c->p.bad_sqrtdet;
  ea.epts = c->d_epts;
  ea.offsets = f->cells.offsets;
  ea.lsurf = f->d_lsurf;
  ea.window = fa.window;
  ea.redo = nullptr;
  ea.redo_out = (windowed && fallback) ? f->d_redo : nullptr;
  ea.check_stride = fa.check_stride;
  ea.e1 = out.e1;
  ea.e2 = out.e2;
  ea.s1 = out.s1;
  ea.s2 = out.s2;
  ea.c12 = out.c12;
  ea.lmax = out.lmax;
  ea.argmax = out.argmax;
  ea.n_above = out.n_above;
  ea.flags = out.flags;
  ea.surface = o.want_surface ? out.surface : nullptr;
  if (f->mixed && f->pos_side <= 1) {
    ea.fit64 = f->cells.fit64;
    ea.sk = c->d_sk;
    ea.logw = f->d_logw;
    ea.num_r = c->p.num_r;
    ea.recheck_rel = kRecheckRel;
    ea.recheck_abs = kRecheckAbs;
  }
  hipError_t e;
  if (queue && !windowed)
    e = launch_fit_queue(fa, *queue, f->mixed, queue_blocks, c->stream);
  else
    e = f->mixed ? launch_fit_mixed(fa, c->stream) : launch_fit_f64(fa, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "fit kernel launch");
  e = launch_estimate(ea, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "estimate kernel launch");
  if (windowed && fallback) {
    fa.window = nullptr;
    fa.check_stride = 0;
    fa.lattice_pass = 0;
    fa.redo = f->d_redo;
    ea.window = nullptr;
    ea.check_stride = 0;
    ea.redo = f->d_redo;
    ea.redo_out = nullptr;
    e = f->mixed ? launch_fit_mixed(fa, c->stream) : launch_fit_f64(fa, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "fit kernel launch (fallback)");
    e = launch_estimate(ea, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "estimate kernel launch (fallback)");
  }
  return RLF_OK;
}

}  // namespace rlf

