// Sequential sky-model refinement around the data-parallel pass (Sec. 2.1:
// the sky model starts circular and each measured shape replaces the
// model's; Sec. 2.4: unreliable fits keep their model and are fitted again at
// the end; Sec. 3.1: with several sources fitted at once the model is updated
// per chunk).  The host orders the chunks.  The residual lives in the
// uv-sorted layout of the first chunk's facet object, which every later
// chunk borrows: it is formed once (the residual DFT of the whole starting
// model, in sorted order), each chunk is extracted from it directly (no
// gather) and fitted on the full grid, and the refined sources' models are
// then swapped in place, R += (old models) - (new models), in one pass over
// the sorted visibilities: the next chunk's extraction makes that pass
// itself when it runs the small-catalogue kernel, otherwise the swap runs
// before it.  The arithmetic is that of the caller-order path
// (rlf_model_vis residual, accumulate and residual modes, then a gather), so
// the results are the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "rlf_objects.h"

using namespace rlf;

namespace {

// Host copy of a subset of a catalogue with the current shapes.
struct SubCat {
  std::vector<double> l, m, flux, alpha, e1, e2, mu;
  rlf_catalog view() const {
    rlf_catalog k{};
    k.n_src = (int64_t)l.size();
    k.l = l.data();
    k.m = m.data();
    k.flux_jy = flux.data();
    k.alpha_arcsec = alpha.data();
    k.e1 = e1.data();
    k.e2 = e2.data();
    k.prior_mu = mu.empty() ? nullptr : mu.data();
    return k;
  }
};

SubCat subset(const rlf_catalog *cat, const std::vector<int64_t> &idx, const std::vector<double> &e1,
              const std::vector<double> &e2) {
  SubCat s;
  for (int64_t i : idx) {
    s.l.push_back(cat->l[i]);
    s.m.push_back(cat->m[i]);
    s.flux.push_back(cat->flux_jy[i]);
    s.alpha.push_back(cat->alpha_arcsec[i]);
    s.e1.push_back(e1[(size_t)i]);
    s.e2.push_back(e2[(size_t)i]);
    if (cat->prior_mu) s.mu.push_back(cat->prior_mu[i]);
  }
  return s;
}

rlf_fit_out offset(const rlf_fit_out &o, int64_t k) {
  rlf_fit_out r{};
  r.e1 = o.e1 ? o.e1 + k : nullptr;
  r.e2 = o.e2 ? o.e2 + k : nullptr;
  r.s1 = o.s1 ? o.s1 + k : nullptr;
  r.s2 = o.s2 ? o.s2 + k : nullptr;
  r.c12 = o.c12 ? o.c12 + k : nullptr;
  r.lmax = o.lmax ? o.lmax + k : nullptr;
  r.argmax = o.argmax ? o.argmax + k : nullptr;
  r.n_above = o.n_above ? o.n_above + k : nullptr;
  r.flags = o.flags + k;
  r.surface = nullptr;
  return r;
}

// Device buffers released on every exit path.
struct Scratch {
  std::vector<void *> ptrs;
  std::vector<rlf_facets *> facets;
  ~Scratch() {
    for (rlf_facets *f : facets) rlf_facets_free(f);
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
  }
  template <class T>
  int alloc(rlf_ctx *c, T **p, int64_t n) {
    if (int e = dalloc(c, p, n)) return e;
    ptrs.push_back((void *)*p);
    return RLF_OK;
  }
};

}  // namespace

extern "C" int rlf_fit_sequential(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, int64_t chunk,
                                  int32_t refit_bad, const rlf_fit_out *out, double *e1_host, double *e2_host) {
  if (!c) return RLF_EINVAL;
  c->err.clear();
  if (!obs || !cat || !out || !out->flags || !out->e1 || !out->e2 || !e1_host || !e2_host)
    return fail(c, RLF_EINVAL, "rlf_fit_sequential: NULL argument (out.flags, out.e1, out.e2 are required)");
  if (chunk < 1) return fail(c, RLF_EINVAL, "rlf_fit_sequential: chunk must be >= 1");
  if (!obs->vis) return fail(c, RLF_EINVAL, "rlf_fit_sequential: obs.vis is NULL");
  if (cat->n_src <= 0 || !cat->e1 || !cat->e2) return fail(c, RLF_EINVAL, "rlf_fit_sequential: catalogue");
  HIPCHK(c, hipSetDevice(c->device));
  const int64_t n = cat->n_src;
  const bool mixed = c->p.precision == RLF_MIXED;
  const int64_t n_vis = obs->n_rows * obs->n_chan;
  std::vector<double> e1(cat->e1, cat->e1 + n), e2(cat->e2, cat->e2 + n);
  Scratch sc;

  // FP64 form: the unweighted residual next to the weighted one the
  // extraction reads (the mixed form keeps R itself in the sorted layout)
  double2 *Rs = nullptr;
  if (!mixed)
    if (int e = sc.alloc(c, &Rs, n_vis)) return e;
  rlf_catalog cur = *cat;
  cur.e1 = e1.data();
  cur.e2 = e2.data();

  rlf_fit_opts full{};
  std::vector<uint32_t> flags((size_t)n, 0u);
  std::vector<double> he1((size_t)n), he2((size_t)n);
  rlf_facets *master = nullptr;
  // the previous chunk's model swap, applied by the next extraction
  UpdateArgs pending{};
  bool has_pending = false;
  for (int64_t c0 = 0; c0 < n; c0 += chunk) {
    const int64_t c1 = std::min(n, c0 + chunk);
    std::vector<int64_t> idx;
    for (int64_t s = c0; s < c1; ++s) idx.push_back(s);
    const SubCat sub = subset(cat, idx, e1, e2);
    const rlf_catalog v = sub.view();
    rlf_facets *f = nullptr;
    if (master && v.n_src == master->n_src) {
      // a chunk of the first chunk's size reuses its facet object
      if (int e = retarget_facets(c, obs, &v, master)) return e;
      f = master;
    } else {
      if (int e = create_facets(c, obs, &v, master, &f)) return e;
      sc.facets.push_back(f);
    }
    if (!master) {
      // residual of the starting model, kept in place from here on
      master = f;
      if (int e = sorted_residual(c, obs, &cur, master, Rs)) return e;
    }
    if (int e = extract_facets(c, obs, &v, nullptr, 0, f, has_pending ? &pending : nullptr)) return e;
    has_pending = false;
    rlf_fit_out o = offset(*out, c0);
    if (int e = rlf_fit_sources(c, f, &full, &o)) return e;
    const size_t m = (size_t)(c1 - c0);
    HIPCHK(c, hipMemcpyAsync(flags.data() + c0, o.flags, m * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(he1.data() + c0, o.e1, m * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(he2.data() + c0, o.e2, m * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (f != master) {
      sc.facets.pop_back();
      rlf_facets_free(f);
    }
    // the chunk's reliable shapes replace their models: R += old - new
    std::vector<int64_t> good;
    for (int64_t s = c0; s < c1; ++s)
      if (!(flags[(size_t)s] & (RLF_FLAG_BAD_VAR | RLF_FLAG_EMPTY)) && std::isfinite(he1[(size_t)s]) &&
          std::isfinite(he2[(size_t)s]) && he1[(size_t)s] * he1[(size_t)s] + he2[(size_t)s] * he2[(size_t)s] < 1.0)
        good.push_back(s);
    if (!good.empty()) {
      const SubCat old_m = subset(cat, good, e1, e2);
      for (int64_t s : good) {
        e1[(size_t)s] = he1[(size_t)s];
        e2[(size_t)s] = he2[(size_t)s];
      }
      const SubCat new_m = subset(cat, good, e1, e2);
      const rlf_catalog vo = old_m.view(), vn = new_m.view();
      if (int e = prepare_update(c, &vo, &vn, master, Rs, pending)) return e;
      has_pending = true;
    }
  }
  if (has_pending)
    if (int e = update_sorted_residual(c, pending, mixed ? 1 : 0)) return e;

  if (refit_bad) {
    std::vector<int64_t> bad;
    for (int64_t s = 0; s < n; ++s)
      if (flags[(size_t)s] & RLF_FLAG_BAD_VAR) bad.push_back(s);
    if (!bad.empty()) {
      const int64_t nb = (int64_t)bad.size();
      const SubCat sub = subset(cat, bad, e1, e2);
      const rlf_catalog v = sub.view();
      rlf_facets *f = nullptr;
      if (int e = create_facets(c, obs, &v, master, &f)) return e;
      sc.facets.push_back(f);
      if (int e = extract_facets(c, obs, &v, nullptr, 0, f)) return e;
      double *t[6];
      int32_t *ti[2], *tidx = nullptr;
      uint32_t *tf = nullptr;
      for (double *&p : t)
        if (int e = sc.alloc(c, &p, nb)) return e;
      for (int32_t *&p : ti)
        if (int e = sc.alloc(c, &p, nb)) return e;
      if (int e = sc.alloc(c, &tf, nb)) return e;
      if (int e = sc.alloc(c, &tidx, nb)) return e;
      std::vector<int32_t> hidx(bad.begin(), bad.end());
      HIPCHK(c, hipMemcpyAsync(tidx, hidx.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, c->stream));
      rlf_fit_out o{};
      o.e1 = t[0];
      o.e2 = t[1];
      o.s1 = t[2];
      o.s2 = t[3];
      o.c12 = t[4];
      o.lmax = t[5];
      o.argmax = ti[0];
      o.n_above = ti[1];
      o.flags = tf;
      if (int e = rlf_fit_sources(c, f, &full, &o)) return e;
      double *dst[6] = {out->e1, out->e2, out->s1, out->s2, out->c12, out->lmax};
      for (int k = 0; k < 6; ++k)
        if (dst[k]) HIPCHK(c, launch_scatter_f64(t[k], tidx, nb, dst[k], c->stream));
      if (out->argmax)
        HIPCHK(c, launch_scatter_u32(reinterpret_cast<uint32_t *>(ti[0]), tidx, nb, 0u,
                                     reinterpret_cast<uint32_t *>(out->argmax), c->stream));
      if (out->n_above)
        HIPCHK(c, launch_scatter_u32(reinterpret_cast<uint32_t *>(ti[1]), tidx, nb, 0u,
                                     reinterpret_cast<uint32_t *>(out->n_above), c->stream));
      HIPCHK(c, launch_scatter_u32(tf, tidx, nb, (uint32_t)RLF_FLAG_REFIT, out->flags, c->stream));
      std::vector<double> r1((size_t)nb), r2((size_t)nb);
      HIPCHK(c, hipMemcpyAsync(r1.data(), t[0], sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(r2.data(), t[1], sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      for (int64_t k = 0; k < nb; ++k)
        if (std::isfinite(r1[(size_t)k]) && std::isfinite(r2[(size_t)k])) {
          e1[(size_t)bad[(size_t)k]] = r1[(size_t)k];
          e2[(size_t)bad[(size_t)k]] = r2[(size_t)k];
        }
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::copy(e1.begin(), e1.end(), e1_host);
  std::copy(e2.begin(), e2.end(), e2_host);
  return RLF_OK;
}
