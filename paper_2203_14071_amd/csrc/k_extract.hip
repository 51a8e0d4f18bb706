// Facet extraction (Sec. 2.3): per (visibility, source) pair, phase-shift the
// residual to the source, add back the source's own model, and accumulate the
// weighted result into the source's facet cell (rint(u theta), rint(v theta)).
//
// Work decomposition.  Lanes are sources: a wave holds 64 sources (one per
// lane, their constants in VGPRs) and walks a chunk of visibilities in the
// facet object's uv-sorted order; each visibility's data is uniform across
// the wave and arrives through scalar loads.  Along the sorted order every
// source stays in one facet cell for long runs, so each lane accumulates
// (count, W, Z) in registers and issues global atomics only when its cell
// changes or the chunk ends: no cross-lane merging is needed.
//
// XCD-aware launch: blocks are dispatched round-robin over the 8 XCDs; the
// grid is laid out so that all blocks of one visibility chunk (all source
// tiles) land on one XCD and share its L2 for the chunk's data.
//
// Integer results are exact (cell index in FP64 exactly as rint(fl(u theta)));
// FP sums are atomic and order-dependent in their last bits.
#include "rlf_devmath.h"
#include "rlf_internal.h"

namespace rlf {

namespace {

constexpr int kXcd = 8;
constexpr int kWaves = 4;          // waves (source tiles) per block
constexpr int kGroup = 4;          // visibilities whose scalar loads are issued together

struct Run {
  int key;                         // cell in the source's dense block, -1 = none
  uint32_t n;
  double w, zr, zi;
};

__device__ __forceinline__ void flush(uint32_t *__restrict__ cnt, double *__restrict__ ws, double *__restrict__ zre,
                                      double *__restrict__ zim, int64_t base, const Run &p) {
  const int64_t k = base + p.key;
  atomicAdd(cnt + k, p.n);
  unsafeAtomicAdd(ws + k, p.w);
  unsafeAtomicAdd(zre + k, p.zr);
  unsafeAtomicAdd(zim + k, p.zi);
}

// The read-only visibility data and the atomic targets are separate
// restrict-qualified kernel parameters: with no possible aliasing the
// compiler keeps the per-visibility loads scalar (s_load) although the loop
// issues atomics.  Visibilities are taken in groups of kGroup whose loads are
// issued together; the sorted arrays are padded so a group never reads past
// the end, and padding carries weight 0.
template <bool kMixed>
__global__ __launch_bounds__(256) void k_extract(ExtractArgs a, const double *__restrict__ su,
                                                 const double *__restrict__ sv, const double *__restrict__ sw,
                                                 const uint32_t *__restrict__ sch4, const void *__restrict__ sres,
                                                 const void *__restrict__ swt, const double *__restrict__ spec_tab,
                                                 uint32_t *__restrict__ cnt, double *__restrict__ ws,
                                                 double *__restrict__ zre, double *__restrict__ zim) {
  __shared__ double2 tab[kCisTable + 1];
  if (!kMixed) {
    cis_table_init(tab);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int bpc = (a.n_tiles + kWaves - 1) / kWaves;           // blocks per chunk
  const int64_t xcd = blockIdx.x % kXcd, local = blockIdx.x / kXcd;
  const int64_t chunk = (local / bpc) * kXcd + xcd;
  const int tile = (int)(local % bpc) * kWaves + wid;
  if (chunk >= a.n_chunks || tile >= a.n_tiles) return;          // uniform per wave

  const int s_raw = tile * 64 + lane;
  const bool active = s_raw < a.n_src;
  const int s = active ? s_raw : a.n_src - 1;
  const SrcGeom g = a.geom[s];
  const int64_t j0 = chunk * (int64_t)a.chunk;
  const int64_t j1 = min(a.sv.n_vis, j0 + (int64_t)a.chunk);
  const bool multi = a.n_chan > 1;

  Run cur{-1, 0u, 0.0, 0.0, 0.0};
  if (!kMixed) {
    const SrcModel p = a.src[s];
    const double2 *__restrict__ res = reinterpret_cast<const double2 *>(sres);
    const double *__restrict__ wt = reinterpret_cast<const double *>(swt);
    for (int64_t jg = j0; jg < j1; jg += kGroup) {
      double wwg[kGroup], ug[kGroup], vg[kGroup], wg[kGroup], spg[kGroup];
      double2 rg[kGroup];
      const uint32_t chg = multi ? sch4[jg / 4] : 0u;
#pragma unroll
      for (int t = 0; t < kGroup; ++t) {
        wwg[t] = wt[jg + t];
        ug[t] = su[jg + t];
        vg[t] = sv[jg + t];
        wg[t] = sw[jg + t];
        rg[t] = res[jg + t];
        spg[t] = spec_tab[(chg >> (8 * t)) & 0xffu];
      }
#pragma unroll
      for (int t = 0; t < kGroup; ++t) {
      const double ww = wwg[t];
      if (!(ww > 0.0)) continue;                                   // uniform
      const double u = ug[t], v = vg[t], w = wg[t];
      const double2 r = rg[t];
      const double spec = spg[t];
      const double ph = fma(u, p.l, fma(v, p.m, w * p.n1));
      const double2 cs = cis2pi_f64(ph, tab);
      double zr = fma(r.x, cs.x, r.y * cs.y);                      // residual * exp(-2 pi i ph)
      const double zi = fma(r.y, cs.x, -(r.x * cs.y));
      const double x = fma(p.q11, u * u, fma(p.q12x2, u * v, fma(p.q22, v * v, 1.0)));
      const double q = rsqrt_f64(x);
      zr = fma(spec * p.flux, q * q * q, zr);                      // own model, real after the shift
      const int ix = (int)rint(__dmul_rn(u, p.theta));
      const int iy = (int)rint(__dmul_rn(v, p.theta));
      const unsigned ox = (unsigned)(ix + g.half), oy = (unsigned)(iy + g.half);
      const bool inb = ox < (unsigned)g.side && oy < (unsigned)g.side;
      const int key = inb ? (int)(oy * (unsigned)g.side + ox) : -1;
      if (key != cur.key) {
        if (cur.key >= 0 && active) flush(cnt, ws, zre, zim, g.base, cur);
        if (!inb && active) atomicOr(a.err, 1u);
        cur.key = key;
        cur.n = 0u;
        cur.w = cur.zr = cur.zi = 0.0;
      }
      cur.n += 1u;
      cur.w += ww;
      cur.zr = fma(ww, zr, cur.zr);
      cur.zi = fma(ww, zi, cur.zi);
      }
    }
  } else {
    const SrcMixed p = a.src32[s];
    const float2 *__restrict__ res = reinterpret_cast<const float2 *>(sres);
    const float *__restrict__ wt = reinterpret_cast<const float *>(swt);
    for (int64_t jg = j0; jg < j1; jg += kGroup) {
      float wwg[kGroup];
      double ug[kGroup], vg[kGroup], wg[kGroup], spg[kGroup];
      float2 rg[kGroup];
      const uint32_t chg = multi ? sch4[jg / 4] : 0u;
#pragma unroll
      for (int t = 0; t < kGroup; ++t) {
        wwg[t] = wt[jg + t];
        ug[t] = su[jg + t];
        vg[t] = sv[jg + t];
        wg[t] = sw[jg + t];
        rg[t] = res[jg + t];
        spg[t] = spec_tab[(chg >> (8 * t)) & 0xffu];
      }
#pragma unroll
      for (int tt = 0; tt < kGroup; ++tt) {
      const float ww = wwg[tt];
      if (!(ww > 0.0f)) continue;                                  // uniform
      const double u = ug[tt], v = vg[tt], w = wg[tt];
      const float2 r = rg[tt];
      const float spec = (float)spg[tt];
      const double ph = fma(u, p.l, fma(v, p.m, w * p.n1));
      const float t = (float)(ph - rint(ph));                      // turns, |t| <= 1/2
      const float sn = __builtin_amdgcn_sinf(t), cs = __builtin_amdgcn_cosf(t);
      float zr = fmaf(r.x, cs, r.y * sn);
      const float zi = fmaf(r.y, cs, -(r.x * sn));
      const float uf = (float)u, vf = (float)v;
      const float x = fmaf(p.q11, uf * uf, fmaf(p.q12x2, uf * vf, fmaf(p.q22, vf * vf, 1.0f)));
      const float q = __builtin_amdgcn_rsqf(x);
      zr = fmaf(spec * p.flux, q * q * q, zr);
      const int ix = (int)rint(__dmul_rn(u, p.theta));
      const int iy = (int)rint(__dmul_rn(v, p.theta));
      const unsigned ox = (unsigned)(ix + g.half), oy = (unsigned)(iy + g.half);
      const bool inb = ox < (unsigned)g.side && oy < (unsigned)g.side;
      const int key = inb ? (int)(oy * (unsigned)g.side + ox) : -1;
      if (key != cur.key) {
        if (cur.key >= 0 && active) flush(cnt, ws, zre, zim, g.base, cur);
        if (!inb && active) atomicOr(a.err, 1u);
        cur.key = key;
        cur.n = 0u;
        cur.w = cur.zr = cur.zi = 0.0;
      }
      const double wd = (double)ww;
      cur.n += 1u;
      cur.w += wd;
      cur.zr = fma(wd, (double)zr, cur.zr);
      cur.zi = fma(wd, (double)zi, cur.zi);
      }
    }
  }
  if (cur.key >= 0 && active) flush(cnt, ws, zre, zim, g.base, cur);
}

}  // namespace

hipError_t launch_extract(const ExtractArgs &a, int mixed, hipStream_t st) {
  const int64_t bpc = (a.n_tiles + kWaves - 1) / kWaves;
  const int64_t blocks = ((a.n_chunks + kXcd - 1) / kXcd) * kXcd * bpc;
  const Sorted &v = a.sv;
  if (mixed)
    hipLaunchKernelGGL(k_extract<true>, dim3((unsigned)blocks), dim3(64 * kWaves), 0, st, a, v.u, v.v, v.w,
                       reinterpret_cast<const uint32_t *>(v.chan), v.res, v.wt, a.chan->spec, a.acc.count, a.acc.wsum, a.acc.zre, a.acc.zim);
  else
    hipLaunchKernelGGL(k_extract<false>, dim3((unsigned)blocks), dim3(64 * kWaves), 0, st, a, v.u, v.v, v.w,
                       reinterpret_cast<const uint32_t *>(v.chan), v.res, v.wt, a.chan->spec, a.acc.count, a.acc.wsum, a.acc.zre, a.acc.zim);
  return hipGetLastError();
}

}  // namespace rlf
