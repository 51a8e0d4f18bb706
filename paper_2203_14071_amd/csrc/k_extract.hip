// Facet extraction (Sec. 2.3): per (visibility, source) pair, phase-shift the
// residual to the source, add back the source's own model, and accumulate the
// weighted result into the source's facet cell (rint(u theta), rint(v theta)).
//
// Work decomposition.  Lanes are sources: a wave holds 64 NS sources (NS per
// lane, their constants in VGPRs; lane slots take the sources in order of
// facet cell size, so the cell changes of a wave's lanes tend to coincide
// and the branches diverge less) and walks a chunk of visibilities in the
// facet object's uv-sorted order; each visibility's data is uniform across
// the wave and arrives through scalar loads.  Along the sorted order a
// source stays in one facet cell for runs of ~100-300 visibilities and,
// near a cell boundary, alternates between the same two cells many times
// (a Morton curve crosses a boundary back and forth).  Each lane therefore
// keeps two runs (count, W, Z) in registers, its current cell's and the
// previous cell's, swaps them when it returns to the previous cell, and
// issues global atomics only when it enters a third cell or the chunk ends:
// on the 1000-source SKA-MID field one atomic flush per ~20 cell changes
// (with one run per lane, every cell change flushed), and no cross-lane
// merging is needed.
//
// XCD-aware launch: blocks are dispatched round-robin over the 8 XCDs; the
// grid is laid out so that all blocks of one visibility chunk (all source
// tiles) land on one XCD and share its L2 for the chunk's data.
//
// Integer results are exact (cell index in FP64 exactly as rint(fl(u theta)));
// FP sums are atomic and order-dependent in their last bits.  Runs are summed
// in FP64 in both forms (the mixed form's FP32 terms are widened per term).
#include <algorithm>

#include "rlf_devmath.h"
#include "rlf_internal.h"
#include "rlf_sky.h"

namespace rlf {

namespace {

constexpr int kXcd = 8;
constexpr int kWaves = 4;          // waves per block (1024-entry table or none)
// FP64 launches of at least kBigTableTiles source tiles take a 2048-entry
// table (32 KB of LDS: sin's x^5 term drops, one FMA per pair) in blocks of
// 8 waves, so that four blocks per CU keep eight waves per SIMD in 128 KB;
// smaller launches, whose blocks hold idle waves, keep the 16 KB table and
// four-wave blocks (eight blocks per CU)
constexpr int kBigTableTiles = 8;
template <bool kMixed, int T>
constexpr int waves_per_block() { return (!kMixed && T == 2048) ? 8 : kWaves; }
constexpr int kNsF64 = 1, kNsMixed = 1;        // sources per lane
constexpr int kGroupF64 = 2, kGroupMixed = 4;  // visibilities whose scalar loads are issued together
constexpr double kNoRun = 1099511627776.0;    // 2^40: "no open run" (run keys are below 2^31 in magnitude)
constexpr int32_t kNoKey = INT32_MIN;          // the same for the previous run's integer key

// One source of a lane: facet geometry and two open runs, the current cell's
// and the cell the lane was in before it.  Near a cell boundary the sorted
// order crosses back and forth between the same two cells many times, so a
// return to the previous cell only swaps the two runs; global memory is
// touched when a third cell is entered (the older run is flushed) and at
// the end of the chunk.  A run key is iy * side + ix (an exact integer in
// FP64); base already holds the offset half * (side + 1) of cell (0, 0) in
// the source's dense block.  Counts are kept relative to the
// lane-independent count nproc of processed visibilities: the current run
// holds nproc - cb visibilities, the other run ocnt.
struct LaneSrc {
  bool active;
  int32_t half;
  int64_t base;
  double side;
  double key, rw, rzr, rzi;        // current cell
  double ow, ozr, ozi;             // the cell before it
  int32_t okey, cb, ocnt;          // okey: the previous cell's key, or kNoKey
};

// Add a run to its dense cell: four FP64 atomics at one address (the count
// is an exact integer in FP64).
__device__ __forceinline__ void flush(double4 *__restrict__ acc, int64_t base, int32_t key, double w, double zr,
                                      double zi, int32_t n) {
  double *c = &acc[base + key].x;
  unsafeAtomicAdd(c, w);
  unsafeAtomicAdd(c + 1, zr);
  unsafeAtomicAdd(c + 2, zi);
  unsafeAtomicAdd(c + 3, (double)n);
}

// Run bookkeeping of one lane source at one visibility (nproc = visibilities
// of the chunk with weight > 0 processed before this one, uniform).  When
// the cell changes: back to the previous cell swaps the two runs; a new cell
// flushes the older run, demotes the current one and opens an empty run
// (after the bounds check).  The caller then adds the visibility's terms to
// the current run.
__device__ __forceinline__ void enter_cell(LaneSrc &L, double4 *__restrict__ acc, uint32_t *err, int32_t nproc,
                                           double xf, double yf) {
  const double k = fma(yf, L.side, xf);
  if (k != L.key) {
    const int32_t tk = L.key == kNoRun ? kNoKey : (int32_t)L.key;
    const double tw = L.rw, tr = L.rzr, ti = L.rzi;
    const int32_t tn = nproc - L.cb;
    if (L.okey != kNoKey && k == (double)L.okey) {
      L.key = (double)L.okey;
      L.rw = L.ow;
      L.rzr = L.ozr;
      L.rzi = L.ozi;
      L.cb = nproc - L.ocnt;
    } else {
      if (L.okey != kNoKey && L.active) flush(acc, L.base, L.okey, L.ow, L.ozr, L.ozi, L.ocnt);
      const double half = (double)L.half;
      const bool inb = fabs(xf) <= half && fabs(yf) <= half;
      if (!inb && L.active) atomicOr(err, 1u);
      L.key = inb ? k : kNoRun;
      L.cb = nproc;
      L.rw = L.rzr = L.rzi = 0.0;
    }
    L.okey = tk;
    L.ow = tw;
    L.ozr = tr;
    L.ozi = ti;
    L.ocnt = tn;
  }
}

// The read-only visibility data and the atomic targets are separate
// restrict-qualified kernel parameters: with no possible aliasing the
// compiler keeps the per-visibility loads scalar (s_load) although the loop
// issues atomics.  Per visibility the wave loads (u, v, w, spec), the
// profile's quadratic terms, the residual and the weight (FP64 form: the
// weighted residual w R and w spec, so that the run sums take the shifted
// residual and the own model in three FMAs and two); flagged visibilities
// carry weight +0 and are skipped on a scalar test of the bits.
// A lane may hold NS sources (NS * 64 per wave) to share each load.
//
// Cell index: ix = rint(fl(u theta)) and iy likewise, in FP64 (exact
// integers); the run key iy side + ix is formed in FP64 too (one FMA, exact:
// |key| < 2^31) and compared as a double, so the common path has no
// conversions.  The facet half-size was sized on the host from the largest
// |u|, |v| with the same rounding chain, so every index is inside its facet;
// the bound is still checked whenever a new cell's run starts (err bit 0).
//
// Occupancy: the FP64 form is held to 64 VGPRs (eight waves per SIMD; the
// few values that spill, the lane's dense-block base among them, are
// reloaded only on the rare third-cell flush and after the loop), the mixed
// form fits eight waves by itself (51 VGPRs) under any bound; its bound
// steers the scalar registers: a minimum of 7 waves gives 94 SGPRs with two
// spilled to VGPR lanes and measured 4.5 % faster than 6 (97 SGPRs, none
// spilled), while 8 spills 17 and is 15 % slower.
// T: entries of the FP64 form's exp table (1024 or 2048; the mixed form has none).
template <bool kMixed, int NS, int G, int T>
__global__ __launch_bounds__((64 * waves_per_block<kMixed, T>()), kMixed ? 7 : 8) void k_extract(
    ExtractArgs a, const double4 *__restrict__ sgeo, const void *__restrict__ squad, const void *__restrict__ sres,
    const uint64_t *__restrict__ swt, double4 *__restrict__ acc) {
  constexpr int kW = waves_per_block<kMixed, T>();
  __shared__ double2 tab[kMixed ? 1 : T];
  if (!kMixed) {
    cis_table_init<T>(tab);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int bpc = (a.n_tiles + kW - 1) / kW;                     // blocks per chunk
  const int64_t xcd = blockIdx.x % kXcd, local = blockIdx.x / kXcd;
  const int64_t chunk = (local / bpc) * kXcd + xcd;
  const int tile = (int)(local % bpc) * kW + wid;
  if (chunk >= a.n_chunks || tile >= a.n_tiles) return;          // uniform per wave

  LaneSrc L[NS];
  int src[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int s_raw = (tile * NS + i) * 64 + lane;
    L[i].active = s_raw < a.n_src;
    src[i] = a.order[L[i].active ? s_raw : a.n_src - 1];
    const SrcGeom g = a.geom[src[i]];
    L[i].base = g.base + (int64_t)g.half * (g.side + 1);
    L[i].half = g.half;
    L[i].side = (double)g.side;
    L[i].key = kNoRun;
    L[i].okey = kNoKey;
    L[i].cb = L[i].ocnt = 0;
    L[i].rw = L[i].rzr = L[i].rzi = 0.0;
    L[i].ow = L[i].ozr = L[i].ozi = 0.0;
  }
  int32_t nproc = 0;
  const int64_t j0 = chunk * (int64_t)a.chunk;
  const int len = (int)(min(a.sv.n_vis, j0 + (int64_t)a.chunk) - j0);
  const double4 *__restrict__ geo = sgeo + j0;
  const uint64_t *__restrict__ wt = swt + j0;                    // weight bits: 0 = skip

  if (!kMixed) {
    // the flux folded into the profile argument: with x' = c0 x and
    // c0 = (3/2 S)^{-2/3}, pow_m32_f64(x') = (2/3) x'^{-3/2} = S x^{-3/2},
    // the own model per unit spectral factor, with no multiplication by S
    // per pair (S = 0: c0 = 1e250, x' >= 1e250 and the term underflows to
    // exactly zero; c0 finite, so no infinity meets a zero coefficient)
    SrcModel p[NS];
    double c0[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      p[i] = a.src[src[i]];
      c0[i] = p[i].flux > 0.0 ? pow(kPowM32Scale * p[i].flux, -2.0 / 3.0) : 1e250;
      p[i].q11 *= c0[i];
      p[i].q12x2 *= c0[i];
      p[i].q22 *= c0[i];
    }
    const double4 *__restrict__ quad = reinterpret_cast<const double4 *>(squad) + j0;
    const double2 *__restrict__ res = reinterpret_cast<const double2 *>(sres) + j0;
    for (int jl = 0; jl < len; jl += G) {
      double4 gg[G], qg[G];
      double2 rg[G];
      uint64_t wwg[G];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        gg[t] = geo[jl + t];
        qg[t] = quad[jl + t];
        rg[t] = res[jl + t];
        wwg[t] = wt[jl + t];
      }
      // the group's values are needed here: the loads the compiler would
      // otherwise sink past the weight test below (a second round trip to
      // memory per group) are issued together with the others
#pragma unroll
      for (int t = 0; t < G; ++t)
        asm volatile("" ::"s"(gg[t].x), "s"(gg[t].y), "s"(gg[t].z), "s"(qg[t].x), "s"(qg[t].y), "s"(qg[t].z));
#pragma unroll
      for (int t = 0; t < G; ++t) {
        if (jl + t >= len) break;                                   // uniform
        if (wwg[t] == 0u) continue;                                  // uniform: flagged or padding
        const double u = gg[t].x, v = gg[t].y, ww = __longlong_as_double((long long)wwg[t]);
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          const double ph = fma(u, p[i].l, fma(v, p[i].m, gg[t].z * p[i].n1));
          const double2 cs = cis2pi_f64<T>(ph, tab);
          const double x = fma(p[i].q11, qg[t].x, fma(p[i].q12x2, qg[t].y, fma(p[i].q22, qg[t].z, c0[i])));
          const double own = pow_m32_f64(x);                        // own model / spec, real after the shift
          enter_cell(L[i], acc, a.err, nproc, rint(__dmul_rn(u, p[i].theta)), rint(__dmul_rn(v, p[i].theta)));
          // w z = (w R) exp(-2 pi i ph) + (w spec) own
          L[i].rw += ww;
          L[i].rzr = fma(rg[t].x, cs.x, fma(rg[t].y, cs.y, fma(qg[t].w, own, L[i].rzr)));
          L[i].rzi = fma(rg[t].y, cs.x, fma(-rg[t].x, cs.y, L[i].rzi));
        }
        ++nproc;
      }
    }
  } else {
    // (the flux stays a multiplication here: folded into the profile
    // argument as in the FP64 form it saves an instruction per pair but
    // measured 0.6 % slower on the 10,000-source field, and again 0.8 %
    // slower on the 1000-source field with the kernel as it is now)
    SrcMixed p[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) p[i] = a.src32[src[i]];
    const float4 *__restrict__ quad = reinterpret_cast<const float4 *>(squad) + j0;
    const float2 *__restrict__ res = reinterpret_cast<const float2 *>(sres) + j0;
    for (int jl = 0; jl < len; jl += G) {
      double4 gg[G];
      float4 qg[G];
      float2 rg[G];
      uint64_t wwg[G];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        gg[t] = geo[jl + t];
        qg[t] = quad[jl + t];
        rg[t] = res[jl + t];
        wwg[t] = wt[jl + t];
      }
      // the group's values are needed here: the loads the compiler would
      // otherwise sink past the weight test below (a second round trip to
      // memory per group) are issued together with the others
#pragma unroll
      for (int t = 0; t < G; ++t)
        asm volatile("" ::"s"(gg[t].x), "s"(gg[t].y), "s"(gg[t].z), "s"(qg[t].x), "s"(qg[t].y), "s"(qg[t].z));
#pragma unroll
      for (int t = 0; t < G; ++t) {
        if (jl + t >= len) break;                                   // uniform
        if (wwg[t] == 0u) continue;                                  // uniform: flagged or padding
        const double u = gg[t].x, v = gg[t].y, ww = __longlong_as_double((long long)wwg[t]);
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          const double ph = fma(u, p[i].l, fma(v, p[i].m, gg[t].z * p[i].n1));
          const float tt = (float)__builtin_amdgcn_fract(ph);        // turns, in [0, 1]
          const float sn = __builtin_amdgcn_sinf(tt), cs = __builtin_amdgcn_cosf(tt);
          float zr = fmaf(rg[t].x, cs, rg[t].y * sn);
          const float zi = fmaf(rg[t].y, cs, -(rg[t].x * sn));
          const float x = fmaf(p[i].q11, qg[t].x, fmaf(p[i].q12x2, qg[t].y, fmaf(p[i].q22, qg[t].z, 1.0f)));
          const float q = __builtin_amdgcn_rsqf(x);
          zr = fmaf(qg[t].w * p[i].flux, q * q * q, zr);
          enter_cell(L[i], acc, a.err, nproc, rint(__dmul_rn(u, p[i].theta)), rint(__dmul_rn(v, p[i].theta)));
          L[i].rw += ww;
          L[i].rzr = fma(ww, (double)zr, L[i].rzr);
          L[i].rzi = fma(ww, (double)zi, L[i].rzi);
        }
        ++nproc;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    if (!L[i].active) continue;
    if (L[i].key != kNoRun) flush(acc, L[i].base, (int32_t)L[i].key, L[i].rw, L[i].rzr, L[i].rzi, nproc - L[i].cb);
    if (L[i].okey != kNoKey) flush(acc, L[i].base, L[i].okey, L[i].ow, L[i].ozr, L[i].ozi, L[i].ocnt);
  }
}

// Visibility-parallel extraction for catalogues of at most kVpSources
// sources (the chunks of a sequential refinement): a wave takes kVpSteps
// steps of 64 consecutive sorted visibilities, one per lane (coalesced
// loads), and evaluates each pair exactly as k_extract does (sources in a
// uniform outer loop, records in SGPRs).  Lanes that fall in one facet cell
// are contiguous runs of the sorted order, so a segmented scan over the
// lanes sums each run; a run that reaches the last lane stays open (its
// sums carried in registers) and continues into the next step, so a cell is
// updated once per run of the sorted order (four FP64 atomics at one
// address), as in k_extract.  A one-source call keeps every lane busy
// instead of one lane in 128.
constexpr int kVpSources = 8;
constexpr int kVpSteps = 32;

// Cross-lane moves by DPP (a VALU operand modifier: no LDS round trip).
// Lanes whose source is outside the pattern, or whose row is masked out,
// receive `old`.
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ int dpp(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, kCtrl, kRowMask, 0xf, false);
}
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ double dpp(double old, double v) {
  return __hiloint2double(dpp<kCtrl, kRowMask>(__double2hiint(old), __double2hiint(v)),
                          dpp<kCtrl, kRowMask>(__double2loint(old), __double2loint(v)));
}
constexpr int kRowShr = 0x110;      // + n: row_shr:n (within rows of 16 lanes)
constexpr int kRowBcast15 = 0x142;  // lane 15 of a row to the whole next row
constexpr int kRowBcast31 = 0x143;  // lane 31 to rows 2 and 3
constexpr int kWaveShr1 = 0x138;    // lane i - 1 to lane i across the wave
constexpr int kWaveShl1 = 0x130;    // lane i + 1 to lane i across the wave

// One level of the segmented scan: add the value `kCtrl` brings in when it
// comes from the same segment.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ void seg_level(double &a, double &b, double &c, double &d, int seg) {
  const bool take = dpp<kCtrl, kRowMask>(-1, seg) == seg;        // segment ids are >= 1
  const double oa = dpp<kCtrl, kRowMask>(0.0, a), ob = dpp<kCtrl, kRowMask>(0.0, b);
  const double oc = dpp<kCtrl, kRowMask>(0.0, c), od = dpp<kCtrl, kRowMask>(0.0, d);
  if (take) {
    a += oa;
    b += ob;
    c += oc;
    d += od;
  }
}

// Inclusive scans of a, b, c, d over the lanes of the same segment (segment
// ids non-decreasing along the lanes, >= 1): shifts by 1, 2, 4 and 8 within
// rows of 16 lanes, then row 0's last lane into row 1 and row 2's into row
// 3, then lane 31 into rows 2 and 3.
__device__ __forceinline__ void seg_scan4(double &a, double &b, double &c, double &d, int seg) {
  seg_level<kRowShr + 1, 0xf>(a, b, c, d, seg);
  seg_level<kRowShr + 2, 0xf>(a, b, c, d, seg);
  seg_level<kRowShr + 4, 0xf>(a, b, c, d, seg);
  seg_level<kRowShr + 8, 0xf>(a, b, c, d, seg);
  seg_level<kRowBcast15, 0xa>(a, b, c, d, seg);
  seg_level<kRowBcast31, 0xc>(a, b, c, d, seg);
}

// The value of lane L (wave-uniform).
template <int L>
__device__ __forceinline__ double read_lane(double x) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), L);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), L);
  return __hiloint2double(hi, lo);
}

// kUpd: the residual kept in sorted order is first updated for changed
// source models (UpdateArgs, as k_update_sorted does, with the same sums),
// in the same pass: each lane updates its visibilities while the first
// source is extracted and the extraction reads the updated values.
template <bool kMixed, bool kUpd>
__global__ __launch_bounds__(256) void k_extract_vp(ExtractArgs a, const double4 *__restrict__ sgeo,
                                                    const void *__restrict__ squad, const void *sres,
                                                    const uint64_t *__restrict__ swt, double4 *__restrict__ acc,
                                                    UpdateArgs u) {
  __shared__ double2 tab[kMixed ? 1 : kCisTable];
  if (!kMixed) {
    cis_table_init(tab);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int64_t jw = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 * kVpSteps);
  if (jw >= a.sv.n_vis) return;                                  // uniform per wave
  for (int s = 0; s < a.n_src; ++s) {                              // uniform
    const SrcGeom g = a.geom[s];
    const int64_t base = g.base + (int64_t)g.half * (g.side + 1);
    const double half = (double)g.half, side = (double)g.side;
    // the open run carried between steps (wave-uniform)
    double ckey = kNoRun, cw = 0.0, cr = 0.0, ci = 0.0, cn = 0.0;
    for (int t = 0; t < kVpSteps; ++t) {
      const int64_t jb = jw + (int64_t)t * 64;
      if (jb >= a.sv.n_vis) break;                               // uniform
      const int64_t j = jb + lane;                               // < n_vis + 64: inside the padded arrays
      const uint64_t wb = swt[j];
      const bool use = j < a.sv.n_vis && wb != 0u;               // flagged and padding entries add nothing
      const double ww = use ? __longlong_as_double((long long)wb) : 0.0;
      const double4 gg = sgeo[j];
      double zr, zi;
      double xf, yf;
      if (!kMixed) {
        const double4 qg = reinterpret_cast<const double4 *>(squad)[j];
        double2 rg;
        if (kUpd && s == 0) {                                    // uniform
          rg = make_double2(0.0, 0.0);
          if (j < a.sv.n_vis) {
            const double2 ao = sum_f64(gg.x, gg.y, gg.z, u.old64, 0, u.n_old, tab);
            const double2 an = sum_f64(gg.x, gg.y, gg.z, u.new64, 0, u.n_new, tab);
            double2 r = u.rs[j];
            r = make_double2(fma(gg.w, ao.x, r.x), fma(gg.w, ao.y, r.y));
            r = make_double2(fma(-gg.w, an.x, r.x), fma(-gg.w, an.y, r.y));
            u.rs[j] = r;
            const double wpos = __longlong_as_double((long long)wb);
            rg = make_double2(wpos * r.x, wpos * r.y);
            reinterpret_cast<double2 *>(u.sv.res)[j] = rg;
          }
        } else {
          rg = reinterpret_cast<const double2 *>(sres)[j];
        }
        const SrcModel p = a.src[s];
        const double ph = fma(gg.x, p.l, fma(gg.y, p.m, gg.z * p.n1));
        const double2 cs = cis2pi_f64(ph, tab);
        const double x = fma(p.q11, qg.x, fma(p.q12x2, qg.y, fma(p.q22, qg.z, 1.0)));
        const double own = (kPowM32Scale * p.flux) * pow_m32_f64(x);
        // w z = (w R) exp(-2 pi i ph) + (w spec) own
        zr = fma(rg.x, cs.x, fma(rg.y, cs.y, qg.w * own));
        zi = fma(rg.y, cs.x, -rg.x * cs.y);
        xf = rint(__dmul_rn(gg.x, p.theta));
        yf = rint(__dmul_rn(gg.y, p.theta));
      } else {
        const float4 qg = reinterpret_cast<const float4 *>(squad)[j];
        float2 rg = reinterpret_cast<const float2 *>(sres)[j];
        if (kUpd && s == 0 && j < a.sv.n_vis) {                  // uniform source test
          const float2 ao = sum_mixed(gg.x, gg.y, gg.z, u.old32, 0, u.n_old);
          const float2 an = sum_mixed(gg.x, gg.y, gg.z, u.new32, 0, u.n_new);
          const float sp = (float)gg.w;
          rg = make_float2(fmaf(sp, ao.x, rg.x), fmaf(sp, ao.y, rg.y));
          rg = make_float2(fmaf(-sp, an.x, rg.x), fmaf(-sp, an.y, rg.y));
          reinterpret_cast<float2 *>(u.sv.res)[j] = rg;
        }
        const SrcMixed p = a.src32[s];
        const double ph = fma(gg.x, p.l, fma(gg.y, p.m, gg.z * p.n1));
        const float tt = (float)__builtin_amdgcn_fract(ph);
        const float sn = __builtin_amdgcn_sinf(tt), cs = __builtin_amdgcn_cosf(tt);
        float fr = fmaf(rg.x, cs, rg.y * sn);
        const float fi = fmaf(rg.y, cs, -(rg.x * sn));
        const float x = fmaf(p.q11, qg.x, fmaf(p.q12x2, qg.y, fmaf(p.q22, qg.z, 1.0f)));
        const float qr = __builtin_amdgcn_rsqf(x);
        fr = fmaf(qg.w * p.flux, qr * qr * qr, fr);
        zr = ww * (double)fr;
        zi = ww * (double)fi;
        xf = rint(__dmul_rn(gg.x, p.theta));
        yf = rint(__dmul_rn(gg.y, p.theta));
      }
      const bool inb = fabs(xf) <= half && fabs(yf) <= half;
      if (use && !inb) atomicOr(a.err, 1u);
      const bool on = use && inb;
      const double key = on ? fma(yf, side, xf) : kNoRun;
      double vw = on ? ww : 0.0, vr = on ? zr : 0.0, vi = on ? zi : 0.0, vn = on ? 1.0 : 0.0;
      // the carried run continues into lane 0's cell, or is closed now
      if (ckey != kNoRun) {                                      // uniform
        if (read_lane<0>(key) == ckey) {
          if (lane == 0) {
            vw += cw;
            vr += cr;
            vi += ci;
            vn += cn;
          }
        } else if (lane == 0) {
          double *c = &acc[base + (int32_t)ckey].x;
          unsafeAtomicAdd(c, cw);
          unsafeAtomicAdd(c + 1, cr);
          unsafeAtomicAdd(c + 2, ci);
          unsafeAtomicAdd(c + 3, cn);
        }
      }
      // segments: runs of equal keys along the lanes
      const double prev = dpp<kWaveShr1>(key, key);
      const bool head = lane == 0 || prev != key;
      const int seg = __popcll(__ballot(head) & (((uint64_t)2 << lane) - 1));
      seg_scan4(vw, vr, vi, vn, seg);
      const int next = dpp<kWaveShl1>(-1, seg);
      if (lane < 63 && next != seg && on) {                      // a run that ends inside this step
        double *c = &acc[base + (int32_t)key].x;
        unsafeAtomicAdd(c, vw);
        unsafeAtomicAdd(c + 1, vr);
        unsafeAtomicAdd(c + 2, vi);
        unsafeAtomicAdd(c + 3, vn);
      }
      // the run reaching lane 63 stays open
      ckey = read_lane<63>(key);
      cw = read_lane<63>(vw);
      cr = read_lane<63>(vr);
      ci = read_lane<63>(vi);
      cn = read_lane<63>(vn);
    }
    if (ckey != kNoRun && lane == 0) {
      double *c = &acc[base + (int32_t)ckey].x;
      unsafeAtomicAdd(c, cw);
      unsafeAtomicAdd(c + 1, cr);
      unsafeAtomicAdd(c + 2, ci);
      unsafeAtomicAdd(c + 3, cn);
    }
  }
}

// Resident blocks of an extraction kernel on the current device (cached).
template <class K>
int64_t resident_blocks(K kernel, int slot, int threads) {
  static int64_t cache[3][16] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 0;
  if (!cache[slot][dev]) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    cache[slot][dev] = (int64_t)per_cu * cus;
  }
  return cache[slot][dev];
}

// Visibilities per wave: near a nominal 2048, sized so the grid is a whole
// number of rounds of resident blocks (a last round nearly empty would leave
// the chip idle for a whole block's duration).
int64_t chunk_size(int64_t n_vis, int64_t bpc, int64_t capacity) {
  constexpr int64_t kNominal = 2048, kMin = 256;
  auto blocks = [&](int64_t chunk) { return ((n_vis + chunk - 1) / chunk + kXcd - 1) / kXcd * kXcd * bpc; };
  if (capacity <= 0 || n_vis <= 0) return kNominal;
  const int64_t b0 = blocks(kNominal);
  const int64_t rounds = std::max<int64_t>(1, (b0 + capacity / 2) / capacity);
  const int64_t max_chunks = std::max<int64_t>(kXcd, (rounds * capacity / bpc) / kXcd * kXcd);
  return std::max(kMin, (n_vis + max_chunks - 1) / max_chunks);
}

}  // namespace

hipError_t launch_extract(const ExtractArgs &a0, int mixed, hipStream_t st, const UpdateArgs *upd) {
  const int ns = mixed ? kNsMixed : kNsF64;
  ExtractArgs a = a0;
  const Sorted &v = a.sv;
  const uint64_t *wt = reinterpret_cast<const uint64_t *>(v.wt);
  // the update is fused only for one changed source (a serial refinement):
  // more sources' sums in the first source's pass lengthen the extraction's
  // latency-bound steps by more than the separate pass costs
  const bool fuse = upd && a.n_src <= kVpSources && upd->n_old <= 1 && upd->n_new <= 1;
  if (upd && !fuse) {
    hipError_t e = launch_update_sorted(*upd, mixed, st);
    if (e != hipSuccess) return e;
  }
  if (a.n_src <= kVpSources) {
    const int64_t waves = (v.n_vis + 64 * kVpSteps - 1) / (64 * kVpSteps);
    const dim3 grid((unsigned)((waves + 3) / 4));
    UpdateArgs u = fuse ? *upd : UpdateArgs{};
    if (fuse) {
      if (mixed)
        hipLaunchKernelGGL((k_extract_vp<true, true>), grid, dim3(256), 0, st, a, v.geo, v.quad, v.res, wt, a.acc.cell, u);
      else
        hipLaunchKernelGGL((k_extract_vp<false, true>), grid, dim3(256), 0, st, a, v.geo, v.quad, v.res, wt, a.acc.cell, u);
    } else {
      if (mixed)
        hipLaunchKernelGGL((k_extract_vp<true, false>), grid, dim3(256), 0, st, a, v.geo, v.quad, v.res, wt, a.acc.cell, u);
      else
        hipLaunchKernelGGL((k_extract_vp<false, false>), grid, dim3(256), 0, st, a, v.geo, v.quad, v.res, wt, a.acc.cell, u);
    }
    return hipGetLastError();
  }
  a.n_tiles = (a.n_src + 64 * ns - 1) / (64 * ns);
  const bool big = !mixed && a.n_tiles >= kBigTableTiles;
  const int waves = big ? waves_per_block<false, 2048>() : kWaves;
  const int64_t bpc = (a.n_tiles + waves - 1) / waves;
  auto kmixed = k_extract<true, kNsMixed, kGroupMixed, 1024>;   // (T unused: no table)
  auto kf64 = k_extract<false, kNsF64, kGroupF64, 1024>;
  auto kf64big = k_extract<false, kNsF64, kGroupF64, 2048>;
  const int64_t capacity = mixed ? resident_blocks(kmixed, 1, 64 * kWaves)
                                 : (big ? resident_blocks(kf64big, 2, 64 * waves) : resident_blocks(kf64, 0, 64 * kWaves));
  a.chunk = (int32_t)chunk_size(v.n_vis, bpc, capacity);
  a.n_chunks = (v.n_vis + a.chunk - 1) / a.chunk;
  const int64_t blocks = ((a.n_chunks + kXcd - 1) / kXcd) * kXcd * bpc;
  auto kern = mixed ? kmixed : (big ? kf64big : kf64);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves), 0, st, a, v.geo, v.quad, v.res, wt, a.acc.cell);
  return hipGetLastError();
}

}  // namespace rlf
