// Likelihood grid (Sec. 2.4): for each source, ellipticity grid point e and
// scale-length knot alpha_k,
//   f_c = (1 + s_k q_c(e))^{-3/2},  q_c(e) = |A_e^{-T} k_c|^2,  s_k = 4 pi^2 alpha_k^2,
//   D_k = sum_c W_c f_c Re Vbar_c,  M_k = sum_c W_c f_c^2,
//   ln L(e, alpha_k) = D_k^2 / (2 M_k) - ln(M_k) / 2            (flux marginalised)
//   ln L(e) = m + ln sum_k exp(ln w_k + ln L(e, alpha_k) - m)   (scale marginalised)
//
// One thread per grid point, all knots of that point in registers (D_k, M_k),
// a uniform loop over the source's cells: each cell record comes in through
// one scalar load shared by the wave; it carries sqrt(W_c) in the profile's
// scale, (W^{-1/6} uc, W^{-1/6} vc, W^{-1/3}, sqrt(W) Re Vbar), so that
// h = (W^{-1/3} + s_k q')^{-3/2} = sqrt(W_c) f_c (q' the quadratic form of the
// scaled centre).  Per (cell, point) the quadratic form costs 6 ops and
// serves all knots; per (cell, point, knot): 1 FMA, x^(-3/2), 2 FMAs
// (D += b h, M += h h).
//   FP64 form:  x^(-3/2) as v_rsq_f64 cubed with a first-order correction
//               (5 ops, relative error < 3e-14), computed as (2/3) x^(-3/2).
//   Mixed form: FP32 cell data and arithmetic (v_rsq_f32 cubed), partial sums of
//               each block of kBlock cells folded into FP64 totals, so the
//               FP32 rounding error grows with kBlock, not with the cell count.
// The epilogue (logs, exps, log-sum-exp over knots) is FP64 in both forms.
//
// Position marginalisation (Sec. 2.4; n_pos offsets x_p on a square grid,
// uniform prior): D is formed per offset from the cross-correlation data
// G[c, p] = sqrt(W_c) Re(Vbar_c exp(-2 pi i k_c.x_p)) and M is shared,
//   ln L(e) = ln sum_k w_k (1/n_pos) sum_p exp(D_kp^2 / (2 M_k) - ln(M_k) / 2).
// The knots run in blocks of KB with the KB * n_pos sums of a block in
// registers; the n_pos values of a cell come in through scalar loads (one
// row of G per cell, G carrying sqrt(W_c) as the records do: the profile
// term h is sqrt(W_c) f_c), so a (cell, point, knot) costs the profile (6
// ops), M (1) and one FMA per offset, plus the quadratic form once per knot
// block.
#include "rlf_cellsums.h"
#include "rlf_devmath.h"
#include "rlf_internal.h"

namespace rlf {

namespace {

constexpr int kBlock = kCellBlock;
constexpr double kLnPowM32Scale = 0.40546510810816438198;   // ln(3/2)

// Knots per pass over the cells: the mixed form with 20 knots takes them in
// two passes of 10 (the quadratic form is formed twice per cell, but half
// the accumulators leave room for twice the resident waves: measured 6 %
// faster); the FP64 form is faster in one pass.
template <int R, bool kMixed>
constexpr int knots_per_pass() { return (kMixed && R == 20) ? 10 : R; }

// ln L(e) of source s at (e1, e2), |e| < 1; NaN for an empty facet.
template <int R, bool kExact, bool kMixed>
__device__ __forceinline__ double loglike_e(const FitArgs &a, int num_r_arg, int s, double e1, double e2) {
  constexpr int KP = knots_per_pass<R, kMixed>();
  const int num_r = kExact ? R : num_r_arg;
  const double det = 1.0 - e1 * e1 - e2 * e2;
  const double g = 1.0 / (det * det);
  const int64_t c0 = a.offsets[s], c1 = a.offsets[s + 1];
  if (c1 == c0) return NAN;
  const double *lw = a.logw + (int64_t)s * a.num_r;
  double mx = -INFINITY, acc = 0.0;
#pragma unroll 1
  for (int k0 = 0; k0 < R; k0 += KP) {
    if (k0 >= num_r) break;
    double D[KP], M[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) D[k] = M[k] = 0.0;
    if (!kMixed) {
      // A^{-T} with its 1/det folded in, so that the knot scales s_k stay
      // wave-uniform (SGPR operands: 40 VGPRs fewer than per-lane s_k g)
      const double id = 1.0 / det;
      const double a11 = (1.0 + e1) * id, a12 = e2 * id, a22 = (1.0 - e1) * id;
      double sk[KP];
#pragma unroll
      for (int k = 0; k < KP; ++k) sk[k] = k0 + k < num_r ? a.sk[k0 + k] : 0.0;
      cell_sums_f64<KP>(a.fit64, c0, c1, a11, a12, a22, sk, num_r - k0, D, M);
    } else {
      const float a11 = (float)(1.0 + e1), a12 = (float)e2, a22 = (float)(1.0 - e1);
      float sk[KP];
#pragma unroll
      for (int k = 0; k < KP; ++k) sk[k] = k0 + k < num_r ? (float)(a.sk[k0 + k] * g) : 0.0f;
      cell_sums_f32<KP>(a.fit32, c0, c1, a11, a12, a22, sk, num_r - k0, D, M);
    }
    // ln(w_k L(e, alpha_k)) in place of D; FP64 form: D and M carry (2/3)
    // and (4/9) of their values, so the ratio term is unchanged and ln M is
    // off by ln(4/9) = -2 ln(3/2)
    double bm = -INFINITY;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      if (k0 + k < num_r) {
        D[k] = lw[k0 + k] + (D[k] * D[k] / (2.0 * M[k]) - 0.5 * log(M[k]) - (kMixed ? 0.0 : kLnPowM32Scale));
        bm = fmax(bm, D[k]);
      }
    }
    const double nm = fmax(mx, bm);
    double bs = 0.0;
#pragma unroll
    for (int k = 0; k < KP; ++k)
      if (k0 + k < num_r) bs += exp(D[k] - nm);
    acc = (mx > -INFINITY ? acc * exp(mx - nm) : 0.0) + bs;
    mx = nm;
  }
  return mx + log(acc);
}

// Knots per block of the position-marginalised sum: KB * NP partial sums
// in registers (FP64, plus as many FP32 ones in the mixed form).
constexpr int pos_knot_block(int np) { return np <= 9 ? 4 : (np <= 25 ? 2 : 1); }

// Position-marginalised ln L(e) of source s at (e1, e2), |e| < 1; NaN for an
// empty facet.
template <int NP, bool kMixed>
__device__ __forceinline__ double loglike_pos(const FitArgs &a, int num_r, int s, double e1, double e2) {
  constexpr int KB = pos_knot_block(NP);
  const double det = 1.0 - e1 * e1 - e2 * e2;
  const double g = 1.0 / (det * det);
  const int64_t c0 = a.offsets[s], c1 = a.offsets[s + 1];
  if (c1 == c0) return NAN;
  const double *lw = a.logw + (int64_t)s * a.num_r;
  double mx = -INFINITY, acc = 0.0;
  for (int k0 = 0; k0 < num_r; k0 += KB) {
    double D[KB][NP], M[KB];
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      M[b] = 0.0;
#pragma unroll
      for (int p = 0; p < NP; ++p) D[b][p] = 0.0;
    }
    if (!kMixed) {
      const double a11 = 1.0 + e1, a12 = e2, a22 = 1.0 - e1;
      double sk[KB];
#pragma unroll
      for (int b = 0; b < KB; ++b) sk[b] = k0 + b < num_r ? a.sk[k0 + b] * g : 0.0;
      const double4 *__restrict__ cells = a.fit64;
      const double *__restrict__ G = a.pos_g64;
      for (int64_t c = c0; c < c1; ++c) {
        const double4 cl = cells[c];
        const double ku = fma(a11, cl.x, a12 * cl.y);
        const double kv = fma(a12, cl.x, a22 * cl.y);
        const double q = fma(ku, ku, kv * kv);
        const double *gc = G + c * NP;
#pragma unroll
        for (int b = 0; b < KB; ++b) {
          const double f = pow_m32_f64(fma(sk[b], q, cl.z));        // (2/3) sqrt(W) f_c
          M[b] = fma(f, f, M[b]);
#pragma unroll
          for (int p = 0; p < NP; ++p) D[b][p] = fma(f, gc[p], D[b][p]);
        }
      }
    } else {
      const float a11 = (float)(1.0 + e1), a12 = (float)e2, a22 = (float)(1.0 - e1);
      float sk[KB];
#pragma unroll
      for (int b = 0; b < KB; ++b) sk[b] = k0 + b < num_r ? (float)(a.sk[k0 + b] * g) : 0.0f;
      const float4 *__restrict__ cells = a.fit32;
      const float *__restrict__ G = a.pos_g32;
      auto block = [&](int64_t cb, int n) {
        float d[KB][NP], m[KB];
#pragma unroll
        for (int b = 0; b < KB; ++b) {
          m[b] = 0.0f;
#pragma unroll
          for (int p = 0; p < NP; ++p) d[b][p] = 0.0f;
        }
        for (int t = 0; t < n; ++t) {
          const float4 cl = cells[cb + t];
          const float ku = fmaf(a11, cl.x, a12 * cl.y);
          const float kv = fmaf(a12, cl.x, a22 * cl.y);
          const float q = fmaf(ku, ku, kv * kv);
          const float *gc = G + (cb + t) * NP;
#pragma unroll
          for (int b = 0; b < KB; ++b) {
            const float r = __builtin_amdgcn_rsqf(fmaf(sk[b], q, cl.z));
            const float f = r * r * r;                                // sqrt(W) f_c
            m[b] = fmaf(f, f, m[b]);
#pragma unroll
            for (int p = 0; p < NP; ++p) d[b][p] = fmaf(f, gc[p], d[b][p]);
          }
        }
#pragma unroll
        for (int b = 0; b < KB; ++b) {
          M[b] += (double)m[b];
#pragma unroll
          for (int p = 0; p < NP; ++p) D[b][p] += (double)d[b][p];
        }
      };
      int64_t cb = c0;
#pragma clang loop unroll(disable)
      for (; cb + kBlock <= c1; cb += kBlock) block(cb, kBlock);
      if (cb < c1) block(cb, (int)(c1 - cb));
    }
    // ln(w_k L(e, alpha_k, x_p)) in place of D, then one rescaling of the
    // running sum per block
    double bm = -INFINITY;
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      if (k0 + b < num_r) {
        const double base = lw[k0 + b] - 0.5 * log(M[b]) - (kMixed ? 0.0 : kLnPowM32Scale);
        const double h = 1.0 / (2.0 * M[b]);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          D[b][p] = fma(D[b][p] * D[b][p], h, base);
          bm = fmax(bm, D[b][p]);
        }
      }
    }
    const double nm = fmax(mx, bm);
    double bs = 0.0;
#pragma unroll
    for (int b = 0; b < KB; ++b)
      if (k0 + b < num_r) {
#pragma unroll
        for (int p = 0; p < NP; ++p) bs += exp(D[b][p] - nm);
      }
    acc = (mx > -INFINITY ? acc * exp(mx - nm) : 0.0) + bs;
    mx = nm;
  }
  return mx + log(acc / (double)NP);
}

// ln L(e): position fixed (NP = 0) or marginalised over NP offsets.
template <int R, bool kExact, bool kMixed, int NP>
__device__ __forceinline__ double loglike(const FitArgs &a, int num_r, int s, double e1, double e2) {
  if constexpr (NP == 0)
    return loglike_e<R, kExact, kMixed>(a, num_r, s, e1, e2);
  else
    return loglike_pos<NP, kMixed>(a, num_r, s, e1, e2);
}

// ln L(e) at valid grid point j (index into the valid-point list) of source s.
template <int R, bool kExact, bool kMixed, int NP = 0>
__device__ __forceinline__ void eval_point(const FitArgs &a, int num_r, int s, int j) {
  const int idx = a.epts[j];
  const int i1 = idx / a.n_e, i2 = idx - (idx / a.n_e) * a.n_e;
  const int ctr = (a.n_e - 1) / 2;
  a.lsurf[(int64_t)s * a.n_valid + j] =
      loglike<R, kExact, kMixed, NP>(a, num_r, s, (double)(i1 - ctr) * a.e_step, (double)(i2 - ctr) * a.e_step);
}

// Refinement level: one thread per point of the source's window at
// resolution e_step / 2^level, e = k * that step, |e| < 1 tested on the
// integers; -inf outside the domain.
template <int R, bool kExact, bool kMixed, int NP = 0>
__global__ __launch_bounds__(256) void k_refine_eval(FitArgs a, RefineArgs r, int num_r) {
  const int s = blockIdx.y;
  const int32_t *w = r.win + (int64_t)s * 5;
  if (!w[0]) return;
  const int n1 = w[3], n2 = w[4];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n1 * n2) return;
  const int64_t k1 = w[1] + t / n2, k2 = w[2] + t % n2;
  const int64_t lim = (int64_t)r.unit << r.level;
  double *out = r.lloc + (int64_t)s * r.max_side * r.max_side + t;
  if (k1 * k1 + k2 * k2 >= lim * lim) {
    *out = -INFINITY;
    return;
  }
  const double res = a.e_step / (double)(1 << r.level);
  *out = loglike<R, kExact, kMixed, NP>(a, num_r, s, (double)k1 * res, (double)k2 * res);
}


// Grid launch: blockIdx.y = source (largest facets first when a.size_order
// is set: blocks are dispatched in index order, and the long blocks of the
// largest facets then do not trail the launch), one thread per valid grid
// point.
template <int R, bool kExact, bool kMixed, int NP = 0>
__global__ __launch_bounds__(256) void k_fit(FitArgs a, int num_r) {
  const int s = a.size_order ? a.size_order[a.n_src - 1 - (int)blockIdx.y] : (int)blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_valid) return;
  if (a.redo && !a.redo[s]) return;
  eval_point<R, kExact, kMixed, NP>(a, num_r, s, j);
}

// Few sources (FP64 form, position fixed, R knots in one pass): the grid of
// one source is only ~100 waves, each walking all of the source's cells, so
// the cells are cut into a.parts ranges (blockIdx.z), each thread writes its
// range's D_k and M_k, and k_fit_join adds the ranges in order and forms
// ln L(e) as loglike_e does.
template <int R>
__global__ __launch_bounds__(256) void k_fit_part(FitArgs a) {
  const int s = blockIdx.y, part = blockIdx.z;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_valid) return;
  if (a.redo && !a.redo[s]) return;
  const int64_t c0 = a.offsets[s], c1 = a.offsets[s + 1];
  const int64_t len = (c1 - c0 + a.parts - 1) / a.parts;
  const int64_t cb = min(c1, c0 + part * len), ce = min(c1, cb + len);
  const int idx = a.epts[j];
  const int i1 = idx / a.n_e, i2 = idx - (idx / a.n_e) * a.n_e;
  const int ctr = (a.n_e - 1) / 2;
  const double e1 = (double)(i1 - ctr) * a.e_step, e2 = (double)(i2 - ctr) * a.e_step;
  const double det = 1.0 - e1 * e1 - e2 * e2;
  const double g = 1.0 / (det * det);
  double D[R], M[R], sk[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    D[k] = M[k] = 0.0;
    sk[k] = a.sk[k] * g;
  }
  cell_sums_f64<R>(a.fit64, cb, ce, 1.0 + e1, e2, 1.0 - e1, sk, R, D, M);
  double *out = a.part_sums + ((int64_t)s * a.parts + part) * (2 * R) * a.n_valid + j;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    out[(int64_t)k * a.n_valid] = D[k];
    out[(int64_t)(R + k) * a.n_valid] = M[k];
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_fit_join(FitArgs a) {
  const int s = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_valid) return;
  if (a.redo && !a.redo[s]) return;
  double *dst = a.lsurf + (int64_t)s * a.n_valid + j;
  if (a.offsets[s + 1] == a.offsets[s]) {
    *dst = NAN;
    return;
  }
  double D[R], M[R];
#pragma unroll
  for (int k = 0; k < R; ++k) D[k] = M[k] = 0.0;
  for (int part = 0; part < a.parts; ++part) {
    const double *in = a.part_sums + ((int64_t)s * a.parts + part) * (2 * R) * a.n_valid + j;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      D[k] += in[(int64_t)k * a.n_valid];
      M[k] += in[(int64_t)(R + k) * a.n_valid];
    }
  }
  const double *lw = a.logw + (int64_t)s * a.num_r;
  double bm = -INFINITY;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    D[k] = lw[k] + (D[k] * D[k] / (2.0 * M[k]) - 0.5 * log(M[k]) - kLnPowM32Scale);
    bm = fmax(bm, D[k]);
  }
  double bs = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k) bs += exp(D[k] - bm);
  *dst = bm + log(bs);
}

// Windowed launch: blockIdx.y = source, one thread per position of the
// source's inclusive box (i1lo, i1hi, i2lo, i2hi) in row-major order, then,
// with a check stride S, per lattice point c + S q (both axes, |q| <= c / S)
// outside the box; invalid points (|e| >= 1) are skipped.  No other point is
// evaluated (the estimator reads no other).  Blocks past a source's positions
// leave at once, so the grid is sized for the largest possible box.  Sources
// largest facet first, as in k_fit.
template <int R, bool kExact, bool kMixed>
__global__ __launch_bounds__(256) void k_fit_window(FitArgs a, int num_r) {
  const int s = a.size_order ? a.size_order[a.n_src - 1 - (int)blockIdx.y] : (int)blockIdx.y;
  // lattice pass 1: the lattice alone (an empty box); pass 2: the lattice
  // values are already in the surface, only the box is evaluated
  int4 b = a.lattice_pass == 1 ? make_int4(1, 0, 1, 0) : reinterpret_cast<const int4 *>(a.window)[s];
  b.x = max(b.x, 0);                          // the box's part on the grid: at most n_e^2 positions
  b.y = min(b.y, a.n_e - 1);
  b.z = max(b.z, 0);
  b.w = min(b.w, a.n_e - 1);
  const int w2 = b.w >= b.z ? b.w - b.z + 1 : 1;
  const int area = (b.y >= b.x && b.w >= b.z) ? (b.y - b.x + 1) * w2 : 0;
  const int ctr = (a.n_e - 1) / 2;
  const int h = a.check_stride > 0 ? ctr / a.check_stride : 0;
  const int nl = (a.check_stride > 0 && a.lattice_pass != 2) ? 2 * h + 1 : 0;
  // a box with at least as many positions as the grid has valid points is
  // walked over the valid points instead (no idle lanes on |e| >= 1)
  const bool by_valid = area >= a.n_valid;
  const int span = by_valid ? a.n_valid : area;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= span + nl * nl) return;
  int i1, i2;
  if (by_valid && t < span) {
    const int f = a.epts[t];
    i1 = f / a.n_e;
    i2 = f - i1 * a.n_e;
    if (i1 >= b.x && i1 <= b.y && i2 >= b.z && i2 <= b.w) eval_point<R, kExact, kMixed>(a, num_r, s, t);
    return;
  }
  if (t < span) {
    i1 = b.x + t / w2;
    i2 = b.z + t % w2;
  } else {
    const int u = t - span;
    i1 = ctr + a.check_stride * (u / nl - h);
    i2 = ctr + a.check_stride * (u % nl - h);
    if (i1 >= b.x && i1 <= b.y && i2 >= b.z && i2 <= b.w) return;   // evaluated with the box
  }
  if (i1 < 0 || i2 < 0 || i1 >= a.n_e || i2 >= a.n_e) return;
  const int j = a.valid_index[i1 * a.n_e + i2];
  if (j >= 0) eval_point<R, kExact, kMixed>(a, num_r, s, j);
}

// Persistent work queue: a grid sized to the resident capacity; each wave
// claims items with one atomic; item -> (rank, piece) by binary search of the
// per-rank item offsets; a rank is a source (ranks ordered by decreasing cell
// count, so the longest items go first), a piece is tile*64 consecutive valid
// grid points.  Every wave leaves when the counter passes the item count.
template <int R, bool kExact, bool kMixed>
__global__ __launch_bounds__(256) void k_fit_queue(FitArgs a, QueueArgs q, int num_r) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    uint32_t item = 0;
    if (lane == 0) item = atomicAdd(q.counter, 1u);
    item = __shfl(item, 0);
    if ((int64_t)item >= q.n_items) break;
    int lo = 0, hi = q.n_rank;                          // item_start[lo] <= item < item_start[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (q.item_start[mid] <= (int64_t)item) lo = mid;
      else hi = mid;
    }
    const int s = q.order[lo];
    const int tile = q.tile[lo];
    const int64_t piece = (int64_t)item - q.item_start[lo];
    for (int t = 0; t < tile; ++t) {
      const int64_t j = (piece * tile + t) * 64 + lane;
      if (j < a.n_valid) eval_point<R, kExact, kMixed>(a, num_r, s, (int)j);
    }
  }
}

// Window seeded by the stride-S lattice (after lattice pass 1): per source,
// the bounding box of the lattice points within the threshold of the lattice
// maximum, widened by S grid steps and clamped to the grid; the whole grid
// for an empty facet.  One wave per source.
__global__ __launch_bounds__(256) void k_lattice_windows(FitArgs a, double log_frac, int32_t *win) {
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= a.n_src) return;                                      // uniform per wave
  int4 *w = reinterpret_cast<int4 *>(win) + s;
  const int S = a.check_stride, ctr = (a.n_e - 1) / 2, h = ctr / S, nl = 2 * h + 1;
  const double *L = a.lsurf + (int64_t)s * a.n_valid;
  double best = -INFINITY;
  if (a.offsets[s + 1] > a.offsets[s]) {
    for (int u = lane; u < nl * nl; u += 64) {
      const int j = a.valid_index[(ctr + S * (u / nl - h)) * a.n_e + ctr + S * (u % nl - h)];
      if (j >= 0) best = fmax(best, L[j]);
    }
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) best = fmax(best, __shfl_xor(best, d));
  if (!(best > -INFINITY)) {
    if (lane == 0) *w = make_int4(0, a.n_e - 1, 0, a.n_e - 1);
    return;
  }
  const double thr = best + log_frac;
  int lo1 = a.n_e, hi1 = -1, lo2 = a.n_e, hi2 = -1;
  for (int u = lane; u < nl * nl; u += 64) {
    const int i1 = ctr + S * (u / nl - h), i2 = ctr + S * (u % nl - h);
    const int j = a.valid_index[i1 * a.n_e + i2];
    if (j >= 0 && L[j] >= thr) {
      lo1 = min(lo1, i1);
      hi1 = max(hi1, i1);
      lo2 = min(lo2, i2);
      hi2 = max(hi2, i2);
    }
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    lo1 = min(lo1, __shfl_xor(lo1, d));
    hi1 = max(hi1, __shfl_xor(hi1, d));
    lo2 = min(lo2, __shfl_xor(lo2, d));
    hi2 = max(hi2, __shfl_xor(hi2, d));
  }
  if (lane == 0)
    *w = make_int4(max(lo1 - S, 0), min(hi1 + S, a.n_e - 1), max(lo2 - S, 0), min(hi2 + S, a.n_e - 1));
}

__global__ void k_reset_counter(uint32_t *c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0u;
}

#define RLF_FIT_DISPATCH(KERNEL, GRID, ...)                                                         \
  do {                                                                                              \
    if (a.num_r == 20)                                                                              \
      hipLaunchKernelGGL((KERNEL<20, true, kMixed>), GRID, dim3(256), 0, st, __VA_ARGS__, 20);     \
    else if (a.num_r == 23)                                                                         \
      hipLaunchKernelGGL((KERNEL<23, true, kMixed>), GRID, dim3(256), 0, st, __VA_ARGS__, 23);     \
    else if (a.num_r <= 8)                                                                          \
      hipLaunchKernelGGL((KERNEL<8, false, kMixed>), GRID, dim3(256), 0, st, __VA_ARGS__, a.num_r); \
    else                                                                                            \
      hipLaunchKernelGGL((KERNEL<kMaxKnots, false, kMixed>), GRID, dim3(256), 0, st, __VA_ARGS__,  \
                         a.num_r);                                                                  \
  } while (0)

// Position-marginalised launches: the offset count selects the kernel (the
// knot count is a run-time bound there).
#define RLF_POS_DISPATCH(KERNEL, GRID, ...)                                                             \
  do {                                                                                                  \
    if (a.n_pos == 9)                                                                                   \
      hipLaunchKernelGGL((KERNEL<1, false, kMixed, 9>), GRID, dim3(256), 0, st, __VA_ARGS__, a.num_r);  \
    else if (a.n_pos == 25)                                                                             \
      hipLaunchKernelGGL((KERNEL<1, false, kMixed, 25>), GRID, dim3(256), 0, st, __VA_ARGS__, a.num_r); \
    else if (a.n_pos == 49)                                                                             \
      hipLaunchKernelGGL((KERNEL<1, false, kMixed, 49>), GRID, dim3(256), 0, st, __VA_ARGS__, a.num_r); \
    else                                                                                                \
      return hipErrorInvalidValue;                                                                      \
  } while (0)

template <bool kMixed>
hipError_t launch(const FitArgs &a, hipStream_t st) {
  if (a.n_pos) {
    if (a.window || a.lattice_pass) return hipErrorInvalidValue;   // full grid only
    RLF_POS_DISPATCH(k_fit, dim3((a.n_valid + 255) / 256, a.n_src), a);
  } else if (a.window || a.lattice_pass == 1) {
    const int h = a.check_stride > 0 ? ((a.n_e - 1) / 2) / a.check_stride : 0;
    const int lattice = (a.check_stride > 0 && a.lattice_pass != 2) ? (2 * h + 1) * (2 * h + 1) : 0;
    const int positions = (a.lattice_pass == 1 ? 0 : a.n_e * a.n_e) + lattice;
    RLF_FIT_DISPATCH(k_fit_window, dim3((positions + 255) / 256, a.n_src), a);
  } else if (!kMixed && a.parts > 1 && a.num_r == 20) {
    const unsigned bx = (unsigned)((a.n_valid + 255) / 256);
    hipLaunchKernelGGL(k_fit_part<20>, dim3(bx, a.n_src, a.parts), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_fit_join<20>, dim3(bx, a.n_src), dim3(256), 0, st, a);
  } else {
    RLF_FIT_DISPATCH(k_fit, dim3((a.n_valid + 255) / 256, a.n_src), a);
  }
  return hipGetLastError();
}

template <bool kMixed>
hipError_t launch_q(const FitArgs &a, const QueueArgs &q, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, q.counter);
  RLF_FIT_DISPATCH(k_fit_queue, dim3(blocks), a, q);
  return hipGetLastError();
}

template <bool kMixed>
int queue_blocks_per_cu(int num_r) {
  int n = 0;
  hipError_t e;
  if (num_r == 20) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fit_queue<20, true, kMixed>, 256, 0);
  else if (num_r == 23) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fit_queue<23, true, kMixed>, 256, 0);
  else if (num_r <= 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fit_queue<8, false, kMixed>, 256, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fit_queue<kMaxKnots, false, kMixed>, 256, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

hipError_t launch_fit_f64(const FitArgs &a, hipStream_t st) { return launch<false>(a, st); }
hipError_t launch_fit_mixed(const FitArgs &a, hipStream_t st) { return launch<true>(a, st); }

hipError_t launch_refine_eval(const FitArgs &a, const RefineArgs &r, int mixed, hipStream_t st) {
  const dim3 grid((r.max_side * r.max_side + 255) / 256, a.n_src);
  if (mixed) {
    constexpr bool kMixed = true;
    if (a.n_pos)
      RLF_POS_DISPATCH(k_refine_eval, grid, a, r);
    else
      RLF_FIT_DISPATCH(k_refine_eval, grid, a, r);
  } else {
    constexpr bool kMixed = false;
    if (a.n_pos)
      RLF_POS_DISPATCH(k_refine_eval, grid, a, r);
    else
      RLF_FIT_DISPATCH(k_refine_eval, grid, a, r);
  }
  return hipGetLastError();
}

hipError_t launch_lattice_windows(const FitArgs &a, double log_frac, int32_t *win, hipStream_t st) {
  if (a.check_stride < 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lattice_windows, dim3((a.n_src + 3) / 4), dim3(256), 0, st, a, log_frac, win);
  return hipGetLastError();
}

hipError_t launch_fit_queue(const FitArgs &a, const QueueArgs &q, int mixed, int blocks, hipStream_t st) {
  return mixed ? launch_q<true>(a, q, blocks, st) : launch_q<false>(a, q, blocks, st);
}

int fit_queue_blocks_per_cu(int mixed, int num_r) {
  return mixed ? queue_blocks_per_cu<true>(num_r) : queue_blocks_per_cu<false>(num_r);
}

}  // namespace rlf
