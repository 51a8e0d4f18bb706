// Internal types shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlf.h"

namespace rlf {

constexpr int kMaxChan = 64;
constexpr int kMaxKnots = 32;
constexpr int kMaxHalf = 32767;

// Per-source constants of the visibility model (Eq. 1), packed so one
// 64-byte scalar load brings a source into SGPRs: every lane of a wave works
// on the same source at the same time.
struct alignas(64) SrcModel {
  double l, m, n1;           // direction cosines; n1 = sqrt(1-l^2-m^2)-1
  double flux;               // S at the reference frequency
  double q11, q12x2, q22;    // 4 pi^2 alpha^2 |A^{-T} k|^2 = q11 u^2 + q12x2 u v + q22 v^2
  double theta;              // facet field of view (radians); cell index = rint(u theta)
};
static_assert(sizeof(SrcModel) == 64, "one 64-byte scalar load per source");

// The same constants for the mixed-precision form: phase terms stay FP64,
// the profile runs in FP32.
struct alignas(64) SrcMixed {
  double l, m, n1;
  float flux, q11, q12x2, q22;
  double theta;
};
static_assert(sizeof(SrcMixed) == 64, "one 64-byte scalar load per source");

// Per-source facet geometry: dense accumulator block [side*side], cells
// centred on the uv origin, index (iy+half)*side + (ix+half).
struct SrcGeom {
  int64_t base;              // offset of the source's dense block
  int32_t half;              // N_s
  int32_t side;              // 2 N_s + 1
};

// Per-channel constants (device table).
struct ChanTable {
  double scale[kMaxChan];    // nu_c / c: metres -> wavelengths
  double spec[kMaxChan];     // (nu_c / nu_ref)^beta
};

// Dense accumulators of one extraction.
struct DenseAcc {
  double4 *cell;             // per dense cell: (W, Z re, Z im, count) -- one address per run flush
};

// Compacted facets (CSR by source, cells sorted by (iy, ix)).
struct Cells {
  int64_t *offsets;          // [n_src+1]
  int64_t *n_nonempty;       // [n_src]
  int32_t *ix, *iy, *count;
  double *wsum, *vre, *vim;
  double4 *fit64;            // (W^{-1/6} uc, W^{-1/6} vc, W^{-1/3}, sqrt(W) Re Vbar) for the FP64 fit
  float4 *fit32;             // same in FP32 for the mixed fit
};

struct ModelArgs {
  const double *u_m, *v_m, *w_m;
  int64_t n_rows;
  int32_t n_chan;
  int32_t mode;
  const ChanTable *chan;
  const SrcModel *src;
  const SrcMixed *src32;
  int32_t s_begin, s_end;
  const void *vis_in;        // RESIDUAL mode only
  void *out;
};

// Per-visibility arrays of a facet object in uv-sorted order (sorted once at
// creation along a Morton curve over (u, v) in wavelengths, so every
// source's facet cells are visited in long contiguous stretches).
struct Sorted {
  int64_t n_vis;
  uint32_t *order;           // sorted position -> visibility index row*n_chan + chan
  double4 *geo;              // (u, v, w) in wavelengths, spectral factor (nu_c/nu_ref)^beta
  void *quad;                // (u^2, u v, v^2, w spec) double4, w spec of the last residual gather |
                             // (u^2, u v, v^2 in FP32 from (float)u, (float)v; spec) float4
  void *res;                 // weighted residual w R, complex128 | residual R, complex64
  double *wt;                // weight, 0 where w <= 0 or NaN (flagged)
};

struct SortKeyArgs {
  const double *u_m, *v_m;
  int64_t n_rows;
  int32_t n_chan;
  const ChanTable *chan;
  double inv_span_u, inv_span_v;   // 1 / (2 max|u|), 1 / (2 max|v|) in wavelengths
  uint32_t *keys, *vals;
};

struct ExtractArgs {
  Sorted sv;
  int32_t n_chan;
  int32_t n_src;
  int32_t n_tiles;           // ceil(n_src / 64)
  int32_t chunk;             // sorted visibilities per wave (set by launch_extract)
  int64_t n_chunks;
  const ChanTable *chan;
  const SrcModel *src;
  const SrcMixed *src32;
  const SrcGeom *geom;
  const int32_t *order;      // [n_src] source of each lane slot: sources by increasing theta
  DenseAcc acc;
  uint32_t *err;             // bit 0: a cell index fell outside its facet (visibility skipped)
};

// Residual in sorted order: res[j] = vis[order[j]] - sum over sources of Eq. 1
// (or a plain gather of a residual given in caller order).
struct ResidualArgs {
  Sorted sv;
  int32_t n_chan;
  int32_t n_src;
  const ChanTable *chan;
  const SrcModel *src;
  const SrcMixed *src32;
  const void *vis;           // caller order
  const void *weight;        // caller order
  int32_t subtract;          // 1: vis - sky; 0: gather only
  double2 *rs;               // optional, FP64 form: the unweighted residual R in sorted order
};

// In-place update of a residual kept in sorted order when some sources'
// models change: R += sum over old models - sum over new models (Eq. 1),
// evaluated and added as rlf_model_vis would (old ones accumulated, then the
// new ones subtracted).  FP64 form: R in rs, and sv.res = w R rewritten;
// mixed form: sv.res holds R itself.
struct UpdateArgs {
  Sorted sv;
  int32_t n_old, n_new;
  const SrcModel *old64, *new64;
  const SrcMixed *old32, *new32;
  double2 *rs;
};

struct CompactArgs {
  int32_t n_src;
  const SrcGeom *geom;
  const SrcModel *src;
  DenseAcc acc;
  Cells cells;
};

struct FitArgs {
  int32_t n_src;
  int32_t n_valid;           // valid grid points (|e| < 1)
  int32_t n_e;
  int32_t num_r;
  double e_step;
  const int32_t *epts;       // [n_valid] flat grid indices, increasing
  const double *sk;          // [num_r] 4 pi^2 alpha_k^2 (radians)
  const double *logw;        // [n_src*num_r] ln(spline weight * prior density)
  const int64_t *offsets;
  const double4 *fit64;
  const float4 *fit32;
  const int32_t *window;     // [n_src*4] inclusive grid boxes, or null (full grid)
  int32_t check_stride;      // windowed launch: also the lattice points (multiples of it from the centre) outside the box
  const int32_t *valid_index; // [n_e*n_e] flat grid index -> valid-point index, -1 if |e| >= 1
  const int32_t *redo;       // fallback pass: [n_src] nonzero = evaluate; null = all
  double *lsurf;             // [n_src*n_valid] ln L(e) of the evaluated points
  // position marginalisation: n_pos offsets (0 = position fixed) and the
  // cross-correlation data [cells * n_pos] of the form in use
  int32_t n_pos;
  const double *pos_g64;
  const float *pos_g32;
  // lattice-seeded window: 1 = evaluate only the check_stride lattice (window
  // ignored); 2 = the lattice values are already in lsurf (box only)
  int32_t lattice_pass;
  // few sources, FP64 form, 20 knots, position fixed, full grid: parts > 1
  // splits each source's cells into that many ranges whose partial sums
  // [n_src][parts][2 * num_r][n_valid] go to part_sums before being joined
  int32_t parts;
  double *part_sums;
  // sources by increasing facet size (null: catalogue order); the full-grid
  // launch takes them from the largest, so the longest blocks start first
  const int32_t *size_order;
};

// Cross-correlation data of the position marginalisation (one row of n_pos
// values per compacted cell).
struct PosPrepArgs {
  int32_t n_src;
  int32_t n_side;            // offsets per axis (odd)
  int32_t n_pos;             // n_side^2
  double step;               // offset spacing in radians
  const SrcModel *src;       // theta per source
  const int64_t *offsets;
  const int32_t *ix, *iy;
  const double *wsum, *vre, *vim;
  double *g64;               // FP64 form
  float *g32;                // mixed form
};

// Adaptive refinement: per source a window of integer lattice indices at
// resolution e_step / 2^level; the estimate of each level decides the next.
struct RefineArgs {
  int32_t n_src;
  int32_t level;             // current level (>= 1)
  int32_t last_level;
  int32_t np_max;            // stop when this many samples lie above the threshold
  int32_t max_side;          // window points per axis, at most
  int32_t unit;              // 1 / e_step (integer): |e| < 1 <=> k1^2 + k2^2 < (unit 2^level)^2
  int32_t n_e, n_valid;
  double e_step;
  double log_frac, bad_sigma, bad_sqrtdet;
  const int32_t *epts;       // coarse grid (level 0)
  const double *lsurf;       // coarse ln L [n_src * n_valid]
  const int64_t *offsets;    // facet cells (empty facets are left alone)
  int32_t *win;              // [n_src * 5]: active, k1lo, k2lo, n1, n2
  double *lloc;              // [n_src * max_side^2] ln L on the window
  double *e1, *e2, *s1, *s2, *c12, *lmax;
  int32_t *n_above;
  uint32_t *flags;
};

// Work queue of the persistent likelihood kernel.
struct QueueArgs {
  const int32_t *order;      // [n_rank] source of each rank (decreasing cell count)
  const int64_t *item_start; // [n_rank+1] first item of each rank
  const int32_t *tile;       // [n_rank] items cover tile*64 valid grid points
  int32_t n_rank;
  int64_t n_items;
  uint32_t *counter;
};

struct EstimateArgs {
  int32_t n_src;
  int32_t n_valid;
  int32_t n_e;
  int32_t half_r2;           // (1/e_step)^2 for the |e| < 1 test
  double e_step;
  double log_frac;
  double bad_sigma, bad_sqrtdet;
  const int32_t *epts;
  const int64_t *offsets;
  double *lsurf;             // written only by the FP64 recheck below
  const int32_t *window;     // null = full grid
  const int32_t *redo;       // fallback pass: only these sources; null = all
  int32_t *redo_out;         // windowed pass with fallback: set where the window is not trusted
  int32_t check_stride;      // lattice check outside the window (0 = off)
  double *e1, *e2, *s1, *s2, *c12, *lmax;
  int32_t *argmax, *n_above;
  uint32_t *flags;
  double *surface;           // [n_src*n_e*n_e] or null
  // Mixed form, position fixed: the decisions of the estimate (the maximum
  // and membership of the thresholded set) are taken on FP64 values.  With
  // delta = recheck_rel * (|max| + recheck_abs), a bound on the error of the
  // FP32-summed ln L, every evaluated point within 2 delta below the maximum
  // or within 2 delta of the threshold is evaluated again in FP64 from the
  // FP64 cell records before the maximum and the set are taken; null fit64 =
  // no recheck (FP64 form).
  const double4 *fit64;
  const double *sk;          // [num_r] 4 pi^2 alpha_k^2
  const double *logw;        // [n_src*num_r]
  int32_t num_r;
  double recheck_rel, recheck_abs;
};

// C[M x N] (FP32, row stride ldc) = A * B, A(m, k) = a[m*sam + k*sak],
// B(k, n) = b[k*sbk + n*sbn], both BF16.
struct GemmArgs {
  const __bf16 *a;
  int64_t sam, sak;
  const __bf16 *b;
  int64_t sbk, sbn;
  float *c;
  int64_t ldc;
  int32_t M, N, K;
  float *ws;                 // split-K partials [split x M x N]
  int64_t ws_floats;
};

// C[M x N] (FP32, row stride ldc) = sum_k A[m lda + k] B[n ldb + k], A and B
// BF16 contiguous along k.
struct GemmNTArgs {
  const __bf16 *a;
  int64_t lda;
  const __bf16 *b;
  int64_t ldb;
  float *c;
  int64_t ldc;
  int32_t M, N, K;
  float *ws;                 // split-K partials [split x M x N]
  int64_t ws_floats;
};

struct FeatureArgs {
  int32_t s0;                // first source of the rows written
  int32_t n_src;             // rows written (sources s0 .. s0 + n_src - 1)
  const int64_t *offsets;
  const int32_t *ix, *iy;
  const double *vre, *vim;
  const SrcModel *src;
  double spec_norm;          // mean over channels of (nu_c / nu_ref)^beta
  __bf16 *x;                 // [n_src * 8192], row r for source s0 + r
};

// Launchers (enqueue on `st`; return the launch status).
hipError_t launch_model(const ModelArgs &a, int mixed, hipStream_t st);
// upd (optional): first update the residual kept in the sorted layout for
// changed source models (fused into the small-catalogue kernel).
hipError_t launch_extract(const ExtractArgs &a, int mixed, hipStream_t st, const UpdateArgs *upd = nullptr);
hipError_t launch_residual_sorted(const ResidualArgs &a, int mixed, hipStream_t st);
hipError_t launch_update_sorted(const UpdateArgs &a, int mixed, hipStream_t st);
hipError_t launch_sort_keys(const SortKeyArgs &a, hipStream_t st);
hipError_t sort_pairs_u32(void *tmp, size_t &tmp_bytes, const uint32_t *kin, uint32_t *kout, const uint32_t *vin,
                          uint32_t *vout, int64_t n, hipStream_t st);
hipError_t launch_sorted_static(const Sorted &sv, const double *u_m, const double *v_m, const double *w_m,
                                int32_t n_chan, const ChanTable *chan, int mixed, hipStream_t st);
hipError_t launch_compact(const CompactArgs &a, int mixed, hipStream_t st);
hipError_t launch_fit_f64(const FitArgs &a, hipStream_t st);
hipError_t launch_fit_mixed(const FitArgs &a, hipStream_t st);
hipError_t launch_fit_queue(const FitArgs &a, const QueueArgs &q, int mixed, int blocks, hipStream_t st);
int fit_queue_blocks_per_cu(int mixed, int num_r);
hipError_t launch_estimate(const EstimateArgs &a, hipStream_t st);
hipError_t launch_absmax(const double *x, int64_t n, double *out2, int slot, hipStream_t st);
hipError_t launch_refine_eval(const FitArgs &a, const RefineArgs &r, int mixed, hipStream_t st);
hipError_t launch_pos_prep(const PosPrepArgs &a, int mixed, hipStream_t st);
hipError_t launch_lattice_windows(const FitArgs &a, double log_frac, int32_t *win, hipStream_t st);
hipError_t launch_refine_start(const RefineArgs &r, hipStream_t st);
hipError_t launch_refine_estimate(const RefineArgs &r, hipStream_t st);
hipError_t launch_scatter_f64(const double *src, const int32_t *idx, int64_t n, double *dst, hipStream_t st);
hipError_t launch_scatter_u32(const uint32_t *src, const int32_t *idx, int64_t n, uint32_t bits, uint32_t *dst,
                              hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_gemm(const GemmArgs &g, int split_k, hipStream_t st);
hipError_t launch_bias_act(const float *c, const float *b, int64_t rows, int cols, float *z, __bf16 *h, int act,
                           hipStream_t st);
hipError_t launch_head(const float *y, const float *t, int64_t n, float *dy, __bf16 *dyb, double *loss,
                       hipStream_t st);
// The 512 -> 6 output layer: forward y = h W4 + b4 (h BF16 [rows x 512],
// W4 BF16 [512 x 6], b4 and y FP32), and backward: gw receives dW4 then db4
// (3,078 FP32, the parameters' order) from h, dY (BF16 for the product, FP32
// for the bias), dh = dY W4^T FP32 [rows x 512]; ws holds row-slice partials.
hipError_t launch_out_forward(const __bf16 *h, const __bf16 *w, const float *b, int64_t rows, float *y,
                              hipStream_t st);
hipError_t launch_out_backward(const __bf16 *h, const __bf16 *dyb, const float *dy, int64_t rows, const __bf16 *w,
                               float *gw, float *dh, float *ws, int64_t ws_floats, hipStream_t st);
// dZ = dH gelu'(Z) as BF16 [rows x cols] and db = column sums of dZ (FP32,
// summed over row slices, then the slices in order), ws holding the slices'
// partial sums.
hipError_t launch_gelu_back_colsum(const float *dh, const float *z, int64_t rows, int cols, __bf16 *dzb, float *db,
                                   float *ws, int64_t ws_floats, hipStream_t st);
hipError_t launch_gemm_nt(const GemmNTArgs &g, int split_k, hipStream_t st);
// dst[c][r] = src[r][c] for up to kMaxTransposeJobs BF16 matrices
// [rows x cols] in one launch.
constexpr int kMaxTransposeJobs = 4;
struct TransposeJob {
  const __bf16 *src;
  int64_t rows, cols;
  __bf16 *dst;
};
hipError_t launch_transpose_bf16(const TransposeJob *jobs, int n_jobs, hipStream_t st);
hipError_t launch_adam(float *w, __bf16 *wb, const float *g, float *m, float *v, int64_t n, float lr, int64_t step,
                       hipStream_t st);
hipError_t launch_to_bf16(const float *x, __bf16 *y, int64_t n, hipStream_t st);
hipError_t launch_features(const FeatureArgs &a, hipStream_t st);
hipError_t launch_posterior_targets(const double *e1, const double *e2, const double *s1, const double *s2,
                                   const float *ln_alpha, int64_t n, double kappa, uint64_t seed, float *t,
                                   hipStream_t st);
hipError_t launch_windows(const float *y, int64_t n, double nsigma, int n_e, double step, int min_half,
                          double full_frac, int32_t *win, hipStream_t st);

}  // namespace rlf
