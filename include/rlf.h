/*
 * rlf.h -- C ABI of the MI355X (gfx950) RadioLensfit hot path.
 *
 * Implements the data-parallel core of Rivi & Miller, "RadioLensfit: an HPC
 * tool for accurate galaxy shape measurement with SKA" (arXiv 2203.14071):
 *   - the sky model, a sum over catalogue sources of the exponential-disk
 *     visibility of Eq. 1 (Sec. 2.2);
 *   - per-source extraction: subtract every other source, phase-shift to the
 *     source, average into a coarse uv grid ("facet") whose field of view is
 *     K times the scale length (Sec. 2.3);
 *   - the shape fit: chi-squared likelihood of the facet under Eq. 1 at the
 *     cell centres, flux marginalised analytically, scale length marginalised
 *     numerically under a log-normal prior (Sec. 2.4), evaluated on a full
 *     (e1, e2) grid, and the thresholded-moment estimate with the variance
 *     test for bad fits (Sec. 2.4, 4.1).
 *
 * Conventions shared by every entry point:
 *   - Pointers documented as "device" are HIP device pointers on the context's
 *     device; "host" pointers are ordinary host memory.  The caller owns every
 *     buffer it passes; the library owns only rlf_ctx and rlf_facets objects.
 *   - Work is enqueued on the context's HIP stream and the call returns
 *     without waiting, unless the entry point says it synchronises.  Results
 *     are valid after rlf_sync() or any later synchronisation of that stream.
 *   - Every call returns RLF_OK (0) or a negative rlf_status; nothing aborts.
 *     rlf_last_error() returns a text description of the last failure on a
 *     context.  A context is not thread-safe; use one per host thread.
 *   - Complex arrays are interleaved (re, im).  Visibility arrays are indexed
 *     [row * n_chan + chan] (channel fastest).
 *   - Precision forms: RLF_FP64 computes everything in FP64 (complex128
 *     visibilities, f64 weights).  RLF_MIXED forms and range-reduces phase
 *     arguments in FP64 and runs sin/cos, the model and the likelihood in
 *     FP32 with compensated (block-FP64) sums (complex64 visibilities, f32
 *     weights).
 */
#ifndef RLF_H
#define RLF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rlf_ctx rlf_ctx;        /* opaque: device, stream, parameters, tables */
typedef struct rlf_facets rlf_facets;  /* opaque: facet geometry + device buffers for one catalogue */
typedef struct rlf_pass rlf_pass;      /* opaque: a captured, replayable pass over all sources */
typedef struct rlf_mlp rlf_mlp;        /* opaque: the grid-narrowing network and its optimiser state */

typedef enum {
  RLF_OK = 0,
  RLF_EINVAL = -1,        /* invalid argument (null pointer, bad size or value)        */
  RLF_ENOMEM = -2,        /* device or host allocation failed                          */
  RLF_EDEVICE = -3,       /* a HIP runtime call failed; rlf_last_error() has its text  */
  RLF_ERANGE = -4,        /* a facet or the visibility count exceeds supported sizes  */
  RLF_EUNSUPPORTED = -5,  /* valid request the library does not implement              */
  RLF_EIO = -6            /* a file could not be opened, read or written, or is not a  */
                          /* checkpoint of this network (rlf_last_error() says which)  */
} rlf_status;

typedef enum { RLF_FP64 = 0, RLF_MIXED = 1 } rlf_precision;

/* Per-source result flags (rlf_fit_out.flags). */
enum {
  RLF_FLAG_BAD_VAR = 1,   /* sigma(e1) or sigma(e2) <= bad_sigma, or sqrt(det C) <= bad_sqrtdet (Sec. 4.1) */
  RLF_FLAG_EMPTY = 2,     /* facet holds no visibility with positive weight; outputs are NaN               */
  RLF_FLAG_EDGE = 4,      /* maximum on the edge of the evaluated ellipticity region                       */
  RLF_FLAG_FALLBACK = 8,  /* narrowed grid rejected; the full grid was evaluated instead                   */
  RLF_FLAG_REFIT = 16,    /* rlf_fit_sequential: fitted again at the end against the final sky model         */
  RLF_FLAG_REFINED = 32   /* rlf_refine_sources: the estimate comes from a finer local grid                  */
};

/* rlf_model_vis modes. */
enum {
  RLF_MODEL_WRITE = 0,      /* out  = sum over sources                        */
  RLF_MODEL_ACCUMULATE = 1, /* out += sum over sources                        */
  RLF_MODEL_RESIDUAL = 2    /* out  = obs->vis - sum over sources (may alias) */
};

/* Algorithm parameters.  Defaults (rlf_params_default) are the paper's:
 * beta = -0.7 (Eq. 1), ADD = -0.93 and ESP = 0.33 (Eq. 4), K = PSF_NAT = 38
 * (Sec. 4.1), R_STD = 0.3136 (Sec. 2.4), [RMIN, RMAX] = [0.3, 3.5] arcsec
 * (Sec. 4.2), 5 % likelihood threshold (Sec. 2.4), bad-fit thresholds 5e-3
 * and 5e-5 (Sec. 4.1); num_r = 20 knots quadratic in the index, an 81 x 81
 * ellipticity grid of step 0.02, FP64. */
typedef struct {
  double beta;            /* spectral index of Eq. 1                                   */
  double ref_freq_hz;     /* reference frequency of the catalogue fluxes               */
  double K;               /* facet field of view = K * scale length                    */
  double add, esp;        /* Eq. 4 coefficients (prior median of the scale length)     */
  double r_std;           /* width of the log-normal scale prior, in ln(alpha)          */
  double rmin_arcsec;     /* scale-length marginalisation interval                      */
  double rmax_arcsec;
  int32_t num_r;          /* knots, 2..32; alpha_k = rmin + (rmax-rmin) (k/(num_r-1))^2  */
  int32_t n_e;            /* ellipticity grid points per axis, odd, 3..255              */
  double e_step;          /* grid step; 1/e_step must be an integer; e = (i-(n_e-1)/2) e_step */
  double frac_thresh;     /* samples with L >= frac_thresh * Lmax enter the moments     */
  double bad_sigma;       /* bad-fit thresholds                                         */
  double bad_sqrtdet;
  int32_t precision;      /* rlf_precision                                              */
  int32_t reserved;       /* must be 0                                                  */
} rlf_params;

/* Observation, structure of arrays.  uvw are in metres in the phase-tracking
 * frame; they are scaled to wavelengths at each channel centre
 * (Sec. 2.2) as u = u_m * (freq / c). */
typedef struct {
  int64_t n_rows;              /* > 0                                                   */
  int32_t n_chan;              /* 1..64                                                 */
  int32_t reserved;            /* must be 0                                             */
  const double *u_m, *v_m, *w_m; /* device [n_rows]                                     */
  const double *freq_hz_host;  /* host [n_chan] channel centres, > 0                    */
  const void *vis;             /* device [n_rows*n_chan] complex128 (FP64) or complex64 (MIXED) */
  const void *weight;          /* device [n_rows*n_chan] f64 (FP64) or f32 (MIXED); w <= 0 = flagged */
} rlf_obs;

/* Source catalogue, structure of arrays, host memory.  Catalogue order is the
 * processing order (Sec. 2.1: decreasing SNR or flux). */
typedef struct {
  int64_t n_src;                 /* > 0                                                */
  const double *l, *m;           /* direction cosines, l^2 + m^2 < 1                   */
  const double *flux_jy;         /* integrated flux at ref_freq_hz, finite, >= 0        */
  const double *alpha_arcsec;    /* scale length, finite, > 0 (rlf_alpha_from_flux when unknown) */
  const double *e1, *e2;         /* sky-model shape, |e| < 1 (0 = circular start, Sec. 2.2) */
  const double *prior_mu;        /* optional [n_src] ln(alpha_median/arcsec) of the scale prior;
                                    NULL = Eq. 4 from flux_jy                           */
} rlf_catalog;

/* Library version (major*10000 + minor*100 + patch). */
int rlf_version(void);

/* Fill *p with the defaults listed above.  Returns RLF_EINVAL if p is NULL. */
int rlf_params_default(rlf_params *p);

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t passed as void*; NULL = the legacy default stream).
 * Validates *p (RLF_EINVAL), builds the ellipticity and knot tables and
 * uploads them; synchronises.  *ctx is set only on success. */
int rlf_create(rlf_ctx **ctx, int device, void *hip_stream, const rlf_params *p);

/* Release a context and its tables (NULL is a no-op).  Facet objects made on
 * it must be freed first. */
int rlf_destroy(rlf_ctx *ctx);

/* Change the stream later calls enqueue on; synchronises the previous one
 * first (the library's small table uploads are staged in host memory that
 * is reused once the stream they were queued on has drained). */
int rlf_set_stream(rlf_ctx *ctx, void *hip_stream);

/* Wait for all work enqueued by this context. */
int rlf_sync(rlf_ctx *ctx);

/* Text of the last error on ctx ("" if none).  Valid until the next call on ctx. */
const char *rlf_last_error(const rlf_ctx *ctx);

/* Eq. 4 (Sec. 2.2): alpha = exp(add + esp * ln(flux / 1 uJy)) arcsec, on the
 * host for n fluxes (> 0). */
int rlf_alpha_from_flux(const double *flux_jy_host, int64_t n, double add, double esp,
                        double *alpha_arcsec_host);

/* Sky model (Sec. 2.2): for every visibility, the sum over catalogue sources
 * src_begin <= s < src_end of Eq. 1 at (u, v, w) in wavelengths,
 * (nu/nu_ref)^beta S exp(2 pi i (u l + v m + w (sqrt(1-l^2-m^2)-1)))
 *     / (1 + 4 pi^2 alpha^2 |A^{-T} (u,v)|^2)^{3/2},
 * with A from Eq. 2 and the catalogue's (e1, e2).  `out` is device
 * [n_rows*n_chan] in the context's complex type; see the mode enum.
 * obs->vis is read only in RLF_MODEL_RESIDUAL and may then alias out. */
int rlf_model_vis(rlf_ctx *ctx, const rlf_obs *obs, const rlf_catalog *cat,
                  int64_t src_begin, int64_t src_end, void *out, int mode);

/* rlf_model_vis for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc): the same computation and
 * result, bit for bit, with the channel and source tables held in one
 * fixed, library-owned device array per GPU (513 KiB, kept until the process
 * ends) instead of memory the context allocates; no hipMalloc, hipFree or
 * other allocating call is made (the host staging it copies from is
 * allocated once by rlf_create).  At most 4096 sources per call
 * (src_end - src_begin), else RLF_EINVAL; larger catalogues are summed in
 * several calls with RLF_MODEL_ACCUMULATE.  The call first waits for the
 * work already queued on the context's stream, then copies the tables and
 * enqueues the kernel; RLF_EUNSUPPORTED while the stream is being captured.
 * Every call on one GPU shares that GPU's array, whichever context makes
 * it: calls on one GPU must not overlap (two contexts on two streams
 * enqueuing at once race on the tables). */
int rlf_model_vis_noalloc(rlf_ctx *ctx, const rlf_obs *obs, const rlf_catalog *cat,
                          int64_t src_begin, int64_t src_end, void *out, int mode);

/* Facet geometry for a catalogue on an observation (Sec. 2.3): per source
 * theta_s = K * alpha_s (alpha in radians, converted first), cell size
 * 1/theta_s, cells centred on the uv origin, half-size
 * N_s = max over visibilities of |rint(u theta_s)|, |rint(v theta_s)|.
 * Allocates the device accumulators, the compacted facet arrays and the
 * per-source scale-prior table (Sec. 2.4), and orders the visibilities once
 * along a Morton curve over (u, v) (a layout for the extraction kernels; no
 * result depends on it beyond FP summation order).  Synchronises.  The
 * observation's uvw and sizes must not change while the object is used.
 * RLF_ERANGE if some N_s > 16383 or there are 2^32 or more visibilities. */
int rlf_facets_create(rlf_ctx *ctx, const rlf_obs *obs, const rlf_catalog *cat,
                      rlf_facets **out);

/* Extraction (Sec. 2.3) of every catalogue source into its facet.  For each
 * source s and visibility with weight w > 0:
 *   z = residual * exp(-2 pi i phi_s) + spec * S_s * profile_s(u, v)
 * where residual = vis - sky (all sources), phi_s the Eq. 1 phase of source s,
 * and the added term is its own model (real after the shift); then, in cell
 * (rint(u theta_s), rint(v theta_s)) (round half to even):
 *   count += 1, W += w, Z += w z.
 * Compaction keeps the cells with count > 0 sorted by (iy, ix) and sets
 * Vbar = Z / W.  `residual` is device, same type and shape as obs->vis
 * (e.g. rlf_model_vis in RLF_MODEL_RESIDUAL mode); NULL means "compute it":
 * the library subtracts the sky model of this catalogue (all sources, their
 * current shapes) from obs->vis itself.  The catalogue must have the same
 * sources and sizes as at rlf_facets_create (RLF_EINVAL otherwise); its
 * shapes may differ.  Integer results (cells, counts) are exact; FP sums are
 * accumulated atomically, so their last bits may vary from run to run. */
int rlf_extract_facets(rlf_ctx *ctx, const rlf_obs *obs, const rlf_catalog *cat,
                       const void *residual, rlf_facets *facets);

/* Sizes of a facet object: sources, non-empty cells of the last extraction
 * (synchronises), and allocated dense cells.  Any output pointer may be NULL. */
int rlf_facets_info(rlf_ctx *ctx, const rlf_facets *facets, int64_t *n_src,
                    int64_t *n_cells_total, int64_t *n_dense_cells);

/* Copy the last extraction to host memory (synchronises).  offsets
 * [n_src+1] (CSR into the cell arrays), ix, iy, count [n_cells_total],
 * wsum [n_cells_total], vbar [2*n_cells_total] (re, im), theta [n_src]
 * radians.  Any output pointer may be NULL. */
int rlf_facets_copy(rlf_ctx *ctx, const rlf_facets *facets, int64_t *offsets, int32_t *ix,
                    int32_t *iy, int32_t *count, double *wsum, double *vbar, double *theta);

/* Free a facet object (NULL is a no-op).  Synchronises its context's stream. */
int rlf_facets_free(rlf_facets *facets);

/* Position marginalisation (Sec. 2.4: the likelihood is marginalised over
 * the source position with a uniform prior, through the cross-correlation of
 * the facet data with the model).  After this call, rlf_fit_sources (full
 * grid) and rlf_refine_sources on `facets` use, for every e and knot,
 *   D_p = sum_c W_c f_c Re(Vbar_c exp(-2 pi i (uc_c dl_p + vc_c dm_p))),
 *   ln L(e) = ln sum_k w_{s,k} (1/n_side^2) sum_p exp(D_p^2 / (2 Mm) - ln(Mm)/2)
 * over the offsets (dl_p, dm_p) = ((p1 - h) step, (p2 - h) step) of an
 * n_side x n_side grid centred on the catalogue position, h = (n_side-1)/2,
 * p = p1 * n_side + p2: a model displaced by x multiplies the facet model
 * by exp(+2 pi i k.x) (the sign of Eq. 1), and the uniform prior over the
 * square the grid spans is integrated as the mean over its points.
 *   n_side        1 (position fixed, the default), 3, 5 or 7
 *   step_arcsec   offset spacing in arcsec (> 0; ignored for n_side = 1)
 * Allocates the cross-correlation rows (n_side^2 values per dense cell, FP64
 * or FP32 with the facets' precision) on first use or growth; each fit
 * recomputes them from the last extraction.  Windowed fits on such facets
 * return RLF_EUNSUPPORTED.  RLF_EINVAL for another n_side or a step <= 0. */
int rlf_facets_set_positions(rlf_ctx *ctx, rlf_facets *facets, int32_t n_side, double step_arcsec);

/* Fit options. */
typedef struct {
  int32_t mode;            /* 0 = full grid; 1 = windowed (window must be set); 2 = windowed on
                              a window the library seeds from a lattice (not in the paper): ln L
                              is first evaluated at the valid points whose offsets from the grid
                              centre are multiples of check_stride (required, 2..n_e-1) on both
                              axes, each source's window is the bounding box of those lattice
                              points within the threshold of the lattice maximum widened by
                              check_stride steps (clamped; the whole grid for an empty facet),
                              and the fit proceeds as mode 1 with fallback and the lattice check
                              (window and fallback are then ignored).  Not available on facets
                              with position marginalisation (RLF_EUNSUPPORTED) nor in a pass.  */
  int32_t want_surface;    /* nonzero: write out->surface                                    */
  const int32_t *window;   /* device [n_src*4] inclusive (i1lo, i1hi, i2lo, i2hi) grid boxes */
  int32_t fallback;        /* windowed mode: nonzero = refit on the full grid (flag
                              RLF_FLAG_FALLBACK) every source of a non-empty facet whose window
                              holds no valid grid point, or where a member of the window's
                              thresholded set has a grid neighbour (|e| < 1) outside the window */
  int32_t check_stride;    /* windowed mode with fallback: 0 = off; S in [2, n_e-1] = also
                              evaluate the valid points outside the window whose offsets from
                              the grid centre are multiples of S on both axes, and refit when
                              one of them reaches the window's thresholded set (a separate
                              region of high likelihood).  Must be 0 otherwise. */
} rlf_fit_opts;

/* Fit outputs, device arrays [n_src] (surface [n_src*n_e*n_e]).  Any pointer
 * may be NULL to skip that output except flags. */
typedef struct {
  double *e1, *e2;         /* likelihood-weighted mean over samples above threshold        */
  double *s1, *s2, *c12;   /* standard deviations and covariance of those samples          */
  double *lmax;            /* maximum of ln L(e) (shape-free constants omitted)            */
  int32_t *argmax;         /* flat grid index i1*n_e + i2 of the maximum (smallest on ties) */
  int32_t *n_above;        /* samples in the thresholded set                                */
  uint32_t *flags;         /* RLF_FLAG_* (required)                                          */
  double *surface;         /* ln L(e) on the full grid, i1 (e1) slow, -inf outside the
                              evaluated region; f64 in both precision forms                 */
} rlf_fit_out;

/* Shape fit (Sec. 2.4) of every source of the last extraction.  For each
 * source, evaluated grid point e (|e| < 1, inside the window if any) and
 * knot alpha_k:
 *   f_c = (1 + 4 pi^2 alpha_k^2 |A_e^{-T} k_c|^2)^{-3/2} at cell centres k_c,
 *   D = sum_c W_c f_c Re Vbar_c,  Mm = sum_c W_c f_c^2,
 *   ln L(e, alpha_k) = D^2 / (2 Mm) - ln(Mm) / 2        (flux marginalised)
 *   ln L(e) = ln sum_k w_{s,k} L(e, alpha_k)              (scale marginalised)
 * with w_{s,k} the natural-cubic-spline quadrature weight of knot k times the
 * log-normal prior density at alpha_k.  Then Lmax, the set
 * {ln L >= ln Lmax + ln frac}, its likelihood-weighted mean and covariance,
 * and the flags.  RLF_MIXED: the set is decided in FP64 -- the maximum and
 * every point whose FP32-sum ln L lies within 2^-16 (|ln Lmax| + 64) of the
 * threshold are evaluated again with FP64 sums over an FP64 copy of the
 * facet's cells before the set is formed (every mode, except on facets with
 * position marginalisation); the surface holds the re-evaluated values. */
int rlf_fit_sources(rlf_ctx *ctx, const rlf_facets *facets, const rlf_fit_opts *opts,
                    rlf_fit_out *out);

/* Adaptive refinement of the estimates of the last full-grid rlf_fit_sources
 * call on `facets` (Sec. 2.4: the likelihood is sampled around its maximum
 * until NP_MAX samples lie above the threshold or the resolution E_RES is
 * reached).  Nested grids: level L has the points e = k * e_step / 2^L, k
 * integer, |e| < 1 tested on the integers; level 0 is the fit's grid.  A
 * source whose thresholded set at level L - 1 holds fewer than np_max points
 * is evaluated at level L on that set's bounding box widened by one level
 * L - 1 step (at most 64 points per axis, else 64 centred on the maximum);
 * the last level is the first with step <= e_res.  Refined sources get the
 * thresholded likelihood-weighted moments of their last window in out (e1,
 * e2, s1, s2, c12, lmax, n_above; argmax keeps the full-grid index), the
 * bad-variance flag re-evaluated with the refined widths, and
 * RLF_FLAG_REFINED; other sources and empty facets are untouched.  `out`
 * holds the full-grid results on entry (flags required).  The paper's
 * values: np_max = 30, e_res = 0.003 (three levels from the 0.02 grid).
 * RLF_EINVAL for np_max < 1 or e_res <= 0 or below e_step / 4096. */
int rlf_refine_sources(rlf_ctx *ctx, rlf_facets *facets, int32_t np_max, double e_res, rlf_fit_out *out);

/* Sequential sky-model refinement (Sec. 2.1, 2.3, 2.4 and the chunked form
 * of Sec. 3.1).  Sources are taken in catalogue order (decreasing flux) in
 * chunks of `chunk`; the sky model starts from the catalogue's shapes (e1, e2;
 * circular at the start of the paper's procedure).  Each chunk's sources are
 * extracted from obs->vis minus the current sky model (their own current
 * model restored) and fitted on the full grid; every chunk source whose fit
 * has neither RLF_FLAG_BAD_VAR nor RLF_FLAG_EMPTY then takes its measured
 * (e1, e2) into the sky model before the next chunk.  With refit_bad
 * nonzero, the sources flagged RLF_FLAG_BAD_VAR are extracted and fitted once
 * more at the end against the final sky model (flag RLF_FLAG_REFIT added),
 * and a finite refit also enters the final shapes.  chunk = 1 is the paper's
 * serial order, chunk = n_src with refit_bad = 0 equals rlf_facets_create +
 * rlf_extract_facets + rlf_fit_sources.
 *   out      device [n_src] final estimate of every source (flags required,
 *            surface ignored)
 *   e1_host, e2_host   host [n_src] final sky-model shapes
 * The residual is kept in the uv-sorted layout of the first chunk's facet
 * object (FP64 form: plus a library-allocated unweighted copy, 16 bytes per
 * visibility) and updated in place (R += old models, R -= new models of the
 * refined sources, with the arithmetic of rlf_model_vis); obs->vis is not
 * modified.  Chunks of the first chunk's size reuse its facet object.
 * Synchronises after every chunk (the host decides which shapes enter the
 * model).  RLF_EINVAL for chunk < 1 or a NULL argument. */
int rlf_fit_sequential(rlf_ctx *ctx, const rlf_obs *obs, const rlf_catalog *cat, int64_t chunk, int32_t refit_bad,
                       const rlf_fit_out *out, double *e1_host, double *e2_host);

/* Batched pass over every source (Sec. 2.2-2.4 in one unit): the residual of
 * this catalogue's sky model (as rlf_extract_facets with residual = NULL),
 * extraction, compaction, the likelihood grid and the estimate, captured
 * once into a HIP graph and replayed by rlf_pass_launch on the context's
 * stream.  The likelihood runs as one persistent work-queue launch: sources
 * in decreasing order of facet cell count, each work item covering tile*64
 * grid points of one source.  The tile for each facet-size bucket (cells
 * < 256, < 1024, < 4096, >= 4096) is autotuned at creation by timing the
 * candidates 1, 2, 4, 8 on the pass's own facets, unless `tune_path` (a text
 * file, may be NULL) already holds a choice for this precision and knot
 * count; new choices are written back to it.  Creation runs the pass once
 * eagerly and synchronises.  Replays read and write the same buffers given
 * here (obs->vis may be refilled between replays); the catalogue, the
 * observation geometry and weights must stay as they were.  opts as for
 * rlf_fit_sources (the windowed mode uses its own windowed launch). */
int rlf_pass_create(rlf_ctx *ctx, const rlf_obs *obs, const rlf_catalog *cat, rlf_facets *facets,
                    const rlf_fit_opts *opts, const rlf_fit_out *out, const char *tune_path,
                    rlf_pass **pass);

/* Enqueue one replay of the pass on the context's stream. */
int rlf_pass_launch(rlf_pass *pass);

/* The chosen tile per bucket, and how it was chosen (0 bucket empty,
 * 1 timed now, 2 read from the table).  Either pointer may be NULL. */
int rlf_pass_tiles(const rlf_pass *pass, int32_t *tiles /*[4]*/, int32_t *tuned /*[4]*/);

/* Free a pass (NULL is a no-op); synchronises. */
int rlf_pass_free(rlf_pass *pass);

/* ---- Grid-narrowing network (not in the paper) --------------------------
 * An MLP maps a facet to (e1, e2, ln alpha) and their log-variances; its
 * predictions centre narrowed ellipticity windows for rlf_fit_sources
 * (mode 1 with fallback), the full-grid fit staying the reference.
 *   input   8192 values: the facet's cells with -32 <= ix, iy <= 31,
 *           Vbar / (S g) (S the catalogue flux at nu_ref, g the observation's
 *           mean spectral factor of Eq. 1) clipped to [-4, 4], Re at (iy+32)*64 + ix+32, Im at
 *           4096 + the same index, 0 for empty cells; BF16 [n x 8192] row-major
 *   layers  z_l = h_{l-1} W_l + b_l, h_l = GELU(z_l) = z Phi(z) (l = 1..3,
 *           width 512), y = h_3 W_4 + b_4 (6 outputs, FP32 [n x 6]:
 *           mu = y[0:3], s = y[3:6] log-variances)
 *   loss    mean over samples of sum_d (s'_d + (t_d - mu_d)^2 exp(-s'_d)) / 2,
 *           s' = max(s, ln 1e-3) (no gradient to s below the floor)
 * Products are BF16 on MFMA with FP32 accumulation; FP32 master weights,
 * Adam (0.9, 0.999, 1e-8).  Parameters, FP32, in this order: W1 [8192 x 512],
 * b1 [512], W2 [512 x 512], b2, W3 [512 x 512], b3, W4 [512 x 6], b4 [6]
 * (weights row-major, input index slow). */

/* Number of parameters (4,723,206). */
int64_t rlf_mlp_num_params(void);

/* Create a network with zero parameters that trains on batches of at most
 * max_batch rows (forward accepts any number of rows). */
int rlf_mlp_create(rlf_ctx *ctx, int64_t max_batch, rlf_mlp **net);

/* Free a network (NULL is a no-op); synchronises. */
int rlf_mlp_free(rlf_mlp *net);

/* Set parameters (host, FP32 [n_params]) and the Adam state (host m, v or
 * NULL for zero; step = updates taken so far).  Synchronises. */
int rlf_mlp_set_state(rlf_mlp *net, const float *params, const float *adam_m, const float *adam_v, int64_t step);

/* Copy parameters, Adam moments and the last gradients to host arrays
 * [n_params] (any may be NULL) and the step count.  Synchronises. */
int rlf_mlp_get_state(rlf_mlp *net, float *params, float *adam_m, float *adam_v, float *grad, int64_t *step);

/* Checkpoint of the training state: FP32 master parameters, Adam moments m
 * and v, and the step count (everything rlf_mlp_train_step reads besides its
 * arguments), written to the file at path (host string).  Format, little-
 * endian: the 8 bytes "RLFMLP01", uint32 format version 1, uint32 0, int64
 * n_params, int64 step, uint64 FNV-1a hash of the payload, then the payload
 * params, m, v as FP32 [n_params] each.  The file is written under a
 * temporary name in the same directory and renamed over path when complete,
 * so a failed save leaves any earlier file at path intact.  Synchronises.
 * RLF_EIO if the file cannot be written. */
int rlf_mlp_save(rlf_mlp *net, const char *path);

/* Restore a checkpoint written by rlf_mlp_save: the network's parameters,
 * Adam moments and step become the file's, so that training continues bit
 * for bit as it would have from the saved state.  The file is read and
 * checked (header, size, payload hash) before anything is changed: on
 * RLF_EIO (unreadable, truncated, another format or network size, hash
 * mismatch) the network keeps its state.  Synchronises. */
int rlf_mlp_load(rlf_mlp *net, const char *path);

/* Network inputs of every source of the last extraction: device BF16
 * [n_src x 8192], Vbar / (S g) with g the mean over the observation's
 * channels of (nu_c / nu_ref)^beta (1 for one channel at nu_ref), each part
 * clipped to [-4, 4]. */
int rlf_mlp_features(rlf_ctx *ctx, const rlf_facets *facets, void *x);

/* y = network(x) for `rows` inputs: x device BF16 [rows x 8192], y device
 * FP32 [rows x 6]. */
int rlf_mlp_forward(rlf_mlp *net, const void *x, int64_t rows, float *y);

/* One Adam step on a batch (rows <= max_batch): x device BF16 [rows x 8192],
 * target device FP32 [rows x 3] (e1, e2, ln alpha), learning rate lr; the
 * batch loss is written to device *loss (FP64). */
int rlf_mlp_train_step(rlf_mlp *net, const void *x, const float *target, int64_t rows, float lr, double *loss);

/* The network on a facet object directly: the inputs of its sources (as
 * rlf_mlp_features forms them) go through the network's own staging buffer
 * in chunks of max_batch, and y (device FP32 [n_src x 6]) receives what
 * rlf_mlp_forward would give for them, bit for bit.  The facet object must
 * belong to the network's context. */
int rlf_mlp_predict(rlf_mlp *net, const rlf_facets *facets, float *y);

/* One Adam step on the sources of a facet object (1 <= n_src <= max_batch),
 * their inputs formed as by rlf_mlp_features; otherwise rlf_mlp_train_step. */
int rlf_mlp_train_facets(rlf_mlp *net, const rlf_facets *facets, const float *target, float lr, double *loss);

/* Training targets around the method's own fits (the network then learns the
 * posterior mean as its mean and, through the NLL, the posterior width plus
 * its own error as its variance): for each of `rows` sources, from its
 * full-grid estimate (e1, e2) and spread (s1, s2) (device FP64 [rows], as
 * rlf_fit_sources writes them) and ln alpha (device FP32 [rows]),
 * target = (e1 + kappa s1 z_{2i}, e2 + kappa s2 z_{2i+1}, ln alpha), device
 * FP32 [rows x 3].  z_j is the j-th standard normal number of stream `seed`:
 * the Box-Muller transform, in FP64, of uniforms from the SplitMix64
 * generator used counter-wise (value k of stream seed is the SplitMix64
 * output mix of seed + k * 0x9E3779B97F4A7C15; u1 = ((h(2j+1) >> 11) + 1)
 * 2^-53, u2 = (h(2j+2) >> 11) 2^-53, z_j = sqrt(-2 ln u1) cos(2 pi u2)).
 * A row whose estimate or spread is not finite gets (0, 0, ln alpha).
 * kappa >= 0 scales the spread. */
int rlf_mlp_posterior_targets(rlf_ctx *ctx, const double *e1, const double *e2, const double *s1, const double *s2,
                              const float *ln_alpha, int64_t rows, double kappa, uint64_t seed, float *target);

/* Window boxes for rlf_fit_sources mode 1 from predictions y (device FP32
 * [rows x 6]): per axis, mu +- nsigma exp(s'/2) (s' the floored
 * log-variance), widened to at least +- min_half grid steps around the
 * nearest grid point, snapped outward and clamped to the grid; a box
 * covering more than full_frac (in [0, 1]) of the n_e x n_e grid becomes the
 * whole grid (a broad prediction gains nothing from a window and would pay
 * for a refit).  Written as device int32 [rows x 4] (i1lo, i1hi, i2lo, i2hi). */
int rlf_mlp_windows(rlf_ctx *ctx, const float *y, int64_t rows, double nsigma, int32_t min_half, double full_frac,
                    int32_t *window);

#ifdef __cplusplus
}
#endif

#endif /* RLF_H */
