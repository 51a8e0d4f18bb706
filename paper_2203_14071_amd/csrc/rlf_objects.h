// Library-private definitions shared by the host-side translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "rlf.h"
#include "rlf_internal.h"

using namespace rlf;

struct rlf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  rlf_params p{};
  std::string err;
  // ellipticity grid
  int n_valid = 0;
  int half_r2 = 0;
  int32_t *d_epts = nullptr;
  int32_t *d_vidx = nullptr;                 // flat grid index -> valid-point index or -1
  // scale-length knots
  std::vector<double> knots, ck;
  double *d_sk = nullptr;
  // channel table (cached by content)
  std::vector<double> chan_key;
  ChanTable *d_chan = nullptr;
  // source tables of rlf_model_vis (two slots, reused by content)
  struct Slot {
    std::vector<double> key;
    SrcModel *d = nullptr;
    SrcMixed *d32 = nullptr;
    int64_t cap = 0;
    uint64_t used = 0;
  } slot[2];
  uint64_t tick = 0;
  uint32_t *d_err = nullptr;
  double *d_absmax = nullptr;
  // partial likelihood sums of split fits (few sources), grown on demand
  double *d_part = nullptr;
  int64_t part_cap = 0;
  // pinned staging ring of the asynchronous table uploads
  char *pinned = nullptr;
  size_t pinned_off = 0;
  // host staging of rlf_model_vis_noalloc's tables (sized at creation)
  std::vector<unsigned char> noalloc_stage;
};

struct rlf_facets {
  rlf_ctx *ctx = nullptr;
  int64_t n_src = 0;
  int64_t dense_total = 0;
  int64_t dense_cap = 0;                     // dense cells the accumulator and cell arrays hold
  int mixed = 0;
  double spec_norm = 1.0;                    // mean spectral factor over the channels
  double mx[2] = {0.0, 0.0};                 // largest |u_m|, |v_m| of the observation
  bool owns_sorted = true;                   // false: sv borrowed from another facet object
  std::vector<double> alpha;                 // catalogue sizes at creation
  std::vector<double> theta;
  std::vector<double> model_key;             // shapes of the uploaded model table
  std::vector<SrcGeom> geom;
  SrcModel *d_src = nullptr;
  SrcMixed *d_src32 = nullptr;
  SrcGeom *d_geom = nullptr;
  int32_t *d_order = nullptr;                // sources by increasing theta (extraction lanes)
  Sorted sv{};                               // uv-sorted visibility layout
  DenseAcc acc{};
  Cells cells{};
  double *d_logw = nullptr;
  double *d_lsurf = nullptr;
  int32_t *d_redo = nullptr;
  int32_t *d_win = nullptr;                  // lattice-seeded windows [n_src * 4]
  int32_t *d_refine_win = nullptr;           // refinement windows [n_src * 5] (made on first use)
  double *d_refine_l = nullptr;              // refinement window values [n_src * side^2]
  // position marginalisation (rlf_facets_set_positions): offsets per axis
  // (1 = position fixed), spacing in radians, cross-correlation data sized
  // for every dense cell
  int32_t pos_side = 1;
  double pos_step = 0.0;
  void *d_pos_g = nullptr;
  int64_t pos_cap = 0;                       // rows x n_pos the buffer holds
};


namespace rlf {

int fail(rlf_ctx *c, int code, const std::string &msg);
int create_facets(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, const rlf_facets *share,
                  rlf_facets **out);
int hip_fail(rlf_ctx *c, hipError_t e, const char *what);

#define HIPCHK(ctx, call)                                    \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return rlf::hip_fail(ctx, e_, #call); \
  } while (0)

template <class T>
int dalloc(rlf_ctx *c, T **p, int64_t n) {
  *p = nullptr;
  if (n <= 0) n = 1;
  hipError_t e = hipMalloc((void **)p, sizeof(T) * (size_t)n);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(c, RLF_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return RLF_OK;
}

template <class T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

// Enqueue the likelihood grid and the estimator for every source of the
// last extraction (rlf_fit_sources without argument checks); `queue` selects
// the persistent work-queue kernel instead of the grid launch.
int enqueue_fit(rlf_ctx *c, const rlf_facets *f, const rlf_fit_opts &o, const rlf_fit_out &out,
                const QueueArgs *queue, int queue_blocks);

// Likelihood arguments of a facet object (position marginalisation
// included); enqueues the cross-correlation data when offsets are set.
int fit_args(rlf_ctx *c, const rlf_facets *f, FitArgs &fa);

// Host-to-device copy of a small table on the context's stream without
// waiting for it: the bytes are staged in a pinned ring, whose space is
// reused only after a synchronisation of the stream (every copy issued from
// it has then run).  Refused while the stream is being captured.
int upload_async(rlf_ctx *c, void *dst, const void *src, size_t bytes);

// The same facet object for another catalogue of as many sources (same
// observation); the uv-sorted layout is kept, the dense arrays reused while
// large enough.
int retarget_facets(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, rlf_facets *f);

// Extraction into f: with `vis`, first the gather into f's sorted layout
// (subtract = 1: minus f's own catalogue models); with vis NULL the sorted
// layout already holds the residual, optionally after a pending update.
int extract_facets(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, const void *vis, int subtract,
                   rlf_facets *f, const UpdateArgs *upd = nullptr);

// A residual kept in the sorted layout of f (sequential refinement): set it
// to obs.vis minus the models of `sky`, then update it as models change.
// FP64 form: rs [n_vis] holds the unweighted residual next to sv.res = w R.
// An update (prepare_update: the two model tables in the context's model
// slots, valid until the next model-table lookup) is applied by its own pass
// or, pending, by the next extraction (extract_facets(..., upd)).
int sorted_residual(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *sky, const rlf_facets *f, double2 *rs);
int prepare_update(rlf_ctx *c, const rlf_catalog *old_m, const rlf_catalog *new_m, const rlf_facets *f,
                   double2 *rs, UpdateArgs &u);
int update_sorted_residual(rlf_ctx *c, const UpdateArgs &u, int mixed);

}  // namespace rlf
