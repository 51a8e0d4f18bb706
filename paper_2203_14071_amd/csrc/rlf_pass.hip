// Batched pass: residual + extraction + likelihood + estimate for every
// source, captured once into a HIP graph and replayed.
//
// The likelihood runs as one persistent work-queue launch: ranks are the
// sources in decreasing order of facet cell count (the longest items are
// claimed first), an item covers tile*64 consecutive valid grid points of one
// source.  The tile per facet-size bucket is chosen by an autotuner that
// times every candidate on the pass's own facets (bucket by bucket) and can
// store its choice in a small text table for later passes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "rlf_objects.h"

namespace {

constexpr int kBuckets = 4;                       // facet cells: <256, <1024, <4096, >=4096
constexpr int kCandidates[] = {1, 2, 4, 8};

int bucket_of(int64_t cells) {
  if (cells < 256) return 0;
  if (cells < 1024) return 1;
  if (cells < 4096) return 2;
  return 3;
}

}  // namespace

struct rlf_pass {
  rlf_ctx *c = nullptr;
  rlf_facets *f = nullptr;
  rlf_fit_opts opts{};
  rlf_fit_out out{};
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t *d_order = nullptr;
  int64_t *d_item_start = nullptr;
  int32_t *d_tile = nullptr;
  uint32_t *d_counter = nullptr;
  QueueArgs q{};
  int blocks = 0;
  int tiles[kBuckets] = {1, 1, 1, 1};
  int tuned[kBuckets] = {0, 0, 0, 0};             // 1 = timed in this pass, 2 = read from the table
};

namespace {

using rlf::dalloc;
using rlf::dfree;
using rlf::fail;
using rlf::hip_fail;

// Build a schedule over `ranks` (source indices, already ordered) into the
// pass's device arrays; tile per rank from its bucket.
int upload_schedule(rlf_pass *ps, const std::vector<int32_t> &ranks, const std::vector<int64_t> &cells,
                    const int tiles[kBuckets]) {
  rlf_ctx *c = ps->c;
  const int n = (int)ranks.size();
  std::vector<int64_t> start((size_t)n + 1, 0);
  std::vector<int32_t> tile((size_t)n);
  for (int r = 0; r < n; ++r) {
    const int t = tiles[bucket_of(cells[(size_t)ranks[(size_t)r]])];
    tile[(size_t)r] = t;
    const int64_t per = 64LL * t;
    start[(size_t)r + 1] = start[(size_t)r] + (c->n_valid + per - 1) / per;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(ps->d_order, ranks.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(ps->d_item_start, start.data(), sizeof(int64_t) * ((size_t)n + 1), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(ps->d_tile, tile.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
  ps->q.order = ps->d_order;
  ps->q.item_start = ps->d_item_start;
  ps->q.tile = ps->d_tile;
  ps->q.n_rank = n;
  ps->q.n_items = start[(size_t)n];
  ps->q.counter = ps->d_counter;
  return RLF_OK;
}

std::string table_key(const rlf_ctx *c, int b) {
  std::ostringstream k;
  k << (c->p.precision == RLF_MIXED ? "mixed" : "fp64") << " " << c->p.num_r << " " << b;
  return k.str();
}

std::map<std::string, int> read_table(const char *path) {
  std::map<std::string, int> t;
  if (!path) return t;
  std::ifstream in(path);
  std::string prec, line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string p;
    int r, b, tile;
    if (ls >> p >> r >> b >> tile) {
      std::ostringstream k;
      k << p << " " << r << " " << b;
      t[k.str()] = tile;
    }
  }
  return t;
}

void write_table(const char *path, const std::map<std::string, int> &t) {
  if (!path) return;
  std::ofstream out(path, std::ios::trunc);
  out << "# likelihood work-queue tiles: precision num_r bucket(cells <256,<1024,<4096,>=4096) tile\n";
  for (const auto &kv : t) out << kv.first << " " << kv.second << "\n";
}

// Time the queue kernel on one bucket's sources for each candidate tile.
int autotune(rlf_pass *ps, const std::vector<int32_t> &ranks, const std::vector<int64_t> &cells, const char *path) {
  rlf_ctx *c = ps->c;
  std::map<std::string, int> table = read_table(path);
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  int rc = RLF_OK;
  bool changed = false;
  for (int b = 0; b < kBuckets && rc == RLF_OK; ++b) {
    std::vector<int32_t> sub;
    for (int32_t s : ranks)
      if (bucket_of(cells[(size_t)s]) == b) sub.push_back(s);
    if (sub.empty()) continue;
    auto it = table.find(table_key(c, b));
    if (it != table.end()) {
      ps->tiles[b] = it->second;
      ps->tuned[b] = 2;
      continue;
    }
    float best = 1e30f;
    for (int cand : kCandidates) {
      int tl[kBuckets];
      std::fill(tl, tl + kBuckets, cand);
      if ((rc = upload_schedule(ps, sub, cells, tl))) break;
      float ms = 1e30f;
      for (int rep = 0; rep < 2 && rc == RLF_OK; ++rep) {
        hipEventRecord(e0, c->stream);
        if ((rc = rlf::enqueue_fit(c, ps->f, rlf_fit_opts{}, ps->out, &ps->q, ps->blocks))) break;
        hipEventRecord(e1, c->stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = hip_fail(c, hipGetLastError(), "autotune timing");
          break;
        }
        float t = 0.f;
        hipEventElapsedTime(&t, e0, e1);
        ms = std::min(ms, t);
      }
      if (ms < best) {
        best = ms;
        ps->tiles[b] = cand;
      }
    }
    ps->tuned[b] = 1;
    table[table_key(c, b)] = ps->tiles[b];
    changed = true;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc == RLF_OK && changed) write_table(path, table);
  return rc;
}

void pass_release(rlf_pass *ps) {
  if (ps->exec) (void)hipGraphExecDestroy(ps->exec);
  if (ps->graph) (void)hipGraphDestroy(ps->graph);
  if (ps->cs) (void)hipStreamDestroy(ps->cs);
  dfree(ps->d_order);
  dfree(ps->d_item_start);
  dfree(ps->d_tile);
  dfree(ps->d_counter);
}

}  // namespace

extern "C" {

int rlf_pass_create(rlf_ctx *c, const rlf_obs *obs, const rlf_catalog *cat, rlf_facets *f,
                    const rlf_fit_opts *opts, const rlf_fit_out *out, const char *tune_path, rlf_pass **res) {
  if (!c) return RLF_EINVAL;
  if (!res || !out || !out->flags || !f || f->ctx != c || !obs || !cat)
    return fail(c, RLF_EINVAL, "rlf_pass_create: NULL argument or facets from another context");
  rlf_fit_opts o{};
  if (opts) o = *opts;
  if ((o.mode != 0 && o.mode != 1) || (o.mode == 1 && !o.window) ||
      (o.check_stride != 0 && (o.mode != 1 || !o.fallback || o.check_stride < 2 || o.check_stride >= c->p.n_e)))
    return fail(c, RLF_EINVAL, "rlf_pass_create: fit options");
  if (o.want_surface && !out->surface) return fail(c, RLF_EINVAL, "want_surface needs out.surface");
  HIPCHK(c, hipSetDevice(c->device));
  rlf_pass *ps = new (std::nothrow) rlf_pass();
  if (!ps) return fail(c, RLF_ENOMEM, "host allocation");
  ps->c = c;
  ps->f = f;
  ps->opts = o;
  ps->out = *out;
  int rc = RLF_OK;
  do {
    // one eager pass: validates the inputs, fixes the facet cells (they depend
    // only on geometry and weights) and leaves every table uploaded
    if ((rc = rlf_extract_facets(c, obs, cat, nullptr, f))) break;
    std::vector<int64_t> off((size_t)f->n_src + 1);
    if (hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(off.data(), f->cells.offsets, sizeof(int64_t) * off.size(), hipMemcpyDeviceToHost) != hipSuccess) {
      rc = hip_fail(c, hipGetLastError(), "rlf_pass_create: reading facet sizes");
      break;
    }
    std::vector<int64_t> cells((size_t)f->n_src);
    std::vector<int32_t> ranks((size_t)f->n_src);
    for (int64_t s = 0; s < f->n_src; ++s) {
      cells[(size_t)s] = off[(size_t)s + 1] - off[(size_t)s];
      ranks[(size_t)s] = (int32_t)s;
    }
    std::stable_sort(ranks.begin(), ranks.end(),
                     [&](int32_t a, int32_t b) { return cells[(size_t)a] > cells[(size_t)b]; });
    if ((rc = dalloc(c, &ps->d_order, f->n_src))) break;
    if ((rc = dalloc(c, &ps->d_item_start, f->n_src + 1))) break;
    if ((rc = dalloc(c, &ps->d_tile, f->n_src))) break;
    if ((rc = dalloc(c, &ps->d_counter, 1))) break;
    int dev_cus = 0;
    if (hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) dev_cus = 256;
    ps->blocks = dev_cus * rlf::fit_queue_blocks_per_cu(f->mixed, c->p.num_r);
    if ((rc = autotune(ps, ranks, cells, tune_path))) break;
    if ((rc = upload_schedule(ps, ranks, cells, ps->tiles))) break;
    // capture on a stream of our own (a graph cannot be captured on the legacy stream)
    if (hipStreamCreateWithFlags(&ps->cs, hipStreamNonBlocking) != hipSuccess) {
      rc = hip_fail(c, hipGetLastError(), "hipStreamCreate");
      break;
    }
    hipStream_t user = c->stream;
    c->stream = ps->cs;
    hipError_t e = hipStreamBeginCapture(ps->cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      rc = rlf_extract_facets(c, obs, cat, nullptr, f);
      if (rc == RLF_OK) rc = rlf::enqueue_fit(c, f, o, ps->out, &ps->q, ps->blocks);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(ps->cs, &g);
      ps->graph = g;
    }
    c->stream = user;
    if (rc != RLF_OK) break;
    if (e != hipSuccess) {
      rc = hip_fail(c, e, "graph capture");
      break;
    }
    e = hipGraphInstantiate(&ps->exec, ps->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      rc = hip_fail(c, e, "hipGraphInstantiate");
      break;
    }
  } while (0);
  if (rc != RLF_OK) {
    pass_release(ps);
    delete ps;
    return rc;
  }
  *res = ps;
  return RLF_OK;
}

int rlf_pass_launch(rlf_pass *ps) {
  if (!ps || !ps->exec) return RLF_EINVAL;
  rlf_ctx *c = ps->c;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipGraphLaunch(ps->exec, c->stream));
  return RLF_OK;
}

int rlf_pass_tiles(const rlf_pass *ps, int32_t *tiles, int32_t *tuned) {
  if (!ps) return RLF_EINVAL;
  for (int b = 0; b < kBuckets; ++b) {
    if (tiles) tiles[b] = ps->tiles[b];
    if (tuned) tuned[b] = ps->tuned[b];
  }
  return RLF_OK;
}

int rlf_pass_free(rlf_pass *ps) {
  if (!ps) return RLF_OK;
  (void)hipSetDevice(ps->c->device);
  (void)hipStreamSynchronize(ps->c->stream);
  if (ps->cs) (void)hipStreamSynchronize(ps->cs);
  pass_release(ps);
  delete ps;
  return RLF_OK;
}

}  // extern "C"
