// Grid-narrowing network: parameters (FP32 master + BF16 copies), Adam state,
// activation buffers, and the forward / training / window entry points.
// Parameter layout (FP32, contiguous): W1 [8192 x 512], b1 [512],
// W2 [512 x 512], b2, W3 [512 x 512], b3, W4 [512 x 6], b4 [6].
#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rlf_objects.h"

namespace {

constexpr int kIn = 8192, kHid = 512, kOut = 6;
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kIn * kHid;
constexpr int64_t kOffW2 = kOffB1 + kHid;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kHid * kHid;
constexpr int64_t kOffW3 = kOffB2 + kHid;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kHid * kHid;
constexpr int64_t kOffW4 = kOffB3 + kHid;
constexpr int64_t kOffB4 = kOffW4 + (int64_t)kHid * kOut;
constexpr int64_t kParams = kOffB4 + kOut;

}  // namespace

struct rlf_mlp {
  rlf_ctx *c = nullptr;
  int64_t max_batch = 0;
  int64_t step = 0;
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  __bf16 *wb = nullptr;
  float *z[3] = {nullptr, nullptr, nullptr};
  __bf16 *h[3] = {nullptr, nullptr, nullptr};
  float *y = nullptr, *cbuf = nullptr, *dy = nullptr, *dh = nullptr;
  float *ws = nullptr;                       // split-K partial products, column-sum slices
  __bf16 *dyb = nullptr, *dzb = nullptr;
  // k-contiguous operands of the NT GEMM: the BF16 weights transposed per
  // layer (W_l^T [out x in] at the offsets of W_l), and per batch the layer
  // input and the gradient dZ transposed ([in x rows], [512 x rows])
  __bf16 *wbt = nullptr;
  __bf16 *xt = nullptr, *ht = nullptr, *dzt = nullptr;
  __bf16 *xf = nullptr;                      // network inputs of a facet object's sources [max_batch x 8192]
};

namespace {

using rlf::dalloc;
using rlf::dfree;
using rlf::fail;
using rlf::hip_fail;

void mlp_release(rlf_mlp *n) {
  dfree(n->w);
  dfree(n->m);
  dfree(n->v);
  dfree(n->g);
  dfree(n->wb);
  for (int l = 0; l < 3; ++l) {
    dfree(n->z[l]);
    dfree(n->h[l]);
  }
  dfree(n->y);
  dfree(n->cbuf);
  dfree(n->dy);
  dfree(n->dh);
  dfree(n->dyb);
  dfree(n->dzb);
  dfree(n->ws);
  dfree(n->wbt);
  dfree(n->xt);
  dfree(n->ht);
  dfree(n->dzt);
  dfree(n->xf);
}

constexpr int kMaxSplitBlocks = 512;                  // tiles x K slices
constexpr int64_t kWsFloats = (int64_t)kMaxSplitBlocks * 128 * 128;

int split_for(int M, int N, int K) {
  const int tiles = ((M + 127) / 128) * ((N + 127) / 128);
  int s = 1;
  while (tiles * s * 2 <= kMaxSplitBlocks && K / (s * 2) >= 64) s *= 2;
  return s;
}

// C[M x N] = A * B with element strides (see GemmArgs).
int gemm(rlf_mlp *net, const __bf16 *a, int64_t sam, int64_t sak, const __bf16 *b, int64_t sbk, int64_t sbn,
         float *out, int M, int N, int K) {
  rlf_ctx *c = net->c;
  GemmArgs ga{};
  ga.a = a;
  ga.sam = sam;
  ga.sak = sak;
  ga.b = b;
  ga.sbk = sbk;
  ga.sbn = sbn;
  ga.c = out;
  ga.ldc = N;
  ga.M = M;
  ga.N = N;
  ga.K = K;
  ga.ws = net->ws;
  ga.ws_floats = kWsFloats;
  hipError_t e = launch_gemm(ga, split_for(M, N, K), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "gemm launch");
  return RLF_OK;
}

// Split of K for the NT GEMM: slices of at least 512 until the grid fills
// the 256 CUs once, then slices of at least 1024 up to two blocks per CU
// (each slice's partial product is written and read back once by the
// reduction, which costs more than it saves on shorter slices).  Measured
// on the network's products: 4096 x 512 x 8192 best at 4 slices, 8192 x 512
// x 4096 at 2, 512 x 512 x 8192 at 16, the 512-deep products unsplit.
int split_nt(int M, int N, int K) {
  const int64_t tiles = (int64_t)((M + 127) / 128) * ((N + 127) / 128);
  int s = 1;
  for (;;) {
    const int64_t s2 = 2 * s;
    const bool fill = tiles * s2 <= 256 && K / s2 >= 512;
    const bool twice = tiles * s2 <= kMaxSplitBlocks && K / s2 >= 1024;
    if (!(fill || twice) || s2 * M * N > kWsFloats) break;
    s = (int)s2;
  }
  return s;
}

// C[M x N] (row stride ldc) = sum_k A[m lda + k] B[n ldb + k].
int gemm_nt(rlf_mlp *net, const __bf16 *a, int64_t lda, const __bf16 *b, int64_t ldb, float *out, int64_t ldc, int M,
            int N, int K) {
  GemmNTArgs ga{};
  ga.a = a;
  ga.lda = lda;
  ga.b = b;
  ga.ldb = ldb;
  ga.c = out;
  ga.ldc = ldc;
  ga.M = M;
  ga.N = N;
  ga.K = K;
  ga.ws = net->ws;
  ga.ws_floats = kWsFloats;
  hipError_t e = launch_gemm_nt(ga, split_nt(M, N, K), net->c->stream);
  if (e != hipSuccess) return hip_fail(net->c, e, "gemm_nt launch");
  return RLF_OK;
}

// The transposed BF16 weights W_l^T [out x in] from W_l [in x out].
int update_wbt(rlf_mlp *n) {
  const int64_t offW[4] = {kOffW1, kOffW2, kOffW3, kOffW4};
  const int64_t din[4] = {kIn, kHid, kHid, kHid}, dout[4] = {kHid, kHid, kHid, kOut};
  TransposeJob jobs[4];
  for (int l = 0; l < 4; ++l) jobs[l] = TransposeJob{n->wb + offW[l], din[l], dout[l], n->wbt + offW[l]};
  hipError_t e = launch_transpose_bf16(jobs, 4, n->c->stream);
  if (e != hipSuccess) return hip_fail(n->c, e, "weight transpose launch");
  return RLF_OK;
}

// Forward of rows [0, nb) of x into the layer buffers; y_out receives the outputs.
int forward_chunk(rlf_mlp *n, const __bf16 *x, int nb, float *y_out) {
  rlf_ctx *c = n->c;
  const __bf16 *hin = x;
  int kin = kIn;
  const int64_t offW[3] = {kOffW1, kOffW2, kOffW3}, offB[3] = {kOffB1, kOffB2, kOffB3};
  for (int l = 0; l < 3; ++l) {
    // z = h W: rows of h and of W^T are both contiguous along the contraction
    if (int e = gemm_nt(n, hin, kin, n->wbt + offW[l], kin, n->cbuf, kHid, nb, kHid, kin)) return e;
    hipError_t e = launch_bias_act(n->cbuf, n->w + offB[l], nb, kHid, n->z[l], n->h[l], 1, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "bias/GELU launch");
    hin = n->h[l];
    kin = kHid;
  }
  hipError_t e = launch_out_forward(hin, n->wb + kOffW4, n->w + kOffB4, nb, y_out, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "output layer launch");
  return RLF_OK;
}

}  // namespace

extern "C" {

int64_t rlf_mlp_num_params(void) { return kParams; }

int rlf_mlp_create(rlf_ctx *c, int64_t max_batch, rlf_mlp **out) {
  if (!c) return RLF_EINVAL;
  if (!out || max_batch < 1 || max_batch > (1 << 20)) return fail(c, RLF_EINVAL, "rlf_mlp_create: max_batch");
  HIPCHK(c, hipSetDevice(c->device));
  rlf_mlp *n = new (std::nothrow) rlf_mlp();
  if (!n) return fail(c, RLF_ENOMEM, "host allocation");
  n->c = c;
  n->max_batch = max_batch;
  const int64_t B = max_batch;
  int rc = RLF_OK;
  do {
    if ((rc = dalloc(c, &n->w, kParams))) break;
    if ((rc = dalloc(c, &n->m, kParams))) break;
    if ((rc = dalloc(c, &n->v, kParams))) break;
    if ((rc = dalloc(c, &n->g, kParams))) break;
    if ((rc = dalloc(c, &n->wb, kParams))) break;
    for (int l = 0; l < 3 && rc == RLF_OK; ++l) {
      if ((rc = dalloc(c, &n->z[l], B * kHid))) break;
      rc = dalloc(c, &n->h[l], B * kHid);
    }
    if (rc) break;
    if ((rc = dalloc(c, &n->y, B * kOut))) break;
    if ((rc = dalloc(c, &n->cbuf, B * kHid))) break;
    if ((rc = dalloc(c, &n->dy, B * kOut))) break;
    if ((rc = dalloc(c, &n->dyb, B * kOut))) break;
    if ((rc = dalloc(c, &n->dh, B * kHid))) break;
    if ((rc = dalloc(c, &n->dzb, B * kHid))) break;
    if ((rc = dalloc(c, &n->ws, kWsFloats))) break;
    if ((rc = dalloc(c, &n->wbt, kParams))) break;
    if ((rc = dalloc(c, &n->xt, B * kIn))) break;
    if ((rc = dalloc(c, &n->ht, B * kHid))) break;
    if ((rc = dalloc(c, &n->dzt, B * kHid))) break;
    if ((rc = dalloc(c, &n->xf, B * kIn))) break;
    hipError_t e = hipMemset(n->w, 0, sizeof(float) * kParams);
    if (e == hipSuccess) e = hipMemset(n->m, 0, sizeof(float) * kParams);
    if (e == hipSuccess) e = hipMemset(n->v, 0, sizeof(float) * kParams);
    if (e == hipSuccess) e = hipMemset(n->wb, 0, sizeof(__bf16) * kParams);
    if (e == hipSuccess) e = hipMemset(n->wbt, 0, sizeof(__bf16) * kParams);
    if (e != hipSuccess) rc = hip_fail(c, e, "rlf_mlp_create: clearing parameters");
  } while (0);
  if (rc) {
    mlp_release(n);
    delete n;
    return rc;
  }
  *out = n;
  return RLF_OK;
}

int rlf_mlp_free(rlf_mlp *n) {
  if (!n) return RLF_OK;
  (void)hipSetDevice(n->c->device);
  (void)hipStreamSynchronize(n->c->stream);
  mlp_release(n);
  delete n;
  return RLF_OK;
}

int rlf_mlp_set_state(rlf_mlp *n, const float *params_host, const float *m_host, const float *v_host, int64_t step) {
  if (!n || !params_host || step < 0) return RLF_EINVAL;
  rlf_ctx *c = n->c;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(n->w, params_host, sizeof(float) * kParams, hipMemcpyHostToDevice));
  if (m_host) HIPCHK(c, hipMemcpy(n->m, m_host, sizeof(float) * kParams, hipMemcpyHostToDevice));
  else HIPCHK(c, hipMemset(n->m, 0, sizeof(float) * kParams));
  if (v_host) HIPCHK(c, hipMemcpy(n->v, v_host, sizeof(float) * kParams, hipMemcpyHostToDevice));
  else HIPCHK(c, hipMemset(n->v, 0, sizeof(float) * kParams));
  n->step = step;
  HIPCHK(c, launch_to_bf16(n->w, n->wb, kParams, c->stream));
  if (int e = update_wbt(n)) return e;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RLF_OK;
}

int rlf_mlp_get_state(rlf_mlp *n, float *params_host, float *m_host, float *v_host, float *grad_host, int64_t *step) {
  if (!n) return RLF_EINVAL;
  rlf_ctx *c = n->c;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (params_host) HIPCHK(c, hipMemcpy(params_host, n->w, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  if (m_host) HIPCHK(c, hipMemcpy(m_host, n->m, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  if (v_host) HIPCHK(c, hipMemcpy(v_host, n->v, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  if (grad_host) HIPCHK(c, hipMemcpy(grad_host, n->g, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  if (step) *step = n->step;
  return RLF_OK;
}

namespace {

constexpr char kCkptMagic[8] = {'R', 'L', 'F', 'M', 'L', 'P', '0', '1'};
constexpr uint32_t kCkptVersion = 1;

struct CkptHeader {
  char magic[8];
  uint32_t version;
  uint32_t reserved;
  int64_t n_params;
  int64_t step;
  uint64_t hash;
};
static_assert(sizeof(CkptHeader) == 40, "checkpoint header layout");

// FNV-1a, 64 bit (offset basis 14695981039346656037, prime 1099511628211).
uint64_t fnv1a(const void *data, size_t n, uint64_t h) {
  const unsigned char *p = static_cast<const unsigned char *>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

uint64_t payload_hash(const std::vector<float> &buf) {
  return fnv1a(buf.data(), buf.size() * sizeof(float), 14695981039346656037ull);
}

}  // namespace

int rlf_mlp_save(rlf_mlp *n, const char *path) {
  if (!n) return RLF_EINVAL;
  rlf_ctx *c = n->c;
  c->err.clear();
  if (!path || !*path) return fail(c, RLF_EINVAL, "rlf_mlp_save: path is NULL or empty");
  std::vector<float> buf;
  try {
    buf.resize(3 * (size_t)kParams);
  } catch (...) {
    return fail(c, RLF_ENOMEM, "rlf_mlp_save: host buffer");
  }
  int64_t step = 0;
  if (int e = rlf_mlp_get_state(n, buf.data(), buf.data() + kParams, buf.data() + 2 * kParams, nullptr, &step))
    return e;
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = kCkptVersion;
  h.n_params = kParams;
  h.step = step;
  h.hash = payload_hash(buf);
  const std::string tmp = std::string(path) + ".tmp";
  FILE *fp = std::fopen(tmp.c_str(), "wb");
  if (!fp) return fail(c, RLF_EIO, "rlf_mlp_save: cannot open " + tmp + ": " + std::strerror(errno));
  const bool ok = std::fwrite(&h, sizeof h, 1, fp) == 1 &&
                  std::fwrite(buf.data(), sizeof(float), buf.size(), fp) == buf.size() && std::fflush(fp) == 0;
  const bool closed = std::fclose(fp) == 0;
  if (!ok || !closed) {
    std::remove(tmp.c_str());
    return fail(c, RLF_EIO, "rlf_mlp_save: write to " + tmp + " failed");
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return fail(c, RLF_EIO, std::string("rlf_mlp_save: cannot rename onto ") + path + ": " + std::strerror(errno));
  }
  return RLF_OK;
}

int rlf_mlp_load(rlf_mlp *n, const char *path) {
  if (!n) return RLF_EINVAL;
  rlf_ctx *c = n->c;
  c->err.clear();
  if (!path || !*path) return fail(c, RLF_EINVAL, "rlf_mlp_load: path is NULL or empty");
  FILE *fp = std::fopen(path, "rb");
  if (!fp) return fail(c, RLF_EIO, std::string("rlf_mlp_load: cannot open ") + path + ": " + std::strerror(errno));
  CkptHeader h{};
  std::vector<float> buf;
  std::string why;
  if (std::fread(&h, sizeof h, 1, fp) != 1) why = "file shorter than the header";
  else if (std::memcmp(h.magic, kCkptMagic, 8) != 0) why = "not a network checkpoint (magic)";
  else if (h.version != kCkptVersion) why = "format version " + std::to_string(h.version);
  else if (h.n_params != kParams) why = "parameter count " + std::to_string(h.n_params) + " of another network";
  else if (h.step < 0) why = "negative step count";
  if (why.empty()) {
    try {
      buf.resize(3 * (size_t)kParams);
    } catch (...) {
      std::fclose(fp);
      return fail(c, RLF_ENOMEM, "rlf_mlp_load: host buffer");
    }
    if (std::fread(buf.data(), sizeof(float), buf.size(), fp) != buf.size()) why = "payload truncated";
    else if (std::fgetc(fp) != EOF) why = "bytes after the payload";
    else if (payload_hash(buf) != h.hash) why = "payload hash mismatch";
  }
  std::fclose(fp);
  if (!why.empty()) return fail(c, RLF_EIO, std::string("rlf_mlp_load: ") + path + ": " + why);
  return rlf_mlp_set_state(n, buf.data(), buf.data() + kParams, buf.data() + 2 * kParams, h.step);
}

namespace {

// Network inputs of sources [s0, s0 + count) of facet object f into x.
hipError_t facet_features(const rlf_facets *f, int64_t s0, int64_t count, __bf16 *x, hipStream_t st) {
  FeatureArgs a{};
  a.s0 = (int32_t)s0;
  a.n_src = (int32_t)count;
  a.offsets = f->cells.offsets;
  a.ix = f->cells.ix;
  a.iy = f->cells.iy;
  a.vre = f->cells.vre;
  a.vim = f->cells.vim;
  a.src = f->d_src;
  a.spec_norm = f->spec_norm;
  a.x = x;
  return launch_features(a, st);
}

}  // namespace

int rlf_mlp_features(rlf_ctx *c, const rlf_facets *f, void *x) {
  if (!c) return RLF_EINVAL;
  if (!f || f->ctx != c || !x) return fail(c, RLF_EINVAL, "rlf_mlp_features: arguments");
  HIPCHK(c, hipSetDevice(c->device));
  if (f->n_src == 0) return RLF_OK;
  HIPCHK(c, facet_features(f, 0, f->n_src, reinterpret_cast<__bf16 *>(x), c->stream));
  return RLF_OK;
}

int rlf_mlp_predict(rlf_mlp *n, const rlf_facets *f, float *y) {
  if (!n) return RLF_EINVAL;
  rlf_ctx *c = n->c;
  if (!f || f->ctx != c || !y) return fail(c, RLF_EINVAL, "rlf_mlp_predict: arguments");
  HIPCHK(c, hipSetDevice(c->device));
  for (int64_t s0 = 0; s0 < f->n_src; s0 += n->max_batch) {
    const int nb = (int)std::min<int64_t>(n->max_batch, f->n_src - s0);
    HIPCHK(c, facet_features(f, s0, nb, n->xf, c->stream));
    if (int e = forward_chunk(n, n->xf, nb, y + s0 * kOut)) return e;
  }
  return RLF_OK;
}

int rlf_mlp_train_facets(rlf_mlp *n, const rlf_facets *f, const float *target, float lr, double *loss) {
  if (!n) return RLF_EINVAL;
  rlf_ctx *c = n->c;
  if (!f || f->ctx != c || !target || !loss || f->n_src < 1 || f->n_src > n->max_batch)
    return fail(c, RLF_EINVAL, "rlf_mlp_train_facets: arguments (1 <= n_src <= max_batch)");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, facet_features(f, 0, f->n_src, n->xf, c->stream));
  return rlf_mlp_train_step(n, n->xf, target, f->n_src, lr, loss);
}

int rlf_mlp_forward(rlf_mlp *n, const void *x, int64_t rows, float *y) {
  if (!n) return RLF_EINVAL;
  rlf_ctx *c = n->c;
  if (!x || !y || rows < 1) return fail(c, RLF_EINVAL, "rlf_mlp_forward: arguments");
  HIPCHK(c, hipSetDevice(c->device));
  const __bf16 *xb = reinterpret_cast<const __bf16 *>(x);
  for (int64_t r0 = 0; r0 < rows; r0 += n->max_batch) {
    const int nb = (int)std::min<int64_t>(n->max_batch, rows - r0);
    if (int e = forward_chunk(n, xb + r0 * kIn, nb, y + r0 * kOut)) return e;
  }
  return RLF_OK;
}

int rlf_mlp_train_step(rlf_mlp *n, const void *x, const float *target, int64_t rows, float lr, double *loss) {
  if (!n) return RLF_EINVAL;
  rlf_ctx *c = n->c;
  if (!x || !target || !loss || rows < 1 || rows > n->max_batch || !(lr >= 0))
    return fail(c, RLF_EINVAL, "rlf_mlp_train_step: arguments (rows must be <= max_batch)");
  HIPCHK(c, hipSetDevice(c->device));
  const int nb = (int)rows;
  const __bf16 *xb = reinterpret_cast<const __bf16 *>(x);
  if (int e = forward_chunk(n, xb, nb, n->y)) return e;
  HIPCHK(c, launch_head(n->y, target, nb, n->dy, n->dyb, loss, c->stream));
  // output layer: dW4 = h3^T dY, db4 = sum dY (together, in the parameters'
  // order), dh3 = dY W4^T
  static_assert(kOffB4 == kOffW4 + (int64_t)kHid * kOut, "b4 follows W4");
  HIPCHK(c, launch_out_backward(n->h[2], n->dyb, n->dy, nb, n->wb + kOffW4, n->g + kOffW4, n->dh, n->ws, kWsFloats,
                                c->stream));
  const int64_t offW[3] = {kOffW1, kOffW2, kOffW3}, offB[3] = {kOffB1, kOffB2, kOffB3};
  // the NT GEMM needs the batch dimension in multiples of 8 for the weight gradients
  const bool nt_rows = nb % 8 == 0;
  for (int l = 2; l >= 0; --l) {
    HIPCHK(c, launch_gelu_back_colsum(n->dh, n->z[l], nb, kHid, n->dzb, n->g + offB[l], n->ws, kWsFloats,
                                      c->stream));
    const __bf16 *hin = l == 0 ? xb : n->h[l - 1];
    const int kin = l == 0 ? kIn : kHid;
    if (nt_rows) {
      // dW = h^T dZ with both operands transposed to [features x rows]
      __bf16 *hin_t = l == 0 ? n->xt : n->ht;
      const TransposeJob jobs[2] = {{hin, nb, kin, hin_t}, {n->dzb, nb, kHid, n->dzt}};
      HIPCHK(c, launch_transpose_bf16(jobs, 2, c->stream));
      if (int e = gemm_nt(n, hin_t, nb, n->dzt, nb, n->g + offW[l], kHid, kin, kHid, nb)) return e;
    } else {
      if (int e = gemm(n, hin, 1, kin, n->dzb, kHid, 1, n->g + offW[l], kin, kHid, nb)) return e;
    }
    // dh = dZ W^T: rows of dZ and of W both run along the output index
    if (l > 0)
      if (int e = gemm_nt(n, n->dzb, kHid, n->wb + offW[l], kHid, n->dh, kHid, nb, kHid, kHid)) return e;
  }
  n->step += 1;
  HIPCHK(c, launch_adam(n->w, n->wb, n->g, n->m, n->v, kParams, lr, n->step, c->stream));
  if (int e = update_wbt(n)) return e;
  return RLF_OK;
}

int rlf_mlp_posterior_targets(rlf_ctx *c, const double *e1, const double *e2, const double *s1, const double *s2,
                              const float *ln_alpha, int64_t rows, double kappa, uint64_t seed, float *target) {
  if (!c) return RLF_EINVAL;
  if (!e1 || !e2 || !s1 || !s2 || !ln_alpha || !target || rows < 1 || !(kappa >= 0.0) || !std::isfinite(kappa))
    return fail(c, RLF_EINVAL, "rlf_mlp_posterior_targets: arguments");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, launch_posterior_targets(e1, e2, s1, s2, ln_alpha, rows, kappa, seed, target, c->stream));
  return RLF_OK;
}

int rlf_mlp_windows(rlf_ctx *c, const float *y, int64_t rows, double nsigma, int32_t min_half, double full_frac,
                    int32_t *window) {
  if (!c) return RLF_EINVAL;
  if (!y || !window || rows < 1 || !(nsigma > 0) || min_half < 0 || !(full_frac >= 0.0 && full_frac <= 1.0))
    return fail(c, RLF_EINVAL, "rlf_mlp_windows: arguments");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, launch_windows(y, rows, nsigma, c->p.n_e, c->p.e_step, min_half, full_frac, window, c->stream));
  return RLF_OK;
}

}  // extern "C"
