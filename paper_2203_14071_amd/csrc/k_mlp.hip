// The grid-narrowing network: features, BF16 MFMA GEMM, epilogues, loss,
// back-propagation helpers, Adam, and the window boxes.
//
// GEMM: C[M x N] (FP32) = A[M x K] * B[K x N], A and B BF16 with arbitrary
// element strides (so X W, dZ W^T and H^T dZ all use one kernel).  Block tile
// 128 x 128 x 32, four waves each owning a 64 x 64 quarter as 2 x 2
// v_mfma_f32_32x32x16_bf16 tiles.  Operand fragments of that instruction:
// lane l holds A[l%32][8(l/32)+t] and B[8(l/32)+t][l%32] (t = 0..7) and
// accumulator r of lane l is C[8(r/4) + 4(l/32) + r%4][l%32].  LDS keeps the
// A tile as [m][k] and the B tile as [n][k] (k contiguous, padded by 8), so
// each fragment is one 16-byte LDS read.  Global loads take 8 contiguous
// BF16 when the operand is contiguous along k (or along m / n, transposing
// into LDS), else single elements; out-of-range elements are zero.
// grid.z splits K; with more than one split each slice writes its partial
// product to a workspace and a second kernel adds the slices in a fixed
// order, so results do not depend on scheduling.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>

#include "rlf_internal.h"

namespace rlf {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBM = 128, kBN = 128, kBK = 32, kPad = 8, kLd = kBK + kPad;
constexpr float kLogVarMin = -6.9077552789821368f;   // ln(1e-3)
constexpr double kFeatureClip = 4.0;

__device__ __forceinline__ __bf16 to_bf16(float x) { return __float2bfloat16(x); }

// Stage rows [r0, r0+128) x k [k0, k0+32) of an operand whose element (r, k)
// is at p[r*sr + k*sk] into lds[r][k]; rows >= nr or k >= nk read as zero.
__device__ __forceinline__ void stage(__bf16 *lds, const __bf16 *__restrict__ p, int64_t sr, int64_t sk, int r0,
                                      int nr, int k0, int nk) {
  const int t = threadIdx.x;
  if (sk == 1 && (sr % 8) == 0) {
    // 128 rows x 4 chunks of 8 k: 512 chunks, 2 per thread
    for (int c = t; c < kBM * (kBK / 8); c += 256) {
      const int r = c / (kBK / 8), kc = (c % (kBK / 8)) * 8;
      const int gr = r0 + r, gk = k0 + kc;
      bf16x8 v;
      if (gr < nr && gk + 8 <= nk) {
        v = *reinterpret_cast<const bf16x8 *>(p + (int64_t)gr * sr + gk);
      } else {
        for (int e = 0; e < 8; ++e)
          v[e] = (gr < nr && gk + e < nk) ? p[(int64_t)gr * sr + (int64_t)(gk + e)] : to_bf16(0.0f);
      }
      *reinterpret_cast<bf16x8 *>(lds + r * kLd + kc) = v;
    }
  } else if (sr == 1 && (sk % 8) == 0) {
    // contiguous along rows: 32 k x 16 chunks of 8 rows
    for (int c = t; c < kBK * (kBM / 8); c += 256) {
      const int k = c / (kBM / 8), rc = (c % (kBM / 8)) * 8;
      const int gk = k0 + k, gr = r0 + rc;
      bf16x8 v;
      if (gk < nk && gr + 8 <= nr) {
        v = *reinterpret_cast<const bf16x8 *>(p + (int64_t)gk * sk + gr);
      } else {
        for (int e = 0; e < 8; ++e)
          v[e] = (gk < nk && gr + e < nr) ? p[(int64_t)gk * sk + (int64_t)(gr + e)] : to_bf16(0.0f);
      }
      for (int e = 0; e < 8; ++e) lds[(rc + e) * kLd + k] = v[e];
    }
  } else {
    for (int c = t; c < kBM * kBK; c += 256) {
      const int r = c / kBK, k = c % kBK;
      const int gr = r0 + r, gk = k0 + k;
      lds[r * kLd + k] = (gr < nr && gk < nk) ? p[(int64_t)gr * sr + (int64_t)gk * sk] : to_bf16(0.0f);
    }
  }
}

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 sa[kBM * kLd];
  __shared__ __attribute__((aligned(16))) __bf16 sb[kBN * kLd];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  const int wm = (wid >> 1) * 64, wn = (wid & 1) * 64;
  // K slices start on kBK boundaries so the 16-byte loads stay aligned
  const int kper = ((g.K + (int)gridDim.z - 1) / (int)gridDim.z + kBK - 1) / kBK * kBK;
  const int kb = blockIdx.z * kper, ke = min(g.K, kb + kper);
  f32x16 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
  for (int k0 = kb; k0 < ke; k0 += kBK) {
    __syncthreads();
    // A tile: rows m, elements A(m, k) = a[m*sam + k*sak]; B tile stored [n][k]: B(k, n) = b[k*sbk + n*sbn]
    stage(sa, g.a, g.sam, g.sak, m0, g.M, k0, ke);
    stage(sb, g.b, g.sbn, g.sbk, n0, g.N, k0, ke);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 16) {
      bf16x8 fa[2], fb[2];
      for (int i = 0; i < 2; ++i)
        fa[i] = *reinterpret_cast<const bf16x8 *>(sa + (wm + i * 32 + (lane & 31)) * kLd + kk + 8 * (lane >> 5));
      for (int j = 0; j < 2; ++j)
        fb[j] = *reinterpret_cast<const bf16x8 *>(sb + (wn + j * 32 + (lane & 31)) * kLd + kk + 8 * (lane >> 5));
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
  }
  float *outp = gridDim.z > 1 ? g.ws + (int64_t)blockIdx.z * g.M * g.N : g.c;
  const int64_t ld = gridDim.z > 1 ? g.N : g.ldc;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int n = n0 + wn + j * 32 + (lane & 31);
        if (m < g.M && n < g.N) outp[(int64_t)m * ld + n] = acc[i][j][r];
      }
}

// GEMM with both operands contiguous along k: C[M x N] (FP32, row stride
// ldc) = sum_k A[m lda + k] B[n ldb + k].  Block tile 128 x 128, k tile 64,
// four waves each owning a 64 x 64 quarter as 2 x 2
// v_mfma_f32_32x32x16_bf16 tiles.  Both k tiles are staged [row][k] in LDS
// (rows padded to 72 BF16, so the eight lanes of one 16-byte read phase hit
// distinct banks) with 16-byte global loads and LDS stores; the LDS holds two
// k tiles and the registers two more, so the global loads of a tile are
// issued two tiles ahead of its MFMAs, and one barrier per tile separates
// the phases.  Rows beyond M or N and k beyond the slice read as
// zero (K a multiple of 8, lda and ldb multiples of 8).  grid.z splits K in
// multiples of 64; with more than one slice each writes its partial product
// to the workspace and k_reduce_split adds the slices in order.
constexpr int kTM = 128, kTN = 128, kTK = 64, kLdT = kTK + 8;

__device__ __forceinline__ void nt_load(bf16x8 (&r)[4], const __bf16 *__restrict__ p, int64_t ld, int r0, int nr,
                                        int k0, int ke) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = threadIdx.x + 256 * j;
    const int row = c >> 3, kc = (c & 7) * 8;
    const int gr = r0 + row, gk = k0 + kc;
    if (gr < nr && gk + 8 <= ke) {
      r[j] = *reinterpret_cast<const bf16x8 *>(p + (int64_t)gr * ld + gk);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) r[j][e] = (gr < nr && gk + e < ke) ? p[(int64_t)gr * ld + gk + e] : to_bf16(0.0f);
    }
  }
}

__device__ __forceinline__ void nt_store(__bf16 *lds, const bf16x8 (&r)[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = threadIdx.x + 256 * j;
    *reinterpret_cast<bf16x8 *>(lds + (c >> 3) * kLdT + (c & 7) * 8) = r[j];
  }
}

// The MFMAs of one k tile from LDS into the wave's 2 x 2 accumulator tiles.
__device__ __forceinline__ void nt_mfma(f32x16 (&acc)[2][2], const __bf16 *A, const __bf16 *B, int wm, int wn,
                                        int lane) {
#pragma unroll
  for (int kk = 0; kk < kTK; kk += 16) {
    bf16x8 fa[2], fb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      fa[i] = *reinterpret_cast<const bf16x8 *>(A + (wm + i * 32 + (lane & 31)) * kLdT + kk + 8 * (lane >> 5));
#pragma unroll
    for (int j = 0; j < 2; ++j)
      fb[j] = *reinterpret_cast<const bf16x8 *>(B + (wn + j * 32 + (lane & 31)) * kLdT + kk + 8 * (lane >> 5));
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
  }
}

// XCD-aware tile order.  Blocks go to the eight XCDs round-robin by linear
// block index; the tile a block computes is chosen so that each XCD takes a
// contiguous run of tiles in (n tile, m tile, k slice) order, i.e. all the
// n tiles of an m tile (which read the same rows of A) share one XCD's L2.
// Without it the four n tiles of a 512-wide product sat on four XCDs and
// each fetched the same A panel.
__device__ __forceinline__ void nt_tile(int &nt, int &mt, int &z) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int n = gx * gy * (int)gridDim.z;
  const int L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int x = L & 7, r = L >> 3, q = n >> 3, rem = n & 7;
  const int T = x * q + min(x, rem) + r;
  nt = T % gx;
  mt = (T / gx) % gy;
  z = T / (gx * gy);
}

__global__ __launch_bounds__(256) void k_gemm_nt(GemmNTArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 sa[2][kTM * kLdT];
  __shared__ __attribute__((aligned(16))) __bf16 sb[2][kTN * kLdT];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int nt, mt, z;
  nt_tile(nt, mt, z);
  const int m0 = mt * kTM, n0 = nt * kTN;
  const int wm = (wid >> 1) * 64, wn = (wid & 1) * 64;
  const int kper = ((g.K + (int)gridDim.z - 1) / (int)gridDim.z + kTK - 1) / kTK * kTK;
  const int kb = z * kper, ke = min(g.K, kb + kper);
  const int T = kb < ke ? (ke - kb + kTK - 1) / kTK : 0;      // k tiles of this slice
  f32x16 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
  // Two register stages: at the start of step t, LDS half t % 2 holds tile t,
  // stage (t + 1) % 2 tile t + 1 and stage t % 2 tile t + 2 (loads in
  // flight).  After the MFMAs of tile t, tile t + 1 goes to the other LDS
  // half and its stage is reloaded with tile t + 3, so a tile's global loads
  // have two steps of MFMAs to arrive.
  bf16x8 ra0[4], rb0[4], ra1[4], rb1[4];
  auto load = [&](bf16x8 (&ra)[4], bf16x8 (&rb)[4], int t) {
    nt_load(ra, g.a, g.lda, m0, g.M, kb + t * kTK, ke);
    nt_load(rb, g.b, g.ldb, n0, g.N, kb + t * kTK, ke);
  };
  if (T > 0) {
    load(ra0, rb0, 0);
    nt_store(sa[0], ra0);
    nt_store(sb[0], rb0);
  }
  if (T > 1) load(ra1, rb1, 1);
  if (T > 2) load(ra0, rb0, 2);
  __syncthreads();
  for (int t = 0; t < T; t += 2) {
    nt_mfma(acc, sa[0], sb[0], wm, wn, lane);
    if (t + 1 < T) {
      nt_store(sa[1], ra1);
      nt_store(sb[1], rb1);
      if (t + 3 < T) load(ra1, rb1, t + 3);
    }
    __syncthreads();
    if (t + 1 >= T) break;
    nt_mfma(acc, sa[1], sb[1], wm, wn, lane);
    if (t + 2 < T) {
      nt_store(sa[0], ra0);
      nt_store(sb[0], rb0);
      if (t + 4 < T) load(ra0, rb0, t + 4);
    }
    __syncthreads();
  }
  float *outp = gridDim.z > 1 ? g.ws + (int64_t)z * g.M * g.N : g.c;
  const int64_t ld = gridDim.z > 1 ? g.N : g.ldc;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int n = n0 + wn + j * 32 + (lane & 31);
        if (m < g.M && n < g.N) outp[(int64_t)m * ld + n] = acc[i][j][r];
      }
}

// dst[c][r] = src[r][c] for BF16 matrices [rows x cols]: 64 x 64 tiles
// through LDS, four BF16 (8 bytes) per global access when the tile is whole
// and the row lengths are multiples of 4, else one element per access.  One
// launch serves several matrices: the blocks run over the tiles of job 0,
// then job 1, ...
struct TransposeBatch {
  int n;
  TransposeJob job[kMaxTransposeJobs];
  int64_t first_tile[kMaxTransposeJobs + 1];   // prefix sums of the jobs' tile counts
  int64_t tiles_x[kMaxTransposeJobs];          // tiles along a job's columns
};

__global__ __launch_bounds__(256) void k_transpose_bf16(TransposeBatch tb) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  __shared__ __bf16 t[64][66];
  const int64_t b = blockIdx.x;
  int jn = 0;
  while (jn + 1 < tb.n && b >= tb.first_tile[jn + 1]) ++jn;
  const TransposeJob &J = tb.job[jn];
  const __bf16 *__restrict__ src = J.src;
  __bf16 *__restrict__ dst = J.dst;
  const int64_t rows = J.rows, cols = J.cols;
  const int64_t local = b - tb.first_tile[jn];
  const int64_t r0 = (local / tb.tiles_x[jn]) * 64, c0 = (local % tb.tiles_x[jn]) * 64;
  const bool whole = r0 + 64 <= rows && c0 + 64 <= cols && (cols % 4) == 0 && (rows % 4) == 0 &&
                     ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 7) == 0;
  if (whole) {
    // 64 rows x 16 groups of 4 columns: 4 per thread
    for (int q = threadIdx.x; q < 64 * 16; q += 256) {
      const int i = q >> 4, c4 = (q & 15) * 4;
      const bf16x4 v = *reinterpret_cast<const bf16x4 *>(src + (r0 + i) * cols + c0 + c4);
      for (int e = 0; e < 4; ++e) t[i][c4 + e] = v[e];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 64 * 16; q += 256) {
      const int j = q >> 4, r4 = (q & 15) * 4;           // output row j = source column c0 + j
      bf16x4 v;
      for (int e = 0; e < 4; ++e) v[e] = t[r4 + e][j];
      *reinterpret_cast<bf16x4 *>(dst + (c0 + j) * rows + r0 + r4) = v;
    }
    return;
  }
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    t[i][tx] = (r < rows && c < cols) ? src[r * cols + c] : to_bf16(0.0f);
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols && r < rows) dst[c * rows + r] = t[tx][i];
  }
}

// One wave per column: lane j adds slices j, j + 64, ... in order, then the
// lanes are added by a fixed butterfly (the same sum on every run).
__global__ __launch_bounds__(256) void k_colsum_join(const float *part, int slices, int cols, float *db) {
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (col >= cols) return;                                   // uniform per wave
  float acc = 0.0f;
  for (int y = lane; y < slices; y += 64) acc += part[(int64_t)y * cols + col];
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d);
  if (lane == 0) db[col] = acc;
}

// c[m][n] = sum over slices z = 0, 1, ... of ws[z][m][n], in that order
__global__ __launch_bounds__(256) void k_reduce_split(const float *ws, int split, int M, int N, float *c,
                                                      int64_t ldc) {
  const int64_t total = (int64_t)M * N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    float acc = ws[i];
    for (int z = 1; z < split; ++z) acc += ws[(int64_t)z * total + i];
    c[(i / N) * ldc + (i % N)] = acc;
  }
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// z = c + b; h = GELU(z) (BF16) or, for the output layer, y = z (FP32)
__global__ __launch_bounds__(256) void k_bias_act(const float *c, const float *b, int64_t rows, int cols, float *z,
                                                  __bf16 *h, int act) {
  const int64_t n = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float v = c[i] + b[i % cols];
    z[i] = v;
    if (act) h[i] = to_bf16(gelu(v));
  }
}

// The output layer (512 -> 6), whose products are too narrow for the MFMA
// tiles: BF16 operands, FP32 sums in a fixed order.
//   forward:  y[r][j] = sum_k h[r][k] W[k][j] + b[j]; a wave per row, lane l
//             sums k = l, l + 64, ..., then a butterfly over the lanes;
//   gradient: dW[k][j] = sum_r h[r][k] dY_bf16[r][j] and db[j] = sum_r dY[r][j]
//             (3,078 values, the order of W4 and b4 in the parameters) as
//             partial sums over slices of 32 rows, then the slices added by a
//             wave per value in a fixed order;
//   input gradient: dh[r][k] = sum_j dY_bf16[r][j] W[k][j], j = 0..5 in order.
constexpr int kOutW = 512 * 6, kOutWB = 512 * 6 + 6;

__global__ __launch_bounds__(256) void k_out_forward(const __bf16 *__restrict__ h, const __bf16 *__restrict__ w,
                                                     const float *__restrict__ b, int64_t rows, float *y) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= rows) return;                                    // whole waves
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int k = lane; k < 512; k += 64) {
    const float hv = (float)h[r * 512 + k];
#pragma unroll
    for (int j = 0; j < 6; ++j) acc[j] = fmaf(hv, (float)w[k * 6 + j], acc[j]);
  }
#pragma unroll
  for (int j = 0; j < 6; ++j)
    for (int d = 32; d > 0; d >>= 1) acc[j] += __shfl_xor(acc[j], d);
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < 6; ++j) y[r * 6 + j] = acc[j] + b[j];
}

__global__ __launch_bounds__(256) void k_out_grad_part(const __bf16 *__restrict__ h, const __bf16 *__restrict__ dyb,
                                                       const float *__restrict__ dy, int64_t rows, int64_t per,
                                                       float *part) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= kOutWB) return;
  const int64_t r0 = (int64_t)blockIdx.y * per, r1 = min(rows, r0 + per);
  const bool wgt = v < kOutW;
  const int k = wgt ? v / 6 : 0, j = wgt ? v - 6 * (v / 6) : v - kOutW;
  float acc = 0.0f;
  // 32 rows per step, their loads issued together; the sum runs in row order
  for (int64_t rb = r0; rb < r1; rb += 32) {
    float a[32], b[32];
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const int64_t r = rb + t;
      const bool in = r < r1;
      a[t] = in ? (wgt ? (float)h[r * 512 + k] : 1.0f) : 0.0f;
      b[t] = in ? (wgt ? (float)dyb[r * 6 + j] : dy[r * 6 + j]) : 0.0f;
    }
#pragma unroll
    for (int t = 0; t < 32; ++t) acc = fmaf(a[t], b[t], acc);
  }
  part[(int64_t)blockIdx.y * kOutWB + v] = acc;
}

// One wave per value: lane l adds slices l, l + 64, ... in order, then the
// lanes are added by a fixed butterfly (the same sum on every run).
__global__ __launch_bounds__(256) void k_out_grad_join(const float *part, int slices, float *out) {
  const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (v >= kOutWB) return;                                  // whole waves
  float acc = 0.0f;
  for (int s = lane; s < slices; s += 64) acc += part[(int64_t)s * kOutWB + v];
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d);
  if (lane == 0) out[v] = acc;
}

__global__ __launch_bounds__(256) void k_out_dh(const __bf16 *__restrict__ dyb, const __bf16 *__restrict__ w,
                                                int64_t rows, float *dh) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows * 512; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i >> 9;
    const int k = (int)(i & 511);
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < 6; ++j) acc = fmaf((float)dyb[r * 6 + j], (float)w[k * 6 + j], acc);
    dh[i] = acc;
  }
}

// Gaussian negative log-likelihood head: y [n x 6] -> loss (written to
// *loss), dY = dL/dy (FP32 for the bias, BF16 for the products).  The
// log-variance is floored at kLogVarMin (variance 1e-3); below the floor it
// gets no gradient.  Blocks of 1024 threads.  Block 0 forms the loss: thread
// i takes rows i, i + 1024, ... and the terms are added in a fixed order
// (per thread, then a butterfly within each wave, then the waves in order),
// so the loss is the same on every run; it loads kHeadRows rows at a time
// before adding any.  Blocks 1, 2, ... write dY, a row per thread, so that
// the strided loads and stores of a large batch are spread over as many CUs
// (one block's memory pipeline took 17 us for 4096 rows).  Both compute the
// terms by the same expressions (head_terms).
constexpr int kHeadRows = 4;

__device__ __forceinline__ void head_terms(float mu, float s_raw, float tv, float nf, double *lt, float *gm,
                                           float *gs) {
  const float s = fmaxf(s_raw, kLogVarMin);
  const float e = tv - mu;
  const float ie = expf(-s);
  *lt = 0.5 * ((double)s + (double)e * e * ie);
  *gm = -e * ie / nf;
  *gs = s_raw < kLogVarMin ? 0.0f : 0.5f * (1.0f - e * e * ie) / nf;
}

__global__ __launch_bounds__(1024) void k_head(const float *__restrict__ y, const float *__restrict__ t, int64_t n,
                                               float *__restrict__ dy, __bf16 *__restrict__ dyb,
                                               double *__restrict__ loss) {
  __shared__ double sh[16];
  const int64_t stride = blockDim.x;
  if (blockIdx.x > 0) {
    const int64_t i = (int64_t)(blockIdx.x - 1) * stride + threadIdx.x;
    if (i >= n) return;
    float yv[6], tv[3];
#pragma unroll
    for (int c = 0; c < 6; ++c) yv[c] = y[i * 6 + c];
#pragma unroll
    for (int d = 0; d < 3; ++d) tv[d] = t[i * 3 + d];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double lt;
      float gm, gs;
      head_terms(yv[d], yv[3 + d], tv[d], (float)n, &lt, &gm, &gs);
      dy[i * 6 + d] = gm;
      dy[i * 6 + 3 + d] = gs;
      dyb[i * 6 + d] = to_bf16(gm);
      dyb[i * 6 + 3 + d] = to_bf16(gs);
    }
    return;
  }
  double acc = 0.0;
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += kHeadRows * stride) {
    float yv[kHeadRows][6], tv[kHeadRows][3];
#pragma unroll
    for (int u = 0; u < kHeadRows; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n) {
#pragma unroll
        for (int c = 0; c < 6; ++c) yv[u][c] = y[i * 6 + c];
#pragma unroll
        for (int d = 0; d < 3; ++d) tv[u][d] = t[i * 3 + d];
      }
    }
#pragma unroll
    for (int u = 0; u < kHeadRows; ++u) {
      if (i0 + u * stride >= n) break;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double lt;
        float gm, gs;
        head_terms(yv[u][d], yv[u][3 + d], tv[u][d], (float)n, &lt, &gm, &gs);
        acc += lt;
      }
    }
  }
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double total = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) total += sh[w];
    *loss = total / (double)n;
  }
}

// The hidden layers' backward epilogue and the first step of their bias
// gradients in one pass: dZ = dH gelu'(Z) (BF16 copy for the products) over
// a block of 64 columns and a slice of rows, with the slice's column sums
// (four row groups, thread g taking rows g, g + 4, ..., the groups added in
// order) written to part[y][col]; k_colsum_join then adds the slices in
// order, so the sums do not depend on scheduling.
__global__ __launch_bounds__(256) void k_gelu_back_colsum(const float *dh, const float *z, int64_t rows, int cols,
                                                          int64_t per, __bf16 *dzb, float *part) {
  __shared__ float sh[4][64];
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int rg = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.y * per, r1 = min(rows, r0 + per);
  float acc = 0.0f;
  if (col < cols)
    for (int64_t r = r0 + rg; r < r1; r += 4) {
      const int64_t i = r * cols + col;
      const float v = dh[i] * gelu_grad(z[i]);
      dzb[i] = to_bf16(v);
      acc += v;
    }
  sh[rg][threadIdx.x & 63] = acc;
  __syncthreads();
  if (rg == 0 && col < cols)
    part[(int64_t)blockIdx.y * cols + col] = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_adam(float *w, __bf16 *wb, const float *g, float *m, float *v, int64_t n,
                                              float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = to_bf16(wi);
  }
}

__global__ __launch_bounds__(256) void k_to_bf16(const float *x, __bf16 *y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = to_bf16(x[i]);
}

// Network input: facet cells inside -32..31 on both axes, Vbar / (S g), g the
// observation's mean spectral factor, clipped to +-kFeatureClip.
__global__ __launch_bounds__(256) void k_features(FeatureArgs a) {
  const int s = a.s0 + (int)blockIdx.x;
  __bf16 *x = a.x + (int64_t)blockIdx.x * 8192;
  for (int i = threadIdx.x; i < 8192; i += blockDim.x) x[i] = to_bf16(0.0f);
  __syncthreads();
  const double inv = 1.0 / (a.src[s].flux * a.spec_norm);
  for (int64_t c = a.offsets[s] + threadIdx.x; c < a.offsets[s + 1]; c += blockDim.x) {
    const int ix = a.ix[c], iy = a.iy[c];
    if (ix < -32 || ix > 31 || iy < -32 || iy > 31) continue;
    const int pos = (iy + 32) * 64 + (ix + 32);
    x[pos] = to_bf16((float)fmin(fmax(a.vre[c] * inv, -kFeatureClip), kFeatureClip));
    x[4096 + pos] = to_bf16((float)fmin(fmax(a.vim[c] * inv, -kFeatureClip), kFeatureClip));
  }
}

// Window boxes from the predictions (decided in FP64 from the FP32 outputs);
// a box covering more than full_frac of the grid becomes the whole grid.
__global__ __launch_bounds__(256) void k_windows(const float *y, int64_t n, double nsigma, int n_e, double step,
                                                 int min_half, double full_frac, int32_t *win) {
  const int c = (n_e - 1) / 2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int box[4];
    for (int d = 0; d < 2; ++d) {
      const double mu = (double)y[i * 6 + d];
      const double sd = exp(0.5 * fmax((double)y[i * 6 + 3 + d], (double)kLogVarMin));
      int lo = (int)floor((mu - nsigma * sd) / step + c);
      int hi = (int)ceil((mu + nsigma * sd) / step + c);
      const int mid = (int)rint(mu / step + c);
      lo = min(lo, mid - min_half);
      hi = max(hi, mid + min_half);
      box[2 * d] = min(max(lo, 0), n_e - 1);
      box[2 * d + 1] = min(max(hi, 0), n_e - 1);
    }
    if ((double)(box[1] - box[0] + 1) * (double)(box[3] - box[2] + 1) > full_frac * (double)n_e * (double)n_e) {
      box[0] = box[2] = 0;
      box[1] = box[3] = n_e - 1;
    }
    for (int q = 0; q < 4; ++q) win[i * 4 + q] = box[q];
  }
}

// SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the output mix of state seed + k * golden gamma,
// used here as a counter-based generator (value k of stream `seed`).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Standard normal number j of stream `seed` by the Box-Muller transform of
// the uniforms u1 = (h(2j+1) >> 11 + 1) 2^-53 in (0, 1] and
// u2 = (h(2j+2) >> 11) 2^-53 in [0, 1), h the counter generator above:
// sqrt(-2 ln u1) cos(2 pi u2), in FP64.
__device__ __forceinline__ double std_normal(uint64_t seed, uint64_t j) {
  const double u1 = ((double)(splitmix64(seed, 2 * j + 1) >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(splitmix64(seed, 2 * j + 2) >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

// Training targets drawn around the method's own estimates: row i gets
// (e1_i + kappa s1_i z_{2i}, e2_i + kappa s2_i z_{2i+1}, ln alpha_i) with z
// the normal numbers of stream `seed`; a row whose estimate or spread is not
// finite gets (0, 0, ln alpha_i).
__global__ __launch_bounds__(256) void k_posterior_targets(const double *e1, const double *e2, const double *s1,
                                                           const double *s2, const float *ln_alpha, int64_t n,
                                                           double kappa, uint64_t seed, float *t) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const bool ok = isfinite(e1[i]) && isfinite(e2[i]) && isfinite(s1[i]) && isfinite(s2[i]);
    t[i * 3 + 0] = ok ? (float)(e1[i] + kappa * s1[i] * std_normal(seed, 2 * (uint64_t)i)) : 0.0f;
    t[i * 3 + 1] = ok ? (float)(e2[i] + kappa * s2[i] * std_normal(seed, 2 * (uint64_t)i + 1)) : 0.0f;
    t[i * 3 + 2] = ln_alpha[i];
  }
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 16384 ? (b > 0 ? b : 1) : 16384);
}

}  // namespace

hipError_t launch_gemm(const GemmArgs &g, int split_k, hipStream_t st) {
  if (split_k > 1 && (!g.ws || (int64_t)split_k * g.M * g.N > g.ws_floats)) return hipErrorInvalidValue;
  const dim3 grid((g.N + kBN - 1) / kBN, (g.M + kBM - 1) / kBM, split_k > 1 ? split_k : 1);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, g);
  if (split_k > 1)
    hipLaunchKernelGGL(k_reduce_split, dim3(grid_for((int64_t)g.M * g.N)), dim3(256), 0, st, g.ws, split_k, g.M, g.N,
                       g.c, g.ldc);
  return hipGetLastError();
}

hipError_t launch_bias_act(const float *c, const float *b, int64_t rows, int cols, float *z, __bf16 *h, int act,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_bias_act, dim3(grid_for(rows * cols)), dim3(256), 0, st, c, b, rows, cols, z, h, act);
  return hipGetLastError();
}

hipError_t launch_out_forward(const __bf16 *h, const __bf16 *w, const float *b, int64_t rows, float *y,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_out_forward, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, h, w, b, rows, y);
  return hipGetLastError();
}

hipError_t launch_out_backward(const __bf16 *h, const __bf16 *dyb, const float *dy, int64_t rows, const __bf16 *w,
                               float *gw, float *dh, float *ws, int64_t ws_floats, hipStream_t st) {
  // slices of 32 rows, longer if their partial sums would not fit the workspace
  const int64_t max_slices = ws_floats / kOutWB;
  if (max_slices < 1) return hipErrorInvalidValue;
  const int64_t per = std::max<int64_t>(32, (rows + max_slices - 1) / max_slices);
  const int slices = (int)((rows + per - 1) / per);
  hipLaunchKernelGGL(k_out_grad_part, dim3((kOutWB + 255) / 256, slices), dim3(256), 0, st, h, dyb, dy, rows, per, ws);
  hipLaunchKernelGGL(k_out_grad_join, dim3((kOutWB + 3) / 4), dim3(256), 0, st, ws, slices, gw);
  hipLaunchKernelGGL(k_out_dh, dim3(grid_for(rows * 512)), dim3(256), 0, st, dyb, w, rows, dh);
  return hipGetLastError();
}

hipError_t launch_head(const float *y, const float *t, int64_t n, float *dy, __bf16 *dyb, double *loss,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_head, dim3(1 + (int)((n + 1023) / 1024)), dim3(1024), 0, st, y, t, n, dy, dyb, loss);
  return hipGetLastError();
}

// Row slices of the two-step column sums: at least 32 rows, at most 256
// slices (one block per slice and 64 columns), within the workspace.
void colsum_slices(int64_t rows, int cols, int64_t ws_floats, int64_t *per, int *nsl) {
  const int64_t slices = std::max<int64_t>(1, std::min<int64_t>({256, (rows + 31) / 32, ws_floats / std::max(1, cols)}));
  *per = (rows + slices - 1) / slices;
  *nsl = (int)((rows + *per - 1) / *per);
}

hipError_t launch_gelu_back_colsum(const float *dh, const float *z, int64_t rows, int cols, __bf16 *dzb, float *db,
                                   float *ws, int64_t ws_floats, hipStream_t st) {
  int64_t per;
  int nsl;
  colsum_slices(rows, cols, ws_floats, &per, &nsl);
  hipLaunchKernelGGL(k_gelu_back_colsum, dim3((cols + 63) / 64, nsl), dim3(256), 0, st, dh, z, rows, cols, per, dzb,
                     ws);
  hipLaunchKernelGGL(k_colsum_join, dim3((cols + 3) / 4), dim3(256), 0, st, ws, nsl, cols, db);
  return hipGetLastError();
}

hipError_t launch_gemm_nt(const GemmNTArgs &g, int split_k, hipStream_t st) {
  if (g.K % 8 || g.lda % 8 || g.ldb % 8) return hipErrorInvalidValue;
  if (split_k > 1 && (!g.ws || (int64_t)split_k * g.M * g.N > g.ws_floats)) return hipErrorInvalidValue;
  const dim3 grid((g.N + kTN - 1) / kTN, (g.M + kTM - 1) / kTM, split_k > 1 ? split_k : 1);
  hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, g);
  if (split_k > 1)
    hipLaunchKernelGGL(k_reduce_split, dim3(grid_for((int64_t)g.M * g.N)), dim3(256), 0, st, g.ws, split_k, g.M, g.N,
                       g.c, g.ldc);
  return hipGetLastError();
}

hipError_t launch_transpose_bf16(const TransposeJob *jobs, int n_jobs, hipStream_t st) {
  if (n_jobs < 1 || n_jobs > kMaxTransposeJobs) return hipErrorInvalidValue;
  TransposeBatch tb{};
  tb.n = n_jobs;
  tb.first_tile[0] = 0;
  for (int j = 0; j < n_jobs; ++j) {
    if (jobs[j].rows < 1 || jobs[j].cols < 1) return hipErrorInvalidValue;
    tb.job[j] = jobs[j];
    tb.tiles_x[j] = (jobs[j].cols + 63) / 64;
    tb.first_tile[j + 1] = tb.first_tile[j] + tb.tiles_x[j] * ((jobs[j].rows + 63) / 64);
  }
  for (int j = n_jobs; j < kMaxTransposeJobs; ++j) tb.first_tile[j + 1] = tb.first_tile[n_jobs];
  hipLaunchKernelGGL(k_transpose_bf16, dim3((unsigned)tb.first_tile[n_jobs]), dim3(256), 0, st, tb);
  return hipGetLastError();
}

hipError_t launch_adam(float *w, __bf16 *wb, const float *g, float *m, float *v, int64_t n, float lr, int64_t step,
                       hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)step)), c2 = (float)(1.0 - std::pow(0.999, (double)step));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, st, w, wb, g, m, v, n, lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float *x, __bf16 *y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n)), dim3(256), 0, st, x, y, n);
  return hipGetLastError();
}

hipError_t launch_features(const FeatureArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_features, dim3(a.n_src), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_posterior_targets(const double *e1, const double *e2, const double *s1, const double *s2,
                                   const float *ln_alpha, int64_t n, double kappa, uint64_t seed, float *t,
                                   hipStream_t st) {
  hipLaunchKernelGGL(k_posterior_targets, dim3(grid_for(n)), dim3(256), 0, st, e1, e2, s1, s2, ln_alpha, n, kappa,
                     seed, t);
  return hipGetLastError();
}

hipError_t launch_windows(const float *y, int64_t n, double nsigma, int n_e, double step, int min_half,
                          double full_frac, int32_t *win, hipStream_t st) {
  hipLaunchKernelGGL(k_windows, dim3(grid_for(n)), dim3(256), 0, st, y, n, nsigma, n_e, step, min_half, full_frac,
                     win);
  return hipGetLastError();
}

}  // namespace rlf
