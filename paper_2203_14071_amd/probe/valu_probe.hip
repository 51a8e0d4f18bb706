// VALU issue-rate probe for gfx950 (measurement of the roofline ceilings the
// benchmark prices the kernels against; not part of the library).
//
// Each kernel runs `iters` iterations of a fixed instruction group on eight
// independent dependency chains per lane (enough independent work to hide
// latency at full occupancy), so the measured time is issue-bound.  The
// groups are single instruction types (FP64 / FP32 FMA, v_rsq_f64, v_rsq_f32,
// v_sin_f32, v_exp_f32) and mixes of one transcendental with k FMAs, which
// show whether transcendentals issue alongside other VALU work.
//
// A second set ("kernel-mix" probes) runs the library kernels' own inner
// loops, the shared device functions of the sky model (sum_f64, sum_mixed)
// and of the likelihood (cell_sums_f64, cell_sums_f32), on synthetic
// sources and cells in small cache-resident arrays read as the kernels
// read them (wave-uniform scalar loads).  Their time is that of the
// kernels' own instruction streams without the kernels' visibility and
// output traffic: the ceiling each kernel is measured against.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "rlf_cellsums.h"
#include "rlf_internal.h"
#include "rlf_sky.h"

namespace {

enum Op : int {
  kFma64 = 0, kFma32 = 1, kRsq64 = 2, kRsq32 = 3, kSin32 = 4, kExp32 = 5,
  kRsq32Fma32x1 = 6, kRsq32Fma32x2 = 7, kRsq32Fma32x4 = 8, kSin32Fma32x2 = 9,
  kRsq64Fma64x2 = 10, kRsq64Fma64x4 = 11, kCvt64to32 = 12, kOps = 13
};

template <int OP>
__global__ __launch_bounds__(256) void k_probe(int64_t iters, float *sink32, double *sink64, uint64_t *clk) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  // shader-clock and fixed 100 MHz counters around the loop (first block)
  uint64_t c0 = 0, r0 = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c0 = __builtin_amdgcn_s_memtime();
    r0 = __builtin_amdgcn_s_memrealtime();
  }
  double a[8];
  float f[8], g[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = 1.0 + 1e-3 * (t + i);
    f[i] = 1.0f + 1e-3f * (float)(t + i);
    g[i] = 0.25f + 1e-4f * (float)(t + i);
  }
  const double b64 = 0.999999, c64 = 1e-7;
  const float b32 = 0.99999f, c32 = 1e-6f;
#pragma unroll 1
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if constexpr (OP == kFma64) a[i] = fma(a[i], b64, c64);
      if constexpr (OP == kFma32) f[i] = fmaf(f[i], b32, c32);
      if constexpr (OP == kRsq64) a[i] = __builtin_amdgcn_rsq(a[i]);
      if constexpr (OP == kRsq32) f[i] = __builtin_amdgcn_rsqf(f[i]);
      if constexpr (OP == kSin32) g[i] = __builtin_amdgcn_sinf(g[i]);
      if constexpr (OP == kExp32) g[i] = __builtin_amdgcn_exp2f(g[i]) - 1.0f;
      if constexpr (OP == kCvt64to32) {
        f[i] = (float)a[i];
        a[i] = (double)f[i] + c64;
      }
      if constexpr (OP == kRsq32Fma32x1 || OP == kRsq32Fma32x2 || OP == kRsq32Fma32x4) {
        g[i] = __builtin_amdgcn_rsqf(g[i] + 1.0f);
        f[i] = fmaf(f[i], b32, c32);
        if constexpr (OP != kRsq32Fma32x1) f[i] = fmaf(f[i], b32, c32);
        if constexpr (OP == kRsq32Fma32x4) {
          f[i] = fmaf(f[i], b32, c32);
          f[i] = fmaf(f[i], b32, c32);
        }
      }
      if constexpr (OP == kSin32Fma32x2) {
        g[i] = __builtin_amdgcn_sinf(g[i]);
        f[i] = fmaf(f[i], b32, c32);
        f[i] = fmaf(f[i], b32, c32);
      }
      if constexpr (OP == kRsq64Fma64x2 || OP == kRsq64Fma64x4) {
        const double r = __builtin_amdgcn_rsq((double)g[i] + 1.0);
        g[i] = (float)r;
        a[i] = fma(a[i], b64, c64);
        a[i] = fma(a[i], b64, c64);
        if constexpr (OP == kRsq64Fma64x4) {
          a[i] = fma(a[i], b64, c64);
          a[i] = fma(a[i], b64, c64);
        }
      }
    }
  }
  float s32 = 0.0f;
  double s64 = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    s32 += f[i] + g[i];
    s64 += a[i];
  }
  sink32[t] = s32;
  sink64[t] = s64;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    clk[0] = __builtin_amdgcn_s_memtime() - c0;
    clk[1] = __builtin_amdgcn_s_memrealtime() - r0;
  }
}

template <int OP>
hipError_t launch(int blocks, int64_t iters, float *s32, double *s64, uint64_t *clk, hipStream_t st) {
  hipLaunchKernelGGL(k_probe<OP>, dim3(blocks), dim3(256), 0, st, iters, s32, s64, clk);
  return hipGetLastError();
}

hipError_t launch_op(int op, int blocks, int64_t iters, float *s32, double *s64, uint64_t *clk, hipStream_t st) {
  switch (op) {
    case kFma64: return launch<kFma64>(blocks, iters, s32, s64, clk, st);
    case kFma32: return launch<kFma32>(blocks, iters, s32, s64, clk, st);
    case kRsq64: return launch<kRsq64>(blocks, iters, s32, s64, clk, st);
    case kRsq32: return launch<kRsq32>(blocks, iters, s32, s64, clk, st);
    case kSin32: return launch<kSin32>(blocks, iters, s32, s64, clk, st);
    case kExp32: return launch<kExp32>(blocks, iters, s32, s64, clk, st);
    case kRsq32Fma32x1: return launch<kRsq32Fma32x1>(blocks, iters, s32, s64, clk, st);
    case kRsq32Fma32x2: return launch<kRsq32Fma32x2>(blocks, iters, s32, s64, clk, st);
    case kRsq32Fma32x4: return launch<kRsq32Fma32x4>(blocks, iters, s32, s64, clk, st);
    case kSin32Fma32x2: return launch<kSin32Fma32x2>(blocks, iters, s32, s64, clk, st);
    case kRsq64Fma64x2: return launch<kRsq64Fma64x2>(blocks, iters, s32, s64, clk, st);
    case kRsq64Fma64x4: return launch<kRsq64Fma64x4>(blocks, iters, s32, s64, clk, st);
    case kCvt64to32: return launch<kCvt64to32>(blocks, iters, s32, s64, clk, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

namespace {

enum MixOp : int { kMixSkyF64 = 0, kMixSkyMixed = 1, kMixFitF64 = 2, kMixFitMixed = 3, kMixOps = 4 };
constexpr int kMixKnots = 20;        // scale-length knots of the likelihood
constexpr int kMixKnotsPass = 10;    // knots per pass of the mixed likelihood kernel

struct MixArgs {
  int64_t iters;
  int n_items;                       // sources (sky model) or cells (likelihood) per iteration
  const rlf::SrcModel *src;
  const rlf::SrcMixed *src32;
  const double4 *c64;
  const float4 *c32;
  const double *sk;                  // kMixKnots knot scales, twice
  double *sink;
  uint64_t *clk;
  int64_t spin_ticks;                // the clock wave's window, fixed-clock ticks (10 ns)
};

// One lane's work: a visibility (ops 0-1) or an ellipticity grid point
// (ops 2-3) taken through `iters` passes of the kernel's own inner loop.
// The FP64 sky-model mix as k_model runs it: a 2048-entry table in blocks
// of 512 threads; the other mixes in blocks of 256.
constexpr int kMixSkyTable = 2048;
template <int OP>
constexpr int mix_threads() { return OP == kMixSkyF64 ? 512 : 256; }

template <int OP>
__device__ __forceinline__ double mix_work(const MixArgs &a, int t, const double2 *tab) {
  double out = 0.0;
  if (OP == kMixSkyF64 || OP == kMixSkyMixed) {
    const double u = 1000.0 + 37.0 * (t & 4095), v = -2000.0 + 53.0 * (t >> 12), w = 11.0 * (t & 63);
    double ar = 0.0, ai = 0.0;
#pragma unroll 1
    for (int64_t it = 0; it < a.iters; ++it) {
      const double ui = u + (double)it;        // a new visibility each pass: nothing is loop-invariant
      if (OP == kMixSkyF64) {
        const double2 z = rlf::sum_f64<kMixSkyTable>(ui, v, w, a.src, 0, a.n_items, tab);
        ar += z.x;
        ai += z.y;
      } else {
        const float2 z = rlf::sum_mixed(ui, v, w, a.src32, 0, a.n_items);
        ar += z.x;
        ai += z.y;
      }
    }
    out = ar + ai;
  } else {
    const double e1 = 0.02 * ((t % 81) - 40) * 0.9, e2 = 0.02 * (((t / 81) % 81) - 40) * 0.9;
    const double det = 1.0 - e1 * e1 - e2 * e2;
#pragma unroll 1
    for (int64_t it = 0; it < a.iters; ++it) {
      const double de = 1e-12 * (double)it;    // a new point each pass
      // the knot scales are loaded per pass, wave-uniform, as the kernel
      // loads them (the alternating copy keeps them from being hoisted out
      // of the loop)
      const double *skp = a.sk + (it & 1) * kMixKnots;
      if (OP == kMixFitF64) {
        double D[kMixKnots], M[kMixKnots], sk[kMixKnots];
#pragma unroll
        for (int k = 0; k < kMixKnots; ++k) {
          D[k] = M[k] = 0.0;
          sk[k] = skp[k];
        }
        const double id = 1.0 / det;
        rlf::cell_sums_f64<kMixKnots>(a.c64, 0, a.n_items, (1.0 + e1 + de) * id, e2 * id, (1.0 - e1) * id, sk,
                                      kMixKnots, D, M);
#pragma unroll
        for (int k = 0; k < kMixKnots; ++k) out += D[k] + M[k];
      } else {
        const double g = 1.0 / (det * det);
#pragma unroll 1
        for (int k0 = 0; k0 < kMixKnots; k0 += kMixKnotsPass) {
          double D[kMixKnotsPass], M[kMixKnotsPass];
          float sk[kMixKnotsPass];
#pragma unroll
          for (int k = 0; k < kMixKnotsPass; ++k) {
            D[k] = M[k] = 0.0;
            sk[k] = (float)(skp[k0 + k] * g);
          }
          rlf::cell_sums_f32<kMixKnotsPass>(a.c32, 0, a.n_items, (float)(1.0 + e1 + de), (float)e2,
                                            (float)(1.0 - e1), sk, kMixKnotsPass, D, M);
#pragma unroll
          for (int k = 0; k < kMixKnotsPass; ++k) out += D[k] + M[k];
        }
      }
    }
  }
  return out;
}

// Shader-clock and fixed 100 MHz counters (inline asm that touches no
// memory; the wait for the result is in the same asm block).
__device__ __forceinline__ uint64_t shader_clock() {
  uint64_t c;
  asm volatile("s_memtime %0\n\ts_waitcnt lgkmcnt(0)" : "=s"(c));
  return c;
}
__device__ __forceinline__ uint64_t fixed_clock() {
  uint64_t c;
  asm volatile("s_memrealtime %0\n\ts_waitcnt lgkmcnt(0)" : "=s"(c));
  return c;
}

// Wave 0 of block 0 is the clock: it reads both counters, sleeps until
// spin_ticks of the fixed clock have passed (the caller sets that below
// the run's duration, so the window lies inside the loaded run) and reads
// them again; it does none of the work.  Every other wave runs the work.
// (A clock read on the working waves' path would make the compiler take
// the loop's loads as possibly clobbered and issue vector loads in place of
// the kernels' scalar loads.)
template <int OP>
__global__ __launch_bounds__(mix_threads<OP>()) void k_mix(MixArgs a) {
  __shared__ double2 tab[OP == kMixSkyF64 ? kMixSkyTable : 1];
  if (OP == kMixSkyF64) {
    rlf::cis_table_init<kMixSkyTable>(tab);
    __syncthreads();
  }
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    if (threadIdx.x == 0) {
      const uint64_t c0 = shader_clock(), r0 = fixed_clock();
      uint64_t r1 = r0;
      while (r1 - r0 < (uint64_t)a.spin_ticks) {
        __builtin_amdgcn_s_sleep(64);
        r1 = fixed_clock();
      }
      a.clk[0] = shader_clock() - c0;
      a.clk[1] = r1 - r0;
    }
    return;
  }
  a.sink[t] = mix_work<OP>(a, t, tab);
}

// `blocks` counts blocks of 256 threads; the FP64 sky-model mix runs the same
// threads in blocks of 512 (blocks must then be even)
hipError_t launch_mix(int op, int blocks, const MixArgs &a, hipStream_t st) {
  switch (op) {
    case kMixSkyF64:
      if (blocks % 2) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_mix<kMixSkyF64>, dim3(blocks / 2), dim3(mix_threads<kMixSkyF64>()), 0, st, a);
      break;
    case kMixSkyMixed: hipLaunchKernelGGL(k_mix<kMixSkyMixed>, dim3(blocks), dim3(256), 0, st, a); break;
    case kMixFitF64: hipLaunchKernelGGL(k_mix<kMixFitF64>, dim3(blocks), dim3(256), 0, st, a); break;
    case kMixFitMixed: hipLaunchKernelGGL(k_mix<kMixFitMixed>, dim3(blocks), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

// Accuracy of v_rsq_f64: for n arguments x = 2^(40 i / n), i < n (spread
// log-uniformly over [1, 2^40), the range of the profile arguments 1 + s q),
// the relative error of the instruction against 1 / sqrt(x) from the
// correctly rounded FP64 square root and division; each block writes its
// largest error.
__global__ __launch_bounds__(256) void k_rsq64_error(int64_t n, double *block_max) {
  __shared__ double sh[256];
  double worst = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double x = exp2(40.0 * (double)i / (double)n);
    const double y = __builtin_amdgcn_rsq(x);
    const double ref = 1.0 / __dsqrt_rn(x);
    worst = fmax(worst, fabs(y - ref) / ref);
  }
  sh[threadIdx.x] = worst;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) block_max[blockIdx.x] = sh[0];
}

// exp(2 pi i phi) by the library's table method (cis2pi_f64) at given
// phases, for each table size the kernels use; a grid-stride loop.
template <int T>
__global__ __launch_bounds__(256) void k_cis_eval(const double *phi, int64_t n, double2 *out) {
  __shared__ double2 tab[T];
  rlf::cis_table_init<T>(tab);
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = rlf::cis2pi_f64<T>(phi[i], tab);
}

// (2/3) x^(-3/2) by the kernels' corrected rsqrt cube (pow_m32_f64) at given
// arguments x >= 1; a grid-stride loop.
__global__ __launch_bounds__(256) void k_pow_m32_eval(const double *x, int64_t n, double *out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = rlf::pow_m32_f64(x[i]);
}

extern "C" {

// Number of probe kernels.
int valu_probe_count(void) { return kOps; }

// Run probe `op` over `blocks` blocks of 256 threads for `iters` iterations,
// `reps` times on a fresh stream; *best_ms receives the fastest run and
// *clock_hz the shader clock over the first block's loop in that run (the
// shader-cycle counter against the fixed 100 MHz one).  Returns 0, or the
// HIP error code.  The device buffers are allocated and freed here.
int valu_probe_run(int op, int blocks, int64_t iters, int reps, double *best_ms, double *clock_hz) {
  if (op < 0 || op >= kOps || blocks < 1 || iters < 1 || reps < 1 || !best_ms || !clock_hz)
    return (int)hipErrorInvalidValue;
  float *s32 = nullptr;
  double *s64 = nullptr;
  uint64_t *clk = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&s32, sizeof(float) * 256 * (size_t)blocks);
  if (e == hipSuccess) e = hipMalloc(&s64, sizeof(double) * 256 * (size_t)blocks);
  if (e == hipSuccess) e = hipMalloc(&clk, sizeof(uint64_t) * 2);
  if (e == hipSuccess) e = hipStreamCreate(&st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  double best = 1e300, hz = 0.0;
  if (e == hipSuccess) e = launch_op(op, blocks, iters, s32, s64, clk, st);    // warm-up
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch_op(op, blocks, iters, s32, s64, clk, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    uint64_t c[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpy(c, clk, sizeof c, hipMemcpyDeviceToHost);
    if (e == hipSuccess && ms < best) {
      best = ms;
      hz = c[1] ? (double)c[0] / ((double)c[1] * 1e-8) : 0.0;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  if (s32) (void)hipFree(s32);
  if (s64) (void)hipFree(s64);
  if (clk) (void)hipFree(clk);
  *best_ms = best;
  *clock_hz = hz;
  return (int)e;
}

// Number of kernel-mix probes (0: sky-model term FP64, 1: mixed; 2:
// likelihood cell sums FP64, 20 knots in one pass; 3: mixed, two passes of
// 10 knots over 32-cell FP32 blocks).
int mix_probe_count(void) { return kMixOps; }

// Run kernel-mix probe `op` over `blocks` blocks of 256 threads, `iters`
// passes over `n_items` synthetic sources (ops 0-1) or cells (ops 2-3),
// `reps` times; *best_ms, *clock_hz as for valu_probe_run, *units the work
// of one run in the kernels' units: (visibility, source) pairs, or
// (cell, e point, knot) triples.  Returns 0, or the HIP error code.  The
// device buffers are allocated and freed here.
int mix_probe_run(int op, int blocks, int64_t iters, int n_items, int reps, double *best_ms, double *clock_hz,
                  double *units) {
  if (op < 0 || op >= kMixOps || blocks < 1 || iters < 1 || n_items < 1 || n_items > (1 << 16) || reps < 1 ||
      !best_ms || !clock_hz || !units)
    return (int)hipErrorInvalidValue;
  std::vector<rlf::SrcModel> hs(n_items);
  std::vector<rlf::SrcMixed> hm(n_items);
  std::vector<double4> h64(n_items);
  std::vector<float4> h32(n_items);
  for (int i = 0; i < n_items; ++i) {
    // sources over a 1-degree field, scale lengths ~1 arcsec; cells on a
    // 17 x 17 patch of a 5,400-wavelength facet lattice
    const double l = 8.7e-3 * ((i * 37) % 101 - 50) / 50.0, m = 8.7e-3 * ((i * 53) % 97 - 48) / 48.0;
    const double q = 4e-10 * (1.0 + (i % 7) * 0.1);
    hs[i] = rlf::SrcModel{l, m, -0.5 * (l * l + m * m), 1e-4, q, 0.2 * q, 1.1 * q, 1.8e-4};
    hm[i] = rlf::SrcMixed{l, m, -0.5 * (l * l + m * m), 1e-4f, (float)q, (float)(0.2 * q), (float)(1.1 * q), 1.8e-4};
    // cells as the library packs them: (W^{-1/6} uc, W^{-1/6} vc, W^{-1/3}, sqrt(W) Re Vbar)
    const double uc = 5400.0 * (i % 17 - 8), vc = 5400.0 * ((i / 17) % 17 - 8);
    const double W = 1.0 + 1e-3 * i, cw = 1.0 / std::cbrt(W), rw = std::sqrt(cw), b = std::sqrt(W) * 1e-3 * (i % 13);
    h64[i] = make_double4(uc * rw, vc * rw, cw, b);
    h32[i] = make_float4((float)(uc * rw), (float)(vc * rw), (float)cw, (float)b);
  }
  double hsk[2 * kMixKnots];
  for (int k = 0; k < kMixKnots; ++k) {
    const double al = (0.3 + 3.2 * k * k / 361.0) * 4.8481368110953599e-6;
    hsk[k] = hsk[kMixKnots + k] = 4.0 * 9.8696044010893586 * al * al;
  }
  MixArgs a{};
  a.iters = iters;
  a.n_items = n_items;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rlf::SrcModel *ds = nullptr;
  rlf::SrcMixed *dm = nullptr;
  double4 *d64 = nullptr;
  float4 *d32 = nullptr;
  double *dsk = nullptr, *sink = nullptr;
  uint64_t *clk = nullptr;
  hipError_t e = hipMalloc(&ds, sizeof(rlf::SrcModel) * n_items);
  if (e == hipSuccess) e = hipMalloc(&dm, sizeof(rlf::SrcMixed) * n_items);
  if (e == hipSuccess) e = hipMalloc(&d64, sizeof(double4) * n_items);
  if (e == hipSuccess) e = hipMalloc(&d32, sizeof(float4) * n_items);
  if (e == hipSuccess) e = hipMalloc(&dsk, sizeof hsk);
  if (e == hipSuccess) e = hipMalloc(&sink, sizeof(double) * 256 * (size_t)blocks);
  if (e == hipSuccess) e = hipMalloc(&clk, sizeof(uint64_t) * 2);
  if (e == hipSuccess) e = hipMemcpy(ds, hs.data(), sizeof(rlf::SrcModel) * n_items, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dm, hm.data(), sizeof(rlf::SrcMixed) * n_items, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d64, h64.data(), sizeof(double4) * n_items, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d32, h32.data(), sizeof(float4) * n_items, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dsk, hsk, sizeof hsk, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreate(&st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  a.src = ds;
  a.src32 = dm;
  a.c64 = d64;
  a.c32 = d32;
  a.sk = dsk;
  a.sink = sink;
  a.clk = clk;
  double best = 1e300, hz = 0.0;
  a.spin_ticks = 0;
  if (e == hipSuccess) e = launch_mix(op, blocks, a, st);      // first launch
  // a second warm-up, timed: the clock window of the measured runs is 70 % of it
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = launch_mix(op, blocks, a, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float warm_ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&warm_ms, e0, e1);
  a.spin_ticks = (int64_t)(0.7 * warm_ms * 1e5);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch_mix(op, blocks, a, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    uint64_t c[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpy(c, clk, sizeof c, hipMemcpyDeviceToHost);
    if (e == hipSuccess && ms < best) {
      best = ms;
      hz = c[1] ? (double)c[0] / ((double)c[1] * 1e-8) : 0.0;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  for (void *ptr : {(void *)ds, (void *)dm, (void *)d64, (void *)d32, (void *)dsk, (void *)sink, (void *)clk})
    if (ptr) (void)hipFree(ptr);
  *best_ms = best;
  *clock_hz = hz;
  const double threads = 256.0 * blocks - 64.0;       // the clock wave does no work
  *units = threads * (double)iters * n_items * (op >= kMixFitF64 ? kMixKnots : 1);
  return (int)e;
}

// Largest relative error of v_rsq_f64 over n arguments spread over [1, 2^40)
// (see k_rsq64_error) into *max_rel.  Returns 0, or the HIP error
// code.  The device buffer is allocated and freed here.
int valu_probe_rsq64_error(int64_t n, double *max_rel) {
  if (n < 1 || !max_rel) return (int)hipErrorInvalidValue;
  constexpr int kBlocks = 1024;
  double *d = nullptr;
  hipError_t e = hipMalloc(&d, sizeof(double) * kBlocks);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_rsq64_error, dim3(kBlocks), dim3(256), 0, 0, n, d);
    e = hipGetLastError();
  }
  double h[kBlocks];
  if (e == hipSuccess) e = hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost);
  if (d) (void)hipFree(d);
  double worst = 0.0;
  for (int b = 0; b < kBlocks && e == hipSuccess; ++b) worst = h[b] > worst ? h[b] : worst;
  *max_rel = worst;
  return (int)e;
}

// (cos 2 pi phi, sin 2 pi phi) by the kernels' table method with a table of
// `table` entries (1024 or 2048), for n phases in turns (host arrays:
// phi_host [n], out_host [2 n] as cos, sin pairs; |phi| < 2^40).
int valu_probe_cis(int table, const double *phi_host, int64_t n, double *out_host) {
  if ((table != 1024 && table != 2048) || n < 1 || n > (int64_t)1 << 24 || !phi_host || !out_host)
    return (int)hipErrorInvalidValue;
  double *dp = nullptr;
  double2 *dout = nullptr;
  hipError_t e = hipMalloc(&dp, sizeof(double) * n);
  if (e == hipSuccess) e = hipMalloc(&dout, sizeof(double2) * n);
  if (e == hipSuccess) e = hipMemcpy(dp, phi_host, sizeof(double) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
    if (table == 1024)
      hipLaunchKernelGGL(k_cis_eval<1024>, dim3(blocks), dim3(256), 0, 0, dp, n, dout);
    else
      hipLaunchKernelGGL(k_cis_eval<2048>, dim3(blocks), dim3(256), 0, 0, dp, n, dout);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(out_host, dout, sizeof(double2) * n, hipMemcpyDeviceToHost);
  if (dp) (void)hipFree(dp);
  if (dout) (void)hipFree(dout);
  return (int)e;
}

// (2/3) x^(-3/2) by the kernels' corrected rsqrt cube for n arguments
// x >= 1 (host arrays x_host [n], out_host [n]).
int valu_probe_pow_m32(const double *x_host, int64_t n, double *out_host) {
  if (n < 1 || n > (int64_t)1 << 24 || !x_host || !out_host) return (int)hipErrorInvalidValue;
  double *dx = nullptr, *dout = nullptr;
  hipError_t e = hipMalloc(&dx, sizeof(double) * n);
  if (e == hipSuccess) e = hipMalloc(&dout, sizeof(double) * n);
  if (e == hipSuccess) e = hipMemcpy(dx, x_host, sizeof(double) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_pow_m32_eval, dim3(blocks), dim3(256), 0, 0, dx, n, dout);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(out_host, dout, sizeof(double) * n, hipMemcpyDeviceToHost);
  if (dx) (void)hipFree(dx);
  if (dout) (void)hipFree(dout);
  return (int)e;
}

}  // extern "C"
