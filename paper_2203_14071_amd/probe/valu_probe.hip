// VALU issue-rate probe for gfx950 (measurement of the roofline ceilings the
// benchmark prices the kernels against; not part of the library).
//
// Each kernel runs `iters` iterations of a fixed instruction group on eight
// independent dependency chains per lane (enough independent work to hide
// latency at full occupancy), so the measured time is issue-bound.  The
// groups are single instruction types (FP64 / FP32 FMA, v_rsq_f64, v_rsq_f32,
// v_sin_f32, v_exp_f32) and mixes of one transcendental with k FMAs, which
// show whether transcendentals issue alongside other VALU work.
#include <hip/hip_runtime.h>
#include <stdint.h>

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

}  // extern "C"
