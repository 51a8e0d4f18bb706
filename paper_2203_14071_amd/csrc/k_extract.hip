// Facet extraction (Sec. 2.3): per (visibility, source) pair, phase-shift the
// residual to the source, add back the source's own model, and accumulate the
// weighted result into the source's facet cell (rint(u theta), rint(v theta)).
//
// Work decomposition.  A wave owns 64*VPT consecutive rows of one channel
// (lane L: rows [L*VPT, (L+1)*VPT)) and a tile of sources; grid.y tiles the
// sources.  Rows are baseline-major with time fastest, so a lane's rows trace
// a short arc of one baseline and usually stay in one facet cell: the lane
// accumulates its rows serially in registers and flushes only when the cell
// changes.  At the end of its rows the wave merges equal cells of adjacent
// lanes with a segmented shuffle reduction, and one lane per run of equal
// cells issues the global atomics.  Integer counts are exact; FP sums are
// atomic (order-dependent in the last bits).
#include "rlf_internal.h"

namespace rlf {

namespace {

constexpr int kVPT = 8;               // rows per lane
constexpr int kSrcTile = 32;          // sources per block (grid.y tiles the catalogue)

struct Partial {
  int key;                            // dense cell index in the source's block, -1 = none
  uint32_t n;
  double w, zr, zi;
};

__device__ __forceinline__ void flush_atomic(const DenseAcc &acc, int64_t base, const Partial &p) {
  const int64_t k = base + p.key;
  atomicAdd(acc.count + k, p.n);
  unsafeAtomicAdd(acc.wsum + k, p.w);
  unsafeAtomicAdd(acc.zre + k, p.zr);
  unsafeAtomicAdd(acc.zim + k, p.zi);
}

// Merge each run of equal keys across the wave (keys of adjacent lanes) and
// flush one partial per run.
__device__ __forceinline__ void wave_flush(const DenseAcc &acc, int64_t base, Partial p) {
  const int lane = __lane_id();
  const int prev = __shfl_up(p.key, 1);
  const bool head = (lane == 0) || (prev != p.key);
  const uint64_t heads = __ballot(head);
  const int seg = __popcll(heads & ((2ull << lane) - 1ull));
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int seg_o = __shfl_down(seg, d);
    const uint32_t n_o = __shfl_down(p.n, d);
    const double w_o = __shfl_down(p.w, d);
    const double zr_o = __shfl_down(p.zr, d);
    const double zi_o = __shfl_down(p.zi, d);
    if (lane + d < 64 && seg_o == seg) {
      p.n += n_o;
      p.w += w_o;
      p.zr += zr_o;
      p.zi += zi_o;
    }
  }
  if (head && p.key >= 0) flush_atomic(acc, base, p);
}

__global__ __launch_bounds__(256) void k_extract_f64(ExtractArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t gwave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int c = (int)(gwave % a.n_chan);
  const int64_t chunk = gwave / a.n_chan;
  const int64_t row0 = chunk * (64 * kVPT) + (int64_t)lane * kVPT;
  if (chunk * (64 * kVPT) >= a.n_rows) return;           // whole wave past the end

  const double sc = a.chan->scale[c];
  const double spec = a.chan->spec[c];
  const double2 *__restrict__ resid = reinterpret_cast<const double2 *>(a.resid);
  const double *__restrict__ wt = reinterpret_cast<const double *>(a.weight);

  double u[kVPT], v[kVPT], w[kVPT], rr[kVPT], ri[kVPT], ww[kVPT];
#pragma unroll
  for (int j = 0; j < kVPT; ++j) {
    const int64_t row = row0 + j;
    if (row < a.n_rows) {
      const int64_t vi = row * a.n_chan + c;
      u[j] = __dmul_rn(a.u_m[row], sc);
      v[j] = __dmul_rn(a.v_m[row], sc);
      w[j] = __dmul_rn(a.w_m[row], sc);
      const double2 r = resid[vi];
      rr[j] = r.x;
      ri[j] = r.y;
      ww[j] = wt[vi];
    } else {
      u[j] = v[j] = w[j] = rr[j] = ri[j] = 0.0;
      ww[j] = 0.0;                                         // skipped like a flagged visibility
    }
  }

  const int s_begin = blockIdx.y * kSrcTile;
  const int s_end = min(a.n_src, s_begin + kSrcTile);
  for (int s = s_begin; s < s_end; ++s) {
    const SrcModel p = a.src[s];
    const SrcGeom g = a.geom[s];
    const double amp = spec * p.flux;
    Partial cur{-1, 0u, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < kVPT; ++j) {
      if (!(ww[j] > 0.0)) continue;
      const double ph = fma(u[j], p.l, fma(v[j], p.m, w[j] * p.n1));
      double sn, cs;
      sincospi(ph + ph, &sn, &cs);
      // residual * exp(-2 pi i ph)
      double zr = fma(rr[j], cs, ri[j] * sn);
      const double zi = fma(ri[j], cs, -(rr[j] * sn));
      // own model, real after the shift
      const double x = fma(p.q11, u[j] * u[j], fma(p.q12x2, u[j] * v[j], fma(p.q22, v[j] * v[j], 1.0)));
      const double r = rsqrt(x);
      zr = fma(amp, r * r * r, zr);
      const int ix = (int)rint(__dmul_rn(u[j], p.theta));
      const int iy = (int)rint(__dmul_rn(v[j], p.theta));
      const unsigned ox = (unsigned)(ix + g.half), oy = (unsigned)(iy + g.half);
      if (ox >= (unsigned)g.side || oy >= (unsigned)g.side) {
        atomicOr(a.err, 1u);
        continue;
      }
      const int key = (int)oy * g.side + (int)ox;
      if (key != cur.key) {
        if (cur.key >= 0) flush_atomic(a.acc, g.base, cur);
        cur.key = key;
        cur.n = 0u;
        cur.w = cur.zr = cur.zi = 0.0;
      }
      cur.n += 1u;
      cur.w += ww[j];
      cur.zr = fma(ww[j], zr, cur.zr);
      cur.zi = fma(ww[j], zi, cur.zi);
    }
    wave_flush(a.acc, g.base, cur);
  }
}

}  // namespace

hipError_t launch_extract_f64(const ExtractArgs &a, hipStream_t st) {
  const int64_t rows_per_wave = 64 * kVPT;
  const int64_t waves = ((a.n_rows + rows_per_wave - 1) / rows_per_wave) * a.n_chan;
  const int64_t blocks = (waves + 3) / 4;
  const int tiles = (a.n_src + kSrcTile - 1) / kSrcTile;
  hipLaunchKernelGGL(k_extract_f64, dim3((unsigned)blocks, (unsigned)tiles), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace rlf
