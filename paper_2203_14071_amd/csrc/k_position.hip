// Position marginalisation (Sec. 2.4): the cross-correlation data of every
// compacted cell c and position offset x_p = (dl_p, dm_p),
//   G[c, p] = sqrt(W_c) Re(Vbar_c exp(-2 pi i (uc_c dl_p + vc_c dm_p))),
// so that the likelihood kernels form D(x_p) = sum_c h_c G[c, p] with the
// same profile values h_c = sqrt(W_c) f_c (as the cell records give them)
// for every offset.  Offsets: an n_side x n_side
// grid at spacing `step` (radians) centred on the catalogue position,
// p = p1 * n_side + p2, dl = (p1 - h) step, dm = (p2 - h) step,
// h = (n_side - 1) / 2.  One block per source, a thread per cell; the
// phases are small (|uc dl| is a fraction of a turn) and are evaluated once
// per extraction, so plain FP64 sincospi serves.
#include "rlf_internal.h"

namespace rlf {

namespace {

template <bool kMixed>
__global__ __launch_bounds__(256) void k_pos_prep(PosPrepArgs a) {
  const int s = blockIdx.x;
  const double theta = a.src[s].theta;
  const int64_t c0 = a.offsets[s], c1 = a.offsets[s + 1];
  const int h = (a.n_side - 1) / 2;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    const double uc = (double)a.ix[c] / theta, vc = (double)a.iy[c] / theta;   // as the compaction
    const double W = a.wsum[c], vr = a.vre[c], vi = a.vim[c];
    for (int p1 = 0; p1 < a.n_side; ++p1) {
      const double dl = (double)(p1 - h) * a.step;
      for (int p2 = 0; p2 < a.n_side; ++p2) {
        const double dm = (double)(p2 - h) * a.step;
        double sn, cs;
        sincospi(2.0 * fma(uc, dl, vc * dm), &sn, &cs);
        const double g = sqrt(W) * fma(vr, cs, vi * sn);
        const int64_t o = c * a.n_pos + p1 * a.n_side + p2;
        if (kMixed)
          a.g32[o] = (float)g;
        else
          a.g64[o] = g;
      }
    }
  }
}

}  // namespace

hipError_t launch_pos_prep(const PosPrepArgs &a, int mixed, hipStream_t st) {
  if (mixed)
    hipLaunchKernelGGL(k_pos_prep<true>, dim3(a.n_src), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_pos_prep<false>, dim3(a.n_src), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace rlf
