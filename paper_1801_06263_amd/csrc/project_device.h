// Pixel-driven gather of the back-projector, shared by the plain
// back-projection kernel and the kernels that fuse an epilogue (primal step,
// step lengths) into it.
#pragma once

#include "device_math.h"
#include "kernels.h"

namespace osscir {

// ----------------------------------------------------------------- back
//
// One thread per pixel, 16 x 16 pixel tiles.  For each view (in order) the
// pixel's four corners are projected onto the detector; every bin whose
// centre falls in that shadow (widened by 0.01 bin) is a candidate ray.
// The few products of one view are summed in FP32; the running sum over
// views is FP64, so the result carries the rounding of the FP32 weights and
// inputs only (the per-pixel 3x3 step blocks built from it are
// ill-conditioned, and FP32 accumulation over thousands of rays would shift
// the MOCCA trajectory measurably).
template <int NCH>
__device__ __forceinline__ void back_accumulate(const ScanDesc &sd, int ix, int iy, const float *__restrict__ q,
                                                int q_stride, double acc[NCH]) {
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
  const float X = (float)ix - sd.c0;
  const float Y = (float)iy - sd.c0;
  const double Xd = (double)ix - sd.c0d;
  const double Yd = (double)iy - sd.c0d;
  const int nb = sd.n_bins;
  for (int v = 0; v < sd.n_views; ++v) {
    const float2 cs = sd.views[v];
    float bmin = 3.0e38f, bmax = -3.0e38f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float x = X + ((k & 1) ? 0.5f : -0.5f);
      const float y = Y + ((k & 2) ? 0.5f : -0.5f);
      const float num = -cs.y * x + cs.x * y;
      const float den = sd.sid_px - cs.x * x - cs.y * y;
      const float b = num / den * sd.bin_scale + sd.cbin;
      bmin = fminf(bmin, b);
      bmax = fmaxf(bmax, b);
    }
    // clamp before the integer conversion (the shadow may lie off the detector)
    bmin = fminf(fmaxf(bmin, -2.0f), (float)nb + 1.0f);
    bmax = fminf(fmaxf(bmax, -2.0f), (float)nb + 1.0f);
    const int d_lo = max(0, (int)ceilf(bmin - 0.01f));
    const int d_hi = min(nb - 1, (int)floorf(bmax + 0.01f));
    const int lv = v * nb;
    float part[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) part[c] = 0.0f;
    for (int d = d_lo; d <= d_hi; ++d) {
      const int l = lv + d;
      const float w = chord_weight(sd.rays[l], Xd, Yd);
#pragma unroll
      for (int c = 0; c < NCH; ++c) part[c] = __fmaf_rn(w, q[c * q_stride + l], part[c]);
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] += (double)part[c];
  }
}


}  // namespace osscir
