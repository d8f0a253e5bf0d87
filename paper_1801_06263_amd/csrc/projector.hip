// Fan-beam projector X (ray-driven) and its exact transpose X^T
// (pixel-driven gather) for gfx950.
//
// Both kernels evaluate the same weight function (device_math.h) on the same
// FP32 per-ray line parameters, so every (ray, pixel) weight is bit-identical
// in X and X^T.  The forward projector visits, per ray, every pixel the line
// can touch; the back-projector visits, per pixel and view, every detector bin
// inside the pixel's shadow (plus a margin of 0.01 bin).  In both, a pair
// whose weight rounds to zero contributes nothing, so the two kernels
// accumulate exactly the same set of products.
#include "device_math.h"
#include "kernels.h"
#include "projector.h"
#include "project_device.h"

namespace osscir {

// ----------------------------------------------------------------- forward
//
// One thread per ray, a workgroup = 256 consecutive detector bins of one view
// (coalesced sinogram writes, neighbouring rays share image cache lines).
// The ray walks its major axis (the image axis closer to its direction); in
// each column (row) the line spans less than one pixel of the minor axis, so
// the two pixels floor(y*) and floor(y*)+1 around the crossing point y* hold
// every non-zero weight.  Within 0.11 degree of 45 degrees rounding could
// make a third pixel's weight non-zero: those rays test one more pixel.
template <int NCH>
__global__ void __launch_bounds__(256) k_forward(ScanDesc sd, const float *__restrict__ f, int f_stride,
                                                  float *__restrict__ p, int p_stride) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (d >= sd.n_bins) return;
  const int l = v * sd.n_bins + d;
  const RayLine ray = sd.rays[l];
  const float nx = (float)ray.nx, ny = (float)ray.ny, s = (float)ray.s;
  const int n = sd.n;
  const float c0 = sd.c0;

  float acc[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = 0.0f;

  const bool xmajor = fabsf(ny) >= fabsf(nx);
  const float nu = xmajor ? nx : ny;  // normal component along the walked axis
  const float nv = xmajor ? ny : nx;  // along the minor axis (|nv| >= 1/sqrt 2)
  const bool near45 = (fabsf(nv) - fabsf(nu)) < 2e-3f;
  const float inv_nv = 1.0f / nv;
  // minor index coordinate of the line at walked index iu:  base + slope * iu
  const float slope = -nu * inv_nv;
  const float base = s * inv_nv + c0 - slope * c0;
  // walked range where the minor coordinate lies in (-1.5, n + 0.5), widened
  int iu_lo = 0, iu_hi = n - 1;
  if (fabsf(slope) > 1e-12f) {
    const float t0 = (-1.5f - base) / slope;
    const float t1 = ((float)n + 0.5f - base) / slope;
    const float lo = fminf(t0, t1), hi = fmaxf(t0, t1);
    iu_lo = max(iu_lo, (int)floorf(fmaxf(lo, -4.0f)) - 1);
    iu_hi = min(iu_hi, (int)ceilf(fminf(hi, (float)n + 4.0f)) + 1);
  } else if (!(base > -1.5f && base < (float)n + 0.5f)) {
    iu_hi = -1;
  }
  for (int iu = iu_lo; iu <= iu_hi; ++iu) {
    const double U = (double)iu - sd.c0d;
    const float ys = __fmaf_rn(slope, (float)iu, base);
    const float fl = floorf(ys);
    const int iv0 = (int)fl;
    int cand[3] = {iv0, iv0 + 1, (ys - fl < 0.5f) ? iv0 - 1 : iv0 + 2};
    const int ncand = near45 ? 3 : 2;
    for (int j = 0; j < ncand; ++j) {
      const int iv = cand[j];
      if (iv < 0 || iv >= n) continue;
      const double V = (double)iv - sd.c0d;
      const double X = xmajor ? U : V;
      const double Y = xmajor ? V : U;
      const float w = chord_weight(ray, X, Y);
      const int idx = xmajor ? (iv * n + iu) : (iu * n + iv);
#pragma unroll
      for (int c = 0; c < NCH; ++c) acc[c] = __fmaf_rn(w, f[c * f_stride + idx], acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) p[c * p_stride + l] = acc[c];
}

template <int NCH>
__global__ void __launch_bounds__(256) k_back(ScanDesc sd, const float *__restrict__ q, int q_stride,
                                               float *__restrict__ b, int b_stride) {
  const int ix = blockIdx.x * 16 + (threadIdx.x & 15);
  const int iy = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (ix >= sd.n || iy >= sd.n) return;
  double acc[NCH];
  back_accumulate<NCH>(sd, ix, iy, q, q_stride, acc);
  const int k = iy * sd.n + ix;
#pragma unroll
  for (int c = 0; c < NCH; ++c) b[c * b_stride + k] = (float)acc[c];
}

// ----------------------------------------------------------------- launchers

template <int NCH>
static hipError_t launch_forward_n(const ScanDesc &sd, const float *f, int f_stride, float *p, int p_stride,
                                   hipStream_t st) {
  dim3 grid((sd.n_bins + 255) / 256, sd.n_views);
  hipLaunchKernelGGL(k_forward<NCH>, grid, dim3(256), 0, st, sd, f, f_stride, p, p_stride);
  return hipGetLastError();
}

hipError_t launch_forward(const ScanDesc &sd, const float *f, int nch, float *p, hipStream_t st) {
  const int fs = sd.n * sd.n, ps = sd.n_rays;
  for (int c0 = 0; c0 < nch;) {
    const int k = (nch - c0 >= 3) ? 3 : (nch - c0);
    hipError_t e;
    if (k == 3)
      e = launch_forward_n<3>(sd, f + (size_t)c0 * fs, fs, p + (size_t)c0 * ps, ps, st);
    else if (k == 2)
      e = launch_forward_n<2>(sd, f + (size_t)c0 * fs, fs, p + (size_t)c0 * ps, ps, st);
    else
      e = launch_forward_n<1>(sd, f + (size_t)c0 * fs, fs, p + (size_t)c0 * ps, ps, st);
    if (e != hipSuccess) return e;
    c0 += k;
  }
  return hipSuccess;
}

template <int NCH>
static hipError_t launch_back_n(const ScanDesc &sd, const float *q, int q_stride, float *b, int b_stride,
                                hipStream_t st) {
  dim3 grid((sd.n + 15) / 16, (sd.n + 15) / 16);
  hipLaunchKernelGGL(k_back<NCH>, grid, dim3(256), 0, st, sd, q, q_stride, b, b_stride);
  return hipGetLastError();
}

hipError_t launch_back(const ScanDesc &sd, const float *q, int nch, float *b, hipStream_t st) {
  const int bs = sd.n * sd.n, qs = sd.n_rays;
  for (int c0 = 0; c0 < nch;) {
    const int left = nch - c0;
    const int k = left >= 9 ? 9 : (left >= 6 ? 6 : (left >= 3 ? 3 : left));
    hipError_t e;
    const float *qq = q + (size_t)c0 * qs;
    float *bb = b + (size_t)c0 * bs;
    switch (k) {
      case 9: e = launch_back_n<9>(sd, qq, qs, bb, bs, st); break;
      case 6: e = launch_back_n<6>(sd, qq, qs, bb, bs, st); break;
      case 3: e = launch_back_n<3>(sd, qq, qs, bb, bs, st); break;
      case 2: e = launch_back_n<2>(sd, qq, qs, bb, bs, st); break;
      default: e = launch_back_n<1>(sd, qq, qs, bb, bs, st); break;
    }
    if (e != hipSuccess) return e;
    c0 += k;
  }
  return hipSuccess;
}

}  // namespace osscir
