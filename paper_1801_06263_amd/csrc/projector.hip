// Fan-beam projector X (ray-driven) and its exact transpose X^T
// (pixel-driven gather) for gfx950.
//
// Both kernels evaluate the same weight function (device_math.h) on the same
// per-ray line parameters and the same FP64 source-to-pixel offsets, so every
// (ray, pixel) weight is bit-identical in X and X^T.  The forward projector
// visits, per ray, every pixel the line can touch; the back-projector visits,
// per pixel and view, every detector bin inside the pixel's shadow (plus a
// margin).  In both, a pair whose weight rounds to zero contributes nothing,
// so the two kernels accumulate exactly the same set of products.
#include "device_math.h"
#include "kernels.h"
#include "project_device.h"
#include "projector.h"

namespace osscir {

// ----------------------------------------------------------------- packing
//
// Up to three planar channels -> two interleaved float4 images: pk_xy[iy][ix]
// (rows contiguous) and pk_yx[ix][iy] (columns contiguous), through a
// 32 x 32 LDS tile for the transposed writes.
__global__ void __launch_bounds__(256) k_pack(const float *__restrict__ f, int n, int nch, float4 *__restrict__ pk_xy,
                                               float4 *__restrict__ pk_yx) {
  __shared__ float4 tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const size_t nn = (size_t)n * n;
  for (int r = ty; r < 32; r += 8) {
    const int ix = bx + tx, iy = by + r;
    float4 val = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (ix < n && iy < n) {
      const size_t k = (size_t)iy * n + ix;
      val.x = f[k];
      if (nch > 1) val.y = f[nn + k];
      if (nch > 2) val.z = f[2 * nn + k];
      pk_xy[k] = val;
    }
    tile[r][tx] = val;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int iy = by + tx, ix = bx + r;
    if (ix < n && iy < n) pk_yx[(size_t)ix * n + iy] = tile[tx][r];
  }
}

// ----------------------------------------------------------------- forward
//
// One thread per ray, a workgroup = 256 consecutive detector bins of one view
// (coalesced sinogram writes).  A ray walks its major axis (the image axis
// closer to its direction); in each column (row) the line spans less than one
// pixel of the minor axis, so the two pixels floor(y*) and floor(y*)+1 around
// its crossing point y* hold every non-zero weight (within 0.11 degree of 45
// degrees a third pixel is tested, against rounding).  Rays walking columns
// read the column-contiguous packed image, rays walking rows the
// row-contiguous one, so neighbouring lanes (neighbouring bins) read
// neighbouring addresses; all lanes of a wave step through the same walk
// index (the wave's union of walk ranges).
__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, 64));
  return x;
}
__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
  return x;
}

template <bool COUNT>
__global__ void __launch_bounds__(256) k_forward(ScanDesc sd, const float4 *__restrict__ pk_xy,
                                                  const float4 *__restrict__ pk_yx, float *__restrict__ p,
                                                  int p_stride, int nch) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  const int n = sd.n;
  const bool active = d < sd.n_bins;
  const ViewGeom vg = sd.views[v];
  RayLine ray{1.0, 0.0, 0.0f, 0.0f, 0.0f, 0.0f};
  bool xmajor = true, near45 = false;
  float slope = 0.0f, base = 0.0f;
  int iu_lo = n, iu_hi = -1;
  if (active) {
    ray = sd.rays[v * sd.n_bins + d];
    // the line in index coordinates: nx ix + ny iy = nx sx + ny sy
    const double sidx = ray.nx * vg.sx + ray.ny * vg.sy;
    xmajor = fabs(ray.ny) >= fabs(ray.nx);
    const double nu = xmajor ? ray.nx : ray.ny;  // along the walked axis
    const double nv = xmajor ? ray.ny : ray.nx;  // along the minor axis, |nv| >= 1/sqrt 2
    near45 = (fabs(nv) - fabs(nu)) < 2e-3;
    slope = (float)(-nu / nv);
    base = (float)(sidx / nv);
    // walked indices where the crossing lies in (-1.5, n + 0.5), widened by one
    iu_lo = 0;
    iu_hi = n - 1;
    if (fabsf(slope) > 1e-12f) {
      const float t0 = (-1.5f - base) / slope;
      const float t1 = ((float)n + 0.5f - base) / slope;
      const float lo = fminf(t0, t1), hi = fmaxf(t0, t1);
      iu_lo = max(iu_lo, (int)floorf(fmaxf(lo, -4.0f)) - 1);
      iu_hi = min(iu_hi, (int)ceilf(fminf(hi, (float)n + 4.0f)) + 1);
    } else if (!(base > -1.5f && base < (float)n + 0.5f)) {
      iu_lo = n;
      iu_hi = -1;
    }
  }
  const int lo = wave_min(iu_lo), hi = wave_max(iu_hi);
  const float4 *__restrict__ img = xmajor ? pk_yx : pk_xy;
  const double s_u = xmajor ? vg.sx : vg.sy;  // source along the walked axis
  const double s_v = xmajor ? vg.sy : vg.sx;
  const int ncand = near45 ? 3 : 2;
  float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
  for (int iu = lo; iu <= hi; ++iu) {
    if (!active) continue;
    const float ys = __fmaf_rn(slope, (float)iu, base);
    const float fl = floorf(ys);
    const int iv0 = (int)fl;
    const int extra = (ys - fl < 0.5f) ? iv0 - 1 : iv0 + 2;
    const double du = s_u - (double)iu;
    const float4 *__restrict__ line = img + (size_t)iu * n;
    for (int j = 0; j < ncand; ++j) {
      const int iv = j == 0 ? iv0 : (j == 1 ? iv0 + 1 : extra);
      if (iv < 0 || iv >= n) continue;
      const double dv = s_v - (double)iv;
      const float w = chord_weight(ray.nx, ray.ny, ray.a, ray.hmax, ray.kappa, xmajor ? du : dv, xmajor ? dv : du);
      if (COUNT) {
        a0 += (w > 0.0f) ? 1.0f : 0.0f;
      } else {
        const float4 fv = line[iv];
        a0 = __fmaf_rn(w, fv.x, a0);
        a1 = __fmaf_rn(w, fv.y, a1);
        a2 = __fmaf_rn(w, fv.z, a2);
      }
    }
  }
  if (!active) return;
  const int l = v * sd.n_bins + d;
  if (COUNT) {
    reinterpret_cast<int *>(p)[l] = (int)a0;
    return;
  }
  p[l] = a0;
  if (nch > 1) p[p_stride + l] = a1;
  if (nch > 2) p[2 * p_stride + l] = a2;
}

// ----------------------------------------------------------------- back

template <int NCH>
__global__ void __launch_bounds__(256) k_back(ScanDesc sd, const float *__restrict__ q, int q_stride,
                                               float *__restrict__ b, int b_stride) {
  __shared__ BpShared sh;
  double acc[NCH];
  back_accumulate<NCH>(sd, blockIdx.x, blockIdx.y, q, q_stride, acc, sh);
  const int ix = blockIdx.x * kBpTile + (threadIdx.x & (kBpTile - 1));
  const int iy = blockIdx.y * kBpTile + (threadIdx.x / kBpTile);
  if (ix >= sd.n || iy >= sd.n) return;
  const int k = iy * sd.n + ix;
#pragma unroll
  for (int c = 0; c < NCH; ++c) b[c * b_stride + k] = (float)acc[c];
}

// ----------------------------------------------------------------- launchers

size_t pack_scratch_bytes(const ScanDesc &sd) { return 2 * (size_t)sd.n * sd.n * sizeof(float4); }

hipError_t launch_forward(const ScanDesc &sd, const float *f, int nch, float *p, void *pack, hipStream_t st) {
  const size_t fs = (size_t)sd.n * sd.n, ps = (size_t)sd.n_rays;
  float4 *pk_xy = reinterpret_cast<float4 *>(pack);
  float4 *pk_yx = pk_xy + fs;
  const dim3 pgrid((sd.n + 31) / 32, (sd.n + 31) / 32);
  const dim3 fgrid((sd.n_bins + 255) / 256, sd.n_views);
  for (int c0 = 0; c0 < nch; c0 += 3) {
    const int k = nch - c0 >= 3 ? 3 : nch - c0;
    hipLaunchKernelGGL(k_pack, pgrid, dim3(256), 0, st, f + c0 * fs, sd.n, k, pk_xy, pk_yx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_forward<false>, fgrid, dim3(256), 0, st, sd, pk_xy, pk_yx, p + c0 * ps, (int)ps, k);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_count(const ScanDesc &sd, int *nnz, hipStream_t st) {
  const dim3 fgrid((sd.n_bins + 255) / 256, sd.n_views);
  hipLaunchKernelGGL(k_forward<true>, fgrid, dim3(256), 0, st, sd, nullptr, nullptr, reinterpret_cast<float *>(nnz),
                     0, 1);
  return hipGetLastError();
}

template <int NCH>
static hipError_t launch_back_n(const ScanDesc &sd, const float *q, int q_stride, float *b, int b_stride,
                                hipStream_t st) {
  const dim3 grid((sd.n + kBpTile - 1) / kBpTile, (sd.n + kBpTile - 1) / kBpTile);
  hipLaunchKernelGGL(k_back<NCH>, grid, dim3(kBpTile * kBpTile), 0, st, sd, q, q_stride, b, b_stride);
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
