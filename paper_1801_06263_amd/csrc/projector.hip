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
#include "forward_device.h"
#include "project_device.h"
#include "projector.h"

namespace osscir {

// ----------------------------------------------------------------- kernels

__global__ void __launch_bounds__(256) k_pack(const float *__restrict__ f, int n, int nch, float4 *__restrict__ pk_xy,
                                               float4 *__restrict__ pk_yx) {
  __shared__ float4 tile[32][33];
  pack_block(f, n, nch, pk_xy, pk_yx, blockIdx.x * 32, blockIdx.y * 32, tile);  // padded coordinates
}

// Rays per forward-projection workgroup (a chunk of consecutive bins of one
// view), each walked by kFpParts waves.
constexpr int kFpRays = 64;
constexpr int kFpBlock = kFpRays * kFpParts;  // threads

// Workgroup -> (view v, bin chunk) of the forward projection.  XCD x takes
// the views [x V / 8, (x + 1) V / 8), an arc whose rays mostly share one
// major axis and hence one packed copy (see xcd_item), and walks it chunk
// rank by chunk rank: the centre chunks of every view of the arc first, the
// edge chunks last.  Central rays cross the most pixels, so the longest
// workgroups are dispatched first and the last ones, which set the tail of
// the launch, are the shortest.
__device__ __forceinline__ bool forward_item(int n_views, int nchunk, int &v, int &chunk) {
  const int b = blockIdx.x, x = b % kXcds, i = b / kXcds;
  const int v0 = (int)((long long)x * n_views / kXcds);
  const int nv = (int)((long long)(x + 1) * n_views / kXcds) - v0;
  if (i >= nv * nchunk) return false;  // also every workgroup of an XCD without views
  const int r = i / nv;                // chunk rank: 0 = centre
  v = v0 + (i - r * nv);
  const int mid = (nchunk - 1) / 2;
  chunk = (r & 1) ? mid + ((r + 1) >> 1) : mid - (r >> 1);  // mid, mid + 1, mid - 1, mid + 2, ...
  return true;
}

template <bool COUNT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) k_forward(ScanDesc sd, const float4 *__restrict__ pk_xy,
                                                  const float4 *__restrict__ pk_yx, float *__restrict__ p,
                                                  int p_stride, int nch) {
  const int nchunk = (sd.n_bins + kFpRays - 1) / kFpRays;
  int v, chunk;
  if (!forward_item(sd.n_views, nchunk, v, chunk)) return;  // uniform over the workgroup
  __shared__ float4 fwd_lds[kFpBlock / 64][kFpWaveRows];  // 4 KB of image rows per wave
  forward_rays<COUNT>(sd, pk_xy, pk_yx, p, p_stride, nch, v, chunk * kFpRays,
                      (float4 OSSCIR_LDS *)fwd_lds[threadIdx.x >> 6]);
}

// ----------------------------------------------------------------- plan

// The staged bins of every (tile, view) of the common back-projection path:
// one thread per pair, tiles in row-major order, views fastest.
__global__ void __launch_bounds__(256) k_tile_bins(ScanDesc sd, TileBins *__restrict__ out) {
  const int nt = (sd.n + kBpTile - 1) / kBpTile;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)nt * nt * sd.n_views) return;
  const int v = (int)(i % sd.n_views), t = (int)(i / sd.n_views);
  ViewTile vt;
  tile_view_bounds(sd, sd.views[v], t % nt, t / nt, vt);
  out[i] = TileBins{vt.d0, vt.nst, vt.K, vt.off};
}

// ----------------------------------------------------------------- back

template <int NCH, bool WIDE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) k_back(ScanDesc sd, const float *__restrict__ q, int q_stride,
                                               float *__restrict__ b, int b_stride) {
  __shared__ BpShared sh;
  const int nt = (sd.n + kBpTile - 1) / kBpTile;
  int item;
  if (!xcd_item(nt * nt, item)) return;
  const int t = as_const(sd.tile_order)[item];
  const int tile_y = t / nt, tile_x = t - tile_y * nt;
  double acc[NCH];
  back_accumulate<NCH, WIDE>(sd, tile_x, tile_y, q, q_stride, acc, sh, 0, sd.n_views);
  int tx, ty;
  bp_pixel_of_thread(threadIdx.x, tx, ty);
  const int ix = tile_x * kBpTile + tx;
  const int iy = tile_y * kBpTile + ty;
  if (ix >= sd.n || iy >= sd.n) return;
  const int k = iy * sd.n + ix;
#pragma unroll
  for (int c = 0; c < NCH; ++c) b[c * b_stride + k] = (float)acc[c];
}

// ----------------------------------------------------------------- launchers

// workgroups of k_forward: the largest arc of views (forward_item) times the
// bin chunks, on every XCD
static unsigned forward_blocks(const ScanDesc &sd) {
  const int nchunk = (sd.n_bins + kFpRays - 1) / kFpRays;
  return (unsigned)(kXcds * ((sd.n_views + kXcds - 1) / kXcds) * nchunk);
}

size_t pack_scratch_bytes(const ScanDesc &sd) {
  const size_t np = (size_t)sd.n + 2 * kPad;
  return 2 * np * np * sizeof(float4);
}

hipError_t launch_forward(const ScanDesc &sd, const float *f, int nch, float *p, void *pack, hipStream_t st) {
  const size_t fs = (size_t)sd.n * sd.n, ps = (size_t)sd.n_rays;
  const size_t np = (size_t)sd.n + 2 * kPad;
  float4 *pk_xy = reinterpret_cast<float4 *>(pack);
  float4 *pk_yx = pk_xy + np * np;
  const dim3 pgrid((unsigned)((np + 31) / 32), (unsigned)((np + 31) / 32));
  const dim3 fgrid(forward_blocks(sd));
  for (int c0 = 0; c0 < nch; c0 += 3) {
    const int k = nch - c0 >= 3 ? 3 : nch - c0;
    hipLaunchKernelGGL(k_pack, pgrid, dim3(256), 0, st, f + c0 * fs, sd.n, k, pk_xy, pk_yx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_forward<false>, fgrid, dim3(kFpBlock), 0, st, sd, pk_xy, pk_yx, p + c0 * ps, (int)ps, k);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_forward_packed(const ScanDesc &sd, const void *pack, float *p, hipStream_t st) {
  const size_t np = (size_t)sd.n + 2 * kPad;
  const float4 *pk_xy = reinterpret_cast<const float4 *>(pack);
  hipLaunchKernelGGL(k_forward<false>, dim3(forward_blocks(sd)), dim3(kFpBlock), 0, st, sd, pk_xy, pk_xy + np * np, p,
                     (int)sd.n_rays, 3);
  return hipGetLastError();
}

hipError_t launch_pack(const ScanDesc &sd, const float *f, int nch, void *pack, hipStream_t st) {
  const size_t np = (size_t)sd.n + 2 * kPad;
  float4 *pk_xy = reinterpret_cast<float4 *>(pack);
  const dim3 pgrid((unsigned)((np + 31) / 32), (unsigned)((np + 31) / 32));
  hipLaunchKernelGGL(k_pack, pgrid, dim3(256), 0, st, f, sd.n, nch, pk_xy, pk_xy + np * np);
  return hipGetLastError();
}

hipError_t launch_count(const ScanDesc &sd, int *nnz, hipStream_t st) {
  const dim3 fgrid(forward_blocks(sd));
  hipLaunchKernelGGL(k_forward<true>, fgrid, dim3(kFpBlock), 0, st, sd, nullptr, nullptr, reinterpret_cast<float *>(nnz),
                     0, 1);
  return hipGetLastError();
}

size_t tile_bins_count(const ScanDesc &sd) {
  const size_t nt = (size_t)(sd.n + kBpTile - 1) / kBpTile;
  return nt * nt * (size_t)sd.n_views;
}

hipError_t launch_tile_bins(const ScanDesc &sd, TileBins *out, hipStream_t st) {
  const size_t count = tile_bins_count(sd);
  hipLaunchKernelGGL(k_tile_bins, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, sd, out);
  return hipGetLastError();
}

// workgroups of the tile-driven kernels: every tile, rounded up to the XCD count
unsigned back_blocks(const ScanDesc &sd) {
  const int nt = (sd.n + kBpTile - 1) / kBpTile;
  return (unsigned)(((nt * nt + kXcds - 1) / kXcds) * kXcds);
}

template <int NCH>
static hipError_t launch_back_n(const ScanDesc &sd, const float *q, int q_stride, float *b, int b_stride,
                                hipStream_t st) {
  const dim3 grid(back_blocks(sd));
  if (sd.bp_wide)
    hipLaunchKernelGGL((k_back<NCH, true>), grid, dim3(kBpTile * kBpTile), 0, st, sd, q, q_stride, b, b_stride);
  else
    hipLaunchKernelGGL((k_back<NCH, false>), grid, dim3(kBpTile * kBpTile), 0, st, sd, q, q_stride, b, b_stride);
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
