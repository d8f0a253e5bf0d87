// Pixel-driven gather of the back-projector, shared by the plain
// back-projection kernel and the kernels that fuse an epilogue (primal step,
// step lengths) into it.
//
// A workgroup owns a 16 x 16 pixel tile, one thread per pixel.  For each view
// (in order):
//   1. one thread projects the tile's four corners onto the detector: every
//      ray that meets the tile has its bin inside that shadow (+0.05 bin);
//   2. the workgroup stages those bins' line parameters and the NCH input
//      values into LDS (coalesced reads of consecutive bins);
//   3. each thread bounds its own pixel's shadow (the linearised projection
//      of the pixel centre, widened to cover the exact corner projections,
//      +0.02 bin) and accumulates w * q over the staged bins in that range.
// The weights are chord_weight() of the same FP32/FP64 inputs as the forward
// projector, so the result is X^T q with X's exact weights.  The few products
// of one view are summed in FP32; the running sum over views is FP64, so the
// result carries the rounding of the FP32 weights and inputs only (the
// per-pixel 3x3 step blocks built from it are ill-conditioned, and FP32
// accumulation over thousands of rays would shift the MOCCA trajectory).
#pragma once

#include "device_math.h"
#include "kernels.h"

namespace osscir {

constexpr int kBpTile = 16;
constexpr int kBpMaxBins = 128;  // bins staged at once; wider shadows are processed in chunks

struct BinLDS {
  double2 n;   // nx, ny
  float4 w0;   // a, hmax, kappa, q0
  float4 w1;   // q1..q4
  float4 w2;   // q5..q8
};

struct BpShared {
  BinLDS bins[kBpMaxBins];
  int range[2][2];  // by view parity: written by thread 0, read by all after a barrier
};

__device__ __forceinline__ float bin_coord(const ScanDesc &sd, const ViewGeom &vg, float X, float Y) {
  const float num = -vg.sb * X + vg.cb * Y;
  const float den = sd.sid_px - vg.cb * X - vg.sb * Y;
  return num / den * sd.bin_scale + sd.cbin;
}

template <int NCH>
__device__ __forceinline__ void back_accumulate(const ScanDesc &sd, int tile_x, int tile_y, const float *__restrict__ q,
                                                int q_stride, double acc[NCH], BpShared &sh) {
  static_assert(NCH >= 1 && NCH <= 9, "1..9 channels");
  const int tid = threadIdx.x;
  const int ix = tile_x * kBpTile + (tid & (kBpTile - 1));
  const int iy = tile_y * kBpTile + (tid / kBpTile);
  const int n = sd.n, nb = sd.n_bins;
  const bool inside = ix < n && iy < n;
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
  const float X = (float)ix - sd.c0;  // centred, for the detector projection
  const float Y = (float)iy - sd.c0;
  for (int v = 0; v < sd.n_views; ++v) {
    const ViewGeom vg = sd.views[v];
    if (tid == 0) {
      const float x0 = (float)(tile_x * kBpTile) - sd.c0 - 0.5f, x1 = x0 + (float)kBpTile;
      const float y0 = (float)(tile_y * kBpTile) - sd.c0 - 0.5f, y1 = y0 + (float)kBpTile;
      const float b00 = bin_coord(sd, vg, x0, y0), b01 = bin_coord(sd, vg, x0, y1);
      const float b10 = bin_coord(sd, vg, x1, y0), b11 = bin_coord(sd, vg, x1, y1);
      float lo = fminf(fminf(b00, b01), fminf(b10, b11));
      float hi = fmaxf(fmaxf(b00, b01), fmaxf(b10, b11));
      lo = fminf(fmaxf(lo, -2.0f), (float)nb + 1.0f);
      hi = fminf(fmaxf(hi, -2.0f), (float)nb + 1.0f);
      sh.range[v & 1][0] = max(0, (int)ceilf(lo - 0.05f));
      sh.range[v & 1][1] = min(nb - 1, (int)floorf(hi + 0.05f));
    }
    __syncthreads();
    const int D0 = sh.range[v & 1][0], D1 = sh.range[v & 1][1];
    // this pixel's candidate bins
    int dlo = D0, dhi = D1;
    {
      const float num = -vg.sb * X + vg.cb * Y;
      const float den = sd.sid_px - vg.cb * X - vg.sb * Y;
      if (den > 4.0f) {
        const float rden = 1.0f / den;
        const float t = num * rden;
        const float dtx = (-vg.sb + vg.cb * t) * rden;
        const float dty = (vg.cb + vg.sb * t) * rden;
        const float hw = 0.5f * (fabsf(dtx) + fabsf(dty)) * (1.0f + 1.5f * rden) * sd.bin_scale;
        const float bc = t * sd.bin_scale + sd.cbin;
        const float lo = fminf(fmaxf(bc - hw, -2.0f), (float)nb + 1.0f);
        const float hi = fminf(fmaxf(bc + hw, -2.0f), (float)nb + 1.0f);
        dlo = max(dlo, (int)ceilf(lo - 0.02f));
        dhi = min(dhi, (int)floorf(hi + 0.02f));
      }
    }
    const double dx = vg.sx - (double)ix;
    const double dy = vg.sy - (double)iy;
    for (int c0 = D0; c0 <= D1; c0 += kBpMaxBins) {
      const int c1 = min(D1, c0 + kBpMaxBins - 1);
      // stage bins c0..c1
      for (int b = tid; b <= c1 - c0; b += blockDim.x) {
        const int l = v * nb + c0 + b;
        const RayLine r = sd.rays[l];
        float qq[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) qq[c] = c < NCH ? q[c * q_stride + l] : 0.0f;
        BinLDS e;
        e.n = make_double2(r.nx, r.ny);
        e.w0 = make_float4(r.a, r.hmax, r.kappa, qq[0]);
        e.w1 = make_float4(qq[1], qq[2], qq[3], qq[4]);
        e.w2 = make_float4(qq[5], qq[6], qq[7], qq[8]);
        sh.bins[b] = e;
      }
      __syncthreads();
      if (inside) {
        float part[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) part[c] = 0.0f;
        const int e0 = max(dlo, c0), e1 = min(dhi, c1);
        for (int d = e0; d <= e1; ++d) {
          const BinLDS &e = sh.bins[d - c0];
          const double2 nn = e.n;
          const float4 w0 = e.w0;
          const float w = chord_weight(nn.x, nn.y, w0.x, w0.y, w0.z, dx, dy);
          float qv[9];
          qv[0] = w0.w;
          if (NCH > 1) {
            const float4 w1 = e.w1;
            qv[1] = w1.x; qv[2] = w1.y; qv[3] = w1.z; qv[4] = w1.w;
          }
          if (NCH > 5) {
            const float4 w2 = e.w2;
            qv[5] = w2.x; qv[6] = w2.y; qv[7] = w2.z; qv[8] = w2.w;
          }
#pragma unroll
          for (int c = 0; c < NCH; ++c) part[c] = __fmaf_rn(w, qv[c], part[c]);
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) acc[c] += (double)part[c];
      }
      __syncthreads();
    }
  }
}

}  // namespace osscir
