// Per-ray spectral model, step lengths and dual step, the fused primal
// update, and the D_TPL reduction (Sec. II of arXiv 1801.06263) for gfx950:
// the single-scan kernels over the device functions of spectral_device.h.
#include "device_math.h"
#include "kernels.h"
#include "projector.h"
#include "project_device.h"
#include "spectral.h"
#include "spectral_device.h"

namespace osscir {

// ---------------------------------------------------------------- model out

template <typename T, bool PB>
__global__ void __launch_bounds__(256) k_spectral_model(ScanDesc sd, const float *__restrict__ p,
                                                         const float *__restrict__ c, float *__restrict__ chat,
                                                         float *__restrict__ r, float *__restrict__ G,
                                                         float *__restrict__ H, float *__restrict__ Hp) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int L = sd.n_rays;
  if (l >= L) return;
  const int d = l % sd.n_bins;
  float g[kWin], af[kWin * kMat], hb[kWin * 6], n0[kWin];
  const float scale = energy_sums_safe<true, true, PB>(sd, p[l], p[L + l], p[2 * L + l], g, af, hb, d);
  ray_n0<PB>(sd, l, d, n0);
  T a[kWin][kMat], cw[kWin], rg[kWin];
#pragma unroll
  for (int w = 0; w < kWin; ++w) {
    const float ch = n0[w] * g[w] * scale;
    const float rw = c[w * L + l] - ch;
    if (chat) chat[w * L + l] = ch;
    if (r) r[w * L + l] = rw;
    cw[w] = (T)c[w * L + l];
    rg[w] = (T)rw / (T)g[w];
#pragma unroll
    for (int m = 0; m < kMat; ++m) {
      const float gw = af[w * kMat + m] / g[w];
      a[w][m] = (T)gw;
      if (G) G[(w * kMat + m) * L + l] = gw;
    }
  }
  if (H || Hp) {
    T h[6], hp[6];
    ray_hessian<T>(a, cw, rg, hb, h);
    if (H)
#pragma unroll
      for (int j = 0; j < 6; ++j) H[j * L + l] = (float)h[j];
    if (Hp) {
      clip_negative_curvature<T, sizeof(T) == 8 ? 8 : 6>(h, hp);
#pragma unroll
      for (int j = 0; j < 6; ++j) Hp[j * L + l] = (float)hp[j];
    }
  }
}

// ---------------------------------------------------------------- dual step

// NEST: pbar (the line integrals of fbar) is read, p is the expansion point's
template <typename T, bool CLIP, bool BLOCK, bool PB, bool NEST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) k_spectral_dual(ScanDesc sd, const float *__restrict__ p,
                                                        const float *__restrict__ c, float *__restrict__ y,
                                                        float *__restrict__ qS, float lambda,
                                                        const float *__restrict__ pbar) {
  spectral_dual_ray<T, CLIP, BLOCK, PB, false, NEST>(sd, p, c, y, qS, lambda, blockIdx.x * blockDim.x + threadIdx.x,
                                                     nullptr, pbar);
}

// energy sums on the matrix cores (shared response table, 64-ray waves)
template <typename T, bool CLIP, bool BLOCK, bool NEST>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4)))
    k_spectral_dual_mfma(ScanDesc sd, const float *__restrict__ p, const float *__restrict__ c, float *__restrict__ y,
                         float *__restrict__ qS, float lambda, const float *__restrict__ pbar) {
  extern __shared__ float stab[];
  stage_table(sd, stab);
  __syncthreads();
  spectral_dual_ray<T, CLIP, BLOCK, false, true, NEST>(sd, p, c, y, qS, lambda,
                                                       blockIdx.x * blockDim.x + threadIdx.x, stab, pbar);
}

// ---------------------------------------------------------------- steps only

template <bool BLOCK>
__global__ void __launch_bounds__(256) k_steps(ScanDesc sd, const float *__restrict__ G, float lambda,
                                                float *__restrict__ sigma, float *__restrict__ terms) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int L = sd.n_rays;
  if (l >= L) return;
  const float rho = sd.rho[l];
  float a[kWin][kMat];
#pragma unroll
  for (int w = 0; w < kWin; ++w)
#pragma unroll
    for (int m = 0; m < kMat; ++m) a[w][m] = G[(w * kMat + m) * L + l];
  const bool hit = rho > 0.0f;
  if (BLOCK) {
    float S[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int w = 0; w < kWin; ++w) {
      const float nrm = sqrtf(a[w][0] * a[w][0] + a[w][1] * a[w][1] + a[w][2] * a[w][2]);
      sigma[w * L + l] = hit ? 1.0f / (lambda * rho * nrm) : 0.0f;
      const float inv = nrm > 0.0f ? 1.0f / nrm : 0.0f;
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int n = m; n < 3; ++n) S[ut(m, n)] += a[w][m] * a[w][n] * inv;
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) terms[j * L + l] = hit ? S[j] : 0.0f;
  } else {
    float h[3] = {0, 0, 0};
#pragma unroll
    for (int w = 0; w < kWin; ++w) {
      const float l1 = fabsf(a[w][0]) + fabsf(a[w][1]) + fabsf(a[w][2]);
      sigma[w * L + l] = hit ? 1.0f / (lambda * rho * l1) : 0.0f;
#pragma unroll
      for (int m = 0; m < 3; ++m) h[m] += fabsf(a[w][m]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) terms[j * L + l] = hit ? h[j] : 0.0f;
  }
}

// scale back-projected terms: block T^-1 = acc / lambda, diag tau = lambda / acc
template <bool BLOCK>
__global__ void k_scale_steps(int count, float lambda, float *__restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float x = v[i];
  v[i] = BLOCK ? x / lambda : (x > 0.0f ? lambda / x : 0.0f);
}

// ---------------------------------------------------------------- primal

// PACK: fbar' is also written into the packed images of the next forward
// projection (pk_xy, pk_yx: interior pixels; borders already zero)
template <bool BLOCK, bool WIDE, bool PACK, bool COPY>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) k_back_primal(ScanDesc sd, const float *__restrict__ qS,
                                                      float *__restrict__ f, float *__restrict__ fbar, float lambda,
                                                      float4 *__restrict__ pk_xy, float4 *__restrict__ pk_yx) {
  __shared__ BpShared sh;
  const int nt = (sd.n + kBpTile - 1) / kBpTile;
  int item;
  if (!xcd_item(nt * nt, item)) return;
  const int t = as_const(sd.tile_order)[item];
  const int tile_y = t / nt;
  back_primal_tile<BLOCK, WIDE, PACK, COPY>(sd, qS, f, fbar, lambda, t - tile_y * nt, tile_y, sh,
                                            PrimalEpilogue{pk_xy, pk_yx, nullptr});
}

// Split back-projection (ScanDesc::bp_parts > 1, grids of few tiles): the
// workgroup of (tile, part) sums the tile's pixels over the part's views and
// leaves the FP64 sums in bp[part][c][pixel]; k_primal_combine adds the
// parts in order and takes the primal step.  The one-workgroup-per-tile
// kernels form the same sums part by part (FOLD), so every path gives the
// same bits.
template <bool BLOCK, bool COPY>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) k_back_partial(ScanDesc sd, const float *__restrict__ qS,
                                                                                     double *__restrict__ bp) {
  __shared__ BpShared sh;
  constexpr int NCH = BLOCK ? 9 : 6;
  const int nt = (sd.n + kBpTile - 1) / kBpTile;
  const int P = sd.bp_parts;
  int item;
  if (!xcd_item(nt * nt * P, item)) return;
  const int ti = item / P, part = item - ti * P;  // the XCD's tiles, every part of each
  const int t = as_const(sd.tile_order)[ti];
  const int tile_y = t / nt, tile_x = t - tile_y * nt;
  const int vb = part * sd.bp_part_views, ve = min(sd.n_views, vb + sd.bp_part_views);
  double acc[NCH];
  back_accumulate<NCH, false, true, COPY>(sd, tile_x, tile_y, qS, 0, acc, sh, vb, ve);
  int tx, ty;
  bp_pixel_of_thread(threadIdx.x, tx, ty);
  const int ix = tile_x * kBpTile + tx, iy = tile_y * kBpTile + ty;
  if (ix >= sd.n || iy >= sd.n) return;
  const size_t nn = (size_t)sd.n * sd.n, k = (size_t)iy * sd.n + ix;
#pragma unroll
  for (int c = 0; c < NCH; ++c) bp[((size_t)part * NCH + c) * nn + k] = acc[c];
}

template <bool BLOCK, bool PACK>
__global__ void __launch_bounds__(256) k_primal_combine(ScanDesc sd, const double *__restrict__ bp, float *__restrict__ f,
                                                        float *__restrict__ fbar, float lambda, float4 *__restrict__ pk_xy,
                                                        float4 *__restrict__ pk_yx) {
  __shared__ float4 tile[kBpTile][kBpTile + 1];
  __shared__ double2 red[kBpThreads / 64];
  constexpr int NCH = BLOCK ? 9 : 6;
  const int nt = (sd.n + kBpTile - 1) / kBpTile;
  int item;
  if (!xcd_item(nt * nt, item)) return;
  const int t = as_const(sd.tile_order)[item];
  const int tile_y = t / nt, tile_x = t - tile_y * nt;
  int tx, ty;
  bp_pixel_of_thread(threadIdx.x, tx, ty);
  const int ix = tile_x * kBpTile + tx, iy = tile_y * kBpTile + ty;
  double acc[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
  if (ix < sd.n && iy < sd.n) {
    const size_t nn = (size_t)sd.n * sd.n, k = (size_t)iy * sd.n + ix;
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = bp[(size_t)c * nn + k];
    for (int p = 1; p < sd.bp_parts; ++p)
#pragma unroll
      for (int c = 0; c < NCH; ++c) acc[c] += bp[((size_t)p * NCH + c) * nn + k];
  }
  primal_epilogue<BLOCK, PACK>(sd, acc, f, fbar, lambda, tile_x, tile_y, tile, red, PrimalEpilogue{pk_xy, pk_yx, nullptr});
}

// ---------------------------------------------------------------- D_TPL

template <bool PB>
__global__ void __launch_bounds__(256) k_dtpl_partial(ScanDesc sd, const float *__restrict__ p,
                                                       const float *__restrict__ c, double *__restrict__ partial) {
  __shared__ double red[256];
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int L = sd.n_rays;
  double term = 0.0;
  if (l < L) {
    const int d = l % sd.n_bins;
    float g[kWin], n0[kWin];
    energy_sums<false, false, false, PB>(sd, p[l], p[L + l], p[2 * L + l], g, nullptr, nullptr, 0.0f, d);
    ray_n0<PB>(sd, l, d, n0);
#pragma unroll
    for (int w = 0; w < kWin; ++w) {
      const double ch = (double)n0[w] * (double)g[w];
      const double cv = (double)c[w * L + l];
      term += ch - cv - (cv > 0.0 ? cv * log(ch / cv) : 0.0);
    }
  }
  red[threadIdx.x] = term;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_sum_partials(const double *__restrict__ partial, int count,
                                                       double *__restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// ---------------------------------------------------------------- basis change

// out[j][k] = sum_m M[j][m] in[m][k] for 3-channel maps (in place allowed):
// the change of material basis of mu-preconditioning.
__global__ void __launch_bounds__(256) k_material_transform(double m00, double m01, double m02, double m10,
                                                             double m11, double m12, double m20, double m21,
                                                             double m22, const float *in, float *out, int npix) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npix) return;
  const double a = in[k], b = in[npix + k], c = in[2 * npix + k];
  out[k] = (float)(m00 * a + m01 * b + m02 * c);
  out[npix + k] = (float)(m10 * a + m11 * b + m12 * c);
  out[2 * npix + k] = (float)(m20 * a + m21 * b + m22 * c);
}

// ---------------------------------------------------------------- launchers

static inline dim3 ray_grid(const ScanDesc &sd) { return dim3((sd.n_rays + 255) / 256); }
static inline dim3 pix_grid(const ScanDesc &sd) { return dim3(back_blocks(sd)); }

hipError_t launch_spectral_model(const ScanDesc &sd, const float *p, const float *c, float *chat, float *r,
                                 float *G, float *H, float *Hp, bool fp64, hipStream_t st) {
#define OSSCIR_MODEL(T, PB) \
  hipLaunchKernelGGL((k_spectral_model<T, PB>), ray_grid(sd), dim3(256), 0, st, sd, p, c, chat, r, G, H, Hp)
  if (sd.per_bin) {
    if (fp64) OSSCIR_MODEL(double, true); else OSSCIR_MODEL(float, true);
  } else {
    if (fp64) OSSCIR_MODEL(double, false); else OSSCIR_MODEL(float, false);
  }
#undef OSSCIR_MODEL
  return hipGetLastError();
}

hipError_t launch_spectral_dual(const ScanDesc &sd, const float *p, const float *c, float *y, float *qS,
                                float lambda, bool clip, bool block, bool fp64, hipStream_t st, const float *pbar) {
  // matrix-core energy sums: a plan property (shared table within 64 KB of LDS)
  // 512-ray workgroups: the table is staged once per eight waves (3% faster than four)
  const size_t mfma_lds = mfma_lds_bytes(sd.n_energy, 8);
  const bool mfma = sd.mfma != 0;
#define OSSCIR_DUAL_N(T, C, B, N)                                                                            \
  do {                                                                                                      \
    if (sd.per_bin)                                                                                         \
      hipLaunchKernelGGL((k_spectral_dual<T, C, B, true, N>), ray_grid(sd), dim3(256), 0, st, sd, p, c, y,   \
                         qS, lambda, pbar);                                                                 \
    else if (mfma)                                                                                          \
      hipLaunchKernelGGL((k_spectral_dual_mfma<T, C, B, N>), dim3((sd.n_rays + 511) / 512), dim3(512),       \
                         mfma_lds, st, sd, p, c, y, qS, lambda, pbar);                                      \
    else                                                                                                    \
      hipLaunchKernelGGL((k_spectral_dual<T, C, B, false, N>), ray_grid(sd), dim3(256), 0, st, sd, p, c, y,  \
                         qS, lambda, pbar);                                                                 \
  } while (0)
#define OSSCIR_DUAL(T, C, B)                      \
  do {                                            \
    if (pbar)                                     \
      OSSCIR_DUAL_N(T, C, B, true);               \
    else                                          \
      OSSCIR_DUAL_N(T, C, B, false);              \
  } while (0)
  if (fp64) {
    if (clip) {
      if (block) OSSCIR_DUAL(double, true, true); else OSSCIR_DUAL(double, true, false);
    } else {
      if (block) OSSCIR_DUAL(double, false, true); else OSSCIR_DUAL(double, false, false);
    }
  } else {
    if (clip) {
      if (block) OSSCIR_DUAL(float, true, true); else OSSCIR_DUAL(float, true, false);
    } else {
      if (block) OSSCIR_DUAL(float, false, true); else OSSCIR_DUAL(float, false, false);
    }
  }
#undef OSSCIR_DUAL
#undef OSSCIR_DUAL_N
  return hipGetLastError();
}

hipError_t launch_back_primal(const ScanDesc &sd, const float *qS, float *f, float *fbar, float lambda, bool block,
                              void *pack, double *bp, hipStream_t st) {
  const size_t np = (size_t)sd.n + 2 * kPad;
  float4 *pk_xy = reinterpret_cast<float4 *>(pack);
  float4 *pk_yx = pack ? pk_xy + np * np : nullptr;
  if (sd.bp_parts > 1 && !sd.bp_wide) {
    if (!bp) return hipErrorInvalidValue;
    const int nt = (sd.n + kBpTile - 1) / kBpTile;
    const unsigned items = (unsigned)(nt * nt * sd.bp_parts);
    const dim3 pgrid((items + kXcds - 1) / kXcds * kXcds);
#define OSSCIR_BPART(B, C) hipLaunchKernelGGL((k_back_partial<B, C>), pgrid, dim3(256), 0, st, sd, qS, bp)
#define OSSCIR_BCOMB(B, P) \
  hipLaunchKernelGGL((k_primal_combine<B, P>), pix_grid(sd), dim3(256), 0, st, sd, bp, f, fbar, lambda, pk_xy, pk_yx)
    if (block) {
      if (sd.bp_copy) OSSCIR_BPART(true, true); else OSSCIR_BPART(true, false);
    } else {
      if (sd.bp_copy) OSSCIR_BPART(false, true); else OSSCIR_BPART(false, false);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (block) {
      if (pack) OSSCIR_BCOMB(true, true); else OSSCIR_BCOMB(true, false);
    } else {
      if (pack) OSSCIR_BCOMB(false, true); else OSSCIR_BCOMB(false, false);
    }
#undef OSSCIR_BCOMB
#undef OSSCIR_BPART
    return hipGetLastError();
  }
#define OSSCIR_BP(B, W, P, C)                                                                                   \
  hipLaunchKernelGGL((k_back_primal<B, W, P, C>), pix_grid(sd), dim3(256), 0, st, sd, qS, f, fbar, lambda, pk_xy, \
                     pk_yx)
#define OSSCIR_BP2(B, P)                           \
  do {                                             \
    if (sd.bp_wide)                                \
      OSSCIR_BP(B, true, P, false);                \
    else if (sd.bp_copy)                           \
      OSSCIR_BP(B, false, P, true);                \
    else                                           \
      OSSCIR_BP(B, false, P, false);               \
  } while (0)
  if (block) {
    if (pack) OSSCIR_BP2(true, true); else OSSCIR_BP2(true, false);
  } else {
    if (pack) OSSCIR_BP2(false, true); else OSSCIR_BP2(false, false);
  }
#undef OSSCIR_BP2
#undef OSSCIR_BP
  return hipGetLastError();
}

hipError_t launch_steps(const ScanDesc &sd, const float *G, float lambda, bool block, float *sigma, float *terms,
                        float *out_img, hipStream_t st) {
  if (block)
    hipLaunchKernelGGL(k_steps<true>, ray_grid(sd), dim3(256), 0, st, sd, G, lambda, sigma, terms);
  else
    hipLaunchKernelGGL(k_steps<false>, ray_grid(sd), dim3(256), 0, st, sd, G, lambda, sigma, terms);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nch = block ? 6 : 3;
  e = launch_back(sd, terms, nch, out_img, st);
  if (e != hipSuccess) return e;
  const int count = nch * sd.n * sd.n;
  if (block)
    hipLaunchKernelGGL(k_scale_steps<true>, dim3((count + 255) / 256), dim3(256), 0, st, count, lambda, out_img);
  else
    hipLaunchKernelGGL(k_scale_steps<false>, dim3((count + 255) / 256), dim3(256), 0, st, count, lambda, out_img);
  return hipGetLastError();
}

hipError_t launch_material_transform(const double M[9], const float *in, float *out, int npix, hipStream_t st) {
  hipLaunchKernelGGL(k_material_transform, dim3((npix + 255) / 256), dim3(256), 0, st, M[0], M[1], M[2], M[3], M[4],
                     M[5], M[6], M[7], M[8], in, out, npix);
  return hipGetLastError();
}

int dtpl_partial_count(const ScanDesc &sd) { return (sd.n_rays + 255) / 256; }

hipError_t launch_dtpl(const ScanDesc &sd, const float *f, const float *c, float *p_scratch, void *pack,
                       double *partial, double *out, hipStream_t st) {
  hipError_t e = launch_forward(sd, f, 3, p_scratch, pack, st);
  if (e != hipSuccess) return e;
  if (sd.per_bin)
    hipLaunchKernelGGL(k_dtpl_partial<true>, ray_grid(sd), dim3(256), 0, st, sd, p_scratch, c, partial);
  else
    hipLaunchKernelGGL(k_dtpl_partial<false>, ray_grid(sd), dim3(256), 0, st, sd, p_scratch, c, partial);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partial, dtpl_partial_count(sd), out);
  return hipGetLastError();
}

}  // namespace osscir
