// Per-ray spectral model, step lengths and dual step, the fused primal
// update, and the D_TPL reduction (Sec. II of arXiv 1801.06263) for gfx950.
//
// One thread per ray.  The energy loop reads the spectral table at a uniform
// address (scalar loads, SGPR operands) and accumulates, per window, the
// model sum g_w, the Jacobian rows a_w = sum_i s_{w,i} softexp'(-z_i) mu_i and,
// for the clipped curvature, Hb_w = sum_i s_{w,i} softexp''(-z_i) mu_i mu_i^T.
// The per-ray tail (3x3 eigen-clip, 4x4 dual solve) runs in FP32 or FP64.
#include "device_math.h"
#include "kernels.h"
#include "projector.h"
#include "project_device.h"
#include "spectral.h"

namespace osscir {

// upper-triangle index of (m, n), m <= n, in a symmetric 3x3
__device__ __forceinline__ constexpr int ut(int m, int n) { return m == 0 ? n : (m == 1 ? 2 + n : 5); }

// SHIFT: the sums are taken with exp(-(z - zshift)) in place of exp(-z), for
// a ray whose every z_i >= zshift > 0 (all energies on the exponential
// branch).  The ratios a_w / g_w and Hb_w / g_w are unchanged; g_w carries
// the factor exp(zshift).
template <bool NEED_A, bool NEED_HB, bool SHIFT = false>
__device__ __forceinline__ void energy_sums(const ScanDesc &sd, float p0, float p1, float p2, float g[kWin],
                                            float a[kWin * kMat], float hb[kWin * 6], float zshift = 0.0f) {
#pragma unroll
  for (int w = 0; w < kWin; ++w) g[w] = 0.0f;
  if (NEED_A) {
#pragma unroll
    for (int j = 0; j < kWin * kMat; ++j) a[j] = 0.0f;
  }
  if (NEED_HB) {
#pragma unroll
    for (int j = 0; j < kWin * 6; ++j) hb[j] = 0.0f;
  }
  const float *__restrict__ tab = sd.tab;
  for (int i = 0; i < sd.n_energy; ++i) {
    const float *t = tab + i * kTab;
    float E, E1, E2;
    if (SHIFT) {
      const float zs = __fmaf_rn(t[kTabMu + 2], p2, __fmaf_rn(t[kTabMu + 1], p1, __fmaf_rn(t[kTabMu], p0, -zshift)));
      E = E1 = E2 = __expf(-zs);
    } else {
      const float z = __fmaf_rn(t[kTabMu + 2], p2, __fmaf_rn(t[kTabMu + 1], p1, t[kTabMu] * p0));
      softexp3(z, E, E1, E2);
    }
#pragma unroll
    for (int w = 0; w < kWin; ++w) g[w] = __fmaf_rn(t[kTabS + w], E, g[w]);
    if (NEED_A) {
#pragma unroll
      for (int j = 0; j < kWin * kMat; ++j) a[j] = __fmaf_rn(t[kTabSMu + j], E1, a[j]);
    }
    if (NEED_HB) {
#pragma unroll
      for (int j = 0; j < kWin * 6; ++j) hb[j] = __fmaf_rn(t[kTabSMuMu + j], E2, hb[j]);
    }
  }
}

// Model sums of one ray with a rescue for transmissions below FP32 range:
// if a window sum underflows (an iterate far outside the physical range),
// the sums are recomputed with the exponent shifted by min_i z_i.  Returns
// the factor (<= 1) that turns the returned g_w into the true sums.
template <bool NEED_A, bool NEED_HB>
__device__ __forceinline__ float energy_sums_safe(const ScanDesc &sd, float p0, float p1, float p2, float g[kWin],
                                                  float a[kWin * kMat], float hb[kWin * 6]) {
  energy_sums<NEED_A, NEED_HB>(sd, p0, p1, p2, g, a, hb);
  const float gmin = fminf(fminf(g[0], g[1]), fminf(g[2], g[3]));
  if (gmin >= 1e-30f) return 1.0f;
  float zmin = 3.0e38f;
  for (int i = 0; i < sd.n_energy; ++i) {
    const float *t = sd.tab + i * kTab;
    zmin = fminf(zmin, __fmaf_rn(t[kTabMu + 2], p2, __fmaf_rn(t[kTabMu + 1], p1, t[kTabMu] * p0)));
  }
  if (!(zmin > 0.0f)) return 1.0f;  // some energy on the linear branch: no underflow possible
  energy_sums<NEED_A, NEED_HB, true>(sd, p0, p1, p2, g, a, hb, zmin);
  return __expf(-zmin);
}

// Per-ray p-space Hessian  H = sum_w c_w a_w a_w^T - sum_w (r_w / g_w) Hb_w
// (the ray-l block of -Z^T diag(B^T r) Z + Z^T A^T diag(chat + r) A Z, using
// chat + r = c), with a_w already divided by g_w.
template <typename T>
__device__ __forceinline__ void ray_hessian(const T a[kWin][kMat], const T cw[kWin], const T rg[kWin],
                                            const float hb[kWin * 6], T H[6]) {
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = m; n < 3; ++n) {
      T h = T(0);
#pragma unroll
      for (int w = 0; w < kWin; ++w) h += cw[w] * a[w][m] * a[w][n] - rg[w] * (T)hb[w * 6 + ut(m, n)];
      H[ut(m, n)] = h;
    }
}

// ---------------------------------------------------------------- model out

template <typename T>
__global__ void __launch_bounds__(256) k_spectral_model(ScanDesc sd, const float *__restrict__ p,
                                                         const float *__restrict__ c, float *__restrict__ chat,
                                                         float *__restrict__ r, float *__restrict__ G,
                                                         float *__restrict__ H, float *__restrict__ Hp) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int L = sd.n_rays;
  if (l >= L) return;
  float g[kWin], af[kWin * kMat], hb[kWin * 6];
  const float scale = energy_sums_safe<true, true>(sd, p[l], p[L + l], p[2 * L + l], g, af, hb);
  T a[kWin][kMat], cw[kWin], rg[kWin];
#pragma unroll
  for (int w = 0; w < kWin; ++w) {
    const float ch = sd.n0[w] * g[w] * scale;
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
//
// y <- y + Sigma (Sigma + D)^-1 (r - y),  q = G^T y,  and the per-ray
// preconditioner terms S (block) or h (diag) for the back-projection.
// CLIP: D = G^+T H^+ G^+ built from the column-equilibrated G and solved as
// (I + Sigma^-1/2 D Sigma^-1/2) z = Sigma^-1/2 (r - y).
template <typename T, bool CLIP, bool BLOCK>
__global__ void __launch_bounds__(256) k_spectral_dual(ScanDesc sd, const float *__restrict__ p,
                                                        const float *__restrict__ c, float *__restrict__ y,
                                                        float *__restrict__ qS, float lambda) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int L = sd.n_rays;
  if (l >= L) return;
  const float rho = sd.rho[l];
  if (!(rho > 0.0f)) {
#pragma unroll
    for (int w = 0; w < kWin; ++w) y[w * L + l] = 0.0f;
#pragma unroll
    for (int j = 0; j < 9; ++j) qS[j * L + l] = 0.0f;
    return;
  }
  float g[kWin], af[kWin * kMat], hb[kWin * 6];
  const float scale = energy_sums_safe<true, CLIP>(sd, p[l], p[L + l], p[2 * L + l], g, af, hb);

  T a[kWin][kMat], cw[kWin], rw[kWin], yw[kWin], sig[kWin];
#pragma unroll
  for (int w = 0; w < kWin; ++w) {
    const float cf = c[w * L + l];
    cw[w] = (T)cf;
    rw[w] = (T)(cf - sd.n0[w] * g[w] * scale);
    yw[w] = (T)y[w * L + l];
    const T ig = T(1) / (T)g[w];
#pragma unroll
    for (int m = 0; m < kMat; ++m) a[w][m] = (T)af[w * kMat + m] * ig;
  }
  // step lengths and the per-ray preconditioner terms
  T extra[6];
  const T lr = (T)lambda * (T)rho;
  if (BLOCK) {
#pragma unroll
    for (int j = 0; j < 6; ++j) extra[j] = T(0);
#pragma unroll
    for (int w = 0; w < kWin; ++w) {
      const T nrm = sqrt(a[w][0] * a[w][0] + a[w][1] * a[w][1] + a[w][2] * a[w][2]);
      sig[w] = T(1) / (lr * nrm);
      const T inv = T(1) / nrm;
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int n = m; n < 3; ++n) extra[ut(m, n)] += a[w][m] * a[w][n] * inv;
    }
  } else {
#pragma unroll
    for (int m = 0; m < 3; ++m) extra[m] = T(0);
#pragma unroll
    for (int w = 0; w < kWin; ++w) {
      const T l1 = fabs(a[w][0]) + fabs(a[w][1]) + fabs(a[w][2]);
      sig[w] = T(1) / (lr * l1);
#pragma unroll
      for (int m = 0; m < 3; ++m) extra[m] += fabs(a[w][m]);
    }
  }
  // dual step
  if (!CLIP) {
#pragma unroll
    for (int w = 0; w < kWin; ++w) yw[w] = (cw[w] * yw[w] + sig[w] * rw[w]) / (cw[w] + sig[w]);
  } else {
    T rg[kWin];
#pragma unroll
    for (int w = 0; w < kWin; ++w) rg[w] = rw[w] / (T)g[w];
    T h[6], hp[6];
    ray_hessian<T>(a, cw, rg, hb, h);
    clip_negative_curvature<T, sizeof(T) == 8 ? 8 : 6>(h, hp);
    // column equilibration of G
    T cn[3], gt[kWin][kMat];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      cn[m] = sqrt(a[0][m] * a[0][m] + a[1][m] * a[1][m] + a[2][m] * a[2][m] + a[3][m] * a[3][m]);
      const T ic = T(1) / cn[m];
#pragma unroll
      for (int w = 0; w < kWin; ++w) gt[w][m] = a[w][m] * ic;
    }
    T gram[6];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int n = m; n < 3; ++n) {
        T s = T(0);
#pragma unroll
        for (int w = 0; w < kWin; ++w) s += gt[w][m] * gt[w][n];
        gram[ut(m, n)] = s;
      }
    T gi[3][3];
    spd3_inverse<T>(gram, gi);
    // P~ = Sigma^-1/2 G~ Gram^-1   (rows w)
    T ss[kWin], P[kWin][3];
#pragma unroll
    for (int w = 0; w < kWin; ++w) {
      ss[w] = sqrt(sig[w]);
      const T is = T(1) / ss[w];
#pragma unroll
      for (int n = 0; n < 3; ++n) P[w][n] = (gt[w][0] * gi[0][n] + gt[w][1] * gi[1][n] + gt[w][2] * gi[2][n]) * is;
    }
    // H^ = C^-1 H^+ C^-1
    T Hh[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int n = 0; n < 3; ++n) Hh[m][n] = hp[m <= n ? ut(m, n) : ut(n, m)] / (cn[m] * cn[n]);
    // M = P~ H^ P~^T
    T PH[kWin][3], Mm[kWin][kWin];
#pragma unroll
    for (int w = 0; w < kWin; ++w)
#pragma unroll
      for (int n = 0; n < 3; ++n) PH[w][n] = P[w][0] * Hh[0][n] + P[w][1] * Hh[1][n] + P[w][2] * Hh[2][n];
#pragma unroll
    for (int w = 0; w < kWin; ++w)
#pragma unroll
      for (int v = 0; v < kWin; ++v) Mm[w][v] = PH[w][0] * P[v][0] + PH[w][1] * P[v][1] + PH[w][2] * P[v][2];
    T bt[kWin], z[kWin];
#pragma unroll
    for (int w = 0; w < kWin; ++w) bt[w] = (rw[w] - yw[w]) / ss[w];
    unit_plus_psd4_solve<T>(Mm, bt, z);
#pragma unroll
    for (int w = 0; w < kWin; ++w) yw[w] = yw[w] + ss[w] * z[w];
  }
  // outputs: y, q = G^T y, and S (block) or h (diag)
#pragma unroll
  for (int w = 0; w < kWin; ++w) y[w * L + l] = (float)yw[w];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const T qm = a[0][m] * yw[0] + a[1][m] * yw[1] + a[2][m] * yw[2] + a[3][m] * yw[3];
    qS[m * L + l] = (float)qm;
  }
  if (BLOCK) {
#pragma unroll
    for (int j = 0; j < 6; ++j) qS[(3 + j) * L + l] = (float)extra[j];
  } else {
#pragma unroll
    for (int j = 0; j < 3; ++j) qS[(3 + j) * L + l] = (float)extra[j];
  }
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
//
// Back-projection of [q; S] (or [q; h]) fused with the primal step and the
// extrapolation:  block  f' = f - lambda (sum_l X S_l)^-1 (sum_l X q_l)
//                 diag   f'_m = f_m - lambda (sum_l X q_l)_m / (sum_l X h_l)_m
//                 fbar'  = 2 f' - f.
// The 3x3 solve takes the FP64 sums directly (equilibrated Cholesky).
template <bool BLOCK, bool WIDE>
__global__ void __launch_bounds__(256) k_back_primal(ScanDesc sd, const float *__restrict__ qS,
                                                      float *__restrict__ f, float *__restrict__ fbar, float lambda) {
  __shared__ BpShared sh;
  constexpr int NCH = BLOCK ? 9 : 6;
  double acc[NCH];
  back_accumulate<NCH, WIDE>(sd, blockIdx.x, blockIdx.y, qS, sd.n_rays, acc, sh);
  const int ix = blockIdx.x * kBpTile + (threadIdx.x & (kBpTile - 1));
  const int iy = blockIdx.y * kBpTile + (threadIdx.x / kBpTile);
  if (ix >= sd.n || iy >= sd.n) return;
  const int nn = sd.n * sd.n;
  const int k = iy * sd.n + ix;
  float fo[3], fn[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) fo[m] = f[m * nn + k];
  const double lam = (double)lambda;
  if (BLOCK) {
    double x[3] = {0.0, 0.0, 0.0};
    if (acc[3] > 0.0 && acc[6] > 0.0 && acc[8] > 0.0) spd3_solve<double>(acc + 3, acc, x);
#pragma unroll
    for (int m = 0; m < 3; ++m) fn[m] = (float)((double)fo[m] - lam * x[m]);
  } else {
#pragma unroll
    for (int m = 0; m < 3; ++m) fn[m] = acc[3 + m] > 0.0 ? (float)((double)fo[m] - lam * acc[m] / acc[3 + m]) : fo[m];
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    f[m * nn + k] = fn[m];
    fbar[m * nn + k] = 2.0f * fn[m] - fo[m];
  }
}

// ---------------------------------------------------------------- D_TPL

__global__ void __launch_bounds__(256) k_dtpl_partial(ScanDesc sd, const float *__restrict__ p,
                                                       const float *__restrict__ c, double *__restrict__ partial) {
  __shared__ double red[256];
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int L = sd.n_rays;
  double term = 0.0;
  if (l < L) {
    float g[kWin];
    energy_sums<false, false>(sd, p[l], p[L + l], p[2 * L + l], g, nullptr, nullptr);
#pragma unroll
    for (int w = 0; w < kWin; ++w) {
      const double ch = (double)sd.n0[w] * (double)g[w];
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

// ---------------------------------------------------------------- launchers

static inline dim3 ray_grid(const ScanDesc &sd) { return dim3((sd.n_rays + 255) / 256); }
static inline dim3 pix_grid(const ScanDesc &sd) {
  return dim3((sd.n + kBpTile - 1) / kBpTile, (sd.n + kBpTile - 1) / kBpTile);
}

hipError_t launch_spectral_model(const ScanDesc &sd, const float *p, const float *c, float *chat, float *r,
                                 float *G, float *H, float *Hp, bool fp64, hipStream_t st) {
  if (fp64)
    hipLaunchKernelGGL(k_spectral_model<double>, ray_grid(sd), dim3(256), 0, st, sd, p, c, chat, r, G, H, Hp);
  else
    hipLaunchKernelGGL(k_spectral_model<float>, ray_grid(sd), dim3(256), 0, st, sd, p, c, chat, r, G, H, Hp);
  return hipGetLastError();
}

hipError_t launch_spectral_dual(const ScanDesc &sd, const float *p, const float *c, float *y, float *qS,
                                float lambda, bool clip, bool block, bool fp64, hipStream_t st) {
#define OSSCIR_DUAL(T, C, B) \
  hipLaunchKernelGGL((k_spectral_dual<T, C, B>), ray_grid(sd), dim3(256), 0, st, sd, p, c, y, qS, lambda)
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
  return hipGetLastError();
}

hipError_t launch_back_primal(const ScanDesc &sd, const float *qS, float *f, float *fbar, float lambda, bool block,
                              bool fp64, hipStream_t st) {
  (void)fp64;
#define OSSCIR_BP(B, W) hipLaunchKernelGGL((k_back_primal<B, W>), pix_grid(sd), dim3(256), 0, st, sd, qS, f, fbar, lambda)
  if (block) {
    if (sd.bp_wide) OSSCIR_BP(true, true); else OSSCIR_BP(true, false);
  } else {
    if (sd.bp_wide) OSSCIR_BP(false, true); else OSSCIR_BP(false, false);
  }
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

int dtpl_partial_count(const ScanDesc &sd) { return (sd.n_rays + 255) / 256; }

hipError_t launch_dtpl(const ScanDesc &sd, const float *f, const float *c, float *p_scratch, void *pack,
                       double *partial, double *out, hipStream_t st) {
  hipError_t e = launch_forward(sd, f, 3, p_scratch, pack, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dtpl_partial, ray_grid(sd), dim3(256), 0, st, sd, p_scratch, c, partial);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partial, dtpl_partial_count(sd), out);
  return hipGetLastError();
}

}  // namespace osscir
