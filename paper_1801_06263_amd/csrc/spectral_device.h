// Per-ray spectral model and dual step, and the per-tile back-projection
// fused with the primal step (Sec. II and III of arXiv 1801.06263), shared by
// the single-scan kernels (spectral.hip) and the batched kernels
// (batch.hip).
//
// One thread per ray.  The energy loop reads the spectral table at a uniform
// address (scalar loads, SGPR operands) and accumulates, per window, the
// model sum g_w, the Jacobian rows a_w = sum_i s_{w,i} softexp'(-z_i) mu_i and,
// for the clipped curvature, Hb_w = sum_i s_{w,i} softexp''(-z_i) mu_i mu_i^T.
// The per-ray tail (3x3 eigen-clip, 4x4 dual solve) runs in FP32 or FP64.
#pragma once

#include "device_math.h"
#include "kernels.h"
#include "project_device.h"

namespace osscir {

// upper-triangle index of (m, n), m <= n, in a symmetric 3x3
__device__ __forceinline__ constexpr int ut(int m, int n) { return m == 0 ? n : (m == 1 ? 2 + n : 5); }

// SHIFT: the sums are taken with exp(-(z - zshift)) in place of exp(-z), for
// a ray whose every z_i >= zshift > 0 (all energies on the exponential
// branch).  The ratios a_w / g_w and Hb_w / g_w are unchanged; g_w carries
// the factor exp(zshift).
// PB: the window responses are those of detector bin d (one float4 per
// energy), the products with mu formed here instead of read from the table.
template <bool NEED_A, bool NEED_HB, bool SHIFT = false, bool PB = false>
__device__ __forceinline__ void energy_sums(const ScanDesc &sd, float p0, float p1, float p2, float g[kWin],
                                            float a[kWin * kMat], float hb[kWin * 6], float zshift = 0.0f,
                                            int d = 0) {
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
  const OSSCIR_CONST float *tab = as_const(sd.tab);
  const float4 *__restrict__ sb = PB ? sd.sbin + d : nullptr;
  for (int i = 0; i < sd.n_energy; ++i) {
    const OSSCIR_CONST float *t = tab + i * kTab;
    float E, E1, E2;
    if (SHIFT) {
      const float zs = __fmaf_rn(t[kTabMu + 2], p2, __fmaf_rn(t[kTabMu + 1], p1, __fmaf_rn(t[kTabMu], p0, -zshift)));
      E = E1 = E2 = __expf(-zs);
    } else {
      const float z = __fmaf_rn(t[kTabMu + 2], p2, __fmaf_rn(t[kTabMu + 1], p1, t[kTabMu] * p0));
      softexp3(z, E, E1, E2);
    }
    if (PB) {
      const float4 s4 = sb[(size_t)i * sd.n_bins];
      const float sw[kWin] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
      for (int w = 0; w < kWin; ++w) g[w] = __fmaf_rn(sw[w], E, g[w]);
      if (NEED_A) {
#pragma unroll
        for (int w = 0; w < kWin; ++w) {
          const float e1 = sw[w] * E1;
#pragma unroll
          for (int m = 0; m < kMat; ++m) a[w * kMat + m] = __fmaf_rn(e1, t[kTabMu + m], a[w * kMat + m]);
        }
      }
      if (NEED_HB) {
#pragma unroll
        for (int w = 0; w < kWin; ++w) {
          const float e2 = sw[w] * E2;
#pragma unroll
          for (int j = 0; j < 6; ++j) hb[w * 6 + j] = __fmaf_rn(e2, t[kTabMuMu + j], hb[w * 6 + j]);
        }
      }
    } else {
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
}

// Model sums of one ray with a rescue for transmissions below FP32 range:
// if a window sum underflows (an iterate far outside the physical range),
// the sums are recomputed with the exponent shifted by min_i z_i.  Returns
// the factor (<= 1) that turns the returned g_w into the true sums.
template <bool NEED_A, bool NEED_HB, bool PB = false>
__device__ __forceinline__ float energy_sums_rescue(const ScanDesc &sd, float p0, float p1, float p2, float g[kWin],
                                                    float a[kWin * kMat], float hb[kWin * 6], int d = 0) {
  const float gmin = fminf(fminf(g[0], g[1]), fminf(g[2], g[3]));
  if (gmin >= 1e-30f) return 1.0f;
  float zmin = 3.0e38f;
  for (int i = 0; i < sd.n_energy; ++i) {
    const OSSCIR_CONST float *t = as_const(sd.tab) + i * kTab;
    zmin = fminf(zmin, __fmaf_rn(t[kTabMu + 2], p2, __fmaf_rn(t[kTabMu + 1], p1, t[kTabMu] * p0)));
  }
  if (!(zmin > 0.0f)) return 1.0f;  // some energy on the linear branch: no underflow possible
  energy_sums<NEED_A, NEED_HB, true, PB>(sd, p0, p1, p2, g, a, hb, zmin, d);
  return __expf(-zmin);
}

template <bool NEED_A, bool NEED_HB, bool PB = false>
__device__ __forceinline__ float energy_sums_safe(const ScanDesc &sd, float p0, float p1, float p2, float g[kWin],
                                                  float a[kWin * kMat], float hb[kWin * 6], int d = 0) {
  energy_sums<NEED_A, NEED_HB, false, PB>(sd, p0, p1, p2, g, a, hb, 0.0f, d);
  return energy_sums_rescue<NEED_A, NEED_HB, PB>(sd, p0, p1, p2, g, a, hb, d);
}

// ---------------------------------------------------------------- MFMA form
//
// With one response table shared by all rays, the energy sums of 64 rays
// are a dense contraction: C[col][ray] = sum_i tab[i][col] B_col[i][ray]
// over the table columns s_w (4), s_w mu_m (12) and s_w mu_m mu_n (24), with
// B = softexp(-z) for the model sums, softexp'(-z) for the Jacobian rows and
// softexp''(-z) for the curvature sums.  A wave runs it on the matrix cores
// (v_mfma_f32_16x16x4f32: 16 table columns x 4 energies x 16 rays per
// instruction, FP32 products and sums) while its VALU forms z and the
// exponentials; the three column blocks are table columns 3..18 (s, s mu),
// 19..34 and 32..47 (s mu mu).  softexp' = softexp unless z < 0: only then
// (a wave-uniform test per 4 energies) the Jacobian rows get the correction
// tab x (softexp' - softexp).  The results are moved to one ray per lane
// through LDS.  Requires the whole wave (64 consecutive rays).
typedef float floatx4_t __attribute__((ext_vector_type(4)));


// All threads of the workgroup: the table into LDS in 16-byte pieces (a
// row is 48 floats), zero rows up to mfma_energies().
__device__ __forceinline__ void stage_table(const ScanDesc &sd, float *stab) {
  const int n = mfma_energies(sd.n_energy) * (kTab / 4), m = sd.n_energy * (kTab / 4);
  const float4 *__restrict__ tab = reinterpret_cast<const float4 *>(sd.tab);
  float4 *s4 = reinterpret_cast<float4 *>(stab);
#pragma unroll 4
  for (int i = threadIdx.x; i < n; i += blockDim.x) s4[i] = i < m ? tab[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Operands of one 4-energy step of energy_sums_mfma: t = the table row of
// this lane's energy (e0 + lane / 16); B operands softexp, softexp' -
// softexp and softexp'' of z for the rays of the four column blocks.
struct MfmaStep {
  float tGA, tH1, tH2;
  float E[4], D1[4], E2[4];
  bool phys;
};

template <bool NEED_HB>
__device__ __forceinline__ void mfma_operands(const float *t, int rn, const float (&pn)[4][3], MfmaStep &o) {
  const float mu0 = t[kTabMu], mu1 = t[kTabMu + 1], mu2 = t[kTabMu + 2];
  o.tGA = t[kTabS + rn];
  if (NEED_HB) {
    o.tH1 = t[kTabSMuMu + rn];
    o.tH2 = t[kTabSMuMu + 13 + rn];
  }
  o.phys = true;
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const float z = __fmaf_rn(mu2, pn[nb][2], __fmaf_rn(mu1, pn[nb][1], mu0 * pn[nb][0]));
    float e, e1, e2;
    softexp3(z, e, e1, e2);
    o.E[nb] = e;
    o.D1[nb] = e1 - e;
    o.E2[nb] = e2;
    o.phys = o.phys && z >= 0.0f;
  }
}

template <bool NEED_HB>
__device__ __forceinline__ void mfma_apply(const MfmaStep &o, floatx4_t (&cGA)[4], floatx4_t (&cH1)[4],
                                           floatx4_t (&cH2)[4]) {
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) cGA[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.tGA, o.E[nb], cGA[nb], 0, 0, 0);
  if (NEED_HB) {
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      cH1[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.tH1, o.E2[nb], cH1[nb], 0, 0, 0);
      cH2[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.tH2, o.E2[nb], cH2[nb], 0, 0, 0);
    }
  }
}

// Every thread of the workgroup calls this (it has barriers); stab holds the
// staged table and is reused for the transposition.
template <bool NEED_HB>
__device__ __forceinline__ void energy_sums_mfma(const ScanDesc &sd, float *stab, float p0, float p1, float p2,
                                                 float g[kWin], float a[kWin * kMat], float hb[kWin * 6]) {
  const int lane = threadIdx.x & 63, rn = lane & 15, kg = lane >> 4;
  float pn[4][3];  // the rays of the four 16-ray column blocks this lane feeds
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int src = nb * 16 + rn;
    pn[nb][0] = __shfl(p0, src, 64);
    pn[nb][1] = __shfl(p1, src, 64);
    pn[nb][2] = __shfl(p2, src, 64);
  }
  const floatx4_t zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
  floatx4_t cGA[4], cCo[4], cH1[4], cH2[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) cGA[nb] = cCo[nb] = cH1[nb] = cH2[nb] = zero4;
  const int ne = mfma_energies(sd.n_energy);
  for (int e0 = 0; e0 < ne; e0 += 8) {  // two independent 4-energy steps per iteration
    MfmaStep s0, s1;
    mfma_operands<NEED_HB>(stab + (e0 + kg) * kTab, rn, pn, s0);
    mfma_operands<NEED_HB>(stab + (e0 + 4 + kg) * kTab, rn, pn, s1);
    mfma_apply<NEED_HB>(s0, cGA, cH1, cH2);
    mfma_apply<NEED_HB>(s1, cGA, cH1, cH2);
    if (!__all(s0.phys && s1.phys)) {
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        cCo[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(s0.tGA, s0.D1[nb], cCo[nb], 0, 0, 0);
        cCo[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(s1.tGA, s1.D1[nb], cCo[nb], 0, 0, 0);
      }
    }
  }
  // lane holds C[4 kg + r][ray nb * 16 + rn]; move one ray's columns to its lane
  __syncthreads();  // every wave is done with the staged table
  float *w = stab + (threadIdx.x >> 6) * kMfmaTileFloats;
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * kg + r;
      w[(nb * 16 + rn) * 17 + i] = cGA[nb][r] + (i >= kWin ? cCo[nb][r] : 0.0f);
    }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kWin; ++c) g[c] = w[lane * 17 + c];
#pragma unroll
  for (int c = 0; c < kWin * kMat; ++c) a[c] = w[lane * 17 + kWin + c];
  if (NEED_HB) {
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) w[(nb * 16 + rn) * 17 + 4 * kg + r] = cH1[nb][r];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) hb[c] = w[lane * 17 + c];
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * kg + r;  // column 32 + i; the curvature sums 16..23 are columns 35..42
        if (i >= 3 && i < 11) w[(nb * 16 + rn) * 17 + i - 3] = cH2[nb][r];
      }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 8; ++c) hb[16 + c] = w[lane * 17 + c];
  }
}

// Incident counts of window w on ray l (detector bin d): the plan's per-ray
// table if it has one, else per detector bin (PB) or shared.
template <bool PB>
__device__ __forceinline__ void ray_n0(const ScanDesc &sd, int l, int d, float n0[kWin]) {
  if (sd.n0ray) {  // uniform
    const float4 v = sd.n0ray[l];
    n0[0] = v.x;
    n0[1] = v.y;
    n0[2] = v.z;
    n0[3] = v.w;
  } else if (PB) {
    const float4 v = sd.n0bin[d];
    n0[0] = v.x;
    n0[1] = v.y;
    n0[2] = v.z;
    n0[3] = v.w;
  } else {
#pragma unroll
    for (int w = 0; w < kWin; ++w) n0[w] = sd.n0[w];
  }
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

// ---------------------------------------------------------------- dual step
//
// y <- y + Sigma (Sigma + D)^-1 (r - y),  q = G^T y,  and the per-ray
// preconditioner terms S (block) or h (diag) for the back-projection.
// CLIP: D = G^+T H^+ G^+ built from the column-equilibrated G and solved as
// (I + Sigma^-1/2 D Sigma^-1/2) z = Sigma^-1/2 (r - y).
// MFMA: the energy sums on the matrix cores (energy_sums_mfma; stab = the
// table staged in LDS); every thread of the workgroup must call it.
// NEST (inner iterations of nested loops): p holds the line integrals of the
// expansion point f0, where the model (G, r, D) and the steps are formed,
// and pbar those of fbar_n (pbar NULL: the step at the expansion point, the
// same arithmetic as NEST = false).  The dual step at v = y + Sigma G pbar with
// u0 = G p is the step above with r replaced by r + D G (pbar - p); with
// D = G^+T H^+ G^+ (G of full column rank) D G = G (G^T G)^-1 H^+.
template <typename T, bool CLIP, bool BLOCK, bool PB = false, bool MFMA = false, bool NEST = false>
__device__ __forceinline__ void spectral_dual_ray(const ScanDesc &sd, const float *__restrict__ p,
                                                  const float *__restrict__ c, float *__restrict__ y,
                                                  float *__restrict__ qS, float lambda, int l, float *stab = nullptr,
                                                  const float *__restrict__ pbar = nullptr) {
  static_assert(!(MFMA && PB), "the MFMA sums need one shared response table");
  const int L = sd.n_rays;
  float g[kWin], af[kWin * kMat], hb[kWin * 6], n0[kWin];
  if (MFMA) {
    const bool in = l < L;
    energy_sums_mfma<CLIP>(sd, stab, in ? p[l] : 0.0f, in ? p[L + l] : 0.0f, in ? p[2 * L + l] : 0.0f, g, af, hb);
  }
  if (l >= L) return;
  const float rho = sd.rho[l];
  float4 *__restrict__ qs4 = reinterpret_cast<float4 *>(qS) + 3 * (size_t)l;
  if (!(rho > 0.0f)) {
#pragma unroll
    for (int w = 0; w < kWin; ++w) y[w * L + l] = 0.0f;
    const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    qs4[0] = z4;
    qs4[1] = z4;
    qs4[2] = z4;
    return;
  }
  const int d = l % sd.n_bins;
  const float scale = MFMA ? energy_sums_rescue<true, CLIP, PB>(sd, p[l], p[L + l], p[2 * L + l], g, af, hb, d)
                           : energy_sums_safe<true, CLIP, PB>(sd, p[l], p[L + l], p[2 * L + l], g, af, hb, d);
  ray_n0<PB>(sd, l, d, n0);

  T a[kWin][kMat], cw[kWin], rw[kWin], yw[kWin], sig[kWin], ig[kWin];
#pragma unroll
  for (int w = 0; w < kWin; ++w) {
    const float cf = c[w * L + l];
    cw[w] = (T)cf;
    rw[w] = (T)(cf - n0[w] * g[w] * scale);
    yw[w] = (T)y[w * L + l];
    ig[w] = T(1) / (T)g[w];
#pragma unroll
    for (int m = 0; m < kMat; ++m) a[w][m] = (T)af[w * kMat + m] * ig[w];
  }
  // step lengths and the per-ray preconditioner terms
  T extra[6];
  const T lr = (T)lambda * (T)rho;
  if (BLOCK) {
    const T ilr = T(1) / lr;
#pragma unroll
    for (int j = 0; j < 6; ++j) extra[j] = T(0);
#pragma unroll
    for (int w = 0; w < kWin; ++w) {
      const T nrm = sqrt(a[w][0] * a[w][0] + a[w][1] * a[w][1] + a[w][2] * a[w][2]);
      const T inv = T(1) / nrm;
      sig[w] = ilr * inv;
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
  T dp[kMat];  // pbar - p (NEST)
  const bool shift = NEST && pbar != nullptr;  // uniform
  if (shift) {
#pragma unroll
    for (int m = 0; m < kMat; ++m) dp[m] = (T)pbar[m * L + l] - (T)p[m * L + l];
  }
  // dual step
  if (!CLIP) {
    if (shift) {
#pragma unroll
      for (int w = 0; w < kWin; ++w) rw[w] += cw[w] * (a[w][0] * dp[0] + a[w][1] * dp[1] + a[w][2] * dp[2]);
    }
#pragma unroll
    for (int w = 0; w < kWin; ++w) yw[w] = (cw[w] * yw[w] + sig[w] * rw[w]) / (cw[w] + sig[w]);
  } else {
    T rg[kWin];
#pragma unroll
    for (int w = 0; w < kWin; ++w) rg[w] = rw[w] * ig[w];
    T h[6], hp[6];
    ray_hessian<T>(a, cw, rg, hb, h);
    clip_negative_curvature<T, sizeof(T) == 8 ? 8 : 6>(h, hp);
    // column equilibration of G
    T ic[3], gt[kWin][kMat];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      ic[m] = T(1) / sqrt(a[0][m] * a[0][m] + a[1][m] * a[1][m] + a[2][m] * a[2][m] + a[3][m] * a[3][m]);
#pragma unroll
      for (int w = 0; w < kWin; ++w) gt[w][m] = a[w][m] * ic[m];
    }
    // The Gram matrix of the equilibrated G and its inverse in FP64 whatever
    // T: the materials' columns of G are close to parallel, and with this
    // inverse in FP32 the maps of the 64^2 edge-ray scan drifted to 1.6e-3 of
    // the oracle after 100 iterations (1e-5 with it in FP64, no slower).
    double gram[6];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int n = m; n < 3; ++n) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kWin; ++w) s += (double)gt[w][m] * (double)gt[w][n];
        gram[ut(m, n)] = s;
      }
    double gid[3][3];
    spd3_inverse<double>(gram, gid);
    T gi[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int n = 0; n < 3; ++n) gi[m][n] = (T)gid[m][n];
    // P~ = Sigma^-1/2 G~ Gram^-1   (rows w)
    T ss[kWin], is[kWin], P[kWin][3];
#pragma unroll
    for (int w = 0; w < kWin; ++w) {
      ss[w] = sqrt(sig[w]);
      is[w] = T(1) / ss[w];
#pragma unroll
      for (int n = 0; n < 3; ++n) P[w][n] = (gt[w][0] * gi[0][n] + gt[w][1] * gi[1][n] + gt[w][2] * gi[2][n]) * is[w];
    }
    // H^ = C^-1 H^+ C^-1
    T Hh[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int n = 0; n < 3; ++n) Hh[m][n] = hp[m <= n ? ut(m, n) : ut(n, m)] * (ic[m] * ic[n]);
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
    if (shift) {
      // G (G^T G)^-1 = (P~ rows scaled back by Sigma^1/2, columns by C^-1)
      T v[3];  // C^-1 H^+ dp
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        T hd = T(0);
#pragma unroll
        for (int m = 0; m < 3; ++m) hd += hp[n <= m ? ut(n, m) : ut(m, n)] * dp[m];
        v[n] = hd * ic[n];
      }
#pragma unroll
      for (int w = 0; w < kWin; ++w) rw[w] += ss[w] * (P[w][0] * v[0] + P[w][1] * v[1] + P[w][2] * v[2]);
    }
    T bt[kWin], z[kWin];
#pragma unroll
    for (int w = 0; w < kWin; ++w) bt[w] = (rw[w] - yw[w]) * is[w];
    unit_plus_psd4_solve<T>(Mm, bt, z);
#pragma unroll
    for (int w = 0; w < kWin; ++w) yw[w] = yw[w] + ss[w] * z[w];
  }
  // outputs: y, q = G^T y, and S (block) or h (diag), the latter two
  // interleaved per ray as 12 floats (q0..2, S0..5 or h0..2 and zeros up to
  // q8, then the ray's kappa a, hmax and a zero)
#pragma unroll
  for (int w = 0; w < kWin; ++w) y[w * L + l] = (float)yw[w];
  float o[12];
#pragma unroll
  for (int m = 0; m < 3; ++m)
    o[m] = (float)(a[0][m] * yw[0] + a[1][m] * yw[1] + a[2][m] * yw[2] + a[3][m] * yw[3]);
#pragma unroll
  for (int j = 0; j < 9; ++j) o[3 + j] = (BLOCK ? j < 6 : j < 3) ? (float)extra[j < 6 ? j : 0] : 0.0f;
  // the last piece also carries the ray's kappa a and hmax, so that the
  // back-projector stages a bin as four 16-byte copies
  const float4 rk = reinterpret_cast<const float4 *>(sd.rays + l)[1];  // kappa a, hmax, kappa, pad
  qs4[0] = make_float4(o[0], o[1], o[2], o[3]);
  qs4[1] = make_float4(o[4], o[5], o[6], o[7]);
  qs4[2] = make_float4(o[8], rk.x, rk.y, 0.0f);
}

// ---------------------------------------------------------------- primal
//
// Back-projection of [q; S] (or [q; h]) fused with the primal step and the
// extrapolation:  block  f' = f - lambda (sum_l X S_l)^-1 (sum_l X q_l)
//                 diag   f'_m = f_m - lambda (sum_l X q_l)_m / (sum_l X h_l)_m
//                 fbar'  = 2 f' - f.
// The 3x3 solve takes the FP64 sums directly (equilibrated Cholesky).
//
// EPI adds fbar' written into the packed images the next forward projection
// reads (interior only; the zero border is written when the images are
// first packed), the column-contiguous copy transposed through LDS; and, if
// partial is set (batched iteration), the tile's FP64 sums of |f' - f|^2 and
// |f'|^2 (fixed-order reduction) for the relative-change stopping rule.
struct PrimalEpilogue {
  float4 *pk_xy, *pk_yx;
  double2 *partial;  // this tile's (sum |f' - f|^2, sum |f'|^2), or null
};

// The primal step of one tile from its FP64 back-projected sums acc (the
// pixel of this thread); every thread of the workgroup calls it (EPI holds a
// workgroup barrier).  tile and red: LDS the workgroup's gather is done with.
template <bool BLOCK, bool EPI>
__device__ __forceinline__ void primal_epilogue(const ScanDesc &sd, const double *acc, float *__restrict__ f,
                                                float *__restrict__ fbar, float lambda, int tile_x, int tile_y,
                                                float4 (&tile)[kBpTile][kBpTile + 1], double2 *red,
                                                const PrimalEpilogue &epi) {
  int tx, ty;
  bp_pixel_of_thread(threadIdx.x, tx, ty);
  const int ix = tile_x * kBpTile + tx;
  const int iy = tile_y * kBpTile + ty;
  const bool inside = ix < sd.n && iy < sd.n;
  if (!EPI && !inside) return;
  const int nn = sd.n * sd.n;
  const int k = iy * sd.n + ix;
  float fo[3] = {0.0f, 0.0f, 0.0f}, fn[3] = {0.0f, 0.0f, 0.0f}, fb[3] = {0.0f, 0.0f, 0.0f};
  if (inside) {
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
      for (int m = 0; m < 3; ++m)
        fn[m] = acc[3 + m] > 0.0 ? (float)((double)fo[m] - lam * acc[m] / acc[3 + m]) : fo[m];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      fb[m] = 2.0f * fn[m] - fo[m];
      f[m * nn + k] = fn[m];
      fbar[m * nn + k] = fb[m];
    }
  }
  if (!EPI) return;
  // packed copies of fbar' and the tile's change sums
  const int np = sd.n + 2 * kPad;
  const float4 v4 = make_float4(fb[0], fb[1], fb[2], 0.0f);
  if (inside) epi.pk_xy[(size_t)(iy + kPad) * np + (ix + kPad)] = v4;
  const bool sums = epi.partial != nullptr;  // uniform
  if (sums) {
    double d2 = 0.0, n2 = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const double dm = (double)fn[m] - (double)fo[m];
      d2 += dm * dm;
      n2 += (double)fn[m] * (double)fn[m];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      d2 += __shfl_xor(d2, o, 64);
      n2 += __shfl_xor(n2, o, 64);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(d2, n2);
  }
  tile[ty][tx] = v4;  // the gather's closing barrier has released the staging slots
  __syncthreads();
  {
    const int cx = threadIdx.x / kBpTile, ry = threadIdx.x & (kBpTile - 1);  // column cx, row ry of the tile
    const int jx = tile_x * kBpTile + cx, jy = tile_y * kBpTile + ry;
    if (jx < sd.n && jy < sd.n) epi.pk_yx[(size_t)(jx + kPad) * np + (jy + kPad)] = tile[ry][cx];
  }
  if (sums && threadIdx.x == 0) {
    double2 s = red[0];
#pragma unroll
    for (int w = 1; w < kBpThreads / 64; ++w) {
      s.x += red[w].x;
      s.y += red[w].y;
    }
    *epi.partial = s;
  }
}

// Back-projection of one tile fused with its primal step.  FOLD: the sum
// over views formed part by part (ScanDesc::bp_part_views), the bits of the
// split back-projection (k_back_partial + k_primal_combine).
template <bool BLOCK, bool WIDE, bool EPI, bool COPY, bool FOLD = false>
__device__ __forceinline__ void back_primal_tile(const ScanDesc &sd, const float *__restrict__ qS,
                                                 float *__restrict__ f, float *__restrict__ fbar, float lambda,
                                                 int tile_x, int tile_y, BpShared &sh, const PrimalEpilogue &epi) {
  constexpr int NCH = BLOCK ? 9 : 6;
  double acc[NCH];
  back_accumulate<NCH, WIDE, true, COPY, FOLD>(sd, tile_x, tile_y, qS, 0, acc, sh, 0, sd.n_views);
  primal_epilogue<BLOCK, EPI>(sd, acc, f, fbar, lambda, tile_x, tile_y, sh.tile, sh.red, epi);
}

}  // namespace osscir
