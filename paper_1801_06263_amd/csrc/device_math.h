// Device-side building blocks shared by every kernel of the library:
// the exact line-intersection weight of the projector, softexp, and the
// small symmetric linear algebra of the per-ray and per-pixel tails.
//
// The whole library is compiled with -ffp-contract=off: every fused
// multiply-add is written out with __fmaf_rn / fma, so the projector weight
// below rounds identically in the forward projector and in the
// back-projector, which makes X^T the exact transpose of X.
#pragma once

#include <hip/hip_runtime.h>

namespace osscir {

// ---------------------------------------------------------------- projector
//
// A ray is a line through the source S of its view with unit normal
// (nx, ny).  The chord of that line through the unit square centred at P
// depends only on the signed distance sig = n . (S - P) of the square's
// centre from the line: it is the trapezoid
//   min(hmax, max(0, (a - |sig|) kappa))  with
//   a     = (|nx| + |ny|) / 2           (half-width of the square's shadow)
//   kappa = 1 / (|nx| |ny|)             (slope of the corner-cutting part)
//   hmax  = 1 / max(|nx|, |ny|)         (chord through a full column/row)
// all multiplied by the pixel size to give centimetres.  This is the exact
// line-intersection length X_{l,k} (the chord of the square, Sec. II's
// "projection along ray l"), evaluated branch-free.  The ray table holds
// the normal and the half-width already scaled by kappa, so the trapezoid is
// min(hmax, max(0, a kappa - |sig kappa|)): one subtraction and one clamp.
//
// Coordinates are pixel units with pixel (ix, iy) centred at (ix, iy); the
// caller passes dx = Sx - ix, dy = Sy - iy in FP64 (sig is a difference of
// numbers as large as the source distance), sig kappa is rounded once to
// FP32 and the trapezoid is FP32.
struct RayLine {
  double nxk, nyk;  // kappa nx, kappa ny
  float ak, hmax;   // kappa a, hmax
  float kappa, pad;
};

// zero: 0.0f (a caller reading the ray from a record may pass the record's
// stored zero instead of the constant, with the same result)
__device__ __forceinline__ float chord_weight(double nxk, double nyk, float ak, float hmax, double dx, double dy,
                                              float zero = 0.0f) {
  const double sigk = fma(nxk, dx, nyk * dy);
  return __builtin_amdgcn_fmed3f(ak - fabsf((float)sigk), zero, hmax);  // clamp to [0, hmax]
}

// ---------------------------------------------------------------- helpers

// floor(x) as an integer in one instruction; x is finite and in int range
// (a NaN gives 0)
__device__ __forceinline__ int floor_to_int(float x) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// min(max(x, 0), hi) for uniform hi >= 0 in one instruction
__device__ __forceinline__ int clamp_0_hi(int x, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(hi));
  return r;
}

// A copy of a (uniform) value held in a VGPR: lets a loop use it as the
// vector operand of an instruction that already reads one SGPR, instead of
// moving it from the SGPR on every iteration.
__device__ __forceinline__ float in_vgpr(float x) {
  float r;
  asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// ---------------------------------------------------------------- softexp
//
// softexp(x) = exp(x) for x <= 0 and x + 1 for x > 0 (Sec. II).  With
// x = -z: E = softexp(-z), E1 = softexp'(-z), E2 = softexp''(-z), the x <= 0
// branch taken at x = 0 (so softexp''(0) = 1).
__device__ __forceinline__ void softexp3(float z, float &E, float &E1, float &E2) {
  const float e = __expf(-z);
  const bool phys = z >= 0.0f;
  E = phys ? e : 1.0f - z;
  E1 = phys ? e : 1.0f;
  E2 = phys ? e : 0.0f;
}

// ---------------------------------------------------------------- 3x3 / 4x4
// Symmetric matrices are kept as their upper triangle
// (00, 01, 02, 11, 12, 22).

template <typename T>
__device__ __forceinline__ T rsqrt_t(T x);
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) { return 1.0f / sqrtf(x); }
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix:
// on return A holds the eigenvalues on its diagonal and V the eigenvectors
// (columns).  A fixed number of sweeps; a rotation whose off-diagonal entry
// is exactly zero is skipped.
template <typename T, int SWEEPS>
__device__ __forceinline__ void jacobi3(T A[3][3], T V[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? T(1) : T(0);
#pragma unroll
  for (int sweep = 0; sweep < SWEEPS; ++sweep) {
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      const int r = 3 - p - q;
      const T apq = A[p][q];
      if (apq != T(0)) {
        const T theta = (A[q][q] - A[p][p]) / (T(2) * apq);
        T t = T(1) / (fabs(theta) + sqrt(theta * theta + T(1)));
        if (theta < T(0)) t = -t;
        const T c = rsqrt_t<T>(t * t + T(1));
        const T s = t * c;
        const T app = A[p][p] - t * apq;
        const T aqq = A[q][q] + t * apq;
        const T arp = c * A[r][p] - s * A[r][q];
        const T arq = s * A[r][p] + c * A[r][q];
        A[p][p] = app;
        A[q][q] = aqq;
        A[p][q] = A[q][p] = T(0);
        A[r][p] = A[p][r] = arp;
        A[r][q] = A[q][r] = arq;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
    }
  }
}

// H^+ = V max(Lambda, 0) V^T.  A positive-definite H (checked on its
// diagonally equilibrated form by Sylvester's criterion) is returned as is.
template <typename T, int SWEEPS>
__device__ __forceinline__ void clip_negative_curvature(const T h[6], T hp[6]) {
  bool pd = h[0] > T(0) && h[3] > T(0) && h[5] > T(0);
  if (pd) {
    const T d0 = rsqrt_t<T>(h[0]), d1 = rsqrt_t<T>(h[3]), d2 = rsqrt_t<T>(h[5]);
    const T b01 = h[1] * d0 * d1, b02 = h[2] * d0 * d2, b12 = h[4] * d1 * d2;
    const T m2 = T(1) - b01 * b01;
    const T det = T(1) + T(2) * b01 * b02 * b12 - b01 * b01 - b02 * b02 - b12 * b12;
    pd = m2 > T(0) && det > T(0);
  }
  if (pd) {
#pragma unroll
    for (int i = 0; i < 6; ++i) hp[i] = h[i];
    return;
  }
  T A[3][3] = {{h[0], h[1], h[2]}, {h[1], h[3], h[4]}, {h[2], h[4], h[5]}};
  T V[3][3];
  jacobi3<T, SWEEPS>(A, V);
  const T l0 = A[0][0] > T(0) ? A[0][0] : T(0);
  const T l1 = A[1][1] > T(0) ? A[1][1] : T(0);
  const T l2 = A[2][2] > T(0) ? A[2][2] : T(0);
  int k = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      hp[k++] = V[i][0] * l0 * V[j][0] + V[i][1] * l1 * V[j][1] + V[i][2] * l2 * V[j][2];
    }
}

// Solve the symmetric positive-definite 3x3 system S x = b (upper triangle
// S[6]) by Cholesky after symmetric diagonal equilibration.
template <typename T>
__device__ __forceinline__ void spd3_solve(const T S[6], const T b[3], T x[3]) {
  const T d0 = rsqrt_t<T>(S[0]), d1 = rsqrt_t<T>(S[3]), d2 = rsqrt_t<T>(S[5]);
  const T a01 = S[1] * d0 * d1, a02 = S[2] * d0 * d2, a12 = S[4] * d1 * d2;
  // Cholesky of [[1,a01,a02],[a01,1,a12],[a02,a12,1]] = L L^T
  const T l11 = sqrt(T(1) - a01 * a01);
  const T l20 = a02;
  const T l21 = (a12 - a02 * a01) / l11;
  const T l22 = sqrt(T(1) - l20 * l20 - l21 * l21);
  const T c0 = b[0] * d0, c1 = b[1] * d1, c2 = b[2] * d2;
  // forward L u = c (l00 = 1, l10 = a01)
  const T u0 = c0;
  const T u1 = (c1 - a01 * u0) / l11;
  const T u2 = (c2 - l20 * u0 - l21 * u1) / l22;
  // backward L^T z = u
  const T z2 = u2 / l22;
  const T z1 = (u1 - l21 * z2) / l11;
  const T z0 = u0 - a01 * z1 - l20 * z2;
  x[0] = z0 * d0;
  x[1] = z1 * d1;
  x[2] = z2 * d2;
}

// Inverse of a symmetric positive-definite 3x3 (upper triangle in, full out)
// by the adjugate.
template <typename T>
__device__ __forceinline__ void spd3_inverse(const T S[6], T inv[3][3]) {
  const T c00 = S[3] * S[5] - S[4] * S[4];
  const T c01 = S[2] * S[4] - S[1] * S[5];
  const T c02 = S[1] * S[4] - S[2] * S[3];
  const T c11 = S[0] * S[5] - S[2] * S[2];
  const T c12 = S[1] * S[2] - S[0] * S[4];
  const T c22 = S[0] * S[3] - S[1] * S[1];
  const T det = S[0] * c00 + S[1] * c01 + S[2] * c02;
  const T id = T(1) / det;
  inv[0][0] = c00 * id; inv[0][1] = c01 * id; inv[0][2] = c02 * id;
  inv[1][0] = c01 * id; inv[1][1] = c11 * id; inv[1][2] = c12 * id;
  inv[2][0] = c02 * id; inv[2][1] = c12 * id; inv[2][2] = c22 * id;
}

// Solve (I + M) z = b for symmetric positive semi-definite M (4x4, full),
// by Cholesky (every pivot is >= 1).
template <typename T>
__device__ __forceinline__ void unit_plus_psd4_solve(const T M[4][4], const T b[4], T z[4]) {
  T L[4][4], il[4];  // il: reciprocal pivots
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      T sum = M[i][j] + (i == j ? T(1) : T(0));
#pragma unroll
      for (int k = 0; k < j; ++k) sum -= L[i][k] * L[j][k];
      if (i == j) {
        L[i][i] = sqrt(sum);
        il[i] = T(1) / L[i][i];
      } else {
        L[i][j] = sum * il[j];
      }
    }
  }
  T u[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T sum = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) sum -= L[i][k] * u[k];
    u[i] = sum * il[i];
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    T sum = u[i];
#pragma unroll
    for (int k = i + 1; k < 4; ++k) sum -= L[k][i] * z[k];
    z[i] = sum * il[i];
  }
}

}  // namespace osscir
