// Forward projector building blocks (packing of the image and the per-ray
// walk), shared by the single-scan kernels (projector.hip) and the batched
// kernels (batch.hip).
#pragma once

#include "device_math.h"
#include "kernels.h"

namespace osscir {

// ----------------------------------------------------------------- packing
//
// Up to three planar channels -> two interleaved float4 images with a zero
// border of kPad pixels: pk_xy[iy + kPad][ix + kPad] (rows contiguous) and
// pk_yx[ix + kPad][iy + kPad] (columns contiguous), written through a 32 x 32
// LDS tile for the transposed copy.  The border lets the forward projector
// read its candidate pixels without bounds checks: a candidate outside the
// image reads 0 and adds w * 0 = 0.
__device__ __forceinline__ void pack_block(const float *__restrict__ f, int n, int nch, float4 *__restrict__ pk_xy,
                                           float4 *__restrict__ pk_yx, int bx, int by, float4 (&tile)[32][33]) {
  const int np = n + 2 * kPad;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const size_t nn = (size_t)n * n;
  for (int r = ty; r < 32; r += 8) {
    const int px = bx + tx, py = by + r;
    const int ix = px - kPad, iy = py - kPad;
    float4 val = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (ix >= 0 && ix < n && iy >= 0 && iy < n) {
      const size_t k = (size_t)iy * n + ix;
      val.x = f[k];
      if (nch > 1) val.y = f[nn + k];
      if (nch > 2) val.z = f[2 * nn + k];
    }
    if (px < np && py < np) pk_xy[(size_t)py * np + px] = val;
    tile[r][tx] = val;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int py = by + tx, px = bx + r;
    if (px < np && py < np) pk_yx[(size_t)px * np + py] = tile[tx][r];
  }
}


// ----------------------------------------------------------------- forward
//
// One thread per ray, a workgroup = a chunk of consecutive detector bins of one view
// (coalesced sinogram writes).  A ray walks its major axis (the image axis
// closer to its direction); in each column (row) the line spans less than one
// pixel of the minor axis, so the two pixels floor(y*) and floor(y*)+1 around
// its crossing point y* hold every non-zero weight (within 0.11 degree of 45
// degrees a third pixel is tested, against rounding).  Rays walking columns
// read the column-contiguous packed image, rays walking rows the
// row-contiguous one, so neighbouring lanes (neighbouring bins) read
// neighbouring addresses; all lanes of a wave step through the same walk
// index (the wave's union of walk ranges), several columns per step with
// every load issued before the weights are formed.
//
// The FP64 offsets from the source are formed exactly as the back-projector
// forms them, one rounded subtraction s - (double)i per pixel index i, so
// every weight is bit-identical to the back-projector's.
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

// Products are summed in FP32 over 16 columns at a time, then into an FP64
// running sum (a ray crosses up to thousands of pixels).  kFpUnroll columns
// are processed per step; the last step may run past the image by up to
// kFpUnroll - 1 columns, which the zero border (kPad >= kFpUnroll) absorbs.
constexpr int kFpUnroll = 4;

static_assert(kPad >= kFpUnroll, "border must cover the unrolled tail");
template <bool XMAJOR, bool THIRD, bool COUNT>
__device__ __forceinline__ void forward_walk(int lo, int hi, int n, const float4 *__restrict__ img, double s_u,
                                             double s_v, float slope, float base, const RayLine &ray, double &s0,
                                             double &s1, double &s2) {
  const int np = n + 2 * kPad;
  constexpr int NC = THIRD ? 3 : 2;
  float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
  int pairs = 0;
  for (int u = lo; u <= hi; u += kFpUnroll) {
    float4 fv[kFpUnroll][NC];
    float w[kFpUnroll][NC];
    int iv0s[kFpUnroll], ives[kFpUnroll];
#pragma unroll
    for (int k = 0; k < kFpUnroll; ++k) {
      const int uu = u + k;
      const float ys = __fmaf_rn(slope, (float)uu, base);
      int iv0, ive = 0;
      if (THIRD) {
        const float fl = floorf(ys);
        iv0 = min(max((int)fl, -2), n);
        ive = (ys - fl < 0.5f) ? iv0 - 1 : iv0 + 2;
      } else {
        iv0 = floor_to_int(__builtin_amdgcn_fmed3f(ys, -2.0f, (float)n));  // in [-2, n]
      }
      iv0s[k] = iv0;
      ives[k] = ive;
      if (!COUNT) {
        // uniform row base, non-negative 32-bit byte offsets (iv0 >= -2, ive >= -3)
        const char *__restrict__ line = reinterpret_cast<const char *>(img + (size_t)(uu + kPad) * np);
        const unsigned o0 = (unsigned)(iv0 + kPad) * 16u;
        fv[k][0] = *reinterpret_cast<const float4 *>(line + o0);
        fv[k][1] = *reinterpret_cast<const float4 *>(line + o0 + 16u);
        if (THIRD) fv[k][2] = *reinterpret_cast<const float4 *>(line + (unsigned)(ive + kPad) * 16u);
      }
      const double du = s_u - (double)uu;
      const double fv0 = (double)iv0;
      const double dv0 = s_v - fv0;
      const double dv1 = s_v - (fv0 + 1.0);
      if (XMAJOR) {
        w[k][0] = chord_weight(ray.nxk, ray.nyk, ray.ak, ray.hmax, du, dv0);
        w[k][1] = chord_weight(ray.nxk, ray.nyk, ray.ak, ray.hmax, du, dv1);
      } else {
        w[k][0] = chord_weight(ray.nxk, ray.nyk, ray.ak, ray.hmax, dv0, du);
        w[k][1] = chord_weight(ray.nxk, ray.nyk, ray.ak, ray.hmax, dv1, du);
      }
      if (THIRD) {
        const double dve = s_v - (double)ive;
        w[k][2] = XMAJOR ? chord_weight(ray.nxk, ray.nyk, ray.ak, ray.hmax, du, dve)
                         : chord_weight(ray.nxk, ray.nyk, ray.ak, ray.hmax, dve, du);
      }
      // a column index past the image reads the zero border (w * 0 adds +0 to
      // the sums); only the counting pass must drop its weights
      if (COUNT && uu >= n) {
#pragma unroll
        for (int j = 0; j < NC; ++j) w[k][j] = 0.0f;
      }
    }
#pragma unroll
    for (int k = 0; k < kFpUnroll; ++k)
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        if (COUNT) {
          const int ivj = j == 0 ? iv0s[k] : (j == 1 ? iv0s[k] + 1 : ives[k]);
          a0 += (w[k][j] > 0.0f && ivj >= 0 && ivj < n) ? 1.0f : 0.0f;
        } else {
          a0 = __fmaf_rn(w[k][j], fv[k][j].x, a0);
          a1 = __fmaf_rn(w[k][j], fv[k][j].y, a1);
          a2 = __fmaf_rn(w[k][j], fv[k][j].z, a2);
        }
      }
    if (++pairs == 16 / kFpUnroll) {
      s0 += (double)a0;
      s1 += (double)a1;
      s2 += (double)a2;
      a0 = a1 = a2 = 0.0f;
      pairs = 0;
    }
  }
  s0 += (double)a0;
  s1 += (double)a1;
  s2 += (double)a2;
}

// The walk of a full wave (all lanes on one major axis, no ray near 45
// degrees) with the image read through LDS.  At a column the crossing is
// monotonic in the bin, and along the walk it is linear in the column, so
// over a step of kFpUnroll columns the candidate rows of the wave's 64 rays
// lie between the crossings of its first and last lanes at the step's first
// and last columns.  The step copies that window of rows (one row per lane,
// 16-byte buffer-to-LDS loads from a scalar offset: no VGPRs, one copy of a
// pixel that neighbouring rays share) for each of its columns, and each lane
// reads its two candidates per column from LDS.  The window keeps one row of
// margin on each side for crossings that FP32 rounding moves across a row
// boundary; a step whose window exceeds 64 rows reads the same pixels
// directly, so the products and their order are exactly those of
// forward_walk.
//
// The loop is rotated: once a step's candidates are in registers, the next
// step's copies are issued and the step's products summed while they are in
// flight (one LDS window per wave, as before).  Two register sets alternate
// so nothing is moved between iterations.
//
// The source lies on a 2^-30-pixel grid (the plan rounds it there), so
// every offset s - i is exact in FP64: the column offset is s_u - u and the
// second candidate's offset is the first's minus one, with the same bits as
// the back-projector's per-pixel offsets.
struct WalkStep {
  int iv0s[kFpUnroll];   // first candidate row per column
  int r0;                // first row of the step's window
  bool via_lds;          // the window fits 64 rows
  float w[kFpUnroll][2];
  float4 fv[kFpUnroll][2];
};

typedef float f32x4_t __attribute__((ext_vector_type(4)));

// min / max of wave-uniform values on the scalar unit (left to itself the
// compiler forms them with vector min3 / max3 and moves them back, seven
// vector instructions per step of a walk bound by vector issue)
__device__ __forceinline__ int uniform_min(int a, int b) {
  int r;
  asm volatile("s_min_i32 %0, %1, %2" : "=s"(r) : "s"(a), "s"(b) : "scc");
  return r;
}
__device__ __forceinline__ int uniform_max(int a, int b) {
  int r;
  asm volatile("s_max_i32 %0, %1, %2" : "=s"(r) : "s"(a), "s"(b) : "scc");
  return r;
}

// Marks loaded candidates as held in registers: without it the compiler
// turns values carried into the next iteration back into loads at their use.
__device__ __forceinline__ void hold(float4 &x) {
  f32x4_t v = __builtin_bit_cast(f32x4_t, x);
  asm volatile("" : "+v"(v));
  x = __builtin_bit_cast(float4, v);
}

template <bool XMAJOR>
__device__ __forceinline__ void forward_walk_lds(int lo, int hi, int n, const float4 *__restrict__ img, double s_u,
                                                 double s_v, float slope, float base, const RayLine &ray, double &s0,
                                                 double &s1, double &s2, float4 OSSCIR_LDS *wb) {
  static_assert(kFpUnroll == 4, "the step window is bounded at its first and last column");
  // A wave whose rays all miss the image has an empty walk range (its lo may
  // lie far past the image): nothing to walk or copy.  Otherwise
  // 0 <= lo <= hi <= n - 1, and every copied column (at most
  // hi + kFpUnroll - 1 + kPad) and row (1 .. n + 6) lies inside the padded image.
  if (lo > hi) return;
  const int np = n + 2 * kPad;
  const int lane = (int)__lane_id();
  // The copies go through a buffer descriptor of the packed image: the
  // lane's 16-byte row offset is fixed, the column's offset is a scalar, and
  // the wave's rows are a scalar LDS address, so forming a step's copies
  // takes no vector instructions (the walk is bound by VALU issue).  Every
  // copied row lies inside the padded image, the descriptor's range.
  wb = (float4 OSSCIR_LDS *)(size_t)__builtin_amdgcn_readfirstlane((unsigned)(size_t)wb);
  const __amdgpu_buffer_rsrc_t img_rsrc =
      __builtin_amdgcn_make_buffer_rsrc((void *)img, 0, np * np * (int)sizeof(float4), kBufferRsrcWord3);
  const unsigned lane_off = (unsigned)lane * 16u;  // this lane's row of a copied window
  float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
  int pairs = 0;
  // the step at column u: candidate rows, window, and the window's copies
  // (wb must be free: the previous step's reads have completed)
  auto fetch = [&](int u, WalkStep &st) {
#pragma unroll
    for (int k = 0; k < kFpUnroll; ++k) {
      const float ys = __fmaf_rn(slope, (float)(u + k), base);
      st.iv0s[k] = floor_to_int(__builtin_amdgcn_fmed3f(ys, -2.0f, (float)n));  // in [-2, n]
    }
    // the step's rows r0 .. r0 + span - 1 (r0 >= -3, r0 + span - 1 <= n + 2)
    const int c00 = __builtin_amdgcn_readlane(st.iv0s[0], 0), c01 = __builtin_amdgcn_readlane(st.iv0s[0], 63);
    const int c30 = __builtin_amdgcn_readlane(st.iv0s[kFpUnroll - 1], 0);
    const int c31 = __builtin_amdgcn_readlane(st.iv0s[kFpUnroll - 1], 63);
    st.r0 = uniform_min(uniform_min(c00, c01), uniform_min(c30, c31)) - 1;
    const int span = uniform_max(uniform_max(c00, c01), uniform_max(c30, c31)) - st.r0 + 3;
    st.via_lds = span <= 64;  // uniform
    if (st.via_lds && lane < span) {
      // a uniform base per column plus the lane's 16-byte row offset
      const unsigned col = (unsigned)((u + kPad) * np + (st.r0 + kPad)) * (unsigned)sizeof(float4);  // uniform
#pragma unroll
      for (int k = 0; k < kFpUnroll; ++k)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(img_rsrc, (void OSSCIR_LDS *)(wb + k * 64), 16, lane_off,
                                                 col + (unsigned)(k * np) * (unsigned)sizeof(float4), 0, 0);
    }
  };
  auto weights = [&](int u, WalkStep &st) {
    const double du0 = s_u - (double)u;  // exact
#pragma unroll
    for (int k = 0; k < kFpUnroll; ++k) {
      const double du = du0 - (double)k;  // exact
      const double dv0 = s_v - (double)st.iv0s[k];
      const double dv1 = dv0 - 1.0;  // exact
      if (XMAJOR) {
        st.w[k][0] = chord_weight(ray.nxk, ray.nyk, ray.ak, ray.hmax, du, dv0);
        st.w[k][1] = chord_weight(ray.nxk, ray.nyk, ray.ak, ray.hmax, du, dv1);
      } else {
        st.w[k][0] = chord_weight(ray.nxk, ray.nyk, ray.ak, ray.hmax, dv0, du);
        st.w[k][1] = chord_weight(ray.nxk, ray.nyk, ray.ak, ray.hmax, dv1, du);
      }
    }
  };
  // after the copies have landed: the candidates
  auto read = [&](int u, WalkStep &st) {
    if (st.via_lds) {
      // generic view of the LDS rows (reads stay ds_read); slot of row r: r - r0
      const float4 *wr = (const float4 *)wb - st.r0;
#pragma unroll
      for (int k = 0; k < kFpUnroll; ++k) {
        st.fv[k][0] = wr[k * 64 + st.iv0s[k]];
        st.fv[k][1] = wr[k * 64 + st.iv0s[k] + 1];
      }
    } else {
#pragma unroll
      for (int k = 0; k < kFpUnroll; ++k) {
        const char *__restrict__ line = reinterpret_cast<const char *>(img + (size_t)(u + k + kPad) * np);
        const unsigned o0 = (unsigned)(st.iv0s[k] + kPad) * 16u;
        st.fv[k][0] = *reinterpret_cast<const float4 *>(line + o0);
        st.fv[k][1] = *reinterpret_cast<const float4 *>(line + o0 + 16u);
      }
    }
#pragma unroll
    for (int k = 0; k < kFpUnroll; ++k) {
      hold(st.fv[k][0]);
      hold(st.fv[k][1]);
    }
  };
  auto sum = [&](const WalkStep &st) {
#pragma unroll
    for (int k = 0; k < kFpUnroll; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        a0 = __fmaf_rn(st.w[k][j], st.fv[k][j].x, a0);
        a1 = __fmaf_rn(st.w[k][j], st.fv[k][j].y, a1);
        a2 = __fmaf_rn(st.w[k][j], st.fv[k][j].z, a2);
      }
    if (++pairs == 16 / kFpUnroll) {
      s0 += (double)a0;
      s1 += (double)a1;
      s2 += (double)a2;
      a0 = a1 = a2 = 0.0f;
      pairs = 0;
    }
  };
  WalkStep A, B;
  __builtin_amdgcn_s_waitcnt(0);
  fetch(lo, A);
  weights(lo, A);
  __builtin_amdgcn_s_waitcnt(0);  // A's copies have landed
  read(lo, A);
  for (int u = lo;; u += 2 * kFpUnroll) {
    // A holds step u; B takes step u + kFpUnroll
    __builtin_amdgcn_s_waitcnt(0);  // A's candidates are in registers: wb is free
    const bool nb = u + kFpUnroll <= hi;  // uniform
    if (nb) fetch(u + kFpUnroll, B);
    __builtin_amdgcn_sched_barrier(0);  // the copies go out before the sums
    sum(A);
    if (!nb) break;
    weights(u + kFpUnroll, B);
    __builtin_amdgcn_s_waitcnt(0);  // B's copies have landed
    read(u + kFpUnroll, B);
    __builtin_amdgcn_s_waitcnt(0);
    const bool na = u + 2 * kFpUnroll <= hi;
    if (na) fetch(u + 2 * kFpUnroll, A);
    __builtin_amdgcn_sched_barrier(0);
    sum(B);
    if (!na) break;
    weights(u + 2 * kFpUnroll, A);
    __builtin_amdgcn_s_waitcnt(0);
    read(u + 2 * kFpUnroll, A);
  }
  s0 += (double)a0;
  s1 += (double)a1;
  s2 += (double)a2;
}

// Each ray is walked by kFpParts waves, each over its own part of the
// columns, and the parts' FP64 sums are added in part order.  A central ray
// crosses ~500 columns and an edge one a few dozen, so a whole-ray wave
// lives for a large share of the launch and the last ones dispatched set its
// tail; parts shorten that (measured at 512^2: 0.376 ms whole, 0.313 / 0.290
// / 0.282 ms with 2 / 3 / 4 parts; 6 and 8 parts were slower again).
constexpr int kFpParts = 4;
constexpr int kFpWaveRows = kFpUnroll * 64;  // float4 rows of LDS per wave (forward_walk_lds)

// One workgroup: rays (v, d0 + 64 g + lane) of one view, g = wave / kFpParts,
// wave w taking part w % kFpParts of its rays' walk range (the range of the
// 64 rays, cut into kFpParts pieces, all but the last a whole number of
// kFpUnroll-column steps, so no column is walked twice).  wb: this wave's
// kFpWaveRows rows of LDS; the waves' buffers are consecutive, part 0's
// first: part k > 0 leaves its sums in its buffer for part 0.  Every wave of
// the workgroup must call this (it holds two workgroup barriers), the same
// number of times.
template <bool COUNT>
__device__ __forceinline__ void forward_rays(const ScanDesc &sd, const float4 *__restrict__ pk_xy,
                                             const float4 *__restrict__ pk_yx, float *__restrict__ p, int p_stride,
                                             int nch, int v, int d0, float4 OSSCIR_LDS *wb) {
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int part = wave % kFpParts;
  const int d = d0 + (wave / kFpParts) * 64 + (int)__lane_id();
  const int n = sd.n;
  const bool active = d < sd.n_bins;
  const ViewGeom vg = load_uniform(sd.views + v);
  RayLine ray{1.0, 0.0, 0.0f, 0.0f, 1.0f, 0.0f};
  bool xmajor = true, near45 = false;
  float slope = 0.0f, base = 0.0f;
  int iu_lo = n, iu_hi = -1;
  if (active) {
    ray = sd.rays[v * sd.n_bins + d];
    // the line in index coordinates: nx ix + ny iy = nx sx + ny sy (here
    // with the normal scaled by kappa > 0, which leaves the line unchanged)
    const double sidx = ray.nxk * vg.sx + ray.nyk * vg.sy;
    xmajor = fabs(ray.nyk) >= fabs(ray.nxk);
    const double nu = xmajor ? ray.nxk : ray.nyk;  // along the walked axis
    const double nv = xmajor ? ray.nyk : ray.nxk;  // along the minor axis, |nv| >= |n| / sqrt 2
    near45 = (fabs(nv) - fabs(nu)) < 2e-3 * (double)ray.kappa;  // |nv| - |nu| < 2e-3 for the unit normal
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
  // the wave's walk range is uniform: keep it (and the walk index) in SGPRs;
  // this wave's part of it
  const int lo0 = __builtin_amdgcn_readfirstlane(wave_min(iu_lo));
  const int hi0 = __builtin_amdgcn_readfirstlane(wave_max(iu_hi));
  int lo = n, hi = -1;  // empty
  if (lo0 <= hi0) {
    const int h = (hi0 - lo0 + kFpUnroll * kFpParts) / (kFpUnroll * kFpParts) * kFpUnroll;  // columns per part
    lo = lo0 + part * h;
    hi = part == kFpParts - 1 ? hi0 : min(hi0, lo + h - 1);
  }
  const bool any45 = __any(near45);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  // the LDS walk needs every lane of the wave on it (all active, one major
  // axis): each lane copies a row for the others
  const bool full = __builtin_amdgcn_read_exec() == ~0ull;
  const bool lds_walk =
      !COUNT && wb != nullptr && full && !any45 && __all(active) && (__all(xmajor) || __all(!xmajor));
  if (active) {
    if (lds_walk) {
      if (xmajor)
        forward_walk_lds<true>(lo, hi, n, pk_yx, vg.sx, vg.sy, slope, base, ray, a0, a1, a2, wb);
      else
        forward_walk_lds<false>(lo, hi, n, pk_xy, vg.sy, vg.sx, slope, base, ray, a0, a1, a2, wb);
    } else if (xmajor) {
      if (any45)
        forward_walk<true, true, COUNT>(lo, hi, n, pk_yx, vg.sx, vg.sy, slope, base, ray, a0, a1, a2);
      else
        forward_walk<true, false, COUNT>(lo, hi, n, pk_yx, vg.sx, vg.sy, slope, base, ray, a0, a1, a2);
    } else {
      if (any45)
        forward_walk<false, true, COUNT>(lo, hi, n, pk_xy, vg.sy, vg.sx, slope, base, ray, a0, a1, a2);
      else
        forward_walk<false, false, COUNT>(lo, hi, n, pk_xy, vg.sy, vg.sx, slope, base, ray, a0, a1, a2);
    }
  }
  // parts 1.. hand their sums to part 0 through their (now idle) LDS rows
  double OSSCIR_LDS *mine = (double OSSCIR_LDS *)wb;
  if (part != 0) {
    const int i = (int)__lane_id();
    mine[i] = a0;
    mine[64 + i] = a1;
    mine[128 + i] = a2;
  }
  __syncthreads();
  if (part == 0 && active) {
    const int i = (int)__lane_id();
#pragma unroll
    for (int k = 1; k < kFpParts; ++k) {
      const double OSSCIR_LDS *o = (const double OSSCIR_LDS *)(wb + k * kFpWaveRows);
      a0 += o[i];
      a1 += o[64 + i];
      a2 += o[128 + i];
    }
    const int l = v * sd.n_bins + d;
    if (COUNT) {
      reinterpret_cast<int *>(p)[l] = (int)a0;
    } else {
      p[l] = (float)a0;
      if (nch > 1) p[p_stride + l] = (float)a1;
      if (nch > 2) p[2 * p_stride + l] = (float)a2;
    }
  }
  __syncthreads();  // the rows are free for the workgroup's next rays
}


}  // namespace osscir
