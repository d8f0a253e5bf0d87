// Batched MOCCA kernels: one launch per stage advances every running slot.
//
// Each kernel walks a host-built work list (forward: one view's chunk of
// rays; spectral: a range of rays; back-projection: a 16 x 16 pixel tile)
// with a fixed number of workgroups, so the launch shapes do not depend on
// which scans are bound and one captured graph serves any mix.  The work of
// an item is the single-scan device function of the same stage, so a slot
// computes bit for bit what the single-scan path computes for its scan: the
// forward walk of a wave depends only on the 64 bins it holds (chunks start
// at multiples of 64), and the per-pixel sums run over views in order.
#include "batch.h"
#include "device_math.h"
#include "forward_device.h"
#include "kernels.h"
#include "project_device.h"
#include "spectral_device.h"

namespace osscir {

// Work lists, slot descriptors and status are read-only while a stage
// kernel runs: read through the scalar cache.
__device__ __forceinline__ int list_count(const WorkList &wl, int x) { return as_const(wl.buf)[x]; }
__device__ __forceinline__ int list_item(const WorkList &wl, int x, int j) {
  return as_const(wl.buf)[kListHeader + x * wl.cap + j];
}
// The slot's descriptor in SGPRs, its buffers marked as global memory (the
// pointers are re-read as pointers: a pointer rebuilt from words would be
// accessed with flat instructions).
__device__ __forceinline__ SlotDesc load_slot(const SlotDesc *slots, int s) {
  SlotDesc d = load_uniform(slots + s);
  const OSSCIR_CONST SlotDesc *q = as_const(slots + s);
  d.sd.rays = as_global(q->sd.rays);
  d.sd.rho = as_global(q->sd.rho);
  d.sd.views = as_global(q->sd.views);
  d.sd.sbin = as_global(q->sd.sbin);
  d.sd.n0bin = as_global(q->sd.n0bin);
  d.sd.n0ray = as_global(q->sd.n0ray);
  d.f = as_global(q->f);
  d.fbar = as_global(q->fbar);
  d.y = as_global(q->y);
  d.c = as_global(q->c);
  d.p = as_global(q->p);
  d.qS = as_global(q->qS);
  d.pk_xy = as_global(q->pk_xy);
  d.pk_yx = as_global(q->pk_yx);
  d.p0 = as_global(q->p0);
  return d;
}

// Nested loops: the slot's step within its outer iteration (0 for a single
// loop).  The first step projects into p0 and forms the model there; the
// others project into p and keep the model at p0.
__device__ __forceinline__ int slot_inner_step(const SlotStatus *status, int s, const SlotDesc &sl) {
  return sl.n_inner > 1 ? as_const(status)[s].iters % sl.n_inner : 0;
}

__device__ __forceinline__ bool slot_running(const SlotStatus *status, int s) {
  return as_const(status)[s].state == kSlotRunning;
}

__global__ void __launch_bounds__(256 * kFpParts) __attribute__((amdgpu_waves_per_eu(5))) kb_forward(const SlotDesc *__restrict__ slots,
                                                                       const SlotStatus *__restrict__ status,
                                                                       WorkList wl) {
  const int x = blockIdx.x % kXcds;
  const int stride = gridDim.x / kXcds;
  const int cnt = list_count(wl, x);
  const int R = blockDim.x / kFpParts;  // rays per item
  extern __shared__ float4 fwd_rows[];  // kFpWaveRows image rows per wave (forward_walk_lds)
  float4 OSSCIR_LDS *wb = (float4 OSSCIR_LDS *)(fwd_rows + (threadIdx.x >> 6) * kFpWaveRows);
  for (int j = blockIdx.x / kXcds; j < cnt; j += stride) {
    const int it = list_item(wl, x, j);
    const int s = item_slot(it), local = item_local(it);
    if (!slot_running(status, s)) continue;
    const SlotDesc sl = load_slot(slots, s);
    const int nchunk = (sl.sd.n_bins + R - 1) / R;
    const int v = local / nchunk;
    float *out = sl.n_inner > 1 && slot_inner_step(status, s, sl) == 0 ? sl.p0 : sl.p;
    forward_rays<false>(sl.sd, sl.pk_xy, sl.pk_yx, out, sl.sd.n_rays, 3, v, (local - v * nchunk) * R, wb);
  }
}

// NESTED: the variant launched while some slot runs nested loops (its
// inner steps take the model from p0 and the dual step at p); the other
// variant serves batches of single-loop slots only.
template <typename T, bool CLIP, bool BLOCK, bool NESTED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) kb_spectral_dual(const SlotDesc *__restrict__ slots,
                                                         const SlotStatus *__restrict__ status, WorkList wl) {
  extern __shared__ float stab[];  // matrix-core sums: the slot's table, then transposition tiles
  const int x = blockIdx.x % kXcds;
  const int stride = gridDim.x / kXcds;
  const int cnt = list_count(wl, x);
  for (int j = blockIdx.x / kXcds; j < cnt; j += stride) {
    const int it = list_item(wl, x, j);
    const int s = item_slot(it), local = item_local(it);
    if (!slot_running(status, s)) continue;
    const SlotDesc sl = load_slot(slots, s);
    const int l = local * (int)blockDim.x + (int)threadIdx.x;
    if (NESTED) {
      // one call per energy-sum mode: a nested slot's inner steps pass pbar
      // (model at p0), its first step and single-loop slots pass none
      const bool nest = sl.n_inner > 1;
      const float *pm = nest ? sl.p0 : sl.p;
      const float *pb = nest && slot_inner_step(status, s, sl) != 0 ? sl.p : nullptr;
      if (sl.sd.per_bin) {
        spectral_dual_ray<T, CLIP, BLOCK, true, false, true>(sl.sd, pm, sl.c, sl.y, sl.qS, sl.lambda, l, nullptr, pb);
      } else if (sl.sd.mfma) {
        __syncthreads();
        stage_table(sl.sd, stab);
        __syncthreads();
        spectral_dual_ray<T, CLIP, BLOCK, false, true, true>(sl.sd, pm, sl.c, sl.y, sl.qS, sl.lambda, l, stab, pb);
      } else {
        spectral_dual_ray<T, CLIP, BLOCK, false, false, true>(sl.sd, pm, sl.c, sl.y, sl.qS, sl.lambda, l, nullptr,
                                                              pb);
      }
    } else if (sl.sd.per_bin) {
      spectral_dual_ray<T, CLIP, BLOCK, true>(sl.sd, sl.p, sl.c, sl.y, sl.qS, sl.lambda, l);
    } else if (sl.sd.mfma) {  // uniform over the workgroup, as in the single-scan kernel
      __syncthreads();        // the previous item is done with the staged table and tiles
      stage_table(sl.sd, stab);
      __syncthreads();
      spectral_dual_ray<T, CLIP, BLOCK, false, true>(sl.sd, sl.p, sl.c, sl.y, sl.qS, sl.lambda, l, stab);
    } else {
      spectral_dual_ray<T, CLIP, BLOCK, false>(sl.sd, sl.p, sl.c, sl.y, sl.qS, sl.lambda, l);
    }
  }
}

template <bool BLOCK, bool WIDE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) kb_back_primal(const SlotDesc *__restrict__ slots,
                                                       const SlotStatus *__restrict__ status, WorkList wl,
                                                       double2 *__restrict__ partial) {
  __shared__ BpShared sh;
  const int x = blockIdx.x % kXcds;
  const int stride = gridDim.x / kXcds;
  const int cnt = list_count(wl, x);
  for (int j = blockIdx.x / kXcds; j < cnt; j += stride) {
    const int it = list_item(wl, x, j);
    const int s = item_slot(it), local = item_local(it);
    if (!slot_running(status, s)) continue;  // uniform over the workgroup
    const SlotDesc sl = load_slot(slots, s);
    const int ntx = (sl.sd.n + kBpTile - 1) / kBpTile;
    const int ty = local / ntx, tx = local - ty * ntx;
    const PrimalEpilogue epi{sl.pk_xy, sl.pk_yx, partial + sl.first_tile + local};
    // the persistent grid keeps four workgroups per CU: global-to-LDS staging;
    // the sums formed part by part, as the scan's own split back-projection
    // forms them
    back_primal_tile<BLOCK, WIDE, true, !WIDE, true>(sl.sd, sl.qS, sl.f, sl.fbar, sl.lambda, tx, ty, sh, epi);
  }
}

// One wave per slot: the tile partial sums in a fixed order, then the
// stopping rule.
__global__ void __launch_bounds__(64) kb_tick(const SlotDesc *__restrict__ slots, SlotStatus *__restrict__ status,
                                               const double2 *__restrict__ partial) {
  const int s = blockIdx.x;
  if (status[s].state != kSlotRunning) return;
  const int first = slots[s].first_tile, nt = slots[s].n_tiles;
  double d2 = 0.0, n2 = 0.0;
  for (int j = threadIdx.x; j < nt; j += 64) {
    const double2 v = partial[first + j];
    d2 += v.x;
    n2 += v.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    d2 += __shfl_xor(d2, o, 64);
    n2 += __shfl_xor(n2, o, 64);
  }
  if (threadIdx.x == 0) {
    SlotStatus st = status[s];
    st.iters += 1;
    st.rel_change = n2 > 0.0 ? sqrt(d2 / n2) : (d2 > 0.0 ? INFINITY : 0.0);
    if (!isfinite(d2) || !isfinite(n2))  // a NaN or an infinity in f (or f - f_prev): stop and report
      st.state = kSlotFailed;
    else if ((st.max_iter > 0 && st.iters >= st.max_iter) || (st.tol > 0.0 && st.rel_change <= st.tol))
      st.state = kSlotDone;
    status[s] = st;
  }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_batch_forward(const SlotDesc *slots, const SlotStatus *status, WorkList wl, int rays_per_wg,
                                hipStream_t st) {
  const int threads = rays_per_wg * kFpParts;  // kFpParts waves per 64 rays
  const size_t lds = (size_t)(threads / 64) * kFpWaveRows * sizeof(float4);
  hipLaunchKernelGGL(kb_forward, dim3((unsigned)wl.wgs), dim3((unsigned)threads), lds, st, slots, status, wl);
  return hipGetLastError();
}

hipError_t launch_batch_spectral_dual(const SlotDesc *slots, const SlotStatus *status, WorkList wl,
                                      int rays_per_wg, size_t lds, bool clip, bool block, bool fp64, bool nested,
                                      hipStream_t st) {
  const dim3 g((unsigned)wl.wgs), b((unsigned)rays_per_wg);
#define OSSCIR_BDUAL(T, C, B)                                                                                  \
  do {                                                                                                        \
    if (nested)                                                                                               \
      hipLaunchKernelGGL((kb_spectral_dual<T, C, B, true>), g, b, lds, st, slots, status, wl);                \
    else                                                                                                      \
      hipLaunchKernelGGL((kb_spectral_dual<T, C, B, false>), g, b, lds, st, slots, status, wl);               \
  } while (0)
  if (fp64) {
    if (clip) {
      if (block) OSSCIR_BDUAL(double, true, true); else OSSCIR_BDUAL(double, true, false);
    } else {
      if (block) OSSCIR_BDUAL(double, false, true); else OSSCIR_BDUAL(double, false, false);
    }
  } else {
    if (clip) {
      if (block) OSSCIR_BDUAL(float, true, true); else OSSCIR_BDUAL(float, true, false);
    } else {
      if (block) OSSCIR_BDUAL(float, false, true); else OSSCIR_BDUAL(float, false, false);
    }
  }
#undef OSSCIR_BDUAL
  return hipGetLastError();
}

hipError_t launch_batch_back_primal(const SlotDesc *slots, const SlotStatus *status, WorkList wl, bool block,
                                    bool wide, double2 *partial, hipStream_t st) {
  const dim3 g((unsigned)wl.wgs), b(kBpThreads);
#define OSSCIR_BBP(B, W) hipLaunchKernelGGL((kb_back_primal<B, W>), g, b, 0, st, slots, status, wl, partial)
  if (block) {
    if (wide) OSSCIR_BBP(true, true); else OSSCIR_BBP(true, false);
  } else {
    if (wide) OSSCIR_BBP(false, true); else OSSCIR_BBP(false, false);
  }
#undef OSSCIR_BBP
  return hipGetLastError();
}

hipError_t launch_batch_tick(const SlotDesc *slots, SlotStatus *status, const double2 *partial, int n_slots,
                             hipStream_t st) {
  hipLaunchKernelGGL(kb_tick, dim3((unsigned)n_slots), dim3(64), 0, st, slots, status, partial);
  return hipGetLastError();
}

}  // namespace osscir
