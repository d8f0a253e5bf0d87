// Batched MOCCA: many independent scans (slots) advanced by one launch per
// stage.  Device-side slot descriptors, per-slot status and the work lists
// the batched kernels walk (batch.hip), and their launchers.
#pragma once

#include "kernels.h"

namespace osscir {

constexpr int kSlotEmpty = 0, kSlotRunning = 1, kSlotDone = 2, kSlotFailed = 3;
constexpr int kMaxSlots = 256;
constexpr int kItemSlotShift = 24;  // work item = slot << 24 | item index within the slot (as unsigned bits)
constexpr int kItemLocalMask = (1 << kItemSlotShift) - 1;

// Work-item codes: the slot in the top 8 bits, the slot's local item index
// (< 2^24, checked when the lists are built) below; encoded and decoded as
// unsigned so that slots 128..255 survive the sign bit.
__host__ __device__ constexpr int item_code(int slot, int local) {
  return (int)(((unsigned)slot << kItemSlotShift) | (unsigned)local);
}
__host__ __device__ constexpr int item_slot(int code) { return (int)((unsigned)code >> kItemSlotShift); }
__host__ __device__ constexpr int item_local(int code) { return code & kItemLocalMask; }
static_assert(kMaxSlots <= (1 << (32 - kItemSlotShift)), "slot index must fit the code's top bits");
static_assert(item_slot(item_code(kMaxSlots - 1, kItemLocalMask)) == kMaxSlots - 1, "slot round trip");
static_assert(item_local(item_code(kMaxSlots - 1, kItemLocalMask)) == kItemLocalMask, "local round trip");
static_assert(item_slot(item_code(128, 0)) == 128 && item_local(item_code(200, 12345)) == 12345, "round trip");
constexpr int kListHeader = 16;     // ints before the items: per-XCD counts (8) and padding

// Everything the batched kernels need of one slot: the plan's scan, the
// caller's state buffers and the slot's regions of the caller workspace.
struct SlotDesc {
  ScanDesc sd;
  float *f, *fbar, *y;
  const float *c;
  float *p, *qS;          // [3][L], [L][12]
  float4 *pk_xy, *pk_yx;  // packed fbar (zero border of kPad)
  float *p0;              // nested loops: X f0 of the current expansion point [3][L] (caller memory)
  float lambda;
  int first_tile;         // the slot's first entry in the per-tile partial sums
  int n_tiles;            // 16 x 16 tiles of the image
  int n_inner;            // inner steps per expansion point (1: single loop); step iters % n_inner of the outer one
};

// Device-owned progress of a slot.  The end-of-iteration kernel advances
// iters, stores the relative change of f and marks the slot done once
// iters reaches max_iter (> 0) or the change falls to tol (> 0), or failed
// once f is no longer finite; the stage kernels skip slots that are not
// running.
struct SlotStatus {
  int state;
  int iters;
  int max_iter;
  int pad;
  double tol;
  double rel_change;  // ||f_{n+1} - f_n|| / ||f_{n+1}|| of the last iteration
};

// A work list of one stage.  buf[0..7]: items per XCD; buf[kListHeader +
// x * cap + j]: item j of XCD x.  Workgroup b runs on XCD b % 8 and takes
// that XCD's items b / 8, b / 8 + wgs / 8, ...
struct WorkList {
  const int *buf;
  int cap;
  int wgs;  // workgroups (multiple of 8)
};

hipError_t launch_batch_forward(const SlotDesc *slots, const SlotStatus *status, WorkList wl, int rays_per_wg,
                                hipStream_t st);
// lds: dynamic LDS bytes, enough for every bound slot with matrix-core energy
// sums (mfma_lds_bytes at rays_per_wg / 64 waves), else 0
// nested: some bound slot has n_inner > 1 (the kernel variant that handles them)
hipError_t launch_batch_spectral_dual(const SlotDesc *slots, const SlotStatus *status, WorkList wl,
                                      int rays_per_wg, size_t lds, bool clip, bool block, bool fp64, bool nested,
                                      hipStream_t st);
hipError_t launch_batch_back_primal(const SlotDesc *slots, const SlotStatus *status, WorkList wl, bool block,
                                    bool wide, double2 *partial, hipStream_t st);
hipError_t launch_batch_tick(const SlotDesc *slots, SlotStatus *status, const double2 *partial, int n_slots,
                             hipStream_t st);

}  // namespace osscir
