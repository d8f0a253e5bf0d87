// Batched MOCCA: many independent scans (slots) advanced by one launch per
// stage.  Device-side slot descriptors, per-slot status and the work lists
// the batched kernels walk (batch.hip), and their launchers.
#pragma once

#include "kernels.h"

namespace osscir {

constexpr int kSlotEmpty = 0, kSlotRunning = 1, kSlotDone = 2;
constexpr int kMaxSlots = 256;
constexpr int kItemSlotShift = 24;  // work item = slot << 24 | item index within the slot
constexpr int kItemLocalMask = (1 << kItemSlotShift) - 1;
constexpr int kListHeader = 16;     // ints before the items: per-XCD counts (8) and padding

// Everything the batched kernels need of one slot: the plan's scan, the
// caller's state buffers and the slot's regions of the caller workspace.
struct SlotDesc {
  ScanDesc sd;
  float *f, *fbar, *y;
  const float *c;
  float *p, *qS;          // [3][L], [L][12]
  float4 *pk_xy, *pk_yx;  // packed fbar (zero border of kPad)
  float lambda;
  int first_tile;         // the slot's first entry in the per-tile partial sums
  int n_tiles;            // 16 x 16 tiles of the image
  int pad;
};

// Device-owned progress of a slot.  The end-of-iteration kernel advances
// iters, stores the relative change of f and marks the slot done once
// iters reaches max_iter (> 0) or the change falls to tol (> 0); the stage
// kernels skip slots that are not running.
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
hipError_t launch_batch_spectral_dual(const SlotDesc *slots, const SlotStatus *status, WorkList wl,
                                      int rays_per_wg, size_t lds, bool clip, bool block, bool fp64, hipStream_t st);
hipError_t launch_batch_back_primal(const SlotDesc *slots, const SlotStatus *status, WorkList wl, bool block,
                                    bool wide, double2 *partial, hipStream_t st);
hipError_t launch_batch_tick(const SlotDesc *slots, SlotStatus *status, const double2 *partial, int n_slots,
                             hipStream_t st);

}  // namespace osscir
