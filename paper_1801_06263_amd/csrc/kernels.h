// Kernel-side data layouts and launch helpers shared by the library's
// translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace osscir {

struct RayLine;

// Bins of one view staged for one 16 x 16 back-projection tile (common
// path): the rays that can meet the tile are bins d0 .. d0 + nst - 1, a
// pixel's window starts at staged index floor(bin_scale t + off) (t its
// centre's detector coordinate) and holds K bins.  One per (tile, view),
// computed once per plan.
struct TileBins {
  int d0, nst, K;
  float off;
};

// Per-view geometry: source position in pixel index coordinates (pixel
// (ix, iy) centred at (ix, iy)), and the view direction for the detector
// projection of pixel corners.
struct ViewGeom {
  double sx, sy;
  float cb, sb, pad0, pad1;
};

constexpr int kMat = 3;   // materials (block SPC works on 3x3 blocks)
constexpr int kWin = 4;   // energy windows
constexpr int kTab = 48;  // floats per energy in the spectral table
constexpr int kPad = 4;   // zero border of the packed images of the forward projector

// Spectral table, one row of kTab floats per energy i:
//   [0..2]   mu_{m,i}
//   [3..6]   s_{w,i}
//   [7..18]  s_{w,i} mu_{m,i}                  (index 7 + 3w + m)
//   [19..42] s_{w,i} mu_{m,i} mu_{n,i}, m <= n (index 19 + 6w + upper(m,n))
//   [43..47] zero
constexpr int kTabMu = 0, kTabS = 3, kTabSMu = 7, kTabSMuMu = 19;
// With per-detector-bin responses the rows hold mu (0..2) and the products
// mu_{m,i} mu_{n,i}, m <= n (7..12); the responses s_{w,d,i} are a separate
// float4 array [I][D] (one 16-byte load per lane and energy, coalesced over
// neighbouring bins).
constexpr int kTabMuMu = 7;

// LDS floats per wave of the matrix-core energy sums' transposition tiles
// (64 rays x 16 columns, +1 against bank conflicts).
constexpr int kMfmaTileFloats = 64 * 17;

// Energies of the matrix-core sums are padded with zero rows to a multiple
// of 8 (two 4-energy steps per loop iteration).
__host__ __device__ inline int mfma_energies(int n_energy) { return (n_energy + 7) & ~7; }

// LDS bytes of a spectral kernel with the matrix-core energy sums: the
// padded table while the sums run, then the per-wave transposition tiles.
inline size_t mfma_lds_bytes(int n_energy, int waves) {
  const size_t tab = (size_t)mfma_energies(n_energy) * kTab * sizeof(float);
  const size_t tiles = (size_t)waves * kMfmaTileFloats * sizeof(float);
  return tab > tiles ? tab : tiles;
}

// Everything a kernel needs to know about one scan.
struct ScanDesc {
  int n;             // image side
  int n_views;
  int n_bins;
  int n_rays;        // n_views * n_bins
  int n_energy;
  float c0;          // (n - 1) / 2
  float sid_px;      // source-isocentre distance, pixel units
  float bin_scale;   // sdd / bin pitch (bins per unit tan)
  float cbin;        // (n_bins - 1) / 2
  float n0[kWin];    // incident counts per window
  int bp_wide;       // some 16x16-tile shadow exceeds the back-projector's staging buffer
  int bp_copy;       // enough workgroups for four per CU: the fused step stages by global-to-LDS copies
  int bp_parts;      // the fused back-projection's views split over this many workgroups per tile (grids of few
                     // tiles), their FP64 sums added in order; 1: one workgroup per tile
  int bp_part_views; // views per part: a multiple of 8 (n_views when bp_parts == 1)
  int per_bin;       // window responses and incident counts per detector bin
  int mfma;          // energy sums on the matrix cores (shared table, fits LDS)
  const float4 *sbin;   // [I][D] s_{w,d,i} (w = x, y, z, w), per_bin only
  const float4 *n0bin;  // [D] incident counts per window, per_bin only
  const float4 *n0ray;  // [L] incident counts per window of every ray (replaces n0 / n0bin), or null
  const int *tile_order;  // [nt * nt] back-projection tiles (ty * nt + tx) in launch order (region_tile_order)
  const TileBins *tile_bins;  // [nt * nt][V] staged bins per (tile, view); null on the wide path
  const float4 *zero;     // 256 bytes of zeros (a null ray record and null inputs)
  const struct RayLine *rays;  // [L]
  const ViewGeom *views;        // [V]
  const float *rho;     // [L]
  const float *tab;     // [I][kTab]
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  xcd_item remaps the flat workgroup index so that XCD x processes the
// contiguous range x of the items: the forward projector's items are (view,
// bin-chunk) pairs, so an XCD takes an arc of views whose rays mostly share
// one major axis and hence one packed copy; the back-projector's items are
// tiles in region order (ScanDesc::tile_order), so an XCD takes a compact
// block of the image and fetches each view's bins into its L2 once.
constexpr int kXcds = 8;

__device__ __forceinline__ bool xcd_item(int nitems, int &item) {
  const int b = blockIdx.x;
  const int per = (nitems + kXcds - 1) / kXcds;
  item = (b % kXcds) * per + b / kXcds;
  return item < nitems;
}

// Pointers into the constant address space: loads through them at a
// uniform address become scalar-cache loads into SGPRs, also after stores
// of the same kernel (the memory is read-only for the kernel's lifetime:
// tables, descriptors, work lists).
#define OSSCIR_CONST __attribute__((address_space(4)))
// Pointers into LDS (the destination of global-to-LDS loads).
#define OSSCIR_LDS __attribute__((address_space(3)))
// Last word of a raw buffer descriptor on gfx9-family GPUs (32-bit data
// format, no swizzle): loads through it read bytes [0, num_records) of the
// base address, with the offsets the instruction gives.
constexpr int kBufferRsrcWord3 = 0x00020000;

template <typename T>
__device__ __forceinline__ const OSSCIR_CONST T *as_const(const T *p) {
  return (const OSSCIR_CONST T *)p;
}

// A pointer loaded from memory is generic (flat loads and stores); the
// round trip through the global address space lets the compiler use global
// memory instructions for it.
template <typename T>
__device__ __forceinline__ T *as_global(T *p) {
  return (T *)(__attribute__((address_space(1))) T *)p;
}

// A copy of *p read word by word through the scalar cache (p uniform over
// the wave); words the caller never uses are not loaded.
template <typename T>
__device__ __forceinline__ T load_uniform(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized structs only");
  const OSSCIR_CONST int *q = (const OSSCIR_CONST int *)p;
  T out;
  int *o = reinterpret_cast<int *>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) o[i] = q[i];
  return out;
}

}  // namespace osscir
