// Launchers of the projector kernels (projector.hip).
#pragma once

#include "kernels.h"

namespace osscir {

// Bytes of the packed-image scratch the forward projector needs.
size_t pack_scratch_bytes(const ScanDesc &sd);

// p[c][l] = sum_k X_{l,k} f[c][k], c < nch (chunks of up to 3 channels);
// pack: device scratch of pack_scratch_bytes().
hipError_t launch_forward(const ScanDesc &sd, const float *f, int nch, float *p, void *pack, hipStream_t st);

// p[c][l] for c < 3 from images already packed by launch_pack (or by the
// primal step's packing epilogue).
hipError_t launch_forward_packed(const ScanDesc &sd, const void *pack, float *p, hipStream_t st);

// Packs up to 3 channels of f into the two padded images of pack (the
// layout launch_forward uses): row-contiguous copy first, then the
// column-contiguous one.
hipError_t launch_pack(const ScanDesc &sd, const float *f, int nch, void *pack, hipStream_t st);

// b[c][k] = sum_l X_{l,k} q[c][l] (chunks of 9, 6, 3, 2 or 1 channels).
hipError_t launch_back(const ScanDesc &sd, const float *q, int nch, float *b, hipStream_t st);

// The common back-projection path's staged bins of every (tile, view):
// tile_bins_count(sd) entries, tiles row-major, views fastest (plan setup).
size_t tile_bins_count(const ScanDesc &sd);
hipError_t launch_tile_bins(const ScanDesc &sd, TileBins *out, hipStream_t st);

// Workgroups of the tile-driven back-projection kernels (all tiles of the
// image in ScanDesc::tile_order, XCD-partitioned).
unsigned back_blocks(const ScanDesc &sd);

// nnz[l] = number of pixels with a non-zero weight on ray l.
hipError_t launch_count(const ScanDesc &sd, int *nnz, hipStream_t st);

}  // namespace osscir
