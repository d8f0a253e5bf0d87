// Host-side internals shared by the library's C-ABI translation units: the
// plan object, the caller workspace layout and the error helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "device_math.h"
#include "kernels.h"
#include "osscir.h"

struct osscir_plan_s {
  int device = -1;
  osscir::ScanDesc sd{};
  osscir::RayLine *d_rays = nullptr;
  osscir::ViewGeom *d_views = nullptr;
  void *d_pack = nullptr;  // packed-image scratch of the standalone projector calls
  float *d_rho = nullptr;
  float *d_tab = nullptr;
  float4 *d_sbin = nullptr;   // per-detector-bin responses [I][D]
  float4 *d_n0bin = nullptr;  // per-detector-bin incident counts [D]
  float4 *d_n0ray = nullptr;  // per-ray incident counts [L] (optional)
  int *d_tile_order = nullptr;  // back-projection tiles in region order
  float4 *d_zero = nullptr;     // 256 zero bytes the back-projector stages for empty slots
  osscir::TileBins *d_tile_bins = nullptr;  // staged bins per (tile, view) of the common back-projection path
};

namespace osscir {

// Sets the thread's last-error message and returns code.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char *what);
void clear_error();
int check_plan(osscir_plan plan);

#define OSSCIR_HIP(call, what)                                  \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return ::osscir::hip_fail(e_, what);  \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Caller workspace regions: p [3][L] f32 | qS [L][12] f32 (q and the step
// terms interleaved per ray; planar scratch for the standalone step calls) |
// partial sums (f64) | packed images of the forward projector | with
// bp_parts > 1, the split back-projection's sums [part][9][n * n] f64.
struct WorkLayout {
  size_t p = 0, qS = 0, partial = 0, pack = 0, bp = 0, total = 0;  // bp: split back-projection sums (bp_parts > 1)
};
WorkLayout work_layout(const ScanDesc &sd);

// The 16 x 16 back-projection tiles (index ty * nt + tx) in region order:
// the image split into 4 bands of rows x 2 halves of columns, regions one
// after the other, row-major inside; consecutive eighths of this order are
// compact blocks of the image (one per XCD).  cus_per_xcd > 0 (one launch
// of every tile): the eighths are instead sectors around the image centre,
// each re-dealt so that the tiles one CU receives (positions congruent
// modulo cus_per_xcd) mix outer and inner tiles.
std::vector<int> region_tile_order(int nt, int cus_per_xcd = 0);

// The per-view sources and per-ray line parameters of a (validated) geometry.
void build_ray_table(const osscir_geometry &g, std::vector<RayLine> &rays, std::vector<ViewGeom> &views);

}  // namespace osscir
