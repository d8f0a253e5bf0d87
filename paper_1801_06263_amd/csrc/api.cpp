// The library's C ABI (include/osscir.h): plan construction on the host in
// FP64, validation, workspace layout and the per-iteration launch sequence.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "device_math.h"
#include "kernels.h"
#include "osscir.h"
#include "plan.h"
#include "projector.h"
#include "project_device.h"
#include "spectral.h"

using namespace osscir;

namespace {
thread_local std::string g_last_error;
}  // namespace

int osscir::fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int osscir::hip_fail(hipError_t e, const char *what) {
  return fail(OSSCIR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void osscir::clear_error() { g_last_error.clear(); }

WorkLayout osscir::work_layout(const ScanDesc &sd) {
  WorkLayout w;
  const size_t L = (size_t)sd.n_rays;
  w.p = 0;
  w.qS = align256(w.p + 3 * L * sizeof(float));
  w.partial = align256(w.qS + 12 * L * sizeof(float));
  w.pack = align256(w.partial + (size_t)dtpl_partial_count(sd) * sizeof(double));
  w.bp = align256(w.pack + pack_scratch_bytes(sd));
  const size_t bp_bytes = sd.bp_parts > 1 ? (size_t)sd.bp_parts * 9 * (size_t)sd.n * sd.n * sizeof(double) : 0;
  w.total = align256(w.bp + bp_bytes);
  return w;
}

std::vector<int> osscir::region_tile_order(int nt, int cus_per_xcd) {
  std::vector<int> order;
  order.reserve((size_t)nt * nt);
  const int rb = (nt + 3) / 4, cb = (nt + 1) / 2;
  for (int band = 0; band < 4; ++band)
    for (int half = 0; half < 2; ++half)
      for (int ty = band * rb; ty < std::min(nt, (band + 1) * rb); ++ty)
        for (int tx = half * cb; tx < std::min(nt, (half + 1) * cb); ++tx) order.push_back(ty * nt + tx);
  if (cus_per_xcd < 1) return order;
  // Balanced for one launch of every tile: a tile's window work over a full
  // orbit grows with its distance from the rotation centre (the outer tiles
  // pass closer to the source, where their shadows are wider; at 512^2 the
  // corner tiles have 1.2x the mean work and the centre ones 0.88x).  The
  // eighths become sectors around the centre (tiles by angle), so every XCD
  // gets the same mix of radii, and within an eighth the tiles at positions
  // congruent modulo the XCD's CU count, which one CU receives, are dealt
  // in a snake over the tiles ranked by radius: each CU takes one tile from
  // every row of ranks, heavy and light alike.
  const int S = cus_per_xcd, n = nt * nt, per = (n + kXcds - 1) / kXcds;
  const double c = 0.5 * nt;
  auto r2 = [&](int t) {
    const double dx = (t % nt) + 0.5 - c, dy = (t / nt) + 0.5 - c;
    return dx * dx + dy * dy;
  };
  auto angle = [&](int t) { return std::atan2((t / nt) + 0.5 - c, (t % nt) + 0.5 - c); };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return angle(a) < angle(b); });
  std::vector<int> out(order);
  for (int x0 = 0; x0 < n; x0 += per) {
    const int m = std::min(per, n - x0);
    std::vector<int> rank(order.begin() + x0, order.begin() + x0 + m);
    std::stable_sort(rank.begin(), rank.end(), [&](int a, int b) { return r2(a) > r2(b); });
    for (int r = 0; r < m; ++r) {
      const int q = r / S, k = r % S;
      const bool full_row = (q + 1) * S <= m;  // a partial last row keeps its order (its positions stay below m)
      const int g = (q % 2 == 1 && full_row) ? S - 1 - k : k;
      out[x0 + q * S + g] = rank[r];
    }
  }
  return out;
}

int osscir::check_plan(osscir_plan plan) {
  if (!plan) return fail(OSSCIR_EINVAL, "null plan");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
    return fail(OSSCIR_EINVAL, "plan was created on device %d, current device is %d", plan->device, dev);
  return OSSCIR_OK;
}

namespace {

void free_plan(osscir_plan p) {
  if (!p) return;
  if (p->d_rays) (void)hipFree(p->d_rays);
  if (p->d_views) (void)hipFree(p->d_views);
  if (p->d_rho) (void)hipFree(p->d_rho);
  if (p->d_tab) (void)hipFree(p->d_tab);
  if (p->d_pack) (void)hipFree(p->d_pack);
  if (p->d_sbin) (void)hipFree(p->d_sbin);
  if (p->d_n0bin) (void)hipFree(p->d_n0bin);
  if (p->d_n0ray) (void)hipFree(p->d_n0ray);
  if (p->d_tile_order) (void)hipFree(p->d_tile_order);
  if (p->d_zero) (void)hipFree(p->d_zero);
  if (p->d_tile_bins) (void)hipFree(p->d_tile_bins);
  delete p;
}

// cos and sin of a view angle, exact (0 and +-1) where the angle is a
// multiple of pi/2: the detector-centre ray of such a view is parallel to an
// image axis, which FP64's cos(pi/2) ~ 6e-17 would turn by rounding alone.
void view_cos_sin(double beta, double &cb, double &sb) {
  cb = std::cos(beta);
  sb = std::sin(beta);
  const bool zc = std::fabs(cb) < 1e-12, zs = std::fabs(sb) < 1e-12;
  if (zc) cb = 0.0, sb = sb > 0 ? 1.0 : -1.0;
  if (zs) sb = 0.0, cb = cb > 0 ? 1.0 : -1.0;
}

// Smallest |t_x t_y| of a ray direction the trapezoid weight is evaluated
// with.  A ray closer to an image axis (exactly parallel at the cardinal
// views) is turned about its source until its minor-axis component is
// +kMinTilt: inside the image it then lies at most ~kMinTilt * 60 cm (well
// under 1e-5 cm) to the + side of the exact line, so a line lying exactly on
// a shared pixel edge is counted once, in the pixel on its + side (pixels
// are half-open), and every weight stays exact with a finite trapezoid slope
// kappa = h / |t_x t_y| <= 8.4e6 h, whose FP32 constants still resolve the
// line's distance from each pixel edge.
constexpr double kMinTilt = 1.0 / 8388608.0;  // 2^-23

}  // namespace

// Per-view source position and per-ray line parameters, in pixel index
// coordinates (pixel (ix, iy) centred at (ix, iy)): normals scaled by kappa
// in FP64, the trapezoid constants rounded to FP32.
void osscir::build_ray_table(const osscir_geometry &g, std::vector<RayLine> &rays, std::vector<ViewGeom> &views) {
  const int V = g.n_views, D = g.n_bins, N = g.n;
  const double h = g.pixel_cm, c0 = 0.5 * (N - 1);
  rays.resize((size_t)V * D);
  views.resize(V);
  for (int v = 0; v < V; ++v) {
    double cb, sb;
    view_cos_sin(g.view0_rad + g.arc_rad * (double)v / (double)V, cb, sb);
    // the source on a 2^-30-pixel grid: with |s| < 2^22 every offset s - i
    // to an integer pixel index is then exact in FP64, so the kernels may
    // step offsets by whole pixels and still agree bit for bit
    const double sx = std::ldexp(std::nearbyint(std::ldexp(g.sid_cm * cb / h + c0, 30)), -30);
    const double sy = std::ldexp(std::nearbyint(std::ldexp(g.sid_cm * sb / h + c0, 30)), -30);
    views[v] = ViewGeom{sx, sy, (float)cb, (float)sb, 0.0f, 0.0f};
    for (int d = 0; d < D; ++d) {
      const double u = ((double)d - 0.5 * (D - 1)) * g.bin_cm;
      const double px = (-(g.sdd_cm - g.sid_cm) * cb - u * sb) / h + c0;
      const double py = (-(g.sdd_cm - g.sid_cm) * sb + u * cb) / h + c0;
      double tx = px - sx, ty = py - sy;
      const double len = std::sqrt(tx * tx + ty * ty);
      tx /= len;
      ty /= len;
      if (std::fabs(tx) * std::fabs(ty) < kMinTilt) {
        const double major = std::sqrt(1.0 - kMinTilt * kMinTilt);
        if (std::fabs(tx) >= std::fabs(ty)) {
          tx = tx > 0 ? major : -major;
          ty = kMinTilt;
        } else {
          ty = ty > 0 ? major : -major;
          tx = kMinTilt;
        }
      }
      const double nx = -ty, ny = tx;
      const double anx = std::fabs(nx), any = std::fabs(ny);
      const double a = 0.5 * (anx + any);
      const double hmax = h / std::max(anx, any);
      const double kappa = h / (anx * any);
      rays[(size_t)v * D + d] = RayLine{nx * kappa, ny * kappa, (float)(a * kappa), (float)hmax, (float)kappa, 0.0f};
    }
  }
}

namespace {

int check_geometry(const osscir_geometry &g) {
  if (g.n < 1 || g.n > 4096) return fail(OSSCIR_EINVAL, "image size n=%d outside [1, 4096]", g.n);
  if (g.n_views < 1 || g.n_bins < 1) return fail(OSSCIR_EINVAL, "need n_views >= 1 and n_bins >= 1");
  if ((int64_t)g.n_views * g.n_bins >= ((int64_t)1 << 31) / 16)
    return fail(OSSCIR_EINVAL, "too many rays (%d x %d)", g.n_views, g.n_bins);
  if (!(g.pixel_cm > 0) || !(g.bin_cm > 0) || !std::isfinite(g.view0_rad) || !std::isfinite(g.arc_rad))
    return fail(OSSCIR_EINVAL, "pixel_cm and bin_cm must be > 0, angles finite");
  const double half_diag = g.n * g.pixel_cm / std::sqrt(2.0);
  if (!(g.sid_cm > half_diag * 1.0001) || !(g.sdd_cm > g.sid_cm + half_diag * 1.0001))
    return fail(OSSCIR_EINVAL, "source and detector must lie outside the image circumcircle");
  if (!(g.sid_cm / g.pixel_cm + g.n < 4194304.0))
    return fail(OSSCIR_EINVAL, "source farther than 2^22 pixels from the image");
  return OSSCIR_OK;
}

}  // namespace

extern "C" {

const char *osscir_last_error(void) { return g_last_error.c_str(); }

const char *osscir_version(void) { return "osscir 0.1 gfx950"; }

int osscir_plan_create(const osscir_geometry *geom, const osscir_spectral *spec, osscir_plan *out) {
  g_last_error.clear();
  if (!out) return fail(OSSCIR_EINVAL, "null output plan pointer");
  *out = nullptr;
  if (!geom || !spec) return fail(OSSCIR_EINVAL, "null geometry or spectral description");
  const osscir_geometry g = *geom;
  if (int rc = check_geometry(g)) return rc;
  if (spec->n_mat != kMat || spec->n_win != kWin)
    return fail(OSSCIR_EINVAL, "supported: n_mat=3, n_win=4 (got %d, %d)", spec->n_mat, spec->n_win);
  const int I = spec->n_energy;
  if (I < 1 || I > 512) return fail(OSSCIR_EINVAL, "n_energy=%d outside [1, 512]", I);
  if (!spec->mu || !spec->s || !spec->n0) return fail(OSSCIR_EINVAL, "null spectral table");
  const int n_resp = spec->n_resp <= 1 ? 1 : spec->n_resp;
  if (n_resp != 1 && n_resp != g.n_bins)
    return fail(OSSCIR_EINVAL, "n_resp=%d must be 0, 1 or n_bins=%d", spec->n_resp, g.n_bins);
  for (int r = 0; r < n_resp; ++r)
    for (int w = 0; w < kWin; ++w) {
      double sum = 0;
      for (int i = 0; i < I; ++i) {
        const double v = spec->s[((size_t)r * kWin + w) * I + i];
        if (!(v >= 0) || !std::isfinite(v))
          return fail(OSSCIR_EINVAL, "s[%d][%d][%d] negative or not finite", r, w, i);
        sum += v;
      }
      if (std::fabs(sum - 1.0) > 1e-6)
        return fail(OSSCIR_EINVAL, "row (%d, %d) of s sums to %.9g, not 1", r, w, sum);
      const double n0 = spec->n0[(size_t)r * kWin + w];
      if (!(n0 > 0) || !std::isfinite(n0)) return fail(OSSCIR_EINVAL, "n0[%d][%d] must be > 0", r, w);
    }
  for (int j = 0; j < kMat * I; ++j)
    if (!std::isfinite(spec->mu[j])) return fail(OSSCIR_EINVAL, "mu not finite");
  if (spec->n0_ray)
    for (size_t j = 0; j < (size_t)g.n_views * g.n_bins * kWin; ++j)
      if (!(spec->n0_ray[j] > 0) || !std::isfinite(spec->n0_ray[j]))
        return fail(OSSCIR_EINVAL, "n0_ray[%zu] must be > 0 and finite", j);

  osscir_plan p = new (std::nothrow) osscir_plan_s;
  if (!p) return fail(OSSCIR_ENOMEM, "host allocation failed");
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(OSSCIR_EDEVICE, "no HIP device");
  }
  const int V = g.n_views, D = g.n_bins, N = g.n;
  const size_t L = (size_t)V * D;
  const double h = g.pixel_cm;

  std::vector<RayLine> rays;
  std::vector<ViewGeom> views;
  build_ray_table(g, rays, views);
  const double c0 = 0.5 * (N - 1);
  // spectral table: shared responses folded with mu, or (per detector bin)
  // mu and its products here and the responses in a per-bin array
  const bool per_bin = n_resp > 1;
  std::vector<float> tab((size_t)I * kTab, 0.0f);
  std::vector<float4> sbin, n0bin;
  for (int i = 0; i < I; ++i) {
    float *t = &tab[(size_t)i * kTab];
    const double mu[3] = {spec->mu[0 * I + i], spec->mu[1 * I + i], spec->mu[2 * I + i]};
    for (int m = 0; m < 3; ++m) t[kTabMu + m] = (float)mu[m];
    if (per_bin) {
      int k = 0;
      for (int m = 0; m < 3; ++m)
        for (int n = m; n < 3; ++n) t[kTabMuMu + (k++)] = (float)(mu[m] * mu[n]);
      continue;
    }
    for (int w = 0; w < kWin; ++w) {
      const double s = spec->s[w * I + i];
      t[kTabS + w] = (float)s;
      for (int m = 0; m < 3; ++m) t[kTabSMu + 3 * w + m] = (float)(s * mu[m]);
      int k = 0;
      for (int m = 0; m < 3; ++m)
        for (int n = m; n < 3; ++n) t[kTabSMuMu + 6 * w + (k++)] = (float)(s * mu[m] * mu[n]);
    }
  }
  if (per_bin) {
    sbin.resize((size_t)I * D);
    n0bin.resize(D);
    for (int d = 0; d < D; ++d) {
      const double *sd_ = spec->s + (size_t)d * kWin * I;
      for (int i = 0; i < I; ++i)
        sbin[(size_t)i * D + d] = make_float4((float)sd_[0 * I + i], (float)sd_[1 * I + i], (float)sd_[2 * I + i],
                                              (float)sd_[3 * I + i]);
      const double *n0 = spec->n0 + (size_t)d * kWin;
      n0bin[d] = make_float4((float)n0[0], (float)n0[1], (float)n0[2], (float)n0[3]);
    }
  }

  std::vector<float4> n0ray;
  if (spec->n0_ray) {
    n0ray.resize(L);
    for (size_t l = 0; l < L; ++l) {
      const double *n0 = spec->n0_ray + l * kWin;
      n0ray[l] = make_float4((float)n0[0], (float)n0[1], (float)n0[2], (float)n0[3]);
    }
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || cus < 1) cus = 256;
  const std::vector<int> tiles = region_tile_order((N + kBpTile - 1) / kBpTile, std::max(1, cus / kXcds));
  hipError_t e;
  if ((e = hipMalloc(&p->d_rays, rays.size() * sizeof(RayLine))) != hipSuccess ||
      (e = hipMalloc(&p->d_views, views.size() * sizeof(ViewGeom))) != hipSuccess ||
      (e = hipMalloc(&p->d_pack, 2 * (size_t)(N + 2 * kPad) * (N + 2 * kPad) * sizeof(float4))) != hipSuccess ||
      (e = hipMalloc(&p->d_rho, L * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&p->d_tab, tab.size() * sizeof(float))) != hipSuccess ||
      (per_bin && (e = hipMalloc(&p->d_sbin, sbin.size() * sizeof(float4))) != hipSuccess) ||
      (per_bin && (e = hipMalloc(&p->d_n0bin, n0bin.size() * sizeof(float4))) != hipSuccess) ||
      (!n0ray.empty() && (e = hipMalloc(&p->d_n0ray, n0ray.size() * sizeof(float4))) != hipSuccess) ||
      (e = hipMalloc(&p->d_tile_order, tiles.size() * sizeof(int))) != hipSuccess ||
      (e = hipMalloc(&p->d_zero, 256)) != hipSuccess) {
    free_plan(p);
    return fail(OSSCIR_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
  }
  if ((e = hipMemcpy(p->d_rays, rays.data(), rays.size() * sizeof(RayLine), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->d_views, views.data(), views.size() * sizeof(ViewGeom), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(p->d_tab, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (per_bin &&
       (e = hipMemcpy(p->d_sbin, sbin.data(), sbin.size() * sizeof(float4), hipMemcpyHostToDevice)) != hipSuccess) ||
      (per_bin && (e = hipMemcpy(p->d_n0bin, n0bin.data(), n0bin.size() * sizeof(float4), hipMemcpyHostToDevice)) !=
                      hipSuccess) ||
      (!n0ray.empty() &&
       (e = hipMemcpy(p->d_n0ray, n0ray.data(), n0ray.size() * sizeof(float4), hipMemcpyHostToDevice)) != hipSuccess) ||
      (e = hipMemcpy(p->d_tile_order, tiles.data(), tiles.size() * sizeof(int), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemset(p->d_zero, 0, 256)) != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "copying plan tables");
  }
  ScanDesc &sd = p->sd;
  sd.n = N;
  sd.n_views = V;
  sd.n_bins = D;
  sd.n_rays = (int)L;
  sd.n_energy = I;
  sd.c0 = 0.5f * (float)(N - 1);
  sd.sid_px = (float)(g.sid_cm / h);
  sd.bin_scale = (float)(g.sdd_cm / g.bin_cm);
  sd.cbin = 0.5f * (float)(D - 1);
  for (int w = 0; w < kWin; ++w) sd.n0[w] = (float)spec->n0[w];
  sd.per_bin = per_bin ? 1 : 0;
  sd.mfma = !per_bin && mfma_lds_bytes(I, 8) <= 65536 ? 1 : 0;
  sd.tile_order = p->d_tile_order;
  sd.zero = p->d_zero;
  sd.sbin = p->d_sbin;
  sd.n0bin = p->d_n0bin;
  sd.n0ray = p->d_n0ray;
  // does any 16x16 tile's shadow exceed a staging slot of the back-projector's
  // grouped path?
  // (the same corner projection the kernel uses, in FP64 with a margin)
  sd.bp_wide = 0;
  {
    const int nt = (N + kBpTile - 1) / kBpTile;
    for (int v = 0; v < V && !sd.bp_wide; ++v) {
      const double cb = views[v].cb, sb = views[v].sb;
      for (int ty = 0; ty < nt && !sd.bp_wide; ++ty)
        for (int tx = 0; tx < nt; ++tx) {
          double lo = 1e300, hi = -1e300;
          for (int k = 0; k < 4; ++k) {
            const double X = tx * kBpTile - c0 - 0.5 + ((k & 1) ? kBpTile : 0);
            const double Y = ty * kBpTile - c0 - 0.5 + ((k & 2) ? kBpTile : 0);
            const double t = (-sb * X + cb * Y) / (g.sid_cm / h - cb * X - sb * Y);
            lo = std::min(lo, t);
            hi = std::max(hi, t);
          }
          const double span = (hi - lo) * (g.sdd_cm / g.bin_cm) + 3.0;
          if (span > kBpSlot - 2) {
            sd.bp_wide = 1;
            break;
          }
        }
    }
  }
  // global-to-LDS staging in the fused back-projection when the tiles fill
  // four workgroups per CU (measured: 4% faster at 1024 tiles on 256 CUs,
  // 8-10% slower at 256 tiles and fewer)
  // A grid of at most two tiles per CU leaves the CUs nearly empty (one
  // 16 x 16 tile is four waves): its views are then split into parts, one
  // workgroup per (tile, part), aiming at four workgroups per CU; a part is
  // a whole number of 8-view FP32 flushes.  Global-to-LDS staging in the
  // fused back-projection when the workgroups fill four per CU (measured:
  // 4% faster at 1024 tiles on 256 CUs, 8-10% slower at 256 tiles and fewer).
  {
    const int nt = (N + kBpTile - 1) / kBpTile, tiles = nt * nt;
    sd.bp_parts = 1;
    sd.bp_part_views = V;
    if (!sd.bp_wide && tiles <= 2 * cus) {
      const int want = (4 * cus + tiles - 1) / tiles;
      const int vp = ((V + want - 1) / want + 7) / 8 * 8;
      const int parts = (V + vp - 1) / vp;
      if (parts > 1) {
        sd.bp_parts = parts;
        sd.bp_part_views = vp;
      }
    }
    sd.bp_copy = tiles * sd.bp_parts >= 4 * cus ? 1 : 0;
  }
  sd.rays = p->d_rays;
  sd.views = p->d_views;
  sd.rho = p->d_rho;
  sd.tab = p->d_tab;
  sd.tile_bins = nullptr;
  if (!sd.bp_wide) {
    // staged bins of every (tile, view), once per plan
    if ((e = hipMalloc(&p->d_tile_bins, tile_bins_count(sd) * sizeof(TileBins))) != hipSuccess) {
      free_plan(p);
      return fail(OSSCIR_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    if ((e = launch_tile_bins(sd, p->d_tile_bins, nullptr)) != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "tabulating the back-projection tiles");
    }
    sd.tile_bins = p->d_tile_bins;
  }

  // rho = X 1 with the library's own projector
  float *ones = nullptr;
  if ((e = hipMalloc(&ones, (size_t)N * N * sizeof(float))) != hipSuccess) {
    free_plan(p);
    return fail(OSSCIR_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
  }
  std::vector<float> h_ones((size_t)N * N, 1.0f);
  e = hipMemcpy(ones, h_ones.data(), h_ones.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_forward(sd, ones, 1, p->d_rho, p->d_pack, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipFree(ones);
  if (e != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "computing ray lengths");
  }
  *out = p;
  return OSSCIR_OK;
}

int osscir_ray_table(const osscir_geometry *geom, double *rays, double *src) {
  clear_error();
  if (!geom || !rays || !src) return fail(OSSCIR_EINVAL, "ray_table: null argument");
  if (int rc = check_geometry(*geom)) return rc;
  std::vector<RayLine> rt;
  std::vector<ViewGeom> vt;
  build_ray_table(*geom, rt, vt);
  for (size_t l = 0; l < rt.size(); ++l) {
    double *o = rays + 6 * l;
    o[0] = rt[l].nxk;
    o[1] = rt[l].nyk;
    o[2] = rt[l].ak;
    o[3] = rt[l].hmax;
    o[4] = rt[l].kappa;
    o[5] = 0.0;
  }
  for (size_t v = 0; v < vt.size(); ++v) {
    src[2 * v] = vt[v].sx;
    src[2 * v + 1] = vt[v].sy;
  }
  return OSSCIR_OK;
}

int osscir_plan_set_energy_sums(osscir_plan plan, int32_t matrix_cores) {
  int rc = check_plan(plan);
  if (rc) return rc;
  ScanDesc &sd = plan->sd;
  if (matrix_cores) {
    if (sd.per_bin || mfma_lds_bytes(sd.n_energy, 8) > 65536)
      return fail(OSSCIR_EINVAL,
                  "energy sums on the matrix cores need one shared response table within 64 KB of LDS "
                  "(per-bin responses or %d energies)", sd.n_energy);
    sd.mfma = 1;
  } else {
    sd.mfma = 0;
  }
  return OSSCIR_OK;
}

int osscir_plan_destroy(osscir_plan plan) {
  if (!plan) return OSSCIR_OK;
  (void)hipDeviceSynchronize();
  free_plan(plan);
  return OSSCIR_OK;
}

int osscir_workspace_bytes(osscir_plan plan, size_t *bytes) {
  if (!plan || !bytes) return fail(OSSCIR_EINVAL, "null argument");
  *bytes = work_layout(plan->sd).total;
  return OSSCIR_OK;
}

int osscir_batch_workspace_bytes(osscir_plan plan, size_t *bytes) {
  if (!plan || !bytes) return fail(OSSCIR_EINVAL, "null argument");
  *bytes = work_layout(plan->sd).bp;  // everything before the split back-projection's region
  return OSSCIR_OK;
}

int osscir_ray_lengths(osscir_plan plan, float *rho, osscir_stream stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!rho) return fail(OSSCIR_EINVAL, "null rho");
  OSSCIR_HIP(hipMemcpyAsync(rho, plan->d_rho, (size_t)plan->sd.n_rays * sizeof(float), hipMemcpyDeviceToDevice,
                            (hipStream_t)stream),
             "copying rho");
  return OSSCIR_OK;
}

int osscir_forward_project(osscir_plan plan, const float *f, int32_t n_ch, float *p, osscir_stream stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!f || !p || n_ch < 1) return fail(OSSCIR_EINVAL, "forward_project: null pointer or n_ch < 1");
  OSSCIR_HIP(launch_forward(plan->sd, f, n_ch, p, plan->d_pack, (hipStream_t)stream), "forward_project launch");
  return OSSCIR_OK;
}

int osscir_back_project(osscir_plan plan, const float *q, int32_t n_ch, float *b, osscir_stream stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!q || !b || n_ch < 1) return fail(OSSCIR_EINVAL, "back_project: null pointer or n_ch < 1");
  OSSCIR_HIP(launch_back(plan->sd, q, n_ch, b, (hipStream_t)stream), "back_project launch");
  return OSSCIR_OK;
}

int osscir_spectral_model(osscir_plan plan, const float *p, const float *c, float *chat, float *r, float *G,
                          float *H, float *Hplus, int32_t fp64_small, osscir_stream stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!p || !c) return fail(OSSCIR_EINVAL, "spectral_model: null p or c");
  OSSCIR_HIP(launch_spectral_model(plan->sd, p, c, chat, r, G, H, Hplus, fp64_small != 0, (hipStream_t)stream),
             "spectral_model launch");
  return OSSCIR_OK;
}

static int steps_common(osscir_plan plan, const float *G, double lambda, float *sigma, float *img, void *work,
                        size_t work_bytes, bool block, osscir_stream stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!G || !sigma || !img || !work) return fail(OSSCIR_EINVAL, "spc_steps: null pointer");
  if (!(lambda > 0) || !std::isfinite(lambda)) return fail(OSSCIR_EINVAL, "lambda must be > 0");
  const WorkLayout wl = work_layout(plan->sd);
  if (work_bytes < wl.total) return fail(OSSCIR_ESTATE, "workspace %zu < %zu bytes", work_bytes, wl.total);
  float *terms = (float *)((char *)work + wl.qS);
  OSSCIR_HIP(launch_steps(plan->sd, G, (float)lambda, block, sigma, terms, img, (hipStream_t)stream),
             "spc_steps launch");
  return OSSCIR_OK;
}

int osscir_block_spc_steps(osscir_plan plan, const float *G, double lambda, float *sigma, float *tinv, void *work,
                           size_t work_bytes, osscir_stream stream) {
  return steps_common(plan, G, lambda, sigma, tinv, work, work_bytes, true, stream);
}

int osscir_diag_spc_steps(osscir_plan plan, const float *G, double lambda, float *sigma, float *tau, void *work,
                          size_t work_bytes, osscir_stream stream) {
  return steps_common(plan, G, lambda, sigma, tau, work, work_bytes, false, stream);
}

namespace {

struct IterArgs {
  float *p, *qS;
  double *partial;
  double *bp;  // split back-projection sums (bp_parts > 1)
  void *pack;
  bool block, clip, fp64;
  float lam;
  const float *pbar = nullptr;  // inner iterations of nested loops: fbar's line integrals (p: the expansion point's)
};

int check_iter(osscir_plan plan, const osscir_params *params, const osscir_state *state, IterArgs *out) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!params || !state) return fail(OSSCIR_EINVAL, "mocca: null params or state");
  if (!state->f || !state->fbar || !state->y || !state->c || !state->work)
    return fail(OSSCIR_EINVAL, "mocca: null state buffer");
  if (!(params->lambda > 0) || !std::isfinite(params->lambda)) return fail(OSSCIR_EINVAL, "lambda must be > 0");
  if (params->precond != OSSCIR_PRECOND_DIAG && params->precond != OSSCIR_PRECOND_BLOCK)
    return fail(OSSCIR_EINVAL, "unknown preconditioner %d", params->precond);
  if (params->curvature != OSSCIR_CURV_WINDOW && params->curvature != OSSCIR_CURV_CLIP)
    return fail(OSSCIR_EINVAL, "unknown curvature %d", params->curvature);
  const WorkLayout wl = work_layout(plan->sd);
  if (state->work_bytes < wl.total)
    return fail(OSSCIR_ESTATE, "workspace %zu < %zu bytes", state->work_bytes, wl.total);
  out->p = (float *)((char *)state->work + wl.p);
  out->qS = (float *)((char *)state->work + wl.qS);
  out->partial = (double *)((char *)state->work + wl.partial);
  out->pack = (char *)state->work + wl.pack;
  out->bp = (double *)((char *)state->work + wl.bp);
  out->block = params->precond == OSSCIR_PRECOND_BLOCK;
  out->clip = params->curvature == OSSCIR_CURV_CLIP;
  out->fp64 = params->fp64_small != 0;
  out->lam = (float)params->lambda;
  return OSSCIR_OK;
}

// packed: the workspace's packed images already hold fbar (written by the
// previous iteration's primal step); pack_next: the primal step writes
// fbar' into them for the next iteration
int run_stage(const ScanDesc &sd, const IterArgs &a, osscir_state *state, int stage, hipStream_t st,
              bool packed = false, bool pack_next = false) {
  switch (stage) {
    case 0:
      if (packed)
        OSSCIR_HIP(launch_forward_packed(sd, a.pack, a.p, st), "mocca: forward projection");
      else
        OSSCIR_HIP(launch_forward(sd, state->fbar, 3, a.p, a.pack, st), "mocca: forward projection");
      break;
    case 1:
      OSSCIR_HIP(launch_spectral_dual(sd, a.p, state->c, state->y, a.qS, a.lam, a.clip, a.block, a.fp64, st, a.pbar),
                 "mocca: spectral model and dual step");
      break;
    case 2:
      OSSCIR_HIP(launch_back_primal(sd, a.qS, state->f, state->fbar, a.lam, a.block, pack_next ? a.pack : nullptr, a.bp,
                                    st),
                 "mocca: back-projection and primal step");
      break;
    default:
      return fail(OSSCIR_EINVAL, "unknown stage %d", stage);
  }
  return OSSCIR_OK;
}

}  // namespace

int osscir_mocca_iterate(osscir_plan plan, const osscir_params *params, osscir_state *state, int32_t n_iter,
                         double *dtpl, osscir_stream stream) {
  IterArgs a;
  int rc = check_iter(plan, params, state, &a);
  if (rc) return rc;
  if (n_iter < 0) return fail(OSSCIR_EINVAL, "n_iter < 0");
  const ScanDesc &sd = plan->sd;
  hipStream_t st = (hipStream_t)stream;
  // without D_TPL (whose forward projection reuses the packed images) the
  // primal step packs fbar' for the next iteration, so only the first
  // iteration of the call runs the packing kernel
  const bool chain = dtpl == nullptr;
  for (int it = 0; it < n_iter; ++it) {
    const bool packed = chain && it > 0, pack_next = chain && it + 1 < n_iter;
    for (int stage = 0; stage < 3; ++stage)
      if ((rc = run_stage(sd, a, state, stage, st, packed, pack_next))) return rc;
    if (dtpl)
      OSSCIR_HIP(launch_dtpl(sd, state->f, state->c, a.p, a.pack, a.partial, dtpl + it, st), "mocca: D_TPL");
  }
  return OSSCIR_OK;
}

int osscir_mocca_iterate_nested(osscir_plan plan, const osscir_params *params, osscir_state *state, int32_t n_outer,
                                int32_t n_inner, float *p0, double *dtpl, osscir_stream stream) {
  IterArgs a;
  int rc = check_iter(plan, params, state, &a);
  if (rc) return rc;
  if (n_outer < 0 || n_inner < 1) return fail(OSSCIR_EINVAL, "nested: need n_outer >= 0 and n_inner >= 1");
  if (n_outer > INT32_MAX / n_inner) return fail(OSSCIR_EINVAL, "nested: n_outer * n_inner overflows");
  if (!p0) return fail(OSSCIR_EINVAL, "nested: null p0");
  const ScanDesc &sd = plan->sd;
  hipStream_t st = (hipStream_t)stream;
  const int total = n_outer * n_inner;
  const bool chain = dtpl == nullptr;  // as in osscir_mocca_iterate
  // the first inner iteration of an outer one is the plain MOCCA step at
  // f0 = fbar, its forward projection kept in p0; the others project fbar
  // into the workspace and take the model from p0
  IterArgs first = a, inner = a;
  first.p = p0;
  inner.pbar = a.p;
  inner.p = p0;
  for (int it = 0; it < total; ++it) {
    const bool packed = chain && it > 0, pack_next = chain && it + 1 < total;
    const bool outer_start = it % n_inner == 0;
    if (outer_start) {
      if ((rc = run_stage(sd, first, state, 0, st, packed, pack_next))) return rc;
      if ((rc = run_stage(sd, first, state, 1, st, packed, pack_next))) return rc;
    } else {
      if ((rc = run_stage(sd, a, state, 0, st, packed, pack_next))) return rc;
      if ((rc = run_stage(sd, inner, state, 1, st, packed, pack_next))) return rc;
    }
    if ((rc = run_stage(sd, a, state, 2, st, packed, pack_next))) return rc;
    if (dtpl)
      OSSCIR_HIP(launch_dtpl(sd, state->f, state->c, a.p, a.pack, a.partial, dtpl + it, st), "mocca: D_TPL");
  }
  return OSSCIR_OK;
}

int osscir_mocca_stage(osscir_plan plan, const osscir_params *params, osscir_state *state, int32_t stage,
                       osscir_stream stream) {
  IterArgs a;
  int rc = check_iter(plan, params, state, &a);
  if (rc) return rc;
  return run_stage(plan->sd, a, state, stage, (hipStream_t)stream);
}

int osscir_mu_pc_basis(const osscir_spectral *spec, double *B, double *mu_out) {
  clear_error();
  if (!spec || !B || !mu_out || !spec->mu || !spec->s) return fail(OSSCIR_EINVAL, "mu_pc_basis: null argument");
  if (spec->n_mat != kMat || spec->n_win < 1) return fail(OSSCIR_EINVAL, "mu_pc_basis: need n_mat = 3, n_win >= 1");
  if (spec->n_resp > 1) return fail(OSSCIR_EINVAL, "mu_pc_basis: needs one shared window response (n_resp <= 1)");
  const int I = spec->n_energy, W = spec->n_win;
  if (I < kMat) return fail(OSSCIR_EINVAL, "mu_pc_basis: need n_energy >= 3");
  // energy weights: the window responses averaged over windows
  std::vector<double> w(I, 0.0);
  for (int i = 0; i < I; ++i) {
    for (int k = 0; k < W; ++k) w[i] += spec->s[k * I + i];
    w[i] /= W;
    if (!(w[i] >= 0) || !std::isfinite(w[i])) return fail(OSSCIR_EINVAL, "mu_pc_basis: bad window response");
  }
  auto dot = [&](const double *u, const double *v) {
    double acc = 0.0;
    for (int i = 0; i < I; ++i) acc += w[i] * u[i] * v[i];
    return acc;
  };
  // Gram-Schmidt of the attenuation rows in material order; row j of B holds
  // the coefficients of the j-th orthonormal function in the original basis
  std::vector<double> q((size_t)kMat * I), v(I);
  double b[kMat][kMat] = {};
  for (int j = 0; j < kMat; ++j) {
    const double *mj = spec->mu + (size_t)j * I;
    for (int i = 0; i < I; ++i) v[i] = mj[i];
    double bj[kMat] = {0.0, 0.0, 0.0};
    bj[j] = 1.0;
    for (int k = 0; k < j; ++k) {
      const double proj = dot(mj, &q[(size_t)k * I]);
      for (int i = 0; i < I; ++i) v[i] -= proj * q[(size_t)k * I + i];
      for (int m = 0; m < kMat; ++m) bj[m] -= proj * b[k][m];
    }
    const double nrm = std::sqrt(dot(v.data(), v.data()));
    if (!(nrm > 1e-10 * std::sqrt(dot(mj, mj))) || !std::isfinite(nrm))
      return fail(OSSCIR_EINVAL, "mu_pc_basis: attenuation rows are linearly dependent under the weights");
    for (int i = 0; i < I; ++i) q[(size_t)j * I + i] = v[i] / nrm;
    for (int m = 0; m < kMat; ++m) b[j][m] = bj[m] / nrm;
  }
  for (int j = 0; j < kMat; ++j)
    for (int m = 0; m < kMat; ++m) B[j * kMat + m] = b[j][m];
  std::memcpy(mu_out, q.data(), q.size() * sizeof(double));
  return OSSCIR_OK;
}

int osscir_material_transform(const double *M, const float *in, float *out, int32_t n_pixels, osscir_stream stream) {
  if (!M || !in || !out || n_pixels < 0) return fail(OSSCIR_EINVAL, "material_transform: null pointer or bad size");
  if (n_pixels == 0) return OSSCIR_OK;
  for (int j = 0; j < 9; ++j)
    if (!std::isfinite(M[j])) return fail(OSSCIR_EINVAL, "material_transform: matrix not finite");
  OSSCIR_HIP(launch_material_transform(M, in, out, n_pixels, (hipStream_t)stream), "material_transform launch");
  return OSSCIR_OK;
}

int osscir_ray_nnz(osscir_plan plan, int32_t *nnz, osscir_stream stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!nnz) return fail(OSSCIR_EINVAL, "null nnz");
  OSSCIR_HIP(launch_count(plan->sd, nnz, (hipStream_t)stream), "ray_nnz launch");
  return OSSCIR_OK;
}

int osscir_dtpl(osscir_plan plan, const float *f, const float *c, double *out, void *work, size_t work_bytes,
                osscir_stream stream) {
  int rc = check_plan(plan);
  if (rc) return rc;
  if (!f || !c || !out || !work) return fail(OSSCIR_EINVAL, "dtpl: null pointer");
  const WorkLayout wl = work_layout(plan->sd);
  if (work_bytes < wl.total) return fail(OSSCIR_ESTATE, "workspace %zu < %zu bytes", work_bytes, wl.total);
  float *p = (float *)((char *)work + wl.p);
  double *partial = (double *)((char *)work + wl.partial);
  OSSCIR_HIP(launch_dtpl(plan->sd, f, c, p, (char *)work + wl.pack, partial, out, (hipStream_t)stream),
             "dtpl launch");
  return OSSCIR_OK;
}

}  // extern "C"
