// Pixel-driven gather of the back-projector, shared by the plain
// back-projection kernel and the kernels that fuse an epilogue (primal step,
// step lengths) into it.
//
// A workgroup owns a 16 x 16 pixel tile, one thread per pixel, and walks the
// views in order.  Projecting the tile's four corners onto the detector
// bounds, for each view, the bins whose rays can meet the tile (+0.05 bin)
// and the half-width hw of every pixel's own shadow; the plan does this once
// for every (tile, view) (TileBins), the wide path per chunk of views.
//
// Common path: views are staged in groups of four, wave w staging the bins
// of the group's view w into LDS (line parameters and the NCH input values,
// one bin per lane, up to 64); slots past a view's shadow hold a null record
// whose weight is exactly 0.  The loads of the next group are issued before
// the current group is processed and stored after it, so a group costs two
// barriers.  With qS as input (the fused primal step) and a grid of at least
// four workgroups per CU, the bins are instead copied straight from memory
// into double-buffered LDS arrays (global-to-LDS loads, one barrier per
// group); both stagings hold the same records.  A pixel's non-zero weights in
// a view lie on the bins strictly inside (tau - hw, tau + hw), tau being its
// centre's detector position: at most K = floor(2 hw) + 1 consecutive bins.
// Every thread reads the group's views in pairs, a pair's window of
// max(K, K') staged bins starting at floor(tau - hw) + 1 in each view,
// clamped into the staged range; the bins of a window outside the pixel's
// shadow have weight exactly 0.  The window length is uniform over the
// workgroup, so the loop carries no per-lane bounds or divergence, and the
// two views' windows are independent work within a step.
//
// Wide path (some tile shadow exceeds 62 bins; chosen by the plan): one view
// at a time, up to 128 bins staged by all four waves, each thread looping
// over its own shadow, views whose shadow exceeds 128 bins in chunks.
//
// The weights are chord_weight() of the same inputs as the forward
// projector, so the result is X^T q with X's exact weights.  Products are
// summed in FP32 over 8 views at a time and the running sum over views is
// FP64, so the result carries the rounding of the FP32 weights and inputs
// only (the per-pixel 3x3 step blocks built from it are ill-conditioned, and
// FP32 accumulation over thousands of rays would shift the MOCCA trajectory).
#pragma once

#include "device_math.h"
#include "kernels.h"

namespace osscir {

constexpr int kBpTile = 16;
constexpr int kBpThreads = kBpTile * kBpTile;
constexpr int kBpMaxBins = 128;   // bins staged per view; wider shadows take a chunked path
constexpr int kBpViewChunk = 128;  // views whose tile bounds are computed together
constexpr int kBpFlush = 8;       // views summed in FP32 before the FP64 running sum
constexpr int kBpGroup = 4;       // views staged together (one wave each) in the common path
constexpr int kBpSlot = 64;       // staged bins per view of a group (one lane each)

// One staged bin.  The 80-byte stride (20 banks) puts the 16-byte pieces of
// eight consecutive bins on 32 distinct LDS banks; a power-of-two stride
// would fold them onto two bank groups.
struct BinLDS {
  double2 n;   // kappa nx, kappa ny
  float4 w0;   // kappa a, hmax, 0, q8
  float4 w1;   // q0..q3
  float4 w2;   // q4..q7
  float4 pad;
};

struct ViewTile {
  int d0, d1;    // bins whose rays can meet the tile
  float hw;      // bound on a pixel's shadow half-width (bins), incl. margin; < 0: use [d0, d1]
  float off;     // cbin - hw - d0 + 1: a pixel's window starts at floor(bin_scale t + off) (staged index)
  int nst;       // staged bins, max(0, d1 - d0 + 1)
  int K;         // window length, min(nst, floor(2 hw) + 1); nst when hw < 0
  int pad0, pad1;
};

// Grouped staging of the fused primal path, filled by global-to-LDS copies
// (16 bytes per lane, lane i at slot i): one array per 16-byte piece of a
// bin: the ray table's (kappa nx, kappa ny) and the three pieces of qS
// (q0..q3, q4..q7, and q8 with the ray's kappa a and hmax, written there by
// the spectral kernel).
struct BpSoa {
  double2 a[kBpGroup][kBpSlot];  // kappa nx, kappa ny
  float4 b[kBpGroup][kBpSlot];   // q0..q3
  float4 c[kBpGroup][kBpSlot];   // q4..q7
  float4 d[kBpGroup][kBpSlot];   // q8, kappa a, hmax, 0
};

struct BpShared {
  union {
    BinLDS bins[2][kBpMaxBins];          // per-view staging (wide shadows)
    BinLDS gbins[kBpGroup][kBpSlot];     // grouped staging (common path, planar q)
    BpSoa soa[2];                        // grouped staging (fused primal path), double-buffered
    float4 tile[kBpTile][kBpTile + 1];  // epilogues, after the last view
  };
  ViewTile vt[kBpViewChunk];
  double2 red[kBpThreads / 64];
};

__device__ __forceinline__ void tile_view_bounds(const ScanDesc &sd, const ViewGeom &vg, int tile_x, int tile_y,
                                                 ViewTile &out) {
  const int nb = sd.n_bins;
  const float x0 = (float)(tile_x * kBpTile) - sd.c0 - 0.5f, x1 = x0 + (float)kBpTile;
  const float y0 = (float)(tile_y * kBpTile) - sd.c0 - 0.5f, y1 = y0 + (float)kBpTile;
  float tmin = 3.0e38f, tmax = -3.0e38f, dmin = 3.0e38f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float X = (k & 1) ? x1 : x0;
    const float Y = (k & 2) ? y1 : y0;
    const float num = -vg.sb * X + vg.cb * Y;
    const float den = sd.sid_px - vg.cb * X - vg.sb * Y;
    const float t = num / den;
    tmin = fminf(tmin, t);
    tmax = fmaxf(tmax, t);
    dmin = fminf(dmin, den);
  }
  float lo = fminf(fmaxf(tmin * sd.bin_scale + sd.cbin, -2.0f), (float)nb + 1.0f);
  float hi = fminf(fmaxf(tmax * sd.bin_scale + sd.cbin, -2.0f), (float)nb + 1.0f);
  out.d0 = max(0, (int)ceilf(lo - 0.05f));
  out.d1 = min(nb - 1, (int)floorf(hi + 0.05f));
  // d t / d X = (-sb + cb t) / den, d t / d Y = (cb + sb t) / den; linear in t,
  // so bounded by the tile's extreme t; den >= dmin at every pixel centre; the
  // exact corner offsets exceed the linearised ones by at most a factor
  // 1 + 1.5 / den (a corner moves den by <= 0.71).
  out.nst = max(0, out.d1 - out.d0 + 1);
  if (dmin > 4.0f) {
    const float A = fmaxf(fabsf(-vg.sb + vg.cb * tmin), fabsf(-vg.sb + vg.cb * tmax));
    const float B = fmaxf(fabsf(vg.cb + vg.sb * tmin), fabsf(vg.cb + vg.sb * tmax));
    out.hw = 0.5f * (A + B) / dmin * (1.0f + 1.5f / dmin) * sd.bin_scale + 0.02f;
    out.off = sd.cbin - out.hw - (float)out.d0 + 1.0f;
    out.K = min(out.nst, (int)floorf(2.0f * out.hw) + 1);
  } else {
    out.hw = -1.0f;
    out.off = 0.0f;
    out.K = out.nst;
  }
}

// Pixel (tx, ty) of the 16 x 16 tile held by thread tid: wave w takes the
// 8 x 8 quadrant (w & 1, w >> 1) and each group of eight lanes a 4 x 2 block.
// An LDS read serves eight lanes at a time, and staged bins 8 apart share
// banks (80-byte stride); the bins of a 4 x 2 block stay within fewer than 8
// of each other for all but the views that see the block magnified most,
// where eight pixels of one row would span up to 19.
__device__ __forceinline__ void bp_pixel_of_thread(int tid, int &tx, int &ty) {
  const int w = tid >> 6, g = (tid >> 3) & 7, k = tid & 7;
  tx = (w & 1) * 8 + (g & 1) * 4 + (k & 3);
  ty = (w >> 1) * 8 + (g >> 1) * 2 + (k >> 2);
}

template <int NCH>
struct BinRegs {
  RayLine r;
  float q[NCH];
};

// Staged bins are spread over the workgroup's four waves in runs of 16
// consecutive bins (lanes 0..15 of each wave, then 16..31, ...), so the
// staging work of a view is shared while loads and LDS stores stay
// contiguous.
__device__ __forceinline__ int stage_bin_of_thread(int tid) {
  return ((tid & 63) >> 4) * 64 + (tid >> 6) * 16 + (tid & 15);
}

// QS12: q holds 12 floats per ray (three float4: channels 0..3, 4..7, 8..11)
// and is staged with three 16-byte loads; otherwise q is planar [c][stride].
template <int NCH, bool QS12>
__device__ __forceinline__ void bin_load(const RayLine *__restrict__ rays, const float *__restrict__ q,
                                         unsigned q_stride, unsigned l, BinRegs<NCH> &b) {
  b.r = rays[l];
  if (QS12) {
    const float4 *__restrict__ q4 = reinterpret_cast<const float4 *>(q) + 3 * (size_t)l;
    const float4 a = q4[0];
    b.q[0] = a.x;
    if (NCH > 1) b.q[1] = a.y;
    if (NCH > 2) b.q[2] = a.z;
    if (NCH > 3) b.q[3] = a.w;
    if (NCH > 4) {
      const float4 c4 = q4[1];
      b.q[4] = c4.x;
      if (NCH > 5) b.q[5] = c4.y;
      if (NCH > 6) b.q[6] = c4.z;
      if (NCH > 7) b.q[7] = c4.w;
    }
    if (NCH > 8) b.q[8] = q4[2].x;
  } else {
#pragma unroll
    for (int c = 0; c < NCH; ++c) b.q[c] = q[c * q_stride + l];
  }
}

template <int NCH>
__device__ __forceinline__ void bin_store(const BinRegs<NCH> &b, BinLDS &e) {
  float qq[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) qq[c] = c < NCH ? b.q[c] : 0.0f;
  e.n = make_double2(b.r.nxk, b.r.nyk);
  e.w0 = make_float4(b.r.ak, b.r.hmax, 0.0f, qq[8]);
  e.w1 = make_float4(qq[0], qq[1], qq[2], qq[3]);
  if (NCH > 4) e.w2 = make_float4(qq[4], qq[5], qq[6], qq[7]);
}

// copy of the fields of a staged bin that NCH channels use
template <int NCH>
__device__ __forceinline__ void load_bin(const BinLDS &src, BinLDS &e) {
  e.n = src.n;
  e.w0 = src.w0;
  e.w1 = src.w1;
  if (NCH > 4) e.w2 = src.w2;
}

template <int NCH>
__device__ __forceinline__ void accumulate_bin(const BinLDS &e, double dx, double dy, float part[NCH]) {
  const double2 nn = e.n;
  const float4 w0 = e.w0;
  const float w = chord_weight(nn.x, nn.y, w0.x, w0.y, dx, dy, w0.z);  // w0.z = 0: the record is read whole
  float qv[9];
  const float4 w1 = e.w1;
  qv[0] = w1.x; qv[1] = w1.y; qv[2] = w1.z; qv[3] = w1.w;
  if (NCH > 4) {
    const float4 w2 = e.w2;
    qv[4] = w2.x; qv[5] = w2.y; qv[6] = w2.z; qv[7] = w2.w;
  }
  qv[8] = w0.w;
#pragma unroll
  for (int c = 0; c < NCH; ++c) part[c] = __fmaf_rn(w, qv[c], part[c]);
}

// bins b0..b1 of the staged view (b0 > b1: none); the first two unrolled
template <int NCH>
__device__ __forceinline__ void accumulate_bins(const BinLDS *__restrict__ bins, int b0, int b1, double dx, double dy,
                                                float part[NCH]) {
  if (b0 <= b1) accumulate_bin<NCH>(bins[b0], dx, dy, part);
  if (b0 + 1 <= b1) accumulate_bin<NCH>(bins[b0 + 1], dx, dy, part);
  for (int b = b0 + 2; b <= b1; ++b) accumulate_bin<NCH>(bins[b], dx, dy, part);
}

// Bins of pixel (X, Y) (centred coordinates) in view vg: the tile's range
// [d0, d1] narrowed to the pixel's bounded shadow.
__device__ __forceinline__ void pixel_bins(const ScanDesc &sd, const ViewGeom &vg, const ViewTile &vt, float X,
                                           float Y, int &dlo, int &dhi) {
  dlo = vt.d0;
  dhi = vt.d1;
  if (vt.hw >= 0.0f) {
    const float num = __fmaf_rn(vg.cb, Y, -vg.sb * X);
    const float den = __fmaf_rn(-vg.sb, Y, __fmaf_rn(-vg.cb, X, sd.sid_px));
    const float bc = __fmaf_rn(num * __builtin_amdgcn_rcpf(den), sd.bin_scale, sd.cbin);
    dlo = max(dlo, (int)ceilf(bc - vt.hw));
    dhi = min(dhi, (int)floorf(bc + vt.hw));
  }
}

// Wide path: one view per barrier; views whose shadow exceeds kBpMaxBins bins
// are staged and accumulated in chunks with extra barriers.
template <int NCH, bool QS12>
__device__ __forceinline__ void back_accumulate_views(const ScanDesc &sd, int tile_x, int tile_y,
                                                      const float *__restrict__ q, int q_stride_i, double acc[NCH],
                                                      BpShared &sh) {
  static_assert(NCH >= 1 && NCH <= 9, "1..9 channels");
  const int tid = threadIdx.x;
  int tx, ty;
  bp_pixel_of_thread(tid, tx, ty);
  const int ix = tile_x * kBpTile + tx;
  const int iy = tile_y * kBpTile + ty;
  const int n = sd.n, V = sd.n_views;
  const unsigned nb = (unsigned)sd.n_bins, q_stride = (unsigned)q_stride_i;
  const RayLine *__restrict__ rays = sd.rays;
  const bool inside = ix < n && iy < n;
  const float X = (float)ix - sd.c0;  // centred, for the detector projection
  const float Y = (float)iy - sd.c0;
  const double fx = (double)ix, fy = (double)iy;
  const int sb = stage_bin_of_thread(tid);
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
  for (int vc = 0; vc < V; vc += kBpViewChunk) {
    const int cnt = min(kBpViewChunk, V - vc);
    __syncthreads();  // the previous chunk is done with sh
    if (tid < cnt) tile_view_bounds(sd, sd.views[vc + tid], tile_x, tile_y, sh.vt[tid]);
    __syncthreads();
    {
      const ViewTile vt = sh.vt[0];
      if (sb < vt.nst && vt.nst <= kBpMaxBins) {
        BinRegs<NCH> b;
        bin_load<NCH, QS12>(rays, q, q_stride, (unsigned)vc * nb + (unsigned)(vt.d0 + sb), b);
        bin_store<NCH>(b, sh.bins[0][sb]);
      }
    }
    __syncthreads();
    for (int j0 = 0; j0 < cnt; j0 += kBpFlush) {
      float part[NCH];
#pragma unroll
      for (int c = 0; c < NCH; ++c) part[c] = 0.0f;
      const int jend = min(cnt, j0 + kBpFlush);
      for (int j = j0; j < jend; ++j) {
        const int v = vc + j;
        const int cur = j & 1;
        const ViewTile vt = sh.vt[j];
        // issue the next view's loads
        BinRegs<NCH> nxt;
        bool have_next = false;
        if (j + 1 < cnt) {
          const ViewTile vn = sh.vt[j + 1];
          have_next = sb < vn.nst && vn.nst <= kBpMaxBins;
          if (have_next) bin_load<NCH, QS12>(rays, q, q_stride, (unsigned)(v + 1) * nb + (unsigned)(vn.d0 + sb), nxt);
        }
        const ViewGeom vg = load_uniform(sd.views + v);
        const double dx = vg.sx - fx;
        const double dy = vg.sy - fy;
        if (vt.nst <= kBpMaxBins) {
          int dlo, dhi;
          pixel_bins(sd, vg, vt, X, Y, dlo, dhi);
          if (inside) accumulate_bins<NCH>(sh.bins[cur], dlo - vt.d0, min(dhi - vt.d0, kBpMaxBins - 1), dx, dy, part);
        } else {
          int dlo, dhi;
          pixel_bins(sd, vg, vt, X, Y, dlo, dhi);
          for (int c0 = vt.d0; c0 <= vt.d1; c0 += kBpMaxBins) {
            const int c1 = min(vt.d1, c0 + kBpMaxBins - 1);
            __syncthreads();
            if (sb <= c1 - c0) {
              BinRegs<NCH> b;
              bin_load<NCH, QS12>(rays, q, q_stride, (unsigned)v * nb + (unsigned)(c0 + sb), b);
              bin_store<NCH>(b, sh.bins[cur][sb]);
            }
            __syncthreads();
            if (inside) accumulate_bins<NCH>(sh.bins[cur], max(dlo, c0) - c0, min(dhi, c1) - c0, dx, dy, part);
          }
        }
        if (have_next) bin_store<NCH>(nxt, sh.bins[cur ^ 1][sb]);
        __syncthreads();
      }
#pragma unroll
      for (int c = 0; c < NCH; ++c) acc[c] += (double)part[c];
    }
  }
}

// Loads of the bin staged by this thread in a group: view j (wave su of the
// group) with staged bins tb, bin d0 + sl.  A thread without a bin (past the
// view's shadow, or past the last view) loads the plan's zero record
// instead, whose weight is exactly 0 (med3((0 - 0) * 0, 0, 0)), so every
// slot of the group is rewritten and no branch or select on the data is
// needed.
template <int NCH, bool QS12>
__device__ __forceinline__ void group_load(const ScanDesc &sd, const float *__restrict__ q, unsigned q_stride,
                                           unsigned nb, const TileBins &tb, int j, bool valid, int sl,
                                           BinRegs<NCH> &b) {
  const bool has = valid && sl < min(tb.nst, kBpSlot);
  const unsigned l = (unsigned)j * nb + (unsigned)(tb.d0 + sl);  // used only if has
  b.r = *(has ? sd.rays + l : reinterpret_cast<const RayLine *>(sd.zero));
  if (QS12) {
    const float4 *__restrict__ q4 = has ? reinterpret_cast<const float4 *>(q) + 3 * (size_t)l : sd.zero;
    const float4 a = q4[0];
    b.q[0] = a.x;
    if (NCH > 1) b.q[1] = a.y;
    if (NCH > 2) b.q[2] = a.z;
    if (NCH > 3) b.q[3] = a.w;
    if (NCH > 4) {
      const float4 c4 = q4[1];
      b.q[4] = c4.x;
      if (NCH > 5) b.q[5] = c4.y;
      if (NCH > 6) b.q[6] = c4.z;
      if (NCH > 7) b.q[7] = c4.w;
    }
    if (NCH > 8) b.q[8] = q4[2].x;
  } else {
    const float *__restrict__ qp = has ? q + l : reinterpret_cast<const float *>(sd.zero);
    const unsigned qs = has ? q_stride : 0u;
#pragma unroll
    for (int c = 0; c < NCH; ++c) b.q[c] = qp[c * qs];
  }
}

// Global-to-LDS copies of one view's bins for the fused primal path (qS with
// 12 floats per ray): wave su stages view j into dst, lane sl bin d0 + sl;
// lanes without a bin copy the plan's zero record.
__device__ __forceinline__ void copy_group_view(const ScanDesc &sd, const float *__restrict__ qS, unsigned nb,
                                                const TileBins &tb, int j, bool valid, int su, int sl,
                                                BpSoa &dst) {
  const bool has = valid && sl < min(tb.nst, kBpSlot);
  const unsigned l0 = (unsigned)j * nb + (unsigned)tb.d0;  // uniform
  const float4 *ra = has ? reinterpret_cast<const float4 *>(sd.rays + l0) + 2 * sl : sd.zero;
  const float4 *qa = has ? reinterpret_cast<const float4 *>(qS) + 3 * ((size_t)l0 + sl) : sd.zero;
  __builtin_amdgcn_global_load_lds(ra, (void OSSCIR_LDS *)&dst.a[su][0], 16, 0, 0);
  __builtin_amdgcn_global_load_lds(qa, (void OSSCIR_LDS *)&dst.b[su][0], 16, 0, 0);
  __builtin_amdgcn_global_load_lds(qa + 1, (void OSSCIR_LDS *)&dst.c[su][0], 16, 0, 0);
  __builtin_amdgcn_global_load_lds(qa + 2, (void OSSCIR_LDS *)&dst.d[su][0], 16, 0, 0);
}

template <int NCH>
__device__ __forceinline__ void load_soa(const BpSoa &S, int u, int idx, BinLDS &e) {
  e.n = S.a[u][idx];
  const float4 d = S.d[u][idx];
  e.w0 = make_float4(d.y, d.z, d.w, d.x);  // kappa a, hmax, 0, q8: the record accumulate_bin reads
  e.w1 = S.b[u][idx];
  if (NCH > 4) e.w2 = S.c[u][idx];
}

// Common path (every tile shadow within kBpSlot - 2 bins; the plan checks):
// views are staged four at a time, one wave per view, and each pixel sums
// the group's views in pairs, a pair reading the window length of its
// longer view.  COPY: the bins go from memory straight into double-buffered
// LDS arrays (global-to-LDS copies, one barrier per group); otherwise they
// are staged through registers into 80-byte records (two barriers per
// group).  Both stagings hold the same records and sum them in the same
// order, so they give the same bits.
// Views vb .. ve - 1 (vb a multiple of kBpFlush).  FOLD: the sum is formed
// part by part, a part being bp_part_views consecutive views from view 0:
// each part's FP64 sum starts from zero and the parts are added in order, so
// the result has the bits of the split back-projection, whose workgroups sum
// one part each (acc = ((p0 + p1) + p2) + ...; with one part, acc = 0 + p0 =
// p0 exactly).
template <int NCH, bool QS12, bool COPY, bool FOLD = false>
__device__ __forceinline__ void back_accumulate_grouped(const ScanDesc &sd, int tile_x, int tile_y,
                                                        const float *__restrict__ q, int q_stride_i, double acc[NCH],
                                                        BpShared &sh, int vb, int ve) {
  static_assert(QS12 || !COPY, "global-to-LDS staging reads qS");
  static_assert(kBpGroup == 4 && kBpGroup * 64 == kBpThreads && kBpSlot == 64, "one wave per view, one lane per bin");
  static_assert(kBpFlush % kBpGroup == 0, "flushes at group ends");
  const int tid = threadIdx.x;
  int tx, ty;
  bp_pixel_of_thread(tid, tx, ty);
  const int ix = tile_x * kBpTile + tx;
  const int iy = tile_y * kBpTile + ty;
  const int V = ve;  // views past ve are not this call's
  const int nt = (sd.n + kBpTile - 1) / kBpTile;
  const unsigned nb = (unsigned)sd.n_bins, q_stride = (unsigned)q_stride_i;
  const float X = (float)ix - sd.c0;  // centred, for the detector projection
  const float Y = (float)iy - sd.c0;
  const float sid = in_vgpr(sd.sid_px);
  const double fx = (double)ix, fy = (double)iy;
  const int su = __builtin_amdgcn_readfirstlane(tid >> 6), sl = tid & 63;  // staged slot: view su, bin sl
  const TileBins *__restrict__ tbs = sd.tile_bins + (size_t)(tile_y * nt + tile_x) * sd.n_views;
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
  double done[FOLD ? NCH : 1];  // FOLD: the parts before the current one
#pragma unroll
  for (int c = 0; c < (FOLD ? NCH : 1); ++c) done[c] = 0.0;
  const int vp = FOLD ? sd.bp_part_views : V;
  float part[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) part[c] = 0.0f;
  BinRegs<NCH> nxt;
  {
    const int j = vb + su;
    const TileBins tb = load_uniform(tbs + min(j, V - 1));
    if (COPY)
      copy_group_view(sd, q, nb, tb, j, j < V, su, sl, sh.soa[0]);
    else
      group_load<NCH, QS12>(sd, q, q_stride, nb, tb, j, j < V, sl, nxt);
  }
  int buf = 0;
  for (int g0 = vb; g0 < V; g0 += kBpGroup) {
    if (COPY) {
      __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of the group have landed
      __syncthreads();                // every wave's have; the other buffer's reads are done
      const int jn = g0 + kBpGroup + su;
      if (g0 + kBpGroup < V) {
        const TileBins tb = load_uniform(tbs + min(jn, V - 1));
        copy_group_view(sd, q, nb, tb, jn, jn < V, su, sl, sh.soa[buf ^ 1]);
      }
    } else {
      __syncthreads();  // the previous group's windows have been read
      bin_store<NCH>(nxt, sh.gbins[su][sl]);
      __syncthreads();
      const int jn = g0 + kBpGroup + su;
      const TileBins tb = load_uniform(tbs + min(jn, V - 1));
      group_load<NCH, QS12>(sd, q, q_stride, nb, tb, jn, jn < V, sl, nxt);
    }
    // the group's views (views past the last one have no staged bins)
    int K[kBpGroup], nst[kBpGroup];
    float t[kBpGroup];
    double dx[kBpGroup], dy[kBpGroup];
#pragma unroll
    for (int u = 0; u < kBpGroup; ++u) {
      const int j = min(g0 + u, V - 1);
      const TileBins tb = load_uniform(tbs + j);
      const ViewGeom vg = load_uniform(sd.views + j);
      nst[u] = g0 + u < V ? min(tb.nst, kBpSlot) : 0;
      K[u] = min(tb.K, nst[u]);
      const float num = __fmaf_rn(vg.cb, Y, -vg.sb * X);
      const float den = __fmaf_rn(-vg.sb, Y, __fmaf_rn(-vg.cb, X, sid));
      t[u] = __fmaf_rn(num * __builtin_amdgcn_rcpf(den), sd.bin_scale, tb.off);
      dx[u] = vg.sx - fx;
      dy[u] = vg.sy - fy;
    }
#pragma unroll
    for (int p = 0; p < kBpGroup; p += 2) {
      // window u: [s, s + kp) inside [0, max(nst, kp)) within the slot,
      // starting at floor(tau - hw) + 1: it covers the staged part of the
      // pixel's shadow, the integers inside (tau - hw, tau + hw) (at most
      // K <= kp of them); slots past nst hold zero records
      const int kp = max(K[p], K[p + 1]);  // uniform
      const int s0 = clamp_0_hi(floor_to_int(t[p]), max(0, nst[p] - kp));
      const int s1 = clamp_0_hi(floor_to_int(t[p + 1]), max(0, nst[p + 1] - kp));
      if (COPY) {
        const BpSoa &S = sh.soa[buf];
        for (int i = 0; i < kp; ++i) {
          BinLDS e0, e1;  // two views' reads in flight before the first weight
          load_soa<NCH>(S, p, s0 + i, e0);
          load_soa<NCH>(S, p + 1, s1 + i, e1);
          accumulate_bin<NCH>(e0, dx[p], dy[p], part);
          accumulate_bin<NCH>(e1, dx[p + 1], dy[p + 1], part);
        }
      } else {
        const BinLDS *w0 = &sh.gbins[p][s0], *w1 = &sh.gbins[p + 1][s1];
        for (int i = 0; i < kp; ++i) {
          BinLDS e0, e1;
          load_bin<NCH>(w0[i], e0);
          load_bin<NCH>(w1[i], e1);
          accumulate_bin<NCH>(e0, dx[p], dy[p], part);
          accumulate_bin<NCH>(e1, dx[p + 1], dy[p + 1], part);
        }
      }
    }
    if ((g0 + kBpGroup) % kBpFlush == 0 || g0 + kBpGroup >= V) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        acc[c] += (double)part[c];
        part[c] = 0.0f;
      }
      if (FOLD && (g0 + kBpGroup) % vp == 0 && g0 + kBpGroup < V) {  // uniform
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          done[c] += acc[c];
          acc[c] = 0.0;
        }
      }
    }
    buf ^= 1;
  }
  if (FOLD) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = done[c] + acc[c];
  }
  __syncthreads();  // every wave is done with the staging buffers, which epilogues reuse
}

// COPY (QS12 only): the grouped path stages by global-to-LDS copies.  Both
// grouped variants give the same bits; the copies pay off when four
// workgroups share a CU (the next group's copies then overlap other
// workgroups' sums), register staging when the grid is small.
// Views vb .. ve - 1 (the grouped path; the wide path always takes every
// view, and its plans have one part).
template <int NCH, bool WIDE, bool QS12 = false, bool COPY = false, bool FOLD = false>
__device__ __forceinline__ void back_accumulate(const ScanDesc &sd, int tile_x, int tile_y, const float *__restrict__ q,
                                                int q_stride_i, double acc[NCH], BpShared &sh, int vb, int ve) {
  static_assert(NCH >= 1 && NCH <= 9, "1..9 channels");
  static_assert(QS12 || !COPY, "global-to-LDS staging reads qS");
  if (WIDE)
    back_accumulate_views<NCH, QS12>(sd, tile_x, tile_y, q, q_stride_i, acc, sh);
  else
    back_accumulate_grouped<NCH, QS12, COPY, FOLD>(sd, tile_x, tile_y, q, q_stride_i, acc, sh, vb, ve);
}

}  // namespace osscir
