// Batched MOCCA over many scans (the osscir_batch_* calls of include/osscir.h):
// slot bookkeeping, work-list construction, graph capture and the
// autotuner.  The kernels are in batch.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "batch.h"
#include "osscir.h"
#include "plan.h"
#include "project_device.h"
#include "projector.h"

using namespace osscir;

namespace {

constexpr int kX = 8;  // XCDs; workgroup b runs on XCD b % 8
enum { kListFp = 0, kListSpec, kListBp, kListBpWide, kLists };

struct HostSlot {
  bool bound = false;
  osscir_plan plan = nullptr;
  osscir_state state{};
  float lambda = 0.0f;
  int n_inner = 1;       // inner steps per expansion point
  float *p0 = nullptr;   // [3][L] caller memory when n_inner > 1
};

struct ListBuf {
  int *d = nullptr;  // kListHeader + kX * cap ints
  int *h = nullptr;  // pinned staging, same size
  int cap = 0;       // items per XCD
  int total = 0;
};

struct Item {
  int code;
  double cost;
};

int list_ints(int cap) { return kListHeader + kX * cap; }

bool valid_rays(int r) { return r == 64 || r == 128 || r == 256; }
bool valid_wgs(int w) { return w >= kX && w <= 65536 && w % kX == 0; }

int check_config(const osscir_batch_config &c) {
  if (!valid_rays(c.fp_rays) || !valid_rays(c.spec_rays))
    return fail(OSSCIR_EINVAL, "rays per workgroup must be 64, 128 or 256 (got %d, %d)", c.fp_rays, c.spec_rays);
  if (!valid_wgs(c.fp_wgs) || !valid_wgs(c.spec_wgs) || !valid_wgs(c.bp_wgs))
    return fail(OSSCIR_EINVAL, "workgroup counts must be multiples of 8 in [8, 65536] (got %d, %d, %d)", c.fp_wgs,
                c.spec_wgs, c.bp_wgs);
  if ((c.fp_xcd | c.spec_xcd | c.bp_xcd) & ~1) return fail(OSSCIR_EINVAL, "xcd flags must be 0 or 1");
  return OSSCIR_OK;
}

// Deal the items (in their logical order) to the XCDs: contiguous ranges of
// equal estimated cost, or round-robin.
void distribute(const std::vector<Item> &items, bool xcd, std::vector<int> (&per)[kX]) {
  for (auto &v : per) v.clear();
  if (!xcd) {
    for (size_t i = 0; i < items.size(); ++i) per[i % kX].push_back(items[i].code);
    return;
  }
  double total = 0.0;
  for (const Item &it : items) total += it.cost;
  double run = 0.0;
  for (const Item &it : items) {
    int x = total > 0.0 ? (int)((run + 0.5 * it.cost) / total * kX) : 0;
    x = std::min(kX - 1, std::max(0, x));
    per[x].push_back(it.code);
    run += it.cost;
  }
}

}  // namespace

struct osscir_batch_s {
  int device = -1;
  int max_slots = 0;
  bool block = true, clip = true, fp64 = true;
  osscir_batch_config cfg{};
  std::vector<HostSlot> slots;
  std::vector<SlotStatus> init_status;  // status entries still to upload
  std::vector<char> status_pending;
  SlotDesc *d_slots = nullptr, *h_slots = nullptr;
  SlotStatus *d_status = nullptr, *h_status = nullptr, *h_status_rb = nullptr;
  double2 *d_partial = nullptr;
  int partial_cap = 0;
  ListBuf lists[kLists];
  bool any_wide = false;
  bool any_nested = false;      // some bound slot runs nested loops
  size_t spec_lds = 0;          // dynamic LDS of the spectral launch
  hipEvent_t staged = nullptr;  // the last upload from the staging buffers
  bool staged_pending = false;
  bool dirty = true;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool graph_ok = false, graph_wide = false, graph_nested = false;
  size_t graph_spec_lds = 0;
};

namespace {

void free_batch(osscir_batch b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->staged) (void)hipEventDestroy(b->staged);
  for (ListBuf &l : b->lists) {
    if (l.d) (void)hipFree(l.d);
    if (l.h) (void)hipHostFree(l.h);
  }
  if (b->d_partial) (void)hipFree(b->d_partial);
  if (b->d_slots) (void)hipFree(b->d_slots);
  if (b->h_slots) (void)hipHostFree(b->h_slots);
  if (b->d_status) (void)hipFree(b->d_status);
  if (b->h_status) (void)hipHostFree(b->h_status);
  if (b->h_status_rb) (void)hipHostFree(b->h_status_rb);
  delete b;
}

int check_batch(osscir_batch b) {
  if (!b) return fail(OSSCIR_EINVAL, "null batch");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
    return fail(OSSCIR_EINVAL, "batch was created on device %d, current device is %d", b->device, dev);
  return OSSCIR_OK;
}

int tiles_of(const ScanDesc &sd) {
  const int nt = (sd.n + kBpTile - 1) / kBpTile;
  return nt * nt;
}

SlotDesc make_desc(const HostSlot &hs) {
  SlotDesc d{};
  const ScanDesc &sd = hs.plan->sd;
  const WorkLayout wl = work_layout(sd);
  char *w = (char *)hs.state.work;
  const size_t np = (size_t)sd.n + 2 * kPad;
  d.sd = sd;
  d.f = hs.state.f;
  d.fbar = hs.state.fbar;
  d.y = hs.state.y;
  d.c = hs.state.c;
  d.p = (float *)(w + wl.p);
  d.qS = (float *)(w + wl.qS);
  d.pk_xy = (float4 *)(w + wl.pack);
  d.pk_yx = d.pk_xy + np * np;
  d.lambda = hs.lambda;
  d.n_tiles = tiles_of(sd);
  d.n_inner = hs.n_inner;
  d.p0 = hs.p0;
  return d;
}

// Grow a device/pinned list pair to hold `cap` items per XCD.  The caller
// has synchronised the stream.
int grow_list(ListBuf &l, int cap) {
  if (l.d) (void)hipFree(l.d);
  if (l.h) (void)hipHostFree(l.h);
  l.d = nullptr;
  l.h = nullptr;
  l.cap = 0;
  const size_t bytes = (size_t)list_ints(cap) * sizeof(int);
  hipError_t e = hipMalloc(&l.d, bytes);
  if (e == hipSuccess) e = hipHostMalloc(&l.h, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return fail(OSSCIR_ENOMEM, "work list allocation (%zu bytes): %s", bytes, hipGetErrorString(e));
  std::memset(l.h, 0, bytes);
  l.cap = cap;
  return OSSCIR_OK;
}

// Rebuild the slot table and work lists and upload them (and pending status
// entries) on stream.
int flush(osscir_batch b, hipStream_t st) {
  if (!b->dirty) return OSSCIR_OK;
  if (b->staged_pending) {
    OSSCIR_HIP(hipEventSynchronize(b->staged), "batch: waiting for the previous upload");
    b->staged_pending = false;
  }
  const osscir_batch_config &c = b->cfg;
  // slot table and tile offsets (slot order)
  int tiles = 0;
  bool any_wide = false, any_nested = false;
  size_t spec_lds = 0;
  std::vector<int> order;
  for (int s = 0; s < b->max_slots; ++s) {
    const HostSlot &hs = b->slots[s];
    if (!hs.bound) {
      std::memset(&b->h_slots[s], 0, sizeof(SlotDesc));
      continue;
    }
    b->h_slots[s] = make_desc(hs);
    b->h_slots[s].first_tile = tiles;
    tiles += b->h_slots[s].n_tiles;
    any_wide |= hs.plan->sd.bp_wide != 0;
    any_nested |= hs.n_inner > 1;
    if (hs.plan->sd.mfma) spec_lds = std::max(spec_lds, mfma_lds_bytes(hs.plan->sd.n_energy, c.spec_rays / 64));
    order.push_back(s);
  }
  // logical order: costliest scans first (the tail of each launch is cheap work)
  auto scan_cost = [&](int s) {
    const ScanDesc &sd = b->slots[s].plan->sd;
    return (double)sd.n * sd.n * sd.n_views;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int z) { return scan_cost(a) > scan_cost(z); });
  std::vector<Item> items[kLists];
  for (int s : order) {
    const ScanDesc &sd = b->slots[s].plan->sd;
    const int nfc = (sd.n_bins + c.fp_rays - 1) / c.fp_rays;
    const int64_t n_fp = (int64_t)sd.n_views * nfc, n_spec = ((int64_t)sd.n_rays + c.spec_rays - 1) / c.spec_rays;
    const int64_t n_bp = (int64_t)tiles_of(sd);
    if (std::max(n_fp, std::max(n_spec, n_bp)) > (int64_t)kItemLocalMask + 1)
      return fail(OSSCIR_EINVAL, "slot %d: %lld work items exceed the %d a slot may hold", s,
                  (long long)std::max(n_fp, std::max(n_spec, n_bp)), kItemLocalMask + 1);
    const int code = item_code(s, 0);
    for (int i = 0; i < sd.n_views * nfc; ++i) items[kListFp].push_back({code | i, (double)c.fp_rays * sd.n});
    const int nsc = (sd.n_rays + c.spec_rays - 1) / c.spec_rays;
    for (int i = 0; i < nsc; ++i) items[kListSpec].push_back({code | i, (double)c.spec_rays * sd.n_energy});
    auto &bl = items[sd.bp_wide ? kListBpWide : kListBp];
    for (int t : region_tile_order((sd.n + kBpTile - 1) / kBpTile)) bl.push_back({code | t, (double)sd.n_views});
  }
  const bool xcd[kLists] = {c.fp_xcd != 0, c.spec_xcd != 0, c.bp_xcd != 0, c.bp_xcd != 0};
  std::vector<int> per[kLists][kX];
  bool regrow = false;
  int need_cap[kLists];
  for (int k = 0; k < kLists; ++k) {
    distribute(items[k], xcd[k], per[k]);
    need_cap[k] = 1;
    for (int x = 0; x < kX; ++x) need_cap[k] = std::max(need_cap[k], (int)per[k][x].size());
    regrow |= need_cap[k] > b->lists[k].cap;
  }
  regrow |= tiles > b->partial_cap;
  if (regrow) {
    OSSCIR_HIP(hipStreamSynchronize(st), "batch: synchronising before growing buffers");
    for (int k = 0; k < kLists; ++k)
      if (need_cap[k] > b->lists[k].cap) {
        int rc = grow_list(b->lists[k], need_cap[k] + need_cap[k] / 4 + 64);
        if (rc) return rc;
      }
    if (tiles > b->partial_cap) {
      if (b->d_partial) (void)hipFree(b->d_partial);
      b->d_partial = nullptr;
      b->partial_cap = 0;
      const int cap = tiles + tiles / 4 + 256;
      hipError_t e = hipMalloc(&b->d_partial, (size_t)cap * sizeof(double2));
      if (e != hipSuccess) return fail(OSSCIR_ENOMEM, "per-tile sums: %s", hipGetErrorString(e));
      b->partial_cap = cap;
    }
    b->graph_ok = false;
  }
  for (int k = 0; k < kLists; ++k) {
    ListBuf &l = b->lists[k];
    std::memset(l.h, 0, kListHeader * sizeof(int));
    l.total = 0;
    for (int x = 0; x < kX; ++x) {
      l.h[x] = (int)per[k][x].size();
      std::copy(per[k][x].begin(), per[k][x].end(), l.h + kListHeader + x * l.cap);
      l.total += l.h[x];
    }
    OSSCIR_HIP(hipMemcpyAsync(l.d, l.h, (size_t)list_ints(l.cap) * sizeof(int), hipMemcpyHostToDevice, st),
               "batch: uploading work lists");
  }
  OSSCIR_HIP(hipMemcpyAsync(b->d_slots, b->h_slots, (size_t)b->max_slots * sizeof(SlotDesc), hipMemcpyHostToDevice,
                            st),
             "batch: uploading the slot table");
  for (int s = 0; s < b->max_slots; ++s) {
    if (!b->status_pending[s]) continue;
    b->h_status[s] = b->init_status[s];
    OSSCIR_HIP(hipMemcpyAsync(b->d_status + s, b->h_status + s, sizeof(SlotStatus), hipMemcpyHostToDevice, st),
               "batch: uploading slot status");
    b->status_pending[s] = 0;
  }
  OSSCIR_HIP(hipEventRecord(b->staged, st), "batch: recording the upload");
  b->staged_pending = true;
  b->any_wide = any_wide;
  b->any_nested = any_nested;
  b->spec_lds = spec_lds;
  b->dirty = false;
  return OSSCIR_OK;
}

WorkList worklist(const osscir_batch b, int k, int wgs) {
  const int maxw = kX * std::max(1, b->lists[k].cap);
  return WorkList{b->lists[k].d, b->lists[k].cap, std::min(wgs, maxw)};
}

// Stage launches of one iteration; ev (optional) receives an event after each stage.
int launch_iteration(osscir_batch b, hipStream_t st, hipEvent_t *ev = nullptr) {
  const osscir_batch_config &c = b->cfg;
  if (ev) OSSCIR_HIP(hipEventRecord(ev[0], st), "batch: event");
  OSSCIR_HIP(launch_batch_forward(b->d_slots, b->d_status, worklist(b, kListFp, c.fp_wgs), c.fp_rays, st),
             "batch: forward projection");
  if (ev) OSSCIR_HIP(hipEventRecord(ev[1], st), "batch: event");
  OSSCIR_HIP(launch_batch_spectral_dual(b->d_slots, b->d_status, worklist(b, kListSpec, c.spec_wgs), c.spec_rays,
                                        b->spec_lds, b->clip, b->block, b->fp64, b->any_nested, st),
             "batch: spectral model and dual step");
  if (ev) OSSCIR_HIP(hipEventRecord(ev[2], st), "batch: event");
  OSSCIR_HIP(launch_batch_back_primal(b->d_slots, b->d_status, worklist(b, kListBp, c.bp_wgs), b->block, false,
                                      b->d_partial, st),
             "batch: back-projection and primal step");
  if (b->any_wide)
    OSSCIR_HIP(launch_batch_back_primal(b->d_slots, b->d_status, worklist(b, kListBpWide, c.bp_wgs), b->block, true,
                                        b->d_partial, st),
               "batch: back-projection and primal step (wide shadows)");
  if (ev) OSSCIR_HIP(hipEventRecord(ev[3], st), "batch: event");
  OSSCIR_HIP(launch_batch_tick(b->d_slots, b->d_status, b->d_partial, b->max_slots, st), "batch: iteration end");
  return OSSCIR_OK;
}

int capture(osscir_batch b, hipStream_t st) {
  if (b->exec) {
    OSSCIR_HIP(hipStreamSynchronize(st), "batch: synchronising before re-capture");
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  OSSCIR_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "batch: begin capture");
  const int rc = launch_iteration(b, b->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (rc != OSSCIR_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "batch: end capture");
  b->graph = g;
  OSSCIR_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "batch: instantiating the graph");
  b->graph_ok = true;
  b->graph_wide = b->any_wide;
  b->graph_nested = b->any_nested;
  b->graph_spec_lds = b->spec_lds;
  return OSSCIR_OK;
}

}  // namespace

extern "C" {

int osscir_batch_create(const osscir_params *modes, int32_t max_slots, osscir_batch *out) {
  clear_error();
  if (!out) return fail(OSSCIR_EINVAL, "null output batch pointer");
  *out = nullptr;
  if (!modes) return fail(OSSCIR_EINVAL, "null modes");
  if (max_slots < 1 || max_slots > kMaxSlots) return fail(OSSCIR_EINVAL, "max_slots=%d outside [1, %d]", max_slots, kMaxSlots);
  if (modes->precond != OSSCIR_PRECOND_DIAG && modes->precond != OSSCIR_PRECOND_BLOCK)
    return fail(OSSCIR_EINVAL, "unknown preconditioner %d", modes->precond);
  if (modes->curvature != OSSCIR_CURV_WINDOW && modes->curvature != OSSCIR_CURV_CLIP)
    return fail(OSSCIR_EINVAL, "unknown curvature %d", modes->curvature);
  osscir_batch b = new (std::nothrow) osscir_batch_s;
  if (!b) return fail(OSSCIR_ENOMEM, "host allocation failed");
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return fail(OSSCIR_EDEVICE, "no HIP device");
  }
  b->max_slots = max_slots;
  b->block = modes->precond == OSSCIR_PRECOND_BLOCK;
  b->clip = modes->curvature == OSSCIR_CURV_CLIP;
  b->fp64 = modes->fp64_small != 0;
  b->cfg = osscir_batch_config{256, 2048, 1, 256, 2048, 1, 2048, 1};
  b->slots.resize(max_slots);
  b->init_status.assign(max_slots, SlotStatus{});
  b->status_pending.assign(max_slots, 0);
  const size_t sbytes = (size_t)max_slots * sizeof(SlotStatus), dbytes = (size_t)max_slots * sizeof(SlotDesc);
  hipError_t e;
  if ((e = hipMalloc(&b->d_slots, dbytes)) != hipSuccess ||
      (e = hipHostMalloc(&b->h_slots, dbytes, hipHostMallocDefault)) != hipSuccess ||
      (e = hipMalloc(&b->d_status, sbytes)) != hipSuccess ||
      (e = hipHostMalloc(&b->h_status, sbytes, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc(&b->h_status_rb, sbytes, hipHostMallocDefault)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
    free_batch(b);
    return fail(OSSCIR_ENOMEM, "batch allocation failed: %s", hipGetErrorString(e));
  }
  std::memset(b->h_slots, 0, dbytes);
  std::memset(b->h_status, 0, sbytes);
  if ((e = hipMemcpy(b->d_slots, b->h_slots, dbytes, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->d_status, b->h_status, sbytes, hipMemcpyHostToDevice)) != hipSuccess) {
    free_batch(b);
    return hip_fail(e, "batch: clearing the slot table");
  }
  *out = b;
  return OSSCIR_OK;
}

int osscir_batch_destroy(osscir_batch batch) {
  if (!batch) return OSSCIR_OK;
  (void)hipDeviceSynchronize();
  free_batch(batch);
  return OSSCIR_OK;
}

int osscir_batch_set_slot_nested(osscir_batch b, int32_t slot, osscir_plan plan, const osscir_state *state,
                                 double lambda, int32_t max_iter, double tol, int32_t n_inner, float *p0,
                                 osscir_stream stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (slot < 0 || slot >= b->max_slots) return fail(OSSCIR_EINVAL, "slot %d outside [0, %d)", slot, b->max_slots);
  if ((rc = check_plan(plan))) return rc;
  if (!state || !state->f || !state->fbar || !state->y || !state->c || !state->work)
    return fail(OSSCIR_EINVAL, "batch: null state buffer");
  if (!(lambda > 0) || !std::isfinite(lambda)) return fail(OSSCIR_EINVAL, "lambda must be > 0");
  if (max_iter < 0 || !(tol >= 0) || !std::isfinite(tol)) return fail(OSSCIR_EINVAL, "need max_iter >= 0, tol >= 0");
  if (n_inner < 1) return fail(OSSCIR_EINVAL, "nested: need n_inner >= 1 (got %d)", n_inner);
  if (n_inner > 1 && !p0) return fail(OSSCIR_EINVAL, "nested: null p0");
  const WorkLayout wl = work_layout(plan->sd);
  if (state->work_bytes < wl.bp)  // the batch does not use the split back-projection's region
    return fail(OSSCIR_ESTATE, "workspace %zu < %zu bytes", state->work_bytes, wl.bp);
  HostSlot &hs = b->slots[slot];
  hs.bound = true;
  hs.plan = plan;
  hs.state = *state;
  hs.lambda = (float)lambda;
  hs.n_inner = n_inner;
  hs.p0 = n_inner > 1 ? p0 : nullptr;
  SlotStatus st{};
  st.state = kSlotRunning;
  st.max_iter = max_iter;
  st.tol = tol;
  st.rel_change = 1.0;
  b->init_status[slot] = st;
  b->status_pending[slot] = 1;
  b->dirty = true;
  OSSCIR_HIP(launch_pack(plan->sd, state->fbar, 3, (char *)state->work + wl.pack, (hipStream_t)stream),
             "batch: packing fbar");
  return OSSCIR_OK;
}

int osscir_batch_set_slot(osscir_batch b, int32_t slot, osscir_plan plan, const osscir_state *state, double lambda,
                          int32_t max_iter, double tol, osscir_stream stream) {
  return osscir_batch_set_slot_nested(b, slot, plan, state, lambda, max_iter, tol, 1, nullptr, stream);
}

int osscir_batch_clear_slot(osscir_batch b, int32_t slot) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (slot < 0 || slot >= b->max_slots) return fail(OSSCIR_EINVAL, "slot %d outside [0, %d)", slot, b->max_slots);
  b->slots[slot] = HostSlot{};
  b->init_status[slot] = SlotStatus{};
  b->status_pending[slot] = 1;
  b->dirty = true;
  return OSSCIR_OK;
}

int osscir_batch_iterate(osscir_batch b, int32_t n_iter, int32_t use_graph, osscir_stream stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (n_iter < 0) return fail(OSSCIR_EINVAL, "n_iter < 0");
  hipStream_t st = (hipStream_t)stream;
  if ((rc = flush(b, st))) return rc;
  if (n_iter == 0) return OSSCIR_OK;
  if (use_graph) {
    if (!b->graph_ok || b->graph_wide != b->any_wide || b->graph_nested != b->any_nested ||
        b->graph_spec_lds != b->spec_lds)
      if ((rc = capture(b, st))) return rc;
    for (int i = 0; i < n_iter; ++i) OSSCIR_HIP(hipGraphLaunch(b->exec, st), "batch: graph launch");
  } else {
    for (int i = 0; i < n_iter; ++i)
      if ((rc = launch_iteration(b, st))) return rc;
  }
  return OSSCIR_OK;
}

int osscir_batch_status(osscir_batch b, osscir_slot_status *out, osscir_stream stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (!out) return fail(OSSCIR_EINVAL, "null status array");
  hipStream_t st = (hipStream_t)stream;
  if ((rc = flush(b, st))) return rc;
  OSSCIR_HIP(hipMemcpyAsync(b->h_status_rb, b->d_status, (size_t)b->max_slots * sizeof(SlotStatus),
                            hipMemcpyDeviceToHost, st),
             "batch: reading slot status");
  OSSCIR_HIP(hipStreamSynchronize(st), "batch: reading slot status");
  for (int s = 0; s < b->max_slots; ++s) {
    out[s].state = b->h_status_rb[s].state;
    out[s].iters = b->h_status_rb[s].iters;
    out[s].rel_change = b->h_status_rb[s].rel_change;
  }
  return OSSCIR_OK;
}

int osscir_batch_get_config(osscir_batch b, osscir_batch_config *cfg) {
  if (!b || !cfg) return fail(OSSCIR_EINVAL, "null argument");
  *cfg = b->cfg;
  return OSSCIR_OK;
}

int osscir_batch_set_config(osscir_batch b, const osscir_batch_config *cfg) {
  if (!b || !cfg) return fail(OSSCIR_EINVAL, "null argument");
  int rc = check_config(*cfg);
  if (rc) return rc;
  b->cfg = *cfg;
  b->dirty = true;
  b->graph_ok = false;
  return OSSCIR_OK;
}

int osscir_batch_tune(osscir_batch b, int32_t iters_per_trial, osscir_batch_config *cfg_out, osscir_stream stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (iters_per_trial < 1 || iters_per_trial > 100) return fail(OSSCIR_EINVAL, "iters_per_trial outside [1, 100]");
  hipStream_t st = (hipStream_t)stream;
  if ((rc = flush(b, st))) return rc;
  OSSCIR_HIP(hipStreamSynchronize(st), "tune: synchronising");
  std::vector<int> bound;
  for (int s = 0; s < b->max_slots; ++s)
    if (b->slots[s].bound) bound.push_back(s);
  if (bound.empty()) {
    if (cfg_out) *cfg_out = b->cfg;
    return OSSCIR_OK;
  }
  // snapshot of f, fbar, y (and p0 of nested slots) and the status table
  std::vector<size_t> off(bound.size() + 1, 0);
  for (size_t i = 0; i < bound.size(); ++i) {
    const HostSlot &hs = b->slots[bound[i]];
    const ScanDesc &sd = hs.plan->sd;
    off[i + 1] = off[i] + 6 * (size_t)sd.n * sd.n + (hs.n_inner > 1 ? 7 : 4) * (size_t)sd.n_rays;
  }
  float *snap = nullptr;
  OSSCIR_HIP(hipMalloc(&snap, off.back() * sizeof(float)), "tune: snapshot allocation");
  std::vector<SlotStatus> saved(b->max_slots);
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr}, ev_end = nullptr;
  auto cleanup = [&]() {
    for (hipEvent_t &e : ev)
      if (e) (void)hipEventDestroy(e);
    if (ev_end) (void)hipEventDestroy(ev_end);
    (void)hipStreamSynchronize(st);
    (void)hipFree(snap);
  };
  auto copy_state = [&](bool save) -> int {
    for (size_t i = 0; i < bound.size(); ++i) {
      const HostSlot &hs = b->slots[bound[i]];
      const ScanDesc &sd = hs.plan->sd;
      const size_t nn3 = 3 * (size_t)sd.n * sd.n, y4 = 4 * (size_t)sd.n_rays;
      float *base = snap + off[i];
      float *bufs[4] = {hs.state.f, hs.state.fbar, hs.state.y, hs.p0};
      const size_t offs[4] = {0, nn3, 2 * nn3, 2 * nn3 + y4};
      const size_t counts[4] = {nn3, nn3, y4, 3 * (size_t)sd.n_rays};
      for (int k = 0; k < (hs.n_inner > 1 ? 4 : 3); ++k) {
        void *dst = save ? (void *)(base + offs[k]) : (void *)bufs[k];
        const void *src = save ? (const void *)bufs[k] : (const void *)(base + offs[k]);
        OSSCIR_HIP(hipMemcpyAsync(dst, src, counts[k] * sizeof(float), hipMemcpyDeviceToDevice, st), "tune: state copy");
      }
      if (!save) {
        const WorkLayout wl = work_layout(sd);
        OSSCIR_HIP(launch_pack(sd, hs.state.fbar, 3, (char *)hs.state.work + wl.pack, st), "tune: repacking fbar");
      }
    }
    return OSSCIR_OK;
  };
  auto put_status = [&](const std::vector<SlotStatus> &v) -> int {
    std::copy(v.begin(), v.end(), b->h_status);
    OSSCIR_HIP(hipMemcpyAsync(b->d_status, b->h_status, v.size() * sizeof(SlotStatus), hipMemcpyHostToDevice, st),
               "tune: status upload");
    OSSCIR_HIP(hipStreamSynchronize(st), "tune: status upload");
    return OSSCIR_OK;
  };
  if ((rc = copy_state(true))) return cleanup(), rc;
  if (hipMemcpyAsync(b->h_status_rb, b->d_status, saved.size() * sizeof(SlotStatus), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(), fail(OSSCIR_EDEVICE, "tune: reading status");
  std::copy(b->h_status_rb, b->h_status_rb + saved.size(), saved.begin());
  // during the trials the running slots run without a stopping rule
  std::vector<SlotStatus> trial = saved;
  for (SlotStatus &s : trial)
    if (s.state == kSlotRunning) s.max_iter = 0, s.tol = 0.0;
  for (hipEvent_t &e : ev)
    if (hipEventCreate(&e) != hipSuccess) return cleanup(), fail(OSSCIR_EDEVICE, "tune: event creation");
  if (hipEventCreate(&ev_end) != hipSuccess) return cleanup(), fail(OSSCIR_EDEVICE, "tune: event creation");

  struct StageCand {
    int rays, wgs, xcd;
  };
  std::vector<StageCand> fp, spec, bp;
  for (int r : {256, 128, 64})
    for (int w : {1024, 2048, 4096, 16384})
      for (int x : {1, 0}) {
        fp.push_back({r, w, x});
        spec.push_back({r, w / 2 < 512 ? 512 : w / 2, x});
      }
  for (int w : {1024, 1280, 2048, 4096, 16384})
    for (int x : {1, 0}) bp.push_back({256, w, x});
  const size_t trials = std::max(fp.size(), std::max(spec.size(), bp.size()));
  std::vector<double> t_fp(fp.size(), 1e300), t_spec(spec.size(), 1e300), t_bp(bp.size(), 1e300);
  const osscir_batch_config orig = b->cfg;
  for (size_t t = 0; t < trials && rc == OSSCIR_OK; ++t) {
    const StageCand &a = fp[t % fp.size()], &s = spec[t % spec.size()], &c = bp[t % bp.size()];
    b->cfg = osscir_batch_config{a.rays, a.wgs, a.xcd, s.rays, s.wgs, s.xcd, c.wgs, c.xcd};
    b->dirty = true;
    if ((rc = flush(b, st))) break;
    if ((rc = put_status(trial))) break;
    if ((rc = launch_iteration(b, st))) break;  // warm-up
    double sum[3] = {0.0, 0.0, 0.0};
    for (int it = 0; it < iters_per_trial && rc == OSSCIR_OK; ++it) {
      if ((rc = launch_iteration(b, st, ev))) break;
      if (hipEventRecord(ev_end, st) != hipSuccess || hipEventSynchronize(ev_end) != hipSuccess) {
        rc = fail(OSSCIR_EDEVICE, "tune: timing");
        break;
      }
      for (int k = 0; k < 3; ++k) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
        sum[k] += ms;
      }
    }
    if (rc) break;
    t_fp[t % fp.size()] = std::min(t_fp[t % fp.size()], sum[0]);
    t_spec[t % spec.size()] = std::min(t_spec[t % spec.size()], sum[1]);
    t_bp[t % bp.size()] = std::min(t_bp[t % bp.size()], sum[2]);
    if ((rc = copy_state(false))) break;
  }
  if (rc == OSSCIR_OK) {
    const size_t i = std::min_element(t_fp.begin(), t_fp.end()) - t_fp.begin();
    const size_t j = std::min_element(t_spec.begin(), t_spec.end()) - t_spec.begin();
    const size_t k = std::min_element(t_bp.begin(), t_bp.end()) - t_bp.begin();
    b->cfg = osscir_batch_config{fp[i].rays, fp[i].wgs, fp[i].xcd, spec[j].rays, spec[j].wgs, spec[j].xcd,
                                 bp[k].wgs, bp[k].xcd};
  } else {
    b->cfg = orig;
  }
  // restore the state and the status table whatever happened
  const int rc_restore = copy_state(false);
  const int rc_status = put_status(saved);
  b->dirty = true;
  b->graph_ok = false;
  cleanup();
  if (rc) return rc;
  if (rc_restore) return rc_restore;
  if (rc_status) return rc_status;
  if ((rc = flush(b, st))) return rc;
  if (cfg_out) *cfg_out = b->cfg;
  return OSSCIR_OK;
}

}  // extern "C"
