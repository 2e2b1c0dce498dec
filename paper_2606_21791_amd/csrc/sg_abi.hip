// C ABI of libsg (include/sg.h): argument validation, contexts and their
// workspaces, prepared scenes, and the orchestration of the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sg_kernels.h"
#include "sg_settings.h"

using namespace sg;

namespace {

thread_local std::string g_err;

sg_status fail(sg_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                                   \
  do {                                                                                                  \
    hipError_t _e = (expr);                                                                             \
    if (_e != hipSuccess) return fail(SG_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

#define SG_TRY(expr)                 \
  do {                               \
    sg_status _s = (expr);           \
    if (_s != SG_OK) return _s;      \
  } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int kMaxViews = 64;

int n_components(int f, int sh_degree) {
  static const int base[5] = {3, 3, 4, 1, 3};
  if (f < 5) return base[f];
  return 3 * ((sh_degree + 1) * (sh_degree + 1) - 1);
}

}  // namespace

// A device buffer that grows on demand.  Bytes are charged to the owning
// context's budget.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Buffers of the calls issued on one HIP stream.  Calls on different
// streams use different workspaces, so their device work may overlap.
struct Workspace {
  hipStream_t stream = nullptr;
  // full renders
  DevBuf rec, depth, rect, diff, flags, clamps, tile_cnt, tile_start, cursor, total, keys, keys_tmp,
      big_prims, big_tiles, big_choff, big_goff, big_split, big_map, parts, work_scene, sites_dev, box_keys, metrics_tmp;
  // batches of variants
  DevBuf vs, ovr, item_off, n_items_v, tiles, bparts, counter, arrive, gmetrics, views_tmp, ssim_tmp;
  unsigned long long* h_total = nullptr;   // pinned
  // pinned staging ring for a batch's sites and variants, read by the variant
  // prep kernel in place; slot k may be rewritten once the batch that last
  // used it (event) has completed
  static constexpr int kRing = 4;
  sg_site* h_sites[kRing] = {};
  sg_variant* h_vars[kRing] = {};
  const sg_site* d_sites[kRing] = {};      // the same memory as seen from the device
  const sg_variant* d_vars[kRing] = {};
  size_t h_sites_cap = 0, h_vars_cap = 0;
  hipEvent_t staged[kRing] = {};
  int ring = 0;
  // pipelined campaign: three buffer sets of batch work items, their
  // partials, per-variant counts and offsets, and a work counter and an
  // arrival counter each (ctl: set s at words 4s and 4s + 1)
  DevBuf st_items[3], st_parts[3], st_off[3], st_n[3], st_ctl;
  // captured incremental batches: one executable graph per shape and buffer set
  struct Graph {
    std::vector<uintptr_t> key;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
};

struct sg_ctx {
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;
  int n_cu = 256;
  int persistent_wgs_per_cu = 0;           // 0: default of the tile size
  int persistent_grid = 0;                 // total workgroups (0: per-CU count)
  int resume_spacing = 64;                 // checkpoint spacing of prepared scenes (0: none)
  bool use_graphs = true;
  std::vector<Workspace*> ws;
  std::vector<hipStream_t> campaign_streams;   // created by sg_campaign, default priority
  // device copies of a pipelined campaign's sites and variants, and the
  // states and touch records of a chunk of its variants; camp_done marks
  // the end of the campaign that last used them; camp_mu serialises
  // campaigns on one context; camp_vargs holds the per-view clean state of a
  // multi-view campaign (its host copy stays alive for the upload)
  DevBuf camp_sites, camp_vars, camp_vs, camp_ovr, camp_views, camp_vargs, camp_scene_of;
  std::vector<ViewArgs> camp_vargs_host;
  std::vector<uint16_t> camp_scene_of_host;
  // the persistent campaign path's two buffer sets (its chunks alternate
  // between them and between two streams): states, touch records, work
  // items, partials, per-variant item ranges, control words, per-view records
  DevBuf pst_vs[2], pst_ovr[2], pst_items[2], pst_parts[2], pst_off[2], pst_n[2], pst_ctl[2], pst_views[2];
  hipEvent_t camp_done = nullptr;
  std::mutex camp_mu;
  // guards ws, in_use and the timing state: sg_campaign enqueues from several
  // host threads, each on its own streams (so each on its own workspaces)
  std::mutex mu;
  // per-pass event timing (sg_ctx_timing)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[SG_N_PASSES];
};

struct sg_prep {
  sg_ctx* ctx;
  // never reused, unlike the object's address: captured graphs of the
  // incremental path are keyed on it, so a graph recorded for a destroyed
  // prepared view (its device buffers freed) never matches a new one
  uint64_t serial = 0;
  DevScene scene;
  sg_scene host_scene;
  DevCam cam;
  DevRaster ras;
  int64_t n_inst = 0;
  DevBuf rec, depth, rect, tile_cnt, tile_start, keys, frame;
  DevBuf stop, ck, ck_off, stop_key;       // resume state of the clean render
  uint32_t ck_group = 0;
};

namespace {

sg_status dev_alloc(sg_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes <= b.bytes) return SG_OK;
  bytes = std::max<size_t>(bytes, 256);
  // a buffer that has to grow again grows by half as much more, so that
  // sizes creeping up call after call (instance counts under a fault storm)
  // reallocate a logarithmic number of times
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    const size_t grown = b.p ? std::max(bytes, b.bytes + b.bytes / 2) : bytes;
    if (!ctx->budget || ctx->in_use - b.bytes + grown <= ctx->budget) bytes = grown;
    if (ctx->budget && ctx->in_use - b.bytes + bytes > ctx->budget)
      return fail(SG_E_NOMEM, "device budget exceeded");
    ctx->in_use += bytes - b.bytes;
  }
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->in_use -= bytes;
    return fail(SG_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  b.p = p;
  b.bytes = bytes;
  return SG_OK;
}

// Variants staged per campaign pre-pass (one view: 562 MB of states and touch records).
constexpr int kCampaignChunk = 1 << 19;

// dev_alloc of `reserve` bytes where the context's budget allows them (and
// they exceed `want`), else of `want`: buffers that later calls are likely
// to need larger are sized for those calls once, since growing a buffer
// frees and reallocates it, which waits for the device.
sg_status dev_reserve(sg_ctx* ctx, DevBuf& b, size_t want, size_t reserve) {
  if (reserve > want && reserve > b.bytes) {
    bool fits;
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      fits = !ctx->budget || ctx->in_use - b.bytes + reserve <= ctx->budget;
    }
    if (fits) return dev_alloc(ctx, b, reserve);
  }
  return dev_alloc(ctx, b, want);
}

void dev_free(sg_ctx* ctx, DevBuf& b) {
  if (b.p) {
    (void)hipFree(b.p);
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->in_use -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

Workspace* workspace(sg_ctx* ctx, hipStream_t st) {
  std::lock_guard<std::mutex> g(ctx->mu);
  for (Workspace* w : ctx->ws)
    if (w->stream == st) return w;
  Workspace* w = new Workspace();
  w->stream = st;
  if (hipHostMalloc((void**)&w->h_total, 8 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
    delete w;
    return nullptr;
  }
  ctx->ws.push_back(w);
  return w;
}

void free_workspace(sg_ctx* ctx, Workspace* w) {
  DevBuf* bufs[] = {&w->rec, &w->depth, &w->rect, &w->diff, &w->flags, &w->clamps, &w->tile_cnt,
                    &w->tile_start, &w->cursor, &w->total, &w->keys, &w->keys_tmp, &w->big_prims, &w->big_tiles,
                    &w->big_choff, &w->big_goff, &w->big_split, &w->big_map,
                    &w->parts, &w->work_scene, &w->sites_dev, &w->box_keys, &w->metrics_tmp, &w->vs, &w->ovr,
                    &w->item_off, &w->n_items_v, &w->tiles, &w->bparts,
                    &w->counter, &w->arrive, &w->gmetrics, &w->views_tmp, &w->ssim_tmp, &w->st_ctl};
  for (auto& g : w->graphs) (void)hipGraphExecDestroy(g.exec);
  w->graphs.clear();
  for (DevBuf* b : bufs) dev_free(ctx, *b);
  for (int k = 0; k < 3; ++k) {
    dev_free(ctx, w->st_items[k]);
    dev_free(ctx, w->st_parts[k]);
    dev_free(ctx, w->st_off[k]);
    dev_free(ctx, w->st_n[k]);
  }
  if (w->h_total) (void)hipHostFree(w->h_total);
  for (int k = 0; k < Workspace::kRing; ++k) {
    if (w->h_sites[k]) (void)hipHostFree(w->h_sites[k]);
    if (w->h_vars[k]) (void)hipHostFree(w->h_vars[k]);
    if (w->staged[k]) (void)hipEventDestroy(w->staged[k]);
  }
  delete w;
}

#define WS_OR_FAIL(W, ctx, st)                                            \
  Workspace* W = workspace(ctx, st);                                      \
  if (!W) return fail(SG_E_NOMEM, "pinned allocation for a workspace failed")

// Copy a batch's sites and variants into the next slot of the workspace's
// pinned ring (waiting for that slot's previous copies), returning the slot.
sg_status stage_batch(Workspace* w, const sg_site* sites, int n_sites, size_t site_cap, const sg_variant* vars, int B,
                      int* slot) {
  const int k = w->ring;
  w->ring = (w->ring + 1) % Workspace::kRing;
  if (site_cap > w->h_sites_cap || (size_t)B > w->h_vars_cap) {
    for (int j = 0; j < Workspace::kRing; ++j) {
      if (w->staged[j]) HIP_TRY(hipEventSynchronize(w->staged[j]));
      if (w->h_sites[j]) (void)hipHostFree(w->h_sites[j]);
      if (w->h_vars[j]) (void)hipHostFree(w->h_vars[j]);
      w->h_sites[j] = nullptr;
      w->h_vars[j] = nullptr;
    }
    const size_t sc = std::max(site_cap, w->h_sites_cap), vc = std::max((size_t)B, w->h_vars_cap);
    for (int j = 0; j < Workspace::kRing; ++j) {
      HIP_TRY(hipHostMalloc((void**)&w->h_sites[j], sc * sizeof(sg_site), hipHostMallocMapped));
      HIP_TRY(hipHostMalloc((void**)&w->h_vars[j], vc * sizeof(sg_variant), hipHostMallocMapped));
      void* d = nullptr;
      HIP_TRY(hipHostGetDevicePointer(&d, w->h_sites[j], 0));
      w->d_sites[j] = static_cast<const sg_site*>(d);
      HIP_TRY(hipHostGetDevicePointer(&d, w->h_vars[j], 0));
      w->d_vars[j] = static_cast<const sg_variant*>(d);
    }
    w->h_sites_cap = sc;
    w->h_vars_cap = vc;
    for (auto& g : w->graphs) (void)hipGraphExecDestroy(g.exec);   // their sources moved
    w->graphs.clear();
  }
  if (!w->staged[k]) HIP_TRY(hipEventCreateWithFlags(&w->staged[k], hipEventDisableTiming));
  else HIP_TRY(hipEventSynchronize(w->staged[k]));
  if (n_sites) std::memcpy(w->h_sites[k], sites, (size_t)n_sites * sizeof(sg_site));
  std::memcpy(w->h_vars[k], vars, (size_t)B * sizeof(sg_variant));
  *slot = k;
  return SG_OK;
}

// Records HIP events around the launches of one pass while timing is on.
// With `at_kernel`, the events are instead handed to a single kernel launch
// (a, b), which records them at that kernel's own start and end.
struct PassScope {
  sg_ctx* c;
  int pass;
  hipStream_t st;
  bool at_kernel = false;
  hipEvent_t a = nullptr, b = nullptr;
  static hipEvent_t get(sg_ctx* c) {
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->ev_pool.empty()) {
      hipEvent_t e = c->ev_pool.back();
      c->ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  PassScope(sg_ctx* c_, int pass_, hipStream_t st_, bool at_kernel_ = false)
      : c(c_), pass(pass_), st(st_), at_kernel(at_kernel_) {
    if (!c->timing) return;
    a = get(c);
    b = get(c);
    if (a && b && !at_kernel) (void)hipEventRecord(a, st);
  }
  ~PassScope() {
    if (a && b) {
      if (!at_kernel) (void)hipEventRecord(b, st);
      std::lock_guard<std::mutex> g(c->mu);
      c->pending[pass].push_back({a, b});
    }
  }
};

template <class T>
T* P(const DevBuf& b) {
  return reinterpret_cast<T*>(b.p);
}

sg_status check_last(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return SG_OK;
}

sg_status to_dev_scene(const sg_scene* s, DevScene* d) {
  if (!s) return fail(SG_E_INVAL, "scene is NULL");
  if (s->n < 1) return fail(SG_E_INVAL, "scene.n must be >= 1");
  if (s->sh_degree < 0 || s->sh_degree > 3) return fail(SG_E_INVAL, "scene.sh_degree must be 0..3");
  if (s->dtype < SG_F32 || s->dtype > SG_BF16) return fail(SG_E_INVAL, "scene.dtype invalid");
  for (int f = 0; f < 6; ++f) {
    const int C = n_components(f, s->sh_degree);
    d->ncomp[f] = C;
    d->ptr[f] = s->ptr[f];
    d->ps[f] = s->prim_stride[f];
    d->cs[f] = s->comp_stride[f];
    if (C == 0) continue;
    if (!s->ptr[f]) return fail(SG_E_INVAL, "scene.ptr[" + std::to_string(f) + "] is NULL");
    if (s->prim_stride[f] < 0 || s->comp_stride[f] < 0) return fail(SG_E_INVAL, "negative stride");
    if (s->dtype != SG_F32 && (reinterpret_cast<uintptr_t>(s->ptr[f]) & 3u))
      return fail(SG_E_INVAL, "16-bit fields must start on a 4-byte boundary");
  }
  d->n = s->n;
  d->sh_degree = s->sh_degree;
  d->dtype = s->dtype;
  return SG_OK;
}

int64_t field_extent(const DevScene& s, int f) {
  if (s.ncomp[f] == 0) return 0;
  return (int64_t)(s.n - 1) * s.ps[f] + (int64_t)(s.ncomp[f] - 1) * s.cs[f] + 1;
}

sg_status to_dev_cam(const sg_camera* c, DevCam* d) {
  if (!c) return fail(SG_E_INVAL, "camera is NULL");
  if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384)
    return fail(SG_E_INVAL, "camera size out of range");
  if (!(c->fx > 0) || !(c->fy > 0)) return fail(SG_E_INVAL, "focal lengths must be positive");
  if (!(c->near_z > 0) || !(c->far_z > c->near_z)) return fail(SG_E_INVAL, "need 0 < near < far");
  for (int i = 0; i < 9; ++i) d->R[i] = c->R[i];
  for (int i = 0; i < 3; ++i) d->t[i] = c->t[i];
  d->fx = c->fx; d->fy = c->fy; d->cx = c->cx; d->cy = c->cy;
  d->nearz = c->near_z; d->farz = c->far_z;
  for (int i = 0; i < 3; ++i) d->campos[i] = -(c->R[0 * 3 + i] * c->t[0] + c->R[1 * 3 + i] * c->t[1] + c->R[2 * 3 + i] * c->t[2]);
  d->limx = 1.3 * (0.5 * c->width) / c->fx;
  d->limy = 1.3 * (0.5 * c->height) / c->fy;
  d->W = c->width;
  d->H = c->height;
  return SG_OK;
}

sg_status to_dev_raster(const sg_raster* r, int W, int H, DevRaster* d) {
  sg_raster def = {16, 0.99f, 1.0f / 255.0f, 1e-4f, 9.0f, 0.3f, {1.f, 1.f, 1.f}};
  if (!r) r = &def;
  int tile = r->tile == 0 ? 16 : r->tile;
  if (tile != 8 && tile != 16 && tile != 32) return fail(SG_E_INVAL, "raster.tile must be 8, 16 or 32");
  if (!(r->alpha_max > 0 && r->alpha_max < 1) || !(r->alpha_min > 0 && r->alpha_min < r->alpha_max) ||
      !(r->t_min > 0 && r->t_min < 1) || !(r->cut_q > 0) || !(r->dilation >= 0))
    return fail(SG_E_INVAL, "raster constants out of range");
  d->tile = tile;
  d->tiles_x = (W + tile - 1) / tile;
  d->tiles_y = (H + tile - 1) / tile;
  d->n_tiles = d->tiles_x * d->tiles_y;
  d->amax = r->alpha_max; d->amin = r->alpha_min; d->tmin = r->t_min; d->cutq = r->cut_q; d->dil = r->dilation;
  for (int i = 0; i < 3; ++i) d->bg[i] = r->bg[i];
  d->qcut2 = (float)((double)r->cut_q * 0.72134752044448170);
  return SG_OK;
}

sg_status to_dev_box(const sg_box* b, uint32_t mask, const DevScene& s, DevBox* d) {
  std::memset(d, 0, sizeof(*d));
  if (!b || !mask) return SG_OK;
  if (mask & ~0x3Fu) return fail(SG_E_INVAL, "box field mask has bits above 5");
  if (b->mode != SG_BOX_GLOBAL && b->mode != SG_BOX_PER_PRIM) return fail(SG_E_INVAL, "box.mode invalid");
  if (b->dtype != s.dtype) return fail(SG_E_INVAL, "box dtype differs from the scene's");
  for (int f = 0; f < 6; ++f) {
    if (!((mask >> f) & 1u) || s.ncomp[f] == 0) continue;
    if (!b->lo[f] || !b->hi[f]) return fail(SG_E_INVAL, "box bounds of a masked field are NULL");
    d->lo[f] = b->lo[f];
    d->hi[f] = b->hi[f];
  }
  d->mode = b->mode;
  d->dtype = b->dtype;
  for (int f = 0; f < 6; ++f)
    if (((mask >> f) & 1u) && s.ncomp[f] > 0) d->mask |= 1u << f;
  return SG_OK;
}

sg_status validate_sites(const DevScene& s, const sg_site* sites, int n) {
  if (n < 0) return fail(SG_E_INVAL, "negative site count");
  if (n > 0 && !sites) return fail(SG_E_INVAL, "sites is NULL");
  const int width = s.dtype == SG_F32 ? 32 : 16;
  for (int k = 0; k < n; ++k) {
    const sg_site& x = sites[k];
    if (x.field > 5 || s.ncomp[x.field] == 0) return fail(SG_E_INVAL, "site " + std::to_string(k) + ": field absent");
    if (x.comp >= s.ncomp[x.field]) return fail(SG_E_INVAL, "site " + std::to_string(k) + ": component out of range");
    if (x.prim >= (uint32_t)s.n) return fail(SG_E_INVAL, "site " + std::to_string(k) + ": primitive out of range");
    if (x.bit >= width) return fail(SG_E_INVAL, "site " + std::to_string(k) + ": bit out of range");
  }
  return SG_OK;
}

sg_status stage_sites(sg_ctx* ctx, const sg_site* sites, int n, DevBuf& dst, hipStream_t st) {
  if (n <= 0) return SG_OK;
  SG_TRY(dev_alloc(ctx, dst, (size_t)n * sizeof(sg_site)));
  HIP_TRY(hipMemcpyAsync(dst.p, sites, (size_t)n * sizeof(sg_site), hipMemcpyHostToDevice, st));
  return SG_OK;
}

// Full render of a scene: project (with optional clamp-on-load), bin, sort,
// composite (with metric partials against `clean` when given).  The record and
// list buffers are either the context's workspaces or a prepared scene's.
sg_status full_render(sg_ctx* ctx, Workspace* W, const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                      DevBuf& rec, DevBuf& depth, DevBuf& rect, DevBuf& tile_cnt,
                      DevBuf& tile_start, DevBuf& keys, float* image, const float* clean, Partial* parts,
                      hipStream_t st, int64_t* n_inst_out, sg_prep* resume = nullptr) {
  const int64_t n = s.n;
  SG_TRY(dev_alloc(ctx, rec, n * sizeof(Rec)));
  SG_TRY(dev_alloc(ctx, depth, n * sizeof(uint32_t)));
  SG_TRY(dev_alloc(ctx, rect, n * sizeof(uint2)));
  const int64_t diff_n = (int64_t)(ras.tiles_x + 1) * (ras.tiles_y + 1);
  SG_TRY(dev_alloc(ctx, W->diff, diff_n * sizeof(int32_t)));
  SG_TRY(dev_alloc(ctx, W->flags, 16));
  SG_TRY(dev_alloc(ctx, W->clamps, 16));
  SG_TRY(dev_alloc(ctx, tile_cnt, ras.n_tiles * sizeof(uint32_t)));
  SG_TRY(dev_alloc(ctx, tile_start, ras.n_tiles * sizeof(uint32_t)));
  SG_TRY(dev_alloc(ctx, W->cursor, ras.n_tiles * sizeof(uint32_t)));
  SG_TRY(dev_alloc(ctx, W->total, 8 * sizeof(unsigned long long)));
  SG_TRY(dev_alloc(ctx, W->big_prims, n * sizeof(uint32_t)));
  SG_TRY(dev_alloc(ctx, W->big_tiles, ras.n_tiles * sizeof(uint32_t)));
  SG_TRY(dev_alloc(ctx, W->big_choff, (ras.n_tiles + 1) * sizeof(uint32_t)));
  SG_TRY(dev_alloc(ctx, W->big_goff, (ras.n_tiles + 1) * sizeof(uint32_t)));
  launch_fill_u32(P<uint32_t>(W->diff), 0u, diff_n, st);
  launch_fill_u32(P<uint32_t>(W->flags), 0u, 4, st);
  launch_fill_u32(P<uint32_t>(W->clamps), 0u, 4, st);
  ProjBuffers pb{P<Rec>(rec), P<uint32_t>(depth), P<uint2>(rect),
                 P<int32_t>(W->diff), P<uint32_t>(W->flags), P<unsigned long long>(W->clamps)};
  {
    PassScope ps(ctx, SG_PASS_PROJECT, st);
    launch_project(s, box, cam, ras, pb, ctx->n_cu, st);
  }
  BinBuffers bb{P<int32_t>(W->diff), P<uint32_t>(tile_cnt), P<uint32_t>(tile_start), P<uint32_t>(W->cursor),
                P<unsigned long long>(W->total), nullptr, nullptr, P<uint32_t>(W->big_prims),
                P<uint32_t>(W->big_tiles), P<uint32_t>(W->big_choff), P<uint32_t>(W->big_goff), nullptr, nullptr,
                0};
  {
    PassScope ps(ctx, SG_PASS_BIN, st);
    launch_tile_prefix(ras, bb, st);
  }
  SG_TRY(check_last("project/binning launch"));
  HIP_TRY(hipMemcpyAsync(W->h_total, W->total.p, 6 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int64_t n_inst = (int64_t)W->h_total[0];
  if (n_inst >= (int64_t)0xffffffffu) return fail(SG_E_UNSUPPORTED, "more than 2^32 primitive-tile instances");
  SG_TRY(dev_alloc(ctx, keys, std::max<int64_t>(n_inst, 1) * sizeof(uint64_t)));
  SG_TRY(dev_alloc(ctx, W->keys_tmp, std::max<int64_t>(n_inst, 1) * sizeof(uint64_t)));
  bb.keys = P<uint64_t>(keys);
  bb.keys_tmp = P<uint64_t>(W->keys_tmp);
  bb.capacity = n_inst;
  {
    PassScope ps(ctx, SG_PASS_BIN, st);
    launch_emit(s.n, P<uint32_t>(depth), P<uint2>(rect), ras, bb, ctx->n_cu, st);
  }
  {
    PassScope ps(ctx, SG_PASS_SORT, st);
    if (W->h_total[3] > (1ull << 31)) return fail(SG_E_UNSUPPORTED, "a tile list longer than 2^31 entries");
    SG_TRY(dev_alloc(ctx, W->big_split, (W->h_total[5] + 1) * sizeof(uint32_t)));
    SG_TRY(dev_alloc(ctx, W->big_map, (W->h_total[5] + W->h_total[4] + 1) * sizeof(uint2)));
    bb.big_split = P<uint32_t>(W->big_split);
    bb.big_map = P<uint2>(W->big_map);
    launch_tile_sort(ras, bb, W->h_total, ctx->n_cu, st);
  }
  CompArgs ca{P<Rec>(rec), P<uint32_t>(tile_start), P<uint32_t>(tile_cnt),
              P<uint64_t>(keys), clean, image, parts, ras, cam.W, cam.H};
  if (resume && resume->ck_group) {
    // checkpoint slots per tile: floor(count / spacing), laid out tile after tile
    const uint32_t g = resume->ck_group;
    std::vector<uint32_t> cnt(ras.n_tiles), off(ras.n_tiles);
    HIP_TRY(hipMemcpyAsync(cnt.data(), tile_cnt.p, ras.n_tiles * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    uint64_t slots = 0;
    for (int t = 0; t < ras.n_tiles; ++t) {
      off[t] = (uint32_t)slots;
      slots += cnt[t] / g;
    }
    if (slots >= 0xffffffffull) return fail(SG_E_UNSUPPORTED, "too many checkpoints; raise the spacing");
    const size_t bs = (size_t)ras.tile * ras.tile;
    SG_TRY(dev_alloc(ctx, resume->stop, (size_t)cam.W * cam.H * sizeof(uint64_t)));
    SG_TRY(dev_alloc(ctx, resume->ck_off, ras.n_tiles * sizeof(uint32_t)));
    SG_TRY(dev_alloc(ctx, resume->stop_key, ras.n_tiles * sizeof(uint64_t)));
    SG_TRY(dev_alloc(ctx, resume->ck, std::max<size_t>(slots, 1) * bs * sizeof(float4)));
    HIP_TRY(hipMemcpyAsync(resume->ck_off.p, off.data(), ras.n_tiles * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));        // `off` is released on return
    ca.stop_out = P<uint64_t>(resume->stop);
    ca.ck_out = P<float4>(resume->ck);
    ca.ck_off = P<uint32_t>(resume->ck_off);
    ca.stop_key_out = P<uint64_t>(resume->stop_key);
    ca.ck_group = g;
  }
  {
    PassScope ps(ctx, SG_PASS_COMPOSITE_FULL, st);
    launch_composite_full(ca, st);
  }
  SG_TRY(check_last("render launch"));
  if (n_inst_out) *n_inst_out = n_inst;
  return SG_OK;
}

}  // namespace

// Scratch memory of the allocation-free metrics call (sg_metrics_noalloc):
// the per-chunk metric partials of up to kScratchBytes / sizeof(Partial)
// (variant, chunk) pairs.  Each device that the library runs on holds its own
// copy until the process ends.  Host code never passes `scratch` itself (its
// host-side name is not a device address): sg_ctx_create records, once per
// device and with that device current, the address hipGetSymbolAddress gives
// for it, and the call uses that address.
constexpr size_t kScratchBytes = (size_t)4 << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kScratchDevices] = {};

static void* scratch_of(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return device >= 0 && device < kScratchDevices ? g_scratch_dev[device] : nullptr;
}

extern "C" {

const char* sg_last_error(void) { return g_err.c_str(); }

sg_status sg_ctx_create(int32_t device, size_t hbm_budget_bytes, sg_ctx** out) {
  if (!out) return fail(SG_E_INVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return fail(SG_E_DEVICE, "no HIP device");
  if (device < 0 || device >= count) return fail(SG_E_INVAL, "device index out of range");
  HIP_TRY(hipSetDevice(device));
  if (device < kScratchDevices) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[device]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(SG_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      g_scratch_dev[device] = p;
    }
  }
  sg_ctx* c = new sg_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0) c->n_cu = ncu;
  *out = c;
  return SG_OK;
}

void sg_ctx_destroy(sg_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (Workspace* w : c->ws) free_workspace(c, w);
  c->ws.clear();
  for (hipStream_t st : c->campaign_streams) (void)hipStreamDestroy(st);
  dev_free(c, c->camp_sites);
  dev_free(c, c->camp_vars);
  dev_free(c, c->camp_vs);
  dev_free(c, c->camp_ovr);
  dev_free(c, c->camp_views);
  dev_free(c, c->camp_vargs);
  dev_free(c, c->camp_scene_of);
  for (int k = 0; k < 2; ++k)
    for (DevBuf* b : {&c->pst_vs[k], &c->pst_ovr[k], &c->pst_items[k], &c->pst_parts[k], &c->pst_off[k], &c->pst_n[k],
                      &c->pst_ctl[k], &c->pst_views[k]})
      dev_free(c, *b);
  if (c->camp_done) (void)hipEventDestroy(c->camp_done);
  for (int p = 0; p < SG_N_PASSES; ++p)
    for (auto& pr : c->pending[p]) c->ev_pool.insert(c->ev_pool.end(), {pr.first, pr.second});
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
}

size_t sg_ctx_bytes(const sg_ctx* c) { return c ? c->in_use : 0; }

}  // extern "C"

SgSettings sg_settings_get(const sg_ctx* c) {
  return {c->device, c->persistent_wgs_per_cu, c->resume_spacing, c->use_graphs ? 1 : 0, c->persistent_grid};
}

sg_status sg_fail(sg_status code, const char* msg) { return fail(code, msg); }

void sg_settings_set(sg_ctx* c, const SgSettings& s) {
  c->persistent_wgs_per_cu = s.wgs_per_cu;
  c->persistent_grid = s.grid;
  c->resume_spacing = s.resume_spacing;
  c->use_graphs = s.graphs != 0;
}

extern "C" {

sg_status sg_ctx_set_resume(sg_ctx* c, int32_t spacing) {
  if (!c) return fail(SG_E_INVAL, "ctx is NULL");
  if (spacing != 0 && (spacing < 16 || spacing > 65536)) return fail(SG_E_INVAL, "resume spacing must be 0 or in [16, 65536]");
  c->resume_spacing = spacing;
  return SG_OK;
}

sg_status sg_ctx_set_persistent_grid(sg_ctx* c, int32_t total_wgs) {
  if (!c || total_wgs < 0 || total_wgs > 65536) return fail(SG_E_INVAL, "total_wgs must be 0..65536");
  c->persistent_grid = total_wgs;
  return SG_OK;
}

sg_status sg_ctx_set_persistent(sg_ctx* c, int32_t wgs_per_cu) {
  if (!c || wgs_per_cu < 0 || wgs_per_cu > 64) return fail(SG_E_INVAL, "wgs_per_cu must be 0..64");
  c->persistent_wgs_per_cu = wgs_per_cu;
  return SG_OK;
}

sg_status sg_ctx_set_graphs(sg_ctx* c, int32_t enable) {
  if (!c) return fail(SG_E_INVAL, "ctx is NULL");
  c->use_graphs = enable != 0;
  return SG_OK;
}

sg_status sg_ctx_timing(sg_ctx* c, int32_t enable) {
  if (!c) return fail(SG_E_INVAL, "ctx is NULL");
  c->timing = enable != 0;
  return SG_OK;
}

sg_status sg_ctx_pass_times(sg_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return fail(SG_E_INVAL, "NULL argument");
  for (int p = 0; p < SG_N_PASSES; ++p) {
    ms[p] = 0.0;
    launches[p] = 0;
    for (auto& pr : c->pending[p]) {
      HIP_TRY(hipEventSynchronize(pr.second));
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second));
      ms[p] += t;
      launches[p] += 1;
      c->ev_pool.push_back(pr.first);
      c->ev_pool.push_back(pr.second);
    }
    c->pending[p].clear();
  }
  return SG_OK;
}

sg_status sg_cast(sg_ctx* ctx, const float* src, void* dst, int64_t n, int32_t dtype, int32_t rounding, void* stream) {
  if (!ctx) return fail(SG_E_INVAL, "ctx is NULL");
  if (n < 0 || (n > 0 && (!src || !dst))) return fail(SG_E_INVAL, "bad cast buffers");
  if (dtype < SG_F32 || dtype > SG_BF16 || rounding < SG_RNE || rounding > SG_RU) return fail(SG_E_INVAL, "bad dtype/rounding");
  if (n == 0) return SG_OK;
  launch_cast(src, dst, n, dtype, rounding, S(stream));
  return check_last("sg_cast");
}

sg_status sg_inject(sg_ctx* ctx, const sg_scene* scene, const sg_site* sites, int32_t n, uint32_t* saved, void* stream) {
  if (!ctx) return fail(SG_E_INVAL, "ctx is NULL");
  DevScene s;
  SG_TRY(to_dev_scene(scene, &s));
  SG_TRY(validate_sites(s, sites, n));
  if (n == 0) return SG_OK;
  WS_OR_FAIL(W, ctx, S(stream));
  SG_TRY(stage_sites(ctx, sites, n, W->sites_dev, S(stream)));
  launch_inject(s, P<sg_site>(W->sites_dev), n, saved, S(stream));
  return check_last("sg_inject");
}

sg_status sg_restore(sg_ctx* ctx, const sg_scene* scene, const sg_site* sites, int32_t n, const uint32_t* saved,
                     void* stream) {
  (void)saved;
  return sg_inject(ctx, scene, sites, n, nullptr, stream);
}

sg_status sg_guard_box(sg_ctx* ctx, const sg_scene* clean, uint32_t field_mask, sg_box* out, void* stream) {
  if (!ctx || !out) return fail(SG_E_INVAL, "ctx/out is NULL");
  DevScene s;
  SG_TRY(to_dev_scene(clean, &s));
  if (field_mask & ~0x3Fu) return fail(SG_E_INVAL, "field mask has bits above 5");
  if (out->mode != SG_BOX_GLOBAL) return fail(SG_E_INVAL, "sg_guard_box fills a SG_BOX_GLOBAL box");
  if (out->dtype != s.dtype) return fail(SG_E_INVAL, "box dtype differs from the scene's");
  for (int f = 0; f < 6; ++f)
    if (((field_mask >> f) & 1u) && s.ncomp[f] > 0 && (!out->lo[f] || !out->hi[f]))
      return fail(SG_E_INVAL, "box bounds of a masked field are NULL");
  hipStream_t st = S(stream);
  WS_OR_FAIL(W, ctx, st);
  SG_TRY(dev_alloc(ctx, W->box_keys, 2 * 64 * sizeof(uint32_t)));
  for (int f = 0; f < 6; ++f) {
    if (!((field_mask >> f) & 1u) || s.ncomp[f] == 0) continue;
    uint32_t* kmin = P<uint32_t>(W->box_keys);
    uint32_t* kmax = kmin + 64;
    launch_fill_u32(kmin, 0xffffffffu, 64, st);
    launch_fill_u32(kmax, 0u, 64, st);
    launch_box_reduce(s, f, kmin, kmax, st);
    launch_box_finalize(kmin, kmax, s.ncomp[f], s.dtype, out->lo[f], out->hi[f], st);
  }
  return check_last("sg_guard_box");
}

sg_status sg_guard(sg_ctx* ctx, const sg_scene* scene, const sg_box* box, uint32_t field_mask,
                   uint64_t health_threshold, uint64_t* clamp_count, uint32_t* health_alert, void* stream) {
  if (!ctx || !box || !clamp_count) return fail(SG_E_INVAL, "ctx/box/clamp_count is NULL");
  DevScene s;
  SG_TRY(to_dev_scene(scene, &s));
  DevBox b;
  SG_TRY(to_dev_box(box, field_mask, s, &b));
  hipStream_t st = S(stream);
  launch_fill_u32(reinterpret_cast<uint32_t*>(clamp_count), 0u, 2, st);
  {
    PassScope ps(ctx, SG_PASS_GUARD, st);
    // rows of contiguous primitives: one vectorised launch (with a
    // per-primitive box, when its rows share the scene rows' alignment);
    // anything else: the per-field kernel
    GuardRows gr;
    gr.n_rows = 0;
    for (int f = 0; f < 6; ++f) {
      if (!((b.mask >> f) & 1u)) continue;
      bool rows = s.ps[f] == 1 && gr.n_rows + s.ncomp[f] <= 64;
      if (b.mode == SG_BOX_PER_PRIM)
        rows = rows && s.cs[f] == s.n && ((uintptr_t)s.ptr[f] & 15) == 0 && ((uintptr_t)b.lo[f] & 15) == 0 &&
               ((uintptr_t)b.hi[f] & 15) == 0;
      if (rows) {
        for (int c = 0; c < s.ncomp[f]; ++c) {
          gr.f[gr.n_rows] = f;
          gr.c[gr.n_rows] = c;
          ++gr.n_rows;
        }
      } else {
        launch_guard(s, b, f, reinterpret_cast<unsigned long long*>(clamp_count), st);
      }
    }
    launch_guard_rows(s, b, gr, reinterpret_cast<unsigned long long*>(clamp_count), st);
  }
  if (health_alert) launch_health(reinterpret_cast<unsigned long long*>(clamp_count), health_threshold, health_alert, st);
  return check_last("sg_guard");
}

sg_status sg_render(sg_ctx* ctx, const sg_scene* scene, const sg_camera* cam, const sg_raster* raster, const sg_box* box,
                    uint32_t box_field_mask, float* image_out, const float* clean_frame, sg_metrics_t* metrics_out,
                    void* stream) {
  if (!ctx) return fail(SG_E_INVAL, "ctx is NULL");
  DevScene s;
  DevCam c;
  DevRaster r;
  DevBox b;
  SG_TRY(to_dev_scene(scene, &s));
  SG_TRY(to_dev_cam(cam, &c));
  SG_TRY(to_dev_raster(raster, c.W, c.H, &r));
  SG_TRY(to_dev_box(box, box_field_mask, s, &b));
  if (metrics_out && !clean_frame) return fail(SG_E_INVAL, "metrics need a clean frame");
  hipStream_t st = S(stream);
  WS_OR_FAIL(W, ctx, st);
  Partial* parts = nullptr;
  if (clean_frame) {
    SG_TRY(dev_alloc(ctx, W->parts, (size_t)r.n_tiles * sizeof(Partial)));
    parts = P<Partial>(W->parts);
  }
  SG_TRY(full_render(ctx, W, s, b, c, r, W->rec, W->depth, W->rect, W->tile_cnt, W->tile_start,
                     W->keys, image_out, clean_frame, parts, st, nullptr));
  if (metrics_out)
    launch_reduce_metrics(parts, nullptr, nullptr, (uint32_t)r.n_tiles, nullptr, P<uint32_t>(W->flags),
                          P<unsigned long long>(W->clamps), (uint32_t)(c.W * c.H), metrics_out, 1, 1u, st,
                          r.tiles_x, r.tiles_y);
  return check_last("sg_render");
}

sg_status sg_prepare(sg_ctx* ctx, const sg_scene* clean, const sg_camera* cam, const sg_raster* raster, sg_prep** out,
                     void* stream) {
  if (!ctx || !out) return fail(SG_E_INVAL, "ctx/out is NULL");
  *out = nullptr;
  static std::atomic<uint64_t> next_serial{1};
  sg_prep* p = new sg_prep();
  p->ctx = ctx;
  p->serial = next_serial.fetch_add(1);
  sg_status rc = to_dev_scene(clean, &p->scene);
  if (rc == SG_OK) rc = to_dev_cam(cam, &p->cam);
  if (rc == SG_OK) rc = to_dev_raster(raster, p->cam.W, p->cam.H, &p->ras);
  if (rc != SG_OK) {
    delete p;
    return rc;
  }
  p->host_scene = *clean;
  p->ck_group = (uint32_t)ctx->resume_spacing;
  DevBox nobox;
  std::memset(&nobox, 0, sizeof(nobox));
  hipStream_t st = S(stream);
  Workspace* W = workspace(ctx, st);
  rc = W ? dev_alloc(ctx, p->frame, (size_t)p->cam.W * p->cam.H * 3 * sizeof(float)) : SG_E_NOMEM;
  if (rc == SG_OK)
    rc = full_render(ctx, W, p->scene, nobox, p->cam, p->ras, p->rec, p->depth, p->rect, p->tile_cnt,
                     p->tile_start, p->keys, P<float>(p->frame), nullptr, nullptr, st, &p->n_inst, p);
  if (rc != SG_OK) {
    sg_prep_destroy(p);
    return rc;
  }
  *out = p;
  return SG_OK;
}

void sg_prep_destroy(sg_prep* p) {
  if (!p) return;
  sg_ctx* c = p->ctx;
  (void)hipDeviceSynchronize();
  DevBuf* bufs[] = {&p->rec, &p->depth, &p->rect, &p->tile_cnt,
                    &p->tile_start, &p->keys, &p->frame, &p->stop,  &p->ck,   &p->ck_off, &p->stop_key};
  for (DevBuf* b : bufs) dev_free(c, *b);
  delete p;
}

const float* sg_prep_frame(const sg_prep* p) { return p ? reinterpret_cast<const float*>(p->frame.p) : nullptr; }
int64_t sg_prep_instances(const sg_prep* p) { return p ? p->n_inst : -1; }

sg_status sg_prep_copy_frame(const sg_prep* p, float* dst, void* stream) {
  if (!p || !dst) return fail(SG_E_INVAL, "prep/dst is NULL");
  HIP_TRY(hipMemcpyAsync(dst, p->frame.p, (size_t)p->cam.W * p->cam.H * 3 * sizeof(float), hipMemcpyDeviceToDevice,
                         S(stream)));
  return SG_OK;
}

// Device buffers of an incremental batch of up to B variants on workspace W.
static sg_status alloc_batch(sg_ctx* ctx, Workspace* W, const sg_prep* prep, int B, hipStream_t st) {
  const DevRaster& ras = prep->ras;
  SG_TRY(dev_alloc(ctx, W->vs, (size_t)B * sizeof(VariantState)));
  SG_TRY(dev_alloc(ctx, W->ovr, (size_t)B * kRecSlots * sizeof(Rec)));
  SG_TRY(dev_alloc(ctx, W->item_off, (size_t)(B + 1) * sizeof(uint32_t)));
  SG_TRY(dev_alloc(ctx, W->n_items_v, (size_t)B * sizeof(uint32_t)));
  SG_TRY(dev_alloc(ctx, W->counter, 16));
  SG_TRY(dev_alloc(ctx, W->tiles, (size_t)B * ras.n_tiles * sizeof(uint4)));
  if (!W->arrive.p) {
    SG_TRY(dev_alloc(ctx, W->arrive, 16));
    launch_fill_u32(P<uint32_t>(W->arrive), 0u, 4, st);   // the variant prep returns it to zero
  }
  SG_TRY(dev_alloc(ctx, W->bparts, (size_t)B * ras.n_tiles * sizeof(Partial)));
  return SG_OK;
}

static BatchBuffers batch_buffers(Workspace* W, const sg_prep* prep, const sg_site* d_sites, const sg_variant* d_vars,
                                  int B) {
  const DevRaster& ras = prep->ras;
  BatchBuffers bb{d_sites, d_vars, B, P<VariantState>(W->vs), P<Rec>(W->ovr), P<uint32_t>(W->item_off),
                  P<uint32_t>(W->n_items_v),
                  P<uint4>(W->tiles), P<uint32_t>(W->counter), P<uint32_t>(W->arrive), ras.tiles_x, ras.tiles_y,
                  ras.n_tiles, prep->ck_group ? P<uint64_t>(prep->stop_key) : nullptr, P<uint32_t>(prep->tile_start),
                  P<uint32_t>(prep->tile_cnt)};
  return bb;
}

static CompArgs item_comp_args(Workspace* W, const sg_prep* prep, float* images_out) {
  CompArgs ca{P<Rec>(prep->rec), P<uint32_t>(prep->tile_start),
              P<uint32_t>(prep->tile_cnt), P<uint64_t>(prep->keys), P<float>(prep->frame), images_out,
              P<Partial>(W->bparts), prep->ras, prep->cam.W, prep->cam.H};
  if (prep->ck_group) {
    ca.stop = P<uint64_t>(prep->stop);
    ca.ck = P<float4>(prep->ck);
    ca.ck_off = P<uint32_t>(prep->ck_off);
    ca.stop_key = P<uint64_t>(prep->stop_key);
    ca.ck_group = prep->ck_group;
  }
  return ca;
}

static ItemArgs item_args(const sg_ctx* ctx, Workspace* W, const sg_prep* prep, int B) {
  const int tile = prep->ras.tile;
  const int per_cu = ctx->persistent_wgs_per_cu > 0 ? ctx->persistent_wgs_per_cu
                                                    : (tile == 32 ? 2 : (tile == 16 ? 8 : 16));
  ItemArgs it{P<VariantState>(W->vs), P<Rec>(W->ovr), P<uint4>(W->tiles), P<uint32_t>(W->item_off),
              P<uint32_t>(W->counter), (int64_t)prep->cam.W * prep->cam.H * 3,
              ctx->persistent_grid > 0 ? ctx->persistent_grid : ctx->n_cu * per_cu, B};
  return it;
}

sg_status sg_render_batch(sg_ctx* ctx, sg_prep* prep, const sg_site* sites, int32_t n_sites, const sg_variant* variants,
                          int32_t B, const sg_box* box, uint32_t box_field_mask, float* images_out,
                          sg_metrics_t* metrics_out, int32_t mode, void* stream) {
  if (!ctx || !prep || !metrics_out) return fail(SG_E_INVAL, "ctx/prep/metrics_out is NULL");
  if (prep->ctx != ctx && prep->ctx->device != ctx->device) return fail(SG_E_INVAL, "prep is on another device");
  if (B < 0 || (B > 0 && !variants)) return fail(SG_E_INVAL, "bad variants");
  if (B > kMaxBatch) return fail(SG_E_INVAL, "at most 2048 variants per launch (sg_campaign splits larger sets)");
  if (mode != SG_INCREMENTAL && mode != SG_FULL) return fail(SG_E_INVAL, "bad mode");
  const DevScene& s = prep->scene;
  SG_TRY(validate_sites(s, sites, n_sites));
  DevBox b;
  SG_TRY(to_dev_box(box, box_field_mask, s, &b));
  std::vector<int> full_idx;
  for (int v = 0; v < B; ++v) {
    const sg_variant& x = variants[v];
    if ((uint64_t)x.site_off + x.n_sites > (uint64_t)n_sites) return fail(SG_E_INVAL, "variant " + std::to_string(v) + ": sites out of range");
    if (x.guard && !b.mask) return fail(SG_E_INVAL, "variant " + std::to_string(v) + ": guard requested without a box");
    if (x.protect > SG_PROTECT_VOTE) return fail(SG_E_INVAL, "variant " + std::to_string(v) + ": unknown protect mode");
    std::vector<uint32_t> prims;
    bool full = mode == SG_FULL;
    for (uint32_t k = 0; k < x.n_sites && !full; ++k) {
      const uint32_t pr = sites[x.site_off + k].prim;
      if (std::find(prims.begin(), prims.end(), pr) == prims.end()) {
        prims.push_back(pr);
        if ((int)prims.size() > kMaxTouch) full = true;
      }
    }
    if (full) full_idx.push_back(v);
  }
  if (B == 0) return SG_OK;
  hipStream_t st = S(stream);
  WS_OR_FAIL(W, ctx, st);
  const DevRaster& ras = prep->ras;
  const int64_t frame_floats = (int64_t)prep->cam.W * prep->cam.H * 3;

  // incremental pipeline over all B (variants needing the full path get no items)
  if ((int)full_idx.size() < B) {
    const size_t site_cap = std::max<size_t>((size_t)n_sites, std::max<size_t>(64, (size_t)4 * B));
    SG_TRY(alloc_batch(ctx, W, prep, B, st));
    SG_TRY(dev_alloc(ctx, W->gmetrics, (size_t)B * sizeof(sg_metrics_t)));
    int slot = 0;
    SG_TRY(stage_batch(W, sites, n_sites, site_cap, variants, B, &slot));
    const int per_cu = ctx->persistent_wgs_per_cu;
    // a graph is replayed when every variant is incremental, no images are
    // requested and timing is off; it writes its metrics to the workspace
    const bool graph = ctx->use_graphs && !ctx->timing && full_idx.empty() && !images_out && st != nullptr;
    sg_metrics_t* mout = graph ? P<sg_metrics_t>(W->gmetrics) : metrics_out;
    auto enqueue = [&]() -> sg_status {
      if (images_out)
        for (int v = 0; v < B; ++v)
          HIP_TRY(hipMemcpyAsync(images_out + v * frame_floats, prep->frame.p, frame_floats * sizeof(float),
                                 hipMemcpyDeviceToDevice, st));
      const BatchBuffers bb = batch_buffers(W, prep, W->d_sites[slot], W->d_vars[slot], B);
      {
        PassScope ps(ctx, SG_PASS_VARIANT_PREP, st);
        launch_variant_prep(s, b, prep->cam, ras, P<Rec>(prep->rec),
                            P<uint32_t>(prep->depth), P<uint2>(prep->rect), bb, st);
      }
      const CompArgs ca = item_comp_args(W, prep, images_out);
      const ItemArgs it = item_args(ctx, W, prep, B);
      {
        PassScope ps(ctx, SG_PASS_COMPOSITE_ITEMS, st);
        launch_composite_items(ca, it, st);
      }
      {
        PassScope ps(ctx, SG_PASS_REDUCE, st);
        launch_reduce_metrics(P<Partial>(W->bparts), P<uint32_t>(W->item_off), P<uint32_t>(W->n_items_v), 0,
                              P<VariantState>(W->vs), nullptr, nullptr, (uint32_t)(prep->cam.W * prep->cam.H), mout,
                              B, 0u, st);
      }
      return SG_OK;
    };
    if (graph) {
      std::vector<uintptr_t> key = {(uintptr_t)prep->serial, (uintptr_t)B, site_cap, (uintptr_t)slot, (uintptr_t)per_cu,
                                    (uintptr_t)ctx->persistent_grid,
                                    (uintptr_t)b.mask, (uintptr_t)b.mode, (uintptr_t)W->vs.p, (uintptr_t)W->ovr.p,
                                    (uintptr_t)W->tiles.p, (uintptr_t)W->bparts.p,
                                    (uintptr_t)W->h_sites[slot], (uintptr_t)W->h_vars[slot], (uintptr_t)W->gmetrics.p,
                                    (uintptr_t)W->counter.p, (uintptr_t)W->item_off.p, (uintptr_t)W->n_items_v.p,
                                    (uintptr_t)W->arrive.p};
      for (int f = 0; f < 6; ++f) { key.push_back((uintptr_t)b.lo[f]); key.push_back((uintptr_t)b.hi[f]); }
      hipGraphExec_t exec = nullptr;
      for (auto& g : W->graphs)
        if (g.key == key) exec = g.exec;
      if (!exec) {
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        sg_status rc = enqueue();
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(st, &gr);
        if (rc != SG_OK) { if (gr) (void)hipGraphDestroy(gr); return rc; }
        if (e != hipSuccess) return fail(SG_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return fail(SG_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        if (W->graphs.size() >= 16) {
          (void)hipGraphExecDestroy(W->graphs.front().exec);
          W->graphs.erase(W->graphs.begin());
        }
        W->graphs.push_back({key, exec});
      }
      HIP_TRY(hipGraphLaunch(exec, st));
      HIP_TRY(hipEventRecord(W->staged[slot], st));
      HIP_TRY(hipMemcpyAsync(metrics_out, W->gmetrics.p, (size_t)B * sizeof(sg_metrics_t), hipMemcpyDeviceToDevice, st));
    } else {
      SG_TRY(enqueue());
      HIP_TRY(hipEventRecord(W->staged[slot], st));
    }
    SG_TRY(check_last("sg_render_batch incremental"));
  }

  // full-render path: a private working copy of the scene per variant
  if (!full_idx.empty()) {
    DevScene w = s;
    size_t total_bytes = 0;
    int64_t off[6];
    const int wb = s.dtype == SG_F32 ? 4 : 2;
    for (int f = 0; f < 6; ++f) {
      off[f] = (int64_t)total_bytes;
      total_bytes += (size_t)((field_extent(s, f) * wb + 255) / 256 * 256);
    }
    SG_TRY(dev_alloc(ctx, W->work_scene, total_bytes));
    SG_TRY(dev_alloc(ctx, W->parts, (size_t)ras.n_tiles * sizeof(Partial)));
    for (int f = 0; f < 6; ++f) w.ptr[f] = P<char>(W->work_scene) + off[f];
    for (int v : full_idx) {
      for (int f = 0; f < 6; ++f)
        if (s.ncomp[f])
          HIP_TRY(hipMemcpyAsync(const_cast<void*>(w.ptr[f]), s.ptr[f], field_extent(s, f) * wb, hipMemcpyDeviceToDevice, st));
      const sg_variant& x = variants[v];
      // sites the variant's emulated defense corrects are not applied
      const int first_protected = s.dtype == SG_F32 ? 23 : (s.dtype == SG_F16 ? 10 : 7);
      std::vector<sg_site> applied;
      for (uint32_t k = 0; k < x.n_sites; ++k) {
        const sg_site& y = sites[x.site_off + k];
        if (x.protect == SG_PROTECT_VOTE || (x.protect == SG_PROTECT_SIGN_EXP && y.bit >= first_protected)) continue;
        applied.push_back(y);
      }
      SG_TRY(stage_sites(ctx, applied.data(), (int)applied.size(), W->sites_dev, st));
      launch_inject(w, P<sg_site>(W->sites_dev), (int)applied.size(), nullptr, st);
      DevBox bx = b;
      if (!x.guard) bx.mask = 0;
      SG_TRY(full_render(ctx, W, w, bx, prep->cam, ras, W->rec, W->depth, W->rect, W->tile_cnt,
                         W->tile_start, W->keys, images_out ? images_out + v * frame_floats : nullptr,
                         P<float>(prep->frame), P<Partial>(W->parts), st, nullptr));
      launch_reduce_metrics(P<Partial>(W->parts), nullptr, nullptr, (uint32_t)ras.n_tiles, nullptr,
                            P<uint32_t>(W->flags), P<unsigned long long>(W->clamps),
                            (uint32_t)(prep->cam.W * prep->cam.H), metrics_out + v, 1, 1u, st, ras.tiles_x, ras.tiles_y);
      SG_TRY(check_last("sg_render_batch full"));
    }
  }
  return SG_OK;
}

sg_status sg_render_batch_views(sg_ctx* ctx, sg_prep* const* preps, int32_t K, const sg_site* sites, int32_t n_sites,
                                const sg_variant* variants, int32_t B, const sg_box* box, uint32_t box_field_mask,
                                sg_metrics_t* metrics_out, sg_metrics_t* per_view_out, int32_t mode, void* stream) {
  if (!ctx || !preps || !metrics_out) return fail(SG_E_INVAL, "ctx/preps/metrics_out is NULL");
  if (K < 1 || K > kMaxViews) return fail(SG_E_INVAL, "K must be in [1, 64]");
  for (int k = 0; k < K; ++k) {
    if (!preps[k]) return fail(SG_E_INVAL, "preps[" + std::to_string(k) + "] is NULL");
    const sg_scene& a = preps[0]->host_scene;
    const sg_scene& b = preps[k]->host_scene;
    bool same = a.n == b.n && a.sh_degree == b.sh_degree && a.dtype == b.dtype;
    for (int f = 0; f < 6 && same; ++f) same = a.ptr[f] == b.ptr[f];
    if (!same) return fail(SG_E_INVAL, "the views are not prepared from one scene");
  }
  if (B == 0) return SG_OK;
  hipStream_t st = S(stream);
  WS_OR_FAIL(W, ctx, st);
  sg_metrics_t* pv = per_view_out;
  if (!pv) {
    SG_TRY(dev_alloc(ctx, W->views_tmp, (size_t)K * B * sizeof(sg_metrics_t)));
    pv = P<sg_metrics_t>(W->views_tmp);
  }
  for (int k = 0; k < K; ++k)
    SG_TRY(sg_render_batch(ctx, preps[k], sites, n_sites, variants, B, box, box_field_mask, nullptr,
                           pv + (int64_t)k * B, mode, stream));
  launch_pool_views(pv, K, B, B, 1, metrics_out, st);
  return check_last("sg_render_batch_views");
}

// sg_campaign(_views) when every variant is incremental.  The campaign's
// sites and variants are copied to the device once.  Per chunk of variants
// and per view, the corrupted primitives are staged and projected by one
// pre-pass launch, and each stream then runs its batches as a pipeline of
// one launch per batch: launch i lists the work items of the stream's batch
// i, composites batch i - 1 and reduces the metrics of batch i - 2, on three
// rotating buffer sets; two more launches drain it.  With K > 1 views the
// per-view records of the chunk are then pooled.  Views of one resolution,
// raster and checkpoint spacing share each launch (its stages count
// variant-views); other view sets follow one another on the device (the
// caller's stream joins every campaign stream before the next pre-pass),
// with no host synchronisation.  With scene_of, the K preps are scenes of
// their own: each scene's pre-pass stages its variants, and every launch
// takes each variant's clean state from the per-scene table.  The records
// are those of sg_render_batch(_views) on the same batches (on each
// variant's own scene).
// The pipelined campaign spreads its streams over the HIP runtime's hardware
// queues (GPU_MAX_HW_QUEUES, read by the runtime when it starts).  On the
// MI355X its rate rises with the queue count up to 23 and collapses at 24;
// at 26 a campaign made no progress for minutes.  The likely cause is that
// the process then holds more user-mode compute queues than the device's
// scheduler keeps mapped at once, so the queues are time-sliced while the
// campaign's streams wait on one another's events.  Larger settings are
// refused rather than risked.
constexpr int kMaxCampaignHwQueues = 23;

static sg_status check_hw_queues() {
  const char* e = std::getenv("GPU_MAX_HW_QUEUES");
  if (!e || !*e) return SG_OK;
  char* end = nullptr;
  const long q = std::strtol(e, &end, 10);
  if (end == e || q <= kMaxCampaignHwQueues) return SG_OK;
  return fail(SG_E_UNSUPPORTED, "GPU_MAX_HW_QUEUES=" + std::string(e) +
                                    ": the pipelined campaign supports at most 23 hardware queues (at 24 its rate "
                                    "collapses and at 26 it stalled)");
}

static sg_status campaign_pipelined(sg_ctx* ctx, sg_prep* const* preps, int K, const sg_site* sites, int32_t n_sites,
                                    const sg_variant* variants, int32_t n_variants, const DevBox& box, int B, int NS,
                                    int NT, sg_metrics_t* metrics_out, hipStream_t caller,
                                    const uint16_t* scene_of = nullptr, const DevBox* scene_boxes = nullptr) {
  SG_TRY(check_hw_queues());
  std::lock_guard<std::mutex> cg(ctx->camp_mu);
  if (ctx->camp_done) HIP_TRY(hipEventSynchronize(ctx->camp_done));   // the previous campaign's buffers are free
  else HIP_TRY(hipEventCreateWithFlags(&ctx->camp_done, hipEventDisableTiming));
  // K views of one resolution, raster and checkpoint spacing, with B * K
  // variant-views within a launch's limit, share each launch: its roles then
  // count variant-views (view k of variant v at v * K + k).  Other view sets
  // run view after view.
  // The per-stream work-item buffers hold every tile of every variant-view
  // (3 sets per stream); views share launches only while those stay within
  // kSharedBytes in all.
  constexpr int64_t kSharedBytes = (int64_t)16 << 30;
  int max_tiles = 0;
  for (int v = 0; v < K; ++v) max_tiles = std::max(max_tiles, preps[v]->ras.n_tiles);
  // scene_of (host, n_variants entries): the K preps are scenes (or views)
  // of their own and each variant is rendered in preps[scene_of[v]] only; all
  // of them share the launches through the per-view table.
  const bool sc = scene_of != nullptr;
  bool mv = sc || (K > 1 && (int64_t)B * K <= kMaxBatch &&
                   (int64_t)B * K * max_tiles * (int64_t)(sizeof(uint4) + sizeof(Partial)) * 3 * NS <= kSharedBytes);
  for (int k = 1; k < K && mv && !sc; ++k) {
    const sg_prep* a = preps[0];
    const sg_prep* c = preps[k];
    mv = a->cam.W == c->cam.W && a->cam.H == c->cam.H && a->ck_group == c->ck_group &&
         std::memcmp(&a->ras, &c->ras, sizeof(DevRaster)) == 0;
  }
  const int per = mv && !sc ? K : 1;                           // variant-views per variant in a launch
  const int64_t cap = mv ? (int64_t)1 << 21 : (int64_t)kCampaignChunk;  // variant-views staged per pre-pass
  const int chunk = (int)std::min<int64_t>(n_variants, std::max<int64_t>(B, (cap / per / B) * B));
  // Single-view campaigns stage a whole pre-pass chunk from the first call on
  // (when the context's budget allows), so that a later, larger campaign
  // reuses the buffers instead of growing them inside its run.
  const size_t rv = mv ? 0 : (size_t)kCampaignChunk;
  SG_TRY(dev_alloc(ctx, ctx->camp_sites, std::max<size_t>(1, (size_t)n_sites) * sizeof(sg_site)));
  SG_TRY(dev_reserve(ctx, ctx->camp_vars, (size_t)n_variants * sizeof(sg_variant), rv * sizeof(sg_variant)));
  SG_TRY(dev_reserve(ctx, ctx->camp_vs, (size_t)chunk * per * sizeof(VariantState), rv * sizeof(VariantState)));
  SG_TRY(dev_reserve(ctx, ctx->camp_ovr, (size_t)chunk * per * kRecSlots * sizeof(Rec), rv * kRecSlots * sizeof(Rec)));
  if (K > 1) SG_TRY(dev_alloc(ctx, ctx->camp_views, (size_t)K * chunk * sizeof(sg_metrics_t)));
  const ViewArgs* d_views = nullptr;
  if (mv) {
    ctx->camp_vargs_host.resize(K);
    for (int k = 0; k < K; ++k) {
      const sg_prep* p = preps[k];
      const bool rs = p->ck_group != 0;
      ctx->camp_vargs_host[k] = ViewArgs{P<Rec>(p->rec),
                                         P<uint32_t>(p->tile_start), P<uint32_t>(p->tile_cnt), P<uint64_t>(p->keys),
                                         P<float>(p->frame), rs ? P<uint64_t>(p->stop) : nullptr,
                                         rs ? P<float4>(p->ck) : nullptr, rs ? P<uint32_t>(p->ck_off) : nullptr,
                                         rs ? P<uint64_t>(p->stop_key) : nullptr, p->ras, p->cam.W, p->cam.H,
                                         p->ck_group};
    }
    SG_TRY(dev_alloc(ctx, ctx->camp_vargs, (size_t)K * sizeof(ViewArgs)));
    HIP_TRY(hipMemcpyAsync(ctx->camp_vargs.p, ctx->camp_vargs_host.data(), (size_t)K * sizeof(ViewArgs),
                           hipMemcpyHostToDevice, caller));
    d_views = P<ViewArgs>(ctx->camp_vargs);
  }
  const uint16_t* d_scene_of = nullptr;
  if (sc) {
    ctx->camp_scene_of_host.assign(scene_of, scene_of + n_variants);
    SG_TRY(dev_alloc(ctx, ctx->camp_scene_of, std::max<size_t>(1, (size_t)n_variants) * sizeof(uint16_t)));
    HIP_TRY(hipMemcpyAsync(ctx->camp_scene_of.p, ctx->camp_scene_of_host.data(), (size_t)n_variants * sizeof(uint16_t),
                           hipMemcpyHostToDevice, caller));
    d_scene_of = P<uint16_t>(ctx->camp_scene_of);
  }
  if (n_sites)
    HIP_TRY(hipMemcpyAsync(ctx->camp_sites.p, sites, (size_t)n_sites * sizeof(sg_site), hipMemcpyHostToDevice, caller));
  HIP_TRY(hipMemcpyAsync(ctx->camp_vars.p, variants, (size_t)n_variants * sizeof(sg_variant), hipMemcpyHostToDevice,
                         caller));
  std::vector<Workspace*> ws(NS);
  for (int k = 0; k < NS; ++k) {
    hipStream_t st = ctx->campaign_streams[k];
    Workspace* W = workspace(ctx, st);
    if (!W) return fail(SG_E_NOMEM, "pinned allocation for a workspace failed");
    for (int q = 0; q < 3; ++q) {
      SG_TRY(dev_alloc(ctx, W->st_items[q], (size_t)B * per * max_tiles * sizeof(uint4)));
      SG_TRY(dev_alloc(ctx, W->st_parts[q], (size_t)B * per * max_tiles * sizeof(Partial)));
      SG_TRY(dev_alloc(ctx, W->st_off[q], (size_t)(B * per + 1) * sizeof(uint32_t)));
      SG_TRY(dev_alloc(ctx, W->st_n[q], (size_t)B * per * sizeof(uint32_t)));
    }
    if (!W->st_ctl.p) {
      SG_TRY(dev_alloc(ctx, W->st_ctl, 3 * 4 * sizeof(uint32_t)));
      launch_fill_u32(P<uint32_t>(W->st_ctl), 0u, 12, st);   // the arrival counters return to zero
    }
    ws[k] = W;
  }
  const sg_site* d_sites = P<sg_site>(ctx->camp_sites);
  const sg_variant* d_vars = P<sg_variant>(ctx->camp_vars);
  VariantState* c_vs = P<VariantState>(ctx->camp_vs);
  Rec* c_ovr = P<Rec>(ctx->camp_ovr);
  sg_metrics_t* per_view = P<sg_metrics_t>(ctx->camp_views);

  std::mutex launch_mu;
  hipError_t launch_err = hipSuccess;
  for (int c0 = 0; c0 < n_variants; c0 += chunk) {
    const int cn = std::min(chunk, n_variants - c0);
    for (int view = 0; view < (mv ? 1 : K); ++view) {
      const sg_prep* prep = preps[view];
      const DevRaster& ras = prep->ras;
      // per-view records: view-major (cn per view) view after view, variant-major (K per variant) when shared
      sg_metrics_t* out = K == 1 || sc ? metrics_out + c0 : per_view + (mv ? 0 : (int64_t)view * cn);
      CompArgs ca0 = item_comp_args(ws[0], prep, nullptr);
      if (mv) ca0.ras.n_tiles = max_tiles;   // work items sit max_tiles apart per variant-view
      const ItemArgs it0 = item_args(ctx, ws[0], prep, B);
      StepArgs base{};
      base.tiles_x = ras.tiles_x;
      base.tiles_y = ras.tiles_y;
      base.n_tiles = mv ? max_tiles : ras.n_tiles;
      base.stop_key = prep->ck_group ? P<uint64_t>(prep->stop_key) : nullptr;
      base.tile_start = P<uint32_t>(prep->tile_start);
      base.tile_cnt = P<uint32_t>(prep->tile_cnt);
      base.n_pixels = (uint32_t)(prep->cam.W * prep->cam.H);
      base.K = per;
      base.views = d_views;
      for (int k = mv ? 0 : view; k < (mv ? K : view + 1); ++k) {
        const sg_prep* pk = preps[k];
        PassScope ps(ctx, SG_PASS_VARIANT_PREP, caller);
        launch_campaign_touch(pk->scene, sc ? scene_boxes[k] : box, pk->cam, pk->ras, P<Rec>(pk->rec), P<uint32_t>(pk->depth), P<uint2>(pk->rect),
                              d_sites, d_vars + c0, cn, c_vs, c_ovr, per, mv && !sc ? k : 0,
                              sc ? d_scene_of + c0 : nullptr, k, caller);
      }
      hipEvent_t staged = nullptr;
      HIP_TRY(hipEventCreateWithFlags(&staged, hipEventDisableTiming));
      HIP_TRY(hipEventRecord(staged, caller));
      for (int k = 0; k < NS; ++k) HIP_TRY(hipStreamWaitEvent(ctx->campaign_streams[k], staged, 0));
      (void)hipEventDestroy(staged);
      const int nb = (cn + B - 1) / B;
      const int per_stream = (nb + NS - 1) / NS;   // batches of the first stream (the most)
      auto worker = [&](int t) {
        (void)hipSetDevice(ctx->device);
        // launch i of every owned stream, then launch i + 1 ...
        for (int i = 0; i < per_stream + 2; ++i)
          for (int k = t; k < NS; k += NT) {
            const int m = nb > k ? (nb - k + NS - 1) / NS : 0;   // batches k, k + NS, ... of the chunk
            if (i > m + 1) continue;
            Workspace* W = ws[k];
            hipStream_t st = ctx->campaign_streams[k];
            auto lb = [&](int pos) { return (pos * NS + k) * B; };   // first variant (in the chunk) of batch `pos`
            auto nvb = [&](int pos) { return std::min(B, cn - lb(pos)); };
            StepArgs a = base;
            if (i < m) {
              const int q = i % 3;
              a.tB = nvb(i) * per;
              a.t_vs = c_vs + (int64_t)lb(i) * per;
              a.t_ovr = c_ovr + (int64_t)lb(i) * per * kRecSlots;
              if (sc) a.t_view_of = d_scene_of + c0 + lb(i);
              a.t_items = P<uint4>(W->st_items[q]);
              a.t_n_items = P<uint32_t>(W->st_n[q]);
              a.t_item_off = P<uint32_t>(W->st_off[q]);
              a.t_counter = P<uint32_t>(W->st_ctl) + 4 * q;
              a.t_arrive = P<uint32_t>(W->st_ctl) + 4 * q + 1;
            }
            a.A = ca0;
            a.I = it0;
            a.I.B = 0;
            if (i >= 1 && i <= m) {
              const int q = (i - 1) % 3;
              a.A.parts = P<Partial>(W->st_parts[q]);
              a.I.vs = c_vs + (int64_t)lb(i - 1) * per;
              a.I.ovr = c_ovr + (int64_t)lb(i - 1) * per * kRecSlots;
              a.I.items = P<uint4>(W->st_items[q]);
              a.I.item_off = P<uint32_t>(W->st_off[q]);
              a.I.counter = P<uint32_t>(W->st_ctl) + 4 * q;
              a.I.B = nvb(i - 1) * per;
              if (sc) a.i_view_of = d_scene_of + c0 + lb(i - 1);
            }
            if (i >= 2) {
              const int q = (i - 2) % 3;
              a.rB = nvb(i - 2) * per;
              a.r_parts = P<Partial>(W->st_parts[q]);
              a.r_item_off = P<uint32_t>(W->st_off[q]);
              a.r_n_items = P<uint32_t>(W->st_n[q]);
              a.r_vs = c_vs + (int64_t)lb(i - 2) * per;
              a.r_out = out + (int64_t)lb(i - 2) * per;
              if (sc) a.r_view_of = d_scene_of + c0 + lb(i - 2);
            }
            if (a.tB == 0 && a.I.B == 0 && a.rB == 0) continue;
            // launches with a compositing role are timed as compositing; the
            // pipeline's fill and drain launches (work items or metrics only)
            // as the reduction pass
            PassScope ps(ctx, a.I.B > 0 ? SG_PASS_COMPOSITE_ITEMS : SG_PASS_REDUCE, st, true);
            launch_campaign_step(a, st, ps.a, ps.b);
          }
        // launch errors are per host thread: each worker reports its own
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
          std::lock_guard<std::mutex> g(launch_mu);
          if (launch_err == hipSuccess) launch_err = e;
        }
      };
      std::vector<std::thread> pool;
      for (int t = 1; t < NT; ++t) pool.emplace_back(worker, t);
      worker(0);
      for (std::thread& th : pool) th.join();
      if (launch_err != hipSuccess)
        return fail(SG_E_DEVICE, std::string("campaign step launch: ") + hipGetErrorString(launch_err));
      for (int k = 0; k < NS; ++k) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(e, ctx->campaign_streams[k]));
        HIP_TRY(hipStreamWaitEvent(caller, e, 0));
        (void)hipEventDestroy(e);
      }
    }
    if (K > 1 && !sc) launch_pool_views(per_view, K, cn, mv ? 1 : cn, mv ? K : 1, metrics_out + c0, caller);
  }
  HIP_TRY(hipEventRecord(ctx->camp_done, caller));
  return check_last("sg_campaign");
}

// Work items one persistent launch can hold per buffer set (16 B record and
// 32 B partial each: 1.6 GB per set).  A chunk's variants are bounded so that
// every one of them may dirty every tile of its view.
constexpr int64_t kPersistItems = (int64_t)1 << 25;
constexpr int64_t kPersistVariants = (int64_t)1 << 18;   // variant-views per chunk

// The persistent campaign: chunks of variants, each rendered by its pre-pass
// (per view or scene), one launch listing every variant's work items
// compactly, one persistent compositing launch over all of them and one
// reduction launch; chunks alternate between two streams and two buffer sets
// so that a chunk's listing overlaps the previous chunk's last items.  With
// K > 1 views (scene_of null) every variant is rendered in every view, the
// views of a variant side by side, and the per-view records are pooled; with
// scene_of, variant v is rendered in preps[scene_of[v]] only.  B > 0 caps the
// variants per chunk.  The records are those of sg_render_batch(_views).
static sg_status campaign_persistent(sg_ctx* ctx, sg_prep* const* preps, int K, const sg_site* sites, int32_t n_sites,
                                     const sg_variant* variants, int32_t n_variants, const DevBox& box, int B,
                                     sg_metrics_t* metrics_out, hipStream_t caller, const uint16_t* scene_of = nullptr,
                                     const DevBox* scene_boxes = nullptr) {
  std::lock_guard<std::mutex> cg(ctx->camp_mu);
  if (ctx->camp_done) HIP_TRY(hipEventSynchronize(ctx->camp_done));   // the previous campaign's buffers are free
  else HIP_TRY(hipEventCreateWithFlags(&ctx->camp_done, hipEventDisableTiming));
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    while ((int)ctx->campaign_streams.size() < 2) {
      hipStream_t st = nullptr;
      HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      ctx->campaign_streams.push_back(st);
    }
  }
  const bool sc = scene_of != nullptr;
  const bool mv = sc || K > 1;
  const int per = mv && !sc ? K : 1;   // variant-views per variant
  int max_tiles = 1;
  for (int k = 0; k < K; ++k) max_tiles = std::max(max_tiles, preps[k]->ras.n_tiles);
  int64_t chunk = std::min<int64_t>(kPersistVariants / per, kPersistItems / ((int64_t)per * max_tiles));
  if (B > 0) chunk = std::min<int64_t>(chunk, B);
  chunk = std::max<int64_t>(1, std::min<int64_t>(chunk, n_variants));
  const int64_t nvv = chunk * per;   // variant-views per chunk
  SG_TRY(dev_alloc(ctx, ctx->camp_sites, std::max<size_t>(1, (size_t)n_sites) * sizeof(sg_site)));
  SG_TRY(dev_reserve(ctx, ctx->camp_vars, (size_t)n_variants * sizeof(sg_variant),
                     mv ? 0 : (size_t)kCampaignChunk * sizeof(sg_variant)));
  for (int k = 0; k < 2; ++k) {
    SG_TRY(dev_alloc(ctx, ctx->pst_vs[k], (size_t)nvv * sizeof(VariantState)));
    SG_TRY(dev_alloc(ctx, ctx->pst_ovr[k], (size_t)nvv * kRecSlots * sizeof(Rec)));
    SG_TRY(dev_alloc(ctx, ctx->pst_items[k], (size_t)nvv * max_tiles * sizeof(uint4)));
    SG_TRY(dev_alloc(ctx, ctx->pst_parts[k], (size_t)nvv * max_tiles * sizeof(Partial)));
    SG_TRY(dev_alloc(ctx, ctx->pst_off[k], (size_t)nvv * sizeof(uint32_t)));
    SG_TRY(dev_alloc(ctx, ctx->pst_n[k], (size_t)nvv * sizeof(uint32_t)));
    SG_TRY(dev_alloc(ctx, ctx->pst_ctl[k], 2 * sizeof(uint32_t)));
    if (per > 1) SG_TRY(dev_alloc(ctx, ctx->pst_views[k], (size_t)nvv * sizeof(sg_metrics_t)));
  }
  const ViewArgs* d_views = nullptr;
  if (mv) {
    ctx->camp_vargs_host.resize(K);
    for (int k = 0; k < K; ++k) {
      const sg_prep* p = preps[k];
      const bool rs = p->ck_group != 0;
      ctx->camp_vargs_host[k] = ViewArgs{P<Rec>(p->rec),
                                         P<uint32_t>(p->tile_start), P<uint32_t>(p->tile_cnt), P<uint64_t>(p->keys),
                                         P<float>(p->frame), rs ? P<uint64_t>(p->stop) : nullptr,
                                         rs ? P<float4>(p->ck) : nullptr, rs ? P<uint32_t>(p->ck_off) : nullptr,
                                         rs ? P<uint64_t>(p->stop_key) : nullptr, p->ras, p->cam.W, p->cam.H,
                                         p->ck_group};
    }
    SG_TRY(dev_alloc(ctx, ctx->camp_vargs, (size_t)K * sizeof(ViewArgs)));
    HIP_TRY(hipMemcpyAsync(ctx->camp_vargs.p, ctx->camp_vargs_host.data(), (size_t)K * sizeof(ViewArgs),
                           hipMemcpyHostToDevice, caller));
    d_views = P<ViewArgs>(ctx->camp_vargs);
  }
  const uint16_t* d_scene_of = nullptr;
  if (sc) {
    ctx->camp_scene_of_host.assign(scene_of, scene_of + n_variants);
    SG_TRY(dev_alloc(ctx, ctx->camp_scene_of, std::max<size_t>(1, (size_t)n_variants) * sizeof(uint16_t)));
    HIP_TRY(hipMemcpyAsync(ctx->camp_scene_of.p, ctx->camp_scene_of_host.data(), (size_t)n_variants * sizeof(uint16_t),
                           hipMemcpyHostToDevice, caller));
    d_scene_of = P<uint16_t>(ctx->camp_scene_of);
  }
  if (n_sites)
    HIP_TRY(hipMemcpyAsync(ctx->camp_sites.p, sites, (size_t)n_sites * sizeof(sg_site), hipMemcpyHostToDevice, caller));
  HIP_TRY(hipMemcpyAsync(ctx->camp_vars.p, variants, (size_t)n_variants * sizeof(sg_variant), hipMemcpyHostToDevice,
                         caller));
  hipStream_t streams[2] = {ctx->campaign_streams[0], ctx->campaign_streams[1]};
  {
    hipEvent_t staged = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&staged, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(staged, caller));
    for (hipStream_t st : streams) HIP_TRY(hipStreamWaitEvent(st, staged, 0));
    (void)hipEventDestroy(staged);
  }
  const sg_site* d_sites = P<sg_site>(ctx->camp_sites);
  const sg_variant* d_vars = P<sg_variant>(ctx->camp_vars);
  const sg_prep* p0 = preps[0];
  const int tile = p0->ras.tile;
  const int occ = persist_occupancy(tile, mv);
  const int grid = ctx->persistent_grid > 0 ? ctx->persistent_grid : ctx->n_cu * occ;
  int set = 0;
  for (int64_t c0 = 0; c0 < n_variants; c0 += chunk, set ^= 1) {
    const int cn = (int)std::min<int64_t>(chunk, n_variants - c0);
    hipStream_t st = streams[set];
    VariantState* vs = P<VariantState>(ctx->pst_vs[set]);
    Rec* ovr = P<Rec>(ctx->pst_ovr[set]);
    uint32_t* ctl = P<uint32_t>(ctx->pst_ctl[set]);
    launch_fill_u32(ctl, 0u, 2, st);   // the list's cursor and the work counter start at zero
    for (int k = 0; k < K; ++k) {
      const sg_prep* pk = preps[k];
      PassScope ps(ctx, SG_PASS_VARIANT_PREP, st);
      launch_campaign_touch(pk->scene, sc ? scene_boxes[k] : box, pk->cam, pk->ras, P<Rec>(pk->rec), P<uint32_t>(pk->depth), P<uint2>(pk->rect), d_sites,
                            d_vars + c0, cn, vs, ovr, per, sc ? 0 : k, sc ? d_scene_of + c0 : nullptr, k, st);
    }
    PersistArgs a{};
    a.A = CompArgs{P<Rec>(p0->rec), P<uint32_t>(p0->tile_start),
                   P<uint32_t>(p0->tile_cnt), P<uint64_t>(p0->keys), P<float>(p0->frame), nullptr,
                   P<Partial>(ctx->pst_parts[set]), p0->ras, p0->cam.W, p0->cam.H};
    if (p0->ck_group) {
      a.A.stop = P<uint64_t>(p0->stop);
      a.A.ck = P<float4>(p0->ck);
      a.A.ck_off = P<uint32_t>(p0->ck_off);
      a.A.stop_key = P<uint64_t>(p0->stop_key);
      a.A.ck_group = p0->ck_group;
    }
    a.vs = vs;
    a.ovr = ovr;
    a.items = P<uint4>(ctx->pst_items[set]);
    a.item_off = P<uint32_t>(ctx->pst_off[set]);
    a.n_items = P<uint32_t>(ctx->pst_n[set]);
    a.ctl = ctl;
    a.nv = cn * per;
    a.grid = grid;
    a.out = per > 1 ? P<sg_metrics_t>(ctx->pst_views[set]) : metrics_out + c0;
    a.n_pixels = (uint32_t)(p0->cam.W * p0->cam.H);
    a.K = per;
    a.views = d_views;
    a.view_of = sc ? d_scene_of + c0 : nullptr;
    {
      PassScope ps(ctx, SG_PASS_VARIANT_PREP, st);
      launch_persist_list(a, st);
    }
    {
      PassScope ps(ctx, SG_PASS_COMPOSITE_ITEMS, st, true);
      launch_persist_composite(a, st, ps.a, ps.b);
    }
    {
      PassScope ps(ctx, SG_PASS_REDUCE, st);
      launch_persist_reduce(a, st);
      if (per > 1) launch_pool_views(a.out, K, cn, 1, K, metrics_out + c0, st);
    }
  }
  for (hipStream_t st : streams) {
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(e, st));
    HIP_TRY(hipStreamWaitEvent(caller, e, 0));
    (void)hipEventDestroy(e);
  }
  HIP_TRY(hipEventRecord(ctx->camp_done, caller));
  return check_last("sg_campaign (persistent)");
}

sg_status sg_campaign_views(sg_ctx* ctx, sg_prep* const* preps, int32_t K, const sg_site* sites, int32_t n_sites,
                            const sg_variant* variants, int32_t n_variants, const sg_box* box, uint32_t box_field_mask,
                            const sg_campaign_cfg* cfg, sg_metrics_t* metrics_out, void* stream) {
  if (!ctx || !preps || !metrics_out) return fail(SG_E_INVAL, "ctx/preps/metrics_out is NULL");
  if (K < 1 || K > kMaxViews) return fail(SG_E_INVAL, "K must be in [1, 64]");
  sg_prep* prep = preps[0];
  if (!prep) return fail(SG_E_INVAL, "preps[0] is NULL");
  for (int k = 0; k < K; ++k) {
    if (!preps[k]) return fail(SG_E_INVAL, "preps[" + std::to_string(k) + "] is NULL");
    if (preps[k]->ctx != ctx && preps[k]->ctx->device != ctx->device)
      return fail(SG_E_INVAL, "preps[" + std::to_string(k) + "] is on another device");
    const sg_scene& a = prep->host_scene;
    const sg_scene& c = preps[k]->host_scene;
    bool same = a.n == c.n && a.sh_degree == c.sh_degree && a.dtype == c.dtype;
    for (int f = 0; f < 6 && same; ++f) same = a.ptr[f] == c.ptr[f];
    if (!same) return fail(SG_E_INVAL, "the views are not prepared from one scene");
  }
  if (n_variants < 0 || (n_variants > 0 && !variants)) return fail(SG_E_INVAL, "bad variants");
  const int engine = cfg ? cfg->engine : SG_ENGINE_PIPELINED;
  if (engine != SG_ENGINE_PIPELINED && engine != SG_ENGINE_PERSISTENT) return fail(SG_E_INVAL, "unknown campaign engine");
  const bool persistent = engine == SG_ENGINE_PERSISTENT;
  const int B = cfg && cfg->batch > 0 ? cfg->batch : (persistent ? 0 : 32);
  const int NS = cfg && cfg->streams > 0 ? cfg->streams : 8;
  const int NT = std::min(cfg && cfg->threads > 0 ? cfg->threads : 2, NS);
  if ((!persistent && B > kMaxBatch) || B < 0 || NS > 64 || NT > 64)
    return fail(SG_E_INVAL, "campaign batch/streams/threads out of range");
  SG_TRY(validate_sites(prep->scene, sites, n_sites));
  for (int v = 0; v < n_variants; ++v)
    if ((uint64_t)variants[v].site_off + variants[v].n_sites > (uint64_t)n_sites)
      return fail(SG_E_INVAL, "variant " + std::to_string(v) + ": sites out of range");
  if (n_variants == 0) return SG_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    while ((int)ctx->campaign_streams.size() < NS) {
      hipStream_t st = nullptr;
      HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      ctx->campaign_streams.push_back(st);
    }
  }
  // the campaign's launches follow the caller's earlier work on `stream` and
  // the caller's later work follows all of them
  hipStream_t caller = S(stream);
  {
    // the pipelined path takes campaigns whose variants all stay incremental
    DevBox b;
    SG_TRY(to_dev_box(box, box_field_mask, prep->scene, &b));
    bool incremental = true;
    std::vector<uint32_t> prims;
    for (int v = 0; v < n_variants && incremental; ++v) {
      const sg_variant& x = variants[v];
      if (x.guard && !b.mask) return fail(SG_E_INVAL, "variant " + std::to_string(v) + ": guard requested without a box");
      if (x.protect > SG_PROTECT_VOTE) return fail(SG_E_INVAL, "variant " + std::to_string(v) + ": unknown protect mode");
      if (x.n_sites <= (uint32_t)kMaxTouch) continue;   // at most kMaxTouch sites: incremental
      prims.clear();
      for (uint32_t k = 0; k < x.n_sites && incremental; ++k) {
        const uint32_t pr = sites[x.site_off + k].prim;
        if (std::find(prims.begin(), prims.end(), pr) == prims.end()) {
          prims.push_back(pr);
          if ((int)prims.size() > kMaxTouch) incremental = false;
        }
      }
    }
    if (incremental)
      return persistent ? campaign_persistent(ctx, preps, K, sites, n_sites, variants, n_variants, b, B, metrics_out, caller)
                        : campaign_pipelined(ctx, preps, K, sites, n_sites, variants, n_variants, b, B, NS, NT,
                                             metrics_out, caller);
  }
  hipEvent_t start = nullptr;
  HIP_TRY(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(start, caller));
  for (int k = 0; k < NS; ++k) HIP_TRY(hipStreamWaitEvent(ctx->campaign_streams[k], start, 0));
  (void)hipEventDestroy(start);

  const int BB = B > 0 && B <= kMaxBatch ? B : 32;   // batches of sg_render_batch
  const int nb = (n_variants + BB - 1) / BB;
  std::mutex err_mu;
  sg_status first_rc = SG_OK;
  std::string first_msg;
  auto worker = [&](int t) {
    (void)hipSetDevice(ctx->device);
    std::vector<sg_variant> local;
    for (int b = 0; b < nb; ++b) {
      const int k = b % NS;
      if (k % NT != t) continue;
      {
        std::lock_guard<std::mutex> g(err_mu);
        if (first_rc != SG_OK) return;
      }
      const int v0 = b * BB, nv = std::min(BB, n_variants - v0);
      // the sites this batch refers to, with its variants' offsets rebased
      uint32_t lo = UINT32_MAX, hi = 0;
      for (int v = v0; v < v0 + nv; ++v) {
        lo = std::min(lo, variants[v].site_off);
        hi = std::max(hi, variants[v].site_off + variants[v].n_sites);
      }
      if (lo > hi) lo = hi = 0;
      local.assign(variants + v0, variants + v0 + nv);
      for (sg_variant& x : local) x.site_off -= lo;
      const sg_status rc =
          K == 1 ? sg_render_batch(ctx, prep, sites + lo, (int32_t)(hi - lo), local.data(), nv, box, box_field_mask,
                                   nullptr, metrics_out + v0, SG_INCREMENTAL, ctx->campaign_streams[k])
                 : sg_render_batch_views(ctx, preps, K, sites + lo, (int32_t)(hi - lo), local.data(), nv, box,
                                         box_field_mask, metrics_out + v0, nullptr, SG_INCREMENTAL,
                                         ctx->campaign_streams[k]);
      if (rc != SG_OK) {
        std::lock_guard<std::mutex> g(err_mu);
        if (first_rc == SG_OK) {
          first_rc = rc;
          first_msg = "batch " + std::to_string(b) + ": " + g_err;
        }
        return;
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < NT; ++t) pool.emplace_back(worker, t);
  worker(0);
  for (std::thread& th : pool) th.join();
  for (int k = 0; k < NS; ++k) {
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(e, ctx->campaign_streams[k]));
    HIP_TRY(hipStreamWaitEvent(caller, e, 0));
    (void)hipEventDestroy(e);
  }
  if (first_rc != SG_OK) return fail(first_rc, first_msg);
  return SG_OK;
}

sg_status sg_campaign(sg_ctx* ctx, sg_prep* prep, const sg_site* sites, int32_t n_sites, const sg_variant* variants,
                      int32_t n_variants, const sg_box* box, uint32_t box_field_mask, const sg_campaign_cfg* cfg,
                      sg_metrics_t* metrics_out, void* stream) {
  return sg_campaign_views(ctx, &prep, 1, sites, n_sites, variants, n_variants, box, box_field_mask, cfg, metrics_out,
                           stream);
}

sg_status sg_campaign_scenes(sg_ctx* ctx, sg_prep* const* preps, int32_t n_preps, const sg_site* sites, int32_t n_sites,
                             const sg_variant* variants, const uint16_t* scene_of, int32_t n_variants,
                             const sg_box* const* boxes, uint32_t box_field_mask, const sg_campaign_cfg* cfg,
                             sg_metrics_t* metrics_out, void* stream) {
  if (!ctx || !preps || !metrics_out) return fail(SG_E_INVAL, "ctx/preps/metrics_out is NULL");
  if (n_preps < 1 || n_preps > kMaxViews) return fail(SG_E_INVAL, "n_preps must be in [1, 64]");
  for (int k = 0; k < n_preps; ++k) {
    if (!preps[k]) return fail(SG_E_INVAL, "preps[" + std::to_string(k) + "] is NULL");
    if (preps[k]->ctx != ctx && preps[k]->ctx->device != ctx->device)
      return fail(SG_E_INVAL, "preps[" + std::to_string(k) + "] is on another device");
    if (preps[k]->ras.tile != preps[0]->ras.tile)
      return fail(SG_E_INVAL, "the prepared scenes must share one tile size");
  }
  if (n_variants < 0 || (n_variants > 0 && (!variants || !scene_of))) return fail(SG_E_INVAL, "bad variants");
  if (n_sites < 0 || (n_sites > 0 && !sites)) return fail(SG_E_INVAL, "bad sites");
  const int engine = cfg ? cfg->engine : SG_ENGINE_PIPELINED;
  if (engine != SG_ENGINE_PIPELINED && engine != SG_ENGINE_PERSISTENT) return fail(SG_E_INVAL, "unknown campaign engine");
  const bool persistent = engine == SG_ENGINE_PERSISTENT;
  const int B = cfg && cfg->batch > 0 ? cfg->batch : (persistent ? 0 : 32);
  const int NS = cfg && cfg->streams > 0 ? cfg->streams : 8;
  const int NT = std::min(cfg && cfg->threads > 0 ? cfg->threads : 2, NS);
  if ((!persistent && B > kMaxBatch) || B < 0 || NS > 64 || NT > 64)
    return fail(SG_E_INVAL, "campaign batch/streams/threads out of range");
  std::vector<DevBox> db(n_preps);
  for (int k = 0; k < n_preps; ++k)
    SG_TRY(to_dev_box(boxes ? boxes[k] : nullptr, box_field_mask, preps[k]->scene, &db[k]));
  // every variant against its own scene: sites in range and valid for that
  // scene, guard only with a box, at most kMaxTouch distinct primitives
  std::vector<uint32_t> prims;
  for (int v = 0; v < n_variants; ++v) {
    const sg_variant& x = variants[v];
    const int sc = scene_of[v];
    if (sc >= n_preps) return fail(SG_E_INVAL, "variant " + std::to_string(v) + ": scene index out of range");
    if ((uint64_t)x.site_off + x.n_sites > (uint64_t)n_sites)
      return fail(SG_E_INVAL, "variant " + std::to_string(v) + ": sites out of range");
    if (x.guard && !db[sc].mask) return fail(SG_E_INVAL, "variant " + std::to_string(v) + ": guard requested without a box");
    if (x.protect > SG_PROTECT_VOTE) return fail(SG_E_INVAL, "variant " + std::to_string(v) + ": unknown protect mode");
    SG_TRY(validate_sites(preps[sc]->scene, sites + x.site_off, (int32_t)x.n_sites));
    prims.clear();
    for (uint32_t k = 0; k < x.n_sites; ++k) {
      const uint32_t pr = sites[x.site_off + k].prim;
      if (std::find(prims.begin(), prims.end(), pr) == prims.end()) prims.push_back(pr);
    }
    if ((int)prims.size() > kMaxTouch)
      return fail(SG_E_UNSUPPORTED, "variant " + std::to_string(v) + ": more than 8 corrupted primitives");
  }
  if (n_variants == 0) return SG_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    while ((int)ctx->campaign_streams.size() < NS) {
      hipStream_t st = nullptr;
      HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      ctx->campaign_streams.push_back(st);
    }
  }
  if (persistent)
    return campaign_persistent(ctx, preps, n_preps, sites, n_sites, variants, n_variants, db[0], B, metrics_out,
                               S(stream), scene_of, db.data());
  return campaign_pipelined(ctx, preps, n_preps, sites, n_sites, variants, n_variants, db[0], B, NS, NT, metrics_out,
                            S(stream), scene_of, db.data());
}

sg_status sg_ssim(sg_ctx* ctx, const float* images, const float* clean, int32_t B, int32_t H, int32_t W, double* out,
                  void* stream) {
  if (!ctx || !images || !clean || !out) return fail(SG_E_INVAL, "NULL argument");
  if (B < 1 || B > 65535 || H < 11 || W < 11)
    return fail(SG_E_INVAL, "B must be in [1, 65535] and the frame at least 11 x 11");
  SsimWeights gw;
  double sum = 0.0;
  for (int t = 0; t < 11; ++t) {
    const double r = (double)(t - 5);
    gw.w[t] = std::exp(-r * r / (2.0 * 1.5 * 1.5));
    sum += gw.w[t];
  }
  for (int t = 0; t < 11; ++t) gw.w[t] /= sum;
  hipStream_t st = S(stream);
  WS_OR_FAIL(WS, ctx, st);
  SG_TRY(dev_alloc(ctx, WS->ssim_tmp, (size_t)B * ssim_blocks(H, W) * sizeof(double)));
  launch_ssim(images, clean, B, H, W, gw, P<double>(WS->ssim_tmp), out, st);
  return check_last("sg_ssim");
}

sg_status sg_metrics(sg_ctx* ctx, const float* images, const float* clean, int32_t B, int32_t K, int32_t H, int32_t W,
                     sg_metrics_t* out, void* stream) {
  if (!ctx || !images || !clean || !out) return fail(SG_E_INVAL, "NULL argument");
  if (B < 1 || K < 1 || H < 1 || W < 1) return fail(SG_E_INVAL, "sizes must be >= 1");
  const int64_t px = (int64_t)K * H * W;
  const int nchunks = (int)std::min<int64_t>(256, (px + 1023) / 1024);
  hipStream_t st = S(stream);
  WS_OR_FAIL(WS, ctx, st);
  SG_TRY(dev_alloc(ctx, WS->metrics_tmp, (size_t)B * nchunks * sizeof(Partial)));
  launch_metrics_partials(images, clean, px, nchunks, B, P<Partial>(WS->metrics_tmp), st);
  launch_reduce_metrics(P<Partial>(WS->metrics_tmp), nullptr, nullptr, (uint32_t)nchunks, nullptr, nullptr, nullptr,
                        (uint32_t)px, out, B, 1u, st);
  return check_last("sg_metrics");
}

sg_status sg_metrics_noalloc(sg_ctx* ctx, const float* images, const float* clean, int32_t B, int32_t K, int32_t H,
                             int32_t W, sg_metrics_t* out, void* stream) {
  if (!ctx || !images || !clean || !out) return fail(SG_E_INVAL, "NULL argument");
  if (B < 1 || K < 1 || H < 1 || W < 1) return fail(SG_E_INVAL, "sizes must be >= 1");
  const int64_t px = (int64_t)K * H * W;
  const int nchunks = (int)std::min<int64_t>(256, (px + 1023) / 1024);
  const size_t need = (size_t)B * (size_t)nchunks * sizeof(Partial);
  if (need > kScratchBytes)
    return fail(SG_E_INVAL, "sg_metrics_noalloc: " + std::to_string(B) + " variants of " + std::to_string(px) +
                                " pixels need " + std::to_string(need) + " bytes of scratch; the limit is " +
                                std::to_string(kScratchBytes) + " (" + std::to_string(kScratchBytes / sizeof(Partial)) +
                                " variant-chunk partials, one chunk per 1,024 pixels up to 256 chunks)");
  Partial* parts = static_cast<Partial*>(scratch_of(ctx->device));
  if (!parts) return fail(SG_E_DEVICE, "no scratch address recorded for this device");
  // every partial is written before the reduction reads it: nothing to clear
  hipStream_t st = S(stream);
  launch_metrics_partials(images, clean, px, nchunks, B, parts, st);
  launch_reduce_metrics(parts, nullptr, nullptr, (uint32_t)nchunks, nullptr, nullptr, nullptr, (uint32_t)px, out, B, 1u,
                        st);
  return check_last("sg_metrics_noalloc");
}

}  // extern "C"
