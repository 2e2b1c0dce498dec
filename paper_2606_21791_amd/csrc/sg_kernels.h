// Host-side launchers of the libsg kernels (defined in the k_*.hip files) and
// small device helpers shared by several kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "sg_types.h"

namespace sg {

// Block-wide reduction of a metric partial in a fixed order (wave butterflies,
// then waves in index order), so the result does not depend on scheduling.
// Every thread of the block must call it; thread 0 writes *out and gets the
// changed-pixel total as the return value (0 elsewhere).  It holds one
// barrier: two calls by one workgroup must be separated by another barrier
// (the per-wave slots are reused), which every caller's control flow has.
__device__ __forceinline__ uint32_t block_reduce_partial(double sse, uint32_t changed, float mx, uint32_t nonfin,
                                                         unsigned long long evals, Partial* out) {
  for (int o = 32; o > 0; o >>= 1) {
    sse += __shfl_xor(sse, o);
    changed += (uint32_t)__shfl_xor((int)changed, o);
    mx = fmaxf(mx, __shfl_xor(mx, o));
    nonfin |= (uint32_t)__shfl_xor((int)nonfin, o);
    evals += __shfl_xor(evals, o);
  }
  __shared__ double s_sse[16];
  __shared__ unsigned long long s_ev[16];
  __shared__ uint32_t s_ch[16], s_nf[16];
  __shared__ float s_mx[16];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { s_sse[w] = sse; s_ch[w] = changed; s_mx[w] = mx; s_nf[w] = nonfin; s_ev[w] = evals; }
  __syncthreads();
  if (threadIdx.x != 0) return 0u;
  const int nw = (blockDim.x + 63) >> 6;
  Partial p;
  p.sse = 0.0; p.evals = 0; p.changed = 0; p.max_abs = 0.f; p.nonfinite = 0; p._pad = 0;
  for (int i = 0; i < nw; ++i) {
    p.sse += s_sse[i]; p.changed += s_ch[i]; p.max_abs = fmaxf(p.max_abs, s_mx[i]); p.nonfinite |= s_nf[i];
    p.evals += s_ev[i];
  }
  *out = p;
  return p.changed;
}

// One wave's sum of the partials parts[off .. off + n) in a fixed order (lane
// j takes entries j, j + 64, ...; then xor butterflies, whose results are
// the same in every lane).  rend (nullable; tiles_x > 0): regions of the
// entries, taken as the tiles of a full frame, that hold a changed pixel.
__device__ __forceinline__ Partial wave_reduce_parts(const Partial* __restrict__ parts, uint32_t off, uint32_t n,
                                                     int tiles_x, int tiles_y, uint64_t* rend) {
  const int lane = threadIdx.x & 63;
  Partial r;
  r.sse = 0.0; r.evals = 0; r.changed = 0; r.max_abs = 0.f; r.nonfinite = 0; r._pad = 0;
  uint64_t rg = 0;
  for (uint32_t k = lane; k < n; k += 64) {
    const Partial p = parts[off + k];
    if (tiles_x > 0 && p.changed) rg |= region_bit((int)k % tiles_x, (int)k / tiles_x, tiles_x, tiles_y);
    r.sse += p.sse;
    r.changed += p.changed;
    r.max_abs = fmaxf(r.max_abs, p.max_abs);
    r.nonfinite |= p.nonfinite;
    r.evals += p.evals;
  }
  for (int o = 32; o > 0; o >>= 1) {
    r.sse += __shfl_xor(r.sse, o);
    r.changed += (uint32_t)__shfl_xor((int)r.changed, o);
    r.max_abs = fmaxf(r.max_abs, __shfl_xor(r.max_abs, o));
    r.nonfinite |= (uint32_t)__shfl_xor((int)r.nonfinite, o);
    r.evals += __shfl_xor(r.evals, o);
    rg |= __shfl_xor(rg, o);
  }
  if (rend) *rend = rg;
  return r;
}

// The record of one variant from its reduced partial (Def. 1 footprint,
// Def. 2 catastrophe, PSNR on [0, 1] images over the three channels).
__device__ __forceinline__ sg_metrics_t make_metrics(const Partial& red, uint32_t extra_nonfinite, uint32_t dirty,
                                                     unsigned long long clamps, uint32_t n_pixels, uint32_t path,
                                                     uint64_t pred_regions = 0, uint64_t rend_regions = 0) {
  sg_metrics_t m;
  m.sse = red.sse;
  m.mse = red.sse / (3.0 * (double)n_pixels);
  m.psnr = m.mse == 0.0 ? __longlong_as_double(0x7ff0000000000000ll) : 10.0 * log10(1.0 / m.mse);
  m.changed_px = red.changed;
  m.footprint = (float)((double)red.changed / (double)n_pixels);
  m.max_abs = red.max_abs;
  m.nonfinite = red.nonfinite | extra_nonfinite;
  m.catastrophic = (m.nonfinite || (double)red.changed > 0.01 * (double)n_pixels) ? 1u : 0u;
  m.dirty_tiles = dirty;
  m.clamps = clamps;
  m.n_pixels = n_pixels;
  m.path = path;
  m.evals = red.evals;
  m.predicted_regions = pred_regions;
  m.rendered_regions = rend_regions;
  return m;
}

// The record of variant v of an incremental batch from its item partials
// and its state (one wave; lane 0 writes out[v]).
__device__ __forceinline__ void reduce_batch_variant(const Partial* __restrict__ parts, const uint32_t* item_off,
                                                     const uint32_t* n_items, const VariantState* vs,
                                                     uint32_t n_pixels, int v, sg_metrics_t* __restrict__ out) {
  const Partial red = wave_reduce_parts(parts, item_off[v], n_items[v], 0, 0, nullptr);
  if ((threadIdx.x & 63) == 0) {
    const VariantState& s = vs[v];
    out[v] = make_metrics(red, s.nonfinite, s.n_dirty, s.clamps, n_pixels, 0u, s.pred_regions, s.rend_regions);
  }
}

// k_ssim.hip: the normalised 1-D Gaussian taps of the SSIM window
struct SsimWeights {
  double w[11];
};
int ssim_blocks(int H, int W);
void launch_ssim(const float* imgs, const float* clean, int B, int H, int W, const SsimWeights& gw, double* partial,
                 double* out, hipStream_t st);

// k_basic.hip
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
void launch_cast(const float* src, void* dst, int64_t n, int dtype, int mode, hipStream_t st);
void launch_inject(const DevScene& s, const sg_site* sites, int n, uint32_t* saved, hipStream_t st);
void launch_box_reduce(const DevScene& s, int f, uint32_t* kmin, uint32_t* kmax, hipStream_t st);
void launch_box_finalize(const uint32_t* kmin, const uint32_t* kmax, int C, int dtype, void* lo, void* hi,
                         hipStream_t st);
void launch_guard(const DevScene& s, const DevBox& b, int f, unsigned long long* count, hipStream_t st);
// Component rows (field, component) guarded by one launch; global box and
// contiguous primitives only.
struct GuardRows {
  int n_rows;
  int f[64];
  int c[64];
};
void launch_guard_rows(const DevScene& s, const DevBox& b, const GuardRows& gr, unsigned long long* count,
                       hipStream_t st);
void launch_health(const unsigned long long* count, unsigned long long thr, uint32_t* alert, hipStream_t st);
void launch_metrics_partials(const float* img, const float* clean, int64_t px_per_var, int nchunks, int B,
                             Partial* out, hipStream_t st);
// Pools the K view records of each of B variants; view k of variant v is
// views[k * view_stride + v * var_stride].
void launch_pool_views(const sg_metrics_t* views, int K, int B, int64_t view_stride, int64_t var_stride,
                       sg_metrics_t* out, hipStream_t st);
// tiles_x > 0 marks per-tile partials of a full render (uniform_items tiles):
// their rendered regions are derived from the tiles with a changed pixel.
void launch_reduce_metrics(const Partial* parts, const uint32_t* item_off, const uint32_t* n_items,
                           uint32_t uniform_items, const VariantState* vs, const uint32_t* flags,
                           const unsigned long long* clamps, uint32_t n_pixels, sg_metrics_t* out, int B,
                           uint32_t path, hipStream_t st, int tiles_x = 0, int tiles_y = 0);

// k_project.hip
struct ProjBuffers {
  Rec* rec;               // one 48-byte record per primitive: a list entry's gather touches one or two lines
  uint32_t* depth;
  uint2* rect;            // (tx0 | ty0 << 16, tx1 | ty1 << 16); x = 0xffffffff when culled
  int32_t* diff;          // (tiles_y + 1) x (tiles_x + 1) 2-D difference grid of tile counts
  uint32_t* flags;        // [0] any stored non-finite, [1] (unused)
  unsigned long long* clamps;
};
void launch_project(const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                    const ProjBuffers& pb, int n_cu, hipStream_t st);

struct BatchBuffers {
  const sg_site* sites;
  const sg_variant* variants;
  int B;
  VariantState* vs;
  Rec* ovr;                 // B * kRecSlots records: each variant's corrupted and clean touch records
  uint32_t* item_off;       // B + 1: first item of each variant, then the total
  uint32_t* n_items_v;      // B: work items (dirty tiles that can change) per variant
  // B x n_tiles work items: variant v's at [v * n_tiles, ...), each
  // {tile, first entry of its clean list, clean list length, 0}
  uint4* items;
  uint32_t* counter;        // compositing work counter, armed by the last prep workgroup
  uint32_t* arrive;         // prep workgroups that have finished (zero between batches)
  int tiles_x, tiles_y, n_tiles;
  const uint64_t* stop_key; // per tile of the prepared view (nullable): see CompArgs
  const uint32_t* tile_start;
  const uint32_t* tile_cnt;
};
void launch_variant_prep(const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                         const Rec* rec, const uint32_t* depth, const uint2* rect, const BatchBuffers& bb,
                         hipStream_t st);
// Campaign pre-pass over n variants: states (touches, clamps, non-finite
// flag) and records (kRecSlots per variant: corrupted, then clean).  Variant
// g's state is vs[g * stride + offset] and its records start at
// ovr[(g * stride + offset) * kRecSlots] (stride K, offset the view: the views
// of a variant side by side).
// view_of (nullable): only the variants g with view_of[g] == view are staged
// (a campaign over several scenes stages each scene's variants in its launch).
void launch_campaign_touch(const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                           const Rec* rec, const uint32_t* depth, const uint2* rect, const sg_site* sites,
                           const sg_variant* variants, int n,
                           VariantState* vs, Rec* ovr, int stride, int offset, const uint16_t* view_of, int view,
                           hipStream_t st);

// k_bin.hip
struct BinBuffers {
  int32_t* diff;
  uint32_t* tile_cnt;
  uint32_t* tile_start;
  uint32_t* cursor;
  // [0] instances, [1] big prims, [2] big tiles (lists longer than one LDS
  // sort), [3] longest big list, [4] LDS chunks of big tiles, [5] merge blocks
  // of big tiles
  unsigned long long* total;
  uint64_t* keys;
  uint64_t* keys_tmp;
  uint32_t* big_prims;
  uint32_t* big_tiles;        // big tiles in tile order
  uint32_t* big_choff;        // per big tile (+1): first LDS chunk
  uint32_t* big_goff;         // per big tile (+1): first merge block
  uint32_t* big_split;        // per merge block: its first output's position in run A
  uint2* big_map;             // per merge block, then per LDS chunk: (tile, index within the tile)
  int64_t capacity;
};
void launch_tile_prefix(const DevRaster& ras, const BinBuffers& bb, hipStream_t st);
void launch_emit(int n, const uint32_t* depth, const uint2* rect, const DevRaster& ras, const BinBuffers& bb,
                 int n_cu, hipStream_t st);
// totals: host copy of bb.total[0..5] after k_tile_prefix
void launch_tile_sort(const DevRaster& ras, const BinBuffers& bb, const unsigned long long* totals, int n_cu,
                      hipStream_t st);

// k_composite.hip
// Per-pixel stop keys of a prepared clean render (CompArgs::stop): list keys
// are (depth bits << 32 | id) with a finite positive depth, so both markers
// compare above every key.
constexpr uint64_t kStopNever = ~0ull;
constexpr uint64_t kStopNonfinite = ~0ull - 1;
struct CompArgs {
  const Rec* rec;         // projected records, by primitive
  const uint32_t* tile_start;
  const uint32_t* tile_cnt;
  const uint64_t* keys;
  const float* clean;     // nullable
  float* image;           // nullable
  Partial* parts;         // per tile / per item; nullable when clean is null
  DevRaster ras;
  int32_t W, H;
  // Resume state of a prepared clean render.  stop[p]: the key of the entry
  // at which pixel p stopped (kStopNever if it never stopped, kStopNonfinite
  // if its colour was not finite).  ck: per tile, the (C, T)
  // state of every pixel after each multiple of ck_group list entries, in
  // slots ck_off[tile] + k - 1 for k = 1 .. count / ck_group.  The clean
  // render of sg_prepare writes them (*_out); the incremental path reads them.
  // stop_key[t]: the key of the entry at which the last pixel of tile t
  // stopped (all ones if a pixel never stopped or was not finite).
  const uint64_t* stop = nullptr;
  const float4* ck = nullptr;
  const uint32_t* ck_off = nullptr;
  const uint64_t* stop_key = nullptr;
  uint64_t* stop_out = nullptr;
  float4* ck_out = nullptr;
  uint64_t* stop_key_out = nullptr;
  uint32_t ck_group = 0;
};
void launch_composite_full(const CompArgs& a, hipStream_t st);
struct ItemArgs {
  VariantState* vs;         // the items OR their regions into it
  const Rec* ovr;
  const uint4* items;       // see BatchBuffers
  const uint32_t* item_off; // B + 1
  uint32_t* counter;
  int64_t image_stride;   // floats per variant image (when a.image != null)
  int grid;
  int B;
};
void launch_composite_items(const CompArgs& a, const ItemArgs& it, hipStream_t st);

// One step of a pipelined campaign stream: the work items of batch j + 1,
// the compositing of batch j and the metric reduction of batch j - 1, each
// in workgroups of their own and on buffers of their own, so that nothing
// in the launch waits for anything else in it.  A role with no batch has
// B = 0.
// The clean state of one prepared view of a multi-view step: a camera view
// of the batch's scene, or one of several scenes of uneven size.
struct ViewArgs {
  const Rec* rec;
  const uint32_t* tile_start;
  const uint32_t* tile_cnt;
  const uint64_t* keys;
  const float* clean;
  const uint64_t* stop;
  const float4* ck;
  const uint32_t* ck_off;
  const uint64_t* stop_key;
  DevRaster ras;        // its tile grid and compositing constants
  int32_t W, H;
  uint32_t ck_group;    // checkpoint spacing of its resume state (0: none)
};

struct StepArgs {
  // work items of the next batch: one workgroup (its first wave) per variant
  int tB;
  VariantState* t_vs;       // the batch's variant states (touches in, n_dirty and regions out)
  const Rec* t_ovr;         // their touch records (kRecSlots per variant)
  uint4* t_items;           // tB x n_tiles
  uint32_t* t_n_items;
  uint32_t* t_item_off;
  uint32_t* t_counter;
  uint32_t* t_arrive;
  int tiles_x, tiles_y, n_tiles;
  const uint64_t* stop_key;
  const uint32_t* tile_start;
  const uint32_t* tile_cnt;
  // metrics of the previous batch: one wave per variant
  int rB;
  const Partial* r_parts;
  const uint32_t* r_item_off;
  const uint32_t* r_n_items;
  const VariantState* r_vs;
  sg_metrics_t* r_out;
  uint32_t n_pixels;
  // compositing of the current batch (I.B = 0: none)
  CompArgs A;
  ItemArgs I;
  // Multi-view steps (views != null): each variant-view takes its view's
  // clean state from views[] in place of the fields of A (and of stop_key,
  // tile_start, tile_cnt, tiles_x, tiles_y and n_pixels above) that differ by
  // view.  Either every variant in K views (K > 1, view k of variant v at
  // index v * K + k), or every variant in one view of its own (*_view_of:
  // the view of each variant of the role's batch).  Work items then sit
  // n_tiles (the largest view's tile count) apart per variant-view.
  int K = 1;
  const ViewArgs* views = nullptr;
  const uint16_t* t_view_of = nullptr;
  const uint16_t* i_view_of = nullptr;
  const uint16_t* r_view_of = nullptr;
};
// e0, e1 (nullable): events recorded at the launch's own start and end.
void launch_campaign_step(const StepArgs& a, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Campaign-wide persistent path.  A chunk of a campaign's variants (or
// variant-views) is rendered by three launches on one stream: one lists the
// work items of every variant compactly, one persistent launch composites all
// of them, one reduces each variant's record.
struct PersistArgs {
  CompArgs A;               // clean state of the single view and the per-item partials A.parts (no images)
  VariantState* vs;         // the chunk's variant states (from the campaign pre-pass)
  const Rec* ovr;           // their touch records, kRecSlots per variant
  uint4* items;             // work items {tile, first entry of its clean list, its length, variant}
  uint32_t* item_off;       // per variant: index of its first item
  uint32_t* n_items;        // per variant: its item count
  uint32_t* ctl;            // [0] items listed so far (the list's cursor), [1] compositing work counter
  int nv;                   // variants (variant-views) of the chunk
  int grid;                 // workgroups of the persistent compositing launch
  sg_metrics_t* out;        // per variant (variant-view): its record
  uint32_t n_pixels;        // single view: pixels of the frame
  // Several views or scenes (views != null), as in StepArgs: each
  // variant-view takes its view's clean state, tile grid and size from
  // views[view_of ? view_of[v] : v % K].
  int K = 1;
  const ViewArgs* views = nullptr;
  const uint16_t* view_of = nullptr;
};
void launch_persist_list(const PersistArgs& a, hipStream_t st);
// e0, e1 (nullable): events recorded at the launch's own start and end.
void launch_persist_composite(const PersistArgs& a, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_persist_reduce(const PersistArgs& a, hipStream_t st);
// Resident workgroups per CU of the persistent compositing kernel at a tile size.
int persist_occupancy(int tile, bool mv);

}  // namespace sg
