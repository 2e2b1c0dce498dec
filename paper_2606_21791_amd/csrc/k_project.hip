// Projection of every primitive (full renders) and of the corrupted
// primitives of each variant (incremental renders), plus the planning of the
// dirty-tile work items of a batch.
#include "sg_batch.h"
#include "sg_device.h"
#include "sg_kernels.h"

#include <algorithm>

namespace sg {

// Projection of every primitive, grid-stride.  All stored words of a
// primitive are loaded first (independent, coalesced loads: field f,
// component c of consecutive primitives are consecutive words in the
// component-major layout), clamped in registers if a box is given, then
// projected.  Each visible primitive adds its tile rectangle to a 2-D
// difference grid; when the grid fits in LDS the block accumulates it there
// and flushes its nonzero entries with one global atomic each.
template <int DEG, bool LDS_GRID>
__global__ void __launch_bounds__(256) k_project(DevScene s, DevBox box, DevCam cam, DevRaster ras, ProjBuffers pb) {
  using L = Layout<DEG>;
  extern __shared__ int s_diff[];
  const int X = ras.tiles_x + 1;
  const int nd = X * (ras.tiles_y + 1);
  if (LDS_GRID) {
    for (int k = threadIdx.x; k < nd; k += blockDim.x) s_diff[k] = 0;
    __syncthreads();
  }
  uint32_t clamps = 0;
  bool nonfin = false;
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < s.n; i0 += (int64_t)gridDim.x * blockDim.x) {
    // The index passes through an empty asm statement, so the compiler forms
    // each word's address from it inside the loop instead of keeping one
    // 64-bit pointer per loaded word, box word and output live across
    // iterations (that strength reduction took SH degree 0 from 153 to 238
    // VGPRs, two waves per SIMD instead of three, and made degree 3 spill).
    int64_t i = i0;
    asm volatile("" : "+v"(i));
    uint32_t w[L::kWords];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int C = f < 5 ? (f == 2 ? 4 : (f == 3 ? 1 : 3)) : L::kRest;
#pragma unroll
      for (int c = 0; c < C; ++c) w[L::off(f) + c] = load_word(s, f, i, c);
    }
    if (box.mask) {
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const int C = f < 5 ? (f == 2 ? 4 : (f == 3 ? 1 : 3)) : L::kRest;
        if (!((box.mask >> f) & 1u)) continue;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          uint32_t lo, hi;
          bool cl;
          box_words(box, f, i, c, s.n, &lo, &hi);
          w[L::off(f) + c] = clamp_word(w[L::off(f) + c], lo, hi, s.dtype, &cl);
          clamps += cl ? 1u : 0u;
        }
      }
    }
    auto get = [&](int f, int c) -> uint32_t { return w[L::off(f) + c]; };
    const ProjOut o = project_prim<DEG>(get, s.dtype, cam, ras);
    nonfin |= o.nonfinite;
    pb.rec[i] = o.rec;
    pb.depth[i] = o.depth;
    pb.rect[i] = o.visible ? make_uint2(o.rect0, o.rect1) : make_uint2(0xffffffffu, 0u);
    if (o.visible) {
      const int tx0 = o.rect0 & 0xffff, ty0 = o.rect0 >> 16, tx1 = o.rect1 & 0xffff, ty1 = o.rect1 >> 16;
      if (LDS_GRID) {
        atomicAdd(s_diff + ty0 * X + tx0, 1);
        atomicAdd(s_diff + ty0 * X + tx1 + 1, -1);
        atomicAdd(s_diff + (ty1 + 1) * X + tx0, -1);
        atomicAdd(s_diff + (ty1 + 1) * X + tx1 + 1, 1);
      } else {
        atomicAdd(pb.diff + ty0 * X + tx0, 1);
        atomicAdd(pb.diff + ty0 * X + tx1 + 1, -1);
        atomicAdd(pb.diff + (ty1 + 1) * X + tx0, -1);
        atomicAdd(pb.diff + (ty1 + 1) * X + tx1 + 1, 1);
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) clamps += (uint32_t)__shfl_xor((int)clamps, o);
  const unsigned long long nf = __ballot(nonfin);
  if ((threadIdx.x & 63) == 0) {
    if (clamps && pb.clamps) atomicAdd(pb.clamps, (unsigned long long)clamps);
    if (nf) atomicOr(pb.flags, 1u);
  }
  if (LDS_GRID) {
    __syncthreads();
    for (int k = threadIdx.x; k < nd; k += blockDim.x) {
      const int v = s_diff[k];
      if (v) atomicAdd(pb.diff + k, v);
    }
  }
}

// Stages a variant's corrupted primitives (at most kMaxTouch distinct ones;
// more set st.full and stage none).  Lane c loads stored word c of each,
// XORs the variant's sites into it and clamps it (if guarded); lane 0
// projects the primitive from the staged words and compares the result with
// its clean record.  st (LDS) receives the touches, the clamp count and the
// non-finite flag (n_dirty and the regions zero); ovr[j] receives touch j's
// corrupted record and ovr[kMaxTouch + j] its clean one (when visible).  One
// 64-thread workgroup; every lane calls it.
template <int DEG>
__device__ void stage_touches(const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                              const Rec* __restrict__ rec, const uint32_t* __restrict__ depth,
                              const uint2* __restrict__ rect, const sg_variant& var, const sg_site* g_sites,
                              VariantState& st, Rec* ovr) {
  using L = Layout<DEG>;
  const int lane = threadIdx.x;
  // read the variant's sites once, staging up to 64 of them in LDS
  __shared__ sg_site s_sites[64];
  __shared__ uint32_t s_w[L::kWords];
  if ((uint32_t)lane < var.n_sites && lane < 64) s_sites[lane] = g_sites[var.site_off + lane];
  const sg_site* sites = var.n_sites <= 64 ? s_sites : g_sites + var.site_off;
  const bool guard = var.guard != 0 && box.mask != 0;
  __syncthreads();
  if (lane == 0) {
    st.n_touch = 0; st.full = 0; st.nonfinite = 0; st.n_dirty = 0; st.clamps = 0; st._pad0 = 0; st._pad = 0;
    st.pred_regions = 0; st.rend_regions = 0;
    for (uint32_t k = 0; k < var.n_sites; ++k) {
      const uint32_t p = sites[k].prim;
      bool seen = false;
      for (uint32_t j = 0; j < st.n_touch; ++j) seen |= st.touch[j].prim == p;
      if (!seen) {
        if (st.n_touch == kMaxTouch) { st.full = 1; break; }
        st.touch[st.n_touch++].prim = p;
      }
    }
    if (st.full) st.n_touch = 0;
  }
  __syncthreads();
  const uint32_t n_touch = st.n_touch;
  for (uint32_t j = 0; j < n_touch; ++j) {
    const uint32_t p = st.touch[j].prim;
    uint32_t cl_count = 0;
    if (lane < L::kWords) {
      const int f = lane < 3 ? 0 : lane < 6 ? 1 : lane < 10 ? 2 : lane < 11 ? 3 : lane < 14 ? 4 : 5;
      const int c = lane - L::off(f);
      uint32_t w = load_word(s, f, p, c);
      for (uint32_t k = 0; k < var.n_sites; ++k) {
        const sg_site x = sites[k];
        if (x.prim == p && x.field == f && x.comp == c && !site_corrected(var.protect, x.bit, s.dtype))
          w ^= 1u << x.bit;
      }
      if (guard && ((box.mask >> f) & 1u)) {
        uint32_t lo, hi;
        bool cl;
        box_words(box, f, p, c, s.n, &lo, &hi);
        w = clamp_word(w, lo, hi, s.dtype, &cl);
        cl_count = cl ? 1u : 0u;
      }
      s_w[lane] = w;
    }
    for (int o = 32; o > 0; o >>= 1) cl_count += (uint32_t)__shfl_xor((int)cl_count, o);
    __syncthreads();
    if (lane == 0) {
      st.clamps += cl_count;
      auto get = [&](int f, int c) -> uint32_t { return s_w[L::off(f) + c]; };
      const ProjOut o = project_prim<DEG>(get, s.dtype, cam, ras);
      st.nonfinite |= o.nonfinite ? 1u : 0u;
      const uint2 orc = rect[p];
      const bool old_vis = orc.x != 0xffffffffu;
      Touch& t = st.touch[j];
      t.old_depth = depth[p];
      t.old_rect0 = orc.x;
      t.old_rect1 = orc.y;
      t.new_depth = o.depth;
      t.new_rect0 = o.rect0;
      t.new_rect1 = o.rect1;
      bool same = old_vis == o.visible;
      if (same && old_vis) {
        const float4 a0 = rec[p].r0, a1 = rec[p].r1, a2 = rec[p].r2;
        same = t.old_depth == t.new_depth && orc.x == o.rect0 && orc.y == o.rect1 &&
               __float_as_uint(a0.x) == __float_as_uint(o.rec.r0.x) && __float_as_uint(a0.y) == __float_as_uint(o.rec.r0.y) &&
               __float_as_uint(a0.z) == __float_as_uint(o.rec.r0.z) && __float_as_uint(a0.w) == __float_as_uint(o.rec.r0.w) &&
               __float_as_uint(a1.x) == __float_as_uint(o.rec.r1.x) && __float_as_uint(a1.y) == __float_as_uint(o.rec.r1.y) &&
               __float_as_uint(a1.z) == __float_as_uint(o.rec.r1.z) && __float_as_uint(a1.w) == __float_as_uint(o.rec.r1.w) &&
               __float_as_uint(a2.x) == __float_as_uint(o.rec.r2.x) && __float_as_uint(a2.y) == __float_as_uint(o.rec.r2.y) &&
               __float_as_uint(a2.z) == __float_as_uint(o.rec.r2.z) && __float_as_uint(a2.w) == __float_as_uint(o.rec.r2.w);
      }
      t.flags = (old_vis ? 1u : 0u) | (o.visible ? 2u : 0u) | (same ? 4u : 0u);
      ovr[j] = o.rec;
      if (old_vis) ovr[kMaxTouch + j] = rec[p];
    }
    __syncthreads();
  }
}

// One 64-thread workgroup per variant of an sg_render_batch batch: stages
// the variant's corrupted primitives, lists its work items and, in the
// workgroup that finishes last, the batch's item offsets.
template <int DEG>
__global__ void __launch_bounds__(64) k_variant_prep(DevScene s, DevBox box, DevCam cam, DevRaster ras,
                                                     const Rec* __restrict__ rec,
                                                     const uint32_t* __restrict__ depth,
                                                     const uint2* __restrict__ rect, BatchBuffers bb) {
  const int v = blockIdx.x;
  __shared__ VariantState st;
  const sg_variant var = bb.variants[v];
  stage_touches<DEG>(s, box, cam, ras, rec, depth, rect, var, bb.sites, st, bb.ovr + (int64_t)v * kRecSlots);
  uint32_t nd, ni;
  uint64_t pred;
  const ReachArgs ra{bb.ovr + (int64_t)v * kRecSlots, ras.tile, cam.W, cam.H, ras.qcut2, ras.amin};
  enumerate_items(st.touch, st.n_touch, bb.tiles_x, bb.tiles_y, bb.stop_key, bb.tile_start, bb.tile_cnt, ra,
                  bb.items + (int64_t)v * bb.n_tiles, &nd, &ni, &pred);
  if (threadIdx.x == 0) {
    st.n_dirty = nd;
    st.pred_regions = pred;
    bb.vs[v] = st;
    bb.n_items_v[v] = ni;
  }
  finish_batch(bb.arrive, gridDim.x, bb.n_items_v, bb.item_off, bb.B, bb.counter);
}

// Campaign pre-pass: the staged corrupted primitives of every variant of a
// campaign chunk at once, one thread per variant, written to the campaign's
// per-variant states and touch records.  The steps are those of
// stage_touches, in its order: the first kMaxTouch distinct primitives of
// the variant's sites (more: st.full and none staged), each primitive's
// stored words with the variant's sites XORed in and the guard clamp
// applied, its projection, and the comparison with its clean record.
template <int DEG>
__global__ void __launch_bounds__(64) k_campaign_touch(DevScene s, DevBox box, DevCam cam, DevRaster ras,
                                                       const Rec* __restrict__ rec,
                                                       const uint32_t* __restrict__ depth,
                                                       const uint2* __restrict__ rect, const sg_site* sites,
                                                       const sg_variant* variants, int n, VariantState* vs, Rec* ovr,
                                                       int stride, int offset, const uint16_t* view_of, int view) {
  using L = Layout<DEG>;
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n) return;
  if (view_of && view_of[g] != view) return;   // a variant of another scene
  const sg_variant var = variants[g];
  const sg_site* vsites = sites + var.site_off;
  const bool guard = var.guard != 0 && box.mask != 0;
  uint32_t prims[kMaxTouch];
  uint32_t n_touch = 0, full = 0;
  for (uint32_t k = 0; k < var.n_sites; ++k) {
    const uint32_t p = vsites[k].prim;
    bool seen = false;
    for (uint32_t j = 0; j < n_touch; ++j) seen |= prims[j] == p;
    if (!seen) {
      if (n_touch == kMaxTouch) { full = 1; break; }
      prims[n_touch++] = p;
    }
  }
  if (full) n_touch = 0;
  const int64_t slot = g * stride + offset;   // this variant's state and records
  VariantState* out = vs + slot;
  unsigned long long clamps = 0;
  uint32_t nonfinite = 0;
  for (uint32_t j = 0; j < n_touch; ++j) {
    const uint32_t p = prims[j];
    uint32_t w[L::kWords];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int C = f < 5 ? (f == 2 ? 4 : (f == 3 ? 1 : 3)) : L::kRest;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        uint32_t x = load_word(s, f, p, c);
        for (uint32_t k = 0; k < var.n_sites; ++k) {
          const sg_site t = vsites[k];
          if (t.prim == p && t.field == f && t.comp == c && !site_corrected(var.protect, t.bit, s.dtype))
            x ^= 1u << t.bit;
        }
        if (guard && ((box.mask >> f) & 1u)) {
          uint32_t lo, hi;
          bool cl;
          box_words(box, f, p, c, s.n, &lo, &hi);
          x = clamp_word(x, lo, hi, s.dtype, &cl);
          clamps += cl ? 1ull : 0ull;
        }
        w[L::off(f) + c] = x;
      }
    }
    auto get = [&](int f, int c) -> uint32_t { return w[L::off(f) + c]; };
    const ProjOut o = project_prim<DEG>(get, s.dtype, cam, ras);
    nonfinite |= o.nonfinite ? 1u : 0u;
    const uint2 orc = rect[p];
    const bool old_vis = orc.x != 0xffffffffu;
    Touch t;
    t.prim = p;
    t.old_depth = depth[p];
    t.old_rect0 = orc.x;
    t.old_rect1 = orc.y;
    t.new_depth = o.depth;
    t.new_rect0 = o.rect0;
    t.new_rect1 = o.rect1;
    bool same = old_vis == o.visible;
    if (same && old_vis) {
      const float4 a0 = rec[p].r0, a1 = rec[p].r1, a2 = rec[p].r2;
      same = t.old_depth == t.new_depth && orc.x == o.rect0 && orc.y == o.rect1 &&
             __float_as_uint(a0.x) == __float_as_uint(o.rec.r0.x) && __float_as_uint(a0.y) == __float_as_uint(o.rec.r0.y) &&
             __float_as_uint(a0.z) == __float_as_uint(o.rec.r0.z) && __float_as_uint(a0.w) == __float_as_uint(o.rec.r0.w) &&
             __float_as_uint(a1.x) == __float_as_uint(o.rec.r1.x) && __float_as_uint(a1.y) == __float_as_uint(o.rec.r1.y) &&
             __float_as_uint(a1.z) == __float_as_uint(o.rec.r1.z) && __float_as_uint(a1.w) == __float_as_uint(o.rec.r1.w) &&
             __float_as_uint(a2.x) == __float_as_uint(o.rec.r2.x) && __float_as_uint(a2.y) == __float_as_uint(o.rec.r2.y) &&
             __float_as_uint(a2.z) == __float_as_uint(o.rec.r2.z) && __float_as_uint(a2.w) == __float_as_uint(o.rec.r2.w);
    }
    t.flags = (old_vis ? 1u : 0u) | (o.visible ? 2u : 0u) | (same ? 4u : 0u);
    out->touch[j] = t;
    ovr[slot * kRecSlots + j] = o.rec;
    if (old_vis) ovr[slot * kRecSlots + kMaxTouch + j] = rec[p];
  }
  out->n_touch = n_touch;
  out->full = full;
  out->nonfinite = nonfinite;
  out->n_dirty = 0;
  out->clamps = clamps;
  out->_pad0 = 0;
  out->_pad = 0;
  out->pred_regions = 0;
  out->rend_regions = 0;
}

// Workgroups of k_project<D, LDS> resident per CU with shm bytes of LDS
// each.  The grid-stride launch uses exactly that many per CU, so that all of
// them run in one round: a partial second round would run with one wave per
// SIMD.  Cached per host thread for the last LDS size asked.
template <int D, bool LDS>
static int project_occupancy(size_t shm) {
  thread_local size_t last_shm = ~(size_t)0;
  thread_local int last = 1;
  if (shm != last_shm) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_project<D, LDS>, 256, shm) != hipSuccess) {
      (void)hipGetLastError();
      nb = 1;
    }
    last_shm = shm;
    last = nb > 0 ? nb : 1;
  }
  return last;
}

void launch_project(const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                    const ProjBuffers& pb, int n_cu, hipStream_t st) {
  const int64_t need = ((int64_t)s.n + 255) / 256;
  const int nd = (ras.tiles_x + 1) * (ras.tiles_y + 1);
  const bool lds = nd <= 16384;
  const size_t shm = lds ? (size_t)nd * sizeof(int) : 0;
  // with the grid in LDS: one round of resident workgroups, each flushing its grid once
#define SG_PROJ(D)                                                                                              \
  if (lds) {                                                                                                    \
    const unsigned blocks = (unsigned)std::min<int64_t>(need, (int64_t)n_cu * project_occupancy<D, true>(shm)); \
    k_project<D, true><<<blocks, 256, shm, st>>>(s, box, cam, ras, pb);                                         \
  } else {                                                                                                      \
    k_project<D, false><<<(unsigned)need, 256, 0, st>>>(s, box, cam, ras, pb);                                  \
  }
  switch (s.sh_degree) {
    case 0: SG_PROJ(0) break;
    case 1: SG_PROJ(1) break;
    case 2: SG_PROJ(2) break;
    default: SG_PROJ(3) break;
  }
#undef SG_PROJ
}

void launch_variant_prep(const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                         const Rec* rec, const uint32_t* depth, const uint2* rect, const BatchBuffers& bb,
                         hipStream_t st) {
  const int grid = bb.B;
  if (grid <= 0) return;
  switch (s.sh_degree) {
    case 0: k_variant_prep<0><<<grid, 64, 0, st>>>(s, box, cam, ras, rec, depth, rect, bb); break;
    case 1: k_variant_prep<1><<<grid, 64, 0, st>>>(s, box, cam, ras, rec, depth, rect, bb); break;
    case 2: k_variant_prep<2><<<grid, 64, 0, st>>>(s, box, cam, ras, rec, depth, rect, bb); break;
    default: k_variant_prep<3><<<grid, 64, 0, st>>>(s, box, cam, ras, rec, depth, rect, bb); break;
  }
}

void launch_campaign_touch(const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                           const Rec* rec, const uint32_t* depth, const uint2* rect, const sg_site* sites,
                           const sg_variant* variants, int n,
                           VariantState* vs, Rec* ovr, int stride, int offset, const uint16_t* view_of, int view,
                           hipStream_t st) {
  if (n <= 0) return;
  const int grid = (n + 63) / 64;
  switch (s.sh_degree) {
    case 0: k_campaign_touch<0><<<grid, 64, 0, st>>>(s, box, cam, ras, rec, depth, rect, sites, variants, n, vs, ovr, stride, offset, view_of, view); break;
    case 1: k_campaign_touch<1><<<grid, 64, 0, st>>>(s, box, cam, ras, rec, depth, rect, sites, variants, n, vs, ovr, stride, offset, view_of, view); break;
    case 2: k_campaign_touch<2><<<grid, 64, 0, st>>>(s, box, cam, ras, rec, depth, rect, sites, variants, n, vs, ovr, stride, offset, view_of, view); break;
    default: k_campaign_touch<3><<<grid, 64, 0, st>>>(s, box, cam, ras, rec, depth, rect, sites, variants, n, vs, ovr, stride, offset, view_of, view); break;
  }
}

}  // namespace sg
