// Projection of every primitive (full renders) and of the corrupted
// primitives of each variant (incremental renders), plus the planning of the
// dirty-tile work items of a batch.
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
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s.n; i += (int64_t)gridDim.x * blockDim.x) {
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
    pb.r0[i] = o.rec.r0;
    pb.r1[i] = o.rec.r1;
    pb.r2[i] = o.rec.r2;
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

__device__ __forceinline__ void set_rect_bits(uint64_t* bm, int row_words, uint32_t r0, uint32_t r1, int lane,
                                              int nlanes) {
  const int tx0 = r0 & 0xffff, ty0 = r0 >> 16, tx1 = r1 & 0xffff, ty1 = r1 >> 16;
  for (int ty = ty0 + lane; ty <= ty1; ty += nlanes) {
    for (int w = tx0 >> 6; w <= (tx1 >> 6); ++w) {
      const int a = max(tx0, w * 64) - w * 64, b = min(tx1, w * 64 + 63) - w * 64;
      const uint64_t m = (b == 63 ? ~0ull : ((1ull << (b + 1)) - 1ull)) & ~((1ull << a) - 1ull);
      bm[ty * row_words + w] |= m;
    }
  }
}

// One 64-thread workgroup per variant.  Lane c loads stored word c of each
// corrupted primitive, XORs the variant's sites into it and clamps it (if
// guarded); lane 0 projects the primitive from the staged words; the lanes
// then mark the tiles of the old and new footprints dirty.  Workgroup v
// first reduces the metrics of variant v of the workspace's previous batch
// when that is pending (the grid then covers both batches).
template <int DEG>
__global__ void __launch_bounds__(64) k_variant_prep(DevScene s, DevBox box, DevCam cam, DevRaster ras,
                                                     const float4* __restrict__ r0, const float4* __restrict__ r1,
                                                     const float4* __restrict__ r2,
                                                     const uint32_t* __restrict__ depth,
                                                     const uint2* __restrict__ rect, BatchBuffers bb) {
  using L = Layout<DEG>;
  const int v = blockIdx.x;
  const int lane = threadIdx.x;
  // the metrics of the previous batch of this workspace, before this batch
  // overwrites its item ranges and states
  if (v < bb.prev_B)
    reduce_batch_variant(bb.prev_parts, bb.item_off, bb.n_items_v, bb.vs, bb.n_pixels, v, bb.prev_out);
  if (v < bb.B) {
    // the batch's variants and sites may sit in pinned host memory: read each
    // once, staging up to 64 sites of the variant in LDS
    const sg_variant var = bb.variants[v];
    __shared__ sg_site s_sites[64];
    if ((uint32_t)lane < var.n_sites && lane < 64) s_sites[lane] = bb.sites[var.site_off + lane];
    const sg_site* sites = var.n_sites <= 64 ? s_sites : bb.sites + var.site_off;
    const bool guard = var.guard != 0 && box.mask != 0;
    __shared__ VariantState st;
    __shared__ uint32_t s_w[L::kWords];
    __shared__ uint32_t s_same;
    uint64_t* bm = bb.bitmap + (int64_t)v * bb.bm_words;
    for (int w = lane; w < bb.bm_words; w += 64) bm[w] = 0ull;
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
    }
    __syncthreads();
    const uint32_t n_touch = st.full ? 0u : st.n_touch;
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
          const float4 a0 = r0[p], a1 = r1[p], a2 = r2[p];
          same = t.old_depth == t.new_depth && orc.x == o.rect0 && orc.y == o.rect1 &&
                 __float_as_uint(a0.x) == __float_as_uint(o.rec.r0.x) && __float_as_uint(a0.y) == __float_as_uint(o.rec.r0.y) &&
                 __float_as_uint(a0.z) == __float_as_uint(o.rec.r0.z) && __float_as_uint(a0.w) == __float_as_uint(o.rec.r0.w) &&
                 __float_as_uint(a1.x) == __float_as_uint(o.rec.r1.x) && __float_as_uint(a1.y) == __float_as_uint(o.rec.r1.y) &&
                 __float_as_uint(a1.z) == __float_as_uint(o.rec.r1.z) && __float_as_uint(a1.w) == __float_as_uint(o.rec.r1.w) &&
                 __float_as_uint(a2.x) == __float_as_uint(o.rec.r2.x) && __float_as_uint(a2.y) == __float_as_uint(o.rec.r2.y) &&
                 __float_as_uint(a2.z) == __float_as_uint(o.rec.r2.z) && __float_as_uint(a2.w) == __float_as_uint(o.rec.r2.w);
        }
        t.flags = (old_vis ? 1u : 0u) | (o.visible ? 2u : 0u) | (same ? 4u : 0u);
        bb.ovr[(int64_t)v * kMaxTouch + j] = o.rec;
        s_same = same ? 1u : 0u;
      }
      __syncthreads();
      if (!s_same) {
        const Touch& t = st.touch[j];
        if (t.flags & 1u) set_rect_bits(bm, bb.row_words, t.old_rect0, t.old_rect1, lane, 64);
        __syncthreads();
        if (t.flags & 2u) set_rect_bits(bm, bb.row_words, t.new_rect0, t.new_rect1, lane, 64);
      }
      __syncthreads();
    }
    // The dirty tiles are the variant's predicted regions.  A dirty tile whose
    // last pixel stopped, in the clean render, before every key the variant
    // removes from or inserts into its list cannot change and gets no work
    // item.  The variant's items (its remaining dirty tiles in row order, each
    // with its clean list range) go to its own slice of the item list.  The
    // dirty tiles of 64 bitmap words are ranked, and lane r takes the tiles of
    // rank r, r + 64, ...: the per-tile reads of 64 tiles are in flight
    // together.
    __shared__ uint64_t s_word[64];
    __shared__ uint32_t s_wpre[65];   // set bits in the words below word k of the chunk
    uint4* my_items = bb.items + (int64_t)v * bb.n_tiles;
    uint32_t nd = 0, ni = 0;
    unsigned long long pred = 0;
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int base = 0; base < bb.bm_words; base += 64) {
      const int w = base + lane;
      const uint64_t word = w < bb.bm_words ? bm[w] : 0ull;
      const uint32_t c = (uint32_t)__popcll(word);
      uint32_t incl = c;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= o) incl += y;
      }
      s_word[lane] = word;
      s_wpre[lane + 1] = incl;
      if (lane == 0) s_wpre[0] = 0;
      __syncthreads();
      const uint32_t D = s_wpre[64];
      nd += D;
      for (uint32_t r0 = 0; r0 < D; r0 += 64) {
        const uint32_t r = r0 + (uint32_t)lane;
        bool keep = false;
        uint4 ent = make_uint4(0u, 0u, 0u, 0u);
        if (r < D) {
          int lo = 0, hi = 64;   // the word holding rank r: s_wpre[lo] <= r < s_wpre[lo + 1]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_wpre[mid] <= r) lo = mid; else hi = mid;
          }
          uint64_t wd = s_word[lo];
          uint32_t k = r - s_wpre[lo];   // rank of the bit within the word
          int bit = 0;
          for (int sh = 32; sh > 0; sh >>= 1) {
            const uint32_t below = (uint32_t)__popcll(wd & ((1ull << sh) - 1ull));
            if (k >= below) { k -= below; wd >>= sh; bit += sh; }
          }
          const int wi = base + lo;
          const int row = wi / bb.row_words, tx = (wi % bb.row_words) * 64 + bit;
          const int t = row * bb.tiles_x + tx;
          pred |= region_bit(tx, row, bb.tiles_x, bb.tiles_y);
          const unsigned long long sk = bb.stop_key ? bb.stop_key[t] : ~0ull;
          ent = make_uint4((uint32_t)t, bb.tile_start[t], bb.tile_cnt[t], 0u);
          keep = !bb.stop_key || tile_min_key(st.touch, n_touch, tx, row) <= sk;
        }
        const unsigned long long kb = __ballot(keep);
        if (keep) my_items[ni + (uint32_t)__popcll(kb & lt)] = ent;
        ni += (uint32_t)__popcll(kb);
      }
      __syncthreads();   // the next chunk reuses s_word and s_wpre
    }
    for (int o = 32; o > 0; o >>= 1) pred |= __shfl_xor(pred, o);
    if (lane == 0) {
      st.n_dirty = nd;
      st.pred_regions = pred;
      bb.vs[v] = st;
      bb.n_items_v[v] = ni;
    }
  }
  // The workgroup that finishes last turns the per-variant item counts into
  // offsets (a scan over B counts) and arms the compositing work counter.
  // Every lane releases its stores before the arrival is counted; the last
  // workgroup acquires them before reading.
  __shared__ uint32_t s_last;
  __threadfence();
  __syncthreads();
  if (lane == 0) s_last = atomicAdd(bb.arrive, 1u) == gridDim.x - 1 ? 1u : 0u;
  __syncthreads();
  if (s_last) {
    __threadfence();
    uint32_t carry = 0;
    for (int base = 0; base < bb.B; base += 64) {
      const int u = base + lane;
      const uint32_t c = u < bb.B ? bb.n_items_v[u] : 0u;
      uint32_t incl = c;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= o) incl += y;
      }
      if (u < bb.B) bb.item_off[u] = carry + incl - c;
      carry += (uint32_t)__shfl((int)incl, 63);
    }
    if (lane == 0) {
      bb.item_off[bb.B] = carry;
      *bb.counter = 0u;
      *bb.arrive = 0u;   // ready for the next batch on this workspace
    }
  }
}

void launch_project(const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                    const ProjBuffers& pb, int n_cu, hipStream_t st) {
  const int64_t need = ((int64_t)s.n + 255) / 256;
  const int nd = (ras.tiles_x + 1) * (ras.tiles_y + 1);
  const bool lds = nd <= 16384;
  const unsigned blocks = (unsigned)(lds ? std::min<int64_t>(need, (int64_t)n_cu * 4) : need);
  const size_t shm = lds ? (size_t)nd * sizeof(int) : 0;
#define SG_PROJ(D)                                                                          \
  if (lds) k_project<D, true><<<blocks, 256, shm, st>>>(s, box, cam, ras, pb);            \
  else k_project<D, false><<<blocks, 256, 0, st>>>(s, box, cam, ras, pb);
  switch (s.sh_degree) {
    case 0: SG_PROJ(0) break;
    case 1: SG_PROJ(1) break;
    case 2: SG_PROJ(2) break;
    default: SG_PROJ(3) break;
  }
#undef SG_PROJ
}

void launch_variant_prep(const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                         const float4* r0, const float4* r1, const float4* r2, const uint32_t* depth,
                         const uint2* rect, const BatchBuffers& bb, hipStream_t st) {
  const int grid = std::max(bb.B, bb.prev_B);
  if (grid <= 0) return;
  switch (s.sh_degree) {
    case 0: k_variant_prep<0><<<grid, 64, 0, st>>>(s, box, cam, ras, r0, r1, r2, depth, rect, bb); break;
    case 1: k_variant_prep<1><<<grid, 64, 0, st>>>(s, box, cam, ras, r0, r1, r2, depth, rect, bb); break;
    case 2: k_variant_prep<2><<<grid, 64, 0, st>>>(s, box, cam, ras, r0, r1, r2, depth, rect, bb); break;
    default: k_variant_prep<3><<<grid, 64, 0, st>>>(s, box, cam, ras, r0, r1, r2, depth, rect, bb); break;
  }
}


}  // namespace sg
