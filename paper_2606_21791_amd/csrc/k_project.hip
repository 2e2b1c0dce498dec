// Projection of every primitive (full renders) and of the corrupted
// primitives of each variant (incremental renders), plus the planning of the
// dirty-tile work items of a batch.
#include "sg_device.h"
#include "sg_kernels.h"

namespace sg {

// One thread per primitive.  Coalesced: field f, component c of primitives
// i .. i+63 are consecutive words in the component-major layout.
__global__ void __launch_bounds__(256) k_project(DevScene s, DevBox box, DevCam cam, DevRaster ras, ProjBuffers pb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  uint32_t clamps = 0;
  bool nonfin = false;
  if (i < s.n) {
    auto get = [&](int f, int c) -> uint32_t {
      uint32_t w = load_word(s, f, i, c);
      if ((box.mask >> f) & 1u) {
        uint32_t lo, hi;
        bool cl;
        box_words(box, f, i, c, s.n, &lo, &hi);
        w = clamp_word(w, lo, hi, s.dtype, &cl);
      }
      return w;
    };
    if (box.mask) {
      for (int f = 0; f < 6; ++f) {
        if (!((box.mask >> f) & 1u)) continue;
        for (int c = 0; c < s.ncomp[f]; ++c) {
          uint32_t lo, hi;
          bool cl;
          box_words(box, f, i, c, s.n, &lo, &hi);
          clamp_word(load_word(s, f, i, c), lo, hi, s.dtype, &cl);
          clamps += cl ? 1u : 0u;
        }
      }
    }
    const ProjOut o = project_prim(get, s.dtype, s.sh_degree, cam, ras);
    nonfin = o.nonfinite;
    pb.r0[i] = o.rec.r0;
    pb.r1[i] = o.rec.r1;
    pb.r2[i] = o.rec.r2;
    pb.depth[i] = o.depth;
    pb.rect[i] = o.visible ? make_uint2(o.rect0, o.rect1) : make_uint2(0xffffffffu, 0u);
    if (o.visible) {
      const int X = ras.tiles_x + 1;
      const int tx0 = o.rect0 & 0xffff, ty0 = o.rect0 >> 16, tx1 = o.rect1 & 0xffff, ty1 = o.rect1 >> 16;
      atomicAdd(pb.diff + ty0 * X + tx0, 1);
      atomicAdd(pb.diff + ty0 * X + tx1 + 1, -1);
      atomicAdd(pb.diff + (ty1 + 1) * X + tx0, -1);
      atomicAdd(pb.diff + (ty1 + 1) * X + tx1 + 1, 1);
    }
  }
  for (int o = 32; o > 0; o >>= 1) clamps += (uint32_t)__shfl_xor((int)clamps, o);
  const unsigned long long nf = __ballot(nonfin);
  if ((threadIdx.x & 63) == 0) {
    if (clamps && pb.clamps) atomicAdd(pb.clamps, (unsigned long long)clamps);
    if (nf) atomicOr(pb.flags, 1u);
  }
}

__device__ __forceinline__ void set_rect_bits(uint64_t* bm, int row_words, uint32_t r0, uint32_t r1) {
  const int tx0 = r0 & 0xffff, ty0 = r0 >> 16, tx1 = r1 & 0xffff, ty1 = r1 >> 16;
  for (int ty = ty0; ty <= ty1; ++ty) {
    for (int w = tx0 >> 6; w <= (tx1 >> 6); ++w) {
      const int a = max(tx0, w * 64) - w * 64, b = min(tx1, w * 64 + 63) - w * 64;
      const uint64_t m = (b == 63 ? ~0ull : ((1ull << (b + 1)) - 1ull)) & ~((1ull << a) - 1ull);
      bm[ty * row_words + w] |= m;
    }
  }
}

// One thread per variant: XOR the variant's sites into the words of each
// corrupted primitive, clamp (if guarded), project, and mark the tiles of the
// old and new footprints dirty.
__global__ void k_variant_prep(DevScene s, DevBox box, DevCam cam, DevRaster ras, const float4* __restrict__ r0,
                               const float4* __restrict__ r1, const float4* __restrict__ r2,
                               const uint32_t* __restrict__ depth, const uint2* __restrict__ rect, BatchBuffers bb) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= bb.B) return;
  const sg_variant var = bb.variants[v];
  const sg_site* sites = bb.sites + var.site_off;
  const bool guard = var.guard != 0 && box.mask != 0;
  VariantState st;
  st.n_touch = 0; st.full = 0; st.nonfinite = 0; st.n_dirty = 0; st.clamps = 0; st.item_off = 0; st._pad = 0;
  for (uint32_t k = 0; k < var.n_sites; ++k) {
    const uint32_t p = sites[k].prim;
    bool seen = false;
    for (uint32_t j = 0; j < st.n_touch; ++j) seen |= st.touch[j].prim == p;
    if (!seen) {
      if (st.n_touch == kMaxTouch) { st.full = 1; break; }
      st.touch[st.n_touch++].prim = p;
    }
  }
  uint64_t* bm = bb.bitmap + (int64_t)v * bb.bm_words;
  for (int w = 0; w < bb.bm_words; ++w) bm[w] = 0ull;
  if (!st.full) {
    for (uint32_t j = 0; j < st.n_touch; ++j) {
      const uint32_t p = st.touch[j].prim;
      auto raw = [&](int f, int c) -> uint32_t {
        uint32_t w = load_word(s, f, p, c);
        for (uint32_t k = 0; k < var.n_sites; ++k) {
          const sg_site x = sites[k];
          if (x.prim == p && x.field == f && x.comp == c) w ^= 1u << x.bit;
        }
        return w;
      };
      auto get = [&](int f, int c) -> uint32_t {
        uint32_t w = raw(f, c);
        if (guard && ((box.mask >> f) & 1u)) {
          uint32_t lo, hi;
          bool cl;
          box_words(box, f, p, c, s.n, &lo, &hi);
          w = clamp_word(w, lo, hi, s.dtype, &cl);
        }
        return w;
      };
      if (guard) {
        for (int f = 0; f < 6; ++f) {
          if (!((box.mask >> f) & 1u)) continue;
          for (int c = 0; c < s.ncomp[f]; ++c) {
            uint32_t lo, hi;
            bool cl;
            box_words(box, f, p, c, s.n, &lo, &hi);
            clamp_word(raw(f, c), lo, hi, s.dtype, &cl);
            st.clamps += cl ? 1u : 0u;
          }
        }
      }
      const ProjOut o = project_prim(get, s.dtype, s.sh_degree, cam, ras);
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
      if (!same) {
        if (old_vis) set_rect_bits(bm, bb.row_words, orc.x, orc.y);
        if (o.visible) set_rect_bits(bm, bb.row_words, o.rect0, o.rect1);
      }
    }
  }
  uint32_t nd = 0;
  for (int w = 0; w < bb.bm_words; ++w) nd += (uint32_t)__popcll(bm[w]);
  st.n_dirty = nd;
  bb.vs[v] = st;
  bb.n_items_v[v] = nd;
}

// Exclusive scan of dirty-tile counts over the batch (one block).
__global__ void k_plan_scan(BatchBuffers bb) {
  __shared__ uint32_t s[1024];
  uint32_t carry = 0;
  for (int base = 0; base < bb.B; base += 1024) {
    const int v = base + threadIdx.x;
    const uint32_t x = v < bb.B ? bb.n_items_v[v] : 0u;
    s[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const uint32_t y = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
      __syncthreads();
      s[threadIdx.x] += y;
      __syncthreads();
    }
    if (v < bb.B) {
      bb.item_off[v] = carry + s[threadIdx.x] - x;
      bb.vs[v].item_off = carry + s[threadIdx.x] - x;
    }
    carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *bb.n_items_total = carry;
}

// One block per variant: dirty-tile bitmap -> work items (variant, tile) in
// increasing tile order.
__global__ void k_expand(BatchBuffers bb, int tiles_x) {
  const int v = blockIdx.x;
  const uint64_t* bm = bb.bitmap + (int64_t)v * bb.bm_words;
  __shared__ uint32_t pre[1024];
  uint32_t off = bb.item_off[v];
  for (int base = 0; base < bb.bm_words; base += 1024) {
    const int w = base + threadIdx.x;
    const uint64_t word = w < bb.bm_words ? bm[w] : 0ull;
    const uint32_t c = (uint32_t)__popcll(word);
    pre[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const uint32_t y = threadIdx.x >= (unsigned)o ? pre[threadIdx.x - o] : 0u;
      __syncthreads();
      pre[threadIdx.x] += y;
      __syncthreads();
    }
    uint32_t pos = off + pre[threadIdx.x] - c;
    uint64_t m = word;
    const int row = w / bb.row_words, col0 = (w % bb.row_words) * 64;
    while (m) {
      const int b = __ffsll((long long)m) - 1;
      m &= m - 1ull;
      bb.items[pos++] = make_uint2((uint32_t)v, (uint32_t)(row * tiles_x + col0 + b));
    }
    off += pre[1023];
    __syncthreads();
  }
}

void launch_project(const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                    const ProjBuffers& pb, hipStream_t st) {
  const int64_t blocks = ((int64_t)s.n + 255) / 256;
  k_project<<<(unsigned)blocks, 256, 0, st>>>(s, box, cam, ras, pb);
}

void launch_variant_prep(const DevScene& s, const DevBox& box, const DevCam& cam, const DevRaster& ras,
                         const float4* r0, const float4* r1, const float4* r2, const uint32_t* depth,
                         const uint2* rect, const BatchBuffers& bb, hipStream_t st) {
  k_variant_prep<<<(bb.B + 63) / 64, 64, 0, st>>>(s, box, cam, ras, r0, r1, r2, depth, rect, bb);
}

void launch_plan_expand(const BatchBuffers& bb, int tiles_x, hipStream_t st) {
  k_plan_scan<<<1, 1024, 0, st>>>(bb);
  k_expand<<<bb.B, 1024, 0, st>>>(bb, tiles_x);
}

}  // namespace sg
