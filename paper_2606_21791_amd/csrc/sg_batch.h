// Device steps of an incremental batch shared by the variant prep kernel and
// the fused campaign step: the dirty-tile work items of a variant and the
// per-batch item offsets.  Each is run by one wave.
#pragma once

#include "sg_device.h"
#include "sg_kernels.h"

namespace sg {

// Orders this wave's memory accesses around a hand-off between its lanes
// (the wave's own barrier: no other wave of the workgroup takes part).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The dirty tiles of a variant are the union of the clean and corrupted tile
// rectangles of its changed primitives (its predicted regions).  One wave
// walks the rectangles' bounding box 64 tiles at a time in row order and
// writes a work item {tile, first entry of its clean list, clean list
// length, tag} for each dirty tile that can change.  A tile is dropped when
// no changed record reaches a pixel centre of it (ra.rec null: no such
// test), or when its last pixel stopped, in the clean render, before every
// key of a change that reaches it (stop_key nullable: none dropped).  With
// items null it only counts.  The results are the same in every lane.
__device__ __forceinline__ void enumerate_items(const Touch* touch, uint32_t n_touch, int tiles_x, int tiles_y,
                                                const uint64_t* stop_key, const uint32_t* tile_start,
                                                const uint32_t* tile_cnt, const ReachArgs& ra, uint4* items,
                                                uint32_t* n_dirty, uint32_t* n_items, uint64_t* pred,
                                                uint32_t tag = 0u) {
  const int lane = threadIdx.x & 63;
  int x0 = tiles_x, y0 = tiles_y, x1 = -1, y1 = -1;
  for (uint32_t j = 0; j < n_touch; ++j) {
    const Touch& t = touch[j];
    if (t.flags & 4u) continue;
    if (t.flags & 1u) {
      x0 = min(x0, (int)(t.old_rect0 & 0xffff)); y0 = min(y0, (int)(t.old_rect0 >> 16));
      x1 = max(x1, (int)(t.old_rect1 & 0xffff)); y1 = max(y1, (int)(t.old_rect1 >> 16));
    }
    if (t.flags & 2u) {
      x0 = min(x0, (int)(t.new_rect0 & 0xffff)); y0 = min(y0, (int)(t.new_rect0 >> 16));
      x1 = max(x1, (int)(t.new_rect1 & 0xffff)); y1 = max(y1, (int)(t.new_rect1 >> 16));
    }
  }
  uint32_t nd = 0, ni = 0;
  uint64_t pr = 0;
  if (x1 >= x0 && y1 >= y0) {
    const uint32_t bw = (uint32_t)(x1 - x0 + 1);
    const uint32_t area = bw * (uint32_t)(y1 - y0 + 1);
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (uint32_t base = 0; base < area; base += 64) {
      const uint32_t i = base + (uint32_t)lane;
      bool dirty = false, keep = false;
      uint4 ent = make_uint4(0u, 0u, 0u, 0u);
      if (i < area) {
        const int tx = x0 + (int)(i % bw), ty = y0 + (int)(i / bw);
        const unsigned long long mk = tile_min_key(touch, n_touch, tx, ty);   // all ones: not dirty
        dirty = mk != ~0ull;
        if (dirty) {
          const int t = ty * tiles_x + tx;
          pr |= region_bit(tx, ty, tiles_x, tiles_y);
          const unsigned long long mr = ra.rec ? tile_min_key_reach(touch, n_touch, ra, tx, ty) : mk;
          const unsigned long long sk = stop_key ? stop_key[t] : ~0ull;
          if (items) ent = make_uint4((uint32_t)t, tile_start[t], tile_cnt[t], tag);
          keep = mr != ~0ull && mr <= sk;
        }
      }
      nd += (uint32_t)__popcll(__ballot(dirty));
      const unsigned long long kb = __ballot(keep);
      if (keep && items) items[ni + (uint32_t)__popcll(kb & lt)] = ent;
      ni += (uint32_t)__popcll(kb);
    }
  }
  for (int o = 32; o > 0; o >>= 1) pr |= __shfl_xor(pr, o);
  *n_dirty = nd;
  *n_items = ni;
  *pred = pr;
}

// Called by one wave of each of the batch's n_groups workgroups after its
// stores.  The workgroup that arrives last turns the per-variant item counts
// into offsets (item_off, B + 1 entries), arms the compositing work counter
// and returns `arrive` to zero.  Every workgroup releases its stores before
// it is counted; the last one acquires them before reading.
__device__ __forceinline__ void finish_batch(uint32_t* arrive, uint32_t n_groups, const uint32_t* n_items_v,
                                             uint32_t* item_off, int B, uint32_t* counter) {
  const int lane = threadIdx.x & 63;
  __threadfence();
  uint32_t last = 0;
  if (lane == 0) last = atomicAdd(arrive, 1u) == n_groups - 1 ? 1u : 0u;
  last = (uint32_t)__shfl((int)last, 0);
  if (!last) return;
  __threadfence();
  uint32_t carry = 0;
  for (int base = 0; base < B; base += 64) {
    const int u = base + lane;
    const uint32_t c = u < B ? n_items_v[u] : 0u;
    uint32_t incl = c;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
      if (lane >= o) incl += y;
    }
    if (u < B) item_off[u] = carry + incl - c;
    carry += (uint32_t)__shfl((int)incl, 63);
  }
  if (lane == 0) {
    item_off[B] = carry;
    *counter = 0u;
    *arrive = 0u;   // ready for the next batch on these buffers
  }
}

}  // namespace sg
