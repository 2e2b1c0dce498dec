// Front-to-back compositing of one tile, fused with the metric partials
// against the clean frame.
//
// One workgroup per tile (TILE x TILE threads, one pixel each).  The tile's
// list is streamed through LDS in batches of TILE*TILE records; every thread
// walks the batch for its own pixel.  A pixel stops at the first contributor
// whose transmittance would fall below t_min (that contributor is not
// blended); the workgroup leaves as soon as all its pixels have stopped.
//
// The incremental path composites the *merged* list of a (variant, tile)
// work item: the clean list with the variant's corrupted primitives removed
// and their new records inserted at their (depth, id) position.  Both paths
// run this same code per pixel, so an incrementally re-composited tile is
// bit-identical to a full render of the variant.
//
// Only the entries a pixel takes (q within the cut and alpha at least
// alpha_min) change its state or stop it, so removing or inserting an entry
// the pixel does not take leaves its walk, its stop and its colour exactly as
// they were.  A pixel is therefore unchanged, and not walked, when every
// changed entry that it takes lies behind the entry at which its clean walk
// stopped (in particular when its walk stopped before the first changed
// entry); the clean render keeps that entry's key per pixel.
//
// Resume: the merged list equals the clean list up to its first differing
// index m0.  The pixels that are walked restart from the clean render's
// checkpoint at the largest multiple of the checkpoint spacing not above m0,
// which holds the exact (C, T) state after that many entries.
//
// k_campaign_step holds, in one launch, the three stages of a campaign
// stream's pipeline on separate buffers: the work items of its next batch,
// the persistent compositing of its current batch and the metric reduction
// of its previous batch.  Its multi-view form (MV) renders every variant of
// a batch in K views of one resolution within the same launch (Def. 1
// averages the footprint over views): each stage then counts variant-views
// and takes each view's clean state from a per-view table.
#include <hip/hip_ext.h>

#include "sg_batch.h"
#include "sg_device.h"
#include "sg_kernels.h"

namespace sg {

struct MergeSpec {
  uint32_t raw_start, raw_len, mlen;
  int n_rm, n_ins;
  uint32_t rm_pos[kMaxTouch];
  uint32_t ins_mpos[kMaxTouch];
  uint32_t ins_src[kMaxTouch];   // index of the inserted entry's record in the touch records
  uint32_t m0;                   // first index at which merged and clean lists differ
  uint32_t start;                // resume index (multiple of the checkpoint spacing, <= m0)
};

// The loop's test of whether a pixel takes an entry (q within the cut and
// alpha at least alpha_min), on the same fp32 operations, with both bounds
// widened by 1e-4 relative: it may say yes where the loop says no, never the
// reverse.
__device__ __forceinline__ bool may_take(float px, float py, float4 a, float4 b, float4 c, float qc, float amin,
                                         float amax) {
  const float ex = px - a.x, ey = py - a.y;
  const float uu = fmaf(ex, a.z, fmaf(ey, a.w, -b.x));
  const float vv = fmaf(ey, a.z, fmaf(-ex, a.w, -b.y));
  const float q = fmaf(vv, vv * b.w, uu * (uu * b.z));
  const float alpha = fminf(amax, c.x * __builtin_amdgcn_exp2f(-q));
  return q <= qc * 1.0001f && alpha >= amin * 0.9999f;
}

// MODE: 0 full render, 1 full render writing the resume state, 2 merged list
// of a (variant, tile) item resumed from the clean state
enum { kFull = 0, kFullWrite = 1, kItem = 2 };


// kItem: s_ids (nullable) holds the ids of the tile's whole clean list;
// walk_in says whether the pixel can change (item_work decides) and cl*_in
// is its clean colour, read by the caller.  Returns the tile's changed-pixel
// count in thread 0 (0 elsewhere, and when part is null).
template <int TILE, int MODE>
__device__ __forceinline__ uint32_t composite_tile(const CompArgs& A, int tile, const MergeSpec* ms, const Rec* ovr,
                                                   float* img, Partial* part, float4* s_r0, float4* s_r1,
                                                   float4* s_r2, const uint32_t* s_ids = nullptr, bool walk_in = true,
                                                   float cl0_in = 0.f, float cl1_in = 0.f, float cl2_in = 0.f) {
  constexpr int BS = TILE * TILE;
  constexpr int NW = BS / 64;            // waves per tile; wave w covers an 8 x 8 pixel block
  constexpr int BPR = TILE / 8;          // blocks per tile row
  // per wave (row w at w * BS): byte offsets into the staged records of the
  // batch entries whose box touches its block, in order.  Every value ever
  // written is a valid offset, and two spare slots close the last row, so the
  // walk may read two slots past its list.
  __shared__ uint16_t s_idx[NW * BS + 2];
  __shared__ uint32_t s_cnt[NW][NW];     // [target wave][loading wave] entry counts
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int tx = tile % A.ras.tiles_x, ty = tile / A.ras.tiles_x;
  const int bx = tx * TILE + (wave % BPR) * 8, by = ty * TILE + (wave / BPR) * 8;
  const int x = bx + (lane & 7), y = by + (lane >> 3);
  const bool inside = x < A.W && y < A.H;
  const float px = (float)x + 0.5f, py = (float)y + 0.5f;
  const float amax = A.ras.amax, amin = A.ras.amin, tmin = A.ras.tmin, qc = A.ras.qcut2;

  uint32_t raw_start, mlen, start = 0;
  if (MODE == kItem) { raw_start = ms->raw_start; mlen = ms->mlen; }
  else { raw_start = A.tile_start[tile]; mlen = A.tile_cnt[tile]; }

  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  bool done = !inside;
  bool same = false;                     // pixel provably equal to the clean frame
  if (MODE == kItem && A.stop) {
    start = ms->start;
    if (inside) {
      if (!walk_in) {
        same = true;
        done = true;
      } else if (start) {
        const float4 st = A.ck[((int64_t)A.ck_off[tile] + start / A.ck_group - 1) * BS + tid];
        C0 = st.x; C1 = st.y; C2 = st.z; T = st.w;
      }
    }
  }
  uint32_t evals = done ? 0u : mlen - start;   // list entries this pixel evaluates
  uint32_t next_ck = A.ck_group;               // kFullWrite: next checkpoint index
  __shared__ uint32_t s_all[NW];         // per wave: every pixel of the wave has stopped
  for (int i = tid; i < NW * BS + 2; i += BS) s_idx[i] = 0;   // ordered before the walk by the loop's barriers
  for (uint32_t base = start; base < mlen; base += BS) {
    // leave once every pixel has stopped (the slots are rewritten only after
    // the two barriers of the compaction below)
    const bool wave_done = __all(done);   // a vote of all 64 lanes, taken outside the lane-0 branch
    if (lane == 0) s_all[wave] = wave_done ? 1u : 0u;
    __syncthreads();
    bool all_done = true;
#pragma unroll
    for (int w = 0; w < NW; ++w) all_done &= s_all[w] != 0u;
    if (all_done) break;
    const uint32_t m = base + tid;
    uint32_t mask = 0;                   // target waves whose block this entry may reach
    if (m < mlen) {
      float4 a, b, c;
      if (MODE != kItem) {
        const uint32_t id = (uint32_t)A.keys[raw_start + m];
        a = A.rec[id].r0; b = A.rec[id].r1; c = A.rec[id].r2;
      } else {
        int before = 0, hit = -1;
        for (int j = 0; j < ms->n_ins; ++j) {
          if (ms->ins_mpos[j] == m) hit = j;
          before += ms->ins_mpos[j] < m ? 1 : 0;
        }
        if (hit >= 0) {
          const Rec r = ovr[ms->ins_src[hit]];
          a = r.r0; b = r.r1; c = r.r2;
        } else {
          uint32_t raw = m - before;
          for (int k = 0; k < ms->n_rm; ++k) raw += ms->rm_pos[k] <= raw ? 1u : 0u;
          const uint32_t id = s_ids ? s_ids[raw] : (uint32_t)A.keys[raw_start + raw];
          a = A.rec[id].r0; b = A.rec[id].r1; c = A.rec[id].r2;
        }
      }
      s_r0[tid] = a; s_r1[tid] = b; s_r2[tid] = c;
      // Conservative extent of the pixels this entry can reach: the ellipse
      // q <= min(cut, 2 ln(o / alpha_min)), from its eigen-decomposition,
      // widened by 0.1% and one pixel against fp32 rounding.
      const float qe = fminf(qc, __log2f(c.x / amin));        // in the scaled units of the loop
      if (qe >= 0.f) {
        const float hl = 0.72134752f;                          // log2(e) / 2
        const float l1 = hl / b.z, l2 = hl / b.w;              // lambda_1, lambda_2
        const float qq = qe / hl;
        const float sxx = a.z * a.z * l1 + a.w * a.w * l2, syy = a.w * a.w * l1 + a.z * a.z * l2;
        const float hx = sqrtf(qq * sxx) * 1.001f + 1.f, hy = sqrtf(qq * syy) * 1.001f + 1.f;
        const float cu = a.x + (b.x * a.z - b.y * a.w), cv = a.y + (b.x * a.w + b.y * a.z);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const float x0 = (float)(tx * TILE + (w % BPR) * 8) + 0.5f, y0 = (float)(ty * TILE + (w / BPR) * 8) + 0.5f;
          const bool hit = (cu + hx >= x0) && (cu - hx <= x0 + 7.f) && (cv + hy >= y0) && (cv - hy <= y0 + 7.f);
          mask |= hit ? (1u << w) : 0u;
        }
      }
    }
    // order-preserving compaction of the batch into one entry list per wave
    unsigned long long bal[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      bal[w] = __ballot((mask >> w) & 1u);
      if (lane == 0) s_cnt[w][wave] = (uint32_t)__popcll(bal[w]);
    }
    __syncthreads();
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      if ((mask >> w) & 1u) {
        uint32_t pos = (uint32_t)__popcll(bal[w] & lt);
        for (int v = 0; v < wave; ++v) pos += s_cnt[w][v];
        s_idx[w * BS + pos] = (uint16_t)(tid * 16);
      }
    }
    uint32_t len = 0;
#pragma unroll
    for (int v = 0; v < NW; ++v) len += s_cnt[wave][v];
    len = __builtin_amdgcn_readfirstlane(len);   // the same in every lane: the walk's bounds stay scalar
    __syncthreads();
    if (!__all(done) && len) {
      // No divergent exits inside the batch: a stopped pixel is masked by
      // `done`; the wave leaves the batch once all of its lanes have stopped.
      // Two entries per iteration; while one is evaluated, the next one's
      // record and the offset of the one after it are read from LDS.
      const uint16_t* idx = s_idx + wave * BS;
      const char* r0b = reinterpret_cast<const char*>(s_r0);
      const char* r1b = reinterpret_cast<const char*>(s_r1);
      const char* r2b = reinterpret_cast<const char*>(s_r2);
      const bool was_done = done;
      uint32_t stop_off = 0;   // offset of the entry at which this pixel stopped in this batch
      auto step = [&](const float4& a, const float4& b, const float4& c, uint32_t off) {
        if (MODE == kFullWrite) {
          // the state before this entry is the state after every entry below it
          while (base + (off >> 4) >= next_ck) {
            A.ck_out[((int64_t)A.ck_off[tile] + next_ck / A.ck_group - 1) * BS + tid] = make_float4(C0, C1, C2, T);
            next_ck += A.ck_group;
          }
        }
        const float ex = px - a.x, ey = py - a.y;
        const float uu = fmaf(ex, a.z, fmaf(ey, a.w, -b.x));
        const float vv = fmaf(ey, a.z, fmaf(-ex, a.w, -b.y));
        const float q = fmaf(vv, vv * b.w, uu * (uu * b.z));
        const float alpha = fminf(amax, c.x * __builtin_amdgcn_exp2f(-q));
        // branch-free: every lane computes the update, and selects keep it
        // only where the entry contributes (the same values the branches
        // would compute)
        const bool take = q <= qc && alpha >= amin && !done;
        const float Tn = T * (1.f - alpha);
        const bool stop = take && Tn < tmin;
        const bool blend = take && !(Tn < tmin);
        const float w = alpha * T;
        C0 = blend ? fmaf(c.y, w, C0) : C0;
        C1 = blend ? fmaf(c.z, w, C1) : C1;
        C2 = blend ? fmaf(c.w, w, C2) : C2;
        T = blend ? Tn : T;
        stop_off = stop ? off : stop_off;
        done = done || stop;
      };
      uint32_t o0 = idx[0], o1 = idx[1];
      float4 a = *reinterpret_cast<const float4*>(r0b + o0), b = *reinterpret_cast<const float4*>(r1b + o0),
             c = *reinterpret_cast<const float4*>(r2b + o0);
      for (uint32_t j = 0; j < len; j += 2) {
        const uint32_t o2 = idx[j + 2];
        const float4 a1 = *reinterpret_cast<const float4*>(r0b + o1), b1 = *reinterpret_cast<const float4*>(r1b + o1),
                     c1 = *reinterpret_cast<const float4*>(r2b + o1);
        step(a, b, c, o0);
        if (j + 1 >= len) break;
        const uint32_t o3 = idx[j + 3];
        a = *reinterpret_cast<const float4*>(r0b + o2);
        b = *reinterpret_cast<const float4*>(r1b + o2);
        c = *reinterpret_cast<const float4*>(r2b + o2);
        step(a1, b1, c1, o1);
        o0 = o2;
        o1 = o3;
        if ((j & 6) == 6 && __all(done)) break;
      }
      if (done && !was_done) evals = base + (stop_off >> 4) + 1u - start;
    }
  }

  if (MODE == kFullWrite && !__all(done)) {
    // pixels that never stopped: their final state is every later checkpoint
    for (; next_ck <= mlen; next_ck += A.ck_group)
      A.ck_out[((int64_t)A.ck_off[tile] + next_ck / A.ck_group - 1) * BS + tid] = make_float4(C0, C1, C2, T);
  }

  double sse = 0.0;
  uint32_t changed = 0, nonfin = 0, my_stop = 0;
  float mx = 0.f;
  if (inside && !same) {
    const float p0 = fmaf(T, A.ras.bg[0], C0), p1 = fmaf(T, A.ras.bg[1], C1), p2 = fmaf(T, A.ras.bg[2], C2);
    nonfin = (isfinite(p0) && isfinite(p1) && isfinite(p2)) ? 0u : 1u;
    const float i0 = fminf(p0, 1.f), i1 = fminf(p1, 1.f), i2 = fminf(p2, 1.f);
    const int64_t off = ((int64_t)y * A.W + x) * 3;
    if (img) { img[off] = i0; img[off + 1] = i1; img[off + 2] = i2; }
    if (MODE == kFullWrite) {
      my_stop = nonfin ? ~0u : (done ? evals - 1u : mlen);
      A.stop_out[(int64_t)y * A.W + x] = nonfin ? kStopNonfinite : (done ? A.keys[raw_start + evals - 1u] : kStopNever);
    }
    if (A.clean) {
      const float c0 = MODE == kItem ? cl0_in : A.clean[off], c1 = MODE == kItem ? cl1_in : A.clean[off + 1],
                  c2 = MODE == kItem ? cl2_in : A.clean[off + 2];
      const double d0 = (double)i0 - (double)c0, d1 = (double)i1 - (double)c1, d2 = (double)i2 - (double)c2;
      sse = d0 * d0 + d1 * d1 + d2 * d2;
      const double dm = fmax(fabs(d0), fmax(fabs(d1), fabs(d2)));
      changed = dm > (1.0 / 255.0) ? 1u : 0u;
      mx = (float)dm;
    }
  }
  if (MODE == kFullWrite) {
    // the key at which the tile's last pixel stopped
    __shared__ uint32_t s_smax;
    if (tid == 0) s_smax = 0;
    __syncthreads();
    if (inside) atomicMax(&s_smax, my_stop);
    __syncthreads();
    if (tid == 0) A.stop_key_out[tile] = s_smax >= mlen ? ~0ull : A.keys[raw_start + s_smax];
  }
  return part ? block_reduce_partial(sse, changed, mx, nonfin, (unsigned long long)evals, part) : 0u;
}

// Full render: one workgroup per tile.  Block b of the grid serves tile
// (b % 8) * chunk + b / 8 so the tiles that one XCD (which receives every
// 8th workgroup) composites form a contiguous band of the frame whose
// primitive records share that XCD's L2.
template <int TILE, int MODE>
__global__ void __launch_bounds__(TILE * TILE) k_composite_full(CompArgs A) {
  __shared__ float4 s_r0[TILE * TILE], s_r1[TILE * TILE], s_r2[TILE * TILE];
  const int nt = A.ras.n_tiles;
  const int chunk = (nt + 7) / 8;
  const int b = blockIdx.x;
  const int tile = (b % 8) * chunk + b / 8;
  if (tile >= nt) return;
  composite_tile<TILE, MODE>(A, tile, nullptr, nullptr, A.image, A.parts ? A.parts + tile : nullptr, s_r0, s_r1, s_r2);
}

// Persistent incremental compositing: a fixed grid of workgroups pops
// (variant, tile) work items from a device counter until the batch's item
// count (known only on the device) is exhausted.  Per item, the positions of
// the corrupted primitives' old keys and new keys in the tile's sorted clean
// list (each target's lower bound) are counted over the whole list, which a
// list of at most KCAP entries brings into registers in one round of loads
// (its ids then stay in LDS for the compositing); a longer list is searched
// in two rounds: the last keys of TILE*TILE equal buckets locate each
// target's bucket, and one pass over that bucket counts the keys below the
// target.  The next item is popped, and the pixel's stop index and clean
// colour are read, while the current item's list is searched.
//
// The variant prep has already dropped every dirty tile whose last pixel
// stopped, in the clean render, before all of the tile's target keys.
// 16 x 16 tiles: registers are held to five resident workgroups per CU, the
// number their LDS allows.
// MV: the items are variant-views and each takes its view's clean state
// from views[]: view v % K of variant-view v, or view_of[v] when given.
// Their work items sit A0.ras.n_tiles apart per variant-view.
// One (variant, tile) work item, run by the whole workgroup.
//
// First, which pixels can change.  Pixel p is walked when some changed entry
// of the variant in the pixel's list (the clean record of a corrupted
// primitive, removed, or its corrupted record, inserted) is one the pixel
// takes and lies at or before the entry at which its clean walk stopped (its
// stop key: every entry when it never stopped; always walked when its clean
// colour was not finite).  Any other pixel's walk, stop and colour are exactly
// the clean ones.  The test needs only the variant's touch records and the
// pixel's stop key, loaded in one round; an item with no pixel to walk writes
// a zero partial and ends there.
//
// Otherwise the positions of the corrupted primitives' old keys and new keys
// in the tile's sorted clean list (each target's lower bound) are counted over
// the whole list, which a list of at most KCAP entries brings into registers
// in one round of loads (its ids then stay in LDS for the compositing); a
// longer list is searched in two rounds: the last keys of TILE*TILE equal
// buckets locate each target's bucket, and one pass over that bucket counts
// the keys below the target.  ent is the item record {tile, first entry of
// its clean list, its length, -}, v its variant (variant-view when MV) and
// `item` its partial's slot.  The caller separates two calls by a barrier.
// MV: the item takes its view's clean state from views[]: view v % K of
// variant-view v, or view_of[v] when given.
template <int TILE, bool MV>
__device__ __forceinline__ void item_work(const CompArgs& A0, VariantState* __restrict__ vs_all, const Rec* ovr,
                                          int64_t image_stride, int K, const ViewArgs* views,
                                          const uint16_t* view_of, uint32_t v, uint4 ent, uint32_t item) {
  constexpr int BS = TILE * TILE;
  constexpr int NW = BS / 64;
  constexpr int NT = 2 * kMaxTouch;
  constexpr int KPT = TILE == 8 ? 8 : (TILE == 16 ? 4 : 2);   // staged list keys per thread
  constexpr int KCAP = KPT * BS;
  constexpr int VSW = (int)(sizeof(VariantState) / sizeof(uint32_t));
  constexpr int BPR = TILE / 8;
  constexpr int RQ = 3 * kRecSlots;        // float4 words of a variant's touch records
  static_assert(sizeof(Rec) == 3 * sizeof(float4) && RQ <= BS, "touch records: one float4 per thread");
  __shared__ float4 s_r0[BS], s_r1[BS], s_r2[BS];
  __shared__ MergeSpec ms;
  __shared__ __align__(8) uint32_t s_vs[VSW];   // the item's VariantState
  __shared__ uint32_t s_ids[KCAP];      // ids of a staged clean list
  __shared__ uint64_t s_tgt[NT];        // removal keys, then insertion keys (sorted)
  __shared__ uint32_t s_cnt[NT], s_fnd[NT], s_bkt[NT];
  __shared__ int s_nr, s_ni;
  __shared__ uint32_t s_walk[NW];       // per wave: a pixel of its block is walked
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pxo = (wave % BPR) * 8 + (lane & 7), pyo = (wave / BPR) * 8 + (lane >> 3);   // as in composite_tile
  CompArgs Am;   // MV: A0 with the clean state of the item's view
  if constexpr (MV) {
    const uint32_t view = view_of ? (uint32_t)view_of[v] : v % (uint32_t)K;
    const ViewArgs& w = views[view];
    Am = A0;
    Am.rec = w.rec;
    Am.tile_start = w.tile_start; Am.tile_cnt = w.tile_cnt; Am.keys = w.keys;
    Am.clean = w.clean; Am.stop = w.stop; Am.ck = w.ck; Am.ck_off = w.ck_off; Am.stop_key = w.stop_key;
    Am.ras = w.ras; Am.W = w.W; Am.H = w.H; Am.ck_group = w.ck_group;
  }
  const CompArgs& A = MV ? Am : A0;
  // Round 1, every load issued before any is waited for (branch-free, from
  // clamped addresses; a lane with nothing to read reads a valid address of
  // the same buffer or the variant's state, and drops the value): the variant
  // state, the variant's touch records (float4 word tid of its kRecSlots
  // records, staged where composite_tile's first list batch later goes: slot
  // j in s_r0/s_r1/s_r2[j]) and the pixel's stop key.
  constexpr int VPT = (VSW + BS - 1) / BS;   // variant-state words per thread
  const uint32_t* vsrc = reinterpret_cast<const uint32_t*>(vs_all + v);
  uint32_t vw[VPT];
#pragma unroll
  for (int k = 0; k < VPT; ++k) vw[k] = vsrc[min(tid + k * BS, VSW - 1)];
  const int tile = (int)ent.x;
  const uint32_t raw_start = ent.y, L = ent.z;
  const int tx = tile % A.ras.tiles_x, ty = tile / A.ras.tiles_x;
  const int x = tx * TILE + pxo, y = ty * TILE + pyo;
  const bool inside = x < A.W && y < A.H;
  const int64_t p = (int64_t)min(y, A.H - 1) * A.W + min(x, A.W - 1);
  const bool resume = A.stop != nullptr;
  const uint64_t pk_w = *(resume ? A.stop + p : reinterpret_cast<const uint64_t*>(vsrc));
  const bool rl = resume && tid < RQ;
  const float4* rbase = reinterpret_cast<const float4*>(ovr);
  const float4 rw = *(rl ? rbase + (int64_t)v * RQ + tid : rbase);
#pragma unroll
  for (int k = 0; k < VPT; ++k)
    if (tid + k * BS < VSW) s_vs[tid + k * BS] = vw[k];
  if (rl) {
    const int slot = tid / 3, comp = tid - 3 * (tid / 3);
    (comp == 0 ? s_r0 : comp == 1 ? s_r1 : s_r2)[slot] = rw;
  }
  if (tid < NT) { s_cnt[tid] = 0; s_fnd[tid] = 0; s_bkt[tid] = 0; }
  __syncthreads();
  const VariantState& vs = *reinterpret_cast<const VariantState*>(s_vs);
  bool walk = inside;
  if (resume && inside) {
    const uint64_t pk = pk_w;
    walk = pk == kStopNonfinite;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const float qc = A.ras.qcut2, amin = A.ras.amin, amax = A.ras.amax;
    const uint32_t n_touch = min(vs.n_touch, (uint32_t)kMaxTouch);
    for (uint32_t j = 0; j < n_touch; ++j) {
      const Touch& t = vs.touch[j];
      if (t.flags & 4u) continue;   // unchanged primitive
      const int so = kMaxTouch + (int)j, sn = (int)j;
      if ((t.flags & 1u) && ((((uint64_t)t.old_depth << 32) | t.prim) <= pk) &&
          may_take(px, py, s_r0[so], s_r1[so], s_r2[so], qc, amin, amax))
        walk = true;
      if ((t.flags & 2u) && ((((uint64_t)t.new_depth << 32) | t.prim) <= pk) &&
          may_take(px, py, s_r0[sn], s_r1[sn], s_r2[sn], qc, amin, amax))
        walk = true;
    }
  }
  const bool wave_walk = __ballot(walk) != 0ull;
  if (lane == 0) s_walk[wave] = wave_walk ? 1u : 0u;
  if (tid == 0) {
    int nr = 0, ni = 0;
    // removal keys fill s_tgt from the front, insertion keys from the back
    for (uint32_t j = 0; j < vs.n_touch; ++j) {
      const Touch t = vs.touch[j];
      if (t.flags & 4u) continue;   // unchanged primitive
      if ((t.flags & 1u) && rect_has(t.old_rect0, t.old_rect1, tx, ty)) s_tgt[nr++] = ((uint64_t)t.old_depth << 32) | t.prim;
      if ((t.flags & 2u) && rect_has(t.new_rect0, t.new_rect1, tx, ty)) {
        s_tgt[NT - 1 - ni] = ((uint64_t)t.new_depth << 32) | t.prim;
        ms.ins_src[ni] = v * kRecSlots + j;
        ++ni;
      }
    }
    // move the insertion keys behind the removals, sorted by key
    for (int j = 0; j < ni; ++j) s_tgt[nr + j] = s_tgt[NT - 1 - j];
    for (int a = 1; a < ni; ++a)
      for (int b = a; b > 0 && s_tgt[nr + b - 1] > s_tgt[nr + b]; --b) {
        const uint64_t k = s_tgt[nr + b]; s_tgt[nr + b] = s_tgt[nr + b - 1]; s_tgt[nr + b - 1] = k;
        const uint32_t z = ms.ins_src[b]; ms.ins_src[b] = ms.ins_src[b - 1]; ms.ins_src[b - 1] = z;
      }
    s_nr = nr;
    s_ni = ni;
  }
  __syncthreads();
  const int nr = __builtin_amdgcn_readfirstlane(s_nr), nt = nr + __builtin_amdgcn_readfirstlane(s_ni);
  bool any_walk = false;
#pragma unroll
  for (int w = 0; w < NW; ++w) any_walk |= s_walk[w] != 0u;
  if (nt == 0 || !any_walk) {   // the variant changes no pixel of this tile
    if (tid == 0) {
      Partial z;
      z.sse = 0.0; z.evals = 0; z.changed = 0; z.max_abs = 0.f; z.nonfinite = 0; z._pad = 0;
      A.parts[item] = z;
    }
    return;
  }
  // Round 2: the clean list (a staged one into registers) and the clean
  // colour of the pixels that are walked.
  const bool staged = L <= (uint32_t)KCAP;
  const uint64_t* keys = A.keys + raw_start;
  uint64_t kr[KPT];
#pragma unroll
  for (int k = 0; k < KPT; ++k) {
    const uint32_t m = (uint32_t)(tid + k * BS);
    const bool have = staged && m < L;
    const uint64_t kv = *(have ? keys + m : reinterpret_cast<const uint64_t*>(vsrc));
    kr[k] = have ? kv : ~0ull;   // padding compares above every key
  }
  const bool use_cl = walk && A.clean;
  const float* csrc = use_cl ? A.clean + 3 * p : reinterpret_cast<const float*>(vsrc);
  const float cw0 = csrc[0], cw1 = csrc[1], cw2 = csrc[2];
  const float cl0 = use_cl ? cw0 : 0.f, cl1 = use_cl ? cw1 : 0.f, cl2 = use_cl ? cw2 : 0.f;
  const uint32_t G = (L + BS - 1) / BS;   // bucket width of a long list
  if (staged) {
#pragma unroll
    for (int k = 0; k < KPT; ++k) {
      const uint32_t m = (uint32_t)(tid + k * BS);
      if (m < L) s_ids[m] = (uint32_t)kr[k];
    }
    for (int j = 0; j < nt; ++j) {
      const uint64_t tgt = s_tgt[j];
      uint32_t c = 0;
      bool eq = false;
#pragma unroll
      for (int k = 0; k < KPT; ++k) {
        c += kr[k] < tgt ? 1u : 0u;
        eq |= kr[k] == tgt;
      }
      for (int o = 32; o > 0; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o);
      const unsigned long long me = __ballot(eq);
      if (lane == 0) {
        if (c) atomicAdd(&s_cnt[j], c);
        if (me) atomicOr(&s_fnd[j], 1u);
      }
    }
  } else {
    // round 1: a target's bucket is the number of buckets whose last key is below it
    uint64_t last = ~0ull;
    if (tid * G < L) last = keys[min(L, (tid + 1) * G) - 1];
    for (int j = 0; j < nt; ++j) {
      const unsigned long long m = __ballot(last < s_tgt[j]);
      if (lane == 0 && m) atomicAdd(&s_bkt[j], (uint32_t)__popcll(m));
    }
    __syncthreads();
    // round 2: keys below the target inside its bucket, and whether it is present
    for (int j = 0; j < nt; ++j) {
      const uint64_t tgt = s_tgt[j];
      const uint32_t b0 = s_bkt[j] * G, b1 = min(L, b0 + G);
      uint32_t c = 0;
      bool eq = false;
      for (uint32_t m = b0 + tid; m < b1; m += BS) {
        const uint64_t key = keys[m];
        c += key < tgt ? 1u : 0u;
        eq |= key == tgt;
      }
      for (int o = 32; o > 0; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o);
      const unsigned long long me = __ballot(eq);
      if (lane == 0) {
        if (c) atomicAdd(&s_cnt[j], c);
        if (me) atomicOr(&s_fnd[j], 1u);
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    // lower bound of target j: the keys below it in its bucket plus the
    // buckets before it (no buckets for a staged list)
    int n_rm = 0;
    for (int j = 0; j < nr; ++j)
      if (s_fnd[j]) ms.rm_pos[n_rm++] = s_cnt[j] + min(s_bkt[j] * G, L);
    for (int a = 1; a < n_rm; ++a)
      for (int b = a; b > 0 && ms.rm_pos[b - 1] > ms.rm_pos[b]; --b) {
        const uint32_t z = ms.rm_pos[b]; ms.rm_pos[b] = ms.rm_pos[b - 1]; ms.rm_pos[b - 1] = z;
      }
    const int ni = nt - nr;
    for (int j = 0; j < ni; ++j) {
      const uint32_t praw = s_cnt[nr + j] + min(s_bkt[nr + j] * G, L);
      uint32_t rm_before = 0;
      for (int k = 0; k < n_rm; ++k) rm_before += ms.rm_pos[k] < praw ? 1u : 0u;
      ms.ins_mpos[j] = praw - rm_before + (uint32_t)j;
    }
    ms.raw_start = raw_start;
    ms.raw_len = L;
    ms.n_rm = n_rm;
    ms.n_ins = ni;
    ms.mlen = L - (uint32_t)n_rm + (uint32_t)ni;
    uint32_t m0 = L;
    if (n_rm) m0 = min(m0, ms.rm_pos[0]);
    if (ni) m0 = min(m0, ms.ins_mpos[0]);
    ms.m0 = m0;
    ms.start = A.ck_group ? (m0 / A.ck_group) * A.ck_group : 0u;
  }
  __syncthreads();
  float* img = A.image ? A.image + (int64_t)v * image_stride : nullptr;
  const uint32_t changed = composite_tile<TILE, kItem>(A, tile, &ms, ovr, img, A.parts + item, s_r0, s_r1, s_r2,
                                                       staged ? s_ids : nullptr, walk, cl0, cl1, cl2);
  if (tid == 0 && changed)
    atomicOr((unsigned long long*)&vs_all[v].rend_regions,
             (unsigned long long)region_bit(tx, ty, A.ras.tiles_x, A.ras.tiles_y));
}

// Persistent incremental compositing of one batch: a fixed grid of
// workgroups pops (variant, tile) work items from a device counter until the
// batch's item count (known only on the device) is exhausted.  Variant v's
// items sit at [v * n_tiles, ...) and its first item index is item_off[v].
// Each workgroup keeps two items ahead: while item i runs, wave 0 locates
// item i + 1 (popped during item i - 1) in the offsets and loads its record,
// and item i + 2 is popped, so an item starts with its variant, tile and list
// range in hand.  (A batch holds a few hundred items over as many
// workgroups, so one pop per item keeps the counter far from its limit.)
//
// The work-item listing has already dropped every dirty tile that no changed
// record reaches and every one whose last pixel stopped, in the clean
// render, before all of the keys of the changes that reach it.
// 16 x 16 tiles: registers are held to five resident workgroups per CU, the
// number their LDS allows.
// MV: the items are variant-views (see item_work); their work items sit
// A0.ras.n_tiles apart per variant-view.
template <int TILE, bool MV = false>
__device__ __forceinline__ void items_role(const CompArgs& A0, const ItemArgs& I, int K = 1,
                                           const ViewArgs* views = nullptr, const uint16_t* view_of = nullptr) {
  constexpr int BS = TILE * TILE;
  __shared__ uint32_t s_cur, s_nxt, s_v;
  __shared__ uint4 s_rec;
  // the variants' first items (B + 1 offsets; B <= kMaxBatch)
  __shared__ uint32_t off[kMaxBatch + 1];
  const int tid = threadIdx.x, lane = tid & 63;
  for (int k = tid; k <= I.B; k += BS) off[k] = I.item_off[k];
  __syncthreads();
  const uint32_t total = off[I.B];
  // Wave 0 only: the variant of item `it` (the largest v with off[v] <= it,
  // counted over the offsets 64 at a time) and the item's record.
  auto locate = [&](uint32_t it, uint32_t* v_out, uint4* rec_out) {
    uint32_t cnt = 0;
    for (int base = 0; base < I.B; base += 64) {
      const int k = base + lane;
      cnt += (uint32_t)__popcll(__ballot(k < I.B && off[k] <= it));
    }
    const uint32_t v = cnt - 1u;
    *v_out = v;
    *rec_out = lane == 0 ? I.items[(int64_t)v * A0.ras.n_tiles + (it - off[v])] : make_uint4(0u, 0u, 0u, 0u);
  };
  if (tid < 64) {
    uint32_t a = 0;
    if (lane == 0) a = atomicAdd(I.counter, 1u);
    a = (uint32_t)__shfl((int)a, 0);
    uint32_t v = 0;
    uint4 rec = make_uint4(0u, 0u, 0u, 0u);
    if (a < total) locate(a, &v, &rec);
    if (lane == 0) {
      s_cur = a;
      s_v = v;
      s_rec = rec;
      s_nxt = atomicAdd(I.counter, 1u);
    }
  }
  __syncthreads();
  for (;;) {
    // item, variant and tile are uniform over the workgroup: keep them scalar
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_cur);
    if (item >= total) break;
    const uint32_t nxt = __builtin_amdgcn_readfirstlane(s_nxt);
    const uint32_t v = __builtin_amdgcn_readfirstlane(s_v);
    const uint4 ent = make_uint4(__builtin_amdgcn_readfirstlane(s_rec.x), __builtin_amdgcn_readfirstlane(s_rec.y),
                                 __builtin_amdgcn_readfirstlane(s_rec.z), __builtin_amdgcn_readfirstlane(s_rec.w));
    uint32_t v_n = 0, nxt2 = 0;
    uint4 rec_n = make_uint4(0u, 0u, 0u, 0u);
    if (tid < 64) {
      if (nxt < total) locate(nxt, &v_n, &rec_n);
      if (lane == 0) nxt2 = atomicAdd(I.counter, 1u);
    }
    item_work<TILE, MV>(A0, I.vs, I.ovr, I.image_stride, K, views, view_of, v, ent, item);
    if (tid == 0) {
      s_cur = nxt;
      s_v = v_n;
      s_rec = rec_n;
      s_nxt = nxt2;
    }
    __syncthreads();
  }
}

// Campaign-wide persistent compositing: the work items of a whole campaign
// chunk (every variant's dirty tiles, compact, each record tagged with its
// variant) in one launch.  ctl[0] holds the item count, ctl[1] the work
// counter.  A workgroup claims kPersistGroup consecutive items at a time:
// increments of one counter are serialized by the device (about 13 ns each
// here), which at one per item would bound the launch by the counter.  It
// keeps its next group claimed ahead and the next item's record loaded
// while an item runs, so an item starts with its record, and therefore its
// variant, tile and list range, already in hand.  Groups are claimed in
// increasing order, so a workgroup that meets an index at or past the count
// holds no claim below it.
constexpr uint32_t kPersistGroup = 4;
template <int TILE, bool MV>
__device__ __forceinline__ void persistent_role(const PersistArgs& P) {
  __shared__ uint32_t s_cur, s_end, s_nbase;
  __shared__ uint4 s_rec;
  const int tid = threadIdx.x;
  const uint32_t total = P.ctl[0];
  if (tid == 0) {
    const uint32_t a = atomicAdd(P.ctl + 1, kPersistGroup);
    s_cur = a;
    s_end = a + kPersistGroup;
    s_rec = a < total ? P.items[a] : make_uint4(0u, 0u, 0u, 0u);
    s_nbase = atomicAdd(P.ctl + 1, kPersistGroup);
  }
  __syncthreads();
  for (;;) {
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_cur);
    if (item >= total) break;
    const uint32_t end = __builtin_amdgcn_readfirstlane(s_end), nbase = __builtin_amdgcn_readfirstlane(s_nbase);
    const uint4 ent = make_uint4(__builtin_amdgcn_readfirstlane(s_rec.x), __builtin_amdgcn_readfirstlane(s_rec.y),
                                 __builtin_amdgcn_readfirstlane(s_rec.z), __builtin_amdgcn_readfirstlane(s_rec.w));
    // the next item: the next one of this group, else the first of the group claimed ahead
    const bool in_group = item + 1u < end;
    const uint32_t nxt = in_group ? item + 1u : nbase;
    uint4 rec_n = make_uint4(0u, 0u, 0u, 0u);
    uint32_t nbase_n = nbase;
    if (tid == 0) {
      if (nxt < total) rec_n = P.items[nxt];
      if (!in_group) nbase_n = atomicAdd(P.ctl + 1, kPersistGroup);
    }
    item_work<TILE, MV>(P.A, P.vs, P.ovr, 0, P.K, P.views, P.view_of, ent.w, ent, item);
    if (tid == 0) {
      s_cur = nxt;
      s_end = in_group ? end : nbase + kPersistGroup;
      s_rec = rec_n;
      s_nbase = nbase_n;
    }
    __syncthreads();
  }
}

template <int TILE>
__global__ void __launch_bounds__(TILE * TILE, TILE == 16 ? 5 : 1) k_composite_items(CompArgs A, ItemArgs I) {
  items_role<TILE>(A, I);
}

// The work items of variant v of a campaign's next batch (variant-view v
// when MV), by the calling wave alone (slot: its LDS copy of the state).
template <bool MV>
__device__ __forceinline__ void tiles_role(const StepArgs& S, int v, VariantState& slot) {
  constexpr int VSW = (int)(sizeof(VariantState) / sizeof(uint32_t));
  const int lane = threadIdx.x & 63;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(S.t_vs + v);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&slot);
  for (int k = lane; k < VSW; k += 64) dst[k] = src[k];
  wave_sync();
  uint32_t nd, ni;
  uint64_t pred;
  const uint64_t* stop_key = S.stop_key;
  const uint32_t* tile_start = S.tile_start;
  const uint32_t* tile_cnt = S.tile_cnt;
  int tiles_x = S.tiles_x, tiles_y = S.tiles_y;
  ReachArgs ra{S.t_ovr ? S.t_ovr + (int64_t)v * kRecSlots : nullptr, S.A.ras.tile, S.A.W, S.A.H, S.A.ras.qcut2,
               S.A.ras.amin};
  if constexpr (MV) {
    const ViewArgs& w = S.views[S.t_view_of ? (int)S.t_view_of[v] : v % S.K];
    stop_key = w.stop_key;
    tile_start = w.tile_start;
    tile_cnt = w.tile_cnt;
    tiles_x = w.ras.tiles_x;
    tiles_y = w.ras.tiles_y;
    ra.tile = w.ras.tile;
    ra.W = w.W;
    ra.H = w.H;
    ra.qc = w.ras.qcut2;
    ra.amin = w.ras.amin;
  }
  enumerate_items(slot.touch, slot.n_touch, tiles_x, tiles_y, stop_key, tile_start, tile_cnt, ra,
                  S.t_items + (int64_t)v * S.n_tiles, &nd, &ni, &pred);
  if (lane == 0) {
    S.t_vs[v].n_dirty = nd;
    S.t_vs[v].pred_regions = pred;
    S.t_n_items[v] = ni;
  }
  finish_batch(S.t_arrive, (uint32_t)S.tB, S.t_n_items, S.t_item_off, S.tB, S.t_counter);
}

// Workgroups [0, ceil(tB / waves)): work items of the next batch, a variant
// (variant-view when MV) per wave; then ceil(rB / waves) workgroups reducing
// the previous batch's metrics, one per wave; then the persistent
// compositing of the current batch.  The waves of the first two roles work
// alone (no barrier).
template <int TILE, bool MV>
__global__ void __launch_bounds__(TILE * TILE, TILE == 16 ? 5 : 1) k_campaign_step(StepArgs S) {
  constexpr int NW = TILE * TILE / 64;
  const int nt = (S.tB + NW - 1) / NW, nr = (S.rB + NW - 1) / NW;
  const int b = blockIdx.x, wave = (int)(threadIdx.x >> 6);
  if (b < nt) {
    __shared__ VariantState s_tv[NW];
    const int v = b * NW + wave;
    if (v < S.tB) tiles_role<MV>(S, v, s_tv[wave]);
    return;
  }
  if (b < nt + nr) {
    const int v = (b - nt) * NW + wave;
    if (v < S.rB) {
      uint32_t n_pixels = S.n_pixels;
      if constexpr (MV) {
        const ViewArgs& w = S.views[S.r_view_of ? (int)S.r_view_of[v] : v % S.K];
        n_pixels = (uint32_t)(w.W * w.H);
      }
      reduce_batch_variant(S.r_parts, S.r_item_off, S.r_n_items, S.r_vs, n_pixels, v, S.r_out);
    }
    return;
  }
  items_role<TILE, MV>(S.A, S.I, S.K, S.views, S.i_view_of);
}

void launch_campaign_step(const StepArgs& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const int nw = a.A.ras.tile * a.A.ras.tile / 64;
  const int grid = (a.tB + nw - 1) / nw + (a.rB + nw - 1) / nw + (a.I.B > 0 ? a.I.grid : 0);
  if (grid <= 0) return;
  if (a.views) {
    switch (a.A.ras.tile) {
      case 8: hipExtLaunchKernelGGL(k_campaign_step<8, true>, dim3(grid), dim3(64), 0, st, e0, e1, 0, a); break;
      case 32: hipExtLaunchKernelGGL(k_campaign_step<32, true>, dim3(grid), dim3(1024), 0, st, e0, e1, 0, a); break;
      default: hipExtLaunchKernelGGL(k_campaign_step<16, true>, dim3(grid), dim3(256), 0, st, e0, e1, 0, a); break;
    }
    return;
  }
  switch (a.A.ras.tile) {
    case 8: hipExtLaunchKernelGGL(k_campaign_step<8, false>, dim3(grid), dim3(64), 0, st, e0, e1, 0, a); break;
    case 32: hipExtLaunchKernelGGL(k_campaign_step<32, false>, dim3(grid), dim3(1024), 0, st, e0, e1, 0, a); break;
    default: hipExtLaunchKernelGGL(k_campaign_step<16, false>, dim3(grid), dim3(256), 0, st, e0, e1, 0, a); break;
  }
}

// The work items of a campaign chunk, one wave per variant (variant-view
// when MV): it counts its items, takes a contiguous range of the chunk's item
// array with one atomic add on the list's cursor, and lists them there in the
// order of enumerate_items, each tagged with the variant.  The order of a
// variant's items, and so its reduction, is that of the batched path.
template <bool MV>
__global__ void __launch_bounds__(256) k_persist_list(PersistArgs P) {
  constexpr int VSW = (int)(sizeof(VariantState) / sizeof(uint32_t));
  __shared__ VariantState s_v[4];
  __shared__ uint32_t s_n[4], s_base[4];
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int v = (int)blockIdx.x * 4 + wave;
  const bool have = v < P.nv;
  VariantState& slot = s_v[wave];
  const uint64_t* stop_key = P.A.stop_key;
  const uint32_t* tile_start = P.A.tile_start;
  const uint32_t* tile_cnt = P.A.tile_cnt;
  int tiles_x = P.A.ras.tiles_x, tiles_y = P.A.ras.tiles_y;
  ReachArgs ra{P.ovr + (int64_t)v * kRecSlots, P.A.ras.tile, P.A.W, P.A.H, P.A.ras.qcut2, P.A.ras.amin};
  uint32_t nd = 0, ni = 0;
  uint64_t pred = 0;
  if (have) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(P.vs + v);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&slot);
    for (int k = lane; k < VSW; k += 64) dst[k] = src[k];
    wave_sync();
    if constexpr (MV) {
      const ViewArgs& w = P.views[P.view_of ? (int)P.view_of[v] : v % P.K];
      stop_key = w.stop_key;
      tile_start = w.tile_start;
      tile_cnt = w.tile_cnt;
      tiles_x = w.ras.tiles_x;
      tiles_y = w.ras.tiles_y;
      ra.tile = w.ras.tile;
      ra.W = w.W;
      ra.H = w.H;
      ra.qc = w.ras.qcut2;
      ra.amin = w.ras.amin;
    }
    enumerate_items(slot.touch, slot.n_touch, tiles_x, tiles_y, stop_key, tile_start, tile_cnt, ra, nullptr, &nd,
                    &ni, &pred);
  }
  // one reservation per workgroup: increments of a single counter are
  // serialized by the device, so one per variant would bound the launch
  if (lane == 0) s_n[wave] = ni;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t tot = s_n[0] + s_n[1] + s_n[2] + s_n[3];
    uint32_t b = tot ? atomicAdd(P.ctl, tot) : 0u;
    for (int w = 0; w < 4; ++w) {
      s_base[w] = b;
      b += s_n[w];
    }
  }
  __syncthreads();
  if (!have) return;
  const uint32_t base = s_base[wave];
  if (ni)
    enumerate_items(slot.touch, slot.n_touch, tiles_x, tiles_y, stop_key, tile_start, tile_cnt, ra, P.items + base,
                    &nd, &ni, &pred, (uint32_t)v);
  if (lane == 0) {
    P.item_off[v] = base;
    P.n_items[v] = ni;
    P.vs[v].n_dirty = nd;
    P.vs[v].pred_regions = pred;
  }
}

// 16 x 16 tiles: registers bounded for eight resident workgroups per CU (the
// LDS allows eight; a few values spill), which outran the five that the
// unbounded build holds when the kernel was first measured (5.0 against
// 4.6 M injections/s on the headline scene).
template <int TILE, bool MV>
__global__ void __launch_bounds__(TILE * TILE, TILE == 16 ? 8 : 1) k_persist_composite(PersistArgs P) {
  persistent_role<TILE, MV>(P);
}

// Each variant's record from its items' partials, one wave per variant.
template <bool MV>
__global__ void __launch_bounds__(256) k_persist_reduce(PersistArgs P) {
  const int v = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (v >= P.nv) return;
  uint32_t n_pixels = P.n_pixels;
  if constexpr (MV) {
    const ViewArgs& w = P.views[P.view_of ? (int)P.view_of[v] : v % P.K];
    n_pixels = (uint32_t)(w.W * w.H);
  }
  reduce_batch_variant(P.A.parts, P.item_off, P.n_items, P.vs, n_pixels, v, P.out);
}

void launch_persist_list(const PersistArgs& a, hipStream_t st) {
  const int grid = (a.nv + 3) / 4;
  if (grid <= 0) return;
  if (a.views) k_persist_list<true><<<grid, 256, 0, st>>>(a);
  else k_persist_list<false><<<grid, 256, 0, st>>>(a);
}

void launch_persist_reduce(const PersistArgs& a, hipStream_t st) {
  const int grid = (a.nv + 3) / 4;
  if (grid <= 0) return;
  if (a.views) k_persist_reduce<true><<<grid, 256, 0, st>>>(a);
  else k_persist_reduce<false><<<grid, 256, 0, st>>>(a);
}

template <int TILE, bool MV>
static int occupancy_of() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist_composite<TILE, MV>, TILE * TILE, 0) != hipSuccess)
    nb = 1;
  return nb > 0 ? nb : 1;
}

int persist_occupancy(int tile, bool mv) {
  static const int occ[3][2] = {{occupancy_of<8, false>(), occupancy_of<8, true>()},
                                {occupancy_of<16, false>(), occupancy_of<16, true>()},
                                {occupancy_of<32, false>(), occupancy_of<32, true>()}};
  return occ[tile == 8 ? 0 : (tile == 32 ? 2 : 1)][mv ? 1 : 0];
}

void launch_persist_composite(const PersistArgs& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (a.grid <= 0 || a.nv <= 0) return;
  const dim3 g(a.grid);
  if (a.views) {
    switch (a.A.ras.tile) {
      case 8: hipExtLaunchKernelGGL(k_persist_composite<8, true>, g, dim3(64), 0, st, e0, e1, 0, a); break;
      case 32: hipExtLaunchKernelGGL(k_persist_composite<32, true>, g, dim3(1024), 0, st, e0, e1, 0, a); break;
      default: hipExtLaunchKernelGGL(k_persist_composite<16, true>, g, dim3(256), 0, st, e0, e1, 0, a); break;
    }
    return;
  }
  switch (a.A.ras.tile) {
    case 8: hipExtLaunchKernelGGL(k_persist_composite<8, false>, g, dim3(64), 0, st, e0, e1, 0, a); break;
    case 32: hipExtLaunchKernelGGL(k_persist_composite<32, false>, g, dim3(1024), 0, st, e0, e1, 0, a); break;
    default: hipExtLaunchKernelGGL(k_persist_composite<16, false>, g, dim3(256), 0, st, e0, e1, 0, a); break;
  }
}

void launch_composite_full(const CompArgs& a, hipStream_t st) {
  const int nt = a.ras.n_tiles;
  const int grid = ((nt + 7) / 8) * 8;
  if (a.ck_out) {
    switch (a.ras.tile) {
      case 8: k_composite_full<8, kFullWrite><<<grid, 64, 0, st>>>(a); break;
      case 32: k_composite_full<32, kFullWrite><<<grid, 1024, 0, st>>>(a); break;
      default: k_composite_full<16, kFullWrite><<<grid, 256, 0, st>>>(a); break;
    }
  } else {
    switch (a.ras.tile) {
      case 8: k_composite_full<8, kFull><<<grid, 64, 0, st>>>(a); break;
      case 32: k_composite_full<32, kFull><<<grid, 1024, 0, st>>>(a); break;
      default: k_composite_full<16, kFull><<<grid, 256, 0, st>>>(a); break;
    }
  }
}

void launch_composite_items(const CompArgs& a, const ItemArgs& it, hipStream_t st) {
  switch (a.ras.tile) {
    case 8: k_composite_items<8><<<it.grid, 64, 0, st>>>(a, it); break;
    case 32: k_composite_items<32><<<it.grid, 1024, 0, st>>>(a, it); break;
    default: k_composite_items<16><<<it.grid, 256, 0, st>>>(a, it); break;
  }
}

}  // namespace sg
