// Tile binning and the per-tile depth sort.
//
// Every visible primitive adds 1 to each tile of its rectangle; the counts
// come from a 2-D difference grid (four atomics per primitive in k_project)
// and two prefix passes.  Instances are scattered into their tile's segment
// with one atomic cursor per tile, as the 64-bit key (fp32 depth bits << 32 |
// primitive id), which is unique; each segment is then sorted by that key, so
// the final order is (depth, id) whatever order the scatter produced.
#include "sg_device.h"
#include "sg_kernels.h"

#include <algorithm>

namespace sg {

constexpr int kSortCap = 4096;       // lists up to this long are sorted in LDS by one block
constexpr int kChunkKeys = 4096;     // longer lists are cut into chunks of this many keys, each sorted by one block
constexpr int kMergeTile = 2048;     // outputs of one block in a merge pass
constexpr int kMergeThreads = kMergeTile / 8;   // 8 outputs per thread
constexpr int kEmitSmall = 32;       // rectangles up to this many tiles are emitted by one thread

constexpr int kPrefixLds = 12288;   // difference-grid entries prefix-summed in LDS (48 KB)

// Inclusive scans of up to three values per thread over the block (1,024
// threads: wave scans by shuffles, then the wave totals), with two barriers.
// tot receives the block totals.
template <int NV>
__device__ __forceinline__ void block_scan(uint32_t (&v)[NV], uint32_t (&tot)[NV], uint32_t (*s_w)[16]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)v[q], o);
      if (lane >= o) v[q] += y;
    }
    if (lane == 63) s_w[q][wave] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    uint32_t off = 0, t = 0;
    for (int w = 0; w < nw; ++w) {
      const uint32_t x = s_w[q][w];
      off += w < wave ? x : 0u;
      t += x;
    }
    v[q] += off;
    tot[q] = t;
  }
  __syncthreads();
}

// Tile counts and list offsets from the difference grid, in one workgroup of
// 1,024 threads: the grid's row and column prefix sums (in LDS when it fits),
// then a scan of the tile counts, then the tiles whose lists exceed one LDS
// sort with the prefix counts of their LDS chunks and merge blocks.
__global__ void __launch_bounds__(1024) k_tile_prefix(DevRaster ras, BinBuffers bb) {
  const int X = ras.tiles_x + 1, Y = ras.tiles_y + 1;
  __shared__ int s_grid[kPrefixLds];
  __shared__ uint32_t s_w[3][16];
  const bool in_lds = X * Y <= kPrefixLds;
  int* grid = in_lds ? s_grid : bb.diff;
  if (in_lds) {
    for (int i = threadIdx.x; i < X * Y; i += blockDim.x) s_grid[i] = bb.diff[i];
    __syncthreads();
  }
  for (int r = threadIdx.x; r < Y; r += blockDim.x) {
    int acc = 0;
    for (int x = 0; x < X; ++x) { acc += grid[r * X + x]; grid[r * X + x] = acc; }
  }
  __syncthreads();
  for (int x = threadIdx.x; x < X; x += blockDim.x) {
    int acc = 0;
    for (int r = 0; r < Y; ++r) { acc += grid[r * X + x]; grid[r * X + x] = acc; }
  }
  __syncthreads();
  unsigned long long carry = 0;
  for (int base = 0; base < ras.n_tiles; base += 1024) {
    const int t = base + threadIdx.x;
    uint32_t c = 0;
    if (t < ras.n_tiles) {
      const int tx = t % ras.tiles_x, ty = t / ras.tiles_x;
      c = (uint32_t)grid[ty * X + tx];
      bb.tile_cnt[t] = c;
      bb.cursor[t] = 0;
    }
    uint32_t v[1] = {c}, tot[1];
    block_scan<1>(v, tot, s_w);
    if (t < ras.n_tiles) bb.tile_start[t] = (uint32_t)(carry + v[0] - c);
    carry += tot[0];
  }
  // tiles whose lists exceed one LDS sort, in tile order, with the prefix
  // counts of their LDS chunks and of their merge blocks
  unsigned long long acc0 = 0, acc1 = 0, acc2 = 0;
  uint32_t mx = 0;
  for (int base = 0; base < ras.n_tiles; base += 1024) {
    const int t = base + threadIdx.x;
    const uint32_t c = t < ras.n_tiles ? bb.tile_cnt[t] : 0u;
    const bool big = c > (uint32_t)kSortCap;
    const uint32_t nch = big ? (c + kChunkKeys - 1) / kChunkKeys : 0u, ngr = big ? (c + kMergeTile - 1) / kMergeTile : 0u;
    uint32_t v[3] = {big ? 1u : 0u, nch, ngr}, tot[3];
    block_scan<3>(v, tot, s_w);
    if (big) {
      const uint32_t k = (uint32_t)(acc0 + v[0] - 1u);
      bb.big_tiles[k] = (uint32_t)t;
      bb.big_choff[k] = (uint32_t)(acc1 + v[1] - nch);
      bb.big_goff[k] = (uint32_t)(acc2 + v[2] - ngr);
      mx = max(mx, c);
    }
    acc0 += tot[0];
    acc1 += tot[1];
    acc2 += tot[2];
  }
  // the longest big list: a block maximum
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o));
  if ((threadIdx.x & 63) == 0) s_w[0][threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = max(m, s_w[0][w]);
    const uint32_t nb = (uint32_t)acc0;
    bb.big_choff[nb] = (uint32_t)acc1;
    bb.big_goff[nb] = (uint32_t)acc2;
    bb.total[0] = carry; bb.total[1] = 0; bb.total[2] = nb; bb.total[3] = m;
    bb.total[4] = acc1; bb.total[5] = acc2;
  }
}

__device__ __forceinline__ void emit_one(const BinBuffers& bb, int t, uint64_t key) {
  const uint32_t pos = bb.tile_start[t] + atomicAdd(bb.cursor + t, 1u);
  bb.keys[pos] = key;
}

__global__ void __launch_bounds__(256) k_emit_small(int n, const uint32_t* __restrict__ depth,
                                                    const uint2* __restrict__ rect, DevRaster ras, BinBuffers bb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint2 r = rect[i];
  if (r.x == 0xffffffffu) return;
  const int tx0 = r.x & 0xffff, ty0 = r.x >> 16, tx1 = r.y & 0xffff, ty1 = r.y >> 16;
  const int area = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
  if (area > kEmitSmall) {
    const unsigned long long b = atomicAdd(bb.total + 1, 1ull);
    bb.big_prims[b] = (uint32_t)i;
    return;
  }
  const uint64_t key = ((uint64_t)depth[i] << 32) | (uint32_t)i;
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx) emit_one(bb, ty * ras.tiles_x + tx, key);
}

__global__ void __launch_bounds__(256) k_emit_big(const uint32_t* __restrict__ depth, const uint2* __restrict__ rect,
                                                  DevRaster ras, BinBuffers bb) {
  const unsigned long long nb = bb.total[1];
  for (unsigned long long b = blockIdx.x; b < nb; b += gridDim.x) {
    const uint32_t i = bb.big_prims[b];
    const uint2 r = rect[i];
    const int tx0 = r.x & 0xffff, ty0 = r.x >> 16, tx1 = r.y & 0xffff, ty1 = r.y >> 16;
    const int w = tx1 - tx0 + 1;
    const int area = w * (ty1 - ty0 + 1);
    const uint64_t key = ((uint64_t)depth[i] << 32) | i;
    for (int k = threadIdx.x; k < area; k += blockDim.x) emit_one(bb, (ty0 + k / w) * ras.tiles_x + tx0 + k % w, key);
  }
}

// Chunked emission: block b handles primitives [b*chunk, (b+1)*chunk).  It
// counts its instances per tile in LDS, reserves each tile's range with one
// global atomic, then scatters with LDS cursors.  Rectangles larger than
// kEmitSmall tiles go to the per-instance path of k_emit_big.
__global__ void __launch_bounds__(1024) k_emit_chunk(int n, int chunk, const uint32_t* __restrict__ depth,
                                                     const uint2* __restrict__ rect, DevRaster ras, BinBuffers bb) {
  extern __shared__ uint32_t s_pos[];
  const int nt = ras.n_tiles;
  for (int k = threadIdx.x; k < nt; k += blockDim.x) s_pos[k] = 0;
  __syncthreads();
  const int i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const uint2 r = rect[i];
    if (r.x == 0xffffffffu) continue;
    const int tx0 = r.x & 0xffff, ty0 = r.x >> 16, tx1 = r.y & 0xffff, ty1 = r.y >> 16;
    if ((tx1 - tx0 + 1) * (ty1 - ty0 + 1) > kEmitSmall) {
      const unsigned long long b = atomicAdd(bb.total + 1, 1ull);
      bb.big_prims[b] = (uint32_t)i;
      continue;
    }
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) atomicAdd(s_pos + ty * ras.tiles_x + tx, 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nt; t += blockDim.x) {
    const uint32_t c = s_pos[t];
    if (c) s_pos[t] = bb.tile_start[t] + atomicAdd(bb.cursor + t, c);
  }
  __syncthreads();
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const uint2 r = rect[i];
    if (r.x == 0xffffffffu) continue;
    const int tx0 = r.x & 0xffff, ty0 = r.x >> 16, tx1 = r.y & 0xffff, ty1 = r.y >> 16;
    if ((tx1 - tx0 + 1) * (ty1 - ty0 + 1) > kEmitSmall) continue;
    const uint64_t key = ((uint64_t)depth[i] << 32) | (uint32_t)i;
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) bb.keys[atomicAdd(s_pos + ty * ras.tiles_x + tx, 1u)] = key;
  }
}

// Tiles with more than kSortCap instances are sorted by the whole grid:
// every chunk of kChunkKeys keys of every such tile is sorted by one block (a
// tile's last chunk may be shorter), then runs are merged pairwise in passes
// of doubling width.  A pass first finds, for
// every kMergeTile-output block, where its outputs start in the two runs
// (merge path, one thread per block), then each block stages its inputs in
// LDS and merges them.  Passes alternate between keys and keys_tmp at the
// tile's own offset; a tile that takes an odd number of passes has its
// sorted chunks written to keys_tmp, so that every tile's last pass ends in
// keys.

// Merge passes a big tile takes: one per width kChunkKeys, 2 kChunkKeys, ...
// below its length.
__device__ __forceinline__ uint32_t merge_passes(uint32_t n) {
  uint32_t p = 0;
  for (uint64_t w = kChunkKeys; w < n; w <<= 1) ++p;
  return p;
}

// The buffer that holds a big tile's keys before merge pass p (after its
// last pass, p = merge_passes(n): keys).
__device__ __forceinline__ uint64_t* pass_buffer(const BinBuffers& bb, uint32_t n, uint32_t p) {
  return ((merge_passes(n) - p) & 1u) ? bb.keys_tmp : bb.keys;
}

// The big tile holding global item g (off has nb + 1 prefix entries).
__device__ __forceinline__ int big_of(const uint32_t* off, int nb, uint32_t g) {
  int lo = 0, hi = nb;   // largest k with off[k] <= g
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Bitonic networks over keys held kPerThread per thread in registers (thread
// t holds elements kPerThread * t + r).  Element i pairs with i ^ J in stage
// (K, J) and the pair sorts ascending when (i & K) == 0.  Partners in the same
// thread are exchanged in registers, partners in the same wave by lane
// permutes on the VALU (no LDS traffic: the LDS pipe bounds a shuffle-based
// network), and the rest through LDS (element i of a block of NT threads at
// sk[(i % kPerThread) * NT + i / kPerThread]).
constexpr int kPerThread = 8;
constexpr int kChunkThreads = kChunkKeys / kPerThread;

__device__ __forceinline__ void bitonic_pair(uint64_t& lo, uint64_t& hi, bool asc) {
  const bool sw = (lo > hi) == asc;
  const uint64_t a = lo;
  lo = sw ? hi : lo;
  hi = sw ? a : hi;
}

// DPP lane permutes of one dword (full row and bank masks: every lane is written).
template <int Ctrl>
__device__ __forceinline__ uint32_t dpp32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, Ctrl, 0xF, 0xF, true);
}

constexpr int kDppXor1 = 0xB1;          // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;          // quad_perm [2,3,0,1]
constexpr int kDppXor3 = 0x1B;          // quad_perm [3,2,1,0]
constexpr int kDppHalfMirror = 0x141;   // lane i of each group of 8 takes lane 7 - i (i ^ 7)
constexpr int kDppRowRor8 = 0x128;      // rotation by 8 within each row of 16 (i ^ 8)

// The dword of lane (lane ^ M), for M < 64, without LDS: DPP for M <= 8,
// the gfx950 row swaps for 16 and 32 (swapping a register with itself gives
// each lane its partner row's value in one of the two results).
template <int M>
__device__ __forceinline__ uint32_t lane_xor32(uint32_t x) {
  if constexpr (M == 1) {
    return dpp32<kDppXor1>(x);
  } else if constexpr (M == 2) {
    return dpp32<kDppXor2>(x);
  } else if constexpr (M == 4) {
    return dpp32<kDppXor3>(dpp32<kDppHalfMirror>(x));   // (i ^ 3) ^ 7 = i ^ 4
  } else if constexpr (M == 8) {
    return dpp32<kDppRowRor8>(x);
  } else if constexpr (M == 16) {
    // odd rows of the first operand swap with even rows of the second
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return (threadIdx.x & 16) ? r[0] : r[1];
  } else {
    static_assert(M == 32, "lane distance");
    // rows 2-3 of the first operand swap with rows 0-1 of the second
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
  }
}

template <int M>
__device__ __forceinline__ uint64_t lane_xor(uint64_t v) {
  const uint32_t lo = lane_xor32<M>((uint32_t)v), hi = lane_xor32<M>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// One stage (K, J) by a block of NT threads.  A wave whose flag live is false
// holds only padding that pairs only with padding (elements at or beyond the
// network's length), so it skips the exchanges and only takes part in the
// barriers.
template <int NT, int J>
__device__ __forceinline__ void bitonic_stage(uint64_t* sk, uint64_t (&v)[kPerThread], int K, bool live) {
  // The thread index passes through an empty asm statement so that each
  // stage forms its lane masks where it uses them: hoisted, the masks of all
  // 78 stages of the chunk sort held 106 SGPRs (with spills), three
  // workgroups per CU instead of four.
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  const int i0 = kPerThread * t;
  if constexpr (J < kPerThread) {
    if (!live) return;
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
      if ((r & J) == 0) {
        // K < kPerThread: the direction depends on r only; otherwise on the thread only
        const bool asc = K < kPerThread ? (r & K) == 0 : (i0 & K) == 0;
        bitonic_pair(v[r], v[r | J], asc);
      }
    }
  } else {
    // the thread's elements share the pair direction and their side of the pair:
    // keep own when (own < partner) agrees with take_min
    const bool take_min = ((i0 & K) == 0) == ((i0 & J) == 0);
    constexpr int M = J / kPerThread;   // partner thread t ^ M, below NT since J < length <= NT * kPerThread
    uint64_t p[kPerThread];
    if constexpr (M >= 64) {
      __syncthreads();
      if (live) {
#pragma unroll
        for (int r = 0; r < kPerThread; ++r) sk[NT * r + t] = v[r];
      }
      __syncthreads();
      if (!live) return;
#pragma unroll
      for (int r = 0; r < kPerThread; ++r) p[r] = sk[NT * r + (t ^ M)];
    } else {
      if (!live) return;
#pragma unroll
      for (int r = 0; r < kPerThread; ++r) p[r] = lane_xor<M>(v[r]);
    }
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) v[r] = (v[r] < p[r]) == take_min ? v[r] : p[r];
  }
}

// The chunk sort: kChunkKeys keys, every stage unrolled, so distances and
// offsets are constants.
template <int K, int J>
__device__ __forceinline__ void bitonic_merge_stages(uint64_t* sk, uint64_t (&v)[kPerThread]) {
  bitonic_stage<kChunkThreads, J>(sk, v, K, true);
  if constexpr (J > 1) bitonic_merge_stages<K, J / 2>(sk, v);
}

template <int K>
__device__ __forceinline__ void bitonic_from(uint64_t* sk, uint64_t (&v)[kPerThread]) {
  bitonic_merge_stages<K, K / 2>(sk, v);
  if constexpr (K < kChunkKeys) bitonic_from<2 * K>(sk, v);
}

// Tiles of up to kSortCap instances: one workgroup of NT threads sorts a
// tile's list with a network of length P (the list's length rounded up to a
// power of two) known only at run time; the waves beyond P idle.
template <int NT, int J>
__device__ __forceinline__ void bitonic_stage_if(uint64_t* sk, uint64_t (&v)[kPerThread], int K, bool live) {
  if constexpr (J < NT * kPerThread) bitonic_stage<NT, J>(sk, v, K, live);
}

template <int NT>
__device__ void bitonic_runtime(uint64_t* sk, uint64_t (&v)[kPerThread], int P) {
  const bool live = (int)(threadIdx.x & ~63u) * kPerThread < P;   // wave-uniform
  for (int K = 2; K <= P; K <<= 1) {
    for (int J = K >> 1; J > 0; J >>= 1) {
      switch (J) {
        case 1: bitonic_stage_if<NT, 1>(sk, v, K, live); break;
        case 2: bitonic_stage_if<NT, 2>(sk, v, K, live); break;
        case 4: bitonic_stage_if<NT, 4>(sk, v, K, live); break;
        case 8: bitonic_stage_if<NT, 8>(sk, v, K, live); break;
        case 16: bitonic_stage_if<NT, 16>(sk, v, K, live); break;
        case 32: bitonic_stage_if<NT, 32>(sk, v, K, live); break;
        case 64: bitonic_stage_if<NT, 64>(sk, v, K, live); break;
        case 128: bitonic_stage_if<NT, 128>(sk, v, K, live); break;
        case 256: bitonic_stage_if<NT, 256>(sk, v, K, live); break;
        case 512: bitonic_stage_if<NT, 512>(sk, v, K, live); break;
        case 1024: bitonic_stage_if<NT, 1024>(sk, v, K, live); break;
        default: bitonic_stage_if<NT, 2048>(sk, v, K, live); break;
      }
    }
  }
}

// Lists of lo..hi instances (hi <= NT * kPerThread); one workgroup per tile.
template <int NT>
__global__ void __launch_bounds__(NT) k_tile_sort(BinBuffers bb, uint32_t lo, uint32_t hi) {
  const int t = blockIdx.x;
  const uint32_t n = bb.tile_cnt[t];
  if (n < lo || n > hi) return;   // another launch's lists (longer than kSortCap: the chunk sort and merges)
  __shared__ uint64_t sk[NT * kPerThread];
  int P = 2;
  while (P < (int)n) P <<= 1;
  uint64_t* g = bb.keys + bb.tile_start[t];
  const int e = kPerThread * threadIdx.x;
  uint64_t v[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) v[r] = e + r < (int)n ? g[e + r] : ~0ull;
  bitonic_runtime<NT>(sk, v, P);
#pragma unroll
  for (int r = 0; r < kPerThread; ++r)
    if (e + r < (int)n) g[e + r] = v[r];
}

// Each merge block's and each LDS chunk's big tile and index within that
// tile (big_map: merge blocks first, then chunks), found once per sort by
// binary searches over the prefix counts, so that the chunk sort and every
// merge pass begin with two dependent loads instead of a search.
__global__ void __launch_bounds__(256) k_big_map(BinBuffers bb) {
  const int nbig = (int)bb.total[2];
  const uint32_t nblk = (uint32_t)bb.total[5], nch = (uint32_t)bb.total[4];
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < nblk + nch; g += gridDim.x * blockDim.x) {
    const bool blk = g < nblk;
    const uint32_t x = blk ? g : g - nblk;
    const uint32_t* off = blk ? bb.big_goff : bb.big_choff;
    const int k = big_of(off, nbig, x);
    bb.big_map[g] = make_uint2(bb.big_tiles[k], x - off[k]);
  }
}

__global__ void __launch_bounds__(kChunkThreads) k_big_chunks(BinBuffers bb) {
  __shared__ uint64_t sk[kChunkKeys];
  const uint32_t nblk = (uint32_t)bb.total[5], nch = (uint32_t)bb.total[4];
  for (uint32_t g = blockIdx.x; g < nch; g += gridDim.x) {
    const uint2 mp = bb.big_map[nblk + g];
    const uint32_t t = mp.x;
    const int n = (int)bb.tile_cnt[t];
    const int c0 = (int)mp.y * kChunkKeys;
    const int m = min(kChunkKeys, n - c0);
    const uint64_t* a = bb.keys + bb.tile_start[t] + c0;
    uint64_t* out = pass_buffer(bb, (uint32_t)n, 0u) + bb.tile_start[t] + c0;
    const int e = kPerThread * threadIdx.x;
    uint64_t v[kPerThread];
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) v[r] = e + r < m ? a[e + r] : ~0ull;
    bitonic_from<2>(sk, v);
#pragma unroll
    for (int r = 0; r < kPerThread; ++r)
      if (e + r < m) out[e + r] = v[r];
    __syncthreads();   // the next chunk's LDS stages reuse sk
  }
}

// Position of one merge block in its tile and run pair for a pass of width w.
struct MergeBlock {
  uint32_t t, n, o0, o1, a0, na, b0, nb;
};

__device__ __forceinline__ MergeBlock merge_block(const BinBuffers& bb, uint32_t g, uint32_t w) {
  MergeBlock m;
  const uint2 mp = bb.big_map[g];
  m.t = mp.x;
  m.n = bb.tile_cnt[m.t];
  m.o0 = mp.y * (uint32_t)kMergeTile;
  m.o1 = min(m.o0 + (uint32_t)kMergeTile, m.n);
  if (m.n <= w) {   // a single run: copied
    m.a0 = 0; m.na = m.n; m.b0 = m.n; m.nb = 0;
    return m;
  }
  m.a0 = m.o0 / (2u * w) * (2u * w);
  m.na = min(w, m.n - m.a0);
  m.b0 = m.a0 + m.na;
  m.nb = m.b0 < m.n ? min(w, m.n - m.b0) : 0u;
  return m;
}

// Number of outputs before diagonal d of the merge of A (na) and B (nb) that come from A.
__device__ __forceinline__ uint32_t merge_split(const uint64_t* A, uint32_t na, const uint64_t* B, uint32_t nb,
                                                uint32_t d) {
  uint32_t lo = d > nb ? d - nb : 0u, hi = min(d, na);
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (A[mid] < B[d - 1 - mid]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Pass p merges runs of width w = kChunkKeys << p.
__global__ void __launch_bounds__(256) k_big_partition(BinBuffers bb, uint32_t w, uint32_t p) {
  const uint32_t nblk = (uint32_t)bb.total[5];
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < nblk; g += gridDim.x * blockDim.x) {
    const MergeBlock m = merge_block(bb, g, w);
    if (m.n <= w) continue;   // the tile is already one sorted run (k_big_merge skips it)
    const uint64_t* src = pass_buffer(bb, m.n, p) + bb.tile_start[m.t];
    bb.big_split[g] = m.nb ? merge_split(src + m.a0, m.na, src + m.b0, m.nb, m.o0 - m.a0) : m.o0 - m.a0;
  }
}

// Each thread merges 8 consecutive outputs into registers, keeping the next
// key of each run in a register (one LDS read per output); the block then
// writes its outputs back into the staging buffer and stores them with
// consecutive threads on consecutive keys.
__global__ void __launch_bounds__(kMergeThreads) k_big_merge(BinBuffers bb, uint32_t w, uint32_t p) {
  __shared__ uint64_t s[kMergeTile];   // the block's inputs (its part of run A, then of run B), then its outputs
  const uint32_t nblk = (uint32_t)bb.total[5];
  for (uint32_t g = blockIdx.x; g < nblk; g += gridDim.x) {
    const MergeBlock m = merge_block(bb, g, w);
    if (m.n <= w) continue;   // the tile is already one sorted run, in keys
    const uint64_t* src = pass_buffer(bb, m.n, p) + bb.tile_start[m.t];
    uint64_t* dst = pass_buffer(bb, m.n, p + 1u) + bb.tile_start[m.t];
    const uint32_t cnt = m.o1 - m.o0;
    if (m.nb == 0) {
      for (uint32_t o = threadIdx.x; o < cnt; o += blockDim.x) dst[m.o0 + o] = src[m.o0 + o];
      continue;
    }
    // this block's inputs: A[ia0, ia1) and B[ib0, ib1)
    const uint32_t ia0 = bb.big_split[g];
    const uint32_t ia1 = m.o1 == m.a0 + m.na + m.nb ? m.na : bb.big_split[g + 1];
    const uint32_t ib0 = (m.o0 - m.a0) - ia0, ib1 = (m.o1 - m.a0) - ia1;
    const uint32_t nA = ia1 - ia0, nB = ib1 - ib0;
    __syncthreads();   // the previous block's outputs have been stored
    for (uint32_t x = threadIdx.x; x < nA; x += blockDim.x) s[x] = src[m.a0 + ia0 + x];
    for (uint32_t x = threadIdx.x; x < nB; x += blockDim.x) s[nA + x] = src[m.b0 + ib0 + x];
    __syncthreads();
    const uint32_t d = 8u * threadIdx.x;   // d + 7 < kMergeTile
    uint64_t out[8];
    if (d < cnt) {
      uint32_t i = merge_split(s, nA, s + nA, nB, d), j = d - i;
      uint64_t ka = i < nA ? s[i] : 0ull, kb = j < nB ? s[nA + j] : 0ull;
#pragma unroll
      for (int q = 0; q < 8; ++q) {   // outputs past cnt are computed but not stored
        const bool take_a = j >= nB || (i < nA && ka < kb);
        out[q] = take_a ? ka : kb;
        if (take_a) {
          ++i;
          ka = i < nA ? s[i] : 0ull;
        } else {
          ++j;
          kb = j < nB ? s[nA + j] : 0ull;
        }
      }
    }
    __syncthreads();   // every thread has read its inputs
    if (d < cnt) {
#pragma unroll
      for (int q = 0; q < 8; ++q) s[d + q] = out[q];
    }
    __syncthreads();
    for (uint32_t o = threadIdx.x; o < cnt; o += blockDim.x) dst[m.o0 + o] = s[o];
  }
}

void launch_tile_prefix(const DevRaster& ras, const BinBuffers& bb, hipStream_t st) {
  k_tile_prefix<<<1, 1024, 0, st>>>(ras, bb);
}

void launch_emit(int n, const uint32_t* depth, const uint2* rect, const DevRaster& ras, const BinBuffers& bb,
                 int n_cu, hipStream_t st) {
  if (ras.n_tiles <= 16384) {
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)n + 255) / 256, (int64_t)n_cu * 4));
    const int chunk = (int)(((int64_t)n + blocks - 1) / blocks);
    k_emit_chunk<<<blocks, 1024, (size_t)ras.n_tiles * sizeof(uint32_t), st>>>(n, chunk, depth, rect, ras, bb);
  } else {
    k_emit_small<<<(n + 255) / 256, 256, 0, st>>>(n, depth, rect, ras, bb);
  }
  k_emit_big<<<1024, 256, 0, st>>>(depth, rect, ras, bb);
}

// Workgroups of k_big_chunks resident per CU: its grid-stride launch uses
// exactly that many per CU, so that all of them run in one round.
static int big_chunks_occupancy() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_big_chunks, kChunkThreads, 0) != hipSuccess) {
    (void)hipGetLastError();
    nb = 1;
  }
  return nb > 0 ? nb : 1;
}

void launch_tile_sort(const DevRaster& ras, const BinBuffers& bb, const unsigned long long* totals, int n_cu,
                      hipStream_t st) {
  // lists of 2..512 keys in one wave (no LDS), 513..2,048 in four, 2,049..kSortCap in eight
  k_tile_sort<64><<<ras.n_tiles, 64, 0, st>>>(bb, 2u, 512u);
  k_tile_sort<256><<<ras.n_tiles, 256, 0, st>>>(bb, 513u, 2048u);
  k_tile_sort<512><<<ras.n_tiles, 512, 0, st>>>(bb, 2049u, (uint32_t)kSortCap);
  if (totals[2] == 0) return;
  const unsigned long long nch = totals[4], nblk = totals[5], maxn = totals[3];
  k_big_map<<<(unsigned)std::min<unsigned long long>((nblk + nch + 255) / 256, (unsigned long long)n_cu * 8), 256, 0,
              st>>>(bb);
  static const int chunk_occ = big_chunks_occupancy();
  k_big_chunks<<<(unsigned)std::min<unsigned long long>(nch, (unsigned long long)n_cu * chunk_occ), kChunkThreads, 0,
                 st>>>(bb);
  const unsigned pgrid = (unsigned)std::max<unsigned long long>(1, (nblk + 255) / 256);
  // one workgroup per merge block (below 2^31 blocks: lists are shorter than 2^31)
  const unsigned mgrid = (unsigned)nblk;
  // Pass p merges runs of width kChunkKeys << p into runs of twice that width,
  // from one buffer into the other, for the tiles still longer than one run;
  // a tile that is already one sorted run has reached keys.
  uint32_t p = 0;
  for (unsigned long long w = kChunkKeys; w < maxn; w <<= 1, ++p) {
    k_big_partition<<<pgrid, 256, 0, st>>>(bb, (uint32_t)w, p);
    k_big_merge<<<mgrid, kMergeThreads, 0, st>>>(bb, (uint32_t)w, p);
  }
}

}  // namespace sg
