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

constexpr int kSortCap = 4096;       // keys sorted in LDS by one block
constexpr int kMergeTile = 2048;     // outputs of one block in a merge pass
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
    const uint32_t nch = big ? (c + kSortCap - 1) / kSortCap : 0u, ngr = big ? (c + kMergeTile - 1) / kMergeTile : 0u;
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

// Bitonic sort of n <= P keys in LDS (P a power of two <= kSortCap).
__device__ __forceinline__ void lds_bitonic(uint64_t* sk, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const uint64_t a = sk[i], b = sk[l];
          const bool asc = (i & k) == 0;
          if ((a > b) == asc) { sk[i] = b; sk[l] = a; }
        }
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(256) k_tile_sort(DevRaster ras, BinBuffers bb) {
  const int t = blockIdx.x;
  const uint32_t n = bb.tile_cnt[t];
  if (n <= 1) return;
  if (n > (uint32_t)kSortCap) return;   // sorted by k_big_chunks and k_big_merge
  __shared__ uint64_t sk[kSortCap];
  int P = 2;
  while (P < (int)n) P <<= 1;
  uint64_t* g = bb.keys + bb.tile_start[t];
  for (int i = threadIdx.x; i < P; i += blockDim.x) sk[i] = i < (int)n ? g[i] : ~0ull;
  __syncthreads();
  lds_bitonic(sk, P);
  for (int i = threadIdx.x; i < (int)n; i += blockDim.x) g[i] = sk[i];
}

// Tiles with more than kSortCap instances are sorted by the whole grid:
// every LDS-sized chunk of every such tile is sorted by one block, then runs
// are merged pairwise in passes of doubling width.  A pass first finds, for
// every kMergeTile-output block, where its outputs start in the two runs
// (merge path, one thread per block), then each block stages its inputs in
// LDS and merges them.  Passes alternate between keys and keys_tmp at the
// tile's own offset.

// The big tile holding global item g (off has nb + 1 prefix entries).
__device__ __forceinline__ int big_of(const uint32_t* off, int nb, uint32_t g) {
  int lo = 0, hi = nb;   // largest k with off[k] <= g
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Element i of a bitonic stage (k, j) keeps min(own, partner) when it is the
// lower element of an ascending pair or the upper one of a descending pair.
__device__ __forceinline__ uint64_t bitonic_keep(uint64_t v, uint64_t p, int i, int k, int j) {
  const bool take_min = ((i & k) == 0) == ((i & j) == 0);
  return take_min ? (v < p ? v : p) : (v < p ? p : v);
}

__device__ __forceinline__ void bitonic_pair(uint64_t& lo, uint64_t& hi, bool asc) {
  if ((lo > hi) == asc) { const uint64_t t = lo; lo = hi; hi = t; }
}

// Ascending sort of 4096 keys by 1024 threads, four keys per thread in
// registers (thread t holds elements 4t..4t+3): partners in the same thread
// are exchanged in registers, partners in the same wave by lane shuffles,
// and the rest through LDS (element i at sk[(i & 3) * 1024 + (i >> 2)]).
__device__ void sort4096(uint64_t* sk, uint64_t& v0, uint64_t& v1, uint64_t& v2, uint64_t& v3) {
  const int t = threadIdx.x;
  const int i0 = 4 * t;
  for (int k = 2; k <= kSortCap; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 256) {
        __syncthreads();
        sk[t] = v0; sk[1024 + t] = v1; sk[2048 + t] = v2; sk[3072 + t] = v3;
        __syncthreads();
        const int pt = t ^ (j >> 2);
        v0 = bitonic_keep(v0, sk[pt], i0, k, j);
        v1 = bitonic_keep(v1, sk[1024 + pt], i0 + 1, k, j);
        v2 = bitonic_keep(v2, sk[2048 + pt], i0 + 2, k, j);
        v3 = bitonic_keep(v3, sk[3072 + pt], i0 + 3, k, j);
      } else if (j >= 4) {
        const int m = j >> 2;
        const uint64_t p0 = __shfl_xor(v0, m), p1 = __shfl_xor(v1, m), p2 = __shfl_xor(v2, m), p3 = __shfl_xor(v3, m);
        v0 = bitonic_keep(v0, p0, i0, k, j);
        v1 = bitonic_keep(v1, p1, i0 + 1, k, j);
        v2 = bitonic_keep(v2, p2, i0 + 2, k, j);
        v3 = bitonic_keep(v3, p3, i0 + 3, k, j);
      } else if (j == 2) {
        bitonic_pair(v0, v2, (i0 & k) == 0);
        bitonic_pair(v1, v3, ((i0 + 1) & k) == 0);
      } else {
        bitonic_pair(v0, v1, (i0 & k) == 0);
        bitonic_pair(v2, v3, ((i0 + 2) & k) == 0);
      }
    }
  }
  __syncthreads();   // the caller may reuse sk
}

__global__ void __launch_bounds__(1024) k_big_chunks(BinBuffers bb) {
  __shared__ uint64_t sk[kSortCap];
  const int nb = (int)bb.total[2];
  const uint32_t nch = (uint32_t)bb.total[4];
  for (uint32_t g = blockIdx.x; g < nch; g += gridDim.x) {
    const int k = big_of(bb.big_choff, nb, g);
    const uint32_t t = bb.big_tiles[k];
    const int n = (int)bb.tile_cnt[t];
    const int c0 = (int)(g - bb.big_choff[k]) * kSortCap;
    const int m = min(kSortCap, n - c0);
    uint64_t* a = bb.keys + bb.tile_start[t] + c0;
    const int e = 4 * threadIdx.x;
    uint64_t v0 = e < m ? a[e] : ~0ull, v1 = e + 1 < m ? a[e + 1] : ~0ull, v2 = e + 2 < m ? a[e + 2] : ~0ull,
             v3 = e + 3 < m ? a[e + 3] : ~0ull;
    sort4096(sk, v0, v1, v2, v3);
    if (e < m) a[e] = v0;
    if (e + 1 < m) a[e + 1] = v1;
    if (e + 2 < m) a[e + 2] = v2;
    if (e + 3 < m) a[e + 3] = v3;
  }
}

// Position of one merge block in its tile and run pair for a pass of width w.
struct MergeBlock {
  uint32_t t, n, o0, o1, a0, na, b0, nb;
};

__device__ __forceinline__ MergeBlock merge_block(const BinBuffers& bb, int nbig, uint32_t g, uint32_t w) {
  MergeBlock m;
  const int k = big_of(bb.big_goff, nbig, g);
  m.t = bb.big_tiles[k];
  m.n = bb.tile_cnt[m.t];
  m.o0 = (g - bb.big_goff[k]) * (uint32_t)kMergeTile;
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

__global__ void __launch_bounds__(256) k_big_partition(BinBuffers bb, uint32_t w, const uint64_t* __restrict__ src_all) {
  const int nbig = (int)bb.total[2];
  const uint32_t nblk = (uint32_t)bb.total[5];
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < nblk; g += gridDim.x * blockDim.x) {
    const MergeBlock m = merge_block(bb, nbig, g, w);
    if (m.n <= w) continue;   // the tile is already one sorted run (k_big_merge skips it)
    const uint64_t* src = src_all + bb.tile_start[m.t];
    bb.big_split[g] = m.nb ? merge_split(src + m.a0, m.na, src + m.b0, m.nb, m.o0 - m.a0) : m.o0 - m.a0;
  }
}

// Merge passes a big tile takes: one per width kSortCap, 2 kSortCap, ...
// below its length.  Its sorted keys end in keys after an even number and in
// keys_tmp after an odd one.
__device__ __forceinline__ uint32_t merge_passes(uint32_t n) {
  uint32_t p = 0;
  for (uint64_t w = kSortCap; w < n; w <<= 1) ++p;
  return p;
}

__global__ void __launch_bounds__(256) k_big_merge(BinBuffers bb, uint32_t w, const uint64_t* __restrict__ src_all,
                                                   uint64_t* __restrict__ dst_all) {
  __shared__ uint64_t s[kMergeTile];
  const int nbig = (int)bb.total[2];
  const uint32_t nblk = (uint32_t)bb.total[5];
  for (uint32_t g = blockIdx.x; g < nblk; g += gridDim.x) {
    // w = 0: the final copy of the tiles whose keys ended in keys_tmp
    const MergeBlock m = merge_block(bb, nbig, g, w ? w : 0xffffffffu);
    if (w ? m.n <= w : (merge_passes(m.n) & 1u) == 0u) continue;   // nothing to move for this tile
    const uint64_t* src = src_all + bb.tile_start[m.t];
    uint64_t* dst = dst_all + bb.tile_start[m.t];
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
    __syncthreads();
    for (uint32_t x = threadIdx.x; x < nA; x += blockDim.x) s[x] = src[m.a0 + ia0 + x];
    for (uint32_t x = threadIdx.x; x < nB; x += blockDim.x) s[nA + x] = src[m.b0 + ib0 + x];
    __syncthreads();
    const uint32_t d = 8u * threadIdx.x;
    if (d < cnt) {
      uint32_t i = merge_split(s, nA, s + nA, nB, d), j = d - i;
      const uint32_t end = min(d + 8u, cnt);
      for (uint32_t o = d; o < end; ++o) {
        if (j >= nB || (i < nA && s[i] < s[nA + j])) dst[m.o0 + o] = s[i++];
        else dst[m.o0 + o] = s[nA + j++];
      }
    }
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

void launch_tile_sort(const DevRaster& ras, const BinBuffers& bb, const unsigned long long* totals, int n_cu,
                      hipStream_t st) {
  k_tile_sort<<<ras.n_tiles, 256, 0, st>>>(ras, bb);
  if (totals[2] == 0) return;
  const unsigned long long nch = totals[4], nblk = totals[5], maxn = totals[3];
  k_big_chunks<<<(unsigned)std::min<unsigned long long>(nch, (unsigned long long)n_cu * 2), 1024, 0, st>>>(bb);
  const unsigned pgrid = (unsigned)std::max<unsigned long long>(1, (nblk + 255) / 256);
  const unsigned mgrid = (unsigned)std::min<unsigned long long>(nblk, (unsigned long long)n_cu * 8);
  // Pass k merges runs of width kSortCap << k into runs of twice that width,
  // from one buffer into the other, for the tiles still longer than one run;
  // a tile that is already one sorted run is left where its last pass put it.
  uint64_t* src = bb.keys;
  uint64_t* dst = bb.keys_tmp;
  int passes = 0;
  for (unsigned long long w = kSortCap; w < maxn; w <<= 1, ++passes) {
    k_big_partition<<<pgrid, 256, 0, st>>>(bb, (uint32_t)w, src);
    k_big_merge<<<mgrid, 256, 0, st>>>(bb, (uint32_t)w, src, dst);
    std::swap(src, dst);
  }
  // the tiles that took an odd number of passes, back into keys
  if (passes) k_big_merge<<<mgrid, 256, 0, st>>>(bb, 0u, bb.keys_tmp, bb.keys);
}

}  // namespace sg
