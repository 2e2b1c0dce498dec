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
constexpr int kEmitSmall = 32;       // rectangles up to this many tiles are emitted by one thread

__global__ void __launch_bounds__(1024) k_tile_prefix(DevRaster ras, BinBuffers bb) {
  const int X = ras.tiles_x + 1, Y = ras.tiles_y + 1;
  for (int r = threadIdx.x; r < Y; r += blockDim.x) {
    int acc = 0;
    for (int x = 0; x < X; ++x) { acc += bb.diff[r * X + x]; bb.diff[r * X + x] = acc; }
  }
  __syncthreads();
  for (int x = threadIdx.x; x < X; x += blockDim.x) {
    int acc = 0;
    for (int r = 0; r < Y; ++r) { acc += bb.diff[r * X + x]; bb.diff[r * X + x] = acc; }
  }
  __syncthreads();
  __shared__ uint32_t s[1024];
  unsigned long long carry = 0;
  for (int base = 0; base < ras.n_tiles; base += 1024) {
    const int t = base + threadIdx.x;
    uint32_t c = 0;
    if (t < ras.n_tiles) {
      const int tx = t % ras.tiles_x, ty = t / ras.tiles_x;
      c = (uint32_t)bb.diff[ty * X + tx];
      bb.tile_cnt[t] = c;
      bb.cursor[t] = 0;
    }
    s[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const uint32_t y = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
      __syncthreads();
      s[threadIdx.x] += y;
      __syncthreads();
    }
    if (t < ras.n_tiles) bb.tile_start[t] = (uint32_t)(carry + s[threadIdx.x] - c);
    carry += s[1023];
    __syncthreads();
  }
  // tiles whose lists exceed one LDS sort, in tile order, with the prefix
  // counts of their LDS chunks and of their 8-key merge groups
  __shared__ unsigned long long s_acc[3];
  __shared__ uint32_t s_max;
  if (threadIdx.x == 0) { s_acc[0] = s_acc[1] = s_acc[2] = 0; s_max = 0; }
  __syncthreads();
  for (int base = 0; base < ras.n_tiles; base += 1024) {
    const int t = base + threadIdx.x;
    const uint32_t c = t < ras.n_tiles ? bb.tile_cnt[t] : 0u;
    const bool big = c > (uint32_t)kSortCap;
    const uint32_t nch = big ? (c + kSortCap - 1) / kSortCap : 0u, ngr = big ? (c + 7) / 8 : 0u;
    // three inclusive scans over the 1024 tiles of this round, in one LDS pass each
    uint32_t v[3] = {big ? 1u : 0u, nch, ngr}, excl[3];
    for (int q = 0; q < 3; ++q) {
      s[threadIdx.x] = v[q];
      __syncthreads();
      for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t y = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
      }
      excl[q] = s[threadIdx.x] - v[q];
      v[q] = s[1023];
      __syncthreads();
    }
    if (big) {
      const uint32_t k = (uint32_t)(s_acc[0] + excl[0]);
      bb.big_tiles[k] = (uint32_t)t;
      bb.big_choff[k] = (uint32_t)(s_acc[1] + excl[1]);
      bb.big_goff[k] = (uint32_t)(s_acc[2] + excl[2]);
      atomicMax(&s_max, c);
    }
    __syncthreads();
    if (threadIdx.x == 0) { s_acc[0] += v[0]; s_acc[1] += v[1]; s_acc[2] += v[2]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint32_t nb = (uint32_t)s_acc[0];
    bb.big_choff[nb] = (uint32_t)s_acc[1];
    bb.big_goff[nb] = (uint32_t)s_acc[2];
    bb.total[0] = carry; bb.total[1] = 0; bb.total[2] = nb; bb.total[3] = s_max;
    bb.total[4] = s_acc[1]; bb.total[5] = s_acc[2];
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
// are merged pairwise in passes of doubling width, each pass spreading its
// 8-key output groups over all threads (merge path per group).  Passes
// alternate between keys and keys_tmp at the tile's own offset.

// The big tile holding global item g (off has nb + 1 prefix entries).
__device__ __forceinline__ int big_of(const uint32_t* off, int nb, uint32_t g) {
  int lo = 0, hi = nb;   // largest k with off[k] <= g
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
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
    __syncthreads();
    for (int i = threadIdx.x; i < kSortCap; i += blockDim.x) sk[i] = i < m ? a[i] : ~0ull;
    __syncthreads();
    lds_bitonic(sk, kSortCap);
    for (int i = threadIdx.x; i < m; i += blockDim.x) a[i] = sk[i];
  }
}

// One pass: runs of width w are merged into runs of 2w (tiles whose list is
// not longer than w are copied).  `src` and `dst` are keys / keys_tmp.
__global__ void __launch_bounds__(256) k_big_merge(BinBuffers bb, uint32_t w, const uint64_t* __restrict__ src_all,
                                                   uint64_t* __restrict__ dst_all) {
  const int nb = (int)bb.total[2];
  const uint32_t ngr = (uint32_t)bb.total[5];
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < ngr; g += gridDim.x * blockDim.x) {
    const int k = big_of(bb.big_goff, nb, g);
    const uint32_t t = bb.big_tiles[k];
    const uint32_t n = bb.tile_cnt[t];
    const uint64_t* src = src_all + bb.tile_start[t];
    uint64_t* dst = dst_all + bb.tile_start[t];
    const uint32_t pos0 = (g - bb.big_goff[k]) * 8u;
    const uint32_t end = min(pos0 + 8u, n);
    if (n <= w) {
      for (uint32_t o = pos0; o < end; ++o) dst[o] = src[o];
      continue;
    }
    const uint32_t a0 = pos0 / (2u * w) * (2u * w);
    const uint32_t na = min(w, n - a0);
    const uint32_t b0 = a0 + na, nbk = b0 < n ? min(w, n - b0) : 0u;
    const uint32_t d = pos0 - a0;
    uint32_t lo = d > nbk ? d - nbk : 0u, hi = min(d, na);
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (src[a0 + mid] < src[b0 + d - 1 - mid]) lo = mid + 1; else hi = mid;
    }
    uint32_t i = lo, j = d - lo;
    for (uint32_t o = pos0; o < end; ++o) {
      if (j >= nbk || (i < na && src[a0 + i] < src[b0 + j])) dst[o] = src[a0 + i++];
      else dst[o] = src[b0 + j++];
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
  const unsigned long long nch = totals[4], ngr = totals[5], maxn = totals[3];
  k_big_chunks<<<(unsigned)std::min<unsigned long long>(nch, (unsigned long long)n_cu * 2), 1024, 0, st>>>(bb);
  const unsigned grid = (unsigned)std::max<unsigned long long>(
      1, std::min<unsigned long long>((ngr + 255) / 256, (unsigned long long)n_cu * 8));
  uint64_t* src = bb.keys;
  uint64_t* dst = bb.keys_tmp;
  int passes = 0;
  for (unsigned long long w = kSortCap; w < maxn; w <<= 1, ++passes) {
    k_big_merge<<<grid, 256, 0, st>>>(bb, (uint32_t)w, src, dst);
    std::swap(src, dst);
  }
  if (passes & 1) k_big_merge<<<grid, 256, 0, st>>>(bb, 0xffffffffu, src, dst);   // back into keys
}

}  // namespace sg
