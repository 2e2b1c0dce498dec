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
  if (threadIdx.x == 0) { bb.total[0] = carry; bb.total[1] = 0; bb.total[2] = 0; }
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
  if (n > (uint32_t)kSortCap) {
    if (threadIdx.x == 0) bb.big_tiles[atomicAdd(bb.total + 2, 1ull)] = (uint32_t)t;
    return;
  }
  __shared__ uint64_t sk[kSortCap];
  int P = 2;
  while (P < (int)n) P <<= 1;
  uint64_t* g = bb.keys + bb.tile_start[t];
  for (int i = threadIdx.x; i < P; i += blockDim.x) sk[i] = i < (int)n ? g[i] : ~0ull;
  __syncthreads();
  lds_bitonic(sk, P);
  for (int i = threadIdx.x; i < (int)n; i += blockDim.x) g[i] = sk[i];
}

// Tiles with more than kSortCap instances: sort chunks of kSortCap in LDS,
// then merge runs pairwise (merge path per 8 outputs) between keys and keys_tmp.
__global__ void __launch_bounds__(1024) k_tile_sort_big(BinBuffers bb) {
  __shared__ uint64_t sk[kSortCap];
  const unsigned long long nbt = bb.total[2];
  for (unsigned long long bt = blockIdx.x; bt < nbt; bt += gridDim.x) {
    const uint32_t t = bb.big_tiles[bt];
    const int n = (int)bb.tile_cnt[t];
    uint64_t* a = bb.keys + bb.tile_start[t];
    uint64_t* b = bb.keys_tmp + bb.tile_start[t];
    for (int c0 = 0; c0 < n; c0 += kSortCap) {
      const int m = min(kSortCap, n - c0);
      __syncthreads();
      for (int i = threadIdx.x; i < kSortCap; i += blockDim.x) sk[i] = i < m ? a[c0 + i] : ~0ull;
      __syncthreads();
      lds_bitonic(sk, kSortCap);
      for (int i = threadIdx.x; i < m; i += blockDim.x) a[c0 + i] = sk[i];
    }
    __syncthreads();
    uint64_t* src = a;
    uint64_t* dst = b;
    for (int w = kSortCap; w < n; w <<= 1) {
      for (int pos0 = threadIdx.x * 8; pos0 < n; pos0 += blockDim.x * 8) {
        const int p = pos0 / (2 * w);
        const int a0 = p * 2 * w, na = min(w, n - a0);
        const int b0 = a0 + na, nb = max(0, min(w, n - b0));
        const int d = pos0 - a0;
        int lo = max(0, d - nb), hi = min(d, na);
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (src[a0 + mid] < src[b0 + d - 1 - mid]) lo = mid + 1; else hi = mid;
        }
        int i = lo, j = d - lo;
        const int end = min(pos0 + 8, a0 + na + nb);
        for (int o = pos0; o < end; ++o) {
          if (j >= nb || (i < na && src[a0 + i] < src[b0 + j])) dst[o] = src[a0 + i++];
          else dst[o] = src[b0 + j++];
        }
      }
      __syncthreads();
      uint64_t* tmp = src; src = dst; dst = tmp;
    }
    if (src != a) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = src[i];
    }
    __syncthreads();
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

void launch_tile_sort(const DevRaster& ras, const BinBuffers& bb, hipStream_t st) {
  k_tile_sort<<<ras.n_tiles, 256, 0, st>>>(ras, bb);
  k_tile_sort_big<<<256, 1024, 0, st>>>(bb);
}

}  // namespace sg
