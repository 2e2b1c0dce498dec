// Element-wise and reduction kernels of libsg: format casts, bit-flip
// injection, the support-box reduction and the guard clamp (Alg. 1), and
// the fixed-order reduction of metric partials.
#include "sg_device.h"
#include "sg_kernels.h"

namespace sg {

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_cast(const float* __restrict__ src, void* __restrict__ dst, int64_t n, int dtype, int mode) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t w = cast_word(src[i], dtype, mode);
    if (dtype == SG_F32) reinterpret_cast<uint32_t*>(dst)[i] = w;
    else reinterpret_cast<uint16_t*>(dst)[i] = (uint16_t)w;
  }
}

// XOR one bit of each addressed word.  16-bit words are flipped with a 32-bit
// atomic on their aligned container so that sites sharing a word compose.
__global__ void k_inject(DevScene s, const sg_site* __restrict__ sites, int n, uint32_t* saved) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const sg_site st = sites[k];
  const int64_t idx = (int64_t)st.prim * s.ps[st.field] + (int64_t)st.comp * s.cs[st.field];
  uint32_t old;
  if (s.dtype == SG_F32) {
    uint32_t* p = const_cast<uint32_t*>(reinterpret_cast<const uint32_t*>(s.ptr[st.field])) + idx;
    old = atomicXor(p, 1u << st.bit);
  } else {
    uintptr_t a = reinterpret_cast<uintptr_t>(reinterpret_cast<const uint16_t*>(s.ptr[st.field]) + idx);
    const uint32_t shift = (a & 2u) ? 16u : 0u;
    uint32_t* p = reinterpret_cast<uint32_t*>(a & ~(uintptr_t)3);
    old = (atomicXor(p, 1u << (st.bit + shift)) >> shift) & 0xffffu;
  }
  if (saved) saved[k] = old;
}

// Box reduction (Alg. 1 precompute): order keys of every component, min and
// max by atomics on the keys (the result does not depend on the order).
__global__ void k_box_reduce(DevScene s, int f, uint32_t* __restrict__ kmin, uint32_t* __restrict__ kmax) {
  const int c = blockIdx.y;
  uint32_t mn = 0xffffffffu, mx = 0u;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s.n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t key = order_key(load_word(s, f, i, c), s.dtype);
    mn = min(mn, key);
    mx = max(mx, key);
  }
  for (int o = 32; o > 0; o >>= 1) {
    mn = min(mn, (uint32_t)__shfl_xor((int)mn, o));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(kmin + c, mn);
    atomicMax(kmax + c, mx);
  }
}

__global__ void k_box_finalize(const uint32_t* kmin, const uint32_t* kmax, int C, int dtype, void* lo, void* hi) {
  const int c = threadIdx.x;
  if (c >= C) return;
  const uint32_t l = key_to_word(kmin[c], dtype), h = key_to_word(kmax[c], dtype);
  if (dtype == SG_F32) {
    reinterpret_cast<uint32_t*>(lo)[c] = l;
    reinterpret_cast<uint32_t*>(hi)[c] = h;
  } else {
    reinterpret_cast<uint16_t*>(lo)[c] = (uint16_t)l;
    reinterpret_cast<uint16_t*>(hi)[c] = (uint16_t)h;
  }
}

// Guard clamp of one field in place (Alg. 1 per frame).  Each thread keeps
// four independent words (and their bounds) in flight; only clamped words are
// written.  Clamps are counted per wave.
__device__ __forceinline__ void guard_one(const DevScene& s, const DevBox& b, int f, int c, int64_t i, uint32_t w,
                                          uint32_t lo, uint32_t hi, uint32_t* local) {
  bool clamped;
  const uint32_t g = clamp_word(w, lo, hi, s.dtype, &clamped);
  if (clamped) {
    const int64_t idx = i * s.ps[f] + (int64_t)c * s.cs[f];
    if (s.dtype == SG_F32) const_cast<uint32_t*>(reinterpret_cast<const uint32_t*>(s.ptr[f]))[idx] = g;
    else const_cast<uint16_t*>(reinterpret_cast<const uint16_t*>(s.ptr[f]))[idx] = (uint16_t)g;
    ++*local;
  }
}

__global__ void __launch_bounds__(256) k_guard(DevScene s, DevBox b, int f, unsigned long long* __restrict__ count) {
  const int c = blockIdx.y;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t local = 0;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; i + 3 * stride < s.n; i += 4 * stride) {
    uint32_t w[4], lo[4], hi[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      w[u] = load_word(s, f, i + u * stride, c);
      box_words(b, f, i + u * stride, c, s.n, &lo[u], &hi[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) guard_one(s, b, f, c, i + u * stride, w[u], lo[u], hi[u], &local);
  }
  for (; i < s.n; i += stride) {
    uint32_t lo, hi;
    box_words(b, f, i, c, s.n, &lo, &hi);
    guard_one(s, b, f, c, i, load_word(s, f, i, c), lo, hi, &local);
  }
  for (int o = 32; o > 0; o >>= 1) local += (uint32_t)__shfl_xor((int)local, o);
  if ((threadIdx.x & 63) == 0 && local) atomicAdd(count, (unsigned long long)local);
}

// Guard of whole component rows against a global box, for rows whose
// primitives are contiguous: 16-byte loads of 4 fp32 or 8 16-bit words, the
// clamp decision per word as in guard_one, a vector written back only when
// one of its words changed.  Block y serves row y of the plan; the few words
// before the row's first 16-byte boundary and after its last are done one by
// one by block x = 0.
template <int ES, bool PER_PRIM>
__global__ void __launch_bounds__(256) k_guard_rows(DevScene s, DevBox b, GuardRows gr,
                                                    unsigned long long* __restrict__ count) {
  constexpr int PER = 16 / ES;   // words per vector
  const int f = gr.f[blockIdx.y], c = gr.c[blockIdx.y];
  const int64_t n = s.n;
  uint32_t glo = 0, ghi = 0;     // global box of this row
  if (!PER_PRIM) box_words(b, f, 0, c, n, &glo, &ghi);
  char* row = const_cast<char*>(reinterpret_cast<const char*>(s.ptr[f])) + (int64_t)c * s.cs[f] * ES;
  // per-primitive bounds: rows of the box arrays, laid out like the scene's
  const char* lrow = PER_PRIM ? reinterpret_cast<const char*>(b.lo[f]) + (int64_t)c * n * ES : nullptr;
  const char* hrow = PER_PRIM ? reinterpret_cast<const char*>(b.hi[f]) + (int64_t)c * n * ES : nullptr;
  const int64_t head = (int64_t)(((16 - ((uintptr_t)row & 15)) & 15) / ES);   // words before alignment
  const int64_t h = head < n ? head : n;
  const int64_t nvec = (n - h) / PER;
  const int64_t tail0 = h + nvec * PER;
  uint32_t local = 0;
  auto word_at = [](const char* r, int64_t i) -> uint32_t {
    return ES == 4 ? reinterpret_cast<const uint32_t*>(r)[i] : reinterpret_cast<const uint16_t*>(r)[i];
  };
  auto one = [&](int64_t i) {
    const uint32_t w = word_at(row, i);
    const uint32_t lo = PER_PRIM ? word_at(lrow, i) : glo, hi = PER_PRIM ? word_at(hrow, i) : ghi;
    bool cl;
    const uint32_t g = clamp_word(w, lo, hi, s.dtype, &cl);
    if (cl) {
      if (ES == 4) reinterpret_cast<uint32_t*>(row)[i] = g;
      else reinterpret_cast<uint16_t*>(row)[i] = (uint16_t)g;
      ++local;
    }
  };
  if (blockIdx.x == 0) {
    for (int64_t i = threadIdx.x; i < h; i += blockDim.x) one(i);
    for (int64_t i = tail0 + threadIdx.x; i < n; i += blockDim.x) one(i);
  }
  uint4* vec = reinterpret_cast<uint4*>(row + h * ES);
  const uint4* lvec = PER_PRIM ? reinterpret_cast<const uint4*>(lrow + h * ES) : nullptr;
  const uint4* hvec = PER_PRIM ? reinterpret_cast<const uint4*>(hrow + h * ES) : nullptr;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nvec; j += stride) {
    const uint4 v = vec[j];
    uint32_t words[4] = {v.x, v.y, v.z, v.w};
    uint32_t los[4] = {glo, glo, glo, glo}, his[4] = {ghi, ghi, ghi, ghi};
    if (PER_PRIM) {
      const uint4 l = lvec[j], u = hvec[j];
      los[0] = l.x; los[1] = l.y; los[2] = l.z; los[3] = l.w;
      his[0] = u.x; his[1] = u.y; his[2] = u.z; his[3] = u.w;
    }
    bool any = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (ES == 4) {
        bool cl;
        words[q] = clamp_word(words[q], los[q], his[q], s.dtype, &cl);
        any |= cl;
        local += cl ? 1u : 0u;
      } else {
        bool c0, c1;
        const uint32_t lo0 = PER_PRIM ? (los[q] & 0xffffu) : glo, hi0 = PER_PRIM ? (his[q] & 0xffffu) : ghi;
        const uint32_t lo1 = PER_PRIM ? (los[q] >> 16) : glo, hi1 = PER_PRIM ? (his[q] >> 16) : ghi;
        const uint32_t a = clamp_word(words[q] & 0xffffu, lo0, hi0, s.dtype, &c0);
        const uint32_t d = clamp_word(words[q] >> 16, lo1, hi1, s.dtype, &c1);
        words[q] = (a & 0xffffu) | (d << 16);
        any |= c0 | c1;
        local += (c0 ? 1u : 0u) + (c1 ? 1u : 0u);
      }
    }
    if (any) vec[j] = make_uint4(words[0], words[1], words[2], words[3]);
  }
  for (int o = 32; o > 0; o >>= 1) local += (uint32_t)__shfl_xor((int)local, o);
  if ((threadIdx.x & 63) == 0 && local) atomicAdd(count, (unsigned long long)local);
}

__global__ void k_health(const unsigned long long* count, unsigned long long threshold, uint32_t* alert) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *alert = (*count > threshold) ? 1u : 0u;
}

// Frame metrics of standalone images: one block per (chunk, variant).
__global__ void k_metrics_partials(const float* __restrict__ img, const float* __restrict__ clean, int64_t px_per_var,
                                   int64_t chunk, Partial* __restrict__ out) {
  const int v = blockIdx.y;
  const int64_t beg = blockIdx.x * chunk, end = min(px_per_var, beg + chunk);
  const float* I = img + (int64_t)v * px_per_var * 3;
  double sse = 0.0;
  uint32_t changed = 0, nonfin = 0;
  float mx = 0.f;
  for (int64_t p = beg + threadIdx.x; p < end; p += blockDim.x) {
    const float* a = I + p * 3;
    const float* c = clean + p * 3;
    double dm = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
      const double d = (double)a[ch] - (double)c[ch];
      if (!isfinite(a[ch])) nonfin = 1;
      sse += d * d;
      dm = fmax(dm, fabs(d));
    }
    changed += dm > (1.0 / 255.0) ? 1u : 0u;
    mx = fmaxf(mx, (float)dm);
  }
  block_reduce_partial(sse, changed, mx, nonfin, 0ull, out + (int64_t)v * gridDim.x + blockIdx.x);
}

// Per variant (one wave): partials[item_off[v] .. + n_items[v]) in a fixed
// order -> metrics.  With vs, the partials are a batch's item partials and
// the record is the one the fused reduction of the next batch's variant prep
// writes (reduce_batch_variant); without, they are per tile (tiles_x > 0) or
// per pixel chunk.
__global__ void __launch_bounds__(64) k_reduce_metrics(const Partial* __restrict__ parts, const uint32_t* __restrict__ item_off,
                                                       const uint32_t* __restrict__ n_items, uint32_t uniform_items,
                                                       const VariantState* vs, const uint32_t* flags,
                                                       const unsigned long long* clamps, uint32_t n_pixels,
                                                       sg_metrics_t* __restrict__ out, uint32_t path, int tiles_x,
                                                       int tiles_y) {
  const int v = blockIdx.x;
  if (vs && item_off && n_items && !flags && path == 0u) {
    reduce_batch_variant(parts, item_off, n_items, vs, n_pixels, v, out);
    return;
  }
  const uint32_t off = item_off ? item_off[v] : v * uniform_items;
  const uint32_t n = n_items ? n_items[v] : uniform_items;
  uint64_t rend = 0;   // full render with per-tile partials: regions of the changed tiles
  const Partial red = wave_reduce_parts(parts, off, n, tiles_x, tiles_y, &rend);
  if (threadIdx.x == 0) {
    uint64_t pr = 0, rr = 0;
    if (vs) { pr = vs[v].pred_regions; rr = vs[v].rend_regions; }
    else if (tiles_x > 0) { pr = ~0ull; rr = rend; }
    out[v] = make_metrics(red, (vs ? vs[v].nonfinite : 0u) | (flags ? (flags[0] & 1u) : 0u), vs ? vs[v].n_dirty : n,
                          vs ? vs[v].clamps : (clamps ? *clamps : 0ull), n_pixels, path, pr, rr);
  }
}

// Pools the records of K views per variant (view-major input, K x B): SSE,
// changed pixels, evaluations, dirty tiles and pixels add up, the largest
// delta and the non-finite flag are kept, the footprint is the mean of the
// per-view footprints (Def. 1), PSNR follows from the pooled MSE, and the
// catastrophe rule (Def. 2) is applied to the pooled footprint.
__global__ void k_pool_views(const sg_metrics_t* __restrict__ views, int K, int B, int64_t view_stride,
                             int64_t var_stride, sg_metrics_t* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= B) return;
  Partial r;
  r.sse = 0.0; r.evals = 0; r.changed = 0; r.max_abs = 0.f; r.nonfinite = 0; r._pad = 0;
  uint32_t dirty = 0, px = 0;
  double foot = 0.0;
  uint64_t pr = 0, rr = 0;
  for (int k = 0; k < K; ++k) {
    const sg_metrics_t& m = views[(int64_t)k * view_stride + (int64_t)v * var_stride];
    pr |= m.predicted_regions;
    rr |= m.rendered_regions;
    r.sse += m.sse;
    r.evals += m.evals;
    r.changed += m.changed_px;
    r.max_abs = fmaxf(r.max_abs, m.max_abs);
    r.nonfinite |= m.nonfinite;
    dirty += m.dirty_tiles;
    px += m.n_pixels;
    foot += (double)m.changed_px / (double)m.n_pixels;
  }
  const sg_metrics_t& m0 = views[(int64_t)v * var_stride];
  sg_metrics_t o = make_metrics(r, 0u, dirty, m0.clamps, px, m0.path, pr, rr);
  o.footprint = (float)(foot / K);
  o.catastrophic = (o.nonfinite || foot / K > 0.01) ? 1u : 0u;
  out[v] = o;
}

// ----------------------------------------------------------------------------
// host launchers

static inline int blocks_for(int64_t n, int bs, int cap = 65535) {
  int64_t b = (n + bs - 1) / bs;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_fill_u32<<<blocks_for(n, 256, 4096), 256, 0, st>>>(p, v, n);
}
void launch_cast(const float* src, void* dst, int64_t n, int dtype, int mode, hipStream_t st) {
  k_cast<<<blocks_for(n, 256, 16384), 256, 0, st>>>(src, dst, n, dtype, mode);
}
void launch_inject(const DevScene& s, const sg_site* sites, int n, uint32_t* saved, hipStream_t st) {
  if (n <= 0) return;
  k_inject<<<(n + 255) / 256, 256, 0, st>>>(s, sites, n, saved);
}
void launch_box_reduce(const DevScene& s, int f, uint32_t* kmin, uint32_t* kmax, hipStream_t st) {
  dim3 g(blocks_for(s.n, 256, 1024), s.ncomp[f]);
  k_box_reduce<<<g, 256, 0, st>>>(s, f, kmin, kmax);
}
void launch_box_finalize(const uint32_t* kmin, const uint32_t* kmax, int C, int dtype, void* lo, void* hi,
                         hipStream_t st) {
  k_box_finalize<<<1, 64, 0, st>>>(kmin, kmax, C, dtype, lo, hi);
}
void launch_guard(const DevScene& s, const DevBox& b, int f, unsigned long long* count, hipStream_t st) {
  dim3 g(blocks_for(s.n, 256, 2048), s.ncomp[f]);
  k_guard<<<g, 256, 0, st>>>(s, b, f, count);
}
void launch_guard_rows(const DevScene& s, const DevBox& b, const GuardRows& gr, unsigned long long* count,
                       hipStream_t st) {
  if (gr.n_rows == 0) return;
  const int es = s.dtype == SG_F32 ? 4 : 2;
  const int64_t nvec = (int64_t)s.n * es / 16;
  // enough blocks per row for several vectors in flight per thread across the device
  dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((nvec + 1023) / 1024, 2048)), gr.n_rows);
  const bool pp = b.mode == SG_BOX_PER_PRIM;
  if (es == 4) {
    if (pp) k_guard_rows<4, true><<<g, 256, 0, st>>>(s, b, gr, count);
    else k_guard_rows<4, false><<<g, 256, 0, st>>>(s, b, gr, count);
  } else {
    if (pp) k_guard_rows<2, true><<<g, 256, 0, st>>>(s, b, gr, count);
    else k_guard_rows<2, false><<<g, 256, 0, st>>>(s, b, gr, count);
  }
}
void launch_health(const unsigned long long* count, unsigned long long thr, uint32_t* alert, hipStream_t st) {
  k_health<<<1, 64, 0, st>>>(count, thr, alert);
}
void launch_metrics_partials(const float* img, const float* clean, int64_t px_per_var, int nchunks, int B,
                             Partial* out, hipStream_t st) {
  const int64_t chunk = (px_per_var + nchunks - 1) / nchunks;
  dim3 g(nchunks, B);
  k_metrics_partials<<<g, 256, 0, st>>>(img, clean, px_per_var, chunk, out);
}
void launch_reduce_metrics(const Partial* parts, const uint32_t* item_off, const uint32_t* n_items,
                           uint32_t uniform_items, const VariantState* vs, const uint32_t* flags,
                           const unsigned long long* clamps, uint32_t n_pixels, sg_metrics_t* out, int B,
                           uint32_t path, hipStream_t st, int tiles_x, int tiles_y) {
  if (B <= 0) return;
  k_reduce_metrics<<<B, 64, 0, st>>>(parts, item_off, n_items, uniform_items, vs, flags, clamps, n_pixels, out,
                                     path, tiles_x, tiles_y);
}

void launch_pool_views(const sg_metrics_t* views, int K, int B, int64_t view_stride, int64_t var_stride,
                       sg_metrics_t* out, hipStream_t st) {
  if (B <= 0) return;
  k_pool_views<<<(B + 255) / 256, 256, 0, st>>>(views, K, B, view_stride, var_stride, out);
}

}  // namespace sg
