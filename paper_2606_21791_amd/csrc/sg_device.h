// Device-side building blocks shared by the libsg kernels: storage-format
// decode/encode, the guard clamp on one word, and the per-primitive
// projection (activation, EWA covariance, eigenframe, colour) that every
// render path uses, so that a primitive projected for a clean frame, a full
// corrupted render or an incremental re-composite yields the same record bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_types.h"

namespace sg {

constexpr double kFltMax = 3.4028234663852886e38;

// ---------------------------------------------------------------------------
// Storage formats (fp32 1|8|23, fp16 1|5|10, bf16 1|8|7).  Words are carried
// zero-extended in uint32.

__device__ __forceinline__ int word_bytes(int dtype) { return dtype == SG_F32 ? 4 : 2; }

__device__ __forceinline__ double decode_word(uint32_t w, int dtype) {
  if (dtype == SG_F32) return (double)__uint_as_float(w);
  if (dtype == SG_BF16) return (double)__uint_as_float(w << 16);
  // fp16: exact via integer fields
  const uint32_t s = (w >> 15) & 1u, e = (w >> 10) & 31u, m = w & 1023u;
  double mag;
  if (e == 31u) mag = m ? __longlong_as_double(0x7ff8000000000000ll) : __longlong_as_double(0x7ff0000000000000ll);
  else if (e == 0u) mag = ldexp((double)m, -24);
  else mag = ldexp((double)(m | 1024u), (int)e - 25);
  return s ? -mag : mag;
}

// fp32 value -> fp16/bf16 word with rounding mode (SG_RNE / SG_RD / SG_RU),
// by integer arithmetic on the fp32 fields.  EB exponent bits, MB mantissa bits.
template <int EB, int MB>
__device__ __forceinline__ uint32_t f32_to_small(float x, int mode) {
  const uint32_t b = __float_as_uint(x);
  const uint32_t sign = b >> 31;
  const uint32_t out_sign = sign << (EB + MB);
  const int e32 = (int)((b >> 23) & 255u);
  const uint32_t m32 = b & 0x7fffffu;
  const uint32_t exp_all = ((1u << EB) - 1u) << MB;
  if (e32 == 255) return out_sign | exp_all | (m32 ? (1u << (MB - 1)) : 0u);   // Inf / quiet NaN
  const int bias = (1 << (EB - 1)) - 1;
  // significand with hidden bit, value = sig * 2^(E - 150)
  uint32_t sig = e32 ? (m32 | 0x800000u) : m32;
  const int E = e32 ? e32 : 1;
  if (sig == 0) return out_sign;
  int e_t = E - 127 + bias;                          // target biased exponent if normal
  int shift = 23 - MB;                               // drop bits for a normal result
  if (e_t < 1 || e32 == 0) { shift += 1 - e_t; e_t = 0; }   // subnormal result (always for fp32 subnormals)
  const bool away = (mode == SG_RU && !sign) || (mode == SG_RD && sign);
  const bool toward0 = (mode == SG_RU && sign) || (mode == SG_RD && !sign);
  if (e_t >= (1 << EB) - 1) {                        // overflow before rounding
    if (mode == SG_RNE || away) return out_sign | exp_all;
    return out_sign | (exp_all - 1u);                // largest finite
  }
  uint32_t q, rem, half;
  if (shift >= 32) { q = 0; rem = sig; half = 0; }
  else { q = sig >> shift; rem = sig & ((1u << shift) - 1u); half = 1u << (shift - 1); }
  uint32_t inc;
  if (mode == SG_RNE) inc = (shift >= 32) ? 0u : ((rem > half) || (rem == half && (q & 1u))) ? 1u : 0u;
  else inc = (away && rem) ? 1u : 0u;
  (void)toward0;
  uint32_t mag;
  if (e_t == 0) mag = q;                              // subnormal: exponent field 0
  else mag = ((uint32_t)e_t << MB) | (q & ((1u << MB) - 1u));
  mag += inc;                                         // carries into the exponent (up to Inf)
  if (mode != SG_RNE && !away && mag >= exp_all) mag = exp_all - 1u;
  return out_sign | mag;
}

__device__ __forceinline__ uint32_t cast_word(float x, int dtype, int mode) {
  if (dtype == SG_F32) return __float_as_uint(x);
  if (dtype == SG_F16) return f32_to_small<5, 10>(x, mode);
  return f32_to_small<8, 7>(x, mode);
}

// Order-preserving unsigned key of a stored word (IEEE total order on
// non-NaN values, -0 below +0), used by the box min/max reduction.
__device__ __forceinline__ uint32_t order_key(uint32_t w, int dtype) {
  const uint32_t sbit = dtype == SG_F32 ? 0x80000000u : 0x8000u;
  const uint32_t all = dtype == SG_F32 ? 0xffffffffu : 0xffffu;
  return (w & sbit) ? (~w & all) : (w | sbit);
}
__device__ __forceinline__ uint32_t key_to_word(uint32_t k, int dtype) {
  const uint32_t sbit = dtype == SG_F32 ? 0x80000000u : 0x8000u;
  const uint32_t all = dtype == SG_F32 ? 0xffffffffu : 0xffffu;
  return (k & sbit) ? (k & ~sbit) : (~k & all);
}

// Alg. 1 clamp of one word: NaN -> lo, x < lo -> lo, x > hi -> hi, else x.
// Sets *clamped when the word changes class.
__device__ __forceinline__ uint32_t clamp_word(uint32_t w, uint32_t lo, uint32_t hi, int dtype, bool* clamped) {
  const double x = decode_word(w, dtype);
  const double l = decode_word(lo, dtype);
  const double h = decode_word(hi, dtype);
  if (x != x || x < l) { *clamped = true; return lo; }
  if (x > h) { *clamped = true; return hi; }
  *clamped = false;
  return w;
}

__device__ __forceinline__ uint32_t load_word(const DevScene& s, int f, int64_t prim, int c) {
  const int64_t idx = prim * s.ps[f] + (int64_t)c * s.cs[f];
  if (s.dtype == SG_F32) return __ldg(reinterpret_cast<const uint32_t*>(s.ptr[f]) + idx);
  return (uint32_t)__ldg(reinterpret_cast<const uint16_t*>(s.ptr[f]) + idx);
}

__device__ __forceinline__ void box_words(const DevBox& b, int f, int64_t prim, int c, int64_t n, uint32_t* lo,
                                          uint32_t* hi) {
  const int64_t idx = b.mode == SG_BOX_GLOBAL ? (int64_t)c : (int64_t)c * n + prim;
  if (b.dtype == SG_F32) {
    *lo = __ldg(reinterpret_cast<const uint32_t*>(b.lo[f]) + idx);
    *hi = __ldg(reinterpret_cast<const uint32_t*>(b.hi[f]) + idx);
  } else {
    *lo = __ldg(reinterpret_cast<const uint16_t*>(b.lo[f]) + idx);
    *hi = __ldg(reinterpret_cast<const uint16_t*>(b.hi[f]) + idx);
  }
}

// ---------------------------------------------------------------------------
// Projected record: what the compositing loop reads per primitive.
//   r0 = (Ux, Uy, c, s): integer part of the screen mean, unit major axis
//   r1 = (k1, k2, i1, i2): fractional mean rotated into the eigenframe
//        (k1 = fx c + fy s, k2 = fy c - fx s) and (log2 e / 2) / lambda_{1,2}
//   r2 = (opacity, r, g, b)
// so that for pixel centre (px, py), with ex = px - Ux, ey = py - Uy,
//   u' = ex c + ey s - k1,  v' = ey c - ex s - k2,
//   q (log2 e / 2) = u'^2 i1 + v'^2 i2.
struct ProjOut {
  Rec rec;
  uint32_t depth;      // fp32 bits of the camera depth (positive)
  uint32_t rect0;      // tx0 | ty0 << 16
  uint32_t rect1;      // tx1 | ty1 << 16  (inclusive); rect0 > rect1 style empty => culled
  bool visible;
  bool nonfinite;      // a stored component is Inf/NaN
};

// Real SH basis of degree <= 3 (3DGS order and signs), normalisations from
// sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) (times sqrt 2 for m != 0).
__device__ __forceinline__ void sh_basis(double x, double y, double z, int deg, double* Y) {
  Y[0] = 0.28209479177387814;                       // 1 / (2 sqrt(pi))
  if (deg < 1) return;
  const double k1 = 0.4886025119029199;             // sqrt(3 / (4 pi))
  Y[1] = -k1 * y; Y[2] = k1 * z; Y[3] = -k1 * x;
  if (deg < 2) return;
  const double k22 = 1.0925484305920792;            // sqrt(15 / pi) / 2
  const double k20 = 0.31539156525252005;           // sqrt(5 / pi) / 4
  const double k2x = 0.5462742152960396;            // sqrt(15 / pi) / 4
  Y[4] = k22 * x * y; Y[5] = -k22 * y * z; Y[6] = k20 * (3.0 * z * z - 1.0);
  Y[7] = -k22 * x * z; Y[8] = k2x * (x * x - y * y);
  if (deg < 3) return;
  const double k33 = 0.5900435899266435;            // sqrt(35 / (2 pi)) / 4
  const double k32 = 2.890611442640554;             // sqrt(105 / pi) / 2
  const double k31 = 0.4570457994644658;            // sqrt(21 / (2 pi)) / 4
  const double k30 = 0.3731763325901154;            // sqrt(7 / pi) / 4
  const double k32b = 1.445305721320277;            // sqrt(105 / pi) / 4
  Y[9] = -k33 * y * (3.0 * x * x - y * y);
  Y[10] = k32 * x * y * z;
  Y[11] = -k31 * y * (5.0 * z * z - 1.0);
  Y[12] = k30 * z * (5.0 * z * z - 3.0);
  Y[13] = -k31 * x * (5.0 * z * z - 1.0);
  Y[14] = k32b * z * (x * x - y * y);
  Y[15] = -k33 * x * (x * x - 3.0 * y * y);
}

__device__ __forceinline__ bool in_range(double v) { return fabs(v) <= kFltMax; }   // false for NaN

// Project one primitive.  `get(f, c)` returns the (already flipped and
// guarded) stored word of field f, component c.  Everything is evaluated in
// fp64 and rounded once into the fp32 record.
// Stored components per primitive at SH degree DEG and the offset of each
// field in a flat per-primitive word array.
template <int DEG>
struct Layout {
  static constexpr int kRest = 3 * ((DEG + 1) * (DEG + 1) - 1);
  static constexpr int kWords = 14 + kRest;
  static constexpr int off(int f) { return f == 0 ? 0 : f == 1 ? 3 : f == 2 ? 6 : f == 3 ? 10 : f == 4 ? 11 : 14; }
};

template <int DEG, class Get>
__device__ __forceinline__ ProjOut project_prim(Get get, int dtype, const DevCam& cam, const DevRaster& ras) {
  constexpr int sh_degree = DEG;
  ProjOut o;
  o.visible = false;
  o.nonfinite = false;
  o.depth = 0;
  o.rect0 = 0xffffffffu;
  o.rect1 = 0;
  o.rec.r0 = o.rec.r1 = o.rec.r2 = make_float4(0.f, 0.f, 0.f, 0.f);
  constexpr int n_rest = Layout<DEG>::kRest;

  double mu[3], ls[3], qv[4], dc[3], logit;
  bool fin = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) { mu[c] = decode_word(get(0, c), dtype); fin &= isfinite(mu[c]); }
#pragma unroll
  for (int c = 0; c < 3; ++c) { ls[c] = decode_word(get(1, c), dtype); fin &= isfinite(ls[c]); }
#pragma unroll
  for (int c = 0; c < 4; ++c) { qv[c] = decode_word(get(2, c), dtype); fin &= isfinite(qv[c]); }
  logit = decode_word(get(3, 0), dtype);
  fin &= isfinite(logit);
#pragma unroll
  for (int c = 0; c < 3; ++c) { dc[c] = decode_word(get(4, c), dtype); fin &= isfinite(dc[c]); }
#pragma unroll
  for (int c = 0; c < n_rest; ++c) fin &= isfinite(decode_word(get(5, c), dtype));
  if (!fin) { o.nonfinite = true; return o; }

  // camera space
  const double* R = cam.R;
  const double px = R[0] * mu[0] + R[1] * mu[1] + R[2] * mu[2] + cam.t[0];
  const double py = R[3] * mu[0] + R[4] * mu[1] + R[5] * mu[2] + cam.t[1];
  const double pz = R[6] * mu[0] + R[7] * mu[1] + R[8] * mu[2] + cam.t[2];
  if (!(pz > cam.nearz && pz <= cam.farz)) return o;

  // activations
  double s[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) { s[k] = exp(ls[k]); if (!in_range(s[k])) return o; }
  const double qa = fmax(fmax(fabs(qv[0]), fabs(qv[1])), fmax(fabs(qv[2]), fabs(qv[3])));
  if (!(qa > 0.0)) return o;
  // reciprocals are taken once and multiplied (fp64 keeps the products within
  // a few units of the last place, far below the fp32 record's rounding)
  const double iqa = 1.0 / qa;
  double qw = qv[0] * iqa, qx = qv[1] * iqa, qy = qv[2] * iqa, qz = qv[3] * iqa;
  const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const double iqn = 1.0 / qn;
  qw *= iqn; qx *= iqn; qy *= iqn; qz *= iqn;
  const double Rq[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy),
                        2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                        2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};

  // EWA: Jacobian with the tangent clamp
  const double ipz = 1.0 / pz;
  const double tx = fmin(cam.limx, fmax(-cam.limx, px * ipz)) * pz;
  const double ty = fmin(cam.limy, fmax(-cam.limy, py * ipz)) * pz;
  const double J00 = cam.fx * ipz, J02 = -cam.fx * tx * ipz * ipz;
  const double J11 = cam.fy * ipz, J12 = -cam.fy * ty * ipz * ipz;
  // U = R * Rq (world-to-camera rotation of the principal axes)
  double U[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) U[i * 3 + j] = R[i * 3 + 0] * Rq[0 * 3 + j] + R[i * 3 + 1] * Rq[1 * 3 + j] + R[i * 3 + 2] * Rq[2 * 3 + j];
  // T = J U (2x3); V = T diag(s)
  double T0[3], T1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T0[k] = J00 * U[0 * 3 + k] + J02 * U[2 * 3 + k];
    T1[k] = J11 * U[1 * 3 + k] + J12 * U[2 * 3 + k];
  }
  double a = 0.0, b = 0.0, c = 0.0, trA = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double v0 = T0[k] * s[k], v1 = T1[k] * s[k];
    if (!in_range(v0) || !in_range(v1)) return o;
    a += v0 * v0; b += v0 * v1; c += v1 * v1;
  }
  trA = a + c;
  a += ras.dil; c += ras.dil;
  if (!in_range(a) || !in_range(b) || !in_range(c)) return o;
  const double hd = 0.5 * (a - c);
  // a, b and c are within the fp32 range here, so the squares cannot leave
  // the fp64 range and no scaled hypot is needed
  const double h = sqrt(hd * hd + b * b);
  const double lam1 = 0.5 * a + 0.5 * c + h;
  if (!in_range(lam1)) return o;
  // det(Sigma') = det A + dil tr A + dil^2 with det A by Cauchy-Binet: the 2x2
  // minors of J U are U^T (J0 x J1), so no difference of large products appears.
  const double n0 = -J02 * J11, n1 = -J00 * J12, n2 = J00 * J11;
  const double m12 = U[0] * n0 + U[3] * n1 + U[6] * n2;
  const double m20 = U[1] * n0 + U[4] * n1 + U[7] * n2;
  const double m01 = U[2] * n0 + U[5] * n1 + U[8] * n2;
  const double t12 = s[1] * s[2] * m12, t20 = s[2] * s[0] * m20, t01 = s[0] * s[1] * m01;
  const double det = t12 * t12 + t20 * t20 + t01 * t01 + ras.dil * trA + (double)ras.dil * ras.dil;
  const double lam2 = det / lam1;
  // unit major axis without cancellation
  double e0, e1;
  if (hd >= 0.0) { e0 = hd + h; e1 = b; } else { e0 = b; e1 = -hd + h; }
  const double en = sqrt(e0 * e0 + e1 * e1);
  if (en > 0.0) { const double ien = 1.0 / en; e0 *= ien; e1 *= ien; } else { e0 = 1.0; e1 = 0.0; }

  const double u = cam.fx * px * ipz + cam.cx;
  const double v = cam.fy * py * ipz + cam.cy;
  if (!in_range(u) || !in_range(v)) return o;

  // colour along the viewing direction
  double dx = mu[0] - cam.campos[0], dy = mu[1] - cam.campos[1], dz = mu[2] - cam.campos[2];
  const double dn = sqrt(dx * dx + dy * dy + dz * dz);
  if (dn > 0.0) { const double idn = 1.0 / dn; dx *= idn; dy *= idn; dz *= idn; }
  double Y[16];
  sh_basis(dx, dy, dz, sh_degree, Y);
  double col[3] = {Y[0] * dc[0], Y[0] * dc[1], Y[0] * dc[2]};
  constexpr int K = (sh_degree + 1) * (sh_degree + 1);
#pragma unroll
  for (int k = 1; k < K; ++k) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) col[ch] += Y[k] * decode_word(get(5, 3 * (k - 1) + ch), dtype);
  }
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    col[ch] += 0.5;
    if (!in_range(col[ch])) return o;
    col[ch] = fmax(col[ch], 0.0);
  }
  const double op = 1.0 / (1.0 + exp(-logit));
  const float opf = (float)op;
  if (!(opf >= ras.amin)) return o;                    // alpha <= opacity < alpha_min everywhere

  // conservative tile rectangle of { q <= min(cut, 2 ln(o / alpha_min)) }
  const double qeff = fmin((double)ras.cutq, 2.0 * log((double)opf / (double)ras.amin));
  const double qbox = qeff * 1.001 + 0.01;
  const double hx = sqrt(qbox * a) * 1.0001 + 1e-3 * (1.0 + 1e-4 * fabs(u));
  const double hy = sqrt(qbox * c) * 1.0001 + 1e-3 * (1.0 + 1e-4 * fabs(v));
  const double xlo = floor(u - hx - 0.5), xhi = ceil(u + hx - 0.5);
  const double ylo = floor(v - hy - 0.5), yhi = ceil(v + hy - 0.5);
  if (xhi < 0.0 || yhi < 0.0 || xlo > (double)(cam.W - 1) || ylo > (double)(cam.H - 1)) return o;
  const double itile = 1.0 / (double)ras.tile;   // exact: the tile size is a power of two
  const int tx0 = (int)fmax(0.0, floor(xlo * itile)), tx1 = (int)fmin((double)(ras.tiles_x - 1), floor(xhi * itile));
  const int ty0 = (int)fmax(0.0, floor(ylo * itile)), ty1 = (int)fmin((double)(ras.tiles_y - 1), floor(yhi * itile));
  if (tx1 < tx0 || ty1 < ty0) return o;

  const float cf = (float)e0, sf = (float)e1;
  const float Ux = (float)floor(u), Uy = (float)floor(v);
  const double fxr = u - (double)Ux, fyr = v - (double)Uy;
  const float k1 = (float)(fxr * (double)cf + fyr * (double)sf);
  const float k2 = (float)(fyr * (double)cf - fxr * (double)sf);
  const double hl = 0.72134752044448170;             // log2(e) / 2
  o.rec.r0 = make_float4(Ux, Uy, cf, sf);
  o.rec.r1 = make_float4(k1, k2, (float)(hl / lam1), (float)(hl / lam2));
  o.rec.r2 = make_float4(opf, (float)col[0], (float)col[1], (float)col[2]);
  o.depth = __float_as_uint((float)pz);
  o.rect0 = (uint32_t)tx0 | ((uint32_t)ty0 << 16);
  o.rect1 = (uint32_t)tx1 | ((uint32_t)ty1 << 16);
  o.visible = true;
  return o;
}

// Whether tile (tx, ty) lies in the packed tile rectangle [r0, r1].
__device__ __forceinline__ bool rect_has(uint32_t r0, uint32_t r1, int tx, int ty) {
  return tx >= (int)(r0 & 0xffff) && tx <= (int)(r1 & 0xffff) && ty >= (int)(r0 >> 16) && ty <= (int)(r1 >> 16);
}

// Smallest (depth, id) key that a variant removes from or inserts into the
// list of tile (tx, ty): the old key of each changed primitive whose clean
// rectangle holds the tile, the new key of each whose corrupted one does.
// All ones when the variant changes nothing in the tile.
__device__ __forceinline__ unsigned long long tile_min_key(const Touch* touch, uint32_t n_touch, int tx, int ty) {
  unsigned long long mk = ~0ull;
  for (uint32_t j = 0; j < n_touch; ++j) {
    const Touch& t = touch[j];
    if (t.flags & 4u) continue;
    if ((t.flags & 1u) && rect_has(t.old_rect0, t.old_rect1, tx, ty))
      mk = min(mk, ((unsigned long long)t.old_depth << 32) | t.prim);
    if ((t.flags & 2u) && rect_has(t.new_rect0, t.new_rect1, tx, ty))
      mk = min(mk, ((unsigned long long)t.new_depth << 32) | t.prim);
  }
  return mk;
}

// Whether some pixel centre of tile (tx, ty) can take record r: whether the
// smallest q of the record over the tile's pixel centres is within
// min(cut, log2(o / alpha_min)) (scaled units, the loop's test), so that the
// tile's pixels cannot change when no record of a variant reaches it.  In
// coordinates relative to the ellipse's centre, q = i1 u^2 + i2 v^2 with
// u = X c + Y s and v = Y c - X s.  q is convex, so its minimum over the box
// of pixel centres is 0 when the box holds the centre, and otherwise lies on
// one of the box's edges, where it is a one-dimensional quadratic minimized
// in closed form (on X = const at Y = X gy, on Y = const at X = Y gx).
// Computed in fp32 with margins (the box widened by 0.05 px, q allowed 1%
// and 0.05 above the bound) well above the rounding of these steps and of
// the loop's q while the centre lies within 4,096 px of the tile; farther
// centres, and records with a non-finite field, are taken to reach the tile.
__device__ __forceinline__ bool rec_reaches_tile(const Rec& r, int tx, int ty, int tile, int W, int H, float qc,
                                                 float amin) {
  const float Ux = r.r0.x, Uy = r.r0.y, c = r.r0.z, s = r.r0.w;
  const float k1 = r.r1.x, k2 = r.r1.y, i1 = r.r1.z, i2 = r.r1.w, o = r.r2.x;
  const float cx = Ux + (k1 * c - k2 * s), cy = Uy + (k1 * s + k2 * c);
  const float x0 = (float)(tx * tile) + 0.45f - cx, x1 = (float)min((tx + 1) * tile, W) - 0.45f - cx;
  const float y0 = (float)(ty * tile) + 0.45f - cy, y1 = (float)min((ty + 1) * tile, H) - 0.45f - cy;
  const float far = fmaxf(fmaxf(fabsf(x0), fabsf(x1)), fmaxf(fabsf(y0), fabsf(y1)));
  if (!(far <= 4096.f) || !(i1 >= 0.f) || !(i2 >= 0.f) || !isfinite(c + s + i1 + i2 + o)) return true;
  if (!(o >= amin)) return false;   // o 2^-q < alpha_min for every q >= 0
  if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return true;
  const float qe = fminf(qc, __log2f(o / amin)) * 1.01f + 0.05f;
  const float cs = c * s * (i2 - i1);
  const float dy = i1 * s * s + i2 * c * c, dx = i1 * c * c + i2 * s * s;
  const float gy = dy > 0.f ? cs / dy : 0.f, gx = dx > 0.f ? cs / dx : 0.f;
  auto q_at = [&](float X, float Y) {
    const float u = X * c + Y * s, v = Y * c - X * s;
    return i1 * u * u + i2 * v * v;
  };
  const float qa = q_at(x0, fminf(fmaxf(x0 * gy, y0), y1));
  const float qb = q_at(x1, fminf(fmaxf(x1 * gy, y0), y1));
  const float qcc = q_at(fminf(fmaxf(y0 * gx, x0), x1), y0);
  const float qd = q_at(fminf(fmaxf(y1 * gx, x0), x1), y1);
  return fminf(fminf(qa, qb), fminf(qcc, qd)) <= qe;
}

// The records a variant's work-item listing tests tiles against: rec (the
// variant's kRecSlots touch records; null: no test) on a raster of tile-pixel
// tiles, W x H pixels, with the loop's cut and alpha_min.
struct ReachArgs {
  const Rec* rec;
  int tile, W, H;
  float qc, amin;
};

// tile_min_key over the changes whose record (clean for a removal, corrupted
// for an insertion) reaches some pixel centre of the tile: all ones when no
// pixel of the tile can change.
__device__ __forceinline__ unsigned long long tile_min_key_reach(const Touch* touch, uint32_t n_touch,
                                                                 const ReachArgs& ra, int tx, int ty) {
  unsigned long long mk = ~0ull;
  for (uint32_t j = 0; j < n_touch; ++j) {
    const Touch& t = touch[j];
    if (t.flags & 4u) continue;
    if ((t.flags & 1u) && rect_has(t.old_rect0, t.old_rect1, tx, ty) &&
        rec_reaches_tile(ra.rec[kMaxTouch + j], tx, ty, ra.tile, ra.W, ra.H, ra.qc, ra.amin))
      mk = min(mk, ((unsigned long long)t.old_depth << 32) | t.prim);
    if ((t.flags & 2u) && rect_has(t.new_rect0, t.new_rect1, tx, ty) &&
        rec_reaches_tile(ra.rec[j], tx, ty, ra.tile, ra.W, ra.H, ra.qc, ra.amin))
      mk = min(mk, ((unsigned long long)t.new_depth << 32) | t.prim);
  }
  return mk;
}

// Whether a site is corrected by the variant's emulated defense (the
// protect field of sg_variant): the sign and exponent bits of the storage
// format, or every bit.
__device__ __forceinline__ bool site_corrected(uint32_t protect, int bit, int dtype) {
  if (protect == SG_PROTECT_VOTE) return true;
  if (protect != SG_PROTECT_SIGN_EXP) return false;
  const int first = dtype == SG_F32 ? 23 : (dtype == SG_F16 ? 10 : 7);
  return bit >= first;
}

}  // namespace sg
