// Structural similarity of B frames against one clean frame (Sec. 3
// "Metrics", after Wang et al. 2004): 11 x 11 Gaussian window of standard
// deviation 1.5 (separable, normalised), C1 = 0.01^2, C2 = 0.03^2 for images
// in [0, 1], biased local variance and covariance, every window position wholly
// inside the frame, mean over positions and the three channels.
//
// One block computes a 16 x 16 tile of window positions of one frame: the
// 26 x 26 patch of both frames is staged in LDS per channel, filtered along
// rows into LDS and then along columns, all in fp64.  Per-block sums are
// reduced per frame in a fixed order by a second kernel.
#include "sg_device.h"
#include "sg_kernels.h"

namespace sg {

constexpr int kWin = 11, kOut = 16, kPatch = kOut + kWin - 1;   // 26

__global__ void __launch_bounds__(256) k_ssim_tiles(const float* __restrict__ imgs, const float* __restrict__ clean,
                                                    int H, int W, SsimWeights gw, double* __restrict__ partial) {
  __shared__ float sx[kPatch][kPatch], sy[kPatch][kPatch];
  __shared__ double h[5][kPatch][kOut];   // row-filtered x, y, x^2, y^2, x*y
  const int b = blockIdx.y;
  const int tiles_x = (W - kWin + 1 + kOut - 1) / kOut;
  const int ox = (blockIdx.x % tiles_x) * kOut, oy = (blockIdx.x / tiles_x) * kOut;
  const int vw = W - kWin + 1, vh = H - kWin + 1;   // valid positions
  const float* x = imgs + (int64_t)b * H * W * 3;
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int c = 0; c < 3; ++c) {
    __syncthreads();
    for (int k = tid; k < kPatch * kPatch; k += blockDim.x) {
      const int r = k / kPatch, q = k % kPatch;
      const int gy = oy + r, gx = ox + q;
      const bool in = gy < H && gx < W;
      const int64_t off = ((int64_t)gy * W + gx) * 3 + c;
      sx[r][q] = in ? x[off] : 0.f;
      sy[r][q] = in ? clean[off] : 0.f;
    }
    __syncthreads();
    for (int k = tid; k < kPatch * kOut; k += blockDim.x) {
      const int r = k / kOut, q = k % kOut;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0;
#pragma unroll
      for (int t = 0; t < kWin; ++t) {
        const double xv = sx[r][q + t], yv = sy[r][q + t], w = gw.w[t];
        a0 = fma(w, xv, a0);
        a1 = fma(w, yv, a1);
        a2 = fma(w, xv * xv, a2);
        a3 = fma(w, yv * yv, a3);
        a4 = fma(w, xv * yv, a4);
      }
      h[0][r][q] = a0; h[1][r][q] = a1; h[2][r][q] = a2; h[3][r][q] = a3; h[4][r][q] = a4;
    }
    __syncthreads();
    const int r = tid / kOut, q = tid % kOut;
    if (oy + r < vh && ox + q < vw) {
      double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < kWin; ++t)
#pragma unroll
        for (int j = 0; j < 5; ++j) m[j] = fma(gw.w[t], h[j][r + t][q], m[j]);
      const double mx = m[0], my = m[1];
      const double vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
      const double c1 = 1e-4, c2 = 9e-4;
      acc += ((2.0 * mx * my + c1) * (2.0 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2));
    }
  }
  // fixed-order block sum
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ double s_w[4];
  if ((tid & 63) == 0) s_w[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) partial[(int64_t)b * gridDim.x + blockIdx.x] = ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}

__global__ void k_ssim_reduce(const double* __restrict__ partial, int nblk, double inv_count, double* __restrict__ out) {
  const int b = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) s += partial[(int64_t)b * nblk + k];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  __shared__ double s_w[4];
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[b] = (((s_w[0] + s_w[1]) + s_w[2]) + s_w[3]) * inv_count;
}

int ssim_blocks(int H, int W) {
  return ((W - kWin + 1 + kOut - 1) / kOut) * ((H - kWin + 1 + kOut - 1) / kOut);
}

void launch_ssim(const float* imgs, const float* clean, int B, int H, int W, const SsimWeights& gw, double* partial,
                 double* out, hipStream_t st) {
  const int nblk = ssim_blocks(H, W);
  k_ssim_tiles<<<dim3(nblk, B), 256, 0, st>>>(imgs, clean, H, W, gw, partial);
  const double count = 3.0 * (double)(H - kWin + 1) * (double)(W - kWin + 1);
  k_ssim_reduce<<<B, 256, 0, st>>>(partial, nblk, 1.0 / count, out);
}

}  // namespace sg
