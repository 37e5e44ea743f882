// Comparison transform round trip and the SSIM quality measure of Section 4.
//
// k_dct_roundtrip: every block through the orthonormal DCT-II in float64
//   (Y = C X C^T), the plan's retention mask, the inverse (C^T Y' C),
//   rounding half up and clamping to 0..255: the reference the approximate
//   transform is compared with (APE), with its per-image SSE.
// k_ssim: mean SSIM over every 11x11 window position inside the image
//   (Gaussian weights, sigma 1.5, K1 = 0.01, K2 = 0.03, peak 255), the five
//   weighted moments filtered separably in float64 through LDS.
#include "device_common.hpp"

namespace adct16 {

// ---------------------------------------------------------------------------
// Exact DCT-II round trip.  A wavefront takes one block at a time: lane l
// owns row l / 4, columns 4 (l % 4) .. + 3 of each 16x16 stage, and the
// stages meet in a float64 tile in LDS.
__device__ __forceinline__ void tile_sync() { wave_lds_sync(); }

__global__ __launch_bounds__(kGroupThreads) void k_dct_roundtrip(Params P) {
  __shared__ double tile_all[kWavesPerGroup][2][256];
  double(*tile)[256] = tile_all[threadIdx.x >> 6];
  const int lane = threadIdx.x & 63, row = lane >> 2, c0 = 4 * (lane & 3);
  const Tables& tb = *P.tables;
  const uint8_t* in = reinterpret_cast<const uint8_t*>(P.in);
  uint8_t* outp = reinterpret_cast<uint8_t*>(P.out);
  StripCursor c;
  if (!cursor_init(c, P)) return;
  SseAcc acc;
  acc.init(P);
  int img = c.img;
  for (;;) {
    const int y0 = c.sy * 16;
    const int y = min(y0 + row, c.d.h - 1);
    const int nb = min(kStripBlocks, c.d.bx - c.sxi * kStripBlocks);
    for (int b = 0; b < nb; ++b) {
      const int x0 = (c.sxi * kStripBlocks + b) * 16;
      // load row `row`, columns c0..c0+3 (edge-extended)
      double xv[4];
      const int64_t off = c.d.offset + (int64_t)y * c.d.pitch;
#pragma unroll
      for (int k = 0; k < 4; ++k) xv[k] = (double)in[off + min(x0 + c0 + k, c.d.w - 1)];
#pragma unroll
      for (int k = 0; k < 4; ++k) tile[0][row * 16 + c0 + k] = xv[k];
      tile_sync();
      // P = X C^T: P[row][j] = sum_m X[row][m] C[j][m]
      double pv[4] = {0, 0, 0, 0};
      for (int m = 0; m < 16; ++m) {
        const double xm = tile[0][row * 16 + m];
#pragma unroll
        for (int k = 0; k < 4; ++k) pv[k] = fma(xm, tb.dctc[(c0 + k) * 16 + m], pv[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) tile[1][row * 16 + c0 + k] = pv[k];
      tile_sync();
      // Y = C P: Y[row][v] = sum_i C[row][i] P[i][v]; retention mask
      double yv[4] = {0, 0, 0, 0};
      for (int i = 0; i < 16; ++i) {
        const double ci = tb.dctc[row * 16 + i];
#pragma unroll
        for (int k = 0; k < 4; ++k) yv[k] = fma(ci, tile[1][i * 16 + c0 + k], yv[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) tile[0][row * 16 + c0 + k] = tb.wkeep[row * 16 + c0 + k] ? yv[k] : 0.0;
      tile_sync();
      // Q = C^T Y: Q[row][v] = sum_u C[u][row] Y[u][v]
      double qv[4] = {0, 0, 0, 0};
      for (int u = 0; u < 16; ++u) {
        const double cu = tb.dctc[u * 16 + row];
#pragma unroll
        for (int k = 0; k < 4; ++k) qv[k] = fma(cu, tile[0][u * 16 + c0 + k], qv[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) tile[1][row * 16 + c0 + k] = qv[k];
      tile_sync();
      // A' = Q C: A'[row][n] = sum_v Q[row][v] C[v][n]
      double av[4] = {0, 0, 0, 0};
      for (int v = 0; v < 16; ++v) {
        const double qrv = tile[1][row * 16 + v];
#pragma unroll
        for (int k = 0; k < 4; ++k) av[k] = fma(qrv, tb.dctc[v * 16 + c0 + k], av[k]);
      }
      tile_sync();
      const bool rowok = y0 + row < c.d.h;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int xx = x0 + c0 + k;
        if (rowok && xx < c.d.w) {
          const int pix = (int)fmin(fmax(floor(av[k] + 0.5), 0.0), 255.0);
          if (outp) outp[off + xx] = (uint8_t)pix;
          const int d = pix - (int)xv[k];
          acc.lane += (unsigned)(d * d);
        }
      }
    }
    const bool changed = cursor_next(c, P);
    const bool done = c.s >= c.s_end;
    if (changed || done) {
      acc.flush(P, img);
      img = c.img;
    }
    if (done) break;
  }
}

hipError_t launch_dct_roundtrip(const Params& P, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_dct_roundtrip, dim3(grid), dim3(kGroupThreads), 0, s, P);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// SSIM.  A workgroup takes a tile of kSsimTh x kSsimTw output positions (the
// top-left corners of the 11x11 windows) of one image.
constexpr int kSsimTh = 16, kSsimTw = 32, kSsimWin = 11;
constexpr int kSsimIh = kSsimTh + kSsimWin - 1, kSsimIw = kSsimTw + kSsimWin - 1;

__global__ __launch_bounds__(256) void k_ssim(Params P, const int64_t* tile_begin, const uint8_t* a, const uint8_t* b,
                                              double* ssim) {
  __shared__ float xa[kSsimIh][kSsimIw], xb[kSsimIh][kSsimIw];
  __shared__ double hm[5][kSsimIh][kSsimTw];  // horizontally filtered a, b, a^2, b^2, ab
  __shared__ double red[4];
  const int64_t t = blockIdx.x;
  // image of this tile: last i with tile_begin[i] <= t
  int lo = 0, hi = P.n_images - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_begin[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const ImageDesc d = P.images[lo];
  const int oh = d.h - (kSsimWin - 1), ow = d.w - (kSsimWin - 1);  // > 0 for images with tiles
  const int tx = (ow + kSsimTw - 1) / kSsimTw;
  const int64_t local = t - tile_begin[lo];
  const int ty0 = (int)(local / tx) * kSsimTh, tx0 = (int)(local % tx) * kSsimTw;
  // input tile (clamped reads; positions past the image feed only masked outputs)
  for (int k = threadIdx.x; k < kSsimIh * kSsimIw; k += 256) {
    const int r = k / kSsimIw, cc = k % kSsimIw;
    const int yy = min(ty0 + r, d.h - 1), xx = min(tx0 + cc, d.w - 1);
    const int64_t o = d.offset + (int64_t)yy * d.pitch + xx;
    xa[r][cc] = (float)a[o];
    xb[r][cc] = (float)b[o];
  }
  __syncthreads();
  const double* g = P.tables->gauss;
  for (int k = threadIdx.x; k < kSsimIh * kSsimTw; k += 256) {
    const int r = k / kSsimTw, cc = k % kSsimTw;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
#pragma unroll
    for (int j = 0; j < kSsimWin; ++j) {
      const double va = xa[r][cc + j], vb = xb[r][cc + j], w = g[j];
      s0 = fma(w, va, s0);
      s1 = fma(w, vb, s1);
      s2 = fma(w, va * va, s2);
      s3 = fma(w, vb * vb, s3);
      s4 = fma(w, va * vb, s4);
    }
    hm[0][r][cc] = s0; hm[1][r][cc] = s1; hm[2][r][cc] = s2; hm[3][r][cc] = s3; hm[4][r][cc] = s4;
  }
  __syncthreads();
  constexpr double c1 = (0.01 * 255.0) * (0.01 * 255.0), c2 = (0.03 * 255.0) * (0.03 * 255.0);
  double sum = 0;
  for (int k = threadIdx.x; k < kSsimTh * kSsimTw; k += 256) {
    const int r = k / kSsimTw, cc = k % kSsimTw;
    if (ty0 + r >= oh || tx0 + cc >= ow) continue;
    double m[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < kSsimWin; ++i) {
      const double w = g[i];
#pragma unroll
      for (int q = 0; q < 5; ++q) m[q] = fma(w, hm[q][r + i][cc], m[q]);
    }
    const double mx = m[0], my = m[1];
    const double sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
    sum += ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2));
  }
  // workgroup sum, one atomic per tile
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) sum += __shfl_xor(sum, m, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(ssim + lo, red[0] + red[1] + red[2] + red[3]);
}

__global__ void k_ssim_finalize(Params P, double* ssim) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P.n_images; i += gridDim.x * blockDim.x) {
    const ImageDesc d = P.images[i];
    const int oh = d.h - (kSsimWin - 1), ow = d.w - (kSsimWin - 1);
    ssim[i] = (oh > 0 && ow > 0) ? ssim[i] / ((double)oh * (double)ow) : __builtin_nan("");
  }
}

__global__ void k_zero_f64(double* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0;
}

hipError_t launch_ssim(const Params& P, const int64_t* tile_begin, int64_t n_tiles, const void* a, const void* b,
                       double* ssim, hipStream_t s) {
  const int g = (P.n_images + 255) / 256;
  hipLaunchKernelGGL(k_zero_f64, dim3(g), dim3(256), 0, s, ssim, P.n_images);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n_tiles > 0) {
    hipLaunchKernelGGL(k_ssim, dim3((unsigned)n_tiles), dim3(256), 0, s, P, tile_begin,
                       reinterpret_cast<const uint8_t*>(a), reinterpret_cast<const uint8_t*>(b), ssim);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ssim_finalize, dim3(g), dim3(256), 0, s, P, ssim);
  return hipGetLastError();
}

}  // namespace adct16
