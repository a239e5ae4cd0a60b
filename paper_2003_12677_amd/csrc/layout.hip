// Streaming kernels around the FFTs (Sec. 3 Eq. (2)): pairing of real slices into complex
// channels (Sec. 3.1), deapodisation, the index shifts that put the image origin and the
// rotation axis at index 0 (so plain FFTs compute the centred transforms), zero padding,
// cropping and the slice-major <-> channel-fastest transposes.  Each block stages a
// 64-point x 32-slice tile in LDS so that both the slice-major side (256-byte runs per
// slice) and the channel-fastest side (128-byte runs per point) are read and written in
// contiguous segments.

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tomo {
namespace {

constexpr int kTile = 64;   // grid points per block
constexpr int kCh = 16;     // complex channels (= 32 real slices) per block

// x[B][n][n] -> X[G][G][C]:  X[(i1-on) mod G][(i2-on) mod G][c] = kd[i1] kd[i2] (x[2c] + i x[2c+1])
__global__ __launch_bounds__(256) void k_embed(const float* __restrict__ x, float2* __restrict__ X,
                                               const float* __restrict__ kd, int B, int n, int G,
                                               int C, int on) {
  __shared__ float tile[2 * kCh][kTile + 1];
  const int g1 = blockIdx.y;
  const int g20 = blockIdx.x * kTile;
  const int c0 = blockIdx.z * kCh;
  int i1 = g1 + on;
  if (i1 >= G) i1 -= G;
  const bool rowok = i1 < n;
  const int tt = threadIdx.x & (kTile - 1);
  const int g2 = g20 + tt;
  int i2 = g2 + on;
  if (i2 >= G) i2 -= G;
  const bool ok = rowok && g2 < G && i2 < n;
  const float k = ok ? kd[i1] * kd[i2] : 0.f;
  for (int sl = threadIdx.x >> 6; sl < 2 * kCh; sl += 4) {
    const int s = 2 * c0 + sl;
    float v = 0.f;
    if (ok && s < B) v = x[((int64_t)s * n + i1) * n + i2] * k;
    tile[sl][tt] = v;
  }
  __syncthreads();
  const int nc = min(kCh, C - c0);
  const int nt = min(kTile, G - g20);
  float2* out = X + ((int64_t)g1 * G + g20) * C + c0;
  for (int e = threadIdx.x; e < nt * nc; e += 256) {
    const int t = e / nc, cl = e - t * nc;
    out[(int64_t)t * C + cl] = make_float2(tile[2 * cl][t], tile[2 * cl + 1][t]);
  }
}

// X[G][G][C] -> x[B][n][n]:  x[s][i1][i2] = scale kd[i1] kd[i2] part_s(X[(i1-on) mod G][(i2-on) mod G][s/2])
__global__ __launch_bounds__(256) void k_crop_image(const float2* __restrict__ X, float* __restrict__ x,
                                                    const float* __restrict__ kd, int B, int n, int G,
                                                    int C, int on, float scale) {
  __shared__ float tile[2 * kCh][kTile + 1];
  const int i1 = blockIdx.y;
  const int i20 = blockIdx.x * kTile;
  const int c0 = blockIdx.z * kCh;
  int g1 = i1 - on;
  if (g1 < 0) g1 += G;
  const int nc = min(kCh, C - c0);
  const int nt = min(kTile, n - i20);
  for (int e = threadIdx.x; e < nt * nc; e += 256) {
    const int t = e / nc, cl = e - t * nc;
    int g2 = i20 + t - on;
    if (g2 < 0) g2 += G;
    const float2 v = X[((int64_t)g1 * G + g2) * C + c0 + cl];
    tile[2 * cl][t] = v.x;
    tile[2 * cl + 1][t] = v.y;
  }
  __syncthreads();
  const int tt = threadIdx.x & (kTile - 1);
  const int i2 = i20 + tt;
  if (i2 >= n) return;
  const float k = scale * kd[i1] * kd[i2];
  for (int sl = threadIdx.x >> 6; sl < 2 * nc; sl += 4) {
    const int s = 2 * c0 + sl;
    if (s < B) x[((int64_t)s * n + i1) * n + i2] = tile[sl][tt] * k;
  }
}

// Y[L][nt][C] -> y[B][nt][np]:  y[s][a][b] = scale part_s(Y[(b - cdet) mod L][a][s/2])
__global__ __launch_bounds__(256) void k_crop_sino(const float2* __restrict__ Y, float* __restrict__ y,
                                                   int B, int nt, int np, int L, int C, int cdet,
                                                   float scale) {
  __shared__ float tile[2 * kCh][kTile + 1];
  const int a = blockIdx.y;
  const int b0 = blockIdx.x * kTile;
  const int c0 = blockIdx.z * kCh;
  const int nc = min(kCh, C - c0);
  const int nb = min(kTile, np - b0);
  for (int e = threadIdx.x; e < nb * nc; e += 256) {
    const int t = e / nc, cl = e - t * nc;
    int m = b0 + t - cdet;
    m %= L;
    if (m < 0) m += L;
    const float2 v = Y[((int64_t)m * nt + a) * C + c0 + cl];
    tile[2 * cl][t] = v.x;
    tile[2 * cl + 1][t] = v.y;
  }
  __syncthreads();
  const int tt = threadIdx.x & (kTile - 1);
  const int b = b0 + tt;
  if (b >= np) return;
  for (int sl = threadIdx.x >> 6; sl < 2 * nc; sl += 4) {
    const int s = 2 * c0 + sl;
    if (s < B) y[((int64_t)s * nt + a) * np + b] = tile[sl][tt] * scale;
  }
}

// y[B][nt][np] -> Y[L][nt][C]:  Y[m][a][c] = y[2c][a][b] + i y[2c+1][a][b], b = (m + cdet) mod L
// (zero where b >= np or the slice does not exist)
__global__ __launch_bounds__(256) void k_pad_sino(const float* __restrict__ y, float2* __restrict__ Y,
                                                  int B, int nt, int np, int L, int C, int cdet) {
  __shared__ float tile[2 * kCh][kTile + 1];
  const int a = blockIdx.y;
  const int m0 = blockIdx.x * kTile;
  const int c0 = blockIdx.z * kCh;
  const int tt = threadIdx.x & (kTile - 1);
  const int m = m0 + tt;
  int b = m + cdet;
  if (b >= L) b -= L;
  const bool ok = m < L && b < np;
  for (int sl = threadIdx.x >> 6; sl < 2 * kCh; sl += 4) {
    const int s = 2 * c0 + sl;
    float v = 0.f;
    if (ok && s < B) v = y[((int64_t)s * nt + a) * np + b];
    tile[sl][tt] = v;
  }
  __syncthreads();
  const int nc = min(kCh, C - c0);
  const int nm = min(kTile, L - m0);
  for (int e = threadIdx.x; e < nm * nc; e += 256) {
    const int t = e / nc, cl = e - t * nc;
    Y[((int64_t)(m0 + t) * nt + a) * C + c0 + cl] = make_float2(tile[2 * cl][t], tile[2 * cl + 1][t]);
  }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

tomo_status launch_embed(const tomo_op* op, const float* x, float2* X, int B, hipStream_t st) {
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  dim3 grid(cdiv(g.G, kTile), (unsigned)g.G, cdiv(C, kCh));
  hipLaunchKernelGGL(k_embed, grid, dim3(256), 0, st, x, X, op->kd_dev, B, g.n, g.G, C, g.on);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_crop_image(const tomo_op* op, const float2* X, float* x, int B, float scale,
                              hipStream_t st) {
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  dim3 grid(cdiv(g.n, kTile), (unsigned)g.n, cdiv(C, kCh));
  hipLaunchKernelGGL(k_crop_image, grid, dim3(256), 0, st, X, x, op->kd_dev, B, g.n, g.G, C, g.on,
                     scale);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_crop_sino(const tomo_op* op, const float2* Y, float* y, int B, float scale,
                             hipStream_t st) {
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  dim3 grid(cdiv(g.np, kTile), (unsigned)g.nt, cdiv(C, kCh));
  hipLaunchKernelGGL(k_crop_sino, grid, dim3(256), 0, st, Y, y, B, g.nt, g.np, g.L, C, g.cdet,
                     scale);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_pad_sino(const tomo_op* op, const float* y, float2* Y, int B, hipStream_t st) {
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  dim3 grid(cdiv(g.L, kTile), (unsigned)g.nt, cdiv(C, kCh));
  hipLaunchKernelGGL(k_pad_sino, grid, dim3(256), 0, st, y, Y, B, g.nt, g.np, g.L, C, g.cdet);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

}  // namespace tomo
