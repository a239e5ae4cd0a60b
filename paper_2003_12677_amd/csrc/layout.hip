// Streaming kernels around the FFTs (Sec. 3 Eq. (2)): pairing of real slices into complex
// channels (Sec. 3.1: channel c = slice 2c + i slice 2c+1), deapodisation, the index shifts that
// put the image origin and the rotation axis at index 0 (so plain FFTs compute the centred
// transforms), zero padding and cropping.
//
// The FFTs run on channel-slowest buffers (Xs[C][G][G], Ys[C][nt][L]: contiguous batched
// transforms), the SpMMs on channel-fastest ones (X[G*G][C], Y[L*nt][C]: one cache line per
// gathered column), so LDS-tiled transposes convert between the two.

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tomo {
namespace {

constexpr int kTP = 64;    // points per transpose tile
constexpr int kTC = 16;    // channels per transpose tile

// x[B][n][n] -> Xs[C][G][G]:  Xs[c][(i1-on) mod G][(i2-on) mod G] = kd[i1] kd[i2] (x[2c] + i x[2c+1])
__global__ __launch_bounds__(256) void k_embed(const float* __restrict__ x, float2* __restrict__ Xs,
                                               const float* __restrict__ kd, int B, int n, int G,
                                               int on) {
  const int g2 = blockIdx.x * 256 + threadIdx.x;
  const int g1 = blockIdx.y, c = blockIdx.z;
  if (g2 >= G) return;
  int i1 = g1 + on, i2 = g2 + on;
  if (i1 >= G) i1 -= G;
  if (i2 >= G) i2 -= G;
  float2 v = make_float2(0.f, 0.f);
  if (i1 < n && i2 < n) {
    const float k = kd[i1] * kd[i2];
    const int64_t off = (int64_t)i1 * n + i2;
    v.x = x[(int64_t)(2 * c) * n * n + off] * k;
    if (2 * c + 1 < B) v.y = x[(int64_t)(2 * c + 1) * n * n + off] * k;
  }
  Xs[((int64_t)c * G + g1) * G + g2] = v;
}

// Xs[C][G][G] -> x[B][n][n]:  x[s][i1][i2] = scale kd[i1] kd[i2] part_s(Xs[s/2][(i1-on) mod G][(i2-on) mod G])
__global__ __launch_bounds__(256) void k_crop_image(const float2* __restrict__ Xs, float* __restrict__ x,
                                                    const float* __restrict__ kd, int B, int n, int G,
                                                    int on, float scale) {
  const int i2 = blockIdx.x * 256 + threadIdx.x;
  const int i1 = blockIdx.y, c = blockIdx.z;
  if (i2 >= n) return;
  int g1 = i1 - on, g2 = i2 - on;
  if (g1 < 0) g1 += G;
  if (g2 < 0) g2 += G;
  const float2 v = Xs[((int64_t)c * G + g1) * G + g2];
  const float k = scale * kd[i1] * kd[i2];
  const int64_t off = (int64_t)i1 * n + i2;
  x[(int64_t)(2 * c) * n * n + off] = v.x * k;
  if (2 * c + 1 < B) x[(int64_t)(2 * c + 1) * n * n + off] = v.y * k;
}

// Ys[C][nt][L] -> y[B][nt][np]:  y[s][a][b] = scale part_s(Ys[s/2][a][(b - cdet) mod L])
__global__ __launch_bounds__(256) void k_crop_sino(const float2* __restrict__ Ys, float* __restrict__ y,
                                                   int B, int nt, int np, int L, int cdet, float scale) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  const int a = blockIdx.y, c = blockIdx.z;
  if (b >= np) return;
  int m = (b - cdet) % L;
  if (m < 0) m += L;
  const float2 v = Ys[((int64_t)c * nt + a) * L + m];
  const int64_t off = (int64_t)a * np + b;
  y[(int64_t)(2 * c) * nt * np + off] = v.x * scale;
  if (2 * c + 1 < B) y[(int64_t)(2 * c + 1) * nt * np + off] = v.y * scale;
}

// y[B][nt][np] -> Ys[C][nt][L]:  Ys[c][a][m] = y[2c][a][b] + i y[2c+1][a][b], b = (m + cdet) mod L
// (zero where b >= np or the slice does not exist)
__global__ __launch_bounds__(256) void k_pad_sino(const float* __restrict__ y, float2* __restrict__ Ys,
                                                  int B, int nt, int np, int L, int cdet) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  const int a = blockIdx.y, c = blockIdx.z;
  if (m >= L) return;
  int b = m + cdet;
  if (b >= L) b -= L;
  float2 v = make_float2(0.f, 0.f);
  if (b < np) {
    const int64_t off = (int64_t)a * np + b;
    v.x = y[(int64_t)(2 * c) * nt * np + off];
    if (2 * c + 1 < B) v.y = y[(int64_t)(2 * c + 1) * nt * np + off];
  }
  Ys[((int64_t)c * nt + a) * L + m] = v;
}

// Y[p][c] *= w[p] (a per-row diagonal on a channel-fastest buffer)
__global__ __launch_bounds__(256) void k_scale_rows(float2* __restrict__ Y, const float* __restrict__ w,
                                                    int64_t total, int C) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const float s = w[i / C];
    const float2 v = Y[i];
    Y[i] = make_float2(v.x * s, v.y * s);
  }
}

// a[C][P] -> b[P][C], tiles of 64 points x 16 channels through LDS
__global__ __launch_bounds__(256) void k_to_fastest(const float2* __restrict__ a, float2* __restrict__ b,
                                                    int64_t P, int C) {
  __shared__ float2 tile[kTC][kTP + 1];
  const int64_t p0 = (int64_t)blockIdx.x * kTP;
  const int c0 = blockIdx.y * kTC;
  const int nc = min(kTC, C - c0);
  const int np = (int)min((int64_t)kTP, P - p0);
  for (int i = threadIdx.x; i < kTC * kTP; i += 256) {
    const int c = i / kTP, p = i % kTP;
    if (c < nc && p < np) tile[c][p] = a[(int64_t)(c0 + c) * P + p0 + p];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < np * nc; i += 256) {
    const int p = i / nc, c = i % nc;
    b[(p0 + p) * C + c0 + c] = tile[c][p];
  }
}

// b[P][C] -> a[C][P]
__global__ __launch_bounds__(256) void k_to_slowest(const float2* __restrict__ b, float2* __restrict__ a,
                                                    int64_t P, int C) {
  __shared__ float2 tile[kTC][kTP + 1];
  const int64_t p0 = (int64_t)blockIdx.x * kTP;
  const int c0 = blockIdx.y * kTC;
  const int nc = min(kTC, C - c0);
  const int np = (int)min((int64_t)kTP, P - p0);
  for (int i = threadIdx.x; i < np * nc; i += 256) {
    const int p = i / nc, c = i % nc;
    tile[c][p] = b[(p0 + p) * C + c0 + c];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kTC * kTP; i += 256) {
    const int c = i / kTP, p = i % kTP;
    if (c < nc && p < np) a[(int64_t)(c0 + c) * P + p0 + p] = tile[c][p];
  }
}

// Yf[kf][a][C] -> Ys[C][a][kf]
__global__ __launch_bounds__(256) void k_polar_to_slowest(const float2* __restrict__ Yf,
                                                          float2* __restrict__ Ys, int L, int nt, int C) {
  __shared__ float2 tile[kTC][kTP + 1];
  const int k0 = blockIdx.x * kTP, a = blockIdx.y, c0 = blockIdx.z * kTC;
  const int nc = min(kTC, C - c0), nk = min(kTP, L - k0);
  for (int i = threadIdx.x; i < nk * nc; i += 256) {
    const int k = i / nc, c = i % nc;
    tile[c][k] = Yf[((int64_t)(k0 + k) * nt + a) * C + c0 + c];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kTC * kTP; i += 256) {
    const int c = i / kTP, k = i % kTP;
    if (c < nc && k < nk) Ys[((int64_t)(c0 + c) * nt + a) * L + k0 + k] = tile[c][k];
  }
}

// Ys[C][a][kf] -> Yf[kf][a][C]
__global__ __launch_bounds__(256) void k_polar_to_fastest(const float2* __restrict__ Ys,
                                                          float2* __restrict__ Yf, int L, int nt, int C) {
  __shared__ float2 tile[kTC][kTP + 1];
  const int k0 = blockIdx.x * kTP, a = blockIdx.y, c0 = blockIdx.z * kTC;
  const int nc = min(kTC, C - c0), nk = min(kTP, L - k0);
  for (int i = threadIdx.x; i < kTC * kTP; i += 256) {
    const int c = i / kTP, k = i % kTP;
    if (c < nc && k < nk) tile[c][k] = Ys[((int64_t)(c0 + c) * nt + a) * L + k0 + k];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nk * nc; i += 256) {
    const int k = i / nc, c = i % nc;
    Yf[((int64_t)(k0 + k) * nt + a) * C + c0 + c] = tile[c][k];
  }
}

// Ys[r][kf] *= phase[kf] (or its conjugate), rows of length L: a fractional rotation-axis bin's
// phase ramp on the library-FFT path
__global__ __launch_bounds__(256) void k_phase_rows(float2* __restrict__ Ys,
                                                    const float2* __restrict__ phase, int L,
                                                    int64_t total, bool conj) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    float2 p = phase[i % L];
    if (conj) p.y = -p.y;
    const float2 v = Ys[i];
    Ys[i] = make_float2(v.x * p.x - v.y * p.y, v.x * p.y + v.y * p.x);
  }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

tomo_status launch_phase_rows(float2* Ys, const float2* phase, int L, int64_t rows, bool conj,
                              hipStream_t st) {
  const int64_t total = rows * L;
  hipLaunchKernelGGL(k_phase_rows, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65535)),
                     dim3(256), 0, st, Ys, phase, L, total, conj);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_scale_rows(float2* Y, const float* w, int64_t P, int C, hipStream_t st) {
  const int64_t total = P * C;
  hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65535)),
                     dim3(256), 0, st, Y, w, total, C);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_embed(const tomo_op* op, const float* x, float2* Xs, int B, hipStream_t st) {
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  hipLaunchKernelGGL(k_embed, dim3(cdiv(g.G, 256), (unsigned)g.G, (unsigned)C), dim3(256), 0, st, x,
                     Xs, op->kd_dev, B, g.n, g.G, g.on);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_crop_image(const tomo_op* op, const float2* Xs, float* x, int B, float scale,
                              hipStream_t st) {
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  hipLaunchKernelGGL(k_crop_image, dim3(cdiv(g.n, 256), (unsigned)g.n, (unsigned)C), dim3(256), 0, st,
                     Xs, x, op->kd_dev, B, g.n, g.G, g.on, scale);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_crop_sino(const tomo_op* op, const float2* Ys, float* y, int B, float scale,
                             hipStream_t st) {
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  hipLaunchKernelGGL(k_crop_sino, dim3(cdiv(g.np, 256), (unsigned)g.nt, (unsigned)C), dim3(256), 0,
                     st, Ys, y, B, g.nt, g.np, g.L, g.cdet, scale);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_pad_sino(const tomo_op* op, const float* y, float2* Ys, int B, hipStream_t st) {
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  hipLaunchKernelGGL(k_pad_sino, dim3(cdiv(g.L, 256), (unsigned)g.nt, (unsigned)C), dim3(256), 0, st,
                     y, Ys, B, g.nt, g.np, g.L, g.cdet);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_to_channel_fastest(const float2* src, float2* dst, int64_t P, int C, hipStream_t st) {
  hipLaunchKernelGGL(k_to_fastest, dim3(cdiv(P, kTP), cdiv(C, kTC)), dim3(256), 0, st, src, dst, P, C);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_to_channel_slowest(const float2* src, float2* dst, int64_t P, int C, hipStream_t st) {
  hipLaunchKernelGGL(k_to_slowest, dim3(cdiv(P, kTP), cdiv(C, kTC)), dim3(256), 0, st, src, dst, P, C);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_polar_to_slowest(const float2* Yf, float2* Ys, int L, int nt, int C, hipStream_t st) {
  hipLaunchKernelGGL(k_polar_to_slowest, dim3(cdiv(L, kTP), (unsigned)nt, cdiv(C, kTC)), dim3(256), 0,
                     st, Yf, Ys, L, nt, C);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_polar_to_fastest(const float2* Ys, float2* Yf, int L, int nt, int C, hipStream_t st) {
  hipLaunchKernelGGL(k_polar_to_fastest, dim3(cdiv(L, kTP), (unsigned)nt, cdiv(C, kTC)), dim3(256), 0,
                     st, Ys, Yf, L, nt, C);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

}  // namespace tomo
