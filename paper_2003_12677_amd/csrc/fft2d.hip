// The Cartesian 2D DFT of Eq. (2) fused with the steps around it, for a power-of-two grid side
// G (16..4096), on the channel-slowest grid Xs[C][G][G]:
//
//   k_rows_embed     x[B][n][n] -> deapodise (k*), centre (pixel i at grid index (i - n/2) mod
//                    G), pair slices 2c / 2c+1 into channel c, zero padding -> DFT of each grid
//                    row (along j2);
//   k_cols           DFT (or inverse) of each grid column (along j1), in place;
//   k_rows_inv_crop  inverse DFT of each grid row -> crop to the image, k*, scale, split the
//                    channel into its two slices.
//
// Rows: one block per (channel, AG consecutive rows), a contiguous stretch of memory.  Columns:
// one block per (channel, W adjacent columns); the W columns of a row are read and written as
// one short run, and blocks of neighbouring column groups are placed on the same XCD so that
// the rest of each cache line is still in that XCD's L2 when its neighbour reads it.  The DFTs
// run in LDS (radix-8 Stockham, fft_lds.h).  With rocFFT the same work takes an embed kernel,
// a row pass, two transposes and a column pass (and an inverse plus a crop kernel).

#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "internal.h"

namespace tomo {
namespace {

using namespace fftk;

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t x = bid & 7, local = bid >> 3;
  const int64_t q = nblocks >> 3, r = nblocks & 7;
  return (x < r) ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// rows per row block: about 32 KB of LDS, so that four blocks share a CU
template <int G>
constexpr int rows_per_block() {
  return G >= 2048 ? 2 : (4096 / G > 16 ? 16 : 4096 / G);
}

// columns per column block: 4 adjacent columns (32-byte runs of a row) while they fit 64 KB
// (measured at G = 2048: 2 columns with twice the blocks per CU took 510 us, 4 columns 410 us)
template <int G>
constexpr int cols_per_block() {
  return G >= 4096 ? 2 : (G >= 2048 ? 4 : (8192 / G > 16 ? 16 : 8192 / G));
}

template <int G, int AG>
__global__ __launch_bounds__(kFB) void k_rows_embed(const float* __restrict__ x,
                                                    float2* __restrict__ Xs,
                                                    const float* __restrict__ kd,
                                                    const float2* __restrict__ tw, int B, int n,
                                                    int on) {
  __shared__ float2 buf[lds_size<AG * G>()];
  constexpr int groups = G / AG;
  // elements per thread, loaded as one batch (all loads issued before the first LDS store)
  constexpr int NE = (AG * G + kFB - 1) / kFB;
  const int c = blockIdx.x / groups, g1_0 = (blockIdx.x % groups) * AG;
  const int64_t plane = (int64_t)n * n;
  const bool odd = 2 * c + 1 < B;
  float re[NE], im[NE], kk[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int i = threadIdx.x + u * kFB;
    const int q = i / G, g2 = i % G;
    const int i1 = (g1_0 + q + on) & (G - 1), i2 = (g2 + on) & (G - 1);
    re[u] = 0.f;
    im[u] = 0.f;
    kk[u] = 0.f;
    if (i < AG * G && i1 < n && i2 < n) {
      const int64_t off = (int64_t)i1 * n + i2;
      kk[u] = kd[i1] * kd[i2];
      re[u] = x[(int64_t)(2 * c) * plane + off];
      if (odd) im[u] = x[(int64_t)(2 * c + 1) * plane + off];
    }
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int i = threadIdx.x + u * kFB;
    if (i < AG * G) buf[lds(i)] = make_float2(re[u] * kk[u], im[u] * kk[u]);
  }
  __syncthreads();
  fft_lds<G, AG, false>(buf, tw);
  float2* dst = Xs + ((int64_t)c * G + g1_0) * G;
  for (int i = threadIdx.x; i < AG * G; i += kFB) dst[i] = buf[lds(i)];
}

template <int G, int W, bool INV>
__global__ __launch_bounds__(kFB) void k_cols(float2* __restrict__ Xs,
                                              const float2* __restrict__ tw) {
  __shared__ float2 buf[lds_size<W * G>()];
  constexpr int groups = G / W;
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  const int c = (int)(blk / groups), j2_0 = (int)(blk % groups) * W;
  float2* base = Xs + (int64_t)c * G * G + j2_0;
  {
    constexpr int NE = (W * G + kFB - 1) / kFB;   // loads per thread, issued as one batch
    float2 v[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      if (i < W * G) v[u] = base[(int64_t)(i / W) * G + i % W];
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      if (i < W * G) buf[lds((i % W) * G + i / W)] = v[u];
    }
  }
  __syncthreads();
  fft_lds<G, W, INV>(buf, tw);
  for (int i = threadIdx.x; i < W * G; i += kFB) {
    const int g1 = i / W, w = i % W;
    base[(int64_t)g1 * G + w] = buf[lds(w * G + g1)];
  }
}

template <int G, int AG>
__global__ __launch_bounds__(kFB) void k_rows_inv_crop(const float2* __restrict__ Xs,
                                                       float* __restrict__ x,
                                                       const float* __restrict__ kd,
                                                       const float2* __restrict__ tw, int B,
                                                       int n, int on, float scale) {
  __shared__ float2 buf[lds_size<AG * G>()];
  constexpr int groups = G / AG;
  const int c = blockIdx.x / groups, g1_0 = (blockIdx.x % groups) * AG;
  const float2* src = Xs + ((int64_t)c * G + g1_0) * G;
  {
    constexpr int NE = (AG * G + kFB - 1) / kFB;  // loads per thread, issued as one batch
    float2 v[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      if (i < AG * G) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      if (i < AG * G) buf[lds(i)] = v[u];
    }
  }
  __syncthreads();
  fft_lds<G, AG, true>(buf, tw);
  const int64_t plane = (int64_t)n * n;
  const bool odd = 2 * c + 1 < B;
  for (int i = threadIdx.x; i < AG * n; i += kFB) {
    const int q = i / n, i2 = i % n;
    const int i1 = (g1_0 + q + on) & (G - 1);
    if (i1 >= n) continue;
    const float2 v = buf[lds(q * G + ((i2 - on) & (G - 1)))];
    const float k = scale * kd[i1] * kd[i2];
    const int64_t off = (int64_t)i1 * n + i2;
    x[(int64_t)(2 * c) * plane + off] = v.x * k;
    if (odd) x[(int64_t)(2 * c + 1) * plane + off] = v.y * k;
  }
}

enum class Step { RowsEmbed, ColsFwd, ColsInv, RowsInvCrop };

template <int G>
tomo_status grid_launch(Step s, const tomo_op* op, const float* xin, float2* Xs, float* xout,
                        int B, float scale, hipStream_t st) {
  constexpr int AG = rows_per_block<G>(), W = cols_per_block<G>();
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  const dim3 grid((unsigned)(C * (G / AG))), cgrid((unsigned)(C * (G / W)));
  switch (s) {
    case Step::RowsEmbed:
      hipLaunchKernelGGL((k_rows_embed<G, AG>), grid, dim3(kFB), 0, st, xin, Xs, op->kd_dev,
                         op->tw2, B, g.n, g.on);
      break;
    case Step::ColsFwd:
      hipLaunchKernelGGL((k_cols<G, W, false>), cgrid, dim3(kFB), 0, st, Xs, op->tw2);
      break;
    case Step::ColsInv:
      hipLaunchKernelGGL((k_cols<G, W, true>), cgrid, dim3(kFB), 0, st, Xs, op->tw2);
      break;
    case Step::RowsInvCrop:
      hipLaunchKernelGGL((k_rows_inv_crop<G, AG>), grid, dim3(kFB), 0, st, Xs, xout, op->kd_dev,
                         op->tw2, B, g.n, g.on, scale);
      break;
  }
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status grid_dispatch(Step s, const tomo_op* op, const float* xin, float2* Xs, float* xout,
                          int B, float scale, hipStream_t st) {
  switch (op->g.G) {
    case 16: return grid_launch<16>(s, op, xin, Xs, xout, B, scale, st);
    case 32: return grid_launch<32>(s, op, xin, Xs, xout, B, scale, st);
    case 64: return grid_launch<64>(s, op, xin, Xs, xout, B, scale, st);
    case 128: return grid_launch<128>(s, op, xin, Xs, xout, B, scale, st);
    case 256: return grid_launch<256>(s, op, xin, Xs, xout, B, scale, st);
    case 512: return grid_launch<512>(s, op, xin, Xs, xout, B, scale, st);
    case 1024: return grid_launch<1024>(s, op, xin, Xs, xout, B, scale, st);
    case 2048: return grid_launch<2048>(s, op, xin, Xs, xout, B, scale, st);
    case 4096: return grid_launch<4096>(s, op, xin, Xs, xout, B, scale, st);
    default: return fail(TOMO_EUNSUPPORTED, "hand-written grid DFT needs G = 2^m in [16, 4096]");
  }
}

}  // namespace

bool grid_fft_supported(const tomo_op* op) {
  const int G = op->g.G;
  return op->tw2 != nullptr && G >= 16 && G <= 4096 && (G & (G - 1)) == 0;
}

tomo_status launch_grid_forward(const tomo_op* op, const float* x, float2* Xs, int B,
                                hipStream_t st) {
  TOMO_TRY(grid_dispatch(Step::RowsEmbed, op, x, Xs, nullptr, B, 1.f, st));
  return grid_dispatch(Step::ColsFwd, op, nullptr, Xs, nullptr, B, 1.f, st);
}

tomo_status launch_grid_inverse(const tomo_op* op, float2* Xs, float* x, int B, float scale,
                                hipStream_t st) {
  TOMO_TRY(grid_dispatch(Step::ColsInv, op, nullptr, Xs, nullptr, B, 1.f, st));
  return grid_dispatch(Step::RowsInvCrop, op, nullptr, Xs, x, B, scale, st);
}

}  // namespace tomo
