// Normal operator A^T A (or A^T D A) in the reduced form that Sec. 4 proposes as the Toeplitz
// approach: with as many detector bins as polar samples per angle, the crop (a circular shift by
// the axis bin's integer part) is a bijection and a fractional part's phase ramp is unitary, so
// the 1D inverse transform followed by its adjoint is 1/L times the identity, and
//     A^T D A x = (1/L) k* . F2D^H W F2D (k* . x),   W = S diag(D) S^dagger.
// W connects Cartesian frequencies that share a polar sample: a fixed (2R+1)^2 stencil with
// per-point weights (R = kw - 1), stored as values only (no column indices).
//
// The kernel works on the 2D FFT's own channel-slowest buffers In/Out[C][G][G] (FFT-ordered),
// so no layout transpose is needed around it.  One thread per grid point: its weights are read
// once (16-byte loads of the zero-padded row) and reused for every channel; lanes run along j2
// so every tap load is coalesced, and the overlapping taps of neighbouring lanes and rows are
// served by L1/L2.  Points whose weights are all zero (outside the sampled disk) write zeros.

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tomo {
namespace {

constexpr int kNormBlock = 256;

struct bf16_t { uint16_t bits; };

template <int S2>
__device__ __forceinline__ void load_weights(const float* row, float (&wt)[S2]) {
#pragma unroll
  for (int q = 0; q < (S2 + 3) / 4; ++q) {
    const float4 v = reinterpret_cast<const float4*>(row)[q];
    const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (4 * q + k < S2) wt[4 * q + k] = e[k];
  }
}

template <int S2>
__device__ __forceinline__ void load_weights(const bf16_t* row, float (&wt)[S2]) {
#pragma unroll
  for (int q = 0; q < (S2 + 7) / 8; ++q) {
    const uint4 v = reinterpret_cast<const uint4*>(row)[q];
    const uint32_t e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (8 * q + k < S2)
        wt[8 * q + k] = __uint_as_float((k & 1) ? (e[k >> 1] & 0xFFFF0000u) : (e[k >> 1] << 16));
  }
}

template <int S2>
__device__ __forceinline__ void load_weights(const _Float16* row, float (&wt)[S2]) {
#pragma unroll
  for (int q = 0; q < (S2 + 7) / 8; ++q) {
    const uint4 v = reinterpret_cast<const uint4*>(row)[q];
    const uint32_t e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (8 * q + k < S2) {
        const uint16_t h = (uint16_t)((k & 1) ? (e[k >> 1] >> 16) : (e[k >> 1] & 0xFFFFu));
        wt[8 * q + k] = (float)*reinterpret_cast<const _Float16*>(&h);
      }
  }
}

template <typename V, int R>
__global__ __launch_bounds__(kNormBlock) void k_normal(const V* __restrict__ w, int stride,
                                                       const float2* __restrict__ in,
                                                       float2* __restrict__ out, int G, int C) {
  constexpr int D = 2 * R + 1, S2 = D * D;
  const int64_t M = (int64_t)G * G;
  const int64_t j = xcd_remap(blockIdx.x, gridDim.x) * kNormBlock + threadIdx.x;
  if (j >= M) return;
  const int j1 = (int)(j / G), j2 = (int)(j - (int64_t)j1 * G);
  float wt[S2];
  load_weights<S2>(w + j * stride, wt);
  bool any = false;
#pragma unroll
  for (int o = 0; o < S2; ++o) any |= (wt[o] != 0.f);
  if (!any) {
    for (int c = 0; c < C; ++c) out[(int64_t)c * M + j] = make_float2(0.f, 0.f);
    return;
  }
  int r1[D], c2[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int v = j1 + a - R;
    v += (v < 0) ? G : 0;
    v -= (v >= G) ? G : 0;
    r1[a] = v * G;
    int u = j2 + a - R;
    u += (u < 0) ? G : 0;
    u -= (u >= G) ? G : 0;
    c2[a] = u;
  }
  for (int c = 0; c < C; ++c) {
    const float2* src = in + (int64_t)c * M;
    float ax = 0.f, ay = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const float2 v = src[r1[a] + c2[b]];
        ax += wt[a * D + b] * v.x;
        ay += wt[a * D + b] * v.y;
      }
    out[(int64_t)c * M + j] = make_float2(ax, ay);
  }
}

// LDS-staged variant: a block owns a kTY x kTX tile of grid points (two adjacent points along j2
// per thread) and walks the channels; for each channel the tile plus an R-wide halo is staged in
// LDS (double-buffered: the next channel's loads are issued before the current one is used), so
// HBM and L2 see each grid value about once and the taps become aligned 16-byte LDS reads.
// The weights of a thread's two points stay in registers for all channels.  A tile whose
// weights are all zero (outside the sampled disk) writes zeros and stages nothing.
constexpr int kTY = 16, kTX = 32;

template <typename V, int R>
__global__ __launch_bounds__(kNormBlock) void k_normal_tiled(const V* __restrict__ w, int stride,
                                                             const float2* __restrict__ in,
                                                             float2* __restrict__ out, int G,
                                                             int C, int tiles_x) {
  constexpr int D = 2 * R + 1, S2 = D * D;
  constexpr int LW = kTX + 2 * R, LH = kTY + 2 * R, NL = LW * LH;
  constexpr int PER = (NL + kNormBlock - 1) / kNormBlock;
  __shared__ __align__(16) float2 buf[2][NL];
  const int64_t M = (int64_t)G * G;
  const int tile = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int j1_0 = (tile / tiles_x) * kTY, j2_0 = (tile % tiles_x) * kTX;
  const int ty = threadIdx.x / (kTX / 2), tx = threadIdx.x % (kTX / 2);
  const int j1 = j1_0 + ty;
  const int j2 = j2_0 + 2 * tx;
  const bool ok0 = j1 < G && j2 < G, ok1 = j1 < G && j2 + 1 < G;
  float wt[2][S2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const bool okp = p ? ok1 : ok0;
    if (okp) {
      load_weights<S2>(w + ((int64_t)j1 * G + j2 + p) * stride, wt[p]);
    } else {
#pragma unroll
      for (int o = 0; o < S2; ++o) wt[p][o] = 0.f;
    }
  }
  bool any = false;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int o = 0; o < S2; ++o) any |= (wt[p][o] != 0.f);
  if (!__syncthreads_or(any)) {
    for (int c = 0; c < C; ++c) {
      if (ok0) out[(int64_t)c * M + (int64_t)j1 * G + j2] = make_float2(0.f, 0.f);
      if (ok1) out[(int64_t)c * M + (int64_t)j1 * G + j2 + 1] = make_float2(0.f, 0.f);
    }
    return;
  }
  // staging slots of this thread: halo position -> wrapped global offset within a channel
  int src[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int q = threadIdx.x + k * kNormBlock;
    src[k] = -1;
    if (q < NL) {
      int g1 = (j1_0 - R + q / LW) % G;
      int g2 = (j2_0 - R + q % LW) % G;
      g1 += (g1 < 0) ? G : 0;
      g2 += (g2 < 0) ? G : 0;
      src[k] = g1 * G + g2;
    }
  }
  float2 stage[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (src[k] >= 0) stage[k] = in[src[k]];
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (src[k] >= 0) buf[0][threadIdx.x + k * kNormBlock] = stage[k];
  __syncthreads();
  for (int c = 0; c < C; ++c) {
    const int b = c & 1;
    if (c + 1 < C) {
      const float2* nxt = in + (int64_t)(c + 1) * M;
#pragma unroll
      for (int k = 0; k < PER; ++k)
        if (src[k] >= 0) stage[k] = nxt[src[k]];
    }
    float a0x = 0.f, a0y = 0.f, a1x = 0.f, a1y = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const float4* row = reinterpret_cast<const float4*>(&buf[b][(ty + a) * LW + 2 * tx]);
      float v[2 * D + 2];
#pragma unroll
      for (int h = 0; h < R + 1; ++h) {
        const float4 q = row[h];
        v[4 * h] = q.x; v[4 * h + 1] = q.y; v[4 * h + 2] = q.z; v[4 * h + 3] = q.w;
      }
#pragma unroll
      for (int bb = 0; bb < D; ++bb) {
        a0x += wt[0][a * D + bb] * v[2 * bb];
        a0y += wt[0][a * D + bb] * v[2 * bb + 1];
        a1x += wt[1][a * D + bb] * v[2 * bb + 2];
        a1y += wt[1][a * D + bb] * v[2 * bb + 3];
      }
    }
    float2* o = out + (int64_t)c * M + (int64_t)j1 * G + j2;
    if (ok0) o[0] = make_float2(a0x, a0y);
    if (ok1) o[1] = make_float2(a1x, a1y);
    if (c + 1 < C) {
#pragma unroll
      for (int k = 0; k < PER; ++k)
        if (src[k] >= 0) buf[b ^ 1][threadIdx.x + k * kNormBlock] = stage[k];
    }
    __syncthreads();
  }
}

template <typename V>
tomo_status normal_impl(const tomo_op* op, const void* w, const float2* in, float2* out, int C,
                        hipStream_t st) {
  const int G = op->g.G;
  const int64_t M = (int64_t)G * G;
  const dim3 grid((unsigned)((M + kNormBlock - 1) / kNormBlock));
  const int stride = op->nrm.stride;
  if (op->tune.normal_tiled && op->nrm.R <= 2) {
    const int tiles_x = (G + kTX - 1) / kTX, tiles_y = (G + kTY - 1) / kTY;
    const dim3 tgrid((unsigned)(tiles_x * tiles_y));
    if (op->nrm.R == 2)
      hipLaunchKernelGGL((k_normal_tiled<V, 2>), tgrid, dim3(kNormBlock), 0, st, (const V*)w,
                         stride, in, out, G, C, tiles_x);
    else
      hipLaunchKernelGGL((k_normal_tiled<V, 0>), tgrid, dim3(kNormBlock), 0, st, (const V*)w,
                         stride, in, out, G, C, tiles_x);
    TOMO_HIP(hipGetLastError());
    return TOMO_OK;
  }
  switch (op->nrm.R) {
    case 0:
      hipLaunchKernelGGL((k_normal<V, 0>), grid, dim3(kNormBlock), 0, st, (const V*)w, stride, in,
                         out, G, C);
      break;
    case 2:
      hipLaunchKernelGGL((k_normal<V, 2>), grid, dim3(kNormBlock), 0, st, (const V*)w, stride, in,
                         out, G, C);
      break;
    case 4:
      hipLaunchKernelGGL((k_normal<V, 4>), grid, dim3(kNormBlock), 0, st, (const V*)w, stride, in,
                         out, G, C);
      break;
    default:
      return fail(TOMO_EUNSUPPORTED, "normal operator needs kw <= 5 (kw=%d)", op->g.kw);
  }
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

}  // namespace

tomo_status launch_normal_stencil(const tomo_op* op, const float2* in, float2* out, int C, int vt,
                                  int filter, hipStream_t st) {
  if (filter < 0 || filter > 3 || vt < 0 || vt > 2 || !op->nrm.val[filter][vt])
    return fail(TOMO_ESTATE, "normal-operator stencil (filter %d, values %d) not built", filter, vt);
  // every value type's stencil is stored in float32 (the normal operator of the matrix with that
  // value type; see ensure_normal)
  return normal_impl<float>(op, op->nrm.val[filter][vt], in, out, C, st);
}

}  // namespace tomo
