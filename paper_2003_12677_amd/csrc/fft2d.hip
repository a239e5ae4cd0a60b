// The Cartesian 2D DFT of Eq. (2) fused with the steps around it, on the channel-slowest grid
// Xs[C][G][G], for a power-of-two grid side G (16..4096), or any other G up to 4096 through
// Bluestein's identity at the power-of-two length M >= 2G - 1 (fft_lds.h):
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

// rows per row block: about 32 KB of LDS, so that four blocks share a CU (M = the transform length
// held in LDS: G itself, or the Bluestein length for other G)
constexpr int rows_per_block(int M) {
  return M >= 8192 ? 1 : (M >= 2048 ? 2 : (4096 / M > 16 ? 16 : 4096 / M));
}

// columns per column block: adjacent columns, each row read and written as one run.  At
// M = 2048, 8 columns (64-byte runs, 135 KB of LDS, one block per CU) beat 4 columns (32-byte
// runs, two blocks per CU): project 1.150 -> 1.128 ms, normal operator 1.517 -> 1.489 ms at
// 2048^2 x 32; 2 columns had taken 510 us per pass against 410 us for 4.  Elsewhere 64 KB.
template <int M>
constexpr int cols_per_block() {
  return M >= 8192 ? 1 : (M >= 4096 ? 2 : (M >= 2048 ? 8 : (8192 / M > 16 ? 16 : 8192 / M)));
}

// The grid side G is t.N: M for power-of-two grids (BL = false), else the DFTs go through
// Bluestein's identity at length M.  Indices below t.N are grid indices; LDS rows have stride M.
// CG (a conjugate-gradient step fused in): x is the search direction p, and before it is
// embedded each pixel takes the deferred step  xsol += alpha[s] p;  p = snew + beta[s] p  (the
// arithmetic of the separate step kernel), both written back in place; the new p is transformed.
template <int M, int AG, bool BL, bool CG>
__global__ __launch_bounds__(kFB) void k_rows_embed(const float* x, float* pout,
                                                    float* __restrict__ xsol,
                                                    const float* __restrict__ snew,
                                                    const double* __restrict__ alpha,
                                                    const double* __restrict__ beta,
                                                    float2* __restrict__ Xs,
                                                    const float* __restrict__ kd, DftTables t,
                                                    int B, int n, int on) {
  __shared__ float2 buf[lds_size<AG * M>()];
  const int G = BL ? t.N : M;
  const int groups = (G + AG - 1) / AG;
  // elements per thread, loaded as one batch (all loads issued before the first LDS store)
  constexpr int NE = (AG * M + kFB - 1) / kFB;
  const int c = blockIdx.x / groups, g1_0 = (blockIdx.x % groups) * AG;
  const int64_t plane = (int64_t)n * n;
  const bool odd = 2 * c + 1 < B;
  float re[NE], im[NE], kk[NE];
  float sr[CG ? NE : 1], si[CG ? NE : 1], xr[CG ? NE : 1], xi[CG ? NE : 1];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int i = threadIdx.x + u * kFB;
    const int q = i / M, g2 = i % M;
    int i1 = g1_0 + q + on, i2 = g2 + on;          // pixel (i1, i2) sits at grid (i - on) mod G
    i1 -= (i1 >= G) ? G : 0;
    i2 -= (i2 >= G) ? G : 0;
    re[u] = 0.f;
    im[u] = 0.f;
    kk[u] = 0.f;
    if (i < AG * M && g1_0 + q < G && g2 < G && i1 < n && i2 < n) {
      const int64_t off = (int64_t)i1 * n + i2;
      kk[u] = kd[i1] * kd[i2];
      re[u] = x[(int64_t)(2 * c) * plane + off];
      if (odd) im[u] = x[(int64_t)(2 * c + 1) * plane + off];
      if constexpr (CG) {
        sr[u] = snew[(int64_t)(2 * c) * plane + off];
        xr[u] = xsol[(int64_t)(2 * c) * plane + off];
        if (odd) {
          si[u] = snew[(int64_t)(2 * c + 1) * plane + off];
          xi[u] = xsol[(int64_t)(2 * c + 1) * plane + off];
        }
      }
    }
  }
  if constexpr (CG) {
    const float fa0 = (float)alpha[2 * c], fb0 = (float)beta[2 * c];
    const float fa1 = odd ? (float)alpha[2 * c + 1] : 0.f, fb1 = odd ? (float)beta[2 * c + 1] : 0.f;
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      const int q = i / M, g2 = i % M;
      int i1 = g1_0 + q + on, i2 = g2 + on;
      i1 -= (i1 >= G) ? G : 0;
      i2 -= (i2 >= G) ? G : 0;
      if (i < AG * M && g1_0 + q < G && g2 < G && i1 < n && i2 < n) {
        const int64_t off = (int64_t)i1 * n + i2;
        float xv = 1.0f * xr[u];
        xv += fa0 * re[u];
        xsol[(int64_t)(2 * c) * plane + off] = xv;
        float nv = 1.0f * sr[u];
        nv += fb0 * re[u];
        pout[(int64_t)(2 * c) * plane + off] = nv;
        re[u] = nv;
        if (odd) {
          float xw = 1.0f * xi[u];
          xw += fa1 * im[u];
          xsol[(int64_t)(2 * c + 1) * plane + off] = xw;
          float nw = 1.0f * si[u];
          nw += fb1 * im[u];
          pout[(int64_t)(2 * c + 1) * plane + off] = nw;
          im[u] = nw;
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int i = threadIdx.x + u * kFB;
    if (i < AG * M) buf[lds(i)] = make_float2(re[u] * kk[u], im[u] * kk[u]);
  }
  __syncthreads();
  dft_lds<M, AG, false, BL>(buf, t);
  const int nq = min(AG, G - g1_0);
  float2* dst = Xs + ((int64_t)c * G + g1_0) * G;
  for (int i = threadIdx.x; i < nq * G; i += kFB) dst[i] = buf[lds((i / G) * M + i % G)];
}

template <int M, int W, bool INV, bool BL>
__global__ __launch_bounds__(kFB) void k_cols(float2* __restrict__ Xs, DftTables t) {
  __shared__ float2 buf[lds_size<W * M>()];
  const int G = BL ? t.N : M;
  const int groups = (G + W - 1) / W;
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  const int c = (int)(blk / groups), j2_0 = (int)(blk % groups) * W;
  const int nw = min(W, G - j2_0);
  float2* base = Xs + (int64_t)c * G * G + j2_0;
  {
    constexpr int NE = (W * M + kFB - 1) / kFB;   // loads per thread, issued as one batch
    float2 v[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      const int g1 = i / W, w = i % W;
      v[u] = make_float2(0.f, 0.f);
      if (i < W * M && g1 < G && w < nw) v[u] = base[(int64_t)g1 * G + w];
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      if (i < W * M) buf[lds((i % W) * M + i / W)] = v[u];
    }
  }
  __syncthreads();
  dft_lds<M, W, INV, BL>(buf, t);
  for (int i = threadIdx.x; i < W * G; i += kFB) {
    const int g1 = i / W, w = i % W;
    if (w < nw) base[(int64_t)g1 * G + w] = buf[lds(w * M + g1)];
  }
}

// With sumsq set, the block also sums the squares of the values it writes (float64), per slice:
// sumsq[s * groups + j] for its group j of grid rows; with dotw set as well, the products of the
// values with dotw (same layout as x) instead of their squares.
template <int M, int AG, bool BL>
__global__ __launch_bounds__(kFB) void k_rows_inv_crop(const float2* __restrict__ Xs,
                                                       float* __restrict__ x,
                                                       const float* __restrict__ kd, DftTables t,
                                                       int B, int n, int on, float scale,
                                                       double* __restrict__ sumsq,
                                                       const float* __restrict__ dotw) {
  __shared__ float2 buf[lds_size<AG * M>()];
  const int G = BL ? t.N : M;
  const int groups = (G + AG - 1) / AG;
  const int c = blockIdx.x / groups, g1_0 = (blockIdx.x % groups) * AG;
  const int nq = min(AG, G - g1_0);
  const float2* src = Xs + ((int64_t)c * G + g1_0) * G;
  {
    constexpr int NE = (AG * M + kFB - 1) / kFB;  // loads per thread, issued as one batch
    float2 v[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      const int q = i / M, g2 = i % M;
      v[u] = make_float2(0.f, 0.f);
      if (i < AG * M && q < nq && g2 < G) v[u] = src[(int64_t)q * G + g2];
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      if (i < AG * M) buf[lds(i)] = v[u];
    }
  }
  __syncthreads();
  dft_lds<M, AG, true, BL>(buf, t);
  const int64_t plane = (int64_t)n * n;
  const bool odd = 2 * c + 1 < B;
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < nq * n; i += kFB) {
    const int q = i / n, i2 = i % n;
    int i1 = g1_0 + q + on;
    i1 -= (i1 >= G) ? G : 0;
    if (i1 >= n) continue;
    const int g2 = i2 - on + ((i2 < on) ? G : 0);
    const float2 v = buf[lds(q * M + g2)];
    const float k = scale * kd[i1] * kd[i2];
    const int64_t off = (int64_t)i1 * n + i2;
    const float re = v.x * k, im = v.y * k;
    x[(int64_t)(2 * c) * plane + off] = re;
    if (odd) x[(int64_t)(2 * c + 1) * plane + off] = im;
    if (dotw) {
      s0 += (double)re * (double)dotw[(int64_t)(2 * c) * plane + off];
      if (odd) s1 += (double)im * (double)dotw[(int64_t)(2 * c + 1) * plane + off];
    } else {
      s0 += (double)re * (double)re;
      s1 += (double)im * (double)im;
    }
  }
  if (sumsq) {
    block_sum2(s0, s1);
    if (threadIdx.x == 0) {
      const int j = blockIdx.x % groups;
      sumsq[(int64_t)(2 * c) * groups + j] = s0;
      if (odd) sumsq[(int64_t)(2 * c + 1) * groups + j] = s1;
    }
  }
}

enum class Step { RowsEmbed, ColsFwd, ColsInv, RowsInvCrop };

constexpr int kMaxCgStepM = 2048;

template <int M, bool BL>
tomo_status grid_launch(Step s, const tomo_op* op, const float* xin, float2* Xs, float* xout,
                        int B, float scale, double* sumsq, const float* dotw, const CgStep* cg,
                        hipStream_t st) {
  constexpr int AG = rows_per_block(M), W = cols_per_block<M>();
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  const DftTables& t = op->dft2;
  const int G = g.G;
  const dim3 grid((unsigned)(C * ((G + AG - 1) / AG))), cgrid((unsigned)(C * ((G + W - 1) / W)));
  switch (s) {
    case Step::RowsEmbed:
      if (cg) {
        // the fused step's extra loads fit the registers up to M = 2048 (kMaxCgStepM)
        if constexpr (M <= kMaxCgStepM)
          hipLaunchKernelGGL((k_rows_embed<M, AG, BL, true>), grid, dim3(kFB), 0, st, xin,
                             const_cast<float*>(xin), cg->x, cg->s, cg->alpha, cg->beta, Xs,
                             op->kd_dev, t, B, g.n, g.on);
        else
          return fail(TOMO_EINVAL, "internal: fused CG step for transform length %d", M);
      } else
        hipLaunchKernelGGL((k_rows_embed<M, AG, BL, false>), grid, dim3(kFB), 0, st, xin, nullptr,
                           nullptr, nullptr, nullptr, nullptr, Xs, op->kd_dev, t, B, g.n, g.on);
      break;
    case Step::ColsFwd:
      hipLaunchKernelGGL((k_cols<M, W, false, BL>), cgrid, dim3(kFB), 0, st, Xs, t);
      break;
    case Step::ColsInv:
      hipLaunchKernelGGL((k_cols<M, W, true, BL>), cgrid, dim3(kFB), 0, st, Xs, t);
      break;
    case Step::RowsInvCrop:
      hipLaunchKernelGGL((k_rows_inv_crop<M, AG, BL>), grid, dim3(kFB), 0, st, Xs, xout, op->kd_dev,
                         t, B, g.n, g.on, scale, sumsq, sumsq ? dotw : nullptr);
      break;
  }
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status grid_dispatch(Step s, const tomo_op* op, const float* xin, float2* Xs, float* xout,
                          int B, float scale, double* sumsq, const float* dotw, const CgStep* cg,
                          hipStream_t st) {
  const bool bl = op->dft2.M != op->g.G;
#define TOMO_GRID(M_)                                                                            \
  case M_:                                                                                      \
    return bl ? grid_launch<M_, true>(s, op, xin, Xs, xout, B, scale, sumsq, dotw, cg, st)      \
              : grid_launch<M_, false>(s, op, xin, Xs, xout, B, scale, sumsq, dotw, cg, st);
  switch (op->dft2.M) {
    TOMO_GRID(16) TOMO_GRID(32) TOMO_GRID(64) TOMO_GRID(128) TOMO_GRID(256) TOMO_GRID(512)
    TOMO_GRID(1024) TOMO_GRID(2048) TOMO_GRID(4096) TOMO_GRID(8192)
    default: return fail(TOMO_EUNSUPPORTED, "hand-written grid DFT: no kernel for length %d", op->dft2.M);
  }
#undef TOMO_GRID
}

}  // namespace

bool grid_fft_supported(const tomo_op* op) { return op->dft2.tw != nullptr; }

bool grid_cg_step_supported(const tomo_op* op) {
  return grid_fft_supported(op) && op->dft2.M <= kMaxCgStepM;
}

int64_t grid_inverse_blocks_per_channel(const tomo_op* op) {
  if (!grid_fft_supported(op)) return 0;
  const int ag = rows_per_block(op->dft2.M);
  return (op->g.G + ag - 1) / ag;
}

tomo_status launch_grid_forward(const tomo_op* op, const float* x, float2* Xs, int B,
                                hipStream_t st, const CgStep* cg) {
  TOMO_TRY(grid_dispatch(Step::RowsEmbed, op, x, Xs, nullptr, B, 1.f, nullptr, nullptr, cg, st));
  return grid_dispatch(Step::ColsFwd, op, nullptr, Xs, nullptr, B, 1.f, nullptr, nullptr, nullptr, st);
}

tomo_status launch_grid_inverse(const tomo_op* op, float2* Xs, float* x, int B, float scale,
                                double* sumsq, hipStream_t st, const float* dotw) {
  TOMO_TRY(grid_dispatch(Step::ColsInv, op, nullptr, Xs, nullptr, B, 1.f, nullptr, nullptr, nullptr, st));
  return grid_dispatch(Step::RowsInvCrop, op, nullptr, Xs, x, B, scale, sumsq, dotw, nullptr, st);
}

}  // namespace tomo
