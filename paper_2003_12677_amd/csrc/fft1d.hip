// The detector-direction transforms of Eq. (2) fused with the layout steps around them, for a
// power-of-two number L of polar samples per angle (16..4096), or any other L up to 4096 through
// Bluestein's identity at the power-of-two length M >= 2L - 1 (fft_lds.h):
//
//   project tail:     Ys[C][nt][L] (written by the staged forward SpMM itself, or a tiled
//                     transpose of its channel-fastest output) -> inverse DFT of each row -> rotation-axis
//                     shift, 1/L, crop to n_p bins, real / imaginary parts to slices 2c / 2c+1
//                     of y[B][nt][np];
//   adjoint front:    y[B][nt][np] -> pad to L with the axis shift, slices paired into complex
//                     channels -> forward DFT of each row -> Yf[L][nt][C], the adjoint SpMM's
//                     channel-fastest input (transform lengths up to 4096), or Ys[C][nt][L]
//                     followed by a tiled transpose.
//
// The project tail and the Ys form of the adjoint front take one block per (channel, AG
// consecutive angles), a contiguous stretch of Ys.  The Yf form takes one block per (angle, CW
// channels) and writes each transformed sample's CW channels as one run; the blocks of one angle
// run side by side on one XCD, so their runs meet in its L2 as whole cache lines.  The rows are
// transformed in LDS with radix-8 Stockham passes (plus one radix-4 or radix-2 pass for the
// remaining factor; each pass reads every butterfly's inputs into registers, synchronises, then
// writes its outputs, so one buffer suffices; the twiddle powers of a butterfly are formed by
// multiplication from one table entry).  This replaces a library FFT and a crop / pad kernel by one
// pass over the data.  Writing the channel-fastest layout in 64-byte runs pays (at 2048 bins x
// 1501 angles x 16 channels: 246 us against 138 + 154 us for the row kernel and the transpose);
// reading it in such runs does not (an 8-channel project tail took 302 us against 141 + 153 us),
// so the project tail keeps channel-slowest rows.  Twiddles exp(-2 pi i j / L), j < L, come
// from a table computed in double.

#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "internal.h"

namespace tomo {
namespace {

using namespace fftk;

// Ys[C][nt][L] (channel-slowest rows after the polar transpose) -> inverse DFT of each row ->
// axis shift, scale, crop, slices 2c / 2c+1.  One block per (channel, AG consecutive angles):
// its rows are one contiguous stretch of memory.  L = t.N: M for power-of-two L (BL = false),
// else the DFTs go through Bluestein's identity at length M; LDS rows have stride M.
// With sumsq set, the block also sums the squares of the values it writes (float64), per slice:
// sumsq[s * agroups + j] for its group j of angles.
template <int M, int AG, bool BL>
__global__ __launch_bounds__(kFB) void k_det_inverse_crop(const float2* __restrict__ Ys,
                                                          float* __restrict__ y, DftTables t,
                                                          int B, int nt, int np, int cdet, float scale,
                                                          double* __restrict__ sumsq,
                                                          const float2* __restrict__ phase) {
  __shared__ float2 buf[lds_size<AG * M>()];
  const int L = BL ? t.N : M;
  const int agroups = (nt + AG - 1) / AG;
  const int c = blockIdx.x / agroups, a0 = (blockIdx.x % agroups) * AG;
  const int na = min(AG, nt - a0);
  const float2* src = Ys + ((int64_t)c * nt + a0) * L;
  {
    constexpr int NE = (AG * M + kFB - 1) / kFB;  // loads per thread, issued as one batch
    float2 v[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      const int q = i / M, m = i % M;
      v[u] = make_float2(0.f, 0.f);
      if (i < AG * M && q < na && m < L) v[u] = src[(int64_t)q * L + m];
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      // a fractional axis bin: the polar row's phase ramp before the inverse DFT
      if (phase && i < AG * M && i % M < L) v[u] = cmul(v[u], phase[i % M]);
      if (i < AG * M) buf[lds(i)] = v[u];
    }
  }
  __syncthreads();
  dft_lds<M, AG, true, BL>(buf, t);
  const int64_t plane = (int64_t)nt * np;
  const bool odd = 2 * c + 1 < B;
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < na * np; i += kFB) {
    const int q = i / np, b = i % np;
    int m = b - cdet;                                 // bin b reads radial index (b - c) mod L
    m += (m < 0) ? L : 0;
    const float2 v = buf[lds(q * M + m)];
    const int64_t off = (int64_t)(a0 + q) * np + b;
    const float re = v.x * scale, im = v.y * scale;
    y[(int64_t)(2 * c) * plane + off] = re;
    if (odd) y[(int64_t)(2 * c + 1) * plane + off] = im;
    s0 += (double)re * (double)re;
    s1 += (double)im * (double)im;
  }
  if (sumsq) {
    block_sum2(s0, s1);
    if (threadIdx.x == 0) {
      const int j = blockIdx.x % agroups;
      sumsq[(int64_t)(2 * c) * agroups + j] = s0;
      if (odd) sumsq[(int64_t)(2 * c + 1) * agroups + j] = s1;
    }
  }
}

// y[B][nt][np] -> pad with the axis shift, slices paired -> forward DFT of each row ->
// Ys[C][nt][L] (channel-slowest rows; the polar transpose follows).
template <int M, int AG, bool BL>
__global__ __launch_bounds__(kFB) void k_det_pad_forward(const float* __restrict__ y,
                                                         float2* __restrict__ Ys, DftTables t,
                                                         int B, int nt, int np, int cdet,
                                                         const float2* __restrict__ phase) {
  __shared__ float2 buf[lds_size<AG * M>()];
  const int L = BL ? t.N : M;
  const int agroups = (nt + AG - 1) / AG;
  const int c = blockIdx.x / agroups, a0 = (blockIdx.x % agroups) * AG;
  const int na = min(AG, nt - a0);
  const int64_t plane = (int64_t)nt * np;
  const bool odd = 2 * c + 1 < B;
  // elements per thread, loaded as one batch (all loads issued before the first LDS store)
  constexpr int NE = (AG * M + kFB - 1) / kFB;
  float2 v[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int i = threadIdx.x + u * kFB;
    const int q = i / M, m = i % M;
    int b = m + cdet;                                 // radial index m holds bin (m + c) mod L
    b -= (b >= L) ? L : 0;
    v[u] = make_float2(0.f, 0.f);
    if (i < AG * M && q < na && m < L && b < np) {
      const int64_t off = (int64_t)(a0 + q) * np + b;
      v[u].x = y[(int64_t)(2 * c) * plane + off];
      if (odd) v[u].y = y[(int64_t)(2 * c + 1) * plane + off];
    }
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int i = threadIdx.x + u * kFB;
    if (i < AG * M) buf[lds(i)] = v[u];
  }
  __syncthreads();
  dft_lds<M, AG, false, BL>(buf, t);
  float2* dst = Ys + ((int64_t)c * nt + a0) * L;
  for (int i = threadIdx.x; i < na * L; i += kFB) {
    float2 w = buf[lds((i / L) * M + i % L)];
    if (phase) w = cmul(w, conj2(phase[i % L]));   // a fractional axis bin's phase ramp
    dst[i] = w;
  }
}

// Rows (angles) per block of the channel-slowest kernels: about 32 KB of LDS, so that four blocks
// share a CU.
constexpr int det_rows_per_block(int M) {
  return M >= 8192 ? 1 : (M >= 2048 ? 2 : (4096 / M > 16 ? 16 : 4096 / M));
}

// Channels per block of the Yf form: 8 (64-byte runs) while their rows fit 128 KB of LDS.
template <int M>
constexpr int det_cw() { return M >= 16384 ? 1 : (16384 / M > 8 ? 8 : 16384 / M); }

// y[B][nt][np] -> pad with the axis shift, slices paired -> forward DFT of each row ->
// Yf[L][nt][C] (polar row k * nt + a, channel fastest).  One block per (angle a, channels c0 ..
// c0 + CW - 1), XCD-remapped so that the channel groups of one angle are neighbours.
// RES (a conjugate-gradient residual step fused in): y is r, updated in place to
// r - alpha[s] q (the arithmetic of the separate update kernel) before it is transformed.
template <int M, int CW, bool BL, bool RES>
__global__ __launch_bounds__(kFB) void k_det_pad_forward_cf(const float* y, float* rnew,
                                                            const float* __restrict__ qv,
                                                            const double* __restrict__ alpha,
                                                            float2* __restrict__ Yf, DftTables t,
                                                            int B, int nt, int np, int cdet,
                                                            const float2* __restrict__ phase) {
  constexpr int PAD = row_skew<M>();
  __shared__ float2 buf[lds_rows_size<CW, M, PAD>()];
  const int L = BL ? t.N : M;
  const int C = (B + 1) / 2;
  const int cgroups = (C + CW - 1) / CW;
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  const int a = (int)(blk / cgroups), c0 = (int)(blk % cgroups) * CW;
  const int nc = min(CW, C - c0);
  const int64_t plane = (int64_t)nt * np;
  constexpr int NE = (CW * M + kFB - 1) / kFB;   // loads per thread, issued as one batch
  float2 v[NE], w[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int i = threadIdx.x + u * kFB;
    const int q = i / M, m = i % M;
    int b = m + cdet;                                 // radial index m holds bin (m + c) mod L
    b -= (b >= L) ? L : 0;
    v[u] = make_float2(0.f, 0.f);
    w[u] = make_float2(0.f, 0.f);
    if (i < CW * M && q < nc && m < L && b < np) {
      const int c = c0 + q;
      const int64_t off = (int64_t)a * np + b;
      v[u].x = y[(int64_t)(2 * c) * plane + off];
      if (RES) w[u].x = qv[(int64_t)(2 * c) * plane + off];
      if (2 * c + 1 < B) {
        v[u].y = y[(int64_t)(2 * c + 1) * plane + off];
        if (RES) w[u].y = qv[(int64_t)(2 * c + 1) * plane + off];
      }
    }
  }
  if constexpr (RES) {
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int i = threadIdx.x + u * kFB;
      const int q = i / M, m = i % M;
      int b = m + cdet;
      b -= (b >= L) ? L : 0;
      if (i < CW * M && q < nc && m < L && b < np) {
        const int c = c0 + q;
        const int64_t off = (int64_t)a * np + b;
        const float f0 = (float)(-1.0 * alpha[2 * c]);
        float r0 = 1.0f * v[u].x;
        r0 += f0 * w[u].x;
        v[u].x = r0;
        rnew[(int64_t)(2 * c) * plane + off] = r0;
        if (2 * c + 1 < B) {
          const float f1 = (float)(-1.0 * alpha[2 * c + 1]);
          float r1 = 1.0f * v[u].y;
          r1 += f1 * w[u].y;
          v[u].y = r1;
          rnew[(int64_t)(2 * c + 1) * plane + off] = r1;
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int i = threadIdx.x + u * kFB;
    if (i < CW * M) buf[ldsr<M, PAD>(i / M, i % M)] = v[u];
  }
  __syncthreads();
  dft_lds<M, CW, false, BL, PAD>(buf, t);
  for (int i = threadIdx.x; i < L * nc; i += kFB) {
    const int k = i / nc, q = i % nc;
    float2 w = buf[ldsr<M, PAD>(q, k)];
    if (phase) w = cmul(w, conj2(phase[k]));       // a fractional axis bin's phase ramp
    Yf[((int64_t)k * nt + a) * C + c0 + q] = w;
  }
}

template <int M, bool BL>
tomo_status det_launch(bool inverse, bool fastest, const tomo_op* op, const float2* Ysin, float2* Ysout,
                       const float* yin, float* yout, int B, float scale, double* sumsq,
                       hipStream_t st) {
  constexpr int AG = det_rows_per_block(M);
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  const dim3 grid((unsigned)(C * ((g.nt + AG - 1) / AG)));
  constexpr int CW = det_cw<M>();
  const dim3 cfgrid((unsigned)(g.nt * ((C + CW - 1) / CW)));
  if (inverse)
    hipLaunchKernelGGL((k_det_inverse_crop<M, AG, BL>), grid, dim3(kFB), 0, st, Ysin, yout, op->dft1,
                       B, g.nt, g.np, g.cdet, scale, sumsq, op->phase_dev);
  else if (fastest)
    hipLaunchKernelGGL((k_det_pad_forward_cf<M, CW, BL, false>), cfgrid, dim3(kFB), 0, st, yin,
                       nullptr, nullptr, nullptr, Ysout, op->dft1, B, g.nt, g.np, g.cdet,
                       op->phase_dev);
  else
    hipLaunchKernelGGL((k_det_pad_forward<M, AG, BL>), grid, dim3(kFB), 0, st, yin, Ysout, op->dft1,
                       B, g.nt, g.np, g.cdet, op->phase_dev);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status det_dispatch(bool inverse, bool fastest, const tomo_op* op, const float2* Yin,
                         float2* Yout, const float* yin, float* yout, int B, float scale,
                         double* sumsq, hipStream_t st) {
  const bool bl = op->dft1.M != op->g.L;
#define TOMO_DET(M_)                                                                             \
  case M_:                                                                                      \
    return bl ? det_launch<M_, true>(inverse, fastest, op, Yin, Yout, yin, yout, B, scale, sumsq, st) \
              : det_launch<M_, false>(inverse, fastest, op, Yin, Yout, yin, yout, B, scale, sumsq, st);
  switch (op->dft1.M) {
    TOMO_DET(16) TOMO_DET(32) TOMO_DET(64) TOMO_DET(128) TOMO_DET(256) TOMO_DET(512) TOMO_DET(1024)
    TOMO_DET(2048) TOMO_DET(4096) TOMO_DET(8192)
    default: return fail(TOMO_EUNSUPPORTED, "fused detector DFT: no kernel for length %d", op->dft1.M);
  }
#undef TOMO_DET
}

template <int M, bool BL>
tomo_status det_residual_launch(const tomo_op* op, float* r, const float* q, const double* alpha,
                                float2* Yf, int B, hipStream_t st) {
  constexpr int CW = det_cw<M>();
  const int C = (B + 1) / 2;
  const dim3 grid((unsigned)(op->g.nt * ((C + CW - 1) / CW)));
  hipLaunchKernelGGL((k_det_pad_forward_cf<M, CW, BL, true>), grid, dim3(kFB), 0, st, r, r, q, alpha,
                     Yf, op->dft1, B, op->g.nt, op->g.np, op->g.cdet, op->phase_dev);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

}  // namespace

bool det_fft_supported(const tomo_op* op) { return op->dft1.tw != nullptr; }

bool det_cf_supported(const tomo_op* op) { return det_fft_supported(op) && op->dft1.M <= 4096; }

tomo_status launch_det_residual_forward(const tomo_op* op, float* r, const float* q,
                                        const double* alpha, float2* Yf, int B, hipStream_t st) {
  if (!det_cf_supported(op))
    return fail(TOMO_EINVAL, "internal: fused residual front needs transform length <= 4096");
  const bool bl = op->dft1.M != op->g.L;
#define TOMO_DETR(M_)                                                                            \
  case M_:                                                                                      \
    return bl ? det_residual_launch<M_, true>(op, r, q, alpha, Yf, B, st)                       \
              : det_residual_launch<M_, false>(op, r, q, alpha, Yf, B, st);
  switch (op->dft1.M) {
    TOMO_DETR(16) TOMO_DETR(32) TOMO_DETR(64) TOMO_DETR(128) TOMO_DETR(256) TOMO_DETR(512)
    TOMO_DETR(1024) TOMO_DETR(2048) TOMO_DETR(4096)
    default: return fail(TOMO_EUNSUPPORTED, "fused detector DFT: no kernel for length %d", op->dft1.M);
  }
#undef TOMO_DETR
}

int64_t det_inverse_blocks_per_channel(const tomo_op* op) {
  if (!det_fft_supported(op)) return 0;
  const int ag = det_rows_per_block(op->dft1.M);
  return (op->g.nt + ag - 1) / ag;
}

tomo_status launch_det_inverse_crop(const tomo_op* op, const float2* Ys, float* y, int B,
                                    float scale, double* sumsq, hipStream_t st) {
  return det_dispatch(true, false, op, Ys, nullptr, nullptr, y, B, scale, sumsq, st);
}

tomo_status launch_det_pad_forward(const tomo_op* op, const float* y, float2* Y, int B,
                                   bool channel_fastest, hipStream_t st) {
  return det_dispatch(false, channel_fastest, op, nullptr, Y, y, nullptr, B, 1.0f, nullptr, st);
}

}  // namespace tomo
