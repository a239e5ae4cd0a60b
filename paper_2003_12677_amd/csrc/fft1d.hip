// The detector-direction transforms of Eq. (2) fused with the layout steps around them, for a
// power-of-two number L of polar samples per angle (16..4096):
//
//   project tail:     Ys[C][nt][L] (the polar data after the tiled transpose from the forward
//                     SpMM's channel-fastest output) -> inverse DFT of each row -> rotation-axis
//                     shift, 1/L, crop to n_p bins, real / imaginary parts to slices 2c / 2c+1
//                     of y[B][nt][np];
//   adjoint front:    y[B][nt][np] -> pad to L with the axis shift, slices paired into complex
//                     channels -> forward DFT of each row -> Ys[C][nt][L] (then transposed for
//                     the adjoint SpMM).
//
// One block per (channel, AG consecutive angles), a contiguous stretch of Ys: the rows are
// transformed in LDS with radix-8 Stockham passes (plus one radix-4 or radix-2 pass for the
// remaining factor; each pass reads every butterfly's inputs into registers, synchronises, then
// writes its outputs, so one buffer suffices; the twiddle powers of a butterfly are formed by
// multiplication from one table entry).  This replaces a library FFT and a crop / pad kernel by one
// pass over the data.  (Gathering straight from the channel-fastest SpMM layout instead reads
// only 4 channels' 32 bytes of each 128-byte row per block and was slower than a separate
// transpose.)  Twiddles exp(-2 pi i j / L), j < L, come from a table computed in double.

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tomo {
namespace {

constexpr int kFB = 512;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// X_q = sum_r v_r exp(-/+ 2 pi i r q / R)
template <bool INV>
__device__ __forceinline__ void dft4(float2 (&v)[4]) {
  const float2 s02 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
  const float2 d02 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
  const float2 s13 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
  const float2 d13 = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
  // -i * d13 (forward) or +i * d13 (inverse)
  const float2 rot = INV ? make_float2(-d13.y, d13.x) : make_float2(d13.y, -d13.x);
  v[0] = make_float2(s02.x + s13.x, s02.y + s13.y);
  v[2] = make_float2(s02.x - s13.x, s02.y - s13.y);
  v[1] = make_float2(d02.x + rot.x, d02.y + rot.y);
  v[3] = make_float2(d02.x - rot.x, d02.y - rot.y);
}

// radix 8 from two radix-4 transforms of the even and odd inputs and the eighth roots of unity
template <bool INV>
__device__ __forceinline__ void dft8(float2 (&v)[8]) {
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  constexpr float h = 0.70710678118654752f;
  // t_q = w8^q o_q, w8 = exp(-/+ 2 pi i / 8)
  const float2 t0 = o[0];
  const float2 t1 = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                        : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
  const float2 t2 = INV ? make_float2(-o[2].y, o[2].x) : make_float2(o[2].y, -o[2].x);
  const float2 t3 = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                        : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
  const float2 t[4] = {t0, t1, t2, t3};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[q] = make_float2(e[q].x + t[q].x, e[q].y + t[q].y);
    v[q + 4] = make_float2(e[q].x - t[q].x, e[q].y - t[q].y);
  }
}

template <bool INV>
__device__ __forceinline__ void dft2(float2 (&v)[2]) {
  const float2 a = v[0], b = v[1];
  v[0] = make_float2(a.x + b.x, a.y + b.y);
  v[1] = make_float2(a.x - b.x, a.y - b.y);
}

// One Stockham pass of radix R on CH transforms of length L stored back to back in `buf`,
// after which sub-transforms of length Ns*R are complete (Ns = 1 << logNs).
template <int L, int CH, int R, bool INV>
__device__ __forceinline__ void stockham_pass(float2* buf, int logNs, const float2* __restrict__ tw) {
  constexpr int NJ = L / R;
  constexpr int TOTAL = CH * NJ;
  constexpr int IT = (TOTAL + kFB - 1) / kFB;
  const int Ns = 1 << logNs;
  const int tstep = L / (R * Ns);
  float2 v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = threadIdx.x + it * kFB;
    if (w < TOTAL) {
      const int ch = w / NJ, j = w % NJ;
      const int k = j & (Ns - 1);
      const float2* src = buf + ch * L + j;
      // w = exp(-/+ 2 pi i k / (R Ns)) from the table, its powers by multiplication
      float2 w = tw[k * tstep];
      if (INV) w.y = -w.y;
      float2 wr = w;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 a = src[r * NJ];
        if (r > 0) {
          a = cmul(a, wr);
          wr = cmul(wr, w);
        }
        v[it][r] = a;
      }
      if constexpr (R == 8) dft8<INV>(v[it]);
      else if constexpr (R == 4) dft4<INV>(v[it]);
      else dft2<INV>(v[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = threadIdx.x + it * kFB;
    if (w < TOTAL) {
      const int ch = w / NJ, j = w % NJ;
      const int idx = ((j >> logNs) << logNs) * R + (j & (Ns - 1));
      float2* dst = buf + ch * L + idx;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns] = v[it][r];
    }
  }
  __syncthreads();
}

// radix-8 passes, then one radix-4 or radix-2 pass for the remaining factor
template <int L, int CH, bool INV>
__device__ __forceinline__ void fft_lds(float2* buf, const float2* __restrict__ tw) {
  int logNs = 0;
  while ((8 << logNs) <= L) {
    stockham_pass<L, CH, 8, INV>(buf, logNs, tw);
    logNs += 3;
  }
  if ((4 << logNs) <= L) stockham_pass<L, CH, 4, INV>(buf, logNs, tw);
  else if ((2 << logNs) <= L) stockham_pass<L, CH, 2, INV>(buf, logNs, tw);
}

// Ys[C][nt][L] (channel-slowest rows after the polar transpose) -> inverse DFT of each row ->
// axis shift, scale, crop, slices 2c / 2c+1.  One block per (channel, AG consecutive angles):
// its rows are one contiguous stretch of memory.
template <int L, int AG>
__global__ __launch_bounds__(kFB) void k_det_inverse_crop(const float2* __restrict__ Ys,
                                                          float* __restrict__ y,
                                                          const float2* __restrict__ tw, int B,
                                                          int nt, int np, int cdet, float scale) {
  __shared__ float2 buf[AG * L];
  const int agroups = (nt + AG - 1) / AG;
  const int c = blockIdx.x / agroups, a0 = (blockIdx.x % agroups) * AG;
  const int na = min(AG, nt - a0);
  const float2* src = Ys + ((int64_t)c * nt + a0) * L;
  for (int i = threadIdx.x; i < AG * L; i += kFB)
    buf[i] = (i < na * L) ? src[i] : make_float2(0.f, 0.f);
  __syncthreads();
  fft_lds<L, AG, true>(buf, tw);
  const int64_t plane = (int64_t)nt * np;
  const bool odd = 2 * c + 1 < B;
  for (int i = threadIdx.x; i < na * np; i += kFB) {
    const int q = i / np, b = i % np;
    const float2 v = buf[q * L + ((b - cdet) & (L - 1))];
    const int64_t off = (int64_t)(a0 + q) * np + b;
    y[(int64_t)(2 * c) * plane + off] = v.x * scale;
    if (odd) y[(int64_t)(2 * c + 1) * plane + off] = v.y * scale;
  }
}

// y[B][nt][np] -> pad with the axis shift, slices paired -> forward DFT of each row ->
// Ys[C][nt][L] (channel-slowest rows; the polar transpose follows).
template <int L, int AG>
__global__ __launch_bounds__(kFB) void k_det_pad_forward(const float* __restrict__ y,
                                                         float2* __restrict__ Ys,
                                                         const float2* __restrict__ tw, int B,
                                                         int nt, int np, int cdet) {
  __shared__ float2 buf[AG * L];
  const int agroups = (nt + AG - 1) / AG;
  const int c = blockIdx.x / agroups, a0 = (blockIdx.x % agroups) * AG;
  const int na = min(AG, nt - a0);
  const int64_t plane = (int64_t)nt * np;
  const bool odd = 2 * c + 1 < B;
  for (int i = threadIdx.x; i < AG * L; i += kFB) {
    const int q = i / L, m = i % L;
    const int b = (m + cdet) & (L - 1);
    float2 v = make_float2(0.f, 0.f);
    if (q < na && b < np) {
      const int64_t off = (int64_t)(a0 + q) * np + b;
      v.x = y[(int64_t)(2 * c) * plane + off];
      if (odd) v.y = y[(int64_t)(2 * c + 1) * plane + off];
    }
    buf[i] = v;
  }
  __syncthreads();
  fft_lds<L, AG, false>(buf, tw);
  float2* dst = Ys + ((int64_t)c * nt + a0) * L;
  for (int i = threadIdx.x; i < na * L; i += kFB) dst[i] = buf[i];
}

template <int L>
tomo_status det_launch(bool inverse, const tomo_op* op, const float2* Ysin, float2* Ysout,
                       const float* yin, float* yout, int B, float scale, hipStream_t st) {
  constexpr int AG = L >= 4096 ? 2 : (L >= 2048 ? 4 : 8192 / L > 16 ? 16 : 8192 / L);
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  const dim3 grid((unsigned)(C * ((g.nt + AG - 1) / AG)));
  if (inverse)
    hipLaunchKernelGGL((k_det_inverse_crop<L, AG>), grid, dim3(kFB), 0, st, Ysin, yout, op->tw1,
                       B, g.nt, g.np, g.cdet, scale);
  else
    hipLaunchKernelGGL((k_det_pad_forward<L, AG>), grid, dim3(kFB), 0, st, yin, Ysout, op->tw1, B,
                       g.nt, g.np, g.cdet);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status det_dispatch(bool inverse, const tomo_op* op, const float2* Yin, float2* Yout,
                         const float* yin, float* yout, int B, float scale, hipStream_t st) {
  switch (op->g.L) {
    case 16: return det_launch<16>(inverse, op, Yin, Yout, yin, yout, B, scale, st);
    case 32: return det_launch<32>(inverse, op, Yin, Yout, yin, yout, B, scale, st);
    case 64: return det_launch<64>(inverse, op, Yin, Yout, yin, yout, B, scale, st);
    case 128: return det_launch<128>(inverse, op, Yin, Yout, yin, yout, B, scale, st);
    case 256: return det_launch<256>(inverse, op, Yin, Yout, yin, yout, B, scale, st);
    case 512: return det_launch<512>(inverse, op, Yin, Yout, yin, yout, B, scale, st);
    case 1024: return det_launch<1024>(inverse, op, Yin, Yout, yin, yout, B, scale, st);
    case 2048: return det_launch<2048>(inverse, op, Yin, Yout, yin, yout, B, scale, st);
    case 4096: return det_launch<4096>(inverse, op, Yin, Yout, yin, yout, B, scale, st);
    default: return fail(TOMO_EUNSUPPORTED, "fused detector FFT needs L = 2^m in [16, 4096]");
  }
}

}  // namespace

bool det_fft_supported(const tomo_op* op) {
  const int L = op->g.L;
  return op->tw1 != nullptr && L >= 16 && L <= 4096 && (L & (L - 1)) == 0;
}

tomo_status launch_det_inverse_crop(const tomo_op* op, const float2* Ys, float* y, int B,
                                    float scale, hipStream_t st) {
  return det_dispatch(true, op, Ys, nullptr, nullptr, y, B, scale, st);
}

tomo_status launch_det_pad_forward(const tomo_op* op, const float* y, float2* Ys, int B,
                                   hipStream_t st) {
  return det_dispatch(false, op, nullptr, Ys, y, nullptr, B, 1.0f, st);
}

}  // namespace tomo
