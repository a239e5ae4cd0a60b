// Radix-8/4/2 Stockham DFTs of several length-L vectors held in LDS, for power-of-two L: the
// shared core of the hand-written transforms (detector rows and Cartesian rows / columns); and
// DFTs of any length N through Bluestein's chirp-z identity on top of them.
// Every pass reads each butterfly's inputs into registers, synchronises the block, then writes
// its outputs back, so the transform is in place in one buffer.  Forward: exp(-2 pi i jk / L);
// inverse: exp(+2 pi i jk / L), unnormalised.  Twiddle table tw[j] = exp(-2 pi i j / L).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tomo {
namespace fftk {

constexpr int kFB = 512;   // threads per block of every kernel that uses these passes

}  // namespace fftk

// Blocks are dispatched round robin over the 8 XCDs (block b to XCD b mod 8).  The remapped index
// of hardware block `bid` makes each XCD walk one contiguous range of logical blocks, so that
// neighbouring logical blocks (which share cache lines or gathered inputs) share one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t x = bid & 7, local = bid >> 3;
  const int64_t q = nblocks >> 3, r = nblocks & 7;
  return (x < r) ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

namespace fftk {

// LDS index of element i: one padding element after every 32 (256 bytes, one row of banks), so
// the stride-R writes of the early passes spread over the banks instead of colliding.
__device__ __forceinline__ int lds(int i) { return i + (i >> 5); }
template <int N>
constexpr int lds_size() { return N + N / 32 + 1; }
// Rows of length L back to back, row ch shifted by ch * PAD further elements: PAD = 8 places the
// same element of 8 consecutive rows in 8 different bank pairs, for reads across rows.  PAD = 0 is
// the plain layout lds(ch * L + j).
template <int L, int PAD>
__device__ __forceinline__ int ldsr(int ch, int j) { return lds(ch * L + j) + ch * PAD; }
template <int CH, int L, int PAD>
constexpr int lds_rows_size() { return lds_size<CH * L>() + CH * PAD; }
// The skew that makes the stride of length-M rows 8 (mod 32) elements: element k of 8
// consecutive rows then lies in 8 different bank pairs, and a wave reading 8 rows x 8
// consecutive k (the transposing loads and stores) is free of bank conflicts.
template <int M>
constexpr int row_skew() { return M >= 32 ? (8 - (M + M / 32) % 32 + 32) % 32 : 0; }

// Sums a and b over the block in float64, in a fixed order (result in thread 0).  Every thread
// of the block must call it.
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double red[2][kFB / 64];
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = b = 0.0;
    for (int w = 0; w < kFB / 64; ++w) {
      a += red[0][w];
      b += red[1][w];
    }
  }
}

__device__ __forceinline__ float2 conj2(float2 a) { return make_float2(a.x, -a.y); }

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
template <int L, int CH, int R, bool INV, int PAD = 0>
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
      // w = exp(-/+ 2 pi i k / (R Ns)) from the table, its powers by multiplication
      float2 w = tw[k * tstep];
      if (INV) w.y = -w.y;
      float2 wr = w;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 a = buf[ldsr<L, PAD>(ch, j + r * NJ)];
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
#pragma unroll
      for (int r = 0; r < R; ++r) buf[ldsr<L, PAD>(ch, idx + r * Ns)] = v[it][r];
    }
  }
  __syncthreads();
}

// radix-8 passes, then one radix-4 or radix-2 pass for the remaining factor
template <int L, int CH, bool INV, int PAD = 0>
__device__ __forceinline__ void fft_lds(float2* buf, const float2* __restrict__ tw) {
  int logNs = 0;
  while ((8 << logNs) <= L) {
    stockham_pass<L, CH, 8, INV, PAD>(buf, logNs, tw);
    logNs += 3;
  }
  if ((4 << logNs) <= L) stockham_pass<L, CH, 4, INV, PAD>(buf, logNs, tw);
  else if ((2 << logNs) <= L) stockham_pass<L, CH, 2, INV, PAD>(buf, logNs, tw);
}

// Length-N DFTs (N not a power of two) of CH vectors held in LDS with row stride M, a power of two
// >= 2N - 1, elements N .. M-1 zero on entry (Bluestein 1970, the chirp-z transform).  With
// w_m = exp(+i pi m^2 / N), n k = (n^2 + k^2 - (k - n)^2) / 2 gives
//   forward: X_k = conj(w_k) sum_n (x_n conj(w_n)) w_{k-n},
//   inverse: X_k =      w_k  sum_n (x_n w_n) conj(w_{k-n}),
// a linear convolution of length < 2N - 1, done as a cyclic one of length M through the radix-8
// transforms.  Tables (from double precision on the host): chirp[n] = conj(w_n), n < N; bhat = the
// length-M DFT of the kernel w (forward) or conj(w) (inverse) wrapped to negative indices, times
// 1/M; tw = the length-M twiddles.  Elements N .. M-1 hold garbage on exit.
template <int M, int CH, bool INV, int PAD = 0>
__device__ __forceinline__ void bluestein_lds(float2* buf, const float2* __restrict__ tw, int N,
                                              const float2* __restrict__ chirp,
                                              const float2* __restrict__ bhat) {
  for (int i = threadIdx.x; i < CH * M; i += kFB) {
    const int m = i % M, e = ldsr<M, PAD>(i / M, m);
    if (m < N) {
      float2 c = chirp[m];
      if (INV) c.y = -c.y;
      buf[e] = cmul(buf[e], c);
    }
  }
  __syncthreads();
  fft_lds<M, CH, false, PAD>(buf, tw);
  for (int i = threadIdx.x; i < CH * M; i += kFB) {
    const int e = ldsr<M, PAD>(i / M, i % M);
    buf[e] = cmul(buf[e], bhat[i % M]);
  }
  __syncthreads();
  fft_lds<M, CH, true, PAD>(buf, tw);
  for (int i = threadIdx.x; i < CH * M; i += kFB) {
    const int m = i % M, e = ldsr<M, PAD>(i / M, m);
    if (m < N) {
      float2 c = chirp[m];
      if (INV) c.y = -c.y;
      buf[e] = cmul(buf[e], c);
    }
  }
  __syncthreads();
}

// Tables of one transform length N for the kernels: the power-of-two case (M = N) needs only the
// twiddles; otherwise M is the Bluestein length and chirp / bhat_f / bhat_i are set.
struct DftTables {
  int N = 0, M = 0;
  const float2* tw = nullptr;
  const float2* chirp = nullptr;
  const float2* bhat_f = nullptr;
  const float2* bhat_i = nullptr;
};

// The length-N DFT (forward or inverse, unnormalised) of CH vectors in LDS with row stride M
// (element j of row ch at ldsr<M, PAD>(ch, j)).
template <int M, int CH, bool INV, bool BL, int PAD = 0>
__device__ __forceinline__ void dft_lds(float2* buf, const DftTables& t) {
  if constexpr (BL)
    bluestein_lds<M, CH, INV, PAD>(buf, t.tw, t.N, t.chirp, INV ? t.bhat_i : t.bhat_f);
  else
    fft_lds<M, CH, INV, PAD>(buf, t.tw);
}

}  // namespace fftk
}  // namespace tomo
