// CSR SpMM kernels for the slicing interpolation (Sec. 2.2: the key step; Sec. 3 Eq. (2)).
//
// Vectors hold C complex channels per grid point, channel-fastest ([point][C] complex64), so
// gathering one column fetches 8*C contiguous bytes (128 B, one cache line, at C = 16).
// A "lane group" of T lanes owns one output row; lane t holds CPL consecutive complex channels
// (CPL = 2 -> one 16-byte load per lane per gathered column).  Accumulation is float32 in a
// fixed order, so results are bitwise reproducible.
//
// Forward (S^dagger, polar rows, <= k_w^2 entries per row): one lane group per row.
// Adjoint (S, Cartesian rows, 0 .. thousands of entries per row): row-binned, no atomics
// (the transpose is stored, Sec. 3.1), in one launch whose block range selects the bin:
//   short rows  -> one lane group per row,
//   medium rows -> one wavefront per row (lane groups stride the entries, shuffle reduction),
//   long rows   -> chunks of entries, one block per chunk, partial sums to a scratch buffer,
//                  followed by a small launch that adds each long row's chunks in order.

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tomo {
namespace {

constexpr int kBlock = 256;

struct bf16_t { uint16_t bits; };

__device__ __forceinline__ float ldv(const float* v, int64_t e) { return v[e]; }
__device__ __forceinline__ float ldv(const bf16_t* v, int64_t e) {
  return __uint_as_float((uint32_t)v[e].bits << 16);
}
__device__ __forceinline__ float ldv(const _Float16* v, int64_t e) { return (float)v[e]; }

// Blocks are dispatched round-robin over the 8 XCDs; remap so that each XCD walks a contiguous
// range of rows and neighbouring rows (which share gathered columns) share one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t x = bid & 7, local = bid >> 3;
  const int64_t q = nblocks >> 3, r = nblocks & 7;
  return (x < r) ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

template <int CPL>
struct Acc {
  float v[2 * CPL];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < 2 * CPL; ++i) v[i] = 0.f;
  }
  __device__ __forceinline__ void fma(float w, const float2* p) {
    if constexpr (CPL == 2) {
      const float4 x = *reinterpret_cast<const float4*>(p);
      v[0] += w * x.x; v[1] += w * x.y; v[2] += w * x.z; v[3] += w * x.w;
    } else {
      const float2 x = *p;
      v[0] += w * x.x; v[1] += w * x.y;
    }
  }
  __device__ __forceinline__ void store(float2* p) const {
    if constexpr (CPL == 2) {
      *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
      *p = make_float2(v[0], v[1]);
    }
  }
  __device__ __forceinline__ void add(const Acc& o) {
#pragma unroll
    for (int i = 0; i < 2 * CPL; ++i) v[i] += o.v[i];
  }
};

// Sum of entries [e0, e1) with stride `step` of one CSR row into acc (lane's channels at p0).
template <int CPL, typename V, bool FILT>
__device__ __forceinline__ void row_dot(const int32_t* __restrict__ col, const V* __restrict__ val,
                                        const float2* __restrict__ src, int C, int cb,
                                        int64_t e0, int64_t e1, int step, const float* dscale,
                                        double inv_nt, Acc<CPL>& acc) {
  int64_t e = e0;
  // four entries per round: the index and value loads of all four are issued before the
  // gathers, so each lane keeps four independent 16-byte loads in flight
  for (; e + 3 * step < e1; e += 4 * step) {
    int c[4];
    float w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c[u] = col[e + u * step];
      w[u] = ldv(val, e + u * step);
    }
    if constexpr (FILT) {
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] *= dscale[(int)(((double)c[u] + 0.5) * inv_nt)];
    }
    const float2* p[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) p[u] = src + (int64_t)c[u] * C + cb;
#pragma unroll
    for (int u = 0; u < 4; ++u) acc.fma(w[u], p[u]);
  }
  for (; e < e1; e += step) {
    const int c = col[e];
    float w = ldv(val, e);
    if constexpr (FILT) w *= dscale[(int)(((double)c + 0.5) * inv_nt)];
    acc.fma(w, src + (int64_t)c * C + cb);
  }
}

// ------------------------------------------------------------------------------------------
// forward: Y = S^dagger X
// ------------------------------------------------------------------------------------------
template <int T, int CPL, typename V>
__global__ __launch_bounds__(kBlock) void k_spmm_fwd(const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col,
                                                     const V* __restrict__ val,
                                                     const float2* __restrict__ X,
                                                     float2* __restrict__ Y, int64_t nrows, int C) {
  constexpr int RPB = kBlock / T;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int64_t row = xcd_remap(blockIdx.x, gridDim.x) * RPB + g;
  const int cb = t * CPL;
  if (row >= nrows || cb >= C) return;
  Acc<CPL> acc;
  acc.zero();
  row_dot<CPL, V, false>(col, val, X, C, cb, rowptr[row], rowptr[row + 1], 1, nullptr, 0.0, acc);
  acc.store(Y + row * C + cb);
}

// ------------------------------------------------------------------------------------------
// adjoint: X = S diag(d) Y, row-binned
// ------------------------------------------------------------------------------------------
struct AdjArgs {
  const int32_t* rowptr;
  const int32_t* col;
  const float2* Y;
  float2* X;
  int C;
  const int32_t* short_rows;  int64_t n_short;  int64_t nb_short;
  const int32_t* medium_rows; int64_t n_medium; int64_t nb_medium;
  const int32_t* chunk_beg;   const int32_t* chunk_end; int64_t n_chunks;
  float2* partials;
  const float* dscale;        // per FFT-ordered radial index, or null
  double inv_nt;              // 1 / n_theta: radial index of polar column c is floor(c / nt)
};

template <int T, int CPL, typename V, bool FILT>
__global__ __launch_bounds__(kBlock) void k_spmm_adj(AdjArgs a, const V* __restrict__ val) {
  constexpr int RPB = kBlock / T;     // lane groups per block
  constexpr int GPW = 64 / T;         // lane groups per wavefront
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int cb = t * CPL;
  const bool active = cb < a.C;
  int64_t bid = blockIdx.x;
  if (bid < a.nb_short) {
    bid = xcd_remap(bid, a.nb_short);
    const int64_t i = bid * RPB + g;
    if (i >= a.n_short || !active) return;
    const int64_t row = a.short_rows[i];
    Acc<CPL> acc;
    acc.zero();
    row_dot<CPL, V, FILT>(a.col, val, a.Y, a.C, cb, a.rowptr[row], a.rowptr[row + 1], 1, a.dscale,
                          a.inv_nt, acc);
    acc.store(a.X + row * a.C + cb);
    return;
  }
  bid -= a.nb_short;
  if (bid < a.nb_medium) {
    const int wave = threadIdx.x >> 6;
    const int gw = (threadIdx.x & 63) / T;           // lane group within the wavefront
    const int64_t i = bid * (kBlock / 64) + wave;
    if (i >= a.n_medium) return;                      // whole wavefront leaves together
    const int64_t row = a.medium_rows[i];
    Acc<CPL> acc;
    acc.zero();
    if (active)
      row_dot<CPL, V, FILT>(a.col, val, a.Y, a.C, cb, a.rowptr[row] + gw, a.rowptr[row + 1], GPW,
                            a.dscale, a.inv_nt, acc);
#pragma unroll
    for (int off = T; off < 64; off <<= 1) {
#pragma unroll
      for (int k = 0; k < 2 * CPL; ++k) acc.v[k] += __shfl_xor(acc.v[k], off, 64);
    }
    if (gw == 0 && active) acc.store(a.X + row * a.C + cb);
    return;
  }
  bid -= a.nb_medium;
  if (bid >= a.n_chunks) return;
  // one chunk of a long row: all lane groups of the block share the chunk's entries
  __shared__ float red[kBlock * 2 * CPL];
  Acc<CPL> acc;
  acc.zero();
  if (active)
    row_dot<CPL, V, FILT>(a.col, val, a.Y, a.C, cb, (int64_t)a.chunk_beg[bid] + g,
                          a.chunk_end[bid], RPB, a.dscale, a.inv_nt, acc);
#pragma unroll
  for (int off = T; off < 64; off <<= 1) {
#pragma unroll
    for (int k = 0; k < 2 * CPL; ++k) acc.v[k] += __shfl_xor(acc.v[k], off, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) < T) {
#pragma unroll
    for (int k = 0; k < 2 * CPL; ++k) red[(wave * T + t) * 2 * CPL + k] = acc.v[k];
  }
  __syncthreads();
  if (threadIdx.x < T && active) {
    Acc<CPL> s;
    s.zero();
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w)
#pragma unroll
      for (int k = 0; k < 2 * CPL; ++k) s.v[k] += red[(w * T + t) * 2 * CPL + k];
    s.store(a.partials + bid * a.C + cb);
  }
}

template <int T, int CPL>
__global__ __launch_bounds__(kBlock) void k_adj_long_reduce(const int32_t* __restrict__ long_rows,
                                                            const int32_t* __restrict__ chunk_ptr,
                                                            const float2* __restrict__ partials,
                                                            float2* __restrict__ X, int64_t n_long,
                                                            int C) {
  constexpr int RPB = kBlock / T;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int64_t i = (int64_t)blockIdx.x * RPB + g;
  const int cb = t * CPL;
  if (i >= n_long || cb >= C) return;
  Acc<CPL> acc;
  acc.zero();
  for (int c = chunk_ptr[i]; c < chunk_ptr[i + 1]; ++c) acc.fma(1.0f, partials + (int64_t)c * C + cb);
  acc.store(X + (int64_t)long_rows[i] * C + cb);
}

// ------------------------------------------------------------------------------------------
// dispatch over (T, CPL, value type)
// ------------------------------------------------------------------------------------------
inline int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

template <int T, int CPL, typename V>
tomo_status fwd_impl(const tomo_op* op, const void* val, const float2* X, float2* Y, int C,
                     hipStream_t st) {
  const int64_t rows = op->fwd.rows;
  constexpr int RPB = kBlock / T;
  const int64_t nb = (rows + RPB - 1) / RPB;
  hipLaunchKernelGGL((k_spmm_fwd<T, CPL, V>), dim3((unsigned)nb), dim3(kBlock), 0, st,
                     op->fwd.rowptr, op->fwd.col, (const V*)val, X, Y, rows, C);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

template <int T, int CPL, typename V>
tomo_status adj_impl(const tomo_op* op, const void* val, const float2* Y, float2* X, int C,
                     const float* dscale, hipStream_t st) {
  constexpr int RPB = kBlock / T;
  AdjArgs a;
  a.rowptr = op->adj.rowptr;
  a.col = op->adj.col;
  a.Y = Y;
  a.X = X;
  a.C = C;
  a.short_rows = op->bins.short_rows;
  a.n_short = op->bins.n_short;
  a.nb_short = (a.n_short + RPB - 1) / RPB;
  a.medium_rows = op->bins.medium_rows;
  a.n_medium = op->bins.n_medium;
  a.nb_medium = (a.n_medium + (kBlock / 64) - 1) / (kBlock / 64);
  a.chunk_beg = op->bins.chunk_beg;
  a.chunk_end = op->bins.chunk_end;
  a.n_chunks = op->bins.n_chunks;
  a.partials = op->partials;
  a.dscale = dscale;
  a.inv_nt = 1.0 / (double)op->g.nt;
  const int64_t nb = a.nb_short + a.nb_medium + a.n_chunks;
  if (nb > 0) {
    if (dscale)
      hipLaunchKernelGGL((k_spmm_adj<T, CPL, V, true>), dim3((unsigned)nb), dim3(kBlock), 0, st, a,
                         (const V*)val);
    else
      hipLaunchKernelGGL((k_spmm_adj<T, CPL, V, false>), dim3((unsigned)nb), dim3(kBlock), 0, st,
                         a, (const V*)val);
    TOMO_HIP(hipGetLastError());
  }
  if (op->bins.n_long > 0) {
    const int64_t nbl = (op->bins.n_long + RPB - 1) / RPB;
    hipLaunchKernelGGL((k_adj_long_reduce<T, CPL>), dim3((unsigned)nbl), dim3(kBlock), 0, st,
                       op->bins.long_rows, op->bins.long_chunk_ptr, op->partials, X,
                       op->bins.n_long, C);
    TOMO_HIP(hipGetLastError());
  }
  return TOMO_OK;
}

template <bool FWD, typename V>
tomo_status dispatch_T(const tomo_op* op, const void* val, const float2* in, float2* out, int C,
                       const float* dscale, hipStream_t st) {
  const int CPL = (C % 2 == 0) ? 2 : 1;
  const int T = next_pow2((C + CPL - 1) / CPL);
#define TOMO_CASE(TT, CC)                                                              \
  if (T == TT && CPL == CC) {                                                          \
    if (FWD) return fwd_impl<TT, CC, V>(op, val, in, out, C, st);                       \
    return adj_impl<TT, CC, V>(op, val, in, out, C, dscale, st);                        \
  }
  TOMO_CASE(1, 1) TOMO_CASE(2, 1) TOMO_CASE(4, 1) TOMO_CASE(8, 1) TOMO_CASE(16, 1)
  TOMO_CASE(32, 1) TOMO_CASE(64, 1)
  TOMO_CASE(1, 2) TOMO_CASE(2, 2) TOMO_CASE(4, 2) TOMO_CASE(8, 2) TOMO_CASE(16, 2)
  TOMO_CASE(32, 2) TOMO_CASE(64, 2)
#undef TOMO_CASE
  return fail(TOMO_EINVAL, "channel count %d not supported", C);
}

template <bool FWD>
tomo_status dispatch(const tomo_op* op, int vt, const float2* in, float2* out, int C,
                     const float* dscale, hipStream_t st) {
  const DevCSR& m = FWD ? op->fwd : op->adj;
  if (vt < 0 || vt > 2 || !m.val[vt])
    return fail(TOMO_ESTATE, "value type %d was not built for this operator", vt);
  if (C < 1 || C > op->cmax) return fail(TOMO_EINVAL, "channel count %d out of range", C);
  switch (vt) {
    case TOMO_VAL_F32: return dispatch_T<FWD, float>(op, m.val[vt], in, out, C, dscale, st);
    case TOMO_VAL_BF16: return dispatch_T<FWD, bf16_t>(op, m.val[vt], in, out, C, dscale, st);
    default: return dispatch_T<FWD, _Float16>(op, m.val[vt], in, out, C, dscale, st);
  }
}

}  // namespace

tomo_status launch_spmm_fwd(const tomo_op* op, const float2* X, float2* Y, int C, int vt,
                            hipStream_t st) {
  return dispatch<true>(op, vt, X, Y, C, nullptr, st);
}

tomo_status launch_spmm_adj(const tomo_op* op, const float2* Y, float2* X, int C, int vt,
                            const float* dscale, hipStream_t st) {
  return dispatch<false>(op, vt, Y, X, C, dscale, st);
}

}  // namespace tomo
