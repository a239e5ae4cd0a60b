// SpMM kernels for the slicing interpolation (Sec. 2.2: the key step; Sec. 3 Eq. (2)).
//
// Vectors hold C complex channels per grid point, channel-fastest ([point][C] complex64), so a
// gathered column is 8*C contiguous bytes (128 B, one cache line, at C = 16).  A lane group of T
// lanes owns one output row; lane t holds CPL consecutive complex channels (CPL = 2: one 16-byte
// load per lane per gathered column).  Accumulation is float32 in a fixed order, so results are
// bitwise reproducible.
//
// These kernels are latency-bound: measured HBM traffic equals the algorithmic bytes, so speed
// comes from keeping the number of dependent memory round trips per row small.  Every row is
// processed in "rounds": first all column indices and values of up to U entries are loaded, then
// all U gathers are issued, then accumulated.
//
// Forward (S^dagger): rows hold at most k_w^2 entries, stored with a constant stride (ELL), so a
// row is one round: indices/values, then k_w^2 gathers.
// Adjoint (S): atomic-free through the stored transpose (Sec. 3.1), one kernel per row layout
// (separate launches, so each gets its own register allocation and full occupancy):
//   sliced ELL  rows with few entries (99% of rows), 8 rows per slice, entries of a slice stored
//               entry-major so the 8 rows' indices of one entry are contiguous;
//   medium      one wavefront per row, lane groups stride the row's entries, shuffle reduction;
//   long        chunks of entries, one block per chunk, partial sums to a scratch buffer,
//               then a small launch adds each long row's chunk sums in order.

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tomo {
namespace {

constexpr int kBlock = 256;
constexpr int kRound = 8;   // entries per round in the adjoint paths

struct bf16_t { uint16_t bits; };

// Blocks interleaved over the XCDs in runs of `chunk`: XCD x takes runs x, x+8, x+16, ... of
// `chunk` consecutive logical blocks, so neighbouring rows still share an L2 while every XCD
// gets a share of each part of the row range (the adjoint's row lengths vary with radius).
// chunk 0 = one contiguous range per XCD (xcd_remap), chunk 1 = the dispatch order itself.
__device__ __forceinline__ int64_t xcd_chunk_remap(int64_t bid, int64_t nblocks, int chunk) {
  if (chunk <= 0) return xcd_remap(bid, nblocks);
  const int64_t span = 8LL * chunk;
  const int64_t full = nblocks / span * span;
  if (bid >= full) return bid;
  const int64_t x = bid & 7, local = bid >> 3;
  return ((local / chunk) * 8 + x) * chunk + (local % chunk);
}

// CPL consecutive complex channels of one lane
template <int CPL>
struct Vec {
  float v[2 * CPL];
};

template <int CPL>
__device__ __forceinline__ Vec<CPL> load_vec(const float2* p) {
  Vec<CPL> r;
  if constexpr (CPL == 1) {
    const float2 a = *p;
    r.v[0] = a.x; r.v[1] = a.y;
  } else {
#pragma unroll
    for (int h = 0; h < CPL / 2; ++h) {
      const float4 a = reinterpret_cast<const float4*>(p)[h];
      r.v[4 * h] = a.x; r.v[4 * h + 1] = a.y; r.v[4 * h + 2] = a.z; r.v[4 * h + 3] = a.w;
    }
  }
  return r;
}

template <int CPL>
__device__ __forceinline__ void store_vec(float2* p, const Vec<CPL>& r) {
  if constexpr (CPL == 1) {
    *p = make_float2(r.v[0], r.v[1]);
  } else {
#pragma unroll
    for (int h = 0; h < CPL / 2; ++h)
      reinterpret_cast<float4*>(p)[h] =
          make_float4(r.v[4 * h], r.v[4 * h + 1], r.v[4 * h + 2], r.v[4 * h + 3]);
  }
}

template <int CPL>
__device__ __forceinline__ void vzero(Vec<CPL>& a) {
#pragma unroll
  for (int i = 0; i < 2 * CPL; ++i) a.v[i] = 0.f;
}

// raw 16/32-bit value storage, converted after every load of a round has been issued
__device__ __forceinline__ uint32_t ldraw(const float* v, int e) { return __float_as_uint(v[e]); }
__device__ __forceinline__ uint32_t ldraw(const bf16_t* v, int e) { return v[e].bits; }
__device__ __forceinline__ uint32_t ldraw(const _Float16* v, int e) {
  return *reinterpret_cast<const uint16_t*>(v + e);
}
__device__ __forceinline__ float cvt(const float*, uint32_t r) { return __uint_as_float(r); }
__device__ __forceinline__ float cvt(const bf16_t*, uint32_t r) { return __uint_as_float(r << 16); }
__device__ __forceinline__ float cvt(const _Float16*, uint32_t r) {
  const uint16_t h = (uint16_t)r;
  return (float)*reinterpret_cast<const _Float16*>(&h);
}

// One round: entries base + u*stride for u < count (count <= U).  Entries with a negative column
// are padding and contribute nothing.  The round is branch-free: every index/value load and
// every gather is issued unconditionally (padding and out-of-round slots read a valid address
// and are replaced by zero with a select), so the compiler keeps all of them in flight instead
// of waiting at each predicated block.
template <int CPL, int U, typename V, bool FILT>
__device__ __forceinline__ void gather_round(const int32_t* __restrict__ col,
                                             const V* __restrict__ val, int base,
                                             int stride, int count,
                                             const float2* __restrict__ src, int C, int cb,
                                             const float* __restrict__ dscale, double inv_nt,
                                             Vec<CPL>& acc) {
  int c[U];
  uint32_t raw[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = (u < count) ? base + u * stride : base;   // entry indices fit in 32 bits
    c[u] = col[e];
    raw[u] = ldraw(val, e);
  }
  bool ok[U];
  float w[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    ok[u] = (u < count) && (c[u] >= 0);
    w[u] = cvt(val, raw[u]);
    if constexpr (FILT) w[u] *= dscale[ok[u] ? (int)(((double)c[u] + 0.5) * inv_nt) : 0];
  }
  Vec<CPL> x[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (u < count)   // uniform in a lane group: slots past the round's end issue no request
      x[u] = load_vec<CPL>(src + (int64_t)(ok[u] ? c[u] : 0) * C + cb);
    else
      vzero(x[u]);
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int i = 0; i < 2 * CPL; ++i) acc.v[i] += w[u] * (ok[u] ? x[u].v[i] : 0.f);
}

// The same round with the metadata loaded once per lane group instead of once per lane, for
// groups of at least 8 lanes: lane t fetches the column and value of entries s*8 + (t & 7) of the
// round (slot s); every lane then reads entry u from lane (u & 7) of its group with a cross-lane
// permute.  All lanes of the group must be active (lanes beyond the channel count still load
// metadata and gather an in-bounds vector).  Split in two phases so that a caller can issue the
// next row's metadata loads before it uses the current row's.
template <int U, typename V>
__device__ __forceinline__ void bcast_meta_load(const int32_t* __restrict__ col,
                                                const V* __restrict__ val, int base, int stride,
                                                int count, int t8, int (&cl)[(U + 7) / 8],
                                                uint32_t (&rl)[(U + 7) / 8]) {
#pragma unroll
  for (int s = 0; s < (U + 7) / 8; ++s) {
    const int u = s * 8 + t8;
    const int e = (u < count) ? base + u * stride : base;
    cl[s] = col[e];
    rl[s] = ldraw(val, e);
  }
}

template <int CPL, int U, typename V, bool FILT>
__device__ __forceinline__ void bcast_meta_use(const V* val, int count, int t8,
                                               const int (&cl_in)[(U + 7) / 8],
                                               const uint32_t (&rl)[(U + 7) / 8],
                                               const float2* __restrict__ src, int C, int cb,
                                               const float* __restrict__ dscale, double inv_nt,
                                               int gbase4, Vec<CPL>& acc) {
  constexpr int S = (U + 7) / 8;
  int cl[S];
  float wl[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const bool ok = (s * 8 + t8 < count) && (cl_in[s] >= 0);
    wl[s] = cvt(val, rl[s]);
    if constexpr (FILT) wl[s] *= dscale[ok ? (int)(((double)cl_in[s] + 0.5) * inv_nt) : 0];
    cl[s] = ok ? cl_in[s] : -1;
  }
  int c[U];
  float w[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int addr = gbase4 + ((u & 7) << 2);
    c[u] = __builtin_amdgcn_ds_bpermute(addr, cl[u >> 3]);
    w[u] = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(wl[u >> 3])));
  }
  Vec<CPL> x[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (u < count)
      x[u] = load_vec<CPL>(src + (int64_t)(c[u] >= 0 ? c[u] : 0) * C + cb);
    else
      vzero(x[u]);
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int i = 0; i < 2 * CPL; ++i) acc.v[i] += w[u] * (c[u] >= 0 ? x[u].v[i] : 0.f);
}

template <int CPL, int U, typename V, bool FILT>
__device__ __forceinline__ void gather_round_bcast(const int32_t* __restrict__ col,
                                                   const V* __restrict__ val, int base,
                                                   int stride, int count,
                                                   const float2* __restrict__ src, int C, int cb,
                                                   const float* __restrict__ dscale,
                                                   double inv_nt, int gbase4, int t8,
                                                   Vec<CPL>& acc) {
  int cl[(U + 7) / 8];
  uint32_t rl[(U + 7) / 8];
  bcast_meta_load<U, V>(col, val, base, stride, count, t8, cl, rl);
  bcast_meta_use<CPL, U, V, FILT>(val, count, t8, cl, rl, src, C, cb, dscale, inv_nt, gbase4, acc);
}

// ------------------------------------------------------------------------------------------
// forward: Y = S^dagger X with a constant row stride W2
// ------------------------------------------------------------------------------------------
template <int CPL, typename V, int W2>
__global__ __launch_bounds__(kBlock) void k_fwd_ell(const int32_t* __restrict__ col,
                                                    const V* __restrict__ val,
                                                    const float2* __restrict__ X,
                                                    float2* __restrict__ Y, int64_t nrows, int C,
                                                    int logT, int w2_runtime) {
  const int g = threadIdx.x >> logT, t = threadIdx.x & ((1 << logT) - 1);
  const int64_t row = xcd_remap(blockIdx.x, gridDim.x) * (kBlock >> logT) + g;
  if (row >= nrows) return;                 // whole lane groups leave together
  const bool store = t * CPL < C;
  const int cb = store ? t * CPL : 0;       // idle channel lanes gather an in-bounds vector
  Vec<CPL> acc;
  vzero(acc);
  if (logT >= 3) {
    const int gbase4 = (int)((threadIdx.x & 63) & ~((1 << logT) - 1)) << 2;
    const int t8 = t & 7;
    if constexpr (W2 > 0) {
      gather_round_bcast<CPL, W2, V, false>(col, val, (int)row * W2, 1, W2, X, C, cb, nullptr,
                                            0.0, gbase4, t8, acc);
    } else {
      for (int e = 0; e < w2_runtime; e += kRound)
        gather_round_bcast<CPL, kRound, V, false>(col, val, (int)row * w2_runtime + e, 1,
                                                  min(kRound, w2_runtime - e), X, C, cb, nullptr,
                                                  0.0, gbase4, t8, acc);
    }
  } else {
    if constexpr (W2 > 0) {
      gather_round<CPL, W2, V, false>(col, val, (int)row * W2, 1, W2, X, C, cb, nullptr, 0.0, acc);
    } else {
      for (int e = 0; e < w2_runtime; e += kRound)
        gather_round<CPL, kRound, V, false>(col, val, (int)row * w2_runtime + e, 1,
                                            min(kRound, w2_runtime - e), X, C, cb, nullptr, 0.0, acc);
    }
  }
  if (store) store_vec(Y + row * C + cb, acc);
}

// Software-pipelined forward for the fixed 9-entry stencil and lane groups of >= 8 lanes: each
// group handles RPG rows (at stride "groups per block", so a wavefront's groups work on
// consecutive rows at every step) and issues the next row's metadata loads before it uses the
// current row's, so the metadata round trip overlaps the previous row's gathers.
template <int CPL, typename V, int RPG>
__global__ __launch_bounds__(kBlock) void k_fwd_pipe(const int32_t* __restrict__ col,
                                                     const V* __restrict__ val,
                                                     const float2* __restrict__ X,
                                                     float2* __restrict__ Y, int64_t nrows, int C,
                                                     int logT) {
  constexpr int W2 = 9, S = (W2 + 7) / 8;
  const int GPB = kBlock >> logT;
  const int g = threadIdx.x >> logT, t = threadIdx.x & ((1 << logT) - 1);
  const int64_t first = xcd_remap(blockIdx.x, gridDim.x) * (int64_t)GPB * RPG + g;
  if (first >= nrows) return;               // later rows of the group are beyond too
  const bool store = t * CPL < C;
  const int cb = store ? t * CPL : 0;
  const int gbase4 = (int)((threadIdx.x & 63) & ~((1 << logT) - 1)) << 2;
  const int t8 = t & 7;
  int cl[2][S];
  uint32_t rl[2][S];
  bcast_meta_load<W2, V>(col, val, (int)first * W2, 1, W2, t8, cl[0], rl[0]);
#pragma unroll
  for (int i = 0; i < RPG; ++i) {
    const int64_t row = first + (int64_t)i * GPB;
    if (i + 1 < RPG) {
      const int64_t nxt = min(row + GPB, nrows - 1);       // past the end: a valid row, unused
      bcast_meta_load<W2, V>(col, val, (int)nxt * W2, 1, W2, t8, cl[(i + 1) & 1],
                             rl[(i + 1) & 1]);
    }
    Vec<CPL> acc;
    vzero(acc);
    bcast_meta_use<CPL, W2, V, false>(val, W2, t8, cl[i & 1], rl[i & 1], X, C, cb, nullptr, 0.0,
                                      gbase4, acc);
    if (store && row < nrows) store_vec(Y + row * C + cb, acc);
  }
}

// ------------------------------------------------------------------------------------------
// adjoint: X = S diag(d) Y
// ------------------------------------------------------------------------------------------
struct AdjArgs {
  const int32_t* slice_ptr;
  const int32_t* slice_rows;
  const int32_t* col;
  int64_t n_slices, nb_sell;
  const int32_t* tail_rows;
  const int32_t* tail_ptr;
  const int32_t* tail_col;
  int64_t n_medium, nb_medium;
  const int32_t* chunk_beg;
  const int32_t* chunk_end;
  int64_t n_chunks;
  float2* partials;
  const float2* Y;
  float2* X;
  int C, logT;
  int sell_chunk, medium_chunk;   // block runs of the XCD interleave (xcd_chunk_remap)
  const float* dscale;        // per FFT-ordered radial index, or null
  double inv_nt;              // 1 / n_theta: radial index of polar column c is floor(c / nt)
};

template <int CPL>
__device__ __forceinline__ void wave_reduce_groups(Vec<CPL>& acc, int T) {
  for (int off = T; off < 64; off <<= 1) {
#pragma unroll
    for (int k = 0; k < 2 * CPL; ++k) acc.v[k] += __shfl_xor(acc.v[k], off, 64);
  }
}

// sliced ELL: one lane group per row slot of a slice
template <int CPL, typename V, bool FILT>
__global__ __launch_bounds__(kBlock) void k_adj_sell(AdjArgs a, const V* __restrict__ val) {
  const int g = threadIdx.x >> a.logT, t = threadIdx.x & ((1 << a.logT) - 1);
  const int64_t gid = xcd_chunk_remap(blockIdx.x, gridDim.x, a.sell_chunk) * (kBlock >> a.logT) + g;
  const int64_t slice = gid / kSliceRows;
  const int j = (int)(gid % kSliceRows);
  const int cb = t * CPL;
  if (slice >= a.n_slices || cb >= a.C) return;
  const int32_t e0 = a.slice_ptr[slice];
  const int len = (a.slice_ptr[slice + 1] - e0) / kSliceRows;
  const int32_t row = a.slice_rows[gid];
  Vec<CPL> acc;
  vzero(acc);
  for (int e = 0; e < len; e += kRound)
    gather_round<CPL, kRound, V, FILT>(a.col, val, e0 + e * kSliceRows + j, kSliceRows,
                                       min(kRound, len - e), a.Y, a.C, cb, a.dscale, a.inv_nt, acc);
  if (row >= 0) store_vec(a.X + (int64_t)row * a.C + cb, acc);
}

// one wavefront per medium row; lane groups stride the row's entries
template <int CPL, typename V, bool FILT>
__global__ __launch_bounds__(kBlock) void k_adj_medium(AdjArgs a, const V* __restrict__ tail_val) {
  const int T = 1 << a.logT;
  const int GPW = 64 >> a.logT;
  const int t = threadIdx.x & (T - 1);
  const int cb = t * CPL;
  const bool active = cb < a.C;
  const int wave = threadIdx.x >> 6;
  const int gw = (threadIdx.x & 63) >> a.logT;
  const int64_t i = xcd_chunk_remap(blockIdx.x, gridDim.x, a.medium_chunk) * (kBlock / 64) + wave;
  if (i >= a.n_medium) return;                       // the whole wavefront leaves together
  const int e1 = a.tail_ptr[i + 1];
  Vec<CPL> acc;
  vzero(acc);
  if (active) {
    for (int e = a.tail_ptr[i] + gw; e < e1; e += kRound * GPW)
      gather_round<CPL, kRound, V, FILT>(a.tail_col, tail_val, e, GPW,
                                         min(kRound, (e1 - e + GPW - 1) / GPW), a.Y, a.C, cb,
                                         a.dscale, a.inv_nt, acc);
  }
  wave_reduce_groups(acc, T);
  if (gw == 0 && active) store_vec(a.X + (int64_t)a.tail_rows[i] * a.C + cb, acc);
}

// one block per chunk of a long row: partial sums to the scratch buffer
template <int CPL, typename V, bool FILT>
__global__ __launch_bounds__(kBlock) void k_adj_chunk(AdjArgs a, const V* __restrict__ tail_val) {
  const int T = 1 << a.logT;
  const int RPB = kBlock >> a.logT;
  const int g = threadIdx.x >> a.logT, t = threadIdx.x & (T - 1);
  const int cb = t * CPL;
  const bool active = cb < a.C;
  const int64_t bid = blockIdx.x;
  __shared__ float red[(kBlock / 64) * 256];              // T * 2 * CPL <= 256 since C <= 128
  const int e1 = a.chunk_end[bid];
  Vec<CPL> acc;
  vzero(acc);
  if (active) {
    for (int e = a.chunk_beg[bid] + g; e < e1; e += kRound * RPB)
      gather_round<CPL, kRound, V, FILT>(a.tail_col, tail_val, e, RPB,
                                         min(kRound, (e1 - e + RPB - 1) / RPB), a.Y, a.C, cb,
                                         a.dscale, a.inv_nt, acc);
  }
  wave_reduce_groups(acc, T);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) < T) {
#pragma unroll
    for (int k = 0; k < 2 * CPL; ++k) red[wave * 256 + t * 2 * CPL + k] = acc.v[k];
  }
  __syncthreads();
  if (threadIdx.x < T && active) {
    Vec<CPL> s;
    vzero(s);
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w)
#pragma unroll
      for (int k = 0; k < 2 * CPL; ++k) s.v[k] += red[w * 256 + t * 2 * CPL + k];
    store_vec(a.partials + bid * a.C + cb, s);
  }
}

// X[row] = sum of the row's chunk partials, in chunk order
template <int CPL>
__global__ __launch_bounds__(kBlock) void k_adj_long_reduce(const int32_t* __restrict__ tail_rows,
                                                            const int32_t* __restrict__ chunk_ptr,
                                                            const float2* __restrict__ partials,
                                                            float2* __restrict__ X, int64_t n_medium,
                                                            int64_t n_long, int C, int logT) {
  const int g = threadIdx.x >> logT, t = threadIdx.x & ((1 << logT) - 1);
  const int64_t li = (int64_t)blockIdx.x * (kBlock >> logT) + g;
  const int cb = t * CPL;
  if (li >= n_long || cb >= C) return;
  Vec<CPL> acc;
  vzero(acc);
  for (int c = chunk_ptr[li]; c < chunk_ptr[li + 1]; ++c) {
    const Vec<CPL> p = load_vec<CPL>(partials + (int64_t)c * C + cb);
#pragma unroll
    for (int k = 0; k < 2 * CPL; ++k) acc.v[k] += p.v[k];
  }
  store_vec(X + (int64_t)tail_rows[n_medium + li] * C + cb, acc);
}

// ------------------------------------------------------------------------------------------
// dispatch
// ------------------------------------------------------------------------------------------
inline int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Largest valid channels-per-lane not above the preference: CPL must divide C (so that every
// lane's vector is whole and 16-byte aligned when CPL >= 2), and lane groups are <= 64 wide.
inline int pick_cpl(int pref, int C) {
  for (int cpl = pref; cpl >= 1; cpl >>= 1)
    if (C % cpl == 0 && (C + cpl - 1) / cpl <= 64) return cpl;
  return 0;
}

template <int CPL, typename V>
tomo_status fwd_impl(const tomo_op* op, const void* val, const float2* X, float2* Y, int C,
                     hipStream_t st) {
  const int logT = ilog2((C + CPL - 1) / CPL);
  const int64_t rows = op->fwd.rows;
  const int64_t rpb = kBlock >> logT;
  const int64_t nb = (rows + rpb - 1) / rpb;
  const int W2 = op->fwd.W2;
  const int rpg = op->tune.fwd_rows_per_group;
  if (W2 == 9 && logT >= 3 && rpg > 1) {
    const int64_t nbp = (rows + rpb * rpg - 1) / (rpb * rpg);
    if (rpg == 2)
      hipLaunchKernelGGL((k_fwd_pipe<CPL, V, 2>), dim3((unsigned)nbp), dim3(kBlock), 0, st,
                         op->fwd.col, (const V*)val, X, Y, rows, C, logT);
    else
      hipLaunchKernelGGL((k_fwd_pipe<CPL, V, 4>), dim3((unsigned)nbp), dim3(kBlock), 0, st,
                         op->fwd.col, (const V*)val, X, Y, rows, C, logT);
    TOMO_HIP(hipGetLastError());
    return TOMO_OK;
  }
  if (W2 == 9)
    hipLaunchKernelGGL((k_fwd_ell<CPL, V, 9>), dim3((unsigned)nb), dim3(kBlock), 0, st,
                       op->fwd.col, (const V*)val, X, Y, rows, C, logT, W2);
  else
    hipLaunchKernelGGL((k_fwd_ell<CPL, V, 0>), dim3((unsigned)nb), dim3(kBlock), 0, st,
                       op->fwd.col, (const V*)val, X, Y, rows, C, logT, W2);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

template <int CPL, typename V>
tomo_status adj_impl(const tomo_op* op, const DevAdj& d, int vt, const float2* Y, float2* X, int C,
                     const float* dscale, hipStream_t st) {
  AdjArgs a;
  a.logT = ilog2((C + CPL - 1) / CPL);
  const int64_t rpb = kBlock >> a.logT;
  a.slice_ptr = d.slice_ptr;
  a.slice_rows = d.slice_rows;
  a.col = d.col;
  a.n_slices = d.n_slices;
  a.nb_sell = (d.n_slices * kSliceRows + rpb - 1) / rpb;
  a.tail_rows = d.tail_rows;
  a.tail_ptr = d.tail_ptr;
  a.tail_col = d.tail_col;
  a.n_medium = d.n_medium;
  a.nb_medium = (d.n_medium + (kBlock / 64) - 1) / (kBlock / 64);
  a.chunk_beg = d.chunk_beg;
  a.chunk_end = d.chunk_end;
  a.n_chunks = d.n_chunks;
  a.partials = op->partials;
  a.Y = Y;
  a.X = X;
  a.C = C;
  a.dscale = dscale;
  a.inv_nt = 1.0 / (double)op->g.nt;
  // XCD interleave runs in blocks from the row counts (0 stays "contiguous")
  auto run_blocks = [](int rows, int64_t rows_per_block) {
    return rows <= 0 ? 0 : (int)std::max<int64_t>(1, rows / rows_per_block);
  };
  a.sell_chunk = run_blocks(op->tune.sell_xcd_rows, rpb);
  a.medium_chunk = run_blocks(op->tune.medium_xcd_rows, kBlock / 64);
  const V* v = (const V*)d.val[vt];
  const V* tv = (const V*)d.tail_val[vt];
#define TOMO_ADJ_LAUNCH(KERNEL, NB, VALS)                                                     \
  if ((NB) > 0) {                                                                          \
    if (dscale)                                                                            \
      hipLaunchKernelGGL((KERNEL<CPL, V, true>), dim3((unsigned)(NB)), dim3(kBlock), 0, st, a, VALS); \
    else                                                                                   \
      hipLaunchKernelGGL((KERNEL<CPL, V, false>), dim3((unsigned)(NB)), dim3(kBlock), 0, st, a, VALS); \
    TOMO_HIP(hipGetLastError());                                                           \
  }
  TOMO_ADJ_LAUNCH(k_adj_sell, a.nb_sell, v)
  TOMO_ADJ_LAUNCH(k_adj_medium, a.nb_medium, tv)
  TOMO_ADJ_LAUNCH(k_adj_chunk, a.n_chunks, tv)
#undef TOMO_ADJ_LAUNCH
  if (d.n_long > 0) {
    const int64_t nbl = (d.n_long + rpb - 1) / rpb;
    hipLaunchKernelGGL((k_adj_long_reduce<CPL>), dim3((unsigned)nbl), dim3(kBlock), 0, st,
                       d.tail_rows, d.long_chunk_ptr, op->partials, X, d.n_medium, d.n_long, C,
                       a.logT);
    TOMO_HIP(hipGetLastError());
  }
  return TOMO_OK;
}

template <typename V>
tomo_status fwd_cpl(const tomo_op* op, const void* val, const float2* X, float2* Y, int C,
                    hipStream_t st) {
  switch (pick_cpl(op->tune.fwd_cpl, C)) {
    case 1: return fwd_impl<1, V>(op, val, X, Y, C, st);
    case 2: return fwd_impl<2, V>(op, val, X, Y, C, st);
    case 4: return fwd_impl<4, V>(op, val, X, Y, C, st);
    default:
      return fail(TOMO_EUNSUPPORTED, "the row kernels take at most 64 lane groups: odd channel "
                  "counts above 64 (%d) need the staged forward (fwd_tiled)", C);
  }
}

template <typename V>
tomo_status adj_cpl(const tomo_op* op, const DevAdj& d, int vt, const float2* Y, float2* X, int C,
                    const float* dscale, hipStream_t st) {
  switch (pick_cpl(op->tune.adj_cpl, C)) {
    case 1: return adj_impl<1, V>(op, d, vt, Y, X, C, dscale, st);
    case 2: return adj_impl<2, V>(op, d, vt, Y, X, C, dscale, st);
    case 4: return adj_impl<4, V>(op, d, vt, Y, X, C, dscale, st);
    default:
      return fail(TOMO_EUNSUPPORTED, "the row kernels take at most 64 lane groups: odd channel "
                  "counts above 64 (%d) need the staged adjoint (adj_tiled)", C);
  }
}

}  // namespace

// The staged kernels run for this channel count and value type (and, for the adjoint, stage its
// dense tiles too): only then can the Cartesian grid be the channel-slowest FFT-side buffer.
bool spmm_fwd_slowest_ok(const tomo_op* op, int C, int vt) {
  return vt >= 0 && vt <= 2 && ((op->tune.fwd_tiled >> vt) & 1) && op->tiles_ready &&
         fwd_tile_supported(op) && fwd_tile_lds_bytes(op, C) <= kMaxTileLds;
}

bool spmm_adj_slowest_ok(const tomo_op* op, int C, int vt) {
  return vt >= 0 && vt <= 2 && op->adj_ready && ((op->tune.adj_tiled >> vt) & 1) &&
         op->tiles_ready && adj_tile_supported(op) && adj_seg_lds_bytes(op, C) <= kMaxTileLds;
}

tomo_status launch_spmm_fwd(const tomo_op* op, const float2* X, float2* Y, int C, int vt,
                            hipStream_t st, bool slow) {
  if (vt < 0 || vt > 2 || !op->fwd.val[vt])
    return fail(TOMO_ESTATE, "value type %d was not built for this operator", vt);
  if (C < 1 || C > op->cmax) return fail(TOMO_EINVAL, "channel count %d out of range", C);
  if (spmm_fwd_slowest_ok(op, C, vt)) return launch_fwd_tile(op, X, Y, C, vt, slow, st);
  if (slow) return fail(TOMO_EINVAL, "internal: channel-slowest grid without the staged forward");
  switch (vt) {
    case TOMO_VAL_F32: return fwd_cpl<float>(op, op->fwd.val[vt], X, Y, C, st);
    case TOMO_VAL_BF16: return fwd_cpl<bf16_t>(op, op->fwd.val[vt], X, Y, C, st);
    default: return fwd_cpl<_Float16>(op, op->fwd.val[vt], X, Y, C, st);
  }
}

tomo_status launch_spmm_adj(const tomo_op* op, const float2* Y, float2* X, int C, int vt,
                            const float* dscale, hipStream_t st, bool slow) {
  if (vt < 0 || vt > 2 || !(op->values & (1u << vt)))
    return fail(TOMO_ESTATE, "value type %d was not built for this operator", vt);
  if (!op->adj_ready) return fail(TOMO_ESTATE, "adjoint layout unavailable (failed re-tuning)");
  if (C < 1 || C > op->cmax) return fail(TOMO_EINVAL, "channel count %d out of range", C);
  auto rows = [&](const DevAdj& d, hipStream_t s) -> tomo_status {
    switch (vt) {
      case TOMO_VAL_F32: return adj_cpl<float>(op, d, vt, Y, X, C, dscale, s);
      case TOMO_VAL_BF16: return adj_cpl<bf16_t>(op, d, vt, Y, X, C, dscale, s);
      default: return adj_cpl<_Float16>(op, d, vt, Y, X, C, dscale, s);
    }
  };
  // the dense tiles' segments: for the FFT-side output (the row kernels write only the channel-
  // fastest grid), for channel counts the row kernels cannot take, and when adj_dense_mode
  // selects them
  if (spmm_adj_slowest_ok(op, C, vt) &&
      (slow || op->tune.adj_dense_mode != 0 || pick_cpl(op->tune.adj_cpl, C) == 0)) {
    if (op->tune.adj_dense_mode == 2)
      return launch_adj_seg(op, Y, X, C, vt, dscale, true, true, slow, st);
    // the dense tiles' segments on a second stream beside the staged tiles (disjoint cells)
    TOMO_HIP(hipEventRecord(op->ev_fork, st));
    TOMO_HIP(hipStreamWaitEvent(op->aux, op->ev_fork, 0));
    TOMO_TRY(launch_adj_seg(op, Y, X, C, vt, dscale, true, false, slow, op->aux));
    TOMO_HIP(hipEventRecord(op->ev_join, op->aux));
    TOMO_TRY(launch_adj_tile(op, Y, X, C, vt, dscale, slow, st));
    TOMO_HIP(hipStreamWaitEvent(st, op->ev_join, 0));
    return TOMO_OK;
  }
  if (slow) return fail(TOMO_EINVAL, "internal: channel-slowest grid without the staged adjoint");
  if (((op->tune.adj_tiled >> vt) & 1) && op->tiles_ready && adj_tile_supported(op) &&
      adj_tile_lds_bytes(op, C) <= kMaxTileLds) {
    // the dense cells' row kernels on two more streams (sliced-ELL rows; wave-per-row and
    // chunked rows), beside the staged tiles: all three write disjoint cells, and the caller's
    // stream waits for the other two
    DevAdj sell = op->adj_dense, tail = op->adj_dense;
    sell.n_medium = sell.n_long = sell.n_chunks = 0;
    tail.n_slices = 0;
    TOMO_HIP(hipEventRecord(op->ev_fork, st));
    TOMO_HIP(hipStreamWaitEvent(op->aux, op->ev_fork, 0));
    TOMO_HIP(hipStreamWaitEvent(op->aux2, op->ev_fork, 0));
    TOMO_TRY(rows(sell, op->aux));
    TOMO_HIP(hipEventRecord(op->ev_join, op->aux));
    TOMO_TRY(rows(tail, op->aux2));
    TOMO_HIP(hipEventRecord(op->ev_join2, op->aux2));
    TOMO_TRY(launch_adj_tile(op, Y, X, C, vt, dscale, false, st));
    TOMO_HIP(hipStreamWaitEvent(st, op->ev_join, 0));
    TOMO_HIP(hipStreamWaitEvent(st, op->ev_join2, 0));
    return TOMO_OK;
  }
  return rows(op->adj, st);
}

}  // namespace tomo
