// LDS-staged SpMM kernels for the slicing interpolation (Sec. 2.2, Sec. 3 Eq. (2)).
//
// Every Cartesian Fourier point is referenced by about nine polar samples (nnz / columns
// touched = 8.4 at 2048^2, 1501 angles), and the row-per-lane-group kernels fetch it from L2
// each time; measured, they are bound by that L2 gather traffic even when the whole grid is
// cache resident.  These kernels stage what a block reads in LDS once:
//
// forward  Y = S^dagger X: samples are grouped by the Cartesian tile (TS x TS) holding their
//          window centre; a block copies the tile plus its halo from X into LDS (the "patch",
//          PS x PS points x up to 16 complex channels) and the work item's sample records
//          (output row, first window slot, k_w^2 window-ordered values) with coalesced loads,
//          then evaluates every sample's k_w x k_w taps from LDS at fixed offsets from its first
//          slot.  A tap the matrix does not hold has value zero (it multiplies a finite patch
//          value).  Per sample the block issues no global load of its own: a tile's patch is one
//          load per point instead of one gather per tap (about 5x fewer line requests).
// adjoint  X = S diag(D) Y: a block owns one Cartesian tile of output cells and stages, with
//          coalesced loads, every polar sample whose window centre lies in the tile's region
//          (the tile grown by h; samples bucketed by centre cell): its row of Y (times D) and
//          its window values.  Cell m then sums, for each window position p, the samples of
//          the bucket at centre cell m + h - p times their value at p, reading only LDS, in a
//          fixed order (no atomics; run-to-run identical).  Regions holding more samples than
//          the block can stage (near the Fourier origin, where rows reach thousands of
//          entries) are left to the row kernels, which run on a layout of just those cells.
//
// A lane group of 8 lanes owns one output row at a time (a polar sample in the forward, a
// Cartesian cell in the adjoint); lane t holds CPL complex channels, so a block covers 8*CPL
// channels (grid.y walks the channel chunks).

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tomo {
namespace {

constexpr int kBlock = 256;
constexpr int kLanes = 8;
constexpr int kGroups = kBlock / kLanes;   // 32 lane groups per block

struct bf16_t { uint16_t bits; };
// Values are loaded raw under the load's predicate and converted afterwards, so that a batch of
// 16-bit loads is issued back to back instead of each waiting for its own conversion.
__device__ __forceinline__ uint32_t ldraw(const float* v, int64_t e) { return __float_as_uint(v[e]); }
__device__ __forceinline__ uint32_t ldraw(const bf16_t* v, int64_t e) { return v[e].bits; }
__device__ __forceinline__ uint32_t ldraw(const _Float16* v, int64_t e) {
  return *reinterpret_cast<const uint16_t*>(v + e);
}
__device__ __forceinline__ float cvt(const float*, uint32_t r) { return __uint_as_float(r); }
__device__ __forceinline__ float cvt(const bf16_t*, uint32_t r) { return __uint_as_float(r << 16); }
__device__ __forceinline__ float cvt(const _Float16*, uint32_t r) {
  const uint16_t h = (uint16_t)r;
  return (float)__builtin_bit_cast(_Float16, h);
}

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t x = bid & 7, local = bid >> 3;
  const int64_t q = nblocks >> 3, r = nblocks & 7;
  return (x < r) ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

template <int CPL>
struct Vec {
  float v[2 * CPL];
};

template <int CPL>
__device__ __forceinline__ void vzero(Vec<CPL>& a) {
#pragma unroll
  for (int i = 0; i < 2 * CPL; ++i) a.v[i] = 0.f;
}

template <int CPL>
__device__ __forceinline__ Vec<CPL> vload(const float2* p) {
  Vec<CPL> r;
  if constexpr (CPL == 1) {
    const float2 a = *p;
    r.v[0] = a.x; r.v[1] = a.y;
  } else {
    const float4 a = *reinterpret_cast<const float4*>(p);
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = a.z; r.v[3] = a.w;
  }
  return r;
}

template <int CPL>
__device__ __forceinline__ void vstore(float2* p, const Vec<CPL>& r) {
  if constexpr (CPL == 1)
    *p = make_float2(r.v[0], r.v[1]);
  else
    *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
}

__device__ __forceinline__ int wrap(int j, int G) { return j < 0 ? j + G : (j >= G ? j - G : j); }

// ------------------------------------------------------------------------------------------
// forward
// ------------------------------------------------------------------------------------------
struct FwdTileArgs {
  const int32_t* wi_tile;
  const int32_t* wi_beg;
  const int32_t* pt_row;
  const int32_t* pt_base;
  const float2* X;
  float2* Y;
  int C, G, oG, TS, NT, TP;
};

// Staging is written as batches of independent loads into registers followed by LDS stores, so
// a block pays one memory round trip per batch instead of one per element.
constexpr int kStageBatch = 8;
constexpr int kMaxTilePoints = 128;

template <int KW>
constexpr int window_stride() { return (KW * KW + 3) / 4 * 4; }   // LDS floats per sample

// MAXP: the most samples a work item may hold (a compile-time bound, so that the staging loops
// issue only the loads a block of that capacity can need)
template <int CPL, typename V, int KW, int PS, int MAXP>
__global__ __launch_bounds__(kBlock) void k_fwd_tile(FwdTileArgs a, const V* __restrict__ val) {
  constexpr int CH = kLanes * CPL, W2 = KW * KW, WP = window_stride<KW>(), H = KW / 2;
  constexpr int PP = PS * PS;
  constexpr int NPL = (PP * kLanes + kBlock - 1) / kBlock;            // patch loads per thread
  constexpr int NVL = (MAXP * W2 + kBlock - 1) / kBlock;              // value loads per thread
  extern __shared__ float2 smem[];
  float2* patch = smem;                                                      // [PP][CH]
  float* s_val = reinterpret_cast<float*>(patch + PP * CH);                  // [TP][WP]
  int* s_row = reinterpret_cast<int*>(s_val + a.TP * WP);                    // [TP]
  int* s_base = s_row + a.TP;                                                // [TP]
  const int wi = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int c0 = blockIdx.y * CH;
  const int nch = min(CH, a.C - c0);
  const int tl = a.wi_tile[wi];
  const int b0 = a.wi_beg[wi], ns = a.wi_beg[wi + 1] - b0;
  const int j01 = -a.oG + (tl / a.NT) * a.TS - H;
  const int j02 = -a.oG + (tl % a.NT) * a.TS - H;
  // issue every load of the block (sample records, then the patch) before the first LDS store
  uint32_t v[NVL];
#pragma unroll
  for (int u = 0; u < NVL; ++u) {
    const int k = threadIdx.x + u * kBlock;
    v[u] = 0;
    if (k < ns * W2) v[u] = ldraw(val, (int64_t)b0 * W2 + k);
  }
  int rw = 0, bs = 0;
  if ((int)threadIdx.x < ns) {
    rw = a.pt_row[b0 + threadIdx.x];
    bs = a.pt_base[b0 + threadIdx.x];
  }
  constexpr int NB = NPL < kStageBatch ? NPL : kStageBatch;
  for (int base = 0; base < NPL; base += NB) {
    Vec<CPL> x[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = threadIdx.x + (base + u) * kBlock;
      const int p = idx / kLanes, l = (idx % kLanes) * CPL;
      if (idx < PP * kLanes && l < nch) {
        const int g1 = wrap(j01 + p / PS, a.G), g2 = wrap(j02 + p % PS, a.G);
        x[u] = vload<CPL>(a.X + ((int64_t)g1 * a.G + g2) * a.C + c0 + l);
      }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = threadIdx.x + (base + u) * kBlock;
      const int p = idx / kLanes, l = (idx % kLanes) * CPL;
      if (idx < PP * kLanes && l < nch) vstore<CPL>(patch + p * CH + l, x[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < NVL; ++u) {
    const int k = threadIdx.x + u * kBlock;
    if (k < ns * W2) s_val[(k / W2) * WP + k % W2] = cvt(val, v[u]);
  }
  if ((int)threadIdx.x < ns) {
    s_row[threadIdx.x] = rw;
    s_base[threadIdx.x] = bs;
  }
  __syncthreads();
  const int g = threadIdx.x / kLanes;
  const int cl = (threadIdx.x % kLanes) * CPL;
  if (cl >= nch) return;
  for (int i = g; i < ns; i += kGroups) {
    const float2* p = patch + s_base[i] * CH + cl;
    const float* w = s_val + i * WP;
    Vec<CPL> acc;
    vzero(acc);
#pragma unroll
    for (int s1 = 0; s1 < KW; ++s1)
#pragma unroll
      for (int s2 = 0; s2 < KW; ++s2) {
        const Vec<CPL> x = vload<CPL>(p + (s1 * PS + s2) * CH);
        const float ws = w[s1 * KW + s2];
#pragma unroll
        for (int k = 0; k < 2 * CPL; ++k) acc.v[k] += ws * x.v[k];
      }
    vstore<CPL>(a.Y + (int64_t)s_row[i] * a.C + c0 + cl, acc);
  }
}

// ------------------------------------------------------------------------------------------
// adjoint
// ------------------------------------------------------------------------------------------
struct AdjWinArgs {
  const int32_t* wi_tile;
  const int32_t* wi_q;
  const uint16_t* wi_boff;
  const int32_t* q_row;
  const float2* Y;
  float2* X;
  const float* dscale;        // per FFT-ordered radial index, or null
  int C, G, oG, NT, nt, QMAX;
};

constexpr int kMaxAdjPoints = 256;

// One block per staged tile, placed by an XCD-aware remap so that neighbouring tiles share an
// L2.  The block loads its list offsets, then its sample rows, values and bucket offsets, then
// the rows of Y those samples name.
template <int CPL, typename V, int KW, int TS, bool SCALE, int MAXP>
__global__ __launch_bounds__(kBlock) void k_adj_win(AdjWinArgs a, const V* __restrict__ val) {
  constexpr int CH = kLanes * CPL, W2 = KW * KW, WP = window_stride<KW>(), H = KW / 2;
  constexpr int RS = TS + 2 * H, NBO = RS * RS + 1;
  constexpr int NBL = (NBO + kBlock - 1) / kBlock;                      // bucket offsets
  constexpr int NVL = (MAXP * W2 + kBlock - 1) / kBlock;                // value loads
  constexpr int NYL = (MAXP * kLanes + kBlock - 1) / kBlock;            // row loads
  extern __shared__ float2 smem[];
  float2* sy = smem;                                                     // [QMAX][CH]
  float* sv = reinterpret_cast<float*>(sy + a.QMAX * CH);                // [QMAX][WP]
  int* sb = reinterpret_cast<int*>(sv + a.QMAX * WP);                    // [NBO]
  const int wi = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int c0 = blockIdx.y * CH;
  const int nch = min(CH, a.C - c0);
  const int tl = a.wi_tile[wi];
  const int q0 = a.wi_q[wi], nq = a.wi_q[wi + 1] - q0;
  int bo[NBL];
#pragma unroll
  for (int u = 0; u < NBL; ++u) {
    const int k = threadIdx.x + u * kBlock;
    bo[u] = (k < NBO) ? (int)a.wi_boff[(int64_t)wi * NBO + k] : 0;
  }
  uint32_t v[NVL];
#pragma unroll
  for (int u = 0; u < NVL; ++u) {
    const int k = threadIdx.x + u * kBlock;
    v[u] = 0;
    if (k < nq * W2) v[u] = ldraw(val, (int64_t)q0 * W2 + k);
  }
  int r[NYL];
#pragma unroll
  for (int u = 0; u < NYL; ++u) {
    const int idx = threadIdx.x + u * kBlock;
    const int l = (idx % kLanes) * CPL;
    r[u] = (idx < nq * kLanes && l < nch) ? a.q_row[q0 + idx / kLanes] : -1;
  }
  Vec<CPL> y[NYL];
#pragma unroll
  for (int u = 0; u < NYL; ++u) {
    const int idx = threadIdx.x + u * kBlock;
    const int l = (idx % kLanes) * CPL;
    if (r[u] >= 0) y[u] = vload<CPL>(a.Y + (int64_t)r[u] * a.C + c0 + l);
  }
  if constexpr (SCALE) {
#pragma unroll
    for (int u = 0; u < NYL; ++u)
      if (r[u] >= 0) {
        const float d = a.dscale[r[u] / a.nt];
#pragma unroll
        for (int k = 0; k < 2 * CPL; ++k) y[u].v[k] *= d;
      }
  }
#pragma unroll
  for (int u = 0; u < NBL; ++u) {
    const int k = threadIdx.x + u * kBlock;
    if (k < NBO) sb[k] = bo[u];
  }
#pragma unroll
  for (int u = 0; u < NVL; ++u) {
    const int k = threadIdx.x + u * kBlock;
    if (k < nq * W2) sv[(k / W2) * WP + k % W2] = cvt(val, v[u]);
  }
#pragma unroll
  for (int u = 0; u < NYL; ++u) {
    const int idx = threadIdx.x + u * kBlock;
    if (r[u] >= 0) vstore<CPL>(sy + (idx / kLanes) * CH + (idx % kLanes) * CPL, y[u]);
  }
  __syncthreads();
  const int g = threadIdx.x / kLanes;
  const int cl = (threadIdx.x % kLanes) * CPL;
  if (cl >= nch) return;
  const int jb1 = -a.oG + (tl / a.NT) * TS, jb2 = -a.oG + (tl % a.NT) * TS;
  for (int c = g; c < TS * TS; c += kGroups) {
    const int m1 = c / TS, m2 = c % TS;
    const int j1 = jb1 + m1, j2 = jb2 + m2;
    if (j1 > a.G - 1 - a.oG || j2 > a.G - 1 - a.oG) continue;   // past the grid's end
    Vec<CPL> acc;
    vzero(acc);
    // for window row p1 the k_w buckets (centre cells (m1 + 2h - p1, m2 + t), t < k_w) are
    // consecutive in the region, so their samples form one run; bucket t holds window column
    // p2 = 2h - t.  One loop per window row instead of one per bucket.
#pragma unroll
    for (int p1 = 0; p1 < KW; ++p1) {
      const int rb = (m1 + 2 * H - p1) * RS + m2;
      int o[KW + 1];
#pragma unroll
      for (int t = 0; t <= KW; ++t) o[t] = sb[rb + t];
      const float* wrow = sv + p1 * KW + 2 * H;
      for (int k = o[0]; k < o[KW]; ++k) {
        int t = 0;
#pragma unroll
        for (int u = 1; u < KW; ++u) t += (k >= o[u]) ? 1 : 0;
        const float w = wrow[k * WP - t];
        const Vec<CPL> x = vload<CPL>(sy + k * CH + cl);
#pragma unroll
        for (int q = 0; q < 2 * CPL; ++q) acc.v[q] += w * x.v[q];
      }
    }
    vstore<CPL>(a.X + ((int64_t)wrap(j1, a.G) * a.G + wrap(j2, a.G)) * a.C + c0 + cl, acc);
  }
}

template <int CPL, typename V>
tomo_status fwd_tile_impl(const tomo_op* op, int vt, const float2* X, float2* Y, int C,
                          hipStream_t st) {
  const DevFwdTiles& d = op->ftile;
  constexpr int CH = kLanes * CPL;
  FwdTileArgs a{d.wi_tile, d.wi_beg, d.pt_row, d.pt_base, X, Y,
                C, op->g.G, op->g.G / 2, d.TS, d.NT, op->tune.tile_points};
  const size_t lds = fwd_tile_lds_bytes(op, C);
  dim3 grid((unsigned)d.n_wi, (unsigned)((C + CH - 1) / CH));
  const V* v = (const V*)d.val[vt];
  const bool small = op->tune.tile_points <= 64;
#define TOMO_FWD_TILE(KW_, TS_)                                                                  \
  if (d.KW == KW_ && d.TS == TS_) {                                                             \
    constexpr int PS_ = TS_ + 2 * (KW_ / 2) + 1;                                                \
    if (small)                                                                                  \
      hipLaunchKernelGGL((k_fwd_tile<CPL, V, KW_, PS_, 64>), grid, dim3(kBlock), lds, st, a, v); \
    else                                                                                        \
      hipLaunchKernelGGL((k_fwd_tile<CPL, V, KW_, PS_, kMaxTilePoints>), grid, dim3(kBlock), lds, \
                         st, a, v);                                                             \
    TOMO_HIP(hipGetLastError());                                                                \
    return TOMO_OK;                                                                             \
  }
  TOMO_FWD_TILE(3, 8) TOMO_FWD_TILE(3, 16) TOMO_FWD_TILE(5, 8) TOMO_FWD_TILE(5, 16)
#undef TOMO_FWD_TILE
  return fail(TOMO_EUNSUPPORTED, "staged forward kernel has no variant for k_w %d, tile %d", d.KW,
              d.TS);
}

template <int CPL, typename V>
tomo_status adj_tile_impl(const tomo_op* op, int vt, const float2* Y, float2* X, int C,
                          const float* dscale, hipStream_t st) {
  const DevAdjWin& d = op->awin;
  if (d.n_wi == 0) return TOMO_OK;
  constexpr int CH = kLanes * CPL;
  AdjWinArgs a{d.wi_tile, d.wi_q, d.wi_boff, d.q_row, Y, X, dscale,
               C, op->g.G, op->g.G / 2, d.NT, op->g.nt, d.QMAX};
  const size_t lds = adj_tile_lds_bytes(op, C);
  dim3 grid((unsigned)d.n_wi, (unsigned)((C + CH - 1) / CH));
  const V* v = (const V*)d.q_val[vt];
  const bool small = d.QMAX <= 128;
#define TOMO_ADJ_WIN_P(KW_, TS_, P_)                                                             \
  if (dscale)                                                                                   \
    hipLaunchKernelGGL((k_adj_win<CPL, V, KW_, TS_, true, P_>), grid, dim3(kBlock), lds, st, a, v); \
  else                                                                                          \
    hipLaunchKernelGGL((k_adj_win<CPL, V, KW_, TS_, false, P_>), grid, dim3(kBlock), lds, st, a, v);
#define TOMO_ADJ_WIN(KW_, TS_)                                                                   \
  if (d.KW == KW_ && d.TS == TS_) {                                                             \
    if (small) {                                                                                \
      TOMO_ADJ_WIN_P(KW_, TS_, 128)                                                             \
    } else {                                                                                    \
      TOMO_ADJ_WIN_P(KW_, TS_, kMaxAdjPoints)                                                   \
    }                                                                                           \
    TOMO_HIP(hipGetLastError());                                                                \
    return TOMO_OK;                                                                             \
  }
  TOMO_ADJ_WIN(3, 8) TOMO_ADJ_WIN(3, 16) TOMO_ADJ_WIN(5, 8) TOMO_ADJ_WIN(5, 16)
#undef TOMO_ADJ_WIN
#undef TOMO_ADJ_WIN_P
  return fail(TOMO_EUNSUPPORTED, "staged adjoint kernel has no variant for k_w %d, tile %d", d.KW,
              d.TS);
}

}  // namespace

bool fwd_tile_supported(const tomo_op* op) {
  const DevFwdTiles& d = op->ftile;
  return (d.KW == 3 || d.KW == 5) && (d.TS == 8 || d.TS == 16) &&
         op->tune.tile_points <= kMaxTilePoints;
}

size_t fwd_tile_lds_bytes(const tomo_op* op, int C) {
  const int cpl = (C % 2 == 0) ? 2 : 1;
  const DevFwdTiles& d = op->ftile;
  const int wp = (d.KW * d.KW + 3) / 4 * 4;
  return (size_t)d.PS * d.PS * kLanes * cpl * sizeof(float2) +
         (size_t)op->tune.tile_points * (wp * sizeof(float) + 2 * sizeof(int));
}

bool adj_tile_supported(const tomo_op* op) {
  const DevAdjWin& d = op->awin;
  return (d.KW == 3 || d.KW == 5) && (d.TS == 8 || d.TS == 16) && d.QMAX <= kMaxAdjPoints;
}

size_t adj_tile_lds_bytes(const tomo_op* op, int C) {
  const int cpl = (C % 2 == 0) ? 2 : 1;
  const DevAdjWin& d = op->awin;
  const int wp = (d.KW * d.KW + 3) / 4 * 4;
  return (size_t)d.QMAX * (kLanes * cpl * sizeof(float2) + wp * sizeof(float)) +
         (size_t)(d.RS * d.RS + 1) * sizeof(int);
}

tomo_status launch_fwd_tile(const tomo_op* op, const float2* X, float2* Y, int C, int vt,
                            hipStream_t st) {
  const bool even = (C % 2 == 0);
  switch (vt) {
    case TOMO_VAL_F32:
      return even ? fwd_tile_impl<2, float>(op, vt, X, Y, C, st) : fwd_tile_impl<1, float>(op, vt, X, Y, C, st);
    case TOMO_VAL_BF16:
      return even ? fwd_tile_impl<2, bf16_t>(op, vt, X, Y, C, st) : fwd_tile_impl<1, bf16_t>(op, vt, X, Y, C, st);
    default:
      return even ? fwd_tile_impl<2, _Float16>(op, vt, X, Y, C, st) : fwd_tile_impl<1, _Float16>(op, vt, X, Y, C, st);
  }
}

tomo_status launch_adj_tile(const tomo_op* op, const float2* Y, float2* X, int C, int vt,
                            const float* dscale, hipStream_t st) {
  const bool even = (C % 2 == 0);
  switch (vt) {
    case TOMO_VAL_F32:
      return even ? adj_tile_impl<2, float>(op, vt, Y, X, C, dscale, st) : adj_tile_impl<1, float>(op, vt, Y, X, C, dscale, st);
    case TOMO_VAL_BF16:
      return even ? adj_tile_impl<2, bf16_t>(op, vt, Y, X, C, dscale, st) : adj_tile_impl<1, bf16_t>(op, vt, Y, X, C, dscale, st);
    default:
      return even ? adj_tile_impl<2, _Float16>(op, vt, Y, X, C, dscale, st) : adj_tile_impl<1, _Float16>(op, vt, Y, X, C, dscale, st);
  }
}

}  // namespace tomo
