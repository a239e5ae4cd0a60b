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

#include <algorithm>
#include <vector>

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
  const float2* X;            // plane == 0: [G*G][C] channel-fastest; else [C][G*G] (plane = G*G)
  float2* Y;                  // yplane == 0: [L*nt][C], row kf*nt + a; else [C][nt][L] (yplane = nt*L)
  int C, G, oG, TS, NT, TP;
  int64_t plane, yplane;
  int nt, L;
};

// Staging is written as batches of independent loads into registers followed by LDS stores, so
// a block pays one memory round trip per batch instead of one per element.
constexpr int kStageBatch = 8;
constexpr int kMaxTilePoints = 128;

template <int KW>
constexpr int window_stride() { return (KW * KW + 3) / 4 * 4; }   // LDS floats per sample

// One forward work item wi (channels c0 .. c0 + 8*CPL - 1) of a block; smem holds the patch, the
// values and the sample records.  MAXP: the most samples a work item may hold (a compile-time
// bound, so that the staging loops issue only the loads a block of that capacity can need).
template <int CPL, typename V, int KW, int PS, int MAXP, bool SLOW>
__device__ __forceinline__ void fwd_tile_body(const FwdTileArgs& a, const V* __restrict__ val,
                                              int wi, int c0, float2* smem) {
  constexpr int CH = kLanes * CPL, W2 = KW * KW, WP = window_stride<KW>(), H = KW / 2;
  constexpr int PP = PS * PS;
  constexpr int NPL = (PP * kLanes + kBlock - 1) / kBlock;            // patch loads per thread
  constexpr int NVL = (MAXP * W2 + kBlock - 1) / kBlock;              // value loads per thread
  float2* patch = smem;                                                      // [PP][CH]
  float* s_val = reinterpret_cast<float*>(patch + PP * CH);                  // [TP][WP]
  int* s_row = reinterpret_cast<int*>(s_val + a.TP * WP);                    // [TP]
  int* s_base = s_row + a.TP;                                                // [TP]
  const int nch = min(CH, a.C - c0);
  const int tl = a.wi_tile[wi];
  const int b0 = a.wi_beg[wi], ns = a.wi_beg[wi + 1] - b0;
  const int j01 = -a.oG + (tl / a.NT) * a.TS - H;
  const int j02 = -a.oG + (tl % a.NT) * a.TS - H;
  // issue every load of the block (sample records, then the patch) before the first LDS store
  uint32_t v[NVL];
#pragma unroll
  for (int u = 0; u < NVL; ++u) {   // every load issued; entries past the item are never stored
    const int k = threadIdx.x + u * kBlock;
    v[u] = ldraw(val, (k < ns * W2) ? (int64_t)b0 * W2 + k : 0);
  }
  int rw = 0, bs = 0;
  if ((int)threadIdx.x < ns) {
    rw = a.pt_row[b0 + threadIdx.x];
    bs = a.pt_base[b0 + threadIdx.x];
  }
  constexpr int NB = NPL < kStageBatch ? NPL : kStageBatch;
  if constexpr (!SLOW) {
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
  } else {
    // channel-slowest grid: point fastest across threads, so that each patch row is one run of
    // PS points in every channel plane
    for (int base = 0; base < NPL; base += NB) {
      Vec<CPL> x[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int idx = threadIdx.x + (base + u) * kBlock;
        const int p = idx % PP, l = (idx / PP) * CPL;
        if (idx < PP * kLanes && l < nch) {
          const int64_t cell = (int64_t)wrap(j01 + p / PS, a.G) * a.G + wrap(j02 + p % PS, a.G);
#pragma unroll
          for (int k = 0; k < CPL; ++k) {
            const float2 v = a.X[(int64_t)(c0 + l + k) * a.plane + cell];
            x[u].v[2 * k] = v.x;
            x[u].v[2 * k + 1] = v.y;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int idx = threadIdx.x + (base + u) * kBlock;
        const int p = idx % PP, l = (idx / PP) * CPL;
        if (idx < PP * kLanes && l < nch) vstore<CPL>(patch + p * CH + l, x[u]);
      }
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
  // lane groups: 8 neighbouring lanes share a sample and split its channels (the channel-
  // fastest output row is one 8*CH-byte run); for the channel-slowest output, 32 neighbouring
  // lanes take 32 consecutive samples of one channel group instead, so that a store covers
  // runs of consecutive radii of each channel plane (measured: project 1.160 -> 1.141 ms at
  // 2048^2 x 32)
  const int g = SLOW ? (int)threadIdx.x % kGroups : (int)threadIdx.x / kLanes;
  const int cl = (SLOW ? (int)threadIdx.x / kGroups : (int)threadIdx.x % kLanes) * CPL;
  if (cl < nch) {
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
      if constexpr (!SLOW) {
        vstore<CPL>(a.Y + (int64_t)s_row[i] * a.C + c0 + cl, acc);
      } else {
        // channel-slowest polar rows: sample (kf, a) at a*L + kf of every channel plane; the
        // samples of a tile are ordered by angle, then radius, so neighbouring lanes write runs
        // of consecutive radii
        const int r = s_row[i], kf = r / a.nt;
        const int64_t at = (int64_t)(r - kf * a.nt) * a.L + kf;
#pragma unroll
        for (int k = 0; k < CPL; ++k)
          a.Y[(int64_t)(c0 + cl + k) * a.yplane + at] = make_float2(acc.v[2 * k], acc.v[2 * k + 1]);
      }
    }
  }
}

// SLOW: the FFT-side layouts (X channel-slowest, Y channel-slowest rows) instead of the
// channel-fastest ones
template <int CPL, typename V, int KW, int PS, int MAXP, bool SLOW>
__global__ __launch_bounds__(kBlock) void k_fwd_tile(FwdTileArgs a, const V* __restrict__ val) {
  extern __shared__ float2 smem[];
  fwd_tile_body<CPL, V, KW, PS, MAXP, SLOW>(a, val, (int)xcd_remap(blockIdx.x, gridDim.x),
                                            blockIdx.y * kLanes * CPL, smem);
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
  float2* X;                  // plane == 0: [G*G][C] channel-fastest; else [C][G*G] (plane = G*G)
  const float* dscale;        // per FFT-ordered radial index, or null
  int C, G, oG, NT, nt, QMAX;
  int64_t plane;
};

// Store the CPL channels ch0 .. of grid cell `cell`: one 8*CPL-byte store into the channel-
// fastest grid, or (SLOW) one float2 per channel plane of the channel-slowest grid (the 8 cells
// of a tile row, held by neighbouring lane groups, then form one 64-byte run per plane).  The
// layout is a compile-time choice, so that the channel-fastest kernels are scheduled on their own.
template <int CPL, bool SLOW>
__device__ __forceinline__ void store_cell(float2* X, int64_t cell, int C, int ch0, int64_t plane,
                                           const Vec<CPL>& v) {
  if constexpr (!SLOW) {
    vstore<CPL>(X + cell * C + ch0, v);
  } else {
#pragma unroll
    for (int k = 0; k < CPL; ++k) X[(int64_t)(ch0 + k) * plane + cell] = make_float2(v.v[2 * k], v.v[2 * k + 1]);
  }
}

// Chunked segments of the dense tiles (and, in one launch, the staged tiles as one-chunk
// segments).  Blocks b < n_first run segments seg0 + b in dispatch order (the long dense
// segments start first, spread over the XCDs); the others run segments seg1 + j, j the
// XCD-aware remap of b - n_first (neighbouring tiles on one XCD).
struct AdjSegArgs {
  AdjWinArgs w;               // chunk arrays (wi_q, wi_boff indexed by chunk), Y, X, scale
  const int32_t* seg_tile;
  const int32_t* seg_chunk;
  const int32_t* seg_slot;
  const int32_t* chunk_tile;  // tile of every chunk
  float2* part;               // [n_slot][TS*TS][C] partial tiles
  int seg0, n_first, seg1;
  int max_chunks;             // most chunks of any segment
};

constexpr int kMaxAdjPoints = 256;

template <int KW, int TS>
struct AdjShape {
  static constexpr int W2 = KW * KW, WP = window_stride<KW>(), H = KW / 2;
  static constexpr int RS = TS + 2 * H, NBO = RS * RS + 1;
};

// Registers of one chunk between its loads and its LDS stores: bucket offsets, raw window values,
// polar rows and the rows of Y they name.
template <int CPL, int KW, int TS, int MAXP>
struct ChunkRegs {
  using S = AdjShape<KW, TS>;
  static constexpr int NBL = (S::NBO + kBlock - 1) / kBlock;             // bucket offsets
  static constexpr int NVL = (MAXP * S::W2 + kBlock - 1) / kBlock;        // value loads
  static constexpr int NYL = (MAXP * kLanes + kBlock - 1) / kBlock;       // row loads
  int bo[NBL];
  uint32_t v[NVL];
  int r[NYL];
  Vec<CPL> y[NYL];
  int nq;
};

// Issue the loads of chunk w's bucket offsets, values and polar rows (samples q0 .. q0+nq-1).
template <int CPL, typename V, int KW, int TS, int MAXP>
__device__ __forceinline__ void chunk_meta(const AdjWinArgs& a, const V* __restrict__ val, int w,
                                           int q0, int nq, int nch, ChunkRegs<CPL, KW, TS, MAXP>& R) {
  using S = AdjShape<KW, TS>;
  using CR = ChunkRegs<CPL, KW, TS, MAXP>;
  R.nq = nq;
#pragma unroll
  for (int u = 0; u < CR::NBL; ++u) {
    const int k = threadIdx.x + u * kBlock;
    R.bo[u] = (k < S::NBO) ? (int)a.wi_boff[(int64_t)w * S::NBO + k] : 0;
  }
  // every value load is issued (entries past the chunk read entry 0 and are never stored): a
  // predicated 16-bit load was compiled into a load-and-wait per value, serialising them
#pragma unroll
  for (int u = 0; u < CR::NVL; ++u) {
    const int k = threadIdx.x + u * kBlock;
    R.v[u] = ldraw(val, (k < nq * S::W2) ? (int64_t)q0 * S::W2 + k : 0);
  }
#pragma unroll
  for (int u = 0; u < CR::NYL; ++u) {
    const int idx = threadIdx.x + u * kBlock;
    const int l = (idx % kLanes) * CPL;
    R.r[u] = (idx < nq * kLanes && l < nch) ? a.q_row[q0 + idx / kLanes] : -1;
  }
}

// Issue the loads of the rows of Y the chunk's samples name.
template <int CPL, int KW, int TS, int MAXP>
__device__ __forceinline__ void chunk_rows(const AdjWinArgs& a, int c0, ChunkRegs<CPL, KW, TS, MAXP>& R) {
  using CR = ChunkRegs<CPL, KW, TS, MAXP>;
#pragma unroll
  for (int u = 0; u < CR::NYL; ++u) {
    const int idx = threadIdx.x + u * kBlock;
    const int l = (idx % kLanes) * CPL;
    if (R.r[u] >= 0) R.y[u] = vload<CPL>(a.Y + (int64_t)R.r[u] * a.C + c0 + l);
  }
}

// Scale the rows by D (SCALE) and store the chunk to LDS.
template <int CPL, typename V, int KW, int TS, bool SCALE, int MAXP>
__device__ __forceinline__ void chunk_store(const AdjWinArgs& a, const V* __restrict__ val,
                                            ChunkRegs<CPL, KW, TS, MAXP>& R, float2* sy, float* sv,
                                            int* sb) {
  using S = AdjShape<KW, TS>;
  using CR = ChunkRegs<CPL, KW, TS, MAXP>;
  constexpr int CH = kLanes * CPL;
  if constexpr (SCALE) {
#pragma unroll
    for (int u = 0; u < CR::NYL; ++u)
      if (R.r[u] >= 0) {
        const float d = a.dscale[R.r[u] / a.nt];
#pragma unroll
        for (int k = 0; k < 2 * CPL; ++k) R.y[u].v[k] *= d;
      }
  }
#pragma unroll
  for (int u = 0; u < CR::NBL; ++u) {
    const int k = threadIdx.x + u * kBlock;
    if (k < S::NBO) sb[k] = R.bo[u];
  }
#pragma unroll
  for (int u = 0; u < CR::NVL; ++u) {
    const int k = threadIdx.x + u * kBlock;
    if (k < R.nq * S::W2) sv[(k / S::W2) * S::WP + k % S::W2] = cvt(val, R.v[u]);
  }
#pragma unroll
  for (int u = 0; u < CR::NYL; ++u) {
    const int idx = threadIdx.x + u * kBlock;
    if (R.r[u] >= 0) vstore<CPL>(sy + (idx / kLanes) * CH + (idx % kLanes) * CPL, R.y[u]);
  }
}

// Stage one chunk (work item) w into LDS: its bucket offsets, window values and the rows of Y
// its samples name (times D when SCALE).  All loads of a kind are issued before the LDS stores.
template <int CPL, typename V, int KW, int TS, bool SCALE, int MAXP>
__device__ __forceinline__ void adj_stage(const AdjWinArgs& a, const V* __restrict__ val, int w,
                                          int c0, int nch, float2* sy, float* sv, int* sb) {
  ChunkRegs<CPL, KW, TS, MAXP> R;
  const int q0 = a.wi_q[w];
  chunk_meta<CPL, V, KW, TS, MAXP>(a, val, w, q0, a.wi_q[w + 1] - q0, nch, R);
  chunk_rows<CPL, KW, TS, MAXP>(a, c0, R);
  chunk_store<CPL, V, KW, TS, SCALE, MAXP>(a, val, R, sy, sv, sb);
}

// Add to acc the staged chunk's contributions to tile cell (m1, m2), channels cl .. cl+CPL-1:
// for window row p1 the k_w buckets (centre cells (m1 + 2h - p1, m2 + t), t < k_w) are
// consecutive in the region, so their samples form one run; bucket t holds window column
// p2 = 2h - t.  One loop per window row instead of one per bucket.
template <int CPL, int KW, int TS>
__device__ __forceinline__ void adj_cell(Vec<CPL>& acc, const float2* sy, const float* sv,
                                         const int* sb, int m1, int m2, int cl) {
  using S = AdjShape<KW, TS>;
  constexpr int CH = kLanes * CPL, WP = S::WP, H = S::H, RS = S::RS;
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
}

// adj_cell summing into float64 totals: each product rounded once in float32, the sums exact to
// float64 (cells near the Fourier origin sum thousands of same-sign terms)
template <int CPL, int KW, int TS>
__device__ __forceinline__ void adj_cell_f64(double (&tot)[2 * CPL], const float2* sy,
                                             const float* sv, const int* sb, int m1, int m2, int cl) {
  using S = AdjShape<KW, TS>;
  constexpr int CH = kLanes * CPL, WP = S::WP, H = S::H, RS = S::RS;
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
      for (int q = 0; q < 2 * CPL; ++q) tot[q] += (double)(w * x.v[q]);
    }
  }
}

// One block per staged tile, placed by an XCD-aware remap so that neighbouring tiles share an
// L2.  The block loads its list offsets, then its sample rows, values and bucket offsets, then
// the rows of Y those samples name.
template <int CPL, typename V, int KW, int TS, bool SCALE, int MAXP, bool SLOW>
__global__ __launch_bounds__(kBlock) void k_adj_win(AdjWinArgs a, const V* __restrict__ val) {
  using S = AdjShape<KW, TS>;
  constexpr int CH = kLanes * CPL;
  extern __shared__ float2 smem[];
  float2* sy = smem;                                                     // [QMAX][CH]
  float* sv = reinterpret_cast<float*>(sy + a.QMAX * CH);                // [QMAX][WP]
  int* sb = reinterpret_cast<int*>(sv + a.QMAX * S::WP);                 // [NBO]
  const int wi = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int c0 = blockIdx.y * CH;
  const int nch = min(CH, a.C - c0);
  const int tl = a.wi_tile[wi];
  adj_stage<CPL, V, KW, TS, SCALE, MAXP>(a, val, wi, c0, nch, sy, sv, sb);
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
    adj_cell<CPL, KW, TS>(acc, sy, sv, sb, m1, m2, cl);
    store_cell<CPL, SLOW>(a.X, (int64_t)wrap(j1, a.G) * a.G + wrap(j2, a.G), a.C, c0 + cl, a.plane, acc);
  }
}

// Segment sg (channels c0 .. c0 + 8*CPL - 1) of a block: its chunks in order, each staged in
// LDS and summed into the cells' registers.  When the next chunk belongs to another tile (a run
// of staged tiles), or at the end, the tile's sums go to X, or to the segment's partial slot when
// its tile is split over several segments; sums run over chunks in order (run-to-run identical).
// (Loading the next chunk while summing the current one needs a second register set; at 106
// VGPRs that halved the blocks per CU and was slower.)
template <int CPL, typename V, int KW, int TS, bool SCALE, int MAXP, bool SLOW>
__device__ __forceinline__ void adj_seg_body(const AdjSegArgs& s, const V* __restrict__ val, int sg,
                                             int c0, float2* smem) {
  using S = AdjShape<KW, TS>;
  constexpr int CH = kLanes * CPL, NC = (TS * TS + kGroups - 1) / kGroups;
  const AdjWinArgs& a = s.w;
  float2* sy = smem;
  float* sv = reinterpret_cast<float*>(sy + a.QMAX * CH);
  int* sb = reinterpret_cast<int*>(sv + a.QMAX * S::WP);
  const int nch = min(CH, a.C - c0);
  const int k0 = s.seg_chunk[sg], n = s.seg_chunk[sg + 1] - k0;
  const int slot = s.seg_slot[sg];
  const int g = threadIdx.x / kLanes;
  const int cl = (threadIdx.x % kLanes) * CPL;
  // every cell's sum in float64 over all its chunks (products rounded once in float32): the cell
  // at the Fourier origin sums 4,743 same-sign terms, up to ~130 of them from one chunk, and
  // float32 sums there (running over the chunks: 3.8e-5; within each chunk: 5e-6) moved a 2048^2
  // back-projection through the DC coefficient by more than the row kernels' tree sums do
  double tot[NC][2 * CPL];
#pragma unroll
  for (int u = 0; u < NC; ++u)
#pragma unroll
    for (int q = 0; q < 2 * CPL; ++q) tot[u][q] = 0.0;
  // chunk bounds and tiles are uniform across the block (scalar loads, issued per chunk)
  int tl = s.chunk_tile[k0];
  for (int i = 0; i < n; ++i) {
    if (i > 0) __syncthreads();                    // the previous chunk's reads are done
    const int q0 = a.wi_q[k0 + i], q1 = a.wi_q[k0 + i + 1];
    const int next_tl = (i + 1 < n) ? s.chunk_tile[k0 + i + 1] : -1;
    {
      ChunkRegs<CPL, KW, TS, MAXP> R;
      chunk_meta<CPL, V, KW, TS, MAXP>(a, val, k0 + i, q0, q1 - q0, nch, R);
      chunk_rows<CPL, KW, TS, MAXP>(a, c0, R);
      chunk_store<CPL, V, KW, TS, SCALE, MAXP>(a, val, R, sy, sv, sb);
    }
    __syncthreads();
    if (cl < nch) {
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const int c = g + u * kGroups;
        if (c < TS * TS) adj_cell_f64<CPL, KW, TS>(tot[u], sy, sv, sb, c / TS, c % TS, cl);
      }
    }
    if (next_tl == tl) continue;
    if (cl < nch) {
      const int jb1 = -a.oG + (tl / a.NT) * TS, jb2 = -a.oG + (tl % a.NT) * TS;
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const int c = g + u * kGroups;
        if (c >= TS * TS) continue;
        Vec<CPL> out;
#pragma unroll
        for (int q = 0; q < 2 * CPL; ++q) out.v[q] = (float)tot[u][q];
        if (slot >= 0) {
          vstore<CPL>(s.part + ((int64_t)slot * TS * TS + c) * a.C + c0 + cl, out);
        } else {
          const int j1 = jb1 + c / TS, j2 = jb2 + c % TS;
          if (j1 <= a.G - 1 - a.oG && j2 <= a.G - 1 - a.oG)   // else past the grid's end
            store_cell<CPL, SLOW>(a.X, (int64_t)wrap(j1, a.G) * a.G + wrap(j2, a.G), a.C, c0 + cl, a.plane,
                            out);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < NC; ++u)
#pragma unroll
      for (int q = 0; q < 2 * CPL; ++q) tot[u][q] = 0.0;
    tl = next_tl;
  }
}

template <int CPL, typename V, int KW, int TS, bool SCALE, int MAXP, bool SLOW>
__global__ __launch_bounds__(kBlock) void k_adj_seg(AdjSegArgs s, const V* __restrict__ val) {
  extern __shared__ float2 smem[];
  const int b = blockIdx.x;
  const int sg = (b < s.n_first) ? s.seg0 + b
                                 : s.seg1 + (int)xcd_remap(b - s.n_first, gridDim.x - s.n_first);
  adj_seg_body<CPL, V, KW, TS, SCALE, MAXP, SLOW>(s, val, sg, blockIdx.y * kLanes * CPL, smem);
}

// Split dense tiles: block i sums partial tiles red_slot[i] .. red_slot[i+1]-1 in order into tile
// red_tile[i] of X; a thread owns one (cell, channel) pair at a time.
__global__ __launch_bounds__(kBlock) void k_adj_seg_reduce(const int32_t* __restrict__ red_tile,
                                                           const int32_t* __restrict__ red_slot,
                                                           const float2* __restrict__ part,
                                                           float2* __restrict__ X, int C, int G,
                                                           int oG, int NT, int TS, int64_t plane) {
  const int i = blockIdx.x;
  const int tl = red_tile[i], s0 = red_slot[i], s1 = red_slot[i + 1];
  const int jb1 = -oG + (tl / NT) * TS, jb2 = -oG + (tl % NT) * TS;
  const int n = TS * TS * C;
  for (int e = threadIdx.x; e < n; e += kBlock) {
    const int c = e / C, ch = e % C;
    const int j1 = jb1 + c / TS, j2 = jb2 + c % TS;
    if (j1 > G - 1 - oG || j2 > G - 1 - oG) continue;
    double ax = 0.0, ay = 0.0;                      // float64 sum of the partial tiles
    for (int sl = s0; sl < s1; ++sl) {
      const float2 p = part[(int64_t)sl * TS * TS * C + e];
      ax += p.x;
      ay += p.y;
    }
    const int64_t cell = (int64_t)wrap(j1, G) * G + wrap(j2, G);
    X[plane == 0 ? cell * C + ch : (int64_t)ch * plane + cell] = make_float2((float)ax, (float)ay);
  }
}

// ------------------------------------------------------------------------------------------
// persistent launches over a stack of operators (one SpMM-pair item per operator and batch)
// ------------------------------------------------------------------------------------------
// Work entry (item, index): forward index = work item * n_cc + channel chunk; adjoint index =
// segment * n_cc + channel chunk; reduction index = split tile.  Blocks walk the list with a
// grid stride; entries [0, n_first) go to blocks in dispatch order (long dense segments spread
// over the XCDs), the rest through the XCD-aware remap (neighbouring tiles on one XCD).
struct StackFwdItem {
  FwdTileArgs a;
  const void* val;
  int cpl, n_cc;
};

struct StackAdjItem {
  AdjSegArgs s;
  const void* val;
  const int32_t* red_tile;
  const int32_t* red_slot;
  int cpl, n_cc;
};

__device__ __forceinline__ int64_t stack_pos(int64_t phys, int64_t n_first, int64_t n_work) {
  return phys < n_first ? phys : n_first + xcd_remap(phys - n_first, n_work - n_first);
}

template <typename V, int KW, int PS, int MAXP>
__global__ __launch_bounds__(kBlock) void k_stack_fwd(const StackFwdItem* __restrict__ items,
                                                      const int2* __restrict__ work, int n_work) {
  extern __shared__ float2 smem[];
  for (int64_t phys = blockIdx.x; phys < n_work; phys += gridDim.x) {
    const int2 e = work[stack_pos(phys, 0, n_work)];
    const StackFwdItem& it = items[e.x];
    const int wi = e.y / it.n_cc, cc = e.y % it.n_cc;
    if (it.cpl == 2)
      fwd_tile_body<2, V, KW, PS, MAXP, false>(it.a, (const V*)it.val, wi, cc * kLanes * 2, smem);
    else
      fwd_tile_body<1, V, KW, PS, MAXP, false>(it.a, (const V*)it.val, wi, cc * kLanes, smem);
    __syncthreads();                                   // LDS is reused by the next entry
  }
}

template <typename V, int KW, int TS, int MAXP>
__global__ __launch_bounds__(kBlock) void k_stack_adj(const StackAdjItem* __restrict__ items,
                                                      const int2* __restrict__ work, int n_work,
                                                      int n_first) {
  extern __shared__ float2 smem[];
  for (int64_t phys = blockIdx.x; phys < n_work; phys += gridDim.x) {
    const int2 e = work[stack_pos(phys, n_first, n_work)];
    const StackAdjItem& it = items[e.x];
    const int sg = e.y / it.n_cc, cc = e.y % it.n_cc;
    if (it.cpl == 2)
      adj_seg_body<2, V, KW, TS, false, MAXP, false>(it.s, (const V*)it.val, sg, cc * kLanes * 2, smem);
    else
      adj_seg_body<1, V, KW, TS, false, MAXP, false>(it.s, (const V*)it.val, sg, cc * kLanes, smem);
    __syncthreads();
  }
}

// split dense tiles of every item: partial tiles summed in order into X
__global__ __launch_bounds__(kBlock) void k_stack_reduce(const StackAdjItem* __restrict__ items,
                                                         const int2* __restrict__ work, int n_work,
                                                         int TS) {
  for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const int2 e = work[w];
    const StackAdjItem& it = items[e.x];
    const AdjWinArgs& a = it.s.w;
    const int i = e.y;
    const int tl = it.red_tile[i], s0 = it.red_slot[i], s1 = it.red_slot[i + 1];
    const int jb1 = -a.oG + (tl / a.NT) * TS, jb2 = -a.oG + (tl % a.NT) * TS;
    const int n = TS * TS * a.C;
    for (int k = threadIdx.x; k < n; k += kBlock) {
      const int c = k / a.C, ch = k % a.C;
      const int j1 = jb1 + c / TS, j2 = jb2 + c % TS;
      if (j1 > a.G - 1 - a.oG || j2 > a.G - 1 - a.oG) continue;
      double ax = 0.0, ay = 0.0;                    // float64 sum of the partial tiles
      for (int sl = s0; sl < s1; ++sl) {
        const float2 p = it.s.part[(int64_t)sl * TS * TS * a.C + k];
        ax += p.x;
        ay += p.y;
      }
      a.X[((int64_t)wrap(j1, a.G) * a.G + wrap(j2, a.G)) * a.C + ch] = make_float2((float)ax, (float)ay);
    }
  }
}

template <int CPL, typename V>
tomo_status fwd_tile_impl(const tomo_op* op, int vt, const float2* X, float2* Y, int C, bool slow,
                          hipStream_t st) {
  const DevFwdTiles& d = op->ftile;
  constexpr int CH = kLanes * CPL;
  FwdTileArgs a{d.wi_tile, d.wi_beg, d.pt_row[slow], d.pt_base[slow], X, Y,
                C, op->g.G, op->g.G / 2, d.TS, d.NT, op->tune.tile_points,
                slow ? (int64_t)op->g.G * op->g.G : 0, slow ? (int64_t)op->g.nt * op->g.L : 0,
                op->g.nt, op->g.L};
  const size_t lds = fwd_tile_lds_bytes(op, C);
  dim3 grid((unsigned)d.n_wi, (unsigned)((C + CH - 1) / CH));
  const V* v = (const V*)d.val[slow][vt];
  const bool small = op->tune.tile_points <= 64;
#define TOMO_FWD_TILE_S(KW_, PS_, MAXP_)                                                          \
  if (slow)                                                                                     \
    hipLaunchKernelGGL((k_fwd_tile<CPL, V, KW_, PS_, MAXP_, true>), grid, dim3(kBlock), lds, st, a, v); \
  else                                                                                          \
    hipLaunchKernelGGL((k_fwd_tile<CPL, V, KW_, PS_, MAXP_, false>), grid, dim3(kBlock), lds, st, a, v);
#define TOMO_FWD_TILE(KW_, TS_)                                                                  \
  if (d.KW == KW_ && d.TS == TS_) {                                                             \
    constexpr int PS_ = TS_ + 2 * (KW_ / 2) + 1;                                                \
    if (small) {                                                                                \
      TOMO_FWD_TILE_S(KW_, PS_, 64)                                                             \
    } else {                                                                                    \
      TOMO_FWD_TILE_S(KW_, PS_, kMaxTilePoints)                                                 \
    }                                                                                           \
    TOMO_HIP(hipGetLastError());                                                                \
    return TOMO_OK;                                                                             \
  }
  TOMO_FWD_TILE(3, 8) TOMO_FWD_TILE(3, 16) TOMO_FWD_TILE(5, 8) TOMO_FWD_TILE(5, 16)
#undef TOMO_FWD_TILE
#undef TOMO_FWD_TILE_S
  return fail(TOMO_EUNSUPPORTED, "staged forward kernel has no variant for k_w %d, tile %d", d.KW,
              d.TS);
}

template <int CPL, typename V>
tomo_status adj_tile_impl(const tomo_op* op, int vt, const float2* Y, float2* X, int C,
                          const float* dscale, bool slow, hipStream_t st) {
  const DevAdjWin& d = op->awin;
  if (d.n_wi == 0) return TOMO_OK;
  constexpr int CH = kLanes * CPL;
  AdjWinArgs a{d.wi_tile, d.wi_q, d.wi_boff, d.q_row, Y, X, dscale,
               C, op->g.G, op->g.G / 2, d.NT, op->g.nt, d.QMAX, slow ? (int64_t)op->g.G * op->g.G : 0};
  const size_t lds = adj_tile_lds_bytes(op, C);
  dim3 grid((unsigned)d.n_wi, (unsigned)((C + CH - 1) / CH));
  const V* v = (const V*)d.q_val[vt];
  const bool small = d.QMAX <= 128;
#define TOMO_ADJ_WIN_P(KW_, TS_, P_)                                                             \
  if (dscale && slow)                                                                           \
    hipLaunchKernelGGL((k_adj_win<CPL, V, KW_, TS_, true, P_, true>), grid, dim3(kBlock), lds, st, a, v); \
  else if (dscale)                                                                              \
    hipLaunchKernelGGL((k_adj_win<CPL, V, KW_, TS_, true, P_, false>), grid, dim3(kBlock), lds, st, a, v); \
  else if (slow)                                                                                \
    hipLaunchKernelGGL((k_adj_win<CPL, V, KW_, TS_, false, P_, true>), grid, dim3(kBlock), lds, st, a, v); \
  else                                                                                          \
    hipLaunchKernelGGL((k_adj_win<CPL, V, KW_, TS_, false, P_, false>), grid, dim3(kBlock), lds, st, a, v);
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

template <int CPL, typename V>
tomo_status adj_seg_impl(const tomo_op* op, int vt, const float2* Y, float2* X, int C,
                         const float* dscale, bool dense, bool staged, bool slow, hipStream_t st) {
  const DevAdjWin& d = op->awin;
  const int n_dense = (int)(d.n_seg - d.n_sseg);
  const int n_first = dense ? n_dense : 0;
  const int nblk = n_first + (staged ? (int)d.n_sseg : 0);
  if (nblk == 0) return TOMO_OK;
  constexpr int CH = kLanes * CPL;
  const int64_t plane = slow ? (int64_t)op->g.G * op->g.G : 0;
  AdjSegArgs a{{d.wi_tile, d.wi_q, d.wi_boff, d.q_row, Y, X, dscale, C, op->g.G, op->g.G / 2, d.NT,
                op->g.nt, d.QMAX, plane},
               d.seg_tile, d.seg_chunk, d.seg_slot, d.chunk_tile, op->seg_partials,
               (int)d.n_sseg, n_first, 0, d.max_seg_chunks};
  const size_t lds = adj_seg_lds_bytes(op, C);
  dim3 grid((unsigned)nblk, (unsigned)((C + CH - 1) / CH));
  const V* v = (const V*)d.q_val[vt];
  const bool small = d.QMAX <= 128;
#define TOMO_ADJ_SEG_P(KW_, TS_, P_)                                                             \
  if (dscale && slow)                                                                           \
    hipLaunchKernelGGL((k_adj_seg<CPL, V, KW_, TS_, true, P_, true>), grid, dim3(kBlock), lds, st, a, v); \
  else if (dscale)                                                                              \
    hipLaunchKernelGGL((k_adj_seg<CPL, V, KW_, TS_, true, P_, false>), grid, dim3(kBlock), lds, st, a, v); \
  else if (slow)                                                                                \
    hipLaunchKernelGGL((k_adj_seg<CPL, V, KW_, TS_, false, P_, true>), grid, dim3(kBlock), lds, st, a, v); \
  else                                                                                          \
    hipLaunchKernelGGL((k_adj_seg<CPL, V, KW_, TS_, false, P_, false>), grid, dim3(kBlock), lds, st, a, v);
#define TOMO_ADJ_SEG(KW_, TS_)                                                                   \
  if (d.KW == KW_ && d.TS == TS_) {                                                             \
    if (small) {                                                                                \
      TOMO_ADJ_SEG_P(KW_, TS_, 128)                                                             \
    } else {                                                                                    \
      TOMO_ADJ_SEG_P(KW_, TS_, kMaxAdjPoints)                                                   \
    }                                                                                           \
    TOMO_HIP(hipGetLastError());                                                                \
    if (dense && d.n_red > 0) {                                                                 \
      hipLaunchKernelGGL(k_adj_seg_reduce, dim3((unsigned)d.n_red), dim3(kBlock), 0, st,         \
                         d.red_tile, d.red_slot, op->seg_partials, X, C, op->g.G, op->g.G / 2,  \
                         d.NT, d.TS, plane);                                                    \
      TOMO_HIP(hipGetLastError());                                                              \
    }                                                                                           \
    return TOMO_OK;                                                                             \
  }
  TOMO_ADJ_SEG(3, 8) TOMO_ADJ_SEG(3, 16) TOMO_ADJ_SEG(5, 8) TOMO_ADJ_SEG(5, 16)
#undef TOMO_ADJ_SEG
#undef TOMO_ADJ_SEG_P
  return fail(TOMO_EUNSUPPORTED, "staged adjoint segment kernel has no variant for k_w %d, tile %d",
              d.KW, d.TS);
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

size_t adj_seg_lds_bytes(const tomo_op* op, int C) { return adj_tile_lds_bytes(op, C); }

tomo_status launch_fwd_tile(const tomo_op* op, const float2* X, float2* Y, int C, int vt,
                            bool slow, hipStream_t st) {
  const bool even = (C % 2 == 0);
  switch (vt) {
    case TOMO_VAL_F32:
      return even ? fwd_tile_impl<2, float>(op, vt, X, Y, C, slow, st) : fwd_tile_impl<1, float>(op, vt, X, Y, C, slow, st);
    case TOMO_VAL_BF16:
      return even ? fwd_tile_impl<2, bf16_t>(op, vt, X, Y, C, slow, st) : fwd_tile_impl<1, bf16_t>(op, vt, X, Y, C, slow, st);
    default:
      return even ? fwd_tile_impl<2, _Float16>(op, vt, X, Y, C, slow, st) : fwd_tile_impl<1, _Float16>(op, vt, X, Y, C, slow, st);
  }
}

tomo_status launch_adj_seg(const tomo_op* op, const float2* Y, float2* X, int C, int vt,
                           const float* dscale, bool dense, bool staged, bool slow, hipStream_t st) {
  const bool even = (C % 2 == 0);
  switch (vt) {
    case TOMO_VAL_F32:
      return even ? adj_seg_impl<2, float>(op, vt, Y, X, C, dscale, dense, staged, slow, st)
                  : adj_seg_impl<1, float>(op, vt, Y, X, C, dscale, dense, staged, slow, st);
    case TOMO_VAL_BF16:
      return even ? adj_seg_impl<2, bf16_t>(op, vt, Y, X, C, dscale, dense, staged, slow, st)
                  : adj_seg_impl<1, bf16_t>(op, vt, Y, X, C, dscale, dense, staged, slow, st);
    default:
      return even ? adj_seg_impl<2, _Float16>(op, vt, Y, X, C, dscale, dense, staged, slow, st)
                  : adj_seg_impl<1, _Float16>(op, vt, Y, X, C, dscale, dense, staged, slow, st);
  }
}

tomo_status launch_adj_tile(const tomo_op* op, const float2* Y, float2* X, int C, int vt,
                            const float* dscale, bool slow, hipStream_t st) {
  const bool even = (C % 2 == 0);
  switch (vt) {
    case TOMO_VAL_F32:
      return even ? adj_tile_impl<2, float>(op, vt, Y, X, C, dscale, slow, st) : adj_tile_impl<1, float>(op, vt, Y, X, C, dscale, slow, st);
    case TOMO_VAL_BF16:
      return even ? adj_tile_impl<2, bf16_t>(op, vt, Y, X, C, dscale, slow, st) : adj_tile_impl<1, bf16_t>(op, vt, Y, X, C, dscale, slow, st);
    default:
      return even ? adj_tile_impl<2, _Float16>(op, vt, Y, X, C, dscale, slow, st) : adj_tile_impl<1, _Float16>(op, vt, Y, X, C, dscale, slow, st);
  }
}

// ------------------------------------------------------------------------------------------
// stack plans
// ------------------------------------------------------------------------------------------
struct StackPlan {
  int device = -1, vt = 0, KW = 0, TS = 0;
  bool fwd_big = false, adj_big = false;        // work-item capacities above 64 / 128 samples
  StackFwdItem* d_fwd = nullptr;
  StackAdjItem* d_adj = nullptr;
  int2 *d_wf = nullptr, *d_wa = nullptr, *d_wr = nullptr;
  int n_wf = 0, n_wa = 0, n_first = 0, n_wr = 0;
  size_t lds_f = 0, lds_a = 0;
  int grid_f = 0, grid_a = 0, grid_r = 0;
  std::vector<float2*> partials;                // per item: its split tiles' partial tiles
};

namespace {

template <typename V, int KW, int TS, int MPF, int MPA>
tomo_status stack_kernels(StackPlan* p, hipStream_t st, bool size_only, int n_cu) {
  constexpr int PS = TS + 2 * (KW / 2) + 1;
  auto kf = k_stack_fwd<V, KW, PS, MPF>;
  auto ka = k_stack_adj<V, KW, TS, MPA>;
  if (size_only) {
    // one grid of resident blocks per kernel (a multiple of the 8 XCDs), no larger than the work
    auto grid = [&](const void* k, size_t lds, int n_work, int* out) -> tomo_status {
      int per_cu = 0;
      TOMO_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlock, lds));
      int g = std::max(8, per_cu * n_cu / 8 * 8);
      *out = std::max(1, std::min(g, n_work));
      return TOMO_OK;
    };
    TOMO_TRY(grid((const void*)kf, p->lds_f, p->n_wf, &p->grid_f));
    TOMO_TRY(grid((const void*)ka, p->lds_a, p->n_wa, &p->grid_a));
    p->grid_r = std::max(1, std::min(p->n_wr, 8 * n_cu));
    return TOMO_OK;
  }
  if (p->n_wf > 0) {
    hipLaunchKernelGGL(kf, dim3((unsigned)p->grid_f), dim3(kBlock), p->lds_f, st, p->d_fwd, p->d_wf,
                       p->n_wf);
    TOMO_HIP(hipGetLastError());
  }
  if (p->n_wa > 0) {
    hipLaunchKernelGGL(ka, dim3((unsigned)p->grid_a), dim3(kBlock), p->lds_a, st, p->d_adj, p->d_wa,
                       p->n_wa, p->n_first);
    TOMO_HIP(hipGetLastError());
  }
  if (p->n_wr > 0) {
    hipLaunchKernelGGL(k_stack_reduce, dim3((unsigned)p->grid_r), dim3(kBlock), 0, st, p->d_adj,
                       p->d_wr, p->n_wr, TS);
    TOMO_HIP(hipGetLastError());
  }
  return TOMO_OK;
}

template <typename V>
tomo_status stack_dispatch_v(StackPlan* p, hipStream_t st, bool size_only, int n_cu) {
#define TOMO_STACK(KW_, TS_)                                                                     \
  if (p->KW == KW_ && p->TS == TS_) {                                                           \
    if (!p->fwd_big && !p->adj_big) return stack_kernels<V, KW_, TS_, 64, 128>(p, st, size_only, n_cu); \
    if (p->fwd_big && !p->adj_big)                                                              \
      return stack_kernels<V, KW_, TS_, kMaxTilePoints, 128>(p, st, size_only, n_cu);            \
    if (!p->fwd_big) return stack_kernels<V, KW_, TS_, 64, kMaxAdjPoints>(p, st, size_only, n_cu); \
    return stack_kernels<V, KW_, TS_, kMaxTilePoints, kMaxAdjPoints>(p, st, size_only, n_cu);    \
  }
  TOMO_STACK(3, 8) TOMO_STACK(3, 16) TOMO_STACK(5, 8) TOMO_STACK(5, 16)
#undef TOMO_STACK
  return fail(TOMO_EUNSUPPORTED, "no stack kernels for k_w %d, tile %d", p->KW, p->TS);
}

tomo_status stack_dispatch(StackPlan* p, hipStream_t st, bool size_only, int n_cu) {
  switch (p->vt) {
    case TOMO_VAL_F32: return stack_dispatch_v<float>(p, st, size_only, n_cu);
    case TOMO_VAL_BF16: return stack_dispatch_v<bf16_t>(p, st, size_only, n_cu);
    default: return stack_dispatch_v<_Float16>(p, st, size_only, n_cu);
  }
}

template <typename T>
tomo_status to_device(T** dst, const std::vector<T>& v) {
  *dst = nullptr;
  if (v.empty()) return TOMO_OK;
  if (hipMalloc((void**)dst, v.size() * sizeof(T)) != hipSuccess) {
    *dst = nullptr;
    return fail(TOMO_ENOMEM, "stack plan: %zu bytes", v.size() * sizeof(T));
  }
  TOMO_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return TOMO_OK;
}

}  // namespace

void stack_plan_destroy(StackPlan* p) {
  if (!p) return;
  (void)hipFree(p->d_fwd);
  (void)hipFree(p->d_adj);
  (void)hipFree(p->d_wf);
  (void)hipFree(p->d_wa);
  (void)hipFree(p->d_wr);
  for (float2* q : p->partials) (void)hipFree(q);
  delete p;
}

tomo_status stack_plan_create(const StackItemSpec* items, int n, int vt, StackPlan** out) {
  *out = nullptr;
  auto* p = new StackPlan();
  p->vt = vt;
  p->device = items[0].op->device;
  std::vector<StackFwdItem> fi;
  std::vector<StackAdjItem> ai;
  std::vector<int2> wf, dense, sparse, wr;
  std::vector<int> dense_len;
  tomo_status status = TOMO_OK;
  for (int i = 0; i < n && status == TOMO_OK; ++i) {
    const tomo_op* op = items[i].op;
    const DevFwdTiles& f = op->ftile;
    const DevAdjWin& d = op->awin;
    const int C = (items[i].batch + 1) / 2;
    const int cpl = (C % 2 == 0) ? 2 : 1, CH = kLanes * cpl, n_cc = (C + CH - 1) / CH;
    if (i == 0) {
      p->KW = f.KW;
      p->TS = f.TS;
    }
    if (f.KW != p->KW || f.TS != p->TS || d.TS != p->TS) {
      status = fail(TOMO_EINVAL, "stack items must share the kernel width and the tile side");
      break;
    }
    p->fwd_big = p->fwd_big || op->tune.tile_points > 64;
    p->adj_big = p->adj_big || d.QMAX > 128;
    p->lds_f = std::max(p->lds_f, fwd_tile_lds_bytes(op, C));
    p->lds_a = std::max(p->lds_a, adj_seg_lds_bytes(op, C));
    FwdTileArgs fa{f.wi_tile, f.wi_beg, f.pt_row[0], f.pt_base[0], (const float2*)items[i].in,
                   (float2*)items[i].out, C, op->g.G, op->g.G / 2, f.TS, f.NT, op->tune.tile_points, 0, 0,
                   op->g.nt, op->g.L};
    fi.push_back(StackFwdItem{fa, f.val[0][vt], cpl, n_cc});
    for (int64_t w = 0; w < f.n_wi; ++w)
      for (int cc = 0; cc < n_cc; ++cc) wf.push_back(make_int2(i, (int)(w * n_cc + cc)));
    float2* part = nullptr;
    if (d.n_slot > 0) {
      const size_t pb = (size_t)d.n_slot * d.TS * d.TS * C * sizeof(float2);
      if (hipMalloc((void**)&part, pb) != hipSuccess) {
        status = fail(TOMO_ENOMEM, "stack partial tiles (%zu B)", pb);
        break;
      }
    }
    p->partials.push_back(part);
    AdjSegArgs sa{{d.wi_tile, d.wi_q, d.wi_boff, d.q_row, (const float2*)items[i].out,
                   (float2*)items[i].aux, nullptr, C, op->g.G, op->g.G / 2, d.NT, op->g.nt, d.QMAX, 0},
                  d.seg_tile, d.seg_chunk, d.seg_slot, d.chunk_tile, part, 0, 0, 0, d.max_seg_chunks};
    ai.push_back(StackAdjItem{sa, d.q_val[vt], d.red_tile, d.red_slot, cpl, n_cc});
    // chunk counts of the dense segments, to start the longest first
    std::vector<int32_t> sc((size_t)d.n_seg + 1);
    if (d.n_seg > d.n_sseg)
      TOMO_HIP(hipMemcpy(sc.data(), d.seg_chunk, sc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int64_t sg = 0; sg < d.n_seg; ++sg)
      for (int cc = 0; cc < n_cc; ++cc) {
        const int2 e = make_int2(i, (int)(sg * n_cc + cc));
        if (sg >= d.n_sseg) {
          dense.push_back(e);
          dense_len.push_back(sc[(size_t)sg + 1] - sc[(size_t)sg]);
        } else {
          sparse.push_back(e);
        }
      }
    for (int64_t r = 0; r < d.n_red; ++r) wr.push_back(make_int2(i, (int)r));
  }
  if (status == TOMO_OK && (p->lds_f > kMaxTileLds || p->lds_a > kMaxTileLds))
    status = fail(TOMO_EUNSUPPORTED, "stack items need more LDS than a block has");
  if (status == TOMO_OK) {
    std::vector<size_t> ord(dense.size());
    for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return dense_len[x] > dense_len[y]; });
    std::vector<int2> wa;
    for (size_t k : ord) wa.push_back(dense[k]);
    wa.insert(wa.end(), sparse.begin(), sparse.end());
    p->n_wf = (int)wf.size();
    p->n_wa = (int)wa.size();
    p->n_first = (int)dense.size();
    p->n_wr = (int)wr.size();
    status = to_device(&p->d_fwd, fi);
    if (status == TOMO_OK) status = to_device(&p->d_adj, ai);
    if (status == TOMO_OK) status = to_device(&p->d_wf, wf);
    if (status == TOMO_OK) status = to_device(&p->d_wa, wa);
    if (status == TOMO_OK) status = to_device(&p->d_wr, wr);
    if (status == TOMO_OK) status = stack_dispatch(p, nullptr, true, items[0].op->n_cu);
  }
  if (status != TOMO_OK) {
    stack_plan_destroy(p);
    return status;
  }
  *out = p;
  return TOMO_OK;
}

tomo_status stack_plan_launch(const StackPlan* p, hipStream_t st) {
  return stack_dispatch(const_cast<StackPlan*>(p), st, false, 0);
}

}  // namespace tomo
