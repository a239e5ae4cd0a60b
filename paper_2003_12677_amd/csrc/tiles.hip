// LDS-staged SpMM kernels for the slicing interpolation (Sec. 2.2, Sec. 3 Eq. (2)).
//
// Every Cartesian Fourier point is referenced by about nine polar samples (nnz / columns
// touched = 8.4 at 2048^2, 1501 angles), and the row-per-lane-group kernels fetch it from L2
// each time; measured, they are bound by that L2 gather traffic even when the whole grid is
// cache resident.  These kernels stage what a block reads in LDS once:
//
// forward  Y = S^dagger X: samples are grouped by the Cartesian tile (TS x TS) holding their
//          window centre; a block copies the tile plus a halo of h = (k_w-1)/2 from X into
//          LDS (the "patch", PS x PS points x up to 16 complex channels) and evaluates every
//          sample's taps from LDS.
// adjoint  X = S diag(D) Y: a block owns one Cartesian tile of output rows; the polar rows its
//          entries reference are staged in LDS in chunks (scaled by D on the way in), together
//          with the chunk's entries (LDS slot, value) and per-row offsets, so the accumulation
//          loop touches only LDS.  Rows near the Fourier origin sum thousands of same-sign
//          terms and their error reaches every pixel through the DC coefficient, so row sums are
//          accumulated in float64 and rounded once.  A block accumulates up to tile_chunks
//          chunks in registers;
//          tiles with more chunks (near the origin) are split over several blocks whose partial
//          sums are added in a fixed order by a small reduction kernel (no atomics).
//
// A lane group of 8 lanes owns one row; lane t holds CPL complex channels, so a block covers
// 8*CPL channels (grid.y walks the channel chunks).

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tomo {
namespace {

constexpr int kBlock = 256;
constexpr int kLanes = 8;
constexpr int kGroups = kBlock / kLanes;   // 32 lane groups per block

struct bf16_t { uint16_t bits; };
__device__ __forceinline__ float ldv(const float* v, int64_t e) { return v[e]; }
__device__ __forceinline__ float ldv(const bf16_t* v, int64_t e) {
  return __uint_as_float((uint32_t)v[e].bits << 16);
}
__device__ __forceinline__ float ldv(const _Float16* v, int64_t e) { return (float)v[e]; }

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
  const uint16_t* pt_slot;   // [P][WS]
  const float2* X;
  float2* Y;
  int C, G, oG, TS, PS, NT, h, WS, n_wi;
};

// Staging is written as batches of independent loads into registers followed by LDS stores, so
// a block pays one memory round trip per batch instead of one per element.
constexpr int kStageBatch = 8;

template <int CPL, typename V, int WS, int SPG>
__global__ __launch_bounds__(kBlock) void k_fwd_tile(FwdTileArgs a, const V* __restrict__ val) {
  extern __shared__ float2 patch[];          // [PS*PS][CH]
  constexpr int CH = kLanes * CPL;
  const int wi = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int c0 = blockIdx.y * CH;
  const int nch = min(CH, a.C - c0);
  const int tl = a.wi_tile[wi];
  const int b0 = a.wi_beg[wi], b1 = a.wi_beg[wi + 1];
  const int g = threadIdx.x / kLanes;
  const int cl = (threadIdx.x % kLanes) * CPL;
  // this group's samples: indices, taps and weights, loaded before the patch is complete
  int row[SPG];
  uint16_t sl[SPG][WS];
  float w[SPG][WS];
#pragma unroll
  for (int q = 0; q < SPG; ++q) {
    const int i = b0 + g + q * kGroups;
    row[q] = -1;
    if (i < b1) {
      row[q] = a.pt_row[i];
#pragma unroll
      for (int s = 0; s < WS; ++s) {
        sl[q][s] = a.pt_slot[(int64_t)i * WS + s];
        w[q][s] = ldv(val, (int64_t)i * WS + s);
      }
    }
  }
  // stage the tile plus halo
  const int j01 = -a.oG + (tl / a.NT) * a.TS - a.h;
  const int j02 = -a.oG + (tl % a.NT) * a.TS - a.h;
  const int PP = a.PS * a.PS;
  for (int base = threadIdx.x; base < PP * kLanes; base += kBlock * kStageBatch) {
    Vec<CPL> v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      const int idx = base + u * kBlock;
      const int p = idx / kLanes, l = (idx % kLanes) * CPL;
      if (idx < PP * kLanes && l < nch) {
        const int g1 = wrap(j01 + p / a.PS, a.G), g2 = wrap(j02 + p % a.PS, a.G);
        v[u] = vload<CPL>(a.X + ((int64_t)g1 * a.G + g2) * a.C + c0 + l);
      }
    }
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      const int idx = base + u * kBlock;
      const int p = idx / kLanes, l = (idx % kLanes) * CPL;
      if (idx < PP * kLanes && l < nch) vstore<CPL>(patch + p * CH + l, v[u]);
    }
  }
  __syncthreads();
  if (cl >= nch) return;
#pragma unroll
  for (int q = 0; q < SPG; ++q) {
    if (row[q] < 0) continue;
    Vec<CPL> acc;
    vzero(acc);
#pragma unroll
    for (int s = 0; s < WS; ++s) {
      if (sl[q][s] != 0xFFFF) {
        const Vec<CPL> x = vload<CPL>(patch + sl[q][s] * CH + cl);
#pragma unroll
        for (int k = 0; k < 2 * CPL; ++k) acc.v[k] += w[q][s] * x.v[k];
      }
    }
    vstore<CPL>(a.Y + (int64_t)row[q] * a.C + c0 + cl, acc);
  }
}

// ------------------------------------------------------------------------------------------
// adjoint
// ------------------------------------------------------------------------------------------
struct AdjTileArgs {
  const int32_t* wi_tile;
  const int32_t* wi_cb;       // first chunk
  const int32_t* wi_ce;       // one past the last chunk
  const int32_t* wi_out;      // -1: write X, else partial slot
  const int32_t* ch_pt_beg;
  const int32_t* ch_pts;
  const int32_t* ch_row_off;  // [chunk][R + 1]
  const uint16_t* en_slot;
  const float2* Y;
  float2* X;
  float2* partials;           // [slot][R][C]
  const float* dscale;        // per FFT-ordered radial index, or null
  double inv_nt;
  int C, G, oG, TS, NT, qmax, emax;
};

constexpr int kRowsPerGroup(int R) { return R / kGroups; }

template <int CPL, typename V, int RPG>
__global__ __launch_bounds__(kBlock) void k_adj_tile(AdjTileArgs a, const V* __restrict__ val) {
  constexpr int CH = kLanes * CPL;
  extern __shared__ float2 smem[];
  float2* pts = smem;                                               // [qmax][CH]
  float* sval = reinterpret_cast<float*>(pts + a.qmax * CH);         // [emax]
  int* soff = reinterpret_cast<int*>(sval + a.emax);                 // [R + 1]
  uint16_t* sslot = reinterpret_cast<uint16_t*>(soff + kGroups * RPG + 1);   // [emax]
  const int R = kGroups * RPG;
  const int wi = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int c0 = blockIdx.y * CH;
  const int nch = min(CH, a.C - c0);
  const int g = threadIdx.x / kLanes;
  const int cl = (threadIdx.x % kLanes) * CPL;
  const bool active = cl < nch;
  double acc[RPG][2 * CPL];
#pragma unroll
  for (int r = 0; r < RPG; ++r)
#pragma unroll
    for (int c = 0; c < 2 * CPL; ++c) acc[r][c] = 0.0;
  for (int ch = a.wi_cb[wi]; ch < a.wi_ce[wi]; ++ch) {
    // stage the chunk: polar rows (times D), entries, row offsets; every phase issues a batch
    // of independent loads before storing to LDS
    const int q0 = a.ch_pt_beg[ch], nq = a.ch_pt_beg[ch + 1] - q0;
    const int* off = a.ch_row_off + (int64_t)ch * (R + 1);
    const int e0 = off[0], ne = off[R] - e0;
    for (int base = threadIdx.x; base < nq * kLanes; base += kBlock * kStageBatch) {
      int pcol[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int idx = base + u * kBlock;
        pcol[u] = (idx < nq * kLanes) ? a.ch_pts[q0 + idx / kLanes] : -1;
      }
      Vec<CPL> v[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int l = ((base + u * kBlock) % kLanes) * CPL;
        if (pcol[u] >= 0 && l < nch) v[u] = vload<CPL>(a.Y + (int64_t)pcol[u] * a.C + c0 + l);
      }
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int idx = base + u * kBlock;
        const int l = (idx % kLanes) * CPL;
        if (pcol[u] < 0 || l >= nch) continue;
        if (a.dscale) {
          const float d = a.dscale[(int)(((double)pcol[u] + 0.5) * a.inv_nt)];
#pragma unroll
          for (int k = 0; k < 2 * CPL; ++k) v[u].v[k] *= d;
        }
        vstore<CPL>(pts + (idx / kLanes) * CH + l, v[u]);
      }
    }
    for (int i = threadIdx.x; i <= R; i += kBlock) soff[i] = off[i] - e0;
    for (int base = threadIdx.x; base < ne; base += kBlock * kStageBatch) {
      uint16_t ts[kStageBatch];
      float tv[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int i = base + u * kBlock;
        if (i < ne) {
          ts[u] = a.en_slot[e0 + i];
          tv[u] = ldv(val, (int64_t)e0 + i);
        }
      }
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int i = base + u * kBlock;
        if (i < ne) {
          sslot[i] = ts[u];
          sval[i] = tv[u];
        }
      }
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int r = 0; r < RPG; ++r) {
        const int rr = g + r * kGroups;
        const int b = soff[rr], e = soff[rr + 1];
        for (int k = b; k < e; ++k) {
          const Vec<CPL> y = vload<CPL>(pts + sslot[k] * CH + cl);
          const float w = sval[k];
#pragma unroll
          for (int c = 0; c < 2 * CPL; ++c) acc[r][c] += (double)(w * y.v[c]);
        }
      }
    }
    __syncthreads();
  }
  if (!active) return;
  const int tl = a.wi_tile[wi];
  const int t1 = tl / a.NT, t2 = tl % a.NT;
  const int out = a.wi_out[wi];
#pragma unroll
  for (int r = 0; r < RPG; ++r) {
    const int rr = g + r * kGroups;
    Vec<CPL> o;
#pragma unroll
    for (int c = 0; c < 2 * CPL; ++c) o.v[c] = (float)acc[r][c];
    if (out >= 0) {
      vstore<CPL>(a.partials + ((int64_t)out * R + rr) * a.C + c0 + cl, o);
    } else {
      const int j1 = -a.oG + t1 * a.TS + rr / a.TS, j2 = -a.oG + t2 * a.TS + rr % a.TS;
      if (j1 > a.G - 1 - a.oG || j2 > a.G - 1 - a.oG) continue;   // outside the grid
      const int64_t m = (int64_t)wrap(j1, a.G) * a.G + wrap(j2, a.G);
      vstore<CPL>(a.X + m * a.C + c0 + cl, o);
    }
  }
}

// tiles split over several blocks: X rows = sum of the blocks' partial sums, in block order
template <int CPL>
__global__ __launch_bounds__(kBlock) void k_adj_tile_reduce(const int32_t* __restrict__ red_tile,
                                                            const int32_t* __restrict__ red_beg,
                                                            const int32_t* __restrict__ red_cnt,
                                                            const float2* __restrict__ partials,
                                                            float2* __restrict__ X, int C, int G,
                                                            int oG, int TS, int NT) {
  constexpr int CH = kLanes * CPL;
  const int R = TS * TS;
  const int i = blockIdx.x;
  const int c0 = blockIdx.y * CH;
  const int nch = min(CH, C - c0);
  const int tl = red_tile[i], t1 = tl / NT, t2 = tl % NT;
  const int cl = (threadIdx.x % kLanes) * CPL;
  if (cl >= nch) return;
  for (int rr = threadIdx.x / kLanes; rr < R; rr += kGroups) {
    const int j1 = -oG + t1 * TS + rr / TS, j2 = -oG + t2 * TS + rr % TS;
    if (j1 > G - 1 - oG || j2 > G - 1 - oG) continue;
    double acc[2 * CPL];
#pragma unroll
    for (int k = 0; k < 2 * CPL; ++k) acc[k] = 0.0;
    for (int s = 0; s < red_cnt[i]; ++s) {
      const Vec<CPL> p = vload<CPL>(partials + ((int64_t)(red_beg[i] + s) * R + rr) * C + c0 + cl);
#pragma unroll
      for (int k = 0; k < 2 * CPL; ++k) acc[k] += (double)p.v[k];
    }
    Vec<CPL> o;
#pragma unroll
    for (int k = 0; k < 2 * CPL; ++k) o.v[k] = (float)acc[k];
    vstore<CPL>(X + ((int64_t)wrap(j1, G) * G + wrap(j2, G)) * C + c0 + cl, o);
  }
}

template <int CPL, typename V>
tomo_status fwd_tile_impl(const tomo_op* op, int vt, const float2* X, float2* Y, int C,
                          hipStream_t st) {
  const DevFwdTiles& d = op->ftile;
  constexpr int CH = kLanes * CPL;
  FwdTileArgs a{d.wi_tile, d.wi_beg, d.pt_row, d.pt_slot, X, Y,
                C, op->g.G, op->g.G / 2, d.TS, d.PS, d.NT, op->g.h, d.WS, (int)d.n_wi};
  const size_t lds = (size_t)d.PS * d.PS * CH * sizeof(float2);
  dim3 grid((unsigned)d.n_wi, (unsigned)((C + CH - 1) / CH));
  const V* v = (const V*)d.val[vt];
  const int spg = (op->tune.tile_points + kGroups - 1) / kGroups;   // samples per lane group
#define TOMO_FWD_TILE(WS_, SPG_)                                                                  \
  if (d.WS == WS_ && spg <= SPG_) {                                                             \
    hipLaunchKernelGGL((k_fwd_tile<CPL, V, WS_, SPG_>), grid, dim3(kBlock), lds, st, a, v);     \
    TOMO_HIP(hipGetLastError());                                                                \
    return TOMO_OK;                                                                             \
  }
  TOMO_FWD_TILE(12, 1) TOMO_FWD_TILE(12, 2) TOMO_FWD_TILE(12, 4)
  TOMO_FWD_TILE(28, 1) TOMO_FWD_TILE(28, 2)
#undef TOMO_FWD_TILE
  return fail(TOMO_EUNSUPPORTED, "staged forward kernel has no variant for %d taps, %d samples",
              d.WS, op->tune.tile_points);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

template <int CPL, typename V>
tomo_status adj_tile_impl(const tomo_op* op, int vt, const float2* Y, float2* X, int C,
                          const float* dscale, hipStream_t st) {
  const DevAdjTiles& d = op->atile;
  constexpr int CH = kLanes * CPL;
  AdjTileArgs a{d.wi_tile, d.wi_cb, d.wi_ce, d.wi_out, d.ch_pt_beg, d.ch_pts, d.ch_row_off,
                d.en_slot, Y, X, op->tile_partials, dscale, 1.0 / (double)op->g.nt,
                C, op->g.G, op->g.G / 2, d.TS, d.NT, d.qmax, d.emax};
  const int R = d.TS * d.TS;
  const size_t lds = (size_t)d.qmax * CH * sizeof(float2) + (size_t)d.emax * sizeof(float) +
                     (size_t)(R + 1) * sizeof(int) + (size_t)d.emax * sizeof(uint16_t);
  dim3 grid((unsigned)d.n_wi, (unsigned)((C + CH - 1) / CH));
  const V* v = (const V*)d.en_val[vt];
  switch (R / kGroups) {
    case 2: hipLaunchKernelGGL((k_adj_tile<CPL, V, 2>), grid, dim3(kBlock), lds, st, a, v); break;
    case 8: hipLaunchKernelGGL((k_adj_tile<CPL, V, 8>), grid, dim3(kBlock), lds, st, a, v); break;
    case 32: hipLaunchKernelGGL((k_adj_tile<CPL, V, 32>), grid, dim3(kBlock), lds, st, a, v); break;
    default: return fail(TOMO_EUNSUPPORTED, "staged adjoint kernel has no variant for tile %d", d.TS);
  }
  TOMO_HIP(hipGetLastError());
  if (d.n_red > 0) {
    hipLaunchKernelGGL((k_adj_tile_reduce<CPL>), dim3((unsigned)d.n_red, grid.y), dim3(kBlock), 0,
                       st, d.red_tile, d.red_beg, d.red_cnt, op->tile_partials, X, C, op->g.G,
                       op->g.G / 2, d.TS, d.NT);
    TOMO_HIP(hipGetLastError());
  }
  return TOMO_OK;
}

}  // namespace

bool fwd_tile_supported(const tomo_op* op) {
  const int spg = (op->tune.tile_points + kGroups - 1) / kGroups;
  return (op->ftile.WS == 12 && spg <= 4) || (op->ftile.WS == 28 && spg <= 2);
}

size_t fwd_tile_lds_bytes(const tomo_op* op, int C) {
  const int cpl = (C % 2 == 0) ? 2 : 1;
  return (size_t)op->ftile.PS * op->ftile.PS * kLanes * cpl * sizeof(float2);
}

size_t adj_tile_lds_bytes(const tomo_op* op, int C) {
  const int cpl = (C % 2 == 0) ? 2 : 1;
  const DevAdjTiles& d = op->atile;
  const int R = d.TS * d.TS;
  return (size_t)d.qmax * kLanes * cpl * sizeof(float2) + (size_t)d.emax * sizeof(float) +
         (size_t)(R + 1) * sizeof(int) + (size_t)d.emax * sizeof(uint16_t);
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
