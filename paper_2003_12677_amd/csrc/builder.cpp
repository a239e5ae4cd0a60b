// Host-side setup stage (Sec. 3.1): geometry -> gridding matrix S^dagger (polar rows) and its
// stored transpose S (Cartesian rows) in float64, adjoint row bins, deapodisation and the
// filter diagonal.  Plain C++17, no HIP calls.
//
// Matrix layout chosen for the device path (differs from the paper's ordering, same matrix):
//   * polar row r = kf * nt + a, where kf = k mod L is the FFT-ordered radial index of the
//     sample at radius k (in Fourier grid units) on angle theta_a; radial-major rows make the
//     1D transform along k a plain strided batch and keep an angle's neighbours adjacent;
//   * Cartesian column / row m = (j1 mod G) * G + (j2 mod G), the FFT-ordered frequency,
//     so the 2D transform needs no shift.
//
// Entries (Sec. 3, Fig. 3): polar point q = k (G/L) (cos theta_a, sin theta_a); window
// j = rint(q) + s, s in [-h, h]^2, h = (k_w - 1)/2; value K(j1 - q1) K(j2 - q2) with the
// Kaiser-Bessel kernel K zero at |t| >= k_w / 2.  Zero entries, entries with |j1| or |j2|
// above ceil(G/2) - 1, and the unpaired radial sample k = -L/2 (even L) are removed, which
// keeps the composed operator exactly real-to-real so that two real slices can share one
// complex channel (Sec. 3.1).

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <thread>

#include "internal.h"

namespace tomo {

namespace {
thread_local std::string g_last_error;

// I0(x) - 1 from the power series sum_{k>=1} (x^2/4)^k / (k!)^2 (Abramowitz & Stegun 9.6.10);
// every term is positive, so the sum has no cancellation.
double bessel_i0_minus_1(double x) {
  const double y = 0.25 * x * x;
  double term = 1.0, sum = 0.0;
  for (int k = 1; k < 1000; ++k) {
    term *= y / ((double)k * (double)k);
    sum += term;
    if (term <= sum * 1e-18) break;
  }
  return sum;
}

inline int64_t mod_pos(int64_t a, int64_t m) {
  int64_t r = a % m;
  return r < 0 ? r + m : r;
}
}  // namespace

tomo_status fail(tomo_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

void clear_error() { g_last_error.clear(); }

const char* last_error_cstr() { return g_last_error.c_str(); }

tomo_status resolve_geometry(const tomo_geometry* in, Geom* g) {
  if (!in) return fail(TOMO_EINVAL, "geometry is NULL");
  Geom r;
  r.n = in->n;
  r.nt = in->n_angles;
  r.np = in->n_det;
  if (r.n < 1 || r.nt < 1 || r.np < 1)
    return fail(TOMO_EINVAL, "n, n_angles and n_det must be positive (got %d, %d, %d)", r.n, r.nt,
                r.np);
  r.G = in->grid ? in->grid : r.np;
  r.L = r.G;
  if (r.G < r.n || r.G < r.np)
    return fail(TOMO_EINVAL, "grid %d must be >= max(n=%d, n_det=%d)", r.G, r.n, r.np);
  if (r.G < 3) return fail(TOMO_EINVAL, "grid must be at least 3");
  r.kw = in->kw ? in->kw : 3;
  if (r.kw < 1 || r.kw > 15 || r.kw % 2 == 0)
    return fail(TOMO_EINVAL, "kernel width kw=%d must be odd and in [1, 15]", r.kw);
  r.h = (r.kw - 1) / 2;
  r.max_batch = in->max_batch;
  if (r.max_batch < 1 || r.max_batch > tomo::kMaxBatch)
    return fail(TOMO_EINVAL, "max_batch=%d must be in [1, %d]", r.max_batch, tomo::kMaxBatch);
  if (in->reserved != 0) return fail(TOMO_EINVAL, "reserved field must be 0");
  r.values = in->values ? in->values : TOMO_VALUES_F32;
  if (r.values & ~(uint32_t)(TOMO_VALUES_F32 | TOMO_VALUES_BF16 | TOMO_VALUES_F16))
    return fail(TOMO_EINVAL, "unknown bits in values mask 0x%x", r.values);
  r.values |= TOMO_VALUES_F32;   // the float32 copy is always kept (refinement residuals)
  const double sigma = (double)r.G / (double)r.n;
  if (std::isnan(in->beta)) {
    // Beatty, Nishimura, Pauly (IEEE TMI 2005), Eq. 5
    const double w = (double)r.kw;
    const double arg = (w / sigma) * (w / sigma) * (sigma - 0.5) * (sigma - 0.5) - 0.8;
    if (arg <= 0) return fail(TOMO_EINVAL, "default beta undefined for kw=%d, G/n=%g", r.kw, sigma);
    r.beta = M_PI * std::sqrt(arg);
  } else {
    r.beta = in->beta;
  }
  if (!(r.beta > 0) || !std::isfinite(r.beta)) return fail(TOMO_EINVAL, "beta must be positive");
  r.center = std::isnan(in->center) ? (double)(r.np / 2) : in->center;
  if (!std::isfinite(r.center)) return fail(TOMO_EINVAL, "center must be finite");
  // c = c0 + f: the integer part shifts the detector bins, the fractional part is a phase ramp
  // on the polar rows (Sec. 3)
  const double c0 = std::floor(r.center);
  if (std::fabs(c0) > 1e9) return fail(TOMO_EINVAL, "center %g out of range", r.center);
  r.cdet = (int)mod_pos((int64_t)c0, r.L);
  r.cfrac = r.center - c0;
  r.jmax = (r.G + 1) / 2 - 1;
  r.on = r.n / 2;
  r.theta.resize(r.nt);
  for (int a = 0; a < r.nt; ++a) {
    r.theta[a] = in->angles ? in->angles[a] : (double)a * M_PI / (double)r.nt;
    if (!std::isfinite(r.theta[a])) return fail(TOMO_EINVAL, "angle %d is not finite", a);
  }
  // index ranges must fit the int32 device arrays
  const double nnz_bound = (double)r.nt * r.L * r.kw * r.kw;
  if (nnz_bound >= 2147483647.0 || (double)r.G * r.G >= 2147483647.0)
    return fail(TOMO_EINVAL, "operator too large for 32-bit indices");
  *g = std::move(r);
  return TOMO_OK;
}

double kernel_value(double t, int W, double beta) {
  const double half = 0.5 * W;
  if (!(std::fabs(t) < half)) return 0.0;
  const double u = 2.0 * t / W;
  const double arg = beta * std::sqrt(std::max(0.0, 1.0 - u * u));
  return bessel_i0_minus_1(arg) / bessel_i0_minus_1(beta);
}

void build_sdag(const Geom& g, HostCSR* out, std::vector<int32_t>* centres) {
  const int64_t N = (int64_t)g.nt * g.L;
  const int64_t M = (int64_t)g.G * g.G;
  const int W = g.kw, h = g.h;
  const double scale = (double)g.G / (double)g.L;
  std::vector<double> ct(g.nt), st(g.nt);
  for (int a = 0; a < g.nt; ++a) {
    ct[a] = std::cos(g.theta[a]);
    st[a] = std::sin(g.theta[a]);
  }
  out->rows = N;
  out->cols = M;
  out->rowptr.assign(N + 1, 0);
  out->col.clear();
  out->val.clear();
  out->col.reserve((size_t)N * W * W);
  out->val.reserve((size_t)N * W * W);
  if (centres) centres->assign((size_t)N * 2, INT32_MIN);
  std::vector<std::pair<int32_t, double>> ent;
  std::vector<double> w1(W), w2(W);
  std::vector<int64_t> j1s(W), j2s(W);
  for (int kf = 0; kf < g.L; ++kf) {
    const bool nyquist = (2 * kf == g.L);
    const int64_t k = (2 * kf < g.L) ? kf : (int64_t)kf - g.L;
    for (int a = 0; a < g.nt; ++a) {
      const int64_t r = (int64_t)kf * g.nt + a;
      if (!nyquist) {
        const double q1 = ((double)k * scale) * ct[a];
        const double q2 = ((double)k * scale) * st[a];
        const double c1 = std::nearbyint(q1);   // round half to even
        const double c2 = std::nearbyint(q2);
        if (centres) {
          (*centres)[(size_t)r * 2] = (int32_t)c1;
          (*centres)[(size_t)r * 2 + 1] = (int32_t)c2;
        }
        for (int s = -h; s <= h; ++s) {
          j1s[s + h] = (int64_t)c1 + s;
          j2s[s + h] = (int64_t)c2 + s;
          w1[s + h] = kernel_value((double)j1s[s + h] - q1, W, g.beta);
          w2[s + h] = kernel_value((double)j2s[s + h] - q2, W, g.beta);
        }
        ent.clear();
        for (int s1 = 0; s1 < W; ++s1) {
          if (std::llabs(j1s[s1]) > g.jmax || w1[s1] == 0.0) continue;
          for (int s2 = 0; s2 < W; ++s2) {
            if (std::llabs(j2s[s2]) > g.jmax) continue;
            const double w = w1[s1] * w2[s2];
            if (w == 0.0) continue;
            const int64_t m = mod_pos(j1s[s1], g.G) * g.G + mod_pos(j2s[s2], g.G);
            ent.emplace_back((int32_t)m, w);
          }
        }
        std::sort(ent.begin(), ent.end(),
                  [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                    return x.first < y.first;
                  });
        for (auto& e : ent) {
          out->col.push_back(e.first);
          out->val.push_back(e.second);
        }
      }
      out->rowptr[r + 1] = (int64_t)out->col.size();
    }
  }
}

void transpose_csr(const HostCSR& a, HostCSR* at) {
  at->rows = a.cols;
  at->cols = a.rows;
  at->rowptr.assign(a.cols + 1, 0);
  const int64_t nnz = a.nnz();
  for (int64_t e = 0; e < nnz; ++e) at->rowptr[a.col[e] + 1]++;
  for (int64_t i = 0; i < a.cols; ++i) at->rowptr[i + 1] += at->rowptr[i];
  at->col.assign(nnz, 0);
  at->val.assign(nnz, 0.0);
  std::vector<int64_t> next(at->rowptr.begin(), at->rowptr.end() - 1);
  for (int64_t r = 0; r < a.rows; ++r) {
    for (int64_t e = a.rowptr[r]; e < a.rowptr[r + 1]; ++e) {
      const int64_t dst = next[a.col[e]]++;
      at->col[dst] = (int32_t)r;   // rows visited in order: columns come out sorted
      at->val[dst] = a.val[e];
    }
  }
}

void build_ell(const HostCSR& a, int W2, HostEll* out) {
  out->W2 = W2;
  out->col.assign((size_t)a.rows * W2, -1);
  out->val.assign((size_t)a.rows * W2, 0.0);
  for (int64_t r = 0; r < a.rows; ++r) {
    int s = 0;
    for (int64_t e = a.rowptr[r]; e < a.rowptr[r + 1]; ++e, ++s) {
      out->col[(size_t)r * W2 + s] = a.col[e];
      out->val[(size_t)r * W2 + s] = a.val[e];
    }
  }
}

tomo_status check_tuning(const Tuning& t) {
  auto cpl_ok = [](int c) { return c == 1 || c == 2 || c == 4; };
  if (t.fwd_tiled < 0 || t.fwd_tiled > 7 || t.adj_tiled < 0 || t.adj_tiled > 7)
    return fail(TOMO_EINVAL, "fwd_tiled / adj_tiled are value-type bit masks in [0, 7]");
  if (t.tile != 8 && t.tile != 16) return fail(TOMO_EINVAL, "tile must be 8 or 16");
  if (t.tile_points < 32 || t.tile_points > 128 || t.tile_points % 32 != 0)
    return fail(TOMO_EINVAL, "tile_points must be 32, 64, 96 or 128");
  if (t.adj_tile_points < 32 || t.adj_tile_points > 256 || t.adj_tile_points % 32 != 0)
    return fail(TOMO_EINVAL, "adj_tile_points must be a multiple of 32 in [32, 256]");
  if (t.normal_tiled != 0 && t.normal_tiled != 1) return fail(TOMO_EINVAL, "normal_tiled must be 0 or 1");
  if (t.sell_xcd_rows < 0 || t.sell_xcd_rows > (1 << 24) || t.medium_xcd_rows < 0 ||
      t.medium_xcd_rows > (1 << 24))
    return fail(TOMO_EINVAL, "XCD interleave rows must be in [0, 2^24]");
  if (t.det_fft < 0 || t.det_fft > 2) return fail(TOMO_EINVAL, "det_fft must be 0, 1 or 2");
  if (t.grid_fft != 0 && t.grid_fft != 1) return fail(TOMO_EINVAL, "grid_fft must be 0 or 1");
  if (t.sell_tiles != 0 && t.sell_tiles != 1) return fail(TOMO_EINVAL, "adj_sell_tiles must be 0 or 1");
  if (t.tile_strip < 0 || t.tile_strip > 4096) return fail(TOMO_EINVAL, "tile_strip must be in [0, 4096]");
  if (t.adj_dense_mode < 0 || t.adj_dense_mode > 2) return fail(TOMO_EINVAL, "adj_dense_mode must be 0, 1 or 2");
  if (t.adj_seg_chunks < 1 || t.adj_seg_chunks > kMaxSegChunks)
    return fail(TOMO_EINVAL, "adj_seg_chunks must be in [1, %d]", kMaxSegChunks);
  if (t.adj_run < 1 || t.adj_run > kMaxSegChunks)
    return fail(TOMO_EINVAL, "adj_run must be in [1, %d]", kMaxSegChunks);
  if (t.fwd_rows_per_group != 1 && t.fwd_rows_per_group != 2 && t.fwd_rows_per_group != 4)
    return fail(TOMO_EINVAL, "fwd_rows_per_group must be 1, 2 or 4");
  if (!cpl_ok(t.fwd_cpl) || !cpl_ok(t.adj_cpl))
    return fail(TOMO_EINVAL, "channels per lane must be 1, 2 or 4 (got %d, %d)", t.fwd_cpl, t.adj_cpl);
  if (t.sell_max < 0 || t.sell_max > 1024) return fail(TOMO_EINVAL, "sell_max %d not in [0, 1024]", t.sell_max);
  if (t.medium_max < t.sell_max || t.medium_max > (1 << 20))
    return fail(TOMO_EINVAL, "medium_max %d must be in [sell_max, 2^20]", t.medium_max);
  if (t.chunk < 8 || t.chunk > 8192) return fail(TOMO_EINVAL, "chunk %d not in [8, 8192]", t.chunk);
  if (t.sell_sigma < 1) return fail(TOMO_EINVAL, "sell_sigma must be >= 1");
  return TOMO_OK;
}

void build_adj_layout(const HostCSR& s, const Tuning& t, HostAdj* o, const std::vector<char>* rows) {
  *o = HostAdj();
  std::vector<int32_t> sell, medium, lng;
  auto len = [&](int64_t r) { return s.rowptr[r + 1] - s.rowptr[r]; };
  for (int64_t r = 0; r < s.rows; ++r) {
    if (rows && !(*rows)[(size_t)r]) continue;
    const int64_t l = len(r);
    if (l <= t.sell_max) sell.push_back((int32_t)r);
    else if (l <= t.medium_max) medium.push_back((int32_t)r);
    else lng.push_back((int32_t)r);
  }
  const int64_t G = (int64_t)std::llround(std::sqrt((double)s.rows));
  if (t.sell_tiles && G * G == s.rows) {
    // Cartesian cells in 4 x 8 tiles of the centred grid (a block of 32 rows is one tile), tiles
    // and the cells inside them in row-major order
    const int64_t oG = G / 2, nt2 = (G + 7) / 8;
    auto key = [&](int32_t r) {
      const int64_t f1 = r / G, f2 = r % G;
      const int64_t u1 = (f1 <= G - 1 - oG ? f1 : f1 - G) + oG;
      const int64_t u2 = (f2 <= G - 1 - oG ? f2 : f2 - G) + oG;
      return ((u1 / 4) * nt2 + u2 / 8) * 32 + (u1 % 4) * 8 + u2 % 8;
    };
    std::stable_sort(sell.begin(), sell.end(), [&](int32_t x, int32_t y) { return key(x) < key(y); });
  } else {
    // sort by decreasing length inside windows of sigma rows (keeps neighbouring rows together)
    for (size_t w = 0; w < sell.size(); w += (size_t)t.sell_sigma) {
      auto b = sell.begin() + w;
      auto e = sell.begin() + std::min(sell.size(), w + (size_t)t.sell_sigma);
      std::stable_sort(b, e, [&](int32_t x, int32_t y) { return len(x) > len(y); });
    }
  }
  o->sell_rows = (int64_t)sell.size();
  const int64_t ns = (o->sell_rows + kSliceRows - 1) / kSliceRows;
  o->slice_rows.assign((size_t)ns * kSliceRows, -1);
  std::copy(sell.begin(), sell.end(), o->slice_rows.begin());
  o->slice_ptr.assign((size_t)ns + 1, 0);
  for (int64_t i = 0; i < ns; ++i) {
    int64_t lmax = 0;
    for (int j = 0; j < kSliceRows; ++j) {
      const int32_t r = o->slice_rows[i * kSliceRows + j];
      if (r >= 0) lmax = std::max(lmax, len(r));
    }
    o->slice_ptr[i + 1] = o->slice_ptr[i] + (int32_t)(lmax * kSliceRows);
  }
  o->col.assign((size_t)o->slice_ptr[ns], -1);
  o->val.assign((size_t)o->slice_ptr[ns], 0.0);
  int64_t used = 0;
  for (int64_t i = 0; i < ns; ++i) {
    for (int j = 0; j < kSliceRows; ++j) {
      const int32_t r = o->slice_rows[i * kSliceRows + j];
      if (r < 0) continue;
      for (int64_t e = 0; e < len(r); ++e) {
        const size_t dst = (size_t)o->slice_ptr[i] + (size_t)e * kSliceRows + j;
        o->col[dst] = s.col[s.rowptr[r] + e];
        o->val[dst] = s.val[s.rowptr[r] + e];
        ++used;
      }
    }
  }
  o->sell_padding = (int64_t)o->col.size() - used;
  // tail CSR: medium rows, then long rows
  o->n_medium = (int64_t)medium.size();
  o->n_long = (int64_t)lng.size();
  o->tail_rows = medium;
  o->tail_rows.insert(o->tail_rows.end(), lng.begin(), lng.end());
  o->tail_ptr.assign(o->tail_rows.size() + 1, 0);
  for (size_t i = 0; i < o->tail_rows.size(); ++i) {
    const int32_t r = o->tail_rows[i];
    o->tail_ptr[i + 1] = o->tail_ptr[i] + (int32_t)len(r);
    for (int64_t e = s.rowptr[r]; e < s.rowptr[r + 1]; ++e) {
      o->tail_col.push_back(s.col[e]);
      o->tail_val.push_back(s.val[e]);
    }
  }
  o->long_chunk_ptr.assign(1, 0);
  for (int64_t i = o->n_medium; i < (int64_t)o->tail_rows.size(); ++i) {
    for (int32_t e = o->tail_ptr[i]; e < o->tail_ptr[i + 1]; e += t.chunk) {
      o->chunk_beg.push_back(e);
      o->chunk_end.push_back(std::min(e + t.chunk, o->tail_ptr[i + 1]));
    }
    o->long_chunk_ptr.push_back((int32_t)o->chunk_beg.size());
  }
}

namespace {
// centred frequency of an FFT-ordered index
inline int centred(int64_t f, int G, int oG) { return (f <= G - 1 - oG) ? (int)f : (int)(f - G); }
// tile index along one axis of the centred coordinate j
inline int tile_of(int j, int oG, int TS) { return (j + oG) / TS; }
// Tile visiting order of the staged kernels: strips `strip` tiles wide, each walked tile row by
// tile row (0, or a strip as wide as the grid: row-major).  Blocks go to the XCDs in contiguous
// runs of this order, so the tiles above and below a tile, whose halos overlap its own, run on
// the same XCD about a strip width earlier or later and find the shared data in its L2.
std::vector<int> tile_order(int NT, int strip) {
  std::vector<int> o;
  o.reserve((size_t)NT * NT);
  if (strip <= 0 || strip >= NT) {
    for (int i = 0; i < NT * NT; ++i) o.push_back(i);
    return o;
  }
  for (int s0 = 0; s0 < NT; s0 += strip)
    for (int t1 = 0; t1 < NT; ++t1)
      for (int t2 = s0; t2 < std::min(NT, s0 + strip); ++t2) o.push_back(t1 * NT + t2);
  return o;
}
}  // namespace

tomo_status build_fwd_tiles(const Geom& g, const HostCSR& sdag, const std::vector<int32_t>& centres,
                            const Tuning& t, HostFwdTiles* o, bool slowest_order) {
  *o = HostFwdTiles();
  const int G = g.G, oG = G / 2, TS = t.tile, h = g.h, kw = g.kw;
  o->TS = TS;
  o->PS = TS + 2 * h + 1;
  o->NT = (G + TS - 1) / TS;
  o->KW = kw;
  o->W2 = kw * kw;
  const int64_t N = sdag.rows;
  const int ntiles = o->NT * o->NT;
  const int origin_tile = tile_of(0, oG, TS) * o->NT + tile_of(0, oG, TS);
  // points are grouped by their tile's place in the visiting order
  const std::vector<int> worder = tile_order(o->NT, t.tile_strip);
  std::vector<int> rank(ntiles);
  for (int i = 0; i < ntiles; ++i) rank[worder[i]] = i;
  std::vector<int32_t> rank_of_row(N);
  std::vector<int64_t> count(ntiles + 1, 0);
  for (int64_t r = 0; r < N; ++r) {
    int tl = origin_tile;   // rows without a window (unpaired Nyquist sample) still write zeros
    const int32_t c1 = centres[(size_t)r * 2], c2 = centres[(size_t)r * 2 + 1];
    if (c1 != INT32_MIN) {
      const int t1 = std::min(std::max(tile_of(c1, oG, TS), 0), o->NT - 1);
      const int t2 = std::min(std::max(tile_of(c2, oG, TS), 0), o->NT - 1);
      tl = t1 * o->NT + t2;
    }
    rank_of_row[r] = rank[tl];
    count[rank[tl] + 1]++;
  }
  for (int i = 0; i < ntiles; ++i) count[i + 1] += count[i];
  std::vector<int32_t> order(N);
  {
    std::vector<int64_t> next(count.begin(), count.end() - 1);
    if (slowest_order) {
      // within a tile, samples by angle, then radius, so that a work item's outputs form runs of
      // consecutive radii in the channel-slowest polar layout
      for (int a = 0; a < g.nt; ++a)
        for (int64_t kf = 0; kf < g.L; ++kf) {
          const int64_t r = kf * g.nt + a;
          order[next[rank_of_row[r]]++] = (int32_t)r;
        }
    } else {
      // row order: neighbouring samples write neighbouring rows of the channel-fastest layout
      for (int64_t r = 0; r < N; ++r) order[next[rank_of_row[r]]++] = (int32_t)r;
    }
  }
  o->pt_row = order;
  o->pt_base.assign((size_t)N, 0);
  o->pt_val.assign((size_t)N * o->W2, 0.0);
  o->wi_beg.push_back(0);
  for (int rk = 0; rk < ntiles; ++rk) {
    const int tl = worder[rk];
    const int j01 = -oG + (tl / o->NT) * TS - h, j02 = -oG + (tl % o->NT) * TS - h;   // patch origin
    for (int64_t i = count[rk]; i < count[rk + 1]; ++i) {
      const int64_t r = order[i];
      const int32_t c1 = centres[(size_t)r * 2], c2 = centres[(size_t)r * 2 + 1];
      if (c1 == INT32_MIN) {
        if (sdag.rowptr[r + 1] != sdag.rowptr[r])
          return fail(TOMO_EINVAL, "internal: row %lld has entries but no window", (long long)r);
        continue;   // base 0, all values zero
      }
      const int b1 = c1 - h - j01, b2 = c2 - h - j02;
      if (b1 < 0 || b2 < 0 || b1 + kw > o->PS || b2 + kw > o->PS)
        return fail(TOMO_EINVAL, "internal: window outside its tile patch (row %lld)", (long long)r);
      o->pt_base[(size_t)i] = b1 * o->PS + b2;
      for (int64_t e = sdag.rowptr[r]; e < sdag.rowptr[r + 1]; ++e) {
        const int s1 = centred(sdag.col[e] / G, G, oG) - c1 + h;
        const int s2 = centred(sdag.col[e] % G, G, oG) - c2 + h;
        if (s1 < 0 || s1 >= kw || s2 < 0 || s2 >= kw)
          return fail(TOMO_EINVAL, "internal: tap outside its window (row %lld)", (long long)r);
        o->pt_val[(size_t)i * o->W2 + s1 * kw + s2] = sdag.val[e];
      }
    }
    for (int64_t b = count[rk]; b < count[rk + 1]; b += t.tile_points) {
      o->wi_tile.push_back(tl);
      o->wi_beg.push_back((int32_t)std::min<int64_t>(b + t.tile_points, count[rk + 1]));
    }
  }
  return TOMO_OK;
}

tomo_status build_adj_win(const Geom& g, const HostCSR& sdag, const std::vector<int32_t>& centres,
                          const Tuning& t, HostAdjWin* o) {
  *o = HostAdjWin();
  const int G = g.G, oG = G / 2, TS = t.tile, h = g.h, kw = g.kw;
  o->TS = TS;
  o->RS = TS + 2 * h;
  o->NT = (G + TS - 1) / TS;
  o->KW = kw;
  o->W2 = kw * kw;
  o->QMAX = t.adj_tile_points;
  const int RS = o->RS, NT = o->NT, W2 = o->W2;
  const int64_t N = sdag.rows;
  // window-ordered values of every polar row, and the rows bucketed by centre cell on the grid
  // extended by h (+1 above: a centre may round onto the grid's upper edge)
  const int E = G + 2 * h + 1;
  std::vector<double> wv((size_t)N * W2, 0.0);
  std::vector<int64_t> cell_ptr((size_t)E * E + 1, 0);
  auto ext = [&](int32_t c) { return (int64_t)c + oG + h; };
  for (int64_t r = 0; r < N; ++r) {
    const int32_t c1 = centres[(size_t)r * 2], c2 = centres[(size_t)r * 2 + 1];
    if (c1 == INT32_MIN) continue;
    if (ext(c1) < 0 || ext(c1) >= E || ext(c2) < 0 || ext(c2) >= E)
      return fail(TOMO_EINVAL, "internal: window centre off the extended grid (row %lld)", (long long)r);
    for (int64_t e = sdag.rowptr[r]; e < sdag.rowptr[r + 1]; ++e) {
      const int s1 = centred(sdag.col[e] / G, G, oG) - c1 + h;
      const int s2 = centred(sdag.col[e] % G, G, oG) - c2 + h;
      if (s1 < 0 || s1 >= kw || s2 < 0 || s2 >= kw)
        return fail(TOMO_EINVAL, "internal: tap outside its window (row %lld)", (long long)r);
      wv[(size_t)r * W2 + s1 * kw + s2] = sdag.val[e];
    }
    cell_ptr[(size_t)(ext(c1) * E + ext(c2)) + 1]++;
  }
  for (size_t i = 1; i < cell_ptr.size(); ++i) cell_ptr[i] += cell_ptr[i - 1];
  std::vector<int32_t> cell_rows((size_t)cell_ptr.back());
  {
    std::vector<int64_t> next(cell_ptr.begin(), cell_ptr.end() - 1);
    for (int64_t r = 0; r < N; ++r) {
      const int32_t c1 = centres[(size_t)r * 2], c2 = centres[(size_t)r * 2 + 1];
      if (c1 != INT32_MIN) cell_rows[(size_t)next[(size_t)(ext(c1) * E + ext(c2))]++] = (int32_t)r;
    }
  }
  o->dense_cell.assign((size_t)G * G, 0);
  o->wi_q.push_back(0);
  std::vector<int> dense_tiles;
  // a tile's samples in bucket order (region cells row-major), with offsets bo[RS*RS + 1]
  auto tile_samples = [&](int t1, int t2, std::vector<int32_t>* rows, std::vector<int64_t>* bo) {
    rows->clear();
    bo->clear();
    for (int a = 0; a < RS; ++a)
      for (int b = 0; b < RS; ++b) {
        bo->push_back((int64_t)rows->size());
        const int64_t e1 = (int64_t)t1 * TS + a, e2 = (int64_t)t2 * TS + b;
        if (e1 >= E || e2 >= E) continue;
        for (int64_t i = cell_ptr[(size_t)(e1 * E + e2)]; i < cell_ptr[(size_t)(e1 * E + e2) + 1]; ++i)
          rows->push_back(cell_rows[(size_t)i]);
      }
    bo->push_back((int64_t)rows->size());
  };
  // one chunk: samples [s0, s1) of a tile's list, bucket offsets clipped to the chunk
  auto push_chunk = [&](const std::vector<int32_t>& rows, const std::vector<int64_t>& bo, int64_t s0,
                        int64_t s1) {
    for (const int64_t b : bo) o->wi_boff.push_back((uint16_t)(std::min(std::max(b, s0), s1) - s0));
    for (int64_t i = s0; i < s1; ++i) {
      const int32_t r = rows[(size_t)i];
      o->q_row.push_back(r);
      o->q_val.insert(o->q_val.end(), wv.begin() + (size_t)r * W2, wv.begin() + (size_t)(r + 1) * W2);
    }
    o->wi_q.push_back((int32_t)o->q_row.size());
  };
  std::vector<int32_t> rows;
  std::vector<int64_t> bo;
  for (const int tl : tile_order(NT, t.tile_strip)) {
    const int t1 = tl / NT, t2 = tl % NT;
    tile_samples(t1, t2, &rows, &bo);
    const int64_t nq = (int64_t)rows.size();
    if (nq > o->QMAX) {
      // a dense tile: chunked segments (the FFT-side form, and adj_dense_mode 1 / 2), and its
      // cells marked for the row kernels (adj_dense_mode 0)
      dense_tiles.push_back(tl);
      for (int a = 0; a < TS; ++a)
        for (int b = 0; b < TS; ++b) {
          const int j1 = -oG + t1 * TS + a, j2 = -oG + t2 * TS + b;
          if (j1 <= G - 1 - oG && j2 <= G - 1 - oG)
            o->dense_cell[(size_t)((j1 % G + G) % G) * G + ((j2 % G + G) % G)] = 1;
        }
      continue;
    }
    o->wi_tile.push_back(tl);
    push_chunk(rows, bo, 0, nq);
  }
  o->n_wi = (int64_t)o->wi_tile.size();
  o->chunk_tile = o->wi_tile;
  // staged tiles: segments of adj_run consecutive tiles in the visiting order
  const int run = t.adj_dense_mode == 2 ? t.adj_run : 1;
  for (int64_t w = 0; w < o->n_wi; w += run) {
    o->seg_tile.push_back(o->wi_tile[(size_t)w]);
    o->seg_chunk.push_back((int32_t)w);
    o->seg_slot.push_back(-1);
  }
  o->n_sseg = (int64_t)o->seg_tile.size();
  // dense tiles: chunks of nearly equal size (<= QMAX samples), segments of nearly equal chunk
  // counts (<= adj_seg_chunks); a tile with several segments is summed from partial tiles
  int32_t chunk = (int32_t)o->n_wi, slot = 0;
  o->red_slot.push_back(0);
  for (const int tl : dense_tiles) {
    tile_samples(tl / NT, tl % NT, &rows, &bo);
    const int64_t nq = (int64_t)rows.size();
    const int64_t nch = (nq + o->QMAX - 1) / o->QMAX;
    const int64_t nseg = (nch + t.adj_seg_chunks - 1) / t.adj_seg_chunks;
    for (int64_t c = 0; c < nch; ++c) {
      push_chunk(rows, bo, nq * c / nch, nq * (c + 1) / nch);
      o->chunk_tile.push_back(tl);
    }
    for (int64_t sg = 0; sg < nseg; ++sg) {
      o->seg_tile.push_back(tl);
      o->seg_chunk.push_back(chunk + (int32_t)(nch * sg / nseg));
      o->seg_slot.push_back(nseg > 1 ? slot++ : -1);
    }
    chunk += (int32_t)nch;
    if (nseg > 1) {
      o->red_tile.push_back(tl);
      o->red_slot.push_back(slot);
    }
  }
  o->seg_chunk.push_back(chunk);
  if (o->q_row.size() >= (size_t)INT32_MAX) return fail(TOMO_EINVAL, "staged adjoint layout too large");
  return TOMO_OK;
}

// Host replay of every kernel layout in float64, following the kernels' traversal, against the
// CSR products; returns the largest relative difference (a self-check of the layout builders).
tomo_status check_layouts(const Geom& g, const HostCSR& sdag, const HostCSR& s,
                          const std::vector<int32_t>& centres, const Tuning& t, double* max_rel) {
  const int64_t N = sdag.rows, M = s.rows;
  const int G = g.G, oG = G / 2;
  std::vector<double> x(M), y(N);
  uint64_t st = 88172645463325252ull;   // xorshift64
  auto rnd = [&]() { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (double)(st >> 11) / 9007199254740992.0 - 0.5; };
  for (auto& v : x) v = rnd();
  for (auto& v : y) v = rnd();
  std::vector<double> yf(N, 0.0), xa(M, 0.0);
  for (int64_t r = 0; r < N; ++r)
    for (int64_t e = sdag.rowptr[r]; e < sdag.rowptr[r + 1]; ++e) yf[r] += sdag.val[e] * x[sdag.col[e]];
  for (int64_t r = 0; r < M; ++r)
    for (int64_t e = s.rowptr[r]; e < s.rowptr[r + 1]; ++e) xa[r] += s.val[e] * y[s.col[e]];
  auto rel = [](const std::vector<double>& a, const std::vector<double>& b) {
    double num = 0, den = 0;
    for (size_t i = 0; i < a.size(); ++i) { num += (a[i] - b[i]) * (a[i] - b[i]); den += b[i] * b[i]; }
    return std::sqrt(num / (den > 0 ? den : 1.0));
  };
  double worst = 0;
  {  // fixed-stride forward
    HostEll ell;
    build_ell(sdag, g.kw * g.kw, &ell);
    std::vector<double> out(N, 0.0);
    for (int64_t r = 0; r < N; ++r)
      for (int k = 0; k < ell.W2; ++k) {
        const int32_t c = ell.col[(size_t)r * ell.W2 + k];
        if (c >= 0) out[r] += ell.val[(size_t)r * ell.W2 + k] * x[c];
      }
    worst = std::max(worst, rel(out, yf));
  }
  // row-binned adjoint kernels over layout h: writes the rows h holds
  auto replay_rows = [&](const HostAdj& h, std::vector<double>& out) {
    const int64_t ns = (int64_t)h.slice_ptr.size() - 1;
    for (int64_t i = 0; i < ns; ++i) {
      const int len = (h.slice_ptr[i + 1] - h.slice_ptr[i]) / kSliceRows;
      for (int j = 0; j < kSliceRows; ++j) {
        const int32_t row = h.slice_rows[i * kSliceRows + j];
        double acc = 0;
        for (int e = 0; e < len; ++e) {
          const size_t k = (size_t)h.slice_ptr[i] + (size_t)e * kSliceRows + j;
          if (h.col[k] >= 0) acc += h.val[k] * y[h.col[k]];
        }
        if (row >= 0) out[row] = acc;
      }
    }
    for (size_t i = 0; i < h.tail_rows.size(); ++i) {
      double acc = 0;
      for (int32_t e = h.tail_ptr[i]; e < h.tail_ptr[i + 1]; ++e) acc += h.tail_val[e] * y[h.tail_col[e]];
      out[h.tail_rows[i]] = acc;
    }
  };
  {  // row-binned adjoint
    HostAdj h;
    build_adj_layout(s, t, &h);
    std::vector<double> out(M, std::nan(""));
    replay_rows(h, out);
    worst = std::max(worst, rel(out, xa));
  }
  for (const bool slowest : {false, true}) {  // staged forward, both sample orders
    HostFwdTiles f;
    TOMO_TRY(build_fwd_tiles(g, sdag, centres, t, &f, slowest));
    std::vector<double> out(N, std::nan(""));
    for (size_t w = 0; w < f.wi_tile.size(); ++w) {
      const int tl = f.wi_tile[w];
      const int j01 = -oG + (tl / f.NT) * f.TS - g.h, j02 = -oG + (tl % f.NT) * f.TS - g.h;
      for (int32_t i = f.wi_beg[w]; i < f.wi_beg[w + 1]; ++i) {
        double acc = 0;
        for (int s1 = 0; s1 < f.KW; ++s1)
          for (int s2 = 0; s2 < f.KW; ++s2) {
            const int sl = f.pt_base[i] + s1 * f.PS + s2;
            if (sl < 0 || sl >= f.PS * f.PS) return fail(TOMO_EINVAL, "internal: tap slot outside the patch");
            const int g1 = ((j01 + sl / f.PS) % G + G) % G, g2 = ((j02 + sl % f.PS) % G + G) % G;
            acc += f.pt_val[(size_t)i * f.W2 + s1 * f.KW + s2] * x[(int64_t)g1 * G + g2];
          }
        out[f.pt_row[i]] = acc;
      }
    }
    worst = std::max(worst, rel(out, yf));
  }
  {  // staged adjoint (window form) and the row kernels on its dense cells
    HostAdjWin a;
    TOMO_TRY(build_adj_win(g, sdag, centres, t, &a));
    const int RS = a.RS, h = g.h, kw = a.KW, NBO = RS * RS + 1, T2 = a.TS * a.TS;
    std::vector<double> out(M, std::nan(""));
    // the cell sums of one chunk added to acc[TS*TS], in the kernels' order
    auto chunk_sums = [&](size_t w, std::vector<double>& acc) -> tomo_status {
      const int32_t q0 = a.wi_q[w];
      const uint16_t* bo = a.wi_boff.data() + w * (size_t)NBO;
      if (a.wi_q[w + 1] - q0 > a.QMAX || bo[NBO - 1] != a.wi_q[w + 1] - q0)
        return fail(TOMO_EINVAL, "internal: staged tile sample count");
      for (int m1 = 0; m1 < a.TS; ++m1)
        for (int m2 = 0; m2 < a.TS; ++m2)
          for (int p1 = 0; p1 < kw; ++p1) {
            const int rb = (m1 + 2 * h - p1) * RS + m2;   // one run per window row
            for (int k = bo[rb]; k < bo[rb + kw]; ++k) {
              int t = 0;
              while (t + 1 < kw && k >= bo[rb + t + 1]) ++t;
              const int p2 = 2 * h - t;
              acc[(size_t)(m1 * a.TS + m2)] +=
                  a.q_val[(size_t)(q0 + k) * a.W2 + p1 * kw + p2] * y[a.q_row[(size_t)(q0 + k)]];
            }
          }
      return TOMO_OK;
    };
    auto store_tile = [&](int tl, const std::vector<double>& acc) {
      const int t1 = tl / a.NT, t2 = tl % a.NT;
      for (int m1 = 0; m1 < a.TS; ++m1)
        for (int m2 = 0; m2 < a.TS; ++m2) {
          const int j1 = -oG + t1 * a.TS + m1, j2 = -oG + t2 * a.TS + m2;
          if (j1 > G - 1 - oG || j2 > G - 1 - oG) continue;
          out[(int64_t)((j1 % G + G) % G) * G + ((j2 % G + G) % G)] = acc[(size_t)(m1 * a.TS + m2)];
        }
    };
    // every segment (runs of staged tiles and dense-tile segments): chunks in order, a tile's
    // sums stored when the next chunk belongs to another tile; then the split tiles' reductions
    const size_t nseg = a.seg_tile.size();
    if (a.seg_chunk.size() != nseg + 1 || a.wi_q.size() != (size_t)a.seg_chunk.back() + 1 ||
        a.chunk_tile.size() + 1 != a.wi_q.size())
      return fail(TOMO_EINVAL, "internal: segment list");
    std::vector<std::vector<double>> slots;
    for (size_t sg = 0; sg < nseg; ++sg) {
      std::vector<double> acc((size_t)T2, 0.0);
      const int32_t c0 = a.seg_chunk[sg], c1 = a.seg_chunk[sg + 1];
      if (c1 - c0 > kMaxSegChunks) return fail(TOMO_EINVAL, "internal: segment too long");
      for (int32_t c = c0; c < c1; ++c) {
        TOMO_TRY(chunk_sums((size_t)c, acc));
        if (c + 1 < c1 && a.chunk_tile[(size_t)c + 1] == a.chunk_tile[(size_t)c]) continue;
        if (a.seg_slot[sg] < 0) {
          store_tile(a.chunk_tile[(size_t)c], acc);
        } else {
          if ((size_t)a.seg_slot[sg] != slots.size() || c0 + 1 > c1 ||
              a.chunk_tile[(size_t)c0] != a.chunk_tile[(size_t)c])
            return fail(TOMO_EINVAL, "internal: partial slot order");
          slots.push_back(acc);
        }
        std::fill(acc.begin(), acc.end(), 0.0);
      }
    }
    for (size_t i = 0; i < a.red_tile.size(); ++i) {
      std::vector<double> acc((size_t)T2, 0.0);
      for (int32_t sl = a.red_slot[i]; sl < a.red_slot[i + 1]; ++sl)
        for (int c = 0; c < T2; ++c) acc[(size_t)c] += slots[(size_t)sl][(size_t)c];
      store_tile(a.red_tile[i], acc);
    }
    worst = std::max(worst, rel(out, xa));   // every cell from the segments
    HostAdj hd;
    build_adj_layout(s, t, &hd, &a.dense_cell);
    replay_rows(hd, out);                     // the dense cells from the row kernels instead
    worst = std::max(worst, rel(out, xa));
  }
  *max_rel = worst;   // NaN if some output row was never written
  return TOMO_OK;
}

void deapod_factors(const Geom& g, std::vector<double>* kd) {
  // kappa(x) = sum_{s=-h..h} K(s) cos(2 pi s x / G), the discrete transform of the kernel taps;
  // k*(i1, i2) = 1 / (kappa(i1 - n/2) kappa(i2 - n/2)) on the image support (Sec. 3).
  std::vector<double> taps(g.h + 1);
  for (int s = 0; s <= g.h; ++s) taps[s] = kernel_value((double)s, g.kw, g.beta);
  kd->resize(g.n);
  for (int i = 0; i < g.n; ++i) {
    const double x = (double)(i - g.on);
    double kap = taps[0];
    for (int s = 1; s <= g.h; ++s) kap += 2.0 * taps[s] * std::cos(2.0 * M_PI * s * x / g.G);
    (*kd)[i] = 1.0 / kap;
  }
}

void filter_diagonal(const Geom& g, int filter, std::vector<double>* d) {
  const int L = g.L;
  d->assign(L, 1.0);
  if (filter == TOMO_FILTER_NONE) return;
  // band-limited ramp h(m) on the circle m in [-L/2, L-1-L/2] (Kak & Slaney 1988)
  std::vector<double> hm(L, 0.0);
  const int m0 = -(L / 2);
  for (int i = 0; i < L; ++i) {
    const int m = m0 + i;
    if (m == 0)
      hm[i] = 0.25;
    else if (m % 2 != 0)
      hm[i] = -1.0 / ((M_PI * m) * (M_PI * m));
  }
  for (int kf = 0; kf < L; ++kf) {
    const int k = (2 * kf < L) ? kf : kf - L;
    double R = 0.0;
    for (int i = 0; i < L; ++i)
      if (hm[i] != 0.0) R += hm[i] * std::cos(2.0 * M_PI * (double)k * (double)(m0 + i) / L);
    double win = 1.0;
    if (filter == TOMO_FILTER_SHEPP) {
      const double x = M_PI * (double)k / L;
      win = (k == 0) ? 1.0 : std::sin(x) / x;
    } else if (filter == TOMO_FILTER_HAMMING) {
      win = 0.54 + 0.46 * std::cos(2.0 * M_PI * (double)k / L);
    }
    (*d)[kf] = R * win;
  }
}

// Row j of W = S diag(d) S^dagger as a (2R+1)^2 stencil, R = kw - 1 (Sec. 4, Toeplitz form of
// A^T A): over the polar samples p of row j of S, add S[j][p] d(p) S^dagger[p][j'] at the slot
// of the offset j' - j, both FFT-ordered Cartesian indices with the offset taken mod G into
// [-G/2, G/2).  Fixed summation order.  False if an entry falls outside the stencil.
bool normal_stencil_row(const Geom& g, const HostCSR& s, const HostCSR& sdag, const double* dk,
                        int64_t j, double* out) {
  const int R = g.kw - 1, D = 2 * R + 1;
  const int64_t G = g.G;
  std::fill(out, out + (size_t)D * D, 0.0);
  const int64_t j1 = j / G, j2 = j % G;
  for (int64_t e = s.rowptr[j]; e < s.rowptr[j + 1]; ++e) {
    const int64_t p = s.col[e];
    const double a = s.val[e] * (dk ? dk[p / g.nt] : 1.0);
    for (int64_t f = sdag.rowptr[p]; f < sdag.rowptr[p + 1]; ++f) {
      const int64_t c = sdag.col[f];
      int64_t d1 = c / G - j1, d2 = c % G - j2;
      if (2 * d1 >= G) d1 -= G;
      if (2 * d1 < -G) d1 += G;
      if (2 * d2 >= G) d2 -= G;
      if (2 * d2 < -G) d2 += G;
      if (d1 < -R || d1 > R || d2 < -R || d2 > R) return false;
      out[(d1 + R) * D + (d2 + R)] += a * sdag.val[f];
    }
  }
  return true;
}

tomo_status build_normal_values(const Geom& g, const HostCSR& s, const HostCSR& sdag,
                                const double* dk, int stride, std::vector<double>* w) {
  const int D = 2 * g.kw - 1;
  const int64_t M = (int64_t)g.G * g.G;
  w->assign((size_t)M * stride, 0.0);
  std::atomic<bool> ok{true};
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t) {
    pool.emplace_back([&, t] {
      std::vector<double> row((size_t)D * D);
      for (int64_t j = M * t / nth; j < M * (t + 1) / nth; ++j) {
        if (!normal_stencil_row(g, s, sdag, dk, j, row.data())) {
          ok = false;
          return;
        }
        std::copy(row.begin(), row.end(), w->begin() + (size_t)j * stride);
      }
    });
  }
  for (auto& th : pool) th.join();
  if (!ok) return fail(TOMO_EINVAL, "S S^dagger entry outside the (2kw-1)^2 stencil");
  return TOMO_OK;
}

uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

}  // namespace tomo
