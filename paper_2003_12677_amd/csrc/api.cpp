// C ABI entry points: operator lifecycle, argument checks, and the composed operators of
// Eq. (2) (Sec. 3): project = F1D^-1 S^dagger F2D k*, backproject = k* F2D^H S F1D^-H.

#include <cmath>
#include <cstring>
#include <memory>

#include <complex>

#include "internal.h"

namespace tomo {
const char* last_error_cstr();

namespace {

template <typename T>
tomo_status upload(T** dst, const T* src, size_t count) {
  *dst = nullptr;
  if (count == 0) return TOMO_OK;
  if (hipMalloc((void**)dst, count * sizeof(T)) != hipSuccess) {
    *dst = nullptr;
    return fail(TOMO_ENOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
  }
  TOMO_HIP(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return TOMO_OK;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

// Upload float64 values as every requested storage type (float32, bfloat16, float16).
tomo_status upload_values(const std::vector<double>& v, uint32_t values, void* dst[3]) {
  const size_t nnz = v.size();
  std::vector<float> vf(nnz);
  for (size_t i = 0; i < nnz; ++i) vf[i] = (float)v[i];
  if (values & TOMO_VALUES_F32) TOMO_TRY(upload((float**)&dst[TOMO_VAL_F32], vf.data(), nnz));
  if (values & TOMO_VALUES_BF16) {
    std::vector<uint16_t> vb(nnz);
    for (size_t i = 0; i < nnz; ++i) vb[i] = f32_to_bf16_rne(vf[i]);
    TOMO_TRY(upload((uint16_t**)&dst[TOMO_VAL_BF16], vb.data(), nnz));
  }
  if (values & TOMO_VALUES_F16) {
    std::vector<_Float16> vh(nnz);
    for (size_t i = 0; i < nnz; ++i) vh[i] = (_Float16)vf[i];
    TOMO_TRY(upload((_Float16**)&dst[TOMO_VAL_F16], vh.data(), nnz));
  }
  return TOMO_OK;
}

void free_adj_layout(DevAdj& d) {
  dfree(d.slice_ptr);
  dfree(d.slice_rows);
  dfree(d.col);
  for (auto& v : d.val) dfree(v);
  dfree(d.tail_rows);
  dfree(d.tail_ptr);
  dfree(d.tail_col);
  for (auto& v : d.tail_val) dfree(v);
  dfree(d.chunk_beg);
  dfree(d.chunk_end);
  dfree(d.long_chunk_ptr);
  d = DevAdj();
}

void free_adj(tomo_op* op) {
  free_adj_layout(op->adj);
  dfree(op->partials);
  op->partials_cap = 0;
}

tomo_status upload_adj_layout(const HostAdj& h, uint32_t values, DevAdj& d) {
  if (h.col.size() >= (size_t)INT32_MAX)
    return fail(TOMO_EINVAL, "sliced-ELL layout exceeds 32-bit entry indices; lower adj_sell_max");
  d.n_slices = (int64_t)h.slice_ptr.size() - 1;
  d.n_medium = h.n_medium;
  d.n_long = h.n_long;
  d.n_chunks = (int64_t)h.chunk_beg.size();
  TOMO_TRY(upload(&d.slice_ptr, h.slice_ptr.data(), h.slice_ptr.size()));
  TOMO_TRY(upload(&d.slice_rows, h.slice_rows.data(), h.slice_rows.size()));
  TOMO_TRY(upload(&d.col, h.col.data(), h.col.size()));
  TOMO_TRY(upload_values(h.val, values, d.val));
  TOMO_TRY(upload(&d.tail_rows, h.tail_rows.data(), h.tail_rows.size()));
  TOMO_TRY(upload(&d.tail_ptr, h.tail_ptr.data(), h.tail_ptr.size()));
  TOMO_TRY(upload(&d.tail_col, h.tail_col.data(), h.tail_col.size()));
  TOMO_TRY(upload_values(h.tail_val, values, d.tail_val));
  TOMO_TRY(upload(&d.chunk_beg, h.chunk_beg.data(), h.chunk_beg.size()));
  TOMO_TRY(upload(&d.chunk_end, h.chunk_end.data(), h.chunk_end.size()));
  TOMO_TRY(upload(&d.long_chunk_ptr, h.long_chunk_ptr.data(), h.long_chunk_ptr.size()));
  return TOMO_OK;
}

// (Re)build the adjoint layout for op->tune on the host and upload it.
tomo_status upload_adj(tomo_op* op) {
  op->adj_ready = false;
  free_adj(op);
  build_adj_layout(op->s, op->tune, &op->hadj);
  const HostAdj& h = op->hadj;
  DevAdj& d = op->adj;
  TOMO_TRY(upload_adj_layout(h, op->g.values, d));
  if (d.n_chunks > 0) {
    const size_t pb = (size_t)d.n_chunks * op->cmax * sizeof(float2);
    if (hipMalloc((void**)&op->partials, pb) != hipSuccess) {
      op->partials = nullptr;
      return fail(TOMO_ENOMEM, "long-row partial sums (%zu B)", pb);
    }
    op->partials_cap = (size_t)d.n_chunks;
  }
  op->adj_ready = true;
  return TOMO_OK;
}

void free_tiles(tomo_op* op) {
  DevFwdTiles& f = op->ftile;
  dfree(f.wi_tile); dfree(f.wi_beg);
  for (int k = 0; k < 2; ++k) {
    dfree(f.pt_row[k]);
    dfree(f.pt_base[k]);
    for (auto& v : f.val[k]) dfree(v);
  }
  f = DevFwdTiles();
  DevAdjWin& a = op->awin;
  dfree(a.wi_tile); dfree(a.wi_q); dfree(a.wi_boff); dfree(a.q_row);
  for (auto& v : a.q_val) dfree(v);
  dfree(a.seg_tile); dfree(a.seg_chunk); dfree(a.seg_slot); dfree(a.red_tile); dfree(a.red_slot);
  dfree(a.chunk_tile);
  a = DevAdjWin();
  dfree(op->seg_partials);
  free_adj_layout(op->adj_dense);
}

// (Re)build the LDS-staged layouts for op->tune on the host and upload them.
tomo_status upload_tiles(tomo_op* op) {
  op->tiles_ready = false;
  free_tiles(op);
  for (int k = 0; k < 2; ++k) {   // row order, then the FFT-side form's angle-radius order
    HostFwdTiles h;
    TOMO_TRY(build_fwd_tiles(op->g, op->sdag, op->centres, op->tune, &h, k == 1));
    DevFwdTiles& d = op->ftile;
    if (k == 0) {
      d.n_wi = (int64_t)h.wi_tile.size();
      d.TS = h.TS; d.PS = h.PS; d.NT = h.NT; d.KW = h.KW;
      TOMO_TRY(upload(&d.wi_tile, h.wi_tile.data(), h.wi_tile.size()));
      TOMO_TRY(upload(&d.wi_beg, h.wi_beg.data(), h.wi_beg.size()));
    }
    TOMO_TRY(upload(&d.pt_row[k], h.pt_row.data(), h.pt_row.size()));
    TOMO_TRY(upload(&d.pt_base[k], h.pt_base.data(), h.pt_base.size()));
    TOMO_TRY(upload_values(h.pt_val, op->g.values, d.val[k]));
  }
  {
    HostAdjWin h;
    TOMO_TRY(build_adj_win(op->g, op->sdag, op->centres, op->tune, &h));
    DevAdjWin& d = op->awin;
    d.n_wi = (int64_t)h.wi_tile.size();
    d.TS = h.TS; d.RS = h.RS; d.NT = h.NT; d.KW = h.KW; d.QMAX = h.QMAX;
    TOMO_TRY(upload(&d.wi_tile, h.wi_tile.data(), h.wi_tile.size()));
    TOMO_TRY(upload(&d.wi_q, h.wi_q.data(), h.wi_q.size()));
    TOMO_TRY(upload(&d.wi_boff, h.wi_boff.data(), h.wi_boff.size()));
    TOMO_TRY(upload(&d.q_row, h.q_row.data(), h.q_row.size()));
    TOMO_TRY(upload_values(h.q_val, op->g.values, d.q_val));
    d.n_wi = h.n_wi;
    d.n_sseg = h.n_sseg;
    d.n_seg = (int64_t)h.seg_tile.size();
    d.max_seg_chunks = 0;
    for (size_t i = 0; i + 1 < h.seg_chunk.size(); ++i)
      d.max_seg_chunks = std::max(d.max_seg_chunks, h.seg_chunk[i + 1] - h.seg_chunk[i]);
    TOMO_TRY(upload(&d.chunk_tile, h.chunk_tile.data(), h.chunk_tile.size()));
    d.n_red = (int64_t)h.red_tile.size();
    d.n_slot = h.red_slot.empty() ? 0 : (int64_t)h.red_slot.back();
    TOMO_TRY(upload(&d.seg_tile, h.seg_tile.data(), h.seg_tile.size()));
    TOMO_TRY(upload(&d.seg_chunk, h.seg_chunk.data(), h.seg_chunk.size()));
    TOMO_TRY(upload(&d.seg_slot, h.seg_slot.data(), h.seg_slot.size()));
    TOMO_TRY(upload(&d.red_tile, h.red_tile.data(), h.red_tile.size()));
    TOMO_TRY(upload(&d.red_slot, h.red_slot.data(), h.red_slot.size()));
    if (d.n_slot > 0) {
      const size_t pb = (size_t)d.n_slot * h.TS * h.TS * op->cmax * sizeof(float2);
      if (hipMalloc((void**)&op->seg_partials, pb) != hipSuccess) {
        op->seg_partials = nullptr;
        return fail(TOMO_ENOMEM, "staged adjoint partial tiles (%zu B)", pb);
      }
    }
    // dense cells: the row kernels' layout over those cells (its long rows are a subset of the
    // full layout's, so the long-row partial-sum buffer already fits them)
    HostAdj hd;
    build_adj_layout(op->s, op->tune, &hd, &h.dense_cell);
    if ((size_t)hd.chunk_beg.size() > op->partials_cap)
      return fail(TOMO_EINVAL, "internal: dense-cell layout has more long-row chunks than the full one");
    TOMO_TRY(upload_adj_layout(hd, op->g.values, op->adj_dense));
  }
  op->tiles_ready = true;
  return TOMO_OK;
}

void free_device(tomo_op* op) {
  if (op->ev_fork) (void)hipEventDestroy(op->ev_fork);
  if (op->ev_join) (void)hipEventDestroy(op->ev_join);
  if (op->ev_join2) (void)hipEventDestroy(op->ev_join2);
  if (op->aux) (void)hipStreamDestroy(op->aux);
  if (op->aux2) (void)hipStreamDestroy(op->aux2);
  op->ev_fork = op->ev_join = op->ev_join2 = nullptr;
  op->aux = op->aux2 = nullptr;
  free_tiles(op);
  destroy_plans(op);
  free_solver(op);
  free_tv(op);
  for (auto& f : op->nrm.val)
    for (auto& v : f) dfree(v);
  dfree(op->fwd.col);
  for (auto& v : op->fwd.val) dfree(v);
  free_adj(op);
  dfree(op->kd_dev);
  dfree(op->phase_dev);
  for (auto* t : {&op->dft1, &op->dft2}) {
    dfree(t->tw);
    dfree(t->chirp);
    dfree(t->bhat_f);
    dfree(t->bhat_i);
    *t = fftk::DftTables();
  }
  dfree(op->dens);
  for (auto& f : op->filt_dev) dfree(f);
  dfree(op->X);
  dfree(op->Y);
  dfree(op->Xs);
  dfree(op->Ys);
}

// Tables of the hand-written DFTs of length N (computed in double): for N = 2^m in [16, 4096] the
// twiddles exp(-2 pi i j / N); for other N in [16, 4096] Bluestein's chirp conj(w_n) =
// exp(-i pi n^2 / N) and, at the power-of-two length M >= 2N - 1, the twiddles and the DFTs of
// the convolution kernels w (forward) and conj(w) (inverse) wrapped to negative indices, times 1/M
// (the DFT in double by the direct sum would be O(M^2); a radix-2 FFT in double is used).
tomo_status upload_dft_tables(int N, fftk::DftTables* t) {
  *t = fftk::DftTables();
  if (N < 16 || N > 4096) return TOMO_OK;
  const bool pow2 = (N & (N - 1)) == 0;
  int M = N;
  if (!pow2)
    for (M = 16; M < 2 * N - 1; M *= 2) {
    }
  auto twiddles = [](int m) {
    std::vector<std::complex<double>> tw(m);
    for (int j = 0; j < m; ++j) tw[j] = std::polar(1.0, -2.0 * M_PI * (double)j / (double)m);
    return tw;
  };
  auto to_f2 = [](const std::vector<std::complex<double>>& v, double scale) {
    std::vector<float2> o(v.size());
    for (size_t i = 0; i < v.size(); ++i)
      o[i] = make_float2((float)(v[i].real() * scale), (float)(v[i].imag() * scale));
    return o;
  };
  const std::vector<std::complex<double>> tw = twiddles(M);
  float2* d_tw = nullptr;
  TOMO_TRY(upload(&d_tw, to_f2(tw, 1.0).data(), (size_t)M));
  t->tw = d_tw;
  t->N = N;
  t->M = M;
  if (pow2) return TOMO_OK;
  // w_m = exp(+i pi m^2 / N) with m^2 reduced mod 2N first (exact in integers)
  auto w = [&](int64_t m) { return std::polar(1.0, M_PI * (double)((m * m) % (2 * (int64_t)N)) / N); };
  std::vector<std::complex<double>> chirp(N);
  for (int n = 0; n < N; ++n) chirp[n] = std::conj(w(n));
  // in-place iterative radix-2 DFT (forward sign) of a length-M sequence in double
  auto dft = [&](std::vector<std::complex<double>>& a) {
    for (int i = 1, j = 0; i < M; ++i) {
      int bit = M >> 1;
      for (; j & bit; bit >>= 1) j ^= bit;
      j ^= bit;
      if (i < j) std::swap(a[i], a[j]);
    }
    for (int len = 2; len <= M; len <<= 1)
      for (int i = 0; i < M; i += len)
        for (int k = 0; k < len / 2; ++k) {
          const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * tw[(size_t)k * (M / len)];
          a[i + k] = u + v;
          a[i + k + len / 2] = u - v;
        }
  };
  std::vector<std::complex<double>> bf(M, 0.0), bi(M, 0.0);
  for (int m = 0; m < N; ++m) {
    bf[m] = w(m);
    bi[m] = std::conj(w(m));
    if (m > 0) {
      bf[M - m] = bf[m];
      bi[M - m] = bi[m];
    }
  }
  dft(bf);
  dft(bi);
  float2 *d_chirp = nullptr, *d_bf = nullptr, *d_bi = nullptr;
  TOMO_TRY(upload(&d_chirp, to_f2(chirp, 1.0).data(), (size_t)N));
  t->chirp = d_chirp;
  TOMO_TRY(upload(&d_bf, to_f2(bf, 1.0 / M).data(), (size_t)M));
  t->bhat_f = d_bf;
  TOMO_TRY(upload(&d_bi, to_f2(bi, 1.0 / M).data(), (size_t)M));
  t->bhat_i = d_bi;
  return TOMO_OK;
}

tomo_status upload_all(tomo_op* op) {
  const Geom& g = op->g;
  op->cmax = (g.max_batch + 1) / 2;
  TOMO_HIP(hipDeviceGetAttribute(&op->n_cu, hipDeviceAttributeMultiprocessorCount, op->device));
  TOMO_HIP(hipStreamCreateWithFlags(&op->aux, hipStreamNonBlocking));
  TOMO_HIP(hipStreamCreateWithFlags(&op->aux2, hipStreamNonBlocking));
  TOMO_HIP(hipEventCreateWithFlags(&op->ev_fork, hipEventDisableTiming));
  TOMO_HIP(hipEventCreateWithFlags(&op->ev_join, hipEventDisableTiming));
  TOMO_HIP(hipEventCreateWithFlags(&op->ev_join2, hipEventDisableTiming));
  {
    HostEll ell;
    build_ell(op->sdag, g.kw * g.kw, &ell);
    op->fwd.rows = op->sdag.rows;
    op->fwd.W2 = ell.W2;
    TOMO_TRY(upload(&op->fwd.col, ell.col.data(), ell.col.size()));
    TOMO_TRY(upload_values(ell.val, g.values, op->fwd.val));
  }
  TOMO_TRY(upload_adj(op));
  TOMO_TRY(upload_tiles(op));
  std::vector<float> kdf(op->kd.begin(), op->kd.end());
  TOMO_TRY(upload(&op->kd_dev, kdf.data(), kdf.size()));
  if (g.cfrac != 0.0) {
    // exp(-2 pi i k f / L) in float64, k the signed frequency of FFT-ordered index kf
    std::vector<float2> ph((size_t)g.L);
    for (int kf = 0; kf < g.L; ++kf) {
      const int k = kf < g.L - g.L / 2 ? kf : kf - g.L;
      const double a = -2.0 * M_PI * (double)k * g.cfrac / (double)g.L;
      ph[(size_t)kf] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    TOMO_TRY(upload(&op->phase_dev, ph.data(), ph.size()));
  }
  for (int f = TOMO_FILTER_RAMLAK; f <= TOMO_FILTER_HAMMING; ++f) {
    std::vector<double> d;
    filter_diagonal(g, f, &d);
    std::vector<float> df(d.begin(), d.end());
    TOMO_TRY(upload(&op->filt_dev[f], df.data(), df.size()));
  }
  TOMO_TRY(upload_dft_tables(g.L, &op->dft1));
  TOMO_TRY(upload_dft_tables(g.G, &op->dft2));
  const size_t xb = (size_t)g.G * g.G * op->cmax * sizeof(float2);
  const size_t yb = (size_t)g.L * g.nt * op->cmax * sizeof(float2);
  if (hipMalloc((void**)&op->X, xb) != hipSuccess) {
    op->X = nullptr;
    return fail(TOMO_ENOMEM, "Cartesian workspace (%zu B)", xb);
  }
  if (hipMalloc((void**)&op->Y, yb) != hipSuccess) {
    op->Y = nullptr;
    return fail(TOMO_ENOMEM, "polar workspace (%zu B)", yb);
  }
  if (hipMalloc((void**)&op->Xs, xb) != hipSuccess) {
    op->Xs = nullptr;
    return fail(TOMO_ENOMEM, "Cartesian FFT workspace (%zu B)", xb);
  }
  if (hipMalloc((void**)&op->Ys, yb) != hipSuccess) {
    op->Ys = nullptr;
    return fail(TOMO_ENOMEM, "polar FFT workspace (%zu B)", yb);
  }
  TOMO_HIP(hipDeviceSynchronize());
  return TOMO_OK;
}

bool misaligned(const void* p, size_t a) { return ((uintptr_t)p) % a != 0; }

}  // namespace

tomo_status check_apply(const tomo_op* op, const void* in, const void* out, int32_t batch,
                        int32_t values) {
  if (!op) return fail(TOMO_EINVAL, "operator is NULL");
  if (op->device < 0) return fail(TOMO_ESTATE, "operator was built without a device");
  if (batch < 0 || batch > op->g.max_batch)
    return fail(TOMO_EINVAL, "batch %d outside [0, max_batch=%d]", batch, op->g.max_batch);
  if (batch > 0 && (!in || !out)) return fail(TOMO_EINVAL, "NULL data pointer");
  if (batch > 0 && (misaligned(in, 16) || misaligned(out, 16)))
    return fail(TOMO_EINVAL, "data pointers must be 16-byte aligned");
  if (values < 0 || values > 2) return fail(TOMO_EINVAL, "unknown value type %d", values);
  if (!(op->values & (1u << values)))
    return fail(TOMO_ESTATE, "value type %d was not built for this operator", values);
  return TOMO_OK;
}


int64_t project_sumsq_blocks(const tomo_op* op) {
  return op->tune.det_fft ? det_inverse_blocks_per_channel(op) : 0;
}

int64_t backproject_sumsq_blocks(const tomo_op* op) {
  return op->tune.grid_fft ? grid_inverse_blocks_per_channel(op) : 0;
}

// project: embed + deapodise -> F2D -> S^dagger -> F1D^-1 -> crop (Eq. (2), first line)
namespace {

// project from the forward grid transform's output in op->Xs onwards: forward SpMM, inverse
// detector DFT, crop
tomo_status project_from_grid(tomo_op* op, float* y, int B, int vt, FFTPlans* p, hipStream_t st,
                              double* sumsq) {
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  if (spmm_fwd_slowest_ok(op, C, vt)) {
    // the staged forward reads its patches from the FFT-side grid and writes the FFT-side polar
    // rows itself
    TOMO_TRY(launch_spmm_fwd(op, op->Xs, op->Ys, C, vt, st, true));
  } else {
    TOMO_TRY(launch_to_channel_fastest(op->Xs, op->X, (int64_t)g.G * g.G, C, st));
    TOMO_TRY(launch_spmm_fwd(op, op->X, op->Y, C, vt, st));
    TOMO_TRY(launch_polar_to_slowest(op->Y, op->Ys, g.L, g.nt, C, st));
  }
  if (op->tune.det_fft && det_fft_supported(op))
    return launch_det_inverse_crop(op, op->Ys, y, B, 1.0f / (float)g.L, sumsq, st);
  if (op->phase_dev)
    TOMO_TRY(launch_phase_rows(op->Ys, op->phase_dev, g.L, (int64_t)C * g.nt, false, st));
  TOMO_TRY(fft_exec(p->inv1, p, op->Ys, st));
  TOMO_TRY(launch_crop_sino(op, op->Ys, y, B, 1.0f / (float)g.L, st));
  return TOMO_OK;
}

}  // namespace

tomo_status apply_project(tomo_op* op, const float* x, float* y, int B, int vt, hipStream_t st,
                          double* sumsq) {
  if (sumsq && project_sumsq_blocks(op) == 0)
    return fail(TOMO_EINVAL, "internal: output norms need the hand-written detector transform");
  FFTPlans* p = nullptr;
  TOMO_TRY(get_plans(op, (B + 1) / 2, &p));
  if (op->tune.grid_fft && grid_fft_supported(op)) {
    TOMO_TRY(launch_grid_forward(op, x, op->Xs, B, st));
  } else {
    TOMO_TRY(launch_embed(op, x, op->Xs, B, st));
    TOMO_TRY(fft_exec(p->fwd2, p, op->Xs, st));
  }
  return project_from_grid(op, y, B, vt, p, st, sumsq);
}

bool project_cg_supported(const tomo_op* op) {
  return op->tune.grid_fft && grid_cg_step_supported(op);
}

tomo_status apply_project_cg(tomo_op* op, float* pdir, const CgStep& cg, float* y, int B, int vt,
                             hipStream_t st, double* sumsq) {
  if (!project_cg_supported(op))
    return fail(TOMO_EINVAL, "internal: the fused CG step needs the hand-written grid transform");
  if (sumsq && project_sumsq_blocks(op) == 0)
    return fail(TOMO_EINVAL, "internal: output norms need the hand-written detector transform");
  FFTPlans* p = nullptr;
  TOMO_TRY(get_plans(op, (B + 1) / 2, &p));
  TOMO_TRY(launch_grid_forward(op, pdir, op->Xs, B, st, &cg));
  return project_from_grid(op, y, B, vt, p, st, sumsq);
}

// backproject: pad -> F1D -> S diag(D) -> F2D^H -> crop + deapodise (Eq. (2), second line)
namespace {

// backproject from the channel-fastest polar data in op->Y onwards: filter, adjoint SpMM, inverse
// 2D DFT, crop + deapodise
tomo_status backproject_from_polar(tomo_op* op, float* x, int B, int vt, int filter,
                                   float extra_scale, FFTPlans* p, hipStream_t st, double* sumsq) {
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  const float* ds = nullptr;
  if (filter == TOMO_FILTER_DENSITY)
    TOMO_TRY(launch_scale_rows(op->Y, op->dens, (int64_t)g.L * g.nt, C, st));
  else if (filter != TOMO_FILTER_NONE)
    ds = op->filt_dev[filter];
  const float scale = extra_scale / (float)g.L;
  if (spmm_adj_slowest_ok(op, C, vt)) {
    // the staged adjoint writes its tiles into the FFT-side grid itself
    TOMO_TRY(launch_spmm_adj(op, op->Y, op->Xs, C, vt, ds, st, true));
  } else {
    TOMO_TRY(launch_spmm_adj(op, op->Y, op->X, C, vt, ds, st));
    TOMO_TRY(launch_to_channel_slowest(op->X, op->Xs, (int64_t)g.G * g.G, C, st));
  }
  if (op->tune.grid_fft && grid_fft_supported(op))
    return launch_grid_inverse(op, op->Xs, x, B, scale, sumsq, st);
  TOMO_TRY(fft_exec(p->inv2, p, op->Xs, st));
  TOMO_TRY(launch_crop_image(op, op->Xs, x, B, scale, st));
  return TOMO_OK;
}

}  // namespace

tomo_status apply_backproject(tomo_op* op, const float* y, float* x, int B, int vt, int filter,
                              float extra_scale, hipStream_t st, double* sumsq) {
  if (sumsq && backproject_sumsq_blocks(op) == 0)
    return fail(TOMO_EINVAL, "internal: output norms need the hand-written grid transform");
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  FFTPlans* p = nullptr;
  TOMO_TRY(get_plans(op, C, &p));
  if (op->tune.det_fft == 1 && det_cf_supported(op)) {
    // the fused transform writes the adjoint SpMM's channel-fastest polar layout itself
    TOMO_TRY(launch_det_pad_forward(op, y, op->Y, B, true, st));
  } else {
    if (op->tune.det_fft && det_fft_supported(op)) {
      TOMO_TRY(launch_det_pad_forward(op, y, op->Ys, B, false, st));
    } else {
      TOMO_TRY(launch_pad_sino(op, y, op->Ys, B, st));
      TOMO_TRY(fft_exec(p->fwd1, p, op->Ys, st));
      if (op->phase_dev)
        TOMO_TRY(launch_phase_rows(op->Ys, op->phase_dev, g.L, (int64_t)C * g.nt, true, st));
    }
    TOMO_TRY(launch_polar_to_fastest(op->Ys, op->Y, g.L, g.nt, C, st));
  }
  return backproject_from_polar(op, x, B, vt, filter, extra_scale, p, st, sumsq);
}

bool backproject_residual_supported(const tomo_op* op) {
  return op->tune.det_fft == 1 && det_cf_supported(op);
}

tomo_status apply_backproject_residual(tomo_op* op, float* r, const float* q, const double* alpha,
                                       float* x, int B, int vt, hipStream_t st, double* sumsq) {
  if (!backproject_residual_supported(op))
    return fail(TOMO_EINVAL, "internal: the fused residual step needs the channel-fastest front");
  if (sumsq && backproject_sumsq_blocks(op) == 0)
    return fail(TOMO_EINVAL, "internal: output norms need the hand-written grid transform");
  FFTPlans* p = nullptr;
  TOMO_TRY(get_plans(op, (B + 1) / 2, &p));
  TOMO_TRY(launch_det_residual_forward(op, r, q, alpha, op->Y, B, st));
  return backproject_from_polar(op, x, B, vt, TOMO_FILTER_NONE, 1.0f, p, st, sumsq);
}

tomo_status normal_supported(const tomo_op* op) {
  const Geom& g = op->g;
  if (g.np != g.L)
    return fail(TOMO_EUNSUPPORTED, "the normal operator needs n_det == grid (n_det=%d, grid=%d)",
                g.np, g.L);
  if (g.kw > 5) return fail(TOMO_EUNSUPPORTED, "the normal operator needs kw <= 5 (kw=%d)", g.kw);
  return TOMO_OK;
}

// Build (host, float64) and upload W = S diag(D) S^dagger for `filter` in every value type the
// operator holds; synchronous, first use per filter.
tomo_status ensure_normal(tomo_op* op, int filter) {
  DevNormal& nrm = op->nrm;
  bool have = false;
  for (int vt = 0; vt < 3; ++vt) have |= nrm.val[filter][vt] != nullptr;
  if (have) return TOMO_OK;
  TOMO_TRY(normal_supported(op));
  const Geom& g = op->g;
  const int R = g.kw - 1, S2 = (2 * R + 1) * (2 * R + 1);
  nrm.R = R;
  nrm.stride = (S2 + 7) / 8 * 8;
  std::vector<double> d;
  if (filter != TOMO_FILTER_NONE) filter_diagonal(g, filter, &d);
  // one float32 stencil per value type, each the normal operator of the forward operator with
  // those values: W = S_v D S_v^dagger from the matrix with its values rounded to the type (so
  // it stays positive semidefinite; rounding W itself to 16 bits does not, and CG on it diverged)
  for (int vt = 0; vt < 3; ++vt) {
    if (!(op->values & (1u << vt))) continue;
    HostCSR sv = op->s, sdv = op->sdag;
    if (vt != TOMO_VAL_F32)
      for (HostCSR* m : {&sv, &sdv})
        for (double& v : m->val) {
          const float f = (float)v;
          if (vt == TOMO_VAL_BF16) {
            const uint32_t b = (uint32_t)f32_to_bf16_rne(f) << 16;
            float r;
            std::memcpy(&r, &b, 4);
            v = r;
          } else {
            v = (double)(float)(_Float16)f;
          }
        }
    std::vector<double> w;
    TOMO_TRY(build_normal_values(g, sv, sdv, d.empty() ? nullptr : d.data(), nrm.stride, &w));
    void* dst[3] = {nullptr, nullptr, nullptr};
    TOMO_TRY(upload_values(w, TOMO_VALUES_F32, dst));
    nrm.val[filter][vt] = dst[TOMO_VAL_F32];
  }
  return TOMO_OK;
}

// A^T D A x = crop(k*, 1/L) F2D^H W F2D embed(k* x), all on the channel-slowest grid buffers
tomo_status apply_normal(tomo_op* op, const float* x, float* out, int B, int vt, int filter,
                         hipStream_t st, const CgStep* cg, double* sumsq, const float* dotw) {
  const Geom& g = op->g;
  const int C = (B + 1) / 2;
  if (cg && !project_cg_supported(op))
    return fail(TOMO_EINVAL, "internal: the fused CG step needs the hand-written grid transform");
  if (sumsq && backproject_sumsq_blocks(op) == 0)
    return fail(TOMO_EINVAL, "internal: output sums need the hand-written grid transform");
  TOMO_TRY(ensure_normal(op, filter));
  FFTPlans* p = nullptr;
  TOMO_TRY(get_plans(op, C, &p));
  const bool hand = op->tune.grid_fft && grid_fft_supported(op);
  if (hand) {
    TOMO_TRY(launch_grid_forward(op, x, op->Xs, B, st, cg));
  } else {
    TOMO_TRY(launch_embed(op, x, op->Xs, B, st));
    TOMO_TRY(fft_exec(p->fwd2, p, op->Xs, st));
  }
  TOMO_TRY(launch_normal_stencil(op, op->Xs, op->X, C, vt, filter, st));
  if (hand) return launch_grid_inverse(op, op->X, out, B, 1.0f / (float)g.L, sumsq, st, dotw);
  TOMO_TRY(fft_exec(p->inv2, p, op->X, st));
  TOMO_TRY(launch_crop_image(op, op->X, out, B, 1.0f / (float)g.L, st));
  return TOMO_OK;
}

}  // namespace tomo

using namespace tomo;

extern "C" {

tomo_status tomo_build_operator(const tomo_geometry* gin, int device, tomo_op** out) {
  clear_error();
  if (!out) return fail(TOMO_EINVAL, "out is NULL");
  *out = nullptr;
  std::unique_ptr<tomo_op> op(new (std::nothrow) tomo_op());
  if (!op) return fail(TOMO_ENOMEM, "host allocation failed");
  TOMO_TRY(resolve_geometry(gin, &op->g));
  try {
    build_sdag(op->g, &op->sdag, &op->centres);
    transpose_csr(op->sdag, &op->s);
    deapod_factors(op->g, &op->kd);
    if (device < 0) build_adj_layout(op->s, op->tune, &op->hadj);
  } catch (const std::bad_alloc&) {
    return fail(TOMO_ENOMEM, "host allocation failed while building the matrices");
  }
  for (double v : op->kd)
    if (!(v > 0) || !std::isfinite(v))
      return fail(TOMO_EINVAL, "deapodisation undefined (kernel transform not positive)");
  for (int64_t r = 0; r < op->s.rows; ++r) op->cols_touched += (op->s.rowptr[r + 1] > op->s.rowptr[r]);
  for (int64_t r = 0; r < op->sdag.rows; ++r)
    op->polar_nonempty += (op->sdag.rowptr[r + 1] > op->sdag.rowptr[r]);
  op->device = device;
  if (device >= 0) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev)
      return fail(TOMO_EINVAL, "device %d not available", device);
    DeviceGuard guard(device);
    if (guard.err != hipSuccess) return fail(TOMO_EHIP, "hipSetDevice(%d) failed", device);
    const tomo_status st = upload_all(op.get());
    if (st != TOMO_OK) {
      free_device(op.get());
      return st;
    }
    op->values = op->g.values;
  } else if (device != -1) {
    return fail(TOMO_EINVAL, "device must be >= 0, or -1 for a host-only operator");
  }
  *out = op.release();
  return TOMO_OK;
}

tomo_status tomo_project(tomo_op* op, const float* x, float* y, int32_t batch, int32_t values,
                         void* stream) {
  clear_error();
  TOMO_TRY(check_apply(op, x, y, batch, values));
  if (batch == 0) return TOMO_OK;
  DeviceGuard guard(op->device);
  return apply_project(op, x, y, batch, values, (hipStream_t)stream);
}

tomo_status tomo_backproject(tomo_op* op, const float* y, float* x, int32_t batch, int32_t values,
                             void* stream) {
  clear_error();
  TOMO_TRY(check_apply(op, y, x, batch, values));
  if (batch == 0) return TOMO_OK;
  DeviceGuard guard(op->device);
  return apply_backproject(op, y, x, batch, values, TOMO_FILTER_NONE, 1.0f, (hipStream_t)stream);
}

tomo_status tomo_irradon(tomo_op* op, const float* y, float* x, int32_t batch, int32_t values,
                         int32_t filter, void* stream) {
  clear_error();
  TOMO_TRY(check_apply(op, y, x, batch, values));
  if (filter < TOMO_FILTER_RAMLAK || filter > TOMO_FILTER_DENSITY)
    return fail(TOMO_EINVAL, "irradon needs a filter (got %d)", filter);
  if (filter == TOMO_FILTER_DENSITY && !op->dens)
    return fail(TOMO_ESTATE, "density weights not computed (tomo_density_filter)");
  if (batch == 0) return TOMO_OK;
  DeviceGuard guard(op->device);
  const float scale = filter == TOMO_FILTER_DENSITY
                          ? (float)((double)op->g.L / ((double)op->g.G * op->g.G))
                          : (float)(M_PI / op->g.nt);
  return apply_backproject(op, y, x, batch, values, filter, scale, (hipStream_t)stream);
}

tomo_status tomo_slice_fwd(tomo_op* op, const float* Xc, float* Yp, int32_t batch, int32_t values,
                           void* stream) {
  clear_error();
  TOMO_TRY(check_apply(op, Xc, Yp, batch, values));
  if (batch == 0) return TOMO_OK;
  DeviceGuard guard(op->device);
  return launch_spmm_fwd(op, (const float2*)Xc, (float2*)Yp, (batch + 1) / 2, values,
                         (hipStream_t)stream);
}

tomo_status tomo_slice_adj(tomo_op* op, const float* Yp, float* Xc, int32_t batch, int32_t values,
                           int32_t filter, void* stream) {
  clear_error();
  TOMO_TRY(check_apply(op, Yp, Xc, batch, values));
  if (filter < TOMO_FILTER_NONE || filter > TOMO_FILTER_HAMMING)
    return fail(TOMO_EINVAL, "unknown filter %d", filter);
  if (batch == 0) return TOMO_OK;
  DeviceGuard guard(op->device);
  const float* ds = (filter == TOMO_FILTER_NONE) ? nullptr : op->filt_dev[filter];
  return launch_spmm_adj(op, (const float2*)Yp, (float2*)Xc, (batch + 1) / 2, values, ds,
                         (hipStream_t)stream);
}

tomo_status tomo_solve(tomo_op* op, const float* b, float* x, int32_t batch,
                       const tomo_solve_opts* opts, void* stream) {
  clear_error();
  if (!opts) return fail(TOMO_EINVAL, "opts is NULL");
  TOMO_TRY(check_apply(op, b, x, batch, opts->values));
  if (opts->method < TOMO_SOLVE_CGLS || opts->method > TOMO_SOLVE_TV_SPLIT_BREGMAN)
    return fail(TOMO_EINVAL, "unknown solver %d", opts->method);
  if (opts->method == TOMO_SOLVE_CGNR || opts->method == TOMO_SOLVE_SIRT_BB_NORMAL)
    TOMO_TRY(normal_supported(op));
  if (opts->iters < 0 || opts->refine_outer < 1)
    return fail(TOMO_EINVAL, "iters must be >= 0 and refine_outer >= 1");
  if (opts->filter < TOMO_FILTER_NONE || opts->filter > TOMO_FILTER_HAMMING)
    return fail(TOMO_EINVAL, "unknown filter %d", opts->filter);
  if (opts->method == TOMO_SOLVE_TV_SPLIT_BREGMAN &&
      (!(opts->tv_mu > 0) || !(opts->tv_lambda > 0) || !std::isfinite(opts->tv_mu) ||
       !std::isfinite(opts->tv_lambda) || opts->use_x0))
    return fail(TOMO_EINVAL, "split Bregman needs finite tv_mu > 0, tv_lambda > 0 and x0 = 0");
  if ((opts->method == TOMO_SOLVE_SIRT_BB || opts->method == TOMO_SOLVE_SIRT_BB_NORMAL) &&
      (opts->refine_outer != 1 || opts->use_x0))
    return fail(TOMO_EUNSUPPORTED, "SIRT-BB runs from zero without refinement");
  if (batch == 0) return TOMO_OK;
  DeviceGuard guard(op->device);
  return run_solve(op, b, x, batch, opts, (hipStream_t)stream);
}

tomo_status tomo_density_filter(tomo_op* op, int32_t iters, double* resid) {
  clear_error();
  if (!op) return fail(TOMO_EINVAL, "operator is NULL");
  if (op->device < 0) return fail(TOMO_ESTATE, "operator was built without a device");
  if (iters < 1 || iters > 100000) return fail(TOMO_EINVAL, "iters must be in [1, 100000]");
  if (!(op->values & TOMO_VALUES_F32)) return fail(TOMO_ESTATE, "needs float32 values");
  DeviceGuard guard(op->device);
  TOMO_HIP(hipDeviceSynchronize());
  TOMO_TRY(run_density(op, iters, resid, nullptr));
  TOMO_HIP(hipDeviceSynchronize());
  return TOMO_OK;
}

tomo_status tomo_export_density(const tomo_op* op, float* w) {
  clear_error();
  if (!op || !w) return fail(TOMO_EINVAL, "NULL argument");
  if (!op->dens) return fail(TOMO_ESTATE, "density weights not computed (tomo_density_filter)");
  DeviceGuard guard(op->device);
  TOMO_HIP(hipMemcpy(w, op->dens, (size_t)op->g.L * op->g.nt * sizeof(float), hipMemcpyDeviceToHost));
  return TOMO_OK;
}

tomo_status tomo_autotune(tomo_op* op, int32_t batch, int32_t values, int32_t rounds,
                          tomo_tuning* best, double* fwd_ms, double* adj_ms) {
  clear_error();
  if (!op) return fail(TOMO_EINVAL, "operator is NULL");
  if (op->device < 0) return fail(TOMO_ESTATE, "operator was built without a device");
  if (batch < 1 || batch > op->g.max_batch)
    return fail(TOMO_EINVAL, "batch %d outside [1, max_batch=%d]", batch, op->g.max_batch);
  if (values < 0 || values > 2 || !(op->values & (1u << values)))
    return fail(TOMO_ESTATE, "value type %d was not built for this operator", values);
  if (rounds < 1 || rounds > 8) return fail(TOMO_EINVAL, "rounds must be in [1, 8]");
  {
    DeviceGuard guard(op->device);
    TOMO_HIP(hipDeviceSynchronize());
    TOMO_TRY(autotune(op, batch, values, rounds, fwd_ms, adj_ms));
  }
  if (best) TOMO_TRY(tomo_get_tuning(op, best));
  return TOMO_OK;
}

tomo_status tomo_normal(tomo_op* op, const float* x, float* out, int32_t batch, int32_t values,
                        int32_t filter, void* stream) {
  clear_error();
  TOMO_TRY(check_apply(op, x, out, batch, values));
  if (filter < TOMO_FILTER_NONE || filter > TOMO_FILTER_HAMMING)
    return fail(TOMO_EINVAL, "unknown filter %d", filter);
  TOMO_TRY(normal_supported(op));
  if (batch == 0) return TOMO_OK;
  DeviceGuard guard(op->device);
  return apply_normal(op, x, out, batch, values, filter, (hipStream_t)stream);
}

tomo_status tomo_export_normal(const tomo_op* op, int32_t filter, double* w) {
  clear_error();
  if (!op || !w) return fail(TOMO_EINVAL, "NULL argument");
  if (filter < TOMO_FILTER_NONE || filter > TOMO_FILTER_HAMMING)
    return fail(TOMO_EINVAL, "unknown filter %d", filter);
  TOMO_TRY(normal_supported(op));
  const Geom& g = op->g;
  const int D = 2 * g.kw - 1;
  std::vector<double> d;
  if (filter != TOMO_FILTER_NONE) filter_diagonal(g, filter, &d);
  std::vector<double> all;
  TOMO_TRY(build_normal_values(g, op->s, op->sdag, d.empty() ? nullptr : d.data(), D * D, &all));
  std::memcpy(w, all.data(), all.size() * sizeof(double));
  return TOMO_OK;
}

namespace {

tomo_status check_tv(const tomo_op* op, const float* x, int32_t batch, double eps, double weight,
                     const float* grad, const double* value) {
  if (!op) return fail(TOMO_EINVAL, "operator is NULL");
  if (op->device < 0) return fail(TOMO_ESTATE, "operator was built without a device");
  if (batch < 0 || batch > op->g.max_batch)
    return fail(TOMO_EINVAL, "batch %d outside [0, max_batch=%d]", batch, op->g.max_batch);
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(TOMO_EINVAL, "eps must be positive and finite");
  if (!std::isfinite(weight)) return fail(TOMO_EINVAL, "weight must be finite");
  if (batch > 0 && !x) return fail(TOMO_EINVAL, "NULL image pointer");
  if (batch > 0 && (misaligned(x, 4) || misaligned(grad, 4) || misaligned(value, 8)))
    return fail(TOMO_EINVAL, "misaligned pointer");
  return TOMO_OK;
}

}  // namespace

tomo_status tomo_tv(tomo_op* op, const float* x, int32_t batch, double eps, double weight,
                    float* grad, double* value, void* stream) {
  clear_error();
  const tomo_status s = check_tv(op, x, batch, eps, weight, grad, value);
  if (s != TOMO_OK) return s;
  if (batch == 0 || (!grad && !value)) return TOMO_OK;
  DeviceGuard guard(op->device);
  return launch_tv(op, x, batch, eps, weight, grad, value, (hipStream_t)stream);
}

tomo_status tomo_tv_noalloc(const tomo_op* op, const float* x, int32_t batch, double eps,
                            double weight, float* grad, double* value, void* stream) {
  clear_error();
  const tomo_status s = check_tv(op, x, batch, eps, weight, grad, value);
  if (s != TOMO_OK) return s;
  if (batch == 0 || (!grad && !value)) return TOMO_OK;
  DeviceGuard guard(op->device);
  if (guard.err != hipSuccess)
    return fail(TOMO_EHIP, "hipSetDevice(%d): %s", op->device, hipGetErrorString(guard.err));
  return launch_tv_noalloc(op, x, batch, eps, weight, grad, value, (hipStream_t)stream);
}

tomo_status tomo_op_info_get(const tomo_op* op, tomo_op_info* out) {
  clear_error();
  if (!op || !out) return fail(TOMO_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof *out);
  const Geom& g = op->g;
  out->n = g.n;
  out->n_angles = g.nt;
  out->n_det = g.np;
  out->grid = g.G;
  out->kw = g.kw;
  out->max_batch = g.max_batch;
  out->beta = g.beta;
  out->center = g.center;
  out->n_polar = op->sdag.rows;
  out->n_cart = op->s.rows;
  out->nnz = op->sdag.nnz();
  out->cols_touched = op->cols_touched;
  out->polar_nonempty = op->polar_nonempty;
  out->adj_sell_rows = op->hadj.sell_rows;
  out->adj_sell_padding = op->hadj.sell_padding;
  out->adj_medium_rows = op->hadj.n_medium;
  out->adj_long_rows = op->hadj.n_long;
  out->adj_long_chunks = (int64_t)op->hadj.chunk_beg.size();
  out->device = op->device;
  out->values = op->values;
  return TOMO_OK;
}

tomo_status tomo_export_csr(const tomo_op* op, int32_t which, int64_t* rowptr, int32_t* col,
                            double* val) {
  clear_error();
  if (!op) return fail(TOMO_EINVAL, "operator is NULL");
  if (which != 0 && which != 1) return fail(TOMO_EINVAL, "which must be 0 or 1");
  const HostCSR& m = which == 0 ? op->sdag : op->s;
  if (rowptr) std::memcpy(rowptr, m.rowptr.data(), m.rowptr.size() * sizeof(int64_t));
  if (col) std::memcpy(col, m.col.data(), m.col.size() * sizeof(int32_t));
  if (val) std::memcpy(val, m.val.data(), m.val.size() * sizeof(double));
  return TOMO_OK;
}

tomo_status tomo_export_factors(const tomo_op* op, int32_t filter, double* kd, double* filt) {
  clear_error();
  if (!op) return fail(TOMO_EINVAL, "operator is NULL");
  if (filter < TOMO_FILTER_NONE || filter > TOMO_FILTER_HAMMING)
    return fail(TOMO_EINVAL, "unknown filter %d", filter);
  if (kd) std::memcpy(kd, op->kd.data(), op->kd.size() * sizeof(double));
  if (filt) {
    std::vector<double> d;
    filter_diagonal(op->g, filter, &d);
    std::memcpy(filt, d.data(), d.size() * sizeof(double));
  }
  return TOMO_OK;
}

tomo_status tomo_check_layouts(const tomo_op* op, double* max_rel_err) {
  clear_error();
  if (!op || !max_rel_err) return fail(TOMO_EINVAL, "NULL argument");
  return check_layouts(op->g, op->sdag, op->s, op->centres, op->tune, max_rel_err);
}

tomo_status tomo_get_tuning(const tomo_op* op, tomo_tuning* out) {
  clear_error();
  if (!op || !out) return fail(TOMO_EINVAL, "NULL argument");
  out->fwd_channels_per_lane = op->tune.fwd_cpl;
  out->adj_channels_per_lane = op->tune.adj_cpl;
  out->adj_sell_max = op->tune.sell_max;
  out->adj_sell_sigma = op->tune.sell_sigma;
  out->adj_medium_max = op->tune.medium_max;
  out->adj_chunk = op->tune.chunk;
  out->fwd_tiled = op->tune.fwd_tiled;
  out->adj_tiled = op->tune.adj_tiled;
  out->tile = op->tune.tile;
  out->tile_points = op->tune.tile_points;
  out->adj_tile_points = op->tune.adj_tile_points;
  out->normal_tiled = op->tune.normal_tiled;
  out->adj_sell_xcd_rows = op->tune.sell_xcd_rows;
  out->adj_medium_xcd_rows = op->tune.medium_xcd_rows;
  out->fwd_rows_per_group = op->tune.fwd_rows_per_group;
  out->det_fft = op->tune.det_fft;
  out->grid_fft = op->tune.grid_fft;
  out->adj_sell_tiles = op->tune.sell_tiles;
  out->tile_strip = op->tune.tile_strip;
  out->adj_dense_mode = op->tune.adj_dense_mode;
  out->adj_seg_chunks = op->tune.adj_seg_chunks;
  out->adj_run = op->tune.adj_run;
  return TOMO_OK;
}

tomo_status tomo_set_tuning(tomo_op* op, const tomo_tuning* in) {
  clear_error();
  if (!op || !in) return fail(TOMO_EINVAL, "NULL argument");
  Tuning t;
  t.fwd_cpl = in->fwd_channels_per_lane;
  t.adj_cpl = in->adj_channels_per_lane;
  t.sell_max = in->adj_sell_max;
  t.sell_sigma = in->adj_sell_sigma;
  t.medium_max = in->adj_medium_max;
  t.chunk = in->adj_chunk;
  t.fwd_tiled = in->fwd_tiled;
  t.adj_tiled = in->adj_tiled;
  t.tile = in->tile;
  t.tile_points = in->tile_points;
  t.adj_tile_points = in->adj_tile_points;
  t.normal_tiled = in->normal_tiled;
  t.sell_xcd_rows = in->adj_sell_xcd_rows;
  t.medium_xcd_rows = in->adj_medium_xcd_rows;
  t.fwd_rows_per_group = in->fwd_rows_per_group;
  t.det_fft = in->det_fft;
  t.grid_fft = in->grid_fft;
  t.sell_tiles = in->adj_sell_tiles;
  t.tile_strip = in->tile_strip;
  t.adj_dense_mode = in->adj_dense_mode;
  t.adj_seg_chunks = in->adj_seg_chunks;
  t.adj_run = in->adj_run;
  return apply_tuning(op, t);
}

}  // extern "C"

namespace tomo {
tomo_status apply_tuning(tomo_op* op, const Tuning& t) {
  TOMO_TRY(check_tuning(t));
  const bool relayout = t.sell_max != op->tune.sell_max || t.sell_sigma != op->tune.sell_sigma ||
                        t.sell_tiles != op->tune.sell_tiles ||
                        t.medium_max != op->tune.medium_max || t.chunk != op->tune.chunk;
  // the staged adjoint's dense cells use a row layout with the same bins, so it is rebuilt too
  const bool retile = relayout || t.tile != op->tune.tile || t.tile_points != op->tune.tile_points ||
                      t.adj_tile_points != op->tune.adj_tile_points || t.tile_strip != op->tune.tile_strip ||
                      t.adj_dense_mode != op->tune.adj_dense_mode ||
                      t.adj_seg_chunks != op->tune.adj_seg_chunks || t.adj_run != op->tune.adj_run;
  op->tune = t;
  if (op->device < 0) {
    if (relayout) build_adj_layout(op->s, op->tune, &op->hadj);
    return TOMO_OK;
  }
  if (!relayout && !retile) return TOMO_OK;
  DeviceGuard guard(op->device);
  TOMO_HIP(hipDeviceSynchronize());
  if (relayout) TOMO_TRY(upload_adj(op));
  if (retile) TOMO_TRY(upload_tiles(op));
  TOMO_HIP(hipDeviceSynchronize());
  return TOMO_OK;
}
}  // namespace tomo

extern "C" {

void tomo_destroy_operator(tomo_op* op) {
  if (!op) return;
  if (op->device >= 0) {
    DeviceGuard guard(op->device);
    (void)hipDeviceSynchronize();
    free_device(op);
  }
  delete op;
}

const char* tomo_last_error(void) { return last_error_cstr(); }

const char* tomo_version(void) { return "1.0.0"; }

}  // extern "C"
