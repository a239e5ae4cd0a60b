// rocFFT plans for the two Fourier steps of Eq. (2), on the channel-slowest buffers, so every
// transform is a contiguous batch:
//   2D: Xs[C][G][G] complex64, C transforms of G x G (the Cartesian grid F2D and its adjoint);
//   1D: Ys[C][nt][L] complex64, C*nt transforms of length L (F1D along each radial line).
// Both are in place and unnormalised (forward e^{-2 pi i}, backward e^{+2 pi i}); the 1/L of
// the detector-side inverse is applied by the crop kernels.  Plans are created on first use for
// each channel count and kept until the operator is destroyed (Sec. 3.1: plans cached until
// the reconstruction restarts).

#include <mutex>

#include "internal.h"

namespace tomo {

namespace {
std::once_flag g_fft_once;
rocfft_status g_fft_setup = rocfft_status_success;

tomo_status make_plan(rocfft_plan* plan, rocfft_transform_type dir, size_t dim, const size_t* lengths,
                      const size_t* strides, size_t distance, size_t batch) {
  rocfft_plan_description desc = nullptr;
  if (rocfft_plan_description_create(&desc) != rocfft_status_success)
    return fail(TOMO_EFFT, "rocfft_plan_description_create failed");
  rocfft_status s = rocfft_plan_description_set_data_layout(
      desc, rocfft_array_type_complex_interleaved, rocfft_array_type_complex_interleaved, nullptr,
      nullptr, dim, strides, distance, dim, strides, distance);
  if (s == rocfft_status_success)
    s = rocfft_plan_create(plan, rocfft_placement_inplace, dir, rocfft_precision_single, dim,
                           lengths, batch, desc);
  rocfft_plan_description_destroy(desc);
  if (s != rocfft_status_success) return fail(TOMO_EFFT, "rocfft_plan_create failed (status %d)", (int)s);
  return TOMO_OK;
}
}  // namespace

tomo_status get_plans(tomo_op* op, int C, FFTPlans** out) {
  auto it = op->plans.find(C);
  if (it != op->plans.end()) {
    *out = &it->second;
    return TOMO_OK;
  }
  std::call_once(g_fft_once, [] { g_fft_setup = rocfft_setup(); });
  if (g_fft_setup != rocfft_status_success) return fail(TOMO_EFFT, "rocfft_setup failed");
  const Geom& g = op->g;
  FFTPlans p;
  const size_t len2[2] = {(size_t)g.G, (size_t)g.G};           // fastest dimension first
  const size_t str2[2] = {1, (size_t)g.G};
  const size_t dist2 = (size_t)g.G * g.G;
  const size_t len1[1] = {(size_t)g.L};
  const size_t str1[1] = {1};
  const size_t dist1 = (size_t)g.L;
  const size_t batch1 = (size_t)g.nt * C;
  tomo_status st = make_plan(&p.fwd2, rocfft_transform_type_complex_forward, 2, len2, str2, dist2, C);
  if (st == TOMO_OK)
    st = make_plan(&p.inv2, rocfft_transform_type_complex_inverse, 2, len2, str2, dist2, C);
  if (st == TOMO_OK)
    st = make_plan(&p.fwd1, rocfft_transform_type_complex_forward, 1, len1, str1, dist1, batch1);
  if (st == TOMO_OK)
    st = make_plan(&p.inv1, rocfft_transform_type_complex_inverse, 1, len1, str1, dist1, batch1);
  if (st == TOMO_OK) {
    size_t w = 0;
    for (rocfft_plan pl : {p.fwd2, p.inv2, p.fwd1, p.inv1}) {
      size_t b = 0;
      rocfft_plan_get_work_buffer_size(pl, &b);
      w = std::max(w, b);
    }
    if (w > 0 && hipMalloc(&p.work, w) != hipSuccess) st = fail(TOMO_ENOMEM, "FFT work buffer (%zu B)", w);
    p.work_bytes = w;
  }
  if (st == TOMO_OK && rocfft_execution_info_create(&p.info) != rocfft_status_success)
    st = fail(TOMO_EFFT, "rocfft_execution_info_create failed");
  if (st == TOMO_OK && p.work &&
      rocfft_execution_info_set_work_buffer(p.info, p.work, p.work_bytes) != rocfft_status_success)
    st = fail(TOMO_EFFT, "rocfft_execution_info_set_work_buffer failed");
  if (st != TOMO_OK) {
    for (rocfft_plan pl : {p.fwd2, p.inv2, p.fwd1, p.inv1})
      if (pl) rocfft_plan_destroy(pl);
    if (p.info) rocfft_execution_info_destroy(p.info);
    if (p.work) (void)hipFree(p.work);
    return st;
  }
  auto res = op->plans.emplace(C, p);
  *out = &res.first->second;
  return TOMO_OK;
}

tomo_status fft_exec(rocfft_plan plan, FFTPlans* p, void* data, hipStream_t st) {
  if (rocfft_execution_info_set_stream(p->info, st) != rocfft_status_success)
    return fail(TOMO_EFFT, "rocfft_execution_info_set_stream failed");
  void* buf[1] = {data};
  const rocfft_status s = rocfft_execute(plan, buf, nullptr, p->info);
  if (s != rocfft_status_success) return fail(TOMO_EFFT, "rocfft_execute failed (status %d)", (int)s);
  return TOMO_OK;
}

void destroy_plans(tomo_op* op) {
  for (auto& kv : op->plans) {
    FFTPlans& p = kv.second;
    for (rocfft_plan pl : {p.fwd2, p.inv2, p.fwd1, p.inv1})
      if (pl) rocfft_plan_destroy(pl);
    if (p.info) rocfft_execution_info_destroy(p.info);
    if (p.work) (void)hipFree(p.work);
  }
  op->plans.clear();
}

}  // namespace tomo
