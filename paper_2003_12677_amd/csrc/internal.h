// Internal declarations of libtomo: host builder, device operator state, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/tomo.h"

namespace tomo {

// ---------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------
tomo_status fail(tomo_status st, const char* fmt, ...);
void clear_error();

#define TOMO_HIP(call)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::tomo::fail(TOMO_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                          __FILE__, __LINE__);                                         \
  } while (0)

#define TOMO_TRY(expr)                 \
  do {                                 \
    tomo_status s_ = (expr);           \
    if (s_ != TOMO_OK) return s_;      \
  } while (0)

// ---------------------------------------------------------------------------------
// geometry and host-side matrices (float64)
// ---------------------------------------------------------------------------------
struct Geom {
  int n = 0, nt = 0, np = 0, G = 0, L = 0, kw = 3, h = 1, max_batch = 0;
  int jmax = 0;            // kept band |j| <= jmax = ceil(G/2) - 1
  int on = 0;              // image origin pixel n/2
  int cdet = 0;            // integer rotation-axis bin
  double beta = 0, center = 0;
  uint32_t values = TOMO_VALUES_F32;
  std::vector<double> theta;
};

struct HostCSR {
  int64_t rows = 0, cols = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  int64_t nnz() const { return (int64_t)col.size(); }
};

// Bin thresholds (nnz per row) for the adjoint SpMM over S's Cartesian rows.
struct BinParams {
  int short_max = 16;   // rows with <= short_max entries: one lane group per row
  int medium_max = 128; // rows with <= medium_max entries: one wavefront per row
  int chunk = 256;      // longer rows: split into chunks of <= chunk entries per block
};

struct HostBins {
  std::vector<int32_t> short_rows, medium_rows;
  std::vector<int32_t> long_rows;          // [n_long]
  std::vector<int32_t> long_chunk_ptr;     // [n_long + 1] into the chunk list
  std::vector<int32_t> chunk_beg, chunk_end;  // [n_chunks] entry ranges
};

tomo_status resolve_geometry(const tomo_geometry* in, Geom* g);
double kernel_value(double t, int W, double beta);
void build_sdag(const Geom& g, HostCSR* sdag);
void transpose_csr(const HostCSR& a, HostCSR* at);
void build_bins(const HostCSR& s, const BinParams& p, HostBins* bins);
void deapod_factors(const Geom& g, std::vector<double>* kd);
void filter_diagonal(const Geom& g, int filter, std::vector<double>* d);   // FFT-ordered k
uint16_t f32_to_bf16_rne(float f);

// ---------------------------------------------------------------------------------
// device state
// ---------------------------------------------------------------------------------
struct DevCSR {
  int64_t rows = 0, nnz = 0;
  int32_t* rowptr = nullptr;    // int32 row pointers (nnz < 2^31 is checked)
  int32_t* col = nullptr;
  void* val[3] = {nullptr, nullptr, nullptr};   // indexed by tomo_value_type
};

struct DevBins {
  int32_t* short_rows = nullptr;  int64_t n_short = 0;
  int32_t* medium_rows = nullptr; int64_t n_medium = 0;
  int32_t* long_rows = nullptr;   int64_t n_long = 0;
  int32_t* long_chunk_ptr = nullptr;
  int32_t* chunk_beg = nullptr;   int32_t* chunk_end = nullptr; int64_t n_chunks = 0;
};

struct FFTPlans {
  rocfft_plan fwd2 = nullptr, inv2 = nullptr, fwd1 = nullptr, inv1 = nullptr;
  rocfft_execution_info info = nullptr;
  void* work = nullptr;
  size_t work_bytes = 0;
};

struct SolverBuffers {
  int B = 0;
  float *p = nullptr, *s = nullptr, *d = nullptr;      // image-sized [B][n][n]
  float *r = nullptr, *q = nullptr, *rb = nullptr;     // sinogram-sized [B][nt][np]
  double* scal = nullptr;                              // per-slice scalars [16][B]
  double* partial = nullptr;                           // dot partial sums [B][kDotBlocks]
};

}  // namespace tomo

struct tomo_op {
  tomo::Geom g;
  tomo::BinParams binp;
  tomo::HostCSR sdag, s;          // float64 host copies (test export)
  tomo::HostBins hbins;
  std::vector<double> kd;         // separable deapodisation factors [n]
  int device = -1;
  uint32_t values = 0;
  int64_t cols_touched = 0, polar_nonempty = 0;
  // device
  tomo::DevCSR fwd, adj;
  tomo::DevBins bins;
  float* kd_dev = nullptr;        // [n]
  float* filt_dev[4] = {nullptr, nullptr, nullptr, nullptr};   // D per tomo_filter, [L]
  int cmax = 0;                   // complex channels the workspace holds
  float2* X = nullptr;            // [G*G][cmax]
  float2* Y = nullptr;            // [L*nt][cmax]
  float2* partials = nullptr;     // [n_chunks][cmax] long-row partial sums
  std::map<int, tomo::FFTPlans> plans;   // keyed by channel count C
  tomo::SolverBuffers sb;
};

namespace tomo {

constexpr int kDotBlocks = 256;   // blocks per slice in the FP64 reductions

// FFT plans for C complex channels (created on first use).
tomo_status get_plans(tomo_op* op, int C, FFTPlans** out);
void destroy_plans(tomo_op* op);
tomo_status fft_exec(rocfft_plan plan, FFTPlans* p, void* data, hipStream_t st);

// kernel launchers (all enqueue on `st`)
tomo_status launch_embed(const tomo_op* op, const float* x, float2* X, int B, hipStream_t st);
tomo_status launch_crop_sino(const tomo_op* op, const float2* Y, float* y, int B, float scale,
                             hipStream_t st);
tomo_status launch_pad_sino(const tomo_op* op, const float* y, float2* Y, int B, hipStream_t st);
tomo_status launch_crop_image(const tomo_op* op, const float2* X, float* x, int B, float scale,
                              hipStream_t st);
tomo_status launch_spmm_fwd(const tomo_op* op, const float2* X, float2* Y, int C, int vt,
                            hipStream_t st);
tomo_status launch_spmm_adj(const tomo_op* op, const float2* Y, float2* X, int C, int vt,
                            const float* dscale, hipStream_t st);

// composite operators on caller buffers
tomo_status apply_project(tomo_op* op, const float* x, float* y, int B, int vt, hipStream_t st);
tomo_status apply_backproject(tomo_op* op, const float* y, float* x, int B, int vt, int filter,
                              float extra_scale, hipStream_t st);

// solver
tomo_status run_solve(tomo_op* op, const float* b, float* x, int B, const tomo_solve_opts* o,
                      hipStream_t st);
void free_solver(tomo_op* op);

// elementwise / reduction launchers used by the solver
tomo_status launch_dot(const float* a, const float* b, int64_t len, int B, double* partial,
                       double* out, hipStream_t st);
tomo_status launch_lincomb(float* out, const float* a, const float* b, const double* ca,
                           const double* cb, double sa, double sb, int64_t len, int B,
                           hipStream_t st);
tomo_status launch_fill(float* out, float v, int64_t len, hipStream_t st);

}  // namespace tomo
