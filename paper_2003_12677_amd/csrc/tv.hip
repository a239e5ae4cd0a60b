// Smoothed isotropic total variation and its gradient for a stack of n x n images: the
// regularisation term of the model-based reconstruction problem (Sec. 2, Reg = total-variation
// norm).  Discretisation: forward differences with a zero difference past the last row and
// column; TV_eps(u) = sum over pixels of sqrt(D1u^2 + D2u^2 + eps); the gradient is D^T p with
// p = Du / sqrt(|Du|^2 + eps).
//
// One pass over the image computes both: a thread owns pixel i and rebuilds p at i, at the pixel
// above and at the pixel to the left (the three p values its gradient entry needs) from seven
// neighbouring samples that the L1/L2 caches serve after the first touch, so HBM sees one read of
// x and one write of the gradient.  Per-slice values are float64 sums in a fixed two-level order.

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "internal.h"

namespace tomo {
namespace {

constexpr int kTvBlock = 256;

// Reduction partials of tomo_tv_noalloc: one float64 per (slice, block), for the largest batch
// an operator accepts.  A file-scope device array (each GPU holds its own copy from the first use
// until the process ends), so that entry point allocates nothing.  Every call on one GPU shares
// it: calls that overlap on a GPU race.  Host code never passes `scratch` itself to a kernel (in
// host code the name is a host-side stand-in); it passes the device address looked up once per
// device by tv_scratch().
constexpr int kTvScratchDoubles = kMaxBatch * kDotBlocks;
__device__ __align__(256) double scratch[kTvScratchDoubles];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxScratchDevices] = {};

__device__ __forceinline__ double tv_wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double tv_block_sum(double v) {
  __shared__ double w[kTvBlock / 64];
  v = tv_wave_sum(v);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (w[0] + w[1]) + (w[2] + w[3]);
  return r;
}

// p = (d1, d2) / sqrt(d1^2 + d2^2 + eps) at pixel (i1, i2) of image u
__device__ __forceinline__ void tv_p(const float* __restrict__ u, int n, int i1, int i2, float eps,
                                     float& p1, float& p2, float& m) {
  const float c = u[(int64_t)i1 * n + i2];
  const float d1 = (i1 < n - 1) ? u[(int64_t)(i1 + 1) * n + i2] - c : 0.f;
  const float d2 = (i2 < n - 1) ? u[(int64_t)i1 * n + i2 + 1] - c : 0.f;
  m = sqrtf(d1 * d1 + d2 * d2 + eps);
  p1 = d1 / m;
  p2 = d2 / m;
}

template <bool GRAD, bool VALUE>
__global__ __launch_bounds__(kTvBlock) void k_tv(const float* __restrict__ x, int n, float eps,
                                                 float weight, float* __restrict__ grad,
                                                 double* __restrict__ partial) {
  const int s = blockIdx.y;
  const int npix = n * n;                 // 32-bit pixel indices (a 64-bit division per pixel is slow)
  const float* u = x + (int64_t)s * npix;
  double acc = 0.0;
  for (int i = blockIdx.x * kTvBlock + threadIdx.x; i < npix; i += gridDim.x * kTvBlock) {
    const int i1 = i / n, i2 = i - i1 * n;
    float p1, p2, m;
    tv_p(u, n, i1, i2, eps, p1, p2, m);
    if constexpr (VALUE) acc += (double)m;
    if constexpr (GRAD) {
      float g = -p1 - p2;
      if (i1 > 0) {
        float q1, q2, mq;
        tv_p(u, n, i1 - 1, i2, eps, q1, q2, mq);
        g += q1;
      }
      if (i2 > 0) {
        float q1, q2, mq;
        tv_p(u, n, i1, i2 - 1, eps, q1, q2, mq);
        g += q2;
      }
      grad[(int64_t)s * npix + i] = weight * g;
    }
  }
  if constexpr (VALUE) {
    const double t = tv_block_sum(acc);
    if (threadIdx.x == 0) partial[(int64_t)s * gridDim.x + blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kTvBlock) void k_tv_final(const double* __restrict__ partial,
                                                       int nblk, double weight,
                                                       double* __restrict__ out) {
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kTvBlock) acc += partial[(int64_t)s * nblk + i];
  const double t = tv_block_sum(acc);
  if (threadIdx.x == 0) out[s] = weight * t;
}

}  // namespace

namespace {

int tv_blocks(const tomo_op* op) {
  const int64_t npix = (int64_t)op->g.n * op->g.n;
  return (int)std::min<int64_t>(kDotBlocks, (npix + kTvBlock - 1) / kTvBlock);
}

// The TV kernels with the per-(slice, block) float64 partials in `partial` (>= B * nblk
// doubles; unused when value is NULL).  Every partial a call reads is written by the same call
// first, so the buffer needs no clearing.
tomo_status run_tv(const tomo_op* op, const float* x, int B, double eps, double weight, float* grad,
                   double* value, double* partial, hipStream_t st) {
  const int n = op->g.n;
  const int nblk = tv_blocks(op);
  const dim3 grid((unsigned)nblk, (unsigned)B);
  const float fe = (float)eps, fw = (float)weight;
  if (grad && value)
    hipLaunchKernelGGL((k_tv<true, true>), grid, dim3(kTvBlock), 0, st, x, n, fe, fw, grad,
                       partial);
  else if (grad)
    hipLaunchKernelGGL((k_tv<true, false>), grid, dim3(kTvBlock), 0, st, x, n, fe, fw, grad,
                       nullptr);
  else
    hipLaunchKernelGGL((k_tv<false, true>), grid, dim3(kTvBlock), 0, st, x, n, fe, fw, nullptr,
                       partial);
  TOMO_HIP(hipGetLastError());
  if (value) {
    hipLaunchKernelGGL(k_tv_final, dim3((unsigned)B), dim3(kTvBlock), 0, st, partial, nblk,
                       weight, value);
    TOMO_HIP(hipGetLastError());
  }
  return TOMO_OK;
}

// Device address of `scratch` on `device` (which must be current), looked up on first use.
tomo_status tv_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxScratchDevices)
    return fail(TOMO_EINVAL, "device %d outside the %d devices the TV scratch array serves", device,
                kMaxScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TOMO_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                  hipGetErrorString(e));
    g_scratch_ptr[device] = (double*)p;
  }
  *out = g_scratch_ptr[device];
  return TOMO_OK;
}

}  // namespace

tomo_status launch_tv(tomo_op* op, const float* x, int B, double eps, double weight, float* grad,
                      double* value, hipStream_t st) {
  if (value && !op->tv_partial) {
    const size_t bytes = (size_t)op->g.max_batch * kDotBlocks * sizeof(double);
    if (hipMalloc(&op->tv_partial, bytes) != hipSuccess) {
      op->tv_partial = nullptr;
      return fail(TOMO_ENOMEM, "TV reduction buffer of %zu bytes", bytes);
    }
  }
  return run_tv(op, x, B, eps, weight, grad, value, op->tv_partial, st);
}

tomo_status launch_tv_noalloc(const tomo_op* op, const float* x, int B, double eps, double weight,
                              float* grad, double* value, hipStream_t st) {
  const int64_t need = (int64_t)B * tv_blocks(op);
  if (need > kTvScratchDoubles)
    return fail(TOMO_EINVAL, "batch %d needs %lld TV partials, beyond the scratch array's %d", B,
                (long long)need, kTvScratchDoubles);
  double* partial = nullptr;
  if (value) {
    const tomo_status s = tv_scratch(op->device, &partial);
    if (s != TOMO_OK) return s;
  }
  return run_tv(op, x, B, eps, weight, grad, value, partial, st);
}

void free_tv(tomo_op* op) {
  if (op->tv_partial) (void)hipFree(op->tv_partial);
  op->tv_partial = nullptr;
}

}  // namespace tomo
