// Iterative reconstruction on the device (Sec. 2.1 least squares; Sec. 3.1 lists CGLS and SIRT
// with Hamming preconditioning and Barzilai-Borwein steps).  Slices are independent, so every
// scalar (step lengths, inner products) is per slice: float64 reductions over each slice with a
// fixed two-level order (bitwise reproducible), stored in device arrays and read by the update
// kernels, so nothing returns to the host inside the loop.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace tomo {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double w[4];
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) w[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (w[0] + w[1]) + (w[2] + w[3]);
  return r;
}

// partial[s][j] = sum over the j-th strided share of slice s of a*b, in float64; four strided
// elements per step with independent accumulators keep four loads in flight per thread, and a
// self product (SELF) loads each element once
template <bool SELF>
__global__ __launch_bounds__(256) void k_dot_partial(const float* __restrict__ a,
                                                     const float* __restrict__ b, int64_t len,
                                                     double* __restrict__ partial) {
  const int s = blockIdx.y;
  const float* pa = a + (int64_t)s * len;
  const float* pb = SELF ? pa : b + (int64_t)s * len;
  const int64_t stride = (int64_t)gridDim.x * 256;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < len; i += 4 * stride) {
    float va[4], vb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) va[u] = pa[i + u * stride];
    if constexpr (!SELF) {
#pragma unroll
      for (int u = 0; u < 4; ++u) vb[u] = pb[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += (double)va[u] * (double)(SELF ? va[u] : vb[u]);
  }
  for (; i < len; i += stride) acc[0] += (double)pa[i] * (double)pb[i];
  const double t = block_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
  if (threadIdx.x == 0) partial[(int64_t)s * gridDim.x + blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ partial, int nblk,
                                                   double* __restrict__ out) {
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) acc += partial[(int64_t)s * nblk + i];
  const double t = block_sum(acc);
  if (threadIdx.x == 0) out[s] = t;
}

// Fused conjugate-gradient vector steps (each saves a pass over an image-sized vector):
//   k_cg_step:     x += alpha[s] p;  p = r + beta[s] p       (the deferred solution update)
//   k_axpy_dot:    r -= alpha[s] q;  partial sums of |r|^2  (residual update and its norm)
__global__ __launch_bounds__(256) void k_cg_step(float* __restrict__ x, float* __restrict__ p,
                                                 const float* __restrict__ r,
                                                 const double* __restrict__ alpha,
                                                 const double* __restrict__ beta, int64_t len) {
  const int s = blockIdx.y;
  const float fa = (float)alpha[s], fb = (float)beta[s];
  const int64_t base = (int64_t)s * len;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) {
    const float pv = p[base + i];
    float xv = 1.0f * x[base + i];
    xv += fa * pv;
    x[base + i] = xv;
    float nv = 1.0f * r[base + i];
    nv += fb * pv;
    p[base + i] = nv;
  }
}

__global__ __launch_bounds__(256) void k_axpy_dot(float* __restrict__ r, const float* __restrict__ q,
                                                  const double* __restrict__ alpha, int64_t len,
                                                  double* __restrict__ partial) {
  const int s = blockIdx.y;
  const float fa = -(float)alpha[s];
  float* pr = r + (int64_t)s * len;
  const float* pq = q + (int64_t)s * len;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) {
    float v = 1.0f * pr[i];
    v += fa * pq[i];
    pr[i] = v;
    acc += (double)v * (double)v;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partial[(int64_t)s * gridDim.x + blockIdx.x] = t;
}

//   k_dot2_partial: partial sums of a.a and a.b in one pass (the two SIRT-BB step inner products)
//   k_sirt_update:  x -= alpha[s] g;  g -= alpha[s] h
__global__ __launch_bounds__(256) void k_dot2_partial(const float* __restrict__ a,
                                                      const float* __restrict__ b, int64_t len,
                                                      double* __restrict__ partial_aa,
                                                      double* __restrict__ partial_ab) {
  const int s = blockIdx.y;
  const float* pa = a + (int64_t)s * len;
  const float* pb = b + (int64_t)s * len;
  double aa = 0.0, ab = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) {
    const double va = (double)pa[i];
    aa += va * va;
    ab += va * (double)pb[i];
  }
  const double taa = block_sum(aa);
  __syncthreads();   // block_sum's shared scratch is reused
  const double tab = block_sum(ab);
  if (threadIdx.x == 0) {
    partial_aa[(int64_t)s * gridDim.x + blockIdx.x] = taa;
    partial_ab[(int64_t)s * gridDim.x + blockIdx.x] = tab;
  }
}

__global__ __launch_bounds__(256) void k_sirt_update(float* __restrict__ x, float* __restrict__ g,
                                                     const float* __restrict__ h,
                                                     const double* __restrict__ alpha, int64_t len) {
  const int s = blockIdx.y;
  const float fa = -(float)alpha[s];
  const int64_t base = (int64_t)s * len;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) {
    const float gv = g[base + i];
    float xv = 1.0f * x[base + i];
    xv += fa * gv;
    x[base + i] = xv;
    float nv = 1.0f * gv;
    nv += fa * h[base + i];
    g[base + i] = nv;
  }
}

// out = sa*ca[s]*a + sb*cb[s]*b per slice (null ca / cb mean 1; null b means no second term);
// out may be a or b (element-wise in place)
__global__ __launch_bounds__(256) void k_lincomb(float* out, const float* a,
                                                 const float* b, const double* __restrict__ ca,
                                                 const double* __restrict__ cb, double sa, double sb,
                                                 int64_t len) {
  const int s = blockIdx.y;
  const float fa = (float)(sa * (ca ? ca[s] : 1.0));
  const float fb = (float)(sb * (cb ? cb[s] : 1.0));
  const int64_t base = (int64_t)s * len;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) {
    float v = fa * a[base + i];
    if (b) v += fb * b[base + i];
    out[base + i] = v;
  }
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ out, float v, int64_t len) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256)
    out[i] = v;
}

// out[s] = den[s] > 0 ? num[s] / den[s] : 0
__global__ void k_ratio(const double* num, const double* den, double* out, int B) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < B) out[s] = den[s] > 0.0 ? num[s] / den[s] : 0.0;
}

// Barzilai-Borwein step (BB1) for the gradient recurrence g_{k+1} = g_k - alpha_k h_k with
// h_k = A^T_D A g_k:  s = -alpha_{k-1} g_{k-1}, y = -alpha_{k-1} h_{k-1} give
// alpha_k = <s,s>/<s,y> = <g_{k-1},g_{k-1}> / <g_{k-1},h_{k-1}>; alpha_0 is the exact line search
// <g_0,g_0>/<g_0,h_0>.  A non-positive <s,y> keeps the previous step.
// state layout per slice: [0] num_k, [1] den_k, [2] num_{k-1}, [3] den_{k-1}, [4] alpha
__global__ void k_sirt_step(double* num, double* den, double* pnum, double* pden, double* alpha,
                            int B, int first) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  if (first) {
    alpha[s] = den[s] > 0.0 ? num[s] / den[s] : 0.0;
  } else if (pden[s] > 0.0 && alpha[s] != 0.0) {
    alpha[s] = pnum[s] / pden[s];
  }
  pnum[s] = num[s];
  pden[s] = den[s];
}

__global__ void k_sqrt(const double* in, double* out, int B) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < B) out[s] = sqrt(in[s] > 0.0 ? in[s] : 0.0);
}

inline unsigned grid_for(int64_t len) {
  int64_t b = (len + 255) / 256;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// scalar slots in SolverBuffers::scal ([16][B] doubles)
enum { kGamma0 = 0, kGamma1, kDelta, kAlpha, kBeta, kNum, kDen, kPNum, kPDen, kTmp, kSlots };

}  // namespace

tomo_status launch_dot(const float* a, const float* b, int64_t len, int B, double* partial,
                       double* out, hipStream_t st) {
  if (a == b)
    hipLaunchKernelGGL(k_dot_partial<true>, dim3(kDotBlocks, B), dim3(256), 0, st, a, b, len, partial);
  else
    hipLaunchKernelGGL(k_dot_partial<false>, dim3(kDotBlocks, B), dim3(256), 0, st, a, b, len, partial);
  TOMO_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_dot_final, dim3(B), dim3(256), 0, st, partial, kDotBlocks, out);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_lincomb(float* out, const float* a, const float* b, const double* ca,
                           const double* cb, double sa, double sb, int64_t len, int B,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb, dim3(grid_for(len), B), dim3(256), 0, st, out, a, b, ca, cb, sa, sb,
                     len);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

// ---- split-Bregman TV: forward differences D (zero past the last row / column) and D^T -----
// (D1 u)(i1,i2) = u(i1+1,i2) - u(i1,i2) for i1 < n-1, else 0; (D2 u) likewise along i2.
// (D^T p)(i) = -p1(i) - p2(i) + p1(i1-1,i2) + p2(i1,i2-1), p1 taken as 0 on the last row and
// p2 on the last column.

__device__ __forceinline__ float tv_dt(const float* __restrict__ p1, const float* __restrict__ p2,
                                       int n, int i1, int i2, int64_t i) {
  const float a = (i1 < n - 1) ? p1[i] : 0.f;
  const float b = (i2 < n - 1) ? p2[i] : 0.f;
  float v = -a - b;
  if (i1 > 0) v += p1[i - n];          // p1(i1-1, i2); i1-1 < n-1 always
  if (i2 > 0) v += p2[i - 1];          // p2(i1, i2-1)
  return v;
}

// The split-Bregman kernels walk one n x n slice per blockIdx.y with 32-bit pixel indices (a
// 64-bit remainder per element made them several times slower than their memory traffic).
#define TOMO_SB_PIXELS                                                                         \
  const int64_t base_ = (int64_t)blockIdx.y * n * n;                                           \
  for (int pix = blockIdx.x * 256 + threadIdx.x; pix < n * n; pix += gridDim.x * 256) {        \
    const int i1 = pix / n, i2 = pix - i1 * n;                                                 \
    const int64_t i = base_ + pix;

// rhs = mu ATf + lam D^T (d - b), per slice of n x n (tv buffers: d1, d2, b1, b2)
__global__ __launch_bounds__(256) void k_sb_rhs(const float* __restrict__ ATf,
                                                const float* __restrict__ d1,
                                                const float* __restrict__ d2,
                                                const float* __restrict__ b1,
                                                const float* __restrict__ b2,
                                                float* __restrict__ rhs, float mu, float lam, int n) {
  TOMO_SB_PIXELS
    // D^T of (d - b): evaluate the two fields at the three points the operator touches
    const float a = (i1 < n - 1) ? d1[i] - b1[i] : 0.f;
    const float c = (i2 < n - 1) ? d2[i] - b2[i] : 0.f;
    float v = -a - c;
    if (i1 > 0) v += d1[i - n] - b1[i - n];
    if (i2 > 0) v += d2[i - 1] - b2[i - 1];
    rhs[i] = mu * ATf[i] + lam * v;
  }
}

// q = mu q + lam D^T D p   (q holds A^T A p on entry)
// With partial set, each block also leaves the float64 sum of p . q (the new q) over its pixels
// in partial[slice * gridDim.x + block].
__global__ __launch_bounds__(256) void k_sb_addlap(const float* __restrict__ p, float* __restrict__ q,
                                                   float mu, float lam, int n,
                                                   double* __restrict__ partial) {
  double acc = 0.0;
  TOMO_SB_PIXELS
    const float c = p[i];
    // D p at (i1, i2), (i1-1, i2) [component 1] and (i1, i2-1) [component 2]
    const float g1 = (i1 < n - 1) ? p[i + n] - c : 0.f;
    const float g2 = (i2 < n - 1) ? p[i + 1] - c : 0.f;
    float v = -g1 - g2;
    if (i1 > 0) v += c - p[i - n];
    if (i2 > 0) v += c - p[i - 1];
    const float o = mu * q[i] + lam * v;
    q[i] = o;
    acc += (double)c * (double)o;
  }
  if (partial) {
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
  }
}

// One quad (4 pixels of a row) of k_sb_addlap4.  Every neighbour load is issued unconditionally,
// with its offset clamped at the slice's edges so that it reads the centre pixel there (whose
// difference is then zero, as the one-pixel form's zero differences past the edges).
struct Quad {
  float4 c, qq, up, dn;
  float lf, rt;
};

__device__ __forceinline__ void quad_load(const float* __restrict__ p, const float* __restrict__ q,
                                          int64_t base, int t, int n, Quad& d) {
  const int pix = 4 * t;
  const int i1 = pix / n, i2 = pix - i1 * n;
  const int64_t i = base + pix;
  d.c = *reinterpret_cast<const float4*>(p + i);
  d.qq = *reinterpret_cast<const float4*>(q + i);
  d.dn = *reinterpret_cast<const float4*>(p + i + ((i1 < n - 1) ? n : 0));
  d.up = *reinterpret_cast<const float4*>(p + i - ((i1 > 0) ? n : 0));
  d.lf = p[i - ((i2 > 0) ? 1 : 0)];
  d.rt = p[i + ((i2 + 4 < n) ? 4 : 3)];
}

__device__ __forceinline__ void quad_store(float* __restrict__ q, int64_t base, int t,
                                           const Quad& d, float mu, float lam, double& acc) {
  // -(D1 p)(i) + (D1 p)(i - row) = (up - c) + (dn - c) with zero differences past the edges;
  // the same along the row with the left / right neighbours
  const float cv[4] = {d.c.x, d.c.y, d.c.z, d.c.w};
  const float uv[4] = {d.up.x, d.up.y, d.up.z, d.up.w};
  const float dv[4] = {d.dn.x, d.dn.y, d.dn.z, d.dn.w};
  const float lv[4] = {d.lf, d.c.x, d.c.y, d.c.z};
  const float rv[4] = {d.c.y, d.c.z, d.c.w, d.rt};
  const float qv[4] = {d.qq.x, d.qq.y, d.qq.z, d.qq.w};
  float o[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float v = -(dv[k] - cv[k]) - (rv[k] - cv[k]);   // the one-pixel form's order of operations
    v += cv[k] - uv[k];
    v += cv[k] - lv[k];
    o[k] = mu * qv[k] + lam * v;
    acc += (double)cv[k] * (double)o[k];
  }
  *reinterpret_cast<float4*>(q + base + 4 * t) = make_float4(o[0], o[1], o[2], o[3]);
}

// The same for n % 4 == 0, four pixels of one row per quad: 16-byte loads of p and q at the
// pixels and at the rows above and below, the left and right neighbours as single loads (the
// one-pixel form issued five 4-byte loads and a division per pixel and ran at ~2.3 TB/s).  A
// thread issues the loads of four quads before computing any of them.
__global__ __launch_bounds__(256) void k_sb_addlap4(const float* __restrict__ p, float* __restrict__ q,
                                                    float mu, float lam, int n,
                                                    double* __restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.y * n * n;
  const int quads = n * n / 4;
  const int stride = gridDim.x * 256;
  double acc = 0.0;
  int t = blockIdx.x * 256 + threadIdx.x;
  for (; t + 3 * stride < quads; t += 4 * stride) {
    Quad d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) quad_load(p, q, base, t + u * stride, n, d[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) quad_store(q, base, t + u * stride, d[u], mu, lam, acc);
  }
  for (; t < quads; t += stride) {
    Quad d;
    quad_load(p, q, base, t, n, d);
    quad_store(q, base, t, d, mu, lam, acc);
  }
  if (partial) {
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = b;
  }
}

// s = D u + b; d = shrink(s, 1/lam) (isotropic); b = s - d
__global__ __launch_bounds__(256) void k_sb_shrink(const float* __restrict__ u, float* __restrict__ d1,
                                                   float* __restrict__ d2, float* __restrict__ b1,
                                                   float* __restrict__ b2, float thr, int n) {
  TOMO_SB_PIXELS
    const float c = u[i];
    const float s1 = ((i1 < n - 1) ? u[i + n] - c : 0.f) + b1[i];
    const float s2 = ((i2 < n - 1) ? u[i + 1] - c : 0.f) + b2[i];
    const float mag = sqrtf(s1 * s1 + s2 * s2);
    const float sc = mag > thr ? (mag - thr) / mag : 0.f;
    const float e1 = sc * s1, e2 = sc * s2;
    d1[i] = e1;
    d2[i] = e2;
    b1[i] = s1 - e1;
    b2[i] = s2 - e2;
  }
}

// out[i] = a value in [-1, 1) from a 32-bit integer hash of (i, seed): timing inputs
__global__ __launch_bounds__(256) void k_fill_hash(float* __restrict__ out, int64_t len,
                                                   uint32_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) {
    uint32_t h = (uint32_t)i * 0x9E3779B9u ^ (uint32_t)(i >> 32) ^ seed;
    h ^= h >> 16; h *= 0x7FEB352Du; h ^= h >> 15; h *= 0x846CA68Bu; h ^= h >> 16;
    out[i] = (float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f;
  }
}

tomo_status launch_fill_hash(float* out, int64_t len, uint32_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_hash, dim3(grid_for(len)), dim3(256), 0, st, out, len, seed);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

tomo_status launch_fill(float* out, float v, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(len)), dim3(256), 0, st, out, v, len);
  TOMO_HIP(hipGetLastError());
  return TOMO_OK;
}

void free_solver(tomo_op* op) {
  SolverBuffers& b = op->sb;
  for (float** p : {&b.p, &b.s, &b.d, &b.t, &b.r, &b.q, &b.rb, &b.tvb}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  if (b.scal) (void)hipFree(b.scal);
  if (b.partial) (void)hipFree(b.partial);
  if (b.norm_partial) (void)hipFree(b.norm_partial);
  b.scal = b.partial = b.norm_partial = nullptr;
  b.norm_blocks = 0;
  b.B = 0;
}

namespace {

tomo_status ensure_solver(tomo_op* op) {
  SolverBuffers& b = op->sb;
  if (b.B) return TOMO_OK;
  const Geom& g = op->g;
  const size_t B = (size_t)g.max_batch;
  const size_t img = B * g.n * g.n * sizeof(float);
  const size_t sino = B * g.nt * g.np * sizeof(float);
  // output-norm partials of either inverse transform, whichever tuning is set later
  const int64_t norm_blocks = std::max<int64_t>(
      1, std::max(det_inverse_blocks_per_channel(op), grid_inverse_blocks_per_channel(op)));
  struct Req { void** p; size_t bytes; } req[] = {
      {(void**)&b.p, img},  {(void**)&b.s, img},  {(void**)&b.d, img},  {(void**)&b.t, img},
      {(void**)&b.tvb, 6 * img},
      {(void**)&b.r, sino}, {(void**)&b.q, sino}, {(void**)&b.rb, sino},
      {(void**)&b.scal, kSlots * B * sizeof(double)},
      {(void**)&b.partial, 2 * B * kDotBlocks * sizeof(double)},     // two reductions at once
      {(void**)&b.norm_partial, B * (size_t)norm_blocks * sizeof(double)}};
  for (auto& r : req) {
    if (hipMalloc(r.p, r.bytes) != hipSuccess) {
      *r.p = nullptr;
      free_solver(op);
      return fail(TOMO_ENOMEM, "solver buffer of %zu bytes", r.bytes);
    }
  }
  b.B = (int)B;
  b.norm_blocks = norm_blocks;
  return TOMO_OK;
}

struct Ctx {
  tomo_op* op;
  int B;
  hipStream_t st;
  int64_t img, sino;
  double* sc(int slot) const { return op->sb.scal + (int64_t)slot * op->g.max_batch; }
  tomo_status dot(const float* a, const float* b, int64_t len, int slot) const {
    return launch_dot(a, b, len, B, op->sb.partial, sc(slot), st);
  }
  // with the deferred step  xs += alpha p; p = s + beta p  (this iteration's alpha and beta
  // slots) fused into the projection's first kernel when it can be, else run on its own first:
  // y = A_vt p and slot = |y|^2
  tomo_status step_project_norm(float* xs, float* p, const float* s, float* y, int vt,
                                int slot) const {
    if (!project_cg_supported(op)) {
      TOMO_TRY(cg_step(xs, p, s, img));
      return project_norm(p, y, vt, slot);
    }
    const CgStep cg{xs, s, sc(kAlpha), sc(kBeta)};
    const int64_t nb = project_sumsq_blocks(op);
    if (nb == 0 || nb > op->sb.norm_blocks) {
      TOMO_TRY(apply_project_cg(op, p, cg, y, B, vt, st));
      return dot(y, y, sino, slot);
    }
    TOMO_TRY(apply_project_cg(op, p, cg, y, B, vt, st, op->sb.norm_partial));
    hipLaunchKernelGGL(k_dot_final, dim3(B), dim3(256), 0, st, op->sb.norm_partial, (int)nb, sc(slot));
    TOMO_HIP(hipGetLastError());
    return TOMO_OK;
  }
  // q = A_vt^T A_vt p through the normal-operator stencil and slot = p . q, the products summed
  // by the last kernel as it writes q; with xs, the deferred step  xs += alpha p; p = s + beta p
  // first, fused into the first kernel.  Each part falls back to its own pass where the
  // hand-written transforms are off.
  tomo_status normal_dot(float* xs, float* p, const float* s, float* q, int vt, int slot) const {
    const bool fuse_step = xs && project_cg_supported(op);
    if (xs && !fuse_step) TOMO_TRY(cg_step(xs, p, s, img));
    const CgStep cg{xs, s, sc(kAlpha), sc(kBeta)};
    const int64_t nb = backproject_sumsq_blocks(op);
    if (nb == 0 || nb > op->sb.norm_blocks) {
      TOMO_TRY(apply_normal(op, p, q, B, vt, TOMO_FILTER_NONE, st, fuse_step ? &cg : nullptr));
      return dot(p, q, img, slot);
    }
    TOMO_TRY(apply_normal(op, p, q, B, vt, TOMO_FILTER_NONE, st, fuse_step ? &cg : nullptr,
                          op->sb.norm_partial, p));
    hipLaunchKernelGGL(k_dot_final, dim3(B), dim3(256), 0, st, op->sb.norm_partial, (int)nb, sc(slot));
    TOMO_HIP(hipGetLastError());
    return TOMO_OK;
  }
  // y = A_vt x and slot = |y|^2, the squares summed by the projection's last kernel as it writes
  // y when it can (no separate pass over y), else by a dot product
  tomo_status project_norm(const float* x, float* y, int vt, int slot) const {
    const int64_t nb = project_sumsq_blocks(op);
    if (nb == 0 || nb > op->sb.norm_blocks) {
      TOMO_TRY(apply_project(op, x, y, B, vt, st));
      return dot(y, y, sino, slot);
    }
    TOMO_TRY(apply_project(op, x, y, B, vt, st, op->sb.norm_partial));
    hipLaunchKernelGGL(k_dot_final, dim3(B), dim3(256), 0, st, op->sb.norm_partial, (int)nb, sc(slot));
    TOMO_HIP(hipGetLastError());
    return TOMO_OK;
  }
  // r -= alpha q, then x = A_vt^T r and slot = |x|^2, the update fused into the adjoint front
  // when it can be
  tomo_status residual_backproject_norm(float* r, const float* q, float* x, int vt, int slot) const {
    if (!backproject_residual_supported(op)) {
      TOMO_TRY(lin(r, r, q, nullptr, sc(kAlpha), 1.0, -1.0, sino));
      return backproject_norm(r, x, vt, slot);
    }
    const int64_t nb = backproject_sumsq_blocks(op);
    if (nb == 0 || nb > op->sb.norm_blocks) {
      TOMO_TRY(apply_backproject_residual(op, r, q, sc(kAlpha), x, B, vt, st));
      return dot(x, x, img, slot);
    }
    TOMO_TRY(apply_backproject_residual(op, r, q, sc(kAlpha), x, B, vt, st, op->sb.norm_partial));
    hipLaunchKernelGGL(k_dot_final, dim3(B), dim3(256), 0, st, op->sb.norm_partial, (int)nb, sc(slot));
    TOMO_HIP(hipGetLastError());
    return TOMO_OK;
  }
  // x = A_vt^T y and slot = |x|^2, likewise
  tomo_status backproject_norm(const float* y, float* x, int vt, int slot) const {
    const int64_t nb = backproject_sumsq_blocks(op);
    if (nb == 0 || nb > op->sb.norm_blocks) {
      TOMO_TRY(apply_backproject(op, y, x, B, vt, TOMO_FILTER_NONE, 1.0f, st));
      return dot(x, x, img, slot);
    }
    TOMO_TRY(apply_backproject(op, y, x, B, vt, TOMO_FILTER_NONE, 1.0f, st, op->sb.norm_partial));
    hipLaunchKernelGGL(k_dot_final, dim3(B), dim3(256), 0, st, op->sb.norm_partial, (int)nb, sc(slot));
    TOMO_HIP(hipGetLastError());
    return TOMO_OK;
  }
  tomo_status lin(float* out, const float* a, const float* b, const double* ca, const double* cb,
                  double sa, double sb, int64_t len) const {
    return launch_lincomb(out, a, b, ca, cb, sa, sb, len, B, st);
  }
  // x += alpha p; p = r + beta p   (alpha, beta: this iteration's slots)
  tomo_status cg_step(float* x, float* p, const float* r, int64_t len) const {
    hipLaunchKernelGGL(k_cg_step, dim3(grid_for(len), B), dim3(256), 0, st, x, p, r, sc(kAlpha),
                       sc(kBeta), len);
    TOMO_HIP(hipGetLastError());
    return TOMO_OK;
  }
  // slot_aa = a.a, slot_ab = a.b in one pass
  tomo_status dot2(const float* a, const float* b, int64_t len, int slot_aa, int slot_ab) const {
    double* p2 = op->sb.partial + (int64_t)B * kDotBlocks;
    hipLaunchKernelGGL(k_dot2_partial, dim3(kDotBlocks, B), dim3(256), 0, st, a, b, len,
                       op->sb.partial, p2);
    TOMO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_dot_final, dim3(B), dim3(256), 0, st, op->sb.partial, kDotBlocks, sc(slot_aa));
    TOMO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_dot_final, dim3(B), dim3(256), 0, st, p2, kDotBlocks, sc(slot_ab));
    TOMO_HIP(hipGetLastError());
    return TOMO_OK;
  }
  // r -= alpha q; slot = |r|^2
  tomo_status axpy_dot(float* r, const float* q, int64_t len, int slot) const {
    hipLaunchKernelGGL(k_axpy_dot, dim3(kDotBlocks, B), dim3(256), 0, st, r, q, sc(kAlpha), len,
                       op->sb.partial);
    TOMO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_dot_final, dim3(B), dim3(256), 0, st, op->sb.partial, kDotBlocks, sc(slot));
    TOMO_HIP(hipGetLastError());
    return TOMO_OK;
  }
};

// CGLS on A_vt from x (zero, or x's contents when use_x0) with rhs b; x is updated in place.
tomo_status cgls(const Ctx& c, const float* b, float* x, int vt, int iters, bool use_x0) {
  SolverBuffers& w = c.op->sb;
  if (use_x0) {
    TOMO_TRY(apply_project(c.op, x, w.q, c.B, vt, c.st));
    TOMO_TRY(c.lin(w.r, b, w.q, nullptr, nullptr, 1.0, -1.0, c.sino));       // r = b - A x
  } else {
    TOMO_TRY(launch_fill(x, 0.f, c.img * c.B, c.st));
    TOMO_TRY(c.lin(w.r, b, nullptr, nullptr, nullptr, 1.0, 0.0, c.sino));    // r = b
  }
  int cur = kGamma0, nxt = kGamma1;
  TOMO_TRY(c.backproject_norm(w.r, w.s, vt, cur));          // s = A^T r; gamma = |s|^2
  TOMO_TRY(c.lin(w.p, w.s, nullptr, nullptr, nullptr, 1.0, 0.0, c.img));     // p = s
  for (int it = 0; it < iters; ++it) {
    if (it == 0) {
      TOMO_TRY(c.project_norm(w.p, w.q, vt, kDelta));       // q = A p; delta = |q|^2
    } else {
      // the previous iteration's x += alpha p; p = s + beta p, then q = A p; delta = |q|^2
      TOMO_TRY(c.step_project_norm(x, w.p, w.s, w.q, vt, kDelta));
    }
    hipLaunchKernelGGL(k_ratio, dim3(1), dim3(256), 0, c.st, c.sc(cur), c.sc(kDelta), c.sc(kAlpha), c.B);
    TOMO_HIP(hipGetLastError());
    // r -= alpha q; s = A^T r; gamma' = |s|^2
    TOMO_TRY(c.residual_backproject_norm(w.r, w.q, w.s, vt, nxt));
    hipLaunchKernelGGL(k_ratio, dim3(1), dim3(256), 0, c.st, c.sc(nxt), c.sc(cur), c.sc(kBeta), c.B);
    TOMO_HIP(hipGetLastError());
    std::swap(cur, nxt);
  }
  // the last iteration's deferred solution update (its new direction is not needed)
  if (iters > 0) TOMO_TRY(c.lin(x, x, w.p, nullptr, c.sc(kAlpha), 1.0, 1.0, c.img));   // x += alpha p
  return TOMO_OK;
}

// Conjugate gradients on the normal equations A^T A x = A^T b with A^T A applied through the
// normal-operator stencil (no 1D FFTs; equal to CGLS in exact arithmetic).
tomo_status cgnr(const Ctx& c, const float* b, float* x, int vt, int iters, bool use_x0) {
  SolverBuffers& w = c.op->sb;
  TOMO_TRY(apply_backproject(c.op, b, w.s, c.B, vt, TOMO_FILTER_NONE, 1.0f, c.st));   // r = A^T b
  if (use_x0) {
    TOMO_TRY(apply_normal(c.op, x, w.t, c.B, vt, TOMO_FILTER_NONE, c.st));
    TOMO_TRY(c.lin(w.s, w.s, w.t, nullptr, nullptr, 1.0, -1.0, c.img));      // r -= A^T A x
  } else {
    TOMO_TRY(launch_fill(x, 0.f, c.img * c.B, c.st));
  }
  TOMO_TRY(c.lin(w.p, w.s, nullptr, nullptr, nullptr, 1.0, 0.0, c.img));     // p = r
  int cur = kGamma0, nxt = kGamma1;
  TOMO_TRY(c.dot(w.s, w.s, c.img, cur));                                      // gamma = |r|^2
  for (int it = 0; it < iters; ++it) {
    // (after the first iteration: x += alpha p; p = r + beta p) q = A^T A p; delta = p.q
    TOMO_TRY(c.normal_dot(it == 0 ? nullptr : x, w.p, w.s, w.t, vt, kDelta));
    hipLaunchKernelGGL(k_ratio, dim3(1), dim3(256), 0, c.st, c.sc(cur), c.sc(kDelta), c.sc(kAlpha), c.B);
    TOMO_HIP(hipGetLastError());
    TOMO_TRY(c.axpy_dot(w.s, w.t, c.img, nxt));          // r -= alpha q; gamma' = |r|^2
    hipLaunchKernelGGL(k_ratio, dim3(1), dim3(256), 0, c.st, c.sc(nxt), c.sc(cur), c.sc(kBeta), c.B);
    TOMO_HIP(hipGetLastError());
    std::swap(cur, nxt);
  }
  // the last iteration's deferred solution update (its new direction is not needed)
  if (iters > 0) TOMO_TRY(c.lin(x, x, w.p, nullptr, c.sc(kAlpha), 1.0, 1.0, c.img));   // x += alpha p
  return TOMO_OK;
}

// Split-Bregman TV (Sec. 3.1, the paper's TV algorithm): min (mu/2)||A x - b||^2 + sum |D x|.
// Each outer step solves (mu A^T A + lam D^T D) x = mu A^T b + lam D^T (d - e) by `inner` CG
// steps from the current x (A^T A through the normal-operator stencil when the geometry allows
// it), then shrinks s = D x + e into d and sets e = s - d.  x0 = 0; d = e = 0.
tomo_status tv_split_bregman(const Ctx& c, const float* b, float* x, int vt, int outer, int inner,
                             double mu, double lam) {
  SolverBuffers& w = c.op->sb;
  const int64_t tot = c.img * c.B;
  float* ATf = w.tvb;
  float* d1 = w.tvb + tot;
  float* d2 = w.tvb + 2 * tot;
  float* e1 = w.tvb + 3 * tot;
  float* e2 = w.tvb + 4 * tot;
  float* rhs = w.tvb + 5 * tot;
  const bool nrm = normal_supported(c.op) == TOMO_OK;
  clear_error();
  const int n = c.op->g.n;
  const dim3 grid(grid_for((int64_t)n * n), (unsigned)c.B);
  // q = mu A^T A v + lam D^T D v.  With step (CG iterations after the first), the deferred
  // update x += alpha v; v = r + beta v comes first (fused into the forward transform's first
  // kernel when it can be); with slot, slot = v . q, summed by the Laplacian kernel as it writes q.
  auto apply_M = [&](float* v, float* q, bool step, int slot) -> tomo_status {
    const bool fuse = step && project_cg_supported(c.op);
    if (step && !fuse) TOMO_TRY(c.cg_step(x, v, w.s, c.img));
    const CgStep cg{x, w.s, c.sc(kAlpha), c.sc(kBeta)};
    if (nrm) {
      TOMO_TRY(apply_normal(c.op, v, q, c.B, vt, TOMO_FILTER_NONE, c.st, fuse ? &cg : nullptr));
    } else {
      if (fuse)
        TOMO_TRY(apply_project_cg(c.op, v, cg, w.q, c.B, vt, c.st));
      else
        TOMO_TRY(apply_project(c.op, v, w.q, c.B, vt, c.st));
      TOMO_TRY(apply_backproject(c.op, w.q, q, c.B, vt, TOMO_FILTER_NONE, 1.0f, c.st));
    }
    double* part = slot >= 0 ? w.partial : nullptr;
    unsigned blocks;
    if (n % 4 == 0) {
      blocks = grid_for((int64_t)n * n / 4);
      if (part) blocks = std::min<unsigned>(blocks, kDotBlocks);
      hipLaunchKernelGGL(k_sb_addlap4, dim3(blocks, (unsigned)c.B), dim3(256), 0, c.st, v, q,
                         (float)mu, (float)lam, n, part);
    } else {
      blocks = grid.x;
      if (part) blocks = std::min<unsigned>(blocks, kDotBlocks);
      hipLaunchKernelGGL(k_sb_addlap, dim3(blocks, (unsigned)c.B), dim3(256), 0, c.st, v, q,
                         (float)mu, (float)lam, n, part);
    }
    TOMO_HIP(hipGetLastError());
    if (part) {
      hipLaunchKernelGGL(k_dot_final, dim3(c.B), dim3(256), 0, c.st, part, (int)blocks, c.sc(slot));
      TOMO_HIP(hipGetLastError());
    }
    return TOMO_OK;
  };
  TOMO_TRY(apply_backproject(c.op, b, ATf, c.B, vt, TOMO_FILTER_NONE, 1.0f, c.st));
  TOMO_TRY(launch_fill(x, 0.f, tot, c.st));
  TOMO_TRY(launch_fill(d1, 0.f, 4 * tot, c.st));                              // d1, d2, e1, e2
  for (int k = 0; k < outer; ++k) {
    hipLaunchKernelGGL(k_sb_rhs, grid, dim3(256), 0, c.st, ATf, d1, d2, e1, e2, rhs,
                       (float)mu, (float)lam, n);
    TOMO_HIP(hipGetLastError());
    // CG on M x = rhs from the current x: r = rhs - M x, p = r
    TOMO_TRY(apply_M(x, w.t, false, -1));
    TOMO_TRY(c.lin(w.s, rhs, w.t, nullptr, nullptr, 1.0, -1.0, c.img));
    TOMO_TRY(c.lin(w.p, w.s, nullptr, nullptr, nullptr, 1.0, 0.0, c.img));
    int cur = kGamma0, nxt = kGamma1;
    TOMO_TRY(c.dot(w.s, w.s, c.img, cur));
    for (int it = 0; it < inner; ++it) {
      // (after the first iteration: x += alpha p; p = r + beta p) q = M p; delta = p . q
      TOMO_TRY(apply_M(w.p, w.t, it > 0, kDelta));
      hipLaunchKernelGGL(k_ratio, dim3(1), dim3(256), 0, c.st, c.sc(cur), c.sc(kDelta), c.sc(kAlpha), c.B);
      TOMO_HIP(hipGetLastError());
      TOMO_TRY(c.axpy_dot(w.s, w.t, c.img, nxt));            // r -= alpha q; gamma' = |r|^2
      hipLaunchKernelGGL(k_ratio, dim3(1), dim3(256), 0, c.st, c.sc(nxt), c.sc(cur), c.sc(kBeta), c.B);
      TOMO_HIP(hipGetLastError());
      std::swap(cur, nxt);
    }
    // the last CG iteration's deferred solution update
    if (inner > 0) TOMO_TRY(c.lin(x, x, w.p, nullptr, c.sc(kAlpha), 1.0, 1.0, c.img));
    hipLaunchKernelGGL(k_sb_shrink, grid, dim3(256), 0, c.st, x, d1, d2, e1, e2,
                       (float)(1.0 / lam), n);
    TOMO_HIP(hipGetLastError());
  }
  return TOMO_OK;
}

// SIRT with the ramp/Hamming preconditioner D in the polar Fourier domain and BB steps:
// g = A^T_D (A x - b), x0 = 0, gradients carried by the recurrence g -= alpha A^T_D A g.
// With `normal`, h = A^T_D A g is applied through the normal-operator stencil of D.
tomo_status sirt_bb(const Ctx& c, const float* b, float* x, int vt, int iters, int filter,
                    bool normal) {
  SolverBuffers& w = c.op->sb;
  TOMO_TRY(launch_fill(x, 0.f, c.img * c.B, c.st));
  TOMO_TRY(apply_backproject(c.op, b, w.s, c.B, vt, filter, 1.0f, c.st));   // s = A^T_D b
  TOMO_TRY(c.lin(w.p, w.s, nullptr, nullptr, nullptr, -1.0, 0.0, c.img));  // g = -A^T_D b
  for (int it = 0; it < iters; ++it) {
    if (normal) {
      TOMO_TRY(apply_normal(c.op, w.p, w.s, c.B, vt, filter, c.st));       // h = A^T_D A g
    } else {
      TOMO_TRY(apply_project(c.op, w.p, w.q, c.B, vt, c.st));              // q = A g
      TOMO_TRY(apply_backproject(c.op, w.q, w.s, c.B, vt, filter, 1.0f, c.st));   // h = A^T_D A g
    }
    TOMO_TRY(c.dot2(w.p, w.s, c.img, kNum, kDen));                           // g.g, g.h
    hipLaunchKernelGGL(k_sirt_step, dim3(1), dim3(256), 0, c.st, c.sc(kNum), c.sc(kDen), c.sc(kPNum),
                       c.sc(kPDen), c.sc(kAlpha), c.B, it == 0 ? 1 : 0);
    TOMO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sirt_update, dim3(grid_for(c.img), c.B), dim3(256), 0, c.st, x, w.p, w.s,
                       c.sc(kAlpha), c.img);                                  // x -= a g; g -= a h
    TOMO_HIP(hipGetLastError());
  }
  return TOMO_OK;
}

}  // namespace

// out[i] = re if i even, 0 if odd (a real vector as one complex channel); dst[i] = src[2 i]
__global__ __launch_bounds__(256) void k_fill_real(float* __restrict__ out, float v, int64_t n2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += (int64_t)gridDim.x * 256)
    out[i] = (i & 1) ? 0.f : v;
}
__global__ __launch_bounds__(256) void k_real_part(const float* __restrict__ src, float* __restrict__ dst,
                                                   int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[i] = src[2 * i];
}

// v(kf, a) and v(L - kf, a) (frequencies k and -k at one angle, FFT-ordered rows kf * nt + a)
// both set to their mean; kf = 0 and, for even L, kf = L/2 have no mirror and stay.
__global__ __launch_bounds__(256) void k_mirror_average(float2* __restrict__ v, int L, int nt) {
  const int64_t pairs = (int64_t)((L - 1) / 2) * nt;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < pairs; i += (int64_t)gridDim.x * 256) {
    const int kf = 1 + (int)(i / nt), a = (int)(i % nt);
    const int64_t p = (int64_t)kf * nt + a, q = (int64_t)(L - kf) * nt + a;
    const float2 x = v[p], y = v[q];
    const float2 m = make_float2(0.5f * (x.x + y.x), 0.5f * (x.y + y.y));
    v[p] = m;
    v[q] = m;
  }
}

// Density filter (Sec. 3): CGLS from zero on S Pi D_v = c 1 over weights even in the frequency
// (Pi the mirror average; see k_mirror_average), c = kappa(0)^2 = 1 / k*(origin), with the
// forward / adjoint SpMMs on one complex channel whose imaginary parts stay zero.  Even weights
// keep the filtered back projection of a real sinogram real, which the pairing of two slices in
// one complex channel needs.
tomo_status run_density(tomo_op* op, int iters, double* resid, hipStream_t st) {
  const Geom& g = op->g;
  const int64_t N = (int64_t)g.L * g.nt, M = (int64_t)g.G * g.G;
  const double kd0 = op->kd[g.on];
  const float target = (float)(1.0 / (kd0 * kd0));
  float *v = nullptr, *s = nullptr, *p = nullptr, *r = nullptr, *q = nullptr;
  double *scal = nullptr, *partial = nullptr;
  struct Req { void** p; size_t bytes; } req[] = {
      {(void**)&v, (size_t)N * 8}, {(void**)&s, (size_t)N * 8}, {(void**)&p, (size_t)N * 8},
      {(void**)&r, (size_t)M * 8}, {(void**)&q, (size_t)M * 8},
      {(void**)&scal, kSlots * sizeof(double)}, {(void**)&partial, kDotBlocks * sizeof(double)}};
  tomo_status status = TOMO_OK;
  for (auto& rq : req)
    if (status == TOMO_OK && hipMalloc(rq.p, rq.bytes) != hipSuccess) {
      *rq.p = nullptr;
      status = fail(TOMO_ENOMEM, "density filter workspace (%zu B)", rq.bytes);
    }
  auto sc = [&](int slot) { return scal + slot; };
  auto dot = [&](const float* a, const float* b, int64_t len, int slot) {
    return launch_dot(a, b, len, 1, partial, sc(slot), st);
  };
  auto lin = [&](float* out, const float* a, const float* b, const double* ca, const double* cb,
                 double sa, double sb, int64_t len) {
    return launch_lincomb(out, a, b, ca, cb, sa, sb, len, 1, st);
  };
  auto body = [&]() -> tomo_status {
    hipLaunchKernelGGL(k_fill_real, dim3(grid_for(2 * M)), dim3(256), 0, st, r, target, 2 * M);
    TOMO_HIP(hipGetLastError());
    TOMO_TRY(launch_fill(v, 0.f, 2 * N, st));
    auto grad = [&]() -> tomo_status {   // s = Pi S^T r
      TOMO_TRY(launch_spmm_fwd(op, (const float2*)r, (float2*)s, 1, TOMO_VAL_F32, st));
      hipLaunchKernelGGL(k_mirror_average, dim3(grid_for((int64_t)((g.L - 1) / 2) * g.nt)), dim3(256),
                         0, st, (float2*)s, g.L, g.nt);
      TOMO_HIP(hipGetLastError());
      return TOMO_OK;
    };
    TOMO_TRY(grad());
    TOMO_TRY(lin(p, s, nullptr, nullptr, nullptr, 1.0, 0.0, 2 * N));
    int cur = kGamma0, nxt = kGamma1;
    TOMO_TRY(dot(s, s, 2 * N, cur));
    for (int it = 0; it < iters; ++it) {
      TOMO_TRY(launch_spmm_adj(op, (const float2*)p, (float2*)q, 1, TOMO_VAL_F32, nullptr, st));
      TOMO_TRY(dot(q, q, 2 * M, kDelta));
      hipLaunchKernelGGL(k_ratio, dim3(1), dim3(256), 0, st, sc(cur), sc(kDelta), sc(kAlpha), 1);
      TOMO_HIP(hipGetLastError());
      TOMO_TRY(lin(v, v, p, nullptr, sc(kAlpha), 1.0, 1.0, 2 * N));
      TOMO_TRY(lin(r, r, q, nullptr, sc(kAlpha), 1.0, -1.0, 2 * M));
      TOMO_TRY(grad());
      TOMO_TRY(dot(s, s, 2 * N, nxt));
      hipLaunchKernelGGL(k_ratio, dim3(1), dim3(256), 0, st, sc(nxt), sc(cur), sc(kBeta), 1);
      TOMO_HIP(hipGetLastError());
      TOMO_TRY(lin(p, s, p, nullptr, sc(kBeta), 1.0, 1.0, 2 * N));
      std::swap(cur, nxt);
    }
    if (!op->dens) {
      if (hipMalloc((void**)&op->dens, (size_t)N * sizeof(float)) != hipSuccess) {
        op->dens = nullptr;
        return fail(TOMO_ENOMEM, "density weights (%lld floats)", (long long)N);
      }
    }
    hipLaunchKernelGGL(k_real_part, dim3(grid_for(N)), dim3(256), 0, st, v, op->dens, N);
    TOMO_HIP(hipGetLastError());
    if (resid) {
      TOMO_TRY(dot(r, r, 2 * M, kTmp));
      double rr = 0;
      TOMO_HIP(hipMemcpyAsync(&rr, sc(kTmp), sizeof(double), hipMemcpyDeviceToHost, st));
      TOMO_HIP(hipStreamSynchronize(st));
      *resid = std::sqrt(rr);
    }
    return TOMO_OK;
  };
  if (status == TOMO_OK) status = body();
  (void)hipStreamSynchronize(st);
  for (auto& rq : req)
    if (*rq.p) (void)hipFree(*rq.p);
  return status;
}

tomo_status run_solve(tomo_op* op, const float* b, float* x, int B, const tomo_solve_opts* o,
                      hipStream_t st) {
  if (B > 256) return fail(TOMO_EINVAL, "batch too large for the scalar kernels");
  TOMO_TRY(ensure_solver(op));
  Ctx c{op, B, st, (int64_t)op->g.n * op->g.n, (int64_t)op->g.nt * op->g.np};
  SolverBuffers& w = op->sb;
  const bool cg_normal = o->method == TOMO_SOLVE_CGNR;
  if (o->method == TOMO_SOLVE_TV_SPLIT_BREGMAN) {
    TOMO_TRY(tv_split_bregman(c, b, x, o->values, o->refine_outer, o->iters, o->tv_mu, o->tv_lambda));
  } else if (o->method == TOMO_SOLVE_SIRT_BB || o->method == TOMO_SOLVE_SIRT_BB_NORMAL) {
    const int filter = o->filter == TOMO_FILTER_NONE ? TOMO_FILTER_HAMMING : o->filter;
    TOMO_TRY(sirt_bb(c, b, x, o->values, o->iters, filter,
                     o->method == TOMO_SOLVE_SIRT_BB_NORMAL));
  } else if (o->refine_outer == 1) {
    if (cg_normal)
      TOMO_TRY(cgnr(c, b, x, o->values, o->iters, o->use_x0 != 0));
    else
      TOMO_TRY(cgls(c, b, x, o->values, o->iters, o->use_x0 != 0));
  } else {
    // iterative refinement: residual with float32 values, correction with `values`
    for (int outer = 0; outer < o->refine_outer; ++outer) {
      const bool have_x = outer > 0 || o->use_x0;
      if (have_x) {
        TOMO_TRY(apply_project(op, x, w.q, B, TOMO_VAL_F32, st));
        TOMO_TRY(c.lin(w.rb, b, w.q, nullptr, nullptr, 1.0, -1.0, c.sino));   // rb = b - A_f32 x
      } else {
        TOMO_TRY(c.lin(w.rb, b, nullptr, nullptr, nullptr, 1.0, 0.0, c.sino));
      }
      if (cg_normal)
        TOMO_TRY(cgnr(c, w.rb, w.d, o->values, o->iters, false));
      else
        TOMO_TRY(cgls(c, w.rb, w.d, o->values, o->iters, false));
      if (have_x)
        TOMO_TRY(c.lin(x, x, w.d, nullptr, nullptr, 1.0, 1.0, c.img));       // x += d
      else
        TOMO_TRY(c.lin(x, w.d, nullptr, nullptr, nullptr, 1.0, 0.0, c.img)); // x = d
    }
  }
  if (o->out_resnorm) {
    TOMO_TRY(apply_project(op, x, w.q, B, TOMO_VAL_F32, st));
    TOMO_TRY(c.lin(w.r, b, w.q, nullptr, nullptr, 1.0, -1.0, c.sino));
    TOMO_TRY(c.dot(w.r, w.r, c.sino, kTmp));
    hipLaunchKernelGGL(k_sqrt, dim3(1), dim3(256), 0, st, c.sc(kTmp), o->out_resnorm, B);
    TOMO_HIP(hipGetLastError());
  }
  return TOMO_OK;
}

}  // namespace tomo
