// Internal declarations of libtomo: host builder, device operator state, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/tomo.h"
#include "fft_lds.h"

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
  int cdet = 0;            // integer part of the rotation-axis bin, mod L
  double cfrac = 0;        // its fractional part, in [0, 1): a phase ramp on the polar rows
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

// Layout parameters of the two SpMMs (the autotuner's search space; tomo_set_tuning).
struct Tuning {
  int fwd_cpl = 2;        // complex channels per lane in the forward kernel (1, 2 or 4)
  int adj_cpl = 4;        // complex channels per lane in the adjoint row kernels (1, 2 or 4)
  int sell_max = 64;      // S rows with <= sell_max entries: sliced ELL, 8 rows per slice
  int sell_sigma = 4096;  // rows are sorted by length within windows of sell_sigma rows
  int medium_max = 256;   // longer rows up to medium_max entries: one wavefront per row
  int chunk = 1024;       // rows above medium_max: chunks of <= chunk entries, one block each
  // staged kernels per value type: bit vt (1 f32, 2 bf16, 4 f16) set = staged, clear = rows
  int fwd_tiled = 7;      // forward: LDS-staged Cartesian tiles
  int adj_tiled = 7;      // adjoint: LDS-staged output tiles (+ row kernels on dense cells)
  int tile = 8;           // Cartesian tile side of the staged kernels (8 or 16)
  int tile_points = 64;   // forward: samples per block
  int adj_tile_points = 128;   // adjoint: most samples a staged tile's region may hold
  int normal_tiled = 1;   // normal operator: LDS-staged grid tiles (1) or direct taps (0)
  int sell_xcd_rows = 8192;   // sliced-ELL adjoint: rows per XCD interleave run (0 = contiguous)
  int medium_xcd_rows = 1024; // wave-per-row adjoint: rows per XCD interleave run
  int fwd_rows_per_group = 2; // forward: rows per lane group in the pipelined kernel (1, 2, 4)
  int det_fft = 1;            // detector transforms: hand-written, the adjoint front writing the
                              // SpMM's layout where the length allows (1) or channel-slowest
                              // rows (2); library (0)
  int grid_fft = 1;           // Cartesian 2D transforms: fused hand-written (1) or library (0)
  int sell_tiles = 1;         // sliced-ELL rows in 4 x 8 Cartesian tiles (1) or grid order (0)
  int tile_strip = 32;        // staged kernels visit tiles in strips this many tiles wide (0 = rows)
  // the staged adjoint's dense tiles (regions holding more than adj_tile_points samples):
  // 0 = row kernels on their cells; 1 = staged in chunks of <= adj_tile_points samples, one block
  // per segment of <= adj_seg_chunks chunks (split tiles summed from partial tiles in a fixed
  // order), on a second stream beside the staged tiles; 2 = the same segments and the staged
  // tiles in one launch, dense segments first
  int adj_dense_mode = 0;
  int adj_seg_chunks = 8;
  // in the one-launch form (adj_dense_mode 2): staged tiles per block, visited in order with the
  // next tile's loads in flight while the current one is summed
  int adj_run = 1;
};

constexpr int kSliceRows = 8;    // rows per slice of the sliced-ELL layout
constexpr int kMaxSegChunks = 256;   // most chunks one segment of the staged adjoint may hold

// S^dagger with a constant row stride W2 = k_w^2 (its rows never hold more): entry s of row r
// at r * W2 + s, padded with column -1 (skipped) and value 0.
struct HostEll {
  int W2 = 0;
  std::vector<int32_t> col;
  std::vector<double> val;
};

// S split by row length: short rows in sliced ELL (slice i holds rows slice_rows[8i .. 8i+8),
// entry e of slot j at slice_ptr[i] + 8 e + j, padded with column -1), the remaining rows as a
// compact CSR ("tail"): medium rows first, then long rows, whose entries are cut into chunks.
struct HostAdj {
  std::vector<int32_t> slice_ptr, slice_rows, col;
  std::vector<double> val;
  std::vector<int32_t> tail_rows, tail_ptr, tail_col;
  std::vector<double> tail_val;
  int64_t n_medium = 0, n_long = 0, sell_rows = 0, sell_padding = 0;
  std::vector<int32_t> chunk_beg, chunk_end, long_chunk_ptr;   // into the tail entries
};

// Forward, LDS-staged, window form: polar samples grouped by the Cartesian tile (side TS) that
// holds their window centre; a block stages the tile plus a halo of h = (k_w-1)/2 below and h+1
// above (patch side PS = TS + 2h + 1: a centre rounded onto the grid's upper edge keeps its whole
// window in the patch) and reads every tap from LDS.  Sample i's k_w x k_w window starts at patch
// slot pt_base[i]; tap (s1, s2) is slot pt_base[i] + s1*PS + s2 with value pt_val[i*W2 + s1*k_w
// + s2] (zero for a tap the matrix does not hold).
struct HostFwdTiles {
  int TS = 0, PS = 0, NT = 0, KW = 0, W2 = 0;
  std::vector<int32_t> wi_tile, wi_beg;    // [n_wi], [n_wi + 1] into the sample list
  std::vector<int32_t> pt_row;             // polar row of each sample
  std::vector<int32_t> pt_base;            // [P] first window slot in the patch
  std::vector<double> pt_val;              // [P][W2] window-ordered values
};

// Adjoint, LDS-staged, window form: a block owns one Cartesian tile (side TS) and stages every
// polar sample whose window centre lies in the tile's region (the tile grown by h on each side,
// side RS = TS + 2h), bucketed by centre cell; output cell m sums, over the k_w^2 centre cells
// m - s (s in [-h, h]^2), the bucket's samples times their window value at position s + h.
// Tiles whose region holds more than adj_tile_points samples (near the Fourier origin) are
// "dense": their cells go to the row kernels through a row layout built over those cells only.
struct HostAdjWin {
  int TS = 0, RS = 0, NT = 0, KW = 0, W2 = 0, QMAX = 0;
  std::vector<int32_t> wi_tile;            // [n_wi] staged tiles
  std::vector<int32_t> wi_q;               // [n_wi + 1] into the tile sample list
  std::vector<uint16_t> wi_boff;           // [n_wi][RS*RS + 1] bucket offsets from wi_q[w]
  std::vector<int32_t> q_row;              // polar row of each tile sample
  std::vector<double> q_val;               // [Q][W2] window-ordered values
  std::vector<char> dense_cell;            // [M] library cell index -> 1 if in a dense tile
  // Dense tiles staged in chunks (always built: the FFT-side form and adj_dense_mode 1 / 2 use
  // them, the channel-fastest form with adj_dense_mode 0 the row kernels).  Chunks extend the
  // work-item arrays:
  // chunk c >= n_wi covers samples [wi_q[c], wi_q[c+1]) with bucket offsets wi_boff[c] (relative
  // to wi_q[c]).  Segment s covers chunks [seg_chunk[s], seg_chunk[s+1]) of tile seg_tile[s];
  // segments 0 .. n_wi-1 are the staged tiles (one chunk each), the rest the dense tiles.  A
  // segment writes its tile's cells to X when seg_slot[s] < 0, else partial tile seg_slot[s];
  // split tile i sums partial tiles [red_slot[i], red_slot[i+1]) in order into tile red_tile[i].
  int64_t n_wi = 0;                        // staged tiles (the first n_wi chunks)
  int64_t n_sseg = 0;                      // segments of staged tiles (runs of adj_run tiles)
  std::vector<int32_t> chunk_tile;         // [n_chunks] tile of every chunk
  std::vector<int32_t> seg_tile, seg_chunk, seg_slot;
  std::vector<int32_t> red_tile, red_slot;
};

tomo_status resolve_geometry(const tomo_geometry* in, Geom* g);
double kernel_value(double t, int W, double beta);
void build_sdag(const Geom& g, HostCSR* sdag, std::vector<int32_t>* centres = nullptr);
// Samples within a tile in polar row order (kf * nt + a: the channel-fastest output's rows
// adjacent), or, with slowest_order, by angle then radius (runs of consecutive radii in the
// channel-slowest rows); the work items (wi_tile, wi_beg) are the same in both.
tomo_status build_fwd_tiles(const Geom& g, const HostCSR& sdag, const std::vector<int32_t>& centres,
                            const Tuning& t, HostFwdTiles* out, bool slowest_order = false);
tomo_status build_adj_win(const Geom& g, const HostCSR& sdag, const std::vector<int32_t>& centres,
                          const Tuning& t, HostAdjWin* out);
void transpose_csr(const HostCSR& a, HostCSR* at);
void build_ell(const HostCSR& a, int W2, HostEll* out);
tomo_status check_tuning(const Tuning& t);
// rows: if non-null, only rows r with (*rows)[r] != 0 are laid out (the others are not written)
void build_adj_layout(const HostCSR& s, const Tuning& t, HostAdj* out,
                      const std::vector<char>* rows = nullptr);
tomo_status check_layouts(const Geom& g, const HostCSR& sdag, const HostCSR& s,
                          const std::vector<int32_t>& centres, const Tuning& t, double* max_rel);
void deapod_factors(const Geom& g, std::vector<double>* kd);
void filter_diagonal(const Geom& g, int filter, std::vector<double>* d);   // FFT-ordered k
uint16_t f32_to_bf16_rne(float f);
bool normal_stencil_row(const Geom& g, const HostCSR& s, const HostCSR& sdag, const double* dk,
                        int64_t j, double* out);
tomo_status build_normal_values(const Geom& g, const HostCSR& s, const HostCSR& sdag,
                                const double* dk, int stride, std::vector<double>* w);

// ---------------------------------------------------------------------------------
// device state
// ---------------------------------------------------------------------------------
struct DevEll {
  int64_t rows = 0;
  int W2 = 0;
  int32_t* col = nullptr;
  void* val[3] = {nullptr, nullptr, nullptr};   // indexed by tomo_value_type
};

// W = S diag(D) S^dagger for the normal operator as a fixed stencil: values [G*G][stride] per
// filter and value type, slot (d1 + R)(2R + 1) + (d2 + R) for the FFT-ordered offset (d1, d2),
// R = kw - 1, stride = (2R+1)^2 rounded up to 8 (zero padded).  Built on first use per filter.
struct DevNormal {
  int R = 0, stride = 0;
  void* val[4][3] = {};   // [tomo_filter][tomo_value_type]
};

struct DevAdj {
  int64_t n_slices = 0, n_medium = 0, n_long = 0, n_chunks = 0;
  int32_t *slice_ptr = nullptr, *slice_rows = nullptr, *col = nullptr;
  void* val[3] = {nullptr, nullptr, nullptr};
  int32_t *tail_rows = nullptr, *tail_ptr = nullptr, *tail_col = nullptr;
  void* tail_val[3] = {nullptr, nullptr, nullptr};
  int32_t *chunk_beg = nullptr, *chunk_end = nullptr, *long_chunk_ptr = nullptr;
};

struct DevFwdTiles {
  int64_t n_wi = 0;
  int TS = 0, PS = 0, NT = 0, KW = 0;
  int32_t *wi_tile = nullptr, *wi_beg = nullptr;
  // [0]: samples in row order (channel-fastest output); [1]: by angle, then radius (the
  // channel-slowest output of the FFT-side form)
  int32_t* pt_row[2] = {nullptr, nullptr};
  int32_t* pt_base[2] = {nullptr, nullptr};
  void* val[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
};

struct DevAdjWin {
  int64_t n_wi = 0;               // staged tiles (one block each)
  int TS = 0, RS = 0, NT = 0, KW = 0, QMAX = 0;
  int32_t *wi_tile = nullptr, *wi_q = nullptr, *q_row = nullptr;
  uint16_t* wi_boff = nullptr;
  void* q_val[3] = {nullptr, nullptr, nullptr};
  // dense tiles in chunked segments (HostAdjWin): n_seg segments in all, the first n_sseg of them
  // runs of staged tiles; n_red split tiles reduced from n_slot partial tiles
  int64_t n_seg = 0, n_sseg = 0, n_red = 0, n_slot = 0;
  int max_seg_chunks = 0;         // most chunks of any segment
  int32_t *seg_tile = nullptr, *seg_chunk = nullptr, *seg_slot = nullptr, *chunk_tile = nullptr;
  int32_t *red_tile = nullptr, *red_slot = nullptr;
};

struct FFTPlans {
  rocfft_plan fwd2 = nullptr, inv2 = nullptr, fwd1 = nullptr, inv1 = nullptr;
  rocfft_execution_info info = nullptr;
  void* work = nullptr;
  size_t work_bytes = 0;
};

struct SolverBuffers {
  int B = 0;
  float *p = nullptr, *s = nullptr, *d = nullptr, *t = nullptr;   // image-sized [B][n][n]
  float *r = nullptr, *q = nullptr, *rb = nullptr;     // sinogram-sized [B][nt][np]
  double* scal = nullptr;                              // per-slice scalars [16][B]
  double* partial = nullptr;                           // dot partial sums [B][kDotBlocks]
  double* norm_partial = nullptr;                      // output-norm partial sums [B][norm_blocks]
  int64_t norm_blocks = 0;
  float* tvb = nullptr;                                // split-Bregman fields [6][B][n][n]
};

}  // namespace tomo

struct tomo_op {
  tomo::Geom g;
  tomo::Tuning tune;
  tomo::HostCSR sdag, s;          // float64 host copies (test export)
  tomo::HostAdj hadj;             // adjoint layout for the current tuning
  std::vector<double> kd;         // separable deapodisation factors [n]
  int device = -1;
  int n_cu = 256;                 // compute units of the device
  // second stream of the staged adjoint: the dense-cell row kernels run there, forked from and
  // joined back to the caller's stream by events, beside the staged kernel (disjoint outputs)
  hipStream_t aux = nullptr, aux2 = nullptr;   // dense sliced-ELL rows; dense longer rows
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
  uint32_t values = 0;
  int64_t cols_touched = 0, polar_nonempty = 0;
  // device
  tomo::DevEll fwd;
  tomo::DevAdj adj;
  float* kd_dev = nullptr;        // [n]
  // polar-row phase of a fractional rotation-axis bin c0 + f: phase[kf] = exp(-2 pi i k f / L)
  // for the signed frequency k of FFT-ordered radial index kf (project multiplies by it before
  // the inverse detector DFT, backproject by its conjugate after the forward one); null when
  // f == 0
  float2* phase_dev = nullptr;    // [L]
  // tables of the hand-written DFTs: detector length L and grid side G (twiddles of the length M
  // held in LDS; chirp and convolution kernels when M is the Bluestein length of L or G)
  tomo::fftk::DftTables dft1, dft2;
  float* dens = nullptr;          // [L*nt] density-filter weights (tomo_density_filter)
  float* filt_dev[4] = {nullptr, nullptr, nullptr, nullptr};   // D per tomo_filter, [L]
  int cmax = 0;                   // complex channels the workspace holds
  float2* X = nullptr;            // [G*G][C]     channel-fastest Cartesian grid (SpMM side)
  float2* Y = nullptr;            // [L*nt][C]    channel-fastest polar data (SpMM side)
  float2* Xs = nullptr;           // [C][G][G]    channel-slowest Cartesian grid (FFT side)
  float2* Ys = nullptr;           // [C][nt][L]   channel-slowest polar data (FFT side)
  float2* partials = nullptr;     // [n_chunks][cmax] long-row partial sums
  size_t partials_cap = 0;        // chunks the partials buffer holds
  bool adj_ready = false;         // false while (or after a failed) adjoint layout upload
  std::vector<int32_t> centres;   // window centre (j1, j2) of every polar row, host
  tomo::DevFwdTiles ftile;        // LDS-staged forward layout
  tomo::DevAdjWin awin;           // LDS-staged adjoint layout
  tomo::DevAdj adj_dense;         // row layout of the staged adjoint's dense cells
  float2* seg_partials = nullptr; // [n_slot][TS*TS][cmax] partial tiles of split dense tiles
  bool tiles_ready = false;
  std::map<int, tomo::FFTPlans> plans;   // keyed by channel count C
  tomo::SolverBuffers sb;
  double* tv_partial = nullptr;   // [max_batch][kDotBlocks] TV partial sums (first use)
  tomo::DevNormal nrm;            // normal-operator stencils (first use per filter)
};

namespace tomo {

// Makes `dev` current for the scope and restores the previous device.
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Argument checks shared by the apply entry points (operator, batch, pointers, value type).
tomo_status check_apply(const tomo_op* op, const void* in, const void* out, int32_t batch,
                        int32_t values);

constexpr int kDotBlocks = 256;   // blocks per slice in the FP64 reductions
constexpr int kMaxBatch = 256;    // largest max_batch an operator accepts

// FFT plans for C complex channels (created on first use).
tomo_status get_plans(tomo_op* op, int C, FFTPlans** out);
void destroy_plans(tomo_op* op);
tomo_status fft_exec(rocfft_plan plan, FFTPlans* p, void* data, hipStream_t st);

// kernel launchers (all enqueue on `st`)
tomo_status launch_embed(const tomo_op* op, const float* x, float2* Xs, int B, hipStream_t st);
tomo_status launch_crop_sino(const tomo_op* op, const float2* Ys, float* y, int B, float scale,
                             hipStream_t st);
tomo_status launch_pad_sino(const tomo_op* op, const float* y, float2* Ys, int B, hipStream_t st);
tomo_status launch_crop_image(const tomo_op* op, const float2* Xs, float* x, int B, float scale,
                              hipStream_t st);
// channel-slowest <-> channel-fastest:  a[C][P] <-> b[P][C] with P = rows (grid points)
tomo_status launch_to_channel_fastest(const float2* src, float2* dst, int64_t P, int C, hipStream_t st);
tomo_status launch_to_channel_slowest(const float2* src, float2* dst, int64_t P, int C, hipStream_t st);
// polar: Yf[kf][a][C] <-> Ys[C][a][kf]
tomo_status launch_polar_to_slowest(const float2* Yf, float2* Ys, int L, int nt, int C, hipStream_t st);
tomo_status launch_polar_to_fastest(const float2* Ys, float2* Yf, int L, int nt, int C, hipStream_t st);
// Ys[r][kf] *= phase[kf] (conj: its conjugate) for rows r < rows of length L
tomo_status launch_phase_rows(float2* Ys, const float2* phase, int L, int64_t rows, bool conj,
                              hipStream_t st);
// `slow` (only when spmm_fwd_slowest_ok / spmm_adj_slowest_ok): the Cartesian grid is the
// channel-slowest [C][G][G] FFT-side buffer, read or written by the staged kernels directly, and
// the forward writes the channel-slowest polar rows [C][nt][L]
tomo_status launch_spmm_fwd(const tomo_op* op, const float2* X, float2* Y, int C, int vt,
                            hipStream_t st, bool slow = false);
bool spmm_fwd_slowest_ok(const tomo_op* op, int C, int vt);
bool spmm_adj_slowest_ok(const tomo_op* op, int C, int vt);
tomo_status launch_spmm_adj(const tomo_op* op, const float2* Y, float2* X, int C, int vt,
                            const float* dscale, hipStream_t st, bool slow = false);

// `slow`: the Cartesian grid is channel-slowest [C][G][G] (the FFT side) instead of [G*G][C], and
// for the forward the polar output too ([C][nt][L] instead of [L*nt][C])
tomo_status launch_fwd_tile(const tomo_op* op, const float2* X, float2* Y, int C, int vt,
                            bool slow, hipStream_t st);
tomo_status launch_adj_tile(const tomo_op* op, const float2* Y, float2* X, int C, int vt,
                            const float* dscale, bool slow, hipStream_t st);
// staged adjoint segments: the dense tiles' segments (+ their reduction) when `dense`, the
// staged tiles as one-chunk segments when `staged` (both: one launch, dense segments first)
tomo_status launch_adj_seg(const tomo_op* op, const float2* Y, float2* X, int C, int vt,
                           const float* dscale, bool dense, bool staged, bool slow, hipStream_t st);
size_t fwd_tile_lds_bytes(const tomo_op* op, int C);
bool fwd_tile_supported(const tomo_op* op);
size_t adj_tile_lds_bytes(const tomo_op* op, int C);
size_t adj_seg_lds_bytes(const tomo_op* op, int C);

// Persistent SpMM pairs over a stack of operators (tiles.hip): one forward kernel and one adjoint
// kernel (+ a reduction of split tiles) walk device work lists covering every item.
struct StackItemSpec {
  const tomo_op* op;
  int batch;
  const float* in;   // Xc, the item's Cartesian input
  float* out;        // Yp = S^dagger Xc
  float* aux;        // Xc' = S Yp
};
struct StackPlan;
tomo_status stack_plan_create(const StackItemSpec* items, int n, int vt, StackPlan** out);
tomo_status stack_plan_launch(const StackPlan* p, hipStream_t st);
void stack_plan_destroy(StackPlan* p);   // the segment kernel's LDS per block
bool adj_tile_supported(const tomo_op* op);
constexpr size_t kMaxTileLds = 65536;   // staged kernels are used when their LDS fits this

// composite operators on caller buffers
// A deferred conjugate-gradient step applied by the forward transform's first kernel to its input
// p before embedding it: x += alpha[s] p; p = s + beta[s] p (p, x updated in place).
struct CgStep {
  float* x;
  const float* s;
  const double* alpha;
  const double* beta;
};
// With sumsq set (project_sumsq_blocks(op) > 0, else an error), the last kernel also leaves the
// float64 partial sums of each output slice's squared norm in sumsq ([B][blocks]).
tomo_status apply_project(tomo_op* op, const float* x, float* y, int B, int vt, hipStream_t st,
                          double* sumsq = nullptr);
// project of p with the deferred CG step fused into the first kernel (project_cg_supported:
// the hand-written grid transform): x += alpha p; p = s + beta p; y = A_vt p.
bool project_cg_supported(const tomo_op* op);
tomo_status apply_project_cg(tomo_op* op, float* p, const CgStep& cg, float* y, int B, int vt,
                             hipStream_t st, double* sumsq = nullptr);
int64_t project_sumsq_blocks(const tomo_op* op);
int64_t backproject_sumsq_blocks(const tomo_op* op);
tomo_status apply_backproject(tomo_op* op, const float* y, float* x, int B, int vt, int filter,
                              float extra_scale, hipStream_t st, double* sumsq = nullptr);
// r -= alpha[s] q (in place, per slice; the arithmetic of the separate update) fused into the
// adjoint front, then x = A_vt^T r (no filter).  Needs the channel-fastest front
// (backproject_residual_supported).
bool backproject_residual_supported(const tomo_op* op);
tomo_status apply_backproject_residual(tomo_op* op, float* r, const float* q, const double* alpha,
                                       float* x, int B, int vt, hipStream_t st,
                                       double* sumsq = nullptr);

// solver
tomo_status run_solve(tomo_op* op, const float* b, float* x, int B, const tomo_solve_opts* o,
                      hipStream_t st);
void free_solver(tomo_op* op);

// Smoothed isotropic TV of `B` n x n images: grad (nullable) = weight * dTV/dx, value
// (nullable, device [B] float64) = weight * TV per slice.
tomo_status launch_tv(tomo_op* op, const float* x, int B, double eps, double weight, float* grad,
                      double* value, hipStream_t st);
// tomo_tv with its reduction partials in the library's file-scope scratch array (no allocation)
tomo_status launch_tv_noalloc(const tomo_op* op, const float* x, int B, double eps, double weight,
                              float* grad, double* value, hipStream_t st);
void free_tv(tomo_op* op);

// Normal operator on the channel-slowest Cartesian grid: Out[c][j] = sum over the stencil of
// W[j][o] In[c][j + offset(o)] (offsets wrap mod G), W for `filter` in value type vt.
// Detector transforms fused with the layout steps (any L with a DFT table: power-of-two lengths
// directly, others through Bluestein's identity).  The inverse reads Ys[C][nt][L]; the forward
// writes Ys or, for the adjoint SpMM, Yf[L][nt][C] (channel fastest; det_cf_supported:
// transform length up to 4096).
bool det_fft_supported(const tomo_op* op);
bool det_cf_supported(const tomo_op* op);
tomo_status launch_det_inverse_crop(const tomo_op* op, const float2* Ys, float* y, int B,
                                    float scale, double* sumsq, hipStream_t st);
tomo_status launch_det_pad_forward(const tomo_op* op, const float* y, float2* Y, int B,
                                   bool channel_fastest, hipStream_t st);
// the channel-fastest forward front with r -= alpha[s] q applied to its input first (r updated
// in place)
tomo_status launch_det_residual_forward(const tomo_op* op, float* r, const float* q,
                                        const double* alpha, float2* Yf, int B, hipStream_t st);
// Cartesian 2D DFT fused with embed (forward) and crop (inverse), any G with a DFT table:
// forward x -> Xs (channel-slowest), inverse Xs (overwritten) -> x.
bool grid_fft_supported(const tomo_op* op);
// cg: the deferred CG step fused into the first kernel (grid_cg_step_supported: transform
// length up to 2048)
bool grid_cg_step_supported(const tomo_op* op);
tomo_status launch_grid_forward(const tomo_op* op, const float* x, float2* Xs, int B,
                                hipStream_t st, const CgStep* cg = nullptr);
tomo_status launch_grid_inverse(const tomo_op* op, float2* Xs, float* x, int B, float scale,
                                double* sumsq, hipStream_t st, const float* dotw = nullptr);
// The output kernels of the inverse transforms can also sum the squares of what they write (or,
// for the grid, its products with dotw), per slice, as float64 partial sums sumsq[s * blocks + j]
// (blocks per channel below; 0 when the operator has no hand-written transform of that kind).
int64_t det_inverse_blocks_per_channel(const tomo_op* op);
int64_t grid_inverse_blocks_per_channel(const tomo_op* op);
// cg: the deferred CG step fused into the first kernel (x is then the direction p, updated in
// place; project_cg_supported); sumsq: partial sums of out . dotw per slice ([B][blocks],
// backproject_sumsq_blocks)
tomo_status apply_normal(tomo_op* op, const float* x, float* out, int B, int vt, int filter,
                         hipStream_t st, const CgStep* cg = nullptr, double* sumsq = nullptr,
                         const float* dotw = nullptr);
tomo_status normal_supported(const tomo_op* op);
tomo_status launch_normal_stencil(const tomo_op* op, const float2* in, float2* out, int C, int vt,
                                  int filter, hipStream_t st);

// elementwise / reduction launchers used by the solver
tomo_status launch_dot(const float* a, const float* b, int64_t len, int B, double* partial,
                       double* out, hipStream_t st);
tomo_status launch_lincomb(float* out, const float* a, const float* b, const double* ca,
                           const double* cb, double sa, double sb, int64_t len, int B,
                           hipStream_t st);
tomo_status launch_fill(float* out, float v, int64_t len, hipStream_t st);
tomo_status launch_fill_hash(float* out, int64_t len, uint32_t seed, hipStream_t st);
// Density-filter weights by CGLS on S (one complex channel); stores op->dens.
tomo_status run_density(tomo_op* op, int iters, double* resid, hipStream_t st);
// Y[p][c] *= w[p] for P rows of C complex channels.
tomo_status launch_scale_rows(float2* Y, const float* w, int64_t P, int C, hipStream_t st);
// Validate and apply a tuning (re-uploading the layouts it changes; synchronises the device).
tomo_status apply_tuning(tomo_op* op, const Tuning& t);
// Coordinate-descent search of the SpMM tuning for `batch` slices in value type vt.
tomo_status autotune(tomo_op* op, int batch, int vt, int rounds, double* fwd_ms, double* adj_ms);

}  // namespace tomo
