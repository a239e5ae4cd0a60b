/*
 * tomo.h - C ABI of the MI355X sparse Fubini-Radon tomography library (libtomo.so).
 *
 * The operator is the paper's Fourier-slice ("Fubini-Radon") factorisation of
 * the parallel-beam Radon transform (Sec. 2.2 Eq. (1), Sec. 3 Eq. (2)):
 *
 *     A   = F1D^-1 . S^dagger . F2D . diag(k*)        (project,  Radon)
 *     A^T = diag(k*) . F2D^H . S . F1D^-H             (backproject, exact transpose)
 *     FBP = (pi / n_theta) . diag(k*) . F2D^H . S . D . F1D^-H      (iRadon)
 *
 * where S (M x N) is the sparse polar-to-Cartesian gridding matrix built from a
 * Kaiser-Bessel window of width k_w (Sec. 3, Fig. 3), stored twice as CSR: once
 * with polar rows (S^dagger, forward) and once with Cartesian rows (S, adjoint),
 * so that neither direction needs atomics (Sec. 3.1: the matrix and its
 * transpose are stored separately).  Pairs of real slices travel as one complex
 * slice (Sec. 3.1), the real parts carrying even slices and the imaginary parts
 * odd slices.
 *
 * Conventions for every entry point:
 *   - Return value: TOMO_OK (0) or a negative tomo_status.  Nothing throws across
 *     the ABI; tomo_last_error() returns a thread-local message for the last error.
 *   - Device pointers are caller-owned, float32, contiguous, 256-byte aligned is
 *     not required but 16-byte alignment is (hipMalloc / torch allocations qualify).
 *     The library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All work is
 *     enqueued on it; no entry point synchronises except tomo_build_operator,
 *     tomo_destroy_operator and the first call that creates FFT plans or
 *     solver buffers for a new batch width (these allocate).
 *   - Precondition failures (NULL pointer, batch < 0 or > max_batch, unsupported
 *     value type, misaligned pointer) return TOMO_EINVAL before anything is launched.
 *   - batch == 0 is a no-op returning TOMO_OK.
 *   - An operator is not thread-safe: calls that share an operator must be ordered
 *     on one stream (its internal workspace is reused by every call).
 *
 * Layouts (row-major, slice index slowest):
 *   image stack     x[batch][n][n]            pixel (i1, i2) at centred position (i1 - n/2, i2 - n/2)
 *   sinogram stack  y[batch][n_theta][n_p]    bin b at detector offset b - center
 *   Cartesian Fourier grid X[G][G][C] complex64, FFT-ordered frequencies, C = ceil(batch/2)
 *   polar Fourier data     Y[L][n_theta][C] complex64, FFT-ordered radial index k
 */
#ifndef TOMO_H
#define TOMO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TOMO_OK = 0,
  TOMO_EINVAL = -1,       /* bad argument or geometry                                */
  TOMO_ENOMEM = -2,       /* host or device allocation failed                        */
  TOMO_EHIP = -3,         /* a HIP runtime call failed                               */
  TOMO_EFFT = -4,         /* a rocFFT call failed                                    */
  TOMO_ESTATE = -5,       /* operator built without a device, or value type absent  */
  TOMO_EUNSUPPORTED = -6  /* valid request this build does not implement             */
} tomo_status;

/* Storage type of the sparse matrix values; accumulation is always float32. */
typedef enum { TOMO_VAL_F32 = 0, TOMO_VAL_BF16 = 1, TOMO_VAL_F16 = 2 } tomo_value_type;

/* Bit mask selecting which value arrays tomo_build_operator keeps on the device. */
#define TOMO_VALUES_F32 (1u << 0)
#define TOMO_VALUES_BF16 (1u << 1)
#define TOMO_VALUES_F16 (1u << 2)

/* Diagonal D of Eq. (2) (Sec. 3: Ram-Lak, Shepp-Logan, Hamming), applied per
 * polar radial index k: D_k = W_k * sum_m h(m) exp(-2 pi i k m / L) with the
 * band-limited ramp h(0) = 1/4, h(odd m) = -1/(pi m)^2, h(even m) = 0 over the
 * circle m in [-L/2, L-1-L/2], and window W = 1, sinc(k/L) or
 * 0.54 + 0.46 cos(2 pi k / L). */
typedef enum {
  TOMO_FILTER_NONE = 0,
  TOMO_FILTER_RAMLAK = 1,
  TOMO_FILTER_SHEPP = 2,
  TOMO_FILTER_HAMMING = 3,
  TOMO_FILTER_DENSITY = 4   /* tomo_irradon only: per-polar-sample weights from
                               tomo_density_filter (Sec. 3 density filter)                    */
} tomo_filter;

/* Experimental parameters of the setup stage (Sec. 3.1: number of pixels, angles,
 * detector bins, and the choice of filters and kernels). */
typedef struct {
  int32_t n;             /* image is n x n pixels (pixel size 1)                          */
  int32_t n_angles;      /* n_theta                                                        */
  int32_t n_det;         /* n_p detector bins (bin size 1)                                 */
  int32_t grid;          /* G = L, Cartesian grid side and polar samples per angle;
                            0 -> n_det.  Must satisfy grid >= max(n, n_det).               */
  int32_t kw;            /* kernel width k_w (odd, 1..15); 0 -> 3 (Fig. 3's stencil)       */
  int32_t max_batch;     /* largest batch (real slices) any call will pass, 1..256         */
  uint32_t values;       /* TOMO_VALUES_* mask; 0 -> TOMO_VALUES_F32                      */
  int32_t reserved;      /* must be 0                                                      */
  double beta;           /* Kaiser-Bessel shape; NaN -> Beatty et al. (2005) rule with
                            oversampling G / n                                             */
  double center;         /* rotation-axis bin c; NaN -> floor(n_det / 2) (Sec. 3, c = n_p/2).
                            c = c0 + f: the integer part c0 shifts the bins, a fractional
                            part f multiplies polar frequency k by exp(-2 pi i k f / L)
                            before the inverse detector DFT (and its conjugate after the
                            forward one), k signed in [-L/2, L/2)                          */
  const double* angles;  /* host array [n_angles] of radians, or NULL -> a * pi / n_angles */
} tomo_geometry;

typedef struct tomo_op tomo_op;

typedef struct {
  int32_t n, n_angles, n_det, grid, kw, max_batch;
  double beta, center;
  int64_t n_polar;        /* N = n_angles * grid rows of S^dagger                    */
  int64_t n_cart;         /* M = grid * grid rows of S                                */
  int64_t nnz;            /* stored entries (same in both CSR copies)                */
  int64_t cols_touched;   /* distinct Cartesian points referenced by S^dagger         */
  int64_t polar_nonempty; /* polar rows with at least one entry                       */
  int64_t adj_sell_rows;   /* S rows held in the sliced-ELL layout                   */
  int64_t adj_sell_padding;/* padding entries of that layout                          */
  int64_t adj_medium_rows; /* S rows processed one wavefront per row                  */
  int64_t adj_long_rows;   /* S rows split into chunks                                */
  int64_t adj_long_chunks; /* chunks (partial sums) used for the long rows            */
  int32_t device;         /* -1 for a host-only operator                             */
  uint32_t values;        /* value arrays present on the device                      */
} tomo_op_info;

/* Kernel layout parameters of the two SpMMs: the search space of an autotuner.
 * Staged kernels are used when their LDS footprint fits 64 KiB (and for k_w 3 or 5), else the
 * row kernels.
 * Defaults (in field order): 2, 4, 64, 4096, 256, 1024, 7, 7, 8, 64, 128, 1, 8192, 1024, 2, 1, 1, 1, 32, 0, 8, 1. */
typedef struct {
  int32_t fwd_channels_per_lane;  /* complex channels per lane in the forward SpMM: 1, 2 or 4
                                     (reduced automatically when it does not divide C)        */
  int32_t adj_channels_per_lane;  /* same for the adjoint SpMM                                */
  int32_t adj_sell_max;           /* S rows with <= this many entries use the sliced-ELL
                                     layout (8 rows per slice); 0..1024                        */
  int32_t adj_sell_sigma;         /* those rows are sorted by length within windows of this
                                     many rows (>= 1; 1 = natural order)                       */
  int32_t adj_medium_max;         /* longer rows up to this many entries: one wavefront each  */
  int32_t adj_chunk;              /* rows above that: chunks of this many entries (8..8192)   */
  int32_t fwd_tiled;              /* value-type bit mask (1 f32, 2 bf16, 4 f16): forward SpMM
                                     stages Cartesian tiles (+ halo) and the tile's sample
                                     records in LDS; clear bit: one lane group per row with
                                     every tap gathered from L2                                */
  int32_t adj_tiled;              /* value-type bit mask: adjoint SpMM stages, per output tile,
                                     the polar samples whose windows reach it in LDS, and runs
                                     the row kernels on the cells of tiles with too many
                                     samples; clear bit: the row-binned layouts for every cell */
  int32_t tile;                   /* Cartesian tile side of the staged kernels: 8 or 16        */
  int32_t tile_points;            /* forward: samples per block (32, 64, 96 or 128)            */
  int32_t adj_tile_points;        /* adjoint: most samples a staged tile may hold (multiple of
                                     32 in [32, 256]); denser tiles go to the row kernels     */
  int32_t normal_tiled;           /* normal operator: 1 stages each channel's grid tile (+ halo)
                                     in LDS; 0 reads every stencil tap through L1/L2           */
  int32_t adj_sell_xcd_rows;      /* sliced-ELL adjoint kernel: its blocks go to the 8 XCDs in runs
                                     covering this many consecutive rows (0 = one contiguous
                                     range per XCD; 1 = dispatch order); 0..2^24                */
  int32_t adj_medium_xcd_rows;    /* the same for the one-wavefront-per-row kernel           */
  int32_t fwd_rows_per_group;     /* forward SpMM (3x3 stencil, >= 8 lanes per row): rows one lane
                                     group handles in a software pipeline (1, 2 or 4)           */
  int32_t det_fft;                /* detector-direction DFTs of project / backproject: one fused
                                     kernel per direction (crop / pad + radix-8 DFT in LDS, other
                                     lengths through Bluestein's identity) on channel-slowest
                                     rows.  1 = backproject's kernel writes the adjoint SpMM's
                                     channel-fastest polar layout itself when the transform length
                                     is at most 4096 (else as 2); 2 = it writes channel-slowest
                                     rows, then a tiled transpose; 0 = rocFFT                   */
  int32_t grid_fft;               /* Cartesian 2D DFTs: 1 = hand-written row and column kernels
                                     fused with the embed / crop steps (power-of-two sides
                                     directly, others through Bluestein's identity); 0 = rocFFT */
  int32_t adj_sell_tiles;         /* order of the sliced-ELL rows: 1 = Cartesian cells in 4 x 8
                                     tiles (a block's rows are neighbouring cells, which share
                                     most of their gathered polar rows); 0 = grid order, sorted
                                     by length within adj_sell_sigma windows                   */
  int32_t tile_strip;             /* order in which the staged kernels visit their tiles: strips
                                     this many tiles wide, each walked tile row by tile row, so
                                     that a tile's neighbours above and below were visited a
                                     strip width earlier and their shared halo samples are still
                                     in the XCD's L2 (0 = row-major over the whole grid); results
                                     do not depend on it; 0..4096                              */
  int32_t adj_dense_mode;         /* staged adjoint, tiles whose region holds more than
                                     adj_tile_points samples (near the Fourier origin), in the
                                     channel-fastest entry points: 0 = the row kernels on their
                                     cells (on two more streams); 1 = staged too, in chunks of
                                     <= adj_tile_points samples, one block per segment of
                                     <= adj_seg_chunks chunks accumulating in registers (a tile
                                     with several segments is summed from partial tiles in a
                                     fixed order), on a second stream beside the other tiles;
                                     2 = the same segments and the other tiles in one launch, the
                                     dense segments first.  Backproject (which writes the FFT
                                     side's channel-slowest grid) and stacks always use the
                                     segments (1 for 0), and so do channel counts the row
                                     kernels cannot take (odd, above 64)                      */
  int32_t adj_seg_chunks;         /* chunks per segment of a dense tile (1..256)             */
  int32_t adj_run;                /* adj_dense_mode 2: the other staged tiles go to blocks in runs
                                     of this many tiles (in the visiting order), each block
                                     loading the next tile while it sums the current one
                                     (1..256)                                                 */
} tomo_tuning;

/* Solver selection and options for tomo_solve (Sec. 2.1; Sec. 3.1 lists SIRT and CGLS). */
typedef enum {
  TOMO_SOLVE_CGLS = 0,           /* CGLS on A (Sec. 3.1)                                        */
  TOMO_SOLVE_SIRT_BB = 1,        /* SIRT, preconditioner D, Barzilai-Borwein steps (Sec. 3.1)  */
  TOMO_SOLVE_CGNR = 2,           /* CG on A^T A x = A^T b with A^T A from tomo_normal (Sec. 4,
                                    Toeplitz approach); needs n_det == grid                   */
  TOMO_SOLVE_SIRT_BB_NORMAL = 3, /* SIRT_BB with A^T_D A from tomo_normal; needs n_det == grid */
  TOMO_SOLVE_TV_SPLIT_BREGMAN = 4 /* min (tv_mu/2)|A x - b|^2 + sum |D x| (isotropic TV, forward
                                    differences) by split Bregman (Sec. 3.1): refine_outer
                                    Bregman steps of `iters` CG steps each on
                                    (mu A^T A + lambda D^T D) x = mu A^T b + lambda D^T (d - e),
                                    then d = shrink(D x + e, 1/lambda), e = D x + e - d;
                                    A^T A from tomo_normal when n_det == grid              */
} tomo_solver;

typedef struct {
  int32_t method;         /* tomo_solver                                                    */
  int32_t iters;          /* iterations per outer step (>= 0)                               */
  int32_t refine_outer;   /* R >= 1 outer refinement steps; 1 = plain solve.  With R > 1 each
                             outer step forms r = b - A_f32 x with float32 values and solves
                             A_values d = r from zero with `iters` inner iterations.         */
  int32_t values;         /* tomo_value_type of the (inner) operator                        */
  int32_t filter;         /* tomo_filter preconditioner D for SIRT_BB (NONE -> HAMMING)     */
  int32_t use_x0;         /* CGLS only: start from the contents of x instead of zero        */
  double* out_resnorm;    /* device [batch] float64 or NULL: |b - A x|_2 per slice at exit   */
  double tv_mu;           /* TV_SPLIT_BREGMAN: data weight mu > 0                            */
  double tv_lambda;       /* TV_SPLIT_BREGMAN: splitting penalty lambda > 0                  */
} tomo_solve_opts;

/* Build the operator for geometry `g` (Sec. 3.1 setup stage): the CSR matrices S^dagger
 * and S in float64 on the host (COO -> zero / out-of-band removal -> CSR, Sec. 3.1),
 * the deapodisation factors, the row bins of S, then the device copies in the
 * requested value types.  `device` is a HIP device ordinal, or -1 for a host-only
 * operator (no HIP call is made; only tomo_op_info and tomo_export_* work on it).
 * The device that is current on entry is current again on return.
 * On success *out owns all device memory; free it with tomo_destroy_operator.
 * Errors: TOMO_EINVAL (geometry), TOMO_ENOMEM, TOMO_EHIP; *out is left NULL. */
tomo_status tomo_build_operator(const tomo_geometry* g, int device, tomo_op** out);

/* Forward projection y = A x (Eq. (2), first line) for `batch` slices.
 * x: device [batch][n][n] f32 (read).  y: device [batch][n_theta][n_det] f32 (written).
 * `values` picks the matrix value type (must have been built).  x and y must not overlap. */
tomo_status tomo_project(tomo_op* op, const float* x, float* y, int32_t batch,
                         int32_t values, void* stream);

/* Back-projection x = A^T y, the exact transpose of tomo_project (D = identity).
 * y: device [batch][n_theta][n_det] f32 (read).  x: device [batch][n][n] f32 (written). */
tomo_status tomo_backproject(tomo_op* op, const float* y, float* x, int32_t batch,
                             int32_t values, void* stream);

/* iRadon / filtered back-projection (Eq. (2), second line), scaled as
 * x = (pi / n_theta) A^T_D y with D = `filter` (TOMO_FILTER_NONE is rejected); with
 * TOMO_FILTER_DENSITY, x = (L / G^2) A^T Diag(D_v) y with the weights of tomo_density_filter
 * (TOMO_ESTATE if they were not computed). */
tomo_status tomo_irradon(tomo_op* op, const float* y, float* x, int32_t batch,
                         int32_t values, int32_t filter, void* stream);

/* The slicing interpolation alone (Sec. 2.2: the key step), as CSR SpMM over
 * C = ceil(batch/2) complex channels:  Yp = S^dagger Xc.
 * Xc: device [G*G][C] complex64 (read, FFT-ordered Cartesian Fourier grid).
 * Yp: device [L*n_theta][C] complex64 (written, row = k_fft * n_theta + angle). */
tomo_status tomo_slice_fwd(tomo_op* op, const float* Xc, float* Yp, int32_t batch,
                           int32_t values, void* stream);

/* Adjoint slicing Xc = S diag(D) Yp, row-binned and atomic-free; D per polar
 * column from `filter` (TOMO_FILTER_NONE -> identity).  Layouts as tomo_slice_fwd. */
tomo_status tomo_slice_adj(tomo_op* op, const float* Yp, float* Xc, int32_t batch,
                           int32_t values, int32_t filter, void* stream);

/* Iterative reconstruction of `batch` slices from sinograms b (Sec. 2.1 least
 * squares; CGLS or SIRT with BB steps, Sec. 3.1).  Per-slice scalars are reduced in
 * float64 on the device; nothing is copied to the host.
 * b: device [batch][n_theta][n_det] f32 (read).  x: device [batch][n][n] f32
 * (written; read first when opts->use_x0).  The first call with a new batch width
 * allocates the solver's device vectors (kept until tomo_destroy_operator). */
tomo_status tomo_solve(tomo_op* op, const float* b, float* x, int32_t batch,
                       const tomo_solve_opts* opts, void* stream);

/* Normal operator out = A^T D A x for `batch` slices in one pass of the Cartesian grid (Sec. 4:
 * the Toeplitz approach, the transform combined with its adjoint without the two 1D FFTs).
 * Exact for this discretisation when n_det == grid (L) and the centre is an integer: then
 *   A^T D A x = (1/L) k* . F2D^H W F2D (k* . x),   W = S diag(D) S^dagger,
 * and W is a fixed (2kw-1)^2 stencil of weights per Cartesian frequency (no column indices).
 * filter: tomo_filter, D in the polar domain (TOMO_FILTER_NONE: A^T A).  `values` selects the
 * matrix whose normal operator is applied: with 16-bit values it is A_v^T D A_v for the forward
 * operator A_v with S's values rounded to that type (the composition of tomo_project and
 * tomo_backproject with those values), its W = S_v diag(D) S_v^dagger formed in float64 and
 * stored in float32, which keeps it positive semidefinite.  The first call per filter builds W on
 * the host in float64 for every value type the operator holds and uploads it (synchronous; kept
 * until tomo_destroy_operator).
 * x: device [batch][n][n] f32 (read); out: device [batch][n][n] f32 (written), 16-byte aligned.
 * Errors: as tomo_project, plus TOMO_EUNSUPPORTED (n_det != grid, or kw > 5). */
tomo_status tomo_normal(tomo_op* op, const float* x, float* out, int32_t batch, int32_t values,
                        int32_t filter, void* stream);

/* Host copy of the normal-operator stencil W = S diag(D) S^dagger for `filter`: w is a host
 * array [grid*grid][(2kw-1)^2] (float64, FFT-ordered Cartesian rows j = j1*G + j2), entry
 * (d1 + R)(2R+1) + (d2 + R) of row j the weight of frequency ((j1+d1) mod G, (j2+d2) mod G),
 * R = kw - 1.  Recomputed on every call (host only, also for host-only operators).
 * Errors: TOMO_EINVAL, TOMO_EUNSUPPORTED (n_det != grid, or kw > 5). */
tomo_status tomo_export_normal(const tomo_op* op, int32_t filter, double* w);

/* Smoothed isotropic total variation of `batch` n x n images and its gradient: the
 * regularisation term mu * Reg(u) of the model-based problem (Sec. 2, Reg = the total-variation
 * norm).  The paper fixes no discretisation; this one uses forward differences with a zero
 * difference past the last row and column,
 *   TV_eps(u) = sum over pixels of sqrt((u[i1+1][i2]-u[i1][i2])^2 + (u[i1][i2+1]-u[i1][i2])^2 + eps).
 * x:     device [batch][n][n] f32, n = the operator's image size (read).
 * grad:  device [batch][n][n] f32 or NULL: overwritten with weight * dTV_eps/dx (float32 math).
 * value: device [batch] f64 or NULL: overwritten with weight * TV_eps per slice (float64 sums
 *        in a fixed order: bitwise reproducible).
 * eps > 0 and finite; weight finite.  The first call with value != NULL allocates a small
 * reduction buffer owned by the operator; calls on one operator must not overlap.
 * Errors: TOMO_EINVAL (NULL op/x, batch outside [0, max_batch], eps, weight, misaligned
 * pointers), TOMO_ESTATE (host-only operator), TOMO_ENOMEM, TOMO_EHIP. */
tomo_status tomo_tv(tomo_op* op, const float* x, int32_t batch, double eps, double weight,
                    float* grad, double* value, void* stream);

/* tomo_tv for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same kernels and results, bit for bit,
 * with the per-(slice, block) float64 reduction partials in a file-scope device array of the
 * library instead of a buffer the operator allocates on first use.  Allocates nothing (no
 * hipMalloc, hipFree or allocating library call); the caller passes x, grad and value as for
 * tomo_tv.  Limit: batch * min(256, ceil(n*n / 256)) <= 65536 partials (512 KiB, held by each GPU
 * the library runs on until the process ends); every batch an operator accepts fits, and larger
 * requests return TOMO_EINVAL.  The array is shared by every call on one GPU (each call writes
 * every partial it reads, so nothing needs clearing): calls that overlap on one GPU, from any
 * operator or stream, race.  The first call on a device looks up the array's device address
 * (hipGetSymbolAddress).  Errors: as tomo_tv, plus TOMO_EHIP if that lookup fails. */
tomo_status tomo_tv_noalloc(const tomo_op* op, const float* x, int32_t batch, double eps,
                            double weight, float* grad, double* value, void* stream);

/* Sizes and statistics of a built operator (host only, no synchronisation). */
tomo_status tomo_op_info_get(const tomo_op* op, tomo_op_info* out);

/* Copy a CSR matrix to host arrays in float64 (test hook; no device access).
 * which = 0: S^dagger, rows = k_fft * n_theta + angle (N + 1 row pointers),
 *            columns = j1_fft * G + j2_fft;
 * which = 1: S, the exact transpose (M + 1 row pointers).
 * rowptr: int64 [rows + 1]; col: int32 [nnz]; val: float64 [nnz].  Any may be NULL. */
tomo_status tomo_export_csr(const tomo_op* op, int32_t which, int64_t* rowptr, int32_t* col,
                            double* val);

/* Copy the separable deapodisation factors kd[n] (k*(i1,i2) = kd[i1] kd[i2]) and,
 * when filt != NULL, the diagonal D for `filter` per FFT-ordered radial index [L]. */
tomo_status tomo_export_factors(const tomo_op* op, int32_t filter, double* kd, double* filt);

/* Read the current kernel layout parameters. */
tomo_status tomo_get_tuning(const tomo_op* op, tomo_tuning* out);

/* Change the kernel layout parameters.  Changing the adjoint bin parameters rebuilds that
 * layout on the host and re-uploads it, synchronising the device; results do not depend on
 * the parameters except through float32 summation order.  Errors: TOMO_EINVAL (out of range;
 * the operator is unchanged), TOMO_ENOMEM. */
tomo_status tomo_set_tuning(tomo_op* op, const tomo_tuning* t);

/* Autotuner: search the SpMM layout parameters for `batch` slices with value type `values` by
 * timing tomo_slice_fwd / tomo_slice_adj on the operator's own work buffers (hashed inputs;
 * HIP events on a private stream), one parameter at a time over short candidate lists
 * (staged or row kernels per value type, tile side and capacities, tile visiting order, the
 * staged adjoint's dense-tile form, segment length and tile runs; forward rows per group and
 * channels per lane; adjoint channels per lane, sliced-ELL and wave-per-row bounds, XCD
 * interleave runs), `rounds` passes (1..8).  The fastest setting is
 * applied to the operator and returned in *best (nullable), with its times in *fwd_ms /
 * *adj_ms (nullable).  Synchronises the device; results of the operator do not depend on the
 * tuning except through float32 summation order.  Overwrites the operator's work buffers, so
 * it must not overlap other calls on the operator.  Errors: TOMO_EINVAL, TOMO_ESTATE,
 * TOMO_ENOMEM, TOMO_EHIP. */
tomo_status tomo_autotune(tomo_op* op, int32_t batch, int32_t values, int32_t rounds,
                          tomo_tuning* best, double* fwd_ms, double* adj_ms);

/* Several operators' work recorded as one HIP graph (stream capture), for stacks of slices of
 * different sizes: each step is one operation of one operator on caller buffers.  Creating the
 * graph runs every step once eagerly (creating FFT plans and normal-operator stencils on first
 * use), then records the same launches; tomo_graph_launch replays them in order with one call.
 * The graph holds the pointers given here: the buffers must stay allocated and the operators
 * alive (and not re-tuned) while the graph is used; replays read the buffers' current
 * contents.  Steps of one operator share its work buffers, so graph replays must not overlap
 * other calls on those operators.  All operators must be on one device. */
typedef enum {
  TOMO_STEP_SPMM_PAIR = 0,     /* in = Xc (cart layout) -> out = Yp (polar) -> aux = Xc' (cart):
                                  tomo_slice_fwd then tomo_slice_adj                          */
  TOMO_STEP_PROJECT = 1,       /* in = x -> out = y (tomo_project)                           */
  TOMO_STEP_BACKPROJECT = 2,   /* in = y -> out = x (tomo_backproject)                       */
  TOMO_STEP_NORMAL = 3         /* in = x -> out = A^T A x (tomo_normal, no filter)            */
} tomo_step_kind;

typedef struct {
  tomo_op* op;
  int32_t kind;          /* tomo_step_kind                                                  */
  int32_t batch;         /* slices (>= 1, <= the operator's max_batch)                     */
  int32_t values;        /* tomo_value_type                                                 */
  int32_t reserved;
  const float* in;       /* device, 16-byte aligned                                         */
  float* out;            /* device, 16-byte aligned                                         */
  float* aux;            /* device, 16-byte aligned; TOMO_STEP_SPMM_PAIR only               */
} tomo_step;

typedef struct tomo_graph tomo_graph;

/* Errors: TOMO_EINVAL (bad step, mixed devices), TOMO_ESTATE, TOMO_EUNSUPPORTED, TOMO_EHIP,
 * TOMO_EFFT; *out is NULL on error. */
tomo_status tomo_graph_create(const tomo_step* steps, int32_t n, tomo_graph** out);
/* Replay on `stream` (a hipStream_t; NULL = the null stream).  Errors: TOMO_EINVAL, TOMO_EHIP. */
tomo_status tomo_graph_launch(tomo_graph* g, void* stream);
/* Free the graph (NULL is a no-op); does not synchronise. */
void tomo_graph_destroy(tomo_graph* g);

/* Persistent SpMM pairs over a stack of operators (uneven stacks, Sec. 3.1: slices in batches,
 * one setup per geometry): item i computes out_i = S_i^dagger in_i, then aux_i = S_i out_i, like
 * TOMO_STEP_SPMM_PAIR, for its operator and batch.  A launch runs one forward kernel whose blocks
 * walk a device work list of (item, staged work item, channel chunk) and one adjoint kernel over
 * (item, segment, channel chunk) with the operators' dense-tile segments first (longest first),
 * then one small kernel that sums split dense tiles; nothing else (no allocation, copy or memset),
 * so a launch may be captured in a HIP graph.  Results equal the items' own tomo_slice_fwd /
 * tomo_slice_adj with the staged kernels, up to float32 summation order.
 * Requirements: operators on one device, one kernel width and tile side, the staged layouts
 * (k_w 3 or 5, tile 8 or 16), value type `values` built for every
 * operator.  Buffers as tomo_slice_fwd / tomo_slice_adj (in: [G*G][C], out: [L*nt][C],
 * aux: [G*G][C] complex64, C = ceil(batch/2), 16-byte aligned); the stack holds the pointers, so
 * they and the operators must stay alive (and not be re-tuned) while it is used.  Launches of one
 * stack, and calls on its operators, must not overlap.  tomo_stack_create allocates the work
 * lists and each item's partial tiles (synchronous).
 * Errors: TOMO_EINVAL (bad item, mixed devices / kernel widths / tiles),
 * TOMO_ESTATE, TOMO_EUNSUPPORTED (no staged layout), TOMO_ENOMEM, TOMO_EHIP. */
typedef struct {
  tomo_op* op;
  int32_t batch;         /* slices (1 .. the operator's max_batch)                          */
  int32_t reserved;      /* must be 0                                                        */
  const float* in;
  float* out;
  float* aux;
} tomo_stack_item;

typedef struct tomo_stack tomo_stack;

tomo_status tomo_stack_create(const tomo_stack_item* items, int32_t n, int32_t values,
                              tomo_stack** out);
/* Enqueue the stack's kernels on `stream` (a hipStream_t; NULL = the null stream). */
tomo_status tomo_stack_launch(tomo_stack* s, void* stream);
/* Free the stack (NULL is a no-op); does not synchronise. */
void tomo_stack_destroy(tomo_stack* s);

/* Density filter (Sec. 3): per-polar-sample weights D_v ~ arg min ||S D_v - c 1|| over the
 * Cartesian grid, c = kappa(0)^2 the mass of the separable gridding kernel, among weights even
 * in the frequency (D_v(k, a) = D_v(-k, a), which keeps the filtered back projection of a real
 * sinogram real), by `iters` (1..100000) CGLS steps from zero with the float32 matrix values
 * (float32 vectors, float64 dots; the least-squares problem is rank deficient, so the weights
 * are defined by this iteration).  Kept in the operator for TOMO_FILTER_DENSITY, replacing
 * earlier weights; *resid (nullable) receives ||S D_v - c 1||_2 from the iteration's residual.
 * Synchronises the device and uses temporary device memory.  Errors: TOMO_EINVAL (NULL op,
 * iters out of range), TOMO_ESTATE (no device, no float32 values), TOMO_ENOMEM, TOMO_EHIP. */
tomo_status tomo_density_filter(tomo_op* op, int32_t iters, double* resid);

/* Host copy of the density weights: w [L * n_theta] float32, FFT-ordered polar rows
 * (k_fft * n_theta + a).  TOMO_ESTATE if they were not computed. */
tomo_status tomo_export_density(const tomo_op* op, float* w);

/* Host self-check (no device access): rebuild every kernel layout for the current tuning on
 * the host, apply each one in float64 following the kernels' traversal, and report the largest
 * relative difference from the CSR products in *max_rel_err (about 1e-16 when correct; NaN if
 * some output row would not be written). */
tomo_status tomo_check_layouts(const tomo_op* op, double* max_rel_err);

/* Free everything the operator owns (synchronises its device first).  NULL is a no-op. */
void tomo_destroy_operator(tomo_op* op);

/* Thread-local message describing the last error in this thread ("" if none). */
const char* tomo_last_error(void);

/* Library version string, e.g. "1.0.0". */
const char* tomo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TOMO_H */
