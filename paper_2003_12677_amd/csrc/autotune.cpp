// Autotuner for the SpMM layout parameters (the tomo_tuning search space): times the forward and
// adjoint SpMMs for one batch width and value type on the operator's own work buffers (filled
// with hashed values), and walks the parameters one at a time (coordinate descent), keeping
// whichever setting is fastest: staged or row kernels for this value type, tile shapes and
// capacities, row bins, channels per lane and XCD interleave.  Row-bin and tile parameters
// change host layouts, so each of their candidates costs a re-layout and upload; the search
// therefore visits a short list per parameter.

#include <algorithm>
#include <functional>
#include <vector>

#include "internal.h"

namespace tomo {
namespace {

struct Timer {
  hipStream_t st = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (st) (void)hipStreamDestroy(st);
  }
};

// average milliseconds of `reps` launches, best of three trials, after two warm-up launches
template <typename F>
tomo_status time_ms(Timer& tm, F launch, int reps, double* out) {
  for (int w = 0; w < 2; ++w) TOMO_TRY(launch());
  double best = 1e30;
  for (int trial = 0; trial < 3; ++trial) {
    TOMO_HIP(hipEventRecord(tm.a, tm.st));
    for (int r = 0; r < reps; ++r) TOMO_TRY(launch());
    TOMO_HIP(hipEventRecord(tm.b, tm.st));
    TOMO_HIP(hipEventSynchronize(tm.b));
    float ms = 0.f;
    TOMO_HIP(hipEventElapsedTime(&ms, tm.a, tm.b));
    best = std::min(best, (double)ms / reps);
  }
  *out = best;
  return TOMO_OK;
}

}  // namespace

tomo_status autotune(tomo_op* op, int batch, int vt, int rounds, double* fwd_ms, double* adj_ms) {
  const Geom& g = op->g;
  const int C = (batch + 1) / 2;
  Timer tm;
  TOMO_HIP(hipStreamCreate(&tm.st));
  TOMO_HIP(hipEventCreate(&tm.a));
  TOMO_HIP(hipEventCreate(&tm.b));
  TOMO_TRY(launch_fill_hash((float*)op->X, (int64_t)g.G * g.G * C * 2, 1u, tm.st));
  TOMO_TRY(launch_fill_hash((float*)op->Y, (int64_t)g.L * g.nt * C * 2, 2u, tm.st));
  const int reps = 10;
  auto fwd = [&] { return launch_spmm_fwd(op, op->X, op->Y, C, vt, tm.st); };
  auto adj = [&] { return launch_spmm_adj(op, op->Y, op->X, C, vt, nullptr, tm.st); };
  // every candidate is timed from the same inputs: the forward reads X and writes Y, so time the
  // adjoint (which reads Y) after refilling Y
  auto measure_fwd = [&](double* ms) { return time_ms(tm, fwd, reps, ms); };
  auto measure_adj = [&](double* ms) {
    TOMO_TRY(launch_fill_hash((float*)op->Y, (int64_t)g.L * g.nt * C * 2, 2u, tm.st));
    return time_ms(tm, adj, reps, ms);
  };

  Tuning best = op->tune;
  double bf = 0, ba = 0;
  TOMO_TRY(measure_fwd(&bf));
  TOMO_TRY(measure_adj(&ba));
  // which SpMM a parameter affects: the forward, the adjoint, or both (the shared tile side)
  enum Side { kFwd, kAdj, kBoth };
  struct Param {
    std::function<int&(Tuning&)> field;
    std::vector<int> values;
    Side side;
  };
  // the staged flags are value-type masks: the search sets or clears this value type's bit
  const int bit = 1 << vt;
  auto mask_values = [&](int cur) { return std::vector<int>{cur & ~bit, cur | bit}; };
  const std::vector<Param> params = {
      {[](Tuning& t) -> int& { return t.fwd_tiled; }, mask_values(best.fwd_tiled), kFwd},
      {[](Tuning& t) -> int& { return t.adj_tiled; }, mask_values(best.adj_tiled), kAdj},
      {[](Tuning& t) -> int& { return t.tile; }, {8, 16}, kBoth},
      {[](Tuning& t) -> int& { return t.tile_points; }, {32, 64, 96, 128}, kFwd},
      {[](Tuning& t) -> int& { return t.adj_tile_points; }, {64, 96, 128, 160, 192, 256}, kAdj},
      {[](Tuning& t) -> int& { return t.tile_strip; }, {0, 16, 32, 128}, kBoth},
      {[](Tuning& t) -> int& { return t.adj_dense_mode; }, {0, 1, 2}, kAdj},
      {[](Tuning& t) -> int& { return t.adj_seg_chunks; }, {2, 4, 8, 16}, kAdj},
      {[](Tuning& t) -> int& { return t.adj_run; }, {1, 4, 16}, kAdj},
      {[](Tuning& t) -> int& { return t.fwd_rows_per_group; }, {1, 2, 4}, kFwd},
      {[](Tuning& t) -> int& { return t.fwd_cpl; }, {1, 2, 4}, kFwd},
      {[](Tuning& t) -> int& { return t.adj_cpl; }, {1, 2, 4}, kAdj},
      {[](Tuning& t) -> int& { return t.sell_max; }, {8, 16, 24, 32, 48, 64, 96}, kAdj},
      {[](Tuning& t) -> int& { return t.medium_max; }, {64, 128, 256, 512}, kAdj},
      {[](Tuning& t) -> int& { return t.sell_sigma; }, {1, 64, 512, 4096, 16384}, kAdj},
      {[](Tuning& t) -> int& { return t.sell_tiles; }, {0, 1}, kAdj},
      {[](Tuning& t) -> int& { return t.chunk; }, {256, 512, 1024, 2048}, kAdj},
      {[](Tuning& t) -> int& { return t.sell_xcd_rows; }, {0, 1, 2048, 4096, 8192, 16384}, kAdj},
      {[](Tuning& t) -> int& { return t.medium_xcd_rows; }, {1, 256, 1024, 4096}, kAdj},
  };
  for (int round = 0; round < std::max(1, rounds); ++round) {
    for (const Param& p : params) {
      for (int v : p.values) {
        Tuning t = best;
        p.field(t) = v;
        if (v == p.field(best) || check_tuning(t) != TOMO_OK) continue;
        TOMO_TRY(apply_tuning(op, t));
        double f = bf, a = ba;
        // a setting the channel count rules out (row kernels with an odd count above 64) is
        // refused before launching anything: skip it
        if ((p.side != kAdj && measure_fwd(&f) != TOMO_OK) ||
            (p.side != kFwd && measure_adj(&a) != TOMO_OK)) {
          clear_error();
          continue;
        }
        if (f + a < bf + ba) {
          best = t;
          bf = f;
          ba = a;
        }
      }
      TOMO_TRY(apply_tuning(op, best));
    }
  }
  clear_error();
  TOMO_HIP(hipStreamSynchronize(tm.st));
  if (fwd_ms) *fwd_ms = bf;
  if (adj_ms) *adj_ms = ba;
  return TOMO_OK;
}

}  // namespace tomo
