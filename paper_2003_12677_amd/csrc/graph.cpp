// Multi-operator steps captured as one HIP graph: a list of (operator, operation, batch, value
// type, buffers) is run once eagerly (which creates FFT plans, normal-operator stencils and
// solver-free workspaces on first use), then the same launches are recorded by stream capture
// and instantiated, so a whole step over many operators of different sizes replays with one
// launch call.  Nothing in the recorded launch paths allocates, copies or synchronises, and
// none of them records a memset.

#include <vector>

#include "internal.h"

struct tomo_graph {
  int device = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace tomo {
namespace {

tomo_status run_step(const tomo_step& s, hipStream_t st) {
  tomo_op* op = s.op;
  const int C = (s.batch + 1) / 2;
  switch (s.kind) {
    case TOMO_STEP_SPMM_PAIR:
      TOMO_TRY(launch_spmm_fwd(op, (const float2*)s.in, (float2*)s.out, C, s.values, st));
      return launch_spmm_adj(op, (const float2*)s.out, (float2*)s.aux, C, s.values, nullptr, st);
    case TOMO_STEP_PROJECT:
      return apply_project(op, s.in, s.out, s.batch, s.values, st);
    case TOMO_STEP_BACKPROJECT:
      return apply_backproject(op, s.in, s.out, s.batch, s.values, TOMO_FILTER_NONE, 1.0f, st);
    case TOMO_STEP_NORMAL:
      return apply_normal(op, s.in, s.out, s.batch, s.values, TOMO_FILTER_NONE, st);
    default:
      return fail(TOMO_EINVAL, "unknown step kind %d", s.kind);
  }
}

tomo_status check_step(const tomo_step& s, int device) {
  if (!s.op) return fail(TOMO_EINVAL, "step without operator");
  if (s.op->device != device) return fail(TOMO_EINVAL, "all steps must use operators of one device");
  if (s.batch < 1) return fail(TOMO_EINVAL, "step batch must be >= 1");
  TOMO_TRY(check_apply(s.op, s.in, s.out, s.batch, s.values));
  if (s.kind == TOMO_STEP_SPMM_PAIR && (!s.aux || ((uintptr_t)s.aux) % 16 != 0))
    return fail(TOMO_EINVAL, "an SpMM pair needs a 16-byte aligned aux buffer");
  if (s.kind == TOMO_STEP_NORMAL) TOMO_TRY(normal_supported(s.op));
  return TOMO_OK;
}

}  // namespace
}  // namespace tomo

using namespace tomo;

extern "C" {

tomo_status tomo_graph_create(const tomo_step* steps, int32_t n, tomo_graph** out) {
  clear_error();
  if (!steps || n < 1 || !out) return fail(TOMO_EINVAL, "need at least one step and an output");
  *out = nullptr;
  const int device = steps[0].op ? steps[0].op->device : -1;
  if (device < 0) return fail(TOMO_ESTATE, "steps need device operators");
  for (int i = 0; i < n; ++i) TOMO_TRY(check_step(steps[i], device));
  DeviceGuard guard(device);
  hipStream_t st = nullptr;
  TOMO_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  tomo_status status = TOMO_OK;
  for (int i = 0; i < n && status == TOMO_OK; ++i) status = run_step(steps[i], st);   // warm-up
  if (status == TOMO_OK && hipStreamSynchronize(st) != hipSuccess)
    status = fail(TOMO_EHIP, "warm-up run failed");
  auto* g = new tomo_graph();
  g->device = device;
  if (status == TOMO_OK && hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
    status = fail(TOMO_EHIP, "hipStreamBeginCapture failed");
  if (status == TOMO_OK) {
    for (int i = 0; i < n && status == TOMO_OK; ++i) status = run_step(steps[i], st);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);   // always end the capture
    g->graph = graph;
    if (status == TOMO_OK && e != hipSuccess)
      status = fail(TOMO_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
  }
  if (status == TOMO_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
    status = fail(TOMO_EHIP, "hipGraphInstantiate failed");
  (void)hipStreamDestroy(st);
  if (status != TOMO_OK) {
    tomo_graph_destroy(g);
    return status;
  }
  *out = g;
  return TOMO_OK;
}

tomo_status tomo_graph_launch(tomo_graph* g, void* stream) {
  clear_error();
  if (!g || !g->exec) return fail(TOMO_EINVAL, "graph is NULL");
  DeviceGuard guard(g->device);
  TOMO_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return TOMO_OK;
}

void tomo_graph_destroy(tomo_graph* g) {
  if (!g) return;
  DeviceGuard guard(g->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
