// A stack of operators of different sizes (Sec. 3.1: slices processed in batches, one setup per
// geometry) run as persistent launches: the forward SpMMs of every (operator, batch) item as one
// kernel over a device work list of (item, staged work item, channel chunk), then the adjoint
// SpMMs as one kernel over (item, segment, channel chunk), the dense segments first, then the
// sums of the split dense tiles.  The work lists are built once; a launch enqueues three kernels
// and nothing else (no allocation, copy or memset), so it can be captured in a HIP graph.

#include <vector>

#include "internal.h"

struct tomo_stack {
  int device = -1;
  tomo::StackPlan* plan = nullptr;
};

using namespace tomo;

extern "C" {

tomo_status tomo_stack_create(const tomo_stack_item* items, int32_t n, int32_t values,
                              tomo_stack** out) {
  clear_error();
  if (!items || n < 1 || !out) return fail(TOMO_EINVAL, "need at least one item and an output");
  *out = nullptr;
  if (values < TOMO_VAL_F32 || values > TOMO_VAL_F16) return fail(TOMO_EINVAL, "bad value type %d", values);
  std::vector<StackItemSpec> spec;
  const int device = items[0].op ? items[0].op->device : -1;
  if (device < 0) return fail(TOMO_ESTATE, "stack items need device operators");
  for (int i = 0; i < n; ++i) {
    const tomo_stack_item& it = items[i];
    if (!it.op) return fail(TOMO_EINVAL, "item %d has no operator", i);
    if (it.op->device != device) return fail(TOMO_EINVAL, "all items must use operators of one device");
    if (it.reserved != 0) return fail(TOMO_EINVAL, "reserved field must be 0");
    if (it.batch < 1) return fail(TOMO_EINVAL, "item %d: batch must be >= 1", i);
    TOMO_TRY(check_apply(it.op, it.in, it.out, it.batch, values));
    if (!it.aux || ((uintptr_t)it.aux) % 16 != 0)
      return fail(TOMO_EINVAL, "item %d needs a 16-byte aligned aux buffer", i);
    if (!it.op->tiles_ready || !fwd_tile_supported(it.op) || !adj_tile_supported(it.op))
      return fail(TOMO_EUNSUPPORTED, "item %d: the staged layouts are not available", i);
    spec.push_back(StackItemSpec{it.op, it.batch, it.in, it.out, it.aux});
  }
  DeviceGuard guard(device);
  if (guard.err != hipSuccess) return fail(TOMO_EHIP, "hipSetDevice(%d) failed", device);
  StackPlan* plan = nullptr;
  TOMO_TRY(stack_plan_create(spec.data(), n, values, &plan));
  auto* s = new tomo_stack();
  s->device = device;
  s->plan = plan;
  *out = s;
  return TOMO_OK;
}

tomo_status tomo_stack_launch(tomo_stack* s, void* stream) {
  clear_error();
  if (!s || !s->plan) return fail(TOMO_EINVAL, "stack is NULL");
  DeviceGuard guard(s->device);
  return stack_plan_launch(s->plan, (hipStream_t)stream);
}

void tomo_stack_destroy(tomo_stack* s) {
  if (!s) return;
  DeviceGuard guard(s->device);
  stack_plan_destroy(s->plan);
  delete s;
}

}  // extern "C"
