// Autotuner: times a small grid of launch parameters of the fused kernels on the plan itself
// and keeps the fastest (lanes per CSR row for SpMV; the plain baseline gets the same
// treatment so comparisons are against a tuned CSR kernel).
#include <algorithm>

#include "plan.h"

namespace sable {

namespace {

template <class F>
float time_ms(F&& f, hipStream_t s, int reps) {
  hipEvent_t a, b;
  HIPC(hipEventCreate(&a));
  HIPC(hipEventCreate(&b));
  f();  // warm
  HIPC(hipEventRecord(a, s));
  for (int r = 0; r < reps; ++r) f();
  HIPC(hipEventRecord(b, s));
  HIPC(hipEventSynchronize(b));
  float ms = 0.f;
  HIPC(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

}  // namespace

void autotune(sable_plan_s& P, int op, int n, const float* x, float* y, hipStream_t s) {
  const int reps = 10;
  if (op == 0) {
    float best = 1e30f;
    int bv = 0;
    for (int v = 0; v <= 10; ++v) {
      P.prm.spmv_variant = v;
      float t = time_ms([&] { launch_spmv(P, x, y, s); }, s, reps);
      if (t < best) { best = t; bv = v; }
    }
    P.prm.spmv_variant = bv;
    if (P.far.npanel && (bv <= 2 || bv >= 8)) {
      P.prm.far_split = 0;
      const float t0 = time_ms([&] { launch_spmv(P, x, y, s); }, s, reps);
      P.prm.far_split = 1;
      const float t1 = time_ms([&] { launch_spmv(P, x, y, s); }, s, reps);
      P.prm.far_split = t1 <= t0 ? 1 : 0;
    }
    best = 1e30f;
    bv = 0;
    for (int v = 0; v <= 12; ++v) {
      P.prm.plain_variant = v;
      float t = time_ms([&] { launch_spmv_plain(P, x, y, s); }, s, reps);
      if (t < best) { best = t; bv = v; }
    }
    P.prm.plain_variant = bv;
  } else {
    // x / y hold X (ncols x n) and Y (nrows x n)
    float best = 1e30f;
    int bm = 0;
    for (int m = 0; m <= 2; ++m) {
      P.prm.spmm_mode = m;
      float t = time_ms([&] { launch_spmm(P, x, y, n, s); }, s, 3);
      if (t < best) { best = t; bm = m; }
    }
    P.prm.spmm_mode = bm;
  }
  HIPC(hipStreamSynchronize(s));
}

}  // namespace sable

extern "C" sable_status sable_autotune(sable_plan_t p, int32_t op, int32_t n, const float* x,
                                       float* y, void* stream) {
  sable::clear_error();
  try {
    if (!p || (op != 0 && op != 1) || n < 1 || (!x && p->ncols) || (!y && p->nrows)) {
      sable::set_error("bad argument");
      return SABLE_ERR_INVALID_ARG;
    }
    if (p->nrows == 0) return SABLE_OK;
    sable::autotune(*p, op, n, x, y, (hipStream_t)stream);
    return SABLE_OK;
  } catch (const sable::Err& e) {
    return e.st;
  } catch (...) {
    return SABLE_ERR_INTERNAL;
  }
}

extern "C" sable_status sable_plan_set_variant(sable_plan_t p, int32_t op, int32_t variant) {
  sable::clear_error();
  if (!p) {
    sable::set_error("NULL plan");
    return SABLE_ERR_INVALID_ARG;
  }
  const int maxv = op == 0 ? 10 : op == 1 ? 2 : op == 2 ? 12 : op == 3 ? 1 : -1;
  if (variant < 0 || variant > maxv) {
    sable::set_error("variant %d out of range for op %d", variant, op);
    return SABLE_ERR_INVALID_ARG;
  }
  if (op == 0) p->prm.spmv_variant = variant;
  else if (op == 1) p->prm.spmm_mode = variant;
  else if (op == 2) p->prm.plain_variant = variant;
  else p->prm.far_split = variant;
  return SABLE_OK;
}
