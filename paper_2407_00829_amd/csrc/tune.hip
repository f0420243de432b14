// Autotuner: times a small grid of launch parameters of the fused kernels on the plan itself
// and keeps the fastest (lanes per CSR row for SpMV; the plain baseline gets the same
// treatment so comparisons are against a tuned CSR kernel).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "plan.h"

namespace sable {

namespace {

// Autotuning cache, process-wide: (structure hash, specialized kernel present, op, n,
// device) -> the chosen variants. A plan whose structure has been tuned before (the same
// matrix pattern, extractor list and thresholds, whatever the values) takes the stored choice
// without timing anything.
struct TuneChoice {
  int spmv_variant, far_split, plain_variant, spmm_mode;
};
typedef std::tuple<uint64_t, int, int, int, int> TuneKey;
std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune_cache;

template <class F>
float time_ms(F&& f, hipStream_t s, int reps) {
  hipEvent_t a, b;
  HIPC(hipEventCreate(&a));
  HIPC(hipEventCreate(&b));
  f();  // warm
  float r3[3];
  for (int round = 0; round < 3; ++round) {
    HIPC(hipEventRecord(a, s));
    for (int r = 0; r < reps; ++r) f();
    HIPC(hipEventRecord(b, s));
    HIPC(hipEventSynchronize(b));
    HIPC(hipEventElapsedTime(&r3[round], a, b));
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::sort(r3, r3 + 3);
  return r3[1] / reps;  // median of three rounds
}

// Index of the variant to keep: the lowest-numbered one within 2% of the fastest, so that
// near-ties resolve the same way from run to run.
int pick(const std::vector<float>& t) {
  const float best = *std::min_element(t.begin(), t.end());
  for (size_t v = 0; v < t.size(); ++v)
    if (t[v] <= 1.02f * best) return (int)v;
  return 0;
}

}  // namespace

void autotune(sable_plan_s& P, int op, int n, const float* x, float* y, hipStream_t s) {
  const int reps = 10;
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  const TuneKey key{P.structure_hash, P.spec_func != nullptr, op, op == 0 ? 1 : n, dev};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      if (op == 0) {
        P.prm.spmv_variant = it->second.spmv_variant;
        P.prm.far_split = it->second.far_split;
        P.prm.plain_variant = it->second.plain_variant;
      } else {
        auto& tuned = P.prm.spmm_tuned;
        tuned.erase(std::remove_if(tuned.begin(), tuned.end(),
                                   [&](const std::pair<int, int>& e) { return e.first == n; }),
                    tuned.end());
        P.prm.spmm_mode = it->second.spmm_mode;
        tuned.push_back({n, P.prm.spmm_mode});
      }
      return;
    }
  }
  if (op == 0) {
    std::vector<float> tp(18);
    for (int v = 0; v <= 17; ++v) {
      P.prm.plain_variant = v;
      tp[v] = time_ms([&] { launch_spmv_plain(P, x, y, s); }, s, reps);
    }
    P.prm.plain_variant = pick(tp);
    if (P.nseg == 0 && P.nblk == 0) {
      // a CSR-only plan runs its SpMV through the plain kernels (the variant just chosen);
      // only a run-time specialized kernel competes with them
      P.prm.far_split = 0;
      P.prm.spmv_variant = 0;
      if (P.spec_func) {
        const float tb = tp[P.prm.plain_variant];
        P.prm.spmv_variant = 11;
        const float t11 = time_ms([&] { launch_spmv(P, x, y, s); }, s, reps);
        if (!(t11 < tb / 1.02f)) P.prm.spmv_variant = 0;
      }
    } else {
      // hybrid SpMV: every variant without the far-column split, then every streamed variant
      // with it; candidates are ranked in that order, so the split is kept only where it is
      // more than 2% faster than every variant without it
      std::vector<float> t;
      std::vector<std::pair<int, int>> cand;  // (variant, far split)
      P.prm.far_split = 0;
      for (int v : {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 13, 14, 15, 16}) {
        P.prm.spmv_variant = v;
        t.push_back(time_ms([&] { launch_spmv(P, x, y, s); }, s, reps));
        cand.push_back({v, 0});
      }
      if (P.spec_func) {  // the run-time specialized kernel, ranked after the generic ones
        P.prm.spmv_variant = 11;
        t.push_back(time_ms([&] { launch_spmv(P, x, y, s); }, s, reps));
        cand.push_back({11, 0});
      }
      if (P.far.npanel) {
        P.prm.far_split = 1;
        for (int v : {0, 1, 2, 8, 9, 10, 15, 16}) {
          P.prm.spmv_variant = v;
          t.push_back(time_ms([&] { launch_spmv(P, x, y, s); }, s, reps));
          cand.push_back({v, 1});
        }
      }
      const int c = pick(t);
      P.prm.spmv_variant = cand[c].first;
      P.prm.far_split = cand[c].second;
    }
  } else {
    // x / y hold X (ncols x n) and Y (nrows x n); the choice is kept per n
    std::vector<float> t(5);
    auto& tuned = P.prm.spmm_tuned;
    tuned.erase(std::remove_if(tuned.begin(), tuned.end(),
                               [&](const std::pair<int, int>& e) { return e.first == n; }),
                tuned.end());
    for (int m = 0; m <= 4; ++m) {
      P.prm.spmm_mode = m;
      t[m] = time_ms([&] { launch_spmm(P, x, y, n, s); }, s, 2);
    }
    P.prm.spmm_mode = pick(t);
    tuned.push_back({n, P.prm.spmm_mode});
  }
  HIPC(hipStreamSynchronize(s));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = TuneChoice{P.prm.spmv_variant, P.prm.far_split, P.prm.plain_variant,
                                 P.prm.spmm_mode};
}

void autotune_cache_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache.clear();
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

extern "C" sable_status sable_autotune_cache_clear(void) {
  sable::clear_error();
  sable::autotune_cache_clear();
  return SABLE_OK;
}

extern "C" sable_status sable_plan_set_variant(sable_plan_t p, int32_t op, int32_t variant) {
  sable::clear_error();
  if (!p) {
    sable::set_error("NULL plan");
    return SABLE_ERR_INVALID_ARG;
  }
  const int maxv = op == 0 ? 16 : op == 1 ? 4 : op == 2 ? 17 : op == 3 ? 1 : -1;
  if (variant < 0 || variant > maxv) {
    sable::set_error("variant %d out of range for op %d", variant, op);
    return SABLE_ERR_INVALID_ARG;
  }
  if (op == 0 && variant == 11 && !p->spec_func) {
    sable::set_error("variant 11 needs sable_plan_specialize first");
    return SABLE_ERR_INVALID_ARG;
  }
  if (op == 0) p->prm.spmv_variant = variant;
  else if (op == 1) {
    p->prm.spmm_mode = variant;
    p->prm.spmm_tuned.clear();
  }
  else if (op == 2) p->prm.plain_variant = variant;
  else p->prm.far_split = variant;
  return SABLE_OK;
}
