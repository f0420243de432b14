// Batched persistent execution of many plans, captured in a hipGraph.
//
// Work units are (item, tile) pairs laid out item by item, in seven lists: SpMV items by
// streamed tile (three tile heights, with and without non-temporal loads) and SpMM items.
// One persistent kernel per non-empty list, each with a grid of every CU times its
// resident workgroups, pull units from their own atomic counter; a unit runs exactly the tile
// body of the standalone product, so each item's result is bitwise equal to its standalone
// launch with the same kernel (SpMV: the streamed tile of the plan's tuned streamed variant,
// 256, 512 or 1024 rows, with or without non-temporal loads, and the 256-row tile for the
// other variants; SpMM: the fused tile in the plan's matrix-core mode, the LDS-staged panel
// tile included). Keeping the lists apart lets each kernel run at the occupancy of its
// standalone kernel. The last unit of an item stamps the GPU wall clock. A reset kernel (no
// memset nodes) clears the counters and stamps the batch start; the kernels are captured
// once and replayed.
#include <algorithm>

#include "exec.h"
#include "spmm_panel.h"

namespace sable {

struct BatchItemDev {
  int op, n, mfma, units;
  int units_per_col, col_chunks;  // SpMM: row tiles x column chunks
  const float* x;
  float* y;
};

namespace {

constexpr int kBatchCounters = 7;  // one per work list

__global__ void k_batch_reset(unsigned* __restrict__ counter, unsigned* __restrict__ done,
                              const BatchItemDev* __restrict__ items, int count,
                              unsigned long long* __restrict__ stamps) {
  __shared__ unsigned long long t0;
  if (threadIdx.x == 0) {
    for (int k = 0; k < kBatchCounters; ++k) counter[k] = 0;
    t0 = wall_clock64();
    stamps[count] = t0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    done[i] = 0;
    if (items[i].units == 0) stamps[i] = t0;  // nothing to run: complete at the start
  }
}

constexpr int kBatchSpmmLds = kMmRows * kMmCols + kMmBlkStage * kBlkDesc;
static_assert(kBatchSpmmLds * 4 >= kPanLdsBytes, "the panel tile fits the SpMM units' LDS");

// Units of one list: list[k] is the item of the k-th entry, off[k] its first unit. OP 0: SpMV
// units of the streamed tile with RPT rows per thread (NT: non-temporal loads); OP 1: SpMM.
template <int OP, int RPT = 1, bool NT = false>
__device__ __forceinline__ void batch_units(const PlanView* __restrict__ views,
                                            const BatchItemDev* __restrict__ items,
                                            const int32_t* __restrict__ list,
                                            const i64* __restrict__ off, int nlist, i64 total,
                                            unsigned* __restrict__ counter,
                                            unsigned* __restrict__ done,
                                            unsigned long long* __restrict__ stamps, float* lds) {
  unsigned* unit = reinterpret_cast<unsigned*>(lds);  // broadcast slot, free between units
  for (;;) {
    __syncthreads();  // the previous unit is done with the LDS
    if (threadIdx.x == 0) unit[0] = atomicAdd(counter, 1u);
    __syncthreads();
    // uniform across the workgroup: scalar registers for the unit, its item and its view
    const i64 u = (i64)(unsigned)__builtin_amdgcn_readfirstlane((int)unit[0]);
    __syncthreads();  // every thread has read the slot before the unit body reuses it
    if (u >= total) break;
    int lo = 0, hi = nlist - 1;  // last list entry whose first unit is <= u
    while (lo < hi) {
      int m = (lo + hi + 1) >> 1;
      if (off[m] <= u) lo = m; else hi = m - 1;
    }
    const int it = list[lo];
    const BatchItemDev I = items[it];
    const PlanView& P = views[it];
    int local = (int)(u - off[lo]);
    if constexpr (OP == 0) {
      spmv_tile_stream<RPT, NT>(P, local, I.x, I.y, lds);  // local = launch slot
    } else {
      int rt = local % I.units_per_col;
      const int cc = local / I.units_per_col;
      if (P.tile_order) rt = P.tile_order[rt];
      if (I.mfma == 3) spmm_tile_panel(P, rt, cc * kMmCols, I.n, I.x, I.y, reinterpret_cast<uint8_t*>(lds));
      else spmm_tile(P, rt * kMmRows, cc * kMmCols, I.n, I.x, I.y, lds, I.mfma);
    }
    __syncthreads();
    // completion count only: nothing in the kernel reads another unit's output, so no
    // fence (on this chip a device-scope release writes back the whole L2)
    if (threadIdx.x == 0 && atomicAdd(&done[it], 1u) + 1u == (unsigned)I.units)
      stamps[it] = wall_clock64();
  }
}

template <int RPT, bool NT>
__global__ __launch_bounds__(256) void k_batch_spmv(const PlanView* __restrict__ views,
                                                    const BatchItemDev* __restrict__ items,
                                                    const int32_t* __restrict__ list,
                                                    const i64* __restrict__ off, int nlist,
                                                    i64 total, unsigned* __restrict__ counter,
                                                    unsigned* __restrict__ done,
                                                    unsigned long long* __restrict__ stamps) {
  __shared__ float lds[kCsrChunk + kSpmvThreads * RPT];
  batch_units<0, RPT, NT>(views, items, list, off, nlist, total, counter, done, stamps, lds);
}

// SpMV group g of a batch: the streamed tile with 1, 2 or 4 rows per thread (g % 3), with
// non-temporal loads for g >= 3; the plan's tuned streamed variant picks its group.
constexpr int kSpmvGroups = 6;
inline int spmv_group(int variant) {
  if (variant >= 0 && variant <= 2) return variant;
  if (variant >= 8 && variant <= 10) return 3 + (variant - 8);
  return 0;  // W-lanes, binned and specialized variants: the 256-row streamed tile
}
typedef void (*BatchKernel)(const PlanView*, const BatchItemDev*, const int32_t*, const i64*, int,
                            i64, unsigned*, unsigned*, unsigned long long*);
const BatchKernel kSpmvKernels[kSpmvGroups] = {k_batch_spmv<1, false>, k_batch_spmv<2, false>,
                                               k_batch_spmv<4, false>, k_batch_spmv<1, true>,
                                               k_batch_spmv<2, true>, k_batch_spmv<4, true>};

__global__ __launch_bounds__(256, 3) void k_batch_spmm(const PlanView* __restrict__ views,
                                                       const BatchItemDev* __restrict__ items,
                                                       const int32_t* __restrict__ list,
                                                       const i64* __restrict__ off, int nlist,
                                                       i64 total, unsigned* __restrict__ counter,
                                                       unsigned* __restrict__ done,
                                                       unsigned long long* __restrict__ stamps) {
  __shared__ __align__(16) float lds[kBatchSpmmLds];  // 40 KB
  batch_units<1>(views, items, list, off, nlist, total, counter, done, stamps, lds);
}

}  // namespace

}  // namespace sable

struct sable_batch_s {
  int count = 0;
  sable::DBuf<sable::PlanView> views;
  sable::DBuf<sable::BatchItemDev> items;
  // work lists: SpMV items by streamed-tile group (6), then SpMM items
  static constexpr int kLists = 7;
  sable::DBuf<int32_t> list[kLists];
  sable::DBuf<sable::i64> off[kLists];  // first unit of each list entry, total at the end
  sable::DBuf<unsigned> counter, done;
  sable::DBuf<unsigned long long> stamps;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last = nullptr;
  double tick_hz = 0.0;
  ~sable_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

static_assert(sable_batch_s::kLists == sable::kBatchCounters, "one work counter per list");

using namespace sable;

extern "C" {

sable_status sable_batch_create(const sable_plan_t* plans, const sable_batch_item* items,
                                int32_t count, void* stream, sable_batch_t* out) {
  if (out) *out = nullptr;
  clear_error();
  sable_batch_s* B = nullptr;
  try {
    if (!plans || !items || !out || count < 1) SB_THROW(SABLE_ERR_INVALID_ARG, "bad argument");
    for (int i = 0; i < count; ++i) {
      const sable_plan_s* p = plans[i];
      const sable_batch_item& it = items[i];
      if (!p || (it.op != 0 && it.op != 1) || it.n < 1 || (it.op == 0 && it.n != 1) ||
          (!it.x && p->ncols) || (!it.y && p->nrows))
        SB_THROW(SABLE_ERR_INVALID_ARG, "item %d: bad argument", i);
      if (it.op == 1 && (((uintptr_t)it.x & 15) || ((uintptr_t)it.y & 15)))
        SB_THROW(SABLE_ERR_INVALID_ARG, "item %d: X and Y must be 16-byte aligned", i);
    }
    hipStream_t s = (hipStream_t)stream;
    B = new sable_batch_s();
    B->count = count;
    std::vector<PlanView> hv(count);
    std::vector<BatchItemDev> hi(count);
    constexpr int NL = sable_batch_s::kLists;
    std::vector<int32_t> lists[NL];
    std::vector<i64> offs[NL];
    for (auto& o : offs) o.push_back(0);
    for (int i = 0; i < count; ++i) {
      const sable_plan_s& P = *plans[i];
      const sable_batch_item& it = items[i];
      BatchItemDev d;
      std::memset(&d, 0, sizeof(d));
      d.op = it.op;
      d.n = it.n;
      d.x = it.x;
      d.y = it.y;
      i64 units = 0;
      int li = kSpmvGroups;  // work list of the item
      if (P.nrows > 0) {
        if (it.op == 0) {
          li = spmv_group(P.prm.spmv_variant);
          hv[i] = make_view(P, P.sched[li % 3], false);
          units = hv[i].ntiles;
        } else {
          hv[i] = make_view(P, P.sched_mm, false);
          d.units_per_col = (P.nrows + kMmRows - 1) / kMmRows;
          d.col_chunks = (it.n + kMmCols - 1) / kMmCols;
          d.mfma = spmm_mfma_mode(P, P.prm.spmm_mode_for(it.n));
          units = (i64)d.units_per_col * d.col_chunks;
        }
      }
      if (units > INT32_MAX) SB_THROW(SABLE_ERR_TOO_LARGE, "item %d: %lld work units", i, (long long)units);
      d.units = (int)units;
      hi[i] = d;
      if (units) {
        lists[li].push_back(i);
        offs[li].push_back(offs[li].back() + units);
      }
    }
    i64 total[NL], all = 0;
    for (int k = 0; k < NL; ++k) all += (total[k] = offs[k].back());
    if (all > (i64)UINT32_MAX / 2) SB_THROW(SABLE_ERR_TOO_LARGE, "too many work units");
    to_dev(B->views, hv, s);
    to_dev(B->items, hi, s);
    for (int k = 0; k < NL; ++k) {
      lists[k].push_back(-1);  // never read: keeps the arrays non-empty
      to_dev(B->list[k], lists[k], s);
      to_dev(B->off[k], offs[k], s);
    }
    B->counter.alloc(NL);
    B->done.alloc(count);
    B->stamps.alloc(count + 1);
    HIPC(hipStreamSynchronize(s));
    int dev = 0, cus = 0, khz = 0;
    HIPC(hipGetDevice(&dev));
    HIPC(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPC(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    B->tick_hz = (double)khz * 1e3;
    // resident workgroups per CU of each kernel (registers and LDS) size its grid
    auto grid_of = [&](const void* kern, i64 units) {
      int per_cu = 0;
      HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0));
      return (unsigned)std::max<i64>(1, std::min<i64>(units, (i64)cus * std::max(1, per_cu)));
    };
    HIPC(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    HIPC(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    k_batch_reset<<<1, 256, 0, B->cap>>>(B->counter.p, B->done.p, B->items.p, count, B->stamps.p);
    for (int g = 0; g < kSpmvGroups; ++g)
      if (total[g])
        kSpmvKernels[g]<<<grid_of((const void*)kSpmvKernels[g], total[g]), 256, 0, B->cap>>>(
            B->views.p, B->items.p, B->list[g].p, B->off[g].p, (int)lists[g].size() - 1, total[g],
            B->counter.p + g, B->done.p, B->stamps.p);
    if (total[kSpmvGroups])
      k_batch_spmm<<<grid_of((const void*)k_batch_spmm, total[kSpmvGroups]), 256, 0, B->cap>>>(
          B->views.p, B->items.p, B->list[kSpmvGroups].p, B->off[kSpmvGroups].p,
          (int)lists[kSpmvGroups].size() - 1, total[kSpmvGroups], B->counter.p + kSpmvGroups,
          B->done.p, B->stamps.p);
    hipError_t ce = hipStreamEndCapture(B->cap, &B->graph);
    if (ce != hipSuccess) SB_THROW(SABLE_ERR_HIP, "stream capture: %s", hipGetErrorString(ce));
    HIPC(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    *out = B;
    return SABLE_OK;
  } catch (const Err& e) {
    delete B;
    return e.st;
  } catch (...) {
    delete B;
    set_error("internal error");
    return SABLE_ERR_INTERNAL;
  }
}

sable_status sable_batch_run(sable_batch_t b, void* stream) {
  clear_error();
  try {
    if (!b) SB_THROW(SABLE_ERR_INVALID_ARG, "NULL batch");
    HIPC(hipGraphLaunch(b->exec, (hipStream_t)stream));
    b->last = (hipStream_t)stream;
    return SABLE_OK;
  } catch (const Err& e) {
    return e.st;
  }
}

sable_status sable_batch_latencies(sable_batch_t b, uint64_t* ticks, double* tick_hz) {
  clear_error();
  try {
    if (!b || !ticks) SB_THROW(SABLE_ERR_INVALID_ARG, "bad argument");
    HIPC(hipStreamSynchronize(b->last));
    std::vector<unsigned long long> h;
    to_host(h, b->stamps.p, b->count + 1, b->last);
    for (int i = 0; i < b->count; ++i) ticks[i] = (uint64_t)(h[i] - h[b->count]);
    if (tick_hz) *tick_hz = b->tick_hz;
    return SABLE_OK;
  } catch (const Err& e) {
    return e.st;
  }
}

sable_status sable_batch_destroy(sable_batch_t b) {
  if (!b) return SABLE_OK;
  (void)hipDeviceSynchronize();
  delete b;
  return SABLE_OK;
}

}  // extern "C"
