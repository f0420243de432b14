// Batched persistent execution of many plans, captured in a hipGraph.
//
// Work units are (item, tile) pairs laid out item by item, SpMV items and SpMM items in two
// lists. Two persistent kernels, one per list, each with a grid of every CU times its
// resident workgroups, pull units from their own atomic counter; a unit runs exactly the tile
// body of the standalone product, so each item's result is bitwise equal to its standalone
// launch with the same kernel (SpMV: the 256-row streamed tile, variant 0; SpMM: the fused
// tile in the plan's matrix-core mode, the LDS-staged panel tile included). Keeping the two apart lets each run at the occupancy
// of its standalone kernel. The last unit of an item stamps the GPU wall clock. A reset kernel
// (no memset nodes) clears the counters and stamps the batch start; the three kernels are
// captured once and replayed.
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

__global__ void k_batch_reset(unsigned* __restrict__ counter, unsigned* __restrict__ done,
                              const BatchItemDev* __restrict__ items, int count,
                              unsigned long long* __restrict__ stamps) {
  __shared__ unsigned long long t0;
  if (threadIdx.x == 0) {
    counter[0] = 0;
    counter[1] = 0;
    t0 = wall_clock64();
    stamps[count] = t0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    done[i] = 0;
    if (items[i].units == 0) stamps[i] = t0;  // nothing to run: complete at the start
  }
}

constexpr int kBatchSpmvLds = kCsrChunk + kSpmvThreads;  // spmv_tile_stream<1>
constexpr int kBatchSpmmLds = kMmRows * kMmCols + kMmBlkStage * kBlkDesc;
static_assert(kBatchSpmmLds * 4 >= kPanLdsBytes, "the panel tile fits the SpMM units' LDS");

// Units of one list: list[k] is the item of the k-th entry, off[k] its first unit.
template <int OP>
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
      spmv_tile_stream<1>(P, local, I.x, I.y, lds);  // local = launch slot
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

__global__ __launch_bounds__(256) void k_batch_spmv(const PlanView* __restrict__ views,
                                                    const BatchItemDev* __restrict__ items,
                                                    const int32_t* __restrict__ list,
                                                    const i64* __restrict__ off, int nlist,
                                                    i64 total, unsigned* __restrict__ counter,
                                                    unsigned* __restrict__ done,
                                                    unsigned long long* __restrict__ stamps) {
  __shared__ float lds[kBatchSpmvLds];
  batch_units<0>(views, items, list, off, nlist, total, counter, done, stamps, lds);
}

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
  sable::DBuf<int32_t> list[2];     // SpMV items, SpMM items
  sable::DBuf<sable::i64> off[2];   // first unit of each list entry, total at the end
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
    std::vector<int32_t> lists[2];
    std::vector<i64> offs[2] = {{0}, {0}};
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
      if (P.nrows > 0) {
        if (it.op == 0) {
          hv[i] = make_view(P, P.sched[0], false);
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
        lists[it.op].push_back(i);
        offs[it.op].push_back(offs[it.op].back() + units);
      }
    }
    const i64 total[2] = {offs[0].back(), offs[1].back()};
    if (total[0] + total[1] > (i64)UINT32_MAX / 2) SB_THROW(SABLE_ERR_TOO_LARGE, "too many work units");
    to_dev(B->views, hv, s);
    to_dev(B->items, hi, s);
    for (int k = 0; k < 2; ++k) {
      lists[k].push_back(-1);  // never read: keeps the arrays non-empty
      to_dev(B->list[k], lists[k], s);
      to_dev(B->off[k], offs[k], s);
    }
    B->counter.alloc(2);
    B->done.alloc(count);
    B->stamps.alloc(count + 1);
    HIPC(hipStreamSynchronize(s));
    int dev = 0, cus = 0, khz = 0;
    HIPC(hipGetDevice(&dev));
    HIPC(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPC(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    B->tick_hz = (double)khz * 1e3;
    // resident workgroups per CU of each kernel (registers and LDS) size its grid
    int per_cu[2] = {0, 0};
    HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[0], k_batch_spmv, 256, 0));
    HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[1], k_batch_spmm, 256, 0));
    unsigned grid[2];
    for (int k = 0; k < 2; ++k)
      grid[k] = (unsigned)std::max<i64>(1, std::min<i64>(total[k], (i64)cus * std::max(1, per_cu[k])));
    HIPC(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    HIPC(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    k_batch_reset<<<1, 256, 0, B->cap>>>(B->counter.p, B->done.p, B->items.p, count, B->stamps.p);
    if (total[0])
      k_batch_spmv<<<grid[0], 256, 0, B->cap>>>(B->views.p, B->items.p, B->list[0].p, B->off[0].p,
                                                (int)lists[0].size() - 1, total[0], B->counter.p,
                                                B->done.p, B->stamps.p);
    if (total[1])
      k_batch_spmm<<<grid[1], 256, 0, B->cap>>>(B->views.p, B->items.p, B->list[1].p, B->off[1].p,
                                                (int)lists[1].size() - 1, total[1], B->counter.p + 1,
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
