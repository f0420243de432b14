// Batched persistent execution of many plans in one launch, captured in a hipGraph.
//
// Work units are (item, tile) pairs laid out item by item. A persistent grid (every CU,
// a few workgroups each) pulls units from one atomic counter; a unit runs exactly the tile
// body of the standalone product (streamed SpMV tiles, or SpMM tiles), so each item's
// result is bitwise equal to its standalone launch with the same kernel variant. The last
// unit of an item stamps the GPU wall clock. A reset kernel (no memset nodes) clears the
// counters and stamps the batch start; both kernels are captured once and replayed.
#include <algorithm>

#include "exec.h"
#include "spmm_tile.h"

namespace sable {

struct BatchItemDev {
  int op, n, rpt, mfma;
  int units_per_col, col_chunks;  // SpMM: row tiles x column chunks
  const float* x;
  float* y;
};

namespace {

__global__ void k_batch_reset(unsigned* __restrict__ counter, unsigned* __restrict__ done,
                              int count, unsigned long long* __restrict__ stamps) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) done[i] = 0;
  if (threadIdx.x == 0) {
    counter[0] = 0;
    stamps[count] = wall_clock64();
  }
}

constexpr int kBatchLds = kMmRows * kMmCols + kMmBlkStage * kBlkDesc;  // >= largest SpMV tile
static_assert(kBatchLds >= kCsrChunk + 1024, "LDS budget");

__global__ __launch_bounds__(256, 3) void k_batch(const PlanView* __restrict__ views,
                                               const BatchItemDev* __restrict__ items,
                                               const i64* __restrict__ unit_off, int count,
                                               i64 total, unsigned* __restrict__ counter,
                                               unsigned* __restrict__ done,
                                               unsigned long long* __restrict__ stamps) {
  __shared__ float lds[kBatchLds];  // exactly 40 KB: four workgroups per CU
  unsigned* unit = reinterpret_cast<unsigned*>(lds);  // broadcast slot, free between units
  for (;;) {
    __syncthreads();  // the previous unit is done with the LDS
    if (threadIdx.x == 0) unit[0] = atomicAdd(counter, 1u);
    __syncthreads();
    const i64 u = (i64)unit[0];
    __syncthreads();  // every thread has read the slot before the unit body reuses it
    if (u >= total) break;
    int lo = 0, hi = count - 1;  // item of unit u
    while (lo < hi) {
      int m = (lo + hi + 1) >> 1;
      if (unit_off[m] <= u) lo = m; else hi = m - 1;
    }
    const int it = lo;
    const BatchItemDev I = items[it];
    const PlanView& P = views[it];
    int local = (int)(u - unit_off[it]);
    if (I.op == 0) {
      if (P.tile_order) local = P.tile_order[local];
      if (I.rpt == 1) spmv_tile_stream<1>(P, local, I.x, I.y, lds);
      else if (I.rpt == 2) spmv_tile_stream<2>(P, local, I.x, I.y, lds);
      else spmv_tile_stream<4>(P, local, I.x, I.y, lds);
    } else {
      int rt = local % I.units_per_col;
      const int cc = local / I.units_per_col;
      if (P.tile_order) rt = P.tile_order[rt];
      spmm_tile(P, rt * kMmRows, cc * kMmCols, I.n, I.x, I.y, lds, I.mfma);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      const unsigned units = (unsigned)(unit_off[it + 1] - unit_off[it]);
      if (atomicAdd(&done[it], 1u) + 1u == units) stamps[it] = wall_clock64();
    }
  }
}

}  // namespace

}  // namespace sable

struct sable_batch_s {
  int count = 0;
  sable::DBuf<sable::PlanView> views;
  sable::DBuf<sable::BatchItemDev> items;
  sable::DBuf<sable::i64> unit_off;
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
    std::vector<i64> off(count + 1, 0);
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
      if (it.op == 0) {
        const int var = P.prm.spmv_variant <= 2 ? P.prm.spmv_variant : 0;
        d.rpt = 1 << var;
        hv[i] = make_view(P, P.sched[var], false);
        units = hv[i].ntiles;
      } else {
        hv[i] = make_view(P, P.sched_mm, false);
        d.units_per_col = (P.nrows + kMmRows - 1) / kMmRows;
        d.col_chunks = (it.n + kMmCols - 1) / kMmCols;
        d.mfma = spmm_mfma_mode(P);
        units = (i64)d.units_per_col * d.col_chunks;
      }
      hi[i] = d;
      off[i + 1] = off[i] + units;
    }
    const i64 total = off[count];
    to_dev(B->views, hv, s);
    to_dev(B->items, hi, s);
    to_dev(B->unit_off, off, s);
    B->counter.alloc(1);
    B->done.alloc(count);
    B->stamps.alloc(count + 1);
    HIPC(hipStreamSynchronize(s));
    int dev = 0, cus = 0, khz = 0;
    HIPC(hipGetDevice(&dev));
    HIPC(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPC(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    B->tick_hz = (double)khz * 1e3;
    int per_cu = 0;  // resident workgroups per CU for this kernel (registers and LDS)
    HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, 256, 0));
    const unsigned grid = (unsigned)std::max<i64>(1, std::min<i64>(total, (i64)cus * std::max(1, per_cu)));
    HIPC(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    HIPC(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    k_batch_reset<<<1, 256, 0, B->cap>>>(B->counter.p, B->done.p, count, B->stamps.p);
    k_batch<<<grid, 256, 0, B->cap>>>(B->views.p, B->items.p, B->unit_off.p, count, total,
                                      B->counter.p, B->done.p, B->stamps.p);
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
