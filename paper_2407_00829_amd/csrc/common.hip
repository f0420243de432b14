// Error state, allocation and library-primitive wrappers (hipCUB sort / scan / RLE).
#include <hipcub/hipcub.hpp>

#include <atomic>
#include <cstdarg>
#include <cstdlib>

#include "common.h"

namespace sable {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = 0; }

const char* last_error() { return g_err; }

static std::atomic<long> g_alloc_count{0};

static long fail_after() {
  static long v = [] {
    const char* e = getenv("SABLE_FAIL_ALLOC_AFTER");
    return e ? atol(e) : -1L;
  }();
  return v;
}

void* dev_alloc(size_t bytes) {
  long k = ++g_alloc_count;
  long f = fail_after();
  if (f >= 0 && k > f) SB_THROW(SABLE_ERR_OOM, "injected allocation failure (#%ld)", k);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    SB_THROW(e == hipErrorOutOfMemory ? SABLE_ERR_OOM : SABLE_ERR_HIP,
             "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  }
  return p;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

int bits_for(uint64_t maxval) {
  int b = 1;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

template <class K>
static void sort_pairs_impl(DBuf<K>& keys, DBuf<int32_t>& vals, i64 n, int end_bit,
                            hipStream_t s) {
  if (n <= 1) return;
  DBuf<K> k2(n);
  DBuf<int32_t> v2(n);
  size_t tmp = 0;
  HIPC(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, keys.p, k2.p, vals.p, v2.p, (int)n, 0,
                                          end_bit, s));
  DBuf<uint8_t> t(tmp);
  HIPC(hipcub::DeviceRadixSort::SortPairs(t.p, tmp, keys.p, k2.p, vals.p, v2.p, (int)n, 0,
                                          end_bit, s));
  keys = std::move(k2);
  vals = std::move(v2);
}

void sort_pairs_u32(DBuf<uint32_t>& keys, DBuf<int32_t>& vals, i64 n, int end_bit,
                    hipStream_t s) {
  sort_pairs_impl(keys, vals, n, end_bit, s);
}

void sort_pairs_u64(DBuf<uint64_t>& keys, DBuf<int32_t>& vals, i64 n, int end_bit,
                    hipStream_t s) {
  sort_pairs_impl(keys, vals, n, end_bit, s);
}

template <class T>
__global__ void k_scan_tail(const T* in, T* out, i64 n) {
  // out[n] = out[n-1] + in[n-1]
  if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = n ? out[n - 1] + in[n - 1] : T(0);
}

template <class T>
static void exclusive_scan_impl(const T* in, T* out, i64 n, hipStream_t s) {
  if (n > 0) {
    size_t tmp = 0;
    HIPC(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, in, out, (int)n, s));
    DBuf<uint8_t> t(tmp);
    HIPC(hipcub::DeviceScan::ExclusiveSum(t.p, tmp, in, out, (int)n, s));
  }
  k_scan_tail<T><<<1, 1, 0, s>>>(in, out, n);
  LAUNCH_CHECK();
}

void exclusive_scan_i32(const int32_t* in, int32_t* out, i64 n, hipStream_t s) {
  exclusive_scan_impl(in, out, n, s);
}

void exclusive_scan_i64(const i64* in, i64* out, i64 n, hipStream_t s) {
  exclusive_scan_impl(in, out, n, s);
}

template <class K>
static i64 rle_impl(const K* keys, i64 n, DBuf<K>& uniq, DBuf<int32_t>& counts,
                    hipStream_t s) {
  uniq.alloc(n > 0 ? n : 1);
  counts.alloc(n > 0 ? n : 1);
  if (n <= 0) return 0;
  DBuf<int32_t> nruns(1);
  size_t tmp = 0;
  HIPC(hipcub::DeviceRunLengthEncode::Encode(nullptr, tmp, keys, uniq.p, counts.p, nruns.p,
                                             (int)n, s));
  DBuf<uint8_t> t(tmp);
  HIPC(hipcub::DeviceRunLengthEncode::Encode(t.p, tmp, keys, uniq.p, counts.p, nruns.p,
                                             (int)n, s));
  int32_t h = 0;
  HIPC(hipMemcpyAsync(&h, nruns.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  return h;
}

i64 rle_u32(const uint32_t* keys, i64 n, DBuf<uint32_t>& uniq, DBuf<int32_t>& counts,
            hipStream_t s) {
  return rle_impl(keys, n, uniq, counts, s);
}

i64 rle_u64(const uint64_t* keys, i64 n, DBuf<uint64_t>& uniq, DBuf<int32_t>& counts,
            hipStream_t s) {
  return rle_impl(keys, n, uniq, counts, s);
}

}  // namespace sable
