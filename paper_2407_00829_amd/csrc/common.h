// Internal helpers of libsable: status propagation, device buffers, launch checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sable.h"

namespace sable {

typedef int64_t i64;

// Thread-local message for sable_last_error().
void set_error(const char* fmt, ...);
void clear_error();

// An error travelling up the internal call stack (never crosses the C interface).
struct Err {
  sable_status st;
};

#define SB_THROW(status, ...)         \
  do {                                \
    ::sable::set_error(__VA_ARGS__);  \
    throw ::sable::Err{status};       \
  } while (0)

#define HIPC(call)                                                                 \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      if (e_ == hipErrorOutOfMemory)                                               \
        SB_THROW(SABLE_ERR_OOM, "%s: %s (%s:%d)", #call, hipGetErrorString(e_),    \
                 __FILE__, __LINE__);                                              \
      SB_THROW(SABLE_ERR_HIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_),      \
               __FILE__, __LINE__);                                                \
    }                                                                              \
  } while (0)

#define LAUNCH_CHECK() HIPC(hipGetLastError())

// Device allocation with an optional injected failure (SABLE_FAIL_ALLOC_AFTER=k makes the
// k-th allocation of a process fail) so out-of-memory paths can be tested from the host.
void* dev_alloc(size_t bytes);
void dev_free(void* p);

// Owning device buffer.
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  explicit DBuf(size_t count) { alloc(count); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { reset(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { reset(); }
  void alloc(size_t count) {
    reset();
    n = count;
    p = (T*)dev_alloc((count ? count : 1) * sizeof(T));
  }
  void reset() {
    if (p) dev_free(p);
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
  T* get() const { return p; }
};

template <class T>
void to_host(std::vector<T>& h, const T* d, size_t count, hipStream_t s) {
  h.resize(count);
  if (count) HIPC(hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
}

template <class T>
void to_dev(DBuf<T>& d, const std::vector<T>& h, hipStream_t s) {
  d.alloc(h.size());
  if (!h.empty())
    HIPC(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

inline unsigned nblocks(i64 work, int per) { return (unsigned)((work + per - 1) / per); }

// Grid-stride helper bound for 1-D kernels (keeps grids within the 2^31 limit).
inline unsigned grid_for(i64 work, int threads, unsigned cap = 1u << 20) {
  i64 b = (work + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > (i64)cap) b = cap;
  return (unsigned)b;
}

// ---- library-primitive wrappers (hipCUB radix sort, scan, run-length encode) -----------
// Sort (key, value) pairs by key, stable. keys/vals are replaced by the sorted arrays.
void sort_pairs_u32(DBuf<uint32_t>& keys, DBuf<int32_t>& vals, i64 n, int end_bit,
                    hipStream_t s);
void sort_pairs_u64(DBuf<uint64_t>& keys, DBuf<int32_t>& vals, i64 n, int end_bit,
                    hipStream_t s);
// out[i] = sum_{j<i} in[j] for i in [0, n]; out must hold n+1 elements.
void exclusive_scan_i32(const int32_t* in, int32_t* out, i64 n, hipStream_t s);
void exclusive_scan_i64(const i64* in, i64* out, i64 n, hipStream_t s);
// Run-length encode sorted keys: unique[k], counts[k]; returns the number of runs.
i64 rle_u32(const uint32_t* keys, i64 n, DBuf<uint32_t>& uniq, DBuf<int32_t>& counts,
            hipStream_t s);
i64 rle_u64(const uint64_t* keys, i64 n, DBuf<uint64_t>& uniq, DBuf<int32_t>& counts,
            hipStream_t s);

int bits_for(uint64_t maxval);

}  // namespace sable
