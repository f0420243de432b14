// Residual matrix (Sec. 3 "Initialize"/"Extract"): validation of the input CSR, the
// residual's entry-to-row map and stream compaction of claimed entries.
#include "plan.h"

namespace sable {

// One thread per row: indptr monotone, columns in range and strictly increasing.
// Row pointers outside [0, nnz] are rejected before any column is read.
__global__ void k_validate(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                           int nrows, int ncols, i64 nnz, int* __restrict__ bad) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < nrows;
       i += (i64)gridDim.x * blockDim.x) {
    int a = ptr[i], b = ptr[i + 1];
    if (a < 0 || b < a || (i64)b > nnz) { atomicOr(bad, 1); continue; }
    int prev = -1;
    for (int k = a; k < b; ++k) {
      int c = col[k];
      if (c < 0 || c >= ncols || c <= prev) { atomicOr(bad, 2); break; }
      prev = c;
    }
  }
}

bool validate_csr_device(const sable_csr& A, hipStream_t s) {
  int32_t ends[2] = {0, 0};
  HIPC(hipMemcpyAsync(&ends[0], A.indptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(&ends[1], A.indptr + A.nrows, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  if (ends[0] != 0 || (i64)ends[1] != A.nnz) return false;
  DBuf<int> bad(1);
  HIPC(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  if (A.nrows > 0) {
    k_validate<<<grid_for(A.nrows, 256), 256, 0, s>>>(A.indptr, A.indices, A.nrows, A.ncols,
                                                      A.nnz, bad.p);
    LAUNCH_CHECK();
  }
  int h = 0;
  HIPC(hipMemcpyAsync(&h, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  return h == 0;
}

__global__ void k_iota(int32_t* __restrict__ a, i64 n) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x)
    a[k] = (int32_t)k;
}

void resid_from_input(Resid& R, const sable_csr& A, hipStream_t s) {
  R.nrows = A.nrows;
  R.ncols = A.ncols;
  R.nnz = A.nnz;
  R.ptr.alloc(A.nrows + 1);
  R.col.alloc(A.nnz);
  R.val.alloc(A.nnz);
  R.id.alloc(A.nnz);
  HIPC(hipMemcpyAsync(R.ptr.p, A.indptr, (A.nrows + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  if (A.nnz) {
    HIPC(hipMemcpyAsync(R.col.p, A.indices, A.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPC(hipMemcpyAsync(R.val.p, A.values, A.nnz * sizeof(float), hipMemcpyDeviceToDevice, s));
    k_iota<<<grid_for(A.nnz, 256), 256, 0, s>>>(R.id.p, A.nnz);
    LAUNCH_CHECK();
  }
}

// rows[k] = row of stored entry k (one thread per row writes its range).
__global__ void k_entry_rows(const int32_t* __restrict__ ptr, int nrows, int32_t* __restrict__ rows) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < nrows;
       i += (i64)gridDim.x * blockDim.x)
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) rows[k] = (int32_t)i;
}

void entry_rows(const Resid& R, DBuf<int32_t>& rows, hipStream_t s) {
  rows.alloc(R.nnz);
  if (R.nnz && R.nrows) {
    k_entry_rows<<<grid_for(R.nrows, 256), 256, 0, s>>>(R.ptr.p, R.nrows, rows.p);
    LAUNCH_CHECK();
  }
}

__global__ void k_keep(const uint8_t* __restrict__ claimed, int32_t* __restrict__ keep, i64 n) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x)
    keep[k] = claimed[k] ? 0 : 1;
}

__global__ void k_compact(const uint8_t* __restrict__ claimed, const int32_t* __restrict__ pos,
                          const int32_t* __restrict__ col, const float* __restrict__ val,
                          const int32_t* __restrict__ id, int32_t* __restrict__ col2,
                          float* __restrict__ val2, int32_t* __restrict__ id2, i64 n) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x) {
    if (claimed[k]) continue;
    int32_t q = pos[k];
    col2[q] = col[k];
    val2[q] = val[k];
    id2[q] = id[k];
  }
}

__global__ void k_newptr(const int32_t* __restrict__ ptr, const int32_t* __restrict__ pos,
                         int32_t* __restrict__ ptr2, int nrows) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i <= nrows;
       i += (i64)gridDim.x * blockDim.x)
    ptr2[i] = pos[ptr[i]];
}

// Remove claimed entries; surviving entries keep their order (rows stay sorted).
void resid_compact(Resid& R, const DBuf<uint8_t>& claimed, hipStream_t s) {
  const i64 n = R.nnz;
  DBuf<int32_t> keep(n), pos(n + 1);
  if (n) {
    k_keep<<<grid_for(n, 256), 256, 0, s>>>(claimed.p, keep.p, n);
    LAUNCH_CHECK();
  }
  exclusive_scan_i32(keep.p, pos.p, n, s);
  int32_t total = 0;
  HIPC(hipMemcpyAsync(&total, pos.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  DBuf<int32_t> ptr2(R.nrows + 1), col2(total), id2(total);
  DBuf<float> val2(total);
  if (n) {
    k_compact<<<grid_for(n, 256), 256, 0, s>>>(claimed.p, pos.p, R.col.p, R.val.p, R.id.p,
                                               col2.p, val2.p, id2.p, n);
    LAUNCH_CHECK();
  }
  k_newptr<<<grid_for(R.nrows + 1, 256), 256, 0, s>>>(R.ptr.p, pos.p, ptr2.p, R.nrows);
  LAUNCH_CHECK();
  HIPC(hipStreamSynchronize(s));
  R.ptr = std::move(ptr2);
  R.col = std::move(col2);
  R.val = std::move(val2);
  R.id = std::move(id2);
  R.nnz = total;
}

}  // namespace sable
