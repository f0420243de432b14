// C interface of libsable: plan construction (Sec. 3), export, value refresh, error norm.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>

#include "plan.h"

namespace sable {

const char* last_error();
bool vbr_paper_fits(i64 nrows, i64 ncols, i64 amin);

namespace {

template <class F>
sable_status guard(F&& f) {
  clear_error();
  try {
    f();
    return SABLE_OK;
  } catch (const Err& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return SABLE_ERR_OOM;
  } catch (...) {
    set_error("internal error");
    return SABLE_ERR_INTERNAL;
  }
}

__global__ void k_csr_owner(const int32_t* __restrict__ rid, i64 n, int8_t* __restrict__ owner,
                            i64* __restrict__ slot) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x) {
    owner[rid[k]] = 2;
    slot[rid[k]] = k;
  }
}

// Refresh every stored value from a new value array with the same structure (aval: the
// whole-input copy, may be null).
template <class T>
__global__ void k_update_values(const T* __restrict__ values, i64 nnz,
                                const int8_t* __restrict__ owner, const i64* __restrict__ slot,
                                T* __restrict__ vdia, T* __restrict__ vbr, T* __restrict__ csr,
                                T* __restrict__ aval) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < nnz; k += (i64)gridDim.x * blockDim.x) {
    const T v = values[k];
    const int8_t o = owner[k];
    const i64 at = slot[k];
    if (o == 0) vdia[at] = v;
    else if (o == 1) vbr[at] = v;
    else csr[at] = v;
    if (aval) aval[k] = v;
  }
}

constexpr int kNormThreads = 256;

__global__ __launch_bounds__(kNormThreads) void k_norm_partial(const float* __restrict__ y,
                                                               const double* __restrict__ yref,
                                                               i64 n, double* __restrict__ part) {
  __shared__ double sd[kNormThreads], sr[kNormThreads];
  double a = 0.0, b = 0.0;
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x) {
    const double d = (double)y[k] - yref[k];
    a += d * d;
    b += yref[k] * yref[k];
  }
  sd[threadIdx.x] = a;
  sr[threadIdx.x] = b;
  __syncthreads();
  for (int w = kNormThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sd[threadIdx.x] += sd[threadIdx.x + w];
      sr[threadIdx.x] += sr[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sd[0];
    part[2 * blockIdx.x + 1] = sr[0];
  }
}

// Adds the nb partial pairs in block order and writes the relative error
// sqrt(sum d^2) / sqrt(sum yref^2) (the absolute one if yref = 0) to out[0].
__global__ void k_norm_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x || blockIdx.x) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nb; ++k) { a += part[2 * k]; b += part[2 * k + 1]; }
  const double num = sqrt(a), den = sqrt(b);
  out[0] = den > 0.0 ? num / den : num;
}

// Partial-sum pairs of the error norm: one per workgroup of k_norm_partial, whose grid is
// capped at this count, so every input length fits.
constexpr int kNormMaxParts = 1024;

int norm_parts(i64 len) {
  return (int)std::min<i64>(kNormMaxParts, std::max<i64>(1, (len + kNormThreads - 1) / kNormThreads));
}

// Scratch of the allocation-free error norm: the partial pairs, then the result slot (unused
// there: that entry point writes the result to the caller's device double). Every GPU the
// library runs on holds its own copy until the process ends.
static __device__ __align__(256) double scratch[2 * kNormMaxParts + 2];

// Device address of this GPU's scratch copy, looked up once per device with that device
// current (the array's name in host code is only a host-side stand-in).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

double* scratch_for_current_device() {
  int dev = -1;
  HIPC(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) SB_THROW(SABLE_ERR_INTERNAL, "device id %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPC(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) SB_THROW(SABLE_ERR_HIP, "no device address for the error-norm scratch");
    g_scratch_ptr[dev] = (double*)ptr;
  }
  return g_scratch_ptr[dev];
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {  // splitmix64 finaliser
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// A wave's 64 partial sums added (mod 2^64) and added once to *out.
__device__ __forceinline__ void add_wave_sum(uint64_t acc, unsigned long long* out) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += (uint64_t)__shfl_xor((unsigned long long)acc, o);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, (unsigned long long)acc);
}

constexpr unsigned kHashBlocks = 2048;  // grid-stride: a few thousand atomics per hash

// sum over k of mix(k, a[k]) mod 2^64 (order-independent, so the atomic sum is exact)
__global__ void k_hash_i32(const int32_t* __restrict__ a, i64 n, uint64_t salt,
                           unsigned long long* __restrict__ out) {
  uint64_t acc = 0;
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x)
    acc += mix64(((uint64_t)k << 32) ^ (uint32_t)a[k] ^ salt);
  add_wave_sum(acc, out);
}

uint64_t mix64_host(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Hash of everything the plan's structure depends on: the sparsity pattern of A, the
// extractor list and the thresholds (not the values). Plans with equal hashes have the same
// formats and schedules, so one autotuning result serves all of them.
uint64_t structure_hash(const sable_csr& A, const sable_extractor* list, int nlist,
                        const sable_thresholds& th, hipStream_t s) {
  DBuf<unsigned long long> d(2);
  HIPC(hipMemsetAsync(d.p, 0, 2 * sizeof(unsigned long long), s));
  k_hash_i32<<<grid_for((i64)A.nrows + 1, 256, kHashBlocks), 256, 0, s>>>(A.indptr, (i64)A.nrows + 1, 0x9e3779b97f4a7c15ull, d.p);
  LAUNCH_CHECK();
  if (A.nnz) {
    k_hash_i32<<<grid_for(A.nnz, 256, kHashBlocks), 256, 0, s>>>(A.indices, A.nnz, 0x7f4a7c159e3779b9ull, d.p + 1);
    LAUNCH_CHECK();
  }
  unsigned long long h2[2];
  HIPC(hipMemcpyAsync(h2, d.p, sizeof(h2), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  uint64_t h = mix64_host(h2[0]) ^ mix64_host(h2[1] + 0x632be59bd9b4e019ull);
  auto put = [&](uint64_t v) { h = mix64_host(h ^ v) + 0x9e3779b97f4a7c15ull; };
  put((uint64_t)(uint32_t)A.nrows); put((uint64_t)(uint32_t)A.ncols); put((uint64_t)A.nnz);
  for (int e = 0; e < nlist; ++e) put(((uint64_t)(uint32_t)list[e].kind << 32) | (uint32_t)list[e].vbr_mode);
  put((uint64_t)(uint32_t)th.delta_band_pm << 32 | (uint32_t)th.delta_block_pm);
  put((uint64_t)th.amin_band); put((uint64_t)th.amin_block);
  put((uint64_t)(uint32_t)th.lseg << 32 | (uint32_t)th.wmax);
  put((uint64_t)(uint32_t)th.dmax << 32 | (uint32_t)th.coverage_pm);
  put((uint64_t)(uint32_t)th.tile_set_mask << 32 | th.flags);
  return h;
}

__global__ void k_hash_owner_slot(const int8_t* __restrict__ owner, const i64* __restrict__ slot,
                                  i64 n, unsigned long long* __restrict__ out) {
  uint64_t acc = 0;
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x)
    acc += mix64(((uint64_t)k << 8 | (uint8_t)owner[k]) ^ mix64((uint64_t)slot[k] + 0x2545f4914f6cdd1dull));
  add_wave_sum(acc, out);
}

// Hash of the partition a plan built: which format holds each entry and where, plus the
// segment and block descriptors that fix the stored fill. Two plans with equal hashes run the
// same kernels over the same layout.
uint64_t partition_hash(const sable_plan_s& P, hipStream_t s) {
  DBuf<unsigned long long> d(6);
  HIPC(hipMemsetAsync(d.p, 0, 6 * sizeof(unsigned long long), s));
  auto h32 = [&](const int32_t* a, i64 n, uint64_t salt, int k) {
    if (n <= 0) return;
    k_hash_i32<<<grid_for(n, 256, kHashBlocks), 256, 0, s>>>(a, n, salt, d.p + k);
    LAUNCH_CHECK();
  };
  if (P.nnz) {
    k_hash_owner_slot<<<grid_for(P.nnz, 256, kHashBlocks), 256, 0, s>>>(P.owner.p, P.slot.p, P.nnz, d.p);
    LAUNCH_CHECK();
  }
  h32(P.blk.p, 4 * (i64)P.nblk, 0x3c6ef372fe94f82bull, 1);
  h32(P.idiag.p, P.nidiag, 0xa54ff53a5f1d36f1ull, 2);
  h32(P.seg_row_start.p, P.nseg, 0x510e527fade682d1ull, 3);
  h32(P.seg_nrows.p, P.nseg, 0x9b05688c2b3e6c1full, 4);
  h32(P.seg_ndiags.p, P.nseg, 0x1f83d9abfb41bd6bull, 5);
  unsigned long long h6[6];
  HIPC(hipMemcpyAsync(h6, d.p, sizeof(h6), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  uint64_t h = 0x6a09e667f3bcc908ull;
  auto put = [&](uint64_t v) { h = mix64_host(h ^ v) + 0x9e3779b97f4a7c15ull; };
  for (int k = 0; k < 6; ++k) put(h6[k]);
  put((uint64_t)(uint32_t)P.nrows << 32 | (uint32_t)P.ncols);
  put((uint64_t)P.nnz); put((uint64_t)P.nidiag); put((uint64_t)(uint32_t)P.nseg << 32 | (uint32_t)P.nblk);
  put((uint64_t)P.vdia_cells); put((uint64_t)P.vbr_cells); put((uint64_t)P.csr_nnz);
  put((uint64_t)P.flags);
  return h;
}

void build_plan(sable_plan_s& P, const sable_csr& A, const sable_extractor* list, int nlist,
                const sable_thresholds& th, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  P.structure_hash = structure_hash(A, list, nlist, th, s);
  P.nrows = A.nrows;
  P.ncols = A.ncols;
  P.nnz = A.nnz;
  P.flags = th.flags;
  P.owner.alloc(A.nnz);
  P.slot.alloc(A.nnz);
  // plain copy of the input (baseline CSR kernel and value refresh)
  P.a_ptr.alloc(A.nrows + 1);
  P.a_col.alloc(A.nnz);
  P.a_val.alloc(A.nnz);
  HIPC(hipMemcpyAsync(P.a_ptr.p, A.indptr, (A.nrows + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  if (A.nnz) {
    HIPC(hipMemcpyAsync(P.a_col.p, A.indices, A.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPC(hipMemcpyAsync(P.a_val.p, A.values, A.nnz * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  if (A.nrows == 0 || A.ncols == 0) {
    // no entry can exist: the plan is an empty CSR part (products give y = 0, or nothing)
    P.csr_nnz = 0;
    P.csr_ptr.alloc(A.nrows + 1);
    P.csr_col.alloc(0);
    P.csr_val.alloc(0);
    HIPC(hipMemsetAsync(P.csr_ptr.p, 0, (A.nrows + 1) * sizeof(int32_t), s));
    for (int e = 0; e < nlist && list[e].kind != SABLE_X_CSR; ++e)
      if (list[e].kind == SABLE_X_VBR) blocks_none(P, th, list[e].vbr_mode);
  } else {
    Resid R;
    resid_from_input(R, A, s);
    for (int e = 0; e < nlist; ++e) {
      if (list[e].kind == SABLE_X_CSR) {
        extract_csr(P, R, s);
        break;
      }
      DBuf<uint8_t> claimed(R.nnz);
      if (R.nnz) HIPC(hipMemsetAsync(claimed.p, 0, R.nnz, s));
      if (list[e].kind == SABLE_X_VDIA) extract_bands(P, R, th, claimed, s);
      else extract_blocks(P, R, th, list[e].vbr_mode, claimed, s);
      resid_compact(R, claimed, s);
    }
    if (P.vbr_cells && (P.flags & SABLE_F_SPLIT_BF16)) build_bf16_split(P, s);
  }
  if (A.nrows > 0) {  // every product entry point returns at once when nrows == 0
    for (int k = 0; k < 3; ++k) {
      build_schedule(P, P.sched[k], 256 << k, true, s, false, true);
      build_schedule(P, P.sched_plain[k], 256 << k, false, s, false, true);
    }
    build_bins(P, P.sched[0], true, s);
    build_bins(P, P.sched_plain[0], false, s);
    build_schedule(P, P.sched_mm, 64, true, s, true);
    build_mm_panels(P, s);
    for (int k = 0; k < 4; ++k) build_schedule(P, P.sched_w[k], 128 >> k, true, s);
    build_far_split(P, s);
  }
  P.partition_hash = partition_hash(P, s);
  HIPC(hipStreamSynchronize(s));
  P.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

void extract_csr(sable_plan_s& P, const Resid& R, hipStream_t s) {
  P.csr_nnz = R.nnz;
  P.csr_ptr.alloc(R.nrows + 1);
  P.csr_col.alloc(R.nnz);
  P.csr_val.alloc(R.nnz);
  HIPC(hipMemcpyAsync(P.csr_ptr.p, R.ptr.p, (R.nrows + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  if (R.nnz) {
    HIPC(hipMemcpyAsync(P.csr_col.p, R.col.p, R.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPC(hipMemcpyAsync(P.csr_val.p, R.val.p, R.nnz * sizeof(float), hipMemcpyDeviceToDevice, s));
    k_csr_owner<<<grid_for(R.nnz, 256), 256, 0, s>>>(R.id.p, R.nnz, P.owner.p, P.slot.p);
    LAUNCH_CHECK();
  }
  HIPC(hipStreamSynchronize(s));
}

}  // namespace sable

sable::i64 sable_plan_s::device_bytes() const {
  sable::i64 b = 0;
  b += vdia_val.bytes() + idiag.bytes() + seg_row_start.bytes() + seg_nrows.bytes() +
       seg_ndiags.bytes() + seg_idiag_ptr.bytes() + seg_val_ptr.bytes();
  b += blk.bytes() + blk_val_ptr.bytes() + vbr_val.bytes() + vbr_mma.bytes() + blk_mma_ptr.bytes();
  b += csr_ptr.bytes() + csr_col.bytes() + csr_val.bytes();
  b += vdia_val64.bytes() + vbr_val64.bytes() + csr_val64.bytes();
  b += a_ptr.bytes() + a_col.bytes() + a_val.bytes() + owner.bytes() + slot.bytes();
  for (int k = 0; k < 11; ++k) {
    const sable::Schedule* S = k < 3 ? &sched[k] : k < 6 ? &sched_plain[k - 3] : k == 6 ? &sched_mm
                                                                                       : &sched_w[k - 7];
    b += S->tile_seg_lo.bytes() + S->tile_seg_hi.bytes() + S->tile_blk_ptr.bytes() +
         S->tile_blk.bytes() + S->order.bytes() + S->row0.bytes() + S->bin_rows.bytes() +
         S->bin_off.bytes() + S->head.bytes();
  }
  b += mm_panels.kcol.bytes() + mm_panels.kptr.bytes() + mm_panels.bpos.bytes() +
       mm_panels.apack.bytes() + mm_panels.amask.bytes() + mm_panels.aptr.bytes() +
       mm_panels.pan_tile.bytes() + mm_panels.pan_pos.bytes();
  b += far.ccol.bytes() + far.far_col.bytes() + far.far_src.bytes() + far.far_val.bytes() +
       far.far_prod.bytes() + far.far_val64.bytes() + far.far_prod64.bytes() + far.chunk.bytes();
  return b;
}

using namespace sable;

extern "C" {

const char* sable_last_error(void) { return sable::last_error(); }

sable_status sable_thresholds_default(sable_thresholds* out) {
  if (!out) {
    set_error("NULL output");
    return SABLE_ERR_INVALID_ARG;
  }
  out->delta_band_pm = 750;
  out->delta_block_pm = 500;
  out->amin_band = 2500;
  out->amin_block = 2500;
  out->lseg = 64;
  out->wmax = 32;
  out->dmax = -1;
  out->coverage_pm = 80;
  out->tile_set_mask = 0;
  out->flags = SABLE_F_SPLIT_BF16;
  return SABLE_OK;
}

sable_status sable_plan(const sable_csr* A, const sable_extractor* list, int32_t nlist,
                        const sable_thresholds* th_in, void* stream, sable_plan_t* out) {
  if (out) *out = nullptr;
  return guard([&] {
    if (!A || !list || !out) SB_THROW(SABLE_ERR_INVALID_ARG, "NULL argument");
    if (A->nrows < 0 || A->ncols < 0 || A->nnz < 0)
      SB_THROW(SABLE_ERR_INVALID_ARG, "negative dimension");
    if (A->nnz >= (i64)INT32_MAX) SB_THROW(SABLE_ERR_TOO_LARGE, "nnz >= 2^31");
    if (!A->indptr || (A->nnz > 0 && (!A->indices || !A->values)))
      SB_THROW(SABLE_ERR_INVALID_ARG, "NULL CSR array");
    if (nlist < 1 || nlist > 3) SB_THROW(SABLE_ERR_INVALID_ARG, "extractor list length %d", nlist);
    if (list[nlist - 1].kind != SABLE_X_CSR)
      SB_THROW(SABLE_ERR_INCOMPLETE, "the extractor list must end with the CSR catch-all");
    for (int e = 0; e < nlist - 1; ++e) {
      if (list[e].kind != SABLE_X_VDIA && list[e].kind != SABLE_X_VBR)
        SB_THROW(SABLE_ERR_INVALID_ARG, "extractor %d: kind %d", e, list[e].kind);
      for (int f = 0; f < e; ++f)
        if (list[f].kind == list[e].kind) SB_THROW(SABLE_ERR_INVALID_ARG, "duplicate extractor kind");
      if (list[e].kind == SABLE_X_VBR) {
        const int m = list[e].vbr_mode;
        if (m < 0 || m > 2) SB_THROW(SABLE_ERR_INVALID_ARG, "vbr_mode %d", m);
      }
    }
    sable_thresholds th;
    sable_thresholds_default(&th);
    if (th_in) th = *th_in;
    for (int e = 0; e < nlist - 1; ++e)
      if (list[e].kind == SABLE_X_VBR && list[e].vbr_mode == SABLE_VBR_PAPER &&
          !vbr_paper_fits(A->nrows, A->ncols, std::max<i64>(1, th.amin_block)))
        SB_THROW(SABLE_ERR_TOO_LARGE, "literal block search over budget for %dx%d", A->nrows,
                 A->ncols);
    if (th.delta_block_pm < 500 || th.delta_block_pm > 1000 || th.delta_band_pm < 1 ||
        th.delta_band_pm > 1000 || th.amin_block < 1 || th.amin_band < 1 || th.lseg < 1 ||
        th.wmax < 0 || th.wmax > 63 || th.coverage_pm < 0 || th.coverage_pm > 1000 || th.tile_set_mask < 0 ||
        th.tile_set_mask > 31)
      SB_THROW(SABLE_ERR_INVALID_ARG, "threshold out of range");
    hipStream_t s = (hipStream_t)stream;
    if (!validate_csr_device(*A, s)) SB_THROW(SABLE_ERR_INVALID_CSR, "input is not canonical CSR");
    sable_plan_s* P = new sable_plan_s();
    try {
      build_plan(*P, *A, list, nlist, th, s);
    } catch (...) {
      (void)hipStreamSynchronize(s);
      delete P;
      throw;
    }
    *out = P;
  });
}

sable_status sable_plan_destroy(sable_plan_t p) {
  return guard([&] {
    if (!p) return;
    (void)hipDeviceSynchronize();
    delete p;
  });
}

sable_status sable_plan_info(sable_plan_t p, sable_plan_stats* o) {
  return guard([&] {
    if (!p || !o) SB_THROW(SABLE_ERR_INVALID_ARG, "NULL argument");
    std::memset(o, 0, sizeof(*o));
    o->nrows = p->nrows;
    o->ncols = p->ncols;
    o->nnz = p->nnz;
    o->nseg = p->nseg;
    o->nidiag = p->nidiag;
    o->vdia_cells = p->vdia_cells;
    o->vdia_nnz = p->vdia_nnz;
    o->nblk = p->nblk;
    o->vbr_mode_used = p->vbr_mode_used;
    o->vbr_tile = p->vbr_tile;
    o->vbr_cells = p->vbr_cells;
    o->vbr_nnz = p->vbr_nnz;
    o->csr_nnz = p->csr_nnz;
    // compulsory bytes of the formats: VDIA values + per-segment metadata, VBR values,
    // CSR values + column indices + row pointers
    o->bytes_matrix = 4 * p->vdia_cells + 20 * (i64)p->nseg + 4 * p->vbr_cells +
                      8 * p->csr_nnz + 4 * ((i64)p->nrows + 1);
    o->device_bytes = p->device_bytes();
    o->structure_hash = p->structure_hash;
    o->partition_hash = p->partition_hash;
    o->mm_panels = p->mm_panels.npanels;
    o->mm_units = p->mm_panels.nunits;
    o->plan_ms = p->plan_ms;
    o->spmv_variant = p->prm.spmv_variant;
    o->spmm_variant = p->prm.spmm_mode;
    o->plain_variant = p->prm.plain_variant;
    o->far_split = (p->far.npanel && p->prm.far_split) ? 1 : 0;
    o->far_nnz = p->far.nfar;
    o->spec_ms = p->spec_ms;
  });
}

sable_status sable_plan_export(sable_plan_t p, const sable_partition_host* o) {
  return guard([&] {
    if (!p || !o) SB_THROW(SABLE_ERR_INVALID_ARG, "NULL argument");
    HIPC(hipDeviceSynchronize());
    auto cp = [&](void* dst, const void* src, size_t bytes) {
      if (dst && bytes) HIPC(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
    };
    cp(o->vdia_val, p->vdia_val.p, p->vdia_cells * sizeof(float));
    cp(o->idiag, p->idiag.p, p->nidiag * sizeof(int32_t));
    cp(o->seg_row_start, p->seg_row_start.p, p->nseg * sizeof(int32_t));
    cp(o->seg_nrows, p->seg_nrows.p, p->nseg * sizeof(int32_t));
    cp(o->seg_ndiags, p->seg_ndiags.p, p->nseg * sizeof(int32_t));
    cp(o->seg_val_ptr, p->seg_val_ptr.p, p->nseg * sizeof(int64_t));
    cp(o->seg_idiag_ptr, p->seg_idiag_ptr.p, p->nseg * sizeof(int32_t));
    cp(o->blk, p->blk.p, 4 * (size_t)p->nblk * sizeof(int32_t));
    cp(o->blk_val_ptr, p->blk_val_ptr.p, p->nblk * sizeof(int64_t));
    cp(o->vbr_val, p->vbr_val.p, p->vbr_cells * sizeof(float));
    cp(o->csr_col, p->csr_col.p, p->csr_nnz * sizeof(int32_t));
    cp(o->csr_val, p->csr_val.p, p->csr_nnz * sizeof(float));
    cp(o->owner, p->owner.p, p->nnz * sizeof(int8_t));
    cp(o->slot, p->slot.p, p->nnz * sizeof(int64_t));
    if (o->csr_ptr) {
      std::vector<int32_t> h(p->nrows + 1);
      HIPC(hipMemcpy(h.data(), p->csr_ptr.p, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
      for (size_t i = 0; i < h.size(); ++i) o->csr_ptr[i] = h[i];
    }
    if (o->vbr_bf16 && p->vbr_cells) {
      // the device copy is row-major per block with the row stride padded to a multiple of 4;
      // the export follows vbr_val's column-major order
      std::fill(o->vbr_bf16, o->vbr_bf16 + p->vbr_cells, 0u);
      if (p->vbr_mma.p) {
        std::vector<int32_t> blk;
        std::vector<i64> vp, mp;
        std::vector<uint32_t> w;
        to_host(blk, p->blk.p, 4 * (size_t)p->nblk, nullptr);
        to_host(vp, p->blk_val_ptr.p, p->nblk, nullptr);
        to_host(mp, p->blk_mma_ptr.p, p->nblk, nullptr);
        to_host(w, p->vbr_mma.p, p->vbr_mma.n, nullptr);
        for (int b = 0; b < p->nblk; ++b) {
          const i64 h = blk[4 * b + 1] - blk[4 * b], wd = blk[4 * b + 3] - blk[4 * b + 2];
          const i64 w4 = (wd + 3) & ~(i64)3;
          for (i64 r = 0; r < h; ++r)
            for (i64 k = 0; k < wd; ++k) o->vbr_bf16[vp[b] + k * h + r] = w[mp[b] + r * w4 + k];
        }
      }
    }
  });
}

sable_status sable_spmv(sable_plan_t p, const float* x, float* y, void* stream) {
  return guard([&] {
    if (!p || (!x && p->ncols) || (!y && p->nrows)) SB_THROW(SABLE_ERR_INVALID_ARG, "NULL argument");
    if (p->nrows == 0) return;
    launch_spmv(*p, x, y, (hipStream_t)stream);
  });
}

sable_status sable_csr_spmv(sable_plan_t p, const float* x, float* y, void* stream) {
  return guard([&] {
    if (!p || (!x && p->ncols) || (!y && p->nrows)) SB_THROW(SABLE_ERR_INVALID_ARG, "NULL argument");
    if (p->nrows == 0) return;
    launch_spmv_plain(*p, x, y, (hipStream_t)stream);
  });
}

sable_status sable_spmm(sable_plan_t p, const float* X, float* Y, int32_t n, void* stream) {
  return guard([&] {
    if (!p || n < 1 || (!X && p->ncols) || (!Y && p->nrows))
      SB_THROW(SABLE_ERR_INVALID_ARG, "NULL argument or n < 1");
    if (((uintptr_t)X & 15) || ((uintptr_t)Y & 15))
      SB_THROW(SABLE_ERR_INVALID_ARG, "X and Y must be 16-byte aligned");
    if (p->nrows == 0) return;
    launch_spmm(*p, X, Y, n, (hipStream_t)stream);
  });
}

sable_status sable_update_values(sable_plan_t p, const float* values, void* stream) {
  return guard([&] {
    if (!p || (!values && p->nnz)) SB_THROW(SABLE_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (p->nnz) {
      k_update_values<float><<<grid_for(p->nnz, 256), 256, 0, s>>>(values, p->nnz, p->owner.p, p->slot.p,
                                                            p->vdia_val.p, p->vbr_val.p,
                                                            p->csr_val.p, p->a_val.p);
      LAUNCH_CHECK();
    }
    if (p->vbr_cells && (p->flags & SABLE_F_SPLIT_BF16)) {
      build_bf16_split(*p, s);
      pack_mm_panels(*p, s);
    }
    refresh_far_values(*p, s);
  });
}

sable_status sable_update_values_f64(sable_plan_t p, const double* values, void* stream) {
  return guard([&] {
    if (!p || (!values && p->nnz)) SB_THROW(SABLE_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (!p->has_f64) {  // first call: fp64 arrays, fill cells zero
      p->vdia_val64.alloc(std::max<i64>(1, p->vdia_cells));
      p->vbr_val64.alloc(std::max<i64>(1, p->vbr_cells));
      p->csr_val64.alloc(std::max<i64>(1, p->csr_nnz));
      HIPC(hipMemsetAsync(p->vdia_val64.p, 0, p->vdia_val64.bytes(), s));
      HIPC(hipMemsetAsync(p->vbr_val64.p, 0, p->vbr_val64.bytes(), s));
      HIPC(hipMemsetAsync(p->csr_val64.p, 0, p->csr_val64.bytes(), s));
    }
    if (p->nnz) {
      k_update_values<double><<<grid_for(p->nnz, 256), 256, 0, s>>>(
          values, p->nnz, p->owner.p, p->slot.p, p->vdia_val64.p, p->vbr_val64.p, p->csr_val64.p,
          nullptr);
      LAUNCH_CHECK();
    }
    refresh_far_values64(*p, s);
    p->has_f64 = true;
  });
}

sable_status sable_spmv_f64(sable_plan_t p, const double* x, double* y, void* stream) {
  return guard([&] {
    if (!p || (!x && p->ncols) || (!y && p->nrows)) SB_THROW(SABLE_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_f64) SB_THROW(SABLE_ERR_INVALID_ARG, "no fp64 values: call sable_update_values_f64 first");
    if (p->nrows == 0) return;
    launch_spmv_f64(*p, x, y, (hipStream_t)stream);
  });
}

sable_status sable_spmm_f64(sable_plan_t p, const double* X, double* Y, int32_t n, void* stream) {
  return guard([&] {
    if (!p || n < 1 || (!X && p->ncols) || (!Y && p->nrows))
      SB_THROW(SABLE_ERR_INVALID_ARG, "NULL argument or n < 1");
    if (!p->has_f64) SB_THROW(SABLE_ERR_INVALID_ARG, "no fp64 values: call sable_update_values_f64 first");
    if (p->nrows == 0) return;
    launch_spmm_f64(*p, X, Y, n, (hipStream_t)stream);
  });
}

sable_status sable_error_norm_f64(const float* y, const double* yref, int64_t len, void* stream,
                                  double* out) {
  return guard([&] {
    if (!out || len < 0 || (len > 0 && (!y || !yref))) SB_THROW(SABLE_ERR_INVALID_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    const int nb = norm_parts(len);
    DBuf<double> part(2 * (size_t)nb), res(1);
    k_norm_partial<<<nb, kNormThreads, 0, s>>>(y, yref, len, part.p);
    LAUNCH_CHECK();
    k_norm_final<<<1, 1, 0, s>>>(part.p, nb, res.p);
    LAUNCH_CHECK();
    double h = 0.0;
    HIPC(hipMemcpyAsync(&h, res.p, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    *out = h;
  });
}

sable_status sable_error_norm_f64_noalloc(const float* y, const double* yref, int64_t len,
                                          void* stream, double* out_dev) {
  return guard([&] {
    if (!out_dev || len < 0 || (len > 0 && (!y || !yref)))
      SB_THROW(SABLE_ERR_INVALID_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    const int nb = norm_parts(len);
    double* part = scratch_for_current_device();
    // k_norm_partial writes all 2 nb slots it uses, so nothing needs clearing
    k_norm_partial<<<nb, kNormThreads, 0, s>>>(y, yref, len, part);
    LAUNCH_CHECK();
    k_norm_final<<<1, 1, 0, s>>>(part, nb, out_dev);
    LAUNCH_CHECK();
  });
}

}  // extern "C"
