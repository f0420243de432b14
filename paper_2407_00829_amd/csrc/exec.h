// Device view of a plan and the fused per-tile product bodies shared by the standalone
// launches and the persistent batched kernel.
#pragma once

#include "plan.h"

namespace sable {

struct PlanView {
  int nrows, ncols;
  int nseg, nblk;
  const float* vdia_val;
  const int32_t* idiag;
  const int32_t* seg_row_start;
  const int32_t* seg_nrows;
  const int32_t* seg_ndiags;
  const i64* seg_val_ptr;
  const int32_t* seg_idiag_ptr;
  const int32_t* blk;
  const i64* blk_val_ptr;
  const float* vbr_val;
  const uint16_t* vbr_hi;
  const uint16_t* vbr_lo;
  const int32_t* csr_ptr;
  const int32_t* csr_col;
  const float* csr_val;
  int rows_per_tile, ntiles;
  const int32_t* tile_seg_lo;
  const int32_t* tile_seg_hi;
  const int32_t* tile_blk_ptr;
  const int32_t* tile_blk;
};

PlanView make_view(const sable_plan_s& P, const Schedule& S, bool plain);

// ---- SpMV tile body --------------------------------------------------------------------
// blockDim.x == rows_per_tile threads; thread t owns row tile*rows_per_tile + t for the band
// and block parts (lane per row: diagonal-major / column-major values are contiguous across
// consecutive rows). The CSR part then runs W lanes per row with a shuffle reduction; the
// per-row band+block partial goes through LDS. Every row's sum has a fixed order:
// y = (sum over segments, diagonals ascending + sum over blocks, columns ascending)
//     + (CSR entries in index order, reduced by a fixed xor tree).
template <int W>
__device__ __forceinline__ void spmv_tile(const PlanView& P, int tile, const float* __restrict__ x,
                                          float* __restrict__ y, float* __restrict__ part) {
  const int RT = P.rows_per_tile;
  const int r0 = tile * RT;
  const int r = r0 + threadIdx.x;
  const bool act = r < P.nrows;
  float acc = 0.f;
  const int slo = P.tile_seg_lo[tile], shi = P.tile_seg_hi[tile];
  for (int s = slo; s < shi; ++s) {
    const int rs = P.seg_row_start[s], nr = P.seg_nrows[s];
    if (act && r >= rs && r < rs + nr) {
      const int nd = P.seg_ndiags[s];
      const int32_t* od = P.idiag + P.seg_idiag_ptr[s];
      const float* v = P.vdia_val + P.seg_val_ptr[s] + (r - rs);
      for (int t = 0; t < nd; ++t) {
        const int c = r + od[t];
        if ((unsigned)c < (unsigned)P.ncols) acc += v[(i64)t * nr] * x[c];
      }
    }
  }
  const int blo = P.tile_blk_ptr[tile], bhi = P.tile_blk_ptr[tile + 1];
  for (int q = blo; q < bhi; ++q) {
    const int b = P.tile_blk[q];
    const int br0 = P.blk[4 * b], br1 = P.blk[4 * b + 1];
    if (act && r >= br0 && r < br1) {
      const int c0 = P.blk[4 * b + 2], c1 = P.blk[4 * b + 3];
      const int h = br1 - br0;
      const float* v = P.vbr_val + P.blk_val_ptr[b] + (r - br0);
      for (int c = c0; c < c1; ++c) acc += v[(i64)(c - c0) * h] * x[c];
    }
  }
  if (W == 1) {
    float cs = 0.f;
    if (act)
      for (int k = P.csr_ptr[r]; k < P.csr_ptr[r + 1]; ++k) cs += P.csr_val[k] * x[P.csr_col[k]];
    if (act) y[r] = acc + cs;
    return;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  const int lane = threadIdx.x & (W - 1);
  const int grp = threadIdx.x / W;
  const int ngrp = RT / W;
  for (int rl = grp; rl < RT; rl += ngrp) {
    const int rr = r0 + rl;
    float cs = 0.f;
    if (rr < P.nrows) {
      const int ke = P.csr_ptr[rr + 1];
      for (int k = P.csr_ptr[rr] + lane; k < ke; k += W) cs += P.csr_val[k] * x[P.csr_col[k]];
    }
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) cs += __shfl_xor(cs, o, W);
    if (lane == 0 && rr < P.nrows) y[rr] = part[rl] + cs;
  }
}

// Plain CSR SpMV body: W lanes per row over the whole matrix (the baseline family).
template <int W>
__device__ __forceinline__ void csr_rows(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                         const float* __restrict__ val, int nrows,
                                         const float* __restrict__ x, float* __restrict__ y,
                                         int row_begin, int nrows_here) {
  const int lane = threadIdx.x & (W - 1);
  const int grp = threadIdx.x / W;
  const int ngrp = blockDim.x / W;
  for (int rl = grp; rl < nrows_here; rl += ngrp) {
    const int r = row_begin + rl;
    float cs = 0.f;
    if (r < nrows) {
      const int ke = ptr[r + 1];
      for (int k = ptr[r] + lane; k < ke; k += W) cs += val[k] * x[col[k]];
    }
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) cs += __shfl_xor(cs, o, W);
    if (lane == 0 && r < nrows) y[r] = cs;
  }
}

}  // namespace sable
