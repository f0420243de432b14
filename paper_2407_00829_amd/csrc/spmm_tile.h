// Fused SpMM tile body: Y[tile rows, column chunk] = A X over bands, blocks and CSR.
//
// A workgroup (4 waves) owns kMmRows output rows and up to kMmCols columns of Y, held in LDS.
//  1. bands (VALU fp32): lanes across columns, one row per lane group; each cell's value is
//     broadcast and multiplied with a coalesced row of X;
//  2. blocks (matrix cores): every block overlapping the tile is a dense (rows x w) operand.
//     With bf16 copies present, each 16x16x16 step runs three bf16 products with fp32
//     accumulation, hi*hi + hi*lo + lo*hi (a = hi + lo split of the fp32 values, X split on
//     the fly), i.e. split-precision products that keep ~16 significant bits per operand.
//     Wave w owns the 16-column chunks w, w+4, ... so each Y element is updated by one lane
//     in block order. Without bf16 copies blocks run in fp32 on the VALU.
//  3. CSR (VALU fp32) accumulated separately, then Y = (bands + blocks) + CSR is stored.
// Every element has a fixed summation order, so results are bitwise reproducible.
#pragma once

#include "exec.h"

namespace sable {

constexpr int kMmRows = 64;
constexpr int kMmCols = 128;
constexpr int kMmThreads = 256;

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf16_rne_dev(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Rows [r0, r0+kMmRows) x columns [cb, cb+nc) of Y; ys = LDS (kMmRows x kMmCols floats).
// tile256 = index of the 256-row schedule tile containing r0 (its lists are a superset).
__device__ __forceinline__ void spmm_tile(const PlanView& P, int r0, int cb, int n,
                                          const float* __restrict__ X, float* __restrict__ Y,
                                          float* __restrict__ ys, bool use_mfma) {
  const int nc = min(kMmCols, n - cb);
  const int rend = min(r0 + kMmRows, P.nrows);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // lanes per row (power of two >= nc/2, at most 64) and rows per wave step
  int lpr = 64;
  while (lpr > 1 && lpr / 2 >= (nc + 1) / 2) lpr >>= 1;
  const int rpw = 64 / lpr;
  const int sub = lane / lpr, cl = lane % lpr;
  const int cA = cl, cB = cl + lpr;  // this lane's (up to) two columns within the chunk
  const bool okA = cA < nc, okB = cB < nc;
  const int tile = r0 / P.rows_per_tile;

  // 1. bands
  for (int rl = wave * rpw + sub; rl < kMmRows; rl += 4 * rpw) {
    const int r = r0 + rl;
    float a0 = 0.f, a1 = 0.f;
    if (r < rend) {
      for (int s = P.tile_seg_lo[tile]; s < P.tile_seg_hi[tile]; ++s) {
        const int rs = P.seg_row_start[s], nr = P.seg_nrows[s];
        if (r < rs || r >= rs + nr) continue;
        const int nd = P.seg_ndiags[s];
        const int32_t* od = P.idiag + P.seg_idiag_ptr[s];
        const float* v = P.vdia_val + P.seg_val_ptr[s] + (r - rs);
        for (int d = 0; d < nd; ++d) {
          const int c = r + od[d];
          if ((unsigned)c >= (unsigned)P.ncols) continue;
          const float a = v[(i64)d * nr];
          const float* xr = X + (i64)c * n + cb;
          if (okA) a0 += a * xr[cA];
          if (okB) a1 += a * xr[cB];
        }
      }
    }
    ys[rl * kMmCols + cA] = a0;
    if (cB < kMmCols) ys[rl * kMmCols + cB] = a1;
  }
  __syncthreads();

  // 2. blocks
  const int blo = P.tile_blk_ptr[tile], bhi = P.tile_blk_ptr[tile + 1];
  for (int qb = blo; qb < bhi; ++qb) {
    const int b = P.tile_blk[qb];
    const int br0 = P.blk[4 * b], br1 = P.blk[4 * b + 1];
    const int lo = max(br0, r0), hi = min(br1, rend);
    if (lo >= hi) continue;
    const int c0 = P.blk[4 * b + 2], c1 = P.blk[4 * b + 3];
    const int h = br1 - br0, w = c1 - c0;
    const i64 vp = P.blk_val_ptr[b];
    if (use_mfma) {
      const int m = lane & 15, kg = lane >> 4;  // MFMA operand coordinates of this lane
      for (int nch = wave; nch * 16 < nc; nch += 4) {
        const int col = nch * 16 + m;  // B / D column within the chunk
        const bool cok = col < nc;
        for (int mt = lo; mt < hi; mt += 16) {
          floatx4_t acc = {0.f, 0.f, 0.f, 0.f};
          const int arow = mt + m;  // A row of this lane
          const bool rok = arow < hi;
          for (int k0 = 0; k0 < w; k0 += 16) {
            bf16x4_t ahi, alo, bhi, blo2;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int k = k0 + 4 * kg + i;
              uint16_t h16 = 0, l16 = 0;
              if (rok && k < w) {
                const i64 at = vp + (i64)k * h + (arow - br0);
                h16 = P.vbr_hi[at];
                l16 = P.vbr_lo[at];
              }
              ahi[i] = (short)h16;
              alo[i] = (short)l16;
              float xv = 0.f;
              if (cok && k < w) xv = X[(i64)(c0 + k) * n + cb + col];
              const uint16_t xh = bf16_rne_dev(xv);
              const uint16_t xl = bf16_rne_dev(xv - bf16_f32(xh));
              bhi[i] = (short)xh;
              blo2[i] = (short)xl;
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo2, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, acc, 0, 0, 0);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int orow = mt + 4 * kg + i;  // D row of this lane
            if (orow < hi && cok) ys[(orow - r0) * kMmCols + col] += acc[i];
          }
        }
      }
    } else {
      for (int rl = wave * rpw + sub; rl < kMmRows; rl += 4 * rpw) {
        const int r = r0 + rl;
        if (r < lo || r >= hi) continue;
        const float* v = P.vbr_val + vp + (r - br0);
        float a0 = 0.f, a1 = 0.f;
        for (int k = 0; k < w; ++k) {
          const float a = v[(i64)k * h];
          const float* xr = X + (i64)(c0 + k) * n + cb;
          if (okA) a0 += a * xr[cA];
          if (okB) a1 += a * xr[cB];
        }
        if (okA) ys[rl * kMmCols + cA] += a0;
        if (okB) ys[rl * kMmCols + cB] += a1;
      }
    }
    __syncthreads();
  }

  // 3. CSR, then store
  for (int rl = wave * rpw + sub; rl < kMmRows; rl += 4 * rpw) {
    const int r = r0 + rl;
    if (r >= rend) continue;
    float a0 = 0.f, a1 = 0.f;
    const int ke = P.csr_ptr[r + 1];
    int k = P.csr_ptr[r];
    for (; k + 2 <= ke; k += 2) {
      const float v0 = P.csr_val[k], v1 = P.csr_val[k + 1];
      const float* x0 = X + (i64)P.csr_col[k] * n + cb;
      const float* x1 = X + (i64)P.csr_col[k + 1] * n + cb;
      if (okA) { a0 += v0 * x0[cA]; a0 += v1 * x1[cA]; }
      if (okB) { a1 += v0 * x0[cB]; a1 += v1 * x1[cB]; }
    }
    for (; k < ke; ++k) {
      const float v0 = P.csr_val[k];
      const float* x0 = X + (i64)P.csr_col[k] * n + cb;
      if (okA) a0 += v0 * x0[cA];
      if (okB) a1 += v0 * x0[cB];
    }
    float* yr = Y + (i64)r * n + cb;
    if (okA) yr[cA] = ys[rl * kMmCols + cA] + a0;
    if (okB) yr[cB] = ys[rl * kMmCols + cB] + a1;
  }
}

}  // namespace sable
