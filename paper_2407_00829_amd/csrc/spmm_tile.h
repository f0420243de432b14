// Fused SpMM tile body: Y[tile rows, column chunk] = A X over bands, blocks and CSR.
//
// A workgroup (4 waves) owns kMmRows output rows and up to kMmCols columns of Y, held in LDS.
//  1. bands (VALU fp32): lanes across columns, one row per lane group; each cell's value is
//     broadcast and multiplied with a coalesced row of X;
//  2. blocks (matrix cores): every block overlapping the tile is a dense (rows x w) operand,
//     zero-padded to 16-row slices and 16-wide k steps. With bf16 copies present, each
//     16x16x16 step runs three bf16 products with fp32 accumulation, hi*hi + hi*lo + lo*hi
//     (a = hi + lo split of the fp32 values, X split on the fly), i.e. split-precision
//     products that keep ~16 significant bits per operand. Wave w owns the 16-column chunks
//     w and w+4 and keeps their accumulators for all four row slices in registers across all
//     blocks (block order), so there is no synchronisation between blocks and each X
//     fragment serves every row slice; the sums are then added to the band partial.
//     Without bf16 copies blocks run in fp32 on the VALU.
//  3. CSR (VALU fp32, eight X rows in flight per lane) accumulated separately, then
//     Y = (bands + blocks) + CSR is stored.
// Every element has a fixed summation order, so results are bitwise reproducible.
#pragma once

#include "exec.h"

namespace sable {

constexpr int kMmRows = 64;
constexpr int kMmCols = 128;
constexpr int kMmThreads = 256;
constexpr int kMmBlkStage = 256;  // block descriptors staged in LDS per pass
constexpr int kBlkDesc = 8;       // ints per staged descriptor

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf16_rne_dev(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Copy nq block descriptors of the tile list (starting at q0) into LDS, all threads.
__device__ __forceinline__ void stage_blocks(const PlanView& P, int q0, int nq, int* sb) {
  __syncthreads();  // the previous pass is done with sb
  for (int j = threadIdx.x; j < nq; j += blockDim.x) {
    const int b = P.tile_blk[q0 + j];
    const i64 vp = P.blk_val_ptr[b];
    const i64 mp = P.blk_mma_ptr ? P.blk_mma_ptr[b] : 0;
    int* d = sb + kBlkDesc * j;
    d[0] = P.blk[4 * b];
    d[1] = P.blk[4 * b + 1];
    d[2] = P.blk[4 * b + 2];
    d[3] = P.blk[4 * b + 3];
    d[4] = (int)(uint32_t)((uint64_t)vp & 0xffffffffu);
    d[5] = (int)(uint32_t)((uint64_t)vp >> 32);
    d[6] = (int)(uint32_t)((uint64_t)mp & 0xffffffffu);
    d[7] = (int)(uint32_t)((uint64_t)mp >> 32);
  }
  __syncthreads();
}

// Rows [r0, r0+kMmRows) x columns [cb, cb+nc) of Y. lds = kMmRows x kMmCols floats for the
// tile of Y, then kMmBlkStage block descriptors (r0, r1, c0, c1, value offset). The view's
// schedule has tiles of kMmRows rows, so tile lists hold exactly the overlapping blocks.
__device__ __forceinline__ void spmm_tile(const PlanView& P, int r0, int cb, int n,
                                          const float* __restrict__ X, float* __restrict__ Y,
                                          float* __restrict__ ys, bool use_mfma) {
  int* sb = reinterpret_cast<int*>(ys + kMmRows * kMmCols);  // [kMmBlkStage][kBlkDesc]
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
  if (use_mfma) {
    // Wave w owns the 16-column chunks w and w+4 of this column block and all four 16-row
    // slices of the tile; products accumulate in registers over the tile's blocks in block
    // order, then are added to the band partial in LDS.
    floatx4_t acc[4][2];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int ci = 0; ci < 2; ++ci) acc[mt][ci] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    const int m = lane & 15, kg = lane >> 4;  // MFMA operand coordinates of this lane
    for (int q0 = blo; q0 < bhi; q0 += kMmBlkStage) {
     const int nq = min(kMmBlkStage, bhi - q0);
     stage_blocks(P, q0, nq, sb);
     for (int j = 0; j < nq; ++j) {
      const int* dsc = sb + kBlkDesc * j;
      const int br0 = dsc[0], br1 = dsc[1];
      const int lo = max(br0, r0), hi = min(br1, rend);
      if (lo >= hi) continue;
      const int c0 = dsc[2], c1 = dsc[3];
      const int w = c1 - c0, w4 = (w + 3) & ~3;
      const i64 mp = (i64)(((uint64_t)(uint32_t)dsc[7] << 32) | (uint32_t)dsc[6]);
      for (int k0 = 0; k0 < w; k0 += 16) {
        const int kk = k0 + 4 * kg;  // first of this lane's four k values
        // B fragments (both column chunks) and A fragments (every 16-row slice) first
        bf16x4_t bh[2], bl[2];
#pragma unroll
        for (int ci = 0; ci < 2; ++ci) {
          const int col = (wave + 4 * ci) * 16 + m;
          const bool cok = col < nc;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = kk + i;
            const float xv = (cok && k < w) ? X[(i64)(c0 + k) * n + cb + col] : 0.f;
            const uint16_t xh = bf16_rne_dev(xv);
            bh[ci][i] = (short)xh;
            bl[ci][i] = (short)bf16_rne_dev(xv - bf16_f32(xh));
          }
        }
        uint4 aw[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const int arow = r0 + 16 * mt + m;
          aw[mt] = make_uint4(0u, 0u, 0u, 0u);
          if (arow >= lo && arow < hi && kk < w4)
            aw[mt] = *reinterpret_cast<const uint4*>(P.vbr_mma + mp + (i64)(arow - br0) * w4 + kk);
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const int m0 = r0 + 16 * mt;
          if (m0 >= hi || m0 + 16 <= lo) continue;
          bf16x4_t ah, al;
          ah[0] = (short)(aw[mt].x & 0xffffu); al[0] = (short)(aw[mt].x >> 16);
          ah[1] = (short)(aw[mt].y & 0xffffu); al[1] = (short)(aw[mt].y >> 16);
          ah[2] = (short)(aw[mt].z & 0xffffu); al[2] = (short)(aw[mt].z >> 16);
          ah[3] = (short)(aw[mt].w & 0xffffu); al[3] = (short)(aw[mt].w >> 16);
#pragma unroll
          for (int ci = 0; ci < 2; ++ci) {
            if ((wave + 4 * ci) * 16 >= nc) continue;
            acc[mt][ci] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh[ci], acc[mt][ci], 0, 0, 0);
            acc[mt][ci] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl[ci], acc[mt][ci], 0, 0, 0);
            acc[mt][ci] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh[ci], acc[mt][ci], 0, 0, 0);
          }
        }
      }
     }
    }
    if (blo < bhi) {
#pragma unroll
      for (int ci = 0; ci < 2; ++ci) {
        const int col = (wave + 4 * ci) * 16 + m;
        if (col >= nc) continue;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
          for (int i = 0; i < 4; ++i) ys[(16 * mt + 4 * kg + i) * kMmCols + col] += acc[mt][ci][i];
      }
      __syncthreads();
    }
  } else {
    for (int q0 = blo; q0 < bhi; q0 += kMmBlkStage) {
     const int nq = min(kMmBlkStage, bhi - q0);
     stage_blocks(P, q0, nq, sb);
     for (int j = 0; j < nq; ++j) {
      const int* dsc = sb + kBlkDesc * j;
      const int br0 = dsc[0], br1 = dsc[1];
      const int lo = max(br0, r0), hi = min(br1, rend);
      if (lo >= hi) continue;
      const int c0 = dsc[2], c1 = dsc[3];
      const int h = br1 - br0, w = c1 - c0;
      const i64 vp = (i64)(((uint64_t)(uint32_t)dsc[5] << 32) | (uint32_t)dsc[4]);
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
    // eight X rows in flight per lane
    for (; k + 8 <= ke; k += 8) {
      float va[8], xa[8], xb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        va[u] = P.csr_val[k + u];
        const float* xr = X + (i64)P.csr_col[k + u] * n + cb;
        xa[u] = okA ? xr[cA] : 0.f;
        xb[u] = okB ? xr[cB] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a0 += va[u] * xa[u];
        a1 += va[u] * xb[u];
      }
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
