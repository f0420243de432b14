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
//     Without bf16 copies, or when the fp32 VALU variant is chosen, blocks run on the VALU
//     in the operand type (each loaded row of X multiplied into up to 8 block rows).
//  3. CSR (VALU, several X rows in flight per lane; when one wave covers a row, its indices
//     and values are loaded 64 at a time and broadcast with readlane) accumulated
//     separately, then Y = (bands + blocks) + CSR is stored.
// Every element has a fixed summation order, so results are bitwise reproducible.
#pragma once

#include "exec.h"

namespace sable {

// Staged block descriptor word: the same for every lane, so it goes to a scalar register
// (block bookkeeping then runs as scalar control flow, not per lane).
__device__ __forceinline__ int desc(const int* d, int i) { return __builtin_amdgcn_readfirstlane(d[i]); }

// Lane l's value of v, for every lane (l wave-uniform).
__device__ __forceinline__ float readlane_val(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane_val(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

constexpr int kMmRows = 64;
constexpr int kMmCols = 128;
constexpr int kMmThreads = 256;
constexpr int kMmBlkStage = 256;  // block descriptors staged in LDS per pass
constexpr int kBlkDesc = 8;       // ints per staged descriptor
constexpr int kMmBatch = 3;       // small blocks whose operand loads are issued together

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

// Packed A fragment (four hi|lo words); read once per product, so loaded non-temporally to
// leave the caches to X, the operand with reuse.
__device__ __forceinline__ uint4 ld_afrag(const uint32_t* p) {
  const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
  return make_uint4(v[0], v[1], v[2], v[3]);
}
typedef float floatx4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf16_rne_dev(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

typedef __bf16 bf16x2v_t __attribute__((ext_vector_type(2)));
typedef float float2v_t __attribute__((ext_vector_type(2)));

// Split four fp32 values into bf16 hi and lo parts (x = hi + lo + O(2^-16 |x|)) with the
// hardware round-to-nearest-even conversion, two values per instruction.
__device__ __forceinline__ void split4(const float (&x)[4], bf16x4_t& hi, bf16x4_t& lo) {
  const uint32_t h01 = __builtin_bit_cast(uint32_t, __builtin_convertvector(float2v_t{x[0], x[1]}, bf16x2v_t));
  const uint32_t h23 = __builtin_bit_cast(uint32_t, __builtin_convertvector(float2v_t{x[2], x[3]}, bf16x2v_t));
  const float2v_t r01 = {x[0] - __uint_as_float(h01 << 16), x[1] - __uint_as_float(h01 & 0xffff0000u)};
  const float2v_t r23 = {x[2] - __uint_as_float(h23 << 16), x[3] - __uint_as_float(h23 & 0xffff0000u)};
  const uint32_t l01 = __builtin_bit_cast(uint32_t, __builtin_convertvector(r01, bf16x2v_t));
  const uint32_t l23 = __builtin_bit_cast(uint32_t, __builtin_convertvector(r23, bf16x2v_t));
  hi = __builtin_bit_cast(bf16x4_t, make_uint2(h01, h23));
  lo = __builtin_bit_cast(bf16x4_t, make_uint2(l01, l23));
}

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

// Which part of the tile's products a wave computes on the matrix cores: 16-column chunks
// c0 and c0 + cstep of the column block, for the 16-row slices whose bit is set in smask.
// Wide column blocks (more than 32 columns) split the chunks over the waves (c0 = wave,
// cstep = 4, every slice); narrow ones (n <= 32) split the slices (c0 = 0, cstep = 1, slice
// wave only), so all four waves have work.
struct MmPart {
  int c0, cstep, smask;
};

// Three split-bf16 products of one 16x16x16 step into acc[0..1] (the wave's two column
// chunks): a = packed hi|lo words of this lane's four k values, b = X fragments.
__device__ __forceinline__ void mfma3(floatx4_t (&acc)[2], const uint4& aw, const bf16x4_t (&bh)[2],
                                      const bf16x4_t (&bl)[2], const MmPart& mp, int nc) {
  bf16x4_t ah, al;
  ah[0] = (short)(aw.x & 0xffffu); al[0] = (short)(aw.x >> 16);
  ah[1] = (short)(aw.y & 0xffffu); al[1] = (short)(aw.y >> 16);
  ah[2] = (short)(aw.z & 0xffffu); al[2] = (short)(aw.z >> 16);
  ah[3] = (short)(aw.w & 0xffffu); al[3] = (short)(aw.w >> 16);
#pragma unroll
  for (int ci = 0; ci < 2; ++ci) {
    if ((mp.c0 + mp.cstep * ci) * 16 >= nc) continue;
    acc[ci] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh[ci], acc[ci], 0, 0, 0);
    acc[ci] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl[ci], acc[ci], 0, 0, 0);
    acc[ci] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh[ci], acc[ci], 0, 0, 0);
  }
}

// cnt (1..kMmBatch) items: k step ik[s] (a multiple of 16) of staged block sb[ib[s]], each
// block overlapping at most two consecutive 16-row slices of the tile. Every operand load of
// the batch is issued first, then the products run item by item (slices ascending), the
// order of the general path.
__device__ __forceinline__ void mfma_small_batch(const PlanView& P, const int* sb, const int (&ib)[kMmBatch],
                                                 const int (&ik)[kMmBatch],
                                                 int cnt, int r0, int rend, int cb, int n, int nc,
                                                 const float* __restrict__ X, const MmPart& part,
                                                 int m, int kg, floatx4_t (&acc)[4][2]) {
  float xr[kMmBatch][2][4];
  uint4 aw[kMmBatch][2];
  int ma[kMmBatch], nsl[kMmBatch];
#pragma unroll
  for (int s = 0; s < kMmBatch; ++s) {
    const bool sv = s < cnt;
    const int* d = sb + kBlkDesc * ib[sv ? s : 0];
    const int k0 = ik[sv ? s : 0];
    const int br0 = desc(d, 0), c0 = desc(d, 2), w = desc(d, 3) - c0;
    const int w4 = (w + 3) & ~3;
    const int lo = max(br0, r0), hi = min(desc(d, 1), rend);
    const i64 mp = (i64)(((uint64_t)(uint32_t)desc(d, 7) << 32) | (uint32_t)desc(d, 6));
    ma[s] = (lo - r0) >> 4;
    nsl[s] = sv ? ((hi - 1 - r0) >> 4) - ma[s] + 1 : 0;
    // every load is issued (addresses clamped into the block and into X) and masked after
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = k0 + 4 * kg + i;
      const float* xrow = X + (i64)(c0 + min(k, w - 1)) * n + cb;
#pragma unroll
      for (int ci = 0; ci < 2; ++ci) {
        const int col = (part.c0 + part.cstep * ci) * 16 + m;
        xr[s][ci][i] = xrow[min(col, nc - 1)];
        if (!(sv && col < nc && k < w)) xr[s][ci][i] = 0.f;
      }
    }
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int arow = r0 + 16 * (ma[s] + sl) + m;
      const int ar = min(max(arow, lo), hi - 1), ak = min(k0 + 4 * kg, w4 - 4);
      aw[s][sl] = ld_afrag(P.vbr_mma + mp + (i64)(ar - br0) * w4 + ak);
      if (!(sl < nsl[s] && arow >= lo && arow < hi && k0 + 4 * kg < w4)) aw[s][sl] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
#pragma unroll
  for (int s = 0; s < kMmBatch; ++s) {
    if (s >= cnt) break;
    bf16x4_t bh[2], bl[2];
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) split4(xr[s][ci], bh[ci], bl[ci]);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {  // slices ascending; ma[s] is wave-uniform
      const int sl = mt - ma[s];
      if (sl < 0 || sl >= nsl[s] || !((part.smask >> mt) & 1)) continue;
      mfma3(acc[mt], sl == 0 ? aw[s][0] : aw[s][1], bh, bl, part, nc);
    }
  }
}

// Blocks on the VALU in the tile's value type: lanes across columns, each loaded row of X
// multiplied into up to 8 block rows; block partials are added to the band partials in ys
// (the tile of Y in LDS).
static_assert(kMmRows == 64, "the VALU block path gives each of the 4 waves 16 tile rows");
template <class T>
__device__ __forceinline__ void spmm_blocks_valu(const PlanView& P, int* sb, int blo, int bhi, int r0,
                                                 int rend, int cb, int n, const T* __restrict__ X,
                                                 T* __restrict__ ys, int wave, int rpw, int sub,
                                                 int cA, int cB, bool okA, bool okB) {
  // Wave w owns tile rows [16 w, 16 w + 16). A block's rows in that range go in chunks of up
  // to 8 rows per lane group (rows rc + sub + rpw i); each block column k loads one row of X
  // (two columns per lane) and multiplies it into every row of the chunk, so a loaded row of
  // X serves all rows of the block; two block columns are in flight together. Per row and
  // column: block columns ascending, blocks in tile-list order.
  const int wr0 = r0 + 16 * wave, wr1 = min(r0 + 16 * wave + 16, rend);
  const int cAc = okA ? cA : 0, cBc = okB ? cB : 0;  // loads stay inside the chunk
  for (int q0 = blo; q0 < bhi; q0 += kMmBlkStage) {
    const int nq = min(kMmBlkStage, bhi - q0);
    stage_blocks(P, q0, nq, sb);  // also orders the band phase's LDS writes before these
    for (int j = 0; j < nq; ++j) {
      const int* dsc = sb + kBlkDesc * j;
      const int br0 = desc(dsc, 0), br1 = desc(dsc, 1);
      const int a = max(br0, wr0), b = min(br1, wr1);
      if (a >= b) continue;
      const int c0 = desc(dsc, 2), c1 = desc(dsc, 3);
      const int h = br1 - br0, w = c1 - c0;
      const i64 vp = (i64)(((uint64_t)(uint32_t)desc(dsc, 5) << 32) | (uint32_t)desc(dsc, 4));
      const T* vb = Vals<T>::vbr(P) + vp;  // cell (r, c0 + k) at vb[k h + r - br0]
      for (int rc = a; rc < b; rc += 8 * rpw) {
        T accA[8], accB[8];
        int off[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int row = rc + sub + rpw * i;
          off[i] = (row < b ? row : a) - br0;  // rows past the chunk read a valid cell
          accA[i] = 0;
          accB[i] = 0;
        }
        int k = 0;
        for (; k + 2 <= w; k += 2) {
          T xa[2], xb[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const T* xr = X + (i64)(c0 + k + u) * n + cb;
            xa[u] = xr[cAc];
            xb[u] = xr[cBc];
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const T* vk = vb + (i64)(k + u) * h;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const T av = vk[off[i]];
              accA[i] += av * xa[u];
              accB[i] += av * xb[u];
            }
          }
        }
        for (; k < w; ++k) {
          const T* xr = X + (i64)(c0 + k) * n + cb;
          const T xa = xr[cAc], xb = xr[cBc];
          const T* vk = vb + (i64)k * h;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const T av = vk[off[i]];
            accA[i] += av * xa;
            accB[i] += av * xb;
          }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int row = rc + sub + rpw * i;
          if (row >= b) continue;
          T* yr = ys + (row - r0) * kMmCols;
          if (okA) yr[cA] += accA[i];
          if (okB) yr[cB] += accB[i];
        }
      }
    }
  }
  __syncthreads();
}

// Rows [r0, r0+kMmRows) x columns [cb, cb+nc) of Y. lds = kMmRows x kMmCols floats for the
// tile of Y, then kMmBlkStage block descriptors (r0, r1, c0, c1, value offset). The view's
// schedule has tiles of kMmRows rows, so tile lists hold exactly the overlapping blocks.
// mfma: 0 = blocks on the VALU, 1 = matrix cores with the automatic work split (slices over
// the waves for n <= 32 columns, chunks otherwise), 2 = matrix cores, chunks over the waves.
template <class T = float>
__device__ __forceinline__ void spmm_tile(const PlanView& P, int r0, int cb, int n,
                                          const T* __restrict__ X, T* __restrict__ Y,
                                          float* __restrict__ lds, int mfma) {
  T* ys = reinterpret_cast<T*>(lds);                          // kMmRows x kMmCols values of T
  int* sb = reinterpret_cast<int*>(ys + kMmRows * kMmCols);  // [kMmBlkStage][kBlkDesc]
  const int nc = min(kMmCols, n - cb);
  const int rend = min(r0 + kMmRows, P.nrows);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
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
    T a0 = 0, a1 = 0;
    if (r < rend) {
      for (int s = P.tile_seg_lo[tile]; s < P.tile_seg_hi[tile]; ++s) {
        const int rs = P.seg_row_start[s], nr = P.seg_nrows[s];
        if (r < rs || r >= rs + nr) continue;
        const int nd = P.seg_ndiags[s];
        const int32_t* od = P.idiag + P.seg_idiag_ptr[s];
        const T* v = Vals<T>::vdia(P) + P.seg_val_ptr[s] + (r - rs);
        for (int d = 0; d < nd; ++d) {
          const int c = r + od[d];
          if ((unsigned)c >= (unsigned)P.ncols) continue;
          const T a = v[(i64)d * nr];
          const T* xr = X + (i64)c * n + cb;
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
  if constexpr (sizeof(T) == 4) {  // matrix cores for the fp32 executor only
   if (mfma) {
    // Each wave owns part of the products (MmPart: two 16-column chunks and a set of 16-row
    // slices); they accumulate in registers over the tile's blocks in block order, then are
    // added to the band partial in LDS. Every output element sees the same operations in
    // either split, so results do not depend on it.
    floatx4_t acc[4][2];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int ci = 0; ci < 2; ++ci) acc[mt][ci] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    const int m = lane & 15, kg = lane >> 4;  // MFMA operand coordinates of this lane
    const MmPart part = (mfma == 1 && nc <= 32) ? MmPart{0, 1, 1 << wave} : MmPart{wave, 4, 0xF};
    for (int q0 = blo; q0 < bhi; q0 += kMmBlkStage) {
     const int nq = min(kMmBlkStage, bhi - q0);
     stage_blocks(P, q0, nq, sb);
     int j = 0, kstart = 0;  // next block and its next 16-wide k step
     while (j < nq) {
      // up to kMmBatch (block, k step) items of blocks overlapping at most two 16-row
      // slices of the tile go together: all their operand loads are issued before any of
      // their products, which then run in (block, k step, slice) order as in the general
      // path below
      int ib[kMmBatch], ik[kMmBatch];
      int cnt = 0, jj = j, kk0 = kstart;
      while (cnt < kMmBatch && jj < nq) {
        const int* d = sb + kBlkDesc * jj;
        const int lo = max(desc(d, 0), r0), hi = min(desc(d, 1), rend);
        if (lo >= hi) { ++jj; kk0 = 0; continue; }
        if (((hi - 1 - r0) >> 4) - ((lo - r0) >> 4) > 1) break;
        ib[cnt] = jj;
        ik[cnt] = kk0;
        ++cnt;
        kk0 += 16;
        if (kk0 >= desc(d, 3) - desc(d, 2)) { ++jj; kk0 = 0; }
      }
      if (cnt > 0) {
        mfma_small_batch(P, sb, ib, ik, cnt, r0, rend, cb, n, nc, X, part, m, kg, acc);
        j = jj;
        kstart = kk0;
        continue;
      }
      if (jj >= nq) break;
      // general block jj: any width and height
      const int* dsc = sb + kBlkDesc * jj;
      j = jj + 1;
      kstart = 0;
      const int br0 = desc(dsc, 0), br1 = desc(dsc, 1);
      const int lo = max(br0, r0), hi = min(br1, rend);
      const int c0 = desc(dsc, 2), c1 = desc(dsc, 3);
      const int w = c1 - c0, w4 = (w + 3) & ~3;
      const i64 mp = (i64)(((uint64_t)(uint32_t)desc(dsc, 7) << 32) | (uint32_t)desc(dsc, 6));
      for (int k0 = 0; k0 < w; k0 += 16) {
        const int kk = k0 + 4 * kg;  // first of this lane's four k values
        // B fragments (both column chunks) and A fragments (every 16-row slice) first
        // every load is issued (addresses clamped into the block and into X), masked after
        float xr[2][4];
#pragma unroll
        for (int ci = 0; ci < 2; ++ci) {
          const int col = (part.c0 + part.cstep * ci) * 16 + m;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = kk + i;
            xr[ci][i] = X[(i64)(c0 + min(k, w - 1)) * n + cb + min(col, nc - 1)];
            if (!(col < nc && k < w)) xr[ci][i] = 0.f;
          }
        }
        uint4 aw[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const int arow = r0 + 16 * mt + m;
          const int ar = min(max(arow, lo), hi - 1), ak = min(kk, w4 - 4);
          aw[mt] = ld_afrag(P.vbr_mma + mp + (i64)(ar - br0) * w4 + ak);
          if (!(arow >= lo && arow < hi && kk < w4)) aw[mt] = make_uint4(0u, 0u, 0u, 0u);
        }
        bf16x4_t bh[2], bl[2];
#pragma unroll
        for (int ci = 0; ci < 2; ++ci) split4(xr[ci], bh[ci], bl[ci]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const int m0 = r0 + 16 * mt;
          if (m0 >= hi || m0 + 16 <= lo || !((part.smask >> mt) & 1)) continue;
          mfma3(acc[mt], aw[mt], bh, bl, part, nc);
        }
      }
     }
    }
    if (blo < bhi) {
#pragma unroll
      for (int ci = 0; ci < 2; ++ci) {
        const int col = (part.c0 + part.cstep * ci) * 16 + m;
        if (col >= nc) continue;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          if (!((part.smask >> mt) & 1)) continue;
#pragma unroll
          for (int i = 0; i < 4; ++i) ys[(16 * mt + 4 * kg + i) * kMmCols + col] += acc[mt][ci][i];
        }
      }
      __syncthreads();
    }
   } else {
    spmm_blocks_valu<T>(P, sb, blo, bhi, r0, rend, cb, n, X, ys, wave, rpw, sub, cA, cB, okA, okB);
   }
  } else {
    spmm_blocks_valu<T>(P, sb, blo, bhi, r0, rend, cb, n, X, ys, wave, rpw, sub, cA, cB, okA, okB);
  }

  // 3. CSR, then store
  for (int rl = wave * rpw + sub; rl < kMmRows; rl += 4 * rpw) {
    const int r = r0 + rl;
    if (r >= rend) continue;
    T a0 = 0, a1 = 0;
    const int ke = P.csr_ptr[r + 1];
    int k = P.csr_ptr[r];
    // eight X rows in flight per lane: indices and values first, then every X load
    // (columns clamped into the chunk, masked when used)
    const int cAc = min(cA, nc - 1), cBc = min(cB, nc - 1);
    if (rpw == 1) {
      // the whole wave is on this row: its entries are loaded 64 at a time, one per lane,
      // and handed to every lane with readlane (two index loads per 64 entries instead of
      // two per entry); the products are added in index order as below
      for (; k < ke; k += 64) {
        const int cnt = min(64, ke - k);
        const int kl = k + min(lane, cnt - 1);
        const int mc = __builtin_nontemporal_load(P.csr_col + kl);
        const T mv = __builtin_nontemporal_load(Vals<T>::csr(P) + kl);
        int u = 0;
        for (; u + 4 <= cnt; u += 4) {
          int cc[4];
          T va[4], xa[4], xb[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            cc[j] = __builtin_amdgcn_readlane(mc, u + j);
            va[j] = readlane_val(mv, u + j);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const T* xr = X + (i64)cc[j] * n + cb;
            xa[j] = xr[cAc];
            xb[j] = xr[cBc];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            a0 += va[j] * (okA ? xa[j] : T(0));
            a1 += va[j] * (okB ? xb[j] : T(0));
          }
        }
        for (; u < cnt; ++u) {
          const T v0 = readlane_val(mv, u);
          const T* x0 = X + (i64)__builtin_amdgcn_readlane(mc, u) * n + cb;
          if (okA) a0 += v0 * x0[cA];
          if (okB) a1 += v0 * x0[cB];
        }
      }
    } else {
      for (; k + 8 <= ke; k += 8) {
        int cc[8];
        T va[8], xa[8], xb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          cc[u] = __builtin_nontemporal_load(P.csr_col + k + u);
          va[u] = __builtin_nontemporal_load(Vals<T>::csr(P) + k + u);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const T* xr = X + (i64)cc[u] * n + cb;
          xa[u] = xr[cAc];
          xb[u] = xr[cBc];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          a0 += va[u] * (okA ? xa[u] : T(0));
          a1 += va[u] * (okB ? xb[u] : T(0));
        }
      }
      for (; k < ke; ++k) {
        const T v0 = Vals<T>::csr(P)[k];
        const T* x0 = X + (i64)P.csr_col[k] * n + cb;
        if (okA) a0 += v0 * x0[cA];
        if (okB) a1 += v0 * x0[cB];
      }
    }
    T* yr = Y + (i64)r * n + cb;
    // Y is written once: non-temporal stores keep it from evicting X
    if (okA) __builtin_nontemporal_store(ys[rl * kMmCols + cA] + a0, yr + cA);
    if (okB) __builtin_nontemporal_store(ys[rl * kMmCols + cB] + a1, yr + cB);
  }
}

}  // namespace sable
