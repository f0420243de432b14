// Fused SpMM tile with the VBR blocks on gfx950 matrix cores, operands staged in LDS.
//
// A workgroup (4 waves) owns kMmRows = 64 output rows and up to kMmCols = 128 columns of Y.
//  1. blocks: the plan lists, per tile, the distinct block columns of the blocks that overlap
//     it (ascending, padded to a multiple of 32). Each run of 32 list positions is one panel:
//       * the 32 rows of X it names are loaded once with 16-byte loads, split into bf16 hi
//         and lo parts (hardware round-to-nearest-even) and stored transposed in LDS, k
//         contiguous per column, the layout of the B operand of v_mfma_f32_16x16x32_bf16;
//       * the panel's A operand, the tile's block cells that fall in it as a zero-filled
//         64 x 32 hi plane and lo plane packed at plan time from the split-bf16 words, is
//         copied into LDS: each thread owns one unit (a row, 8 columns) and loads it with
//         two 16-byte loads if the panel's occupancy mask says a cell falls in it (only such
//         units are stored), else writes zeros;
//       * both loads of the next panel are issued before this panel's products run;
//       * each wave then runs, for its 16-column chunks and 16-row slices, three
//         16x16x32 products hi*hi + hi*lo + lo*hi with fp32 accumulation in registers.
//     One k step of 32 covers a C3 6x18 strip with room to spare, and each X row a tile needs
//     is loaded once per tile, however many of the tile's blocks read it.
//  2. the accumulators go to the tile of Y in LDS (reusing the panel buffers);
//  3. rows: bands (VALU fp32) + blocks, then + CSR (VALU fp32), stored; for a full 128-column
//     chunk every X access is a 16-byte load and a wave takes two CSR entries at a time.
// Every element has a fixed summation order, so results are bitwise reproducible.
#pragma once

#include "spmm_tile.h"

namespace sable {

constexpr int kPanK = 32;                        // panel width = k of one matrix-core step
constexpr int kPanLd = 40;                       // LDS row pitch in bf16 (80 bytes)
constexpr int kPanA = kMmRows * kPanLd;          // bf16 per A plane
constexpr int kPanB = kMmCols * kPanLd;          // bf16 per B plane
constexpr int kPanBytes = 4 * (kPanA + kPanB);   // A hi, A lo, B hi, B lo (2 bytes each)
constexpr int kPanLdsBytes = kPanBytes > kMmRows * kMmCols * 4 ? kPanBytes : kMmRows * kMmCols * 4;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// Band part of row r for this lane's two columns (cA, cB) of the chunk at cb.
template <class T>
__device__ __forceinline__ void spmm_band_row(const PlanView& P, int tile, int r, int cb, int n,
                                              const T* __restrict__ X, int cA, int cB, bool okA,
                                              bool okB, T& a0, T& a1) {
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

// CSR part of row r for columns (cA, cB): entries in index order, several X rows in flight;
// when one wave covers the row (rpw == 1) its entries are loaded 64 at a time, one per lane,
// and handed to every lane with readlane.
template <class T>
__device__ __forceinline__ void spmm_csr_row(const PlanView& P, int r, int cb, int n, int nc,
                                             const T* __restrict__ X, int rpw, int lane, int cA,
                                             int cB, bool okA, bool okB, T& a0, T& a1) {
  const int ke = P.csr_ptr[r + 1];
  int k = P.csr_ptr[r];
  const int cAc = min(cA, nc - 1), cBc = min(cB, nc - 1);
  if (rpw == 1) {
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
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Rows of the tile for one full 128-column chunk of a row-major X with n % 4 == 0: wave w
// takes rows w, w + 4, ...; lane l holds columns 4 (l % 32) .. + 3 and, in the CSR part, the
// entries of parity l / 32, so every load of X is a 16-byte load and one wave instruction
// fetches two whole 512-byte rows (four times fewer load instructions per entry than lanes
// across single columns, and four times the bytes in flight). The row's indices and values
// are loaded 64 at a time, one per lane, and handed to the lanes with bpermute. Per element:
// (bands + blocks) + (even-numbered CSR entries + odd-numbered ones), each part in index order.
__device__ __forceinline__ void spmm_rows_quad(const PlanView& P, int tile, int r0, int rend, int cb,
                                               int n, const float* __restrict__ X,
                                               float* __restrict__ Y, const float* __restrict__ ys,
                                               int wave, int lane) {
  const int h = lane >> 5, cq = 4 * (lane & 31);
  // the tile's row bounds, lane l holding the start of row r0 + l; a wave reads them with
  // readlane (its rows are wave-uniform)
  const int rb_lane = P.csr_ptr[min(r0 + lane, rend)];
  const int rb_end = P.csr_ptr[rend];
  auto row_begin = [&](int rl) { return __builtin_amdgcn_readlane(rb_lane, rl); };
  auto row_end = [&](int rl) { return rl + 1 < rend - r0 ? __builtin_amdgcn_readlane(rb_lane, rl + 1) : rb_end; };
  // the first 64 indices and values of the wave's next row are loaded while the current
  // row's gathers run
  int mc = 0;
  float mv = 0.f;
  if (wave < rend - r0) {
    const int k0 = row_begin(wave), k1 = row_end(wave);
    if (k0 < k1) {
      const int kl = k0 + min(lane, k1 - k0 - 1);
      mc = __builtin_nontemporal_load(P.csr_col + kl);
      mv = __builtin_nontemporal_load(P.csr_val + kl);
    }
  }
  for (int rl = wave; rl < rend - r0; rl += 4) {
    const int r = r0 + rl;
    const int kb = row_begin(rl), ke = row_end(rl);
    int mc_n = 0;
    float mv_n = 0.f;
    if (rl + 4 < rend - r0) {
      const int k0 = row_begin(rl + 4), k1 = row_end(rl + 4);
      if (k0 < k1) {
        const int kl = k0 + min(lane, k1 - k0 - 1);
        mc_n = __builtin_nontemporal_load(P.csr_col + kl);
        mv_n = __builtin_nontemporal_load(P.csr_val + kl);
      }
    }
    f32x4_t a = {0.f, 0.f, 0.f, 0.f};
    if (h == 0) {
      for (int s = P.tile_seg_lo[tile]; s < P.tile_seg_hi[tile]; ++s) {
        const int rs = P.seg_row_start[s], nr = P.seg_nrows[s];
        if (r < rs || r >= rs + nr) continue;
        const int nd = P.seg_ndiags[s];
        const int32_t* od = P.idiag + P.seg_idiag_ptr[s];
        const float* v = P.vdia_val + P.seg_val_ptr[s] + (r - rs);
        for (int d = 0; d < nd; ++d) {
          const int c = r + od[d];
          if ((unsigned)c >= (unsigned)P.ncols) continue;
          a += v[(i64)d * nr] * *reinterpret_cast<const f32x4_t*>(X + (i64)c * n + cb + cq);
        }
      }
      a += *reinterpret_cast<const f32x4_t*>(ys + rl * kMmCols + cq);
    }
    f32x4_t cs = {0.f, 0.f, 0.f, 0.f};
    for (int k = kb; k < ke; k += 64) {
      const int cnt = min(64, ke - k);
      if (k > kb) {  // rows longer than 64 entries: the next 64
        const int kl = k + min(lane, cnt - 1);
        mc = __builtin_nontemporal_load(P.csr_col + kl);
        mv = __builtin_nontemporal_load(P.csr_val + kl);
      }
      int u = 0;
      for (; u + 16 <= cnt; u += 16) {  // eight entries per half in flight
        int cc[8];
        float va[8];
        f32x4_t xv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          cc[j] = __shfl(mc, u + 2 * j + h);
          va[j] = __shfl(mv, u + 2 * j + h);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) xv[j] = *reinterpret_cast<const f32x4_t*>(X + (i64)cc[j] * n + cb + cq);
#pragma unroll
        for (int j = 0; j < 8; ++j) cs += va[j] * xv[j];
      }
      if (u < cnt) {  // the last 1..15 entries in one batch; lanes past the end idle
        int cc[8];
        float va[8];
        f32x4_t xv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = min(u + 2 * j + h, cnt - 1);
          cc[j] = __shfl(mc, e);
          va[j] = __shfl(mv, e);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (u + 2 * j + h < cnt) xv[j] = *reinterpret_cast<const f32x4_t*>(X + (i64)cc[j] * n + cb + cq);
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (u + 2 * j + h < cnt) cs += va[j] * xv[j];
      }
    }
    mc = mc_n;
    mv = mv_n;
    f32x4_t o;
    o.x = __shfl_xor(cs.x, 32);
    o.y = __shfl_xor(cs.y, 32);
    o.z = __shfl_xor(cs.z, 32);
    o.w = __shfl_xor(cs.w, 32);
    if (h == 0)
      __builtin_nontemporal_store(a + (cs + o), reinterpret_cast<f32x4_t*>(Y + (i64)r * n + cb + cq));
  }
}

// The panel's X rows (list positions kp .. kp + 31 of kcol, -1 = none) as bf16 hi / lo in
// LDS, transposed: plane[col * kPanLd + k]. Thread t takes k = 4 (t % 8) .. + 3 and columns
// 4 (t / 8) .. + 3 of the chunk (the eight lanes of one column group write 64 consecutive
// bytes of a column, so a half wave's 8-byte stores cover all banks once); columns >= nc are
// stored as 0. load_x_panel reads the values into registers (so they can be in flight while
// the previous panel's products run), store_x_panel splits and writes them.
struct XPanel {
  float v[4][4];  // [k][column]
};

// Thread t loads panel rows 4 (t % 8) .. + 3 (X rows row[0..3], -1 for padding) at columns
// cb + 4 (t / 8) .. + 3.
__device__ __forceinline__ void load_x_panel(const int (&row)[4], const float* __restrict__ X,
                                             int n, int cb, int nc, XPanel& xp) {
  const int t = threadIdx.x;
  const int c0 = 4 * (t >> 3);
  if ((n & 3) == 0 && c0 + 4 <= nc) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const float4 q = row[kk] >= 0
                           ? *reinterpret_cast<const float4*>(X + (i64)row[kk] * n + cb + c0)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
      xp.v[kk][0] = q.x; xp.v[kk][1] = q.y; xp.v[kk][2] = q.z; xp.v[kk][3] = q.w;
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        xp.v[kk][c] = (row[kk] >= 0 && c0 + c < nc) ? X[(i64)row[kk] * n + cb + c0 + c] : 0.f;
  }
}

__device__ __forceinline__ void store_x_panel(const XPanel& xp, uint16_t* bh, uint16_t* bl) {
  const int t = threadIdx.x;
  const int k0 = 4 * (t & 7), c0 = 4 * (t >> 3);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float col4[4] = {xp.v[0][c], xp.v[1][c], xp.v[2][c], xp.v[3][c]};
    bf16x4_t h, l;
    split4(col4, h, l);
    *reinterpret_cast<bf16x4_t*>(bh + (c0 + c) * kPanLd + k0) = h;
    *reinterpret_cast<bf16x4_t*>(bl + (c0 + c) * kPanLd + k0) = l;
  }
}

// Rows [r0, r0 + kMmRows) x columns [cb, cb + nc) of Y for tile `tile` of the view's 64-row
// schedule; lds holds kPanLdsBytes.
static_assert(kMmThreads * 8 == kMmRows * kPanK && kMmThreads == 256,
              "one unit of 8 bf16 per thread covers a 64 x 32 plane; four 64-bit occupancy words");

__device__ __forceinline__ void spmm_tile_panel(const PlanView& P, int tile, int cb, int n,
                                                const float* __restrict__ X, float* __restrict__ Y,
                                                uint8_t* __restrict__ lds) {
  uint16_t* ah = reinterpret_cast<uint16_t*>(lds);
  uint16_t* al = ah + kPanA;
  uint16_t* bh = al + kPanA;
  uint16_t* bl = bh + kPanB;
  float* ys = reinterpret_cast<float*>(lds);  // after the block phase
  const int r0 = tile * kMmRows;
  const int nc = min(kMmCols, n - cb);
  const int rend = min(r0 + kMmRows, P.nrows);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int m = lane & 15, g = lane >> 4;  // matrix-core operand coordinates of this lane
  const MmPart part = nc <= 32 ? MmPart{0, 1, 1 << wave} : MmPart{wave, 4, 0xF};

  // 1. blocks
  floatx4_t acc[4][2];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) acc[mt][ci] = floatx4_t{0.f, 0.f, 0.f, 0.f};
  // no panels: a plan without blocks (bands and CSR only)
  const int kb = P.mm_kptr ? __builtin_amdgcn_readfirstlane(P.mm_kptr[tile]) : 0;
  const int ke = P.mm_kptr ? __builtin_amdgcn_readfirstlane(P.mm_kptr[tile + 1]) : 0;
  // Panel g = kp / 32 goes through three stages, one panel apart: its indices (this thread's
  // four X row numbers, the occupancy mask and the first unit of A), then its data (this
  // thread's unit of A: row t / 4, columns 8 (t % 4) .. + 7, two 16-byte loads of hi and lo
  // words when the mask has it, else zero; and its 4 x 4 piece of the 32 rows of X), then its
  // products from LDS. While panel g's products run, the data of g + 1 and the indices of
  // g + 2 are in flight, so a panel waits for one round trip at most.
  const int at = threadIdx.x;
  const int arow = at >> 2, acol = 8 * (at & 3);
  const int xk0 = 4 * (at & 7);
  const uint4 zero4 = make_uint4(0u, 0u, 0u, 0u);
  struct PanIdx {
    int row[4];
    uint64_t m0, m1, m2, m3;
    i64 base;
  };
  auto load_idx = [&](int pg, PanIdx& q) {
    const int4 r4 = *reinterpret_cast<const int4*>(P.mm_kcol + (i64)pg * kPanK + xk0);
    q.row[0] = r4.x; q.row[1] = r4.y; q.row[2] = r4.z; q.row[3] = r4.w;
    const uint64_t* mk = P.mm_amask + 4 * (i64)pg;
    q.m0 = mk[0]; q.m1 = mk[1]; q.m2 = mk[2]; q.m3 = mk[3];
    q.base = P.mm_aptr[pg];
  };
  uint4 aw_h = zero4, aw_l = zero4;
  XPanel xp;
  auto load_data = [&](const PanIdx& q) {
    const uint64_t mw = wave == 0 ? q.m0 : wave == 1 ? q.m1 : wave == 2 ? q.m2 : q.m3;
    const int before = (wave > 0 ? __popcll(q.m0) : 0) + (wave > 1 ? __popcll(q.m1) : 0) +
                       (wave > 2 ? __popcll(q.m2) : 0);
    aw_h = zero4;
    aw_l = zero4;
    if ((mw >> lane) & 1ull) {
      const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mw >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)mw, 0u));
      const uint4* src = P.mm_apack + 2 * (q.base + before + rank);
      aw_h = src[0];
      aw_l = src[1];
    }
    load_x_panel(q.row, X, n, cb, nc, xp);
  };
  PanIdx qn;  // indices of the panel after the one whose data is in flight
  if (kb < ke) {
    PanIdx q0;
    load_idx(kb / kPanK, q0);
    if (kb + kPanK < ke) load_idx(kb / kPanK + 1, qn);
    load_data(q0);
  }
  for (int kp = kb; kp < ke; kp += kPanK) {
    __syncthreads();  // the previous panel's operands have been read
    *reinterpret_cast<uint4*>(ah + arow * kPanLd + acol) = aw_h;
    *reinterpret_cast<uint4*>(al + arow * kPanLd + acol) = aw_l;
    store_x_panel(xp, bh, bl);
    if (kp + kPanK < ke) {
      const PanIdx q = qn;
      if (kp + 2 * kPanK < ke) load_idx(kp / kPanK + 2, qn);
      load_data(q);
    }
    __syncthreads();
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) {
      const int col = (part.c0 + part.cstep * ci) * 16;
      if (col >= nc) continue;
      const bf16x8_t xh = *reinterpret_cast<const bf16x8_t*>(bh + (col + m) * kPanLd + 8 * g);
      const bf16x8_t xl = *reinterpret_cast<const bf16x8_t*>(bl + (col + m) * kPanLd + 8 * g);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        if (!((part.smask >> mt) & 1)) continue;
        const bf16x8_t wh = *reinterpret_cast<const bf16x8_t*>(ah + (16 * mt + m) * kPanLd + 8 * g);
        const bf16x8_t wl = *reinterpret_cast<const bf16x8_t*>(al + (16 * mt + m) * kPanLd + 8 * g);
        acc[mt][ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xh, acc[mt][ci], 0, 0, 0);
        acc[mt][ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xl, acc[mt][ci], 0, 0, 0);
        acc[mt][ci] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, xh, acc[mt][ci], 0, 0, 0);
      }
    }
  }
  // 2. block sums to the tile of Y in LDS (every (slice, column < nc) has one owner wave)
  __syncthreads();
#pragma unroll
  for (int ci = 0; ci < 2; ++ci) {
    const int col = (part.c0 + part.cstep * ci) * 16 + m;
    if (col >= nc) continue;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      if (!((part.smask >> mt) & 1)) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) ys[(16 * mt + 4 * g + i) * kMmCols + col] = acc[mt][ci][i];
    }
  }
  __syncthreads();

  // 3. rows: (bands + blocks) + CSR
  if (nc == kMmCols && (n & 3) == 0) {
    spmm_rows_quad(P, tile, r0, rend, cb, n, X, Y, ys, wave, lane);
    return;
  }
  int lpr = 64;
  while (lpr > 1 && lpr / 2 >= (nc + 1) / 2) lpr >>= 1;
  const int rpw = 64 / lpr;
  const int sub = lane / lpr, cl = lane % lpr;
  const int cA = cl, cB = cl + lpr;
  const bool okA = cA < nc, okB = cB < nc;
  for (int rl = wave * rpw + sub; rl < kMmRows; rl += 4 * rpw) {
    const int r = r0 + rl;
    if (r >= rend) continue;
    float a0 = 0.f, a1 = 0.f;
    spmm_band_row<float>(P, tile, r, cb, n, X, cA, cB, okA, okB, a0, a1);
    if (okA) a0 += ys[rl * kMmCols + cA];
    if (okB) a1 += ys[rl * kMmCols + cB];
    float s0 = 0.f, s1 = 0.f;
    spmm_csr_row<float>(P, r, cb, n, nc, X, rpw, lane, cA, cB, okA, okB, s0, s1);
    float* yr = Y + (i64)r * n + cb;
    if (okA) __builtin_nontemporal_store(a0 + s0, yr + cA);
    if (okB) __builtin_nontemporal_store(a1 + s1, yr + cB);
  }
}

}  // namespace sable
