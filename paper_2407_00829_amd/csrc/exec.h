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
  const uint32_t* vbr_mma;
  const i64* blk_mma_ptr;
  const int32_t* csr_ptr;
  const int32_t* csr_col;
  const float* csr_val;
  int rows_per_tile, ntiles;
  const int32_t* tile_seg_lo;
  const int32_t* tile_seg_hi;
  const int32_t* tile_blk_ptr;
  const int32_t* tile_blk;
  const int32_t* tile_order;  // launch order of the streamed kernels (may be null)
  const TileHead* tile_head;  // streamed kernels: per launch slot (null for other schedules)
  const int32_t* tile_row0;   // tile row bounds (entry-balanced tiling; null: uniform)
  // fp64 copies of the values (FP64 executor; null until set)
  const double* vdia_val64;
  const double* vbr_val64;
  const double* csr_val64;
  // far-column split: when far_prod is set, csr_col holds negative codes -(1 + q) for entries
  // whose product far_prod[q] the gather pass has already computed
  const float* far_prod;
  const double* far_prod64;  // the same for the fp64 executor
  // matrix-core SpMM panels of the 64-row SpMM schedule (null without them)
  const int32_t* mm_kcol;
  const int32_t* mm_kptr;
  const int32_t* mm_bpos;
  const uint4* mm_apack;
  const uint64_t* mm_amask;
  const i64* mm_aptr;
};

// Value arrays of the view for the executor's value type.
template <class T>
struct Vals;
template <>
struct Vals<float> {
  __device__ static const float* vdia(const PlanView& P) { return P.vdia_val; }
  __device__ static const float* vbr(const PlanView& P) { return P.vbr_val; }
  __device__ static const float* csr(const PlanView& P) { return P.csr_val; }
  __device__ static const float* far(const PlanView& P) { return P.far_prod; }
};
template <>
struct Vals<double> {
  __device__ static const double* vdia(const PlanView& P) { return P.vdia_val64; }
  __device__ static const double* vbr(const PlanView& P) { return P.vbr_val64; }
  __device__ static const double* csr(const PlanView& P) { return P.csr_val64; }
  __device__ static const double* far(const PlanView& P) { return P.far_prod64; }
};

// far = true: the view with the far-column split, if the plan has one and it is enabled.
PlanView make_view(const sable_plan_s& P, const Schedule& S, bool plain, bool far = false);

// Rows [r0, rend) of tile t of the view's schedule.
__device__ __forceinline__ void tile_rows(const PlanView& P, int t, int& r0, int& rend) {
  if (P.tile_row0) {
    r0 = P.tile_row0[t];
    rend = P.tile_row0[t + 1];
  } else {
    r0 = t * P.rows_per_tile;
    rend = min(r0 + P.rows_per_tile, P.nrows);
  }
}

// Tile of row r (r < nrows).
__device__ __forceinline__ int tile_of_row(const PlanView& P, int r) {
  if (!P.tile_row0) return r / P.rows_per_tile;
  int l = 0, h = P.ntiles - 1;  // last tile whose first row is <= r
  while (l < h) { const int m = (l + h + 1) >> 1; if (P.tile_row0[m] <= r) l = m; else h = m - 1; }
  return l;
}


// ---- SpMV tile body --------------------------------------------------------------------
// 256 threads over a tile of rows_per_tile <= 256 rows (256 / W rows in the W-lanes
// schedules); thread t owns row r0 + t for the band part (lane per row: diagonal-major values
// are contiguous across consecutive rows), and for blocks when W == 1. For W > 1 each row's
// W lanes take its block columns (c0 + lane, c0 + lane + W, ...) and then its CSR entries,
// and a shuffle reduction adds them; the band partial goes through LDS. Every row's sum has a
// fixed order: W == 1: (bands, diagonals ascending + blocks, columns ascending) + CSR in
// index order; W > 1: bands + (per lane: blocks, then CSR, strided by W; xor tree over lanes).
template <int W>
__device__ __forceinline__ void spmv_tile(const PlanView& P, int tile, const float* __restrict__ x,
                                          float* __restrict__ y, float* __restrict__ part) {
  const int RT = P.rows_per_tile;
  int r0, rend;
  tile_rows(P, tile, r0, rend);
  const int r = r0 + threadIdx.x;
  const bool act = r < rend;
  // W > 1: the first row of this lane group; its row pointers are loaded before anything
  // else, so they are in flight together with the tile's format lists
  const int grp0 = threadIdx.x / W;
  int kb0 = 0, ke0 = 0;
  if (W > 1 && grp0 < RT && r0 + grp0 < rend) {
    kb0 = P.csr_ptr[r0 + grp0];
    ke0 = P.csr_ptr[r0 + grp0 + 1];
  }
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
  if (W == 1) {  // blocks lane per row (W > 1: by the row's W lanes, with its CSR entries)
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
  }
  if (W == 1) {
    float cs = 0.f;
    if (act)
      for (int k = P.csr_ptr[r]; k < P.csr_ptr[r + 1]; ++k) cs += P.csr_val[k] * x[P.csr_col[k]];
    if (act) y[r] = acc + cs;
    return;
  }
  const bool bands = slo < shi;  // same for the whole tile: without bands, no LDS exchange
  if (bands) {
    part[threadIdx.x] = acc;
    __syncthreads();
  }
  const int lane = threadIdx.x & (W - 1);
  const int grp = threadIdx.x / W;
  const int ngrp = (int)blockDim.x / W;  // row groups of W lanes
  for (int rl = grp; rl < RT; rl += ngrp) {
    const int rr = r0 + rl;
    float cs = 0.f;
    if (rr < rend) {
      for (int q = blo; q < bhi; ++q) {  // block columns c0 + lane, c0 + lane + W, ...
        const int b = P.tile_blk[q];
        const int br0 = P.blk[4 * b], br1 = P.blk[4 * b + 1];
        if (rr < br0 || rr >= br1) continue;
        const int c0 = P.blk[4 * b + 2], c1 = P.blk[4 * b + 3];
        const int h = br1 - br0;
        const float* v = P.vbr_val + P.blk_val_ptr[b] + (rr - br0);
        for (int c = c0 + lane; c < c1; c += W) cs += v[(i64)(c - c0) * h] * x[c];
      }
      const bool first = rl == grp0;
      const int ke = first ? ke0 : P.csr_ptr[rr + 1];
      for (int k = (first ? kb0 : P.csr_ptr[rr]) + lane; k < ke; k += W)
        cs += P.csr_val[k] * x[P.csr_col[k]];
    }
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) cs += __shfl_xor(cs, o, W);
    if (lane == 0 && rr < rend) y[rr] = (bands ? part[rl] : 0.f) + cs;
  }
}

// ---- SpMV tile body, streamed variant ---------------------------------------------------
// Tile = up to 256*RPT rows, 256 threads; thread t owns rows r0 + t + 256*q (q < RPT).
//  0. every per-tile index load that depends on nothing else is issued at once, then the
//     first pass of CSR entries (U per thread: column, value, gathered x), so that the
//     longest dependent chain of the tile is in flight while the bands run;
//  1. bands: lane per row, diagonals unrolled by 4 (independent value and x loads); the next
//     segment's descriptor is loaded while the current one is processed;
//  2. blocks: each block's rows in the tile x column slices are spread over all threads;
//     slice partials meet in LDS and are added per row in slice order;
//  3. CSR: the tile's entries are contiguous and are taken in passes of 256*U; each
//     thread multiplies U entries by gathered x values (far entries of a split plan:
//     their stored products) into LDS, then every row adds its own products in index order.
// Per row: y = (bands + blocks) + CSR, in a fixed order (bitwise reproducible).
constexpr int kSpmvThreads = 256;
constexpr int kCsrUMax = 16;                        // CSR entries per thread per pass (max)
constexpr int kCsrChunk = kCsrUMax * kSpmvThreads;  // LDS products per pass (max)
template <int RPT>
struct CsrPass {
  static constexpr int U = RPT == 1 ? 8 : kCsrUMax;  // entries per thread per pass
};

__host__ __device__ __forceinline__ int xcd_tile(int bid, int ntiles) {
  // blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of tiles so
  // neighbouring rows (and their x entries) share one L2
  const int per = (ntiles + 7) >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// Matrix values and indices are read exactly once per product; with NT they are loaded with
// the non-temporal hint so they do not evict x (the only reused operand) from the L2.
template <bool NT, class T>
__device__ __forceinline__ T ld(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// One CSR pass: thread t takes entries e0 + t + 256*u (u < U) below e_end (e0 < e_end).
// csr_issue loads columns, values and the gathered operands; csr_finish forms the products
// later, so other loads can be issued while the gathers are in flight. Indices past e_end
// load entry e_end - 1 again and contribute 0, so every load is unconditional.
template <class T, int U>
struct CsrFlight {
  int j[U];
  T a[U], v[U];
};

template <class T, bool NT, int U>
__device__ __forceinline__ void csr_issue_idx(const PlanView& P, int e0, int e_end, CsrFlight<T, U>& f) {
  const T* val = Vals<T>::csr(P);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = min(e0 + (int)threadIdx.x + kSpmvThreads * u, e_end - 1);
    f.j[u] = ld<NT>(P.csr_col + k);
    f.a[u] = ld<NT>(val + k);
  }
}

template <class T, int U>
__device__ __forceinline__ void csr_issue_x(const PlanView& P, const T* __restrict__ x, CsrFlight<T, U>& f) {
  const T* fp = Vals<T>::far(P) ? Vals<T>::far(P) : x;  // stored far-column products
#pragma unroll
  for (int u = 0; u < U; ++u) f.v[u] = *(f.j[u] >= 0 ? x + f.j[u] : fp + (-1 - f.j[u]));
}

template <class T, bool NT, int U>
__device__ __forceinline__ void csr_issue(const PlanView& P, int e0, int e_end,
                                          const T* __restrict__ x, CsrFlight<T, U>& f) {
  csr_issue_idx<T, NT, U>(P, e0, e_end, f);
  csr_issue_x<T, U>(P, x, f);
}

template <class T, int U>
__device__ __forceinline__ void csr_finish(const CsrFlight<T, U>& f, int e0, int e_end, T (&pv)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const T pr = f.j[u] >= 0 ? f.a[u] * f.v[u] : f.v[u];
    pv[u] = e0 + (int)threadIdx.x + kSpmvThreads * u < e_end ? pr : T(0);
  }
}

// A streamed tile between the arrival of its record and its body: the row pointers of this
// thread's rows and the first CSR pass's columns and values (loads issued, x not yet read).
template <int RPT, class T>
struct StreamTile {
  TileHead H;
  int kb[RPT], ke[RPT];
  CsrFlight<T, CsrPass<RPT>::U> fl;
};

// The loads of a tile that need only its record.
template <int RPT, bool NT, class T>
__device__ __forceinline__ void stream_prefetch(const PlanView& P, StreamTile<RPT, T>& S) {
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = S.H.r0 + (int)threadIdx.x + kSpmvThreads * q;
    S.kb[q] = r < S.H.rend ? P.csr_ptr[r] : 0;
    S.ke[q] = r < S.H.rend ? P.csr_ptr[r + 1] : 0;
  }
  if (S.H.e0 < S.H.e1) csr_issue_idx<T, NT, CsrPass<RPT>::U>(P, S.H.e0, S.H.e1, S.fl);
}

// The rest of the tile: the first pass's gathers of x, bands, blocks, CSR, stores.
template <int RPT, bool NT, class T>
__device__ __forceinline__ void stream_body(const PlanView& P, StreamTile<RPT, T>& S,
                                            const T* __restrict__ x, T* __restrict__ y,
                                            float* __restrict__ lds) {
  constexpr int RT = kSpmvThreads * RPT;
  constexpr int U = CsrPass<RPT>::U;
  constexpr int kPass = U * kSpmvThreads;
  T* prod = reinterpret_cast<T*>(lds);  // kPass products (lds holds kCsrChunk + RT values of T)
  T* part = prod + kCsrChunk;           // RT block partials
  const TileHead& H = S.H;
  const int r0 = H.r0, rend = H.rend;
  const int t = threadIdx.x;
  // 0. the first CSR pass's gathers
  const int e_begin = H.e0, e_end = H.e1;
  const int slo = H.slo, shi = H.shi;
  const int blo = H.blo, bhi = H.bhi;
  int(&kb)[RPT] = S.kb;
  int(&ke)[RPT] = S.ke;
  int rs = H.rs, nr = H.nr, nd = H.nd;
  i64 svp = H.svp;
  int sip = H.sip;
  CsrFlight<T, U>& fl = S.fl;
  if (e_begin < e_end) csr_issue_x<T, U>(P, x, fl);

  T acc[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) acc[q] = 0;
  // 1. band segments
  for (int s = slo; s < shi; ++s) {
    const int32_t* od = P.idiag + sip;
    const T* vb = Vals<T>::vdia(P) + svp;
    const int crs = rs, cnr = nr, cnd = nd;
    if (s + 1 < shi) {  // next descriptor
      rs = P.seg_row_start[s + 1];
      nr = P.seg_nrows[s + 1];
      nd = P.seg_ndiags[s + 1];
      svp = P.seg_val_ptr[s + 1];
      sip = P.seg_idiag_ptr[s + 1];
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = r0 + t + kSpmvThreads * q;
      if (r < crs || r >= crs + cnr || r >= rend) continue;
      const T* v = vb + (r - crs);
      // groups of four diagonals with predicated loads (a ribbon of 3 is one group)
      for (int d = 0; d < cnd; d += 4) {
        int c[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // offsets past the segment's last read it again
          const int o = od[min(d + u, cnd - 1)];
          c[u] = d + u < cnd ? r + o : -1;
          ok[u] = (unsigned)c[u] < (unsigned)P.ncols;
        }
        T vv[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          vv[u] = ok[u] ? ld<NT>(v + (i64)(d + u) * cnr) : T(0);
          xv[u] = ok[u] ? x[c[u]] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (ok[u]) acc[q] += vv[u] * xv[u];
      }
    }
  }
  // 2. blocks; the next block's descriptor (list entry -> rectangle and value offset) is
  // loaded while the current block computes, so a block waits only for its values
  int4 bd = make_int4(0, 0, 0, 0);
  i64 bvp = 0;
  if (blo < bhi) {
    const int b = P.tile_blk[blo];
    bd = *reinterpret_cast<const int4*>(P.blk + 4 * b);
    bvp = P.blk_val_ptr[b];
  }
  for (int qb = blo; qb < bhi; ++qb) {
    const int br0 = bd.x, br1 = bd.y, c0 = bd.z, c1 = bd.w;
    const i64 vp = bvp;
    if (qb + 1 < bhi) {
      const int b = P.tile_blk[qb + 1];
      bd = *reinterpret_cast<const int4*>(P.blk + 4 * b);
      bvp = P.blk_val_ptr[b];
    }
    const int h = br1 - br0, w = c1 - c0;
    const int lo = max(br0, r0), hi = min(br1, rend);
    const int nrb = hi - lo;
    if (nrb <= 0) continue;
    const int S = nrb >= kSpmvThreads ? 1 : kSpmvThreads / nrb;
    const int cw = (w + S - 1) / S;
    const T* vb = Vals<T>::vbr(P) + vp;
    __syncthreads();
    for (int i = t; i < nrb * S; i += kSpmvThreads) {
      const int rl = i % nrb, sl = i / nrb;
      const int row = lo + rl;
      const int cb = c0 + sl * cw, ce = min(c1, cb + cw);
      const T* v = vb + (row - br0);
      T p0 = 0, p1 = 0, p2 = 0, p3 = 0, p4 = 0, p5 = 0, p6 = 0, p7 = 0;
      int c = cb;
      for (; c + 8 <= ce; c += 8) {
        const T* vc = v + (i64)(c - c0) * h;
        const T a0 = ld<NT>(vc), a1 = ld<NT>(vc + h), a2 = ld<NT>(vc + 2 * (i64)h),
                    a3 = ld<NT>(vc + 3 * (i64)h), a4 = ld<NT>(vc + 4 * (i64)h),
                    a5 = ld<NT>(vc + 5 * (i64)h), a6 = ld<NT>(vc + 6 * (i64)h),
                    a7 = ld<NT>(vc + 7 * (i64)h);
        p0 += a0 * x[c];
        p1 += a1 * x[c + 1];
        p2 += a2 * x[c + 2];
        p3 += a3 * x[c + 3];
        p4 += a4 * x[c + 4];
        p5 += a5 * x[c + 5];
        p6 += a6 * x[c + 6];
        p7 += a7 * x[c + 7];
      }
      for (; c < ce; ++c) p0 += ld<NT>(v + (i64)(c - c0) * h) * x[c];
      p0 += p4;
      p1 += p5;
      p2 += p6;
      p3 += p7;
      part[i] = (p0 + p1) + (p2 + p3);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = r0 + t + kSpmvThreads * q;
      if (r < lo || r >= hi) continue;
      T sacc = 0;
      for (int sl = 0; sl < S; ++sl) sacc += part[sl * nrb + (r - lo)];
      acc[q] += sacc;
    }
  }
  // 3. CSR: the first pass is already in registers
  T cs[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) cs[q] = 0;
  T pv[U];
  for (int e0 = e_begin; e0 < e_end; e0 += kPass) {
    if (e0 != e_begin) csr_issue<T, NT, U>(P, e0, e_end, x, fl);
    csr_finish<T, U>(fl, e0, e_end, pv);
    const int n = min(kPass, e_end - e0);
    __syncthreads();  // previous pass's row sums are done with prod
#pragma unroll
    for (int u = 0; u < U; ++u) prod[t + kSpmvThreads * u] = pv[u];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      // the row's products in index order; eight LDS reads are issued before their adds, so
      // a long row costs one LDS round trip per eight entries instead of one per entry
      const int a = max(kb[q], e0), b = min(ke[q], e0 + n);
      int k = a;
      for (; k + 8 <= b; k += 8) {
        T v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = prod[k - e0 + i];
#pragma unroll
        for (int i = 0; i < 8; ++i) cs[q] += v[i];
      }
      for (; k < b; ++k) cs[q] += prod[k - e0];
    }
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = r0 + t + kSpmvThreads * q;
    if (r < rend) y[r] = acc[q] + cs[q];
  }
}

// slot: the launch slot (the tile is the slot's record's).
template <int RPT, bool NT = false, class T = float>
__device__ __forceinline__ void spmv_tile_stream(const PlanView& P, int slot,
                                                 const T* __restrict__ x,
                                                 T* __restrict__ y, float* __restrict__ lds) {
  StreamTile<RPT, T> S;
  S.H = P.tile_head[slot];  // uniform: one scalar load of the whole record
  stream_prefetch<RPT, NT, T>(P, S);
  stream_body<RPT, NT, T>(P, S, x, y, lds);
}

// ---- SpMV tile body, row-length bins ----------------------------------------------------
// Rows of the CSR part are binned by length: 0, 1-4, 5-8, 9-16, 17-32, 33-64, > 64 entries
// (bins 0..6). The plan keeps, per tile, its rows grouped by bin (stable) and the bin
// boundaries. 256 threads over a tile of up to 256 rows:
//  1. bands and blocks lane per row (as the W = 1 tile body); a row without CSR entries is
//     stored at once, the others leave their partial in LDS;
//  2. bin by bin, each row of the bin is taken by a subwave of kBinWidth[u][bin] lanes
//     (u = the plan's entries-per-lane setting: about 1, 2 or 4 entries per lane), the
//     lanes stride over the row's entries and an xor tree adds their sums.
// Per row: y = (bands + blocks) + CSR (lane partials in index-strided order, xor tree).
constexpr int kNumBins = 7;
__host__ __device__ __forceinline__ int csr_bin(int len) {
  return len == 0 ? 0 : len <= 4 ? 1 : len <= 8 ? 2 : len <= 16 ? 3 : len <= 32 ? 4 : len <= 64 ? 5 : 6;
}
// lanes per row of each bin for 1, 2 and 4 entries per lane (bin 0 unused)
__host__ __device__ __forceinline__ int bin_width(int u, int bin) {
  const int maxlen = bin >= 6 ? 256 : 2 << bin;  // 4, 8, 16, 32, 64; long rows get a wave
  int w = maxlen >> u;                            // u = log2(entries per lane)
  return w < 1 ? 1 : w > 64 ? 64 : w;
}

__device__ __forceinline__ void spmv_tile_binned(const PlanView& P, int tile, const int32_t* __restrict__ brow,
                                                 const int32_t* __restrict__ boff, int u,
                                                 const float* __restrict__ x, float* __restrict__ y,
                                                 float* __restrict__ part) {
  int r0, rend;
  tile_rows(P, tile, r0, rend);
  const int t = threadIdx.x;
  const int r = r0 + t;
  const bool act = r < rend;
  int kb = 0, ke = 0;
  if (act) {
    kb = P.csr_ptr[r];
    ke = P.csr_ptr[r + 1];
  }
  float acc = 0.f;
  const int slo = P.tile_seg_lo[tile], shi = P.tile_seg_hi[tile];
  for (int s = slo; s < shi; ++s) {
    const int rs = P.seg_row_start[s], nr = P.seg_nrows[s];
    if (act && r >= rs && r < rs + nr) {
      const int nd = P.seg_ndiags[s];
      const int32_t* od = P.idiag + P.seg_idiag_ptr[s];
      const float* v = P.vdia_val + P.seg_val_ptr[s] + (r - rs);
      for (int d = 0; d < nd; ++d) {
        const int c = r + od[d];
        if ((unsigned)c < (unsigned)P.ncols) acc += v[(i64)d * nr] * x[c];
      }
    }
  }
  for (int q = P.tile_blk_ptr[tile]; q < P.tile_blk_ptr[tile + 1]; ++q) {
    const int b = P.tile_blk[q];
    const int br0 = P.blk[4 * b], br1 = P.blk[4 * b + 1];
    if (act && r >= br0 && r < br1) {
      const int c0 = P.blk[4 * b + 2], c1 = P.blk[4 * b + 3];
      const float* v = P.vbr_val + P.blk_val_ptr[b] + (r - br0);
      for (int c = c0; c < c1; ++c) acc += v[(i64)(c - c0) * (br1 - br0)] * x[c];
    }
  }
  if (act) {
    if (ke == kb) y[r] = acc;
    else part[t] = acc;
  }
  __syncthreads();
  const int* off = boff + (i64)tile * (kNumBins + 1);
  for (int bin = 1; bin < kNumBins; ++bin) {
    const int pa = off[bin], pz = off[bin + 1];
    if (pa >= pz) continue;
    const int W = bin_width(u, bin);
    const int lane = t & (W - 1), grp = t / W, ngrp = kSpmvThreads / W;
    for (int pos = pa + grp; pos - grp < pz; pos += ngrp) {  // whole subwaves iterate together
      const bool on = pos < pz;
      const int rr = on ? brow[pos] : r0;
      float cs = 0.f;
      if (on) {
        const int e1 = P.csr_ptr[rr + 1];
        for (int k = P.csr_ptr[rr] + lane; k < e1; k += W) cs += P.csr_val[k] * x[P.csr_col[k]];
      }
      for (int o = W >> 1; o > 0; o >>= 1) cs += __shfl_xor(cs, o);
      if (on && lane == 0) y[rr] = part[rr - r0] + cs;
    }
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
