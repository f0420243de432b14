// Block extractor (Sec. 4.1; Alg. 1 Partition/Decompose, Alg. 2 FindBlock) -> VBR blocks.
//
// Literal search ("paper" mode), allowed while nrows*ncols*max(nrows,ncols) <= 2^37:
//   prefix tables give the histogram H of Alg. 2 for any outer span in O(1) per inner index:
//     PT[j][r] = entries of column j in rows < r  (row pass: H[j] = PT[j][o1+1] - PT[j][o0])
//     QT[i][c] = entries of row i in columns < c  (column pass)
//   FindBlock runs one lane per (o0, o1) pair, each lane doing the two-pointer window scan of
//   Alg. 2 over the inner dimension; lanes with consecutive o1 read consecutive table words.
//   The best candidate is the highest score, ties broken by the smallest (o0, o1, i1): the
//   result of the sequential loop order with strict improvement. Scores compare exactly via
//   score^2 = (2n - a)^3 / (8a). Decompose recurses on the host; Trim runs on the GPU with
//   O(1) edge counts from the same tables.
// Tiled delta-dense detection ("tiled" mode; a scalable reading, not in the paper):
//   per tile size T the tile counts come from a radix sort of tile keys and run-length
//   encoding; hot tiles are grown into rectangles greedily in row-major order on the host;
//   Trim (one wave per rectangle) and the density / area / width tests run on the GPU; the
//   tile size covering the most nonzeros wins (ties: larger T).
#include <algorithm>
#include <climits>

#include "plan.h"

namespace sable {

namespace {

struct Cand {
  i64 nnz, area;  // nnz < 0: none
  int32_t o0, o1, i0, i1;
};

struct U128 {
  uint64_t hi, lo;
};

__host__ __device__ inline U128 mul64(uint64_t a, uint64_t b) {
#ifdef __HIP_DEVICE_COMPILE__
  return U128{__umul64hi(a, b), a * b};
#else
  unsigned __int128 r = (unsigned __int128)a * b;
  return U128{(uint64_t)(r >> 64), (uint64_t)r};
#endif
}

// x * y for x < 2^128 / y (no overflow past 128 bits by construction)
__host__ __device__ inline U128 mul128_64(U128 x, uint64_t y) {
  U128 lo = mul64(x.lo, y);
  return U128{x.hi * y + lo.hi, lo.lo};
}

__host__ __device__ inline bool gt128(U128 a, U128 b) {
  return a.hi != b.hi ? a.hi > b.hi : a.lo > b.lo;
}

// score(n1, a1) > score(n2, a2) with score^2 = (2n - a)^3 / (8a); n < 0 encodes "none" (-1).
__host__ __device__ inline bool score_gt(i64 n1, i64 a1, i64 n2, i64 a2) {
  if (n1 < 0) return false;
  if (n2 < 0) return true;
  const uint64_t t1 = (uint64_t)(2 * n1 - a1), t2 = (uint64_t)(2 * n2 - a2);
  U128 l = mul128_64(mul64(t1 * t1, t1), (uint64_t)a2);
  U128 r = mul128_64(mul64(t2 * t2, t2), (uint64_t)a1);
  return gt128(l, r);
}

__host__ __device__ inline bool cand_better(const Cand& a, const Cand& b) {
  if (score_gt(a.nnz, a.area, b.nnz, b.area)) return true;
  if (score_gt(b.nnz, b.area, a.nnz, a.area)) return false;
  if (a.nnz < 0) return false;
  if (b.nnz < 0) return true;
  if (a.o0 != b.o0) return a.o0 < b.o0;
  if (a.o1 != b.o1) return a.o1 < b.o1;
  return a.i1 < b.i1;
}

__global__ void k_occupancy(const int32_t* __restrict__ rptr, const int32_t* __restrict__ rcol,
                            int nrows, int ncols, uint8_t* __restrict__ occ) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < nrows; i += (i64)gridDim.x * blockDim.x)
    for (int k = rptr[i]; k < rptr[i + 1]; ++k) occ[i * (i64)ncols + rcol[k]] = 1;
}

// PT[j][r], r in [0, nrows]: one thread per column.
__global__ void k_col_prefix(const uint8_t* __restrict__ occ, int nrows, int ncols,
                             int32_t* __restrict__ PT) {
  for (i64 j = blockIdx.x * (i64)blockDim.x + threadIdx.x; j < ncols; j += (i64)gridDim.x * blockDim.x) {
    int32_t acc = 0;
    int32_t* out = PT + j * (i64)(nrows + 1);
    out[0] = 0;
    for (int r = 0; r < nrows; ++r) {
      acc += occ[r * (i64)ncols + j];
      out[r + 1] = acc;
    }
  }
}

// QT[i][c], c in [0, ncols]: one thread per row.
__global__ void k_row_prefix(const uint8_t* __restrict__ occ, int nrows, int ncols,
                             int32_t* __restrict__ QT) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < nrows; i += (i64)gridDim.x * blockDim.x) {
    int32_t acc = 0;
    int32_t* out = QT + i * (i64)(ncols + 1);
    const uint8_t* row = occ + i * (i64)ncols;
    out[0] = 0;
    for (int c = 0; c < ncols; ++c) {
      acc += row[c];
      out[c + 1] = acc;
    }
  }
}

constexpr int kFBThreads = 256;

// Alg. 2 for one pass. T: prefix table with row stride S; H[i] over outer span [o0, o1] is
// T[(in0+i)*S + out0+o1+1] - T[(in0+i)*S + out0+o0]. Grid: x = o1 chunks, y = o0.
__global__ __launch_bounds__(kFBThreads) void k_findblock(
    const int32_t* __restrict__ T, i64 S, int in0, int out0, int Lout, int Lin, i64 amin, int p,
    int smin, Cand* __restrict__ blockbest) {
  __shared__ Cand sh[kFBThreads];
  const int o0 = blockIdx.y;
  const int o1 = o0 + smin - 1 + blockIdx.x * kFBThreads + threadIdx.x;
  Cand best;
  best.nnz = -1; best.area = 0; best.o0 = o0; best.o1 = o1; best.i0 = 0; best.i1 = 0;
  if (o1 < Lout) {
    const i64 s = o1 - o0 + 1;
    const int32_t* hiT = T + in0 * S + out0 + o1 + 1;
    const int32_t* loT = T + in0 * S + out0 + o0;
    i64 nnz = 0;
    int i0 = 0;
    for (int i1 = 0; i1 < Lin; ++i1) {
      nnz += hiT[i1 * S] - loT[i1 * S];
      while (i0 <= i1) {
        const i64 a = s * (i1 - i0 + 1);
        if (a < amin) break;
        if (1000 * nnz >= (i64)p * a) {
          if (score_gt(nnz, a, best.nnz, best.area)) {
            best.nnz = nnz; best.area = a; best.i0 = i0; best.i1 = i1;
          }
          break;
        }
        nnz -= hiT[(i64)i0 * S] - loT[(i64)i0 * S];
        ++i0;
      }
    }
  }
  sh[threadIdx.x] = best;
  __syncthreads();
  for (int w = kFBThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w && cand_better(sh[threadIdx.x + w], sh[threadIdx.x]))
      sh[threadIdx.x] = sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) blockbest[(i64)blockIdx.y * gridDim.x + blockIdx.x] = sh[0];
}

// ---- the sparse window scan --------------------------------------------------------------
// The same search over the non-empty inner lines only. Lines are the residual's rows (column
// pass) or columns (row pass, from a transpose): lidx[lptr[l] .. lptr[l + 1]) are the outer
// indices of line l, ascending. A workgroup serves one o0 and 256 consecutive o1: it first
// lists, in inner order, every line of the region with an entry at an outer index in
// [o0, largest o1 of the workgroup] (its first such index `first`, and the range of its
// entries inside the region's outer range); each lane then runs the window rule over the
// lines with first <= its o1, counting a line's entries in [o0, o1] by binary search. Runs of
// empty inner indices are crossed in one step: with `win` entries in the window, the scan
// keeps dropping left columns iff the width exceeds T(win) = max(ceil(A_min / s) - 1,
// floor(1000 win / (p s))), so an empty run either grows the window up to T(win) or slides it,
// and within a stretch of constant `win` only the first candidate can be a strict
// improvement (the score falls as the area grows). Results equal the dense scan's.
struct SpanLine {
  int32_t pos, lo, end, first;  // inner index; entries [lo, end) from outer o0 on; first outer
};

__device__ inline int line_count_le(const int32_t* __restrict__ lidx, int lo, int end, int lim) {
  int a = lo, b = end;  // entries in [lo, end) with outer index <= lim
  while (a < b) {
    const int m = (a + b) >> 1;
    if (lidx[m] <= lim) a = m + 1; else b = m;
  }
  return a - lo;
}

__global__ __launch_bounds__(kFBThreads) void k_findblock_sparse(
    const int32_t* __restrict__ lptr, const int32_t* __restrict__ lidx, int in0, int out0, int Lout,
    int Lin, i64 amin, int p, int smin, int o0_base, SpanLine* __restrict__ scratch,
    Cand* __restrict__ blockbest) {
  __shared__ int wsum[kFBThreads / 64];
  __shared__ Cand sh[kFBThreads];
  const int o0 = o0_base + blockIdx.y;
  const int o1_first = o0 + smin - 1 + blockIdx.x * kFBThreads;
  const int o1 = o1_first + threadIdx.x;
  const int o1max = min(Lout - 1, o1_first + kFBThreads - 1);
  SpanLine* list = scratch + ((i64)blockIdx.y * gridDim.x + blockIdx.x) * Lin;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int m = 0;
  if (o1_first < Lout) {  // the same for the whole workgroup
    for (int ib = 0; ib < Lin; ib += kFBThreads) {
      const int i = ib + threadIdx.x;
      SpanLine L;
      bool keep = false;
      if (i < Lin) {
        const int a = lptr[in0 + i], b = lptr[in0 + i + 1];
        int lo = a, hi = b;  // first entry at outer >= out0 + o0
        while (lo < hi) { const int mm = (lo + hi) >> 1; if (lidx[mm] < out0 + o0) lo = mm + 1; else hi = mm; }
        if (lo < b && lidx[lo] - out0 <= o1max) {
          int e0 = lo, e1 = b;  // end of the entries inside the region's outer range
          while (e0 < e1) { const int mm = (e0 + e1) >> 1; if (lidx[mm] < out0 + Lout) e0 = mm + 1; else e1 = mm; }
          L.pos = i; L.lo = lo; L.end = e0; L.first = lidx[lo] - out0;
          keep = true;
        }
      }
      const uint64_t bal = __ballot(keep);
      if (lane == 0) wsum[wv] = __popcll(bal);
      __syncthreads();
      int before = m;
      for (int w = 0; w < wv; ++w) before += wsum[w];
      if (keep) list[before + __popcll(bal & ((1ull << lane) - 1ull))] = L;
      for (int w = 0; w < kFBThreads / 64; ++w) m += wsum[w];
      __syncthreads();
    }
  }
  Cand best;
  best.nnz = -1; best.area = 0; best.o0 = o0; best.o1 = o1; best.i0 = 0; best.i1 = 0;
  if (o1 < Lout) {
    const i64 s = o1 - o0 + 1;
    const i64 A = amin > 0 ? (amin + s - 1) / s : 0;  // smallest width that is large enough
    const i64 wmin = A > 1 ? A : 1;
    const i64 pd = (i64)p * s;
    auto T = [&](i64 win) -> i64 {
      const i64 D = p > 0 ? (1000 * win) / pd : ((i64)1 << 60);
      return D > A - 1 ? D : A - 1;
    };
    auto valid = [&](int k) {  // next listed line visible to this lane, from k on
      while (k < m && list[k].first > o1) ++k;
      return k;
    };
    auto posk = [&](int k) -> i64 { return k < m ? list[k].pos : Lin; };
    auto cntk = [&](int k) -> i64 { return line_count_le(lidx, list[k].lo, list[k].end, out0 + o1); };
    int kr = valid(0), kl = kr;
    i64 i0 = 0, i1 = -1, win = 0;
    bool tested = false;
    auto shrink = [&]() {
      for (;;) {
        const i64 w = i1 - i0 + 1, t = T(win);
        if (w <= t) return;
        const i64 z = posk(kl) - i0;
        if (z > 0) { i0 += z < w - t ? z : w - t; continue; }
        win -= cntk(kl);
        kl = valid(kl + 1);
        ++i0;
        tested = false;
      }
    };
    auto test = [&]() {
      const i64 w = i1 - i0 + 1;
      if (tested || w < wmin) return;
      tested = true;
      const i64 a = s * w;
      if (score_gt(win, a, best.nnz, best.area)) {
        best.nnz = win; best.area = a; best.i0 = (int32_t)i0; best.i1 = (int32_t)i1;
      }
    };
    for (;;) {
      i64 rem = posk(kr) - (i1 + 1);  // empty inner indices before the next listed line
      while (rem > 0) {
        const i64 w = i1 - i0 + 1, t = T(win);
        if (w < t) {  // the window grows, nothing leaves
          const i64 k = rem < t - w ? rem : t - w;
          const i64 wc = w + 1 > wmin ? w + 1 : wmin;
          if (!tested && wc <= w + k) { i1 += wc - w; test(); i1 += w + k - wc; }
          else i1 += k;
          rem -= k;
          continue;
        }
        const i64 z = posk(kl) - i0;  // w == t: each step drops a column at the left
        if (z > 0) {
          const i64 k = rem < z ? rem : z;
          ++i1; ++i0; test();
          i1 += k - 1; i0 += k - 1;
          rem -= k;
          continue;
        }
        ++i1; shrink(); test(); --rem;
      }
      if (kr >= m) break;
      i1 = list[kr].pos;
      win += cntk(kr);
      kr = valid(kr + 1);
      tested = false;
      shrink(); test();
    }
  }
  sh[threadIdx.x] = best;
  __syncthreads();
  for (int w = kFBThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w && cand_better(sh[threadIdx.x + w], sh[threadIdx.x]))
      sh[threadIdx.x] = sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) blockbest[(i64)o0 * gridDim.x + blockIdx.x] = sh[0];
}

// Transpose of the residual's pattern: rows of every column, ascending (keys column:row).
__global__ void k_colrow_keys(const int32_t* __restrict__ rows, const int32_t* __restrict__ col,
                              i64 nnz, uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
                              int32_t* __restrict__ ccount) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < nnz; k += (i64)gridDim.x * blockDim.x) {
    keys[k] = ((uint64_t)(uint32_t)col[k] << 32) | (uint32_t)rows[k];
    vals[k] = 0;
    atomicAdd(&ccount[col[k]], 1);
  }
}

__global__ void k_key_low(const uint64_t* __restrict__ keys, i64 n, int32_t* __restrict__ out) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x)
    out[k] = (int32_t)(uint32_t)(keys[k] & 0xffffffffu);
}

__global__ __launch_bounds__(1024) void k_reduce_cand(const Cand* __restrict__ in, i64 n,
                                                      Cand* __restrict__ out) {
  __shared__ Cand sh[1024];
  Cand best;
  best.nnz = -1; best.area = 0; best.o0 = INT_MAX; best.o1 = INT_MAX; best.i0 = 0; best.i1 = INT_MAX;
  for (i64 k = threadIdx.x; k < n; k += blockDim.x)
    if (cand_better(in[k], best)) best = in[k];
  sh[threadIdx.x] = best;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w && cand_better(sh[threadIdx.x + w], sh[threadIdx.x]))
      sh[threadIdx.x] = sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

struct TrimOut {
  int32_t r0, r1, c0, c1;
  i64 nnz;
};

__device__ inline bool dens_gt(i64 n1, i64 a1, i64 n2, i64 a2) {
  U128 l = mul64((uint64_t)n1, (uint64_t)a2), r = mul64((uint64_t)n2, (uint64_t)a1);
  return gt128(l, r);
}

// Trim (Alg. 1) with table counts; single thread. Ties: top, bottom, left, right.
__global__ void k_trim_tables(const int32_t* __restrict__ PT, const int32_t* __restrict__ QT,
                              int nrows, int ncols, int r0, int r1, int c0, int c1,
                              TrimOut* __restrict__ out) {
  if (threadIdx.x || blockIdx.x) return;
  const i64 SP = nrows + 1, SQ = ncols + 1;
  auto rowc = [&](int r, int a, int b) -> i64 { return QT[r * SQ + b] - QT[r * SQ + a]; };
  auto colc = [&](int c, int a, int b) -> i64 { return PT[c * SP + b] - PT[c * SP + a]; };
  i64 nnz = 0;
  for (int r = r0; r < r1; ++r) nnz += rowc(r, c0, c1);
  for (;;) {
    const i64 h = r1 - r0, w = c1 - c0, area = h * w;
    int be = -1;
    i64 bn = nnz, ba = area;
    for (int e = 0; e < 4; ++e) {
      i64 cnt, len;
      if (e < 2) {
        if (h < 2) continue;
        cnt = rowc(e == 0 ? r0 : r1 - 1, c0, c1);
        len = w;
      } else {
        if (w < 2) continue;
        cnt = colc(e == 2 ? c0 : c1 - 1, r0, r1);
        len = h;
      }
      const i64 n2 = nnz - cnt, a2 = area - len;
      if (dens_gt(n2, a2, bn, ba)) { be = e; bn = n2; ba = a2; }
    }
    if (be < 0) break;
    if (be == 0) ++r0; else if (be == 1) --r1; else if (be == 2) ++c0; else --c1;
    nnz = bn;
  }
  TrimOut o;
  o.r0 = r0; o.r1 = r1; o.c0 = c0; o.c1 = c1; o.nnz = nnz;
  out[0] = o;
}

// ---- tiled mode kernels -----------------------------------------------------------------

__global__ void k_tile_keys(const int32_t* __restrict__ rows, const int32_t* __restrict__ col,
                            i64 nnz, int T, i64 ntc, uint64_t* __restrict__ keys,
                            int32_t* __restrict__ vals) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < nnz; k += (i64)gridDim.x * blockDim.x) {
    keys[k] = (uint64_t)(rows[k] / T) * (uint64_t)ntc + (uint64_t)(col[k] / T);
    vals[k] = 0;
  }
}

__global__ void k_hot_flags(const uint64_t* __restrict__ uniq, const int32_t* __restrict__ cnt,
                            i64 nt, int T, i64 ntc, int nrows, int ncols, int p,
                            int32_t* __restrict__ flag) {
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < nt; t += (i64)gridDim.x * blockDim.x) {
    const i64 I = (i64)(uniq[t] / (uint64_t)ntc), J = (i64)(uniq[t] % (uint64_t)ntc);
    const i64 h = min((I + 1) * T, (i64)nrows) - I * T;
    const i64 w = min((J + 1) * T, (i64)ncols) - J * T;
    flag[t] = (1000 * (i64)cnt[t] >= (i64)p * h * w) ? 1 : 0;
  }
}

__global__ void k_scatter_hot(const uint64_t* __restrict__ uniq, const int32_t* __restrict__ flag,
                              const int32_t* __restrict__ pos, i64 nt, uint64_t* __restrict__ hot) {
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < nt; t += (i64)gridDim.x * blockDim.x)
    if (flag[t]) hot[pos[t]] = uniq[t];
}

__device__ inline int row_count_dev(const int32_t* __restrict__ rptr, const int32_t* __restrict__ rcol,
                                    int r, int c0, int c1) {  // entries of row r in [c0, c1)
  int a = rptr[r], b = rptr[r + 1];
  int lo = a, hi = b;
  while (lo < hi) { int m = (lo + hi) >> 1; if (rcol[m] < c0) lo = m + 1; else hi = m; }
  int s = lo;
  lo = s; hi = b;
  while (lo < hi) { int m = (lo + hi) >> 1; if (rcol[m] < c1) lo = m + 1; else hi = m; }
  return lo - s;
}

__device__ inline i64 wave_sum64(i64 v) {
  for (int o = 32; o > 0; o >>= 1) {
    int lo = __shfl_xor((int)(uint32_t)(v & 0xffffffffu), o, 64);
    int hi = __shfl_xor((int)(v >> 32), o, 64);
    v += (i64)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
  }
  return v;
}

// One wave per rectangle: nnz, then Trim (Alg. 1) with counts from the residual CSR.
__global__ __launch_bounds__(64) void k_trim_rects(const int32_t* __restrict__ rptr,
                                                   const int32_t* __restrict__ rcol,
                                                   const BlkRec* __restrict__ rects, int nrect,
                                                   TrimOut* __restrict__ out) {
  const int b = blockIdx.x;
  if (b >= nrect) return;
  const int lane = threadIdx.x;
  int r0 = rects[b].r0, r1 = rects[b].r1, c0 = rects[b].c0, c1 = rects[b].c1;
  i64 part = 0;
  for (int r = r0 + lane; r < r1; r += 64) part += row_count_dev(rptr, rcol, r, c0, c1);
  i64 nnz = wave_sum64(part);
  for (;;) {
    const i64 h = r1 - r0, w = c1 - c0, area = h * w;
    i64 cnt[4] = {0, 0, 0, 0};
    if (h >= 2) {
      cnt[0] = row_count_dev(rptr, rcol, r0, c0, c1);
      cnt[1] = row_count_dev(rptr, rcol, r1 - 1, c0, c1);
    }
    if (w >= 2) {
      i64 pl = 0, pr = 0;
      for (int r = r0 + lane; r < r1; r += 64) {
        pl += row_count_dev(rptr, rcol, r, c0, c0 + 1);
        pr += row_count_dev(rptr, rcol, r, c1 - 1, c1);
      }
      cnt[2] = wave_sum64(pl);
      cnt[3] = wave_sum64(pr);
    }
    int be = -1;
    i64 bn = nnz, ba = area;
    for (int e = 0; e < 4; ++e) {
      if (e < 2 && h < 2) continue;
      if (e >= 2 && w < 2) continue;
      const i64 len = e < 2 ? w : h;
      const i64 n2 = nnz - cnt[e], a2 = area - len;
      if (dens_gt(n2, a2, bn, ba)) { be = e; bn = n2; ba = a2; }
    }
    if (be < 0) break;
    if (be == 0) ++r0; else if (be == 1) --r1; else if (be == 2) ++c0; else --c1;
    nnz = bn;
  }
  if (lane == 0) {
    TrimOut o;
    o.r0 = r0; o.r1 = r1; o.c0 = c0; o.c1 = c1; o.nnz = nnz;
    out[b] = o;
  }
}

// One thread per (block, block row): copy the row's entries inside the block column-major.
__global__ void k_pack_vbr(const int32_t* __restrict__ rpre, int nblk, i64 total,
                           const BlkRec* __restrict__ blks, const i64* __restrict__ bvp,
                           const int32_t* __restrict__ rptr, const int32_t* __restrict__ rcol,
                           const float* __restrict__ rval, const int32_t* __restrict__ rid,
                           float* __restrict__ val, uint8_t* __restrict__ claimed,
                           int8_t* __restrict__ owner, i64* __restrict__ slot) {
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < total; t += (i64)gridDim.x * blockDim.x) {
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
      int m = (lo + hi + 1) >> 1;
      if ((i64)rpre[m] <= t) lo = m; else hi = m - 1;
    }
    const BlkRec B = blks[lo];
    const int r = B.r0 + (int)(t - rpre[lo]);
    const int h = B.r1 - B.r0;
    int a = rptr[r], e = rptr[r + 1];
    int l2 = a, h2 = e;
    while (l2 < h2) { int m = (l2 + h2) >> 1; if (rcol[m] < B.c0) l2 = m + 1; else h2 = m; }
    for (int k = l2; k < e && rcol[k] < B.c1; ++k) {
      const i64 at = bvp[lo] + (i64)(rcol[k] - B.c0) * h + (r - B.r0);
      val[at] = rval[k];
      claimed[k] = 1;
      owner[rid[k]] = 1;
      slot[rid[k]] = at;
    }
  }
}

// ---- host side ----------------------------------------------------------------------------

bool dense_enough(i64 nnz, i64 area, int p) { return (__int128)1000 * nnz >= (__int128)p * area; }

i64 ceil_sqrt(i64 a) {
  i64 s = 0;
  while (s * s < a) ++s;
  return s;
}

bool paper_fits(i64 nrows, i64 ncols);

struct PaperCtx {
  const Resid* R;
  const sable_thresholds* th;
  hipStream_t s;
  bool sparse = false;           // window scans over non-empty inner lines (equal results)
  DBuf<int32_t> PT, QT;          // dense scan: prefix tables
  DBuf<int32_t> cptr, crow;      // sparse scan: the residual's columns (rows ascending)
  DBuf<SpanLine> lines;          // sparse scan: per-workgroup line lists
  DBuf<Cand> blockbest, best1;
  std::vector<char> used_r, used_c;
  std::vector<TrimOut> out;
};

Cand find_block(PaperCtx& C, const BlkRec& reg, bool by_rows) {
  const Resid& R = *C.R;
  const int Lout = by_rows ? reg.r1 - reg.r0 : reg.c1 - reg.c0;
  const int Lin = by_rows ? reg.c1 - reg.c0 : reg.r1 - reg.r0;
  const int smin = (int)ceil_sqrt(C.th->amin_block);
  Cand none;
  none.nnz = -1; none.area = 0; none.o0 = none.o1 = none.i0 = none.i1 = 0;
  if (Lout < smin || Lout <= 0 || Lin <= 0) return none;
  const int n_o1 = Lout - smin + 1;  // o1 - o0 offsets from smin-1 up to Lout-1
  dim3 grid(nblocks(n_o1, kFBThreads), Lout);
  const i64 nbest = (i64)grid.x * grid.y;
  if ((i64)C.blockbest.n < nbest) C.blockbest.alloc(nbest);
  if (C.sparse) {
    // inner lines: columns (row pass, from the transpose) or rows (column pass)
    const int32_t* lptr = by_rows ? C.cptr.p : R.ptr.p;
    const int32_t* lidx = by_rows ? C.crow.p : R.col.p;
    const int in0 = by_rows ? reg.c0 : reg.r0;
    const int out0 = by_rows ? reg.r0 : reg.c0;
    // o0 in batches whose line lists fit 256 MB of scratch
    const i64 per_o0 = (i64)grid.x * Lin;
    const int batch = (int)std::max<i64>(1, std::min<i64>(Lout, ((i64)1 << 24) / std::max<i64>(1, per_o0)));
    if ((i64)C.lines.n < per_o0 * batch) C.lines.alloc(per_o0 * batch);
    for (int ob = 0; ob < Lout; ob += batch) {
      dim3 g2(grid.x, std::min(batch, Lout - ob));
      k_findblock_sparse<<<g2, kFBThreads, 0, C.s>>>(lptr, lidx, in0, out0, Lout, Lin,
                                                     C.th->amin_block, C.th->delta_block_pm, smin,
                                                     ob, C.lines.p, C.blockbest.p);
      LAUNCH_CHECK();
    }
    k_reduce_cand<<<1, 1024, 0, C.s>>>(C.blockbest.p, nbest, C.best1.p);
    LAUNCH_CHECK();
    std::vector<Cand> h;
    to_host(h, C.best1.p, 1, C.s);
    return h[0];
  }
  const int32_t* T = by_rows ? C.PT.p : C.QT.p;
  const i64 S = by_rows ? R.nrows + 1 : R.ncols + 1;
  const int in0 = by_rows ? reg.c0 : reg.r0;
  const int out0 = by_rows ? reg.r0 : reg.c0;
  k_findblock<<<grid, kFBThreads, 0, C.s>>>(T, S, in0, out0, Lout, Lin, C.th->amin_block,
                                            C.th->delta_block_pm, smin, C.blockbest.p);
  LAUNCH_CHECK();
  k_reduce_cand<<<1, 1024, 0, C.s>>>(C.blockbest.p, nbest, C.best1.p);
  LAUNCH_CHECK();
  std::vector<Cand> h;
  to_host(h, C.best1.p, 1, C.s);
  return h[0];
}

BlkRec cand_rect(const Cand& c, const BlkRec& reg, bool by_rows) {
  if (by_rows) return {reg.r0 + c.o0, reg.r0 + c.o1 + 1, reg.c0 + c.i0, reg.c0 + c.i1 + 1};
  return {reg.r0 + c.i0, reg.r0 + c.i1 + 1, reg.c0 + c.o0, reg.c0 + c.o1 + 1};
}

void decompose(PaperCtx& C, BlkRec reg) {
  const sable_thresholds& th = *C.th;
  if (reg.r1 <= reg.r0 || reg.c1 <= reg.c0) return;
  if ((i64)(reg.r1 - reg.r0) * (reg.c1 - reg.c0) < th.amin_block) return;
  Cand b = find_block(C, reg, true);
  Cand b2 = find_block(C, reg, false);
  const bool use_csc = score_gt(b2.nnz, b2.area, b.nnz, b.area);
  const Cand bc = use_csc ? b2 : b;
  if (bc.nnz < 0 || bc.area < th.amin_block) return;
  BlkRec B = cand_rect(bc, reg, !use_csc);
  for (int r = B.r0; r < B.r1; ++r) if (C.used_r[r]) return;
  for (int c = B.c0; c < B.c1; ++c) if (C.used_c[c]) return;
  DBuf<TrimOut> d(1);
  if (C.sparse) {  // counts from the residual's rows
    DBuf<BlkRec> rb(1);
    std::vector<BlkRec> hb{B};
    to_dev(rb, hb, C.s);
    k_trim_rects<<<1, 64, 0, C.s>>>(C.R->ptr.p, C.R->col.p, rb.p, 1, d.p);
  } else {
    k_trim_tables<<<1, 1, 0, C.s>>>(C.PT.p, C.QT.p, C.R->nrows, C.R->ncols, B.r0, B.r1, B.c0,
                                    B.c1, d.p);
  }
  LAUNCH_CHECK();
  std::vector<TrimOut> t;
  to_host(t, d.p, 1, C.s);
  const TrimOut o = t[0];
  const i64 area = (i64)(o.r1 - o.r0) * (o.c1 - o.c0);
  if (!dense_enough(o.nnz, area, th.delta_block_pm) || area < th.amin_block) return;
  C.out.push_back(o);
  for (int r = o.r0; r < o.r1; ++r) C.used_r[r] = 1;
  for (int c = o.c0; c < o.c1; ++c) C.used_c[c] = 1;
  decompose(C, {reg.r0, o.r0, reg.c0, reg.c1});
  decompose(C, {o.r1, reg.r1, reg.c0, reg.c1});
  decompose(C, {o.r0, o.r1, reg.c0, o.c0});
  decompose(C, {o.r0, o.r1, o.c1, reg.c1});
}

std::vector<TrimOut> blocks_paper(const Resid& R, const sable_thresholds& th, hipStream_t s) {
  PaperCtx C;
  C.R = &R;
  C.th = &th;
  C.s = s;
  C.best1.alloc(1);
  C.sparse = (th.flags & SABLE_F_SPARSE_SEARCH) || !paper_fits(R.nrows, R.ncols);
  if (C.sparse) {
    DBuf<int32_t> rows;
    entry_rows(R, rows, s);
    DBuf<uint64_t> keys(R.nnz);
    DBuf<int32_t> vals(R.nnz), cnt(R.ncols);
    if (R.ncols) HIPC(hipMemsetAsync(cnt.p, 0, R.ncols * sizeof(int32_t), s));
    if (R.nnz) {
      k_colrow_keys<<<grid_for(R.nnz, 256), 256, 0, s>>>(rows.p, R.col.p, R.nnz, keys.p, vals.p, cnt.p);
      LAUNCH_CHECK();
      sort_pairs_u64(keys, vals, R.nnz, 64, s);
    }
    C.crow.alloc(R.nnz);
    if (R.nnz) {
      k_key_low<<<grid_for(R.nnz, 256), 256, 0, s>>>(keys.p, R.nnz, C.crow.p);
      LAUNCH_CHECK();
    }
    C.cptr.alloc((i64)R.ncols + 1);
    exclusive_scan_i32(cnt.p, C.cptr.p, R.ncols, s);
    HIPC(hipStreamSynchronize(s));
  } else {
    DBuf<uint8_t> occ((i64)R.nrows * R.ncols);
    if (occ.n) HIPC(hipMemsetAsync(occ.p, 0, occ.n, s));
    if (R.nnz)
      k_occupancy<<<grid_for(R.nrows, 256), 256, 0, s>>>(R.ptr.p, R.col.p, R.nrows, R.ncols, occ.p);
    LAUNCH_CHECK();
    C.PT.alloc((i64)R.ncols * (R.nrows + 1));
    C.QT.alloc((i64)R.nrows * (R.ncols + 1));
    if (R.ncols) k_col_prefix<<<grid_for(R.ncols, 64), 64, 0, s>>>(occ.p, R.nrows, R.ncols, C.PT.p);
    LAUNCH_CHECK();
    if (R.nrows) k_row_prefix<<<grid_for(R.nrows, 64), 64, 0, s>>>(occ.p, R.nrows, R.ncols, C.QT.p);
    LAUNCH_CHECK();
    HIPC(hipStreamSynchronize(s));
  }
  C.used_r.assign(R.nrows, 0);
  C.used_c.assign(R.ncols, 0);
  decompose(C, {0, R.nrows, 0, R.ncols});
  std::vector<TrimOut> kept;
  for (auto& b : C.out)
    if (b.c1 - b.c0 != 1) kept.push_back(b);  // width-1 blocks are discarded (Alg. 1)
  HIPC(hipStreamSynchronize(s));
  return kept;
}

// Greedy rectangles over hot tiles (sorted keys I*ntc + J), row-major order.
std::vector<BlkRec> greedy_rects(const std::vector<uint64_t>& hot, i64 ntr, i64 ntc, int T,
                                 int nrows, int ncols) {
  std::vector<char> claimed(hot.size(), 0);
  auto find = [&](i64 I, i64 J) -> i64 {
    if (I < 0 || J < 0 || I >= ntr || J >= ntc) return -1;
    const uint64_t key = (uint64_t)I * (uint64_t)ntc + (uint64_t)J;
    auto it = std::lower_bound(hot.begin(), hot.end(), key);
    if (it == hot.end() || *it != key) return -1;
    return it - hot.begin();
  };
  auto avail = [&](i64 I, i64 J) {
    i64 k = find(I, J);
    return k >= 0 && !claimed[k];
  };
  std::vector<BlkRec> rects;
  for (size_t q = 0; q < hot.size(); ++q) {
    if (claimed[q]) continue;
    const i64 I = (i64)(hot[q] / (uint64_t)ntc), J = (i64)(hot[q] % (uint64_t)ntc);
    i64 w = 1;
    while (avail(I, J + w)) ++w;
    i64 h = 1;
    for (;;) {
      bool ok = true;
      for (i64 t = 0; t < w && ok; ++t) ok = avail(I + h, J + t);
      if (!ok) break;
      ++h;
    }
    for (i64 a = 0; a < h; ++a)
      for (i64 t = 0; t < w; ++t) claimed[find(I + a, J + t)] = 1;
    BlkRec b;
    b.r0 = (int32_t)(I * T);
    b.r1 = (int32_t)std::min<i64>((I + h) * T, nrows);
    b.c0 = (int32_t)(J * T);
    b.c1 = (int32_t)std::min<i64>((J + w) * T, ncols);
    rects.push_back(b);
  }
  return rects;
}

std::vector<TrimOut> tiled_for_T(const Resid& R, const DBuf<int32_t>& rows,
                                 const sable_thresholds& th, int T, i64& cov, hipStream_t s) {
  const i64 ntr = (R.nrows + T - 1) / T, ntc = (R.ncols + T - 1) / T;
  DBuf<uint64_t> keys(R.nnz);
  DBuf<int32_t> vals(R.nnz);
  k_tile_keys<<<grid_for(R.nnz, 256), 256, 0, s>>>(rows.p, R.col.p, R.nnz, T, ntc, keys.p, vals.p);
  LAUNCH_CHECK();
  sort_pairs_u64(keys, vals, R.nnz, bits_for((uint64_t)(ntr * ntc)), s);
  DBuf<uint64_t> uniq;
  DBuf<int32_t> cnt;
  const i64 nt = rle_u64(keys.p, R.nnz, uniq, cnt, s);
  DBuf<int32_t> flag(nt), pos(nt + 1);
  k_hot_flags<<<grid_for(nt, 256), 256, 0, s>>>(uniq.p, cnt.p, nt, T, ntc, R.nrows, R.ncols,
                                                th.delta_block_pm, flag.p);
  LAUNCH_CHECK();
  exclusive_scan_i32(flag.p, pos.p, nt, s);
  int32_t nhot = 0;
  HIPC(hipMemcpyAsync(&nhot, pos.p + nt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  DBuf<uint64_t> hot(nhot);
  if (nt) k_scatter_hot<<<grid_for(nt, 256), 256, 0, s>>>(uniq.p, flag.p, pos.p, nt, hot.p);
  LAUNCH_CHECK();
  std::vector<uint64_t> h_hot;
  to_host(h_hot, hot.p, nhot, s);
  std::vector<BlkRec> rects = greedy_rects(h_hot, ntr, ntc, T, R.nrows, R.ncols);
  std::vector<TrimOut> out;
  cov = 0;
  if (rects.empty()) return out;
  DBuf<BlkRec> d_rects;
  to_dev(d_rects, rects, s);
  DBuf<TrimOut> d_out(rects.size());
  k_trim_rects<<<(unsigned)rects.size(), 64, 0, s>>>(R.ptr.p, R.col.p, d_rects.p,
                                                     (int)rects.size(), d_out.p);
  LAUNCH_CHECK();
  std::vector<TrimOut> h;
  to_host(h, d_out.p, rects.size(), s);
  for (auto& o : h) {
    const i64 area = (i64)(o.r1 - o.r0) * (o.c1 - o.c0);
    if (!dense_enough(o.nnz, area, th.delta_block_pm) || area < th.amin_block || o.c1 - o.c0 < 2)
      continue;
    out.push_back(o);
    cov += o.nnz;
  }
  return out;
}

const int kTileSizes[5] = {4, 6, 8, 16, 32};

// Tile size reported for a residual without entries: the largest size in the candidate set.
int tile_for_empty(const sable_thresholds& th) {
  for (int t = 4; t >= 0; --t)
    if (!th.tile_set_mask || (th.tile_set_mask & (1 << t))) return kTileSizes[t];
  return 0;
}

std::vector<TrimOut> blocks_tiled(const Resid& R, const sable_thresholds& th, int& chosen,
                                  hipStream_t s) {
  const int* Ts = kTileSizes;
  chosen = 0;
  std::vector<TrimOut> best;
  if (R.nnz == 0) {
    chosen = tile_for_empty(th);
    return best;
  }
  DBuf<int32_t> rows;
  entry_rows(R, rows, s);
  i64 best_cov = -1;
  for (int t = 0; t < 5; ++t) {
    if (th.tile_set_mask && !(th.tile_set_mask & (1 << t))) continue;
    i64 cov = 0;
    std::vector<TrimOut> b = tiled_for_T(R, rows, th, Ts[t], cov, s);
    if (cov >= best_cov) { best_cov = cov; best.swap(b); chosen = Ts[t]; }
  }
  return best;
}

bool paper_fits(i64 nrows, i64 ncols) {
  const unsigned __int128 m = (unsigned __int128)std::max(nrows, ncols);
  return (unsigned __int128)nrows * (unsigned __int128)ncols * m <= ((unsigned __int128)1 << 37);
}

typedef unsigned __int128 u128;
constexpr u128 kSearchBudget = (u128)1 << 37;

// Spans (o0, o1) of one pass with o1 - o0 + 1 >= smin over n outer slices.
u128 span_pairs(i64 n, i64 smin) {
  const u128 k = n >= smin ? (u128)(n - smin + 1) : 0;
  return k * (k + 1) / 2;
}

// Work of the sparse scan over one pass: over the spans (o0, o1), o1 - o0 + 1 >= smin, one step
// plus min(Lin, entries of the span). The entries grow with o1, so for each o0 a binary search
// over the prefix sums P finds where they reach Lin, and the sum below that point comes from
// the prefix sums of P.
u128 scan_cost(const std::vector<i64>& cnt, i64 Lin, i64 smin) {
  const i64 n = (i64)cnt.size();
  std::vector<i64> P(n + 1, 0), Q(n + 2, 0);
  for (i64 i = 0; i < n; ++i) P[i + 1] = P[i] + cnt[i];
  for (i64 i = 0; i <= n; ++i) Q[i + 1] = Q[i] + P[i];
  u128 total = 0;
  for (i64 o0 = 0; o0 < n; ++o0) {
    const i64 a = o0 + smin - 1;
    if (a >= n) break;
    const i64 t = (i64)(std::lower_bound(P.begin() + a + 1, P.end(), P[o0] + Lin) - P.begin()) - 1;
    total += (u128)(n - a);
    total += (u128)((Q[t + 1] - Q[a + 1]) - (t - a) * P[o0]);
    total += (u128)(n - t) * (u128)Lin;
  }
  return total;
}

// Budget of the literal search on the VBR extractor's input: the dense scan's bound
// nrows * ncols * max(nrows, ncols) <= 2^37, or the sparse scan's work on this residual
// (rows pass + columns pass) <= 2^37.
bool paper_allowed(const Resid& R, const sable_thresholds& th, hipStream_t s) {
  if (paper_fits(R.nrows, R.ncols)) return true;
  const i64 smin = ceil_sqrt(th.amin_block);
  if (span_pairs(R.nrows, smin) + span_pairs(R.ncols, smin) > kSearchBudget) return false;
  std::vector<int32_t> ptr, col;
  to_host(ptr, R.ptr.p, (size_t)R.nrows + 1, s);
  to_host(col, R.col.p, (size_t)R.nnz, s);
  std::vector<i64> rc(R.nrows), cc(R.ncols, 0);
  for (int i = 0; i < R.nrows; ++i) rc[i] = ptr[i + 1] - ptr[i];
  for (int32_t c : col) cc[c] += 1;
  const u128 rows = scan_cost(rc, R.ncols, smin);
  return rows <= kSearchBudget && rows + scan_cost(cc, R.nrows, smin) <= kSearchBudget;
}

}  // namespace

// Before any GPU work: false only when even one step per span exceeds the budget (then no
// residual of these dimensions can be searched literally).
bool vbr_paper_fits(i64 nrows, i64 ncols, i64 amin) {
  if (paper_fits(nrows, ncols)) return true;
  const i64 smin = ceil_sqrt(amin);
  return span_pairs(nrows, smin) + span_pairs(ncols, smin) <= kSearchBudget;
}

void blocks_none(sable_plan_s& P, const sable_thresholds& th, int mode) {
  if (mode == SABLE_VBR_AUTO) mode = paper_fits(P.nrows, P.ncols) ? SABLE_VBR_PAPER : SABLE_VBR_TILED;
  P.vbr_mode_used = mode;
  P.vbr_tile = mode == SABLE_VBR_TILED ? tile_for_empty(th) : 0;
}

void extract_blocks(sable_plan_s& P, const Resid& R, const sable_thresholds& th, int mode,
                    DBuf<uint8_t>& claimed, hipStream_t s) {
  if (mode == SABLE_VBR_AUTO) mode = paper_allowed(R, th, s) ? SABLE_VBR_PAPER : SABLE_VBR_TILED;
  else if (mode == SABLE_VBR_PAPER && !paper_allowed(R, th, s))
    SB_THROW(SABLE_ERR_TOO_LARGE, "literal block search over budget for this %dx%d residual",
             R.nrows, R.ncols);
  std::vector<TrimOut> B;
  int T = 0;
  if (mode == SABLE_VBR_PAPER) B = blocks_paper(R, th, s);
  else B = blocks_tiled(R, th, T, s);
  i64 cov = 0;
  for (auto& b : B) cov += b.nnz;
  if ((__int128)1000 * cov < (__int128)th.coverage_pm * R.nnz) B.clear();  // coverage cutoff
  std::sort(B.begin(), B.end(), [](const TrimOut& a, const TrimOut& b) {
    return a.r0 != b.r0 ? a.r0 < b.r0 : a.c0 < b.c0;
  });
  P.vbr_mode_used = mode;
  P.vbr_tile = T;
  const int nb = (int)B.size();
  std::vector<int32_t> blk(4 * (size_t)nb), rpre(nb);
  std::vector<i64> bvp(nb);
  std::vector<BlkRec> recs(nb);
  i64 cells = 0, rows_total = 0, nnz = 0;
  for (int k = 0; k < nb; ++k) {
    const TrimOut& b = B[k];
    blk[4 * k] = b.r0; blk[4 * k + 1] = b.r1; blk[4 * k + 2] = b.c0; blk[4 * k + 3] = b.c1;
    recs[k] = BlkRec{b.r0, b.r1, b.c0, b.c1};
    bvp[k] = cells;
    rpre[k] = (int32_t)rows_total;
    cells += (i64)(b.r1 - b.r0) * (b.c1 - b.c0);
    rows_total += b.r1 - b.r0;
    nnz += b.nnz;
  }
  P.nblk = nb;
  P.vbr_cells = cells;
  P.vbr_nnz = nnz;
  to_dev(P.blk, blk, s);
  to_dev(P.blk_val_ptr, bvp, s);
  P.vbr_val.alloc(cells);
  if (cells) HIPC(hipMemsetAsync(P.vbr_val.p, 0, cells * sizeof(float), s));
  if (nb) {
    DBuf<int32_t> d_rpre;
    DBuf<BlkRec> d_recs;
    to_dev(d_rpre, rpre, s);
    to_dev(d_recs, recs, s);
    k_pack_vbr<<<grid_for(rows_total, 256), 256, 0, s>>>(d_rpre.p, nb, rows_total, d_recs.p,
                                                         P.blk_val_ptr.p, R.ptr.p, R.col.p,
                                                         R.val.p, R.id.p, P.vbr_val.p, claimed.p,
                                                         P.owner.p, P.slot.p);
    LAUNCH_CHECK();
    HIPC(hipStreamSynchronize(s));
  }
  HIPC(hipStreamSynchronize(s));
}

}  // namespace sable
