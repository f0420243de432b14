// Executor: tile schedule, fused SpMV / SpMM launches, plain CSR baseline, bf16 split.
#include <algorithm>
#include <cmath>

#include "exec.h"
#include "spmm_panel.h"

namespace sable {

void build_tiles(sable_plan_s& P, Schedule& S, int RT, bool with_formats, bool col_order,
                 hipStream_t s);

PlanView make_view(const sable_plan_s& P, const Schedule& S, bool plain, bool far) {
  PlanView v;
  std::memset(&v, 0, sizeof(v));
  v.nrows = P.nrows;
  v.ncols = P.ncols;
  v.rows_per_tile = S.rows_per_tile;
  v.ntiles = S.ntiles;
  v.tile_seg_lo = S.tile_seg_lo.p;
  v.tile_seg_hi = S.tile_seg_hi.p;
  v.tile_blk_ptr = S.tile_blk_ptr.p;
  v.tile_blk = S.tile_blk.p;
  v.tile_order = S.order.p;
  v.tile_head = S.head.p;
  v.tile_row0 = S.row0.p;
  v.vdia_val64 = P.vdia_val64.p;
  v.vbr_val64 = P.vbr_val64.p;
  v.csr_val64 = P.csr_val64.p;
  if (plain) {
    v.csr_ptr = P.a_ptr.p;
    v.csr_col = P.a_col.p;
    v.csr_val = P.a_val.p;
    return v;
  }
  v.nseg = P.nseg;
  v.nblk = P.nblk;
  v.vdia_val = P.vdia_val.p;
  v.idiag = P.idiag.p;
  v.seg_row_start = P.seg_row_start.p;
  v.seg_nrows = P.seg_nrows.p;
  v.seg_ndiags = P.seg_ndiags.p;
  v.seg_val_ptr = P.seg_val_ptr.p;
  v.seg_idiag_ptr = P.seg_idiag_ptr.p;
  v.blk = P.blk.p;
  v.blk_val_ptr = P.blk_val_ptr.p;
  v.vbr_val = P.vbr_val.p;
  v.vbr_mma = P.vbr_mma.p;
  v.blk_mma_ptr = P.blk_mma_ptr.p;
  v.csr_ptr = P.csr_ptr.p;
  v.csr_col = P.csr_col.p;
  v.csr_val = P.csr_val.p;
  if (&S == &P.sched_mm && P.mm_panels.kptr.p) {
    v.mm_kcol = P.mm_panels.kcol.p;
    v.mm_kptr = P.mm_panels.kptr.p;
    v.mm_bpos = P.mm_panels.bpos.p;
    v.mm_apack = P.mm_panels.apack.p;
    v.mm_amask = P.mm_panels.amask.p;
    v.mm_aptr = P.mm_panels.aptr.p;
  }
  if (far && P.far.npanel && P.prm.far_split) {
    v.csr_col = P.far.ccol.p;
    v.far_prod = P.far.far_prod.p;
    v.far_prod64 = P.far.far_prod64.p;
  }
  return v;
}

namespace {

// ---- schedule ----------------------------------------------------------------------------

// Rows [a, b) of tile t: from the row bound table if there is one, else uniform tiles of RT.
__device__ __forceinline__ void sched_rows(const int32_t* row0, int RT, int nrows, i64 t, int& a, int& b) {
  if (row0) {
    a = row0[t];
    b = row0[t + 1];
  } else {
    a = (int)(t * RT);
    b = (int)min((i64)nrows, (t + 1) * RT);
  }
}

// Tile of row r.
__device__ __forceinline__ int sched_tile(const int32_t* row0, int RT, int ntiles, int r) {
  if (!row0) return r / RT;
  int l = 0, h = ntiles - 1;
  while (l < h) { const int m = (l + h + 1) >> 1; if (row0[m] <= r) l = m; else h = m - 1; }
  return l;
}

__global__ void k_tile_segs(const int32_t* __restrict__ srs, const int32_t* __restrict__ snr,
                            int nseg, int RT, const int32_t* __restrict__ row0, int ntiles,
                            int nrows, int32_t* __restrict__ lo, int32_t* __restrict__ hi) {
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < ntiles; t += (i64)gridDim.x * blockDim.x) {
    int a, b;
    sched_rows(row0, RT, nrows, t, a, b);
    int l = 0, h = nseg;  // first segment whose end > a (ends are sorted: segments disjoint)
    while (l < h) { int m = (l + h) >> 1; if (srs[m] + snr[m] <= a) l = m + 1; else h = m; }
    lo[t] = l;
    l = 0; h = nseg;      // first segment starting at or after b
    while (l < h) { int m = (l + h) >> 1; if (srs[m] < b) l = m + 1; else h = m; }
    hi[t] = l;
  }
}

__global__ void k_blk_tile_counts(const int32_t* __restrict__ blk, int nblk, int RT,
                                  const int32_t* __restrict__ row0, int ntiles,
                                  int32_t* __restrict__ cnt) {
  for (i64 b = blockIdx.x * (i64)blockDim.x + threadIdx.x; b < nblk; b += (i64)gridDim.x * blockDim.x)
    cnt[b] = sched_tile(row0, RT, ntiles, blk[4 * b + 1] - 1) - sched_tile(row0, RT, ntiles, blk[4 * b]) + 1;
}

// (tile, block) pairs keyed by tile, then by rank[b] (the block's position in the order a
// tile visits its blocks; the block index itself when rank is null).
__global__ void k_blk_tile_pairs(const int32_t* __restrict__ blk, const int32_t* __restrict__ off,
                                 const int32_t* __restrict__ rank, int nblk, int RT,
                                 const int32_t* __restrict__ row0, int ntiles,
                                 uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
  for (i64 b = blockIdx.x * (i64)blockDim.x + threadIdx.x; b < nblk; b += (i64)gridDim.x * blockDim.x) {
    const int t0 = sched_tile(row0, RT, ntiles, blk[4 * b]);
    const int t1 = sched_tile(row0, RT, ntiles, blk[4 * b + 1] - 1);
    const uint64_t low = (uint64_t)(uint32_t)(rank ? rank[b] : (int32_t)b);
    for (int t = t0; t <= t1; ++t) {
      keys[off[b] + (t - t0)] = ((uint64_t)t << 32) | low;
      vals[off[b] + (t - t0)] = (int32_t)b;
    }
  }
}

__global__ void k_tile_ptr(const uint64_t* __restrict__ keys, i64 n, int ntiles,
                           int32_t* __restrict__ ptr) {
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t <= ntiles; t += (i64)gridDim.x * blockDim.x) {
    const uint64_t key = (uint64_t)t << 32;
    i64 l = 0, h = n;
    while (l < h) { i64 m = (l + h) >> 1; if (keys[m] < key) l = m + 1; else h = m; }
    ptr[t] = (int32_t)l;
  }
}

// Estimated cost of each tile: CSR entries (weight 2: index, value and a gathered x) plus
// VBR cells plus VDIA cells of the tile.
__global__ void k_tile_cost(const int32_t* __restrict__ ptr, int nrows, int RT,
                            const int32_t* __restrict__ row0, int ntiles,
                            const int32_t* __restrict__ slo, const int32_t* __restrict__ shi,
                            const int32_t* __restrict__ srs, const int32_t* __restrict__ snr,
                            const int32_t* __restrict__ snd, const int32_t* __restrict__ bptr,
                            const int32_t* __restrict__ tblk, const int32_t* __restrict__ blk,
                            i64* __restrict__ cost) {
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < ntiles; t += (i64)gridDim.x * blockDim.x) {
    int a, b;
    sched_rows(row0, RT, nrows, t, a, b);
    i64 c = 2 * (i64)(ptr[b] - ptr[a]);
    if (slo)
      for (int s = slo[t]; s < shi[t]; ++s)
        c += (i64)(min(b, srs[s] + snr[s]) - max(a, srs[s])) * snd[s];
    for (int q = bptr[t]; q < bptr[t + 1]; ++q) {
      const int* B = blk + 4 * tblk[q];
      c += (i64)(min(b, B[1]) - max(a, B[0])) * (B[3] - B[2]);
    }
    cost[t] = c;
  }
}

// Keys (first column, first row) of every block, for the column-major visiting order.
__global__ void k_blk_col_keys(const int32_t* __restrict__ blk, int nblk, uint64_t* __restrict__ keys,
                               int32_t* __restrict__ ids) {
  for (i64 b = blockIdx.x * (i64)blockDim.x + threadIdx.x; b < nblk; b += (i64)gridDim.x * blockDim.x) {
    keys[b] = ((uint64_t)(uint32_t)blk[4 * b + 2] << 32) | (uint64_t)(uint32_t)blk[4 * b];
    ids[b] = (int32_t)b;
  }
}

__global__ void k_rank_of(const int32_t* __restrict__ ids, int n, int32_t* __restrict__ rank) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    rank[ids[i]] = (int32_t)i;
}

__global__ void k_zero_i32(int32_t* __restrict__ a, i64 n) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x) a[k] = 0;
}

// ---- bf16 split (round to nearest even) -----------------------------------------------------

__device__ inline uint16_t to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// One workgroup per block: element (r, k) of the block (column-major in vbr_val) becomes the
// word hi | lo << 16 at row-major position r * w4 + k; padding columns k >= w hold 0.
__global__ void k_split_mma(const int32_t* __restrict__ blk, const i64* __restrict__ bvp,
                            const i64* __restrict__ mptr, const float* __restrict__ val,
                            uint32_t* __restrict__ out) {
  const int b = blockIdx.x;
  const int h = blk[4 * b + 1] - blk[4 * b], w = blk[4 * b + 3] - blk[4 * b + 2];
  const int w4 = (w + 3) & ~3;
  const i64 vp = bvp[b], mp = mptr[b];
  for (i64 e = threadIdx.x; e < (i64)h * w4; e += blockDim.x) {
    const int r = (int)(e / w4), k = (int)(e % w4);
    uint32_t word = 0;
    if (k < w) {
      const float v = val[vp + (i64)k * h + r];
      const uint16_t hi = to_bf16_rne(v);
      const uint16_t lo = to_bf16_rne(v - __uint_as_float((uint32_t)hi << 16));
      word = (uint32_t)hi | ((uint32_t)lo << 16);
    }
    out[mp + e] = word;
  }
}

// ---- products ---------------------------------------------------------------------------------

template <int W>
__global__ __launch_bounds__(256) void k_spmv_fused(PlanView P, const float* __restrict__ x,
                                                   float* __restrict__ y) {
  __shared__ float part[256];
  spmv_tile<W>(P, blockIdx.x, x, y, part);
}

template <int RPT, bool NT>
__global__ __launch_bounds__(256) void k_spmv_stream(PlanView P, const float* __restrict__ x,
                                                    float* __restrict__ y) {
  __shared__ float lds[kCsrChunk + kSpmvThreads * RPT];
  const int slot = xcd_tile(blockIdx.x, P.ntiles);
  if (slot >= P.ntiles) return;
  spmv_tile_stream<RPT, NT>(P, slot, x, y, lds);
}

// Persistent streamed SpMV (256-row tiles): nw workgroups per XCD; workgroup j of XCD xs
// takes the launch slots j, j + nw, ... of that XCD's contiguous run of slots. While one
// tile's body runs, the next tile's record is loaded; its row pointers and first CSR pass are
// issued as soon as the body's stores are, so each tile starts with only its gathers of x
// outstanding instead of the chain record -> row pointers -> entries -> x. Every tile runs
// the streamed body unchanged (results equal the one-tile-per-workgroup launch bit for bit).
template <bool NT>
__device__ __forceinline__ void spmv_persist(const PlanView& P, const float* __restrict__ x,
                                             float* __restrict__ y, int nw, float* lds) {
  const int per = (P.ntiles + 7) >> 3;
  const int xs = blockIdx.x & 7;
  const int s1 = min(P.ntiles, (xs + 1) * per);
  int slot = xs * per + (int)(blockIdx.x >> 3);
  if (slot >= s1) return;
  StreamTile<1, float> S;
  S.H = P.tile_head[slot];
  stream_prefetch<1, NT, float>(P, S);
  for (;;) {
    const int next = slot + nw;
    const bool more = next < s1;
    TileHead Hn;
    if (more) Hn = P.tile_head[next];
    stream_body<1, NT, float>(P, S, x, y, lds);
    if (!more) break;
    S.H = Hn;
    stream_prefetch<1, NT, float>(P, S);
    slot = next;
  }
}

template <bool NT>
__global__ __launch_bounds__(256) void k_spmv_persist(PlanView P, const float* __restrict__ x,
                                                     float* __restrict__ y, int nw) {
  __shared__ float lds[kCsrChunk + kSpmvThreads];
  spmv_persist<NT>(P, x, y, nw, lds);
}

// The plain CSR baseline's persistent variants (the same body over the input as one CSR).
template <bool NT>
__global__ __launch_bounds__(256) void k_csr_persist(PlanView P, const float* __restrict__ x,
                                                    float* __restrict__ y, int nw) {
  __shared__ float lds[kCsrChunk + kSpmvThreads];
  spmv_persist<NT>(P, x, y, nw, lds);
}

// Row-length bins: subwave widths per bin (u = log2 of entries per lane).
__global__ __launch_bounds__(256) void k_spmv_binned(PlanView P, const int32_t* __restrict__ brow,
                                                    const int32_t* __restrict__ boff, int u,
                                                    const float* __restrict__ x,
                                                    float* __restrict__ y) {
  __shared__ float part[kSpmvThreads];
  int tile = xcd_tile(blockIdx.x, P.ntiles);
  if (tile >= P.ntiles) return;
  if (P.tile_order) tile = P.tile_order[tile];
  spmv_tile_binned(P, tile, brow, boff, u, x, y, part);
}

// The plain CSR baseline's binned variants (the same body over the input as one CSR matrix).
__global__ __launch_bounds__(256) void k_csr_binned(PlanView P, const int32_t* __restrict__ brow,
                                                   const int32_t* __restrict__ boff, int u,
                                                   const float* __restrict__ x,
                                                   float* __restrict__ y) {
  __shared__ float part[kSpmvThreads];
  int tile = xcd_tile(blockIdx.x, P.ntiles);
  if (tile >= P.ntiles) return;
  if (P.tile_order) tile = P.tile_order[tile];
  spmv_tile_binned(P, tile, brow, boff, u, x, y, part);
}

// Far-column gather: workgroup b runs on XCD b mod 8 and takes that XCD's (b / 8)-th work
// item (begin, end, panel); it stages the panel's x slice in LDS with coalesced loads, then
// multiplies its entries by x values read from LDS.
template <class T>
__global__ __launch_bounds__(kFarThreads) void k_far_gather(const int32_t* __restrict__ chunk,
                                                           int per_xcd, int ncols,
                                                           const uint16_t* __restrict__ col,
                                                           const T* __restrict__ val,
                                                           const T* __restrict__ x,
                                                           T* __restrict__ prod) {
  __shared__ T xs[kFarPanelCols];  // fp32: 32 KB, fp64: 64 KB
  const int* c = chunk + 3 * ((blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3));
  const int b = c[0], e = c[1], panel = c[2];
  if (b < 0) return;
  const int t = threadIdx.x;
  const int base = panel * kFarPanelCols;
  const int w = min(kFarPanelCols, ncols - base);
  // this thread's entries first (independent of the slice), then the slice
  int j[8];
  T a[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = b + t + kFarThreads * u;
    j[u] = k < e ? (int)__builtin_nontemporal_load(col + k) : 0;
    a[u] = k < e ? __builtin_nontemporal_load(val + k) : T(0);
  }
  // slice: all loads of a thread in flight together (fp32: float4 when x is 16-byte aligned)
  bool vec = false;
  if constexpr (sizeof(T) == 4) {
    vec = ((uintptr_t)x & 15) == 0 && w == kFarPanelCols;
    if (vec) {
      constexpr int kV = kFarPanelCols / (4 * kFarThreads);  // float4 per thread
      float4 v[kV];
      const float4* x4 = reinterpret_cast<const float4*>(x + base);
#pragma unroll
      for (int u = 0; u < kV; ++u) v[u] = x4[t + kFarThreads * u];
#pragma unroll
      for (int u = 0; u < kV; ++u) reinterpret_cast<float4*>(xs)[t + kFarThreads * u] = v[u];
    }
  }
  if (!vec) {
    for (int i0 = 0; i0 < w; i0 += 8 * kFarThreads) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + t + kFarThreads * u;
        v[u] = i < w ? x[base + i] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + t + kFarThreads * u;
        if (i < w) xs[i] = v[u];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = b + t + kFarThreads * u;
    if (k < e) prod[k] = a[u] * xs[j[u]];
  }
}

// The plain CSR baseline's streamed variants: the same tile body over the input as one CSR
// matrix, under a kernel name of its own so profiles keep the two apart.
template <int RPT, bool NT>
__global__ __launch_bounds__(256) void k_csr_stream(PlanView P, const float* __restrict__ x,
                                                   float* __restrict__ y) {
  __shared__ float lds[kCsrChunk + kSpmvThreads * RPT];
  const int slot = xcd_tile(blockIdx.x, P.ntiles);
  if (slot >= P.ntiles) return;
  spmv_tile_stream<RPT, NT>(P, slot, x, y, lds);
}

template <int W>
__global__ __launch_bounds__(256) void k_spmv_plain(const int32_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ col,
                                                   const float* __restrict__ val, int nrows,
                                                   const float* __restrict__ x, float* __restrict__ y) {
  const int rows_per_block = 256 / W;
  csr_rows<W>(ptr, col, val, nrows, x, y, blockIdx.x * rows_per_block, rows_per_block);
}

// Blocks on matrix cores (mfma 1 or 2; the VALU block path is compiled out, so it does not
// set this kernel's register budget).
__global__ __launch_bounds__(kMmThreads, 4) void k_spmm_tile(PlanView P, const float* __restrict__ X,
                                                         float* __restrict__ Y, int n, int mfma) {
  __shared__ float ys[kMmRows * kMmCols + kMmBlkStage * kBlkDesc];
  const int ntile = (P.nrows + kMmRows - 1) / kMmRows;
  int t = xcd_tile(blockIdx.x, ntile);
  if (t >= ntile) return;
  if (P.tile_order) t = P.tile_order[t];
  spmm_tile(P, t * kMmRows, blockIdx.y * kMmCols, n, X, Y, ys, mfma == 2 ? 2 : 1);
}

// Blocks on the VALU in fp32 (the same tile, mfma = 0).
__global__ __launch_bounds__(kMmThreads, 4) void k_spmm_tile_valu(PlanView P, const float* __restrict__ X,
                                                              float* __restrict__ Y, int n) {
  __shared__ float ys[kMmRows * kMmCols + kMmBlkStage * kBlkDesc];
  const int ntile = (P.nrows + kMmRows - 1) / kMmRows;
  int t = xcd_tile(blockIdx.x, ntile);
  if (t >= ntile) return;
  if (P.tile_order) t = P.tile_order[t];
  spmm_tile(P, t * kMmRows, blockIdx.y * kMmCols, n, X, Y, ys, 0);
}

// One workgroup per panel: the tile's block cells that fall in the panel's 32 list positions
// are placed in a zero-filled 64 x 32 hi plane and lo plane in LDS, with the units (row, 8
// columns) that receive a cell marked. write == 0: the panel's occupancy mask is stored;
// write == 1: its marked units are stored in mask order from apack[2 aptr[g]] on.
__global__ __launch_bounds__(256) void k_pack_panels(PlanView P, const int32_t* __restrict__ pan_tile,
                                                    const int32_t* __restrict__ pan_pos,
                                                    uint64_t* __restrict__ amask,
                                                    const i64* __restrict__ aptr,
                                                    uint4* __restrict__ apack, int write) {
  __shared__ __align__(16) uint16_t pl[2 * kMmRows * kPanK];
  __shared__ uint8_t occ[kMmRows * kPanK / 8];
  const i64 g = blockIdx.x;
  const int tile = pan_tile[g], pj = pan_pos[g];
  const int r0 = tile * kMmRows, rend = min(r0 + kMmRows, P.nrows);
  for (int i = threadIdx.x; i < 2 * kMmRows * kPanK / 4; i += blockDim.x)  // both planes
    reinterpret_cast<uint64_t*>(pl)[i] = 0ull;
  for (int i = threadIdx.x; i < kMmRows * kPanK / 8; i += blockDim.x) occ[i] = 0;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int q = P.tile_blk_ptr[tile] + wave; q < P.tile_blk_ptr[tile + 1]; q += 4) {
    const int b = P.tile_blk[q], p0 = P.mm_bpos[q];
    const int br0 = P.blk[4 * b], br1 = P.blk[4 * b + 1];
    const int w = P.blk[4 * b + 3] - P.blk[4 * b + 2];
    const int ka = max(p0, pj), kz = min(p0 + w, pj + kPanK);
    const int ra = max(br0, r0), rz = min(br1, rend);
    if (ka >= kz || ra >= rz) continue;
    const int nk = kz - ka, cells = (rz - ra) * nk, w4 = (w + 3) & ~3;
    const uint32_t* src = P.vbr_mma + P.blk_mma_ptr[b];
    for (int c = lane; c < cells; c += 64) {
      const int r = ra + c / nk, kk = ka + c % nk;
      const uint32_t word = src[(i64)(r - br0) * w4 + (kk - p0)];
      const int e = (r - r0) * kPanK + (kk - pj);
      pl[e] = (uint16_t)(word & 0xffffu);
      pl[kMmRows * kPanK + e] = (uint16_t)(word >> 16);
      occ[e >> 3] = 1;  // the same value from every writer
    }
  }
  __syncthreads();
  const int u = threadIdx.x;  // one unit per thread (256 units)
  const bool set = occ[u] != 0;
  const uint64_t m = __ballot(set);
  if (!write) {
    if (lane == 0) amask[4 * g + wave] = m;
    return;
  }
  int before = 0;
  for (int i = 0; i < wave; ++i) before += __popcll(amask[4 * g + i]);
  if (set) {
    const int rank = before + __popcll(m & ((1ull << lane) - 1ull));
    uint4* out = apack + 2 * (aptr[g] + rank);
    out[0] = reinterpret_cast<const uint4*>(pl)[u];
    out[1] = reinterpret_cast<const uint4*>(pl + kMmRows * kPanK)[u];
  }
}

// Blocks on matrix cores from LDS-staged panels (16x16x32 bf16 steps).
__global__ __launch_bounds__(kMmThreads, 5) void k_spmm_panel(PlanView P, const float* __restrict__ X,
                                                          float* __restrict__ Y, int n) {
  __shared__ __align__(16) uint8_t lds[kPanLdsBytes];
  const int ntile = (P.nrows + kMmRows - 1) / kMmRows;
  int t = xcd_tile(blockIdx.x, ntile);
  if (t >= ntile) return;
  if (P.tile_order) t = P.tile_order[t];
  spmm_tile_panel(P, t, blockIdx.y * kMmCols, n, X, Y, lds);
}

// FP64 executor: the same streamed SpMV tile body and SpMM tile (blocks on the VALU) over the
// plan's fp64 value copies.
template <int RPT>
__global__ __launch_bounds__(256) void k_spmv_stream_f64(PlanView P, const double* __restrict__ x,
                                                        double* __restrict__ y) {
  __shared__ double lds[kCsrChunk + kSpmvThreads * RPT];
  const int slot = xcd_tile(blockIdx.x, P.ntiles);
  if (slot >= P.ntiles) return;
  spmv_tile_stream<RPT, false, double>(P, slot, x, y, reinterpret_cast<float*>(lds));
}

__global__ __launch_bounds__(kMmThreads) void k_spmm_tile_f64(PlanView P, const double* __restrict__ X,
                                                             double* __restrict__ Y, int n) {
  __shared__ double ys[kMmRows * kMmCols + kMmBlkStage * kBlkDesc / 2];
  const int ntile = (P.nrows + kMmRows - 1) / kMmRows;
  int t = xcd_tile(blockIdx.x, ntile);
  if (t >= ntile) return;
  if (P.tile_order) t = P.tile_order[t];
  spmm_tile<double>(P, t * kMmRows, blockIdx.y * kMmCols, n, X, Y, reinterpret_cast<float*>(ys), 0);
}

// Fused SpMM (VALU): one wave per row, lanes across 64-column chunks of X / Y.
__global__ __launch_bounds__(256) void k_spmm_fused_valu(PlanView P, const float* __restrict__ X,
                                                        float* __restrict__ Y, int n) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + wave;
  if (r >= P.nrows) return;
  // band segment containing r
  int s = -1;
  {
    int lo = 0, hi = P.nseg - 1;
    while (lo <= hi) {
      int m = (lo + hi) >> 1;
      if (P.seg_row_start[m] <= r) { s = m; lo = m + 1; } else hi = m - 1;
    }
    if (s >= 0 && r >= P.seg_row_start[s] + P.seg_nrows[s]) s = -1;
  }
  const int tile = tile_of_row(P, r);
  for (int cb = 0; cb < n; cb += 64) {
    const int c = cb + lane;
    const bool ok = c < n;
    float acc = 0.f;
    if (s >= 0) {
      const int rs = P.seg_row_start[s], nr = P.seg_nrows[s], nd = P.seg_ndiags[s];
      const int32_t* od = P.idiag + P.seg_idiag_ptr[s];
      const float* v = P.vdia_val + P.seg_val_ptr[s] + (r - rs);
      for (int t = 0; t < nd; ++t) {
        const int col = r + od[t];
        if ((unsigned)col < (unsigned)P.ncols && ok) acc += v[(i64)t * nr] * X[(i64)col * n + c];
      }
    }
    for (int q = P.tile_blk_ptr[tile]; q < P.tile_blk_ptr[tile + 1]; ++q) {
      const int b = P.tile_blk[q];
      const int br0 = P.blk[4 * b], br1 = P.blk[4 * b + 1];
      if (r < br0 || r >= br1) continue;
      const int c0 = P.blk[4 * b + 2], c1 = P.blk[4 * b + 3], h = br1 - br0;
      const float* v = P.vbr_val + P.blk_val_ptr[b] + (r - br0);
      if (ok)
        for (int cc = c0; cc < c1; ++cc) acc += v[(i64)(cc - c0) * h] * X[(i64)cc * n + c];
    }
    float cs = 0.f;
    if (ok)
      for (int k = P.csr_ptr[r]; k < P.csr_ptr[r + 1]; ++k) cs += P.csr_val[k] * X[(i64)P.csr_col[k] * n + c];
    if (ok) Y[(i64)r * n + c] = acc + cs;
  }
}

}  // namespace

static void build_order(const sable_plan_s& P, Schedule& S, bool with_formats, hipStream_t s,
                        bool coarse);

static void build_heads(const sable_plan_s& P, Schedule& S, bool with_formats, hipStream_t s);

void build_schedule(sable_plan_s& P, Schedule& S, int RT, bool with_formats, hipStream_t s,
                    bool col_order, bool balance) {
  S.row0.reset();
  if (balance && P.nrows > 0) {  // entry-balanced tile bounds from the CSR row pointers
    std::vector<int32_t> ptr, r0;
    to_host(ptr, with_formats ? P.csr_ptr.p : P.a_ptr.p, (size_t)P.nrows + 1, s);
    // at most max(4096, 8 RT) entries per tile; on small inputs fewer (down to 512), so that
    // there are about 2048 tiles (8 per CU) and no workgroup carries a long serial chain
    const i64 total = ptr[P.nrows];
    const i64 emax = std::min<i64>(std::max<i64>(4096, 8 * (i64)RT),
                                   std::max<i64>(512, (total + 2047) / 2048));
    bool split = false;
    for (int r = 0; r < P.nrows;) {
      int r1 = std::min(P.nrows, r + RT);
      if (ptr[r1] - ptr[r] > emax) {  // largest r1 > r with at most emax entries (>= 1 row)
        int lo = r + 1, hi = r1;
        while (lo < hi) { const int m = (lo + hi + 1) / 2; if (ptr[m] - ptr[r] <= emax) lo = m; else hi = m - 1; }
        r1 = lo;
        split = true;
      }
      r0.push_back(r);
      r = r1;
    }
    r0.push_back(P.nrows);
    if (split) to_dev(S.row0, r0, s);  // uniform tiling already balanced: keep it implicit
  }
  build_tiles(P, S, RT, with_formats, col_order, s);
  build_order(P, S, with_formats, s, col_order);
  if (balance) build_heads(P, S, with_formats, s);
}

// One record per launch slot of a streamed SpMV schedule (host-side from the tile tables).
static void build_heads(const sable_plan_s& P, Schedule& S, bool with_formats, hipStream_t s) {
  S.head.reset();
  const int nt = S.ntiles;
  if (nt == 0) return;
  std::vector<int32_t> ptr, row0, ord, slo, shi, bptr;
  to_host(ptr, with_formats ? P.csr_ptr.p : P.a_ptr.p, (size_t)P.nrows + 1, s);
  if (S.row0.p) to_host(row0, S.row0.p, (size_t)nt + 1, s);
  if (S.order.p) to_host(ord, S.order.p, (size_t)nt, s);
  to_host(slo, S.tile_seg_lo.p, (size_t)nt, s);
  to_host(shi, S.tile_seg_hi.p, (size_t)nt, s);
  to_host(bptr, S.tile_blk_ptr.p, (size_t)nt + 1, s);
  const int nseg = with_formats ? P.nseg : 0;
  std::vector<int32_t> srs, snr, snd, sip;
  std::vector<i64> svp;
  if (nseg) {
    to_host(srs, P.seg_row_start.p, nseg, s);
    to_host(snr, P.seg_nrows.p, nseg, s);
    to_host(snd, P.seg_ndiags.p, nseg, s);
    to_host(sip, P.seg_idiag_ptr.p, nseg, s);
    to_host(svp, P.seg_val_ptr.p, nseg, s);
  }
  std::vector<TileHead> h(nt);
  for (int k = 0; k < nt; ++k) {
    const int t = S.order.p ? ord[k] : k;
    TileHead& H = h[k];
    std::memset(&H, 0, sizeof(H));
    H.tile = t;
    H.r0 = S.row0.p ? row0[t] : t * S.rows_per_tile;
    H.rend = S.row0.p ? row0[t + 1] : std::min(P.nrows, (t + 1) * S.rows_per_tile);
    H.e0 = ptr[H.r0];
    H.e1 = ptr[H.rend];
    H.slo = slo[t];
    H.shi = shi[t];
    H.blo = bptr[t];
    H.bhi = bptr[t + 1];
    if (H.slo < H.shi) {
      H.rs = srs[H.slo];
      H.nr = snr[H.slo];
      H.nd = snd[H.slo];
      H.sip = sip[H.slo];
      H.svp = svp[H.slo];
    }
  }
  to_dev(S.head, h, s);
  HIPC(hipStreamSynchronize(s));
}

// coarse: costs are compared in half-octave classes, so tiles of about the same cost keep their
// row order (SpMM: neighbouring tiles read many of the same X rows, which then meet in L2);
// tiles much heavier than the rest still go first.
static void build_order(const sable_plan_s& P, Schedule& S, bool with_formats, hipStream_t s,
                        bool coarse) {
  const int nt = S.ntiles;
  if (nt < 2) return;
  DBuf<i64> cost(nt);
  const bool fm = with_formats && P.nseg;
  k_tile_cost<<<grid_for(nt, 256), 256, 0, s>>>(
      with_formats ? P.csr_ptr.p : P.a_ptr.p, P.nrows, S.rows_per_tile, S.row0.p, nt,
      fm ? S.tile_seg_lo.p : nullptr, fm ? S.tile_seg_hi.p : nullptr, P.seg_row_start.p,
      P.seg_nrows.p, P.seg_ndiags.p, S.tile_blk_ptr.p, S.tile_blk.p,
      with_formats ? P.blk.p : nullptr, cost.p);
  LAUNCH_CHECK();
  std::vector<i64> hc;
  to_host(hc, cost.p, nt, s);
  if (coarse)
    for (auto& c : hc) c = (i64)std::floor(2.0 * std::log2(1.0 + (double)c));
  // slot i of XCD run x holds tile xcd_tile(8*i + x); sort each run's tiles by cost
  const int per = (nt + 7) >> 3;
  std::vector<int32_t> ord(nt);
  for (int t = 0; t < nt; ++t) ord[t] = t;
  for (int x = 0; x < 8; ++x) {
    const int a = std::min(nt, x * per), b = std::min(nt, (x + 1) * per);
    std::stable_sort(ord.begin() + a, ord.begin() + b,
                     [&](int32_t u, int32_t v) { return hc[u] > hc[v]; });
  }
  to_dev(S.order, ord, s);
  HIPC(hipStreamSynchronize(s));
}

// col_order: each tile visits its blocks by (first column, first row) instead of block
// order (SpMM: blocks that read overlapping rows of X run back to back).
void build_tiles(sable_plan_s& P, Schedule& S, int RT, bool with_formats, bool col_order,
                 hipStream_t s) {
  S.rows_per_tile = RT;
  S.ntiles = S.row0.p ? (int)S.row0.n - 1 : (P.nrows + RT - 1) / RT;
  const int nt = S.ntiles;
  S.tile_seg_lo.alloc(nt);
  S.tile_seg_hi.alloc(nt);
  S.tile_blk_ptr.alloc(nt + 1);
  const int nseg = with_formats ? P.nseg : 0;
  const int nblk = with_formats ? P.nblk : 0;
  if (nt) {
    if (nseg) {
      k_tile_segs<<<grid_for(nt, 256), 256, 0, s>>>(P.seg_row_start.p, P.seg_nrows.p, nseg, RT,
                                                    S.row0.p, nt, P.nrows, S.tile_seg_lo.p,
                                                    S.tile_seg_hi.p);
    } else {
      k_zero_i32<<<grid_for(nt, 256), 256, 0, s>>>(S.tile_seg_lo.p, nt);
      LAUNCH_CHECK();
      k_zero_i32<<<grid_for(nt, 256), 256, 0, s>>>(S.tile_seg_hi.p, nt);
    }
    LAUNCH_CHECK();
  }
  if (!nblk) {
    S.tile_blk.alloc(1);
    k_zero_i32<<<grid_for(nt + 1, 256), 256, 0, s>>>(S.tile_blk_ptr.p, nt + 1);
    LAUNCH_CHECK();
    HIPC(hipStreamSynchronize(s));
    return;
  }
  DBuf<int32_t> cnt(nblk), off(nblk + 1);
  k_blk_tile_counts<<<grid_for(nblk, 256), 256, 0, s>>>(P.blk.p, nblk, RT, S.row0.p, nt, cnt.p);
  LAUNCH_CHECK();
  exclusive_scan_i32(cnt.p, off.p, nblk, s);
  int32_t npairs = 0;
  HIPC(hipMemcpyAsync(&npairs, off.p + nblk, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  DBuf<int32_t> rank;
  if (col_order) {
    DBuf<uint64_t> ck(nblk);
    DBuf<int32_t> ids(nblk);
    k_blk_col_keys<<<grid_for(nblk, 256), 256, 0, s>>>(P.blk.p, nblk, ck.p, ids.p);
    LAUNCH_CHECK();
    sort_pairs_u64(ck, ids, nblk, 64, s);
    rank.alloc(nblk);
    k_rank_of<<<grid_for(nblk, 256), 256, 0, s>>>(ids.p, nblk, rank.p);
    LAUNCH_CHECK();
  }
  DBuf<uint64_t> keys(npairs);
  DBuf<int32_t> vals(npairs);
  k_blk_tile_pairs<<<grid_for(nblk, 256), 256, 0, s>>>(P.blk.p, off.p, rank.p, nblk, RT, S.row0.p,
                                                       nt, keys.p, vals.p);
  LAUNCH_CHECK();
  sort_pairs_u64(keys, vals, npairs, 32 + bits_for((uint64_t)nt), s);
  k_tile_ptr<<<grid_for(nt + 1, 256), 256, 0, s>>>(keys.p, npairs, nt, S.tile_blk_ptr.p);
  LAUNCH_CHECK();
  HIPC(hipStreamSynchronize(s));
  S.tile_blk = std::move(vals);
}

void build_bf16_split(sable_plan_s& P, hipStream_t s) {
  if (!P.nblk) return;
  if (!P.blk_mma_ptr.p) {
    std::vector<int32_t> blk;
    to_host(blk, P.blk.p, 4 * (size_t)P.nblk, s);
    std::vector<i64> mp(P.nblk);
    i64 acc = 0;
    for (int b = 0; b < P.nblk; ++b) {
      mp[b] = acc;
      const i64 h = blk[4 * b + 1] - blk[4 * b], w = blk[4 * b + 3] - blk[4 * b + 2];
      acc += h * ((w + 3) & ~(i64)3);
    }
    to_dev(P.blk_mma_ptr, mp, s);
    P.vbr_mma.alloc(acc);
  }
  k_split_mma<<<(unsigned)P.nblk, 256, 0, s>>>(P.blk.p, P.blk_val_ptr.p, P.blk_mma_ptr.p,
                                               P.vbr_val.p, P.vbr_mma.p);
  LAUNCH_CHECK();
}

#define SABLE_STREAM_LAUNCH(KERNEL)                                                            \
  static void launch_##KERNEL(const PlanView& v, int rpt, bool nt, const float* x, float* y,  \
                              hipStream_t s) {                                                 \
    const unsigned nb = (unsigned)(((v.ntiles + 7) / 8) * 8);                                  \
    if (nt) {                                                                                  \
      switch (rpt) {                                                                           \
        case 1: KERNEL<1, true><<<nb, kSpmvThreads, 0, s>>>(v, x, y); break;                   \
        case 2: KERNEL<2, true><<<nb, kSpmvThreads, 0, s>>>(v, x, y); break;                   \
        default: KERNEL<4, true><<<nb, kSpmvThreads, 0, s>>>(v, x, y); break;                  \
      }                                                                                        \
    } else {                                                                                   \
      switch (rpt) {                                                                           \
        case 1: KERNEL<1, false><<<nb, kSpmvThreads, 0, s>>>(v, x, y); break;                  \
        case 2: KERNEL<2, false><<<nb, kSpmvThreads, 0, s>>>(v, x, y); break;                  \
        default: KERNEL<4, false><<<nb, kSpmvThreads, 0, s>>>(v, x, y); break;                 \
      }                                                                                        \
    }                                                                                          \
    LAUNCH_CHECK();                                                                            \
  }
SABLE_STREAM_LAUNCH(k_spmv_stream)
SABLE_STREAM_LAUNCH(k_csr_stream)
#undef SABLE_STREAM_LAUNCH

// Workgroups per XCD of a persistent kernel: its resident workgroups per CU times the CUs of
// one XCD (queried once per kernel; the device's CU count / 8), at most the XCD's slots.
template <bool NT, bool PLAIN>
static int persist_nw(int ntiles) {
  static const int per_xcd = [] {
    const void* kern = PLAIN ? (const void*)k_csr_persist<NT> : (const void*)k_spmv_persist<NT>;
    int occ = 0, dev = 0, cus = 0;
    HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kSpmvThreads, 0));
    HIPC(hipGetDevice(&dev));
    HIPC(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return std::max(1, occ) * std::max(1, cus / 8);
  }();
  return std::max(1, std::min(per_xcd, (ntiles + 7) / 8));
}

template <bool NT, bool PLAIN>
static void launch_persist(const PlanView& v, const float* x, float* y, hipStream_t s) {
  const int nw = persist_nw<NT, PLAIN>(v.ntiles);
  if (PLAIN) k_csr_persist<NT><<<(unsigned)(8 * nw), kSpmvThreads, 0, s>>>(v, x, y, nw);
  else k_spmv_persist<NT><<<(unsigned)(8 * nw), kSpmvThreads, 0, s>>>(v, x, y, nw);
  LAUNCH_CHECK();
}

void launch_spmv(const sable_plan_s& P, const float* x, float* y, hipStream_t s) {
  const int var = P.prm.spmv_variant;
  if (var == 11) {
    launch_spmv_spec(P, x, y, s);
    return;
  }
  if (P.nseg == 0 && P.nblk == 0) {
    // the plan is its CSR part alone, which is the input in its own order: the plain CSR
    // kernels run it (the plain variant)
    launch_spmv_plain(P, x, y, s);
    return;
  }
  if (var >= 15) {  // persistent streamed tiles (with the far-column pass when enabled)
    const PlanView v = make_view(P, P.sched[0], false, true);
    if (v.far_prod) {
      k_far_gather<float><<<(unsigned)(8 * P.far.per_xcd), kFarThreads, 0, s>>>(
          P.far.chunk.p, P.far.per_xcd, P.ncols, P.far.far_col.p, P.far.far_val.p, x,
          P.far.far_prod.p);
      LAUNCH_CHECK();
    }
    if (var == 16) launch_persist<true, false>(v, x, y, s);
    else launch_persist<false, false>(v, x, y, s);
    return;
  }
  if (var >= 12) {
    const Schedule& S = P.sched[0];
    const PlanView v = make_view(P, S, false);
    const unsigned nb = (unsigned)(((v.ntiles + 7) / 8) * 8);
    k_spmv_binned<<<nb, kSpmvThreads, 0, s>>>(v, S.bin_rows.p, S.bin_off.p, var - 12, x, y);
    LAUNCH_CHECK();
    return;
  }
  if (var <= 2 || var >= 8) {
    const int k = var <= 2 ? var : var - 8;
    const PlanView v = make_view(P, P.sched[k], false, true);
    if (v.far_prod) {
      k_far_gather<float><<<(unsigned)(8 * P.far.per_xcd), kFarThreads, 0, s>>>(
          P.far.chunk.p, P.far.per_xcd, P.ncols, P.far.far_col.p, P.far.far_val.p, x,
          P.far.far_prod.p);
      LAUNCH_CHECK();
    }
    launch_k_spmv_stream(v, 1 << k, var >= 8, x, y, s);
    return;
  }
  // W lanes per CSR row: tiles of 256 / W rows, so every thread of a workgroup has a row
  const PlanView v = make_view(P, var == 3 ? P.sched[0] : P.sched_w[var - 4], false);
  const unsigned nb = (unsigned)v.ntiles;
  switch (var) {
    case 3: k_spmv_fused<1><<<nb, 256, 0, s>>>(v, x, y); break;
    case 4: k_spmv_fused<2><<<nb, 256, 0, s>>>(v, x, y); break;
    case 5: k_spmv_fused<4><<<nb, 256, 0, s>>>(v, x, y); break;
    case 6: k_spmv_fused<8><<<nb, 256, 0, s>>>(v, x, y); break;
    default: k_spmv_fused<16><<<nb, 256, 0, s>>>(v, x, y); break;
  }
  LAUNCH_CHECK();
}

void launch_spmv_plain(const sable_plan_s& P, const float* x, float* y, hipStream_t s) {
  const int var = P.prm.plain_variant;
  if (var >= 16) {
    const PlanView v = make_view(P, P.sched_plain[0], true);
    if (var == 17) launch_persist<true, true>(v, x, y, s);
    else launch_persist<false, true>(v, x, y, s);
    return;
  }
  if (var >= 13) {
    const Schedule& S = P.sched_plain[0];
    const PlanView v = make_view(P, S, true);
    const unsigned nb = (unsigned)(((v.ntiles + 7) / 8) * 8);
    k_csr_binned<<<nb, kSpmvThreads, 0, s>>>(v, S.bin_rows.p, S.bin_off.p, var - 13, x, y);
    LAUNCH_CHECK();
    return;
  }
  if (var <= 2 || var >= 10) {
    const int k = var <= 2 ? var : var - 10;
    launch_k_csr_stream(make_view(P, P.sched_plain[k], true), 1 << k, var >= 10, x, y, s);
    return;
  }
  const int W = 1 << (var - 3);
  const int rpb = 256 / W;
  const unsigned nb = (unsigned)((P.nrows + rpb - 1) / rpb);
  switch (W) {
    case 1: k_spmv_plain<1><<<nb, 256, 0, s>>>(P.a_ptr.p, P.a_col.p, P.a_val.p, P.nrows, x, y); break;
    case 2: k_spmv_plain<2><<<nb, 256, 0, s>>>(P.a_ptr.p, P.a_col.p, P.a_val.p, P.nrows, x, y); break;
    case 4: k_spmv_plain<4><<<nb, 256, 0, s>>>(P.a_ptr.p, P.a_col.p, P.a_val.p, P.nrows, x, y); break;
    case 8: k_spmv_plain<8><<<nb, 256, 0, s>>>(P.a_ptr.p, P.a_col.p, P.a_val.p, P.nrows, x, y); break;
    case 16: k_spmv_plain<16><<<nb, 256, 0, s>>>(P.a_ptr.p, P.a_col.p, P.a_val.p, P.nrows, x, y); break;
    case 32: k_spmv_plain<32><<<nb, 256, 0, s>>>(P.a_ptr.p, P.a_col.p, P.a_val.p, P.nrows, x, y); break;
    default: k_spmv_plain<64><<<nb, 256, 0, s>>>(P.a_ptr.p, P.a_col.p, P.a_val.p, P.nrows, x, y); break;
  }
  LAUNCH_CHECK();
}

int spmm_mfma_mode(const sable_plan_s& P, int mode) {
  // the panel tile also serves plans without blocks (bands and CSR only)
  if (mode == 4) return P.nblk == 0 || P.mm_panels.kptr.p ? 3 : 0;
  if (!P.vbr_mma.p || P.nblk == 0) return 0;
  return mode == 0 ? 1 : mode == 3 ? 2 : 0;
}

void build_bins(const sable_plan_s& P, Schedule& S, bool with_formats, hipStream_t s) {
  S.bin_rows.reset();
  S.bin_off.reset();
  if (S.ntiles == 0 || S.rows_per_tile > kSpmvThreads) return;
  std::vector<int32_t> ptr, row0;
  to_host(ptr, with_formats ? P.csr_ptr.p : P.a_ptr.p, (size_t)P.nrows + 1, s);
  if (S.row0.p) to_host(row0, S.row0.p, (size_t)S.ntiles + 1, s);
  std::vector<int32_t> rows(P.nrows), off((size_t)S.ntiles * (kNumBins + 1));
  int at = 0;
  for (int t = 0; t < S.ntiles; ++t) {
    const int a = S.row0.p ? row0[t] : t * S.rows_per_tile;
    const int b = S.row0.p ? row0[t + 1] : std::min(P.nrows, (t + 1) * S.rows_per_tile);
    int cnt[kNumBins] = {0};
    for (int r = a; r < b; ++r) cnt[csr_bin(ptr[r + 1] - ptr[r])]++;
    int* o = off.data() + (size_t)t * (kNumBins + 1);
    o[0] = at;
    for (int k = 0; k < kNumBins; ++k) o[k + 1] = o[k] + cnt[k];
    int fill[kNumBins];
    for (int k = 0; k < kNumBins; ++k) fill[k] = o[k];
    for (int r = a; r < b; ++r) rows[fill[csr_bin(ptr[r + 1] - ptr[r])]++] = r;
    at = o[kNumBins];
  }
  to_dev(S.bin_rows, rows, s);
  to_dev(S.bin_off, off, s);
  HIPC(hipStreamSynchronize(s));
}

void build_mm_panels(sable_plan_s& P, hipStream_t s) {
  MmPanels& M = P.mm_panels;
  M.kcol.reset();
  M.kptr.reset();
  M.bpos.reset();
  M.apack.reset();
  M.amask.reset();
  M.aptr.reset();
  M.nunits = 0;
  M.pan_tile.reset();
  M.pan_pos.reset();
  M.npanels = 0;
  const Schedule& S = P.sched_mm;
  if (!P.vbr_mma.p || P.nblk == 0 || S.ntiles == 0) return;
  std::vector<int32_t> blk, tptr, tblk;
  to_host(blk, P.blk.p, 4 * (size_t)P.nblk, s);
  to_host(tptr, S.tile_blk_ptr.p, (size_t)S.ntiles + 1, s);
  to_host(tblk, S.tile_blk.p, (size_t)tptr[S.ntiles], s);
  std::vector<int32_t> kcol, kptr(S.ntiles + 1), bpos(tblk.size());
  kptr[0] = 0;
  for (int t = 0; t < S.ntiles; ++t) {
    // the tile's blocks are listed by first column: one sweep gives the distinct columns
    const size_t base = kcol.size();
    int covered = INT32_MIN;  // every column below this is listed already
    for (int q = tptr[t]; q < tptr[t + 1]; ++q) {
      const int c0 = blk[4 * tblk[q] + 2], c1 = blk[4 * tblk[q] + 3];
      for (int c = std::max(c0, covered); c < c1; ++c) kcol.push_back(c);
      covered = std::max(covered, c1);
    }
    for (int q = tptr[t]; q < tptr[t + 1]; ++q) {
      const int c0 = blk[4 * tblk[q] + 2];
      bpos[q] = (int32_t)(std::lower_bound(kcol.begin() + base, kcol.end(), c0) - (kcol.begin() + base));
    }
    while ((kcol.size() - base) % kPanK) kcol.push_back(-1);
    if (kcol.size() > (size_t)INT32_MAX) SB_THROW(SABLE_ERR_TOO_LARGE, "panel list too long");
    kptr[t + 1] = (int32_t)kcol.size();
  }
  to_dev(M.kcol, kcol, s);
  to_dev(M.kptr, kptr, s);
  to_dev(M.bpos, bpos, s);
  std::vector<int32_t> ptile, ppos;
  for (int t = 0; t < S.ntiles; ++t)
    for (int k = kptr[t]; k < kptr[t + 1]; k += kPanK) {
      ptile.push_back(t);
      ppos.push_back(k - kptr[t]);
    }
  M.npanels = (i64)ptile.size();
  to_dev(M.pan_tile, ptile, s);
  to_dev(M.pan_pos, ppos, s);
  // occupancy masks first, then the unit offsets, then the units
  M.amask.alloc((size_t)M.npanels * 4);
  const PlanView v = make_view(P, P.sched_mm, false);
  for (i64 g0 = 0; g0 < M.npanels; g0 += (1 << 30)) {  // grid.x limit
    const unsigned nb = (unsigned)std::min<i64>(M.npanels - g0, 1 << 30);
    k_pack_panels<<<nb, 256, 0, s>>>(v, M.pan_tile.p + g0, M.pan_pos.p + g0, M.amask.p + 4 * g0,
                                     nullptr, nullptr, 0);
    LAUNCH_CHECK();
  }
  std::vector<uint64_t> mask;
  to_host(mask, M.amask.p, (size_t)M.npanels * 4, s);
  std::vector<i64> aptr((size_t)M.npanels + 1);
  aptr[0] = 0;
  for (i64 g = 0; g < M.npanels; ++g) {
    int c = 0;
    for (int i = 0; i < 4; ++i) c += __builtin_popcountll(mask[4 * g + i]);
    aptr[g + 1] = aptr[g] + c;
  }
  M.nunits = aptr[M.npanels];
  to_dev(M.aptr, aptr, s);
  M.apack.alloc((size_t)std::max<i64>(1, 2 * M.nunits));
  pack_mm_panels(P, s);
}

void pack_mm_panels(sable_plan_s& P, hipStream_t s) {
  MmPanels& M = P.mm_panels;
  if (!M.npanels || !P.vbr_mma.p) return;
  const PlanView v = make_view(P, P.sched_mm, false);
  for (i64 g0 = 0; g0 < M.npanels; g0 += (1 << 30)) {  // grid.x limit
    const unsigned nb = (unsigned)std::min<i64>(M.npanels - g0, 1 << 30);
    k_pack_panels<<<nb, 256, 0, s>>>(v, M.pan_tile.p + g0, M.pan_pos.p + g0, M.amask.p + 4 * g0,
                                     M.aptr.p + g0, M.apack.p, 1);
    LAUNCH_CHECK();
  }
  HIPC(hipStreamSynchronize(s));
}

void launch_spmm(const sable_plan_s& P, const float* X, float* Y, int n, hipStream_t s) {
  const int mode = P.prm.spmm_mode_for(n);
  const PlanView v = make_view(P, mode == 2 ? P.sched[0] : P.sched_mm, false);
  if (mode == 2) {
    const unsigned nb = (unsigned)((P.nrows + 3) / 4);
    k_spmm_fused_valu<<<nb, 256, 0, s>>>(v, X, Y, n);
  } else {
    const int ntile = (P.nrows + kMmRows - 1) / kMmRows;
    dim3 grid((unsigned)(((ntile + 7) / 8) * 8), (unsigned)((n + kMmCols - 1) / kMmCols));
    const int mfma = spmm_mfma_mode(P, mode);
    if (mfma == 3) k_spmm_panel<<<grid, kMmThreads, 0, s>>>(v, X, Y, n);
    else if (mfma) k_spmm_tile<<<grid, kMmThreads, 0, s>>>(v, X, Y, n, mfma);
    else k_spmm_tile_valu<<<grid, kMmThreads, 0, s>>>(v, X, Y, n);
  }
  LAUNCH_CHECK();
}

void launch_spmv_f64(const sable_plan_s& P, const double* x, double* y, hipStream_t s) {
  // the streamed variant's tile size (rows per thread) if one is selected, else 1
  const int var = P.prm.spmv_variant;
  const int k = var <= 2 ? var : (var >= 8 && var <= 10) ? var - 8 : 0;
  const PlanView v = make_view(P, P.sched[k], false, P.far.far_prod64.p != nullptr);
  if (v.far_prod64) {  // far-column products first, as in the fp32 path
    k_far_gather<double><<<(unsigned)(8 * P.far.per_xcd), kFarThreads, 0, s>>>(
        P.far.chunk.p, P.far.per_xcd, P.ncols, P.far.far_col.p, P.far.far_val64.p, x,
        P.far.far_prod64.p);
    LAUNCH_CHECK();
  }
  const unsigned nb = (unsigned)(((v.ntiles + 7) / 8) * 8);
  switch (k) {
    case 0: k_spmv_stream_f64<1><<<nb, kSpmvThreads, 0, s>>>(v, x, y); break;
    case 1: k_spmv_stream_f64<2><<<nb, kSpmvThreads, 0, s>>>(v, x, y); break;
    default: k_spmv_stream_f64<4><<<nb, kSpmvThreads, 0, s>>>(v, x, y); break;
  }
  LAUNCH_CHECK();
}

void launch_spmm_f64(const sable_plan_s& P, const double* X, double* Y, int n, hipStream_t s) {
  const PlanView v = make_view(P, P.sched_mm, false);
  const int ntile = (P.nrows + kMmRows - 1) / kMmRows;
  dim3 grid((unsigned)(((ntile + 7) / 8) * 8), (unsigned)((n + kMmCols - 1) / kMmCols));
  k_spmm_tile_f64<<<grid, kMmThreads, 0, s>>>(v, X, Y, n);
  LAUNCH_CHECK();
}

}  // namespace sable
