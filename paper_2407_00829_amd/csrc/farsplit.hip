// Far-column split of the CSR remainder for the streamed SpMV (built on the GPU at plan time).
//
// An entry (r, c) of the CSR part is far when |c - r| > kFarWindow. Far entries are sorted
// by (panel of c, CSR index), so each panel holds its entries in row order. The gather work
// list gives each workgroup one chunk of one panel, and puts panel p's chunks on XCD p mod 8
// (workgroups are dealt to the XCDs round-robin). Nothing here changes the partition:
// csr_ptr / csr_col / csr_val remain the CSR format of the plan.
#include <algorithm>

#include "exec.h"

namespace sable {

namespace {

__global__ void k_far_flags(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                            int nrows, int32_t* __restrict__ isfar) {
  for (i64 r = blockIdx.x * (i64)blockDim.x + threadIdx.x; r < nrows; r += (i64)gridDim.x * blockDim.x)
    for (int k = ptr[r]; k < ptr[r + 1]; ++k) {
      const i64 d = (i64)col[k] - r;
      isfar[k] = (d > kFarWindow || d < -kFarWindow) ? 1 : 0;
    }
}

// Far entry k at compacted position pos[k]: key (panel, k); near entries keep their column
// in the encoded copy.
__global__ void k_far_keys(const int32_t* __restrict__ col, const int32_t* __restrict__ isfar,
                           const int32_t* __restrict__ pos, i64 nnz, int panel_cols,
                           uint64_t* __restrict__ keys, int32_t* __restrict__ idx,
                           int32_t* __restrict__ ccol) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < nnz; k += (i64)gridDim.x * blockDim.x) {
    if (!isfar[k]) {
      ccol[k] = col[k];
      continue;
    }
    const i64 q = pos[k];
    keys[q] = ((uint64_t)(col[k] / panel_cols) << 32) | (uint64_t)(uint32_t)k;
    idx[q] = (int32_t)k;
  }
}

// Sorted position q of far entry k = idx[q]: copy the column within its panel and the value,
// encode -(1 + q).
__global__ void k_far_fill(const int32_t* __restrict__ idx, i64 nfar, const int32_t* __restrict__ col,
                           const float* __restrict__ val, int panel_cols,
                           uint16_t* __restrict__ fcol, float* __restrict__ fval,
                           int32_t* __restrict__ fsrc, int32_t* __restrict__ ccol) {
  for (i64 q = blockIdx.x * (i64)blockDim.x + threadIdx.x; q < nfar; q += (i64)gridDim.x * blockDim.x) {
    const int k = idx[q];
    fcol[q] = (uint16_t)(col[k] % panel_cols);
    fval[q] = val[k];
    fsrc[q] = k;
    ccol[k] = (int32_t)(-1 - q);
  }
}

// panel_ptr[p] = first sorted key with panel >= p, p in [0, npanel].
__global__ void k_panel_ptr(const uint64_t* __restrict__ keys, i64 n, int npanel,
                            int32_t* __restrict__ pp) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > npanel) return;
  const uint64_t key = (uint64_t)p << 32;
  i64 l = 0, h = n;
  while (l < h) { i64 m = (l + h) >> 1; if (keys[m] < key) l = m + 1; else h = m; }
  pp[p] = (int32_t)l;
}

template <class T>
__global__ void k_gather_vals(const T* __restrict__ src, const int32_t* __restrict__ idx, i64 n,
                              T* __restrict__ out) {
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    out[i] = src[idx[i]];
}

}  // namespace

void build_far_split(sable_plan_s& P, hipStream_t s) {
  FarSplit& F = P.far;
  F = FarSplit();
  const i64 nnz = P.csr_nnz;
  if (P.nrows == 0 || nnz < kFarMinEntries || P.ncols < kFarMinCols) return;
  const int panel_cols = kFarPanelCols;
  const int npanel = (int)(((i64)P.ncols + panel_cols - 1) / panel_cols);

  DBuf<int32_t> isfar(nnz), pos(nnz + 1);
  k_far_flags<<<grid_for(P.nrows, 256), 256, 0, s>>>(P.csr_ptr.p, P.csr_col.p, P.nrows, isfar.p);
  LAUNCH_CHECK();
  exclusive_scan_i32(isfar.p, pos.p, nnz, s);
  int32_t nfar = 0;
  HIPC(hipMemcpyAsync(&nfar, pos.p + nnz, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  if (nfar < kFarMinEntries) return;

  DBuf<uint64_t> keys(nfar);
  DBuf<int32_t> idx(nfar);
  F.ccol.alloc(nnz);
  k_far_keys<<<grid_for(nnz, 256), 256, 0, s>>>(P.csr_col.p, isfar.p, pos.p, nnz, panel_cols,
                                                 keys.p, idx.p, F.ccol.p);
  LAUNCH_CHECK();
  sort_pairs_u64(keys, idx, nfar, 32 + bits_for((uint64_t)npanel), s);
  F.far_col.alloc(nfar);
  F.far_val.alloc(nfar);
  F.far_src.alloc(nfar);
  F.far_prod.alloc(nfar);
  k_far_fill<<<grid_for(nfar, 256), 256, 0, s>>>(idx.p, nfar, P.csr_col.p, P.csr_val.p, panel_cols,
                                                  F.far_col.p, F.far_val.p, F.far_src.p, F.ccol.p);
  LAUNCH_CHECK();
  DBuf<int32_t> pp(npanel + 1);
  k_panel_ptr<<<grid_for(npanel + 1, 256), 256, 0, s>>>(keys.p, nfar, npanel, pp.p);
  LAUNCH_CHECK();
  // gather work list (begin, end, panel) per workgroup: panel p's chunks go to XCD p mod 8
  std::vector<int32_t> hp;
  to_host(hp, pp.p, npanel + 1, s);
  std::vector<std::vector<int32_t>> per(8);
  for (int p = 0; p < npanel; ++p)
    for (int b = hp[p]; b < hp[p + 1]; b += kFarChunk) {
      per[p & 7].push_back(b);
      per[p & 7].push_back(std::min(b + kFarChunk, hp[p + 1]));
      per[p & 7].push_back(p);
    }
  size_t mx = 0;
  for (auto& v : per) mx = std::max(mx, v.size() / 3);
  std::vector<int32_t> ch(24 * mx, -1);
  for (int x = 0; x < 8; ++x)
    for (size_t i = 0; i < per[x].size() / 3; ++i)
      for (int f = 0; f < 3; ++f) ch[3 * (x * mx + i) + f] = per[x][3 * i + f];
  to_dev(F.chunk, ch, s);
  F.npanel = npanel;
  F.panel_cols = panel_cols;
  F.per_xcd = (int)mx;
  F.nfar = nfar;
  HIPC(hipStreamSynchronize(s));
}

void refresh_far_values64(sable_plan_s& P, hipStream_t s) {
  FarSplit& F = P.far;
  if (!F.npanel) return;
  if (!F.far_val64.p) {
    F.far_val64.alloc(F.nfar);
    F.far_prod64.alloc(F.nfar);
  }
  k_gather_vals<double><<<grid_for(F.nfar, 256), 256, 0, s>>>(P.csr_val64.p, F.far_src.p, F.nfar,
                                                              F.far_val64.p);
  LAUNCH_CHECK();
}

void refresh_far_values(sable_plan_s& P, hipStream_t s) {
  FarSplit& F = P.far;
  if (!F.npanel) return;
  k_gather_vals<float><<<grid_for(F.nfar, 256), 256, 0, s>>>(P.csr_val.p, F.far_src.p, F.nfar, F.far_val.p);
  LAUNCH_CHECK();
}

}  // namespace sable
