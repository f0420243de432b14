// Learned planner: matrix features on the GPU, an MLP 140-128-128-15 (forward, backward,
// Adam) in hand-written kernels, native inference with an exhaustive timed search as the
// fallback and yardstick.
//
// Label space (15 classes): extractor list {CSR, VDIA+CSR, VBR+CSR, VDIA+VBR+CSR,
// VBR+VDIA+CSR} x delta {0.5, 0.7, 0.9} (bands and blocks share delta). The plan search of
// the paper is a user choice of extractor order (Sec. 4.3) and of delta (Sec. 4.1, Sec. 5);
// the planner predicts the fastest choice from structure features instead of timing all.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "plan.h"

namespace sable {

namespace {

// ---- features ---------------------------------------------------------------------------

__global__ void k_feat_keys(const int32_t* __restrict__ rows, const int32_t* __restrict__ col,
                            i64 nnz, int nrows, uint32_t* __restrict__ dkey,
                            int32_t* __restrict__ rowv, uint64_t* __restrict__ tkey, i64 ntc,
                            int32_t* __restrict__ dummy) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < nnz; k += (i64)gridDim.x * blockDim.x) {
    const int r = rows[k], c = col[k];
    dkey[k] = (uint32_t)((i64)c - r + nrows - 1);
    rowv[k] = r;
    tkey[k] = (uint64_t)(r / 16) * (uint64_t)ntc + (uint64_t)(c / 16);
    dummy[k] = 0;
  }
}

__device__ __forceinline__ int log_bin(i64 L) {  // 4 bins per octave, 64 bins
  int e = 63 - __clzll((unsigned long long)L);
  if (e >= 16) return 63;
  int b = 4 * e + (int)((L << 2) >> e) - 4;
  return b > 63 ? 63 : b;
}

// run starts along diagonals in the (d, row)-sorted order
__global__ void k_run_flags(const uint32_t* __restrict__ skey, const int32_t* __restrict__ srow,
                            i64 n, int32_t* __restrict__ flag) {
  for (i64 p = blockIdx.x * (i64)blockDim.x + threadIdx.x; p < n; p += (i64)gridDim.x * blockDim.x)
    flag[p] = (p == 0 || skey[p] != skey[p - 1] || srow[p] != srow[p - 1] + 1) ? 1 : 0;
}

// Block-private counters in LDS, merged into global memory with one atomic per nonzero
// counter per block (global atomics on a few shared addresses serialise).
template <int NB>
__device__ __forceinline__ void lds_zero(unsigned long long* h) {
  for (int i = threadIdx.x; i < NB; i += blockDim.x) h[i] = 0;
  __syncthreads();
}

template <int NB>
__device__ __forceinline__ void lds_merge_add(const unsigned long long* h, unsigned long long* g) {
  __syncthreads();
  for (int i = threadIdx.x; i < NB; i += blockDim.x)
    if (h[i]) atomicAdd(&g[i], h[i]);
}

// run r starts at start[r]: rid[p] (exclusive scan of the run-start flags) numbers the runs
__global__ void k_run_starts(const int32_t* __restrict__ flag, const int32_t* __restrict__ rid,
                             i64 n, int32_t* __restrict__ start) {
  for (i64 p = blockIdx.x * (i64)blockDim.x + threadIdx.x; p < n; p += (i64)gridDim.x * blockDim.x)
    if (flag[p]) start[rid[p]] = (int32_t)p;
}

// hist[log_bin(L)] += L over the run lengths L
__global__ void k_run_hist(const int32_t* __restrict__ start, i64 nruns, i64 n,
                           unsigned long long* __restrict__ hist) {
  __shared__ unsigned long long h[64];
  lds_zero<64>(h);
  for (i64 r = blockIdx.x * (i64)blockDim.x + threadIdx.x; r < nruns; r += (i64)gridDim.x * blockDim.x) {
    const i64 L = (r + 1 < nruns ? (i64)start[r + 1] : n) - start[r];
    atomicAdd(&h[log_bin(L)], (unsigned long long)L);
  }
  lds_merge_add<64>(h, hist);
}

__global__ void k_tile_hist(const uint64_t* __restrict__ uniq, const int32_t* __restrict__ cnt,
                            i64 nt, i64 ntc, int nrows, int ncols,
                            unsigned long long* __restrict__ hist,
                            unsigned long long* __restrict__ dense_nnz) {
  __shared__ unsigned long long h[65];  // 64 density bins, nnz in half-dense tiles
  lds_zero<65>(h);
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < nt; t += (i64)gridDim.x * blockDim.x) {
    const i64 I = (i64)(uniq[t] / (uint64_t)ntc), J = (i64)(uniq[t] % (uint64_t)ntc);
    const i64 hh = min((I + 1) * 16, (i64)nrows) - I * 16;
    const i64 w = min((J + 1) * 16, (i64)ncols) - J * 16;
    const i64 c = cnt[t];
    int b = (int)((64 * c) / (hh * w));
    if (b > 63) b = 63;
    atomicAdd(&h[b], (unsigned long long)c);
    if (2 * c >= hh * w) atomicAdd(&h[64], (unsigned long long)c);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 65; i += blockDim.x)
    if (h[i]) atomicAdd(i < 64 ? &hist[i] : dense_nnz, h[i]);
}

__global__ void k_diag_stats(const uint32_t* __restrict__ uniq, const int32_t* __restrict__ cnt,
                             i64 nd, int nrows, unsigned long long* __restrict__ out) {
  // out[0] = nnz on d = 0, out[1] = nnz with |d| <= 32, out[2] = max count
  __shared__ unsigned long long h[3];
  lds_zero<3>(h);
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < nd; t += (i64)gridDim.x * blockDim.x) {
    const i64 d = (i64)uniq[t] - (nrows - 1);
    if (d == 0) atomicAdd(&h[0], (unsigned long long)cnt[t]);
    if (d >= -32 && d <= 32) atomicAdd(&h[1], (unsigned long long)cnt[t]);
    atomicMax(&h[2], (unsigned long long)cnt[t]);
  }
  __syncthreads();
  if (threadIdx.x < 2 && h[threadIdx.x]) atomicAdd(&out[threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x == 2 && h[2]) atomicMax(&out[2], h[2]);
}

__global__ void k_row_stats(const int32_t* __restrict__ ptr, int nrows,
                            unsigned long long* __restrict__ out) {
  // out[0] = sum len^2, out[1] = max len, out[2] = empty rows
  __shared__ unsigned long long h[3];
  lds_zero<3>(h);
  for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < nrows; i += (i64)gridDim.x * blockDim.x) {
    const unsigned long long L = (unsigned long long)(ptr[i + 1] - ptr[i]);
    atomicAdd(&h[0], L * L);
    atomicMax(&h[1], L);
    if (L == 0) atomicAdd(&h[2], 1ull);
  }
  __syncthreads();
  if ((threadIdx.x == 0 || threadIdx.x == 2) && h[threadIdx.x]) atomicAdd(&out[threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x == 1 && h[1]) atomicMax(&out[1], h[1]);
}

}  // namespace

void compute_features(const sable_csr& A, hipStream_t s, float* out) {
  std::fill(out, out + SABLE_NFEAT, 0.f);
  const i64 nnz = A.nnz;
  const int n = A.nrows, m = A.ncols;
  std::vector<unsigned long long> rh(64, 0), th(64, 0), ds(3, 0), rs(3, 0), dn(1, 0);
  i64 ndiag = 0;
  if (nnz > 0) {
    Resid R;
    resid_from_input(R, A, s);
    DBuf<int32_t> rows;
    entry_rows(R, rows, s);
    const i64 ntc = (m + 15) / 16, ntr = (n + 15) / 16;
    DBuf<uint32_t> dkey(nnz);
    DBuf<int32_t> rowv(nnz), dummy(nnz);
    DBuf<uint64_t> tkey(nnz);
    k_feat_keys<<<grid_for(nnz, 256), 256, 0, s>>>(rows.p, R.col.p, nnz, n, dkey.p, rowv.p, tkey.p,
                                                   ntc, dummy.p);
    LAUNCH_CHECK();
    sort_pairs_u32(dkey, rowv, nnz, bits_for((uint64_t)n + m), s);
    // diagonal runs
    DBuf<int32_t> flag(nnz), rid(nnz + 1);
    k_run_flags<<<grid_for(nnz, 256), 256, 0, s>>>(dkey.p, rowv.p, nnz, flag.p);
    LAUNCH_CHECK();
    exclusive_scan_i32(flag.p, rid.p, nnz, s);
    int32_t nruns = 0;
    HIPC(hipMemcpyAsync(&nruns, rid.p + nnz, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    DBuf<int32_t> start(nruns);
    k_run_starts<<<grid_for(nnz, 256), 256, 0, s>>>(flag.p, rid.p, nnz, start.p);
    LAUNCH_CHECK();
    // hist: [0,64) run lengths, [64,128) tile densities, 128..130 diagonal stats,
    // 131..133 row stats, 134 nnz in half-dense tiles
    DBuf<unsigned long long> hist(135);
    HIPC(hipMemsetAsync(hist.p, 0, hist.bytes(), s));
    k_run_hist<<<grid_for(nruns, 256, 1024), 256, 0, s>>>(start.p, nruns, nnz, hist.p);
    LAUNCH_CHECK();
    // diagonal counts
    DBuf<uint32_t> du;
    DBuf<int32_t> dc;
    ndiag = rle_u32(dkey.p, nnz, du, dc, s);
    k_diag_stats<<<grid_for(ndiag, 256, 1024), 256, 0, s>>>(du.p, dc.p, ndiag, n, hist.p + 128);
    LAUNCH_CHECK();
    // tiles of 16 x 16
    sort_pairs_u64(tkey, dummy, nnz, bits_for((uint64_t)(ntr * ntc)), s);
    DBuf<uint64_t> tu;
    DBuf<int32_t> tc;
    const i64 nt = rle_u64(tkey.p, nnz, tu, tc, s);
    k_tile_hist<<<grid_for(nt, 256, 1024), 256, 0, s>>>(tu.p, tc.p, nt, ntc, n, m, hist.p + 64,
                                                  hist.p + 134);
    LAUNCH_CHECK();
    if (n) k_row_stats<<<grid_for(n, 256, 1024), 256, 0, s>>>(R.ptr.p, n, hist.p + 131);
    LAUNCH_CHECK();
    std::vector<unsigned long long> h;
    to_host(h, hist.p, hist.n, s);
    for (int b = 0; b < 64; ++b) { rh[b] = h[b]; th[b] = h[64 + b]; }
    ds = {h[128], h[129], h[130]};
    rs = {h[131], h[132], h[133]};
    dn[0] = h[134];
  } else if (n) {
    rs[2] = (unsigned long long)n;
  }
  const double dnnz = (double)std::max<i64>(nnz, 1);
  for (int b = 0; b < 64; ++b) {
    out[b] = (float)((double)rh[b] / dnnz);
    out[64 + b] = (float)((double)th[b] / dnnz);
  }
  const double dn_rows = (double)std::max(n, 1);
  const double mean = (double)nnz / dn_rows;
  const double var = std::max(0.0, (double)rs[0] / dn_rows - mean * mean);
  out[128] = (float)std::log1p(mean);
  out[129] = (float)std::log1p(std::sqrt(var));
  out[130] = (float)std::log1p((double)rs[1]);
  out[131] = (float)std::log((double)std::max(n, 1));
  out[132] = (float)std::log((double)std::max(m, 1));
  out[133] = (float)std::log((double)std::max<i64>(nnz, 1));
  out[134] = (float)((double)ds[0] / dnnz);
  out[135] = (float)((double)ds[1] / dnnz);
  out[136] = (float)((double)ds[2] / dn_rows);
  out[137] = (float)((double)ndiag / (double)std::max<i64>((i64)n + m - 1, 1));
  out[138] = (float)((double)dn[0] / dnnz);
  out[139] = (float)((double)rs[2] / dn_rows);
}

// ---- MLP kernels ----------------------------------------------------------------------------

namespace {

constexpr int kIn = SABLE_NFEAT, kH = 128, kOut = SABLE_NCLASS;
constexpr i64 oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH,
              oW3 = ob2 + kH, ob3 = oW3 + kOut * kH, kNP = ob3 + kOut;
static_assert(kNP == SABLE_MLP_NPARAM, "parameter layout");

// C[i][j] = sum_k A[i*sai + k*sak] * B[k*sbk + j*sbj] (+ bias[j]); optional ReLU.
// One thread per output element, k ascending: deterministic.
__global__ void k_gemm(const float* __restrict__ A, i64 sai, i64 sak, const float* __restrict__ B,
                       i64 sbk, i64 sbj, const float* __restrict__ bias, float* __restrict__ C,
                       int M, int N, int K, int relu) {
  const i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  if (idx >= (i64)M * N) return;
  const int i = (int)(idx / N), j = (int)(idx % N);
  float acc = 0.f;
  for (int k = 0; k < K; ++k) acc += A[i * sai + k * sak] * B[k * sbk + j * sbj];
  if (bias) acc += bias[j];
  if (relu && acc < 0.f) acc = 0.f;
  C[idx] = acc;
}

// softmax cross-entropy: G = (softmax(Z) - onehot) / B, loss[i] = -log softmax(Z)[label]
__global__ void k_softmax_ce(const float* __restrict__ Z, const int32_t* __restrict__ lab, int B,
                             int C, float* __restrict__ G, float* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const float* z = Z + (i64)i * C;
  float mx = z[0];
  for (int c = 1; c < C; ++c) mx = fmaxf(mx, z[c]);
  float se = 0.f;
  for (int c = 0; c < C; ++c) se += expf(z[c] - mx);
  const float lse = mx + logf(se);
  const int y = lab[i];
  for (int c = 0; c < C; ++c) G[(i64)i * C + c] = (expf(z[c] - lse) - (c == y ? 1.f : 0.f)) / (float)B;
  loss[i] = lse - z[y];
}

// G = dH * (Z > 0)
__global__ void k_relu_grad(const float* __restrict__ dH, const float* __restrict__ H, i64 n,
                            float* __restrict__ G) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x)
    G[k] = H[k] > 0.f ? dH[k] : 0.f;
}

// db[j] = sum_i G[i][j] (i ascending)
__global__ void k_colsum(const float* __restrict__ G, int B, int N, float* __restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
  for (int i = 0; i < B; ++i) s += G[(i64)i * N + j];
  db[j] = s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, i64 n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x) {
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / c1, vh = vk / c2;
    p[k] -= lr * mh / (sqrtf(vh) + eps);
  }
}

void gemm(const float* A, i64 sai, i64 sak, const float* B, i64 sbk, i64 sbj, const float* bias,
          float* C, int M, int N, int K, int relu, hipStream_t s) {
  const i64 tot = (i64)M * N;
  if (tot <= 0) return;
  k_gemm<<<nblocks(tot, 256), 256, 0, s>>>(A, sai, sak, B, sbk, sbj, bias, C, M, N, K, relu);
  LAUNCH_CHECK();
}

struct Acts {
  DBuf<float> H1, H2, Z3;
};

void forward(const float* P, const float* X, int B, Acts& a, hipStream_t s) {
  a.H1.alloc((i64)B * kH);
  a.H2.alloc((i64)B * kH);
  a.Z3.alloc((i64)B * kOut);
  // H1 = relu(X W1^T + b1): A = X (B x 140), B-operand element (k, j) = W1[j][k]
  gemm(X, kIn, 1, P + oW1, 1, kIn, P + ob1, a.H1.p, B, kH, kIn, 1, s);
  gemm(a.H1.p, kH, 1, P + oW2, 1, kH, P + ob2, a.H2.p, B, kH, kH, 1, s);
  gemm(a.H2.p, kH, 1, P + oW3, 1, kH, P + ob3, a.Z3.p, B, kOut, kH, 0, s);
}

}  // namespace

void mlp_forward(const float* params, const float* feats, int B, float* logits, hipStream_t s) {
  Acts a;
  forward(params, feats, B, a, s);
  HIPC(hipMemcpyAsync(logits, a.Z3.p, (size_t)B * kOut * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIPC(hipStreamSynchronize(s));
}

float mlp_train_step(float* P, float* G, float* m, float* v, const float* X, const int32_t* lab,
                     int B, float lr, float b1, float b2, float eps, int t, hipStream_t s) {
  Acts a;
  forward(P, X, B, a, s);
  DBuf<float> G3((i64)B * kOut), loss(B), dH2((i64)B * kH), G2((i64)B * kH), dH1((i64)B * kH),
      G1((i64)B * kH);
  k_softmax_ce<<<nblocks(B, 128), 128, 0, s>>>(a.Z3.p, lab, B, kOut, G3.p, loss.p);
  LAUNCH_CHECK();
  // layer 3: dW3[j][k] = sum_i G3[i][j] H2[i][k]; db3 = colsum(G3); dH2 = G3 W3
  gemm(G3.p, 1, kOut, a.H2.p, kH, 1, nullptr, G + oW3, kOut, kH, B, 0, s);
  k_colsum<<<1, 128, 0, s>>>(G3.p, B, kOut, G + ob3);
  LAUNCH_CHECK();
  gemm(G3.p, kOut, 1, P + oW3, kH, 1, nullptr, dH2.p, B, kH, kOut, 0, s);
  k_relu_grad<<<grid_for((i64)B * kH, 256), 256, 0, s>>>(dH2.p, a.H2.p, (i64)B * kH, G2.p);
  LAUNCH_CHECK();
  // layer 2
  gemm(G2.p, 1, kH, a.H1.p, kH, 1, nullptr, G + oW2, kH, kH, B, 0, s);
  k_colsum<<<1, 128, 0, s>>>(G2.p, B, kH, G + ob2);
  LAUNCH_CHECK();
  gemm(G2.p, kH, 1, P + oW2, kH, 1, nullptr, dH1.p, B, kH, kH, 0, s);
  k_relu_grad<<<grid_for((i64)B * kH, 256), 256, 0, s>>>(dH1.p, a.H1.p, (i64)B * kH, G1.p);
  LAUNCH_CHECK();
  // layer 1
  gemm(G1.p, 1, kH, X, kIn, 1, nullptr, G + oW1, kH, kIn, B, 0, s);
  k_colsum<<<1, 128, 0, s>>>(G1.p, B, kH, G + ob1);
  LAUNCH_CHECK();
  if (t > 0) {
    const float c1 = 1.f - std::pow(b1, (float)t), c2 = 1.f - std::pow(b2, (float)t);
    k_adam<<<grid_for(kNP, 256), 256, 0, s>>>(P, G, m, v, kNP, lr, b1, b2, eps, c1, c2);
    LAUNCH_CHECK();
  }
  std::vector<float> hl;
  to_host(hl, loss.p, B, s);
  double sum = 0.0;
  for (float x : hl) sum += x;
  return (float)(sum / std::max(B, 1));
}

void class_plan(int c, sable_extractor* list, int32_t* nlist, sable_thresholds* th) {
  static const int lists[5][3] = {{SABLE_X_CSR, 0, 0},
                                  {SABLE_X_VDIA, SABLE_X_CSR, 0},
                                  {SABLE_X_VBR, SABLE_X_CSR, 0},
                                  {SABLE_X_VDIA, SABLE_X_VBR, SABLE_X_CSR},
                                  {SABLE_X_VBR, SABLE_X_VDIA, SABLE_X_CSR}};
  static const int len[5] = {1, 2, 2, 3, 3};
  static const int deltas[3] = {500, 700, 900};
  const int L = c / 3, d = deltas[c % 3];
  *nlist = len[L];
  for (int e = 0; e < len[L]; ++e) {
    list[e].kind = lists[L][e];
    list[e].vbr_mode = SABLE_VBR_TILED;
  }
  sable_thresholds_default(th);
  th->delta_band_pm = d;
  th->delta_block_pm = d;
}

namespace {

// Time of one fused SpMV: three rounds of `reps` back-to-back launches between two events;
// the median of the three per-launch averages (per-launch events are too coarse for launches
// of a few microseconds).
float median_launch_ms(const sable_plan_s& P, const float* x, float* y, int reps, hipStream_t s,
                       bool plain = false) {
  hipEvent_t ev[6];
  for (auto& e : ev) HIPC(hipEventCreate(&e));
  auto launch = [&] {
    if (plain) launch_spmv_plain(P, x, y, s);
    else launch_spmv(P, x, y, s);
  };
  launch();  // warm-up
  for (int r = 0; r < 3; ++r) {
    HIPC(hipEventRecord(ev[2 * r], s));
    for (int k = 0; k < reps; ++k) launch();
    HIPC(hipEventRecord(ev[2 * r + 1], s));
  }
  HIPC(hipStreamSynchronize(s));
  float t[3];
  for (int r = 0; r < 3; ++r) {
    HIPC(hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]));
    t[r] /= reps;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  std::sort(t, t + 3);
  return t[1];
}

}  // namespace

// Plan A with every class; autotune each plan's SpMV kernels, time the chosen one; keep the
// fastest. CSR-only classes share one plan (their time is recorded for all three, and ties
// go to the lowest class index). ref (may be null) receives, timed the same way, the plain
// CSR baseline (the CSR-only plan's tuned plain kernel) and the paper's default list
// [VDIA, VBR, CSR] at delta 0.75 / 0.5 (tuned).
void plan_exhaustive(const sable_csr& A, const float* x, float* y, int reps, hipStream_t s,
                     sable_plan_t* out, int32_t* best_class, float* times, float* ref) {
  float best = 1e30f;
  int bc = -1;
  sable_plan_t bp = nullptr;
  if (ref) {  // the default plan, tuned and timed as the classes below
    sable_extractor list[3] = {{SABLE_X_VDIA, SABLE_VBR_TILED}, {SABLE_X_VBR, SABLE_VBR_TILED},
                               {SABLE_X_CSR, 0}};
    sable_thresholds th;
    sable_thresholds_default(&th);
    sable_plan_t p = nullptr;
    sable_status st = sable_plan(&A, list, 3, &th, s, &p);
    if (st != SABLE_OK) throw Err{st};
    try {
      if (p->nrows) autotune(*p, 0, 1, x, y, s);
      ref[1] = p->nrows ? median_launch_ms(*p, x, y, reps, s) : 0.f;
    } catch (...) {
      sable_plan_destroy(p);
      throw;
    }
    sable_plan_destroy(p);
  }
  // classes whose extraction yields the same partition run the same kernels: they are timed
  // once and share that time, so the fastest-class label is not decided by timing noise
  // between identical plans
  uint64_t seen_hash[SABLE_NCLASS];
  float seen_t[SABLE_NCLASS];
  int nseen = 0;
  for (int c = 0; c < SABLE_NCLASS; ++c) {
    float t;
    if (c < 3 && c > 0) {
      t = times[0];
    } else {
      sable_extractor list[3];
      int32_t nl = 0;
      sable_thresholds th;
      class_plan(c, list, &nl, &th);
      sable_plan_t p = nullptr;
      sable_status st = sable_plan(&A, list, nl, &th, s, &p);
      if (st != SABLE_OK) {
        if (bp) sable_plan_destroy(bp);
        throw Err{st};
      }
      int dup = -1;
      for (int k = 0; k < nseen; ++k)
        if (seen_hash[k] == p->partition_hash) dup = k;
      if (dup >= 0) {
        sable_plan_destroy(p);
        times[c] = seen_t[dup];
        continue;
      }
      try {
        if (p->nrows) autotune(*p, 0, 1, x, y, s);
        t = p->nrows ? median_launch_ms(*p, x, y, reps, s) : 0.f;
        if (c == 0 && ref) ref[0] = p->nrows ? median_launch_ms(*p, x, y, reps, s, true) : 0.f;
        seen_hash[nseen] = p->partition_hash;
        seen_t[nseen++] = t;
      } catch (...) {
        sable_plan_destroy(p);
        if (bp) sable_plan_destroy(bp);
        throw;
      }
      if (t < best) {
        if (bp) sable_plan_destroy(bp);
        bp = p;
        best = t;
        bc = c;
      } else {
        sable_plan_destroy(p);
      }
    }
    times[c] = t;
  }
  *out = bp;
  *best_class = bc;
}

}  // namespace sable

using namespace sable;

namespace {
template <class F>
sable_status guard2(F&& f) {
  clear_error();
  try {
    f();
    return SABLE_OK;
  } catch (const Err& e) {
    return e.st;
  } catch (...) {
    set_error("internal error");
    return SABLE_ERR_INTERNAL;
  }
}
}  // namespace

extern "C" {

sable_status sable_features(const sable_csr* A, void* stream, float* out) {
  return guard2([&] {
    if (!A || !out || A->nrows < 0 || A->ncols < 0 || A->nnz < 0 || !A->indptr ||
        (A->nnz && (!A->indices || !A->values)))
      SB_THROW(SABLE_ERR_INVALID_ARG, "bad argument");
    if (A->nnz >= (i64)INT32_MAX) SB_THROW(SABLE_ERR_TOO_LARGE, "nnz >= 2^31");
    hipStream_t s = (hipStream_t)stream;
    if (!validate_csr_device(*A, s)) SB_THROW(SABLE_ERR_INVALID_CSR, "input is not canonical CSR");
    compute_features(*A, s, out);
  });
}

sable_status sable_plan_exhaustive(const sable_csr* A, const float* x, float* y, int32_t reps,
                                   void* stream, sable_plan_t* out, int32_t* best_class,
                                   float* times_ms, float* ref_ms) {
  if (out) *out = nullptr;
  return guard2([&] {
    if (!A || !out || !best_class || reps < 1 || (!x && A->ncols) || (!y && A->nrows))
      SB_THROW(SABLE_ERR_INVALID_ARG, "bad argument");
    float t[SABLE_NCLASS];
    plan_exhaustive(*A, x, y, reps, (hipStream_t)stream, out, best_class, t, ref_ms);
    if (times_ms) std::copy(t, t + SABLE_NCLASS, times_ms);
  });
}

sable_status sable_plan_auto(const sable_csr* A, const float* params, const float* feat_mean,
                             const float* feat_std, float tau_conf, const float* x, float* y,
                             void* stream, sable_plan_t* out, int32_t* chosen_class,
                             float* confidence, int32_t* fell_back) {
  if (out) *out = nullptr;
  return guard2([&] {
    if (!A || !params || !feat_mean || !feat_std || !out || !chosen_class || !confidence ||
        !fell_back)
      SB_THROW(SABLE_ERR_INVALID_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    if (!validate_csr_device(*A, s)) SB_THROW(SABLE_ERR_INVALID_CSR, "input is not canonical CSR");
    float f[SABLE_NFEAT];
    compute_features(*A, s, f);
    for (int k = 0; k < SABLE_NFEAT; ++k)
      f[k] = (f[k] - feat_mean[k]) / (feat_std[k] > 0.f ? feat_std[k] : 1.f);
    DBuf<float> df(SABLE_NFEAT), dl(SABLE_NCLASS);
    HIPC(hipMemcpyAsync(df.p, f, sizeof(f), hipMemcpyHostToDevice, s));
    mlp_forward(params, df.p, 1, dl.p, s);
    float z[SABLE_NCLASS];
    HIPC(hipMemcpyAsync(z, dl.p, sizeof(z), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    int c = 0;
    for (int k = 1; k < SABLE_NCLASS; ++k) if (z[k] > z[c]) c = k;
    double se = 0.0;
    for (int k = 0; k < SABLE_NCLASS; ++k) se += std::exp((double)z[k] - z[c]);
    *confidence = (float)(1.0 / se);
    if (*confidence >= tau_conf) {
      sable_extractor list[3];
      int32_t nl = 0;
      sable_thresholds th;
      class_plan(c, list, &nl, &th);
      sable_status st = sable_plan(A, list, nl, &th, stream, out);
      if (st != SABLE_OK) throw Err{st};
      *chosen_class = c;
      *fell_back = 0;
      return;
    }
    if ((!x && A->ncols) || (!y && A->nrows)) SB_THROW(SABLE_ERR_INVALID_ARG, "fallback needs x and y");
    float t[SABLE_NCLASS];
    plan_exhaustive(*A, x, y, 5, s, out, chosen_class, t, nullptr);
    *fell_back = 1;
  });
}

sable_status sable_class_plan(int32_t c, sable_extractor* list, int32_t* nlist,
                              sable_thresholds* th) {
  return guard2([&] {
    if (!list || !nlist || !th || c < 0 || c >= SABLE_NCLASS) SB_THROW(SABLE_ERR_INVALID_ARG, "bad argument");
    class_plan(c, list, nlist, th);
  });
}

sable_status sable_mlp_forward(const float* params, const float* feats, int32_t batch,
                               float* logits, void* stream) {
  return guard2([&] {
    if (!params || !feats || !logits || batch < 1) SB_THROW(SABLE_ERR_INVALID_ARG, "bad argument");
    mlp_forward(params, feats, batch, logits, (hipStream_t)stream);
  });
}

sable_status sable_mlp_train_step(float* params, float* grads, float* m, float* v,
                                  const float* feats, const int32_t* labels, int32_t batch,
                                  float lr, float beta1, float beta2, float eps, int32_t t,
                                  void* stream, float* loss) {
  return guard2([&] {
    if (!params || !grads || !feats || !labels || !loss || batch < 1 || t < 0 ||
        (t > 0 && (!m || !v)))
      SB_THROW(SABLE_ERR_INVALID_ARG, "bad argument");
    *loss = mlp_train_step(params, grads, m, v, feats, labels, batch, lr, beta1, beta2, eps, t,
                           (hipStream_t)stream);
  });
}

}  // extern "C"
