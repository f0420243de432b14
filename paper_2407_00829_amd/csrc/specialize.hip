// Per-matrix specialization (the paper's code-generation idea, Sec. 3.3 - 3.4, Fig. 1, carried
// to the GPU with hipRTC): for a small plan, emit HIP source for its SpMV in which every band
// segment's rows, diagonal offsets and value offset, and every block's rectangle and value
// offset, are literal constants. Work is dispatched per 256-row tile (one workgroup): a
// switch on the tile lists only the segments and blocks overlapping it, so each thread runs
// straight-line code for its row; the tile's CSR entries stream through LDS in coalesced
// passes (first pass issued before the band and block work). The source is compiled at run
// time for the device's architecture and kept in the plan.
//
// Per row the sum is (band diagonals ascending, then blocks in block order with columns
// ascending) + CSR entries in index order: fixed, so results are bitwise reproducible.
#include <hip/hiprtc.h>

#include <algorithm>
#include <chrono>
#include <sstream>
#include <string>

#include "exec.h"

namespace sable {

namespace {

constexpr int kSpecRows = 256;      // rows per workgroup (one thread per row)
constexpr int kSpecMaxTiles = 4096;
constexpr i64 kSpecMaxItems = 16384;  // (tile, segment or block) pairs in the source
constexpr int kSpecMaxDiags = 128;

std::string spec_source(const sable_plan_s& P, const std::vector<int32_t>& srs,
                        const std::vector<int32_t>& snr, const std::vector<int32_t>& snd,
                        const std::vector<i64>& svp, const std::vector<int32_t>& sip,
                        const std::vector<int32_t>& idiag, const std::vector<int32_t>& blk,
                        const std::vector<i64>& bvp, int ntiles) {
  std::ostringstream o;
  o << "extern \"C\" __global__ __launch_bounds__(" << kSpecRows << ") void sable_spec_spmv(\n"
       "    const float* __restrict__ vdia, const float* __restrict__ vbr,\n"
       "    const int* __restrict__ cptr, const int* __restrict__ ccol,\n"
       "    const float* __restrict__ cval, const float* __restrict__ x, float* __restrict__ y) {\n"
       "  __shared__ float prod[" << 8 * kSpecRows << "];\n"
       "  const int t = threadIdx.x;\n"
       "  const int r0 = blockIdx.x * " << kSpecRows << ";\n"
       "  const int rend = min(r0 + " << kSpecRows << ", " << P.nrows << ");\n"
       "  const int r = r0 + t;\n"
       "  const bool act = r < rend;\n"
       "  // CSR entries of the tile: first pass issued before the bands and blocks\n"
       "  const int eb = cptr[r0], ee = cptr[rend];\n"
       "  const int kb = act ? cptr[r] : 0, ke = act ? cptr[r + 1] : 0;\n"
       "  int jj[8]; float aa[8], vv[8];\n"
       "  if (eb < ee) {\n"
       "#pragma unroll\n"
       "    for (int u = 0; u < 8; ++u) { const int k = min(eb + t + " << kSpecRows << " * u, ee - 1); jj[u] = ccol[k]; aa[u] = cval[k]; }\n"
       "#pragma unroll\n"
       "    for (int u = 0; u < 8; ++u) vv[u] = x[jj[u]];\n"
       "  }\n"
       "  float acc = 0.f;\n"
       "  if (act) switch (blockIdx.x) {\n";
  size_t s = 0, b = 0;  // segments and blocks are sorted by first row
  for (int t = 0; t < ntiles; ++t) {
    const i64 a = (i64)t * kSpecRows, e = std::min<i64>(P.nrows, a + kSpecRows);
    std::ostringstream body;
    while (s < srs.size() && (i64)srs[s] + snr[s] <= a) ++s;
    for (size_t q = s; q < srs.size() && srs[q] < e; ++q) {
      body << "    if (r >= " << srs[q] << " && r < " << (i64)srs[q] + snr[q] << ") {\n"
           << "      const float* v = vdia + " << svp[q] << "ll + (r - " << srs[q] << ");\n";
      for (int d = 0; d < snd[q]; ++d) {
        const i64 off = idiag[sip[q] + d];
        // the bound check is emitted only where the diagonal can leave the matrix
        const bool check = (i64)srs[q] + off < 0 || (i64)srs[q] + snr[q] - 1 + off >= P.ncols;
        if (check)
          body << "      if ((unsigned)(r + " << off << ") < " << P.ncols << "u) ";
        else
          body << "      ";
        body << "acc += v[" << (i64)d * snr[q] << "ll] * x[r + " << off << "];\n";
      }
      body << "    }\n";
    }
    while (b < bvp.size() && blk[4 * b + 1] <= a) ++b;
    for (size_t q = b; q < bvp.size() && blk[4 * q] < e; ++q) {
      const int r0 = blk[4 * q], r1 = blk[4 * q + 1], c0 = blk[4 * q + 2], c1 = blk[4 * q + 3];
      if (r1 <= a) continue;
      body << "    if (r >= " << r0 << " && r < " << r1 << ") {\n"
           << "      const float* v = vbr + " << bvp[q] << "ll + (r - " << r0 << ");\n"
           << "#pragma unroll 8\n"
           << "      for (int k = 0; k < " << (c1 - c0) << "; ++k) acc += v[k * " << (r1 - r0)
           << "] * x[" << c0 << " + k];\n"
           << "    }\n";
    }
    const std::string bs = body.str();
    if (!bs.empty()) o << "  case " << t << ": {\n" << bs << "    break;\n  }\n";
  }
  o << "  default: break;\n  }\n"
       "  // CSR passes of " << 8 * kSpecRows << " entries: products in LDS, each row adds its own in index order\n"
       "  float cs = 0.f;\n"
       "  for (int e0 = eb; e0 < ee; e0 += " << 8 * kSpecRows << ") {\n"
       "    if (e0 != eb) {\n"
       "#pragma unroll\n"
       "      for (int u = 0; u < 8; ++u) { const int k = min(e0 + t + " << kSpecRows << " * u, ee - 1); jj[u] = ccol[k]; aa[u] = cval[k]; }\n"
       "#pragma unroll\n"
       "      for (int u = 0; u < 8; ++u) vv[u] = x[jj[u]];\n"
       "    }\n"
       "    __syncthreads();\n"
       "#pragma unroll\n"
       "    for (int u = 0; u < 8; ++u) prod[t + " << kSpecRows << " * u] = e0 + t + " << kSpecRows << " * u < ee ? aa[u] * vv[u] : 0.f;\n"
       "    __syncthreads();\n"
       "    const int a = max(kb, e0), b = min(ke, e0 + " << 8 * kSpecRows << ");\n"
       "    int k = a;\n"
       "    for (; k + 8 <= b; k += 8) {\n"
       "      float v[8];\n"
       "#pragma unroll\n"
       "      for (int i = 0; i < 8; ++i) v[i] = prod[k - e0 + i];\n"
       "#pragma unroll\n"
       "      for (int i = 0; i < 8; ++i) cs += v[i];\n"
       "    }\n"
       "    for (; k < b; ++k) cs += prod[k - e0];\n"
       "  }\n"
       "  if (act) y[r] = acc + cs;\n"
       "}\n";
  return o.str();
}

}  // namespace

}  // namespace sable

sable_plan_s::~sable_plan_s() {
  if (spec_module) (void)hipModuleUnload((hipModule_t)spec_module);
}

using namespace sable;

namespace sable {

void launch_spmv_spec(const sable_plan_s& P, const float* x, float* y, hipStream_t s) {
  if (!P.spec_func) SB_THROW(SABLE_ERR_INVALID_ARG, "the plan has no specialized kernel");
  const float* vdia = P.vdia_val.p;
  const float* vbr = P.vbr_val.p;
  const int* cptr = P.csr_ptr.p;
  const int* ccol = P.csr_col.p;
  const float* cval = P.csr_val.p;
  void* args[] = {&vdia, &vbr, &cptr, &ccol, &cval, &x, &y};
  const unsigned nb = (unsigned)((P.nrows + kSpecRows - 1) / kSpecRows);
  HIPC(hipModuleLaunchKernel((hipFunction_t)P.spec_func, nb, 1, 1, kSpecRows, 1, 1, 0, s, args,
                             nullptr));
}

}  // namespace sable

extern "C" sable_status sable_plan_specialize(sable_plan_t p, void* stream) {
  clear_error();
  hiprtcProgram prog = nullptr;
  try {
    if (!p) SB_THROW(SABLE_ERR_INVALID_ARG, "NULL plan");
    if (p->spec_func) return SABLE_OK;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    const int ntiles = (p->nrows + kSpecRows - 1) / kSpecRows;
    if (ntiles > kSpecMaxTiles) SB_THROW(SABLE_ERR_TOO_LARGE, "%d row tiles (at most %d)", ntiles, kSpecMaxTiles);
    std::vector<int32_t> srs, snr, snd, sip, idiag, blk;
    std::vector<i64> svp, bvp;
    to_host(srs, p->seg_row_start.p, p->nseg, s);
    to_host(snr, p->seg_nrows.p, p->nseg, s);
    to_host(snd, p->seg_ndiags.p, p->nseg, s);
    to_host(svp, p->seg_val_ptr.p, p->nseg, s);
    to_host(sip, p->seg_idiag_ptr.p, p->nseg, s);
    to_host(idiag, p->idiag.p, p->nidiag, s);
    to_host(blk, p->blk.p, 4 * (size_t)p->nblk, s);
    to_host(bvp, p->blk_val_ptr.p, p->nblk, s);
    i64 items = 0;  // (tile, item) pairs the source will hold
    for (int q = 0; q < p->nseg; ++q) {
      if (snd[q] > kSpecMaxDiags) SB_THROW(SABLE_ERR_TOO_LARGE, "segment with %d diagonals", snd[q]);
      items += (i64)(srs[q] + snr[q] - 1) / kSpecRows - srs[q] / kSpecRows + 1;
    }
    for (int q = 0; q < p->nblk; ++q)
      items += (i64)(blk[4 * q + 1] - 1) / kSpecRows - blk[4 * q] / kSpecRows + 1;
    if (items > kSpecMaxItems) SB_THROW(SABLE_ERR_TOO_LARGE, "%lld tile items (at most %lld)", (long long)items, (long long)kSpecMaxItems);
    const std::string src = spec_source(*p, srs, snr, snd, svp, sip, idiag, blk, bvp, ntiles);

    int dev = 0;
    HIPC(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPC(hipGetDeviceProperties(&prop, dev));
    const std::string arch = std::string("--offload-arch=") + prop.gcnArchName;
    const char* opts[] = {arch.c_str(), "-O3", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    if (hiprtcCreateProgram(&prog, src.c_str(), "sable_spec.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
      SB_THROW(SABLE_ERR_HIP, "hiprtcCreateProgram failed");
    const hiprtcResult cr = hiprtcCompileProgram(prog, 6, opts);
    if (cr != HIPRTC_SUCCESS) {
      size_t n = 0;
      hiprtcGetProgramLogSize(prog, &n);
      std::string log(n, '\0');
      if (n) hiprtcGetProgramLog(prog, &log[0]);
      SB_THROW(SABLE_ERR_HIP, "hipRTC: %s: %.400s", hiprtcGetErrorString(cr), log.c_str());
    }
    size_t csz = 0;
    if (hiprtcGetCodeSize(prog, &csz) != HIPRTC_SUCCESS || csz == 0) SB_THROW(SABLE_ERR_HIP, "hipRTC: no code");
    std::vector<char> code(csz);
    if (hiprtcGetCode(prog, code.data()) != HIPRTC_SUCCESS) SB_THROW(SABLE_ERR_HIP, "hipRTC: code");
    hiprtcDestroyProgram(&prog);
    prog = nullptr;
    hipModule_t mod = nullptr;
    HIPC(hipModuleLoadData(&mod, code.data()));
    hipFunction_t fn = nullptr;
    const hipError_t fe = hipModuleGetFunction(&fn, mod, "sable_spec_spmv");
    if (fe != hipSuccess) {
      (void)hipModuleUnload(mod);
      SB_THROW(SABLE_ERR_HIP, "hipModuleGetFunction: %s", hipGetErrorString(fe));
    }
    p->spec_module = mod;
    p->spec_func = fn;
    p->spec_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return SABLE_OK;
  } catch (const Err& e) {
    if (prog) hiprtcDestroyProgram(&prog);
    return e.st;
  } catch (...) {
    if (prog) hiprtcDestroyProgram(&prog);
    set_error("internal error");
    return SABLE_ERR_INTERNAL;
  }
}
