// Band extractor (Sec. 4.2; Alg. 3 ExtractBands, Alg. 4 GrowSegments) -> VDIA (Sec. 4.2.1).
//
// GPU data flow:
//   1. key(entry) = column - row (+ nrows-1 bias); a stable radix sort by key gives, for every
//      diagonal d, the rows that carry an entry on d in increasing order (diagonal-major
//      index) and the counts M[d] by run-length encoding.
//   2. Candidates: diagonals with M[d] >= l_seg (count threshold), ranked by M descending,
//      then d ascending, with a 64-bit key radix sort.
//   3. Candidates are processed in order, in speculative batches: FitRibbon runs one thread
//      per (candidate, present row) and also records which offsets within W_max of the
//      diagonal are present (two 64-bit masks); GrowSegments runs one wave per candidate,
//      64 rows per step with wave scans and mask popcounts. A candidate reads only the rows on its diagonal (their used
//      flag and their own entries), so its result is exact unless a candidate accepted
//      earlier in the same batch claimed one of those rows; the host checks this with row
//      spans and re-runs the batch from the first conflicting candidate.
//   4. Accepted segments are packed diagonal-major and their entries claimed.
// Density tests are exact integer tests 1000*z >= p*area.
#include <algorithm>
#include <climits>

#include "plan.h"

namespace sable {

namespace {

constexpr uint32_t kNoKey = 0xffffffffu;

__global__ void k_diag_keys(const int32_t* __restrict__ rows, const int32_t* __restrict__ col,
                            i64 nnz, int nrows, int dmax, uint32_t* __restrict__ keys,
                            int32_t* __restrict__ vals) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < nnz; k += (i64)gridDim.x * blockDim.x) {
    const i64 d = (i64)col[k] - rows[k];
    bool ok = dmax < 0 || (d <= dmax && d >= -(i64)dmax);
    keys[k] = ok ? (uint32_t)(d + nrows - 1) : kNoKey;
    vals[k] = (int32_t)k;
  }
}

// Rank key: count descending, then diagonal ascending; non-candidates sort last.
__global__ void k_cand_keys(const uint32_t* __restrict__ uniq, const int32_t* __restrict__ cnt,
                            i64 nruns, int tau, uint64_t* __restrict__ rk, int32_t* __restrict__ idx,
                            int* __restrict__ ncand) {
  for (i64 r = blockIdx.x * (i64)blockDim.x + threadIdx.x; r < nruns; r += (i64)gridDim.x * blockDim.x) {
    bool c = uniq[r] != kNoKey && cnt[r] >= tau;
    rk[r] = c ? ((uint64_t)(0x7fffffffu - (uint32_t)cnt[r]) << 32) | uniq[r] : ~0ull;
    idx[r] = (int32_t)r;
    if (c) atomicAdd(ncand, 1);
  }
}

__global__ void k_gather_rows(const int32_t* __restrict__ perm, const int32_t* __restrict__ rows,
                              i64 n, int32_t* __restrict__ srow) {
  for (i64 k = blockIdx.x * (i64)blockDim.x + threadIdx.x; k < n; k += (i64)gridDim.x * blockDim.x)
    srow[k] = rows[perm[k]];
}

// FitRibbon reading (Alg. 3): starting at the centre cell, extend by the nearest present cell
// below or above (smaller gap first, below on ties) while the ribbon stays delta-dense; each
// side is capped at wmax. Present cells of a ribbon are consecutive entries of the row, so the
// nearest present cell on each side is the neighbouring entry.
__global__ void k_fit_ribbon(const int32_t* __restrict__ bpre, int nb, const i64* __restrict__ cstart,
                             const int32_t* __restrict__ cd, i64 items,
                             const int32_t* __restrict__ perm, const int32_t* __restrict__ srow,
                             const int32_t* __restrict__ rptr, const int32_t* __restrict__ rcol,
                             const uint8_t* __restrict__ used, int p, int wmax,
                             int32_t* __restrict__ Lp, int32_t* __restrict__ Up,
                             int32_t* __restrict__ Kp, uint64_t* __restrict__ Mlo,
                             uint64_t* __restrict__ Mhi) {
  for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < items; t += (i64)gridDim.x * blockDim.x) {
    int lo = 0, hi = nb - 1;  // last c with bpre[c] <= t
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if ((i64)bpre[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int c = lo;
    const i64 pos = cstart[c] + (t - bpre[c]);
    const int i = srow[pos];
    const int e = perm[pos];
    int l = 0, u = 0, k = 0;
    if (!used[i]) {
      const int d = cd[c];
      const int rs = rptr[i], re = rptr[i + 1];
      int elo = e, ehi = e;
      k = 1;
      for (;;) {
        int glo = INT_MAX, ghi = INT_MAX;
        if (elo > rs) {
          int g = (i + d - l) - rcol[elo - 1];
          if (l + g <= wmax) glo = g;
        }
        if (ehi + 1 < re) {
          int g = rcol[ehi + 1] - (i + d + u);
          if (u + g <= wmax) ghi = g;
        }
        bool applied = false;
        // first candidate: smaller gap, below on ties; then the other one
        for (int pass = 0; pass < 2 && !applied; ++pass) {
          bool below = (glo <= ghi) ? (pass == 0) : (pass == 1);
          int g = below ? glo : ghi;
          if (g == INT_MAX) continue;
          if (1000LL * (k + 1) >= (long long)p * (l + u + 1 + g)) {
            if (below) { l += g; --elo; } else { u += g; ++ehi; }
            ++k;
            applied = true;
          }
        }
        if (!applied) break;
      }
    }
    Lp[pos] = l;
    Up[pos] = u;
    Kp[pos] = k;
    // presence masks around the centre: bit t of lo = offset d-1-t, bit t of hi = offset d+t
    uint64_t mlo = 0, mhi = 0;
    if (k) {
      const int d = cd[c];
      const int rs = rptr[i], re = rptr[i + 1];
      for (int q = e; q < re; ++q) {
        const int t = rcol[q] - (i + d);
        if (t > wmax) break;
        mhi |= 1ull << t;
      }
      for (int q = e - 1; q >= rs; --q) {
        const int t = (i + d) - 1 - rcol[q];
        if (t >= wmax) break;
        mlo |= 1ull << t;
      }
    }
    Mlo[pos] = mlo;
    Mhi[pos] = mhi;
  }
}

__device__ inline i64 shfl64(i64 v, int src) {
  int lo = __shfl((int)(uint32_t)(v & 0xffffffffu), src, 64);
  int hi = __shfl((int)(v >> 32), src, 64);
  return (i64)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ inline i64 shfl_up64(i64 v, int delta) {
  int lo = __shfl_up((int)(uint32_t)(v & 0xffffffffu), delta, 64);
  int hi = __shfl_up((int)(v >> 32), delta, 64);
  return (i64)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ inline i64 wave_incl_sum(i64 v, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    i64 t = shfl_up64(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ inline i64 wave_sum(i64 v) {
  for (int o = 32; o > 0; o >>= 1) v += shfl64(v, (threadIdx.x & 63) ^ o);
  return v;
}

__device__ inline int wave_incl_max(int v, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v = max(v, t);
  }
  return v;
}

__device__ inline int first_lane(unsigned long long m) { return m ? __ffsll((long long)m) - 1 : 64; }

struct CandStat {
  i64 area, z;
  int32_t nseg, rmin, rmax, first_row, last_row, pad;
};

// Present cells of a row in offsets [d-L, d+U] from its presence masks (L <= 64, U <= 63).
__device__ __forceinline__ int mask_count(uint64_t mlo, uint64_t mhi, int L, int U) {
  const uint64_t ml = L >= 64 ? ~0ull : ((1ull << L) - 1ull);
  const uint64_t mh = U >= 63 ? ~0ull : ((1ull << (U + 1)) - 1ull);
  return __popcll(mlo & ml) + __popcll(mhi & mh);
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  return (uint64_t)shfl64((i64)v, src);
}

// GrowSegments (Alg. 4), one 64-lane wave per candidate diagonal. Lanes hold 64 consecutive
// positions of the candidate's row list (64 consecutive rows while the run lasts); window
// counts come from presence masks, so a segment that breaks inside a chunk restarts at the
// breaking lane without reloading anything.
__global__ __launch_bounds__(64) void k_grow(
    int nb, const i64* __restrict__ cstart, const int32_t* __restrict__ ccnt,
    const int32_t* __restrict__ cd, const int32_t* __restrict__ srow,
    const int32_t* __restrict__ Lp, const int32_t* __restrict__ Up,
    const int32_t* __restrict__ Kp, const uint64_t* __restrict__ Mlo,
    const uint64_t* __restrict__ Mhi, int nrows, int p, int lseg, SegRec* __restrict__ segs,
    int* __restrict__ nsegs, int seg_cap, CandStat* __restrict__ stat) {
  const int c = blockIdx.x;
  if (c >= nb) return;
  const int lane = threadIdx.x;
  const i64 st = cstart[c];
  const int cnt = ccnt[c];
  const int d = cd[c];
  i64 area_sum = 0, z_sum = 0;
  int nseg = 0, rmin = INT_MAX, rmax = -1;

  auto emit = [&](int i0, int jend, int L, int U, i64 z) {
    if (jend - i0 < lseg) return;
    area_sum += (i64)(L + U + 1) * (jend - i0);
    z_sum += z;
    ++nseg;
    rmin = min(rmin, i0);
    rmax = max(rmax, jend - 1);
    if (lane == 0) {
      int slot = atomicAdd(nsegs, 1);
      if (slot < seg_cap) {
        SegRec rec;
        rec.i0 = i0; rec.j = jend; rec.L = L; rec.U = U; rec.d = d; rec.cand = c; rec.z = z;
        segs[slot] = rec;
      }
    }
  };

  int q = 0;
  while (q < cnt) {
    // next position with k > 0 starts a segment
    bool found = false;
    while (q < cnt) {
      const int pq = q + lane;
      const bool ok = pq < cnt && Kp[st + pq] > 0;
      const unsigned long long m = __ballot(ok);
      if (m) { q += first_lane(m); found = true; break; }
      q += 64;
    }
    if (!found) break;
    int qs = q;                      // position of the current segment's first row
    const int row0_first = srow[st + qs];
    int i0 = row0_first;
    int L = Lp[st + qs], U = Up[st + qs];
    i64 z = Kp[st + qs];
    int cpos = qs;                   // position held by lane 0 of the current chunk
    int row0 = row0_first;           // row of lane 0 when the run continues
    int base = 1;                    // first lane still to examine
    bool done = false;
    while (!done) {
      const int pq = cpos + lane;
      const int pc = pq < cnt ? pq : cnt - 1;
      const bool valid = pq < cnt && row0 + lane < nrows && srow[st + pc] == row0 + lane &&
                         Kp[st + pc] > 0;
      const int lv = valid ? Lp[st + pc] : 0, uv = valid ? Up[st + pc] : 0;
      const int kv = valid ? Kp[st + pc] : 0;
      const uint64_t mlo = valid ? Mlo[st + pc] : 0ull, mhi = valid ? Mhi[st + pc] : 0ull;
      const unsigned long long inval = __ballot(!valid);
      while (base < 64) {
        const unsigned long long above = ~0ull << base;
        const int f = first_lane(inval & above);   // first invalid lane at or after base
        const int Lm = max(L, wave_incl_max(lane >= base ? lv : 0, lane));
        const int Um = max(U, wave_incl_max(lane >= base ? uv : 0, lane));
        const bool widen = lane >= base && lane < f && (Lm != L || Um != U);
        const int w = first_lane(__ballot(widen));
        const int lim = min(f, w);
        const i64 cv = (lane >= base && lane < lim) ? mask_count(mlo, mhi, L, U) : 0;
        const i64 zp = z + wave_incl_sum(cv, lane);
        const i64 area = (i64)(L + U + 1) * (row0 + lane - i0 + 1);
        const bool brk = lane >= base && lane < lim && 1000LL * zp < (long long)p * area;
        const int b = first_lane(__ballot(brk));
        if (b < lim) {
          emit(i0, row0 + b, L, U, b > base ? shfl64(zp, b - 1) : z);
          i0 = row0 + b;
          L = __shfl(lv, b, 64);
          U = __shfl(uv, b, 64);
          z = __shfl(kv, b, 64);
          qs = cpos + b;
          base = b + 1;
          continue;
        }
        if (w < f) {
          z = w > base ? shfl64(zp, w - 1) : z;
          const int L2 = __shfl(Lm, w, 64), U2 = __shfl(Um, w, 64);
          // exact recount over the segment's rows with the widened extents
          i64 part = 0;
          for (int pp = qs + lane; pp < cpos; pp += 64)
            part += mask_count(Mlo[st + pp], Mhi[st + pp], L2, U2);
          const int from = max(qs - cpos, 0);
          if (lane >= from && lane <= w) part += mask_count(mlo, mhi, L2, U2);
          const i64 z2 = wave_sum(part);
          const i64 area2 = (i64)(L2 + U2 + 1) * (row0 + w - i0 + 1);
          if (1000LL * z2 < (long long)p * area2) {
            emit(i0, row0 + w, L, U, z);
            i0 = row0 + w;
            L = __shfl(lv, w, 64);
            U = __shfl(uv, w, 64);
            z = __shfl(kv, w, 64);
            qs = cpos + w;
          } else {
            L = L2; U = U2; z = z2;
          }
          base = w + 1;
          continue;
        }
        z = f > base ? shfl64(zp, f - 1) : z;
        if (f < 64) {  // the run of k > 0 rows ends before lane f
          emit(i0, row0 + f, L, U, z);
          q = cpos + f;
          done = true;
        }
        base = 64;
      }
      if (!done) {
        cpos += 64;
        row0 += 64;
        base = 0;
      }
    }
  }
  if (lane == 0) {
    CandStat s;
    s.area = area_sum; s.z = z_sum; s.nseg = nseg; s.rmin = rmin; s.rmax = rmax;
    s.first_row = cnt ? srow[st] : 0;
    s.last_row = cnt ? srow[st + cnt - 1] : -1;
    s.pad = 0;
    stat[c] = s;
  }
}

__global__ void k_mark_used(const SegRec* __restrict__ segs, int n, uint8_t* __restrict__ used) {
  const SegRec s = segs[blockIdx.x];
  for (int r = s.i0 + threadIdx.x; r < s.j; r += blockDim.x) used[r] = 1;
}

// One thread per row: the row's segment (if any) receives its window's entries.
__global__ void k_pack_vdia(int nrows, int nseg, const int32_t* __restrict__ srs,
                            const int32_t* __restrict__ snr, const int32_t* __restrict__ snd,
                            const i64* __restrict__ svp, const int32_t* __restrict__ sip,
                            const int32_t* __restrict__ idiag, const int32_t* __restrict__ rptr,
                            const int32_t* __restrict__ rcol, const float* __restrict__ rval,
                            const int32_t* __restrict__ rid, float* __restrict__ val,
                            uint8_t* __restrict__ claimed, int8_t* __restrict__ owner,
                            i64* __restrict__ slot) {
  for (i64 r = blockIdx.x * (i64)blockDim.x + threadIdx.x; r < nrows; r += (i64)gridDim.x * blockDim.x) {
    int lo = 0, hi = nseg - 1, s = -1;
    while (lo <= hi) {
      int mid = (lo + hi) >> 1;
      if (srs[mid] <= r) { s = mid; lo = mid + 1; } else hi = mid - 1;
    }
    if (s < 0 || r >= (i64)srs[s] + snr[s]) continue;
    const int nr = snr[s], nd = snd[s];
    const int o0 = idiag[sip[s]];
    const i64 clo = r + o0, chi = r + o0 + nd - 1;
    for (int k = rptr[r]; k < rptr[r + 1]; ++k) {
      const i64 c = rcol[k];
      if (c < clo || c > chi) continue;
      const i64 at = svp[s] + (c - clo) * nr + (r - srs[s]);
      val[at] = rval[k];
      claimed[k] = 1;
      owner[rid[k]] = 0;
      slot[rid[k]] = at;
    }
  }
}

}  // namespace

void extract_bands(sable_plan_s& P, const Resid& R, const sable_thresholds& th,
                   DBuf<uint8_t>& claimed, hipStream_t s) {
  const int n = R.nrows;
  const int p = th.delta_band_pm;
  const int tau = th.lseg;
  std::vector<SegRec> accepted;
  if (R.nnz > 0 && n > 0) {
    // 1. diagonal keys, stable sort, run-length counts M[d]
    DBuf<int32_t> rows;
    entry_rows(R, rows, s);
    DBuf<uint32_t> keys(R.nnz);
    DBuf<int32_t> perm(R.nnz);
    k_diag_keys<<<grid_for(R.nnz, 256), 256, 0, s>>>(rows.p, R.col.p, R.nnz, n, th.dmax, keys.p,
                                                     perm.p);
    LAUNCH_CHECK();
    sort_pairs_u32(keys, perm, R.nnz, bits_for((uint64_t)n + R.ncols), s);
    DBuf<uint32_t> uniq;
    DBuf<int32_t> cnt;
    const i64 nruns = rle_u32(keys.p, R.nnz, uniq, cnt, s);
    DBuf<int32_t> off(nruns + 1);
    exclusive_scan_i32(cnt.p, off.p, nruns, s);
    DBuf<int32_t> srow(R.nnz);
    k_gather_rows<<<grid_for(R.nnz, 256), 256, 0, s>>>(perm.p, rows.p, R.nnz, srow.p);
    LAUNCH_CHECK();
    // 2. candidate ranking
    DBuf<uint64_t> rk(nruns);
    DBuf<int32_t> ridx(nruns);
    DBuf<int> ncand_d(1);
    HIPC(hipMemsetAsync(ncand_d.p, 0, sizeof(int), s));
    k_cand_keys<<<grid_for(nruns, 256), 256, 0, s>>>(uniq.p, cnt.p, nruns, tau, rk.p, ridx.p,
                                                     ncand_d.p);
    LAUNCH_CHECK();
    sort_pairs_u64(rk, ridx, nruns, 64, s);
    int ncand = 0;
    HIPC(hipMemcpyAsync(&ncand, ncand_d.p, sizeof(int), hipMemcpyDeviceToHost, s));
    std::vector<int32_t> h_ridx, h_cnt, h_off;
    std::vector<uint32_t> h_uniq;
    to_host(h_ridx, ridx.p, ncand, s);
    to_host(h_cnt, cnt.p, nruns, s);
    to_host(h_off, off.p, nruns, s);
    to_host(h_uniq, uniq.p, nruns, s);
    std::vector<i64> c_start(ncand);
    std::vector<int32_t> c_cnt(ncand), c_d(ncand);
    for (int c = 0; c < ncand; ++c) {
      const int r = h_ridx[c];
      c_start[c] = h_off[r];
      c_cnt[c] = h_cnt[r];
      c_d[c] = (int32_t)((i64)h_uniq[r] - (n - 1));
    }
    // 3. candidates in speculative batches
    DBuf<uint8_t> used(n);
    HIPC(hipMemsetAsync(used.p, 0, n, s));
    DBuf<int32_t> Lp(R.nnz), Up(R.nnz), Kp(R.nnz);
    DBuf<uint64_t> Mlo(R.nnz), Mhi(R.nnz);
    int b0 = 0, bsize = 1;
    const i64 item_budget = (i64)1 << 26;
    while (b0 < ncand) {
      int b1 = b0;
      i64 items = 0;
      while (b1 < ncand && b1 - b0 < bsize && (b1 == b0 || items + c_cnt[b1] <= item_budget)) {
        items += c_cnt[b1];
        ++b1;
      }
      const int nb = b1 - b0;
      std::vector<int32_t> bpre(nb);
      i64 acc = 0;
      i64 seg_cap = 0;
      for (int c = 0; c < nb; ++c) {
        bpre[c] = (int32_t)acc;
        acc += c_cnt[b0 + c];
        seg_cap += c_cnt[b0 + c] / std::max(1, th.lseg) + 1;
      }
      std::vector<i64> bst(c_start.begin() + b0, c_start.begin() + b1);
      std::vector<int32_t> bcnt(c_cnt.begin() + b0, c_cnt.begin() + b1);
      std::vector<int32_t> bd(c_d.begin() + b0, c_d.begin() + b1);
      DBuf<int32_t> d_bpre, d_bcnt, d_bd;
      DBuf<i64> d_bst;
      to_dev(d_bpre, bpre, s);
      to_dev(d_bst, bst, s);
      to_dev(d_bcnt, bcnt, s);
      to_dev(d_bd, bd, s);
      k_fit_ribbon<<<grid_for(items, 256), 256, 0, s>>>(d_bpre.p, nb, d_bst.p, d_bd.p, items,
                                                        perm.p, srow.p, R.ptr.p, R.col.p, used.p,
                                                        p, th.wmax, Lp.p, Up.p, Kp.p, Mlo.p, Mhi.p);
      LAUNCH_CHECK();
      DBuf<SegRec> segs(seg_cap);
      DBuf<int> nsegs(1);
      DBuf<CandStat> stat(nb);
      HIPC(hipMemsetAsync(nsegs.p, 0, sizeof(int), s));
      k_grow<<<nb, 64, 0, s>>>(nb, d_bst.p, d_bcnt.p, d_bd.p, srow.p, Lp.p, Up.p, Kp.p, Mlo.p,
                               Mhi.p, n, p, th.lseg, segs.p, nsegs.p, (int)seg_cap, stat.p);
      LAUNCH_CHECK();
      std::vector<CandStat> hs;
      to_host(hs, stat.p, nb, s);
      int hn = 0;
      HIPC(hipMemcpyAsync(&hn, nsegs.p, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      if (hn > seg_cap) SB_THROW(SABLE_ERR_INTERNAL, "segment buffer overflow");
      std::vector<SegRec> hseg;
      to_host(hseg, segs.p, hn, s);
      // host walk in candidate order: conflicts end the batch
      std::vector<std::pair<int, int>> spans;
      std::vector<char> acc_c(nb, 0);
      int stop = nb;
      for (int c = 0; c < nb; ++c) {
        bool conflict = false;
        for (auto& sp : spans)
          if (!(hs[c].last_row < sp.first || hs[c].first_row > sp.second)) { conflict = true; break; }
        if (conflict) { stop = c; break; }
        if (hs[c].nseg == 0) continue;
        if (hs[c].area < th.amin_band || (__int128)1000 * hs[c].z < (__int128)p * hs[c].area) continue;
        acc_c[c] = 1;
        spans.push_back({hs[c].rmin, hs[c].rmax});
      }
      std::vector<SegRec> newly;
      for (auto& sg : hseg)
        if (sg.cand < stop && acc_c[sg.cand]) newly.push_back(sg);
      if (!newly.empty()) {
        DBuf<SegRec> d_new;
        to_dev(d_new, newly, s);
        k_mark_used<<<(unsigned)newly.size(), 256, 0, s>>>(d_new.p, (int)newly.size(), used.p);
        LAUNCH_CHECK();
        HIPC(hipStreamSynchronize(s));
        accepted.insert(accepted.end(), newly.begin(), newly.end());
      }
      HIPC(hipStreamSynchronize(s));
      b0 += stop;
      if (stop == nb) bsize = std::min(bsize * 2, 1 << 14);
      else bsize = std::max(1, bsize / 2);
    }
  }
  // 4. pack (segments are row-disjoint; export order = row start)
  std::sort(accepted.begin(), accepted.end(),
            [](const SegRec& a, const SegRec& b) { return a.i0 < b.i0; });
  const int ns = (int)accepted.size();
  std::vector<int32_t> srs(ns), snr(ns), snd(ns), sip(ns), idg;
  std::vector<i64> svp(ns);
  i64 cells = 0, z = 0;
  for (int k = 0; k < ns; ++k) {
    const SegRec& g = accepted[k];
    srs[k] = g.i0;
    snr[k] = g.j - g.i0;
    snd[k] = g.L + g.U + 1;
    svp[k] = cells;
    sip[k] = (int32_t)idg.size();
    for (int t = 0; t < snd[k]; ++t) idg.push_back(g.d - g.L + t);
    cells += (i64)snr[k] * snd[k];
    z += g.z;
  }
  P.nseg = ns;
  P.nidiag = (i64)idg.size();
  P.vdia_cells = cells;
  P.vdia_nnz = z;
  to_dev(P.seg_row_start, srs, s);
  to_dev(P.seg_nrows, snr, s);
  to_dev(P.seg_ndiags, snd, s);
  to_dev(P.seg_val_ptr, svp, s);
  to_dev(P.seg_idiag_ptr, sip, s);
  to_dev(P.idiag, idg, s);
  P.vdia_val.alloc(cells);
  if (cells) HIPC(hipMemsetAsync(P.vdia_val.p, 0, cells * sizeof(float), s));
  if (ns && R.nnz) {
    k_pack_vdia<<<grid_for(n, 256), 256, 0, s>>>(n, ns, P.seg_row_start.p, P.seg_nrows.p,
                                                 P.seg_ndiags.p, P.seg_val_ptr.p, P.seg_idiag_ptr.p,
                                                 P.idiag.p, R.ptr.p, R.col.p, R.val.p, R.id.p,
                                                 P.vdia_val.p, claimed.p, P.owner.p, P.slot.p);
    LAUNCH_CHECK();
  }
  HIPC(hipStreamSynchronize(s));
}

}  // namespace sable
