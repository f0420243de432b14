// Internal plan representation: formats in HBM plus the execution schedule.
#pragma once

#include <utility>
#include <vector>

#include "common.h"

namespace sable {

// Residual matrix on the device: CSR (int32 row pointers, nnz < 2^31) plus, per stored
// entry, its index in the input matrix (to build the owner/slot map and refresh values).
struct Resid {
  int nrows = 0, ncols = 0;
  i64 nnz = 0;
  DBuf<int32_t> ptr, col, id;
  DBuf<float> val;
};

struct SegRec {  // band segment produced by the band extractor: rows [i0, j), [d-L, d+U]
  int32_t i0, j, L, U, d, cand;
  i64 z;
};

struct BlkRec {  // block rectangle rows [r0, r1), columns [c0, c1)
  int32_t r0, r1, c0, c1;
};

// Launch parameters of the fused kernels (autotuned).
// SpMV kernel variants: 0..2 = streamed tile body with 1, 2, 4 rows per thread (tiles of
// 256, 512, 1024 rows); 3..7 = row-per-lane bands/blocks with 1, 2, 4, 8, 16 lanes per CSR
// row (tiles of 256 / W rows); 8..10 = 0..2 with non-temporal matrix loads; 11 = run-time
// specialized; 12..14 = row-length bins with subwave widths for about 1, 2, 4 entries per
// lane. The plain CSR baseline: 0..2 streamed, 3..9 = 1..64 lanes per row, 10..12 = 0..2
// non-temporal, 13..15 = row-length bins as 12..14.
struct ExecParams {
  int spmv_variant = 1;
  int plain_variant = 1;
  int spmm_mode = 0;  // fused SpMM variant: 0 tiled, matrix cores (automatic work split),
                      // 1 tiled fp32 VALU, 2 wave per row, 3 tiled, matrix cores (chunk split),
                      // 4 tiled, matrix cores on LDS-staged panels (16x16x32 steps)
  int far_split = 1;  // streamed SpMV: gather far-column CSR entries in a separate pass
  // SpMM variant the autotuner chose for each number of right-hand sides it was run with;
  // an explicit sable_plan_set_variant for SpMM clears it
  std::vector<std::pair<int, int>> spmm_tuned;  // (n, mode)
  int spmm_mode_for(int n) const {
    for (const auto& t : spmm_tuned)
      if (t.first == n) return t.second;
    return spmm_mode;
  }
};

// Far-column split of the CSR remainder (streamed SpMV variants). An entry whose column lies
// more than kFarWindow columns from its row would pull a whole cache line of x for one
// 4-byte value, and a wave of such entries issues 64 separate cache requests. Such entries
// are grouped by column panel (x slices of kFarPanelCols columns); a gather pass stages a
// panel's x slice in LDS with coalesced loads and multiplies the panel's entries by it,
// writing the products in panel order (panel p's workgroups run on XCD p mod 8, so repeated
// slice loads hit one L2). The tile kernel walks the CSR part as usual over ccol, a copy of
// csr_col in which a far entry's column is replaced by -(1 + position of its product), and
// takes the stored product for it. The order of every row's sum is unchanged, so results
// equal those without the split bit for bit.
constexpr int kFarWindow = 1 << 17;      // |column - row| above this is far
constexpr int kFarPanelCols = 1 << 13;   // x slice per panel: 32 KB of fp32 in LDS
constexpr int kFarThreads = 1024;
constexpr int kFarChunk = 8 * kFarThreads;  // entries per gather workgroup
constexpr int kFarMinEntries = 1 << 16;  // below this the extra pass is not worth a launch
constexpr int kFarMinCols = 1 << 20;     // x below 4 MB stays L2-resident anyway
static_assert(kFarPanelCols <= 65536, "panel-relative far columns are 16-bit");

struct FarSplit {
  int npanel = 0;  // 0: no split
  int panel_cols = 0;
  int per_xcd = 0;  // gather workgroups per XCD
  i64 nfar = 0;
  DBuf<int32_t> ccol;                 // csr_col with far entries encoded as -(1 + q)
  DBuf<uint16_t> far_col;             // column within its panel; panel-major, row order inside
  DBuf<int32_t> far_src;              // CSR index of each far entry
  DBuf<float> far_val, far_prod;
  DBuf<double> far_val64, far_prod64;  // fp64 executor (after fp64 values are set)
  DBuf<int32_t> chunk;  // [8][per_xcd] (begin, end) entry ranges, begin < 0 = none
};

// Matrix-core SpMM panels (16x16x32 bf16 steps) of the 64-row SpMM schedule: for every tile,
// the distinct block columns its blocks touch, ascending, padded with -1 to a multiple of 32
// (32 list positions = one panel = one k step); for every entry of the tile -> block list
// (ordered by first column), the list position of the block's first column.
struct MmPanels {
  DBuf<int32_t> kcol;  // tile t: kcol[kptr[t] .. kptr[t + 1])
  DBuf<int32_t> kptr;  // ntiles + 1 offsets, multiples of 32
  DBuf<int32_t> bpos;  // aligned with the schedule's tile_blk
  // The A operand of every panel, packed at plan time from the split-bf16 words. Panel g
  // (g = kptr[t] / 32 + j for panel j of tile t) is a 64 x 32 bf16 operand cut into 256 units
  // of one row and 8 consecutive columns (unit u = 4 row + column / 8, the piece one thread
  // loads). amask[4 g .. 4 g + 3] has bit u set when a block cell falls in unit u; the set
  // units are stored in order from apack[2 aptr[g]] on, each as its hi then its lo 16 bytes
  // (zero where no cell falls). A thread of the SpMM loads its unit with two 16-byte loads,
  // or nothing when the unit is empty. pan_tile / pan_pos: tile and tile-relative first list
  // position of each panel.
  DBuf<uint4> apack;
  DBuf<uint64_t> amask;
  DBuf<i64> aptr;
  DBuf<int32_t> pan_tile, pan_pos;
  i64 npanels = 0, nunits = 0;
};

// What a streamed SpMV tile needs before its first dependent load, one 64-byte record per
// launch slot (slot k runs tile order[k]): the tile, its rows, its CSR entry range, its band
// segment and block list ranges and its first segment's descriptor. One load of the record
// replaces the chain order -> row bounds -> row pointers -> descriptors.
struct TileHead {
  int32_t tile, r0, rend, e0, e1, slo, shi, blo, bhi, rs, nr, nd, sip, pad;
  i64 svp;
};
static_assert(sizeof(TileHead) == 64, "tile records are 64 bytes");

struct Schedule {
  int rows_per_tile = 0;
  int ntiles = 0;
  DBuf<int32_t> tile_seg_lo, tile_seg_hi;  // VDIA segments overlapping each tile
  DBuf<int32_t> tile_blk_ptr, tile_blk;    // VBR blocks overlapping each tile
  // Launch order of the streamed kernels: workgroup slot i runs tile order[i]. Within each
  // XCD's contiguous run of slots the tiles are sorted by estimated cost, heaviest first, so
  // the few expensive tiles (dense blocks, long rows) do not finish last.
  DBuf<int32_t> order;
  // Entry-balanced tiling (SpMV schedules): tile t is rows [row0[t], row0[t+1]), at most
  // rows_per_tile rows and, unless it is a single row, at most
  // min(max(4096, 8 rows_per_tile), max(512, CSR entries / 2048)) CSR entries, so a run of
  // long rows is spread over several workgroups and a small input still gives about 2048
  // tiles. Empty: tile t is rows [t rows_per_tile, (t+1) rows_per_tile).
  DBuf<int32_t> row0;
  // Row-length bins of the CSR part (binned SpMV variants; tiles of at most 256 rows): the
  // rows of each tile grouped by bin, stable (bin_rows, absolute row ids, tile after tile),
  // and per tile the kNumBins + 1 bin boundaries in bin_rows (empty for other schedules).
  DBuf<int32_t> bin_rows, bin_off;
  DBuf<TileHead> head;  // streamed SpMV schedules: one record per launch slot
};

}  // namespace sable

struct sable_plan_s {
  int nrows = 0, ncols = 0;
  sable::i64 nnz = 0;
  // VDIA (Sec. 4.2.1)
  int nseg = 0;
  sable::i64 nidiag = 0, vdia_cells = 0, vdia_nnz = 0;
  sable::DBuf<float> vdia_val;
  sable::DBuf<int32_t> idiag, seg_row_start, seg_nrows, seg_ndiags, seg_idiag_ptr;
  sable::DBuf<sable::i64> seg_val_ptr;
  // VBR (App. B): blk = (r0, r1, c0, c1) per block, values column-major per block
  int nblk = 0;
  int vbr_mode_used = 0, vbr_tile = 0;
  sable::i64 vbr_cells = 0, vbr_nnz = 0;
  sable::DBuf<int32_t> blk;
  sable::DBuf<sable::i64> blk_val_ptr;
  sable::DBuf<float> vbr_val;
  // bf16 split copies for matrix-core SpMM: per block row-major with the row stride padded
  // to a multiple of 4 (w4), each element one 32-bit word (hi | lo << 16)
  sable::DBuf<uint32_t> vbr_mma;
  sable::DBuf<sable::i64> blk_mma_ptr;
  // CSR remainder
  sable::i64 csr_nnz = 0;
  sable::DBuf<int32_t> csr_ptr, csr_col;
  sable::DBuf<float> csr_val;
  // fp64 copies of the format values for the FP64 executor (empty until
  // sable_update_values_f64); same layouts as vdia_val / vbr_val / csr_val
  sable::DBuf<double> vdia_val64, vbr_val64, csr_val64;
  bool has_f64 = false;
  // Whole input as CSR (plain baseline) and owner/slot map of every input entry
  sable::DBuf<int32_t> a_ptr, a_col;
  sable::DBuf<float> a_val;
  sable::DBuf<int8_t> owner;
  sable::DBuf<sable::i64> slot;
  // schedule and tuned parameters
  sable::Schedule sched[3];        // tiles of 256, 512, 1024 rows with the formats
  sable::Schedule sched_plain[3];  // the same tilings for the whole input as CSR
  sable::Schedule sched_mm;        // 64-row tiles of the fused SpMM
  sable::MmPanels mm_panels;       // matrix-core panels of sched_mm (with the bf16 copies)
  sable::Schedule sched_w[4];      // tiles of 256 / W rows, W = 2, 4, 8, 16 lanes per CSR row
  sable::FarSplit far;             // far-column split of the CSR part (streamed SpMV)
  sable::ExecParams prm;
  uint32_t flags = 0;
  double plan_ms = 0.0;
  uint64_t structure_hash = 0;  // pattern of A, extractor list, thresholds (autotuning cache key)
  uint64_t partition_hash = 0;  // owner and slot of every entry, VDIA segments, VBR blocks
  // run-time specialized SpMV (hipRTC module and kernel; null until sable_plan_specialize)
  void* spec_module = nullptr;
  void* spec_func = nullptr;
  double spec_ms = 0.0;
  sable::i64 device_bytes() const;
  ~sable_plan_s();
};

namespace sable {

// Extractors (each claims entries of R, fills its part of the plan, marks claimed[k]).
void extract_bands(sable_plan_s& P, const Resid& R, const sable_thresholds& th,
                   DBuf<uint8_t>& claimed, hipStream_t s);
// What extract_blocks records (mode used, tile size) for an input that has no entries.
void blocks_none(sable_plan_s& P, const sable_thresholds& th, int mode);
void extract_blocks(sable_plan_s& P, const Resid& R, const sable_thresholds& th, int mode,
                    DBuf<uint8_t>& claimed, hipStream_t s);
void extract_csr(sable_plan_s& P, const Resid& R, hipStream_t s);

// Residual management.
void resid_from_input(Resid& R, const sable_csr& A, hipStream_t s);
void resid_compact(Resid& R, const DBuf<uint8_t>& claimed, hipStream_t s);
void entry_rows(const Resid& R, DBuf<int32_t>& rows, hipStream_t s);
bool validate_csr_device(const sable_csr& A, hipStream_t s);

// Schedules and kernels.
void build_schedule(sable_plan_s& P, Schedule& S, int rows_per_tile, bool with_formats,
                    hipStream_t s, bool col_order = false, bool balance = false);
void build_bf16_split(sable_plan_s& P, hipStream_t s);
void build_mm_panels(sable_plan_s& P, hipStream_t s);
// (Re)pack the panels' A operands from the split-bf16 words (after a value refresh).
void pack_mm_panels(sable_plan_s& P, hipStream_t s);
void build_bins(const sable_plan_s& P, Schedule& S, bool with_formats, hipStream_t s);
void build_far_split(sable_plan_s& P, hipStream_t s);
void refresh_far_values(sable_plan_s& P, hipStream_t s);
// fp64 copies of the far entries' values (from csr_val64), allocated on first use.
void refresh_far_values64(sable_plan_s& P, hipStream_t s);
void launch_spmv(const sable_plan_s& P, const float* x, float* y, hipStream_t s);
// Time the plan's kernel variants and keep the fastest (op 0 SpMV, 1 SpMM with n columns).
void autotune(sable_plan_s& P, int op, int n, const float* x, float* y, hipStream_t s);
void launch_spmv_plain(const sable_plan_s& P, const float* x, float* y, hipStream_t s);
void launch_spmm(const sable_plan_s& P, const float* X, float* Y, int n, hipStream_t s);
// Matrix-core mode of the tiled SpMM for the plan's variant (0 none, 1 auto split, 2 chunks).
int spmm_mfma_mode(const sable_plan_s& P, int mode);
void launch_spmv_f64(const sable_plan_s& P, const double* x, double* y, hipStream_t s);
void launch_spmv_spec(const sable_plan_s& P, const float* x, float* y, hipStream_t s);
void launch_spmm_f64(const sable_plan_s& P, const double* X, double* Y, int n, hipStream_t s);

}  // namespace sable
