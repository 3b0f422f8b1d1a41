// rtg_internal.h -- launchers of the gfx950 kernels, shared by the host
// pipeline (rtg_host.cpp) and the kernels (rtg_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtgk {

constexpr int kBlock = 256;          // threads per block: four 64-wide waves
constexpr int kWaves = kBlock / 64;  // waves per block
constexpr int kKeysPerThread = 16;   // radix-sort / scan elements per thread
constexpr int kTile = kBlock * kKeysPerThread;  // 4096 elements per tile
constexpr int kPairTile = 64;        // points per tile in the cell-pair kernel
constexpr int kRadixBits = 8;        // digit width of one radix pass
constexpr int kMaxDim = 64;

// Where each axis of a cell vector sits in the packed 64-bit key.
struct KeyLayout {
  int32_t d;
  int32_t cell_bits;           // sum of bits[] (segment id sits above)
  uint8_t shift[kMaxDim];      // bit offset of axis j
  uint8_t bits[kMaxDim];       // width of axis j
};

// Tests of a squared distance against r^2: FP32 screen plus FP64 band.
struct PairTest {
  float lo;      // accept if d2_f32 <= lo  (lo <= r2 (1 - 2^-16))
  float hi;      // reject if d2_f32 >  hi  (hi >= r2 (1 + 2^-16))
  double r2;     // FP64 decision in between: s <= r2
  int32_t pair_bits;  // bits of one index in a packed (i,j) pair
  // An FP32 bound on |a - o|^2 + |b - o|^2 for three points a, b, o of one
  // grid cell (twice the squared cell diagonal, with margin), used by the
  // matrix-core screen when the cell keys are exact; 0: none.
  float s_bound;
};

// Optional hook around kernel launches (HIP-event timing, byte accounting).
struct LaunchTimer {
  void* self = nullptr;
  void (*begin)(void* self, int kid) = nullptr;
  void (*end)(void* self, int kid, double bytes) = nullptr;
  void on_begin(int kid) const {
    if (begin) begin(self, kid);
  }
  void on_end(int kid, double bytes) const {
    if (end) end(self, kid, bytes);
  }
};

// Device scalars to bring back with one copy (launch_gather).
struct Gather {
  const void* src[8] = {};
  int bytes[8] = {};
  int count = 0;
  void add(const void* p, int nbytes) {
    src[count] = p;
    bytes[count] = nbytes;
    ++count;
  }
};
void launch_gather(const Gather& g, uint64_t* dst, hipStream_t s);
// Writes words 32-bit words of src (or, with src null, the scalars of *g as
// u64) to pinned host memory at host, then seq to *host_seq with a
// system-scope release once every value is visible (one block).
void launch_mailbox(const uint32_t* src, uint32_t words, const Gather* g, uint32_t* host,
                    uint64_t* host_seq, uint64_t seq, hipStream_t s);
// rec[i][0..d) = rows[i][0..d), rec[i][d..rs) = 0 (padding, then the
// signature word in the last two floats), for i < n.
void launch_records(const float* rows, int64_t n, int d, int rs, float* rec, hipStream_t s);

// --- batches ------------------------------------------------------------------
// A batch is a set of instances (queries) of the same dimension d run through
// one pass of the pipeline.  Their points are concatenated (instance q owns
// batch points [pt_off, pt_off + n)); every (instance, grid) pair is one
// segment of the key space, numbered instance-major.  Kernels that work per
// point use blocks of kBlock points that never span two instances: instance
// q owns blocks [blk_first, blk_first + ceil(n / kBlock)).
struct InstDesc {
  const float* pts;   // the caller's row-major [n][d] points
  int64_t pt_off;     // first batch point of the instance
  int64_t n;          // points
  double inv_c;       // 1 / (alpha r)
  int32_t k;          // grids
  int32_t tr_off;     // first transform of the instance in R / u / klo
  int32_t seg_first;  // segment of (instance, grid 0); grid t is seg_first + t
  int32_t blk_first;  // first point block of the instance
};
struct SegDesc {
  int64_t key_off;    // first key of the segment within its pass
  int32_t inst;       // instance
  int32_t t;          // grid of the instance
};

// --- staging --------------------------------------------------------------
// For every instance: copy its points into the batch's SoA [d][npts] (and
// row-major aos [npts][d] when aos is not null), *bad = 1 if a value is not
// finite (else 0), and per-axis min/max as order-preserving uint32
// encodings in bbox[q][2d] (min at 2j, max at 2j+1).  nblocks = the
// instances' point blocks; part holds nblocks * 2d elements.  With rec, also
// the point records of the pair kernels' tile loads: rec[i][0..d) = the
// point, rec[i][d..rs) = 0 (the signature word, in the last two floats, is
// filled by the key kernel).  zero64[0, nzero), if given, is cleared first
// in the same launch as bbox and bad.
void launch_stage(const InstDesc* inst, uint32_t m, uint32_t nblocks, int d, int64_t npts,
                  float* soa, float* aos, uint32_t* bad, uint32_t* bbox, uint32_t* part,
                  float* rec, int rs, hipStream_t s, uint64_t* zero64 = nullptr,
                  uint32_t nzero = 0, bool cleared = false);

// --- cell keys ------------------------------------------------------------
// For every batch point and each of its instance's segments in [sa, sb):
// key = (segment - sa) << cell_bits | packed cell, written at
// segs[segment].key_off + the point's index in its instance; the value is
// the batch point index.  With idx_bits > 0 the point index rides in the
// key's low bits (key << idx_bits | point) and vals is unused.  If sig is
// not null, sig[point * kmax + grid] = the packed cell (u64 if sig64, else
// u32).  err |= 1 if some |y| >= 2^31.
struct KeysArgs {
  const InstDesc* inst;
  uint32_t m, nblocks;
  int d;
  int64_t npts;
  const float* soa;
  int sa, sb;
  const SegDesc* segs;
  const double *R, *u;
  const int64_t* klo;
  const KeyLayout* layout;
  uint64_t* keys;
  uint32_t* vals;
  uint32_t* err;
  uint64_t* sig;     // neighbourhood signatures (see PairFilter), or null
  int sig_stride, sig_b, sig_gpw;  // sig_stride: words from one point's signature to the next
  int idx_bits;
  int sig_fresh;     // 1: this pass covers every grid, so signature words are stored, not ORed
};
void launch_keys(const KeysArgs& a, hipStream_t s);
// kappa [n][d] = floor(y) for one transform (stage check).
void launch_cell_coords(const float* soa, int64_t n, int d, const double* R, const double* u,
                        double inv_c, int64_t* kappa, uint32_t* err, hipStream_t s);

// --- generic helpers ------------------------------------------------------
void launch_fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t s);
void launch_fill_u64(uint64_t* p, uint64_t v, size_t count, hipStream_t s);

// Exclusive prefix sum of count elements; total (device, optional) receives
// the sum.  scratch must hold scan_scratch_elems(count) elements.  With
// dcount (device) the elements are the first min(count, *dcount): count is
// then only the host's bound.
size_t scan_scratch_elems(size_t count);
void scan_exclusive_u32(const uint32_t* in, uint32_t* out, size_t count, uint32_t* total,
                        uint32_t* scratch, hipStream_t s, const uint32_t* dcount = nullptr);
void scan_exclusive_u64(const uint64_t* in, uint64_t* out, size_t count, uint64_t* total,
                        uint64_t* scratch, hipStream_t s, const uint32_t* dcount = nullptr);

// --- radix sort -----------------------------------------------------------
// Stable LSD sort of count 64-bit keys (and optional u32 values) on bits
// [begin_bit, end_bit), 8-bit digits.  Ping-pongs between (keys, vals) and
// (keys_alt, vals_alt); returns 0 if the result ends in keys/vals, 1 if in
// the *_alt.  scratch must hold radix_scratch_bytes(count, ...) bytes (any
// algorithm).  *err |= 2 if a look-back wait gave up (the output is then
// wrong but every write stays in bounds).  timer (optional) sees the
// histogram launches as kid_hist and each digit pass as kid_scatter.
//
// Segmented sorts (reduce-then-scan only): with a tile table, each tile
// covers keys [start, start + len) of one segment (len <= kTile) and its
// digit counts go to slot + digit * stride of a histogram table laid out
// segment by segment, digit by digit, tile by tile; the scan of that table
// then keeps every key inside its segment, so bits above end_bit (the
// segment id) need no pass.  ntiles_table tiles; the scratch needs
// radix_scratch_bytes(count, ..., ntiles_table - tiles_for(count)).
enum { kSortOnesweep = 0, kSortReduceScan = 1 };
struct SortTile {
  uint64_t start;
  uint32_t len;
  uint32_t slot;    // histogram index of digit 0
  uint32_t stride;  // distance between digits (the segment's tiles)
  uint32_t pad;
};
size_t radix_scratch_bytes(size_t count, int begin_bit, int end_bit, size_t extra_tiles = 0);
int radix_sort(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
               size_t count, int begin_bit, int end_bit, void* scratch, uint32_t* err,
               hipStream_t s, const LaunchTimer* timer = nullptr, int kid_hist = 0,
               int kid_scatter = 0, int algo = kSortOnesweep, const SortTile* tiles = nullptr,
               uint32_t ntiles_table = 0);

// --- cells ----------------------------------------------------------------
// Runs of equal keys >> shift with length >= 2 in a sorted key array: per
// tile counts of run heads and run tails (u32 each, ntiles entries), and the
// head and tail bits themselves, masks[2 g] and masks[2 g + 1] for the keys
// [64 g, 64 g + 64) (run_mask_words(count) words).
void launch_run_count(const uint64_t* keys, size_t count, int shift, uint32_t* head_cnt,
                      uint32_t* tail_cnt, uint64_t* masks, hipStream_t s);
size_t run_mask_words(size_t count);
// Writes start[c] / end[c] of run c (ordered by position) from the masks
// given the scanned per-tile offsets; or, with tot, given the raw per-tile
// counts (the kernel adds up the earlier tiles' counts itself, writes tot[0]
// = runs (heads), tot[1] = tails, and clears *zero if given).
void launch_run_write(const uint64_t* masks, size_t count, const uint32_t* head_off,
                      const uint32_t* tail_off, uint32_t* start, uint32_t* end, uint32_t* tot,
                      unsigned long long* zero, hipStream_t s);
// units[c] = work units of run c (see UnitDesc), tests[c] = L(L-1)/2, and
// *members += sum of L, for c < ncells (c < min(ncells, *dcells) when the
// device count dcells is given; ncells is then the host's bound).
void launch_cell_work(const uint32_t* start, const uint32_t* end, uint32_t ncells,
                      const uint32_t* dcells, uint32_t cell_unit_tiles, uint32_t* units,
                      uint64_t* tests, unsigned long long* members, hipStream_t s);
// launch_cell_work followed by the in-place exclusive scans of units and
// tests (totals to *utotal, *ttotal; usums / tsums hold one sum per 2048
// cells), in three launches, when ncells needs at most 2048 such sums;
// returns false, having launched nothing, otherwise.
bool launch_cell_work_scanned(const uint32_t* start, const uint32_t* end, uint32_t ncells,
                              const uint32_t* dcells, uint32_t cell_unit_tiles, uint32_t* units,
                              uint64_t* tests, unsigned long long* members, uint32_t* usums,
                              uint32_t* utotal, uint64_t* tsums, uint64_t* ttotal, hipStream_t s);
// A work unit of the pair kernels: the 64-point tiles ta in [ta_begin,
// ta_end) of a cell, each tested against the cell's tiles tb >= ta.  A cell
// of at most cell_unit_tiles tiles is one unit; a larger cell has one unit
// per tile.
struct UnitDesc {
  uint32_t s0;        // first sorted position of the cell
  uint32_t len;       // points in the cell
  uint32_t ta_begin;  // the unit's first A tile
  uint32_t ta_end;    // one past its last A tile
  uint32_t t;         // grid of the cell
  uint32_t inst;      // instance of the cell
  uint32_t pad[2];
};
// desc[unit_off[c] + q] for the units q of cell c; a cell's segment is
// sa + (its key >> seg_shift) (sa when seg_shift >= 64).
// work (optional) receives each unit's tile pairs.
void launch_unit_fill(const uint32_t* start, const uint32_t* end, const uint32_t* unit_off,
                      uint32_t ncells, const uint32_t* dcells, uint32_t cell_unit_tiles,
                      const uint64_t* skeys, int seg_shift, int sa, const SegDesc* segs,
                      UnitDesc* desc, uint64_t* work, hipStream_t s);

// --- cell pairs -----------------------------------------------------------
// Neighbourhood signatures for the first-owner rule, which keeps a pair
// found under grid t only if no grid t' < t put both points in one cell.
// Under grid t a point's group holds the low b bits of each axis field
// (kappa_j - origin_j), g = d b bits, at bit (t % gpw) g of word t / gpw of
// the point's W-word row.  For two points within r every axis differs by at
// most 2^b - 1 cells (b is at least the key packing's minimum field width),
// so equal groups mean equal cells.
//
// The pair kernels read every unit's points by sorted position: their
// coordinates spts[l][p] and signature words ssig[w][p], gathered once by
// launch_gather_units.  One 64-wide wave per unit emits packed pairs
// (min << pair_bits | max) for same-cell pairs within r.  The output has
// nseg segments of cap entries each (segment s at cand + s cap, taken by
// blocks b with b % nseg == s, so that the segments' counters are not all
// contended by every XCD); cand_count[s] is segment s's running total (it
// may exceed cap: then the overflow is only counted).  rechecks counts FP64
// band re-tests.
struct PairsArgs {
  const UnitDesc* units;
  uint32_t total_units;
  const float* spts;       // [d][N] unit points' coordinates by sorted position (direct == 0)
  const uint64_t* ssig;    // [W][N] their signature words (direct == 0 and first_owner)
  int first_owner;         // 1: keep a pair only under the first grid whose cell holds both
  size_t N;                // plane stride of spts / ssig
  int direct;              // 1: read rows by point index from pts / sigp instead
  const uint64_t* sigp;    // [npts][W] signature words by point (direct reads)
  const uint64_t* skeys;   // sorted keys
  const uint32_t* sidx;    // sorted point indices (null when in skeys)
  int idx_bits;            // > 0: point index in the low idx_bits of skeys
  const float* pts;        // batch points, row-major [npts][d] (FP64 band re-test)
  const float* rows;       // tile loads (direct): point i's coordinates at rows + i row_stride
  int row_stride;
  int sig_stride;          // words from point i's signature (sigp) to point i + 1's
  int d;
  const PairTest* tests;   // per instance
  int W, g, gpw;           // signature layout
  uint64_t lows, highs;    // lowest and highest bit of each signature group
  uint64_t* cand;
  uint64_t cap;            // entries per segment
  unsigned long long *cand_count, *rechecks;  // cand_count: [nseg]
  uint32_t nseg;           // output segments (0 or 1: one)
  int gram;                // 1: matrix-core screen (d <= 16), 0: vector screen
  // 1: every unit holds the points of one grid cell (no two cells share a
  // key), so the matrix-core screen may take its band from tests[].s_bound
  int unit_band;
  uint32_t max_blocks;     // grid size cap (0: default)
  // [pair_waves + 1]: wave w takes units [wave_first[w], wave_first[w + 1])
  // (launch_wave_ranges); null: every pair_waves-th unit from its own index
  const uint32_t* wave_first;
};
// Waves of the pair kernels' grid for these arguments.
uint32_t pair_waves(const PairsArgs& a);
// first[0..nwaves] from the exclusive prefix work_off of the units' tile
// pairs (total their sum, on the device): contiguous runs of units with
// about equal work.
void launch_wave_ranges(const uint64_t* work_off, uint32_t nunits, const uint64_t* total,
                        uint32_t nwaves, uint32_t* first, hipStream_t s);
// --- MR-metric filter -----------------------------------------------------
// Under the MR-metric (the sum of the robots' Euclidean displacements, each
// robot a block of sub consecutive axes) the pair kernels run the Euclidean
// test with a radius a little above r, which keeps every MR neighbour, and
// this pass keeps the packed pairs (a << pair_bits | b) whose MR distance is
// at most r.  The instance of a pair is the last one with pt_off <= a; pairs
// of Euclidean instances (sub == 0) are kept as they are.  Kept pairs are
// appended to out in no particular order; out_count must start at zero.
struct MrInst {
  int64_t pt_off;  // first row of the instance
  double r;
  int32_t sub;     // axes per robot; 0: Euclidean instance
  int32_t pad;
};
struct MrFilterArgs {
  const uint64_t* in;
  uint64_t count;
  int pair_bits;
  int d;
  const float* rows_a;  // row-major [.][d]: rows of the pairs' first indices
  const float* rows_b;  // and of their second indices
  const MrInst* inst;   // [m], pt_off ascending, inst[0].pt_off = 0
  int m;
  uint64_t* out;        // room for count pairs
  unsigned long long* out_count;
};
void launch_mr_filter(const MrFilterArgs& a, hipStream_t s);

// --- bitmap de-duplication --------------------------------------------------
// Keeps the first arrival of each packed pair (a << pair_bits | b, a < b, both
// in the instance with the last pt_off <= a): instance q owns bits
// [bit_off, bit_off + n (n - 1) / 2) of bits, the pair of local indices
// a' < b' bit b'(b'-1)/2 + a'.  bits must start at zero; kept pairs are
// appended to out in no particular order; out_count must start at zero.
struct BitmapInst {
  int64_t pt_off;
  int64_t bit_off;
};
struct BitmapArgs {
  const uint64_t* in;
  uint64_t count;
  int pair_bits;
  int m;
  const BitmapInst* inst;  // [m], pt_off ascending, inst[0].pt_off = 0
  uint32_t* bits;
  uint64_t* out;           // room for count pairs
  unsigned long long* out_count;
};
void launch_bitmap_unique(const BitmapArgs& a, hipStream_t s);

// --- query mode -------------------------------------------------------------
// One sorted grid of an index: its n sorted keys (cell prefix above the point
// index when the keys carry it) and the grid's segment id within its sort.
struct QueryGrid {
  const uint64_t* keys;
  const uint32_t* idx;  // point indices when the keys do not carry them
  uint64_t seg;
  int32_t idx_bits;     // > 0: the point index in the low idx_bits of the keys
  int32_t pad;
};
struct QueryArgs {
  const float* queries;     // [m][d] row-major
  int64_t m;
  int d, k;
  const double *R, *u;      // [k][d][d], [k][d]
  double inv_c, r2;
  const int64_t* klo;       // [k][d] field origins
  const KeyLayout* layout;
  int cell_bits;            // packed cell bits of the index's keys
  const QueryGrid* grids;   // [k]
  int64_t n;                // indexed points
  const float* pts;         // [n][d] indexed points
  const uint64_t* sig;      // [n][W] their signatures (null: no first-owner rule)
  int W, sig_b, g, gpw;
  uint64_t lows, highs;
  uint64_t* qkey;           // [m][k] cell prefix of each query under each grid
  uint64_t* qsig;           // [m][W] signature words of each query
  uint32_t* err;            // bit 0: a cell coordinate out of range, bit 1: not finite
  int pb;                   // bits of an index in a packed (query, point) pair
  uint64_t* cand;
  uint64_t cap;
  unsigned long long* cand_count;
};
void launch_query_keys(const QueryArgs& a, hipStream_t s);
void launch_query_pairs(const QueryArgs& a, hipStream_t s);

// spts / ssig for the positions of every unit, from the batch rows and the
// per-point signatures sig [npts][W] (ssig untouched when sig is null).
void launch_gather_units(const PairsArgs& a, const uint64_t* sig, float* spts, uint64_t* ssig,
                         hipStream_t s);
void launch_cell_pairs(const PairsArgs& a, hipStream_t s);

// --- small instances --------------------------------------------------------
// One instance of n <= kTinyPoints points (d <= 8, n d <= kTinyFloats,
// k n <= kTinyCells, k d (d + 1) <= kTinyTransform) in two launches:
// TinyArgs::parts workgroups per grid each find the grid's cells (32-bit
// keys, sorted in LDS), test their share of its pairs in FP64 and append
// the pairs of the first grid that holds both points to pairs; workgroups
// of 512 rows each build the CSR lists from them.
constexpr int kTinyPoints = 4096;
constexpr int kTinyFloats = 12288;    // n d at most (the points are staged in LDS)
constexpr int kTinyTransform = 2048;  // k d (d + 1) at most (the transforms too)
constexpr int kTinyCells = 12288;     // k n at most (every grid's packed cells)
constexpr int kTinyBinBits = 12;      // counting sort up to 2^12 cells, else bitonic
constexpr int kTinyBins = 1 << kTinyBinBits;
constexpr int kTinyListLds = 32768;   // list entries built in LDS (more: in stage)
constexpr uint64_t kTinyPairCap = 131072;
constexpr uint32_t kTinyMaxDeg = 128;
struct TinyArgs {
  const float* pts;           // [n][d] FP32
  int n;
  double r2, inv_c;           // r^2; 1 / (alpha r)
  const double* R;            // [k][d][d]
  const double* u;            // [k][d]
  int k;
  uint32_t parts;             // workgroups per grid, each testing a slice of its pairs
  uint64_t* pairs;            // [cap]: (min << 32) | max
  uint64_t cap;
  unsigned long long* count;  // [0] pairs, [1] tests, [2] cells, [3] entries written
  uint32_t* err;              // bits: 1 non-finite point, 2 cell out of range,
                              // 4 key wider than 31 bits, 8 row over kTinyMaxDeg
  int upper;                  // 1: one orientation
  int64_t* row_ptr;           // [n + 1]
  int32_t* col;               // [2 cap]
  int32_t* stage;             // [2 cap]: the entries before their rows are ordered
};
void launch_tiny(const TinyArgs& a, int d, int k, hipStream_t s);
// dst[0, sum cnt) = the segments' entries in segment order: segment s holds
// src[s seg_cap, s seg_cap + cnt[s]).  dst must not overlap src.
void launch_seg_compact(const uint64_t* src, uint64_t seg_cap, const unsigned long long* cnt,
                        uint32_t nseg, uint64_t max_count, uint64_t* dst, hipStream_t s);

// --- unique + CSR -----------------------------------------------------------
void launch_unique_count(const uint64_t* keys, size_t count, uint32_t* tile_cnt, hipStream_t s);
void launch_unique_write(const uint64_t* keys, size_t count, const uint32_t* tile_off,
                         uint64_t* out, hipStream_t s);
// swapped[p] = (j << b) | i for pairs[p] = (i << b) | j.
void launch_swap_pairs(const uint64_t* pairs, size_t count, int pair_bits, uint64_t* swapped,
                       hipStream_t s);
// For a key array sorted by row (row = key >> pair_bits): rstart[row] = first
// position, rend[row] = one past the last (untouched rows keep their value).
void launch_row_runs(const uint64_t* keys, size_t count, int pair_bits, uint32_t* rstart,
                     uint32_t* rend, hipStream_t s);
// deg[i] = (lo_end - lo_start) + (up_end - up_start); lo_* may be null.
void launch_row_degree(const uint32_t* lo_start, const uint32_t* lo_end, const uint32_t* up_start,
                       const uint32_t* up_end, int64_t n, uint64_t* deg, hipStream_t s);
// col[row_ptr[i] + lo_cnt(i) + (p - up_start[i])] = j for upper entries, and
// col[row_ptr[j] + (q - lo_start[j])] = i for the swapped entries.
void launch_csr_fill_upper(const uint64_t* up, size_t count, int pair_bits, const int64_t* row_ptr,
                           const uint32_t* lo_start, const uint32_t* lo_end,
                           const uint32_t* up_start, int32_t* col, hipStream_t s);
void launch_csr_fill_lower(const uint64_t* lo, size_t count, int pair_bits, const int64_t* row_ptr,
                           const uint32_t* lo_start, int32_t* col, hipStream_t s);

// --- neighbour lists by row buckets -------------------------------------------
// Directed entries of the pairs (both orientations when both != 0) go to
// buckets of 2^rb rows (rb <= 11) as 32-bit keys (row mod 2^rb) << pb | col
// (needs rb + pb <= 32).  Blocks take `chunk` pairs each; part / offs are
// [nbuckets][nblocks] counts / their exclusive scan (bucket-major).
constexpr int kBucketMaxEntries = 16384;  // entries one block holds in LDS
constexpr int kBucketMaxRows = 1024;      // rows per bucket (rb <= 10)
// threads: block size of the two partition kernels (256 or 1024).  The
// pairs are one array of count entries (nseg = 0), or the pair kernels' nseg
// output segments as they left them (segment s at pairs + s seg_cap with
// seg_cnt[s] entries on the device; count their total, nblocks a multiple of
// nseg).
struct PairSource {
  const uint64_t* pairs;
  const unsigned long long* seg_cnt = nullptr;
  uint64_t seg_cap = 0;
  uint32_t nseg = 0;
};
// Also clears *zero_word (when given): the oversized count of the CSR step.
void launch_bucket_hist(const PairSource& src, size_t count, int pb, int rb, int both,
                        uint32_t nbuckets, uint32_t chunk, uint32_t nblocks, int threads,
                        uint32_t* part, uint32_t* zero_word, hipStream_t s);
void launch_bucket_scatter(const PairSource& src, size_t count, int pb, int rb, int both,
                           uint32_t nbuckets, uint32_t chunk, uint32_t nblocks, int threads,
                           const uint32_t* offs, uint32_t* entries, hipStream_t s);
// Writes col and row_ptr (row_ptr[n] = nnz) for every bucket of at most
// cap (<= kBucketMaxEntries) entries: entries of unique pairs, so a bucket's
// start in the entry array is its start in col.  Larger buckets, and
// buckets with a row of more than 1024 entries, are listed in oversized[]
// (count in *n_oversized, cleared beforehand) for the caller.
void launch_bucket_csr(const uint32_t* entries, const uint32_t* offs, uint32_t nbuckets,
                       uint32_t nblocks, const uint32_t* total, uint32_t* oversized,
                       uint32_t* n_oversized, uint32_t cap, int pb, int rb, int64_t n,
                       int64_t nnz, int64_t* row_ptr, int32_t* col, hipStream_t s);
// Every oversized bucket at once: ids[q] (q < nover) are their bucket ids.
// launch_over_extent gives each one's first entry and entry count (part is
// the scanned partition table, part[np] its total); with off the exclusive
// scan of cnt and tot its sum, launch_over_gather tags each entry with q
// above bit sh = rb + pb, and launch_over_emit writes col and row_ptr from
// those keys sorted on bits [0, sh + bits of q).
void launch_over_extent(const uint32_t* ids, uint32_t nover, const uint32_t* part,
                        uint32_t nblocks, uint32_t nbuckets, size_t np, uint32_t* start,
                        uint32_t* cnt, hipStream_t s);
void launch_over_gather(const uint32_t* entries, const uint32_t* start, const uint32_t* off,
                        uint32_t nover, uint32_t tot, int sh, uint64_t* w, hipStream_t s);
void launch_over_emit(const uint64_t* keys, uint32_t tot, const uint32_t* ids,
                      const uint32_t* start, const uint32_t* cnt, const uint32_t* off, int pb,
                      int rb, int64_t n, int64_t* row_ptr, int32_t* col, hipStream_t s);

void launch_u32_to_u64(const uint32_t* src, size_t count, uint64_t* dst, hipStream_t s);

// --- memory for callers that cannot allocate ----------------------------------
// Bytes of the file-scope device array that rtg_all_pairs_noalloc takes all
// of its device memory from (one copy per device, held until the process
// ends).
constexpr size_t kNoallocBytes = size_t(256) << 20;
// That array's address on the current device (hipGetSymbolAddress); 0 on
// success, else the HIP error code (*ptr is then null).
int noalloc_scratch_address(void** ptr);

// --- per-instance lists of a batch ------------------------------------------
// out[q] = row_ptr[first batch point of instance q], out[m] = row_ptr[npts].
void launch_rowptr_at(const InstDesc* inst, uint32_t m, const int64_t* row_ptr, int64_t npts,
                      int64_t* out, hipStream_t s);
// Instance q's rows of the batch lists into out_rp[q] (n+1) / out_col[q],
// with row starts and column indices local to the instance (device pointer
// tables); at = launch_rowptr_at's output, total = at[m] entries.
void launch_localize(const InstDesc* inst, uint32_t m, uint32_t nblocks, const int64_t* row_ptr,
                     const int32_t* col, const int64_t* at, int64_t total, int64_t* const* out_rp,
                     int32_t* const* out_col, hipStream_t s);

}  // namespace rtgk
