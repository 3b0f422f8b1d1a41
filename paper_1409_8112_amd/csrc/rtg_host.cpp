// rtg_host.cpp -- host side of the RTG library: C-ABI, context, device-memory
// arena, transform generator, key-packing plan and the pipeline that drives
// the gfx950 kernels (rtg_kernels.hip).
#include "../../include/rtg.h"
#include "rtg_internal.h"
#include "rtg_runtime.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

using namespace rtgk;

namespace rtg {

// ---------------------------------------------------------------------------
// transforms: SplitMix64 (Steele, Lea & Flood 2014) streams, uniform shifts,
// Gaussian rows by Marsaglia's polar method, rows orthonormalised by modified
// Gram-Schmidt applied twice.

namespace {

struct SplitMix64 {
  uint64_t state;
  uint64_t next() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double unit() { return (double)(next() >> 11) * 0x1p-53; }
};

void polar_normals(SplitMix64& g, double* out2) {
  for (;;) {
    const double a = 2.0 * g.unit() - 1.0;
    const double b = 2.0 * g.unit() - 1.0;
    const double s = a * a + b * b;
    if (s < 1.0 && s != 0.0) {
      const double f = std::sqrt(-2.0 * std::log(s) / s);
      out2[0] = a * f;
      out2[1] = b * f;
      return;
    }
  }
}

}  // namespace

int make_transforms(uint64_t seed, int32_t k, int32_t d, uint32_t flags, double* R, double* u) {
  if (k < 1 || d < 1 || d > kMaxDim || !R || !u) return RTG_EINVAL;
  std::vector<double> gauss((size_t)d * d + 1);
  SplitMix64 parent{seed};
  for (int32_t t = 0; t < k; ++t) {
    SplitMix64 g{parent.next()};  // stream t starts at the (t+1)-th output of seed
    double* ut = u + (size_t)t * d;
    double* Rt = R + (size_t)t * d * d;
    for (int32_t j = 0; j < d; ++j) ut[j] = g.unit();
    if (flags & RTG_NO_ROTATE) {
      for (int32_t a = 0; a < d; ++a)
        for (int32_t b = 0; b < d; ++b) Rt[(size_t)a * d + b] = (a == b) ? 1.0 : 0.0;
      continue;
    }
    const int32_t dd = d * d;
    for (int32_t e = 0; e < dd; e += 2) polar_normals(g, &gauss[e]);
    for (int32_t row = 0; row < d; ++row) {
      double* v = &gauss[(size_t)row * d];
      for (int sweep = 0; sweep < 2; ++sweep) {
        for (int32_t prev = 0; prev < row; ++prev) {
          const double* q = Rt + (size_t)prev * d;
          double dot = 0.0;
          for (int32_t l = 0; l < d; ++l) dot = dot + v[l] * q[l];
          for (int32_t l = 0; l < d; ++l) v[l] = v[l] - dot * q[l];
        }
      }
      double nrm2 = 0.0;
      for (int32_t l = 0; l < d; ++l) nrm2 = nrm2 + v[l] * v[l];
      const double nrm = std::sqrt(nrm2);
      if (!(nrm > 0.0)) return RTG_ERANGE;
      for (int32_t l = 0; l < d; ++l) Rt[(size_t)row * d + l] = v[l] / nrm;
    }
  }
  return RTG_OK;
}

// ---------------------------------------------------------------------------
// arena

Arena::Arena(char* base, size_t bytes) {
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  const uintptr_t a = (b + kAlign - 1) & ~(uintptr_t)(kAlign - 1);
  base_ = reinterpret_cast<char*>(a);
  size_ = bytes > (a - b) ? (bytes - (a - b)) & ~(size_t)(kAlign - 1) : 0;
  if (size_) add_free(0, size_);
}

void Arena::add_free(size_t off, size_t len) {
  free_[off] = len;
  by_size_.emplace(len, off);
}

void Arena::drop_free(std::map<size_t, size_t>::iterator it) {
  auto range = by_size_.equal_range(it->second);
  for (auto s = range.first; s != range.second; ++s)
    if (s->second == it->first) {
      by_size_.erase(s);
      break;
    }
  free_.erase(it);
}

void* Arena::alloc(size_t bytes) {
  bytes = std::max<size_t>(bytes, 1);
  bytes = (bytes + kAlign - 1) & ~(size_t)(kAlign - 1);
  auto s = by_size_.lower_bound(bytes);  // the smallest free block that fits
  if (s == by_size_.end()) return nullptr;
  const size_t off = s->second, len = s->first;
  by_size_.erase(s);
  free_.erase(off);
  if (len > bytes) add_free(off + bytes, len - bytes);
  used_[off] = bytes;
  in_use_ += bytes;
  peak_ = std::max(peak_, in_use_);
  return base_ + off;
}

void Arena::release(void* p) {
  if (!p) return;
  const size_t off = (size_t)(static_cast<char*>(p) - base_);
  auto u = used_.find(off);
  if (u == used_.end()) return;
  size_t start = off, len = u->second;
  in_use_ -= len;
  used_.erase(u);
  auto next = free_.lower_bound(start);
  if (next != free_.end() && start + len == next->first) {
    len += next->second;
    drop_free(next);
  }
  auto prev = free_.lower_bound(start);
  if (prev != free_.begin()) {
    --prev;
    if (prev->first + prev->second == start) {
      start = prev->first;
      len += prev->second;
      drop_free(prev);
    }
  }
  add_free(start, len);
}

void Arena::shrink(void* p, size_t bytes) {
  if (!p) return;
  const size_t off = (size_t)(static_cast<char*>(p) - base_);
  auto u = used_.find(off);
  if (u == used_.end()) return;
  bytes = (std::max<size_t>(bytes, 1) + kAlign - 1) & ~(size_t)(kAlign - 1);
  if (bytes >= u->second) return;
  const size_t tail = u->second - bytes;
  u->second = bytes;
  in_use_ -= tail;
  size_t start = off + bytes, len = tail;
  auto next = free_.lower_bound(start);
  if (next != free_.end() && start + len == next->first) {
    len += next->second;
    drop_free(next);
  }
  add_free(start, len);
}

size_t Arena::largest_free() const { return by_size_.empty() ? 0 : by_size_.rbegin()->first; }

// ---------------------------------------------------------------------------
// helpers

namespace {

int ceil_log2(uint64_t x) {
  int b = 0;
  while (b < 64 && (1ull << b) < x) ++b;
  return b;
}

// FP32 thresholds of the screen: lo <= r2 (1 - 2^-16) <= r2 (1 + 2^-16) <= hi.
// The FP32 sum of d <= 64 squared FP32 differences is within a relative
// (d + 2) 2^-24 < 2^-17.9 of the exact value, and the FP64 sum within
// (d + 2) 2^-53, so a value at or below lo is within r in FP64 and a value
// above hi is not; only the band between is re-tested in FP64.
//
// s_bound: two points of one cell of side c lie within its diagonal, so
// |a - b|^2 <= d c^2 (the cell coordinates floor(R p / c + u) agree; R is
// orthogonal and the FP64 rounding of R p / c + u is far below the 2^-10
// margin, which also covers the FP32 centring and norms).  With o a point
// of the cell, |a - o|^2 + |b - o|^2 <= 2 d c^2.
PairTest make_pair_test(double r2, int pair_bits, int d, double cell_side) {
  PairTest t;
  const double sb = 2.0 * d * cell_side * cell_side * (1.0 + 0x1p-10);
  t.s_bound = (sb < 0x1p100) ? (float)sb : 0.0f;
  const double lo_d = r2 * (1.0 - 0x1p-16);
  float lo = (float)lo_d;
  if ((double)lo > lo_d) lo = std::nextafter(lo, -INFINITY);
  const double hi_d = r2 * (1.0 + 0x1p-16);
  float hi = (float)hi_d;
  if ((double)hi < hi_d) hi = std::nextafter(hi, INFINITY);
  t.lo = lo;
  t.hi = hi;
  t.r2 = r2;
  t.pair_bits = pair_bits;
  return t;
}

// The squared radius of the Euclidean test that finds the candidates of an
// MR-metric query.  A pair within r under the MR-metric in FP64 has
// Euclidean distance at most its exact MR distance (triangle inequality),
// which is at most r (1 + (2 d + 4) 2^-53); its FP64 squared distance is then
// at most r*r (1 + (5 d + 12) 2^-53) < r*r (1 + 2^-40) for d <= 64, so the
// Euclidean test against this radius keeps every MR neighbour.
double mr_screen_r2(double r) {
  const double x = (r * r) * (1.0 + 0x1p-40);
  return std::nextafter(x, INFINITY);
}

// The volume of the d-ball of radius r over that of the cube of side
// alpha r: no more than this share of the pairs of points that share a cell
// lie within r of each other (the cube's edges only lower the share).
double ball_share(int d, double alpha) {
  const double v = std::pow(M_PI, 0.5 * d) / std::tgamma(0.5 * d + 1.0);
  return std::min(1.0, v / std::pow(alpha, d));
}

// Whether the matrix-core pair screen suits an instance: its band, relative
// to r^2, is about (2K + d + 8) * 1.5 * 2^-24 * 2 d alpha^2 for cells of side
// alpha r (K = d + 2 rounded up to even); up to 2^-8 it sends few pairs to
// FP64.  Wider bands stay exact but slow, so they take the vector screen.
bool gram_suits(int d, double alpha) {
  if (d > 16) return false;
  const int K = (d + 3) & ~1;
  const double band = 1.5 * (2.0 * K + d + 8) * 0x1p-24 * 2.0 * d * alpha * alpha;
  return band <= 0x1p-8;
}

float decode_order(uint32_t e) {
  const uint32_t b = (e & 0x80000000u) ? (e & 0x7FFFFFFFu) : ~e;
  float f;
  std::memcpy(&f, &b, 4);
  return f;
}

}  // namespace

// Smallest field width b >= 1 such that two points whose cells coincide in
// the low b bits of some axis but differ on that axis are more than r apart:
// they differ by >= 2^b cells, so ||p - q|| >= (2^b - 1 - eps) alpha r with
// eps < 1e-3 covering FP64 rounding of y for |y| < 2^31; (2^b - 1.001) alpha
// >= 1.001 then puts them beyond r with margin, and such pairs are rejected.
int min_field_bits(double alpha) {
  for (int b = 1; b <= 32; ++b)
    if ((std::ldexp(1.0, b) - 1.001) * alpha >= 1.001) return b;
  return 33;
}

uint64_t cand_per_key(uint32_t flags) {
  // First owner: every pair once, about nu / (2k) per key at nu neighbours.
  // Sort-unique and bitmap keep every grid's repeats until the union.
  return (flags & (RTG_DEDUP_SORT | RTG_DEDUP_BITMAP)) ? 8 : 4;
}

size_t Ctx::pass_bytes_bound(int64_t n, int32_t d, int32_t k, double alpha, uint32_t flags) const {
  const double N = (double)n * (double)k;
  const int b = std::min(32, min_field_bits(alpha));
  const int g = d * b;
  const int gpw = g <= 64 ? 64 / g : 1;
  const double W = (double)((k + gpw - 1) / gpw);
  const double rs = (double)((d + 2 + 3) & ~3);
  // per point: SoA and concatenated rows, bounding-box partials, point
  // records or signature rows
  double bytes = (double)n * (8.0 * d + d / 32.0 + std::max(4.0 * rs, 8.0 * W) + 16.0);
  // per key: two key buffers and two value buffers (worst case), cell
  // starts / ends / unit counts (6), unit descriptors (16.5), cell tests (4),
  // unit work and its scan (4.2 + 0.1), cell head and tail bits (0.25),
  // sort and scan scratch (1)
  bytes += N * (16.0 + 8.0 + 6.0 + 16.5 + 4.0 + 4.3 + 0.25 + 1.0);
  if (!gather_direct) bytes += N * (4.0 * d + 8.0 * W);
  // candidates: the pair kernels' segments (a quarter to spare) and the
  // compacted copy, then the list build (entries and the result) after the
  // key buffers are gone -- the larger of the two phases
  const double C = (double)cand_per_key(flags) * N;
  bytes += std::max(8.0 * 1.25 * C + 8.0 * kCandSegments * 1024 + 8.0 * C,
                    8.0 * C + 8.0 * C + 12.0 * 2.0 * C + 8.0 * (double)n);
  if (flags & RTG_DEDUP_BITMAP)
    bytes += std::min((double)kBitmapMaxBytes, (double)n * (double)(n - 1) / 16.0);
  // transforms, descriptors, tables, alignment
  bytes += 8.0 * k * d * (d + 2) + (double)(2 << 20);
  return (size_t)bytes;
}

int plan_batch(int d, uint32_t m, const int64_t* k, const int64_t* n, const double* R,
               const double* u, const double* inv_c, const double* alpha, const float* lo,
               const float* hi, size_t budget_bytes, Packing& P) {
  int64_t S_total = 0, nmax = 0, elems_all = 0;
  for (uint32_t q = 0; q < m; ++q) {
    S_total += k[q];
    nmax = std::max(nmax, n[q]);
    elems_all += n[q] * k[q];
  }
  std::vector<int> need(d, 1);
  P.klo.assign((size_t)S_total * d, 0);
  P.wrapped = false;
  int bmin = 1;
  int64_t tr = 0;
  for (uint32_t q = 0; q < m; ++q) {
    bmin = std::max(bmin, min_field_bits(alpha[q]));
    const float* lq = lo + (size_t)q * d;
    const float* hq = hi + (size_t)q * d;
    for (int64_t t = 0; t < k[q]; ++t, ++tr) {
      for (int j = 0; j < d; ++j) {
        const double* Rj = R + ((size_t)tr * d + j) * d;
        double zlo = 0.0, zhi = 0.0;
        for (int l = 0; l < d; ++l) {
          const double a = Rj[l] * (double)lq[l], b = Rj[l] * (double)hq[l];
          zlo += std::min(a, b);
          zhi += std::max(a, b);
        }
        const double ylo = zlo * inv_c[q] + u[(size_t)tr * d + j];
        const double yhi = zhi * inv_c[q] + u[(size_t)tr * d + j];
        int bits = 32;
        int64_t klo = 0;
        if (std::fabs(ylo) < 0x1p31 && std::fabs(yhi) < 0x1p31) {
          // one cell of slack on each side covers the rounding of y
          klo = (int64_t)std::floor(ylo) - 1;
          const int64_t khi = (int64_t)std::floor(yhi) + 1;
          bits = std::max(1, ceil_log2((uint64_t)(khi - klo + 1)));
        } else {
          P.wrapped = true;  // 32-bit fields of cell coordinates beyond 2^31
        }
        P.klo[(size_t)tr * d + j] = klo;
        need[j] = std::max(need[j], std::min(bits, 32));
      }
    }
  }
  if (bmin > 32) return RTG_ERANGE;
  for (int j = 0; j < d; ++j) need[j] = std::max(need[j], bmin);

  // Segments per pass: as many as the key bits, the 32-bit element index of
  // the sort and the memory budget allow.
  int64_t tb = S_total;
  for (;;) {
    const int seg_bits = tb > 1 ? ceil_log2((uint64_t)tb) : 0;
    const int avail = 64 - seg_bits;
    std::vector<int> b = need;
    int total = 0;
    for (int j = 0; j < d; ++j) total += b[j];
    // Narrow the widest fields first, never below bmin.
    while (total > avail) {
      int jw = -1;
      for (int j = 0; j < d; ++j)
        if (b[j] > bmin && (jw < 0 || b[j] > b[jw])) jw = j;
      if (jw < 0) break;
      --b[jw];
      --total;
    }
    const uint64_t elems = (uint64_t)std::min<int64_t>(elems_all, tb * nmax);
    const size_t bytes = (size_t)elems * 28;  // two key/value buffers + cells
    const bool fits = total <= avail && elems < (1ull << 32) && (bytes <= budget_bytes || tb == 1);
    if (fits) {
      P.tb = (int)tb;
      P.seg_bits = seg_bits;
      P.layout.d = d;
      P.layout.cell_bits = total;
      int sh = 0;
      P.truncated = false;
      for (int j = 0; j < d; ++j) {
        P.layout.shift[j] = (uint8_t)sh;
        P.layout.bits[j] = (uint8_t)b[j];
        if (b[j] < need[j]) P.truncated = true;
        sh += b[j];
      }
      P.key_bits = total + seg_bits;
      return RTG_OK;
    }
    if (tb == 1) return total > avail ? RTG_ERANGE : RTG_ENOMEM;
    tb = (tb + 1) / 2;
  }
}

// ---------------------------------------------------------------------------
// context

Ctx::Ctx(int dev) : device(dev) {
  // Reduce-then-scan is the default radix sort: on MI355X its per-pass
  // histogram + scan + scatter beat onesweep, whose look-back reads cross
  // the XCDs' L2s.  RTG_SORT=onesweep selects onesweep.
  const char* e = std::getenv("RTG_SORT");
  defaults.sort_algo = (e && std::strcmp(e, "onesweep") == 0) ? kSortOnesweep : kSortReduceScan;
  // RTG_BATCH_POINTS lowers the points per batch of rtg_all_pairs_batched
  // and of the request loop (tests use it to split small batches).
  const char* bp = std::getenv("RTG_BATCH_POINTS");
  batch_points = kBatchPoints;
  if (bp) {
    const long long v = std::strtoll(bp, nullptr, 10);
    if (v >= 2 && v < kBatchPoints) batch_points = v;
  }
  // RTG_PAIRS: "vector" forces the vector pair screen, "matrix" the
  // matrix-core one wherever d <= 16 (default: matrix cores where they suit).
  if (const char* e = std::getenv("RTG_PAIRS")) {
    if (std::strcmp(e, "vector") == 0) pair_screen = 1;
    if (std::strcmp(e, "matrix") == 0) pair_screen = 2;
  }
  // RTG_BAND: "tile" makes the matrix-core screen bound its FP32 band by each
  // tile pair's largest norms instead of the cell diagonal (narrower band,
  // fewer FP64 re-tests, two wave reductions per tile pair).
  if (const char* e = std::getenv("RTG_BAND")) unit_band = std::strcmp(e, "tile") != 0;
  // RTG_SMALL=0: small instances take the general pipeline too.
  if (const char* e = std::getenv("RTG_SMALL")) small_path = std::strcmp(e, "0") != 0;
  // RTG_GATHER: "sorted" makes the pair kernels read a copy of the cell
  // members' rows gathered in sorted order instead of the rows by index.
  if (const char* e = std::getenv("RTG_GATHER")) gather_direct = std::strcmp(e, "sorted") != 0;
  // RTG_UNIT_TILES: cells of at most this many 64-point tiles are one work
  // unit of the pair kernels (larger cells: one unit per tile).
  if (const char* e = std::getenv("RTG_UNIT_TILES"))
    defaults.unit_tiles = (uint32_t)std::max(1, std::min(64, std::atoi(e)));
  // RTG_PAIR_BLOCKS: grid size of the pair kernels (default: from the work).
  if (const char* e = std::getenv("RTG_PAIR_BLOCKS"))
    pair_blocks = (uint32_t)std::max(1, std::min(1 << 20, std::atoi(e)));
  // RTG_LANES: passes of the request loop that may run at once (1..4).
  if (const char* e = std::getenv("RTG_LANES"))
    server_lanes = std::max(1, std::min(4, std::atoi(e)));
  // RTG_BUCKET_CAP lowers the entries a neighbour-list bucket may hold in
  // LDS (tests use it to send buckets down the global-sort fallback).
  const char* bc = std::getenv("RTG_BUCKET_CAP");
  if (const char* e = std::getenv("RTG_BUCKET_BLOCKS"))
    defaults.bucket_blocks = (uint32_t)std::max(1, std::min(4096, std::atoi(e)));
  if (const char* e = std::getenv("RTG_BATCH_LANES")) batch_lanes = std::max(1, std::min(3, std::atoi(e)));
  // RTG_PART_THREADS: block size of the neighbour-list partition kernels
  if (const char* e = std::getenv("RTG_PART_THREADS"))
    defaults.part_threads = std::atoi(e) >= 1024 ? 1024 : 256;
  if (const char* e = std::getenv("RTG_UNITS"))
    balanced_units = std::strcmp(e, "roundrobin") != 0;
  bucket_cap = kBucketMaxEntries;
  if (bc) {
    const long v = std::strtol(bc, nullptr, 10);
    if (v >= 1 && v < kBucketMaxEntries) bucket_cap = (uint32_t)v;
  }
}

Tuning Ctx::tuning_for(int d, int64_t npts) {
  std::lock_guard<std::mutex> lk(tmu);
  auto it = tuned.find({d, ceil_log2((uint64_t)std::max<int64_t>(npts, 1))});
  return it == tuned.end() ? defaults : it->second;
}

Ctx::~Ctx() {
  stop_server();
  for (auto& L : side) L->fini();
  if (side_ready) (void)hipEventDestroy(side_ready);
  main.fini();
  if (own_arena && arena_mem) (void)hipFree(arena_mem);
}

int Ctx::hip_fail(hipError_t e, const char* what) {
  if (e == hipSuccess) return RTG_OK;
  std::fprintf(stderr, "rtg: %s failed: %s\n", what, hipGetErrorString(e));
  poisoned = true;
  return RTG_EDEVICE;
}

void* Ctx::dalloc(size_t bytes) {
  std::lock_guard<std::mutex> lk(amu);
  return arena->alloc(bytes);
}

void* Ctx::dalloc_noalloc(size_t bytes) {
  std::lock_guard<std::mutex> lk(amu);
  return noalloc_arena ? noalloc_arena->alloc(bytes) : nullptr;
}

size_t Ctx::largest_free_noalloc() {
  std::lock_guard<std::mutex> lk(amu);
  return noalloc_arena ? noalloc_arena->largest_free() : 0;
}

Arena* Ctx::arena_of(const void* p) {
  const char* c = static_cast<const char*>(p);
  const char* b = static_cast<const char*>(noalloc_base);
  if (noalloc_arena && c >= b && c < b + kNoallocBytes) return noalloc_arena.get();
  return arena.get();
}

void Ctx::dfree(void* p) {
  std::lock_guard<std::mutex> lk(amu);
  arena_of(p)->release(p);
}

void Ctx::dshrink(void* p, size_t bytes) {
  std::lock_guard<std::mutex> lk(amu);
  arena_of(p)->shrink(p, bytes);
}

size_t Ctx::largest_free() {
  std::lock_guard<std::mutex> lk(amu);
  return arena->largest_free();
}

size_t Ctx::free_bytes() {
  std::lock_guard<std::mutex> lk(amu);
  return arena->size() - arena->in_use();
}

uint64_t Ctx::new_handle() {
  std::lock_guard<std::mutex> lk(amu);
  return next_handle++;
}

uint64_t Ctx::keep_result(uint64_t h, void* mem, int64_t n, int64_t nnz, int64_t pairs,
                          int64_t* row_ptr, int32_t* col) {
  std::lock_guard<std::mutex> lk(amu);
  if (!h) h = next_handle++;
  results[h] = Result{mem, n, nnz, pairs, row_ptr, col};
  return h;
}

int Ctx::release_many(const uint64_t* handles, int32_t count) {
  int rc = RTG_OK;
  bool any = false;
  {
    std::lock_guard<std::mutex> lk(amu);
    for (int32_t i = 0; i < count; ++i) {
      auto it = results.find(handles[i]);
      if (it != results.end()) {
        arena_of(it->second.mem)->release(it->second.mem);
        results.erase(it);
        any = true;
        continue;
      }
      auto ix = indexes.find(handles[i]);
      if (ix == indexes.end()) {
        rc = RTG_ENOENT;
        continue;
      }
      for (void* p : ix->second->blocks) arena->release(p);
      indexes.erase(ix);
      any = true;
    }
  }
  if (any) wake_server();
  return rc;
}

int Ctx::release(uint64_t h) { return release_many(&h, 1); }

bool Ctx::holds_results() {
  std::lock_guard<std::mutex> lk(amu);
  return !results.empty() || !indexes.empty();
}

bool Ctx::find_result(uint64_t h, rtg_csr* out) {
  std::lock_guard<std::mutex> lk(amu);
  auto it = results.find(h);
  if (it == results.end()) return false;
  out->n = it->second.n;
  out->nnz = it->second.nnz;
  out->row_ptr = it->second.row_ptr;
  out->col = it->second.nnz ? it->second.col : nullptr;
  out->pairs = it->second.pairs;
  out->handle = h;
  return true;
}

// ---------------------------------------------------------------------------
// lanes

int Lane::init(Ctx* c, hipStream_t s, bool create_stream) {
  ctx = c;
  stream = s;
  if (create_stream) {
    // default priority (streams of different priorities are avoided)
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return RTG_EDEVICE;
    own_stream = true;
  }
  if (hipHostMalloc(&host_stage, 4096) != hipSuccess) return RTG_EDEVICE;
  host_stage_bytes = 4096;
  if (hipHostMalloc(&host_up, 65536) != hipSuccess) return RTG_EDEVICE;
  host_up_bytes = 65536;
  if (hipEventCreateWithFlags(&up_done, hipEventDisableTiming) != hipSuccess) return RTG_EDEVICE;
  if (hipHostMalloc((void**)&mail, kMailBytes + 256) != hipSuccess) return RTG_EDEVICE;
  mail[0] = 0;
  gather_dev = c->dalloc(64);
  if (!gather_dev) return RTG_ENOMEM;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) return RTG_EDEVICE;
  return RTG_OK;
}

void Lane::fini() {
  if (stream || own_stream) (void)hipStreamSynchronize(stream);
  if (host_stage) (void)hipHostFree(host_stage);
  host_stage = nullptr;
  if (host_up) (void)hipHostFree(host_up);
  host_up = nullptr;
  if (mail) (void)hipHostFree(mail);
  mail = nullptr;
  if (up_done) (void)hipEventDestroy(up_done);
  up_done = nullptr;
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : kev) (void)hipEventDestroy(e);
  kev.clear();
  if (gather_dev && ctx) ctx->dfree(gather_dev);
  gather_dev = nullptr;
  if (own_stream) (void)hipStreamDestroy(stream);
  own_stream = false;
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  cap_stream = nullptr;
}

int Lane::hip_fail(hipError_t e, const char* what) { return ctx->hip_fail(e, what); }

void Lane::dfree(void* p) { ctx->dfree(p); }

int Lane::sync() { return hip_fail(hipStreamSynchronize(stream), "hipStreamSynchronize"); }

// Read-backs go through the pinned mailbox: a one-block kernel copies the
// values and then posts a sequence number, which the host waits for by
// spinning -- no stream synchronisation and its wake-up latency on the
// critical path.  A wait longer than kMailSpinUs (a long pass queued before
// the read) synchronises the stream instead.
constexpr double kMailSpinUs = 20000.0;

int Lane::wait_mail(uint64_t seq) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    if (__atomic_load_n(&mail[0], __ATOMIC_ACQUIRE) == seq) return RTG_OK;
    const double us = std::chrono::duration<double, std::micro>(
                          std::chrono::steady_clock::now() - t0).count();
    if (us > kMailSpinUs) break;
  }
  int rc = sync();
  if (rc) return rc;
  return __atomic_load_n(&mail[0], __ATOMIC_ACQUIRE) == seq
             ? RTG_OK
             : hip_fail(hipErrorUnknown, "read-back mailbox");
}

int Lane::read_back(const void* dev, size_t bytes, void* host) {
  if (bytes <= kMailBytes && bytes % 4 == 0 && !(reinterpret_cast<uintptr_t>(dev) & 3u)) {
    const uint64_t seq = ++mail_seq;
    launch_mailbox(static_cast<const uint32_t*>(dev), (uint32_t)(bytes / 4), nullptr,
                   reinterpret_cast<uint32_t*>(mail + 32), mail, seq, stream);
    int rc = hip_fail(hipGetLastError(), "read-back launch");
    if (!rc) rc = wait_mail(seq);
    if (rc) return rc;
    std::memcpy(host, mail + 32, bytes);
    return RTG_OK;
  }
  if (bytes > host_stage_bytes) {
    // every earlier read-back has completed (each one waits)
    const size_t grown = std::max(bytes, 2 * host_stage_bytes);
    void* p = nullptr;
    if (hipHostMalloc(&p, grown) != hipSuccess) return hip_fail(hipErrorOutOfMemory, "hipHostMalloc");
    (void)hipHostFree(host_stage);
    host_stage = p;
    host_stage_bytes = grown;
  }
  hipError_t e = hipMemcpyAsync(host_stage, dev, bytes, hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync D2H");
  int rc = sync();
  if (rc) return rc;
  std::memcpy(host, host_stage, bytes);
  return RTG_OK;
}

int Lane::gather_back(const rtgk::Gather& g, uint64_t* host) {
  const uint64_t seq = ++mail_seq;
  launch_mailbox(nullptr, 0, &g, reinterpret_cast<uint32_t*>(mail + 32), mail, seq, stream);
  int rc = hip_fail(hipGetLastError(), "read-back launch");
  if (!rc) rc = wait_mail(seq);
  if (rc) return rc;
  std::memcpy(host, mail + 32, sizeof(uint64_t) * (size_t)g.count);
  return RTG_OK;
}

int Lane::download(void* host, const void* dev, size_t bytes) {
  if (bytes == 0) return RTG_OK;
  hipError_t e = hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync D2H");
  return sync();
}

int Lane::upload(void* dev, const void* host, size_t bytes) {
  return hip_fail(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, stream),
                  "hipMemcpyAsync H2D");
}

int Lane::up_room(size_t bytes) {
  if (up_pending) {
    if (hipEventSynchronize(up_done) != hipSuccess) return hip_fail(hipErrorUnknown, "upload wait");
    up_pending = false;
  }
  if (bytes > host_up_bytes) {
    const size_t grown = std::max(bytes, 2 * host_up_bytes);
    void* p = nullptr;
    if (hipHostMalloc(&p, grown) != hipSuccess) return hip_fail(hipErrorOutOfMemory, "hipHostMalloc");
    (void)hipHostFree(host_up);
    host_up = p;
    host_up_bytes = grown;
  }
  return RTG_OK;
}

void Lane::mark(int phase) {
  if (timing_mask & RTG_TIME_PHASES) (void)hipEventRecord(ev[phase], stream);
}

void Lane::kbegin(int kid) {
  if (!(timing_mask & (1u << kid))) return;
  const size_t pair = kpending.size();
  while (kev.size() < 2 * (pair + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    kev.push_back(e);
  }
  (void)hipEventRecord(kev[2 * pair], stream);
  kpending.emplace_back(kid, (int)pair);
}

void Lane::kend(int kid, double bytes) {
  if (kstats) {
    kstats->kernel_launches[kid] += 1;
    kstats->kernel_bytes[kid] += bytes;
  }
  if (!(timing_mask & (1u << kid)) || kpending.empty()) return;
  const auto& last = kpending.back();
  if (last.first != kid) return;
  (void)hipEventRecord(kev[2 * last.second + 1], stream);
}

void Lane::kfinish() {
  for (const auto& pk : kpending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, kev[2 * pk.second], kev[2 * pk.second + 1]) == hipSuccess &&
        kstats)
      kstats->kernel_ms[pk.first] += ms;
  }
  kpending.clear();
}

static void timer_begin(void* self, int kid) { static_cast<Lane*>(self)->kbegin(kid); }
static void timer_end(void* self, int kid, double bytes) {
  static_cast<Lane*>(self)->kend(kid, bytes);
}

rtgk::LaunchTimer Lane::timer() {
  rtgk::LaunchTimer t;
  t.self = this;
  t.begin = timer_begin;
  t.end = timer_end;
  return t;
}

// Device-side validity of a caller pointer: it must be device memory (or
// memory the device can address) of this context's device.
int check_device_pointer(const void* p, int device) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return RTG_EINVAL;
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return RTG_EINVAL;
  if (attr.type == hipMemoryTypeDevice && attr.device != device) return RTG_EINVAL;
  return RTG_OK;
}

int axes_per_robot(int32_t d, uint32_t flags) {
  constexpr uint32_t known =
      RTG_NO_ROTATE | RTG_UPPER_ONLY | RTG_DEDUP_SORT | RTG_DEDUP_BITMAP | RTG_ROBOTS_MASK;
  if (flags & ~known) return -1;
  if ((flags & RTG_DEDUP_SORT) && (flags & RTG_DEDUP_BITMAP)) return -1;
  const int robots = (int)((flags & RTG_ROBOTS_MASK) >> RTG_ROBOTS_SHIFT);
  if (robots <= 1) return 0;
  if (d < 1 || robots > d || d % robots) return -1;
  return d / robots;
}

int validate_query(const float* points, int64_t n, int32_t d, double r, int32_t k, double alpha) {
  if (d < 1 || d > kMaxDim || k < 1 || n < 0 || n >= (int64_t(1) << 31)) return RTG_EINVAL;
  if (!std::isfinite(r) || !(r > 0.0) || !std::isfinite(alpha) || !(alpha > 0.0)) return RTG_EINVAL;
  if (n > 0 && (!points || (reinterpret_cast<uintptr_t>(points) & 3u))) return RTG_EINVAL;
  return RTG_OK;
}

// ---------------------------------------------------------------------------
// the plain pipeline

namespace {

// Host arrays bound for the device in one transfer: add() reserves a
// 256-byte aligned slot and returns its offset; send() copies every slot
// from the lane's pinned staging into one device block with one
// hipMemcpyAsync, ordered on the lane's stream.
class Uploads {
 public:
  explicit Uploads(Lane& lane) : L_(lane) {}
  size_t add(const void* host, size_t bytes) {
    const size_t off = total_;
    parts_.push_back(Part{host, bytes, off});
    total_ = (off + bytes + 255) & ~(size_t)255;
    return off;
  }
  size_t total() const { return total_; }
  int send(void* dev) {
    if (!total_) return RTG_OK;
    int rc = L_.up_room(total_);
    if (rc) return rc;
    for (const Part& p : parts_)
      if (p.bytes) std::memcpy(static_cast<char*>(L_.host_up) + p.off, p.host, p.bytes);
    rc = L_.hip_fail(hipMemcpyAsync(dev, L_.host_up, total_, hipMemcpyHostToDevice, L_.stream),
                     "hipMemcpyAsync H2D");
    if (rc) return rc;
    rc = L_.hip_fail(hipEventRecord(L_.up_done, L_.stream), "hipEventRecord");
    if (!rc) L_.up_pending = true;
    return rc;
  }

 private:
  struct Part {
    const void* host;
    size_t bytes, off;
  };
  Lane& L_;
  std::vector<Part> parts_;
  size_t total_ = 0;
};

// The tile table of a segmented key sort: segment q holds keys
// [off[q], off[q] + len[q]); tiles stay inside segments and the histogram
// table runs segment by segment (see rtgk::SortTile).
std::vector<SortTile> segment_tiles(const std::vector<uint64_t>& off,
                                    const std::vector<uint64_t>& len) {
  std::vector<SortTile> tab;
  uint64_t slot = 0;
  for (size_t q = 0; q < off.size(); ++q) {
    const uint32_t nts = (uint32_t)((len[q] + kTile - 1) / kTile);
    for (uint32_t t = 0; t < nts; ++t) {
      const uint64_t st0 = (uint64_t)t * kTile;
      tab.push_back(SortTile{off[q] + st0, (uint32_t)std::min<uint64_t>(kTile, len[q] - st0),
                             (uint32_t)(slot + t), nts, 0u});
    }
    slot += (uint64_t)256 * nts;
  }
  return tab;
}

// Frees every arena block taken through it when it goes out of scope.
// Blocks are returned only after the lane's stream has drained, so that
// another lane cannot reuse memory a kernel of this one still touches.
struct Scratch {
  Lane& c;
  void* outer;                                    // the lane's Scratch before this one
  std::vector<std::pair<void*, size_t>> held;     // in use
  // Dropped blocks.  Their last use is queued on this lane's stream, so the
  // lane's later work may take them at once (stream order); the arena, and
  // so the other lanes, gets them back only once the stream has drained.
  std::vector<std::pair<void*, size_t>> pool;
  // A plan's workspace (the same addresses on every run, which its captured
  // graph needs): while carve is set, requests are cut from [carve, carve +
  // carve_left) in order and never given back one by one; if it runs short
  // the rest come from the arena (carve_short).  With record set, the sizes
  // such requests would take are summed in recorded.
  char* carve = nullptr;
  size_t carve_left = 0;
  bool carve_short = false;
  bool record = false;
  size_t recorded = 0;
  // Set by a caller whose last stream operation was a read-back that waited
  // for every kernel before it: the blocks go back without a stream wait.
  bool drained = false;
  explicit Scratch(Lane& lane) : c(lane), outer(lane.scratch) { lane.scratch = this; }
  ~Scratch() {
    c.scratch = outer;
    if (held.empty() && pool.empty()) return;
    if (!drained) (void)hipStreamSynchronize(c.stream);
    for (auto& b : held) c.dfree(b.first);
    for (auto& b : pool) c.dfree(b.first);
  }
  template <class T>
  T* get(size_t count) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    const size_t cut = (bytes + Arena::kAlign - 1) & ~(size_t)(Arena::kAlign - 1);
    if (record) recorded += cut;
    if (carve) {
      if (cut <= carve_left) {
        void* p = carve;
        carve += cut;
        carve_left -= cut;
        return static_cast<T*>(p);
      }
      carve = nullptr;
      carve_short = true;
    }
    // a dropped block that fits without wasting more than its request
    size_t best = pool.size();
    for (size_t i = 0; i < pool.size(); ++i)
      if (pool[i].second >= bytes && pool[i].second <= 2 * bytes + 4096 &&
          (best == pool.size() || pool[i].second < pool[best].second))
        best = i;
    if (best < pool.size()) {
      held.push_back(pool[best]);
      pool.erase(pool.begin() + (std::ptrdiff_t)best);
      return static_cast<T*>(held.back().first);
    }
    void* p = c.dalloc(bytes);
    if (p) held.push_back({p, bytes});
    return static_cast<T*>(p);
  }
  void drop(void* p) {
    for (size_t i = 0; i < held.size(); ++i)
      if (held[i].first == p) {
        if (c.keep_drops) {
          pool.push_back(held[i]);
        } else {
          (void)hipStreamSynchronize(c.stream);
          c.dfree(p);
        }
        held.erase(held.begin() + (std::ptrdiff_t)i);
        return;
      }
  }
  // Gives the dropped blocks back to the arena (after the stream drains);
  // false if there were none.
  bool flush() {
    if (pool.empty()) return false;
    (void)hipStreamSynchronize(c.stream);
    for (auto& b : pool) c.ctx->dfree(b.first);
    pool.clear();
    return true;
  }
};

// Result block: row_ptr (n+1 int64) then col (nnz int32), one arena block.
int alloc_result(Lane& c, int64_t n, size_t nnz, void** res, int64_t** row_ptr, int32_t** col) {
  const size_t rp = ((sizeof(int64_t) * (size_t)(n + 1)) + Arena::kAlign - 1) &
                    ~(size_t)(Arena::kAlign - 1);
  *res = c.dalloc(rp + sizeof(int32_t) * std::max<size_t>(nnz, 1));
  if (!*res) return RTG_ENOMEM;
  *row_ptr = static_cast<int64_t*>(*res);
  *col = reinterpret_cast<int32_t*>(static_cast<char*>(*res) + rp);
  return RTG_OK;
}

// Neighbour lists by row buckets (see the bucket kernels): partition the
// directed entries of the unique pairs into buckets of 2^rb rows, then put
// each bucket in (row, col) order in LDS and write col and row_ptr; buckets
// too large for LDS go through the global radix sort.
int csr_by_buckets(Lane& c, Scratch& S, const Tuning& T, const PairSource& pairs, size_t count,
                   int64_t n, int pb, bool both, uint32_t* err, const LaunchTimer* tm, void** res,
                   int64_t** row_ptr, int32_t** col, size_t* nnz_out, uint32_t* err_host = nullptr,
                   bool* drained = nullptr) {
  if (drained) *drained = false;
  hipStream_t s = c.stream;
  int rc;
  const size_t E = both ? 2 * count : count;
  // at most 2^14 buckets of at most 2^10 rows, as few as keep the mean
  // bucket within 7/8 of what one block holds in LDS (the rest is headroom
  // for uneven buckets; one that overflows takes the global sort): fewer,
  // larger buckets give the partition blocks longer runs to write and the
  // per-bucket blocks more entries per fixed step
  int rb = std::max(0, ceil_log2((uint64_t)n) - 14);
  if ((1 << rb) > kBucketMaxRows) return RTG_ENOMEM;  // callers keep n <= 2^22
  const double per_row = (double)E / (double)n;
  while ((2 << rb) <= kBucketMaxRows && rb + 1 + pb <= 32 &&
         per_row * (double)(1u << (rb + 1)) <= (double)T.bucket_entries)
    ++rb;
  const uint32_t nbuckets = (uint32_t)((n + ((int64_t)1 << rb) - 1) >> rb);
  uint32_t nblocks = (uint32_t)std::max<size_t>(
      1, std::min<size_t>(T.bucket_blocks, (count + 4095) / 4096));
  // pairs still in output segments: every segment gets the same number of
  // blocks
  if (pairs.nseg) nblocks = (nblocks + pairs.nseg - 1) / pairs.nseg * pairs.nseg;
  const uint32_t chunk = (uint32_t)((count + nblocks - 1) / nblocks);
  const size_t np = (size_t)nbuckets * nblocks;
  uint32_t* part = S.get<uint32_t>(np + 1);
  uint32_t* pscr = S.get<uint32_t>(scan_scratch_elems(np) + 1);
  uint32_t* entries = S.get<uint32_t>(E);
  uint32_t* over = S.get<uint32_t>((size_t)nbuckets + 1);  // [0] count, then bucket ids
  if (!part || !pscr || !entries || !over) return RTG_ENOMEM;
  if ((rc = alloc_result(c, n, E, res, row_ptr, col))) return rc;
  if (tm) tm->on_begin(RTG_K_CSR);
  const int pt = (int)T.part_threads;
  // the histogram launch also clears the oversized count; the CSR launch
  // also writes row_ptr[n]
  launch_bucket_hist(pairs, count, pb, rb, both ? 1 : 0, nbuckets, chunk, nblocks, pt, part, over,
                     s);
  scan_exclusive_u32(part, part, np, part + np, pscr, s);
  launch_bucket_scatter(pairs, count, pb, rb, both ? 1 : 0, nbuckets, chunk, nblocks, pt, part,
                        entries, s);
  launch_bucket_csr(entries, part, nbuckets, nblocks, part + np, over + 1, over, c.ctx->bucket_cap, pb,
                    rb, n, (int64_t)E, *row_ptr, *col, s);
  // read the pairs twice, write and read the entries, write col and row_ptr
  if (tm) tm->on_end(RTG_K_CSR, 16.0 * (double)count + 8.0 * (double)E + 4.0 * (double)E +
                                    8.0 * (double)(n + 1));
  // one read for the oversized count and the error bits of everything so far
  uint64_t got[8];
  Gather g;
  g.add(over, 4);
  g.add(err, 4);
  if ((rc = c.gather_back(g, got))) {
    c.dfree(*res);
    return rc;
  }
  const uint32_t nover = (uint32_t)got[0];
  if (err_host) *err_host = (uint32_t)got[1];
  if (drained) *drained = nover == 0;
  if (nover) {
    // Buckets beyond LDS capacity (heavy rows, or rows that cluster in index
    // order), all in one global radix sort of their entries tagged with the
    // bucket's place in the list.
    uint32_t* ext = S.get<uint32_t>(3 * (size_t)nover + 1);  // start, cnt, off, total
    uint32_t* escr = S.get<uint32_t>(scan_scratch_elems(nover) + 1);
    uint32_t tot = 0;
    rc = (!ext || !escr) ? RTG_ENOMEM : RTG_OK;
    if (!rc) {
      launch_over_extent(over + 1, nover, part, nblocks, nbuckets, np, ext, ext + nover, s);
      scan_exclusive_u32(ext + nover, ext + 2 * (size_t)nover, nover, ext + 3 * (size_t)nover,
                         escr, s);
      rc = c.read_back(ext + 3 * (size_t)nover, sizeof(tot), &tot);
    }
    if (!rc && tot) {
      const int sh = rb + pb;
      const int bits = sh + std::max(1, ceil_log2((uint64_t)nover));
      uint64_t* w = S.get<uint64_t>(tot);
      uint64_t* w_alt = S.get<uint64_t>(tot);
      void* scr = S.get<char>(radix_scratch_bytes(tot, 0, bits));
      if (!w || !w_alt || !scr) {
        rc = RTG_ENOMEM;
      } else {
        launch_over_gather(entries, ext, ext + 2 * (size_t)nover, nover, tot, sh, w, s);
        const int where = radix_sort(w, nullptr, w_alt, nullptr, tot, 0, bits, scr, err, s);
        launch_over_emit(where ? w_alt : w, tot, over + 1, ext, ext + nover,
                         ext + 2 * (size_t)nover, pb, rb, n, *row_ptr, *col, s);
      }
    }
    if (rc) {
      c.dfree(*res);
      return rc;
    }
  }
  *nnz_out = E;
  return RTG_OK;
}

// Neighbour lists from pairs sorted by (i, j): upper rows are runs of the
// sorted list; lower rows come from a second sort of the swapped pairs.
int csr_from_sorted(Lane& c, Scratch& S, const Tuning& T, const uint64_t* uniq, size_t U,
                    int64_t n, int pb, bool both, uint32_t* err, int64_t* row_ptr, int32_t* col) {
  hipStream_t s = c.stream;
  uint32_t* up_s = S.get<uint32_t>((size_t)n);
  uint32_t* up_e = S.get<uint32_t>((size_t)n);
  uint32_t* lo_s = both ? S.get<uint32_t>((size_t)n) : nullptr;
  uint32_t* lo_e = both ? S.get<uint32_t>((size_t)n) : nullptr;
  uint64_t* deg = S.get<uint64_t>((size_t)n);
  uint64_t* dscr = S.get<uint64_t>(scan_scratch_elems((size_t)n));
  if (!up_s || !up_e || (both && (!lo_s || !lo_e)) || !deg || !dscr) return RTG_ENOMEM;
  c.kbegin(RTG_K_CSR);
  launch_fill_u32(up_s, 0u, (size_t)n, s);
  launch_fill_u32(up_e, 0u, (size_t)n, s);
  if (both) {
    launch_fill_u32(lo_s, 0u, (size_t)n, s);
    launch_fill_u32(lo_e, 0u, (size_t)n, s);
  }
  const uint64_t* lower = nullptr;
  launch_row_runs(uniq, U, pb, up_s, up_e, s);
  if (both) {
    uint64_t* sw = S.get<uint64_t>(U);
    uint64_t* sw_alt = S.get<uint64_t>(U);
    void* scr = S.get<char>(radix_scratch_bytes(U, 0, 2 * pb));
    if (!sw || !sw_alt || !scr) return RTG_ENOMEM;
    launch_swap_pairs(uniq, U, pb, sw, s);
    const int where = radix_sort(sw, nullptr, sw_alt, nullptr, U, 0, 2 * pb, scr, err, s, nullptr,
                                 0, 0, T.sort_algo);
    lower = where ? sw_alt : sw;
    launch_row_runs(lower, U, pb, lo_s, lo_e, s);
  }
  launch_row_degree(lo_s, lo_e, up_s, up_e, n, deg, s);
  scan_exclusive_u64(deg, reinterpret_cast<uint64_t*>(row_ptr), (size_t)n,
                     reinterpret_cast<uint64_t*>(row_ptr) + n, dscr, s);
  launch_csr_fill_upper(uniq, U, pb, row_ptr, lo_s, lo_e, up_s, col, s);
  if (both) launch_csr_fill_lower(lower, U, pb, row_ptr, lo_s, col, s);
  const size_t nnz = both ? 2 * U : U;
  c.kend(RTG_K_CSR, (both ? 16.0 : 8.0) * (double)U + 8.0 * (double)(n + 1) + 4.0 * (double)nnz);
  return RTG_OK;
}


}  // namespace

// Device memory from the arena; when it has none to give, the dropped blocks
// of this lane's open Scratch objects go back to it first.
void* Lane::dalloc(size_t bytes) {
  auto get = [&] { return noalloc ? ctx->dalloc_noalloc(bytes) : ctx->dalloc(bytes); };
  void* p = get();
  for (Scratch* s = static_cast<Scratch*>(scratch); !p && s; s = static_cast<Scratch*>(s->outer))
    if (s->flush()) p = get();
  return p;
}

size_t Lane::largest_free() { return noalloc ? ctx->largest_free_noalloc() : ctx->largest_free(); }

int Lane::make_empty_result(int64_t n, rtg_csr* out, uint64_t handle) {
  void* mem = dalloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!mem) return RTG_ENOMEM;
  launch_fill_u64(static_cast<uint64_t*>(mem), 0ull, (size_t)(n + 1), stream);
  int rc = sync();
  if (rc) {
    dfree(mem);
    return rc;
  }
  out->n = n;
  out->nnz = 0;
  out->row_ptr = static_cast<int64_t*>(mem);
  out->col = nullptr;
  out->pairs = 0;
  out->handle = ctx->keep_result(handle, mem, n, 0, 0, out->row_ptr, nullptr);
  return RTG_OK;
}

// Argument checks of one query that need no device work beyond a pointer
// query: the shared rules, a device pointer of this context's device, and
// r*r inside the range where the FP32 screen's band is sound.
int Ctx::check_query(const float* points, int64_t n, int32_t d, double r, int32_t k,
                     double alpha, uint32_t flags) {
  int rc = validate_query(points, n, d, r, k, alpha);
  if (rc) return rc;
  if (axes_per_robot(d, flags) < 0) return RTG_EINVAL;
  if (n > 0 && check_device_pointer(points, device)) return RTG_EINVAL;
  const double r2 = r * r;
  if (!(r2 >= 0x1p-100 && r2 <= 0x1p120)) return RTG_ERANGE;
  return RTG_OK;
}

// Whether an instance is within the two-launch small path's limits.
bool Ctx::small_fits(int64_t n, int32_t d, int32_t k, uint32_t flags) const {
  return small_path && n > 1 && n <= kTinyPoints && n * d <= kTinyFloats && d <= 8 &&
         (int64_t)k * n <= kTinyCells && (int64_t)k * d * (d + 1) <= kTinyTransform &&
         axes_per_robot(d, flags) == 0;
}

// Device bytes the small path takes at most for an instance: the uploaded
// transforms, the pair list, the list staging, the counts and the result
// block before it gives back its tail (with room for alignment).
size_t Ctx::small_bytes(int64_t n, int32_t d, int32_t k) const {
  auto up = [](size_t b) { return (b + Arena::kAlign - 1) / Arena::kAlign * Arena::kAlign; };
  return up(sizeof(double) * (size_t)k * d * (d + 1)) + up(sizeof(uint64_t) * kTinyPairCap) +
         up(sizeof(int32_t) * 2 * kTinyPairCap) + up(64) + up(sizeof(int64_t) * (size_t)(n + 1)) +
         up(sizeof(int32_t) * 2 * kTinyPairCap) + (64u << 10);
}

// Lists for a query of n <= 1 points: empty, after the finiteness check.
int Lane::tiny_query(const float* points, int64_t n, int32_t d, rtg_csr* out, uint64_t handle) {
  if (n == 1) {
    std::vector<float> h(d);
    if (download(h.data(), points, sizeof(float) * d)) return RTG_EDEVICE;
    for (float v : h)
      if (!std::isfinite(v)) return RTG_EINVAL;
  }
  return make_empty_result(n, out, handle);
}

int Ctx::all_pairs(const float* points, int64_t n, int32_t d, double r, int32_t k, double alpha,
                   const double* R, const double* u, uint32_t flags, rtg_csr* out) {
  if (poisoned) return RTG_EDEVICE;
  int rc = check_query(points, n, d, r, k, alpha, flags);
  if (rc) return rc;
  rtg_stats st{};
  st.n = n;
  st.d = d;
  st.k = k;
  st.point_transforms = n * k;
  if (n <= 1) {
    rc = main.tiny_query(points, n, d, out, 0);
    if (!rc) stats = st;
    return rc;
  }
  Job job{points, n, d, r, alpha, k, flags, R, u, out};
  if (small_fits(n, d, k, flags)) {
    rc = main.run_tiny(job, st);
    if (rc != Lane::kTinyFallback) {
      if (!rc) stats = st;
      return rc;
    }
  }
  std::vector<Job*> jobs{&job};
  rc = main.run_batch(jobs, st);
  if (!rc) stats = st;
  return rc;
}

// One small instance: k workgroups find each grid's cells and test their
// pairs (first grid only), one builds the lists into a result block sized
// for the most pairs the small path takes, which then gives back its tail.
// One read-back for the counts.
int Lane::run_tiny(Job& j, rtg_stats& st) {
  const int d = j.d;
  int rc;
  kstats = &st;
  kpending.clear();
  struct Detach {
    Lane& c;
    ~Detach() {
      c.kpending.clear();
      c.kstats = nullptr;
    }
  } detach{*this};
  Scratch S(*this);
  mark(0);
  // the transforms and the zeroed counters ([0..3] counts, [4] error
  // bits) go up in one copy: no separate launch clears the counters
  static const unsigned long long kZeroCounts[8] = {};
  Uploads U(*this);
  const size_t o_R = U.add(j.R, sizeof(double) * (size_t)j.k * d * d);
  const size_t o_u = U.add(j.u, sizeof(double) * (size_t)j.k * d);
  const size_t o_cnt = U.add(kZeroCounts, sizeof(kZeroCounts));
  char* up = S.get<char>(U.total());
  uint64_t* pairs = S.get<uint64_t>(kTinyPairCap);
  int32_t* stage = S.get<int32_t>(2 * kTinyPairCap);
  if (!up || !pairs || !stage) return RTG_ENOMEM;
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(up + o_cnt);
  if ((rc = U.send(up))) return rc;
  void* res = nullptr;
  int64_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  if ((rc = alloc_result(*this, j.n, 2 * kTinyPairCap, &res, &row_ptr, &col))) return rc;
  TinyArgs a{};
  a.pts = j.pts;
  a.n = (int)j.n;
  a.r2 = j.r * j.r;
  a.inv_c = 1.0 / (j.alpha * j.r);
  a.R = reinterpret_cast<const double*>(up + o_R);
  a.u = reinterpret_cast<const double*>(up + o_u);
  a.k = j.k;
  // up to 8 workgroups per grid (each finds the grid's cells, then tests
  // its slice of the pairs), no more than 256 in all unless k is larger
  a.parts = (uint32_t)std::max(1, std::min(8, 256 / std::max(1, j.k)));
  a.pairs = pairs;
  a.cap = kTinyPairCap;
  a.count = cnt;
  a.err = reinterpret_cast<uint32_t*>(cnt + 4);
  a.upper = (j.flags & RTG_UPPER_ONLY) ? 1 : 0;
  a.row_ptr = row_ptr;
  a.col = col;
  a.stage = stage;
  kbegin(RTG_K_PAIRS);
  launch_tiny(a, d, j.k, stream);
  // points read per grid and pair; pairs, lists and row offsets written
  kend(RTG_K_PAIRS, 4.0 * (double)j.n * d * j.k);
  if ((rc = hip_fail(hipGetLastError(), "kernel launch"))) {
    dfree(res);
    return rc;
  }
  uint64_t got[8];
  Gather g;
  g.add(cnt, 8);
  g.add(cnt + 1, 8);
  g.add(cnt + 2, 8);
  g.add(cnt + 3, 8);
  g.add(cnt + 4, 4);
  if ((rc = gather_back(g, got))) {
    dfree(res);
    return rc;
  }
  const uint64_t npairs = got[0], nnz = got[3];
  const uint32_t err = (uint32_t)got[4];
  kfinish();
  if (err & 1u) {
    dfree(res);
    return RTG_EINVAL;
  }
  if (err & 2u) {
    dfree(res);
    return RTG_ERANGE;
  }
  if (err || npairs > kTinyPairCap) {
    dfree(res);
    return kTinyFallback;
  }
  const size_t rp = ((sizeof(int64_t) * (size_t)(j.n + 1)) + Arena::kAlign - 1) &
                    ~(size_t)(Arena::kAlign - 1);
  ctx->dshrink(res, rp + sizeof(int32_t) * std::max<uint64_t>(nnz, 1));
  const bool both = !(j.flags & RTG_UPPER_ONLY);
  st.cells = (int64_t)got[2];
  st.tests = (int64_t)got[1];
  st.candidates = (int64_t)npairs;
  st.unique_pairs = (int64_t)npairs;
  st.transforms_per_sort = 1;
  j.out->n = j.n;
  j.out->nnz = (int64_t)nnz;
  j.out->row_ptr = row_ptr;
  j.out->col = nnz ? col : nullptr;
  j.out->pairs = (int64_t)(both ? nnz / 2 : nnz);
  j.out->handle = ctx->keep_result(j.handle, res, j.n, (int64_t)nnz, j.out->pairs, row_ptr, col);
  mark(8);
  S.drained = true;  // the counts' read-back came after both launches
  return RTG_OK;
}

// rtg_all_pairs into the caller's buffers with every device byte from the
// no-allocation arena: the usual pass on the main lane, its result copied
// out and given back.  Size limits keep the pass inside the array and every
// host transfer inside the main lane's pinned staging (sized at creation),
// so nothing is allocated on the device or pinned on the host.
int Ctx::all_pairs_noalloc(const float* points, int64_t n, int32_t d, double r, int32_t k,
                           double alpha, const double* R, const double* u, uint32_t flags,
                           int64_t* row_ptr, int32_t* col, int64_t col_capacity, int64_t* nnz) {
  if (poisoned) return RTG_EDEVICE;
  if (!noalloc_arena) return RTG_EDEVICE;
  int rc = check_query(points, n, d, r, k, alpha, flags);
  if (rc) return rc;
  if ((reinterpret_cast<uintptr_t>(row_ptr) & 7u) || (reinterpret_cast<uintptr_t>(col) & 3u) ||
      check_device_pointer(row_ptr, device) ||
      (col_capacity > 0 && check_device_pointer(col, device)))
    return RTG_EINVAL;
  // uploads of one pass (transforms, field origins, segment tiles) and the
  // working set (points excluded) against the limits
  const double staging = 8.0 * k * d * (d + 2) + 24.0 * k + 24.0 * k * ((double)n / kTile + 2.0) +
                         8192.0;
  if (staging > (double)kNoallocStaging ||
      pass_bytes_bound(n, d, k, alpha, flags) > kNoallocBytes)
    return RTG_ENOMEM;
  rtg_stats st{};
  st.n = n;
  st.d = d;
  st.k = k;
  st.point_transforms = n * k;
  rtg_csr out{};
  const uint32_t timing = main.timing_mask;
  main.timing_mask = 0;  // no timing events are made in this call
  main.noalloc = true;
  if (n <= 1) {
    rc = main.tiny_query(points, n, d, &out, 0);
  } else {
    Job job{points, n, d, r, alpha, k, flags, R, u, &out};
    std::vector<Job*> jobs{&job};
    rc = main.run_batch(jobs, st);
  }
  main.noalloc = false;
  main.timing_mask = timing;
  if (rc) return rc;
  const int64_t need = out.nnz;
  if (need > col_capacity) {
    release(out.handle);
    *nnz = need;
    return RTG_ENOMEM;
  }
  rc = hip_fail(hipMemcpyAsync(row_ptr, out.row_ptr, sizeof(int64_t) * (size_t)(n + 1),
                               hipMemcpyDeviceToDevice, main.stream),
                "copy row_ptr");
  if (!rc && need)
    rc = hip_fail(hipMemcpyAsync(col, out.col, sizeof(int32_t) * (size_t)need,
                                 hipMemcpyDeviceToDevice, main.stream),
                  "copy col");
  if (!rc) rc = main.sync();
  release(out.handle);
  if (rc) return rc;
  *nnz = need;
  stats = st;
  return RTG_OK;
}

// One pass of the pipeline over a batch of instances of one dimension d
// sharing the RTG_UPPER_ONLY / RTG_DEDUP_SORT flags (every instance has
// n >= 2 and passed check_query).  On success each job's out is filled.
int Lane::run_batch(std::vector<Job*>& jobs, rtg_stats& st, PassPlan* pp) {
  const uint32_t m = (uint32_t)jobs.size();
  const int d = jobs[0]->d;
  const uint32_t flags = jobs[0]->flags;
  const bool both = !(flags & RTG_UPPER_ONLY);
  int rc;

  kstats = &st;
  kpending.clear();
  struct Detach {
    Lane& c;
    ~Detach() {
      c.kpending.clear();
      c.kstats = nullptr;
    }
  } detach{*this};
  const LaunchTimer tm = timer();
  Scratch S(*this);
  if (pp && pp->ws) {
    S.carve = static_cast<char*>(pp->ws);
    S.carve_left = pp->head_bytes;
  } else if (pp) {
    S.record = true;  // the first run sizes the plan's workspace
  }
  mark(0);

  // --- the batch's instances and segments (host) -----------------------------
  std::vector<InstDesc> inst(m);
  int64_t npts = 0;
  uint32_t nblk = 0;
  int32_t S_total = 0, kmax = 0;
  for (uint32_t q = 0; q < m; ++q) {
    const Job& j = *jobs[q];
    inst[q].pts = j.pts;
    inst[q].pt_off = npts;
    inst[q].n = j.n;
    inst[q].inv_c = 1.0 / (j.alpha * j.r);
    inst[q].k = j.k;
    inst[q].tr_off = S_total;
    inst[q].seg_first = S_total;
    inst[q].blk_first = (int32_t)nblk;
    npts += j.n;
    nblk += (uint32_t)((j.n + kBlock - 1) / kBlock);
    S_total += j.k;
    kmax = std::max(kmax, j.k);
  }
  if (npts >= (int64_t(1) << 31)) return RTG_ENOMEM;
  const Tuning T = ctx->tuning_for(d, npts);
  const int pair_bits = std::max(1, ceil_log2((uint64_t)npts));
  std::vector<PairTest> tests(m);
  std::vector<int> sub(m);  // MR-metric axes per robot (0: Euclidean)
  bool any_mr = false;
  std::vector<double> Rh((size_t)S_total * d * d), uh((size_t)S_total * d);
  for (uint32_t q = 0; q < m; ++q) {
    const Job& j = *jobs[q];
    sub[q] = axes_per_robot(d, j.flags);
    tests[q] = make_pair_test(sub[q] ? mr_screen_r2(j.r) : j.r * j.r, pair_bits, d,
                              j.alpha * j.r);
    any_mr = any_mr || sub[q] > 0;
    std::memcpy(&Rh[(size_t)inst[q].tr_off * d * d], j.R, sizeof(double) * (size_t)j.k * d * d);
    std::memcpy(&uh[(size_t)inst[q].tr_off * d], j.u, sizeof(double) * (size_t)j.k * d);
  }

  Uploads U1(*this);
  const size_t o_inst = U1.add(inst.data(), sizeof(InstDesc) * m);
  const size_t o_tests = U1.add(tests.data(), sizeof(PairTest) * m);
  const size_t o_R = U1.add(Rh.data(), sizeof(double) * Rh.size());
  const size_t o_u = U1.add(uh.data(), sizeof(double) * uh.size());
  // A few boxes: their identities, *bad and the pass's counters go up with
  // the descriptors (cleared by the copy, not by a launch).
  const size_t nbox = (size_t)m * 2 * d;
  const bool box_up = nbox <= 1024;
  std::vector<uint32_t> box_init;
  static const unsigned long long kZeroCounters[kCounterWords] = {};
  size_t o_box = 0, o_cnt = 0;
  if (box_up) {
    box_init.resize(nbox + 1);
    for (size_t e = 0; e < nbox; ++e) box_init[e] = (e & 1) ? 0u : 0xFFFFFFFFu;
    box_init[nbox] = 0u;  // bad
    o_box = U1.add(box_init.data(), sizeof(uint32_t) * box_init.size());
    o_cnt = U1.add(kZeroCounters, sizeof(kZeroCounters));
  }
  char* up1 = S.get<char>(U1.total());
  if (!up1) return RTG_ENOMEM;
  InstDesc* inst_d = reinterpret_cast<InstDesc*>(up1 + o_inst);
  PairTest* tests_d = reinterpret_cast<PairTest*>(up1 + o_tests);
  double* Rd = reinterpret_cast<double*>(up1 + o_R);
  double* ud = reinterpret_cast<double*>(up1 + o_u);
  float* soa = S.get<float>((size_t)npts * d);
  float* aos = m > 1 ? S.get<float>((size_t)npts * d) : nullptr;
  uint32_t* part = S.get<uint32_t>((size_t)nblk * 2 * d);
  uint32_t* bbox = box_up ? reinterpret_cast<uint32_t*>(up1 + o_box)
                         : S.get<uint32_t>((size_t)m * 2 * d + 1);  // + [bad]
  // -, rechecks, filter count, members, the pair-output segments' counts,
  // then err (read back with them after each pass's pair kernel)
  unsigned long long* counters =
      box_up ? reinterpret_cast<unsigned long long*>(up1 + o_cnt)
             : S.get<unsigned long long>(kCounterWords);
  if (!soa || (m > 1 && !aos) || !part || !bbox || !counters) return RTG_ENOMEM;
  uint32_t* bad = bbox + (size_t)m * 2 * d;
  uint32_t* err = reinterpret_cast<uint32_t*>(counters + kErrWord);
  if ((rc = U1.send(up1))) return rc;

  // First-owner filter (default): each pair is emitted only by the first grid
  // whose cell holds both points, so the union needs no de-duplication.  It
  // compares neighbourhood signatures: per grid the low sig_b bits of every
  // axis field, sig_b the widest minimum field width of the batch.  Groups
  // wider than a word (small alpha at high d) take sort-unique instead.
  int sig_b = 1;
  for (uint32_t q = 0; q < m; ++q) sig_b = std::max(sig_b, min_field_bits(jobs[q]->alpha));
  const int sig_g = d * sig_b;
  // Bitmaps of every instance's unordered pairs, when asked for and small
  // enough; otherwise the first-owner rule where the signatures fit.
  uint64_t bitmap_words = 0;
  std::vector<BitmapInst> bmi;
  if (flags & RTG_DEDUP_BITMAP) {
    uint64_t bits = 0;
    for (uint32_t q = 0; q < m; ++q) {
      bmi.push_back(BitmapInst{inst[q].pt_off, (int64_t)bits});
      const uint64_t nq = (uint64_t)inst[q].n;
      bits += nq * (nq - 1) / 2;
    }
    const uint64_t words = (bits + 31) / 32;
    const uint64_t limit = std::min<uint64_t>(kBitmapMaxBytes, largest_free() / 4);
    if (4 * words <= limit) bitmap_words = std::max<uint64_t>(words, 1);
  }
  const bool bitmap = bitmap_words > 0;
  const bool first_owner = !(flags & RTG_DEDUP_SORT) && !bitmap && sig_g <= 64;
  const int sig_gpw = sig_g <= 64 ? 64 / sig_g : 1;
  const int sig_W = (kmax + sig_gpw - 1) / sig_gpw;
  uint64_t* sig = nullptr;   // [npts][W], or in the point records
  uint64_t* ssig = nullptr;  // [W][NB] by sorted position (gathered copy)
  // With one signature word, tile loads by point index and d <= 6, every
  // point gets a 32-byte record (coordinates, padding, then the signature
  // word in the last 8 bytes): a tile load reads one aligned run per lane
  // instead of a row and a word apart (uniform d6 pair kernel about 1.5%
  // faster; wider records at d = 12 cost more than they saved).  The stage
  // kernel writes them while it reads the points.
  const int rs = (d + 2 + 3) & ~3;
  float* rec = nullptr;
  int sig_stride = sig_W;
  if (first_owner && sig_W == 1 && ctx->gather_direct && d <= 6) {
    rec = S.get<float>((size_t)npts * rs);
    if (!rec) return RTG_ENOMEM;
    sig = reinterpret_cast<uint64_t*>(rec + rs - 2);
    sig_stride = rs / 2;
  }
  // --- stage: SoA copy (+ concatenated rows), finiteness, bounding boxes -------
  kbegin(RTG_K_STAGE);
  // (its first launch also clears the boxes and the pass's counters, unless the upload did)
  launch_stage(inst_d, m, nblk, d, npts, soa, aos, bad, bbox, part, rec, rs, stream,
               reinterpret_cast<uint64_t*>(counters), kCounterWords, box_up);
  kend(RTG_K_STAGE, (aos ? 12.0 : 8.0) * (double)npts * d + (rec ? 4.0 * rs * (double)npts : 0.0));
  mark(1);
  std::vector<uint32_t> hb((size_t)m * 2 * d + 1);
  if ((rc = read_back(bbox, sizeof(uint32_t) * hb.size(), hb.data()))) return rc;
  if (hb[(size_t)m * 2 * d]) return RTG_EINVAL;
  const float* pts_rows = aos ? aos : jobs[0]->pts;

  // --- key layout shared by the batch ---------------------------------------------
  Packing P;
  {
    std::vector<float> lo((size_t)m * d), hi((size_t)m * d);
    for (size_t e = 0; e < (size_t)m * d; ++e) {
      lo[e] = decode_order(hb[2 * e]);
      hi[e] = decode_order(hb[2 * e + 1]);
    }
    std::vector<double> alphas(m), inv_cs(m);
    std::vector<int64_t> ns(m), ks(m);
    for (uint32_t q = 0; q < m; ++q) {
      alphas[q] = jobs[q]->alpha;
      inv_cs[q] = inst[q].inv_c;
      ns[q] = jobs[q]->n;
      ks[q] = jobs[q]->k;
    }
    rc = plan_batch(d, m, ks.data(), ns.data(), Rh.data(), uh.data(), inv_cs.data(),
                    alphas.data(), lo.data(), hi.data(), largest_free() / 2, P);
    if (rc) return rc;
  }
  st.key_bits = std::max(st.key_bits, P.key_bits);

  st.pair_bits = 2 * pair_bits;
  st.transforms_per_sort = P.tb;



  // Passes: consecutive ranges of P.tb segments; key offsets restart per pass.
  std::vector<SegDesc> segs((size_t)S_total);
  size_t NB = 0;
  for (int32_t sa = 0; sa < S_total; sa += P.tb) {
    const int32_t sb = std::min(S_total, sa + P.tb);
    int64_t off = 0;
    for (uint32_t q = 0; q < m; ++q)
      for (int32_t t = 0; t < jobs[q]->k; ++t) {
        const int32_t s = inst[q].seg_first + t;
        if (s < sa || s >= sb) continue;
        segs[s].key_off = off;
        segs[s].inst = (int32_t)q;
        segs[s].t = t;
        off += jobs[q]->n;
      }
    NB = std::max(NB, (size_t)off);
  }
  // Each pass of several segments sorts within them (reduce-then-scan):
  // its table of sort tiles goes up with the layout, in one copy.
  std::vector<std::vector<SortTile>> pass_tabs;
  for (int32_t sa = 0; sa < S_total; sa += P.tb) {
    const int32_t sb = std::min(S_total, sa + P.tb);
    pass_tabs.emplace_back();
    if (sb - sa > 1 && T.sort_algo == kSortReduceScan) {
      std::vector<uint64_t> soff, slen;
      for (int32_t sg = sa; sg < sb; ++sg) {
        soff.push_back((uint64_t)segs[sg].key_off);
        slen.push_back((uint64_t)jobs[segs[sg].inst]->n);
      }
      pass_tabs.back() = segment_tiles(soff, slen);
    }
  }
  Uploads U2(*this);
  const size_t o_layout = U2.add(&P.layout, sizeof(KeyLayout));
  const size_t o_klo = U2.add(P.klo.data(), sizeof(int64_t) * P.klo.size());
  const size_t o_segs = U2.add(segs.data(), sizeof(SegDesc) * segs.size());
  std::vector<size_t> o_tabs;
  for (const auto& tab : pass_tabs)
    o_tabs.push_back(U2.add(tab.data(), sizeof(SortTile) * tab.size()));
  char* up2 = S.get<char>(U2.total());
  if (!up2) return RTG_ENOMEM;
  KeyLayout* layout_d = reinterpret_cast<KeyLayout*>(up2 + o_layout);
  int64_t* klo_d = reinterpret_cast<int64_t*>(up2 + o_klo);
  SegDesc* segs_d = reinterpret_cast<SegDesc*>(up2 + o_segs);
  if ((rc = U2.send(up2))) return rc;

  // The point index rides in the low bits of the key when both fit in 64
  // bits: the sort then moves 8 bytes per element instead of 12.
  const int idx_bits = (P.key_bits + pair_bits <= 64) ? pair_bits : 0;
  uint64_t* keys = S.get<uint64_t>(NB);
  uint64_t* keys_alt = S.get<uint64_t>(NB);
  uint32_t* vals = idx_bits ? nullptr : S.get<uint32_t>(NB);
  uint32_t* vals_alt = idx_bits ? nullptr : S.get<uint32_t>(NB);
  const size_t ntiles = (NB + kTile - 1) / kTile;
  void* sort_scr = S.get<char>(radix_scratch_bytes(NB, 0, P.key_bits, (size_t)S_total));
  uint32_t* run_scr = S.get<uint32_t>(2 * ntiles + 8 + scan_scratch_elems(ntiles));
  uint64_t* run_masks = S.get<uint64_t>(run_mask_words(NB));  // cell heads and tails
  const size_t max_cells = NB / 2 + 1;
  const size_t max_units = max_cells + NB / kPairTile + 1;
  uint32_t* cstart = S.get<uint32_t>(max_cells);
  uint32_t* cend = S.get<uint32_t>(max_cells);
  uint32_t* units = S.get<uint32_t>(max_cells);
  UnitDesc* udesc = S.get<UnitDesc>(max_units);
  // unit points by sorted position: only when the pair kernels read a gathered copy
  float* spts = ctx->gather_direct ? nullptr : S.get<float>((size_t)d * NB);
  uint64_t* tests_c = S.get<uint64_t>(max_cells);
  const size_t s64 = scan_scratch_elems(max_cells);
  uint64_t* scan64 = S.get<uint64_t>(s64 + 4);
  uint32_t* scan32 = S.get<uint32_t>(s64 + 4);
  // the units' tile pairs, their prefix, and each pair-kernel wave's run of units
  const bool balanced = ctx->balanced_units;
  const size_t su = scan_scratch_elems(max_units);
  uint64_t* uwork = balanced ? S.get<uint64_t>(max_units) : nullptr;
  uint64_t* uscan = balanced ? S.get<uint64_t>(su + 4) : nullptr;
  const size_t max_waves = (size_t)std::max<uint32_t>(ctx->pair_blocks, kMaxPairBlocks) * kWaves;
  uint32_t* wfirst = balanced ? S.get<uint32_t>(max_waves + 1) : nullptr;
  if (!keys || !keys_alt || (!idx_bits && (!vals || !vals_alt)) || !sort_scr || !run_scr ||
      !run_masks ||
      !cstart || !cend || !units || !udesc || (!ctx->gather_direct && !spts) || !tests_c ||
      !scan64 || !scan32 ||
      (balanced && (!uwork || !uscan || !wfirst)))
    return RTG_ENOMEM;

  if (first_owner) {
    // signature words by sorted position: only for the gathered copy
    if (!ctx->gather_direct) {
      ssig = S.get<uint64_t>((size_t)sig_W * NB);
      if (!ssig) return RTG_ENOMEM;
    }
    if (!rec) {
      sig = S.get<uint64_t>((size_t)npts * sig_W);
      if (!sig) return RTG_ENOMEM;
      // the key kernel ORs into the words when its passes split the grids
      if (P.tb < S_total) launch_fill_u64(sig, 0ull, (size_t)npts * sig_W, stream);
    }
  }

  uint64_t cap = 0;
  uint64_t* cand = nullptr;
  uint64_t cand_total = 0;  // exact number of candidates so far
  // One pass whose first-owner pairs go straight to the row-bucket lists: the
  // list build reads the pair kernel's output segments as they are, so they
  // are not first copied into one array.
  const bool lists_from_segments = P.tb >= S_total && first_owner && !any_mr &&
                                   pair_bits <= 24 && ceil_log2((uint64_t)npts) <= 22 &&
                                   ceil_log2((uint64_t)npts) - 14 + pair_bits <= 32;
  PairSource seg_src{nullptr};
  uint64_t rechecks_seen = 0;

  // Pair screen: matrix cores when every instance suits them.  Their Gram
  // form squares and sums coordinates, so it needs |coordinate| <= 2^60
  // (no FP32 overflow for d <= 16); the vector screen takes the rest.
  bool coords_small = true;
  for (size_t e = 0; e < (size_t)m * d; ++e)
    coords_small = coords_small && std::fabs(decode_order(hb[2 * e])) <= 0x1p60f &&
                   std::fabs(decode_order(hb[2 * e + 1])) <= 0x1p60f;
  bool use_gram = ctx->pair_screen != 1 && coords_small;
  for (uint32_t q = 0; q < m && use_gram; ++q) use_gram = gram_suits(d, jobs[q]->alpha);
  if (ctx->pair_screen == 2) use_gram = d <= 16 && coords_small;

  for (int32_t sa = 0; sa < S_total; sa += P.tb) {
    const int32_t sb = std::min(S_total, sa + P.tb);
    size_t N = 0, pass_pts = 0;
    for (int32_t s = sa; s < sb; ++s) {
      N += (size_t)jobs[segs[s].inst]->n;
      if (s == sa || segs[s].inst != segs[s - 1].inst) pass_pts += (size_t)jobs[segs[s].inst]->n;
    }
    const int seg_bits = (sb - sa) > 1 ? ceil_log2((uint64_t)(sb - sa)) : 0;
    const int key_bits = seg_bits + P.layout.cell_bits;
    // Several segments in the pass: sort within segments (tiles that stay
    // inside one segment), so only the cell bits take passes; the segment
    // bits above them are already in order.
    const bool segmented = seg_bits > 0 && T.sort_algo == kSortReduceScan;
    uint32_t ntab = 0;
    SortTile* tab_d = nullptr;
    if (segmented) {
      const size_t pass = (size_t)(sa / P.tb);
      ntab = (uint32_t)pass_tabs[pass].size();
      tab_d = reinterpret_cast<SortTile*>(up2 + o_tabs[pass]);
    }
    const int sort_end = idx_bits + (segmented ? P.layout.cell_bits : key_bits);
    const size_t nt = (N + kTile - 1) / kTile;
    uint32_t* hcnt = run_scr;
    uint32_t* tcnt = run_scr + nt;
    uint32_t* tot = run_scr + 2 * nt;  // [0] heads, [1] tails
    uint32_t* sscr = run_scr + 2 * nt + 2;
    // up to 2048 tiles the writing kernel adds up the earlier tiles' counts
    // itself (and clears the member counter of the cell-work kernel); its
    // reads grow as the square of the tiles, so more take the scans
    const bool counts_direct = nt >= 1 && nt <= 2048;
    const uint32_t cell_bound = (uint32_t)std::min<size_t>(max_cells, N / 2 + 1);
    int where = 0;
    // From the key kernel to the unit descriptors every size is on the
    // device: the stretch a plan captures as a graph.
    auto stretch = [&]() {
      KeysArgs ka{inst_d, m, nblk, d, npts, soa, sa, sb, segs_d, Rd, ud, klo_d, layout_d,
                  keys, vals, err, sig, sig_stride, sig_b, sig_gpw, idx_bits,
                  P.tb >= S_total ? 1 : 0};
      kbegin(RTG_K_KEYS);
      launch_keys(ka, stream);
      kend(RTG_K_KEYS, 4.0 * (double)pass_pts * d + (idx_bits ? 8.0 : 12.0) * (double)N +
                           (sig ? 16.0 * (double)pass_pts * sig_W : 0.0));
      mark(2);
      where = radix_sort(keys, vals, keys_alt, vals_alt, N, idx_bits, sort_end, sort_scr,
                                   err, stream, &tm, RTG_K_KEY_HIST, RTG_K_KEY_SCATTER,
                                   T.sort_algo, tab_d, ntab);
      st.key_passes = std::max(st.key_passes, (sort_end - idx_bits + kRadixBits - 1) / kRadixBits);
      const uint64_t* skeys = where ? keys_alt : keys;
      mark(3);
      // cells with >= 2 points
      kbegin(RTG_K_CELLS);
      launch_run_count(skeys, N, idx_bits, hcnt, tcnt, run_masks, stream);
      if (counts_direct) {
        launch_run_write(run_masks, N, hcnt, tcnt, cstart, cend, tot, counters + 3, stream);
      } else {
        scan_exclusive_u32(hcnt, hcnt, nt, tot, sscr, stream);
        scan_exclusive_u32(tcnt, tcnt, nt, tot + 1, sscr, stream);
        launch_run_write(run_masks, N, hcnt, tcnt, cstart, cend, nullptr, nullptr, stream);
      }
      kend(RTG_K_CELLS, 8.5 * (double)N);  // keys once, head and tail bits out and back
      // Cell work, unit counts and their scans and the unit descriptors run on
      // the device's own cell count (tot[0]; the host knows only the bound
      // max_cells), so one read-back after them serves the whole cell stage.
      kbegin(RTG_K_CELLS);
      if (!counts_direct) launch_fill_u64(reinterpret_cast<uint64_t*>(counters) + 3, 0ull, 1, stream);
      if (!launch_cell_work_scanned(cstart, cend, cell_bound, tot, T.unit_tiles, units, tests_c,
                                    counters + 3, scan32, scan32 + s64, scan64, scan64 + s64,
                                    stream)) {
        launch_cell_work(cstart, cend, cell_bound, tot, T.unit_tiles, units, tests_c, counters + 3,
                         stream);
        scan_exclusive_u32(units, units, cell_bound, scan32 + s64, scan32, stream, tot);
        scan_exclusive_u64(tests_c, tests_c, cell_bound, scan64 + s64, scan64, stream, tot);
      }
      launch_unit_fill(cstart, cend, units, cell_bound, tot, T.unit_tiles, skeys,
                       seg_bits > 0 ? idx_bits + P.layout.cell_bits : 64, sa, segs_d, udesc, uwork,
                       stream);
      kend(RTG_K_CELLS, 0.0);
    };
    // A plan's single-pass stretch is captured once and then replayed:
    // its arguments (workspace addresses and sizes) must match the capture.
    constexpr uint32_t kStretchTimed = (1u << RTG_K_KEYS) | (1u << RTG_K_KEY_HIST) |
                                       (1u << RTG_K_KEY_SCATTER) | (1u << RTG_K_CELLS) |
                                       (1u << RTG_K_SCAN) | RTG_TIME_PHASES;
    const bool graph = pp && pp->ws && !S.carve_short && P.tb >= S_total &&
                       !(timing_mask & kStretchTimed);
    std::vector<int64_t> shape;
    if (graph) {
      for (const void* ptr : {(const void*)inst_d, (const void*)soa, (const void*)segs_d,
                              (const void*)Rd, (const void*)ud, (const void*)klo_d,
                              (const void*)layout_d, (const void*)keys, (const void*)keys_alt,
                              (const void*)vals, (const void*)vals_alt, (const void*)err,
                              (const void*)sig, (const void*)sort_scr, (const void*)tab_d,
                              (const void*)run_scr, (const void*)cstart, (const void*)cend,
                              (const void*)units, (const void*)tests_c, (const void*)scan32,
                              (const void*)scan64, (const void*)udesc, (const void*)uwork,
                              (const void*)counters, (const void*)run_masks})
        shape.push_back((int64_t)reinterpret_cast<uintptr_t>(ptr));
      for (int64_t v : {(int64_t)m, (int64_t)nblk, (int64_t)d, npts, (int64_t)sa, (int64_t)sb,
                        (int64_t)N, (int64_t)pass_pts, (int64_t)idx_bits, (int64_t)key_bits,
                        (int64_t)P.layout.cell_bits, (int64_t)sort_end, (int64_t)ntab,
                        (int64_t)T.sort_algo, (int64_t)T.unit_tiles, (int64_t)sig_stride,
                        (int64_t)sig_b, (int64_t)sig_gpw, (int64_t)cell_bound,
                        (int64_t)counts_direct, (int64_t)seg_bits, (int64_t)NB,
                        (int64_t)max_cells})
        shape.push_back(v);
    }
    if (graph && pp->exec && shape == pp->shape) {
      if ((rc = hip_fail(hipGraphLaunch(pp->exec, stream), "hipGraphLaunch"))) return rc;
      where = pp->where;  // the buffer the sort's last pass wrote
      for (int q = 0; q < RTG_NKERNELS; ++q) {
        st.kernel_launches[q] += pp->launches[q];
        st.kernel_bytes[q] += pp->bytes[q];
      }
      st.key_passes = std::max(st.key_passes, pp->key_passes);
      ++pp->replays;
    } else if (graph) {
      if (pp->exec) (void)hipGraphExecDestroy(pp->exec);
      pp->exec = nullptr;
      rtg_stats before = st;
      hipGraph_t g = nullptr;
      // the stretch's launches go to the capturing stream while it records
      if (!own_stream && !cap_stream)
        (void)hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
      const hipStream_t lane_stream = stream;
      const hipStream_t cs = own_stream ? stream : cap_stream;
      bool captured =
          cs && hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) == hipSuccess;
      if (captured) {
        stream = cs;
        stretch();
        stream = lane_stream;
        captured = hipStreamEndCapture(cs, &g) == hipSuccess && g != nullptr;
        if (captured)
          captured = hipGraphInstantiate(&pp->exec, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
      }
      if (!captured) (void)hipGetLastError();  // the failed capture's error
      if (captured) {
        for (int q = 0; q < RTG_NKERNELS; ++q) {
          pp->launches[q] = st.kernel_launches[q] - before.kernel_launches[q];
          pp->bytes[q] = st.kernel_bytes[q] - before.kernel_bytes[q];
        }
        pp->key_passes = st.key_passes;
        pp->where = where;
        pp->shape = shape;
        ++pp->captures;
        if ((rc = hip_fail(hipGraphLaunch(pp->exec, stream), "hipGraphLaunch"))) return rc;
      } else {
        // no graph: the stretch runs as ordinary launches
        pp->exec = nullptr;
        st = before;
        stretch();
      }
    } else {
      stretch();
    }
    const uint64_t* skeys = where ? keys_alt : keys;
    const uint32_t* sidx = idx_bits ? nullptr : (where ? vals_alt : vals);
    uint64_t got[8];
    Gather g1;
    g1.add(tot, 4);
    g1.add(err, 4);
    g1.add(scan64 + s64, 8);
    g1.add(scan32 + s64, 4);
    if ((rc = gather_back(g1, got))) return rc;
    const uint32_t ncells_h = (uint32_t)got[0], errh0 = (uint32_t)got[1];
    // A cell coordinate out of range makes the grouping meaningless: stop
    // before the pair kernel sees it.
    if (errh0 & 1u) return RTG_ERANGE;
    if (errh0) return hip_fail(hipErrorUnknown, "radix sort look-back");
    const uint64_t tests_total = ncells_h ? got[2] : 0;
    const uint32_t units_total = ncells_h ? (uint32_t)got[3] : 0u;
    st.kernel_bytes[RTG_K_CELLS] += 24.0 * (double)ncells_h;
    mark(4);
    // a plan's workspace ends here: what follows is sized by the pass's pairs
    S.carve = nullptr;
    S.record = false;
    st.cells += ncells_h;
    st.tests += (int64_t)tests_total;
    if (units_total == 0) continue;
    PairsArgs pa{};
    pa.units = udesc;
    pa.total_units = units_total;
    pa.spts = spts;
    pa.ssig = first_owner ? ssig : nullptr;
    pa.first_owner = first_owner ? 1 : 0;
    pa.N = NB;
    pa.direct = ctx->gather_direct ? 1 : 0;
    // about 90k pair tests per wave: enough work to hide a wave's start, and
    // waves small enough that the last ones do not run alone for long
    pa.max_blocks = ctx->pair_blocks
                        ? ctx->pair_blocks
                        : (uint32_t)std::min<uint64_t>(
                              kMaxPairBlocks,
                              std::max<uint64_t>(2048, tests_total / ((uint64_t)T.tests_per_wave *
                                                                      kWaves) + 1));
    // (with no more units than waves every wave takes at most one either way,
    // and the every-n-th dealing needs no ranges)
    if (balanced && units_total > pair_waves(pa)) {
      // each wave takes a contiguous run of units with an equal share of the
      // tile pairs, so that no wave (and no block) runs far longer than the rest
      scan_exclusive_u64(uwork, uwork, units_total, uscan + su, uscan, stream);
      launch_wave_ranges(uwork, units_total, uscan + su, pair_waves(pa), wfirst, stream);
      pa.wave_first = wfirst;
    }
    pa.sigp = first_owner ? sig : nullptr;
    pa.skeys = skeys;
    pa.sidx = sidx;
    pa.idx_bits = idx_bits;
    pa.pts = pts_rows;
    pa.rows = rec ? rec : pts_rows;
    pa.row_stride = rec ? rs : d;
    pa.sig_stride = sig_stride;
    pa.d = d;
    pa.tests = tests_d;
    pa.gram = use_gram ? 1 : 0;
    pa.unit_band = (ctx->unit_band && !P.truncated && !P.wrapped) ? 1 : 0;
    if (first_owner) {
      pa.W = sig_W;
      pa.g = sig_g;
      pa.gpw = sig_gpw;
      for (int z = 0; z < sig_gpw; ++z) {
        pa.lows |= 1ull << (z * sig_g);
        pa.highs |= 1ull << (z * sig_g + sig_g - 1);
      }
    }
    // the unit points' coordinates and signature words by sorted position
    if (!pa.direct) {
      kbegin(RTG_K_GATHER);
      launch_gather_units(pa, first_owner ? sig : nullptr, spts, ssig, stream);
      kend(RTG_K_GATHER, 0.0);
    }

    // This pass's pairs go to kCandSegments output segments, room for them
    // from a guess first and from the largest count on overflow; then one
    // copy puts them after the earlier passes' pairs in cand.
    const uint32_t nseg = kCandSegments;
    unsigned long long* segcnt = counters + 4;
    // The guess: the tests times the share of a cell's pairs that can lie
    // within r -- for two points of one cube of side alpha r at most the
    // unit ball's volume over alpha^d (the cube's edges only lower it), with a
    // quarter to spare and a sixteenth as the floor -- but at most
    // cand_per_key pairs per (point, grid) key: where few tested pairs lie
    // within r (high d, clustered points) the tests overstate the pairs a
    // thousandfold.  The cap keeps the pass inside pass_bytes_bound.
    double share = 1.0 / 16;
    for (int32_t sg = sa; sg < sb; ++sg)
      share = std::max(share, 1.25 * ball_share(d, jobs[segs[sg].inst]->alpha));
    const uint64_t per_key = cand_per_key(flags);
    const uint64_t guess = std::min<uint64_t>(
        {tests_total, std::max<uint64_t>(1u << 16, (uint64_t)(share * (double)tests_total)),
         per_key * N});
    // Where that cannot be had, a quarter of it: an overflow then costs one
    // more pair pass.
    const uint64_t lean = std::max<uint64_t>(1, guess / 4);
    uint64_t seg_cap = guess / nseg + guess / (4 * nseg) + 1024;
    for (int attempt = 0; attempt < 2; ++attempt) {
      uint64_t* sbuf = S.get<uint64_t>((size_t)nseg * seg_cap);
      if (!sbuf && attempt == 0 && lean < guess) {
        seg_cap = lean / nseg + lean / (4 * nseg) + 1024;
        sbuf = S.get<uint64_t>((size_t)nseg * seg_cap);
      }
      if (!sbuf) return RTG_ENOMEM;
      // the stage's first launch cleared them for the first pair launch
      if (sa > 0 || attempt > 0)
        launch_fill_u64(reinterpret_cast<uint64_t*>(segcnt), 0ull, nseg, stream);
      pa.cand = sbuf;
      pa.cap = seg_cap;
      pa.cand_count = segcnt;
      pa.nseg = nseg;
      pa.rechecks = counters + 1;
      kbegin(RTG_K_PAIRS);
      launch_cell_pairs(pa, stream);
      if (use_gram) st.matrix_screen_launches += 1;
      kend(RTG_K_PAIRS, 0.0);
      std::vector<unsigned long long> cnt(4 + (size_t)nseg);
      if ((rc = read_back(counters, sizeof(unsigned long long) * cnt.size(), cnt.data())))
        return rc;
      rechecks_seen = cnt[1];  // FP64 re-tests so far (a running total)
      uint64_t total = 0, most = 0;
      for (uint32_t g = 0; g < nseg; ++g) {
        total += cnt[4 + g];
        most = std::max<uint64_t>(most, cnt[4 + g]);
      }
      // every member of a multi-point cell read once (index + coordinates;
      // counters[3] = members, summed by the cell-work kernel of this pass),
      // every pair within r written once
      st.kernel_bytes[RTG_K_PAIRS] += (4.0 + 4.0 * d) * (double)cnt[3] + 8.0 * (double)total;
      if (attempt == 0 && !pa.direct)  // the gather: index, row, words in; row, words out
        st.kernel_bytes[RTG_K_GATHER] +=
            (8.0 + 8.0 * d + (first_owner ? 16.0 * sig_W : 0.0)) * (double)cnt[3];
      if (most <= seg_cap && lists_from_segments && 2 * total < (1ull << 32)) {
        seg_src = PairSource{sbuf, segcnt, seg_cap, nseg};
        cand_total += total;
        break;
      }
      if (most <= seg_cap) {
        if (cand_total + total > cap) {
          const uint64_t want = cand_total + total;
          uint64_t* grown = S.get<uint64_t>(std::max<uint64_t>(want, 1));
          if (!grown) return RTG_ENOMEM;
          if (cand && cand_total)
            if ((rc = hip_fail(hipMemcpyAsync(grown, cand, sizeof(uint64_t) * cand_total,
                                              hipMemcpyDeviceToDevice, stream),
                               "grow candidates")))
              return rc;
          if (cand) S.drop(cand);
          cand = grown;
          cap = want;
        }
        kbegin(RTG_K_COMPACT);
        launch_seg_compact(sbuf, seg_cap, segcnt, nseg, most, cand + cand_total, stream);
        kend(RTG_K_COMPACT, 16.0 * (double)total);
        cand_total += total;
        S.drop(sbuf);
        break;
      }
      S.drop(sbuf);
      seg_cap = most;
      if (attempt == 1) return RTG_ENOMEM;
    }
    mark(5);
  }
  // (each pass checked err after its key sort; the pair kernels set none)
  st.band_rechecks += (int64_t)rechecks_seen;

  // Key buffers are no longer needed.
  for (void* p : {(void*)keys, (void*)keys_alt, (void*)vals, (void*)vals_alt, (void*)cstart,
                  (void*)cend, (void*)units, (void*)udesc, (void*)spts, (void*)tests_c,
                  (void*)sig, (void*)ssig, (void*)rec})
    S.drop(p);

  // --- MR-metric: keep the Euclidean candidates within r under the MR-metric -----
  if (any_mr && cand_total > 0) {
    std::vector<MrInst> mi(m);
    for (uint32_t q = 0; q < m; ++q) mi[q] = MrInst{inst[q].pt_off, jobs[q]->r, sub[q], 0};
    MrInst* mi_d = S.get<MrInst>(m);
    uint64_t* kept = S.get<uint64_t>(cand_total);
    if (!mi_d || !kept) return RTG_ENOMEM;
    if ((rc = upload(mi_d, mi.data(), sizeof(MrInst) * m))) return rc;
    launch_fill_u64(reinterpret_cast<uint64_t*>(counters) + 2, 0ull, 1, stream);
    MrFilterArgs fa{cand, cand_total, pair_bits, d, pts_rows, pts_rows, mi_d, (int)m, kept,
                    counters + 2};
    kbegin(RTG_K_COMPACT);
    launch_mr_filter(fa, stream);
    kend(RTG_K_COMPACT, (8.0 + 8.0 * d) * (double)cand_total);  // pairs and both rows read
    unsigned long long nk = 0;
    if ((rc = read_back(counters + 2, sizeof(nk), &nk))) return rc;
    st.kernel_bytes[RTG_K_COMPACT] += 8.0 * (double)nk;  // kept pairs written
    st.band_rechecks += (int64_t)cand_total;
    S.drop(cand);
    cand = kept;
    cand_total = nk;
  }
  st.candidates += (int64_t)cand_total;

  // --- bitmap de-duplication: first arrival of each pair --------------------------
  if (bitmap && cand_total > 0) {
    BitmapInst* bmi_d = S.get<BitmapInst>(m);
    uint32_t* bits = S.get<uint32_t>(bitmap_words);
    uint64_t* uniq = S.get<uint64_t>(cand_total);
    if (!bmi_d || !bits || !uniq) return RTG_ENOMEM;
    if ((rc = upload(bmi_d, bmi.data(), sizeof(BitmapInst) * m))) return rc;
    kbegin(RTG_K_UNIQUE);
    launch_fill_u32(bits, 0u, bitmap_words, stream);
    launch_fill_u64(reinterpret_cast<uint64_t*>(counters) + 2, 0ull, 1, stream);
    BitmapArgs ba{cand, cand_total, pair_bits, (int)m, bmi_d, bits, uniq, counters + 2};
    launch_bitmap_unique(ba, stream);
    // the bitmap cleared, the candidates read, one word touched per candidate
    kend(RTG_K_UNIQUE, 4.0 * (double)bitmap_words + 12.0 * (double)cand_total);
    unsigned long long nu = 0;
    if ((rc = read_back(counters + 2, sizeof(nu), &nu))) return rc;
    st.kernel_bytes[RTG_K_UNIQUE] += 8.0 * (double)nu;  // unique pairs written
    S.drop(bits);
    S.drop(cand);
    cand = uniq;
    cand_total = nu;
  }

  // --- union and neighbour lists ------------------------------------------------
  const bool unique_pairs = first_owner || bitmap;  // no repeats among the candidates
  const size_t C = cand_total;
  if (C >= (1ull << 32)) return RTG_ENOMEM;
  // Row buckets need a 32-bit local entry (rb row bits + pair_bits) and at
  // most 2^14 buckets; larger batches take the sorted-pair build below.
  const bool bucket_ok = pair_bits <= 24 && ceil_log2((uint64_t)npts) <= 22 &&
                         ceil_log2((uint64_t)npts) - 14 + pair_bits <= 32 &&
                         (both ? 2 * C : C) < (1ull << 32);
  const uint64_t* pairs = cand;  // pairs for the neighbour-list build
  size_t npairs = C;
  if (C > 0 && (!unique_pairs || !bucket_ok)) {
    if (seg_src.pairs) return hip_fail(hipErrorUnknown, "pair segments without a row-bucket build");
    // Global sort of the packed pairs; with RTG_DEDUP_SORT also drop repeats
    // (sort-unique over every grid's candidates).
    uint64_t* cand_alt = S.get<uint64_t>(C);
    uint32_t* scr = static_cast<uint32_t*>(
        static_cast<void*>(S.get<char>(radix_scratch_bytes(C, 0, 2 * pair_bits))));
    if (!cand_alt || !scr) return RTG_ENOMEM;
    const int where = radix_sort(cand, nullptr, cand_alt, nullptr, C, 0, 2 * pair_bits, scr, err,
                                 stream, &tm, RTG_K_PAIR_HIST, RTG_K_PAIR_SCATTER, T.sort_algo);
    const uint64_t* sc = where ? cand_alt : cand;
    uint64_t* dst = where ? cand : cand_alt;
    mark(6);
    if (unique_pairs) {
      pairs = sc;  // every pair is there once
    } else {
      const size_t nt = (C + kTile - 1) / kTile;
      uint32_t* tc = scr;
      uint32_t* tot = scr + nt;
      kbegin(RTG_K_UNIQUE);
      launch_unique_count(sc, C, tc, stream);
      scan_exclusive_u32(tc, tc, nt, tot, tot + 1, stream);
      launch_unique_write(sc, C, tc, dst, stream);
      kend(RTG_K_UNIQUE, 16.0 * (double)C);
      uint32_t uh = 0;
      if ((rc = read_back(tot, sizeof(uh), &uh))) return rc;
      st.kernel_bytes[RTG_K_UNIQUE] += 8.0 * (double)uh;
      pairs = dst;
      npairs = uh;
    }
    mark(7);
  } else {
    mark(6);
    mark(7);
  }

  void* res = nullptr;
  int64_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  size_t nnz = 0;
  // drained: the list build read err after its last kernel and nothing ran since
  bool drained = false;
  uint32_t err_seen = 0;
  if (npairs == 0) {
    if ((rc = alloc_result(*this, npts, 0, &res, &row_ptr, &col))) return rc;
    launch_fill_u64(reinterpret_cast<uint64_t*>(row_ptr), 0ull, (size_t)(npts + 1), stream);
  } else if (bucket_ok) {
    const PairSource psrc = seg_src.pairs ? seg_src : PairSource{pairs};
    rc = csr_by_buckets(*this, S, T, psrc, npairs, npts, pair_bits, both, err, &tm, &res, &row_ptr,
                        &col, &nnz, &err_seen, &drained);
    if (rc) return rc;
  } else {
    nnz = both ? 2 * npairs : npairs;
    if ((rc = alloc_result(*this, npts, nnz, &res, &row_ptr, &col))) return rc;
    rc = csr_from_sorted(*this, S, T, pairs, npairs, npts, pair_bits, both, err, row_ptr, col);
    if (rc) {
      dfree(res);
      return rc;
    }
  }
  st.unique_pairs += (int64_t)(both ? nnz / 2 : nnz);

  // --- per-instance lists ------------------------------------------------------------
  if (m == 1) {
    Job& j = *jobs[0];
    j.out->n = j.n;
    j.out->nnz = (int64_t)nnz;
    j.out->row_ptr = row_ptr;
    j.out->col = nnz ? col : nullptr;
    j.out->pairs = (int64_t)(both ? nnz / 2 : nnz);
  } else {
    std::vector<int64_t> at(m + 1);
    int64_t* at_d = S.get<int64_t>(m + 1);
    if (!at_d) {
      dfree(res);
      return RTG_ENOMEM;
    }
    launch_rowptr_at(inst_d, m, row_ptr, npts, at_d, stream);
    if ((rc = read_back(at_d, sizeof(int64_t) * (m + 1), at.data()))) {
      dfree(res);
      return rc;
    }
    std::vector<void*> mem(m, nullptr);
    std::vector<int64_t*> rps(m);
    std::vector<int32_t*> cols(m);
    for (uint32_t q = 0; q < m && !rc; ++q) {
      const size_t nq = (size_t)((q + 1 < m ? at[q + 1] : at[m]) - at[q]);
      rc = alloc_result(*this, jobs[q]->n, nq, &mem[q], &rps[q], &cols[q]);
    }
    // both pointer tables in one copy from pinned memory
    Uploads Ul(*this);
    const size_t o_rp = Ul.add(rps.data(), sizeof(int64_t*) * m);
    const size_t o_col = Ul.add(cols.data(), sizeof(int32_t*) * m);
    char* tabs = rc ? nullptr : S.get<char>(Ul.total());
    if (!rc && !tabs) rc = RTG_ENOMEM;
    int64_t** rp_tab = tabs ? reinterpret_cast<int64_t**>(tabs + o_rp) : nullptr;
    int32_t** col_tab = tabs ? reinterpret_cast<int32_t**>(tabs + o_col) : nullptr;
    if (!rc) rc = Ul.send(tabs);
    if (!rc) {
      kbegin(RTG_K_CSR);
      launch_localize(inst_d, m, nblk, row_ptr, col, at_d, at[m], rp_tab, col_tab, stream);
      kend(RTG_K_CSR, 16.0 * (double)(npts + m) + 8.0 * (double)at[m]);
      rc = sync();
    }
    dfree(res);
    if (rc) {
      for (void* p : mem) dfree(p);
      return rc;
    }
    for (uint32_t q = 0; q < m; ++q) {
      Job& j = *jobs[q];
      const int64_t nq = (q + 1 < m ? at[q + 1] : at[m]) - at[q];
      j.out->n = j.n;
      j.out->nnz = nq;
      j.out->row_ptr = rps[q];
      j.out->col = nq ? cols[q] : nullptr;
      j.out->pairs = both ? nq / 2 : nq;
      j.out->handle = ctx->keep_result(j.handle, mem[q], j.n, nq, j.out->pairs, rps[q], cols[q]);
    }
  }
  mark(8);
  if ((rc = hip_fail(hipGetLastError(), "kernel launch"))) {
    if (m == 1) dfree(res);
    return rc;
  }
  {
    // Wait for the pass (the read waits) and check the sorts' error bits,
    // unless the list build already did after the last kernel (phase
    // timing needs the final event, so it always waits).
    uint32_t errh2 = err_seen;
    if (!(m == 1 && drained) || (timing_mask & RTG_TIME_PHASES))
      rc = read_back(err, sizeof(errh2), &errh2);
    if (rc || errh2) {
      if (m == 1) dfree(res);
      return rc ? rc : hip_fail(hipErrorUnknown, "radix sort look-back");
    }
  }
  kfinish();
  if (timing_mask & RTG_TIME_PHASES) {
    float ms[8] = {0};
    for (int q = 0; q < 8; ++q) (void)hipEventElapsedTime(&ms[q], ev[q], ev[q + 1]);
    st.ms_stage += ms[0];
    if (P.tb >= S_total) {
      st.ms_keys += ms[1];
      st.ms_key_sort += ms[2];
      st.ms_cells += ms[3];
      st.ms_pairs += ms[4];
    }
    st.ms_pair_sort += ms[5];
    st.ms_unique += ms[6];
    st.ms_csr += ms[7];
    float tot_ms = 0;
    (void)hipEventElapsedTime(&tot_ms, ev[0], ev[8]);
    st.ms_total += tot_ms;
  }
  if (m == 1)
    jobs[0]->out->handle =
        ctx->keep_result(jobs[0]->handle, res, jobs[0]->n, (int64_t)nnz, jobs[0]->out->pairs,
                         row_ptr, col);
  // A plan's first run leaves it a workspace of the sizes the run took up to
  // the cell stage; its later runs cut those buffers from it, at the same
  // addresses each time.  Without room the plan runs as before and tries
  // again next time.
  if (pp && !pp->ws && S.recorded) {
    pp->ws = ctx->dalloc(S.recorded);
    if (pp->ws) pp->head_bytes = S.recorded;
  }
  // The pass's last stream operation was a read-back after its last kernel
  // (the list build's, the error bits' or the localization's wait).
  S.drained = true;
  return RTG_OK;
}

// The extra lanes of the batched call (count of them), made with this
// context's device current (as the request loop's lanes are).
int Ctx::side_lanes(int count) {
  if ((int)side.size() >= count) return RTG_OK;
  if (hipSetDevice(device) != hipSuccess) return RTG_EDEVICE;
  if (!side_ready && hipEventCreateWithFlags(&side_ready, hipEventDisableTiming) != hipSuccess)
    return RTG_EDEVICE;
  while ((int)side.size() < count) {
    std::unique_ptr<Lane> L(new (std::nothrow) Lane());
    if (!L) return RTG_ENOMEM;
    const int rc = L->init(this, nullptr, true);
    if (rc) {
      L->fini();
      return rc;
    }
    side.push_back(std::move(L));
  }
  return RTG_OK;
}

// Adds the counts and times of b to a (widths: the larger).
static void add_stats(rtg_stats& a, const rtg_stats& b) {
  a.cells += b.cells;
  a.tests += b.tests;
  a.candidates += b.candidates;
  a.band_rechecks += b.band_rechecks;
  a.unique_pairs += b.unique_pairs;
  a.key_bits = std::max(a.key_bits, b.key_bits);
  a.key_passes = std::max(a.key_passes, b.key_passes);
  a.pair_bits = std::max(a.pair_bits, b.pair_bits);
  a.transforms_per_sort = std::max(a.transforms_per_sort, b.transforms_per_sort);
  a.ms_stage += b.ms_stage;
  a.ms_keys += b.ms_keys;
  a.ms_key_sort += b.ms_key_sort;
  a.ms_cells += b.ms_cells;
  a.ms_pairs += b.ms_pairs;
  a.ms_pair_sort += b.ms_pair_sort;
  a.ms_unique += b.ms_unique;
  a.ms_csr += b.ms_csr;
  a.ms_total += b.ms_total;
  for (int i = 0; i < RTG_NKERNELS; ++i) {
    a.kernel_launches[i] += b.kernel_launches[i];
    a.kernel_bytes[i] += b.kernel_bytes[i];
    a.kernel_ms[i] += b.kernel_ms[i];
  }
  a.matrix_screen_launches += b.matrix_screen_launches;
}

// Many queries: grouped by dimension and list flags, each group split into
// batches of at most batch_points points (an instance larger than that runs
// alone), every batch one pass of run_batch.
std::vector<std::vector<int32_t>> Ctx::batch_groups(const rtg_query* q, int32_t nq) {
  std::map<std::pair<int, uint32_t>, std::vector<int32_t>> groups;
  for (int32_t i = 0; i < nq; ++i)
    if (q[i].n > 1) groups[{q[i].d, q[i].flags & kListFlags}].push_back(i);
  std::vector<std::vector<int32_t>> batches;
  for (auto& g : groups) {
    size_t b = 0;
    while (b < g.second.size()) {
      std::vector<int32_t> batch;
      int64_t pts = 0;
      while (b < g.second.size() && (batch.empty() || pts + q[g.second[b]].n <= batch_points)) {
        pts += q[g.second[b]].n;
        batch.push_back(g.second[b]);
        ++b;
      }
      batches.push_back(std::move(batch));
    }
  }
  return batches;
}

int Ctx::batched(const rtg_query* q, int32_t nq, rtg_csr* outs,
                 std::vector<std::unique_ptr<PassPlan>>* plan) {
  if (poisoned) return RTG_EDEVICE;
  int rc;
  for (int32_t i = 0; i < nq; ++i)
    if ((rc = check_query(q[i].points, q[i].n, q[i].d, q[i].r, q[i].k, q[i].alpha, q[i].flags)))
      return rc;
  std::vector<std::vector<double>> R(nq), u(nq);
  for (int32_t i = 0; i < nq; ++i) {
    R[i].resize((size_t)q[i].k * q[i].d * q[i].d);
    u[i].resize((size_t)q[i].k * q[i].d);
    if ((rc = make_transforms(q[i].seed, q[i].k, q[i].d, q[i].flags, R[i].data(), u[i].data())))
      return rc;
  }
  const std::vector<std::vector<int32_t>> groups = batch_groups(q, nq);
  if (plan) {
    if (plan->empty())
      for (size_t b = 0; b < groups.size(); ++b) plan->emplace_back(new PassPlan);
    if (plan->size() != groups.size()) return RTG_EINVAL;
  }
  std::vector<rtg_csr> res(nq);
  std::vector<char> done(nq, 0);
  auto undo = [&](int code) {
    for (int32_t i = 0; i < nq; ++i)
      if (done[i]) release(res[i].handle);
    return code;
  };
  rtg_stats st{};
  std::vector<Job> jobs(nq);
  for (int32_t i = 0; i < nq; ++i) {
    st.n += q[i].n;
    st.point_transforms += q[i].n * q[i].k;
    if (q[i].n <= 1) {
      if ((rc = main.tiny_query(q[i].points, q[i].n, q[i].d, &res[i], 0))) return undo(rc);
      done[i] = 1;
      continue;
    }
    jobs[i] = Job{q[i].points, q[i].n, q[i].d, q[i].r, q[i].alpha, q[i].k, q[i].flags,
                  R[i].data(), u[i].data(), &res[i], 0};
  }
  // One small instance: the two-launch path, as rtg_all_pairs takes it
  // (nothing is captured for it)
  if (nq == 1 && small_fits(q[0].n, q[0].d, q[0].k, q[0].flags)) {
    rc = main.run_tiny(jobs[0], st);
    if (rc != Lane::kTinyFallback) {
      if (rc) return rc;
      outs[0] = res[0];
      st.d = q[0].d;
      st.k = q[0].k;
      stats = st;
      return RTG_OK;
    }
  }
  std::vector<std::vector<Job*>> batches;
  for (const auto& g : groups) {
    batches.emplace_back();
    for (int32_t i : g) batches.back().push_back(&jobs[i]);
  }
  auto pass_plan = [&](size_t b) { return plan ? (*plan)[b].get() : nullptr; };
  // Several batches: two lanes take them in turn.  A batch that runs out of
  // memory beside the other lane's pass runs again alone afterwards.
  constexpr int kNotRun = 1 << 20;
  std::vector<int> brc(batches.size(), kNotRun);
  const int extra = (int)std::min<size_t>(batch_lanes - 1, batches.size() - 1);
  if (batches.size() >= 2 && extra > 0 && side_lanes(extra) == RTG_OK) {
    if ((rc = hip_fail(hipEventRecord(side_ready, main.stream), "hipEventRecord"))) return undo(rc);
    for (int l = 0; l < extra; ++l) {
      if ((rc = hip_fail(hipStreamWaitEvent(side[l]->stream, side_ready, 0), "hipStreamWaitEvent")))
        return undo(rc);
      side[l]->timing_mask = main.timing_mask;
    }
    std::atomic<size_t> next{0};
    std::atomic<bool> failed{false};
    auto work = [&](Lane& L, rtg_stats& s) {
      for (;;) {
        if (failed) return;
        const size_t b = next++;
        if (b >= batches.size()) return;
        brc[b] = L.run_batch(batches[b], s, pass_plan(b));
        if (brc[b] == RTG_OK)
          for (Job* j : batches[b]) done[j->out - res.data()] = 1;
        else if (brc[b] != RTG_ENOMEM)
          failed = true;
      }
    };
    std::vector<rtg_stats> sst(extra, rtg_stats{});
    std::vector<std::thread> threads;
    for (int l = 0; l < extra; ++l)
      threads.emplace_back([&, l] {
        (void)hipSetDevice(device);
        work(*side[l], sst[l]);
      });
    work(main, st);
    for (auto& t : threads) t.join();
    // The extra lanes go with the call: their streams would otherwise keep
    // hardware queues (a few per process) that the request loop's lanes need.
    for (auto& L : side) L->fini();
    side.clear();
    for (const auto& s2 : sst) add_stats(st, s2);
    for (int r : brc)
      if (r != RTG_OK && r != RTG_ENOMEM && r != kNotRun) return undo(r);
  }
  for (size_t b = 0; b < batches.size(); ++b) {
    if (brc[b] == RTG_OK) continue;
    if ((rc = main.run_batch(batches[b], st, pass_plan(b)))) return undo(rc);
    for (Job* j : batches[b]) done[j->out - res.data()] = 1;
  }
  for (int32_t i = 0; i < nq; ++i) outs[i] = res[i];
  st.d = nq ? q[0].d : 0;
  st.k = nq ? q[0].k : 0;
  stats = st;
  return RTG_OK;
}

int Ctx::debug_cell_coords(const float* points, int64_t n, int32_t d, double r, double alpha,
                           const double* R, const double* u, int64_t* kappa_host) {
  if (poisoned) return RTG_EDEVICE;
  int rc = validate_query(points, n, d, r, 1, alpha);
  if (rc) return rc;
  if (n == 0) return RTG_OK;
  if (check_device_pointer(points, device)) return RTG_EINVAL;
  Lane& L = main;
  Scratch S(L);
  float* soa = S.get<float>((size_t)n * d);
  uint32_t* flags_dev = S.get<uint32_t>(2 + 2 * kMaxDim);
  double* Rd = S.get<double>((size_t)d * d);
  double* ud = S.get<double>((size_t)d);
  int64_t* kap = S.get<int64_t>((size_t)n * d);
  if (!soa || !flags_dev || !Rd || !ud || !kap) return RTG_ENOMEM;
  if ((rc = L.upload(Rd, R, sizeof(double) * d * d)) || (rc = L.upload(ud, u, sizeof(double) * d)))
    return rc;
  const uint32_t nblk = (uint32_t)((n + kBlock - 1) / kBlock);
  uint32_t* stage_part = S.get<uint32_t>((size_t)nblk * 2 * d);
  InstDesc* inst_d = S.get<InstDesc>(1);
  if (!stage_part || !inst_d) return RTG_ENOMEM;
  InstDesc one{};
  one.pts = points;
  one.n = n;
  if ((rc = L.upload(inst_d, &one, sizeof(one)))) return rc;
  launch_fill_u32(flags_dev + 1, 0u, 1, L.stream);
  launch_stage(inst_d, 1, nblk, d, n, soa, nullptr, flags_dev, flags_dev + 2, stage_part, nullptr,
               0, L.stream);
  launch_cell_coords(soa, n, d, Rd, ud, 1.0 / (alpha * r), kap, flags_dev + 1, L.stream);
  uint32_t fl[2];
  if ((rc = L.read_back(flags_dev, sizeof(fl), fl))) return rc;
  if (fl[0]) return RTG_EINVAL;
  if (fl[1]) return RTG_ERANGE;
  return L.download(kappa_host, kap, sizeof(int64_t) * (size_t)n * d);
}

// ---------------------------------------------------------------------------
// parameter choice

namespace {

// Quadrature of the recall model: radii at the midpoints of v in [0, 1]
// with rho / r = v^(1/d) (which turns the density d x^(d-1) into a uniform
// one), directions from a fixed SplitMix64 stream of Gaussian vectors.
constexpr int kModelRadii = 48;
constexpr int kModelDirs = 2048;
constexpr int kModelDirsFixed = 512;  // directions kept per radius for shift-only grids

struct RecallModel {
  int d = 0;
  std::vector<double> x;      // rho / r at the quadrature radii
  std::vector<double> dirs;   // [kModelDirs][d] |u_j| of unit directions

  explicit RecallModel(int dim) : d(dim) {
    for (int i = 0; i < kModelRadii; ++i)
      x.push_back(std::pow((i + 0.5) / kModelRadii, 1.0 / d));
    SplitMix64 g{0x5EEDC0FFEEull + (uint64_t)d};
    dirs.resize((size_t)kModelDirs * d);
    for (int q = 0; q < kModelDirs; ++q) {
      double nrm = 0.0;
      for (int j = 0; j < d; j += 2) {
        double pr[2];
        polar_normals(g, pr);
        for (int e = 0; e < 2 && j + e < d; ++e) {
          dirs[(size_t)q * d + j + e] = pr[e];
          nrm += pr[e] * pr[e];
        }
      }
      nrm = std::sqrt(nrm);
      for (int j = 0; j < d; ++j) dirs[(size_t)q * d + j] = std::fabs(dirs[(size_t)q * d + j]) / nrm;
    }
  }

  // P(one grid holds the pair) for displacement x * r along direction q
  double cocell(int q, double xr_over_c) const {
    double p = 1.0;
    for (int j = 0; j < d && p > 0.0; ++j) p *= std::max(0.0, 1.0 - xr_over_c * dirs[(size_t)q * d + j]);
    return p;
  }

  // One-grid probabilities at the quadrature radii for cell factor alpha:
  // averaged over directions (rotate), else per (radius, direction).
  std::vector<double> probs(double alpha, bool rotate) const {
    std::vector<double> p(rotate ? x.size() : x.size() * kModelDirsFixed, 0.0);
    for (size_t i = 0; i < x.size(); ++i) {
      const double s = x[i] / alpha;
      if (rotate) {
        for (int q = 0; q < kModelDirs; ++q) p[i] += cocell(q, s) / kModelDirs;
      } else {
        for (int q = 0; q < kModelDirsFixed; ++q) p[i * kModelDirsFixed + q] = cocell(q, s);
      }
    }
    return p;
  }

  // E[1 - (1 - p)^k] over the quadrature (p from probs()).
  static double recall_of(const std::vector<double>& p, int k, bool rotate) {
    double acc = 0.0;
    for (double pi : p) acc += 1.0 - std::pow(1.0 - pi, k);
    return acc / (double)(rotate ? kModelRadii : (size_t)kModelRadii * kModelDirsFixed);
  }

  double recall(int k, double alpha, bool rotate) const {
    return recall_of(probs(alpha, rotate), k, rotate);
  }
};

// Relative cost of one pair test against one point under one grid, from the
// measured time split of the uniform d6 benchmark (keys, sort, cells and
// lists per point-grid against the pair screen per test).
constexpr double kTestCost = 0.0134;

double unit_ball_volume(int d) { return std::pow(M_PI, d / 2.0) / std::tgamma(d / 2.0 + 1.0); }

}  // namespace

int model_recall(int32_t d, int32_t k, double alpha, uint32_t flags, double* recall) {
  if (d < 1 || d > kMaxDim || k < 1 || !(alpha > 0.0) || !std::isfinite(alpha) || !recall)
    return RTG_EINVAL;
  RecallModel M(d);
  *recall = M.recall(k, alpha, !(flags & RTG_NO_ROTATE));
  return RTG_OK;
}

int least_grids(int32_t d, double alpha, double target, uint32_t flags, int32_t kmax,
                int32_t* k_out, double* recall_out) {
  if (d < 1 || d > kMaxDim || !(alpha > 0.0) || !(target > 0.0 && target < 1.0) || kmax < 1)
    return RTG_EINVAL;
  const bool rotate = !(flags & RTG_NO_ROTATE);
  RecallModel M(d);
  const std::vector<double> p = M.probs(alpha, rotate);
  if (RecallModel::recall_of(p, kmax, rotate) < target) return RTG_ERANGE;
  int lo = 1, hi = kmax;
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    if (RecallModel::recall_of(p, mid, rotate) >= target) hi = mid;
    else lo = mid + 1;
  }
  *k_out = lo;
  *recall_out = RecallModel::recall_of(p, lo, rotate);
  return RTG_OK;
}

int choose_params(int32_t d, double target, double nu, uint32_t flags, int32_t* k_out,
                  double* alpha_out, double* recall_out) {
  if (d < 1 || d > kMaxDim || !(target > 0.0 && target < 1.0) || !(nu > 0.0) ||
      !std::isfinite(nu) || !k_out || !alpha_out || !recall_out)
    return RTG_EINVAL;
  const bool rotate = !(flags & RTG_NO_ROTATE);
  RecallModel M(d);
  const double zeta = unit_ball_volume(d);
  double best = INFINITY, best_alpha = 0.0, best_recall = 0.0;
  int best_k = 0;
  for (int a = 32; a <= 256; a += 2) {
    const double alpha = a / 64.0;
    const std::vector<double> p = M.probs(alpha, rotate);
    // least k reaching the target: recall rises with k (bisection)
    int lo = 1, hi = 1024;
    if (RecallModel::recall_of(p, hi, rotate) < target) continue;
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (RecallModel::recall_of(p, mid, rotate) >= target) hi = mid;
      else lo = mid + 1;
    }
    const double cost = lo * (1.0 + kTestCost * nu * std::pow(alpha, d) / (2.0 * zeta));
    if (cost < best) {
      best = cost;
      best_k = lo;
      best_alpha = alpha;
      best_recall = RecallModel::recall_of(p, lo, rotate);
    }
  }
  if (!best_k) return RTG_ERANGE;
  *k_out = best_k;
  *alpha_out = best_alpha;
  *recall_out = best_recall;
  return RTG_OK;
}

// ---------------------------------------------------------------------------
// query mode

// The sorted grids of one point set (steps A1-A3 of the pipeline, single
// instance), kept with a copy of the points and their signatures.
int Lane::build_index(const float* points, int64_t n, int32_t d, double r, int32_t k,
                      double alpha, const double* R, const double* u, Index& I) {
  int rc;
  I.n = n;
  I.d = d;
  I.k = k;
  I.r = r;
  I.alpha = alpha;
  auto own = [&](size_t bytes) -> void* {
    void* p = dalloc(std::max<size_t>(bytes, 1));
    if (p) I.blocks.push_back(p);
    return p;
  };
  I.R = static_cast<double*>(own(sizeof(double) * (size_t)k * d * d));
  I.u = static_cast<double*>(own(sizeof(double) * (size_t)k * d));
  I.grids = static_cast<QueryGrid*>(own(sizeof(QueryGrid) * (size_t)k));
  I.layout = static_cast<KeyLayout*>(own(sizeof(KeyLayout)));
  I.klo = static_cast<int64_t*>(own(sizeof(int64_t) * (size_t)k * d));
  if (!I.R || !I.u || !I.grids || !I.layout || !I.klo) return RTG_ENOMEM;
  if ((rc = upload(I.R, R, sizeof(double) * (size_t)k * d * d))) return rc;
  if ((rc = upload(I.u, u, sizeof(double) * (size_t)k * d))) return rc;
  if (n == 0) return sync();

  Scratch S(*this);
  I.pts = static_cast<float*>(own(sizeof(float) * (size_t)n * d));
  if (!I.pts) return RTG_ENOMEM;
  if ((rc = hip_fail(hipMemcpyAsync(I.pts, points, sizeof(float) * (size_t)n * d,
                                    hipMemcpyDeviceToDevice, stream),
                     "copy index points")))
    return rc;

  // stage: SoA copy, finiteness, bounding box
  const uint32_t nblk = (uint32_t)((n + kBlock - 1) / kBlock);
  InstDesc one{};
  one.pts = I.pts;
  one.n = n;
  one.inv_c = 1.0 / (alpha * r);
  one.k = k;
  InstDesc* inst_d = S.get<InstDesc>(1);
  float* soa = S.get<float>((size_t)n * d);
  uint32_t* part = S.get<uint32_t>((size_t)nblk * 2 * d);
  uint32_t* bbox = S.get<uint32_t>((size_t)2 * d + 2);
  SegDesc* segs_d = S.get<SegDesc>((size_t)k);
  if (!inst_d || !soa || !part || !bbox || !segs_d) return RTG_ENOMEM;
  uint32_t* bad = bbox + 2 * d;
  uint32_t* err = bad + 1;
  if ((rc = upload(inst_d, &one, sizeof(one)))) return rc;
  launch_fill_u32(err, 0u, 1, stream);
  launch_stage(inst_d, 1, nblk, d, n, soa, nullptr, bad, bbox, part, nullptr, 0, stream);
  std::vector<uint32_t> hb((size_t)2 * d + 1);
  if ((rc = download(hb.data(), bbox, sizeof(uint32_t) * hb.size()))) return rc;
  if (hb[(size_t)2 * d]) return RTG_EINVAL;
  std::vector<float> lo(d), hi(d);
  for (int j = 0; j < d; ++j) {
    lo[j] = decode_order(hb[2 * j]);
    hi[j] = decode_order(hb[2 * j + 1]);
  }
  const int64_t kk = k, nn = n;
  if ((rc = plan_batch(d, 1, &kk, &nn, R, u, &one.inv_c, &alpha, lo.data(), hi.data(),
                       ctx->largest_free() / 2, I.P)))
    return rc;
  if ((rc = upload(I.layout, &I.P.layout, sizeof(KeyLayout)))) return rc;
  if ((rc = upload(I.klo, I.P.klo.data(), sizeof(int64_t) * I.P.klo.size()))) return rc;

  // signatures of the first-owner rule (keys that fit imply groups that fit)
  I.sig_b = min_field_bits(alpha);
  I.sig_g = d * I.sig_b;
  if (I.sig_g > 64) return RTG_ERANGE;
  I.sig_gpw = 64 / I.sig_g;
  I.sig_W = (k + I.sig_gpw - 1) / I.sig_gpw;
  for (int z = 0; z < I.sig_gpw; ++z) {
    I.lows |= 1ull << (z * I.sig_g);
    I.highs |= 1ull << (z * I.sig_g + I.sig_g - 1);
  }
  I.sig = static_cast<uint64_t*>(own(sizeof(uint64_t) * (size_t)n * I.sig_W));
  if (!I.sig) return RTG_ENOMEM;
  launch_fill_u64(I.sig, 0ull, (size_t)n * I.sig_W, stream);

  // keys and sort, pass by pass; each grid's n sorted keys are kept
  std::vector<SegDesc> segs((size_t)k);
  std::vector<QueryGrid> grids((size_t)k);
  const int pair_bits = std::max(1, ceil_log2((uint64_t)n));
  for (int32_t sa = 0; sa < k; sa += I.P.tb) {
    const int32_t sb = std::min(k, sa + I.P.tb);
    for (int32_t t = sa; t < sb; ++t) segs[t] = SegDesc{(int64_t)(t - sa) * n, 0, t};
  }
  if ((rc = upload(segs_d, segs.data(), sizeof(SegDesc) * segs.size()))) return rc;
  for (int32_t sa = 0; sa < k; sa += I.P.tb) {
    const int32_t sb = std::min(k, sa + I.P.tb);
    const size_t N = (size_t)(sb - sa) * n;
    const int seg_bits = (sb - sa) > 1 ? ceil_log2((uint64_t)(sb - sa)) : 0;
    const int key_bits = seg_bits + I.P.layout.cell_bits;
    const int idx_bits = (key_bits + pair_bits <= 64) ? pair_bits : 0;
    uint64_t* keys = static_cast<uint64_t*>(own(sizeof(uint64_t) * N));
    uint64_t* keys_alt = static_cast<uint64_t*>(own(sizeof(uint64_t) * N));
    uint32_t* vals = idx_bits ? nullptr : static_cast<uint32_t*>(own(sizeof(uint32_t) * N));
    uint32_t* vals_alt = idx_bits ? nullptr : static_cast<uint32_t*>(own(sizeof(uint32_t) * N));
    void* scr = S.get<char>(radix_scratch_bytes(N, 0, key_bits, (size_t)(sb - sa)));
    if (!keys || !keys_alt || (!idx_bits && (!vals || !vals_alt)) || !scr) return RTG_ENOMEM;
    KeysArgs ka{inst_d, 1, nblk, d, n, soa, sa, sb, segs_d, I.R, I.u, I.klo, I.layout,
                keys, vals, err, I.sig, I.sig_W, I.sig_b, I.sig_gpw, idx_bits};
    launch_keys(ka, stream);
    // several grids in the sort: within grids, on the cell bits only
    const bool segmented = seg_bits > 0 && ctx->defaults.sort_algo == kSortReduceScan;
    SortTile* tab_d = nullptr;
    uint32_t ntab = 0;
    if (segmented) {
      std::vector<uint64_t> soff, slen;
      for (int32_t t = sa; t < sb; ++t) {
        soff.push_back((uint64_t)(t - sa) * (uint64_t)n);
        slen.push_back((uint64_t)n);
      }
      const std::vector<SortTile> tab = segment_tiles(soff, slen);
      ntab = (uint32_t)tab.size();
      Uploads Ut(*this);
      const size_t o_tab = Ut.add(tab.data(), sizeof(SortTile) * tab.size());
      char* tab_mem = S.get<char>(Ut.total());
      if (!tab_mem) return RTG_ENOMEM;
      tab_d = reinterpret_cast<SortTile*>(tab_mem + o_tab);
      if ((rc = Ut.send(tab_mem))) return rc;
    }
    const int sort_end = idx_bits + (segmented ? I.P.layout.cell_bits : key_bits);
    const int where = radix_sort(keys, vals, keys_alt, vals_alt, N, idx_bits, sort_end, scr, err,
                                 stream, nullptr, 0, 0, ctx->defaults.sort_algo, tab_d, ntab);
    uint64_t* sorted = where ? keys_alt : keys;
    uint32_t* sorted_idx = idx_bits ? nullptr : (where ? vals_alt : vals);
    if ((rc = sync())) return rc;  // the other buffers go back below
    for (void* p : {(void*)(where ? keys : keys_alt), (void*)(where ? vals : vals_alt)}) {
      if (!p) continue;
      auto it = std::find(I.blocks.begin(), I.blocks.end(), p);
      if (it != I.blocks.end()) I.blocks.erase(it);
      dfree(p);
    }
    for (int32_t t = sa; t < sb; ++t)
      grids[t] = QueryGrid{sorted + (size_t)(t - sa) * n,
                           sorted_idx ? sorted_idx + (size_t)(t - sa) * n : nullptr,
                           (uint64_t)(t - sa), idx_bits, 0};
  }
  if ((rc = upload(I.grids, grids.data(), sizeof(QueryGrid) * grids.size()))) return rc;
  uint32_t errh = 0;
  if ((rc = read_back(err, sizeof(errh), &errh))) return rc;
  if (errh & 1u) return RTG_ERANGE;
  if (errh) return hip_fail(hipErrorUnknown, "radix sort look-back");
  return RTG_OK;
}

int Lane::query_index(const Index& I, const float* queries, int64_t m, rtg_stats& st,
                      rtg_csr* out) {
  int rc;
  if (m == 0 || I.n == 0) return make_empty_result(m, out, 0);
  kstats = &st;
  kpending.clear();
  struct Detach {
    Lane& c;
    ~Detach() {
      c.kpending.clear();
      c.kstats = nullptr;
    }
  } detach{*this};
  Scratch S(*this);
  const int k = I.k, d = I.d;
  uint64_t* qkey = S.get<uint64_t>((size_t)m * k);
  uint64_t* qsig = S.get<uint64_t>((size_t)m * I.sig_W);
  uint32_t* err = S.get<uint32_t>(2);
  unsigned long long* counter = S.get<unsigned long long>(1);
  if (!qkey || !qsig || !err || !counter) return RTG_ENOMEM;
  launch_fill_u32(err, 0u, 2, stream);
  QueryArgs A{};
  A.queries = queries;
  A.m = m;
  A.d = d;
  A.k = k;
  A.R = I.R;
  A.u = I.u;
  A.inv_c = 1.0 / (I.alpha * I.r);
  A.r2 = I.sub ? mr_screen_r2(I.r) : I.r * I.r;
  A.klo = I.klo;
  A.layout = I.layout;
  A.cell_bits = I.P.layout.cell_bits;
  A.grids = I.grids;
  A.n = I.n;
  A.pts = I.pts;
  A.sig = I.sig;
  A.W = I.sig_W;
  A.sig_b = I.sig_b;
  A.g = I.sig_g;
  A.gpw = I.sig_gpw;
  A.lows = I.lows;
  A.highs = I.highs;
  A.qkey = qkey;
  A.qsig = qsig;
  A.err = err;
  A.pb = std::max(1, ceil_log2((uint64_t)std::max<int64_t>(I.n, m)));
  launch_query_keys(A, stream);
  uint32_t errh = 0;
  if ((rc = read_back(err, sizeof(errh), &errh))) return rc;
  if (errh & 2u) return RTG_EINVAL;
  if (errh & 1u) return RTG_ERANGE;

  // pairs (query, point); room from a guess, the exact count on overflow
  uint64_t cap = std::max<uint64_t>(1u << 20, (uint64_t)m * 32);
  uint64_t* cand = nullptr;
  uint64_t C = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (cand) S.drop(cand);
    cand = S.get<uint64_t>(cap);
    if (!cand) return RTG_ENOMEM;
    launch_fill_u64(reinterpret_cast<uint64_t*>(counter), 0ull, 1, stream);
    A.cand = cand;
    A.cap = cap;
    A.cand_count = counter;
    kbegin(RTG_K_PAIRS);
    launch_query_pairs(A, stream);
    kend(RTG_K_PAIRS, 0.0);
    unsigned long long cnt = 0;
    if ((rc = read_back(counter, sizeof(cnt), &cnt))) return rc;
    C = cnt;
    if (C <= cap) break;
    if (attempt == 1) return RTG_ENOMEM;
    cap = C;
  }
  if (I.sub && C > 0) {
    // MR-metric: keep the Euclidean candidates within r under the MR-metric
    MrInst mi{0, I.r, I.sub, 0};
    MrInst* mi_d = S.get<MrInst>(1);
    uint64_t* kept = S.get<uint64_t>(C);
    if (!mi_d || !kept) return RTG_ENOMEM;
    if ((rc = upload(mi_d, &mi, sizeof(mi)))) return rc;
    launch_fill_u64(reinterpret_cast<uint64_t*>(counter), 0ull, 1, stream);
    MrFilterArgs fa{cand, C, A.pb, d, queries, I.pts, mi_d, 1, kept, counter};
    kbegin(RTG_K_COMPACT);
    launch_mr_filter(fa, stream);
    kend(RTG_K_COMPACT, (8.0 + 8.0 * d) * (double)C);
    unsigned long long nk = 0;
    if ((rc = read_back(counter, sizeof(nk), &nk))) return rc;
    st.kernel_bytes[RTG_K_COMPACT] += 8.0 * (double)nk;
    st.band_rechecks = (int64_t)C;
    S.drop(cand);
    cand = kept;
    C = nk;
  }
  st.candidates = (int64_t)C;
  st.unique_pairs = (int64_t)C;

  // lists: rows are the queries, one orientation
  void* res = nullptr;
  int64_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  size_t nnz = 0;
  const int pb = A.pb;
  const bool bucket_ok = pb <= 24 && ceil_log2((uint64_t)m) <= 22 &&
                         ceil_log2((uint64_t)m) - 14 + pb <= 32 && C < (1ull << 32);
  if (C == 0) {
    if ((rc = alloc_result(*this, m, 0, &res, &row_ptr, &col))) return rc;
    launch_fill_u64(reinterpret_cast<uint64_t*>(row_ptr), 0ull, (size_t)(m + 1), stream);
  } else if (bucket_ok) {
    if ((rc = csr_by_buckets(*this, S, ctx->defaults, PairSource{cand}, C, m, pb, false, err + 1,
                             nullptr, &res, &row_ptr, &col, &nnz)))
      return rc;
  } else {
    uint64_t* alt = S.get<uint64_t>(C);
    void* scr = S.get<char>(radix_scratch_bytes(C, 0, 2 * pb));
    if (!alt || !scr) return RTG_ENOMEM;
    launch_fill_u32(err + 1, 0u, 1, stream);
    const int where = radix_sort(cand, nullptr, alt, nullptr, C, 0, 2 * pb, scr, err + 1, stream,
                                 nullptr, 0, 0, ctx->defaults.sort_algo);
    nnz = C;
    if ((rc = alloc_result(*this, m, nnz, &res, &row_ptr, &col))) return rc;
    if ((rc = csr_from_sorted(*this, S, ctx->defaults, where ? alt : cand, C, m, pb, false,
                              err + 1, row_ptr, col))) {
      dfree(res);
      return rc;
    }
  }
  if ((rc = sync())) {
    dfree(res);
    return rc;
  }
  out->n = m;
  out->nnz = (int64_t)nnz;
  out->row_ptr = row_ptr;
  out->col = nnz ? col : nullptr;
  out->pairs = (int64_t)nnz;
  out->handle = ctx->keep_result(0, res, m, (int64_t)nnz, (int64_t)nnz, row_ptr, col);
  kfinish();
  return RTG_OK;
}

}  // namespace rtg

// ===========================================================================
// C-ABI

using rtg::Ctx;

extern "C" {

int rtg_create(rtg_ctx** out, int device, void* arena, size_t arena_bytes, void* hip_stream) {
  if (!out || arena_bytes < (1u << 20)) return RTG_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RTG_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return RTG_EDEVICE;
  Ctx* c = new (std::nothrow) Ctx(device);
  if (!c) return RTG_ENOMEM;
  if (!arena) {
    if (hipMalloc(&c->arena_mem, arena_bytes) != hipSuccess) {
      delete c;
      return RTG_ENOMEM;
    }
    c->own_arena = true;
    arena = c->arena_mem;
  }
  c->arena.reset(new rtg::Arena(static_cast<char*>(arena), arena_bytes));
  c->load_tuning_from_env();
  int rc = c->main.init(c, static_cast<hipStream_t>(hip_stream), false);
  // pinned staging large enough that rtg_all_pairs_noalloc never grows it
  if (!rc) rc = c->main.up_room(rtg::kNoallocStaging);
  if (rc) {
    delete c;
    return rc;
  }
  // The no-allocation entry point's device array on this device (current).
  void* np = nullptr;
  if (rtgk::noalloc_scratch_address(&np) == 0 && np) {
    c->noalloc_base = np;
    c->noalloc_arena.reset(new rtg::Arena(static_cast<char*>(np), rtgk::kNoallocBytes));
  }
  *out = reinterpret_cast<rtg_ctx*>(c);
  return RTG_OK;
}

int rtg_destroy(rtg_ctx* ctx) {
  if (!ctx) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  c->stop_server();
  (void)hipStreamSynchronize(c->main.stream);
  delete c;
  return RTG_OK;
}

int rtg_all_pairs(rtg_ctx* ctx, const float* points, int64_t n, int32_t d, double r, int32_t k,
                  double alpha, uint64_t seed, uint32_t flags, rtg_csr* out) {
  if (!ctx || !out) return RTG_EINVAL;
  int rc = rtg::validate_query(points, n, d, r, k, alpha);
  if (rc) return rc;
  std::vector<double> R((size_t)k * d * d), u((size_t)k * d);
  if ((rc = rtg::make_transforms(seed, k, d, flags, R.data(), u.data()))) return rc;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  return c->all_pairs(points, n, d, r, k, alpha, R.data(), u.data(), flags, out);
}

int rtg_all_pairs_with_transforms(rtg_ctx* ctx, const float* points, int64_t n, int32_t d, double r,
                                  int32_t k, double alpha, const double* R, const double* u,
                                  uint32_t flags, rtg_csr* out) {
  if (!ctx || !out || !R || !u) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  return c->all_pairs(points, n, d, r, k, alpha, R, u, flags, out);
}

int rtg_all_pairs_noalloc(rtg_ctx* ctx, const float* points, int64_t n, int32_t d, double r,
                          int32_t k, double alpha, uint64_t seed, uint32_t flags, int64_t* row_ptr,
                          int32_t* col, int64_t col_capacity, int64_t* nnz) {
  if (!ctx || !row_ptr || !nnz || col_capacity < 0 || (col_capacity > 0 && !col))
    return RTG_EINVAL;
  int rc = rtg::validate_query(points, n, d, r, k, alpha);
  if (rc) return rc;
  std::vector<double> R((size_t)k * d * d), u((size_t)k * d);
  if ((rc = rtg::make_transforms(seed, k, d, flags, R.data(), u.data()))) return rc;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  return c->all_pairs_noalloc(points, n, d, r, k, alpha, R.data(), u.data(), flags, row_ptr, col,
                              col_capacity, nnz);
}

int rtg_release(rtg_ctx* ctx, uint64_t handle) {
  if (!ctx) return RTG_EINVAL;
  return reinterpret_cast<Ctx*>(ctx)->release(handle);
}

int rtg_release_many(rtg_ctx* ctx, const uint64_t* handles, int32_t count) {
  if (!ctx || count < 0 || (count > 0 && !handles)) return RTG_EINVAL;
  return reinterpret_cast<Ctx*>(ctx)->release_many(handles, count);
}

int rtg_index_build(rtg_ctx* ctx, const float* points, int64_t n, int32_t d, double r, int32_t k,
                    double alpha, uint64_t seed, uint32_t flags, uint64_t* index) {
  if (!ctx || !index) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->poisoned) return RTG_EDEVICE;
  int rc = c->check_query(points, n, d, r, k, alpha, flags);
  if (rc) return rc;
  std::vector<double> R((size_t)k * d * d), u((size_t)k * d);
  if ((rc = rtg::make_transforms(seed, k, d, flags, R.data(), u.data()))) return rc;
  std::unique_ptr<rtg::Index> I(new (std::nothrow) rtg::Index());
  if (!I) return RTG_ENOMEM;
  I->sub = rtg::axes_per_robot(d, flags);
  rc = c->main.build_index(points, n, d, r, k, alpha, R.data(), u.data(), *I);
  if (rc) {
    (void)hipStreamSynchronize(c->main.stream);
    for (void* p : I->blocks) c->dfree(p);
    return rc;
  }
  const uint64_t h = c->new_handle();
  {
    std::lock_guard<std::mutex> alk(c->amu);
    c->indexes[h] = std::move(I);
  }
  *index = h;
  return RTG_OK;
}

int rtg_index_query(rtg_ctx* ctx, uint64_t index, const float* queries, int64_t m,
                    rtg_csr* out) {
  if (!ctx || !out) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->poisoned) return RTG_EDEVICE;
  const rtg::Index* I = nullptr;
  {
    std::lock_guard<std::mutex> alk(c->amu);
    auto it = c->indexes.find(index);
    if (it == c->indexes.end()) return RTG_ENOENT;
    I = it->second.get();
  }
  if (m < 0 || m >= (int64_t(1) << 31)) return RTG_EINVAL;
  if (m > 0 && (!queries || (reinterpret_cast<uintptr_t>(queries) & 3u) ||
                rtg::check_device_pointer(queries, c->device)))
    return RTG_EINVAL;
  rtg_stats st{};
  st.n = m;
  st.d = I->d;
  st.k = I->k;
  const int rc = c->main.query_index(*I, queries, m, st, out);
  if (!rc) c->stats = st;
  return rc;
}

int rtg_choose_params(int32_t d, double target_recall, double mean_neighbours, uint32_t flags,
                      int32_t* k, double* alpha, double* recall) {
  return rtg::choose_params(d, target_recall, mean_neighbours, flags, k, alpha, recall);
}

int rtg_model_recall(int32_t d, int32_t k, double alpha, uint32_t flags, double* recall) {
  return rtg::model_recall(d, k, alpha, flags, recall);
}

int rtg_make_transforms(uint64_t seed, int32_t k, int32_t d, uint32_t flags, double* R, double* u) {
  return rtg::make_transforms(seed, k, d, flags, R, u);
}

int rtg_set_timing(rtg_ctx* ctx, uint32_t mask) {
  if (!ctx) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  c->main.timing_mask = mask;
  return RTG_OK;
}

int rtg_get_stats(rtg_ctx* ctx, rtg_stats* out) {
  if (!ctx || !out) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  {
    std::lock_guard<std::mutex> lk(c->mu);
    *out = c->stats;
  }
  out->served_requests = c->served_requests;
  out->served_batches = c->served_batches;
  out->served_small = c->served_small;
  return RTG_OK;
}

int rtg_debug_cell_coords(rtg_ctx* ctx, const float* points, int64_t n, int32_t d, double r,
                          double alpha, const double* R, const double* u, int64_t* kappa) {
  if (!ctx || !R || !u || (n > 0 && !kappa)) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  return c->debug_cell_coords(points, n, d, r, alpha, R, u, kappa);
}

const char* rtg_strerror(int status) {
  switch (status) {
    case RTG_OK: return "ok";
    case RTG_EAGAIN: return "request not finished";
    case RTG_EINVAL: return "invalid argument";
    case RTG_ENOMEM: return "does not fit the device-memory budget";
    case RTG_ERANGE: return "out of range (cell coordinate, radius, or key bits)";
    case RTG_EDEVICE: return "device error";
    case RTG_ENOENT: return "unknown ticket or handle";
    default: return "unknown status";
  }
}

}  // extern "C"
