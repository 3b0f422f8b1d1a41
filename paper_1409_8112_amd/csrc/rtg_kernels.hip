// rtg_kernels.hip -- gfx950 kernels of the RTG all-pairs r-NN pipeline.
//
// Steps (Sec. III, Alg. "Randomly Shifted Grids" with random orientations):
//   stage      AoS -> SoA copy of the points, finiteness check, bounding box
//   keys       cell of every (point, grid) in FP64, packed into a 64-bit key
//   sort       stable LSD radix sort of (key, point) -- groups equal cells
//   cells      runs of equal keys with >= 2 points and their 64x64 tile pairs
//   pairs      one wave per tile pair: FP32 screen, FP64 band re-test,
//              ballot-compacted output of pairs within r
//   unique     sort of packed pairs and removal of repeats (Sec. III-B)
//   csr        symmetric neighbour lists (Sec. III-B)
//
// The whole file is compiled with FMA contraction off: the cell coordinate
// y = (R p) / c + u and the FP64 re-test must round every product and sum on
// its own, in the order written, to match the FP64 definition bit for bit.
// Where a fused multiply-add is wanted (the FP32 screen) it is written out.
#pragma clang fp contract(off)

#include "rtg_internal.h"

#include <math.h>

#include <algorithm>
#include <type_traits>
#include <utility>

namespace rtgk {
namespace {

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of m below this lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Orders the LDS traffic of one wave: every lane's earlier LDS writes are
// seen by every lane's later LDS reads, and no access moves across.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// v from another lane by a DPP pattern (row_mask / bank_mask select the
// written rows and banks; lanes whose source falls outside the row, or that
// are not written, get old).  Every lane of the wave must be active.
template <int Ctrl, int RowMask = 0xf, int BankMask = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, Ctrl, RowMask, BankMask, false);
}

// The value of lane l (a constant or wave-uniform l), in every lane.
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ unsigned long long lane_value(unsigned long long v, int l) {
  const uint32_t lo = lane_value((uint32_t)v, l), hi = lane_value((uint32_t)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// DPP controls: row_shr:n = 0x110 + n, row_mirror = 0x140,
// row_half_mirror = 0x141, row_bcast:15 = 0x142, row_bcast:31 = 0x143;
// quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  if constexpr (sizeof(T) == 4) {
    // within each row of 16 lanes (shifts 1, 2, 4, 8), then row 0's total
    // into rows 1 and 3, then rows 0-1's total into rows 2 and 3
    uint32_t x = (uint32_t)v;
    x += dpp_u32<0x111>(0u, x);
    x += dpp_u32<0x112>(0u, x);
    x += dpp_u32<0x114>(0u, x);
    x += dpp_u32<0x118>(0u, x);
    x += dpp_u32<0x142, 0xa>(0u, x);
    x += dpp_u32<0x143, 0xc>(0u, x);
    return (T)x;
  } else {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      T t = __shfl_up(v, o, 64);
      if (lane >= (uint32_t)o) v += t;
    }
    return v;
  }
}

// Exclusive scan of one value per thread over a 256-thread block.  wsum
// must be a __shared__ array of kWaves elements; total receives the sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* wsum, T& total) {
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  T inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) {
    T x = wsum[q];
    if (q < w) before += x;
    all += x;
  }
  __syncthreads();
  total = all;
  return before + inc - v;
}

// Order-preserving encoding of a finite float as uint32.
__device__ __forceinline__ uint32_t float_order(float f) {
  uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// ---------------------------------------------------------------------------
// fill

template <typename T>
__global__ void k_fill(T* p, T v, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// stage: one thread per point.

// Instance that owns point block blk: the largest q with blk_first <= blk.
__device__ __forceinline__ uint32_t block_instance(const InstDesc* __restrict__ inst, uint32_t m,
                                                   uint32_t blk) {
  uint32_t lo = 0, hi = m;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((uint32_t)inst[mid].blk_first <= blk) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Each block writes its own per-axis min/max (order-preserving encodings)
// to part[block][2d]; k_bbox_reduce folds them per instance.  (Atomics on
// the 2d words of one bounding box would all meet at one address per axis.)
__global__ __launch_bounds__(kBlock) void k_stage(const InstDesc* __restrict__ inst, uint32_t m,
                                                  int d, int64_t npts, float* __restrict__ soa,
                                                  float* __restrict__ aos, uint32_t* bad,
                                                  uint32_t* __restrict__ part,
                                                  float* __restrict__ rec, int rs) {
  __shared__ uint32_t smin[kWaves][kMaxDim], smax[kWaves][kMaxDim];
  const uint32_t q = block_instance(inst, m, blockIdx.x);
  const float* pts = inst[q].pts;
  const int64_t i = (int64_t)(blockIdx.x - (uint32_t)inst[q].blk_first) * kBlock + threadIdx.x;
  const bool live = i < inst[q].n;
  const int64_t g = inst[q].pt_off + i;
  const int w = threadIdx.x >> 6;
  bool nonfinite = false;
  for (int l = 0; l < d; ++l) {
    float v = live ? pts[i * d + l] : 0.0f;
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    if (live) {
      soa[(int64_t)l * npts + g] = v;
      if (aos) aos[g * d + l] = v;
      if (rec) rec[g * rs + l] = v;
      if (!isfinite(v)) nonfinite = true;
      else lo = hi = float_order(v);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
      hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
    }
    if (lane_id() == 0) {
      smin[w][l] = lo;
      smax[w][l] = hi;
    }
  }
  if (ballot(nonfinite) && lane_id() == 0) atomicOr(bad, 1u);
  if (rec && live)
    for (int l = d; l < rs; ++l) rec[g * rs + l] = 0.0f;  // padding, then the signature word
  __syncthreads();
  if (threadIdx.x < (unsigned)d) {
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
    for (int q2 = 0; q2 < kWaves; ++q2) {
      lo = min(lo, smin[q2][threadIdx.x]);
      hi = max(hi, smax[q2][threadIdx.x]);
    }
    part[(size_t)blockIdx.x * 2 * d + 2 * threadIdx.x] = lo;
    part[(size_t)blockIdx.x * 2 * d + 2 * threadIdx.x + 1] = hi;
  }
}

// The minimum and maximum of lo / hi over the wave (every lane active), in
// every lane: quads, half rows and rows by DPP, then the four rows' values.
__device__ __forceinline__ void wave_minmax_u32(uint32_t& lo, uint32_t& hi) {
  auto step = [&](auto ctrl) {
    constexpr int C = decltype(ctrl)::value;
    lo = min(lo, dpp_u32<C>(lo, lo));
    hi = max(hi, dpp_u32<C>(hi, hi));
  };
  step(std::integral_constant<int, 0xB1>{});
  step(std::integral_constant<int, 0x4E>{});
  step(std::integral_constant<int, 0x141>{});
  step(std::integral_constant<int, 0x140>{});
  lo = min(min(lane_value(lo, 0), lane_value(lo, 16)), min(lane_value(lo, 32), lane_value(lo, 48)));
  hi = max(max(lane_value(hi, 0), lane_value(hi, 16)), max(lane_value(hi, 32), lane_value(hi, 48)));
}

// k_stage for d = D <= 16: every coordinate of the thread's point loaded at
// once, wave minima and maxima by DPP, and the point record (when asked
// for: the coordinates, then zeros -- padding and the signature word the
// key kernel writes) stored 16 bytes at a time.
template <int D>
__global__ __launch_bounds__(kBlock) void k_stage_d(const InstDesc* __restrict__ inst, uint32_t m,
                                                    int64_t npts, float* __restrict__ soa,
                                                    float* __restrict__ aos, uint32_t* bad,
                                                    uint32_t* __restrict__ part,
                                                    float* __restrict__ rec) {
  constexpr int RS = (D + 2 + 3) & ~3;  // record floats (used for D <= 6)
  __shared__ uint32_t smin[kWaves][D], smax[kWaves][D];
  const uint32_t q = block_instance(inst, m, blockIdx.x);
  const float* pts = inst[q].pts;
  const int64_t i = (int64_t)(blockIdx.x - (uint32_t)inst[q].blk_first) * kBlock + threadIdx.x;
  const bool live = i < inst[q].n;
  const int64_t g = inst[q].pt_off + i;
  const int w = threadIdx.x >> 6;
  float v[D];
#pragma unroll
  for (int l = 0; l < D; ++l) v[l] = live ? pts[i * D + l] : 0.0f;
  bool nonfinite = false;
#pragma unroll
  for (int l = 0; l < D; ++l) {
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    if (live) {
      soa[(int64_t)l * npts + g] = v[l];
      if (aos) aos[g * D + l] = v[l];
      if (!isfinite(v[l])) nonfinite = true;
      else lo = hi = float_order(v[l]);
    }
    wave_minmax_u32(lo, hi);
    if (lane_id() == 0) {
      smin[w][l] = lo;
      smax[w][l] = hi;
    }
  }
  if (ballot(nonfinite) && lane_id() == 0) atomicOr(bad, 1u);
  if constexpr (D <= 6) {
    if (rec && live) {
      float4* r4 = reinterpret_cast<float4*>(rec + g * RS);
#pragma unroll
      for (int c4 = 0; c4 < RS / 4; ++c4) {
        float4 x;
        x.x = 4 * c4 + 0 < D ? v[4 * c4 + 0] : 0.0f;
        x.y = 4 * c4 + 1 < D ? v[4 * c4 + 1] : 0.0f;
        x.z = 4 * c4 + 2 < D ? v[4 * c4 + 2] : 0.0f;
        x.w = 4 * c4 + 3 < D ? v[4 * c4 + 3] : 0.0f;
        r4[c4] = x;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)D) {
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
    for (int q2 = 0; q2 < kWaves; ++q2) {
      lo = min(lo, smin[q2][threadIdx.x]);
      hi = max(hi, smax[q2][threadIdx.x]);
    }
    part[(size_t)blockIdx.x * 2 * D + 2 * threadIdx.x] = lo;
    part[(size_t)blockIdx.x * 2 * D + 2 * threadIdx.x + 1] = hi;
  }
}

// Before the stage: bbox of every instance to the identities of min and
// max (bits of the order-preserving encoding), *bad to 0, and the caller's
// zero64[0, nzero) to 0 (counters of the pass), in one launch.
__global__ void k_stage_init(uint32_t* __restrict__ bbox, uint32_t count, uint32_t* bad,
                             uint64_t* __restrict__ zero64, uint32_t nzero) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) bbox[e] = (e & 1u) ? 0u : 0xFFFFFFFFu;
  if (e < nzero) zero64[e] = 0ull;
  if (e == 0) *bad = 0u;
}

// Block (q, y) folds slice y of instance q's per-block boxes into bbox with
// atomic min / max (one per axis and block): one instance spreads over up
// to kBboxBlocks blocks.
constexpr uint32_t kBboxBlocks = 64;
__global__ __launch_bounds__(kBlock) void k_bbox_reduce(const InstDesc* __restrict__ inst, int d,
                                                        const uint32_t* __restrict__ part,
                                                        uint32_t* __restrict__ bbox) {
  const uint32_t q = blockIdx.x;
  const uint32_t b0 = inst[q].blk_first;
  const uint32_t nb = (uint32_t)((inst[q].n + kBlock - 1) / kBlock);
  const uint32_t per = (nb + gridDim.y - 1) / gridDim.y;
  const uint32_t lo_b = blockIdx.y * per, hi_b = min(nb, lo_b + per);
  if (lo_b >= hi_b) return;
  const int w = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  for (int l = w; l < d; l += kWaves) {
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (uint32_t b = lo_b + lane; b < hi_b; b += 64) {
      lo = min(lo, part[(size_t)(b0 + b) * 2 * d + 2 * l]);
      hi = max(hi, part[(size_t)(b0 + b) * 2 * d + 2 * l + 1]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
      hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
    }
    if (lane == 0) {
      atomicMin(&bbox[(size_t)q * 2 * d + 2 * l], lo);
      atomicMax(&bbox[(size_t)q * 2 * d + 2 * l + 1], hi);
    }
  }
}

// ---------------------------------------------------------------------------
// keys: y_j = ((R_j0 p_0 + R_j1 p_1) + ...) * inv_c + u_j, each operation
// rounded on its own (contraction is off), kappa_j = floor(y_j).

template <int D>
__device__ __forceinline__ double cell_y(const double* __restrict__ Rj, const float* p_reg,
                                         const float* __restrict__ soa, int64_t n, int64_t i,
                                         int d, double inv_c, double uj) {
  double z;
  if (D > 0) {
    z = Rj[0] * (double)p_reg[0];
#pragma unroll
    for (int l = 1; l < D; ++l) z = z + Rj[l] * (double)p_reg[l];
  } else {
    z = Rj[0] * (double)soa[i];
    for (int l = 1; l < d; ++l) z = z + Rj[l] * (double)soa[(int64_t)l * n + i];
  }
  return z * inv_c + uj;
}

// One thread per batch point; writes the keys of the point's segments in
// [sa, sb): key = (segment - sa) << cell_bits | packed cell, at
// segs[segment].key_off + the point's index in its instance.
template <int D>
__global__ __launch_bounds__(kBlock) void k_keys(const InstDesc* __restrict__ inst, uint32_t m,
                                                 int d_rt, int64_t npts,
                                                 const float* __restrict__ soa, int sa, int sb,
                                                 const SegDesc* __restrict__ segs,
                                                 const double* __restrict__ R,
                                                 const double* __restrict__ u,
                                                 const int64_t* __restrict__ klo,
                                                 const KeyLayout* __restrict__ layout,
                                                 uint64_t* __restrict__ keys,
                                                 uint32_t* __restrict__ vals, uint32_t* err,
                                                 uint64_t* __restrict__ sig, int sig_stride,
                                                 int sig_b, int sig_gpw, int idx_bits,
                                                 int sig_fresh) {
  const int d = D > 0 ? D : d_rt;
  const uint32_t q = block_instance(inst, m, blockIdx.x);
  const int64_t i = (int64_t)(blockIdx.x - (uint32_t)inst[q].blk_first) * kBlock + threadIdx.x;
  if (i >= inst[q].n) return;
  const int64_t g = inst[q].pt_off + i;
  const int seg_first = inst[q].seg_first;
  const int t_lo = max(0, sa - seg_first), t_hi = min(inst[q].k, sb - seg_first);
  const double inv_c = inst[q].inv_c;
  float p[D > 0 ? D : 1];
  if (D > 0) {
#pragma unroll
    for (int l = 0; l < (D > 0 ? D : 1); ++l) p[l] = soa[(int64_t)l * npts + g];
  }
  const int cell_bits = layout->cell_bits;
  const uint64_t bmask = (1ull << sig_b) - 1ull;
  const int gbits = d * sig_b;
  uint64_t sword = 0;  // signature word being filled
  int sw = -1;         // its index
  bool bad = false;
  for (int t = t_lo; t < t_hi; ++t) {
    const int s = seg_first + t;
    const int tr = inst[q].tr_off + t;
    const double* Rt = R + (size_t)tr * d * d;
    const double* ut = u + (size_t)tr * d;
    const int64_t* kl = klo + (size_t)tr * d;
    uint64_t cell = 0, grp = 0;
    for (int j = 0; j < d; ++j) {
      double y = cell_y<D>(Rt + (size_t)j * d, p, soa, npts, g, d, inv_c, ut[j]);
      bool ok = fabs(y) < 2147483648.0;
      bad |= !ok;
      // |y| < 2^31: the floor fits 32 bits, and one native conversion takes it
      int64_t kap = ok ? (int64_t)(int32_t)floor(y) : 0;
      uint64_t mask = (1ull << layout->bits[j]) - 1ull;
      cell |= ((uint64_t)(kap - kl[j]) & mask) << layout->shift[j];
      grp |= ((uint64_t)(kap - kl[j]) & bmask) << (j * sig_b);
    }
    if (sig) {
      // the point owns its row: earlier passes' bits are read back and kept
      const int w = t / sig_gpw;
      if (w != sw) {
        if (sw >= 0) {
          uint64_t* dst = sig + (size_t)g * sig_stride + sw;
          *dst = sig_fresh ? sword : (*dst | sword);
        }
        sword = 0;
        sw = w;
      }
      sword |= grp << ((t - w * sig_gpw) * gbits);
    }
    const uint64_t key = (cell_bits < 64) ? (((uint64_t)(s - sa) << cell_bits) | cell) : cell;
    const int64_t pos = segs[s].key_off + i;
    if (idx_bits) {
      keys[pos] = (key << idx_bits) | (uint64_t)g;
    } else {
      keys[pos] = key;
      vals[pos] = (uint32_t)g;
    }
  }
  if (sig && sw >= 0) {
    uint64_t* dst = sig + (size_t)g * sig_stride + sw;
    *dst = sig_fresh ? sword : (*dst | sword);
  }
  if (bad) atomicOr(err, 1u);
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_cell_coords(const float* __restrict__ soa, int64_t n,
                                                        int d_rt, const double* __restrict__ R,
                                                        const double* __restrict__ u, double inv_c,
                                                        int64_t* __restrict__ kappa,
                                                        uint32_t* err) {
  const int d = D > 0 ? D : d_rt;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float p[D > 0 ? D : 1];
  if (D > 0) {
#pragma unroll
    for (int l = 0; l < (D > 0 ? D : 1); ++l) p[l] = soa[(int64_t)l * n + i];
  }
  bool bad = false;
  for (int j = 0; j < d; ++j) {
    double y = cell_y<D>(R + (size_t)j * d, p, soa, n, i, d, inv_c, u[j]);
    bool ok = fabs(y) < 2147483648.0;
    bad |= !ok;
    kappa[i * d + j] = ok ? (int64_t)(int32_t)floor(y) : 0;
  }
  if (bad) atomicOr(err, 1u);
}

// ---------------------------------------------------------------------------
// scan: 256 threads x 8 consecutive elements per block.

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;
// Up to this many tile sums, every apply block adds up its predecessors' sums
// itself (at most 8 KB read per block).
constexpr int kFusedScanSums = 2048;

// With dcount the element count is min(count, *dcount): count is then the
// grid's capacity and the elements beyond the device count read as zero.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const T* __restrict__ in, size_t count,
                                                        T* __restrict__ sums,
                                                        const uint32_t* __restrict__ dcount) {
  __shared__ T wsum[kWaves];
  if (dcount) count = min(count, (size_t)*dcount);
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  T s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q)
    if (base + q < count) s += in[base + q];
  T total;
  block_exclusive_scan<T>(s, wsum, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Scans each block's tile and adds its offset: offsets[block] (already
// scanned), or with FROM_SUMS the sum of the earlier blocks' tile sums, added
// up by the block itself (no separate scan of the sums; for few blocks).
template <typename T, bool FROM_SUMS = false>
__global__ __launch_bounds__(kBlock) void k_scan_apply(const T* in, T* out, size_t count,
                                                       const T* __restrict__ offsets, T* total,
                                                       const uint32_t* __restrict__ dcount) {
  __shared__ T wsum[kWaves];
  if (dcount) count = min(count, (size_t)*dcount);
  T from_sums = 0;
  if (FROM_SUMS) {
    T part = 0;
    for (uint32_t p = threadIdx.x; p < blockIdx.x; p += kBlock) part += offsets[p];
    block_exclusive_scan<T>(part, wsum, from_sums);
  }
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = (base + q < count) ? in[base + q] : (T)0;
    s += v[q];
  }
  T tile_total;
  T run = block_exclusive_scan<T>(s, wsum, tile_total);
  const T off = FROM_SUMS ? from_sums : (offsets ? offsets[blockIdx.x] : (T)0);
  run += off;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    if (base + q < count) out[base + q] = run;
    run += v[q];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tile_total;
}

// ---------------------------------------------------------------------------
// radix sort: tiles of 4096 elements; element e of a tile is held by wave
// e / 1024, round (e % 1024) / 64, lane e % 64, so every load is one
// contiguous 64-element run.  Two drivers share the tile code:
//   reduce-then-scan (the default): per pass, tile histograms, a
//     device-wide scan, then the scatter (one more read of the keys per
//     pass); it can sort within segments, leaving their bits out of the
//     passes;
//   onesweep: one histogram read for all digit passes, then per pass one
//     kernel in which each tile takes the next tile id, publishes its digit
//     counts and looks back over earlier tiles' published counts (decoupled
//     look-back) to find where its digits start; its look-back reads cross
//     the XCDs' L2s, and it measured slower.

// LDS of one tile: staged keys/values and the per-wave digit counters.
// (Values are staged in key[] too, after the keys have gone out: the tile
// needs no separate value area, so a sort with values keeps the occupancy of
// one without.)
template <bool HAS_VAL>
struct TileLds {
  uint64_t key[kTile];
  uint32_t wcnt[kWaves][256];
  uint32_t dstart[256];
  uint64_t goff[256];
  uint32_t wsum[kWaves];
};

// Loads tile `tile` and ranks every element among the elements of its wave
// with the same digit (stable: wave order, then round, then lane).  After
// the call wcnt[w][dg] holds wave w's count of digit dg.
template <bool HAS_VAL>
__device__ __forceinline__ void tile_rank(TileLds<HAS_VAL>& S, const uint64_t* __restrict__ kin,
                                          const uint32_t* __restrict__ vin, size_t tile_base,
                                          size_t tile_end, int shift, int nbits, uint64_t* k_,
                                          uint32_t* v_, uint32_t* r_) {
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  const uint32_t mask = (1u << nbits) - 1u;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) S.wcnt[q][threadIdx.x] = 0u;
  __syncthreads();
  const size_t wave_base = tile_base + (size_t)w * (kTile / kWaves);
  const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int q = 0; q < kKeysPerThread; ++q) {
    const size_t e = wave_base + (size_t)q * 64 + lane;
    const bool valid = e < tile_end;
    const uint64_t key = valid ? kin[e] : ~0ull;
    k_[q] = key;
    if (HAS_VAL) v_[q] = valid ? vin[e] : 0u;
    const uint32_t dg = (uint32_t)(key >> shift) & mask;
    uint64_t peers = ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (dg >> b) & 1u;
      const uint64_t m = ballot(bit);
      peers &= bit ? m : ~m;
    }
    uint32_t before = 0;
    if (valid) before = S.wcnt[w][dg];
    r_[q] = before + (uint32_t)__popcll(peers & lt);
    wave_lds_sync();
    if (valid && (peers & lt) == 0ull) S.wcnt[w][dg] = before + (uint32_t)__popcll(peers);
    wave_lds_sync();
  }
  __syncthreads();
}

// Thread dg: the tile's count of digit dg; sets dstart[dg] (its first
// position in the tile) and turns wcnt[w][dg] into wave w's first position.
template <bool HAS_VAL>
__device__ __forceinline__ uint32_t tile_layout(TileLds<HAS_VAL>& S) {
  const uint32_t dg = threadIdx.x;
  uint32_t c[kWaves];
  uint32_t tot = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) {
    c[q] = S.wcnt[q][dg];
    tot += c[q];
  }
  uint32_t all;
  const uint32_t start = block_exclusive_scan<uint32_t>(tot, S.wsum, all);
  S.dstart[dg] = start;
  uint32_t run = start;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) {
    S.wcnt[q][dg] = run;
    run += c[q];
  }
  return tot;
}

// Sorts the tile into LDS and writes it out at goff[dg] + rank in digit.
template <bool HAS_VAL>
__device__ __forceinline__ void tile_scatter(TileLds<HAS_VAL>& S, uint64_t* __restrict__ kout,
                                             uint32_t* __restrict__ vout, size_t count,
                                             size_t tile_base, size_t tile_end, int shift,
                                             int nbits, const uint64_t* k_, const uint32_t* v_,
                                             const uint32_t* r_) {
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  const uint32_t mask = (1u << nbits) - 1u;
  const size_t wave_base = tile_base + (size_t)w * (kTile / kWaves);
  uint32_t pos_[HAS_VAL ? kKeysPerThread : 1];
#pragma unroll
  for (int q = 0; q < kKeysPerThread; ++q) {
    const size_t e = wave_base + (size_t)q * 64 + lane;
    if (e < tile_end) {
      const uint32_t dg = (uint32_t)(k_[q] >> shift) & mask;
      const uint32_t pos = S.wcnt[w][dg] + r_[q];
      S.key[pos] = k_[q];
      if (HAS_VAL) pos_[q] = pos;
    }
  }
  __syncthreads();
  const size_t rem = tile_end - tile_base;
  const uint32_t tile_count = rem < (size_t)kTile ? (uint32_t)rem : (uint32_t)kTile;
  // the digit of each slot this thread writes out, a byte each, for the values
  uint32_t dg4[HAS_VAL ? kKeysPerThread / 4 : 1] = {};
#pragma unroll 4
  for (int q = 0; q < kKeysPerThread; ++q) {
    const uint32_t s = (uint32_t)q * kBlock + threadIdx.x;
    if (s < tile_count) {
      const uint64_t key = S.key[s];
      const uint32_t dg = (uint32_t)(key >> shift) & mask;
      const uint64_t g = S.goff[dg] + (s - S.dstart[dg]);
      if (g < count) kout[g] = key;  // always in range when the offsets are right
      if (HAS_VAL) dg4[q / 4] |= dg << (8 * (q % 4));
    }
  }
  if (HAS_VAL) {
    // the values through the same slots, once every key has been read out
    __syncthreads();
    uint32_t* sval = reinterpret_cast<uint32_t*>(S.key);
#pragma unroll
    for (int q = 0; q < kKeysPerThread; ++q) {
      const size_t e = wave_base + (size_t)q * 64 + lane;
      if (e < tile_end) sval[pos_[q]] = v_[q];
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < kKeysPerThread; ++q) {
      const uint32_t s = (uint32_t)q * kBlock + threadIdx.x;
      if (s < tile_count) {
        const uint32_t dg = (dg4[q / 4] >> (8 * (q % 4))) & 0xFFu;
        const uint64_t g = S.goff[dg] + (s - S.dstart[dg]);
        if (g < count) vout[g] = sval[s];
      }
    }
  }
}

// --- reduce-then-scan ---------------------------------------------------------

// Tile b of a sort: its keys [start, start + len) and the place of its
// digit counts in the histogram table, slot + digit * stride.  Without a
// table, tile b is keys [b kTile, ...) with slot b and stride ntiles; with
// one, tiles stay inside segments and the table is segment-major, so its
// exclusive scan orders by segment, then digit, then tile.
struct TileSpan {
  size_t start, end;
  size_t slot, stride;
};
__device__ __forceinline__ TileSpan tile_span(const SortTile* tiles, size_t count,
                                              uint32_t ntiles, uint32_t b) {
  TileSpan t;
  if (tiles) {
    const SortTile d = tiles[b];
    t.start = d.start;
    t.end = d.start + d.len;
    t.slot = d.slot;
    t.stride = d.stride;
  } else {
    t.start = (size_t)b * kTile;
    t.end = min(count, t.start + (size_t)kTile);
    t.slot = b;
    t.stride = ntiles;
  }
  return t;
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                       size_t count, int shift, int nbits,
                                                       uint32_t* __restrict__ tile_hist,
                                                       uint32_t ntiles,
                                                       const SortTile* __restrict__ tiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t mask = (1u << nbits) - 1u;
  const TileSpan t = tile_span(tiles, count, ntiles, blockIdx.x);
#pragma unroll 4
  for (int q = 0; q < kKeysPerThread; ++q) {
    size_t e = t.start + (size_t)q * kBlock + threadIdx.x;
    if (e < t.end) atomicAdd(&h[(uint32_t)(keys[e] >> shift) & mask], 1u);
  }
  __syncthreads();
  tile_hist[t.slot + (size_t)threadIdx.x * t.stride] = h[threadIdx.x];
}

template <bool HAS_VAL>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, size_t count, int shift, int nbits,
    const uint32_t* __restrict__ tile_off, uint32_t ntiles, const SortTile* __restrict__ tiles) {
  __shared__ TileLds<HAS_VAL> S;
  uint64_t k_[kKeysPerThread];
  uint32_t v_[kKeysPerThread];
  uint32_t r_[kKeysPerThread];
  const TileSpan t = tile_span(tiles, count, ntiles, blockIdx.x);
  tile_rank<HAS_VAL>(S, kin, vin, t.start, t.end, shift, nbits, k_, v_, r_);
  tile_layout<HAS_VAL>(S);
  S.goff[threadIdx.x] = tile_off[t.slot + (size_t)threadIdx.x * t.stride];
  __syncthreads();
  tile_scatter<HAS_VAL>(S, kout, vout, count, t.start, t.end, shift, nbits, k_, v_, r_);
}

// --- onesweep -------------------------------------------------------------------

constexpr int kHistBlockTiles = 4;  // tiles per block of the all-pass histogram
constexpr int kMaxPasses = 8;

// part[block][p][dg]: this block's count of digit dg in pass p.
__global__ __launch_bounds__(kBlock) void k_hist_all(const uint64_t* __restrict__ keys,
                                                     size_t count, int begin_bit, int end_bit,
                                                     uint32_t* __restrict__ part) {
  __shared__ uint32_t h[kWaves][kMaxPasses][256];
  const int w = threadIdx.x >> 6;
  const int npass = (end_bit - begin_bit + kRadixBits - 1) / kRadixBits;
  for (int p = 0; p < npass; ++p)
#pragma unroll
    for (int q = 0; q < kWaves; ++q) h[q][p][threadIdx.x] = 0u;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * kHistBlockTiles * kTile;
  for (int q = 0; q < kHistBlockTiles * kKeysPerThread; ++q) {
    const size_t e = base + (size_t)q * kBlock + threadIdx.x;
    if (e >= count) break;
    const uint64_t key = keys[e];
    for (int p = 0; p < npass; ++p) {
      const int b = begin_bit + p * kRadixBits;
      const int nb = min(kRadixBits, end_bit - b);
      atomicAdd(&h[w][p][(uint32_t)(key >> b) & ((1u << nb) - 1u)], 1u);
    }
  }
  __syncthreads();
  for (int p = 0; p < npass; ++p) {
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) s += h[q][p][threadIdx.x];
    part[((size_t)blockIdx.x * npass + p) * 256 + threadIdx.x] = s;
  }
}

// One block per pass: digit_off[p][dg] = number of keys with a smaller digit.
__global__ __launch_bounds__(kBlock) void k_hist_scan(const uint32_t* __restrict__ part,
                                                      uint32_t nblocks, int npass,
                                                      uint64_t* __restrict__ digit_off) {
  __shared__ uint64_t wsum[kWaves];
  const int p = blockIdx.x;
  uint64_t s = 0;
  for (uint32_t b = 0; b < nblocks; ++b) s += part[((size_t)b * npass + p) * 256 + threadIdx.x];
  uint64_t all;
  digit_off[p * 256 + threadIdx.x] = block_exclusive_scan<uint64_t>(s, wsum, all);
}

// Status word of (tile, digit): flag in the top two bits (0 not yet
// published, 1 this tile's count, 2 count of this and all earlier tiles).
constexpr uint64_t kStAggregate = 1ull << 62;
constexpr uint64_t kStInclusive = 2ull << 62;
constexpr uint64_t kStValue = (1ull << 62) - 1ull;
constexpr uint32_t kSpinLimit = 1u << 22;

template <bool HAS_VAL>
__global__ __launch_bounds__(kBlock) void k_onesweep(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, size_t count, int shift, int nbits,
    const uint64_t* __restrict__ digit_off, unsigned long long* status, unsigned int* tile_counter,
    unsigned int* err) {
  __shared__ TileLds<HAS_VAL> S;
  __shared__ uint32_t s_tile;
  // Tile ids in the order blocks start: every earlier tile is already
  // running, so each look-back wait ends.
  if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const size_t tile = s_tile;
  uint64_t k_[kKeysPerThread];
  uint32_t v_[kKeysPerThread];
  uint32_t r_[kKeysPerThread];
  const size_t tile_base = tile * kTile;
  const size_t tile_end = min(count, tile_base + (size_t)kTile);
  tile_rank<HAS_VAL>(S, kin, vin, tile_base, tile_end, shift, nbits, k_, v_, r_);
  const uint32_t tot = tile_layout<HAS_VAL>(S);
  const uint32_t dg = threadIdx.x;
  if (dg < (1u << nbits)) {
    unsigned long long* mine = status + tile * 256 + dg;
    __hip_atomic_store(mine, kStAggregate | (uint64_t)tot, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    for (size_t p = tile; p-- > 0;) {
      uint64_t st;
      uint32_t spins = 0;
      do {
        st = __hip_atomic_load(status + p * 256 + dg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } while ((st >> 62) == 0 && ++spins < kSpinLimit);
      if ((st >> 62) == 0) {  // never published: give up, report, keep writes in bounds
        atomicOr(err, 2u);
        break;
      }
      excl += st & kStValue;
      if ((st >> 62) == 2) break;
    }
    __hip_atomic_store(mine, kStInclusive | (excl + tot), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    S.goff[dg] = digit_off[dg] + excl;
  }
  __syncthreads();
  tile_scatter<HAS_VAL>(S, kout, vout, count, tile_base, tile_end, shift, nbits, k_, v_, r_);
}

// ---------------------------------------------------------------------------
// runs of equal keys (cells with >= 2 points), unique keys.

// Whether element e begins or ends a run of at least two equal keys.  The
// wave's lanes hold 64 consecutive elements (e = 64-aligned base + lane):
// each loads its own key, takes its neighbours' from the adjacent lanes, and
// only the first and last lanes load the keys beyond the wave's ends.
__device__ __forceinline__ void run_flags(const uint64_t* __restrict__ keys, size_t count, size_t e,
                                          uint32_t lane, int shift, bool& head, bool& tail) {
  const bool in = e < count;
  const uint64_t k = in ? keys[e] >> shift : 0ull;
  uint64_t kp = __shfl_up(k, 1, 64);
  uint64_t kn = __shfl_down(k, 1, 64);
  if (lane == 0 && in && e > 0) kp = keys[e - 1] >> shift;
  if (lane == 63 && e + 1 < count) kn = keys[e + 1] >> shift;
  const bool prev_same = in && e > 0 && kp == k;
  const bool next_same = in && e + 1 < count && kn == k;
  head = !prev_same && next_same;
  tail = prev_same && !next_same;
}

__global__ __launch_bounds__(kBlock) void k_run_count(const uint64_t* __restrict__ keys,
                                                      size_t count, int shift, uint32_t* head_cnt,
                                                      uint32_t* tail_cnt,
                                                      uint64_t* __restrict__ masks) {
  __shared__ uint32_t sh[kWaves], st[kWaves];
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  const size_t wave_base = (size_t)blockIdx.x * kTile + (size_t)w * (kTile / kWaves);
  const size_t ngroups = (count + 63) / 64;
  uint32_t hc = 0, tc = 0;
  for (int q = 0; q < kKeysPerThread; ++q) {
    bool h, t;
    run_flags(keys, count, wave_base + (size_t)q * 64 + lane, lane, shift, h, t);
    const uint64_t hb = ballot(h), tb = ballot(t);
    hc += (uint32_t)__popcll(hb);
    tc += (uint32_t)__popcll(tb);
    // the writing kernel reads these bits instead of the keys again
    const size_t g = (wave_base >> 6) + (size_t)q;
    if (g < ngroups && lane < 2) masks[2 * g + lane] = lane ? tb : hb;
  }
  if (lane == 0) {
    sh[w] = hc;
    st[w] = tc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0, b = 0;
    for (int q = 0; q < kWaves; ++q) {
      a += sh[q];
      b += st[q];
    }
    head_cnt[blockIdx.x] = a;
    tail_cnt[blockIdx.x] = b;
  }
}

// head_off / tail_off: each tile's scanned offsets, or with FROM_COUNTS the
// raw per-tile counts, which each block then adds up for the tiles before it
// itself (the last block writes the totals to tot; block 0 clears *zero).
template <bool FROM_COUNTS>
__global__ __launch_bounds__(kBlock) void k_run_write(const uint64_t* __restrict__ masks,
                                                      size_t count,
                                                      const uint32_t* __restrict__ head_off,
                                                      const uint32_t* __restrict__ tail_off,
                                                      uint32_t* __restrict__ start,
                                                      uint32_t* __restrict__ end,
                                                      uint32_t* __restrict__ tot,
                                                      unsigned long long* __restrict__ zero) {
  __shared__ uint32_t sh[kWaves], st[kWaves];
  __shared__ uint32_t wsum[kWaves];
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  const size_t wave_base = (size_t)blockIdx.x * kTile + (size_t)w * (kTile / kWaves);
  const size_t ngroups = (count + 63) / 64;
  uint32_t hmask = 0, tmask = 0, hc = 0, tc = 0;
  for (int q = 0; q < kKeysPerThread; ++q) {
    const size_t g = (wave_base >> 6) + (size_t)q;
    uint64_t hb = 0, tb = 0;
    if (g < ngroups) {
      hb = masks[2 * g];
      tb = masks[2 * g + 1];
    }
    hmask |= (uint32_t)((hb >> lane) & 1ull) << q;
    tmask |= (uint32_t)((tb >> lane) & 1ull) << q;
    hc += (uint32_t)__popcll(hb);
    tc += (uint32_t)__popcll(tb);
  }
  if (lane == 0) {
    sh[w] = hc;
    st[w] = tc;
  }
  __syncthreads();
  uint32_t hbase, tbase;
  if (FROM_COUNTS) {
    uint32_t ph = 0, pt = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kBlock) {
      ph += head_off[b];
      pt += tail_off[b];
    }
    block_exclusive_scan<uint32_t>(ph, wsum, hbase);
    block_exclusive_scan<uint32_t>(pt, wsum, tbase);
    if (threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) {
      uint32_t a = 0, b = 0;
      for (int q = 0; q < kWaves; ++q) {
        a += sh[q];
        b += st[q];
      }
      tot[0] = hbase + a;
      tot[1] = tbase + b;
    }
    if (zero && threadIdx.x == 0 && blockIdx.x == 0) *zero = 0ull;
  } else {
    hbase = head_off[blockIdx.x];
    tbase = tail_off[blockIdx.x];
  }
  for (int q = 0; q < w; ++q) {
    hbase += sh[q];
    tbase += st[q];
  }
  for (int q = 0; q < kKeysPerThread; ++q) {
    const size_t e = wave_base + (size_t)q * 64 + lane;
    const bool h = (hmask >> q) & 1u, t = (tmask >> q) & 1u;
    const uint64_t hb = ballot(h), tbm = ballot(t);
    if (h) start[hbase + rank_below(hb)] = (uint32_t)e;
    if (t) end[tbase + rank_below(tbm)] = (uint32_t)(e + 1);
    hbase += (uint32_t)__popcll(hb);
    tbase += (uint32_t)__popcll(tbm);
  }
}

__global__ __launch_bounds__(kBlock) void k_cell_work(const uint32_t* __restrict__ start,
                                                      const uint32_t* __restrict__ end,
                                                      uint32_t ncells,
                                                      const uint32_t* __restrict__ dcells,
                                                      uint32_t cell_unit_tiles,
                                                      uint32_t* __restrict__ units,
                                                      uint64_t* __restrict__ tests,
                                                      unsigned long long* members) {
  // cells [0, ncells), or [0, min(ncells, *dcells)) with the device count
  if (dcells) ncells = min(ncells, *dcells);
  uint64_t L = 0;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncells;
       c += gridDim.x * blockDim.x) {
    const uint64_t Lc = end[c] - start[c];
    const uint32_t nt = (uint32_t)((Lc + kPairTile - 1) / kPairTile);
    units[c] = nt <= cell_unit_tiles ? 1u : nt;
    tests[c] = Lc * (Lc - 1) / 2;
    L += Lc;
  }
  // one atomic per block: a single counter's device-scope atomics serialise
  // across the XCDs
  __shared__ unsigned long long wm[kWaves];
  unsigned long long m = L;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m += __shfl_xor(m, o, 64);
  if (lane_id() == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long all = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) all += wm[q];
    if (all) atomicAdd(members, all);
  }
}

// k_cell_work by scan tiles: block b takes cells [b kScanTile, (b + 1)
// kScanTile), kScanItems consecutive cells per thread as the scan kernels
// hold them, and also writes the tile's sums of units and tests, so that
// the two scans need only their apply launches (each block adds up the
// sums before its own tile).
__global__ __launch_bounds__(kBlock) void k_cell_work_tiles(
    const uint32_t* __restrict__ start, const uint32_t* __restrict__ end, uint32_t ncells,
    const uint32_t* __restrict__ dcells, uint32_t cell_unit_tiles, uint32_t* __restrict__ units,
    uint64_t* __restrict__ tests, unsigned long long* members, uint32_t* __restrict__ usums,
    uint64_t* __restrict__ tsums) {
  if (dcells) ncells = min(ncells, *dcells);
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  uint64_t L = 0, tt = 0;
  uint32_t uu = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const size_t c = base + q;
    if (c < ncells) {
      const uint64_t Lc = end[c] - start[c];
      const uint32_t nt = (uint32_t)((Lc + kPairTile - 1) / kPairTile);
      const uint32_t u = nt <= cell_unit_tiles ? 1u : nt;
      const uint64_t t = Lc * (Lc - 1) / 2;
      units[c] = u;
      tests[c] = t;
      uu += u;
      tt += t;
      L += Lc;
    }
  }
  __shared__ unsigned long long wl[kWaves], wt[kWaves];
  __shared__ uint32_t wu[kWaves];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    L += __shfl_xor(L, o, 64);
    tt += __shfl_xor(tt, o, 64);
    uu += __shfl_xor(uu, o, 64);
  }
  if (lane_id() == 0) {
    wl[threadIdx.x >> 6] = L;
    wt[threadIdx.x >> 6] = tt;
    wu[threadIdx.x >> 6] = uu;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long all = 0, tall = 0;
    uint32_t uall = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
      all += wl[q];
      tall += wt[q];
      uall += wu[q];
    }
    usums[blockIdx.x] = uall;
    tsums[blockIdx.x] = tall;
    if (all) atomicAdd(members, all);
  }
}

__global__ __launch_bounds__(kBlock) void k_unique_count(const uint64_t* __restrict__ keys,
                                                         size_t count, uint32_t* tile_cnt) {
  __shared__ uint32_t sh[kWaves];
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  const size_t wave_base = (size_t)blockIdx.x * kTile + (size_t)w * (kTile / kWaves);
  uint32_t c = 0;
  for (int q = 0; q < kKeysPerThread; ++q) {
    const size_t e = wave_base + (size_t)q * 64 + lane;
    const bool f = e < count && (e == 0 || keys[e] != keys[e - 1]);
    c += (uint32_t)__popcll(ballot(f));
  }
  if (lane == 0) sh[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0;
    for (int q = 0; q < kWaves; ++q) a += sh[q];
    tile_cnt[blockIdx.x] = a;
  }
}

__global__ __launch_bounds__(kBlock) void k_unique_write(const uint64_t* __restrict__ keys,
                                                         size_t count,
                                                         const uint32_t* __restrict__ tile_off,
                                                         uint64_t* __restrict__ out) {
  __shared__ uint32_t sh[kWaves];
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  const size_t wave_base = (size_t)blockIdx.x * kTile + (size_t)w * (kTile / kWaves);
  uint32_t fmask = 0, c = 0;
  for (int q = 0; q < kKeysPerThread; ++q) {
    const size_t e = wave_base + (size_t)q * 64 + lane;
    const bool f = e < count && (e == 0 || keys[e] != keys[e - 1]);
    fmask |= (uint32_t)f << q;
    c += (uint32_t)__popcll(ballot(f));
  }
  if (lane == 0) sh[w] = c;
  __syncthreads();
  uint32_t base = tile_off[blockIdx.x];
  for (int q = 0; q < w; ++q) base += sh[q];
  for (int q = 0; q < kKeysPerThread; ++q) {
    const size_t e = wave_base + (size_t)q * 64 + lane;
    const bool f = (fmask >> q) & 1u;
    const uint64_t m = ballot(f);
    if (f) out[base + rank_below(m)] = keys[e];
    base += (uint32_t)__popcll(m);
  }
}

// ---------------------------------------------------------------------------
// cell pairs.  A work unit is (cell, tile a) with tiles of 64 points; its wave
// tests tile a against the tiles b >= a of the same cell.  Unit points are
// read by sorted position from spts / ssig (gathered once), so every tile
// load is a direct, coalesced read; the next B tile is loaded while the
// current one is tested.  Accepted pairs go through the first-owner filter
// (a pair is kept only if no earlier grid put both points in one cell: the
// signature words of the two points are compared) and are written as
// (min << pair_bits) | max.

constexpr int kSigWords = 2;  // signature words kept per point (more: read on demand)
constexpr int kOutBuf = 256;  // staged pairs per wave

// Whether x = a ^ b (signature words of two points within r) has an all-zero
// group among the first n groups: with L the lowest and H the highest bit of
// every group, (x - L) & ~x & H is nonzero exactly when some group of x is
// zero; a borrow only runs upward, out of a zero group, so masking to the
// first n groups keeps the test exact.
__device__ __forceinline__ bool zero_group(uint64_t x, int n, const PairsArgs& P) {
  const uint64_t keep = (n * P.g >= 64) ? ~0ull : ((1ull << (n * P.g)) - 1ull);
  return (((x - P.lows) & ~x & P.highs) & keep) != 0ull;
}

// Signature word q of the point at sorted position p with index i.
__device__ __forceinline__ uint64_t sig_word(const PairsArgs& P, int q, uint32_t p, uint32_t i) {
  return P.direct ? P.sigp[(size_t)i * P.sig_stride + q] : P.ssig[(size_t)q * P.N + p];
}

// Whether two points within r shared a cell under a grid t < tcell; word q of
// their signatures is aq / bq for q < kSigWords, and is read on demand (the
// points at sorted positions pa, pb with indices ia, ib) beyond that.
__device__ __forceinline__ bool shared_earlier_cell(const uint64_t* aq, const uint64_t* bq,
                                                    int tcell, uint32_t pa, uint32_t ia,
                                                    uint32_t pb, uint32_t ib,
                                                    const PairsArgs& P) {
  const int nw = (tcell - 1) / P.gpw + 1;
  bool same = false;
#pragma unroll
  for (int q = 0; q < kSigWords; ++q)
    if (q < nw) same |= zero_group(aq[q] ^ bq[q], min(P.gpw, tcell - q * P.gpw), P);
  for (int q = kSigWords; q < nw && !same; ++q)
    same = zero_group(sig_word(P, q, pa, ia) ^ sig_word(P, q, pb, ib),
                      min(P.gpw, tcell - q * P.gpw), P);
  return same;
}

// Point index at sorted position p: the low idx_bits of the sorted key when
// keys carry it, else the separate index array.
__device__ __forceinline__ uint32_t point_at(const PairsArgs& P, uint32_t p) {
  return P.idx_bits ? (uint32_t)(P.skeys[p] & ((1ull << P.idx_bits) - 1ull)) : P.sidx[p];
}

template <typename T>
__device__ __forceinline__ T uniform(T v) {
  return (T)__builtin_amdgcn_readfirstlane((int)v);
}

// One tile's data for this lane (lane < n): coordinates, point index and the
// first signature words.
template <int D>
struct TileRegs {
  float c[D];
  uint32_t idx;
  uint64_t sw[kSigWords];
};

template <int D>
__device__ __forceinline__ void load_tile(const PairsArgs& P, uint32_t p0, uint32_t n, int nw,
                                          uint32_t lane, TileRegs<D>& R) {
  const bool ok = lane < n;
  const uint32_t p = p0 + lane;
  R.idx = ok ? point_at(P, p) : 0u;
  if (P.direct) {
    const float* row = P.rows + (size_t)R.idx * P.row_stride;
#pragma unroll
    for (int l = 0; l < D; ++l) R.c[l] = (ok && l < P.d) ? row[l] : 0.0f;
#pragma unroll
    for (int q = 0; q < kSigWords; ++q)
      R.sw[q] = (ok && q < nw) ? P.sigp[(size_t)R.idx * P.sig_stride + q] : 0ull;
  } else {
#pragma unroll
    for (int l = 0; l < D; ++l) R.c[l] = (ok && l < P.d) ? P.spts[(size_t)l * P.N + p] : 0.0f;
#pragma unroll
    for (int q = 0; q < kSigWords; ++q)
      R.sw[q] = (ok && q < nw) ? P.ssig[(size_t)q * P.N + p] : 0ull;
  }
}

// A unit's fields, uniform across the wave (ok = false past the last unit).
struct UnitView {
  uint32_t s0, L, ta_begin, ta_end, nt, inst;
  int tcell, nw;  // grid; signature words to compare (0: no filtering)
  bool ok;
};

__device__ __forceinline__ UnitView unit_view(const PairsArgs& P, uint32_t u, uint32_t u_end) {
  UnitView v;
  v.ok = u < u_end;
  if (!v.ok) {
    v.s0 = v.L = v.ta_begin = v.ta_end = v.nt = v.inst = 0u;
    v.tcell = v.nw = 0;
    return v;
  }
  const UnitDesc U = P.units[u];
  v.s0 = uniform(U.s0);
  v.L = uniform(U.len);
  v.ta_begin = uniform(U.ta_begin);
  v.ta_end = uniform(U.ta_end);
  v.tcell = (int)uniform(U.t);
  v.inst = uniform(U.inst);
  v.nt = (v.L + kPairTile - 1) / kPairTile;
  v.nw = (P.first_owner && v.tcell > 0) ? (v.tcell - 1) / P.gpw + 1 : 0;
  return v;
}

__device__ __forceinline__ uint32_t tile_len(const UnitView& V, uint32_t t) {
  return min((uint32_t)kPairTile, V.L - t * kPairTile);
}

// A row's tile pairs (ta, tb): its diagonal first, then its B tiles from the
// last down to ta + 1, so that a row ends on the next row's own tile.
__device__ __forceinline__ uint32_t row_step_tile(const UnitView& V, uint32_t ta, uint32_t s) {
  return s == 0 ? ta : V.nt - s;
}

// Loads the tile after (ta, tb) in the wave's stream of tile pairs: the
// row's next B tile, else -- the row ending on tile ta + 1 -- that tile again
// (kept from R_cur, not loaded) for the next row, in this unit or in the next
// one when that is the same cell's next row, else the first tile of the next
// unit Vn (nothing when the stream ends).
template <int D>
__device__ __forceinline__ void load_next(const PairsArgs& P, const UnitView& V,
                                          const UnitView& Vn, uint32_t ta, uint32_t tb,
                                          uint32_t lane, const TileRegs<D>& R_cur,
                                          TileRegs<D>& R) {
  uint32_t t = ~0u;  // the unit's next tile to load
  if (tb == ta) {
    if (V.nt > ta + 1) t = V.nt - 1;
  } else if (tb > ta + 1) {
    t = tb - 1;
  } else if (ta + 1 < V.ta_end || (Vn.ok && Vn.s0 == V.s0 && Vn.ta_begin == ta + 1)) {
    R = R_cur;  // tb = ta + 1: the next row's tile, in registers already
    return;
  }
  uint32_t p0 = 0, n = 0;
  int nw = 0;
  if (t != ~0u) {
    p0 = V.s0 + t * kPairTile;
    n = tile_len(V, t);
    nw = V.nw;
  } else if (Vn.ok) {
    p0 = Vn.s0 + Vn.ta_begin * kPairTile;
    n = tile_len(Vn, Vn.ta_begin);
    nw = Vn.nw;
  }
  if (n) load_tile<D>(P, p0, n, nw, lane, R);
}

// Appends this lane's pairs (ai, partner(j)) for the bits j of acc to the
// wave's staging buffer, flushing it to cand as needed.
struct OutStage {
  uint64_t* buf;  // kOutBuf entries of this wave
  uint32_t n = 0;
  uint64_t* dst;               // this block's output segment
  unsigned long long* count;   // and its running total
  uint64_t cap;                // the segment's capacity
};

__device__ __forceinline__ OutStage out_stage(const PairsArgs& P, uint64_t* buf) {
  OutStage O;
  O.buf = buf;
  const uint32_t seg = P.nseg > 1 ? blockIdx.x % P.nseg : 0u;
  O.dst = P.cand + (size_t)seg * P.cap;
  O.count = P.cand_count + seg;
  O.cap = P.cap;
  return O;
}

__device__ __forceinline__ void flush_out(const PairsArgs& P, OutStage& O, uint32_t lane) {
  wave_lds_sync();
  if (O.n) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(O.count, (unsigned long long)O.n);
    base = lane_value(base, 0);
    for (uint32_t e = lane; e < O.n; e += 64) {
      const uint64_t g = base + e;
      if (g < O.cap) O.dst[g] = O.buf[e];
    }
    O.n = 0;
  }
  wave_lds_sync();
}

// Writes the pairs of acc; pair_of(bit) gives the packed pair of a bit.
template <typename PairOf>
__device__ __forceinline__ void emit_pairs(const PairsArgs& P, OutStage& O, uint32_t lane,
                                           uint64_t acc, PairOf pair_of) {
  const uint32_t cnt = (uint32_t)__popcll(acc);
  const uint32_t incl = wave_inclusive_scan(cnt);
  const uint32_t total = lane_value(incl, 63);
  if (!total) return;
  if (O.n + total > (uint32_t)kOutBuf) flush_out(P, O, lane);
  if (total > (uint32_t)kOutBuf) {
    // more than the buffer holds: straight out
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(O.count, (unsigned long long)total);
    base = lane_value(base, 0);
    uint64_t pos = base + incl - cnt;
    while (acc) {
      const int b = __builtin_ctzll(acc);
      acc &= acc - 1;
      if (pos < O.cap) O.dst[pos] = pair_of(b);
      ++pos;
    }
  } else {
    uint32_t pos = O.n + incl - cnt;
    while (acc) {
      const int b = __builtin_ctzll(acc);
      acc &= acc - 1;
      O.buf[pos++] = pair_of(b);
    }
    O.n += total;
  }
}

__device__ __forceinline__ uint64_t pack_pair(uint64_t x, uint64_t y, int pair_bits) {
  return (min(x, y) << pair_bits) | max(x, y);
}

// Appends pair (when keep) to the wave's staging buffer: one slot per
// keeping lane, in lane order, flushing first if they would not fit.
__device__ __forceinline__ void append_pair(const PairsArgs& P, OutStage& O, uint32_t lane,
                                            bool keep, uint64_t pair) {
  const uint64_t kb = ballot(keep);
  const uint32_t nk = (uint32_t)__popcll(kb);
  if (!nk) return;
  if (O.n + nk > (uint32_t)kOutBuf) flush_out(P, O, lane);
  if (keep) O.buf[O.n + rank_below(kb)] = pair;
  O.n += nk;
}

// Accepted pairs of a tile pair listed for the first-owner check, at most
// this many per wave (more: each lane checks its own, one by one).
constexpr uint32_t kPend = 256;

// --- vector screen --------------------------------------------------------
// Lane l holds point a_l of tile a in registers and tests it against every
// point b_j of tile b, read from LDS by broadcast: FP32 squared differences
// summed with FMA; accepted j in one bit mask, j whose FP32 value lies in the
// band around r^2 in a second mask, re-tested in FP64.
template <int D>
__global__ __launch_bounds__(kBlock) void k_cell_pairs(const PairsArgs P) {
  // LDS row stride: rows of 4 floats read with 128-bit loads
  constexpr int DP = D <= 2 ? D : ((D + 3) / 4) * 4;
  __shared__ __attribute__((aligned(16))) float sB[kWaves][kPairTile][DP];
  __shared__ uint32_t sBi[kWaves][kPairTile];
  __shared__ uint64_t sBw[kWaves][kSigWords][kPairTile];
  __shared__ uint64_t sOut[kWaves][kOutBuf];

  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  unsigned long long nre = 0;
  OutStage O = out_stage(P, sOut[w]);

  const uint32_t wave_id = blockIdx.x * kWaves + w;
  const uint32_t nwaves = gridDim.x * kWaves;
  // The wave's units form one stream of tiles, each loaded while the tile
  // pair before it is tested.
  // The wave's units: a contiguous run holding about an equal share of the
  // tile pairs (wave_first), else every nwaves-th unit.
  uint32_t u = wave_id, u_end = P.total_units, step = nwaves;
  if (P.wave_first) {
    u = uniform(P.wave_first[wave_id]);
    u_end = uniform(P.wave_first[wave_id + 1]);
    step = 1;
  }
  UnitView V = unit_view(P, u, u_end);
  TileRegs<D> cur, nxt;
  if (V.ok)
    load_tile<D>(P, V.s0 + V.ta_begin * kPairTile, tile_len(V, V.ta_begin), V.nw, lane, cur);
  while (V.ok) {
    const UnitView Vn = unit_view(P, u + step, u_end);
    const PairTest T = P.tests[V.inst];
    for (uint32_t ta = V.ta_begin; ta < V.ta_end; ++ta) {
      const uint32_t nA = tile_len(V, ta);
      const uint32_t pa0 = V.s0 + ta * kPairTile;
      const bool rowok = lane < nA;
      const TileRegs<D> A = cur;  // the row's tile, also its diagonal B tile
      for (uint32_t s = 0; s < V.nt - ta; ++s) {
      const uint32_t tb = row_step_tile(V, ta, s);
      const uint32_t pb0 = V.s0 + tb * kPairTile;
      const uint32_t nB = tile_len(V, tb);
      wave_lds_sync();
      if (lane < nB) {
        sBi[w][lane] = cur.idx;
#pragma unroll
        for (int l = 0; l < DP; ++l) sB[w][lane][l] = (l < D) ? cur.c[l] : 0.0f;
#pragma unroll
        for (int q = 0; q < kSigWords; ++q) sBw[w][q][lane] = cur.sw[q];
      }
      wave_lds_sync();
      load_next<D>(P, V, Vn, ta, tb, lane, cur, nxt);

      // lane l tests j only when j > lim: every pair once in a diagonal tile
      const int lim = rowok ? (ta == tb ? (int)lane : -1) : 64;
      uint32_t accw[2] = {0u, 0u}, bandw[2] = {0u, 0u};
      auto test = [&](int j, int q, uint32_t& am, uint32_t& bm) {
        float b[DP];
#pragma unroll
        for (int l = 0; l < DP; ++l) b[l] = sB[w][j][l];
        float d2 = 0.0f;
#pragma unroll
        for (int l = 0; l < D; ++l) {
          const float df = A.c[l] - b[l];
          d2 = __builtin_fmaf(df, df, d2);
        }
        // bitwise, not short-circuit: every lane computes every test, so
        // the loop stays free of branches and its LDS reads can run ahead
        const uint32_t ok = (uint32_t)(j > lim);
        const uint32_t in_lo = (uint32_t)(d2 <= T.lo);
        const uint32_t in_hi = (uint32_t)(d2 <= T.hi);
        am |= (ok & in_lo) << q;
        bm |= (ok & in_hi & (in_lo ^ 1u)) << q;
      };
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int jb = h * 32;
        const int jn = min((int)nB - jb, 32);
        if (jn <= 0) break;
        uint32_t am = 0u, bm = 0u;
        if (jn == 32) {
#pragma unroll 8
          for (int q = 0; q < 32; ++q) test(jb + q, q, am, bm);
        } else {
          for (int q = 0; q < jn; ++q) test(jb + q, q, am, bm);
        }
        accw[h] = am;
        bandw[h] = bm;
      }
      uint64_t acc = ((uint64_t)accw[1] << 32) | accw[0];
      uint64_t band = ((uint64_t)bandw[1] << 32) | bandw[0];

      // Band: decide in FP64 exactly as the definition does.  Padding
      // coordinates are zero on both sides and add nothing.
      while (band) {
        const int j = __builtin_ctzll(band);
        band &= band - 1;
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) {
          const double dl = (double)A.c[l] - (double)sB[w][j][l];
          s = s + dl * dl;
        }
        if (s <= T.r2) acc |= 1ull << j;
        ++nre;
      }

      // First owner: drop a pair that an earlier grid put in one cell.
      if (V.nw && ballot(acc != 0ull)) {
        uint64_t m = acc;
        while (m) {
          const int j = __builtin_ctzll(m);
          m &= m - 1;
          uint64_t bw[kSigWords];
#pragma unroll
          for (int q = 0; q < kSigWords; ++q) bw[q] = sBw[w][q][j];
          if (shared_earlier_cell(A.sw, bw, V.tcell, pa0 + lane, A.idx, pb0 + (uint32_t)j,
                                  sBi[w][j], P))
            acc &= ~(1ull << j);
        }
      }

      const uint64_t ai = A.idx;
      emit_pairs(P, O, lane, acc,
                 [&](int j) { return pack_pair(ai, sBi[w][j], T.pair_bits); });
      cur = nxt;
      }
    }
    u += step;
    V = Vn;
  }
  flush_out(P, O, lane);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nre += __shfl_xor(nre, o, 64);
  if (lane == 0 && nre) atomicAdd(P.rechecks, nre);
}

// --- matrix-core screen -----------------------------------------------------
// The squared distances of a 64 x 64 tile pair come from Gram blocks.  With
// the A tile's first point o as origin, a' = a - o and b' = b - o in FP32;
// the rows [a', |a'|^2, 1] and [-2 b', 1, |b'|^2] have dot product
// |a'|^2 + |b'|^2 - 2 a'.b' = |a' - b'|^2, and v_mfma_f32_32x32x2f32
// accumulates 32 x 32 of them over K/2 steps.
//
// The screen accepts v <= lo and rejects v > hi, lo and hi = r^2 -/+ E,
// where E bounds |v - s| for s the FP64 squared distance of the definition:
// recursive-summation bounds for the K products and sums of the expansion
// and for the norms, the rounding of a - o and of r^2 to FP32, all
// proportional to S = max |a'|^2 + max |b'|^2 over the tile pair, with a
// factor 1.5 to spare.  E is set per tile pair, so it widens by itself when
// a cell's points lie far apart (aliased keys, very large cells): the screen
// stays exact and only sends more pairs to FP64.  Pairs with v in between
// are decided in FP64 from the original coordinates.

// v_mfma_f32_32x32x2f32 lane layout: lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32]; result register i of lane l holds D[row][l % 32] with
// row = 8 (i / 4) + 4 (l / 32) + i % 4.
__device__ __forceinline__ uint32_t mfma32_row(uint32_t i, uint32_t lane) {
  return 8u * (i >> 2) + 4u * (lane >> 5) + (i & 3u);
}

typedef float floatx16 __attribute__((ext_vector_type(16)));

// The least float above x (x not NaN; +inf stays +inf).
__device__ __forceinline__ float next_up(float x) {
  const uint32_t b = __float_as_uint(x);
  if (x == 0.0f) return __uint_as_float(1u);
  if (b & 0x80000000u) return __uint_as_float(b - 1u);
  return (x == INFINITY) ? x : __uint_as_float(b + 1u);
}

// The maximum over the wave, uniform: quads (xor 1, xor 2), half rows and
// rows by mirroring, then the four rows' maxima read out.
__device__ __forceinline__ float wave_max_f(float v) {
  auto step = [](float x, uint32_t y) { return fmaxf(x, __uint_as_float(y)); };
  v = step(v, dpp_u32<0xB1>(__float_as_uint(v), __float_as_uint(v)));
  v = step(v, dpp_u32<0x4E>(__float_as_uint(v), __float_as_uint(v)));
  v = step(v, dpp_u32<0x141>(__float_as_uint(v), __float_as_uint(v)));
  v = step(v, dpp_u32<0x140>(__float_as_uint(v), __float_as_uint(v)));
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
}

// Bits of a tile pair's 64-bit masks: bit 16 (2R + C) + 15 - i is register
// i of block (R, C), i.e. row 32 R + mfma32_row(i, lane), column 32 C + l32.
__device__ __forceinline__ uint32_t gram_row(int b, uint32_t lane) {
  return 32u * ((uint32_t)b >> 5) + mfma32_row(15u - ((uint32_t)b & 15u), lane);
}
__device__ __forceinline__ uint32_t gram_col(int b, uint32_t lane) {
  return 32u * (((uint32_t)b >> 4) & 1u) + (lane & 31u);
}

// The screen's band for S = max |a'|^2 + max |b'|^2 (or a bound on it).  The
// products carry lo into the sums (the B rows hold |b'|^2 - lo), so each
// output is x = v - lo: x < 0 accepts, x > W rejects, anything between is
// decided in FP64.  E bounds the rounding of x, including the lo term; a
// band that reaches 0 (cells far wider than r) is decided in FP64 throughout.
struct GramBand {
  float lo;
  uint32_t Wu;    // W as bits: x <= W for x >= 0
  bool all_fp64;
};
__device__ __forceinline__ GramBand gram_band(float S, float r2f, float gain) {
  constexpr float kU = 0x1p-24f;
  const float E = (S + r2f) * gain + r2f * (4.0f * kU) + 1e-36f;
  GramBand b;
  b.all_fp64 = !(E < r2f);
  b.lo = b.all_fp64 ? 0.0f : (r2f - E) * (1.0f - 0x1p-20f);
  const float hi = (r2f + E) * (1.0f + 0x1p-20f);
  b.Wu = __float_as_uint(next_up(hi - b.lo));
  return b;
}

// The matrix cores' operands of a tile from its rows, one row per lane:
// block X (rows 32 X .. 32 X + 31) takes, in lane l, element 2 q + (l >> 5)
// of row 32 X + (l & 31).  Lanes 0-31 of block 0 keep their own even
// elements and lanes 32-63 need the odd elements of lanes 0-31; block 1
// the reverse.  Swapping the upper half of row[2 q] with the lower half of
// row[2 q + 1] across the wave (v_permlane32_swap) leaves block 0's
// operand in the first and block 1's in the second: no trip through LDS.
template <int KS>
__device__ __forceinline__ void gram_operands(const float* row, float (&op)[2][KS]) {
#pragma unroll
  for (int q = 0; q < KS; ++q) {
    const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(row[2 * q]),
                                                     __float_as_uint(row[2 * q + 1]), false, false);
    op[0][q] = __uint_as_float(sw[0]);
    op[1][q] = __uint_as_float(sw[1]);
  }
}

// Four waves per SIMD up to D = 9 (at most 128 registers: a few spills at
// D = 9 cost less than the lost wave); three above, where the registers the
// wider rows need would spill more.
template <int D>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(D <= 9 ? 4 : 3))) void
k_cell_pairs_gram(
    const PairsArgs P) {
  constexpr int KA = (D + 3) & ~1;  // augmented row length, even
  constexpr int KS = KA / 2;        // MFMA steps per block
  constexpr float kGain = 1.5f * (float)(2 * KA + D + 8) * 0x1p-24f;
  // the A and B tiles' signature words
  constexpr int kRegion = 2 * kSigWords * kPairTile;
  __shared__ __attribute__((aligned(16))) float sAreg[kWaves][kRegion];
  __shared__ __attribute__((aligned(16))) float sBreg[kWaves][kRegion];
  __shared__ uint32_t sAi[kWaves][kPairTile];
  __shared__ uint32_t sBi[kWaves][kPairTile];
  __shared__ uint64_t sOut[kWaves][kOutBuf];
  __shared__ uint16_t sPend[kWaves][kPend];  // accepted (lane << 6 | bit) codes

  const uint32_t lane = lane_id();
  const uint32_t l32 = lane & 31u, h = lane >> 5;
  const int w = threadIdx.x >> 6;
  uint64_t (*sAw)[kPairTile] = reinterpret_cast<uint64_t (*)[kPairTile]>(sAreg[w]);
  uint64_t (*sBw)[kPairTile] = reinterpret_cast<uint64_t (*)[kPairTile]>(sBreg[w]);
  unsigned long long nre = 0;
  OutStage O = out_stage(P, sOut[w]);

  const uint32_t wave_id = blockIdx.x * kWaves + w;
  const uint32_t nwaves = gridDim.x * kWaves;
  // The wave's units form one stream of tiles, each loaded while the tile
  // pair before it is tested.
  // The wave's units: a contiguous run holding about an equal share of the
  // tile pairs (wave_first), else every nwaves-th unit.
  uint32_t u = wave_id, u_end = P.total_units, step = nwaves;
  if (P.wave_first) {
    u = uniform(P.wave_first[wave_id]);
    u_end = uniform(P.wave_first[wave_id + 1]);
    step = 1;
  }
  UnitView V = unit_view(P, u, u_end);
  TileRegs<D> cur, nxt;
  if (V.ok)
    load_tile<D>(P, V.s0 + V.ta_begin * kPairTile, tile_len(V, V.ta_begin), V.nw, lane, cur);
  while (V.ok) {
    const UnitView Vn = unit_view(P, u + step, u_end);
    const PairTest T = P.tests[V.inst];
    const float r2f = (float)T.r2;
    // When every unit is one grid cell, S <= s_bound for all of the unit's
    // tile pairs: one band for the unit, no per-tile maxima.
    const float s_bound =
        __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(T.s_bound)));
    const bool unit_band = P.unit_band && s_bound > 0.0f;
    const GramBand ub = gram_band(s_bound, r2f, kGain);
    // origin: the first point of the unit's first tile (lane 0; wave-uniform)
    float o[D];
#pragma unroll
    for (int l = 0; l < D; ++l)
      o[l] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(cur.c[l])));
    for (uint32_t ta = V.ta_begin; ta < V.ta_end; ++ta) {
    const uint32_t nA = tile_len(V, ta);
    const uint32_t pa0 = V.s0 + ta * kPairTile;
    // tile a: centred rows, norms; invalid rows get a huge norm (rejected)
    wave_lds_sync();
    float na = 0.0f;
    float areg[2][KS];
    {
      float row[KA];
      if (lane < nA) {
        float n2 = 0.0f;
#pragma unroll
        for (int l = 0; l < D; ++l) {
          const float v = cur.c[l] - o[l];
          row[l] = v;
          n2 = __builtin_fmaf(v, v, n2);
        }
        row[D] = n2;
        na = n2;
      } else {
#pragma unroll
        for (int l = 0; l < D; ++l) row[l] = 0.0f;
        row[D] = 1e30f;
      }
      row[D + 1] = 1.0f;
#pragma unroll
      for (int l = D + 2; l < KA; ++l) row[l] = 0.0f;
      sAi[w][lane] = cur.idx;
      gram_operands<KS>(row, areg);
    }
    const float amax = unit_band ? 0.0f : wave_max_f(na);
    if (V.nw) {
#pragma unroll
      for (int q = 0; q < kSigWords; ++q) sAw[q][lane] = cur.sw[q];
    }
    wave_lds_sync();  // the A indices and words, before lanes read each other's

    for (uint32_t s = 0; s < V.nt - ta; ++s) {
      const uint32_t tb = row_step_tile(V, ta, s);
      const uint32_t pb0 = V.s0 + tb * kPairTile;
      const uint32_t nB = min((uint32_t)kPairTile, V.L - tb * kPairTile);
      wave_lds_sync();
      float nb = 0.0f;
      uint64_t bsw[kSigWords];
      float row[KA];
      if (lane < nB) {
        float n2 = 0.0f;
#pragma unroll
        for (int l = 0; l < D; ++l) {
          const float v = cur.c[l] - o[l];
          row[l] = -2.0f * v;
          n2 = __builtin_fmaf(v, v, n2);
        }
        nb = n2;
      } else {
#pragma unroll
        for (int l = 0; l < D; ++l) row[l] = 0.0f;
      }
      row[D] = 1.0f;
#pragma unroll
      for (int l = D + 2; l < KA; ++l) row[l] = 0.0f;
#pragma unroll
      for (int q = 0; q < kSigWords; ++q) bsw[q] = cur.sw[q];
      // the tile pair's band: the unit's, else from this pair's maxima
      GramBand bd = ub;
      if (!unit_band) bd = gram_band(amax + wave_max_f(nb), r2f, kGain);
      const bool all_fp64 = bd.all_fp64;
      const float lo = bd.lo;
      const uint32_t Wu = bd.Wu;
      row[D + 1] = lane < nB ? nb - lo : 1e30f;
      sBi[w][lane] = cur.idx;
      float breg[2][KS];
      gram_operands<KS>(row, breg);
      wave_lds_sync();  // the B indices, before lanes read each other's
      load_next<D>(P, V, Vn, ta, tb, lane, cur, nxt);

      const bool diag = (ta == tb);
      uint64_t acc = 0ull, band = 0ull;
#pragma unroll
      for (int R = 0; R < 2; ++R) {
        if (R == 1 && nA <= 32u) break;
#pragma unroll
        for (int C = 0; C < 2; ++C) {
          if (C == 1 && nB <= 32u) break;
          if (diag && R > C) continue;  // rows above the columns: no pairs
          floatx16 v = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f,
                        0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int q = 0; q < KS; ++q)
            v = __builtin_amdgcn_mfma_f32_32x32x2f32(areg[R][q], breg[C][q], v, 0, 0, 0);
          // Bit 15 - i of am: x[i] < 0, its sign shifted in from the right
          // (x is finite: the host keeps coordinates small enough).  The
          // least x >= 0 as bits (negative x are larger as unsigned) tells
          // whether any x lies in the band; only then are its bits built:
          // bit 15 - i of cm is x[i] <= W.
          uint32_t am = 0u, mn = 0xFFFFFFFFu;
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            am = __builtin_amdgcn_alignbit(am, __float_as_uint(v[i]), 31);
            mn = min(mn, __float_as_uint(v[i]));
          }
          uint32_t cm = 0u;
          if (ballot(mn <= Wu) || all_fp64) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
              cm = __builtin_amdgcn_alignbit(cm, __float_as_uint(v[i]) - (Wu + 1u), 31);
            if (all_fp64) {
              // every pair of real points is decided in FP64; the padding
              // rows and columns of a short tile hold no points
              const bool col_in = 32u * (uint32_t)C + l32 < nB;
              uint32_t in = 0u;
#pragma unroll
              for (int i = 0; i < 16; ++i)
                in = (in << 1) |
                     ((col_in && 32u * (uint32_t)R + mfma32_row((uint32_t)i, lane) < nA) ? 1u : 0u);
              cm = in;
              am = 0u;
            }
          }
          uint32_t valid = 0xFFFFu;
          if (diag && R == C) {
            // row < col holds for registers i < cnt (rows rise with i)
            const int x = (int)l32 - 4 * (int)h;
            int cnt = 0;
#pragma unroll
            for (int g = 0; g < 4; ++g) cnt += min(max(x - 8 * g, 0), 4);
            valid = (0xFFFFu << (16 - cnt)) & 0xFFFFu;
          }
          const int sh = (R * 2 + C) * 16;
          am &= valid;
          acc |= (uint64_t)am << sh;
          band |= (uint64_t)(cm & valid & ~am) << sh;
          // one block's accumulators at a time
          __builtin_amdgcn_sched_barrier(0);
        }
      }

      // Band: decide in FP64 exactly as the definition does.
      while (band) {
        const int b = __builtin_ctzll(band);
        band &= band - 1;
        const uint32_t pa = sAi[w][gram_row(b, lane)], pb = sBi[w][gram_col(b, lane)];
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) {
          const double dl = (double)P.pts[(size_t)pa * D + l] - (double)P.pts[(size_t)pb * D + l];
          s = s + dl * dl;
        }
        if (s <= T.r2) acc |= 1ull << b;
        ++nre;
      }

      // First owner: drop a pair that an earlier grid put in one cell.  The
      // B rows are in registers by now: their space takes the B words.  The
      // accepted bits are listed in LDS as (lane, bit) codes, each lane
      // writing its own in turn, and are then worked one per lane -- the
      // pair's row and column, the check, the packed pair -- so the per-pair
      // work takes ceil(count / 64) rounds rather than the most any one lane
      // holds.
      const uint32_t cnt = (uint32_t)__popcll(acc);
      const uint32_t incl = wave_inclusive_scan(cnt);
      const uint32_t total = lane_value(incl, 63);
      const bool check = V.nw != 0;
      if (total && check) {
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < kSigWords; ++q) sBw[q][lane] = bsw[q];
      }
      if (total && total <= kPend) {
        uint32_t pos = incl - cnt;
        uint64_t m = acc;
        while (m) {
          const int b = __builtin_ctzll(m);
          m &= m - 1;
          sPend[w][pos++] = (uint16_t)((lane << 6) | (uint32_t)b);
        }
        wave_lds_sync();
        for (uint32_t e0 = 0; e0 < total; e0 += 64) {
          const uint32_t e = e0 + lane;
          bool keep = e < total;
          uint64_t pair = 0;
          if (keep) {
            const uint32_t code = sPend[w][e];
            const int b = (int)(code & 63u);
            const uint32_t row = gram_row(b, code >> 6), col = gram_col(b, code >> 6);
            const uint32_t ia = sAi[w][row], ib = sBi[w][col];
            if (check) {
              uint64_t aq[kSigWords], bq[kSigWords];
#pragma unroll
              for (int q = 0; q < kSigWords; ++q) {
                aq[q] = sAw[q][row];
                bq[q] = sBw[q][col];
              }
              keep = !shared_earlier_cell(aq, bq, V.tcell, pa0 + row, ia, pb0 + col, ib, P);
            }
            pair = pack_pair(ia, ib, T.pair_bits);
          }
          append_pair(P, O, lane, keep, pair);
        }
        wave_lds_sync();  // sPend is rewritten by the next tile pair
      } else if (total) {
        // more than the list holds: each lane checks and writes its own
        if (check) {
          wave_lds_sync();
          uint64_t m = acc;
          while (m) {
            const int b = __builtin_ctzll(m);
            m &= m - 1;
            const uint32_t row = gram_row(b, lane), col = gram_col(b, lane);
            uint64_t aq[kSigWords], bq[kSigWords];
#pragma unroll
            for (int q = 0; q < kSigWords; ++q) {
              aq[q] = sAw[q][row];
              bq[q] = sBw[q][col];
            }
            if (shared_earlier_cell(aq, bq, V.tcell, pa0 + row, sAi[w][row], pb0 + col,
                                    sBi[w][col], P))
              acc &= ~(1ull << b);
          }
        }
        emit_pairs(P, O, lane, acc, [&](int b) {
          return pack_pair(sAi[w][gram_row(b, lane)], sBi[w][gram_col(b, lane)], T.pair_bits);
        });
      }
      cur = nxt;
    }
    }
    u += step;
    V = Vn;
  }
  flush_out(P, O, lane);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nre += __shfl_xor(nre, o, 64);
  if (lane == 0 && nre) atomicAdd(P.rechecks, nre);
}

// ---------------------------------------------------------------------------
// query mode.  A query point takes the role of one more point of the indexed
// set: under grid t it falls in the cell floor((R_t q)/(alpha r) + u_t),
// computed in FP64 in the same order as the points' cells, and is reported
// with the indexed points of that cell within r, once (first-owner rule with
// the query's own signature).

// Cell prefix (segment and packed cell fields) of every query under every
// grid, and the query's signature words.  One thread per query.
template <int D>
__global__ __launch_bounds__(kBlock) void k_query_keys(const QueryArgs A) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= A.m) return;
  const int d = D > 0 ? D : A.d;
  float p[D > 0 ? D : 1];
  bool finite = true;
  if (D > 0) {
#pragma unroll
    for (int l = 0; l < (D > 0 ? D : 1); ++l) p[l] = A.queries[q * d + l];
  }
  for (int l = 0; l < d; ++l) finite = finite && isfinite(A.queries[q * d + l]);
  if (!finite) {
    atomicOr(A.err, 2u);
    return;
  }
  const uint64_t bmask = (1ull << A.sig_b) - 1ull;
  uint64_t sword = 0;
  int sw = -1;
  bool bad = false;
  for (int t = 0; t < A.k; ++t) {
    const double* Rt = A.R + (size_t)t * d * d;
    const double* ut = A.u + (size_t)t * d;
    const int64_t* kl = A.klo + (size_t)t * d;
    uint64_t cell = 0, grp = 0;
    for (int j = 0; j < d; ++j) {
      // same operation order as the points' keys (the key kernel)
      double z;
      if (D > 0) {
        z = Rt[(size_t)j * d] * (double)p[0];
        for (int l = 1; l < d; ++l) z = z + Rt[(size_t)j * d + l] * (double)p[l];
      } else {
        z = Rt[(size_t)j * d] * (double)A.queries[q * d];
        for (int l = 1; l < d; ++l) z = z + Rt[(size_t)j * d + l] * (double)A.queries[q * d + l];
      }
      const double y = z * A.inv_c + ut[j];
      const bool ok = fabs(y) < 2147483648.0;
      bad |= !ok;
      const int64_t kap = ok ? (int64_t)(int32_t)floor(y) : 0;
      const uint64_t mask = (1ull << A.layout->bits[j]) - 1ull;
      cell |= ((uint64_t)(kap - kl[j]) & mask) << A.layout->shift[j];
      grp |= ((uint64_t)(kap - kl[j]) & bmask) << (j * A.sig_b);
    }
    const uint64_t prefix = A.cell_bits < 64 ? ((A.grids[t].seg << A.cell_bits) | cell) : cell;
    A.qkey[(size_t)q * A.k + t] = prefix;
    if (A.sig) {
      const int w = t / A.gpw;
      if (w != sw) {
        if (sw >= 0) A.qsig[(size_t)q * A.W + sw] = sword;
        sword = 0;
        sw = w;
      }
      sword |= grp << ((t - w * A.gpw) * A.g);
    }
  }
  if (A.sig && sw >= 0) A.qsig[(size_t)q * A.W + sw] = sword;
  if (bad) atomicOr(A.err, 1u);
}

// First position in keys[0..n) whose cell prefix is >= K.
__device__ __forceinline__ uint32_t prefix_lower_bound(const uint64_t* keys, uint32_t n, int shift,
                                                       uint64_t K) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if ((keys[mid] >> shift) < K) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Pairs (query, indexed point): one wave per query; lane t finds grid t's
// cell by binary search, then the wave tests that cell's members.
template <int D>
__global__ __launch_bounds__(kBlock) void k_query_pairs(const QueryArgs A) {
  __shared__ uint64_t sOut[kWaves][kOutBuf];
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  const int d = D > 0 ? D : A.d;
  PairsArgs P{};  // output staging shares the pair kernels' machinery
  P.cand = A.cand;
  P.cap = A.cap;
  P.cand_count = A.cand_count;
  OutStage O = out_stage(P, sOut[w]);
  const uint32_t n = (uint32_t)A.n;
  const int64_t wave_id = (int64_t)blockIdx.x * kWaves + w;
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  for (int64_t q = wave_id; q < A.m; q += nwaves) {
    double qc[D > 0 ? D : 1];
    if (D > 0) {
#pragma unroll
      for (int l = 0; l < (D > 0 ? D : 1); ++l) qc[l] = (double)A.queries[q * d + l];
    }
    uint64_t qw[kSigWords] = {0ull, 0ull};
    if (A.sig)
#pragma unroll
      for (int x = 0; x < kSigWords; ++x) qw[x] = x < A.W ? A.qsig[(size_t)q * A.W + x] : 0ull;
    for (int t0 = 0; t0 < A.k; t0 += 64) {
      // lane t: the range of grid t0 + t
      uint32_t rlo = 0, rhi = 0;
      const int tl = t0 + (int)lane;
      if (tl < A.k) {
        const uint64_t K = A.qkey[(size_t)q * A.k + tl];
        const uint64_t* keys = A.grids[tl].keys;
        const int sh = A.grids[tl].idx_bits;
        rlo = prefix_lower_bound(keys, n, sh, K);
        rhi = rlo;
        while (rhi < n && (keys[rhi] >> sh) == K && rhi - rlo < 8u) ++rhi;
        if (rhi < n && (keys[rhi] >> sh) == K)
          rhi = K == ~0ull ? n : prefix_lower_bound(keys + rhi, n - rhi, sh, K + 1ull) + rhi;
      }
      const int tn = min(64, A.k - t0);
      for (int tt = 0; tt < tn; ++tt) {
        const int t = t0 + tt;
        const uint32_t lo = lane_value(rlo, tt);
        const uint32_t hi = lane_value(rhi, tt);
        const QueryGrid G = A.grids[t];
        const uint64_t imask = G.idx_bits ? ((1ull << G.idx_bits) - 1ull) : 0ull;
        for (uint32_t base = lo; base < hi; base += 64) {
          const uint32_t pos = base + lane;
          bool hit = false;
          uint32_t i = 0;
          if (pos < hi) {
            i = G.idx_bits ? (uint32_t)(G.keys[pos] & imask) : G.idx[pos];
            const float* row = A.pts + (size_t)i * d;
            double s2 = 0.0;
            if (D > 0) {
#pragma unroll
              for (int l = 0; l < (D > 0 ? D : 1); ++l) {
                const double dl = qc[l] - (double)row[l];
                s2 = s2 + dl * dl;
              }
            } else {
              for (int l = 0; l < d; ++l) {
                const double dl = (double)A.queries[q * d + l] - (double)row[l];
                s2 = s2 + dl * dl;
              }
            }
            hit = s2 <= A.r2;
            if (hit && A.sig && t > 0) {
              // dropped if an earlier grid put the query and the point in one cell
              const int nw = (t - 1) / A.gpw + 1;
              for (int x = 0; x < nw && hit; ++x) {
                const uint64_t xw =
                    (x < kSigWords ? qw[x] : A.qsig[(size_t)q * A.W + x]) ^ A.sig[(size_t)i * A.W + x];
                const int ng = min(A.gpw, t - x * A.gpw);
                const uint64_t keep = (ng * A.g >= 64) ? ~0ull : ((1ull << (ng * A.g)) - 1ull);
                hit = (((xw - A.lows) & ~xw & A.highs) & keep) == 0ull;
              }
            }
          }
          const uint64_t pair = ((uint64_t)q << A.pb) | i;
          emit_pairs(P, O, lane, hit ? 1ull : 0ull, [&](int) { return pair; });
        }
      }
    }
  }
  flush_out(P, O, lane);
}

// The MR-metric's FP64 decision for one candidate pair: the robots' squared
// displacements summed in axis order, their square roots (correctly rounded)
// added in robot order, the sum tested against r.
__device__ __forceinline__ bool mr_keep(const MrFilterArgs& A, uint64_t v) {
  const uint64_t a = v >> A.pair_bits, b = v & ((1ull << A.pair_bits) - 1ull);
  int lo = 0, hi = A.m - 1;  // the last instance with pt_off <= a
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (A.inst[mid].pt_off <= (int64_t)a) lo = mid;
    else hi = mid - 1;
  }
  const MrInst I = A.inst[lo];
  if (I.sub <= 0) return true;
  const float* ra = A.rows_a + (size_t)a * A.d;
  const float* rb = A.rows_b + (size_t)b * A.d;
  double s = 0.0;
  for (int o = 0; o < A.d; o += I.sub) {
    double t = 0.0;
    for (int l = o; l < o + I.sub; ++l) {
      const double dl = (double)ra[l] - (double)rb[l];
      t = t + dl * dl;
    }
    s = s + __builtin_sqrt(t);
  }
  return s <= I.r;
}

// Keeps the packed pairs v of in[0, count) with keep(v), appended to out in
// no particular order.  One block per tile of kBlock * kCompactPer pairs
// (coalesced reads, one lane per pair and step); a tile's kept pairs take
// one atomic on out_count.  Every lane of a block runs the same tiles.
constexpr int kCompactPer = 16;
template <class Keep>
__device__ __forceinline__ void compact_tiles(const uint64_t* __restrict__ in, uint64_t count,
                                              uint64_t* __restrict__ out,
                                              unsigned long long* out_count, Keep keep) {
  __shared__ uint32_t sWave[kWaves];
  __shared__ unsigned long long sBase;
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  const uint64_t tile = (uint64_t)kBlock * kCompactPer;
  for (uint64_t t0 = (uint64_t)blockIdx.x * tile; t0 < count; t0 += (uint64_t)gridDim.x * tile) {
    uint64_t v[kCompactPer], km[kCompactPer];
    uint32_t tot = 0;
#pragma unroll
    for (int i = 0; i < kCompactPer; ++i) {
      const uint64_t p = t0 + (uint64_t)i * kBlock + threadIdx.x;
      v[i] = p < count ? in[p] : 0ull;
    }
#pragma unroll
    for (int i = 0; i < kCompactPer; ++i) {
      const uint64_t p = t0 + (uint64_t)i * kBlock + threadIdx.x;
      km[i] = ballot(p < count && keep(v[i]));
      tot += (uint32_t)__popcll(km[i]);
    }
    if (lane == 0) sWave[w] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t all = 0;
#pragma unroll
      for (int x = 0; x < kWaves; ++x) all += sWave[x];
      sBase = all ? atomicAdd(out_count, (unsigned long long)all) : 0ull;
    }
    __syncthreads();
    unsigned long long at = sBase;
    for (int x = 0; x < w; ++x) at += sWave[x];
#pragma unroll
    for (int i = 0; i < kCompactPer; ++i) {
      if ((km[i] >> lane) & 1ull) out[at + rank_below(km[i])] = v[i];
      at += (uint32_t)__popcll(km[i]);
    }
    __syncthreads();  // sWave and sBase are rewritten by the next tile
  }
}

__global__ __launch_bounds__(kBlock) void k_mr_filter(const MrFilterArgs A) {
  compact_tiles(A.in, A.count, A.out, A.out_count, [&](uint64_t v) { return mr_keep(A, v); });
}

// Repeats removed with one bit per unordered pair of an instance (the
// upper triangle, a' < b' local indices, bit b'(b'-1)/2 + a'): the
// candidate whose atomic OR sets the bit is kept, any later one is not.
// Which of equal candidates survives does not matter: they are equal.
__device__ __forceinline__ bool bitmap_first(const BitmapArgs& A, uint64_t v) {
  const uint64_t a = v >> A.pair_bits, b = v & ((1ull << A.pair_bits) - 1ull);
  int lo = 0, hi = A.m - 1;  // the last instance with pt_off <= a
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (A.inst[mid].pt_off <= (int64_t)a) lo = mid;
    else hi = mid - 1;
  }
  const BitmapInst I = A.inst[lo];
  const uint64_t la = a - (uint64_t)I.pt_off, lb = b - (uint64_t)I.pt_off;
  const uint64_t bit = (uint64_t)I.bit_off + lb * (lb - 1) / 2 + la;
  const uint32_t m = 1u << (bit & 31u);
  return (atomicOr(A.bits + (bit >> 5), m) & m) == 0u;
}

__global__ __launch_bounds__(kBlock) void k_bitmap_unique(const BitmapArgs A) {
  compact_tiles(A.in, A.count, A.out, A.out_count, [&](uint64_t v) { return bitmap_first(A, v); });
}

// Segment blockIdx.y of the pair output to its place in dst.
__global__ __launch_bounds__(kBlock) void k_seg_compact(const uint64_t* __restrict__ src,
                                                        uint64_t seg_cap,
                                                        const unsigned long long* __restrict__ cnt,
                                                        uint64_t* __restrict__ dst) {
  const uint32_t g = blockIdx.y;
  uint64_t off = 0;
  for (uint32_t h = 0; h < g; ++h) off += cnt[h];
  const uint64_t n = cnt[g];
  const uint64_t* s = src + (size_t)g * seg_cap;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock)
    dst[off + i] = s[i];
}

// Unit descriptors of cell c: the whole cell, or one unit per tile.
__global__ void k_unit_fill(const uint32_t* __restrict__ start, const uint32_t* __restrict__ end,
                            const uint32_t* __restrict__ unit_off, uint32_t ncells,
                            const uint32_t* __restrict__ dcells, uint32_t cell_unit_tiles,
                            const uint64_t* __restrict__ skeys, int seg_shift, int sa,
                            const SegDesc* __restrict__ segs, UnitDesc* __restrict__ desc,
                            uint64_t* __restrict__ work) {
  if (dcells) ncells = min(ncells, *dcells);
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncells;
       c += gridDim.x * blockDim.x) {
  const uint32_t s0 = start[c], L = end[c] - s0;
  const uint32_t nt = (L + kPairTile - 1) / kPairTile;
  const int seg = sa + (seg_shift >= 64 ? 0 : (int)(skeys[s0] >> seg_shift));
  UnitDesc D;
  D.s0 = s0;
  D.len = L;
  D.t = (uint32_t)segs[seg].t;
  D.inst = (uint32_t)segs[seg].inst;
  D.pad[0] = D.pad[1] = 0u;
  const uint32_t o = unit_off[c];
  if (nt <= cell_unit_tiles) {
    D.ta_begin = 0;
    D.ta_end = nt;
    desc[o] = D;
    if (work) work[o] = (uint64_t)nt * (nt + 1) / 2;  // tile pairs of the unit
  } else {
    for (uint32_t q = 0; q < nt; ++q) {
      D.ta_begin = q;
      D.ta_end = q + 1;
      desc[o + q] = D;
      if (work) work[o + q] = nt - q;
    }
  }
  }
}

// first[w] = the first unit whose exclusive prefix of tile pairs reaches
// w total / nwaves, for w <= nwaves: wave w takes units [first[w],
// first[w + 1]), a contiguous run with about an equal share of the work.
__global__ void k_wave_ranges(const uint64_t* __restrict__ work_off, uint32_t nunits,
                              const uint64_t* __restrict__ total, uint32_t nwaves,
                              uint32_t* __restrict__ first) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w > nwaves) return;
  // w total / nwaves without overflow: total < 2^56 (units x tile pairs)
  const uint64_t T = *total;
  const uint64_t target = (T / nwaves) * w + (T % nwaves) * w / nwaves;
  uint32_t lo = 0, hi = nunits;  // first index with work_off >= target
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (work_off[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  first[w] = w == nwaves ? nunits : lo;
}

// spts[l][p] and ssig[w][p] for the positions p of every unit (one wave per
// unit, one lane per position).  All loads of a lane are issued before its
// stores.
template <int D>
__global__ __launch_bounds__(kBlock) void k_gather_units(const PairsArgs P,
                                                         const uint64_t* __restrict__ sig,
                                                         float* __restrict__ spts,
                                                         uint64_t* __restrict__ ssig) {
  const uint32_t u = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (u >= P.total_units) return;
  const UnitDesc U = P.units[u];
  const uint32_t lane = lane_id();
  for (uint32_t ta = U.ta_begin; ta < U.ta_end; ++ta) {
  const uint32_t n = min((uint32_t)kPairTile, U.len - ta * kPairTile);
  if (lane >= n) break;
  const uint32_t p = U.s0 + ta * kPairTile + lane;
  const uint32_t i = point_at(P, p);
  const int d = D > 0 ? D : P.d;
  const float* __restrict__ row = P.pts + (size_t)i * d;
  if (D > 0) {
    float c[D > 0 ? D : 1];
#pragma unroll
    for (int l = 0; l < (D > 0 ? D : 1); ++l) c[l] = row[l];
    uint64_t w[kSigWords];
#pragma unroll
    for (int q = 0; q < kSigWords; ++q) w[q] = (sig && q < P.W) ? sig[(size_t)i * P.W + q] : 0ull;
#pragma unroll
    for (int l = 0; l < (D > 0 ? D : 1); ++l) spts[(size_t)l * P.N + p] = c[l];
#pragma unroll
    for (int q = 0; q < kSigWords; ++q)
      if (sig && q < P.W) ssig[(size_t)q * P.N + p] = w[q];
  } else {
    for (int l = 0; l < d; ++l) spts[(size_t)l * P.N + p] = row[l];
  }
  if (sig)
    for (int q = (D > 0 ? kSigWords : 0); q < P.W; ++q)
      ssig[(size_t)q * P.N + p] = sig[(size_t)i * P.W + q];
  }
}

// ---------------------------------------------------------------------------
// CSR

__global__ void k_swap_pairs(const uint64_t* __restrict__ pairs, size_t count, int pb,
                             uint64_t* __restrict__ out) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const uint64_t k = pairs[p];
  const uint64_t mask = (1ull << pb) - 1ull;
  out[p] = ((k & mask) << pb) | (k >> pb);
}

__global__ void k_row_runs(const uint64_t* __restrict__ keys, size_t count, int pb,
                           uint32_t* __restrict__ rstart, uint32_t* __restrict__ rend) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const uint64_t row = keys[p] >> pb;
  if (p == 0 || (keys[p - 1] >> pb) != row) rstart[row] = (uint32_t)p;
  if (p + 1 == count || (keys[p + 1] >> pb) != row) rend[row] = (uint32_t)(p + 1);
}

__global__ void k_row_degree(const uint32_t* __restrict__ lo_start, const uint32_t* __restrict__ lo_end,
                             const uint32_t* __restrict__ up_start, const uint32_t* __restrict__ up_end,
                             int64_t n, uint64_t* __restrict__ deg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t c = (uint64_t)(up_end[i] - up_start[i]);
  if (lo_start) c += (uint64_t)(lo_end[i] - lo_start[i]);
  deg[i] = c;
}

__global__ void k_csr_fill_upper(const uint64_t* __restrict__ up, size_t count, int pb,
                                 const int64_t* __restrict__ row_ptr,
                                 const uint32_t* __restrict__ lo_start,
                                 const uint32_t* __restrict__ lo_end,
                                 const uint32_t* __restrict__ up_start, int32_t* __restrict__ col) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const uint64_t k = up[p];
  const uint64_t i = k >> pb, j = k & ((1ull << pb) - 1ull);
  int64_t pos = row_ptr[i] + (int64_t)(p - up_start[i]);
  if (lo_start) pos += (int64_t)(lo_end[i] - lo_start[i]);
  col[pos] = (int32_t)j;
}

__global__ void k_csr_fill_lower(const uint64_t* __restrict__ lo, size_t count, int pb,
                                 const int64_t* __restrict__ row_ptr,
                                 const uint32_t* __restrict__ lo_start, int32_t* __restrict__ col) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const uint64_t k = lo[q];
  const uint64_t j = k >> pb, i = k & ((1ull << pb) - 1ull);
  col[row_ptr[j] + (int64_t)(q - lo_start[j])] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// Neighbour lists by row buckets.  Directed entries (row, col) -- both
// orientations of every pair, or only (i, j) for upper-only lists -- are
// partitioned into buckets of 2^rb consecutive rows: per-block bucket counts,
// one device-wide scan in bucket-major order, and a scatter in which each
// block places its entries through LDS cursors.  An entry is stored as the
// 32-bit local key (row mod 2^rb) << pb | col.  Each bucket is then sorted in
// LDS (bitonic) with repeats removed, and the emit step writes col and the
// bucket's slice of row_ptr.  The order of entries inside a bucket before the
// local sort does not matter: the sort makes it canonical.

// The pairs a partition block reads: a chunk of one array, or -- when the
// pairs are still in the pair kernels' nseg output segments (segment s at
// pairs + s seg_cap, seg_cnt[s] entries) -- an equal share of one segment
// (block b takes segment b % nseg; nblocks is a multiple of nseg).
struct PairRange {
  const uint64_t* src;
  size_t base, end;
};
__device__ __forceinline__ PairRange pair_range(const uint64_t* pairs, size_t count,
                                                uint32_t chunk, uint32_t nblocks,
                                                const unsigned long long* seg_cnt,
                                                uint64_t seg_cap, uint32_t nseg) {
  PairRange r;
  if (nseg) {
    const uint32_t seg = blockIdx.x % nseg, bps = nblocks / nseg, part = blockIdx.x / nseg;
    const size_t cnt = (size_t)min((unsigned long long)seg_cap, seg_cnt[seg]);
    const size_t ch = (cnt + bps - 1) / bps;
    r.src = pairs + (size_t)seg * seg_cap;
    r.base = min(cnt, (size_t)part * ch);
    r.end = min(cnt, r.base + ch);
  } else {
    r.src = pairs;
    r.base = (size_t)blockIdx.x * chunk;
    r.end = min(count, r.base + chunk);
  }
  return r;
}

template <int TH>
__global__ __launch_bounds__(TH) void k_bucket_hist(const uint64_t* __restrict__ pairs,
                                                    size_t count, int pb, int rb, int both,
                                                    uint32_t nbuckets, uint32_t chunk,
                                                    uint32_t nblocks,
                                                    const unsigned long long* __restrict__ seg_cnt,
                                                    uint64_t seg_cap, uint32_t nseg,
                                                    uint32_t* __restrict__ part,
                                                    uint32_t* __restrict__ zero_word) {
  extern __shared__ uint32_t h[];
  if (zero_word && blockIdx.x == 0 && threadIdx.x == 0) *zero_word = 0u;
  for (uint32_t b = threadIdx.x; b < nbuckets; b += TH) h[b] = 0u;
  __syncthreads();
  const PairRange pr = pair_range(pairs, count, chunk, nblocks, seg_cnt, seg_cap, nseg);
  const uint64_t* __restrict__ src = pr.src;
  const size_t base = pr.base, end = pr.end;
  const uint64_t cmask = (1ull << pb) - 1ull;
  // eight loads in flight per thread, then their atomics
  for (size_t q0 = base; q0 < end; q0 += 8 * TH) {
    uint64_t k8[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      const size_t q = q0 + (size_t)x * TH + threadIdx.x;
      k8[x] = q < end ? src[q] : ~0ull;
    }
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      if (k8[x] == ~0ull) continue;
      atomicAdd(&h[(uint32_t)((k8[x] >> pb) >> rb)], 1u);
      if (both) atomicAdd(&h[(uint32_t)((k8[x] & cmask) >> rb)], 1u);
    }
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nbuckets; b += TH)
    part[(size_t)b * nblocks + blockIdx.x] = h[b];
}

template <int TH>
__global__ __launch_bounds__(TH) void k_bucket_scatter(const uint64_t* __restrict__ pairs,
                                                       size_t count, int pb, int rb, int both,
                                                       uint32_t nbuckets, uint32_t chunk,
                                                       uint32_t nblocks,
                                                       const unsigned long long* __restrict__ seg_cnt,
                                                       uint64_t seg_cap, uint32_t nseg,
                                                       const uint32_t* __restrict__ offs,
                                                       uint32_t* __restrict__ entries) {
  extern __shared__ uint32_t cur[];
  for (uint32_t b = threadIdx.x; b < nbuckets; b += TH)
    cur[b] = offs[(size_t)b * nblocks + blockIdx.x];
  __syncthreads();
  const PairRange pr = pair_range(pairs, count, chunk, nblocks, seg_cnt, seg_cap, nseg);
  const uint64_t* __restrict__ src = pr.src;
  const size_t base = pr.base, end = pr.end;
  const uint64_t cmask = (1ull << pb) - 1ull;
  const uint32_t rmask = (1u << rb) - 1u;
  for (size_t q0 = base; q0 < end; q0 += 8 * TH) {
    uint64_t k8[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      const size_t q = q0 + (size_t)x * TH + threadIdx.x;
      k8[x] = q < end ? src[q] : ~0ull;
    }
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      if (k8[x] == ~0ull) continue;
      const uint32_t i = (uint32_t)(k8[x] >> pb), j = (uint32_t)(k8[x] & cmask);
      entries[atomicAdd(&cur[i >> rb], 1u)] = ((i & rmask) << pb) | j;
      if (both) entries[atomicAdd(&cur[j >> rb], 1u)] = ((j & rmask) << pb) | i;
    }
  }
}

__device__ __forceinline__ void bucket_range(const uint32_t* __restrict__ offs, uint32_t b,
                                             uint32_t nbuckets, uint32_t nblocks, uint32_t total,
                                             uint32_t& start, uint32_t& cnt) {
  start = offs[(size_t)b * nblocks];
  const uint32_t stop = (b + 1 < nbuckets) ? offs[(size_t)(b + 1) * nblocks] : total;
  cnt = stop - start;
}

// One block per bucket: put the bucket's entries in row order and write
// them out as the bucket's part of col and row_ptr.  The input pairs are
// unique, so every entry is kept, the bucket's start in the entry array is
// its start in col, and the columns of a row are distinct.  The block's
// 1024 threads load the whole bucket into registers at once, count rows
// (LDS histogram) and scatter the entries by row into LDS.  An entry of a
// row of at most kShortRow entries takes its place in the row as the number
// of smaller columns; a longer row is sorted in place by one wave.  Buckets
// larger than cap or with a row longer than kLongRow are listed in
// oversized for the caller.
constexpr uint32_t kLongRow = 1024;
constexpr uint32_t kShortRow = 64;
constexpr uint32_t kMaxLongRows = 512;  // long rows per bucket handled in LDS

// Ascending sort of v[0..len) in LDS by one wave (len <= 1024): a bitonic
// network in its flip form, where every compare-exchange puts the smaller
// key at the lower index, so the missing tail of the power-of-two size acts
// as +infinity and the sort runs in place.
__device__ __forceinline__ void wave_sort_lds(uint32_t* v, uint32_t len, uint32_t lane) {
  uint32_t P = 1;
  while (P < len) P <<= 1;
  for (uint32_t size = 2; size <= P; size <<= 1) {
    const uint32_t half = size >> 1;
    for (uint32_t i = lane; i < (P >> 1); i += 64) {
      const uint32_t blk = i / half, off = i % half;
      const uint32_t a = blk * size + off, b = blk * size + size - 1 - off;
      if (b < len) {
        const uint32_t x = v[a], y = v[b];
        if (y < x) {
          v[a] = y;
          v[b] = x;
        }
      }
    }
    wave_lds_sync();
    for (uint32_t st = half >> 1; st >= 1; st >>= 1) {
      for (uint32_t i = lane; i < (P >> 1); i += 64) {
        const uint32_t a = 2 * st * (i / st) + (i % st), b = a + st;
        if (b < len) {
          const uint32_t x = v[a], y = v[b];
          if (y < x) {
            v[a] = y;
            v[b] = x;
          }
        }
      }
      wave_lds_sync();
    }
  }
}
constexpr int kCsrThreads = 1024;
constexpr int kCsrWaves = kCsrThreads / 64;
constexpr int kCsrItems = kBucketMaxEntries / kCsrThreads;

__device__ __forceinline__ uint32_t csr_block_exclusive_scan(uint32_t v, uint32_t* wsum,
                                                             uint32_t& total) {
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int q = 0; q < kCsrWaves; ++q) {
    const uint32_t x = wsum[q];
    if (q < w) before += x;
    all += x;
  }
  __syncthreads();
  total = all;
  return before + inc - v;
}

__global__ __launch_bounds__(kCsrThreads) void k_bucket_csr(
    const uint32_t* __restrict__ entries, const uint32_t* __restrict__ offs, uint32_t nbuckets,
    uint32_t nblocks, const uint32_t* __restrict__ total_p, uint32_t* __restrict__ oversized,
    uint32_t* __restrict__ n_oversized, uint32_t cap, int pb, int rb, int64_t n, int64_t nnz,
    int64_t* __restrict__ row_ptr, int32_t* __restrict__ col) {
  __shared__ uint32_t s[kBucketMaxEntries];
  __shared__ uint32_t rstart[kBucketMaxRows], rcur[kBucketMaxRows];
  __shared__ uint32_t wsum[kCsrWaves];
  __shared__ uint32_t s_long, s_nlong;
  __shared__ uint32_t s_longrows[kMaxLongRows];
  const uint32_t b = blockIdx.x;
  if (b == 0 && threadIdx.x == 0) row_ptr[n] = nnz;
  uint32_t start, cnt;
  bucket_range(offs, b, nbuckets, nblocks, *total_p, start, cnt);
  if (cnt > cap) {
    if (threadIdx.x == 0) oversized[atomicAdd(n_oversized, 1u)] = b;
    return;
  }
  const uint32_t nrows = 1u << rb;
  const uint32_t cmask = (1u << pb) - 1u;
  uint32_t e_[kCsrItems];
#pragma unroll
  for (int q = 0; q < kCsrItems; ++q) {
    const uint32_t i = threadIdx.x + (uint32_t)q * kCsrThreads;
    e_[q] = i < cnt ? entries[start + i] : 0u;
  }
  for (uint32_t r = threadIdx.x; r < nrows; r += kCsrThreads) rcur[r] = 0u;
  if (threadIdx.x == 0) {
    s_long = 0u;
    s_nlong = 0u;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kCsrItems; ++q)
    if (threadIdx.x + (uint32_t)q * kCsrThreads < cnt) atomicAdd(&rcur[e_[q] >> pb], 1u);
  __syncthreads();
  // row starts: each thread scans a contiguous run of rows
  const uint32_t per = (nrows + kCsrThreads - 1) / kCsrThreads;
  const uint32_t r0 = threadIdx.x * per;
  uint32_t mine = 0;
  for (uint32_t r = r0; r < r0 + per && r < nrows; ++r) {
    mine += rcur[r];
    if (rcur[r] > kLongRow) s_long = 1u;
    if (rcur[r] > kShortRow) {
      const uint32_t q = atomicAdd(&s_nlong, 1u);
      if (q < kMaxLongRows) s_longrows[q] = r;
      else s_long = 1u;  // too many long rows: the caller sorts the bucket
    }
  }
  uint32_t all;
  uint32_t run = csr_block_exclusive_scan(mine, wsum, all);
  for (uint32_t r = r0; r < r0 + per && r < nrows; ++r) {
    rstart[r] = run;
    const int64_t row = ((int64_t)b << rb) + r;
    if (row < n) row_ptr[row] = (int64_t)start + run;
    run += rcur[r];
  }
  __syncthreads();
  if (s_long) {
    if (threadIdx.x == 0) oversized[atomicAdd(n_oversized, 1u)] = b;
    return;
  }
  for (uint32_t r = threadIdx.x; r < nrows; r += kCsrThreads) rcur[r] = rstart[r];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kCsrItems; ++q)
    if (threadIdx.x + (uint32_t)q * kCsrThreads < cnt) s[atomicAdd(&rcur[e_[q] >> pb], 1u)] = e_[q];
  __syncthreads();
  // Short rows: thread t takes the entries at positions t, t + 1024, ... of
  // the row-ordered array, so the lanes of a wave cover a few whole rows and
  // read the same row element at each step (broadcast reads, no bank
  // conflicts).  Each entry's place is the number of smaller columns in its
  // row (the row bits are equal, so whole entries compare as columns).
#pragma unroll
  for (int q = 0; q < kCsrItems; ++q) {
    const uint32_t x = threadIdx.x + (uint32_t)q * kCsrThreads;
    if (x < cnt) {
      const uint32_t e = s[x];
      const uint32_t r = e >> pb;
      const uint32_t lo = rstart[r], hi = rcur[r];
      if (hi - lo <= kShortRow) {
        uint32_t rank = 0, y = lo;
        for (; y + 4 <= hi; y += 4)
          rank += (s[y] < e ? 1u : 0u) + (s[y + 1] < e ? 1u : 0u) + (s[y + 2] < e ? 1u : 0u) +
                  (s[y + 3] < e ? 1u : 0u);
        for (; y < hi; ++y) rank += s[y] < e ? 1u : 0u;
        col[(size_t)start + lo + rank] = (int32_t)(e & cmask);
      }
    }
  }
  // long rows: one wave sorts each in place (the row bits are equal, so the
  // whole entries order as the columns)
  const uint32_t nlong = s_nlong;
  const uint32_t lane = lane_id();
  for (uint32_t q = threadIdx.x >> 6; q < nlong; q += kCsrWaves) {
    const uint32_t r = s_longrows[q];
    const uint32_t lo = rstart[r], len = rcur[r] - lo;
    wave_sort_lds(s + lo, len, lane);
    for (uint32_t x = lane; x < len; x += 64) col[(size_t)start + lo + x] = (int32_t)(s[lo + x] & cmask);
  }
}

// Buckets beyond LDS capacity, all in one global sort.  Bucket ids[q] holds
// entries [start[q], start[q] + cnt[q]) of the entry array (and of col).
__global__ void k_over_extent(const uint32_t* __restrict__ ids, uint32_t nover,
                              const uint32_t* __restrict__ part, uint32_t nblocks,
                              uint32_t nbuckets, size_t np, uint32_t* __restrict__ start,
                              uint32_t* __restrict__ cnt) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nover) return;
  const uint32_t b = ids[q];
  const uint32_t st = part[(size_t)b * nblocks];
  const uint32_t nx = (b + 1 < nbuckets) ? part[(size_t)(b + 1) * nblocks] : part[np];
  start[q] = st;
  cnt[q] = nx - st;
}

// The largest q with off[q] <= i (off ascending, off[0] = 0).
__device__ __forceinline__ uint32_t over_of(const uint32_t* __restrict__ off, uint32_t nover,
                                            uint32_t i) {
  uint32_t lo = 0, hi = nover - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// w[off[q] + e] = q << sh | entry e of oversized bucket q: one sort orders
// every oversized bucket's entries, bucket by bucket.
__global__ void k_over_gather(const uint32_t* __restrict__ entries,
                              const uint32_t* __restrict__ start, const uint32_t* __restrict__ off,
                              uint32_t nover, uint32_t tot, int sh, uint64_t* __restrict__ w) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tot) return;
  const uint32_t q = over_of(off, nover, i);
  w[i] = ((uint64_t)q << sh) | entries[(size_t)start[q] + (i - off[q])];
}

// col and row_ptr of every oversized bucket from the sorted tagged entries.
__global__ void k_over_emit(const uint64_t* __restrict__ keys, uint32_t tot,
                            const uint32_t* __restrict__ ids, const uint32_t* __restrict__ start,
                            const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ off,
                            int pb, int rb, int64_t n, int64_t* __restrict__ row_ptr,
                            int32_t* __restrict__ col) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tot) return;
  const int sh = rb + pb;
  const uint64_t emask = (1ull << sh) - 1ull;
  const uint64_t key = keys[i];
  const uint32_t q = (uint32_t)(key >> sh);
  const uint32_t e = (uint32_t)(key & emask);
  const uint32_t rr = e >> pb;
  const uint32_t local = i - off[q];
  const int64_t base = (int64_t)ids[q] << rb;
  const int64_t at = (int64_t)start[q] + local;
  col[at] = (int32_t)(e & ((1u << pb) - 1u));
  // the first entry of each row sets row_ptr for it and the empty rows before
  const uint32_t from = local == 0 ? 0u : (uint32_t)((keys[i - 1] & emask) >> pb) + 1u;
  for (uint32_t r = from; r <= rr; ++r)
    if (base + r < n) row_ptr[base + r] = at;
  // the bucket's last entry sets the empty rows after it
  if (local + 1 == cnt[q])
    for (uint32_t r = rr + 1; r < (1u << rb); ++r)
      if (base + r < n) row_ptr[base + r] = (int64_t)start[q] + cnt[q];
}

// dst[q] = src[q], zero-extended.
__global__ void k_widen(const uint32_t* __restrict__ src, size_t count, uint64_t* __restrict__ dst) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < count) dst[q] = src[q];
}

// dst[q] = the 4- or 8-byte device scalar at src[q], zero-extended: several
// scalars come back to the host with one copy.
__global__ void k_gather(Gather g, uint64_t* __restrict__ dst) {
  const int q = threadIdx.x;
  if (q >= g.count) return;
  dst[q] = g.bytes[q] == 8 ? *static_cast<const uint64_t*>(g.src[q])
                           : (uint64_t)*static_cast<const uint32_t*>(g.src[q]);
}

// Read-backs into pinned host memory: the values (words of a device buffer,
// or the scalars of a Gather), then -- after every thread's stores are
// visible at system scope -- the sequence number the host waits for.
__global__ __launch_bounds__(kBlock) void k_mailbox(const uint32_t* __restrict__ src,
                                                    uint32_t words, Gather g,
                                                    uint32_t* __restrict__ host,
                                                    uint64_t* __restrict__ host_seq,
                                                    uint64_t seq) {
  if (src) {
    for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) host[i] = src[i];
  } else if (threadIdx.x < (unsigned)g.count) {
    const int q = threadIdx.x;
    const uint64_t v = g.bytes[q] == 8 ? *static_cast<const uint64_t*>(g.src[q])
                                       : (uint64_t)*static_cast<const uint32_t*>(g.src[q]);
    reinterpret_cast<uint64_t*>(host)[q] = v;
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(host_seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Point records for tile loads: the coordinates, then zeros up to rs floats
// (the last two hold the point's signature word, written by the key kernel).
__global__ void k_records(const float* __restrict__ rows, int64_t n, int d, int rs,
                          float* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float* r = rec + (size_t)i * rs;
  for (int l = 0; l < d; ++l) r[l] = rows[(size_t)i * d + l];
  for (int l = d; l < rs; ++l) r[l] = 0.0f;
}

// out[q] = row_ptr[first point of instance q] for q < m, out[m] = row_ptr[npts].
__global__ void k_rowptr_at(const InstDesc* __restrict__ inst, uint32_t m,
                            const int64_t* __restrict__ row_ptr, int64_t npts,
                            int64_t* __restrict__ out) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) out[q] = row_ptr[inst[q].pt_off];
  if (q == m) out[m] = row_ptr[npts];
}

// One thread per batch point (point blocks as in the stage): the point's
// row start in its instance's own row_ptr, relative to the instance.
__global__ __launch_bounds__(kBlock) void k_localize_rows(const InstDesc* __restrict__ inst,
                                                          uint32_t m,
                                                          const int64_t* __restrict__ row_ptr,
                                                          int64_t* const* __restrict__ out_rp) {
  const uint32_t q = block_instance(inst, m, blockIdx.x);
  const int64_t n = inst[q].n;
  const int64_t i = (int64_t)(blockIdx.x - (uint32_t)inst[q].blk_first) * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t off = inst[q].pt_off;
  const int64_t base = row_ptr[off];
  int64_t* rp = out_rp[q];
  rp[i] = row_ptr[off + i] - base;
  if (i == n - 1) rp[n] = row_ptr[off + n] - base;
}

constexpr int kLocalizePer = 16;  // entries per thread of the column copy

// The batch's col copied into the instances' own col arrays, indices made
// local: each block a contiguous run of kLocalizePer * kBlock entries (loads
// and stores coalesced); at[q] is instance q's first entry, at[m] the total.
// Each thread finds the instance of its first entry by bisection and steps
// forward past instance ends (several instances may share a run).
__global__ __launch_bounds__(kBlock) void k_localize_cols(const InstDesc* __restrict__ inst,
                                                          uint32_t m,
                                                          const int64_t* __restrict__ at,
                                                          const int32_t* __restrict__ col,
                                                          int32_t* const* __restrict__ out_col) {
  const int64_t total = at[m];
  const int64_t e0 = (int64_t)blockIdx.x * (kLocalizePer * kBlock) + threadIdx.x;
  if (e0 >= total) return;
  uint32_t lo = 0, hi = m - 1;  // the last q with at[q] <= e0
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (at[mid] <= e0) lo = mid; else hi = mid - 1;
  }
  uint32_t q = lo;
  int64_t q_end = at[q + 1], q_begin = at[q];
  int32_t* dst = out_col[q];
  int32_t off = (int32_t)inst[q].pt_off;
#pragma unroll 4
  for (int j = 0; j < kLocalizePer; ++j) {
    const int64_t e = e0 + (int64_t)j * kBlock;
    if (e >= total) break;
    while (e >= q_end) {
      ++q;
      q_begin = q_end;
      q_end = at[q + 1];
      dst = out_col[q];
      off = (int32_t)inst[q].pt_off;
    }
    dst[e - q_begin] = col[e] - off;
  }
}

inline unsigned grid_for(size_t count, unsigned block = kBlock) {
  size_t g = (count + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

inline unsigned tiles_for(size_t count) { return (unsigned)((count + kTile - 1) / kTile); }

// ---------------------------------------------------------------------------
// Small instances in two launches.  For n <= kTinyPoints (and d <= 8) the
// whole pipeline fits a few workgroups per grid: block (t, part) computes
// every point's cell under grids 0..t (the FP64 formula of k_keys) and
// packs each cell's fields into 32 bits (field widths from the block's own
// minimum and maximum), sorts grid t's keys -- cell and point index -- in
// LDS (counting sort over few cells, else bitonic), tests its slice of the
// pairs of the cells in FP64 in the definition's order, keeps a pair within
// r only if no earlier
// grid's packed cells of the two points are equal, and appends it to one
// pair list.  A second launch turns the list into the CSR lists.
// Anything outside these limits -- wider keys, more pairs than the list
// holds (kTinyPairCap), a row longer than kTinyMaxDeg -- is flagged and the
// caller runs the general pipeline instead.

constexpr int kTinyThreads = 512;
constexpr int kTinyWaves = kTinyThreads / 64;
constexpr int kTinyPer = kTinyPoints / kTinyThreads;

__device__ __forceinline__ uint32_t tiny_block_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int q = 0; q < kTinyWaves; ++q) {
    const uint32_t x = wsum[q];
    if (q < w) before += x;
    all += x;
  }
  __syncthreads();
  total = all;
  return before + inc - v;
}

// The wave's staged pairs (kTinyOut per wave) go to the list in one block
// of slots; every lane of the wave takes part.
constexpr uint32_t kTinyOut = 256;
struct TinyOut {
  uint64_t* buf;
  uint32_t n;
};
__device__ __forceinline__ void tiny_flush(const TinyArgs& A, TinyOut& O, uint32_t lane) {
  wave_lds_sync();
  if (O.n) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(A.count, (unsigned long long)O.n);
    base = lane_value(base, 0);
    for (uint32_t e = lane; e < O.n; e += 64)
      if (base + e < A.cap) A.pairs[base + e] = O.buf[e];
    O.n = 0;
  }
  wave_lds_sync();
}
__device__ __forceinline__ void tiny_append(const TinyArgs& A, TinyOut& O, uint32_t lane,
                                            bool keep, uint64_t val) {
  const uint64_t m = ballot(keep);
  const uint32_t c = (uint32_t)__popcll(m);
  if (!c) return;
  if (O.n + c > kTinyOut) tiny_flush(A, O, lane);
  if (keep) O.buf[O.n + rank_below(m)] = val;
  O.n += c;
}

template <int D>
__global__ __launch_bounds__(kTinyThreads) void k_tiny_grids(const TinyArgs A) {
  __shared__ float sp[kTinyFloats];         // the points, [n][D]
  __shared__ double sT[kTinyTransform];     // R then u of every grid
  __shared__ uint32_t sC[kTinyCells];       // packed cells of grids 0..t, [g][n]
  __shared__ uint32_t skey[kTinyPoints];    // (cell << idx_bits) | point, sorted
  __shared__ union {
    uint32_t hist[kTinyBins];                // the counting sort's bins
    uint64_t out[kTinyWaves][kTinyOut];      // then each wave's staged pairs
  } sU;
  __shared__ int32_t wlo[kTinyWaves][D], whi[kTinyWaves][D];
  __shared__ uint32_t wsum[kTinyWaves];
  __shared__ uint32_t sflag;
  // k parts workgroups: workgroup (t, part) tests slice part of grid t's
  // pairs (every part finds the grid's cells itself)
  const int t = (int)(blockIdx.x / A.parts);
  const uint32_t part = blockIdx.x % A.parts;
  const int n = A.n;
  const uint32_t lane = lane_id();
  const int w = threadIdx.x >> 6;
  if (threadIdx.x == 0) sflag = 0u;
  uint32_t bad = 0u;
  for (int e = (int)threadIdx.x; e < n * D; e += kTinyThreads) {
    const float v = A.pts[e];
    if (!isfinite(v)) bad |= 1u;
    sp[e] = v;
  }
  const int nR = A.k * D * D;
  for (int e = (int)threadIdx.x; e < nR + A.k * D; e += kTinyThreads)
    sT[e] = e < nR ? A.R[e] : A.u[e - nR];
  if (bad) atomicOr(&sflag, bad);
  __syncthreads();
  int idx_bits = 1;
  while ((1 << idx_bits) < n) ++idx_bits;

  // The packed cell of every point under grids 0..t: the fields (the key
  // kernel's FP64 formula) less their minimum over the instance, side by
  // side.  Grid t's cells key the sort; the earlier grids' decide, by one
  // comparison, whether a pair was already some earlier grid's.
  int cell_bits = 0;
  for (int g = 0; g <= t; ++g) {
    const double* Rg = sT + (size_t)g * D * D;
    const double* ug = sT + nR + (size_t)g * D;
    int32_t lo[D], hi[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      lo[j] = INT32_MAX;
      hi[j] = INT32_MIN;
    }
    bad = 0u;
    for (int i = (int)threadIdx.x; i < n; i += kTinyThreads) {
      float p[D];
#pragma unroll
      for (int l = 0; l < D; ++l) p[l] = sp[i * D + l];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double y = cell_y<D>(Rg + (size_t)j * D, p, nullptr, 0, 0, D, A.inv_c, ug[j]);
        const bool ok = fabs(y) < 2147483648.0;
        const int32_t kj = ok ? (int32_t)floor(y) : 0;
        if (!ok) bad |= 2u;
        lo[j] = min(lo[j], kj);
        hi[j] = max(hi[j], kj);
      }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        lo[j] = min(lo[j], __shfl_xor(lo[j], o, 64));
        hi[j] = max(hi[j], __shfl_xor(hi[j], o, 64));
      }
      if (lane == 0) {
        wlo[w][j] = lo[j];
        whi[w][j] = hi[j];
      }
    }
    if (bad) atomicOr(&sflag, bad);
    __syncthreads();
    int shift[D], total = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      lo[j] = wlo[0][j];
      hi[j] = whi[0][j];
#pragma unroll
      for (int q = 1; q < kTinyWaves; ++q) {
        lo[j] = min(lo[j], wlo[q][j]);
        hi[j] = max(hi[j], whi[q][j]);
      }
      int b = 0;
      while (b < 32 && ((int64_t)1 << b) < (int64_t)hi[j] - (int64_t)lo[j] + 1) ++b;
      shift[j] = total;
      total += b;
    }
    uint32_t flag = sflag;
    // grid t's key holds the point index too (and must not match the
    // bitonic sort's padding); the earlier grids' cells only need 32 bits
    if (g == t ? total + idx_bits > 31 : total > 32) flag |= 4u;
    if (flag) {
      if (threadIdx.x == 0) atomicOr(A.err, flag);
      return;  // uniform: every thread read the same flag
    }
    cell_bits = total;
    for (int i = (int)threadIdx.x; i < n; i += kTinyThreads) {
      float p[D];
#pragma unroll
      for (int l = 0; l < D; ++l) p[l] = sp[i * D + l];
      uint32_t cell = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double y = cell_y<D>(Rg + (size_t)j * D, p, nullptr, 0, 0, D, A.inv_c, ug[j]);
        cell |= (uint32_t)((int32_t)floor(y) - lo[j]) << shift[j];
      }
      sC[(size_t)g * n + i] = cell;
    }
    __syncthreads();  // wlo / whi are reused by the next grid
  }
  const uint32_t* cur = sC + (size_t)t * n;

  // Grid t's keys in cell order: a counting sort over the cells when they
  // are few, else a bitonic sort of the whole keys.
  if (cell_bits <= kTinyBinBits) {
    const int nb = 1 << cell_bits;
    for (int c = (int)threadIdx.x; c < nb; c += kTinyThreads) sU.hist[c] = 0u;
    __syncthreads();
    for (int i = (int)threadIdx.x; i < n; i += kTinyThreads) atomicAdd(&sU.hist[cur[i]], 1u);
    __syncthreads();
    constexpr int per = kTinyBins / kTinyThreads;
    uint32_t mine = 0;
#pragma unroll
    for (int e = 0; e < per; ++e) {
      const int c = (int)threadIdx.x * per + e;
      if (c < nb) mine += sU.hist[c];
    }
    uint32_t all;
    uint32_t run = tiny_block_scan(mine, wsum, all);
#pragma unroll
    for (int e = 0; e < per; ++e) {
      const int c = (int)threadIdx.x * per + e;
      if (c < nb) {
        const uint32_t h = sU.hist[c];
        sU.hist[c] = run;
        run += h;
      }
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < n; i += kTinyThreads) {
      const uint32_t c = cur[i];
      skey[atomicAdd(&sU.hist[c], 1u)] = (c << idx_bits) | (uint32_t)i;
    }
    __syncthreads();
  } else {
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (int i = (int)threadIdx.x; i < np2; i += kTinyThreads)
      skey[i] = i < n ? (cur[i] << idx_bits) | (uint32_t)i : 0xFFFFFFFFu;
    __syncthreads();
    for (int size = 2; size <= np2; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int x = (int)threadIdx.x; x < np2 / 2; x += kTinyThreads) {
          const int a = 2 * stride * (x / stride) + (x % stride), b = a + stride;
          const bool up = (a & size) == 0;
          const uint32_t ka = skey[a], kb = skey[b];
          if ((ka > kb) == up) {
            skey[a] = kb;
            skey[b] = ka;
          }
        }
        __syncthreads();
      }
    }
  }

  // Pairs per sorted position: c_p = the positions after p in p's cell
  // (the cell's end: the counting sort's cursor, else found by bisection);
  // their exclusive prefix goes where grid t's cells were (no longer read).
  const uint32_t imask = (1u << idx_bits) - 1u;
  uint32_t* pre = sC + (size_t)t * n;
  uint32_t cnt[kTinyPer];
  uint32_t mine = 0, cells = 0;
#pragma unroll
  for (int e = 0; e < kTinyPer; ++e) {
    const int p = (int)threadIdx.x * kTinyPer + e;
    cnt[e] = 0;
    if (p < n) {
      const uint32_t cp = skey[p] >> idx_bits;
      int lo = p + 1, hi = n;  // the first position past p's cell
      if (cell_bits <= kTinyBinBits) {
        lo = (int)sU.hist[cp];
      } else {
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if ((skey[mid] >> idx_bits) == cp) lo = mid + 1; else hi = mid;
        }
      }
      cnt[e] = (uint32_t)(lo - p - 1);
      if (cnt[e] && (p == 0 || (skey[p - 1] >> idx_bits) != cp)) ++cells;
      mine += cnt[e];
    }
  }
  uint32_t T;
  uint32_t run = tiny_block_scan(mine, wsum, T);  // barriers: every c_p is read
#pragma unroll
  for (int e = 0; e < kTinyPer; ++e) {
    const int p = (int)threadIdx.x * kTinyPer + e;
    if (p < n) {
      pre[p] = run;
      run += cnt[e];
    }
  }
  __syncthreads();

  // The workgroup's slice [s0, s1) of the grid's T pairs (p, q), p < q in
  // one cell, in position order, in one contiguous run per thread: its
  // first p by bisection of pre, then q steps to the cell's end and p on to
  // the next position with pairs.  The order of a cell's points may differ
  // between the parts (the counting sort's scatter is atomic), so slices
  // hold whole cells: a nominal bound T * part / parts moves down to the
  // first pair of the cell that holds it, a value every part finds alike.
  auto cell_bound = [&](uint32_t part_i) -> uint32_t {
    const uint32_t s = (uint32_t)((uint64_t)T * part_i / A.parts);
    if (s >= T) return T;
    int lo = 0, hi = n - 1;  // the position whose pairs hold index s
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= s) lo = mid; else hi = mid - 1;
    }
    const uint32_t c = skey[lo] >> idx_bits;
    int a0 = 0, a1 = lo;  // the first position of that cell
    while (a0 < a1) {
      const int mid = (a0 + a1) >> 1;
      if ((skey[mid] >> idx_bits) < c) a0 = mid + 1; else a1 = mid;
    }
    return pre[a0];
  };
  const uint32_t s0 = cell_bound(part);
  const uint32_t s1 = cell_bound(part + 1);
  const uint32_t chunk = (s1 - s0 + kTinyThreads - 1) / kTinyThreads;
  uint32_t e = s0 + threadIdx.x * chunk;
  const uint32_t e_end = min(s1, e + chunk);
  int p = 0, q = 0;
  uint32_t pend = 0;  // pre of the position after p
  uint32_t a = 0;
  float pa[D];
  if (e < e_end) {
    int lo = 0, hi = n - 1;  // the last position with pre <= e
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= e) lo = mid; else hi = mid - 1;
    }
    p = lo;
    q = p + 1 + (int)(e - pre[p]);
    pend = p + 1 < n ? pre[p + 1] : T;
    a = skey[p] & imask;
#pragma unroll
    for (int l = 0; l < D; ++l) pa[l] = sp[a * D + l];
  }
  TinyOut O{sU.out[w], 0u};
  // sU.hist was last read before the prefix scan's barriers
  for (uint32_t round = 0; round < chunk; ++round, ++e) {
    bool keep = false;
    uint64_t val = 0;
    if (e < e_end) {
      if (e == pend) {  // on to the next position that has pairs
        do {
          ++p;
          pend = p + 1 < n ? pre[p + 1] : T;
        } while (pend == pre[p]);
        q = p + 1;
        a = skey[p] & imask;
#pragma unroll
        for (int l = 0; l < D; ++l) pa[l] = sp[a * D + l];
      }
      const uint32_t b = skey[q] & imask;
      double s2 = 0.0;
#pragma unroll
      for (int l = 0; l < D; ++l) {
        const double dl = (double)pa[l] - (double)sp[b * D + l];
        s2 = s2 + dl * dl;
      }
      keep = s2 <= A.r2;
      // first owner: no earlier grid with both points in one cell
      for (int g = 0; keep && g < t; ++g)
        if (sC[(size_t)g * n + a] == sC[(size_t)g * n + b]) keep = false;
      val = ((uint64_t)min(a, b) << 32) | (uint64_t)max(a, b);
      ++q;
    }
    tiny_append(A, O, lane, keep, val);
  }
  tiny_flush(A, O, lane);
  // the grid's cells and tests (T), counted by its first part
  if (part == 0) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cells += __shfl_xor(cells, o, 64);
    if (lane == 0 && cells) atomicAdd(A.count + 2, (unsigned long long)cells);
    if (threadIdx.x == 0 && T) atomicAdd(A.count + 1, (unsigned long long)T);
  }
}

// The pair list to CSR lists, the rows split over the workgroups
// (kTinyThreads rows each): every workgroup counts every row's degree and
// takes the offsets of all of them, places the entries of its own rows --
// in LDS when they fit, else in A.stage -- and writes each at its rank
// within its row (rows of at most kTinyMaxDeg entries).  count[3] receives
// the entries written.
__global__ __launch_bounds__(kTinyThreads) void k_tiny_lists(const TinyArgs A) {
  __shared__ uint32_t cur[kTinyPoints];
  __shared__ int32_t scol[kTinyListLds];
  __shared__ uint32_t wsum[kTinyWaves];
  __shared__ uint32_t smax, sbase, send;
  constexpr int kB = 8;  // pairs in flight per thread
  const uint64_t P = A.count[0];
  if (P > A.cap || *A.err) return;  // uniform: the caller reruns or fails
  const int n = A.n;
  const uint32_t r0 = blockIdx.x * kTinyThreads, r1 = min((uint32_t)n, r0 + kTinyThreads);
  for (int i = (int)threadIdx.x; i < n; i += kTinyThreads) cur[i] = 0u;
  if (threadIdx.x == 0) smax = 0u;
  __syncthreads();
  for (uint32_t base = 0; base < (uint32_t)P; base += kB * kTinyThreads) {
    uint64_t v[kB];
#pragma unroll
    for (int e = 0; e < kB; ++e) {
      const uint32_t x = base + e * kTinyThreads + threadIdx.x;
      v[e] = x < P ? A.pairs[x] : ~0ull;
    }
#pragma unroll
    for (int e = 0; e < kB; ++e) {
      if (v[e] == ~0ull) continue;
      atomicAdd(&cur[(uint32_t)(v[e] >> 32)], 1u);
      if (!A.upper) atomicAdd(&cur[(uint32_t)v[e]], 1u);
    }
  }
  __syncthreads();
  // row offsets: thread t takes the rows [t kTinyPer, (t + 1) kTinyPer);
  // cur becomes the placement cursor of the workgroup's rows and the end
  // of every other row (so a row's start is always its predecessor's cur)
  uint32_t dg[kTinyPer];
  uint32_t mine = 0, mx = 0;
#pragma unroll
  for (int e = 0; e < kTinyPer; ++e) {
    const int i = (int)threadIdx.x * kTinyPer + e;
    dg[e] = i < n ? cur[i] : 0u;
    mine += dg[e];
    mx = max(mx, dg[e]);
  }
  atomicMax(&smax, mx);
  uint32_t all;
  uint32_t run = tiny_block_scan(mine, wsum, all);
  if (smax > kTinyMaxDeg) {
    if (threadIdx.x == 0) atomicOr(A.err, 8u);
    return;  // uniform after the scan's barriers
  }
#pragma unroll
  for (int e = 0; e < kTinyPer; ++e) {
    const uint32_t i = threadIdx.x * kTinyPer + e;
    if (i < (uint32_t)n) {
      const bool own = i >= r0 && i < r1;
      if (own) A.row_ptr[i] = (int64_t)run;
      cur[i] = own ? run : run + dg[e];
      if (i == r0) sbase = run;
      if (i + 1 == r1) send = run + dg[e];
    }
    run += dg[e];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    A.row_ptr[n] = (int64_t)all;
    A.count[3] = all;
  }
  __syncthreads();
  const uint32_t base = sbase;
  const bool in_lds = send - base <= (uint32_t)kTinyListLds;
  // entry at list position x: scol[x - base] or A.stage[x]
  int32_t* stage = in_lds ? scol : A.stage;
  const uint32_t off = in_lds ? base : 0u;
  for (uint32_t b0 = 0; b0 < (uint32_t)P; b0 += kB * kTinyThreads) {
    uint64_t v[kB];
#pragma unroll
    for (int e = 0; e < kB; ++e) {
      const uint32_t x = b0 + e * kTinyThreads + threadIdx.x;
      v[e] = x < P ? A.pairs[x] : ~0ull;
    }
#pragma unroll
    for (int e = 0; e < kB; ++e) {
      if (v[e] == ~0ull) continue;
      const uint32_t a = (uint32_t)(v[e] >> 32), b = (uint32_t)v[e];
      if (a >= r0 && a < r1) stage[atomicAdd(&cur[a], 1u) - off] = (int32_t)b;
      if (!A.upper && b >= r0 && b < r1) stage[atomicAdd(&cur[b], 1u) - off] = (int32_t)a;
    }
  }
  // the workgroup's own stores to A.stage are visible after the barrier
  __threadfence_block();
  __syncthreads();
  // A row's entries are distinct, so each one's rank within the row is its
  // place: kR entries at a time are held in registers and compared with
  // every entry of the row, read kR at a time (INT32_MAX past the row's
  // end counts below none).  One row per thread.
  constexpr int kR = 16;
  const uint32_t i = r0 + threadIdx.x;
  if (i >= r1) return;
  const uint32_t s = i ? cur[i - 1] : 0u, len = cur[i] - s;
  const int32_t* row = stage + (s - off);
  for (uint32_t x0 = 0; x0 < len; x0 += kR) {
    int32_t v[kR];
    uint32_t rank[kR];
#pragma unroll
    for (int x = 0; x < kR; ++x) {
      v[x] = x0 + x < len ? row[x0 + x] : INT32_MAX;
      rank[x] = 0;
    }
    for (uint32_t y0 = 0; y0 < len; y0 += kR) {
      int32_t wv[kR];
#pragma unroll
      for (int y = 0; y < kR; ++y) wv[y] = y0 + y < len ? row[y0 + y] : INT32_MAX;
#pragma unroll
      for (int y = 0; y < kR; ++y)
#pragma unroll
        for (int x = 0; x < kR; ++x) rank[x] += wv[y] < v[x] ? 1u : 0u;
    }
#pragma unroll
    for (int x = 0; x < kR; ++x)
      if (x0 + x < len) A.col[s + rank[x]] = v[x];
  }
}

}  // namespace


// ===========================================================================
// launchers

void launch_fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t s) {
  if (!count) return;
  size_t g = (count + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3((unsigned)g), dim3(kBlock), 0, s, p, v, count);
}

void launch_fill_u64(uint64_t* p, uint64_t v, size_t count, hipStream_t s) {
  if (!count) return;
  size_t g = (count + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_fill<uint64_t>, dim3((unsigned)g), dim3(kBlock), 0, s, p, v, count);
}

void launch_stage(const InstDesc* inst, uint32_t m, uint32_t nblocks, int d, int64_t npts,
                  float* soa, float* aos, uint32_t* bad, uint32_t* bbox, uint32_t* part,
                  float* rec, int rs, hipStream_t s, uint64_t* zero64, uint32_t nzero,
                  bool cleared) {
  const uint32_t nbox = m * 2u * (uint32_t)d;
  if (!cleared)
    hipLaunchKernelGGL(k_stage_init, dim3(grid_for(std::max(nbox, nzero))), dim3(kBlock), 0, s,
                       bbox, nbox, bad, zero64, nzero);
  if (!nblocks) return;
#define RTG_STAGE(DD)                                                                         \
  hipLaunchKernelGGL(k_stage_d<DD>, dim3(nblocks), dim3(kBlock), 0, s, inst, m, npts, soa, aos, \
                     bad, part, rec)
  // records are made for d <= 6 only, rs = (d + 5) & ~3 as k_stage_d assumes
  switch (d) {
    case 1: RTG_STAGE(1); break;
    case 2: RTG_STAGE(2); break;
    case 3: RTG_STAGE(3); break;
    case 4: RTG_STAGE(4); break;
    case 5: RTG_STAGE(5); break;
    case 6: RTG_STAGE(6); break;
    case 7: RTG_STAGE(7); break;
    case 8: RTG_STAGE(8); break;
    case 9: RTG_STAGE(9); break;
    case 10: RTG_STAGE(10); break;
    case 11: RTG_STAGE(11); break;
    case 12: RTG_STAGE(12); break;
    case 13: RTG_STAGE(13); break;
    case 14: RTG_STAGE(14); break;
    case 15: RTG_STAGE(15); break;
    case 16: RTG_STAGE(16); break;
    default:
      hipLaunchKernelGGL(k_stage, dim3(nblocks), dim3(kBlock), 0, s, inst, m, d, npts, soa, aos,
                         bad, part, rec, rs);
  }
#undef RTG_STAGE
  // blocks per instance: about 256 per-block boxes each (four per lane), at
  // most kBboxBlocks
  uint32_t gy = (uint32_t)std::min<uint64_t>(kBboxBlocks, (nblocks / m + 255) / 256);
  if (gy < 1) gy = 1;
  hipLaunchKernelGGL(k_bbox_reduce, dim3(m, gy), dim3(kBlock), 0, s, inst, d, part, bbox);
}

template <int D>
static void keys_dispatch(const KeysArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_keys<D>, dim3(a.nblocks), dim3(kBlock), 0, s, a.inst, a.m, a.d, a.npts,
                     a.soa, a.sa, a.sb, a.segs, a.R, a.u, a.klo, a.layout, a.keys, a.vals, a.err,
                     a.sig, a.sig_stride, a.sig_b, a.sig_gpw, a.idx_bits, a.sig_fresh);
}

void launch_keys(const KeysArgs& a, hipStream_t s) {
  if (!a.nblocks) return;
  switch (a.d) {
    case 1: keys_dispatch<1>(a, s); break;
    case 2: keys_dispatch<2>(a, s); break;
    case 3: keys_dispatch<3>(a, s); break;
    case 4: keys_dispatch<4>(a, s); break;
    case 5: keys_dispatch<5>(a, s); break;
    case 6: keys_dispatch<6>(a, s); break;
    case 7: keys_dispatch<7>(a, s); break;
    case 8: keys_dispatch<8>(a, s); break;
    case 9: keys_dispatch<9>(a, s); break;
    case 10: keys_dispatch<10>(a, s); break;
    case 11: keys_dispatch<11>(a, s); break;
    case 12: keys_dispatch<12>(a, s); break;
    case 13: keys_dispatch<13>(a, s); break;
    case 14: keys_dispatch<14>(a, s); break;
    case 15: keys_dispatch<15>(a, s); break;
    case 16: keys_dispatch<16>(a, s); break;
    default: keys_dispatch<0>(a, s);
  }
}

template <int D>
static void coords_dispatch(const float* soa, int64_t n, int d, const double* R, const double* u,
                            double inv_c, int64_t* kappa, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_coords<D>, dim3(grid_for((size_t)n)), dim3(kBlock), 0, s, soa, n, d, R,
                     u, inv_c, kappa, err);
}

void launch_cell_coords(const float* soa, int64_t n, int d, const double* R, const double* u,
                        double inv_c, int64_t* kappa, uint32_t* err, hipStream_t s) {
  if (n <= 0) return;
#define RTG_COORDS_CASE(DV) \
  case DV: coords_dispatch<DV>(soa, n, d, R, u, inv_c, kappa, err, s); break;
  switch (d) {
    RTG_COORDS_CASE(1) RTG_COORDS_CASE(2) RTG_COORDS_CASE(3) RTG_COORDS_CASE(4)
    RTG_COORDS_CASE(5) RTG_COORDS_CASE(6) RTG_COORDS_CASE(7) RTG_COORDS_CASE(8)
    RTG_COORDS_CASE(9) RTG_COORDS_CASE(10) RTG_COORDS_CASE(11) RTG_COORDS_CASE(12)
    RTG_COORDS_CASE(13) RTG_COORDS_CASE(14) RTG_COORDS_CASE(15) RTG_COORDS_CASE(16)
    default: coords_dispatch<0>(soa, n, d, R, u, inv_c, kappa, err, s);
  }
#undef RTG_COORDS_CASE
}

size_t scan_scratch_elems(size_t count) {
  size_t total = 0;
  while (count > (size_t)kScanTile) {
    count = (count + kScanTile - 1) / kScanTile;
    total += count;
  }
  return total + 1;
}

template <typename T>
static void scan_rec(const T* in, T* out, size_t count, T* total, T* scratch, hipStream_t s,
                     const uint32_t* dcount = nullptr) {
  if (count == 0) {
    if (total) hipLaunchKernelGGL(k_fill<T>, dim3(1), dim3(64), 0, s, total, (T)0, (size_t)1);
    return;
  }
  if (count <= (size_t)kScanTile) {
    hipLaunchKernelGGL(k_scan_apply<T>, dim3(1), dim3(kBlock), 0, s, in, out, count,
                       (const T*)nullptr, total, dcount);
    return;
  }
  const size_t nb = (count + kScanTile - 1) / kScanTile;
  T* sums = scratch;
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)nb), dim3(kBlock), 0, s, in, count, sums,
                     dcount);
  if (nb <= (size_t)kFusedScanSums) {
    // each block adds up the sums before it: two launches instead of three
    hipLaunchKernelGGL((k_scan_apply<T, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, in, out,
                       count, (const T*)sums, total, dcount);
    return;
  }
  scan_rec<T>(sums, sums, nb, (T*)nullptr, scratch + nb, s);
  hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, count,
                     (const T*)sums, total, dcount);
}

void scan_exclusive_u32(const uint32_t* in, uint32_t* out, size_t count, uint32_t* total,
                        uint32_t* scratch, hipStream_t s, const uint32_t* dcount) {
  scan_rec<uint32_t>(in, out, count, total, scratch, s, dcount);
}

void scan_exclusive_u64(const uint64_t* in, uint64_t* out, size_t count, uint64_t* total,
                        uint64_t* scratch, hipStream_t s, const uint32_t* dcount) {
  scan_rec<uint64_t>(in, out, count, total, scratch, s, dcount);
}

size_t radix_scratch_bytes(size_t count, int begin_bit, int end_bit, size_t extra_tiles) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t ntiles = tiles_for(count) + extra_tiles;
  const int npass = std::max(1, (end_bit - begin_bit + kRadixBits - 1) / kRadixBits);
  const size_t nbh = (count + (size_t)kHistBlockTiles * kTile - 1) / ((size_t)kHistBlockTiles * kTile);
  const size_t onesweep = up(nbh * npass * 256 * 4) + up((size_t)npass * 256 * 8) +
                          up(ntiles * 256 * 8) + up((size_t)npass * 4);
  const size_t h = (size_t)256 * ntiles;
  const size_t rts = up(4 * (h + scan_scratch_elems(h)));
  return std::max(onesweep, rts) + 256;
}

int radix_sort(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
               size_t count, int begin_bit, int end_bit, void* scratch, uint32_t* err,
               hipStream_t s, const LaunchTimer* timer, int kid_hist, int kid_scatter, int algo,
               const SortTile* tiles, uint32_t ntiles_table) {
  const LaunchTimer none;
  const LaunchTimer& tm = timer ? *timer : none;
  const double elem = vals ? 12.0 : 8.0;
  if (count <= 1 || end_bit <= begin_bit) return 0;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const unsigned ntiles = tiles_for(count);
  char* base = static_cast<char*>(scratch);
  uint64_t *kin = keys, *kout = keys_alt;
  uint32_t *vin = vals, *vout = vals_alt;
  int where = 0;
  if (algo == kSortOnesweep) {
    const int npass = (end_bit - begin_bit + kRadixBits - 1) / kRadixBits;
    const size_t nbh =
        (count + (size_t)kHistBlockTiles * kTile - 1) / ((size_t)kHistBlockTiles * kTile);
    uint32_t* part = reinterpret_cast<uint32_t*>(base);
    base += up(nbh * npass * 256 * 4);
    uint64_t* digit_off = reinterpret_cast<uint64_t*>(base);
    base += up((size_t)npass * 256 * 8);
    unsigned long long* status = reinterpret_cast<unsigned long long*>(base);
    base += up((size_t)ntiles * 256 * 8);
    unsigned int* counters = reinterpret_cast<unsigned int*>(base);
    tm.on_begin(kid_hist);
    hipLaunchKernelGGL(k_hist_all, dim3((unsigned)nbh), dim3(kBlock), 0, s, kin, count, begin_bit,
                       end_bit, part);
    hipLaunchKernelGGL(k_hist_scan, dim3(npass), dim3(kBlock), 0, s, part, (uint32_t)nbh, npass,
                       digit_off);
    tm.on_end(kid_hist, 8.0 * (double)count);
    hipLaunchKernelGGL(k_fill<unsigned int>, dim3(1), dim3(64), 0, s, counters, 0u, (size_t)npass);
    for (int p = 0; p < npass; ++p) {
      const int b = begin_bit + p * kRadixBits;
      const int nbits = std::min(kRadixBits, end_bit - b);
      launch_fill_u64(reinterpret_cast<uint64_t*>(status), 0ull, (size_t)ntiles * 256, s);
      tm.on_begin(kid_scatter);
      if (vals)
        hipLaunchKernelGGL(k_onesweep<true>, dim3(ntiles), dim3(kBlock), 0, s, kin, vin, kout, vout,
                           count, b, nbits, digit_off + (size_t)p * 256, status, counters + p, err);
      else
        hipLaunchKernelGGL(k_onesweep<false>, dim3(ntiles), dim3(kBlock), 0, s, kin,
                           (const uint32_t*)nullptr, kout, (uint32_t*)nullptr, count, b, nbits,
                           digit_off + (size_t)p * 256, status, counters + p, err);
      tm.on_end(kid_scatter, 2.0 * elem * (double)count);
      std::swap(kin, kout);
      std::swap(vin, vout);
      where ^= 1;
    }
    return where;
  }
  const unsigned nt = tiles ? ntiles_table : ntiles;
  if (nt == 0) return 0;
  uint32_t* hist = reinterpret_cast<uint32_t*>(base);
  uint32_t* sscr = hist + (size_t)256 * nt;
  for (int b = begin_bit; b < end_bit; b += kRadixBits) {
    const int nbits = (end_bit - b) < kRadixBits ? (end_bit - b) : kRadixBits;
    tm.on_begin(kid_hist);
    hipLaunchKernelGGL(k_radix_hist, dim3(nt), dim3(kBlock), 0, s, kin, count, b, nbits, hist, nt,
                       tiles);
    tm.on_end(kid_hist, 8.0 * (double)count);
    scan_rec<uint32_t>(hist, hist, (size_t)256 * nt, (uint32_t*)nullptr, sscr, s);
    tm.on_begin(kid_scatter);
    if (vals)
      hipLaunchKernelGGL(k_radix_scatter<true>, dim3(nt), dim3(kBlock), 0, s, kin, vin, kout,
                         vout, count, b, nbits, hist, nt, tiles);
    else
      hipLaunchKernelGGL(k_radix_scatter<false>, dim3(nt), dim3(kBlock), 0, s, kin,
                         (const uint32_t*)nullptr, kout, (uint32_t*)nullptr, count, b, nbits, hist,
                         nt, tiles);
    tm.on_end(kid_scatter, 2.0 * elem * (double)count);
    std::swap(kin, kout);
    std::swap(vin, vout);
    where ^= 1;
  }
  return where;
}

size_t run_mask_words(size_t count) { return 2 * ((count + 63) / 64); }

void launch_run_count(const uint64_t* keys, size_t count, int shift, uint32_t* head_cnt,
                      uint32_t* tail_cnt, uint64_t* masks, hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_run_count, dim3(tiles_for(count)), dim3(kBlock), 0, s, keys, count, shift,
                     head_cnt, tail_cnt, masks);
}

void launch_run_write(const uint64_t* masks, size_t count, const uint32_t* head_off,
                      const uint32_t* tail_off, uint32_t* start, uint32_t* end, uint32_t* tot,
                      unsigned long long* zero, hipStream_t s) {
  if (!count) return;
  if (tot)
    hipLaunchKernelGGL(k_run_write<true>, dim3(tiles_for(count)), dim3(kBlock), 0, s, masks, count,
                       head_off, tail_off, start, end, tot, zero);
  else
    hipLaunchKernelGGL(k_run_write<false>, dim3(tiles_for(count)), dim3(kBlock), 0, s, masks,
                       count, head_off, tail_off, start, end, (uint32_t*)nullptr,
                       (unsigned long long*)nullptr);
}

// Grid of the cell kernels: one thread per cell up to 2048 blocks, then
// every thread takes more (with a device count the host knows only a bound).
static unsigned cell_grid(uint32_t ncells) {
  return (unsigned)std::min<size_t>(grid_for(ncells), 2048);
}

void launch_cell_work(const uint32_t* start, const uint32_t* end, uint32_t ncells,
                      const uint32_t* dcells, uint32_t cell_unit_tiles, uint32_t* units,
                      uint64_t* tests, unsigned long long* members, hipStream_t s) {
  if (!ncells) return;
  hipLaunchKernelGGL(k_cell_work, dim3(cell_grid(ncells)), dim3(kBlock), 0, s, start, end, ncells,
                     dcells, cell_unit_tiles, units, tests, members);
}

bool launch_cell_work_scanned(const uint32_t* start, const uint32_t* end, uint32_t ncells,
                              const uint32_t* dcells, uint32_t cell_unit_tiles, uint32_t* units,
                              uint64_t* tests, unsigned long long* members, uint32_t* usums,
                              uint32_t* utotal, uint64_t* tsums, uint64_t* ttotal, hipStream_t s) {
  const size_t nb = ((size_t)ncells + kScanTile - 1) / kScanTile;
  if (!ncells || nb > (size_t)kFusedScanSums) return false;
  hipLaunchKernelGGL(k_cell_work_tiles, dim3((unsigned)nb), dim3(kBlock), 0, s, start, end, ncells,
                     dcells, cell_unit_tiles, units, tests, members, usums, tsums);
  hipLaunchKernelGGL((k_scan_apply<uint32_t, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, units,
                     units, (size_t)ncells, (const uint32_t*)usums, utotal, dcells);
  hipLaunchKernelGGL((k_scan_apply<uint64_t, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, tests,
                     tests, (size_t)ncells, (const uint64_t*)tsums, ttotal, dcells);
  return true;
}

void launch_unit_fill(const uint32_t* start, const uint32_t* end, const uint32_t* unit_off,
                      uint32_t ncells, const uint32_t* dcells, uint32_t cell_unit_tiles,
                      const uint64_t* skeys, int seg_shift, int sa, const SegDesc* segs,
                      UnitDesc* desc, uint64_t* work, hipStream_t s) {
  if (!ncells) return;
  hipLaunchKernelGGL(k_unit_fill, dim3(cell_grid(ncells)), dim3(kBlock), 0, s, start, end,
                     unit_off, ncells, dcells, cell_unit_tiles, skeys, seg_shift, sa, segs, desc,
                     work);
}

uint32_t pair_waves(const PairsArgs& a) {
  uint64_t blocks = ((uint64_t)a.total_units + kWaves - 1) / kWaves;
  const uint64_t max_blocks = a.max_blocks ? a.max_blocks : 256ull * 8ull;
  if (blocks > max_blocks) blocks = max_blocks;
  if (blocks < 1) blocks = 1;
  return (uint32_t)blocks * kWaves;
}

void launch_wave_ranges(const uint64_t* work_off, uint32_t nunits, const uint64_t* total,
                        uint32_t nwaves, uint32_t* first, hipStream_t s) {
  hipLaunchKernelGGL(k_wave_ranges, dim3(grid_for((size_t)nwaves + 1)), dim3(kBlock), 0, s,
                     work_off, nunits, total, nwaves, first);
}

void launch_gather_units(const PairsArgs& a, const uint64_t* sig, float* spts, uint64_t* ssig,
                         hipStream_t s) {
  if (!a.total_units) return;
  const unsigned blocks = (unsigned)(((uint64_t)a.total_units + kWaves - 1) / kWaves);
#define RTG_GATHER(DD) \
  hipLaunchKernelGGL(k_gather_units<DD>, dim3(blocks), dim3(kBlock), 0, s, a, sig, spts, ssig)
  switch (a.d) {
    case 1: RTG_GATHER(1); break;
    case 2: RTG_GATHER(2); break;
    case 3: RTG_GATHER(3); break;
    case 4: RTG_GATHER(4); break;
    case 5: RTG_GATHER(5); break;
    case 6: RTG_GATHER(6); break;
    case 7: RTG_GATHER(7); break;
    case 8: RTG_GATHER(8); break;
    case 9: RTG_GATHER(9); break;
    case 10: RTG_GATHER(10); break;
    case 11: RTG_GATHER(11); break;
    case 12: RTG_GATHER(12); break;
    case 13: RTG_GATHER(13); break;
    case 14: RTG_GATHER(14); break;
    case 15: RTG_GATHER(15); break;
    case 16: RTG_GATHER(16); break;
    default: RTG_GATHER(0); break;
  }
#undef RTG_GATHER
}

void launch_query_keys(const QueryArgs& a, hipStream_t s) {
  if (a.m <= 0) return;
  const unsigned blocks = (unsigned)((a.m + kBlock - 1) / kBlock);
#define RTG_QK(DD) hipLaunchKernelGGL(k_query_keys<DD>, dim3(blocks), dim3(kBlock), 0, s, a)
  switch (a.d) {
    case 1: RTG_QK(1); break;
    case 2: RTG_QK(2); break;
    case 3: RTG_QK(3); break;
    case 4: RTG_QK(4); break;
    case 5: RTG_QK(5); break;
    case 6: RTG_QK(6); break;
    case 7: RTG_QK(7); break;
    case 8: RTG_QK(8); break;
    case 9: RTG_QK(9); break;
    case 10: RTG_QK(10); break;
    case 11: RTG_QK(11); break;
    case 12: RTG_QK(12); break;
    case 16: RTG_QK(16); break;
    default: RTG_QK(0); break;
  }
#undef RTG_QK
}

void launch_seg_compact(const uint64_t* src, uint64_t seg_cap, const unsigned long long* cnt,
                        uint32_t nseg, uint64_t max_count, uint64_t* dst, hipStream_t s) {
  if (nseg == 0 || max_count == 0) return;
  uint64_t bx = (max_count + kBlock * 4 - 1) / (kBlock * 4);
  if (bx > 512) bx = 512;
  hipLaunchKernelGGL(k_seg_compact, dim3((unsigned)bx, nseg), dim3(kBlock), 0, s, src, seg_cap,
                     cnt, dst);
}

static unsigned compact_blocks(uint64_t count) {
  const uint64_t tile = (uint64_t)kBlock * kCompactPer;
  const uint64_t blocks = (count + tile - 1) / tile;
  return (unsigned)(blocks > 4096 ? 4096 : blocks);
}

void launch_mr_filter(const MrFilterArgs& a, hipStream_t s) {
  if (a.count == 0) return;
  hipLaunchKernelGGL(k_mr_filter, dim3(compact_blocks(a.count)), dim3(kBlock), 0, s, a);
}

void launch_bitmap_unique(const BitmapArgs& a, hipStream_t s) {
  if (a.count == 0) return;
  hipLaunchKernelGGL(k_bitmap_unique, dim3(compact_blocks(a.count)), dim3(kBlock), 0, s, a);
}

void launch_query_pairs(const QueryArgs& a, hipStream_t s) {
  if (a.m <= 0 || a.n <= 0) return;
  uint64_t blocks = ((uint64_t)a.m + kWaves - 1) / kWaves;
  if (blocks > 4096) blocks = 4096;
#define RTG_QP(DD) hipLaunchKernelGGL(k_query_pairs<DD>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a)
  switch (a.d) {
    case 1: RTG_QP(1); break;
    case 2: RTG_QP(2); break;
    case 3: RTG_QP(3); break;
    case 4: RTG_QP(4); break;
    case 5: RTG_QP(5); break;
    case 6: RTG_QP(6); break;
    case 7: RTG_QP(7); break;
    case 8: RTG_QP(8); break;
    case 9: RTG_QP(9); break;
    case 10: RTG_QP(10); break;
    case 11: RTG_QP(11); break;
    case 12: RTG_QP(12); break;
    case 16: RTG_QP(16); break;
    default: RTG_QP(0); break;
  }
#undef RTG_QP
}

template <int D>
static void pairs_dispatch(const PairsArgs& a, hipStream_t s) {
  // 256 CUs, several resident blocks each (the grid wave_first was made for)
  const uint64_t blocks = pair_waves(a) / kWaves;
  if constexpr (D <= 16) {
    if (a.gram && a.d == D) {
      hipLaunchKernelGGL((k_cell_pairs_gram<D>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
      return;
    }
  }
  hipLaunchKernelGGL((k_cell_pairs<D>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
}

void launch_tiny(const TinyArgs& a, int d, int k, hipStream_t s) {
#define RTG_TINY(DD) \
  hipLaunchKernelGGL(k_tiny_grids<DD>, dim3(k * a.parts), dim3(kTinyThreads), 0, s, a)
  switch (d) {
    case 1: RTG_TINY(1); break;
    case 2: RTG_TINY(2); break;
    case 3: RTG_TINY(3); break;
    case 4: RTG_TINY(4); break;
    case 5: RTG_TINY(5); break;
    case 6: RTG_TINY(6); break;
    case 7: RTG_TINY(7); break;
    case 8: RTG_TINY(8); break;
    default: return;
  }
#undef RTG_TINY
  hipLaunchKernelGGL(k_tiny_lists, dim3((a.n + kTinyThreads - 1) / kTinyThreads),
                     dim3(kTinyThreads), 0, s, a);
}

void launch_cell_pairs(const PairsArgs& a, hipStream_t s) {
  if (!a.total_units) return;
  const int d = a.d;
#define RTG_PAIRS_ARGS a, s
  // Instantiations for d <= 16 exactly; larger d run the next wider one with
  // zero padding, which adds exact zeros to both sums.
  switch (d) {
    case 1: pairs_dispatch<1>(RTG_PAIRS_ARGS); break;
    case 2: pairs_dispatch<2>(RTG_PAIRS_ARGS); break;
    case 3: pairs_dispatch<3>(RTG_PAIRS_ARGS); break;
    case 4: pairs_dispatch<4>(RTG_PAIRS_ARGS); break;
    case 5: pairs_dispatch<5>(RTG_PAIRS_ARGS); break;
    case 6: pairs_dispatch<6>(RTG_PAIRS_ARGS); break;
    case 7: pairs_dispatch<7>(RTG_PAIRS_ARGS); break;
    case 8: pairs_dispatch<8>(RTG_PAIRS_ARGS); break;
    case 9: pairs_dispatch<9>(RTG_PAIRS_ARGS); break;
    case 10: pairs_dispatch<10>(RTG_PAIRS_ARGS); break;
    case 11: pairs_dispatch<11>(RTG_PAIRS_ARGS); break;
    case 12: pairs_dispatch<12>(RTG_PAIRS_ARGS); break;
    case 13: pairs_dispatch<13>(RTG_PAIRS_ARGS); break;
    case 14: pairs_dispatch<14>(RTG_PAIRS_ARGS); break;
    case 15: pairs_dispatch<15>(RTG_PAIRS_ARGS); break;
    case 16: pairs_dispatch<16>(RTG_PAIRS_ARGS); break;
    default:
      if (d <= 24) pairs_dispatch<24>(RTG_PAIRS_ARGS);
      else if (d <= 32) pairs_dispatch<32>(RTG_PAIRS_ARGS);
      else if (d <= 48) pairs_dispatch<48>(RTG_PAIRS_ARGS);
      else pairs_dispatch<64>(RTG_PAIRS_ARGS);
  }
#undef RTG_PAIRS_ARGS
}

void launch_unique_count(const uint64_t* keys, size_t count, uint32_t* tile_cnt, hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_unique_count, dim3(tiles_for(count)), dim3(kBlock), 0, s, keys, count,
                     tile_cnt);
}

void launch_unique_write(const uint64_t* keys, size_t count, const uint32_t* tile_off,
                         uint64_t* out, hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_unique_write, dim3(tiles_for(count)), dim3(kBlock), 0, s, keys, count,
                     tile_off, out);
}

void launch_swap_pairs(const uint64_t* pairs, size_t count, int pair_bits, uint64_t* swapped,
                       hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_swap_pairs, dim3(grid_for(count)), dim3(kBlock), 0, s, pairs, count,
                     pair_bits, swapped);
}

void launch_row_runs(const uint64_t* keys, size_t count, int pair_bits, uint32_t* rstart,
                     uint32_t* rend, hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_row_runs, dim3(grid_for(count)), dim3(kBlock), 0, s, keys, count, pair_bits,
                     rstart, rend);
}

void launch_row_degree(const uint32_t* lo_start, const uint32_t* lo_end, const uint32_t* up_start,
                       const uint32_t* up_end, int64_t n, uint64_t* deg, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_row_degree, dim3(grid_for((size_t)n)), dim3(kBlock), 0, s, lo_start, lo_end,
                     up_start, up_end, n, deg);
}

void launch_csr_fill_upper(const uint64_t* up, size_t count, int pair_bits, const int64_t* row_ptr,
                           const uint32_t* lo_start, const uint32_t* lo_end,
                           const uint32_t* up_start, int32_t* col, hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_csr_fill_upper, dim3(grid_for(count)), dim3(kBlock), 0, s, up, count,
                     pair_bits, row_ptr, lo_start, lo_end, up_start, col);
}

void launch_csr_fill_lower(const uint64_t* lo, size_t count, int pair_bits, const int64_t* row_ptr,
                           const uint32_t* lo_start, int32_t* col, hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_csr_fill_lower, dim3(grid_for(count)), dim3(kBlock), 0, s, lo, count,
                     pair_bits, row_ptr, lo_start, col);
}

// --- row buckets ------------------------------------------------------------

void launch_bucket_hist(const PairSource& src, size_t count, int pb, int rb, int both,
                        uint32_t nbuckets, uint32_t chunk, uint32_t nblocks, int threads,
                        uint32_t* part, uint32_t* zero_word, hipStream_t s) {
  if (!nblocks) {
    if (zero_word) launch_fill_u32(zero_word, 0u, 1, s);
    return;
  }
  const size_t lds = nbuckets * sizeof(uint32_t);
  if (threads >= 1024)
    hipLaunchKernelGGL(k_bucket_hist<1024>, dim3(nblocks), dim3(1024), lds, s, src.pairs, count,
                       pb, rb, both, nbuckets, chunk, nblocks, src.seg_cnt, src.seg_cap,
                       src.nseg, part, zero_word);
  else
    hipLaunchKernelGGL(k_bucket_hist<kBlock>, dim3(nblocks), dim3(kBlock), lds, s, src.pairs,
                       count, pb, rb, both, nbuckets, chunk, nblocks, src.seg_cnt, src.seg_cap,
                       src.nseg, part, zero_word);
}

void launch_bucket_scatter(const PairSource& src, size_t count, int pb, int rb, int both,
                           uint32_t nbuckets, uint32_t chunk, uint32_t nblocks, int threads,
                           const uint32_t* offs, uint32_t* entries, hipStream_t s) {
  if (!nblocks) return;
  const size_t lds = nbuckets * sizeof(uint32_t);
  if (threads >= 1024)
    hipLaunchKernelGGL(k_bucket_scatter<1024>, dim3(nblocks), dim3(1024), lds, s, src.pairs,
                       count, pb, rb, both, nbuckets, chunk, nblocks, src.seg_cnt, src.seg_cap,
                       src.nseg, offs, entries);
  else
    hipLaunchKernelGGL(k_bucket_scatter<kBlock>, dim3(nblocks), dim3(kBlock), lds, s, src.pairs,
                       count, pb, rb, both, nbuckets, chunk, nblocks, src.seg_cnt, src.seg_cap,
                       src.nseg, offs, entries);
}

void launch_bucket_csr(const uint32_t* entries, const uint32_t* offs, uint32_t nbuckets,
                       uint32_t nblocks, const uint32_t* total, uint32_t* oversized,
                       uint32_t* n_oversized, uint32_t cap, int pb, int rb, int64_t n,
                       int64_t nnz, int64_t* row_ptr, int32_t* col, hipStream_t s) {
  if (!nbuckets) {
    launch_fill_u64(reinterpret_cast<uint64_t*>(row_ptr + n), (uint64_t)nnz, 1, s);
    return;
  }
  if (cap > (uint32_t)kBucketMaxEntries) cap = kBucketMaxEntries;
  hipLaunchKernelGGL(k_bucket_csr, dim3(nbuckets), dim3(kCsrThreads), 0, s, entries, offs,
                     nbuckets, nblocks, total, oversized, n_oversized, cap, pb, rb, n, nnz, row_ptr,
                     col);
}

void launch_over_extent(const uint32_t* ids, uint32_t nover, const uint32_t* part,
                        uint32_t nblocks, uint32_t nbuckets, size_t np, uint32_t* start,
                        uint32_t* cnt, hipStream_t s) {
  if (!nover) return;
  hipLaunchKernelGGL(k_over_extent, dim3(grid_for(nover)), dim3(kBlock), 0, s, ids, nover, part,
                     nblocks, nbuckets, np, start, cnt);
}

void launch_over_gather(const uint32_t* entries, const uint32_t* start, const uint32_t* off,
                        uint32_t nover, uint32_t tot, int sh, uint64_t* w, hipStream_t s) {
  if (!nover || !tot) return;
  hipLaunchKernelGGL(k_over_gather, dim3(grid_for(tot)), dim3(kBlock), 0, s, entries, start, off,
                     nover, tot, sh, w);
}

void launch_over_emit(const uint64_t* keys, uint32_t tot, const uint32_t* ids,
                      const uint32_t* start, const uint32_t* cnt, const uint32_t* off, int pb,
                      int rb, int64_t n, int64_t* row_ptr, int32_t* col, hipStream_t s) {
  if (!tot) return;
  hipLaunchKernelGGL(k_over_emit, dim3(grid_for(tot)), dim3(kBlock), 0, s, keys, tot, ids, start,
                     cnt, off, pb, rb, n, row_ptr, col);
}

void launch_u32_to_u64(const uint32_t* src, size_t count, uint64_t* dst, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_widen, dim3(grid_for(count)), dim3(kBlock), 0, s, src, count, dst);
}

void launch_mailbox(const uint32_t* src, uint32_t words, const Gather* g, uint32_t* host,
                    uint64_t* host_seq, uint64_t seq, hipStream_t s) {
  hipLaunchKernelGGL(k_mailbox, dim3(1), dim3(kBlock), 0, s, src, words, g ? *g : Gather{}, host,
                     host_seq, seq);
}

void launch_gather(const Gather& g, uint64_t* dst, hipStream_t s) {
  if (g.count <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3(1), dim3(64), 0, s, g, dst);
}

void launch_records(const float* rows, int64_t n, int d, int rs, float* rec, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_records, dim3(grid_for((size_t)n)), dim3(kBlock), 0, s, rows, n, d, rs,
                     rec);
}

void launch_rowptr_at(const InstDesc* inst, uint32_t m, const int64_t* row_ptr, int64_t npts,
                      int64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_rowptr_at, dim3(grid_for((size_t)m + 1)), dim3(kBlock), 0, s, inst, m,
                     row_ptr, npts, out);
}

void launch_localize(const InstDesc* inst, uint32_t m, uint32_t nblocks, const int64_t* row_ptr,
                     const int32_t* col, const int64_t* at, int64_t total, int64_t* const* out_rp,
                     int32_t* const* out_col, hipStream_t s) {
  if (nblocks)
    hipLaunchKernelGGL(k_localize_rows, dim3(nblocks), dim3(kBlock), 0, s, inst, m, row_ptr,
                       out_rp);
  if (total > 0 && m > 0)
    hipLaunchKernelGGL(k_localize_cols,
                       dim3((unsigned)((total + kLocalizePer * kBlock - 1) / (kLocalizePer * kBlock))),
                       dim3(kBlock), 0, s, inst, m, at, col, out_col);
}

// --- memory for callers that cannot allocate ----------------------------------
// All scratch and the result of rtg_all_pairs_noalloc live here.  In host
// code the name is only a stand-in for the array, not a device address: the
// host side uses the address that noalloc_scratch_address returns for the
// current device, and the kernels get pointers into it as arguments.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

int noalloc_scratch_address(void** ptr) {
  *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return (int)e;
  }
  return 0;
}

}  // namespace rtgk
