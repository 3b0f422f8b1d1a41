// rtg_runtime.h -- host runtime of the RTG library: device-memory arena,
// context, key-packing plan.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/rtg.h"
#include "rtg_internal.h"

namespace rtg {

// First-fit sub-allocator over one device buffer (the context's memory
// budget).  Host-side bookkeeping only; blocks are 256-byte aligned.
class Arena {
 public:
  static constexpr size_t kAlign = 256;
  Arena(char* base, size_t bytes);
  void* alloc(size_t bytes);  // nullptr when no free block is large enough
  void release(void* p);
  size_t largest_free() const;
  size_t size() const { return size_; }
  size_t in_use() const { return in_use_; }
  size_t peak() const { return peak_; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, in_use_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> used_;  // offset -> length
};

// How cell vectors are packed into the sort key for one query.
struct Packing {
  rtgk::KeyLayout layout{};
  std::vector<int64_t> klo;  // [k][d] origin of each packed field
  int tb = 1;                // segments (instance, grid) per sort
  int seg_bits = 0;          // bits of the grid id above the cell fields
  int key_bits = 0;          // seg_bits + cell_bits
  bool truncated = false;    // some field narrower than its span (aliasing)
};

int make_transforms(uint64_t seed, int32_t k, int32_t d, uint32_t flags, double* R, double* u);
int min_field_bits(double alpha);
int validate_query(const float* points, int64_t n, int32_t d, double r, int32_t k, double alpha);
int check_device_pointer(const void* p, int device);

// One query of a batch, with its transforms (host arrays).
struct Job {
  const float* pts;
  int64_t n;
  int32_t d;
  double r, alpha;
  int32_t k;
  uint32_t flags;
  const double* R;  // [k][d][d]
  const double* u;  // [k][d]
  rtg_csr* out;
};

// Points per batch of rtg_all_pairs_batched (an instance larger runs alone):
// keeps the neighbour-list build on row buckets and the packed sort keys.
constexpr int64_t kBatchPoints = int64_t(1) << 22;

int plan_batch(int d, uint32_t m, const int64_t* k, const int64_t* n, const double* R,
               const double* u, const double* inv_c, const double* alpha, const float* lo,
               const float* hi, size_t budget_bytes, Packing& P);

struct Result {
  void* mem;
  int64_t n, nnz;
  int64_t* row_ptr;
  int32_t* col;
};

struct Ctx {
  Ctx(int dev, hipStream_t s);
  ~Ctx();

  int device;
  hipStream_t stream;
  bool own_arena = false;
  void* arena_mem = nullptr;
  std::unique_ptr<Arena> arena;
  void* host_stage = nullptr;  // pinned staging for scalar read-backs
  void* gather_dev = nullptr;  // 8 device u64 that gather_back fills
  bool poisoned = false;
  uint32_t timing_mask = 0;  // bit i: time kernel id i; RTG_TIME_PHASES: phases
  int sort_algo = 0;         // rtgk::kSortOnesweep or rtgk::kSortReduceScan
  uint32_t bucket_cap = rtgk::kBucketMaxEntries;  // entries per LDS-sorted bucket
  int64_t batch_points = kBatchPoints;             // points per batch
  hipEvent_t ev[9] = {};
  rtg_stats stats{};
  // per-launch timing: a pool of event pairs and the launches of this call
  std::vector<hipEvent_t> kev;
  std::vector<std::pair<int, int>> kpending;  // (kernel id, event pair)
  rtg_stats* kstats = nullptr;                // stats of the call in flight
  std::mutex mu;  // one pipeline call at a time
  std::map<uint64_t, Result> results;
  uint64_t next_handle = 1;

  int hip_fail(hipError_t e, const char* what);
  void* dalloc(size_t bytes);
  void dfree(void* p);
  int sync();
  int read_back(const void* dev, size_t bytes, void* host);
  // Several device scalars in one copy (one sync).
  int gather_back(const rtgk::Gather& g, uint64_t* host);
  int upload(void* dev, const void* host, size_t bytes);
  void mark(int phase);
  void kbegin(int kid);
  void kend(int kid, double bytes);
  void kfinish();  // after a sync: add the timed launches to *kstats
  rtgk::LaunchTimer timer();
  uint64_t keep_result(void* mem, int64_t n, int64_t nnz, int64_t* row_ptr, int32_t* col);
  int release(uint64_t handle);
  int make_empty_result(int64_t n, rtg_csr* out);

  int all_pairs(const float* points, int64_t n, int32_t d, double r, int32_t k, double alpha,
                const double* R, const double* u, uint32_t flags, rtg_csr* out);
  int batched(const rtg_query* q, int32_t nq, rtg_csr* outs);
  int run_batch(std::vector<Job*>& jobs, rtg_stats& st);
  int check_query(const float* points, int64_t n, int32_t d, double r, int32_t k, double alpha);
  int tiny_query(const float* points, int64_t n, int32_t d, rtg_csr* out);
  int debug_cell_coords(const float* points, int64_t n, int32_t d, double r, double alpha,
                        const double* R, const double* u, int64_t* kappa_host);

  // request loop (rtg_server.cpp)
  void stop_server() {}
};

}  // namespace rtg
