// rtg_runtime.h -- host runtime of the RTG library: device-memory arena,
// context, key-packing plan.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
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

// Best-fit sub-allocator over one device buffer (the context's memory
// budget): free blocks indexed by offset (for coalescing) and by length
// (for the search).  Host-side bookkeeping only; blocks are 256-byte aligned.
class Arena {
 public:
  static constexpr size_t kAlign = 256;
  Arena(char* base, size_t bytes);
  void* alloc(size_t bytes);  // nullptr when no free block is large enough
  void release(void* p);
  void shrink(void* p, size_t bytes);  // gives back the tail of a block past bytes
  size_t largest_free() const;
  size_t size() const { return size_; }
  size_t in_use() const { return in_use_; }
  size_t peak() const { return peak_; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, in_use_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;            // offset -> length
  std::multimap<size_t, size_t> by_size_;    // length -> offset (the same free blocks)
  std::map<size_t, size_t> used_;            // offset -> length
  void add_free(size_t off, size_t len);
  void drop_free(std::map<size_t, size_t>::iterator it);
};

// How cell vectors are packed into the sort key for one query.
struct Packing {
  rtgk::KeyLayout layout{};
  std::vector<int64_t> klo;  // [k][d] origin of each packed field
  int tb = 1;                // segments (instance, grid) per sort
  int seg_bits = 0;          // bits of the grid id above the cell fields
  int key_bits = 0;          // seg_bits + cell_bits
  bool truncated = false;    // some field narrower than its span (aliasing)
  bool wrapped = false;      // some field's span beyond 32 bits (aliasing)
};

int make_transforms(uint64_t seed, int32_t k, int32_t d, uint32_t flags, double* R, double* u);
int model_recall(int32_t d, int32_t k, double alpha, uint32_t flags, double* recall);
int choose_params(int32_t d, double target, double nu, uint32_t flags, int32_t* k_out,
                  double* alpha_out, double* recall_out);
// The least k <= kmax whose modelled recall at cell factor alpha reaches
// target (RTG_ERANGE if none does), and that recall.
int least_grids(int32_t d, double alpha, double target, uint32_t flags, int32_t kmax,
                int32_t* k_out, double* recall_out);
int min_field_bits(double alpha);
// Candidate pairs a pass makes room for per (point, grid) key before it
// learns the exact count (a pass that needs more runs its pair kernel again).
uint64_t cand_per_key(uint32_t flags);
int validate_query(const float* points, int64_t n, int32_t d, double r, int32_t k, double alpha);
// Flags that shape a pass's output (instances batched together share them).
constexpr uint32_t kListFlags = RTG_UPPER_ONLY | RTG_DEDUP_SORT | RTG_DEDUP_BITMAP;
// Largest default grid of the pair kernels.
constexpr uint32_t kMaxPairBlocks = 8192;
// Output segments of the pair kernels (each with its own counter).
constexpr uint32_t kCandSegments = 32;
// The pass counters: [0] unused, [1] FP64 re-tests, [2] filter count,
// [3] cell members, [4, 4 + kCandSegments) segment counts, then the
// pipeline's error bits (a u32 in the low half of the last word).
constexpr uint32_t kErrWord = 4 + kCandSegments;
constexpr uint32_t kCounterWords = kErrWord + 1;
// Largest pair bitmap of one pass (RTG_DEDUP_BITMAP): beyond it the pass
// removes repeats by the first-owner rule instead.
constexpr uint64_t kBitmapMaxBytes = uint64_t(4) << 30;

// Axes per robot of the MR-metric that flags select (0: Euclidean), or -1
// for flags the library does not know or a robot count that does not
// divide d.
int axes_per_robot(int32_t d, uint32_t flags);
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
  uint64_t handle = 0;  // result handle to use (0: a new one)
};

// Points per batch of rtg_all_pairs_batched (an instance larger runs alone):
// keeps the neighbour-list build on row buckets and the packed sort keys.
constexpr int64_t kBatchPoints = int64_t(1) << 22;
// Pinned upload staging of the main lane, made at rtg_create: everything
// rtg_all_pairs_noalloc uploads fits it.
constexpr size_t kNoallocStaging = size_t(256) << 10;

int plan_batch(int d, uint32_t m, const int64_t* k, const int64_t* n, const double* R,
               const double* u, const double* inv_c, const double* alpha, const float* lo,
               const float* hi, size_t budget_bytes, Packing& P);

struct Result {
  void* mem;
  int64_t n, nnz, pairs;
  int64_t* row_ptr;
  int32_t* col;
};

// Query mode: the sorted grids of one point set, kept on the device.
struct Index {
  int64_t n = 0;
  int32_t d = 0, k = 0;
  double r = 0.0, alpha = 0.0;
  int32_t sub = 0;  // MR-metric: axes per robot; 0: Euclidean
  Packing P;
  int sig_b = 0, sig_g = 0, sig_gpw = 1, sig_W = 0;
  uint64_t lows = 0, highs = 0;
  float* pts = nullptr;       // [n][d] copy of the points
  uint64_t* sig = nullptr;    // [n][W] signatures
  double *R = nullptr, *u = nullptr;
  int64_t* klo = nullptr;
  rtgk::KeyLayout* layout = nullptr;
  rtgk::QueryGrid* grids = nullptr;  // device [k]
  std::vector<void*> blocks;         // arena blocks the index owns
};

// Launch settings of one pass (rtg_tuning in rtg.h): the context's
// defaults, or what the autotuner found for the pass's dimension and size.
struct Tuning {
  uint32_t tests_per_wave = 90000;  // pair kernels: grid of about this many tests per wave
  uint32_t unit_tiles = 1;          // cells of at most this many tiles are one unit
  uint32_t part_threads = 256;      // neighbour-list partition block size (256 or 1024)
  uint32_t bucket_blocks = 256;     // neighbour-list partition blocks
  uint32_t bucket_entries = rtgk::kBucketMaxEntries / 8 * 7;  // target entries per bucket
  int sort_algo = rtgk::kSortReduceScan;
};

// One batch pass that a plan (rtg_plan) runs again and again with the same
// shape: the pass's leading allocations come from the plan's workspace, so
// their addresses repeat from run to run, and the stretch from the key
// kernel to the unit descriptors -- whose sizes are all on the device -- is
// captured once as a HIP graph and replayed.
struct PassPlan {
  void* ws = nullptr;            // workspace (an arena block of head_bytes)
  size_t head_bytes = 0;
  std::vector<int64_t> shape;    // launch arguments of the captured stretch
  hipGraphExec_t exec = nullptr;
  int64_t launches[RTG_NKERNELS] = {};  // the stretch's launches and bytes (stats)
  double bytes[RTG_NKERNELS] = {};
  int key_passes = 0;
  int where = 0;                 // which key buffer holds the sorted keys
  int64_t captures = 0, replays = 0;
};

struct Ctx;
struct Server;

// An execution lane: one HIP stream with its own staging buffers and timing
// state.  A pass of the pipeline runs on one lane and is ordered on its
// stream; passes on different lanes run concurrently and share the
// context's arena and results.
struct Lane {
  Ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // A stream that only records graphs (made on first use) for a lane whose
  // stream cannot be captured (the caller's, possibly the null stream); the
  // graphs are launched on the lane's stream.
  hipStream_t cap_stream = nullptr;
  void* scratch = nullptr;     // the innermost open scratch set of this lane (rtg_host.cpp)
  // Blocks a pass drops are kept for the pass's own later allocations (no
  // wait); off for the request loop's lanes, whose admission reads the
  // arena's free bytes and needs them back at once.
  bool keep_drops = true;
  // Allocations of this lane come from the context's no-allocation arena
  // (the file-scope device array) instead of its budget: set for the
  // duration of an rtg_all_pairs_noalloc call.
  bool noalloc = false;
  void* host_stage = nullptr;  // pinned staging for read-backs
  size_t host_stage_bytes = 0;
  void* host_up = nullptr;     // pinned staging for batched uploads
  size_t host_up_bytes = 0;
  hipEvent_t up_done = nullptr;  // recorded after the last batched upload's copy
  bool up_pending = false;
  void* gather_dev = nullptr;  // 8 device u64 that gather_back fills
  // Pinned mailbox of the read-backs: a sequence word, then kMailBytes of
  // values (see wait_mail).
  static constexpr size_t kMailBytes = 64 << 10;
  uint64_t* mail = nullptr;
  uint64_t mail_seq = 0;
  // Waits for the mailbox kernel just queued to post seq: spins, then after
  // a while synchronises the stream (which also reports a failed kernel).
  int wait_mail(uint64_t seq);
  uint32_t timing_mask = 0;    // bit i: time kernel id i; RTG_TIME_PHASES: phases
  hipEvent_t ev[9] = {};
  std::vector<hipEvent_t> kev;                // pool of event pairs
  std::vector<std::pair<int, int>> kpending;  // (kernel id, event pair) of this pass
  rtg_stats* kstats = nullptr;                // stats of the pass in flight

  int init(Ctx* c, hipStream_t s, bool create_stream);
  void fini();
  int hip_fail(hipError_t e, const char* what);
  void* dalloc(size_t bytes);
  void dfree(void* p);
  size_t largest_free();  // in the arena this lane allocates from
  int sync();
  int read_back(const void* dev, size_t bytes, void* host);
  // Several device scalars in one copy (one sync).
  int gather_back(const rtgk::Gather& g, uint64_t* host);
  int upload(void* dev, const void* host, size_t bytes);
  // Room for bytes in the pinned upload staging, once the previous batched
  // upload has left it.
  int up_room(size_t bytes);
  int download(void* host, const void* dev, size_t bytes);  // ordered on the stream, waits
  void mark(int phase);
  void kbegin(int kid);
  void kend(int kid, double bytes);
  void kfinish();  // after a sync: add the timed launches to *kstats
  rtgk::LaunchTimer timer();

  int make_empty_result(int64_t n, rtg_csr* out, uint64_t handle);
  int build_index(const float* points, int64_t n, int32_t d, double r, int32_t k, double alpha,
                  const double* R, const double* u, Index& I);
  int query_index(const Index& I, const float* queries, int64_t m, rtg_stats& st,
                  rtg_csr* out);
  int tiny_query(const float* points, int64_t n, int32_t d, rtg_csr* out, uint64_t handle);
  // One pass of the pipeline over a batch of instances of one dimension
  // (pp: the pass of a plan, or null).
  int run_batch(std::vector<Job*>& jobs, rtg_stats& st, PassPlan* pp = nullptr);
  // One small instance in two launches (kTinyPoints, d <= 8, Euclidean);
  // kTinyFallback when it is outside the small path's limits.
  static constexpr int kTinyFallback = 1000;
  int run_tiny(Job& job, rtg_stats& st);
};

struct Ctx {
  explicit Ctx(int dev);
  ~Ctx();

  int device;
  bool own_arena = false;
  void* arena_mem = nullptr;
  std::unique_ptr<Arena> arena;
  // rtg_all_pairs_noalloc: the file-scope device array of this device
  // (address from hipGetSymbolAddress at rtg_create) and the arena over it.
  void* noalloc_base = nullptr;
  std::unique_ptr<Arena> noalloc_arena;
  std::atomic<bool> poisoned{false};
  uint32_t bucket_cap = rtgk::kBucketMaxEntries;  // entries per LDS-sorted bucket
  int64_t batch_points = kBatchPoints;             // points per batch
  int server_lanes = 2;  // passes of the request loop that may run at once
  int pair_screen = 0;   // 0 auto, 1 vector, 2 matrix cores (d <= 16)
  bool unit_band = true;  // matrix-core band from the cell diagonal where keys are exact
  bool small_path = true;  // one small instance in two launches (Lane::run_tiny)
  bool small_fits(int64_t n, int32_t d, int32_t k, uint32_t flags) const;
  size_t small_bytes(int64_t n, int32_t d, int32_t k) const;  // device bytes it takes at most
  bool gather_direct = true;  // pair kernels read rows by point index
  uint32_t pair_blocks = 0;      // pair-kernel grid (0: from the tuning's tests per wave)
  bool balanced_units = true;    // pair-kernel waves take equal shares of the tile pairs
  // Launch settings: the defaults (environment), and the autotuner's entries
  // by (dimension, log2 of the points of a pass), under tmu.
  Tuning defaults;
  std::map<std::pair<int, int>, Tuning> tuned;
  std::mutex tmu;
  Tuning tuning_for(int d, int64_t npts);
  // the autotuner (rtg_tune.cpp)
  int autotune(const rtg_query* q, int32_t nq, int32_t reps, rtg_tuning* out);
  int set_tuning(const rtg_tuning& t);
  int save_tuning(const char* path);
  int load_tuning(const char* path);
  void load_tuning_from_env();
  int tune_params(const float* points, int64_t n, int32_t d, double r, double target,
                  uint32_t flags, int32_t reps, int32_t* k, double* alpha, double* recall,
                  double* ms);
  Lane main;          // the caller's stream: blocking calls
  // More lanes for rtg_all_pairs_batched: batches run batch_lanes at a time
  // (the caller's lane and batch_lanes - 1 more), so one pass's host work and
  // waits overlap the others' kernels (RTG_BATCH_LANES, 1 to 3).  Made for
  // each call that has several batches and released at its end.
  int batch_lanes = 3;
  std::vector<std::unique_ptr<Lane>> side;
  hipEvent_t side_ready = nullptr;  // the caller's stream reached the call
  int side_lanes(int count);
  rtg_stats stats{};  // of the last blocking call
  std::mutex mu;      // one blocking call at a time
  std::mutex amu;     // arena, results, handles
  std::map<uint64_t, Result> results;
  std::map<uint64_t, std::unique_ptr<Index>> indexes;
  uint64_t next_handle = 1;
  Server* server = nullptr;  // request loop, started by the first rtg_submit
  std::mutex server_mu;      // guards the server pointer

  int hip_fail(hipError_t e, const char* what);
  void* dalloc(size_t bytes);
  void* dalloc_noalloc(size_t bytes);   // from the no-allocation arena
  size_t largest_free_noalloc();
  void dfree(void* p);                  // to whichever arena holds p
  void dshrink(void* p, size_t bytes);  // a block's tail back to its arena
  Arena* arena_of(const void* p);       // (under amu)
  // Device bytes one pass of the pipeline takes for an instance (points
  // excluded), while its candidates stay within cand_per_key per key.
  size_t pass_bytes_bound(int64_t n, int32_t d, int32_t k, double alpha, uint32_t flags) const;
  size_t largest_free();
  size_t free_bytes();
  uint64_t new_handle();
  uint64_t keep_result(uint64_t h, void* mem, int64_t n, int64_t nnz, int64_t pairs,
                       int64_t* row_ptr, int32_t* col);
  int release(uint64_t handle);
  int release_many(const uint64_t* handles, int32_t count);
  bool find_result(uint64_t handle, rtg_csr* out);

  int all_pairs(const float* points, int64_t n, int32_t d, double r, int32_t k, double alpha,
                const double* R, const double* u, uint32_t flags, rtg_csr* out);
  int all_pairs_noalloc(const float* points, int64_t n, int32_t d, double r, int32_t k,
                        double alpha, const double* R, const double* u, uint32_t flags,
                        int64_t* row_ptr, int32_t* col, int64_t col_capacity, int64_t* nnz);
  // Many queries: one pass per batch; with plan, batch b runs as plan[b].
  int batched(const rtg_query* q, int32_t nq, rtg_csr* outs,
              std::vector<std::unique_ptr<PassPlan>>* plan = nullptr);
  // The batches batched() forms: query indices, grouped by dimension and
  // list flags, at most batch_points points each.
  std::vector<std::vector<int32_t>> batch_groups(const rtg_query* q, int32_t nq);
  int check_query(const float* points, int64_t n, int32_t d, double r, int32_t k, double alpha,
                  uint32_t flags);
  int debug_cell_coords(const float* points, int64_t n, int32_t d, double r, double alpha,
                        const double* R, const double* u, int64_t* kappa_host);

  // request loop (rtg_server.cpp)
  int submit(const rtg_query& q, uint64_t* ticket);
  int poll(uint64_t ticket, rtg_csr* out);
  void stop_server();
  void wake_server();   // memory came back: requests waiting for it may run
  bool holds_results();  // results or indexes held in the arena
  std::atomic<int64_t> served_requests{0}, served_batches{0}, served_small{0};
};

}  // namespace rtg
