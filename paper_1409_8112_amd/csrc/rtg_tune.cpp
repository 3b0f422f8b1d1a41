// rtg_tune.cpp -- the autotuner.
//
// Launch settings.  A pass of the pipeline runs with the settings the context
// holds for its dimension and size (points of the pass, rounded up to a power
// of two), else with the defaults.  rtg_autotune times the caller's own
// workload -- one all-pairs query or a batch of one dimension -- under each
// candidate value of each setting in turn (coordinate descent from the
// current entry, the median of reps calls per candidate) and keeps the
// fastest; the entries go to and come from a JSON file.
//
// Parameters for a target recall.  rtg_tune_params applies the rule of the
// paper's parameter study (Sec. IV-A, Table II: the fastest (m, c~) that
// reaches the success rate) with the modelled recall of rtg_choose_params in
// place of a brute-force count and measured time in place of the cost model:
// for every cell factor on a grid, the least number of grids whose modelled
// recall reaches the target is timed on the caller's points, and the fastest
// is returned.
#include "../../include/rtg.h"
#include "rtg_runtime.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace rtg {

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

double median(std::vector<double> v) {
  std::sort(v.begin(), v.end());
  return v.empty() ? 0.0 : v[v.size() / 2];
}

int log2_up(int64_t x) {
  int b = 0;
  while (b < 62 && (int64_t(1) << b) < x) ++b;
  return b;
}

// One tunable setting: its candidate values and where it lives.
struct Knob {
  const char* name;
  std::vector<uint32_t> values;
  uint32_t* (*field)(Tuning&);
};

uint32_t* f_tpw(Tuning& t) { return &t.tests_per_wave; }
uint32_t* f_unit(Tuning& t) { return &t.unit_tiles; }
uint32_t* f_part(Tuning& t) { return &t.part_threads; }
uint32_t* f_bblk(Tuning& t) { return &t.bucket_blocks; }
uint32_t* f_bent(Tuning& t) { return &t.bucket_entries; }
uint32_t* f_sort(Tuning& t) { return reinterpret_cast<uint32_t*>(&t.sort_algo); }

const std::vector<Knob>& knobs() {
  static const std::vector<Knob> k = {
      {"tests_per_wave", {30000, 60000, 90000, 180000, 360000}, f_tpw},
      {"unit_tiles", {1, 2, 4}, f_unit},
      {"part_threads", {256, 1024}, f_part},
      {"bucket_blocks", {128, 256, 512}, f_bblk},
      {"bucket_entries", {7168, 10240, 14336}, f_bent},
      {"sort", {(uint32_t)rtgk::kSortOnesweep, (uint32_t)rtgk::kSortReduceScan}, f_sort},
  };
  return k;
}

bool valid(const rtg_tuning& t) {
  return t.d >= 1 && t.d <= rtgk::kMaxDim && t.log2_points >= 0 && t.log2_points <= 31 &&
         t.tests_per_wave >= 1000 && t.tests_per_wave <= 10000000 && t.unit_tiles >= 1 &&
         t.unit_tiles <= 64 && (t.part_threads == 256 || t.part_threads == 1024) &&
         t.bucket_blocks >= 1 && t.bucket_blocks <= 4096 && t.bucket_entries >= 256 &&
         t.bucket_entries <= rtgk::kBucketMaxEntries && (t.sort == 0 || t.sort == 1);
}

Tuning from_abi(const rtg_tuning& t) {
  Tuning x;
  x.tests_per_wave = (uint32_t)t.tests_per_wave;
  x.unit_tiles = (uint32_t)t.unit_tiles;
  x.part_threads = (uint32_t)t.part_threads;
  x.bucket_blocks = (uint32_t)t.bucket_blocks;
  x.bucket_entries = (uint32_t)t.bucket_entries;
  x.sort_algo = t.sort ? rtgk::kSortReduceScan : rtgk::kSortOnesweep;
  return x;
}

rtg_tuning to_abi(int d, int log2n, const Tuning& x, double ms) {
  rtg_tuning t{};
  t.d = d;
  t.log2_points = log2n;
  t.tests_per_wave = (int32_t)x.tests_per_wave;
  t.unit_tiles = (int32_t)x.unit_tiles;
  t.part_threads = (int32_t)x.part_threads;
  t.bucket_blocks = (int32_t)x.bucket_blocks;
  t.bucket_entries = (int32_t)x.bucket_entries;
  t.sort = x.sort_algo == rtgk::kSortReduceScan ? 1 : 0;
  t.ms = ms;
  return t;
}

// The integer after "key": in an object's text, or false.
bool json_int(const std::string& obj, const char* key, long long* v) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = obj.find(k);
  if (p == std::string::npos) return false;
  p = obj.find(':', p + k.size());
  if (p == std::string::npos) return false;
  char* end = nullptr;
  *v = std::strtoll(obj.c_str() + p + 1, &end, 10);
  return end != obj.c_str() + p + 1;
}

}  // namespace

// Times nq queries (one dimension) under the context's current settings:
// the median over reps calls of the batched pipeline (results released).
static int time_queries(Ctx& c, const rtg_query* q, int32_t nq, int32_t reps, double* ms) {
  std::vector<rtg_csr> outs((size_t)nq);
  std::vector<uint64_t> hs((size_t)nq);
  std::vector<double> t;
  for (int32_t r = 0; r <= reps; ++r) {  // the first call is not timed
    const double t0 = now_ms();
    const int rc = c.batched(q, nq, outs.data());
    const double t1 = now_ms();
    if (rc) return rc;
    for (int32_t i = 0; i < nq; ++i) hs[(size_t)i] = outs[(size_t)i].handle;
    (void)c.release_many(hs.data(), nq);
    if (r) t.push_back(t1 - t0);
  }
  *ms = median(t);
  return RTG_OK;
}

int Ctx::autotune(const rtg_query* q, int32_t nq, int32_t reps, rtg_tuning* out) {
  if (nq < 1 || reps < 1 || reps > 100) return RTG_EINVAL;
  const int d = q[0].d;
  int64_t pts = 0;
  for (int32_t i = 0; i < nq; ++i) {
    if (q[i].d != d) return RTG_EINVAL;
    pts += q[i].n;
  }
  // a pass holds at most batch_points points (a larger query runs alone)
  int64_t pass = std::min<int64_t>(pts, batch_points);
  for (int32_t i = 0; i < nq; ++i) pass = std::max<int64_t>(pass, q[i].n);
  const int key = log2_up(std::max<int64_t>(pass, 1));
  Tuning best = tuning_for(d, pass);
  auto install = [&](const Tuning& t) {
    std::lock_guard<std::mutex> lk(tmu);
    tuned[{d, key}] = t;
  };
  install(best);
  double best_ms = 0.0;
  int rc = time_queries(*this, q, nq, reps, &best_ms);
  if (rc) return rc;
  for (const Knob& kb : knobs()) {
    const uint32_t start = *kb.field(best);
    for (uint32_t v : kb.values) {
      if (v == start) continue;
      Tuning t = best;
      *kb.field(t) = v;
      install(t);
      double ms = 0.0;
      if ((rc = time_queries(*this, q, nq, reps, &ms))) {
        install(best);
        return rc;
      }
      // a candidate must win by more than the timing noise to replace the
      // current value
      if (ms < best_ms * 0.98) {
        best = t;
        best_ms = ms;
      }
    }
    install(best);
  }
  *out = to_abi(d, key, best, best_ms);
  return RTG_OK;
}

int Ctx::set_tuning(const rtg_tuning& t) {
  if (!valid(t)) return RTG_EINVAL;
  std::lock_guard<std::mutex> lk(tmu);
  tuned[{t.d, t.log2_points}] = from_abi(t);
  return RTG_OK;
}

int Ctx::save_tuning(const char* path) {
  std::vector<rtg_tuning> all;
  {
    std::lock_guard<std::mutex> lk(tmu);
    for (const auto& e : tuned) all.push_back(to_abi(e.first.first, e.first.second, e.second, 0.0));
  }
  FILE* f = std::fopen(path, "w");
  if (!f) return RTG_EINVAL;
  std::fprintf(f, "{\"rtg_tuning\": 1, \"entries\": [");
  for (size_t i = 0; i < all.size(); ++i) {
    const rtg_tuning& t = all[i];
    std::fprintf(f,
                 "%s\n {\"d\": %d, \"log2_points\": %d, \"tests_per_wave\": %d, "
                 "\"unit_tiles\": %d, \"part_threads\": %d, \"bucket_blocks\": %d, "
                 "\"bucket_entries\": %d, \"sort\": %d}",
                 i ? "," : "", t.d, t.log2_points, t.tests_per_wave, t.unit_tiles,
                 t.part_threads, t.bucket_blocks, t.bucket_entries, t.sort);
  }
  std::fprintf(f, "\n]}\n");
  return std::fclose(f) == 0 ? RTG_OK : RTG_EINVAL;
}

int Ctx::load_tuning(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return RTG_ENOENT;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  if (text.find("\"rtg_tuning\"") == std::string::npos) return RTG_EINVAL;
  size_t p = text.find("\"entries\"");
  if (p == std::string::npos) return RTG_EINVAL;
  std::vector<rtg_tuning> got_entries;
  while ((p = text.find('{', p + 1)) != std::string::npos) {
    const size_t e = text.find('}', p);
    if (e == std::string::npos) return RTG_EINVAL;
    const std::string obj = text.substr(p, e - p + 1);
    long long v[8];
    const char* names[8] = {"d", "log2_points", "tests_per_wave", "unit_tiles",
                            "part_threads", "bucket_blocks", "bucket_entries", "sort"};
    for (int i = 0; i < 8; ++i)
      if (!json_int(obj, names[i], &v[i]) || v[i] < 0 || v[i] > 100000000) return RTG_EINVAL;
    rtg_tuning t{};
    t.d = (int32_t)v[0];
    t.log2_points = (int32_t)v[1];
    t.tests_per_wave = (int32_t)v[2];
    t.unit_tiles = (int32_t)v[3];
    t.part_threads = (int32_t)v[4];
    t.bucket_blocks = (int32_t)v[5];
    t.bucket_entries = (int32_t)v[6];
    t.sort = (int32_t)v[7];
    if (!valid(t)) return RTG_EINVAL;
    got_entries.push_back(t);
    p = e;
  }
  std::lock_guard<std::mutex> lk(tmu);
  for (const rtg_tuning& t : got_entries) tuned[{t.d, t.log2_points}] = from_abi(t);
  return RTG_OK;
}

int Ctx::tune_params(const float* points, int64_t n, int32_t d, double r, double target,
                     uint32_t flags, int32_t reps, int32_t* k_out, double* alpha_out,
                     double* recall_out, double* ms_out) {
  if (!(target > 0.0 && target < 1.0) || reps < 1 || reps > 100) return RTG_EINVAL;
  int rc = check_query(points, n, d, r, 1, 1.0, flags);
  if (rc) return rc;
  if (n < 2) return RTG_EINVAL;
  double best_ms = INFINITY, best_alpha = 0.0, best_rec = 0.0;
  int32_t best_k = 0;
  for (int a = 20; a <= 50; ++a) {
    const double alpha = a / 20.0;  // 1.0, 1.05, ..., 2.5
    int32_t k = 0;
    double rec = 0.0;
    if (least_grids(d, alpha, target, flags, 128, &k, &rec)) continue;
    std::vector<double> R((size_t)k * d * d), u((size_t)k * d);
    if ((rc = make_transforms(0, k, d, flags, R.data(), u.data()))) return rc;
    std::vector<double> t;
    for (int32_t i = 0; i <= reps; ++i) {
      rtg_csr out{};
      const double t0 = now_ms();
      rc = all_pairs(points, n, d, r, k, alpha, R.data(), u.data(), flags, &out);
      const double t1 = now_ms();
      if (rc == RTG_ENOMEM || rc == RTG_ERANGE) break;  // not a candidate at this size
      if (rc) return rc;
      (void)release(out.handle);
      if (i) t.push_back(t1 - t0);
    }
    if ((int32_t)t.size() < reps) continue;
    const double ms = median(t);
    if (ms < best_ms) {
      best_ms = ms;
      best_k = k;
      best_alpha = alpha;
      best_rec = rec;
    }
  }
  if (!best_k) return RTG_ERANGE;
  *k_out = best_k;
  *alpha_out = best_alpha;
  *recall_out = best_rec;
  *ms_out = best_ms;
  return RTG_OK;
}

void Ctx::load_tuning_from_env() {
  if (const char* p = std::getenv("RTG_TUNING_FILE"))
    if (load_tuning(p) != RTG_OK)
      std::fprintf(stderr, "rtg: RTG_TUNING_FILE %s not loaded\n", p);
}

}  // namespace rtg

using rtg::Ctx;

extern "C" {

int rtg_autotune(rtg_ctx* ctx, const rtg_query* queries, int32_t nq, int32_t reps,
                 rtg_tuning* out) {
  if (!ctx || !queries || !out) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->poisoned) return RTG_EDEVICE;
  return c->autotune(queries, nq, reps, out);
}

int rtg_set_tuning(rtg_ctx* ctx, const rtg_tuning* t) {
  if (!ctx || !t) return RTG_EINVAL;
  return reinterpret_cast<Ctx*>(ctx)->set_tuning(*t);
}

int rtg_get_tuning(rtg_ctx* ctx, int32_t d, int64_t points, rtg_tuning* out) {
  if (!ctx || !out || d < 1 || d > rtgk::kMaxDim || points < 1) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  *out = rtg::to_abi(d, rtg::log2_up(points), c->tuning_for(d, points), 0.0);
  return RTG_OK;
}

int rtg_save_tuning(rtg_ctx* ctx, const char* path) {
  if (!ctx || !path) return RTG_EINVAL;
  return reinterpret_cast<Ctx*>(ctx)->save_tuning(path);
}

int rtg_load_tuning(rtg_ctx* ctx, const char* path) {
  if (!ctx || !path) return RTG_EINVAL;
  return reinterpret_cast<Ctx*>(ctx)->load_tuning(path);
}

int rtg_tune_params(rtg_ctx* ctx, const float* points, int64_t n, int32_t d, double r,
                    double target_recall, uint32_t flags, int32_t reps, int32_t* k,
                    double* alpha, double* recall, double* ms) {
  if (!ctx || !k || !alpha || !recall || !ms) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->poisoned) return RTG_EDEVICE;
  return c->tune_params(points, n, d, r, target_recall, flags, reps, k, alpha, recall, ms);
}

}  // extern "C"
