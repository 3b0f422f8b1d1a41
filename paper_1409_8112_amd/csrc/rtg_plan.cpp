// rtg_plan.cpp -- plans: batched calls of one fixed shape, repeated.
//
// A plan holds, for each batch its calls form, a device workspace and a HIP
// graph of the batch pass's device-sized stretch (cell keys, the segmented
// sort, cells, cell work and unit descriptors: every size in it is read on
// the device, so no host wait falls inside).  The first run sizes the
// workspaces, the second captures the graphs, and later runs upload their
// tables to the same addresses and launch the graphs instead of some twenty
// kernels each.  Anything that changes a captured argument (another cell-key
// layout for new data, another radius's signature width) is caught by
// comparing the arguments and recaptures; the results are those of
// rtg_all_pairs_batched either way.
#include "../../include/rtg.h"
#include "rtg_runtime.h"

#include <memory>
#include <mutex>
#include <vector>

namespace rtg {

struct Plan {
  Ctx* ctx = nullptr;
  struct Shape {
    int64_t n;
    int32_t d, k;
    uint32_t flags;
    bool operator==(const Shape& o) const {
      return n == o.n && d == o.d && k == o.k && flags == o.flags;
    }
  };
  std::vector<Shape> shape;
  std::vector<std::unique_ptr<PassPlan>> passes;
};

namespace {

std::vector<Plan::Shape> shape_of(const rtg_query* q, int32_t nq) {
  std::vector<Plan::Shape> s((size_t)nq);
  for (int32_t i = 0; i < nq; ++i) s[i] = Plan::Shape{q[i].n, q[i].d, q[i].k, q[i].flags};
  return s;
}

}  // namespace

}  // namespace rtg

using rtg::Ctx;
using rtg::Plan;

extern "C" {

int rtg_plan_create(rtg_ctx* ctx, const rtg_query* queries, int32_t nq, rtg_plan** out) {
  if (!ctx || !out || nq < 0 || (nq > 0 && !queries)) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  for (int32_t i = 0; i < nq; ++i) {
    const rtg_query& q = queries[i];
    const int rc = c->check_query(q.points, q.n, q.d, q.r, q.k, q.alpha, q.flags);
    if (rc) return rc;
  }
  Plan* p = new Plan;
  p->ctx = c;
  p->shape = rtg::shape_of(queries, nq);
  *out = reinterpret_cast<rtg_plan*>(p);
  return RTG_OK;
}

int rtg_plan_run(rtg_plan* plan, const rtg_query* queries, int32_t nq, rtg_csr* outs) {
  if (!plan || nq < 0 || (nq > 0 && (!queries || !outs))) return RTG_EINVAL;
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (rtg::shape_of(queries, nq) != p->shape) return RTG_EINVAL;
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  return p->ctx->batched(queries, nq, outs, &p->passes);
}

int rtg_plan_info(const rtg_plan* plan, int64_t* captures, int64_t* replays,
                  int64_t* workspace_bytes) {
  if (!plan || !captures || !replays || !workspace_bytes) return RTG_EINVAL;
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  *captures = *replays = *workspace_bytes = 0;
  for (const auto& pp : p->passes) {
    *captures += pp->captures;
    *replays += pp->replays;
    if (pp->ws) *workspace_bytes += (int64_t)pp->head_bytes;
  }
  return RTG_OK;
}

int rtg_plan_destroy(rtg_plan* plan) {
  if (!plan) return RTG_EINVAL;
  Plan* p = reinterpret_cast<Plan*>(plan);
  {
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    // runs are blocking, so nothing queued reads the workspaces any more
    (void)hipStreamSynchronize(p->ctx->main.stream);
    for (auto& pp : p->passes) {
      if (pp->exec) (void)hipGraphExecDestroy(pp->exec);
      if (pp->ws) p->ctx->dfree(pp->ws);
    }
  }
  delete p;
  return RTG_OK;
}

}  // extern "C"
