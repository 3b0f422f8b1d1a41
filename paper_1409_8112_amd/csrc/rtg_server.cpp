// rtg_server.cpp -- batched entry point and request loop.
//
// Interim form: the batched call runs its queries one after another through
// the plain pipeline, and a submitted request runs at submit time.  Results
// are identical to rtg_all_pairs for each query.
#include "../../include/rtg.h"
#include "rtg_runtime.h"

#include <vector>

using rtg::Ctx;

extern "C" {

int rtg_all_pairs_batched(rtg_ctx* ctx, const rtg_query* q, int32_t nq, rtg_csr* outs) {
  if (!ctx || (nq > 0 && (!q || !outs)) || nq < 0) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::vector<rtg_csr> done;
  for (int32_t i = 0; i < nq; ++i) {
    rtg_csr o{};
    int rc = rtg_all_pairs(ctx, q[i].points, q[i].n, q[i].d, q[i].r, q[i].k, q[i].alpha,
                           q[i].seed, q[i].flags, &o);
    if (rc) {
      for (auto& x : done) rtg_release(ctx, x.handle);
      return rc;
    }
    done.push_back(o);
  }
  (void)c;
  for (int32_t i = 0; i < nq; ++i) outs[i] = done[i];
  return RTG_OK;
}

int rtg_submit(rtg_ctx* ctx, const rtg_query* q, uint64_t* ticket) {
  if (!ctx || !q || !ticket) return RTG_EINVAL;
  rtg_csr o{};
  int rc = rtg_all_pairs(ctx, q->points, q->n, q->d, q->r, q->k, q->alpha, q->seed, q->flags, &o);
  if (rc) return rc;
  *ticket = o.handle;
  return RTG_OK;
}

int rtg_poll(rtg_ctx* ctx, uint64_t ticket, rtg_csr* out) {
  if (!ctx || !out) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->results.find(ticket);
  if (it == c->results.end()) return RTG_ENOENT;
  out->n = it->second.n;
  out->nnz = it->second.nnz;
  out->row_ptr = it->second.row_ptr;
  out->col = it->second.col;
  out->handle = ticket;
  out->pairs = it->second.nnz / 2;
  return RTG_OK;
}

}  // extern "C"
