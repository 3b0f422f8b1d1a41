// rtg_server.cpp -- batched entry point and request loop.
//
// The batched call groups queries by dimension and runs each group through
// the batch pipeline (one pass per batch of instances).  Interim request
// loop: a submitted request runs at submit time.
#include "../../include/rtg.h"
#include "rtg_runtime.h"

#include <vector>

using rtg::Ctx;

extern "C" {

int rtg_all_pairs_batched(rtg_ctx* ctx, const rtg_query* q, int32_t nq, rtg_csr* outs) {
  if (!ctx || nq < 0 || (nq > 0 && (!q || !outs))) return RTG_EINVAL;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  return c->batched(q, nq, outs);
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
