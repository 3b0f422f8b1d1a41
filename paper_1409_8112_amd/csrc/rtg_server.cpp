// rtg_server.cpp -- batched entry point and the request loop.
//
// The request loop is continuous batching over the batch pipeline.  A
// submitted query's points are copied into the arena before rtg_submit
// returns, then the query waits in a FIFO queue.  Each lane (a HIP stream
// driven by its own worker thread) repeatedly takes the queue's head and
// every other waiting query of the same dimension and list flags that fits,
// runs them as one pass of the pipeline, and files the results under their
// tickets.  Queries that arrive while a pass runs join the next pass on a
// free lane, so passes of different lanes overlap on the device.
//
// Admission is by device memory: a pass starts when its working-set bound
// (Ctx::pass_bytes_bound) fits the arena's free bytes -- which already count
// the finished results the caller has not released -- less the bounds of
// the passes already running (the head of the queue always starts on an
// idle device).  A pass that still runs out of memory, or fails on one of
// its queries, is split: its queries go back to the front of the queue to
// run alone, on an idle device, so each query gets its own result or error.
// A query that runs out of memory alone while other requests' points or
// unreleased results hold part of the budget waits until memory comes back
// (a release, or a pass that ends) and runs again; it fails with ENOMEM
// only when nothing else holds memory.  A query's result never depends on
// its batch-mates: no step of a pass mixes instances.
//
// A query within the small-instance limits of rtg_all_pairs that reaches
// the head of the queue while the device is idle runs alone on that path's
// two launches, and no other pass starts meanwhile: its workgroups take a
// CU's LDS each and would otherwise wait for another pass's kernels to
// drain.  On a busy device it heads or joins a batch pass like any other.
#include "../../include/rtg.h"
#include "rtg_runtime.h"

#include <algorithm>
#include <cstdlib>
#include <vector>

namespace rtg {

namespace {

enum { kQueued = 0, kRunning = 1, kDone = 2 };

struct Request {
  uint64_t ticket = 0;
  rtg_query q{};          // q.points: the staged copy in the arena
  void* pts_mem = nullptr;
  std::vector<double> R, u;
  size_t est = 0;
  int state = kQueued;
  int rc = RTG_OK;
  bool solo = false;      // run alone on an idle device
  bool small = false;     // within the small path's limits
  bool tiny_run = false;  // picked to run alone on the small path
  // Ran alone and ran out of memory while other requests' points or results
  // held part of the budget: waits until some memory is given back (the
  // server's release count passes wait_gen).
  bool waiting = false;
  uint64_t wait_gen = 0;
  rtg_csr out{};
};

uint32_t group_of(const rtg_query& q) {
  return ((uint32_t)q.d << 8) | (q.flags & kListFlags);
}

}  // namespace

struct Server {
  explicit Server(Ctx& ctx) : c(ctx) {}
  Ctx& c;

  std::mutex m;  // guards everything below except the copy lane
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<std::unique_ptr<Lane>> lanes;
  std::vector<size_t> reserved;  // estimate of the pass on each lane (0: idle)
  std::vector<std::thread> workers;
  int running = 0;
  bool solo_running = false;
  bool stop = false;
  uint64_t gen = 0;  // device memory given back (results released, points dropped)

  std::mutex copy_mu;  // the copy lane: staging of submitted points
  Lane copy;
  hipEvent_t ready = nullptr;

  int start(int nlanes);
  void shutdown();
  int submit(const rtg_query& q, uint64_t* ticket);
  int poll(uint64_t ticket, rtg_csr* out);
  bool pick(std::vector<Request*>& batch, size_t& est);
  void work(int li);
  // Called when the caller releases a result or an index: a request waiting
  // for memory may run again.
  void wake() {
    {
      std::lock_guard<std::mutex> lk(m);
      ++gen;
    }
    cv.notify_all();
  }
};

int Server::start(int nlanes) {
  if (hipSetDevice(c.device) != hipSuccess) return RTG_EDEVICE;
  int rc = copy.init(&c, nullptr, true);
  if (rc) return rc;
  if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) return RTG_EDEVICE;
  for (int i = 0; i < nlanes; ++i) {
    lanes.emplace_back(new Lane());
    if ((rc = lanes.back()->init(&c, nullptr, true))) return rc;
    lanes.back()->keep_drops = false;  // admission reads the free bytes
  }
  reserved.assign(nlanes, 0);
  for (int i = 0; i < nlanes; ++i) workers.emplace_back(&Server::work, this, i);
  return RTG_OK;
}

void Server::shutdown() {
  {
    std::lock_guard<std::mutex> lk(m);
    stop = true;
  }
  cv.notify_all();
  for (auto& w : workers) w.join();
  workers.clear();
  // Queued queries never ran: drop their staged points.  Finished results
  // stay in the context until released or destroyed.
  for (Request* r : queue) c.dfree(r->pts_mem);
  queue.clear();
  for (auto& l : lanes) l->fini();
  copy.fini();
  if (ready) (void)hipEventDestroy(ready);
  ready = nullptr;
}

int Server::submit(const rtg_query& q, uint64_t* ticket) {
  std::unique_ptr<Request> req(new Request());
  req->q = q;
  req->R.resize((size_t)q.k * q.d * q.d);
  req->u.resize((size_t)q.k * q.d);
  int rc = make_transforms(q.seed, q.k, q.d, q.flags, req->R.data(), req->u.data());
  if (rc) return rc;
  const size_t pts_bytes = sizeof(float) * (size_t)q.n * (size_t)q.d;
  req->est = c.pass_bytes_bound(q.n, q.d, q.k, q.alpha, q.flags);
  req->small = c.small_fits(q.n, q.d, q.k, q.flags);
  if (req->small) req->est = std::max(req->est, c.small_bytes(q.n, q.d, q.k));
  if (req->est + pts_bytes > c.arena->size()) return RTG_ENOMEM;
  const uint64_t t = c.new_handle();
  req->ticket = t;
  {
    std::lock_guard<std::mutex> lk(copy_mu);
    if (q.n <= 1) {
      // nothing to pair: the (empty) result is ready at once
      if ((rc = copy.tiny_query(q.points, q.n, q.d, &req->out, t))) return rc;
      req->state = kDone;
    } else {
      req->pts_mem = c.dalloc(pts_bytes);
      if (!req->pts_mem) return RTG_EAGAIN;  // no room to stage it now
      // The copy follows the work the caller queued on the context's stream.
      rc = c.hip_fail(hipEventRecord(ready, c.main.stream), "hipEventRecord");
      if (!rc) rc = c.hip_fail(hipStreamWaitEvent(copy.stream, ready, 0), "hipStreamWaitEvent");
      if (!rc)
        rc = c.hip_fail(hipMemcpyAsync(req->pts_mem, q.points, pts_bytes,
                                       hipMemcpyDeviceToDevice, copy.stream),
                        "stage points");
      if (!rc) rc = copy.sync();
      if (rc) {
        c.dfree(req->pts_mem);
        return rc;
      }
      req->q.points = static_cast<const float*>(req->pts_mem);
    }
  }
  {
    std::lock_guard<std::mutex> lk(m);
    Request* r = req.get();
    reqs[t] = std::move(req);
    if (r->state == kQueued) queue.push_back(r);
  }
  cv.notify_all();
  *ticket = t;
  return RTG_OK;
}

int Server::poll(uint64_t t, rtg_csr* out) {
  std::unique_lock<std::mutex> lk(m);
  auto it = reqs.find(t);
  if (it == reqs.end()) {
    lk.unlock();
    // a ticket already collected: its result, while not released
    return c.find_result(t, out) ? RTG_OK : RTG_ENOENT;
  }
  Request* r = it->second.get();
  if (r->state != kDone) return RTG_EAGAIN;
  const int rc = r->rc;
  if (rc == RTG_OK) {
    *out = r->out;
    out->handle = t;
  }
  reqs.erase(it);
  return rc;
}

// Under m: the next pass for an idle lane, or false to wait.  The pass
// starts with the first queued request that is not waiting for memory.
bool Server::pick(std::vector<Request*>& batch, size_t& est) {
  batch.clear();
  if (queue.empty() || solo_running) return false;
  Request* h = nullptr;
  for (Request* r : queue) {
    if (r->waiting && r->wait_gen == gen) continue;
    r->waiting = false;
    h = r;
    break;
  }
  if (!h) return false;
  if (h->solo && running > 0) return false;
  size_t others = 0;
  for (size_t v : reserved) others += v;
  const size_t free = c.free_bytes();
  const size_t avail = free > others ? free - others : 0;
  if (running > 0 && h->est > avail) return false;  // wait for memory
  batch.push_back(h);
  est = h->est;
  int64_t pts = h->q.n;
  h->tiny_run = h->small && running == 0;
  if (!h->solo && !h->tiny_run) {
    const uint32_t g = group_of(h->q);
    for (size_t i = 0; i < queue.size(); ++i) {
      Request* r = queue[i];
      if (r == h || r->solo || r->waiting || group_of(r->q) != g) continue;
      if (pts + r->q.n > c.batch_points || est + r->est > avail) continue;
      batch.push_back(r);
      est += r->est;
      pts += r->q.n;
    }
  }
  std::deque<Request*> rest;
  for (Request* r : queue)
    if (std::find(batch.begin(), batch.end(), r) == batch.end()) rest.push_back(r);
  queue.swap(rest);
  return true;
}

void Server::work(int li) {
  (void)hipSetDevice(c.device);
  Lane& L = *lanes[li];
  std::vector<Request*> batch;
  std::unique_lock<std::mutex> lk(m);
  for (;;) {
    size_t est = 0;
    while (!stop && !pick(batch, est)) cv.wait(lk);
    if (stop) return;
    const bool solo = batch.size() == 1 && (batch[0]->solo || batch[0]->tiny_run);
    for (Request* r : batch) r->state = kRunning;
    reserved[li] = est;
    ++running;
    if (solo) solo_running = true;
    lk.unlock();

    std::vector<Job> jobs(batch.size());
    std::vector<Job*> ptrs(batch.size());
    for (size_t i = 0; i < batch.size(); ++i) {
      const rtg_query& q = batch[i]->q;
      jobs[i] = Job{q.points, q.n,       q.d,           q.r,  q.alpha, q.k, q.flags,
                    batch[i]->R.data(), batch[i]->u.data(), &batch[i]->out, batch[i]->ticket};
      ptrs[i] = &jobs[i];
    }
    rtg_stats st{};
    int rc = RTG_EDEVICE;
    if (!c.poisoned) {
      rc = Lane::kTinyFallback;
      if (batch.size() == 1 && batch[0]->tiny_run) {
        rc = L.run_tiny(jobs[0], st);
        if (rc == RTG_OK) c.served_small += 1;
      }
      if (rc == Lane::kTinyFallback) rc = L.run_batch(ptrs, st);
    }

    lk.lock();
    --running;
    reserved[li] = 0;
    if (solo) solo_running = false;
    // A request that ran alone on an idle device and still ran out of
    // memory: if other requests' points or finished results hold part of the
    // budget it waits for some of it to come back; only with nothing else
    // held is the budget too small for it.
    bool others_hold = false;
    if (rc == RTG_ENOMEM && solo) {
      others_hold = running > 0 || c.holds_results();
      for (Request* r : queue) others_hold = others_hold || r->pts_mem != nullptr;
    }
    if (rc != RTG_OK && rc != RTG_EDEVICE &&
        (batch.size() > 1 || (rc == RTG_ENOMEM && (!solo || others_hold)))) {
      // split: every query runs alone, in its original order, at the front
      for (size_t i = batch.size(); i-- > 0;) {
        batch[i]->state = kQueued;
        batch[i]->solo = true;
        if (solo) {
          batch[i]->waiting = true;
          batch[i]->wait_gen = gen;
        }
        queue.push_front(batch[i]);
      }
    } else {
      for (Request* r : batch) {
        r->state = kDone;
        r->rc = rc;
        c.dfree(r->pts_mem);
        r->pts_mem = nullptr;
      }
      ++gen;  // their staged points are back
      c.served_requests += (int64_t)batch.size();
      c.served_batches += 1;
    }
    cv.notify_all();
  }
}

// ---------------------------------------------------------------------------

int Ctx::submit(const rtg_query& q, uint64_t* ticket) {
  if (poisoned) return RTG_EDEVICE;
  int rc = check_query(q.points, q.n, q.d, q.r, q.k, q.alpha, q.flags);
  if (rc) return rc;
  Server* s = nullptr;
  {
    std::lock_guard<std::mutex> lk(server_mu);
    if (!server) {
      std::unique_ptr<Server> sv(new Server(*this));
      if ((rc = sv->start(server_lanes))) {
        sv->shutdown();
        return rc;
      }
      server = sv.release();
    }
    s = server;
  }
  return s->submit(q, ticket);
}

int Ctx::poll(uint64_t ticket, rtg_csr* out) {
  Server* s = nullptr;
  {
    std::lock_guard<std::mutex> lk(server_mu);
    s = server;
  }
  if (!s) return find_result(ticket, out) ? RTG_OK : RTG_ENOENT;
  return s->poll(ticket, out);
}

void Ctx::wake_server() {
  std::lock_guard<std::mutex> lk(server_mu);
  if (server) server->wake();
}

void Ctx::stop_server() {
  Server* s = nullptr;
  {
    std::lock_guard<std::mutex> lk(server_mu);
    s = server;
    server = nullptr;
  }
  if (!s) return;
  s->shutdown();
  delete s;
}

}  // namespace rtg

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
  return reinterpret_cast<Ctx*>(ctx)->submit(*q, ticket);
}

int rtg_poll(rtg_ctx* ctx, uint64_t ticket, rtg_csr* out) {
  if (!ctx || !out) return RTG_EINVAL;
  return reinterpret_cast<Ctx*>(ctx)->poll(ticket, out);
}

}  // extern "C"
