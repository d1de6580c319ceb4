// Serving loop: continuous batching of convolution requests.
//
// Requests name a resident table and bring their own PDF batch.  A scheduler
// thread admits queued requests whenever a stream lane and request slots are
// free: all queued requests on the same table that fit the lane's staging
// memory are coalesced into one pass over the table (their replica columns
// are concatenated, the GPU may only pay off for a large enough batch per
// Section 3-4), and passes run concurrently on the lanes' streams, several
// on one table if its requests keep arriving.  Each lane runs a table's
// passes with scratch memory of its own (a copy of the table's plan that
// shares the table and descriptors), so passes never share scratch with one
// another or with direct calls.  Every output column is computed by the
// same arithmetic whatever the other columns of its pass are, so a
// request's result does not depend on the mix it was served in.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include <memory>

#include "runtime.h"

using namespace fk;

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Ticket {
  fk_request req;
  int64_t table = 0;  // resolved (fallback applied)
  int state = FK_QUEUED;
  uint64_t t_submit = 0, t_admit = 0, t_done = 0;
  size_t need = 0;    // staging bytes for this request alone
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void *arena = nullptr;
  size_t bytes = 0;
  bool busy = false;
  int64_t table = 0;
  std::vector<int64_t> tickets;
  // the lane's copies of the table plans it has run, with private scratch
  std::unordered_map<int64_t, std::unique_ptr<Plan>> plans;
};

constexpr size_t kKeepDone = 65536;  // finished ticket records kept

}  // namespace

struct fk_serve {
  fk_ctx *ctx = nullptr;
  int nslots = 0;
  std::vector<Lane> lanes;
  std::vector<std::pair<void *, size_t>> allocs;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  std::deque<int64_t> queue;
  std::unordered_map<int64_t, Ticket> tickets;
  std::deque<int64_t> finished;  // finished tickets, oldest first
  int64_t next = 1;
  int inflight = 0;
  size_t max_queue = 1 << 20;

  void loop();
  bool dispatch(Lane &lane);
  void complete(Lane &lane, bool ok);
};

void fk_serve::complete(Lane &lane, bool ok) {
  const uint64_t t = now_ns();
  {
    std::lock_guard<std::mutex> lk(mu);
    for (int64_t id : lane.tickets) {
      auto it = tickets.find(id);
      if (it == tickets.end()) continue;
      it->second.state = ok ? FK_DONE : FK_FAILED;
      it->second.t_done = t;
      finished.push_back(id);
    }
    inflight -= (int)lane.tickets.size();
    while (finished.size() > kKeepDone) {
      tickets.erase(finished.front());
      finished.pop_front();
    }
  }
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (Table *tb = find_table(ctx, lane.table)) tb->busy--;
  }
  lane.tickets.clear();
  lane.busy = false;
}

// Pick the oldest queued request and coalesce the queued requests on its
// table into one pass on ``lane``.  Returns true if a pass started (or a
// request was failed).
bool fk_serve::dispatch(Lane &lane) {
  std::vector<Ticket *> batch;
  std::vector<int64_t> ids;
  int64_t table = 0;
  Plan *plan = nullptr;
  Table *tab = nullptr;
  size_t rtot = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (queue.empty() || inflight >= nslots) return false;
    std::lock_guard<std::mutex> lk2(ctx->mu);
    const int64_t id0 = queue.front();
    Ticket &t0 = tickets[id0];
    Table *tb = find_table(ctx, t0.table);
    Plan *pl = tb ? find_plan(ctx, t0.table) : nullptr;
    auto fail_front = [&]() {
      t0.state = FK_FAILED;
      t0.t_done = now_ns();
      finished.push_back(id0);
      queue.pop_front();
      return true;
    };
    if (!tb || !pl) return fail_front();  // unloaded behind our back
    auto &mine = lane.plans[t0.table];
    if (!mine) {
      auto q = std::make_unique<Plan>();
      if (clone_forward_scratch(ctx, *pl, *q, &allocs) != FK_OK) {
        lane.plans.erase(t0.table);
        return fail_front();
      }
      mine = std::move(q);
    }
    table = t0.table;
    tab = tb;
    plan = mine.get();
    const size_t per_col = ((size_t)tab->F * tab->X + (size_t)tab->N) * sizeof(float);
    for (auto qi = queue.begin(); qi != queue.end();) {
      Ticket &t = tickets[*qi];
      if (t.table != table) {
        ++qi;
        continue;
      }
      if (inflight + (int)batch.size() >= nslots) break;
      if ((rtot + t.req.nrep) * per_col > lane.bytes) break;
      rtot += t.req.nrep;
      batch.push_back(&t);
      ids.push_back(*qi);
      qi = queue.erase(qi);
    }
    if (batch.empty()) return false;
    const uint64_t t = now_ns();
    for (Ticket *b : batch) {
      b->state = FK_RUNNING;
      b->t_admit = t;
    }
    inflight += (int)batch.size();
    tab->busy++;
  }
  // enqueue: wait for the producers of the PDFs, gather the PDF columns,
  // one pass, scatter the outputs
  const int F = tab->F, X = tab->X, N = tab->N;
  float *pdf = (float *)lane.arena;
  float *out = pdf + (size_t)F * X * rtot;
  hipError_t e = hipSuccess;
  for (Ticket *b : batch)
    if (e == hipSuccess && b->req.ready)
      e = hipStreamWaitEvent(lane.stream, (hipEvent_t)b->req.ready, 0);
  size_t col = 0;
  for (Ticket *b : batch) {
    const size_t w = (size_t)b->req.nrep * sizeof(float);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(pdf + col, rtot * sizeof(float), b->req.pdf, w, w, (size_t)F * X,
                           hipMemcpyDeviceToDevice, lane.stream);
    col += b->req.nrep;
  }
  if (e == hipSuccess) e = run_forward(*plan, pdf, (int)rtot, out, lane.stream, nullptr, ctx->kernels.load());
  col = 0;
  for (Ticket *b : batch) {
    const size_t w = (size_t)b->req.nrep * sizeof(float);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(b->req.out, w, out + col, rtot * sizeof(float), w, (size_t)N,
                           hipMemcpyDeviceToDevice, lane.stream);
    col += b->req.nrep;
  }
  if (e == hipSuccess) e = hipEventRecord(lane.done, lane.stream);
  lane.table = table;
  lane.tickets = ids;
  lane.busy = true;
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(lane.stream);
    complete(lane, false);
  }
  return true;
}

void fk_serve::loop() {
  (void)hipSetDevice(ctx->device);
  for (;;) {
    bool active = false;
    for (auto &lane : lanes) {
      if (!lane.busy) continue;
      active = true;
      const hipError_t q = hipEventQuery(lane.done);
      if (q == hipSuccess)
        complete(lane, true);
      else if (q != hipErrorNotReady)
        complete(lane, false);
    }
    bool started = false;
    for (auto &lane : lanes)
      if (!lane.busy && dispatch(lane)) started = true;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stop && queue.empty() && inflight == 0) break;
      if (!started && !active) {
        cv.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
    }
    if (!started) std::this_thread::yield();
  }
}

extern "C" {

fk_status fk_serve_start(fk_ctx *ctx, int32_t nslots, int32_t nstreams,
                         uint64_t request_budget_bytes) {
  if (!ctx) return FK_E_ARG;
  if (nslots < 1 || nstreams < 1 || nstreams > 64 || request_budget_bytes < 4096)
    return set_err(ctx, FK_E_ARG, "fk_serve_start: need nslots>=1, 1<=nstreams<=64, budget>=4096");
  if (ctx->serve) return set_err(ctx, FK_E_STATE, "fk_serve_start: already serving");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, FK_E_HIP, "hipSetDevice failed");
  auto *s = new fk_serve();
  s->ctx = ctx;
  s->nslots = nslots;
  s->lanes.resize(nstreams);
  const size_t per = (size_t)(request_budget_bytes / nstreams) / 256 * 256;
  for (auto &lane : s->lanes) {
    fk_status st = dev_alloc(ctx, per, &lane.arena, &s->allocs);
    hipError_t e = hipSuccess;
    if (st == FK_OK) e = hipStreamCreateWithFlags(&lane.stream, hipStreamNonBlocking);
    if (st == FK_OK && e == hipSuccess) e = hipEventCreateWithFlags(&lane.done, hipEventDisableTiming);
    if (st != FK_OK || e != hipSuccess) {
      for (auto &l : s->lanes) {
        if (l.stream) (void)hipStreamDestroy(l.stream);
        if (l.done) (void)hipEventDestroy(l.done);
      }
      dev_free_all(ctx, s->allocs);
      delete s;
      return st != FK_OK ? st : set_err(ctx, FK_E_HIP, "fk_serve_start: %s", hipGetErrorString(e));
    }
    lane.bytes = per;
  }
  ctx->serve = s;
  s->th = std::thread([s]() { s->loop(); });
  return FK_OK;
}

fk_status fk_serve_stop(fk_ctx *ctx) {
  if (!ctx) return FK_E_ARG;
  fk_serve *s = ctx->serve;
  if (!s) return FK_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  s->th.join();
  (void)hipSetDevice(ctx->device);
  for (auto &l : s->lanes) {
    (void)hipStreamSynchronize(l.stream);
    (void)hipStreamDestroy(l.stream);
    (void)hipEventDestroy(l.done);
  }
  dev_free_all(ctx, s->allocs);
  ctx->serve = nullptr;
  delete s;
  return FK_OK;
}

fk_status fk_table_set_fallback(fk_ctx *ctx, fk_table table, fk_table fallback) {
  if (!ctx) return FK_E_ARG;
  std::lock_guard<std::mutex> lk(ctx->mu);
  Table *t = find_table(ctx, table);
  Table *f = fallback ? find_table(ctx, fallback) : nullptr;
  if (!t || (fallback && !f))
    return set_err(ctx, FK_E_HANDLE, "fk_table_set_fallback: unknown table handle");
  if (f && (f->kind != t->kind || f->N != t->N || f->F != t->F || f->X != t->X))
    return set_err(ctx, FK_E_SHAPE, "fk_table_set_fallback: fallback has a different shape");
  t->fallback = fallback;
  return FK_OK;
}

fk_status fk_submit(fk_ctx *ctx, const fk_request *req, fk_ticket *out) {
  if (!ctx) return FK_E_ARG;
  if (!req || !out) return set_err(ctx, FK_E_ARG, "fk_submit: NULL argument");
  *out = 0;
  fk_serve *s = ctx->serve;
  if (!s) return set_err(ctx, FK_E_STATE, "fk_submit: serving loop not started");
  if (req->nrep < 1 || !req->pdf || !req->out)
    return set_err(ctx, FK_E_ARG, "fk_submit: need nrep>=1 and non-NULL pdf/out");
  Ticket t;
  t.req = *req;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    Table *tb = find_table(ctx, req->table);
    if (!tb) return set_err(ctx, FK_E_HANDLE, "fk_submit: %lld is not a loaded table", (long long)req->table);
    t.table = req->table;
    if (tb->fallback && tb->dtype != FK_F32 && (req->precision == FK_F32 || tb->route_fallback))
      t.table = tb->fallback;
    t.need = ((size_t)tb->F * tb->X + (size_t)tb->N) * sizeof(float) * (size_t)req->nrep;
  }
  if (t.need > s->lanes[0].bytes)
    return set_err(ctx, FK_E_TOO_LARGE, "fk_submit: request needs %llu staging bytes, a lane has %llu",
                   (unsigned long long)t.need, (unsigned long long)s->lanes[0].bytes);
  t.t_submit = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->queue.size() >= s->max_queue) return set_err(ctx, FK_E_QUEUE_FULL, "fk_submit: queue full");
    const int64_t id = s->next++;
    s->tickets[id] = t;
    s->queue.push_back(id);
    *out = id;
  }
  s->cv.notify_one();
  return FK_OK;
}

fk_status fk_poll(fk_ctx *ctx, fk_ticket ticket, int32_t *state) {
  if (!ctx || !state) return FK_E_ARG;
  fk_serve *s = ctx->serve;
  if (!s) return set_err(ctx, FK_E_STATE, "fk_poll: serving loop not started");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return set_err(ctx, FK_E_HANDLE, "fk_poll: unknown ticket");
  *state = it->second.state;
  return FK_OK;
}

fk_status fk_ticket_times(fk_ctx *ctx, fk_ticket ticket, uint64_t *t_submit, uint64_t *t_admit,
                          uint64_t *t_done) {
  if (!ctx) return FK_E_ARG;
  fk_serve *s = ctx->serve;
  if (!s) return set_err(ctx, FK_E_STATE, "fk_ticket_times: serving loop not started");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return set_err(ctx, FK_E_HANDLE, "fk_ticket_times: unknown ticket");
  if (t_submit) *t_submit = it->second.t_submit;
  if (t_admit) *t_admit = it->second.t_admit;
  if (t_done) *t_done = it->second.t_done;
  return FK_OK;
}

}  // extern "C"
