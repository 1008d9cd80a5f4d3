// Serving loop: a persistent pool of solve slots fed from a FIFO of requests.
//
// Each slot owns a library context (its device buffers stay resident between
// requests) and a HIP stream, and is driven by its own host thread; a request
// is admitted to a free slot as soon as the device memory of all slots (the
// buffers each one holds, or the estimated footprint of the request it runs)
// leaves room for it, and so does the sum of the work in flight (grid nodes
// plus targets).  A slot whose resident buffers push the total over the
// budget after a request releases them.  Requests that arrive while
// others are running therefore start immediately and their kernels overlap on
// the GPU with the others'; the work bound stops several large requests from
// dividing the GPU between them, which would stretch each one's latency.  A
// request's result does not depend on which slot ran it or on what ran beside
// it: every slot runs the same deterministic kernels on its own buffers.
//
// Fused launches: a slot that admits the head of the queue also takes later
// queued requests of the same shape (device inputs and outputs, multipole
// method) while the bounds allow, and solves them as one forest with
// pp_solve_grid_batch: one set of launches, each result still bitwise the
// request's lone solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pp.h"
#include "internal.h"

namespace {

using clk = std::chrono::steady_clock;

struct Job {
  uint64_t ticket = 0;
  pp_request req{};
  bool device_io = false;  // every input and the output in device memory (may join a batch)
  std::vector<double> f_copy, tx_copy, ty_copy;  // host inputs copied at submission
  uint64_t footprint = 0;
  uint64_t work = 0;
  clk::time_point t_submit, t_start, t_end;
  int slot = -1;
  pp_status status = PP_OK;
  bool done = false;
  bool cancelled = false;
  std::string err;
};

bool host_memory(const void* p) {
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return true;
  }
  return !(a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged);
}

// A request pp_solve_grid_batch takes (device inputs and output, the
// multipole method, 33 to 16384 nodes a side), and requests it can solve
// together (one shape).
bool batchable(const Job& j) {
  const int n = std::max(j.req.nx, j.req.ny);
  return j.device_io && j.req.params.method == PP_METHOD_FMM && n >= 33 && n <= 16384;
}
bool same_shape(const pp_request& a, const pp_request& b) {
  const pp_params &p = a.params, &q = b.params;
  return a.nx == b.nx && a.ny == b.ny && a.x0 == b.x0 && a.y0 == b.y0 && a.h == b.h && p.p == q.p &&
         p.theta == q.theta && p.leaf_max == q.leaf_max && p.precision == q.precision && p.self_mode == q.self_mode &&
         p.method == q.method;
}

}  // namespace

struct pp_server {
  pp_server_cfg cfg{};
  clk::time_point t0 = clk::now();
  std::mutex mu;
  std::condition_variable cv_work;  // workers: queue changed or memory freed
  std::condition_variable cv_done;  // waiters: a job finished
  std::deque<std::shared_ptr<Job>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
  uint64_t next_ticket = 1;
  uint64_t inflight_bytes = 0;
  uint64_t inflight_work = 0;
  int inflight = 0;
  bool stopping = false;
  std::vector<std::thread> workers;
  std::vector<pp_ctx*> ctxs;
  std::vector<hipStream_t> streams;
  // device bytes each slot's context holds between requests (its buffers stay
  // resident), and the footprint of the request a slot is running (0 = idle)
  std::vector<uint64_t> held;
  std::vector<uint64_t> running_fp;
  std::string err;
};

extern "C" uint64_t pp_footprint_estimate(int32_t nx, int32_t ny, int64_t m, int32_t p, int32_t leaf_max) {
  if (nx < 1 || ny < 1 || m < 0 || p < 1 || leaf_max < 1) return 0;
  const uint64_t g = (uint64_t)nx * (uint64_t)ny;
  int k = 0;
  while ((1 << k) < std::max(nx, ny)) ++k;
  // per grid node: f staging, key, packed index, weight, three FP32 record planes, ingest tiles
  const uint64_t src = g * (8 + 4 + 4 + 8 + 12 + 1);
  // per target: coordinates, keys/permutations (x2), offsets, leaf, self data, far, near parts, output
  const uint64_t tgt = (uint64_t)m * (16 + 16 + 8 + 16 + 4 + 4 + 8 + 8 + 8 * 8 + 8);
  // cells: bounded by the tree capacity; arrays, records, expansions, lists
  const uint64_t cells = std::min<uint64_t>(((uint64_t)1 << (2 * k + 2)) / 3 + 1,
                                            1 + 4 * (uint64_t)std::max(k, 1) * ((g + m) / (leaf_max + 1) + 1));
  const uint64_t cell = cells * (uint64_t)(15 * 4 + 16 + 4 * 16 + 3 * 16 * (p + 1) + 64 * 4 + 27 * 4);
  return src + tgt + cell + (64u << 10);
}

namespace {

void worker_loop(pp_server* s, int slot) {
  (void)hipSetDevice(s->cfg.device);
  pp_ctx* ctx = s->ctxs[slot];
  hipStream_t stream = s->streams[slot];
  std::vector<std::shared_ptr<Job>> batch;  // the head, then the requests solved with it
  for (;;) {
    std::shared_ptr<Job> job;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] {
        if (s->stopping && s->queue.empty()) return true;
        if (s->queue.empty()) return false;
        const Job& head = *s->queue.front();
        // FIFO admission: the head runs when the memory and work bounds leave
        // room for it (always when nothing else is in flight)
        if (s->inflight == 0) return true;
        // device memory once the head runs here: every other slot's resident
        // buffers (or its running request's footprint, if larger) plus this
        // slot's buffers grown to the head's footprint
        uint64_t resident = std::max(s->held[slot], head.footprint);
        for (int o = 0; o < (int)s->held.size(); ++o)
          if (o != slot) resident += std::max(s->held[o], s->running_fp[o]);
        const bool mem_ok = s->cfg.hbm_budget_bytes == 0 || resident <= s->cfg.hbm_budget_bytes;
        const bool work_ok =
            s->cfg.work_budget_points == 0 || s->inflight_work + head.work <= s->cfg.work_budget_points;
        return mem_ok && work_ok;
      });
      if (s->queue.empty()) return;  // stopping and drained
      job = s->queue.front();
      s->queue.pop_front();
      batch.assign(1, job);
      uint64_t fp = job->footprint;
      // fused launches: later queued requests of the head's shape join it (in
      // queue order) while the memory bound leaves room.  The batch is one
      // solve whose time grows far more slowly than its work (the launch
      // chain and its host round trips dominate at these sizes), so it counts
      // as the head's work for the work bound.
      if (s->cfg.max_batch > 1 && batchable(*job)) {
        uint64_t others = 0;
        for (int o = 0; o < (int)s->held.size(); ++o)
          if (o != slot) others += std::max(s->held[o], s->running_fp[o]);
        const int cap = std::min<int>(s->cfg.max_batch, pp::kMaxBatch);
        for (auto it = s->queue.begin(); it != s->queue.end() && (int)batch.size() < cap;) {
          const Job& o = **it;
          const bool fits_mem = s->cfg.hbm_budget_bytes == 0 ||
                                others + std::max(s->held[slot], fp + o.footprint) <= s->cfg.hbm_budget_bytes;
          if (batchable(o) && same_shape(o.req, job->req) && fits_mem) {
            fp += o.footprint;
            batch.push_back(*it);
            it = s->queue.erase(it);
          } else {
            ++it;
          }
        }
      }
      s->inflight += (int)batch.size();
      s->inflight_bytes += fp;
      s->inflight_work += job->work;
      s->running_fp[slot] = fp;
      const auto now = clk::now();
      for (auto& b : batch) {
        b->slot = slot;
        b->t_start = now;
      }
      // a request that starts alone on the GPU runs its near field on the
      // context's second stream; beside other requests it keeps one stream
      if (s->cfg.max_slots > 1) pp::ctx_set_near_stream(ctx, s->inflight == (int)batch.size());
    }
    std::vector<pp_status> sts(batch.size(), PP_OK);
    std::vector<std::string> errs(batch.size());
    auto solve_one = [&](size_t i) {
      const Job& jb = *batch[i];
      const pp_request& r = jb.req;
      const double* f = jb.f_copy.empty() ? r.f : jb.f_copy.data();
      const double* tx = jb.tx_copy.empty() ? r.tx : jb.tx_copy.data();
      const double* ty = jb.ty_copy.empty() ? r.ty : jb.ty_copy.data();
      sts[i] = pp_solve_grid(ctx, r.nx, r.ny, r.x0, r.y0, r.h, f, r.m, tx, ty, &r.params, r.p_out, (void*)stream);
      if (sts[i] != PP_OK) errs[i] = pp_last_error(ctx);
    };
    if (batch.size() == 1) {
      solve_one(0);
    } else {
      const int n = (int)batch.size();
      std::vector<const double*> fs(n), txs(n), tys(n);
      std::vector<double*> outs(n);
      std::vector<int64_t> ms(n);
      for (int i = 0; i < n; ++i) {
        const pp_request& r = batch[i]->req;
        fs[i] = r.f;
        txs[i] = r.tx;
        tys[i] = r.ty;
        outs[i] = r.p_out;
        ms[i] = r.m;
      }
      const pp_request& r0 = batch[0]->req;
      const pp_status st = pp_solve_grid_batch(ctx, n, r0.nx, r0.ny, r0.x0, r0.y0, r0.h, fs.data(), ms.data(),
                                               txs.data(), tys.data(), &r0.params, outs.data(), (void*)stream);
      if (st != PP_OK && st != PP_ERR_DEVICE) {
        for (int i = 0; i < n; ++i) solve_one(i);  // each request gets its own status
      } else if (st != PP_OK) {
        for (int i = 0; i < n; ++i) {
          sts[i] = st;
          errs[i] = pp_last_error(ctx);
        }
      }
    }
    pp_status st = PP_OK;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      const auto now = clk::now();
      for (size_t i = 0; i < batch.size(); ++i) {
        Job& jb = *batch[i];
        jb.status = sts[i];
        if (sts[i] != PP_OK) jb.err = errs[i];
        if (sts[i] == PP_ERR_DEVICE) st = PP_ERR_DEVICE;
        jb.t_end = now;
        jb.done = true;
        jb.f_copy.clear();
        jb.f_copy.shrink_to_fit();
        jb.tx_copy.clear();
        jb.tx_copy.shrink_to_fit();
        jb.ty_copy.clear();
        jb.ty_copy.shrink_to_fit();
        s->inflight -= 1;
        s->inflight_bytes -= jb.footprint;
      }
      s->inflight_work -= batch[0]->work;
      s->running_fp[slot] = 0;
      // a slot whose buffers push the resident total over the budget (after a
      // request larger than the others) gives them back
      s->held[slot] = pp::ctx_held_bytes(ctx);
      if (s->cfg.hbm_budget_bytes) {
        uint64_t total = 0;
        for (int o = 0; o < (int)s->held.size(); ++o) total += std::max(s->held[o], s->running_fp[o]);
        if (total > s->cfg.hbm_budget_bytes) {
          pp::ctx_trim(ctx);
          s->held[slot] = pp::ctx_held_bytes(ctx);
        }
      }
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
    if (st == PP_ERR_DEVICE) {
      // this slot's context is unusable; replace it so the slot keeps serving
      pp_destroy(ctx);
      ctx = nullptr;
      if (pp_create(s->cfg.device, 0, &ctx) != PP_OK) return;
      if (s->cfg.max_slots > 1) pp::ctx_set_near_stream(ctx, false);
      std::lock_guard<std::mutex> lk(s->mu);
      s->ctxs[slot] = ctx;
      s->held[slot] = 0;
    }
  }
}

}  // namespace

extern "C" {

pp_status pp_server_create(const pp_server_cfg* cfg, pp_server** out) {
  if (!cfg || !out || cfg->max_slots < 1 || cfg->max_slots > 64 || cfg->max_batch < 0 ||
      cfg->max_batch > pp::kMaxBatch)
    return PP_ERR_ARG;
  *out = nullptr;
  auto* s = new pp_server();
  s->cfg = *cfg;
  if (hipSetDevice(cfg->device) != hipSuccess) {
    delete s;
    return PP_ERR_DEVICE;
  }
  for (int i = 0; i < cfg->max_slots; ++i) {
    pp_ctx* c = nullptr;
    hipStream_t st = nullptr;
    if (pp_create(cfg->device, 0, &c) != PP_OK ||
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      if (c) pp_destroy(c);
      for (auto* x : s->ctxs) pp_destroy(x);
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return PP_ERR_DEVICE;
    }
    // with several slots the concurrency comes from the requests: each slot keeps
    // its whole solve on its own stream (a second stream per slot only adds
    // contention for the hardware queues)
    if (cfg->max_slots > 1) pp::ctx_set_near_stream(c, false);
    s->ctxs.push_back(c);
    s->streams.push_back(st);
    s->held.push_back(0);
    s->running_fp.push_back(0);
  }
  for (int i = 0; i < cfg->max_slots; ++i) s->workers.emplace_back(worker_loop, s, i);
  *out = s;
  return PP_OK;
}

pp_status pp_server_submit(pp_server* s, const pp_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return PP_ERR_ARG;
  if (r->m < 0 || r->nx < 1 || r->ny < 1 || !r->f || (r->m > 0 && (!r->tx || !r->ty || !r->p_out)))
    return PP_ERR_ARG;
  auto job = std::make_shared<Job>();
  job->req = *r;
  const int64_t ng = (int64_t)r->nx * r->ny;
  if (host_memory(r->f)) job->f_copy.assign(r->f, r->f + ng);
  if (r->m > 0 && host_memory(r->tx)) job->tx_copy.assign(r->tx, r->tx + r->m);
  if (r->m > 0 && host_memory(r->ty)) job->ty_copy.assign(r->ty, r->ty + r->m);
  job->device_io = job->f_copy.empty() && job->tx_copy.empty() && job->ty_copy.empty() && r->m > 0 &&
                   !host_memory(r->p_out);
  job->footprint = pp_footprint_estimate(r->nx, r->ny, r->m, r->params.p, r->params.leaf_max);
  job->work = (uint64_t)ng + (uint64_t)r->m;
  job->t_submit = clk::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return PP_ERR_ARG;
    job->ticket = s->next_ticket++;
    *ticket = job->ticket;
    s->jobs[job->ticket] = job;
    s->queue.push_back(job);
  }
  s->cv_work.notify_all();
  return PP_OK;
}

pp_status pp_server_wait(pp_server* s, uint64_t ticket, int64_t timeout_us, pp_ticket_info* info) {
  if (!s) return PP_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return PP_ERR_ARG;
  std::shared_ptr<Job> job = it->second;
  auto ready = [&] { return job->done; };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return PP_ERR_TIMEOUT;
  }
  if (info) {
    using us = std::chrono::duration<double, std::micro>;
    info->status = job->status;
    info->slot = job->slot;
    info->queue_us = us(job->t_start - job->t_submit).count();
    info->run_us = us(job->t_end - job->t_start).count();
    info->total_us = us(job->t_end - job->t_submit).count();
    info->start_us = us(job->t_start - s->t0).count();
    info->end_us = us(job->t_end - s->t0).count();
  }
  const pp_status st = job->status;
  if (st != PP_OK) s->err = job->err;
  s->jobs.erase(it);
  return st;
}

pp_status pp_server_cancel(pp_server* s, uint64_t ticket) {
  if (!s) return PP_ERR_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return PP_ERR_ARG;
    std::shared_ptr<Job> job = it->second;
    auto q = std::find(s->queue.begin(), s->queue.end(), job);
    if (q == s->queue.end()) return PP_ERR_BUSY;  // running or finished
    s->queue.erase(q);
    job->cancelled = true;
    job->done = true;
    job->status = PP_ERR_CANCELLED;
    job->err = "cancelled before it started";
    job->t_start = job->t_end = clk::now();
    job->f_copy.clear();
    job->tx_copy.clear();
    job->ty_copy.clear();
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();  // the next request may now be the head
  return PP_OK;
}

pp_status pp_server_destroy(pp_server* s) {
  if (!s) return PP_ERR_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv_work.notify_all();
  for (auto& w : s->workers) w.join();
  for (auto* c : s->ctxs)
    if (c) pp_destroy(c);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return PP_OK;
}

const char* pp_server_last_error(const pp_server* s) { return s ? s->err.c_str() : "null server"; }

uint64_t pp_server_device_bytes(pp_server* s) {
  if (!s) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  uint64_t total = 0;
  for (uint64_t b : s->held) total += b;
  return total;
}

}  // extern "C"
