// Serving: clustering jobs arrive one by one (host buffers), a scheduler
// runs them on the GPU with continuous batching and reports latency.
//
//   * every job is validated at submit; a bad job fails alone;
//   * `slots` worker threads, each with its own HIP stream, context (device
//     arena, kept and reused) and device I/O buffers, take work from one FIFO
//     queue, so work of several jobs is on the device at once;
//   * continuous batching: a worker that takes a small job (n below
//     batch_cut) also takes every other queued small job, up to
//     batch_max_points / batch_max_jobs, and runs them as one batched call
//     (independent sets of one pass); large jobs run alone;
//   * admission: the budget bounds the device memory the slots hold, which
//     outlives the jobs (each slot keeps its arena and I/O buffers for the
//     next one).  A job (or batch) starts on a slot only if that slot's
//     memory after the job (grown, if needed, to the job's scratch, in the
//     batched layout for a batch, and I/O) fits next to what the other slots
//     hold; when it does not, idle slots give their memory back, and if it
//     still does not fit the job waits for running ones.  A job that could
//     never fit fails with DBSCAN_ETOOBIG;
//   * a batch that fails on a non-finite coordinate is re-run job by job so
//     only the offending job reports the error;
//   * latency = completion - submit; p50/p99 over completed jobs.
// A fake executor (no GPU: sleeps for a time proportional to the points)
// drives the same scheduler in CPU tests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dbscan_mi355x.h"

// what the server needs from a context (api.cpp)
namespace dbx {
uint64_t ctx_arena_bytes(const dbscan_ctx* c);
void ctx_set_budget(dbscan_ctx* c, uint64_t bytes);
int ctx_release_arena(dbscan_ctx* c);
uint64_t batched_scratch_bytes(int64_t n, uint32_t sets, bool any_core);
}  // namespace dbx

namespace {

using clock_t_ = std::chrono::steady_clock;

double now_s() {
  return std::chrono::duration<double>(clock_t_::now().time_since_epoch()).count();
}

struct Job {
  uint64_t ticket = 0;
  const float* pts = nullptr;
  int64_t n = 0;
  float eps = 0.f;
  int32_t min_pts = 0;
  int32_t* labels = nullptr;
  double t_submit = 0, t_done = 0;
  int status = 0;
  bool done = false;
};

struct Slot {
  dbscan_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  float* d_pts = nullptr;
  int32_t* d_lab = nullptr;
  size_t cap = 0;          // points the device I/O buffers hold
  uint64_t arena = 0;      // bytes of the context's arena
  uint64_t held = 0;       // device bytes charged to the slot (held, or reserved while busy)
  bool busy = false;
  uint64_t arena_cap = 0;  // the budget the next call's arena may grow to (0: none)
  size_t io_target = 0;    // points the I/O buffers grow to for the next call
  uint64_t arena_target = 0;  // the arena the next call will hold (fake executor)
  std::thread th;
};

}  // namespace

struct dbscan_server {
  dbscan_server_options opt{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
  uint64_t next_ticket = 1;
  uint64_t held_bytes = 0, peak_bytes = 0;  // device bytes the slots hold or have reserved
  int running = 0;
  bool stop = false;
  std::vector<std::unique_ptr<Slot>> slots;
  // statistics
  std::vector<double> latencies;
  uint64_t submitted = 0, completed = 0, failed = 0, points = 0, batches = 0, batched_jobs = 0;
  double first_submit = -1, last_done = 0;
};

namespace {

constexpr uint64_t IO_BYTES_PER_POINT = 16;  // points in (12) and labels out (4)

// Arena bytes of a job (one set) or a batch (several sets, batched layout).
uint64_t scratch_of(const std::vector<Job*>& b) {
  int64_t total = 0;
  bool any_core = false;
  for (Job* j : b) {
    total += j->n;
    any_core |= j->min_pts > 2;
  }
  if (b.size() == 1) return dbscan_scratch_bytes(total, b[0]->min_pts, DBSCAN_ALGO_FDBSCAN);
  return dbx::batched_scratch_bytes(total, uint32_t(b.size()), any_core);
}

// Bytes a buffer of `have` grows to for `need` within `limit` (0: none): 1/8
// headroom when that fits, else exactly `need`; unchanged if it holds it.
uint64_t grown(uint64_t have, uint64_t need, uint64_t limit) {
  if (need <= have) return have;
  const uint64_t want = need + need / 8;
  return limit && want > limit ? need : want;
}

// I/O buffers of at least n points (s->io_target when they grow).
int grow_io(Slot* s, size_t n) {
  if (n <= s->cap) return DBSCAN_OK;
  if (s->d_pts) (void)hipFree(s->d_pts);
  if (s->d_lab) (void)hipFree(s->d_lab);
  s->d_pts = nullptr;
  s->d_lab = nullptr;
  s->cap = 0;
  const size_t want = std::max(n, s->io_target);
  if (hipMalloc(&s->d_pts, want * 12) != hipSuccess || hipMalloc(&s->d_lab, want * 4) != hipSuccess) {
    (void)hipGetLastError();
    return DBSCAN_ENOMEM;
  }
  s->cap = want;
  return DBSCAN_OK;
}

// Give back an idle slot's device memory (lock held; the slot runs nothing).
void release(dbscan_server* S, Slot* s) {
  if (!S->opt.fake_executor) {
    if (s->ctx) (void)dbx::ctx_release_arena(s->ctx);
    if (s->d_pts) (void)hipFree(s->d_pts);
    if (s->d_lab) (void)hipFree(s->d_lab);
  }
  s->d_pts = nullptr;
  s->d_lab = nullptr;
  s->cap = 0;
  s->arena = 0;
  S->held_bytes -= s->held;
  s->held = 0;
}

enum class Admit { RUN, WAIT, NEVER };

// May slot s run a batch needing `scratch` arena bytes and `total` points of
// I/O now (lock held)?  On RUN the slot's charge is raised to what it will
// hold afterwards and s->arena_cap is the cap its arena may grow to.
Admit admit(dbscan_server* S, Slot* s, uint64_t scratch, int64_t total) {
  const uint64_t B = S->opt.hbm_budget_bytes;
  const uint64_t io_need = uint64_t(total) * IO_BYTES_PER_POINT;
  if (B && scratch + io_need > B) return Admit::NEVER;
  auto others = [&] { return S->held_bytes - s->held; };
  // what the slot holds afterwards, with no headroom: the least it can be
  auto least = [&] {
    return std::max(s->arena, scratch) + std::max(uint64_t(s->cap) * IO_BYTES_PER_POINT, io_need);
  };
  if (B && others() + least() > B) {
    for (auto& o : S->slots)  // idle slots give their memory back
      if (o.get() != s && !o->busy && o->held) release(S, o.get());
  }
  if (B && others() + least() > B) {
    bool others_busy = false;
    for (auto& o : S->slots) others_busy |= o.get() != s && o->busy;
    if (others_busy) return Admit::WAIT;
    release(S, s);  // alone on the device: start from nothing
    if (others() + least() > B) return Admit::WAIT;  // cannot happen: checked above
  }
  // within what is left, the arena grows with headroom where it fits, then the I/O
  const uint64_t room = B ? B - others() : 0;
  const uint64_t io_after = std::max(uint64_t(s->cap) * IO_BYTES_PER_POINT, io_need);
  const uint64_t arena_after = grown(s->arena, scratch, B ? room - io_after : 0);
  const uint64_t io_final = grown(uint64_t(s->cap) * IO_BYTES_PER_POINT, io_need,
                                  B ? room - arena_after : 0);
  s->arena_cap = B ? room - io_final : 0;
  s->arena_target = arena_after;
  s->io_target = size_t(io_final / IO_BYTES_PER_POINT);
  S->held_bytes += arena_after + io_final - s->held;
  s->held = arena_after + io_final;
  S->peak_bytes = std::max(S->peak_bytes, S->held_bytes);
  return Admit::RUN;
}

// Runs a batch (one job = a plain call) on the slot's stream; fills each
// job's status.  Host buffers are copied in and out on the same stream.
void execute(dbscan_server* S, Slot* s, std::vector<Job*>& batch) {
  int64_t total = 0;
  for (Job* j : batch) total += j->n;
  if (S->opt.fake_executor) {  // holds what a real run would hold, allocates nothing
    const double us = S->opt.fake_us_per_mpoint * double(total) / 1e6 + 1.0;
    std::this_thread::sleep_for(std::chrono::duration<double, std::micro>(us));
    for (Job* j : batch) {
      for (int64_t i = 0; i < j->n; ++i) j->labels[i] = -1;
      j->status = DBSCAN_OK;
    }
    s->arena = std::max(s->arena, s->arena_target);
    s->cap = std::max(s->cap, std::max(size_t(total), s->io_target));
    return;
  }
  dbx::ctx_set_budget(s->ctx, s->arena_cap);
  int st = grow_io(s, size_t(total));
  if (st == DBSCAN_OK) {
    int64_t o = 0;
    for (Job* j : batch) {
      if (j->n && hipMemcpyAsync(s->d_pts + 3 * o, j->pts, size_t(j->n) * 12,
                                 hipMemcpyHostToDevice, s->stream) != hipSuccess)
        st = DBSCAN_EDEVICE;
      o += j->n;
    }
  }
  if (st == DBSCAN_OK) {
    dbscan_options opt{};
    opt.algorithm = DBSCAN_ALGO_FDBSCAN;
    if (batch.size() == 1) {
      Job* j = batch[0];
      st = dbscan_cluster_ex(s->ctx, s->d_pts, j->n, j->eps, j->min_pts, s->d_lab, s->stream, &opt);
    } else {
      std::vector<int64_t> off(batch.size() + 1, 0);
      std::vector<float> eps(batch.size());
      std::vector<int32_t> mp(batch.size());
      for (size_t k = 0; k < batch.size(); ++k) {
        off[k + 1] = off[k] + batch[k]->n;
        eps[k] = batch[k]->eps;
        mp[k] = batch[k]->min_pts;
      }
      st = dbscan_cluster_batched(s->ctx, s->d_pts, off.data(), int32_t(batch.size()), eps.data(),
                                  mp.data(), s->d_lab, s->stream, &opt);
    }
  }
  if (st == DBSCAN_OK) {
    int64_t o = 0;
    for (Job* j : batch) {
      if (j->n && hipMemcpyAsync(j->labels, s->d_lab + o, size_t(j->n) * 4,
                                 hipMemcpyDeviceToHost, s->stream) != hipSuccess)
        st = DBSCAN_EDEVICE;
      o += j->n;
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess) st = DBSCAN_EDEVICE;
  }
  s->arena = dbx::ctx_arena_bytes(s->ctx);
  if (st == DBSCAN_ENONFINITE && batch.size() > 1) {
    // isolate the offending job(s): run the batch again one job at a time
    // (each needs less than the batch, which the slot already holds)
    for (Job* j : batch) {
      std::vector<Job*> one{j};
      execute(S, s, one);
    }
    return;
  }
  for (Job* j : batch) j->status = st;
}

// The batch a slot takes: the queue's head, plus (if it is small) every
// other queued small job within the batch limits (lock held).
std::vector<Job*> take_batch(dbscan_server* S) {
  std::vector<Job*> batch;
  Job* head = S->queue.front();
  S->queue.pop_front();
  batch.push_back(head);
  int64_t total = head->n;
  bool any_core = head->min_pts > 2;
  const uint64_t B = S->opt.hbm_budget_bytes;
  if (head->n < S->opt.batch_cut) {
    for (auto it = S->queue.begin(); it != S->queue.end();) {
      Job* j = *it;
      const int64_t t2 = total + j->n;
      const bool c2 = any_core || j->min_pts > 2;
      // a batch that could never fit the budget is not formed
      const bool fits = !B || dbx::batched_scratch_bytes(t2, uint32_t(batch.size() + 1), c2) +
                                      uint64_t(t2) * IO_BYTES_PER_POINT <= B;
      if (j->n < S->opt.batch_cut && t2 <= S->opt.batch_max_points &&
          int32_t(batch.size()) < S->opt.batch_max_jobs && fits) {
        batch.push_back(j);
        total = t2;
        any_core = c2;
        it = S->queue.erase(it);
      } else {
        ++it;
      }
    }
  }
  return batch;
}

void finish_job(dbscan_server* S, Job* j, double t) {
  j->t_done = t;
  j->done = true;
  if (j->status == DBSCAN_OK) {
    ++S->completed;
    S->points += uint64_t(j->n);
    S->latencies.push_back(t - j->t_submit);
    S->last_done = std::max(S->last_done, t);
  } else {
    ++S->failed;
  }
}

void worker(dbscan_server* S, Slot* s) {
  if (!S->opt.fake_executor) (void)hipSetDevice(S->opt.device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
    if (S->queue.empty()) {
      if (S->stop) return;
      continue;
    }
    std::vector<Job*> batch = take_batch(S);
    int64_t total = 0;
    for (Job* j : batch) total += j->n;
    Admit a = admit(S, s, scratch_of(batch), total);
    if (a == Admit::NEVER && batch.size() > 1) {
      // the batch is too big for the budget: its jobs go back to run alone
      for (auto it = batch.rbegin(); it != batch.rend(); ++it) S->queue.push_front(*it);
      S->cv_work.notify_all();
      batch.resize(1);
      S->queue.pop_front();
      total = batch[0]->n;
      a = admit(S, s, scratch_of(batch), total);
    }
    if (a == Admit::NEVER) {  // a job that can never fit
      batch[0]->status = DBSCAN_ETOOBIG;
      finish_job(S, batch[0], now_s());
      S->cv_done.notify_all();
      continue;
    }
    if (a == Admit::WAIT) {  // back to the head of the queue until a running job ends
      for (auto it = batch.rbegin(); it != batch.rend(); ++it) S->queue.push_front(*it);
      S->cv_work.wait(lk);
      continue;
    }
    s->busy = true;
    ++S->running;
    if (batch.size() > 1) {
      ++S->batches;
      S->batched_jobs += batch.size();
    }
    lk.unlock();
    execute(S, s, batch);
    const double t = now_s();
    lk.lock();
    // charge what the slot holds now
    const uint64_t held = s->arena + uint64_t(s->cap) * IO_BYTES_PER_POINT;
    S->held_bytes = S->held_bytes - s->held + held;
    s->held = held;
    S->peak_bytes = std::max(S->peak_bytes, S->held_bytes);
    s->busy = false;
    --S->running;
    for (Job* j : batch) finish_job(S, j, t);
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0;
  std::sort(v.begin(), v.end());
  const double pos = q * double(v.size() - 1);
  const size_t a = size_t(pos);
  const size_t b = std::min(a + 1, v.size() - 1);
  return v[a] + (v[b] - v[a]) * (pos - double(a));
}

}  // namespace

extern "C" {

int dbscan_server_create(const dbscan_server_options* opts, dbscan_server** out) {
  if (!out) return DBSCAN_EINVAL;
  auto S = std::make_unique<dbscan_server>();
  if (opts) S->opt = *opts;
  dbscan_server_options& o = S->opt;
  if (o.slots <= 0) o.slots = 4;
  if (o.slots > 64) return DBSCAN_EINVAL;
  if (o.batch_cut <= 0) o.batch_cut = 1 << 18;
  if (o.batch_max_points <= 0) o.batch_max_points = 1 << 24;
  if (o.batch_max_jobs <= 0) o.batch_max_jobs = 1024;
  if (!o.fake_executor) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || o.device < 0 || o.device >= count)
      return DBSCAN_EINVAL;
    if (hipSetDevice(o.device) != hipSuccess) return DBSCAN_EDEVICE;
  }
  for (int k = 0; k < o.slots; ++k) {
    auto s = std::make_unique<Slot>();
    if (!o.fake_executor) {
      if (dbscan_ctx_create(o.device, 0, &s->ctx) != DBSCAN_OK) return DBSCAN_EDEVICE;
      if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
        return DBSCAN_EDEVICE;
    }
    S->slots.push_back(std::move(s));
  }
  dbscan_server* raw = S.release();
  for (auto& s : raw->slots) s->th = std::thread(worker, raw, s.get());
  *out = raw;
  return DBSCAN_OK;
}

int dbscan_server_submit(dbscan_server* S, const float* host_pts, int64_t n, float eps,
                         int32_t min_pts, int32_t* host_labels, uint64_t* ticket) {
  if (!S || !ticket) return DBSCAN_EINVAL;
  if (n < 0 || n >= (int64_t(1) << 30)) return DBSCAN_EINVAL;
  if (n > 0 && (!host_pts || !host_labels)) return DBSCAN_EINVAL;
  if (!(eps >= 0.0f) || std::isinf(eps) || std::isinf(eps * eps) || min_pts < 1)
    return DBSCAN_EINVAL;
  auto j = std::make_unique<Job>();
  j->pts = host_pts;
  j->n = n;
  j->eps = eps;
  j->min_pts = min_pts;
  j->labels = host_labels;
  j->t_submit = now_s();
  std::lock_guard<std::mutex> g(S->mu);
  j->ticket = S->next_ticket++;
  *ticket = j->ticket;
  ++S->submitted;
  if (S->first_submit < 0) S->first_submit = j->t_submit;
  Job* raw = j.get();
  S->jobs.emplace(raw->ticket, std::move(j));
  if (n == 0) {
    raw->done = true;
    raw->t_done = raw->t_submit;
    ++S->completed;
    S->latencies.push_back(0.0);
  } else {
    S->queue.push_back(raw);
    S->cv_work.notify_one();
  }
  return DBSCAN_OK;
}

int dbscan_server_poll(dbscan_server* S, uint64_t ticket, int32_t* job_status) {
  if (!S) return DBSCAN_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return DBSCAN_EINVAL;
  if (!it->second->done) return 0;
  if (job_status) *job_status = it->second->status;
  return 1;
}

int dbscan_server_wait(dbscan_server* S, uint64_t ticket, double timeout_s, int32_t* job_status) {
  if (!S) return DBSCAN_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return DBSCAN_EINVAL;
  Job* j = it->second.get();
  const auto pred = [&] { return j->done; };
  if (timeout_s < 0) S->cv_done.wait(lk, pred);
  else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return 0;
  if (job_status) *job_status = j->status;
  return 1;
}

int dbscan_server_job_times(dbscan_server* S, uint64_t ticket, double* submit_s, double* done_s) {
  if (!S) return DBSCAN_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end() || !it->second->done) return DBSCAN_EINVAL;
  if (submit_s) *submit_s = it->second->t_submit;
  if (done_s) *done_s = it->second->t_done;
  return DBSCAN_OK;
}

int dbscan_server_stats(dbscan_server* S, dbscan_serving_stats* out) {
  if (!S || !out) return DBSCAN_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  dbscan_serving_stats r{};
  r.submitted = S->submitted;
  r.completed = S->completed;
  r.failed = S->failed;
  r.points = S->points;
  r.batches = S->batches;
  r.batched_jobs = S->batched_jobs;
  r.peak_in_flight_bytes = S->peak_bytes;
  r.p50_ms = percentile(S->latencies, 0.50) * 1e3;
  r.p99_ms = percentile(S->latencies, 0.99) * 1e3;
  double sum = 0, mx = 0;
  for (double v : S->latencies) { sum += v; mx = std::max(mx, v); }
  r.mean_ms = S->latencies.empty() ? 0 : sum / double(S->latencies.size()) * 1e3;
  r.max_ms = mx * 1e3;
  const double span = S->last_done - S->first_submit;
  r.mpoints_per_s = span > 0 ? double(S->points) / span / 1e6 : 0;
  *out = r;
  return DBSCAN_OK;
}

int dbscan_server_destroy(dbscan_server* S) {
  if (!S) return DBSCAN_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& s : S->slots)
    if (s->th.joinable()) s->th.join();
  for (auto& s : S->slots) {
    if (s->d_pts) (void)hipFree(s->d_pts);
    if (s->d_lab) (void)hipFree(s->d_lab);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->ctx) dbscan_ctx_destroy(s->ctx);
  }
  delete S;
  return DBSCAN_OK;
}

}  // extern "C"
