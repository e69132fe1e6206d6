// Construction server: continuous batching of build requests under an HBM
// budget.
//
// One device pool of the budget's size holds the working memory of every
// build in flight.  Requests wait in arrival order; each slot (a host thread
// with its own stream) takes the oldest waiting requests that fit into a free
// region of the pool -- as many as fit, up to a per-launch limit -- builds
// them as one batch (one persistent search launch for all of them), and
// returns the region.  Slots run concurrently, so requests that arrive while
// others are on the GPU are admitted as soon as a slot and memory are free,
// and their kernels overlap with the ones already running.  Every result is
// the one rs_build makes of the request alone: the build does not depend on
// the schedule.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "rs_host.h"

using namespace rs;

namespace {

// A launch of at least this many keys counts as large (its search holds the
// whole device for milliseconds).
constexpr uint64_t kLargeLaunchKeys = 1ull << 20;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  rs_job job;
  size_t footprint = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int status = RS_PENDING;
  rs_mphf* out = nullptr;
  uint32_t slot = 0, batch_jobs = 0;
};

// First-fit allocator of byte ranges of the pool.
struct Regions {
  std::map<size_t, size_t> free;  // offset -> size
  size_t align = 4096;
  bool take(size_t bytes, size_t* off) {
    bytes = (bytes + align - 1) / align * align;
    for (auto it = free.begin(); it != free.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free.erase(it);
        if (rest) free[at] = rest;
        return true;
      }
    }
    return false;
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& f : free) m = f.second > m ? f.second : m;
    return m;
  }
  void give(size_t off, size_t bytes) {
    bytes = (bytes + align - 1) / align * align;
    auto it = free.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free.erase(nx);
    }
    if (it != free.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free.erase(it);
      }
    }
  }
};

}  // namespace

struct rs_server {
  Device* dev = nullptr;
  rs_server_config cfg{};
  char* pool = nullptr;
  Regions regions;
  std::vector<Context*> ctx;
  std::vector<std::thread> threads;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> waiting;
  std::map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  uint32_t workers_max = 0;
  uint32_t workers_cap = 0;      // search grid of a launch: the device minus the reserve
  uint32_t reserve_workers = 0;  // the reserve (reserve_per_cu workers on every CU)
  uint32_t large_running = 0;  // large launches in progress
  std::condition_variable cv_large;
  uint64_t large_seq = 0;            // admission number of the next large launch
  std::set<uint64_t> large_pending;  // large launches admitted, not yet started
  rs_server_stats st{};
  size_t in_use = 0;
  size_t usable = 0;  // pool bytes in whole regions
};

namespace {

size_t job_footprint(const rs_job& j, uint32_t workers_max) {
  std::vector<JobPlan> one(1);
  one[0].n = j.n;
  one[0].b = j.bucket_size;
  one[0].l = j.leaf_size;
  one[0].flags = j.flags;
  return batch_footprint(one, workers_max);
}

void slot_loop(rs_server* S, uint32_t slot) {
  Context& c = *S->ctx[slot];
  (void)hipSetDevice(S->dev->id);  // a new thread starts on device 0
  for (;;) {
    std::vector<uint64_t> tickets;
    std::vector<JobPlan> plan;
    size_t off = 0, bytes = 0;
    bool backlog = false, large = false;
    uint64_t seq = 0;
    {
      std::unique_lock<std::mutex> lock(S->mu);
      for (;;) {
        if (S->stopping) return;
        if (!S->waiting.empty()) {
          // The oldest requests that fit one free region, in arrival order.
          // A large request is always built alone, so no smaller request
          // waits for the end of its search.  With a short queue (latency
          // first) small ones are batched only while their keys stay below
          // the large-launch size; with a backlog (at least one request per
          // slot waiting: throughput first) up to the per-launch limit.
          backlog = S->waiting.size() >= S->ctx.size();
          const size_t room = S->regions.largest();
          std::vector<JobPlan> trial;
          size_t need = 0;
          uint64_t batch_keys = 0;
          for (uint64_t t : S->waiting) {
            if (trial.size() >= S->cfg.max_jobs_per_launch) break;
            const Request& r = S->reqs[t];
            if (!trial.empty() &&
                (r.job.n >= kLargeLaunchKeys || batch_keys >= kLargeLaunchKeys ||
                 (!backlog && batch_keys + r.job.n >= kLargeLaunchKeys)))
              break;
            batch_keys += r.job.n;
            JobPlan p;
            p.keys = reinterpret_cast<const Key*>(r.job.keys);
            p.n = r.job.n;
            p.l = r.job.leaf_size;
            p.b = r.job.bucket_size;
            p.flags = r.job.flags;
            trial.push_back(p);
            const size_t f = batch_footprint(trial, S->workers_max);
            if (f > room) {
              trial.pop_back();
              break;
            }
            need = f;
          }
          if (!trial.empty() && S->regions.take(need, &off)) {
            bytes = need;
            plan.swap(trial);
            const double t = now_s();
            for (size_t k = 0; k < plan.size(); ++k) {
              const uint64_t tk = S->waiting.front();
              S->waiting.pop_front();
              Request& r = S->reqs[tk];
              r.t_admit = t;
              r.slot = slot;
              r.batch_jobs = (uint32_t)plan.size();
              tickets.push_back(tk);
            }
            S->in_use += bytes;
            if (S->in_use > S->st.peak_bytes) S->st.peak_bytes = S->in_use;
            S->st.launches += 1;
            uint64_t keys = 0;
            for (const JobPlan& p : plan) keys += p.n;
            large = keys >= kLargeLaunchKeys;
            if (large) {
              seq = S->large_seq++;
              S->large_pending.insert(seq);
            }
            break;
          }
        }
        S->cv_work.wait(lock);
      }
    }
    // Device sharing.  A large launch holds the device for a long time and
    // leaves the reserve free; without a backlog large launches run one at a
    // time, in the order they were admitted (with one, they overlap and fill
    // each other's tails).  A small launch that starts while a large one runs
    // is sized to the reserve, so it finishes without waiting for the large
    // one; otherwise a small launch takes the whole device (it ends soon).
    uint32_t cap = 0;
    if (large) {
      {
        std::unique_lock<std::mutex> lock(S->mu);
        if (!backlog)
          S->cv_large.wait(lock, [&] {
            return S->stopping || (!S->large_running && *S->large_pending.begin() == seq);
          });
        S->large_pending.erase(seq);
        S->large_running += 1;
        cap = S->workers_cap;
      }
      S->cv_large.notify_all();  // the next large launch in order may now wait its turn
    } else {
      std::lock_guard<std::mutex> lock(S->mu);
      if (S->large_running && S->reserve_workers) cap = S->reserve_workers;
    }
    int rc = build_jobs(c, plan, S->pool + off, bytes, cap);
    if (rc) {
      (void)hipStreamSynchronize(c.s);
      (void)hipGetLastError();
    }
    if (large) {
      std::lock_guard<std::mutex> lock(S->mu);
      S->large_running -= 1;
    }
    if (large) S->cv_large.notify_all();
    {
      std::lock_guard<std::mutex> lock(S->mu);
      const double t = now_s();
      for (size_t k = 0; k < plan.size(); ++k) {
        Request& r = S->reqs[tickets[k]];
        if (rc) {
          mphf_release(plan[k].out);
          r.status = rc;
          r.out = nullptr;
        } else {
          r.status = plan[k].status;
          r.out = plan[k].status ? nullptr : plan[k].out;
        }
        r.t_done = t;
        S->st.completed += 1;
        S->st.keys_completed += r.job.n;
      }
      S->regions.give(off, bytes);
      S->in_use -= bytes;
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

int rs_server_create(const rs_server_config* cfg, rs_server** out) {
  if (!cfg || !out || cfg->max_slots < 1 || cfg->max_slots > 64 || cfg->hbm_budget_bytes < (1u << 20))
    return RS_ERR_INVALID_ARG;
  *out = nullptr;
  rs_server* S = new (std::nothrow) rs_server();
  if (!S) return RS_ERR_OOM;
  S->cfg = *cfg;
  if (S->cfg.max_jobs_per_launch < 1) S->cfg.max_jobs_per_launch = 1;
  int rc = device_get(&S->dev);
  if (rc) {
    delete S;
    return rc;
  }
  S->workers_max = max_workers(*S->dev);
  {
    const uint64_t cus = (uint64_t)S->dev->cus;
    const uint64_t keep = (uint64_t)cfg->reserve_per_cu * cus;
    S->workers_cap = keep + cus <= S->workers_max ? (uint32_t)(S->workers_max - keep) : (uint32_t)cus;
    S->reserve_workers = (uint32_t)(S->workers_max - S->workers_cap);
  }
  if (hipMalloc(reinterpret_cast<void**>(&S->pool), cfg->hbm_budget_bytes) != hipSuccess) {
    delete S;
    return RS_ERR_OOM;
  }
  S->usable = cfg->hbm_budget_bytes / S->regions.align * S->regions.align;
  S->regions.free[0] = S->usable;
  for (uint32_t i = 0; i < cfg->max_slots; ++i) {
    Context* c = new (std::nothrow) Context();
    if (!c || context_init(*c, S->dev)) {
      delete c;
      rs_server_destroy(S);
      return RS_ERR_DEVICE;
    }
    S->ctx.push_back(c);
  }
  for (uint32_t i = 0; i < cfg->max_slots; ++i) S->threads.emplace_back(slot_loop, S, i);
  *out = S;
  return RS_OK;
}

int rs_server_submit(rs_server* S, const rs_job* job, uint64_t* ticket) {
  if (!S || !job || !ticket) return RS_ERR_INVALID_ARG;
  if (!job_args_ok(job->keys, job->n, job->leaf_size, job->bucket_size, job->flags))
    return RS_ERR_INVALID_ARG;
  const size_t fp = job_footprint(*job, S->workers_max);
  const size_t al = S->regions.align;
  if ((fp + al - 1) / al * al > S->usable) return RS_ERR_OOM;  // can never be admitted
  {
    std::lock_guard<std::mutex> lock(S->mu);
    const uint64_t t = S->next_ticket++;
    Request& r = S->reqs[t];
    r.job = *job;
    r.footprint = fp;
    r.t_submit = now_s();
    S->waiting.push_back(t);
    S->st.submitted += 1;
    *ticket = t;
  }
  S->cv_work.notify_all();
  return RS_OK;
}

int rs_server_poll(rs_server* S, uint64_t ticket, int wait, rs_mphf** out, int* status,
                   rs_request_times* times) {
  if (!S || !out || !status) return RS_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lock(S->mu);
  if (S->reqs.find(ticket) == S->reqs.end()) return RS_ERR_INVALID_ARG;
  // Another thread polling the same ticket may collect (and erase) it while
  // this one waits, so the entry is looked up again after every wake-up
  // instead of holding an iterator across the wait.
  if (wait)
    S->cv_done.wait(lock, [&] {
      auto w = S->reqs.find(ticket);
      return w == S->reqs.end() || w->second.status != RS_PENDING;
    });
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return RS_ERR_INVALID_ARG;  // collected by another poll
  Request& r = it->second;
  if (r.status == RS_PENDING) return RS_PENDING;
  *out = r.out;
  *status = r.status;
  if (times) {
    times->submit = r.t_submit;
    times->admit = r.t_admit;
    times->done = r.t_done;
    times->slot = r.slot;
    times->batch_jobs = r.batch_jobs;
  }
  S->reqs.erase(it);  // the caller owns the structure now
  return RS_OK;
}

int rs_server_get_stats(rs_server* S, rs_server_stats* st) {
  if (!S || !st) return RS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(S->mu);
  *st = S->st;
  st->waiting = S->waiting.size();
  st->bytes_in_use = S->in_use;
  return RS_OK;
}

void rs_server_destroy(rs_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lock(S->mu);
    S->stopping = true;
  }
  S->cv_work.notify_all();
  S->cv_large.notify_all();
  for (std::thread& t : S->threads) t.join();
  for (Context* c : S->ctx) {
    context_destroy(*c);
    delete c;
  }
  for (auto& kv : S->reqs) mphf_release(kv.second.out);
  if (S->pool) (void)hipFree(S->pool);
  delete S;
}

}  // extern "C"
