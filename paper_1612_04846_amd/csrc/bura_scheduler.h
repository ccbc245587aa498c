// Scheduling of the request server (bura_server_*), independent of the device.
//
// Requests (grid, alpha, k, tolerance, precision, f, u) are queued on submit.
// A dispatcher thread assigns each to the resident plan of its key -- grid,
// precision and a class of term counts (13 or 17 term slots per right-hand
// side, the smaller that holds k+1) -- creating the plan, outside the lock,
// if there is none.  Every plan has a worker thread:
//
// * BURA_MIXED (continuous batching): the worker admits queued requests into
//   free right-hand-side slots of the running solve at every outer
//   refinement-step boundary, advances all admitted systems by one outer step,
//   and hands each request its result as soon as its own systems have
//   finished, freeing the slot for the next one.  Requests join and leave a
//   solve that is already running.
// * BURA_FP64: each solve takes up to max_group queued requests of the key as
//   its right-hand sides; the next batch starts when it finishes.
//
// At most max_concurrent plans have work at once.  New plans are admitted
// against an HBM budget; idle plans are evicted least recently used first
// when the budget would be exceeded, and a key whose plan cannot fit while
// other plans are busy waits for them.
//
// The device work is behind Executor: the library drives slot plans on HIP
// streams (bura_server.cpp); the scheduler itself makes no device call, so it
// can also be driven by a host-only executor.
#ifndef BURA_SCHEDULER_H
#define BURA_SCHEDULER_H

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/bura.h"

namespace bura {
namespace sched {

using Clock = std::chrono::steady_clock;

constexpr int kMaxTerms = 17;   // k <= 16 poles: up to 17 terms per request

// term slots per right-hand side of the plan a request goes to: 13 (k <= 12,
// the serving range) or 17; a finer split (8 / 13 / 17) measured worse, as it
// doubles the plans of a grid and same-grid requests share fewer steps
inline int term_class(int nterms) { return nterms <= 13 ? 13 : kMaxTerms; }

// The device side of a plan.  create/destroy are called by the dispatcher (and
// the destructor), everything else by the plan's worker thread only.
struct Executor {
  virtual ~Executor() = default;
  // make the device current on a scheduler thread
  virtual void bind_thread() {}
  // resources for key q: a slot plan with K term slots for each of max_group
  // right-hand sides; budget_left > 0 caps its bytes (BURA_ENOMEM if it does
  // not fit), 0 = unlimited.  *bytes: what it holds.
  virtual int create(const bura_request_t& q, int K, int max_group, size_t budget_left, void** plan,
                     size_t* bytes) = 0;
  virtual void destroy(void* plan) = 0;
  // continuous batching (BURA_MIXED): no slot in use; stage f into a slot and
  // start its systems; one outer step of every active system (returns the
  // systems still active, or a negative status); whether a slot has finished
  // (1: u written, *rep filled; 0: not yet; < 0: status)
  virtual int reset(void* plan) = 0;
  virtual int admit(void* plan, int slot, const double* f, int nterms, const double* w, const double* s,
                    double tol) = 0;
  virtual int step(void* plan) = 0;
  virtual int slot_done(void* plan, int slot, double* u, bura_report_t* rep) = 0;
  // one solve of g requests (BURA_FP64): f[i] -> u[i] with nterms[i] terms at
  // w + i K, s + i K and tolerance tol[i]; returns when every u[i] is written
  virtual int solve(void* plan, int g, const double* const* f, double* const* u, const int* nterms,
                    const double* w, const double* s, const double* tol, bura_report_t* rep) = 0;
};

struct Req {
  uint64_t id = 0;
  bura_request_t q{};
  double w[kMaxTerms] = {}, s[kMaxTerms] = {};   // the request's terms (weights, shifts)
  double E = 0.0;
  const double* f = nullptr;
  double* u = nullptr;
  Clock::time_point t_submit, t_done;
  bool done = false;
  int status = BURA_PENDING;
  bura_report_t rep{};
};

struct Entry {
  std::string key;
  bura_request_t q{};
  int K = kMaxTerms;
  void* plan = nullptr;   // the executor's
  size_t bytes = 0;
  Clock::time_point last_used;
  // scheduling state (under the scheduler's lock)
  bool creating = true;                          // plan being created by the dispatcher
  bool stop = false;
  bool holds_token = false;                      // counts towards max_concurrent
  std::deque<std::shared_ptr<Req>> pending;      // assigned, not yet admitted
  std::vector<std::shared_ptr<Req>> slot;        // running requests by rhs slot
  int running = 0;
  std::thread worker;
  bool idle() const { return !creating && pending.empty() && running == 0; }
};

inline std::string key_of(const bura_request_t& q) {
  char b[64];
  std::snprintf(b, sizeof(b), "%d/%d/%d/%d", q.dim, q.n, q.precision, term_class(q.k + 1));
  return b;
}

class Scheduler {
 public:
  Scheduler(Executor* ex, size_t budget, int max_concurrent, int max_group)
      : ex_(ex), budget_(budget), max_concurrent_(max_concurrent), max_group_(max_group) {
    dispatcher_ = std::thread([this]() { loop(); });
  }

  // Waits for queued and running requests, then frees every plan.
  ~Scheduler() {
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&]() {
        if (!queue_.empty()) return false;
        for (auto& kv : plans_)
          if (!kv.second->idle()) return false;
        return true;
      });
      stop_ = true;
      cv_.notify_all();
    }
    if (dispatcher_.joinable()) dispatcher_.join();
    for (auto& kv : plans_) destroy_entry(kv.second.get());
    plans_.clear();
  }

  // Queue a request whose terms (weights w, shifts s, nterms = k+1) the
  // caller computed; *ticket identifies it.
  int submit(const bura_request_t& q, const double* w, const double* s, double E, const double* f, double* u,
             uint64_t* ticket) {
    auto r = std::make_shared<Req>();
    r->q = q;
    r->f = f;
    r->u = u;
    r->E = E;
    for (int j = 0; j <= q.k; ++j) {
      r->w[j] = w[j];
      r->s[j] = s[j];
    }
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(mu_);
    r->id = next_id_++;
    tickets_[r->id] = r;
    queue_.push_back(r);
    ++submitted_;
    *ticket = r->id;
    cv_.notify_all();
    return BURA_OK;
  }

  int poll(uint64_t ticket, bura_report_t* rep) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end()) return BURA_EINVAL;
    if (!it->second->done) return BURA_PENDING;
    if (rep) *rep = it->second->rep;
    const int st = it->second->status;
    tickets_.erase(it);
    return st;
  }

  int wait(uint64_t ticket, bura_report_t* rep) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end()) return BURA_EINVAL;
    std::shared_ptr<Req> r = it->second;
    cv_.wait(lk, [&]() { return r->done; });
    if (rep) *rep = r->rep;
    tickets_.erase(ticket);
    return r->status;
  }

  void stats(bura_server_stats_t* st) {
    std::lock_guard<std::mutex> lk(mu_);
    std::memset(st, 0, sizeof(*st));
    st->submitted = submitted_;
    st->completed = completed_;
    st->failed = failed_;
    st->batches = batches_;
    st->plans_created = created_;
    st->plans_evicted = evicted_;
    st->unknown_pole_solves = unknown_pole_;
    st->mean_batch = batches_ ? batched_requests_ / batches_ : 0.0;
    st->resident_bytes = resident_;
    st->joined_running = joined_;
    std::vector<double> l = latencies_;
    if (!l.empty()) {
      std::sort(l.begin(), l.end());
      st->p50_latency_s = l[(size_t)(0.50 * (l.size() - 1))];
      st->p99_latency_s = l[(size_t)(0.99 * (l.size() - 1))];
    }
  }

  void reset_latency() {
    std::lock_guard<std::mutex> lk(mu_);
    latencies_.clear();
  }

 private:
  Executor* ex_;
  size_t budget_ = 0;
  int max_concurrent_ = 4;
  int max_group_ = 4;
  std::mutex mu_;
  std::condition_variable cv_;
  std::list<std::shared_ptr<Req>> queue_;   // submitted, not yet assigned to a plan
  std::map<uint64_t, std::shared_ptr<Req>> tickets_;
  std::map<std::string, std::unique_ptr<Entry>> plans_;
  std::thread dispatcher_;
  bool stop_ = false;
  uint64_t next_id_ = 1;
  int tokens_ = 0;   // plans with work (<= max_concurrent)
  // statistics
  long long submitted_ = 0, completed_ = 0, failed_ = 0, batches_ = 0, created_ = 0, evicted_ = 0, joined_ = 0;
  double unknown_pole_ = 0.0;
  double batched_requests_ = 0.0;
  std::vector<double> latencies_;
  size_t resident_ = 0;

  // ---- completion (under mu_) ----
  void complete(const std::shared_ptr<Req>& r, int rc, const bura_report_t* rep) {
    const auto now = Clock::now();
    r->status = rc;
    if (rep) r->rep = *rep;
    r->rep.status = rc;
    r->rep.nterms = r->q.k + 1;
    r->rep.E = r->E;
    r->t_done = now;
    r->done = true;
    ++completed_;
    if (rc != BURA_OK) ++failed_;
    latencies_.push_back(std::chrono::duration<double>(now - r->t_submit).count());
    long long N = 1;
    for (int a = 0; a < r->q.dim; ++a) N *= r->q.n;
    if (rc == BURA_OK) unknown_pole_ += (double)N * (r->q.k + 1);
  }

  // an idle worker gives its max_concurrent token back at once (waiting with
  // it would starve other keys' workers); under mu_
  void release_token_if_idle(Entry* e) {
    if (e->running == 0 && e->pending.empty() && e->holds_token) {
      e->holds_token = false;
      --tokens_;
      e->last_used = Clock::now();
      cv_.notify_all();
    }
  }

  // ---- plan workers ----
  void worker_mixed(Entry* e) {
    ex_->bind_thread();
    const int R = max_group_;
    int rc = ex_->reset(e->plan);
    std::vector<std::pair<int, std::shared_ptr<Req>>> admit;
    for (;;) {
      admit.clear();
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&]() {
          if (e->stop || e->running > 0) return true;
          if (e->pending.empty()) return false;
          return e->holds_token || tokens_ < max_concurrent_;
        });
        if (e->stop && e->running == 0 && e->pending.empty()) break;
        if (!e->holds_token && (e->running > 0 || !e->pending.empty())) {
          e->holds_token = true;
          ++tokens_;
        }
        const bool was_running = e->running > 0;
        for (int i = 0; i < R && !e->pending.empty(); ++i) {
          if (e->slot[i]) continue;
          std::shared_ptr<Req> r = e->pending.front();
          e->pending.pop_front();
          if (rc != BURA_OK) {   // the plan cannot serve (reset failed)
            complete(r, rc, nullptr);
            continue;
          }
          if (was_running) ++joined_;   // admitted into a solve already running
          e->slot[i] = r;
          ++e->running;
          admit.emplace_back(i, r);
        }
        if (rc != BURA_OK) cv_.notify_all();
      }
      for (auto& a : admit) {
        const Req& q = *a.second;
        const int ar = ex_->admit(e->plan, a.first, q.f, q.q.k + 1, q.w, q.s, q.q.tol);
        if (ar != BURA_OK) {
          std::lock_guard<std::mutex> lk(mu_);
          complete(a.second, ar, nullptr);
          e->slot[a.first].reset();
          --e->running;
          cv_.notify_all();
        }
      }
      int running;
      {
        std::lock_guard<std::mutex> lk(mu_);
        running = e->running;
        if (running > 0) {
          ++batches_;
          batched_requests_ += running;
        }
      }
      if (running == 0) {
        std::lock_guard<std::mutex> lk(mu_);
        release_token_if_idle(e);
        continue;
      }
      const int st = ex_->step(e->plan);
      for (int i = 0; i < R; ++i) {
        std::shared_ptr<Req> r;
        {
          std::lock_guard<std::mutex> lk(mu_);
          r = e->slot[i];
        }
        if (!r) continue;
        bura_report_t rep{};
        const int d = st < 0 ? st : ex_->slot_done(e->plan, i, r->u, &rep);
        if (d == 0) continue;
        std::lock_guard<std::mutex> lk(mu_);
        complete(r, d == 1 ? rep.status : d, d == 1 ? &rep : nullptr);
        e->slot[i].reset();
        --e->running;
        cv_.notify_all();
      }
      if (st < 0) rc = ex_->reset(e->plan);   // device error: the plan's state is lost; restart it
      std::lock_guard<std::mutex> lk(mu_);
      release_token_if_idle(e);
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (e->holds_token) {
      e->holds_token = false;
      --tokens_;
    }
    cv_.notify_all();
  }

  void worker_fp64(Entry* e) {
    ex_->bind_thread();
    const int R = max_group_;
    std::vector<const double*> f(R);
    std::vector<double*> u(R);
    std::vector<int> nterms(R);
    std::vector<double> w((size_t)R * e->K), sh((size_t)R * e->K), tol(R);
    for (;;) {
      std::vector<std::shared_ptr<Req>> group;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&]() {
          return e->stop || (!e->pending.empty() && (e->holds_token || tokens_ < max_concurrent_));
        });
        if (e->pending.empty()) break;   // stop requested
        if (!e->holds_token) {
          e->holds_token = true;
          ++tokens_;
        }
        while ((int)group.size() < R && !e->pending.empty()) {
          group.push_back(e->pending.front());
          e->pending.pop_front();
        }
        e->running = (int)group.size();
        ++batches_;
        batched_requests_ += (double)group.size();
      }
      const int g = (int)group.size();
      std::fill(w.begin(), w.end(), 0.0);
      std::fill(sh.begin(), sh.end(), 0.0);
      for (int i = 0; i < g; ++i) {
        const Req& q = *group[i];
        f[i] = q.f;
        u[i] = q.u;
        nterms[i] = q.q.k + 1;
        tol[i] = q.q.tol;
        for (int j = 0; j <= q.q.k; ++j) {
          w[(size_t)i * e->K + j] = q.w[j];
          sh[(size_t)i * e->K + j] = q.s[j];
        }
      }
      bura_report_t rep{};
      const int rc = ex_->solve(e->plan, g, f.data(), u.data(), nterms.data(), w.data(), sh.data(), tol.data(), &rep);
      std::lock_guard<std::mutex> lk(mu_);
      for (auto& r : group) complete(r, rc, &rep);
      e->running = 0;
      e->last_used = Clock::now();
      if (e->pending.empty() && e->holds_token) {
        e->holds_token = false;
        --tokens_;
      }
      cv_.notify_all();
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (e->holds_token) {
      e->holds_token = false;
      --tokens_;
    }
    cv_.notify_all();
  }

  // ---- plan creation and eviction (dispatcher thread, outside mu_) ----
  void destroy_entry(Entry* e) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      e->stop = true;
      cv_.notify_all();
    }
    if (e->worker.joinable()) e->worker.join();
    if (e->plan) ex_->destroy(e->plan);
    e->plan = nullptr;
  }

  // Create the plan of entry e; over the budget, evict idle plans one at a
  // time, least recently used first, trying again after each.  Returns a status.
  int create_plan(Entry* e) {
    for (;;) {
      size_t left = 0;
      int rc = BURA_OK;
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (budget_ > 0) {
          if (budget_ <= resident_) rc = BURA_ENOMEM;
          else left = budget_ - resident_;
        }
      }
      if (rc == BURA_OK) {
        void* p = nullptr;
        size_t bytes = 0;
        rc = ex_->create(e->q, e->K, max_group_, left, &p, &bytes);
        if (rc == BURA_OK) {
          e->plan = p;
          e->bytes = bytes;
          std::lock_guard<std::mutex> lk(mu_);
          resident_ += bytes;
          ++created_;
          return BURA_OK;
        }
      }
      if (rc != BURA_ENOMEM) return rc;
      // over budget: take the least recently used idle plan out of service
      std::unique_ptr<Entry> victim;
      {
        std::lock_guard<std::mutex> lk(mu_);
        Entry* lru = nullptr;
        for (auto& kv : plans_) {
          Entry* v = kv.second.get();
          if (v != e && v->idle() && (!lru || v->last_used < lru->last_used)) lru = v;
        }
        if (!lru) return BURA_ENOMEM;
        auto it = plans_.find(lru->key);
        victim = std::move(it->second);
        plans_.erase(it);
        resident_ -= std::min(resident_, victim->bytes);
        ++evicted_;
      }
      destroy_entry(victim.get());
    }
  }

  bool any_running() {
    for (auto& kv : plans_)
      if (kv.second->running > 0 || !kv.second->pending.empty()) return true;
    return false;
  }

  void loop() {
    ex_->bind_thread();
    std::unique_lock<std::mutex> lk(mu_);
    while (!stop_) {
      // assign queued requests to the plans of their keys (FIFO)
      Entry* to_create = nullptr;
      for (auto it = queue_.begin(); it != queue_.end();) {
        const std::string key = key_of((*it)->q);
        auto pe = plans_.find(key);
        if (pe == plans_.end()) {
          if (!to_create) {
            auto e = std::make_unique<Entry>();
            e->key = key;
            e->q = (*it)->q;
            e->K = term_class((*it)->q.k + 1);
            e->slot.assign(max_group_, nullptr);
            to_create = e.get();
            plans_[key] = std::move(e);
          }
          ++it;
          continue;
        }
        if (pe->second->creating) {
          ++it;
          continue;
        }
        pe->second->pending.push_back(*it);
        it = queue_.erase(it);
        cv_.notify_all();
      }
      if (to_create) {
        lk.unlock();
        const int rc = create_plan(to_create);
        lk.lock();
        if (rc == BURA_OK) {
          to_create->creating = false;
          to_create->last_used = Clock::now();
          Entry* e = to_create;
          e->worker = std::thread([this, e]() {
            if (e->q.precision == BURA_MIXED) worker_mixed(e);
            else worker_fp64(e);
          });
        } else if (rc == BURA_ENOMEM && any_running()) {
          // wait for memory to free up: drop the entry, keep its requests queued
          auto pe = plans_.find(to_create->key);
          std::unique_ptr<Entry> e = std::move(pe->second);
          plans_.erase(pe);
          lk.unlock();
          destroy_entry(e.get());
          lk.lock();
          cv_.wait_for(lk, std::chrono::milliseconds(2));
        } else {
          // the key cannot be served: fail its queued requests
          const std::string key = to_create->key;
          for (auto it = queue_.begin(); it != queue_.end();) {
            if (key_of((*it)->q) == key) {
              complete(*it, rc, nullptr);
              it = queue_.erase(it);
            } else {
              ++it;
            }
          }
          auto pe = plans_.find(key);
          std::unique_ptr<Entry> e = std::move(pe->second);
          plans_.erase(pe);
          lk.unlock();
          destroy_entry(e.get());
          lk.lock();
          cv_.notify_all();
        }
        continue;
      }
      cv_.wait(lk, [&]() {
        if (stop_) return true;
        for (auto& r : queue_)
          if (!plans_.count(key_of(r->q)) || !plans_[key_of(r->q)]->creating) return true;
        return false;
      });
    }
  }
};

}  // namespace sched
}  // namespace bura

#endif  // BURA_SCHEDULER_H
