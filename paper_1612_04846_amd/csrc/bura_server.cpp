// Request server with continuous batching for fractional solves on one GPU.
//
// Requests (grid, alpha, k, tolerance, precision, f, u) are queued on submit.
// A dispatcher thread assigns each to the resident slot plan
// (bura_plan_create_slots) of its key -- grid, precision and a class of term
// counts (13 or 17 term slots per right-hand side, the smaller that holds
// k+1) -- creating the plan, outside the server's lock, if there is none.
// Every plan has a worker thread:
//
// * BURA_MIXED (continuous batching): the worker admits queued requests into
//   free right-hand-side slots of the running solve at every outer
//   refinement-step boundary (bura::serve_admit), advances all admitted
//   systems by one outer step (bura::serve_step), and hands each request its
//   result as soon as its own systems have finished (bura::serve_slot_done),
//   freeing the slot for the next one.  Requests join and leave a solve that
//   is already running.
// * BURA_FP64: each solve takes up to nrhs_max queued requests of the key as
//   its right-hand sides (bura_solve_slots); the next batch starts when it
//   finishes.
//
// Plans of different keys run concurrently on their own streams (at most
// max_concurrent with work at once).  New plans are admitted against an HBM
// budget; idle plans are evicted least recently used first when the budget
// would be exceeded.  A request's result depends only on its own right-hand
// side and terms: every system's arithmetic and fixed-order reductions are
// its own, and a system admitted at a step boundary goes through the same
// operations as in a solve by itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "bura_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kMaxTerms = 17;   // k <= 16 poles: up to 17 terms per request

// term slots per right-hand side of the plan a request goes to: 13 (k <= 12,
// the serving range) or 17; a finer split (8 / 13 / 17) measured worse, as it
// doubles the plans of a grid and same-grid requests share fewer steps
int term_class(int nterms) { return nterms <= 13 ? 13 : kMaxTerms; }

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
  bura_plan_t plan = nullptr;
  hipStream_t stream = nullptr;   // the plan's caller stream; also carries the staging copies
  size_t bytes = 0;
  long long N = 0;
  Clock::time_point last_used;
  // scheduling state (under the server's lock)
  bool creating = true;                          // plan being created by the dispatcher
  bool stop = false;
  bool holds_token = false;                      // counts towards max_concurrent
  std::deque<std::shared_ptr<Req>> pending;      // assigned, not yet admitted
  std::vector<std::shared_ptr<Req>> slot;        // running requests by rhs slot
  int running = 0;
  std::thread worker;
  double* f_stage = nullptr;   // FP64 batches of several requests
  double* u_stage = nullptr;
  bool idle() const { return !creating && pending.empty() && running == 0; }
};

std::string key_of(const bura_request_t& q) {
  char b[64];
  std::snprintf(b, sizeof(b), "%d/%d/%d/%d", q.dim, q.n, q.precision, term_class(q.k + 1));
  return b;
}

}  // namespace

struct bura_server_s {
  size_t budget = 0;
  int max_concurrent = 4;
  int max_group = 4;
  std::mutex mu;
  std::condition_variable cv;
  std::list<std::shared_ptr<Req>> queue;   // submitted, not yet assigned to a plan
  std::map<uint64_t, std::shared_ptr<Req>> tickets;
  std::map<std::string, std::unique_ptr<Entry>> plans;
  std::thread dispatcher;
  bool stop = false;
  uint64_t next_id = 1;
  int device = 0;
  int tokens = 0;   // plans with work (<= max_concurrent)
  // statistics
  long long submitted = 0, completed = 0, failed = 0, batches = 0, created = 0, evicted = 0, joined = 0;
  double unknown_pole = 0.0;
  double batched_requests = 0.0;
  std::vector<double> latencies;
  size_t resident = 0;

  // ---- completion (under mu) ----
  void complete(const std::shared_ptr<Req>& r, int rc, const bura_report_t* rep) {
    const auto now = Clock::now();
    r->status = rc;
    if (rep) r->rep = *rep;
    r->rep.status = rc;
    r->rep.nterms = r->q.k + 1;
    r->rep.E = r->E;
    r->t_done = now;
    r->done = true;
    ++completed;
    if (rc != BURA_OK) ++failed;
    latencies.push_back(std::chrono::duration<double>(now - r->t_submit).count());
    long long N = 1;
    for (int a = 0; a < r->q.dim; ++a) N *= r->q.n;
    if (rc == BURA_OK) unknown_pole += (double)N * (r->q.k + 1);
  }

  // ---- plan workers ----
  void worker_mixed(Entry* e) {
    hipSetDevice(device);
    const int R = max_group;
    int rc = bura::serve_reset(e->plan);
    std::vector<std::pair<int, std::shared_ptr<Req>>> admit;
    for (;;) {
      admit.clear();
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&]() {
          if (e->stop || e->running > 0) return true;
          if (e->pending.empty()) return false;
          return e->holds_token || tokens < max_concurrent;
        });
        if (e->stop && e->running == 0 && e->pending.empty()) break;
        if (!e->holds_token && (e->running > 0 || !e->pending.empty())) {
          e->holds_token = true;
          ++tokens;
        }
        for (int i = 0; i < R && !e->pending.empty(); ++i) {
          if (e->slot[i]) continue;
          std::shared_ptr<Req> r = e->pending.front();
          e->pending.pop_front();
          if (rc != BURA_OK) {   // the plan cannot serve (reset failed)
            complete(r, rc, nullptr);
            continue;
          }
          if (e->running > 0) ++joined;   // admitted into a solve already running
          e->slot[i] = r;
          ++e->running;
          admit.emplace_back(i, r);
        }
        if (rc != BURA_OK) cv.notify_all();
      }
      for (auto& a : admit) {
        const Req& q = *a.second;
        const int ar = bura::serve_admit(e->plan, a.first, q.f, q.q.k + 1, q.w, q.s, q.q.tol);
        if (ar != BURA_OK) {
          std::lock_guard<std::mutex> lk(mu);
          complete(a.second, ar, nullptr);
          e->slot[a.first].reset();
          --e->running;
          cv.notify_all();
        }
      }
      int running;
      {
        std::lock_guard<std::mutex> lk(mu);
        running = e->running;
        if (running > 0) {
          ++batches;
          batched_requests += running;
        }
      }
      if (running == 0) {
        std::lock_guard<std::mutex> lk(mu);
        if (e->holds_token && e->pending.empty()) {
          e->holds_token = false;
          --tokens;
          e->last_used = Clock::now();
          cv.notify_all();
        }
        continue;
      }
      const int st = bura::serve_step(e->plan);
      for (int i = 0; i < R; ++i) {
        std::shared_ptr<Req> r;
        {
          std::lock_guard<std::mutex> lk(mu);
          r = e->slot[i];
        }
        if (!r) continue;
        bura_report_t rep{};
        const int d = st < 0 ? st : bura::serve_slot_done(e->plan, i, r->u, &rep);
        if (d == 0) continue;
        std::lock_guard<std::mutex> lk(mu);
        complete(r, d == 1 ? rep.status : d, d == 1 ? &rep : nullptr);
        e->slot[i].reset();
        --e->running;
        cv.notify_all();
      }
      if (st < 0) {   // device error: the plan's state is lost; restart it
        rc = bura::serve_reset(e->plan);
      }
      // an idle worker gives its max_concurrent token back at once (waiting
      // with it would starve other keys' workers)
      std::lock_guard<std::mutex> lk(mu);
      if (e->running == 0 && e->pending.empty() && e->holds_token) {
        e->holds_token = false;
        --tokens;
        e->last_used = Clock::now();
        cv.notify_all();
      }
    }
    std::lock_guard<std::mutex> lk(mu);
    if (e->holds_token) {
      e->holds_token = false;
      --tokens;
    }
    cv.notify_all();
  }

  void worker_fp64(Entry* e) {
    hipSetDevice(device);
    const int R = max_group;
    for (;;) {
      std::vector<std::shared_ptr<Req>> group;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&]() { return e->stop || (!e->pending.empty() && (e->holds_token || tokens < max_concurrent)); });
        if (e->pending.empty()) break;   // stop requested
        if (!e->holds_token) {
          e->holds_token = true;
          ++tokens;
        }
        while ((int)group.size() < R && !e->pending.empty()) {
          group.push_back(e->pending.front());
          e->pending.pop_front();
        }
        e->running = (int)group.size();
        ++batches;
        batched_requests += (double)group.size();
      }
      const int g = (int)group.size();
      int nterms[64];
      double w[64 * kMaxTerms] = {}, sh[64 * kMaxTerms] = {}, tol[64];
      for (int i = 0; i < g; ++i) {
        const Req& q = *group[i];
        nterms[i] = q.q.k + 1;
        tol[i] = q.q.tol;
        for (int j = 0; j <= q.q.k; ++j) {
          w[i * e->K + j] = q.w[j];
          sh[i * e->K + j] = q.s[j];
        }
      }
      const double* f = group[0]->f;
      double* u = group[0]->u;
      if (g > 1) {
        for (int i = 0; i < g; ++i)
          hipMemcpyAsync(e->f_stage + (size_t)i * e->N, group[i]->f, e->N * 8, hipMemcpyDeviceToDevice, e->stream);
        f = e->f_stage;
        u = e->u_stage;
      }
      bura_report_t rep{};
      const int rc = bura_solve_slots(e->plan, f, u, g, nterms, w, sh, tol, &rep);
      if (g > 1 && rc != BURA_EINVAL) {
        for (int i = 0; i < g; ++i)
          hipMemcpyAsync(group[i]->u, e->u_stage + (size_t)i * e->N, e->N * 8, hipMemcpyDeviceToDevice, e->stream);
      }
      hipStreamSynchronize(e->stream);
      std::lock_guard<std::mutex> lk(mu);
      for (auto& r : group) complete(r, rc, &rep);
      e->running = 0;
      e->last_used = Clock::now();
      if (e->pending.empty() && e->holds_token) {
        e->holds_token = false;
        --tokens;
      }
      cv.notify_all();
    }
    std::lock_guard<std::mutex> lk(mu);
    if (e->holds_token) {
      e->holds_token = false;
      --tokens;
    }
    cv.notify_all();
  }

  // ---- plan creation and eviction (dispatcher thread, outside mu) ----
  void destroy_entry(Entry* e) {
    {
      std::lock_guard<std::mutex> lk(mu);
      e->stop = true;
      cv.notify_all();
    }
    if (e->worker.joinable()) e->worker.join();
    if (e->plan) bura_plan_destroy(e->plan);
    if (e->f_stage) hipFree(e->f_stage);
    if (e->u_stage) hipFree(e->u_stage);
    if (e->stream) hipStreamDestroy(e->stream);
  }

  // Create the plan of entry e; over the budget, evict idle plans (least
  // recently used first) and try once more.  Returns a status.
  int create_plan(Entry* e) {
    const bura_request_t& q = e->q;
    const bool fp64 = q.precision == BURA_FP64;
    for (int attempt = 0; attempt < 2; ++attempt) {
      bura_grid_t g{};
      g.dim = q.dim;
      g.n = q.n;
      bura_opts_t o;
      bura_opts_default(&o);
      o.precision = q.precision;
      o.nrhs_max = max_group;
      long long N = 1;
      for (int a = 0; a < g.dim; ++a) N *= g.n;
      const size_t staging = fp64 && max_group > 1 ? 2 * (size_t)max_group * N * 8 : 0;
      int rc = BURA_OK;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (budget > 0) {
          if (budget <= resident + staging) rc = BURA_ENOMEM;
          else o.hbm_budget = budget - resident - staging;
        }
      }
      hipStream_t es = nullptr;
      bura_plan_t p = nullptr;
      if (rc == BURA_OK) {
        if (hipStreamCreateWithFlags(&es, hipStreamNonBlocking) != hipSuccess) return BURA_EDEVICE;
        o.stream = es;
        rc = bura_plan_create_slots(&g, e->K, &o, &p);
        if (rc != BURA_OK) hipStreamDestroy(es);
      }
      if (rc == BURA_OK) {
        e->plan = p;
        e->stream = es;
        e->N = N;
        size_t pb = 0;
        bura_plan_info(p, nullptr, nullptr, &pb);
        e->bytes = pb;
        if (staging > 0) {
          if (hipMalloc(&e->f_stage, (size_t)max_group * N * 8) != hipSuccess ||
              hipMalloc(&e->u_stage, (size_t)max_group * N * 8) != hipSuccess) {
            return BURA_ENOMEM;
          }
          e->bytes += staging;
        }
        std::lock_guard<std::mutex> lk(mu);
        resident += e->bytes;
        ++created;
        return BURA_OK;
      }
      if (rc != BURA_ENOMEM) return rc;
      // over budget: take the idle plans out of service, then free them
      std::vector<std::unique_ptr<Entry>> victims;
      {
        std::lock_guard<std::mutex> lk(mu);
        std::vector<Entry*> idle;
        for (auto& kv : plans)
          if (kv.second.get() != e && kv.second->idle()) idle.push_back(kv.second.get());
        std::sort(idle.begin(), idle.end(), [](Entry* a, Entry* b) { return a->last_used < b->last_used; });
        for (Entry* v : idle) {
          auto it = plans.find(v->key);
          victims.push_back(std::move(it->second));
          plans.erase(it);
          resident -= std::min(resident, v->bytes);
          ++evicted;
        }
      }
      if (victims.empty()) break;
      for (auto& v : victims) destroy_entry(v.get());
    }
    return BURA_ENOMEM;
  }

  bool any_running() {
    for (auto& kv : plans)
      if (kv.second->running > 0 || !kv.second->pending.empty()) return true;
    return false;
  }

  void loop() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
      // assign queued requests to the plans of their keys (FIFO)
      Entry* to_create = nullptr;
      for (auto it = queue.begin(); it != queue.end();) {
        const std::string key = key_of((*it)->q);
        auto pe = plans.find(key);
        if (pe == plans.end()) {
          if (!to_create) {
            auto e = std::make_unique<Entry>();
            e->key = key;
            e->q = (*it)->q;
            e->K = term_class((*it)->q.k + 1);
            e->slot.assign(max_group, nullptr);
            to_create = e.get();
            plans[key] = std::move(e);
          }
          ++it;
          continue;
        }
        if (pe->second->creating) {
          ++it;
          continue;
        }
        pe->second->pending.push_back(*it);
        it = queue.erase(it);
        cv.notify_all();
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
          auto pe = plans.find(to_create->key);
          std::unique_ptr<Entry> e = std::move(pe->second);
          plans.erase(pe);
          lk.unlock();
          destroy_entry(e.get());
          lk.lock();
          cv.wait_for(lk, std::chrono::milliseconds(2));
        } else {
          // the key cannot be served: fail its queued requests
          const std::string key = to_create->key;
          for (auto it = queue.begin(); it != queue.end();) {
            if (key_of((*it)->q) == key) {
              complete(*it, rc, nullptr);
              it = queue.erase(it);
            } else {
              ++it;
            }
          }
          auto pe = plans.find(key);
          std::unique_ptr<Entry> e = std::move(pe->second);
          plans.erase(pe);
          lk.unlock();
          destroy_entry(e.get());
          lk.lock();
          cv.notify_all();
        }
        continue;
      }
      cv.wait(lk, [&]() {
        if (stop) return true;
        for (auto& r : queue)
          if (!plans.count(key_of(r->q)) || !plans[key_of(r->q)]->creating) return true;
        return false;
      });
    }
  }
};

extern "C" {

int bura_server_create(size_t hbm_budget, int max_concurrent, int max_group, bura_server_t* out) {
  if (!out || max_concurrent < 1 || max_group < 1 || max_group > 64) return BURA_EINVAL;
  auto* s = new bura_server_s();
  s->budget = hbm_budget;
  s->max_concurrent = max_concurrent;
  s->max_group = max_group;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return BURA_EDEVICE;
  }
  s->dispatcher = std::thread([s]() { s->loop(); });
  *out = s;
  return BURA_OK;
}

int bura_server_submit(bura_server_t s, const bura_request_t* req, const double* f_dev, double* u_dev,
                       uint64_t* ticket) {
  if (!s || !req || !f_dev || !u_dev || !ticket) return BURA_EINVAL;
  if ((req->dim != 2 && req->dim != 3) || req->n < 1 || !(req->alpha > 0 && req->alpha < 1) || req->k < 1 ||
      req->k > 16 || !(req->tol > 0) || (req->precision != BURA_FP64 && req->precision != BURA_MIXED))
    return BURA_EINVAL;
  auto r = std::make_shared<Req>();
  r->q = *req;
  r->f = f_dev;
  r->u = u_dev;
  // the request's terms, eq. (16): weights c_j and shifts -d_j (cached per (alpha, k))
  double c[kMaxTerms], d[kMaxTerms];
  const int rc = bura_coefficients(req->alpha, 1, req->k, c, d, &r->E);
  if (rc != BURA_OK) return rc;
  for (int j = 0; j <= req->k; ++j) {
    r->w[j] = c[j];
    r->s[j] = -d[j];
  }
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  s->tickets[r->id] = r;
  s->queue.push_back(r);
  ++s->submitted;
  *ticket = r->id;
  s->cv.notify_all();
  return BURA_OK;
}

int bura_server_poll(bura_server_t s, uint64_t ticket, bura_report_t* rep) {
  if (!s) return BURA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return BURA_EINVAL;
  if (!it->second->done) return BURA_PENDING;
  if (rep) *rep = it->second->rep;
  const int st = it->second->status;
  s->tickets.erase(it);
  return st;
}

int bura_server_wait(bura_server_t s, uint64_t ticket, bura_report_t* rep) {
  if (!s) return BURA_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return BURA_EINVAL;
  std::shared_ptr<Req> r = it->second;
  s->cv.wait(lk, [&]() { return r->done; });
  if (rep) *rep = r->rep;
  s->tickets.erase(ticket);
  return r->status;
}

int bura_server_stats(bura_server_t s, bura_server_stats_t* st) {
  if (!s || !st) return BURA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(st, 0, sizeof(*st));
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->failed = s->failed;
  st->batches = s->batches;
  st->plans_created = s->created;
  st->plans_evicted = s->evicted;
  st->unknown_pole_solves = s->unknown_pole;
  st->mean_batch = s->batches ? s->batched_requests / s->batches : 0.0;
  st->resident_bytes = s->resident;
  st->joined_running = s->joined;
  std::vector<double> l = s->latencies;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    st->p50_latency_s = l[(size_t)(0.50 * (l.size() - 1))];
    st->p99_latency_s = l[(size_t)(0.99 * (l.size() - 1))];
  }
  return BURA_OK;
}

int bura_server_reset_latency(bura_server_t s) {
  if (!s) return BURA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  s->latencies.clear();
  return BURA_OK;
}

void bura_server_destroy(bura_server_t s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // let queued and in-flight solves finish
    s->cv.wait(lk, [&]() {
      if (!s->queue.empty()) return false;
      for (auto& kv : s->plans)
        if (!kv.second->idle()) return false;
      return true;
    });
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->dispatcher.joinable()) s->dispatcher.join();
  for (auto& kv : s->plans) s->destroy_entry(kv.second.get());
  s->plans.clear();
  delete s;
}

}  // extern "C"
