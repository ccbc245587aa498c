// Request server with continuous batching for fractional solves on one GPU.
//
// Requests (grid, alpha, k, tolerance, precision, f, u) are queued on submit.
// A dispatcher thread keeps one slot plan (bura_plan_create_slots) resident per
// (dim, n, precision): every right-hand side of a slot plan's solve carries its
// own partial-fraction terms and tolerance, so queued requests for the same
// grid are batched into one solve whatever their alpha, k and tolerance.  Each
// plan runs one solve at a time on its own stream, and several plans run
// concurrently, so work of different grids overlaps on the device; a request
// never waits for requests of other grids.  New plans are admitted against an
// HBM budget; idle plans are evicted least recently used first when the budget
// would be exceeded.  Each request's result depends only on its own
// right-hand side and terms (the solver's per-system arithmetic and
// fixed-order reductions do not depend on the other systems of a batch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
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

constexpr int kSlotTerms = 17;   // k <= 16 poles: up to 17 terms per request

struct Req {
  uint64_t id = 0;
  bura_request_t q{};
  double w[kSlotTerms] = {}, s[kSlotTerms] = {};   // the request's terms (weights, shifts)
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
  bura_plan_t plan = nullptr;
  bool busy = false;
  bura_ticket_t ticket = 0;   // the running solve
  std::vector<std::shared_ptr<Req>> group;
  double* f_stage = nullptr;
  double* u_stage = nullptr;
  size_t bytes = 0;
  long long N = 0;
  Clock::time_point last_used;
  hipStream_t stream = nullptr;   // the plan's caller stream; also carries the staging copies
};

std::string key_of(const bura_request_t& q) {
  char b[64];
  std::snprintf(b, sizeof(b), "%d/%d/%d", q.dim, q.n, q.precision);
  return b;
}

}  // namespace

struct bura_server_s {
  size_t budget = 0;
  int max_concurrent = 4;
  int max_group = 4;
  std::mutex mu;
  std::condition_variable cv;
  std::list<std::shared_ptr<Req>> queue;   // erase keeps other iterators valid
  std::map<uint64_t, std::shared_ptr<Req>> tickets;
  std::map<std::string, std::unique_ptr<Entry>> plans;
  std::thread dispatcher;
  bool stop = false;
  uint64_t next_id = 1;
  int device = 0;
  // statistics
  long long submitted = 0, completed = 0, failed = 0, batches = 0, created = 0, evicted = 0;
  double unknown_pole = 0.0;
  double batched_requests = 0.0;
  std::vector<double> latencies;
  size_t resident = 0;

  void destroy_entry(Entry* e) {
    if (e->plan) bura_plan_destroy(e->plan);
    if (e->f_stage) hipFree(e->f_stage);
    if (e->u_stage) hipFree(e->u_stage);
    if (e->stream) hipStreamDestroy(e->stream);
    resident -= std::min(resident, e->bytes);
  }

  // create the plan for a request's key, evicting idle plans if the budget needs it
  Entry* admit(const std::shared_ptr<Req>& r, int* err) {
    const std::string key = key_of(r->q);
    auto it = plans.find(key);
    if (it != plans.end()) return it->second.get();
    for (int attempt = 0; attempt < 2; ++attempt) {
      bura_grid_t g{};
      g.dim = r->q.dim;
      g.n = r->q.n;
      bura_opts_t o;
      bura_opts_default(&o);
      o.precision = r->q.precision;
      o.nrhs_max = max_group;
      long long N = 1;
      for (int a = 0; a < g.dim; ++a) N *= g.n;
      const size_t staging = max_group > 1 ? 2 * (size_t)max_group * N * 8 : 0;
      if (budget > 0) {
        if (budget <= resident + staging) {
          *err = BURA_ENOMEM;
        } else {
          o.hbm_budget = budget - resident - staging;
        }
      }
      // the plan is ordered against this entry's own stream (never the legacy
      // null stream, which must not be used while other plans capture graphs)
      hipStream_t es = nullptr;
      if (hipStreamCreateWithFlags(&es, hipStreamNonBlocking) != hipSuccess) {
        *err = BURA_EDEVICE;
        return nullptr;
      }
      o.stream = es;
      bura_plan_t p = nullptr;
      int rc = (*err == BURA_ENOMEM) ? BURA_ENOMEM : bura_plan_create_slots(&g, kSlotTerms, &o, &p);
      if (rc != BURA_OK) hipStreamDestroy(es);
      if (rc == BURA_OK) {
        auto e = std::make_unique<Entry>();
        e->key = key;
        e->q = r->q;
        e->plan = p;
        e->N = N;
        e->stream = es;
        size_t pb = 0;
        bura_plan_info(p, nullptr, nullptr, &pb);
        e->bytes = pb;
        if (max_group > 1) {
          if (hipMalloc(&e->f_stage, (size_t)max_group * N * 8) != hipSuccess ||
              hipMalloc(&e->u_stage, (size_t)max_group * N * 8) != hipSuccess) {
            destroy_entry(e.get());
            *err = BURA_ENOMEM;
            return nullptr;
          }
          e->bytes += staging;
        }
        e->last_used = Clock::now();
        resident += e->bytes;
        ++created;
        Entry* raw = e.get();
        plans[key] = std::move(e);
        *err = BURA_OK;
        return raw;
      }
      if (rc != BURA_ENOMEM) {
        *err = rc;
        return nullptr;
      }
      // over budget: evict idle plans, least recently used first, then retry once
      *err = BURA_OK;
      std::vector<Entry*> idle;
      for (auto& kv : plans)
        if (!kv.second->busy) idle.push_back(kv.second.get());
      if (idle.empty()) break;
      std::sort(idle.begin(), idle.end(), [](Entry* a, Entry* b) { return a->last_used < b->last_used; });
      for (Entry* e : idle) {
        destroy_entry(e);
        plans.erase(e->key);
        ++evicted;
      }
    }
    *err = BURA_ENOMEM;
    return nullptr;
  }

  void finish(Entry* e, int rc, const bura_report_t& rep) {
    const size_t g = e->group.size();
    if (g > 1 && rc != BURA_EINVAL) {
      for (size_t i = 0; i < g; ++i)
        hipMemcpyAsync(e->group[i]->u, e->u_stage + i * e->N, e->N * 8, hipMemcpyDeviceToDevice, e->stream);
      hipStreamSynchronize(e->stream);
    }
    const auto now = Clock::now();
    for (auto& r : e->group) {
      r->status = rc;
      r->rep = rep;
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
    e->group.clear();
    e->busy = false;
    e->last_used = now;
  }

  void fail(const std::shared_ptr<Req>& r, int rc) {
    r->status = rc;
    r->rep.status = rc;
    r->t_done = Clock::now();
    r->done = true;
    ++completed;
    ++failed;
  }

  void loop() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
      bool progressed = false;
      int active = 0;
      // completions
      for (auto& kv : plans) {
        Entry* e = kv.second.get();
        if (!e->busy) continue;
        bura_report_t rep{};
        const int rc = bura_poll(e->ticket, &rep);
        if (rc == BURA_PENDING) {
          ++active;
          continue;
        }
        finish(e, rc, rep);
        progressed = true;
      }
      if (progressed) cv.notify_all();
      // dispatch: first-come first-served per key; a busy plan never blocks other keys
      for (auto it = queue.begin(); it != queue.end() && active < max_concurrent;) {
        std::shared_ptr<Req> r = *it;
        int err = BURA_OK;
        Entry* e = admit(r, &err);
        if (!e) {
          if (err == BURA_ENOMEM) {
            bool any_busy = false;
            for (auto& kv : plans) any_busy |= kv.second->busy;
            if (any_busy) {   // wait for memory to free up
              ++it;
              continue;
            }
          }
          fail(r, err);
          it = queue.erase(it);
          cv.notify_all();
          continue;
        }
        if (e->busy) {
          ++it;
          continue;
        }
        // batch: this request and later queued ones with the same key
        e->group.clear();
        e->group.push_back(r);
        it = queue.erase(it);
        for (auto jt = it; jt != queue.end() && (int)e->group.size() < max_group;) {
          if (key_of((*jt)->q) == e->key) {
            if (jt == it) {
              e->group.push_back(*jt);
              jt = queue.erase(jt);
              it = jt;
            } else {
              e->group.push_back(*jt);
              jt = queue.erase(jt);
            }
          } else {
            ++jt;
          }
        }
        const int g = (int)e->group.size();
        const double* f = r->f;
        double* u = r->u;
        int nterms[64];
        double w[64 * kSlotTerms] = {}, sh[64 * kSlotTerms] = {}, tol[64];
        for (int i = 0; i < g; ++i) {
          const Req& q = *e->group[i];
          nterms[i] = q.q.k + 1;
          tol[i] = q.q.tol;
          for (int j = 0; j <= q.q.k; ++j) {
            w[i * kSlotTerms + j] = q.w[j];
            sh[i * kSlotTerms + j] = q.s[j];
          }
        }
        if (g > 1) {
          for (int i = 0; i < g; ++i)
            hipMemcpyAsync(e->f_stage + (size_t)i * e->N, e->group[i]->f, e->N * 8, hipMemcpyDeviceToDevice,
                           e->stream);
          hipStreamSynchronize(e->stream);
          f = e->f_stage;
          u = e->u_stage;
        }
        const int rc = bura_submit_slots(e->plan, f, u, g, nterms, w, sh, tol, &e->ticket);
        if (rc != BURA_OK) {
          for (auto& q : e->group) fail(q, rc);
          e->group.clear();
          cv.notify_all();
          continue;
        }
        e->busy = true;
        ++batches;
        batched_requests += g;
        ++active;
        progressed = true;
      }
      if (!progressed) cv.wait_for(lk, std::chrono::microseconds(100));
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
  double c[kSlotTerms], d[kSlotTerms];
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
        if (kv.second->busy) return false;
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
