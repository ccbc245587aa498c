// TEST INFRASTRUCTURE: a host-only executor for the request server's
// scheduler (paper_1612_04846_amd/csrc/bura_scheduler.h), so that admission,
// continuous batching, concurrency limits and the HBM budget can be tested
// without a GPU.  A plan is a host record with a footprint computed from its
// key; a request's solve is a countdown of outer steps (more for tighter
// tolerances), each step sleeping for a fixed time; a finished request's
// u[0] receives f[0] + the sum of its weights, so a test can see that every
// result reached its own output.
#include <atomic>
#include <chrono>
#include <cmath>
#include <thread>
#include <vector>

#include "../../paper_1612_04846_amd/csrc/bura_scheduler.h"

namespace {

struct StubPlan {
  int R = 0, K = 0;
  std::vector<int> left;     // outer steps left per rhs slot (< 0: free)
  std::vector<double> val;   // what the slot's u[0] receives
};

int steps_for(double tol) { return std::max(1, (int)std::ceil(-std::log10(tol) / 3.0)); }

struct StubExecutor final : bura::sched::Executor {
  int step_us = 1000;
  std::atomic<int> busy{0}, max_busy{0};
  std::atomic<long long> creates{0}, destroys{0};

  static size_t footprint(const bura_request_t& q, int K, int R) {
    long long N = 1;
    for (int a = 0; a < q.dim; ++a) N *= q.n;
    return (size_t)N * K * R * 8 * 4 + (q.precision == BURA_FP64 && R > 1 ? 2 * (size_t)R * N * 8 : 0);
  }
  void enter() {
    const int b = ++busy;
    int m = max_busy.load();
    while (b > m && !max_busy.compare_exchange_weak(m, b)) {
    }
  }
  void leave() { --busy; }
  void nap(int steps) { std::this_thread::sleep_for(std::chrono::microseconds((long long)step_us * steps)); }

  int create(const bura_request_t& q, int K, int R, size_t budget_left, void** plan, size_t* bytes) override {
    const size_t b = footprint(q, K, R);
    if (budget_left > 0 && b > budget_left) return BURA_ENOMEM;
    auto* p = new StubPlan();
    p->R = R;
    p->K = K;
    p->left.assign(R, -1);
    p->val.assign(R, 0.0);
    *plan = p;
    *bytes = b;
    ++creates;
    return BURA_OK;
  }
  void destroy(void* plan) override {
    delete static_cast<StubPlan*>(plan);
    ++destroys;
  }
  int reset(void* plan) override {
    auto* p = static_cast<StubPlan*>(plan);
    std::fill(p->left.begin(), p->left.end(), -1);
    return BURA_OK;
  }
  int admit(void* plan, int slot, const double* f, int nterms, const double* w, const double*, double tol) override {
    auto* p = static_cast<StubPlan*>(plan);
    if (slot < 0 || slot >= p->R || p->left[slot] >= 0) return BURA_EINVAL;
    double s = f[0];
    for (int j = 0; j < nterms; ++j) s += w[j];
    p->val[slot] = s;
    p->left[slot] = steps_for(tol);
    return BURA_OK;
  }
  int step(void* plan) override {
    auto* p = static_cast<StubPlan*>(plan);
    enter();
    nap(1);
    int active = 0;
    for (int& l : p->left)
      if (l > 0) active += --l > 0;
    leave();
    return active;
  }
  int slot_done(void* plan, int slot, double* u, bura_report_t* rep) override {
    auto* p = static_cast<StubPlan*>(plan);
    if (p->left[slot] != 0) return 0;
    u[0] = p->val[slot];
    p->left[slot] = -1;
    rep->status = BURA_OK;
    return 1;
  }
  int solve(void* plan, int g, const double* const* f, double* const* u, const int* nterms, const double* w,
            const double*, const double* tol, bura_report_t* rep) override {
    const int K = static_cast<StubPlan*>(plan)->K;
    enter();
    int steps = 1;
    for (int i = 0; i < g; ++i) steps = std::max(steps, steps_for(tol[i]));
    nap(steps);
    for (int i = 0; i < g; ++i) {
      double s = f[i][0];
      for (int j = 0; j < nterms[i]; ++j) s += w[(size_t)i * K + j];
      u[i][0] = s;
    }
    leave();
    rep->status = BURA_OK;
    return BURA_OK;
  }
};

struct StubServer {
  StubExecutor ex;
  std::unique_ptr<bura::sched::Scheduler> sched;
};

}  // namespace

extern "C" {

void* stub_server_create(size_t budget, int max_concurrent, int max_group, int step_us) {
  auto* s = new StubServer();
  s->ex.step_us = step_us;
  s->sched = std::make_unique<bura::sched::Scheduler>(&s->ex, budget, max_concurrent, max_group);
  return s;
}

// request terms: weights 1, 2, ..., k+1 (shifts 0), so a finished request's
// u[0] is f[0] + (k+1)(k+2)/2
int stub_server_submit(void* h, int dim, int n, double alpha, int k, double tol, int precision, const double* f,
                       double* u, uint64_t* ticket) {
  auto* s = static_cast<StubServer*>(h);
  bura_request_t q{};
  q.dim = dim;
  q.n = n;
  q.alpha = alpha;
  q.k = k;
  q.tol = tol;
  q.precision = precision;
  double w[bura::sched::kMaxTerms] = {}, sh[bura::sched::kMaxTerms] = {};
  for (int j = 0; j <= k; ++j) w[j] = j + 1.0;
  return s->sched->submit(q, w, sh, 0.0, f, u, ticket);
}

int stub_server_poll(void* h, uint64_t ticket) { return static_cast<StubServer*>(h)->sched->poll(ticket, nullptr); }

int stub_server_wait(void* h, uint64_t ticket) { return static_cast<StubServer*>(h)->sched->wait(ticket, nullptr); }

void stub_server_stats(void* h, bura_server_stats_t* st) { static_cast<StubServer*>(h)->sched->stats(st); }

void stub_server_counters(void* h, long long* creates, long long* destroys, int* max_busy) {
  auto* s = static_cast<StubServer*>(h);
  *creates = s->ex.creates;
  *destroys = s->ex.destroys;
  *max_busy = s->ex.max_busy;
}

size_t stub_plan_bytes(int dim, int n, int k, int precision, int max_group) {
  bura_request_t q{};
  q.dim = dim;
  q.n = n;
  q.precision = precision;
  return StubExecutor::footprint(q, bura::sched::term_class(k + 1), max_group);
}

void stub_server_destroy(void* h) { delete static_cast<StubServer*>(h); }

}  // extern "C"
