// Request server with continuous batching for fractional solves on one GPU:
// the scheduler of bura_scheduler.h driving slot plans (bura_plan_create_slots)
// on HIP streams.
//
// Every plan runs on its own non-blocking stream.  BURA_MIXED plans are
// driven through the engine's serving API (bura::serve_*): right-hand sides
// join and leave a running solve at outer refinement-step boundaries.
// BURA_FP64 plans solve a group of requests per bura_solve_slots call, their
// right-hand sides staged into one contiguous batch.  A request's result
// depends only on its own right-hand side and terms: every system's arithmetic
// and fixed-order reductions are its own, and a system admitted at a step
// boundary goes through the same operations as in a solve by itself.
#include <hip/hip_runtime.h>

#include <memory>

#include "bura_internal.h"
#include "bura_scheduler.h"

namespace {

struct HipPlan {
  bura_plan_t plan = nullptr;
  hipStream_t stream = nullptr;   // the plan's caller stream; also carries the staging copies
  double* f_stage = nullptr;      // FP64 groups of several requests
  double* u_stage = nullptr;
  long long N = 0;
};

struct HipExecutor final : bura::sched::Executor {
  int device = 0;

  void bind_thread() override { hipSetDevice(device); }

  int create(const bura_request_t& q, int K, int max_group, size_t budget_left, void** out,
             size_t* bytes) override {
    const bool fp64 = q.precision == BURA_FP64;
    long long N = 1;
    for (int a = 0; a < q.dim; ++a) N *= q.n;
    const size_t staging = fp64 && max_group > 1 ? 2 * (size_t)max_group * N * 8 : 0;
    bura_grid_t g{};
    g.dim = q.dim;
    g.n = q.n;
    bura_opts_t o;
    bura_opts_default(&o);
    o.precision = q.precision;
    o.nrhs_max = max_group;
    if (budget_left > 0) {
      if (budget_left <= staging) return BURA_ENOMEM;
      o.hbm_budget = budget_left - staging;
    }
    auto h = std::make_unique<HipPlan>();
    h->N = N;
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return BURA_EDEVICE;
    o.stream = h->stream;
    int rc = bura_plan_create_slots(&g, K, &o, &h->plan);
    if (rc == BURA_OK && staging > 0 &&
        (hipMalloc(&h->f_stage, (size_t)max_group * N * 8) != hipSuccess ||
         hipMalloc(&h->u_stage, (size_t)max_group * N * 8) != hipSuccess))
      rc = BURA_ENOMEM;
    if (rc != BURA_OK) {
      destroy(h.release());
      return rc;
    }
    size_t pb = 0;
    bura_plan_info(h->plan, nullptr, nullptr, &pb);
    *bytes = pb + staging;
    *out = h.release();
    return BURA_OK;
  }

  void destroy(void* p) override {
    auto* h = static_cast<HipPlan*>(p);
    if (!h) return;
    hipSetDevice(device);
    if (h->plan) bura_plan_destroy(h->plan);
    if (h->f_stage) hipFree(h->f_stage);
    if (h->u_stage) hipFree(h->u_stage);
    if (h->stream) hipStreamDestroy(h->stream);
    delete h;
  }

  int reset(void* p) override { return bura::serve_reset(static_cast<HipPlan*>(p)->plan); }

  int admit(void* p, int slot, const double* f, int nterms, const double* w, const double* s, double tol) override {
    return bura::serve_admit(static_cast<HipPlan*>(p)->plan, slot, f, nterms, w, s, tol);
  }

  int step(void* p) override { return bura::serve_step(static_cast<HipPlan*>(p)->plan); }

  int slot_done(void* p, int slot, double* u, bura_report_t* rep) override {
    return bura::serve_slot_done(static_cast<HipPlan*>(p)->plan, slot, u, rep);
  }

  int solve(void* p, int g, const double* const* f, double* const* u, const int* nterms, const double* w,
            const double* s, const double* tol, bura_report_t* rep) override {
    auto* h = static_cast<HipPlan*>(p);
    const double* fb = f[0];
    double* ub = u[0];
    if (g > 1) {
      for (int i = 0; i < g; ++i)
        hipMemcpyAsync(h->f_stage + (size_t)i * h->N, f[i], h->N * 8, hipMemcpyDeviceToDevice, h->stream);
      fb = h->f_stage;
      ub = h->u_stage;
    }
    const int rc = bura_solve_slots(h->plan, fb, ub, g, nterms, w, s, tol, rep);
    if (g > 1 && rc != BURA_EINVAL) {
      for (int i = 0; i < g; ++i)
        hipMemcpyAsync(u[i], h->u_stage + (size_t)i * h->N, h->N * 8, hipMemcpyDeviceToDevice, h->stream);
    }
    hipStreamSynchronize(h->stream);
    return rc;
  }
};

}  // namespace

struct bura_server_s {
  HipExecutor ex;
  std::unique_ptr<bura::sched::Scheduler> sched;
};

extern "C" {

int bura_server_create(size_t hbm_budget, int max_concurrent, int max_group, bura_server_t* out) {
  if (!out || max_concurrent < 1 || max_group < 1 || max_group > 64) return BURA_EINVAL;
  auto* s = new bura_server_s();
  if (hipGetDevice(&s->ex.device) != hipSuccess) {
    delete s;
    return BURA_EDEVICE;
  }
  s->sched = std::make_unique<bura::sched::Scheduler>(&s->ex, hbm_budget, max_concurrent, max_group);
  *out = s;
  return BURA_OK;
}

int bura_server_submit(bura_server_t s, const bura_request_t* req, const double* f_dev, double* u_dev,
                       uint64_t* ticket) {
  if (!s || !req || !f_dev || !u_dev || !ticket) return BURA_EINVAL;
  if ((req->dim != 2 && req->dim != 3) || req->n < 1 || !(req->alpha > 0 && req->alpha < 1) || req->k < 1 ||
      req->k > 16 || !(req->tol > 0) || (req->precision != BURA_FP64 && req->precision != BURA_MIXED))
    return BURA_EINVAL;
  // the request's terms, eq. (16): weights c_j and shifts -d_j (cached per (alpha, k))
  constexpr int M = bura::sched::kMaxTerms;
  double c[M], d[M], w[M], sh[M], E = 0.0;
  const int rc = bura_coefficients(req->alpha, 1, req->k, c, d, &E);
  if (rc != BURA_OK) return rc;
  for (int j = 0; j <= req->k; ++j) {
    w[j] = c[j];
    sh[j] = -d[j];
  }
  return s->sched->submit(*req, w, sh, E, f_dev, u_dev, ticket);
}

int bura_server_poll(bura_server_t s, uint64_t ticket, bura_report_t* rep) {
  if (!s) return BURA_EINVAL;
  return s->sched->poll(ticket, rep);
}

int bura_server_wait(bura_server_t s, uint64_t ticket, bura_report_t* rep) {
  if (!s) return BURA_EINVAL;
  return s->sched->wait(ticket, rep);
}

int bura_server_stats(bura_server_t s, bura_server_stats_t* st) {
  if (!s || !st) return BURA_EINVAL;
  s->sched->stats(st);
  return BURA_OK;
}

int bura_server_reset_latency(bura_server_t s) {
  if (!s) return BURA_EINVAL;
  s->sched->reset_latency();
  return BURA_OK;
}

void bura_server_destroy(bura_server_t s) {
  if (!s) return;
  s->sched.reset();   // waits for queued and running requests, then frees every plan
  delete s;
}

}  // extern "C"
