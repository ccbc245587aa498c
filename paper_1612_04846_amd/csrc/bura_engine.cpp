// Solver engine and C ABI: operator hierarchy, device workspace, the PCG /
// iterative-refinement loops over batches of shifted systems, and the combine
// u = sum_j c_j (A - d_j I)^-1 f of Section 2.2, eq. (16).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bura_internal.h"

using namespace bura;

namespace {

thread_local std::string g_last_error;

#define HIPCHK(expr)                                        \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) {                                 \
      g_last_error = hipGetErrorString(e_);                 \
      return e_ == hipErrorOutOfMemory ? BURA_ENOMEM : BURA_EDEVICE; \
    }                                                       \
  } while (0)

constexpr size_t kLdsCap = 64 * 1024;

struct HostLevel {
  int n = 0;
  long long N = 0;
  double wc = 0.0;                       // constant face weight a/(Lambda h_l^2)
  std::vector<double> wf[3];             // variable face weights, scaled
  double* d_wf64[3] = {nullptr, nullptr, nullptr};
  float* d_wf32[3] = {nullptr, nullptr, nullptr};
};

template <typename T>
struct Work {
  T* x = nullptr;   // PCG iterate (FP64 path: the solution; MIXED: the correction e)
  T* r = nullptr;
  T* z = nullptr;
  T* zt = nullptr;
  T* p = nullptr;
  T* p2 = nullptr;  // p ping-pong partner (p_new = z + beta p_old is written to the other buffer)
  T* q = nullptr;
  T* r2 = nullptr;  // r ping-pong partner when the residual update is folded into the down kernel
  std::vector<T*> xl, tl, bl;   // levels 1..lc (index by level)
  T* shift = nullptr;
};

size_t face_count(int dim, int n, int axis) {
  size_t c = (size_t)(n + 1);
  for (int a = 1; a < dim; ++a) c *= (size_t)n;
  (void)axis;
  return c;
}

inline double hmean(double a, double b) { return 2.0 * a * b / (a + b); }

// One stage of a sequential form: solve the terms [tb, te) against an input
// vector (the caller's f, an earlier stage's output, or the solution of one
// term) and write out = base_w * base + sum_j w_j x_j, where base is the
// stage buffer (the previous stage's output) or nothing.  Stages run in order;
// the last one writes the caller's u.  Used for the multi-step BURA
// (Section 4.4) and the zero-pole product form (remark on the product form in
// Section 2.2).
struct Stage {
  enum Input { F = 0, PREV = 1, SOL = 2 };
  int tb = 0, te = 0;
  int input = F;
  int sol_term = 0;      // input == SOL: the term whose solution is the right-hand side
  bool base = false;     // add base_w * (previous stage output)
  double base_w = 0.0;
};

}  // namespace

struct bura_plan_s {
  int dim = 2, n = 0;
  long long N = 0;
  bool var = false;
  double lambda = 0.0;
  // rational form u = sum_j w_j (A + s_j)^-1 f
  int nterms = 0;
  std::vector<double> w, s;   // weights c_j and shifts s_j = -d_j
  // outputs: output i combines the terms [out_begin[i], out_end[i]) (several
  // fractional powers of the same operator solved in one batch)
  int nout = 1;
  std::vector<int> out_begin, out_end;
  std::vector<Stage> stages;   // empty: all terms at once against f
  double* d_buf = nullptr;     // stage output between stages, nrhs_max x N FP64
  double E = 0.0;
  bura_opts_t opts{};
  hipStream_t stream = nullptr;
  int device = 0;
  // hierarchy
  std::vector<HostLevel> lev;
  int lc = -1;                 // first level solved in LDS; -1: no multigrid (Jacobi PCG)
  bool unfused = false;        // the one-kernel-per-step V-cycle (BURA_VARIANT_UNFUSED)
  // PCG vector updates folded into other passes: x += alpha p deferred to the
  // next stencil-product pass, r -= alpha q done by the first fine-level
  // pre-smoothing kernel (the fused down kernel in 2D, k_jacobi0_rup
  // otherwise) into a second residual buffer (off with BURA_VARIANT_NO_FOLDXR)
  bool foldxr = false;
  size_t lds_bytes = 0;
  // launch-shape variant of the 2D stencil product and, per global level, of
  // the fused down and up kernels (0 = default; chosen by tune_tiles)
  int tile_spmv = 0;
  std::vector<int> tile_down, tile_up;
  int S = 0;                   // systems = nterms * nrhs_max
  // slot plan (bura_plan_create_slots): weights, shifts and tolerances are set
  // per solve and per rhs; d_wsys / d_tol hold them per system, h_slot is the
  // pinned staging area of one solve's per-system values
  bool slots = false;
  double* d_wsys = nullptr;
  double* d_tol = nullptr;
  void* h_slot = nullptr;
  // device buffers
  Work<double> w64;
  Work<float> w32;
  double* x64 = nullptr;       // MIXED: FP64 solutions
  double* partial = nullptr;
  size_t partial_len = 0;
  double* d_w = nullptr;       // combine weights
  double* d_shift64 = nullptr;
  float* d_shift32 = nullptr;
  SysState st{};
  void* state_block = nullptr;
  int* h_flags = nullptr;      // pinned host mirror of active flags
  std::vector<void*> allocs;
  size_t device_bytes = 0;
  // bura_solve_static: every device buffer is carved from the caller-provided
  // region [ws_base, ws_base + ws_cap) instead of hipMalloc; the plan then
  // runs on the caller's stream (no own stream, event or graphs) and keeps its
  // host mirrors in ordinary host memory instead of pinned allocations
  char* ws_base = nullptr;
  size_t ws_cap = 0, ws_used = 0;
  bool owns_stream = true;
  std::vector<char> host_mirror;
  // profiling (events around launches + device byte counters per kernel class)
  struct Prof {
    bool on = false;
    unsigned mask = 0;                        // kernel classes timed with events
    unsigned long long* d_ctr = nullptr;
    std::vector<hipEvent_t> pool;             // eager-mode events, reused after each flush
    size_t used = 0;
    std::vector<std::pair<int, size_t>> rec;   // pending (class, index of the start event; stop = +1)
    double ms[BURA_K_COUNT] = {};
    long long launches[BURA_K_COUNT] = {};
  } prof;
  // graphs: one captured chunk of PCG iterations per (precision, batch, tolerance)
  struct Graph {
    hipGraphExec_t exec = nullptr;
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> ev;   // events recorded inside the graph
  };
  std::map<std::string, Graph> graphs;
  bool capturing = false;
  bool capture_failed = false;
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> cap_ev;
  bool use_graphs = true;
  bool fold = false;                   // scalar updates folded into the producing kernels
  unsigned int* d_cnt = nullptr;       // per-system block counters for the folded updates
  hipStream_t user_stream = nullptr;   // caller's stream (opts.stream)
  hipEvent_t join_ev = nullptr;
  void* h_state = nullptr;             // pinned mirror of the scalar state for reports
  double run_tol = 0.0;                // stopping tolerance of the solve in progress
  // a posteriori error bound (see do_solve): a guaranteed lower bound of the
  // spectrum of the scaled operator, the combine weights as applied, the
  // squared norms of the outputs (device, and their host copy after the state)
  double lam_lb = 0.0;
  std::vector<double> w_applied;
  double* d_upart = nullptr;   // rows x ceil(N/256) partial sums
  double* d_unorm = nullptr;   // rows = nout x nrhs_max
  double* d_tol_err = nullptr; // MIXED: per-system refinement tolerances set by opts.err_tol
  // continuous batching (bura::serve_*): the slots' right-hand sides, the
  // systems being initialised, and the host copy of each slot's terms
  double* d_fserve = nullptr;  // [nrhs_max][N]
  int* d_init = nullptr;       // [S]
  std::vector<int> serve_nterms;
  std::vector<double> serve_w, serve_s, serve_tol;
  // asynchronous solves: a FIFO of submitted solves run in order by one
  // worker thread; exec_mu serialises them with synchronous solves
  struct Job {
    const double* f = nullptr;
    double* u = nullptr;
    int nrhs = 0;
    double tol = 0.0;
    uint64_t ticket = 0;
    bool slots = false;
    std::vector<int> nterms;
    std::vector<double> w, s, tolv;
  };
  std::mutex exec_mu;
  std::mutex q_mu;
  std::condition_variable q_cv;
  std::deque<Job> queue;
  int running = 0;
  bool stop = false;
  std::thread worker;
};

namespace {

int dev_alloc(bura_plan_t P, void** ptr, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (P->ws_base) {
    // static workspace: 256-byte aligned carve-outs, nothing is freed
    const size_t at = (P->ws_used + 255) & ~(size_t)255;
    if (at > P->ws_cap || bytes > P->ws_cap - at) {
      g_last_error = "workspace larger than the static scratch array";
      *ptr = nullptr;
      return BURA_ETOOBIG;
    }
    *ptr = P->ws_base + at;
    P->ws_used = at + bytes;
    P->device_bytes += bytes;
    return BURA_OK;
  }
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    g_last_error = hipGetErrorString(e);
    *ptr = nullptr;
    return BURA_ENOMEM;
  }
  P->allocs.push_back(*ptr);
  P->device_bytes += bytes;
  return BURA_OK;
}

// Clear device memory of the plan: a fill kernel for a static-workspace plan
// (whose caller may be capturing the stream), hipMemsetAsync otherwise.
int dev_zero(bura_plan_t P, void* ptr, size_t bytes) {
  if (P->ws_base) {
    launch_zero(ptr, bytes, P->stream);
    return BURA_OK;
  }
  return hipMemsetAsync(ptr, 0, bytes, P->stream) == hipSuccess ? BURA_OK : BURA_EDEVICE;
}

// Records start/stop events around one launch of class `cls` when profiling;
// `ctr` is the device byte counter the kernel adds to (nullptr otherwise).
struct ProfScope {
  bura_plan_t P;
  long idx = -1;
  hipEvent_t e1 = nullptr;
  unsigned long long* ctr = nullptr;
  ProfScope(bura_plan_t P_, int cls) : P(P_) {
    auto& pr = P->prof;
    if (!pr.on) return;
    ctr = pr.d_ctr + cls;
    if (!(pr.mask & (1u << cls))) return;
    if (P->capturing) {
      // events recorded inside the graph being captured (owned by that graph)
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) { P->capture_failed = true; return; }
      if (hipEventCreate(&b) != hipSuccess) { hipEventDestroy(a); P->capture_failed = true; return; }
      // external record nodes: the replayed graph writes real timestamps
      if (hipEventRecordWithFlags(a, P->stream, hipEventRecordExternal) != hipSuccess) P->capture_failed = true;
      P->cap_ev.emplace_back(cls, a, b);
      e1 = b;
      return;
    }
    while (pr.pool.size() < pr.used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      pr.pool.push_back(e);
    }
    idx = (long)pr.used;
    pr.used += 2;
    pr.rec.emplace_back(cls, (size_t)idx);
    hipEventRecord(pr.pool[idx], P->stream);
  }
  ~ProfScope() {
    if (e1) {
      if (hipEventRecordWithFlags(e1, P->stream, hipEventRecordExternal) != hipSuccess) P->capture_failed = true;
    } else if (idx >= 0) {
      hipEventRecord(P->prof.pool[idx + 1], P->stream);
    }
  }
};

// after a stream synchronisation: fold the pending eager events into the totals
void prof_flush(bura_plan_t P) {
  auto& pr = P->prof;
  for (const auto& r : pr.rec) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, pr.pool[r.second], pr.pool[r.second + 1]) == hipSuccess) {
      pr.ms[r.first] += t;
      pr.launches[r.first] += 1;
    }
  }
  pr.rec.clear();
  pr.used = 0;
  (void)hipGetLastError();   // an unreadable event must not surface as a later launch error
}

void prof_graph(bura_plan_t P, const bura_plan_s::Graph& g) {
  if (!P->prof.on) return;
  for (const auto& e : g.ev) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, std::get<1>(e), std::get<2>(e)) == hipSuccess) {
      P->prof.ms[std::get<0>(e)] += t;
      P->prof.launches[std::get<0>(e)] += 1;
    }
  }
  (void)hipGetLastError();
}

void destroy_graphs(bura_plan_t P) {
  for (auto& kv : P->graphs) {
    if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
    for (auto& e : kv.second.ev) {
      hipEventDestroy(std::get<1>(e));
      hipEventDestroy(std::get<2>(e));
    }
  }
  P->graphs.clear();
}

template <typename T>
LevelDev<T> level_view(const bura_plan_t P, int l) {
  const HostLevel& H = P->lev[l];
  LevelDev<T> L;
  L.n = H.n;
  L.N = H.N;
  L.wc = (T)H.wc;
  if (P->var) {
    if (sizeof(T) == 8) {
      L.wf0 = (const T*)H.d_wf64[0];
      L.wf1 = (const T*)H.d_wf64[1];
      L.wf2 = (const T*)H.d_wf64[2];
    } else {
      L.wf0 = (const T*)H.d_wf32[0];
      L.wf1 = (const T*)H.d_wf32[1];
      L.wf2 = (const T*)H.d_wf32[2];
    }
  } else {
    L.wf0 = L.wf1 = L.wf2 = nullptr;
  }
  return L;
}

double default_omega(int dim) { return dim == 2 ? 0.8 : 6.0 / 7.0; }

// Damping of the nu sweeps of a half-cycle.  opts.omega > 0: that weight for
// every sweep.  Otherwise FP64 solves use the uniform default_omega, and the
// FP32 inner solves of BURA_MIXED use the reciprocals of the roots of the
// degree-nu Chebyshev polynomial on [lo, 2] (D^-1 A has its spectrum in
// (0, 2], its high-frequency part above ~0.5 in 2D and ~1/3 in 3D for full
// coarsening), which damp that range by 1/T_nu((2 + lo)/(2 - lo)) instead of
// max|1 - omega t|^nu (2D, nu = 2: 0.21 against 0.36).  The Chebyshev weights
// shorten the 1e-5 inner solves (7 % less time on the 1023^2 three-alpha
// workload, 4-7 % on 255^3) but lengthen the 1e-10 FP64 solves (+5 %
// iterations: they damp the poles with large shifts, whose spectrum sits near
// 1, less than omega = 0.8 does), hence the split.  lo was chosen by timing:
// 0.4 in 2D, 0.5 in 3D (0.4 and 0.6 were slower there).  The weights are
// polynomials in the same operator, so the smoother stays symmetric in any
// order.
template <typename T>
Sweeps<T> sweep_weights(const bura_plan_t P, int nu) {
  Sweeps<T> s{};
  const double om = P->opts.omega;
  const double lo = nu >= 3 ? 0.3 : (P->dim == 3 ? 0.5 : 0.4);
  const bool cheb = !(om > 0) && sizeof(T) == 4;
  for (int i = 0; i < 3; ++i) {
    double w = om > 0 ? om : default_omega(P->dim);
    if (cheb && i < nu) {
      const double pi = 3.141592653589793;
      const double th = (lo + 2.0) / 2 + (2.0 - lo) / 2 * std::cos((2 * i + 1) * pi / (2 * nu));
      w = 1.0 / th;
    }
    s.w[i] = (T)w;
  }
  return s;
}

// ---------------------------------------------------------------------------
// hierarchy on the host (Section 1.4 scaling; coarse operators by
// rediscretisation with series/parallel averaging of the face coefficients)
// ---------------------------------------------------------------------------
int build_levels(bura_plan_t P, const bura_grid_t* g) {
  const int dim = P->dim, n = P->n;
  const double h = 1.0 / (n + 1);
  // fine faces (unscaled a_f) and Gershgorin bound of A~ = h^-2 * flux form
  HostLevel L0;
  L0.n = n;
  L0.N = 1;
  for (int a = 0; a < dim; ++a) L0.N *= n;
  const int m = n + 2;
  auto A = [&](int i, int j, int k) -> double {   // lattice value, 0..n+1 per axis
    return g->coeff[((size_t)k * m + j) * m + i];
  };
  if (P->var) {
    for (int a = 0; a < dim; ++a) L0.wf[a].assign(face_count(dim, n, a), 0.0);
    const int nk = dim == 3 ? n : 1;
    for (int k = 0; k < nk; ++k)
      for (int j = 0; j < n; ++j)
        for (int f = 0; f <= n; ++f) {
          const int K = dim == 3 ? k + 1 : 0;
          L0.wf[0][((size_t)k * n + j) * (n + 1) + f] = hmean(A(f, j + 1, K), A(f + 1, j + 1, K));
        }
    for (int k = 0; k < nk; ++k)
      for (int f = 0; f <= n; ++f)
        for (int i = 0; i < n; ++i) {
          const int K = dim == 3 ? k + 1 : 0;
          L0.wf[1][((size_t)k * (n + 1) + f) * n + i] = hmean(A(i + 1, f, K), A(i + 1, f + 1, K));
        }
    if (dim == 3)
      for (int f = 0; f <= n; ++f)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i)
            L0.wf[2][((size_t)f * n + j) * n + i] = hmean(A(i + 1, j + 1, f), A(i + 1, j + 1, f + 1));
  }
  // Gershgorin: row i of A~ has diagonal sum_f a_f and off-diagonals -a_f for
  // faces to interior neighbours: bound = max_i sum_f a_f (1 + [nb interior]) / h^2
  double gb = 0.0;
  {
    const int nk = dim == 3 ? n : 1;
    for (int k = 0; k < nk; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double row = 0.0;
          auto face = [&](int axis, size_t idx, bool nb_interior) {
            const double a = P->var ? L0.wf[axis][idx] : 1.0;
            row += a * (nb_interior ? 2.0 : 1.0);
          };
          face(0, ((size_t)k * n + j) * (n + 1) + i, i > 0);
          face(0, ((size_t)k * n + j) * (n + 1) + i + 1, i < n - 1);
          face(1, ((size_t)k * (n + 1) + j) * n + i, j > 0);
          face(1, ((size_t)k * (n + 1) + j + 1) * n + i, j < n - 1);
          if (dim == 3) {
            face(2, ((size_t)k * n + j) * n + i, k > 0);
            face(2, ((size_t)(k + 1) * n + j) * n + i, k < n - 1);
          }
          gb = std::max(gb, row);
          if (!P->var && (dim == 2 || n > 2) && i == 1 && j == 1 && (dim == 2 || k == 1)) {
            // constant coefficient: an interior node with all neighbours interior attains the max
            k = nk; j = n; i = n;
          }
        }
    gb /= h * h;
    // constant coefficients: the paper's scaling 4d/h^2 (h^2/8 in 2D) for every
    // n; Gershgorin's bound equals it for n >= 3 and is smaller below that
    if (!P->var) gb = 4.0 * dim / (h * h);
  }
  if (g->lambda_upper > 0.0) {
    P->lambda = g->lambda_upper;   // caller's bound (cannot be verified cheaply)
  } else {
    P->lambda = gb;
  }
  // lower bound of the spectrum of A = A~/Lambda: the Laplacian's smallest
  // eigenvalue 4 dim sin^2(pi h/2)/h^2; with coefficients x^T A~ x =
  // h^-2 sum_faces a_f (x_i - x_nb)^2 >= a_min x^T A~_Laplacian x
  {
    double amin = P->var ? HUGE_VAL : 1.0;
    if (P->var)
      for (int a = 0; a < dim; ++a)
        for (double v : L0.wf[a]) amin = std::min(amin, v);
    const double sn = std::sin(3.14159265358979323846 * h / 2.0);
    P->lam_lb = amin * 4.0 * dim * sn * sn / (h * h) / P->lambda * (1.0 - 1e-12);
  }
  const double scale0 = 1.0 / (P->lambda * h * h);
  L0.wc = scale0;
  if (P->var)
    for (int a = 0; a < dim; ++a)
      for (double& v : L0.wf[a]) v *= scale0;
  P->lev.clear();
  P->lev.push_back(std::move(L0));
  // coarse levels
  while (true) {
    const HostLevel& F = P->lev.back();
    if (F.n < 3 || (F.n % 2) == 0) break;
    HostLevel C;
    C.n = (F.n - 1) / 2;
    C.N = 1;
    for (int a = 0; a < dim; ++a) C.N *= C.n;
    C.wc = F.wc * 0.25;
    if (P->var) {
      const int nf = F.n, nc = C.n;
      const double wt[3] = {0.25, 0.5, 0.25};
      for (int a = 0; a < dim; ++a) C.wf[a].assign(face_count(dim, nc, a), 0.0);
      const int nkc = dim == 3 ? nc : 1;
      // axis-a coarse face between coarse nodes X-1 and X (along a) spans fine faces 2X and 2X+1;
      // transverse fine rows 2T+1+dt, weights (1/4,1/2,1/4).
      for (int a = 0; a < dim; ++a) {
        for (int K = 0; K < (a == 2 ? nc + 1 : nkc); ++K)
          for (int J = 0; J < (a == 1 ? nc + 1 : nc); ++J)
            for (int I = 0; I < (a == 0 ? nc + 1 : nc); ++I) {
              double acc = 0.0;
              const int dkmin = (dim == 3 && a != 2) ? -1 : 0, dkmax = (dim == 3 && a != 2) ? 1 : 0;
              const int djmin = (a != 1) ? -1 : 0, djmax = (a != 1) ? 1 : 0;
              const int dimin = (a != 0) ? -1 : 0, dimax = (a != 0) ? 1 : 0;
              for (int dk = dkmin; dk <= dkmax; ++dk)
                for (int dj = djmin; dj <= djmax; ++dj)
                  for (int di = dimin; di <= dimax; ++di) {
                    double wgt = 1.0;
                    int fi, fj, fk;
                    if (a == 0) { fi = 2 * I; } else { fi = 2 * I + 1 + di; wgt *= wt[di + 1]; }
                    if (a == 1) { fj = 2 * J; } else { fj = 2 * J + 1 + dj; wgt *= wt[dj + 1]; }
                    if (dim == 3) {
                      if (a == 2) { fk = 2 * K; } else { fk = 2 * K + 1 + dk; wgt *= wt[dk + 1]; }
                    } else {
                      fk = 0;
                    }
                    // two fine faces in series along axis a
                    size_t i1, i2;
                    if (a == 0) {
                      i1 = ((size_t)fk * nf + fj) * (nf + 1) + fi;
                      i2 = i1 + 1;
                    } else if (a == 1) {
                      i1 = ((size_t)fk * (nf + 1) + fj) * nf + fi;
                      i2 = i1 + nf;
                    } else {
                      i1 = ((size_t)fk * nf + fj) * nf + fi;
                      i2 = i1 + (size_t)nf * nf;
                    }
                    acc += wgt * hmean(F.wf[a][i1], F.wf[a][i2]);
                  }
              size_t ci;
              if (a == 0) ci = ((size_t)K * nc + J) * (nc + 1) + I;
              else if (a == 1) ci = ((size_t)K * (nc + 1) + J) * nc + I;
              else ci = ((size_t)K * nc + J) * nc + I;
              C.wf[a][ci] = 0.25 * acc;
            }
      }
    }
    P->lev.push_back(std::move(C));
  }
  return BURA_OK;
}

// choose the first LDS level: the largest level l >= 1 whose sub-hierarchy fits in LDS
void choose_lds(bura_plan_t P, size_t elem) {
  const int L = (int)P->lev.size();
  if (L < 2) {
    P->lc = -1;
    P->lds_bytes = 0;
    return;
  }
  for (int l = 1; l < L; ++l) {
    size_t tot = 0;
    for (int q = l; q < L; ++q) tot += 3 * (size_t)P->lev[q].N * elem;
    if (tot <= kLdsCap && (L - l) <= kMaxLdsLevels) {
      P->lc = l;
      P->lds_bytes = tot;
      return;
    }
  }
  // the coarsest level alone does not fit (coarsening stopped early at a
  // large even n, e.g. 201 -> 100): no exact coarse solve is possible, so the
  // plan falls back to Jacobi-preconditioned CG on the fine level
  P->lc = -1;
  P->lds_bytes = 0;
}

template <typename T>
LdsHierarchy<T> lds_view(const bura_plan_t P) {
  LdsHierarchy<T> H{};
  const int L = (int)P->lev.size();
  H.nlev = L - P->lc;
  int off = 0;
  for (int q = 0; q < H.nlev; ++q) {
    H.lev[q] = level_view<T>(P, P->lc + q);
    H.off[q] = off;
    off += 3 * (int)P->lev[P->lc + q].N;
  }
  H.cycles = 1;   // one V-cycle through the in-LDS levels: the hierarchy is then a plain V-cycle
  H.nu = 2;
  H.bottom_sweeps = 8 * P->lev[L - 1].n + 8;
  H.omega = (T)(P->opts.omega > 0 ? P->opts.omega : default_omega(P->dim));
  H.pre = sweep_weights<T>(P, H.nu);
  return H;
}

bool fused_ok(const bura_plan_t P);

// q = (A + s) p needs a buffer unless the kernel that takes the PCG residual
// update forms it from p: the fused 2D down kernel, the 3D first fine sweep
// (the PCG updates folded into the level kernels)
bool q_stored(const bura_plan_t P) { return !(P->foldxr && (fused_ok(P) || P->dim == 3)); }

template <typename T>
int alloc_work(bura_plan_t P, Work<T>& W) {
  const size_t S = (size_t)P->S;
  const size_t vb = S * (size_t)P->N * sizeof(T);
  int rc;
  if ((rc = dev_alloc(P, (void**)&W.x, vb))) return rc;
  if ((rc = dev_alloc(P, (void**)&W.r, vb))) return rc;
  if ((rc = dev_alloc(P, (void**)&W.z, vb))) return rc;
  if ((rc = dev_alloc(P, (void**)&W.zt, vb))) return rc;
  if ((rc = dev_alloc(P, (void**)&W.p, vb))) return rc;
  if ((rc = dev_alloc(P, (void**)&W.p2, vb))) return rc;
  if (q_stored(P) && (rc = dev_alloc(P, (void**)&W.q, vb))) return rc;
  if (P->foldxr) {
    if ((rc = dev_alloc(P, (void**)&W.r2, vb))) return rc;
    if ((rc = dev_zero(P, W.r2, vb))) return rc;
  }
  const int L = (int)P->lev.size();
  W.xl.assign(L, nullptr);
  W.tl.assign(L, nullptr);
  W.bl.assign(L, nullptr);
  if (P->lc > 0) {
    for (int l = 1; l <= P->lc; ++l) {
      const size_t b = S * (size_t)P->lev[l].N * sizeof(T);
      if ((rc = dev_alloc(P, (void**)&W.xl[l], b))) return rc;
      if ((rc = dev_alloc(P, (void**)&W.bl[l], b))) return rc;
      if (l < P->lc && (rc = dev_alloc(P, (void**)&W.tl[l], b))) return rc;
    }
  }
  if ((rc = dev_alloc(P, (void**)&W.shift, S * sizeof(T)))) return rc;
  std::vector<T> sh(S);
  const int R = P->opts.nrhs_max;
  for (size_t i = 0; i < S; ++i) sh[i] = (T)P->s[i / R];
  HIPCHK(hipMemcpyAsync(W.shift, sh.data(), S * sizeof(T), hipMemcpyHostToDevice, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  for (void* ptr : {(void*)W.x, (void*)W.r, (void*)W.z, (void*)W.zt, (void*)W.p, (void*)W.p2, (void*)W.q})
    if (ptr && (rc = dev_zero(P, ptr, vb))) return rc;
  return BURA_OK;
}

size_t footprint(const bura_plan_t P, size_t elem, bool mixed) {
  const size_t S = (size_t)P->S;
  size_t t = (6 + (P->foldxr ? 1 : 0) + (q_stored(P) ? 1 : 0)) * S * (size_t)P->N * elem;
  if (P->lc > 0)
    for (int l = 1; l <= P->lc; ++l) t += 3 * S * (size_t)P->lev[l].N * elem;
  if (mixed) t += S * (size_t)P->N * 8;
  if (!P->stages.empty()) t += (size_t)P->opts.nrhs_max * P->N * 8;
  t += S * (size_t)max_partial_blocks(P->dim, P->n, P->N) * 8;
  for (const auto& L : P->lev)
    for (int a = 0; a < P->dim; ++a) t += L.wf[a].size() * 12;
  return t;
}

int upload_faces(bura_plan_t P) {
  if (!P->var) return BURA_OK;
  for (auto& L : P->lev) {
    for (int a = 0; a < P->dim; ++a) {
      const size_t cnt = L.wf[a].size();
      int rc;
      if ((rc = dev_alloc(P, (void**)&L.d_wf64[a], cnt * 8))) return rc;
      if ((rc = dev_alloc(P, (void**)&L.d_wf32[a], cnt * 4))) return rc;
      std::vector<float> f32(L.wf[a].begin(), L.wf[a].end());
      HIPCHK(hipMemcpyAsync(L.d_wf64[a], L.wf[a].data(), cnt * 8, hipMemcpyHostToDevice, P->stream));
      HIPCHK(hipMemcpyAsync(L.d_wf32[a], f32.data(), cnt * 4, hipMemcpyHostToDevice, P->stream));
      HIPCHK(hipStreamSynchronize(P->stream));
    }
  }
  return BURA_OK;
}

// ---------------------------------------------------------------------------
// preconditioner z = M r on a batch (V-cycle, or Jacobi without a hierarchy);
// the last sweep writes the per-block partials of r.z into `partial`.
// ---------------------------------------------------------------------------
// the fused level kernels exist for 2D hierarchies with 1..3 sweeps
bool fused_ok(const bura_plan_t P) {
  if (P->lc <= 0 || P->unfused || P->opts.nu_pre < 1 || P->opts.nu_post < 1) return false;
  if (P->dim == 2) return P->opts.nu_pre <= 3 && P->opts.nu_post <= 3;
  // 3D: constant coefficients, up to two sweeps (the z-marching kernels hold
  // every sweep's planes in LDS)
  return !P->var && P->opts.nu_pre <= 2 && P->opts.nu_post <= 2;
}

// The PCG residual update folded into the fine down kernel: r_new = r_old -
// alpha q is formed while staging, written to rnew (a different buffer) with
// its squared norm; `after` runs once that kernel is queued (the convergence
// test on |r_new|).  The fused 2D down kernel and the 3D first fine sweep
// take the search direction p and form q = (A + s) p themselves (the stencil
// product then stores no q); the 2D unfused first sweep reads q.
template <typename T>
struct ResidUpdate {
  const T* rold;
  T* rnew;
  const T* q;   // (A + s) p, for the 2D unfused first sweep (nullptr: form it from p)
  const T* p;   // p, for the fused down kernel and the 3D first sweep
  const double* alpha;
  Fin fin;
  std::function<void()> after;
};

template <typename T>
void precondition(bura_plan_t P, Work<T>& W, size_t sys0, int nsys, const int* active, double* partial,
                  Fin fin = Fin(), const ResidUpdate<T>* ru = nullptr) {
  hipStream_t st = P->stream;
  const int dim = P->dim;
  const bool var = P->var;
  const T* shift = W.shift + sys0;
  auto off = [&](T* base, int l) { return base + sys0 * (size_t)P->lev[l].N; };
  if (P->lc < 0) {
    // Jacobi preconditioner: z = D^-1 r
    ProfScope ps(P, BURA_K_SMOOTH_FINE);
    Launch<T>::jacobi(dim, var, level_view<T>(P, 0), off(W.r, 0), nullptr, off(W.z, 0), shift, active, T(1), true,
                      partial, nsys, st, ps.ctr, fin);
    return;
  }
  const int lc = P->lc;
  const int nu1 = std::max(1, P->opts.nu_pre), nu2 = std::max(1, P->opts.nu_post);
  const Sweeps<T> wpre = sweep_weights<T>(P, nu1), wpost = sweep_weights<T>(P, nu2);
  auto w_at = [](const Sweeps<T>& sw, int i) { return sw.w[std::min(i, 2)]; };
  if (fused_ok(P)) {
    // two LDS-tiled kernels per level: down (nu1 sweeps + residual + restriction)
    // writes the pre-smoothed iterate into A_l; up (prolongation + nu2 sweeps)
    // writes the final iterate into B_l (B_0 = z).
    auto A = [&](int l) { return l == 0 ? off(W.zt, 0) : off(W.tl[l], l); };
    auto Bv = [&](int l) { return l == 0 ? off(W.z, 0) : off(W.xl[l], l); };
    auto bl = [&](int l) { return l == 0 ? (ru ? ru->rnew : off(W.r, 0)) : off(W.bl[l], l); };
    for (int l = 0; l < lc; ++l) {
      {
        ProfScope ps(P, l > 0 ? BURA_K_SMOOTH_COARSE : ru ? BURA_K_DOWN_FINE : BURA_K_DOWN_FINE_PLAIN);
        if (l == 0 && ru)
          Launch<T>::fused_down(dim, var, nu1, level_view<T>(P, 0), level_view<T>(P, 1), ru->rold, A(0), bl(1),
                                shift, active, wpre, nsys, st, ps.ctr, ru->p, ru->alpha, ru->rnew, partial,
                                ru->fin, P->tile_down[0], P->tile_up[0]);
        else
          Launch<T>::fused_down(dim, var, nu1, level_view<T>(P, l), level_view<T>(P, l + 1), bl(l), A(l),
                                bl(l + 1), shift, active, wpre, nsys, st, ps.ctr, nullptr, nullptr, nullptr,
                                nullptr, Fin(), P->tile_down[l], P->tile_up[l]);
      }
      if (l == 0 && ru && ru->after) ru->after();
    }
    {
      ProfScope ps(P, BURA_K_COARSE_LDS);
      Launch<T>::coarse_solve(dim, var, lds_view<T>(P), bl(lc), off(W.xl[lc], lc), shift, active, nsys,
                              P->lds_bytes, st, ps.ctr);
    }
    for (int l = lc - 1; l >= 0; --l) {
      ProfScope ps(P, l == 0 ? BURA_K_UP_FINE : BURA_K_SMOOTH_COARSE);
      const T* xc = l + 1 == lc ? off(W.xl[lc], lc) : Bv(l + 1);
      Launch<T>::fused_up(dim, var, nu2, level_view<T>(P, l + 1), level_view<T>(P, l), xc, A(l), bl(l), Bv(l),
                          shift, active, wpost, l == 0 ? partial : nullptr, nsys, st, ps.ctr,
                          l == 0 ? fin : Fin(), P->tile_up[l]);
    }
    return;
  }
  // per level: right-hand side, the buffer holding the iterate, the spare buffer.
  // nu1 + nu2 sweeps alternate between two buffers; the first sweep writes the
  // buffer that makes the last one land in xa (xa = z on the fine level).
  std::vector<T*> bcur(lc + 1), cur(lc + 1), spare(lc + 1);
  bcur[0] = ru ? ru->rnew : off(W.r, 0);
  for (int l = 1; l <= lc; ++l) bcur[l] = off(W.bl[l], l);
  for (int l = 0; l < lc; ++l) {
    const LevelDev<T> L = level_view<T>(P, l);
    T* xa = l == 0 ? off(W.z, 0) : off(W.xl[l], l);
    T* xb = l == 0 ? off(W.zt, 0) : off(W.tl[l], l);
    const bool odd = ((nu1 + nu2) % 2) == 1;
    T* out = odd ? xa : xb;
    T* other = odd ? xb : xa;
    const int scls = l == 0 ? BURA_K_SMOOTH_FINE : BURA_K_SMOOTH_COARSE;
    if (l == 0 && ru) {
      {
        ProfScope ps(P, BURA_K_SMOOTH_FINE_RUP);
        Launch<T>::jacobi_rup(dim, var, L, ru->rold, ru->q, ru->alpha, ru->rnew, out, shift, active, w_at(wpre, 0),
                              partial, nsys, st, ps.ctr, ru->fin, ru->p);
      }
      if (ru->after) ru->after();
    } else {
      ProfScope ps(P, scls);
      Launch<T>::jacobi(dim, var, L, bcur[l], nullptr, out, shift, active, w_at(wpre, 0), true, nullptr, nsys, st,
                        ps.ctr);
    }
    for (int s = 1; s < nu1; ++s) {
      ProfScope ps(P, scls);
      Launch<T>::jacobi(dim, var, L, bcur[l], out, other, shift, active, w_at(wpre, s), false, nullptr, nsys, st,
                        ps.ctr);
      std::swap(out, other);
    }
    cur[l] = out;
    spare[l] = other;
    ProfScope ps(P, BURA_K_RESTRICT);
    Launch<T>::restrict_residual(dim, var, L, level_view<T>(P, l + 1), bcur[l], cur[l], bcur[l + 1], shift, active,
                                 nsys, st, ps.ctr);
  }
  cur[lc] = off(W.xl[lc], lc);
  {
    ProfScope ps(P, BURA_K_COARSE_LDS);
    Launch<T>::coarse_solve(dim, var, lds_view<T>(P), bcur[lc], cur[lc], shift, active, nsys, P->lds_bytes, st,
                            ps.ctr);
  }
  for (int l = lc - 1; l >= 0; --l) {
    const LevelDev<T> L = level_view<T>(P, l);
    {
      ProfScope ps(P, BURA_K_PROLONG);
      Launch<T>::prolong_add(dim, level_view<T>(P, l + 1), L, cur[l + 1], cur[l], active, nsys, st, ps.ctr);
    }
    const int scls = l == 0 ? BURA_K_SMOOTH_FINE : BURA_K_SMOOTH_COARSE;
    for (int s = 0; s < nu2; ++s) {
      const bool last = (l == 0 && s == nu2 - 1);
      ProfScope ps(P, scls);
      Launch<T>::jacobi(dim, var, L, bcur[l], cur[l], spare[l], shift, active, w_at(wpost, nu2 - 1 - s), false,
                        last ? partial : nullptr, nsys, st, ps.ctr, last ? fin : Fin());
      std::swap(cur[l], spare[l]);
    }
  }
}

// which kernel wrote the r.z partials (for the reduction's block count)
int rz_blocks(const bura_plan_t P) {
  return fused_ok(P) ? up_blocks(P->dim, P->n, P->tile_up[0]) : stencil_blocks(P->dim, P->n);
}

SysState state_at(const bura_plan_t P, size_t sys0) {
  SysState s = P->st;
  s.bnorm2 += sys0; s.rho += sys0; s.alpha += sys0; s.beta += sys0; s.relres += sys0;
  s.active += sys0; s.iters += sys0; s.total_iters += sys0; s.flags += sys0;
  s.fnorm2 += sys0; s.relres64 += sys0; s.active64 += sys0; s.outer += sys0;
  if (s.tol_pcg) s.tol_pcg += sys0;
  if (s.tol_outer) s.tol_outer += sys0;
  if (s.tol_inner) s.tol_inner += sys0;
  return s;
}

int count_active(bura_plan_t P, const int* dev_flags, size_t sys0, int nsys) {
  if (hipMemcpyAsync(P->h_flags, dev_flags + sys0, nsys * sizeof(int), hipMemcpyDeviceToHost, P->stream) !=
      hipSuccess)
    return -1;
  if (hipStreamSynchronize(P->stream) != hipSuccess) return -1;
  prof_flush(P);
  int c = 0;
  for (int i = 0; i < nsys; ++i) c += P->h_flags[i] != 0;
  return c;
}

// PCG on systems [sys0, sys0+nsys): r holds b, x holds 0, OP_INIT done.
// defer_finish: leave each system's last deferred x update pending (the
// caller's next kernel applies it: k_x_from_e in the refinement loop).
template <typename T>
int run_pcg(bura_plan_t P, Work<T>& W, size_t sys0, int nsys, double tol, int max_iter, bool defer_finish = false) {
  hipStream_t st = P->stream;
  const int dim = P->dim;
  const LevelDev<T> L0 = level_view<T>(P, 0);
  const size_t o = sys0 * (size_t)P->N;
  const SysState S = state_at(P, sys0);
  double* part = P->partial;
  const int nb_flat = flat_blocks(P->N);
  const int check = std::max(1, P->opts.check_every);
  auto scal = [&](int op, int nblk) {
    ProfScope ps(P, BURA_K_OTHER);
    launch_scalars(op, part, nblk, nsys, S, tol, max_iter, st);
  };
  T* pold = W.p + o;
  T* pnew = W.p2 + o;
  // one PCG iteration for the systems of this batch (converged systems are
  // skipped by their blocks); p_new = z + beta p_old goes to the other buffer
  auto fin = [&](int op) {
    Fin f;
    if (!P->fold) return f;
    f.op = op;
    f.cnt = P->d_cnt + sys0;
    f.st = S;
    f.tol = tol;
    f.max_iter = max_iter;
    return f;
  };
  const bool fx = P->foldxr;
  // blocks of the kernel that writes the |r_new|^2 partials
  const int nb_down = !fx ? 0 : fused_ok(P) ? down_blocks(dim, P->n, P->tile_down[0]) : stencil_blocks(dim, P->n);
  // the fused down kernel forms q from p: the stencil product stores no q
  const bool qfree = !q_stored(P);
  auto body = [&](T* po, T* pn, T* ro, T* rn) {
    {
      ProfScope ps(P, BURA_K_SPMV);
      Launch<T>::spmv_p(dim, P->var, L0, W.z + o, po, pn, qfree ? nullptr : W.q + o, S.beta, W.shift + sys0, S.active,
                        part, nsys, st, ps.ctr, fin(OP_ALPHA), fx ? W.x + o : nullptr, S.alpha, P->tile_spmv);
    }
    if (!P->fold) scal(OP_ALPHA, spmv_blocks(dim, P->n, P->tile_spmv));
    if (fx) {
      ResidUpdate<T> ru{ro, rn, qfree ? nullptr : W.q + o, pn, S.alpha, fin(OP_RESID), [&]() {
                          if (!P->fold) scal(OP_RESID, nb_down);
                        }};
      precondition<T>(P, W, sys0, nsys, S.active, part, fin(OP_BETA), &ru);
    } else {
      {
        ProfScope ps(P, BURA_K_UPDATE_XR);
        Launch<T>::update_xr(L0, dim, W.x + o, W.r + o, pn, W.q + o, S.alpha, S.active, part, nsys, st, ps.ctr,
                             fin(OP_RESID));
      }
      if (!P->fold) scal(OP_RESID, nb_flat);
      precondition<T>(P, W, sys0, nsys, S.active, part, fin(OP_BETA));
    }
    if (!P->fold) scal(OP_BETA, rz_blocks(P));
  };
  T* rold = W.r + o;
  T* rnew = fx ? W.r2 + o : W.r + o;
  precondition<T>(P, W, sys0, nsys, S.active, part, fin(OP_BETA));
  if (!P->fold) scal(OP_BETA, rz_blocks(P));
  // chunks of an even number of iterations, so p_old is W.p at every chunk start
  const int chunk = std::max(2, check + (check & 1));
  const int nchunks = max_iter / chunk + 1;
  bura_plan_s::Graph* g = nullptr;
  if (P->use_graphs) {
    char key[160];
    std::snprintf(key, sizeof(key), "%zu/%zu/%d/%.17g/%d/%d", sizeof(T), sys0, nsys, tol, max_iter, chunk);
    auto it = P->graphs.find(key);
    if (it != P->graphs.end()) {
      g = &it->second;
    } else {
      // capture the chunk once; replays cost one launch
      HIPCHK(hipStreamSynchronize(st));
      prof_flush(P);
      P->capturing = true;
      P->capture_failed = false;
      P->cap_ev.clear();
      hipGraph_t graph = nullptr;
      bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        T* a = pold;
        T* b = pnew;
        T* ra = rold;
        T* rb = rnew;
        for (int c = 0; c < chunk; ++c) {
          body(a, b, ra, rb);
          std::swap(a, b);
          std::swap(ra, rb);
        }
        ok = hipStreamEndCapture(st, &graph) == hipSuccess && graph != nullptr && !P->capture_failed;
      }
      P->capturing = false;
      bura_plan_s::Graph G;
      G.ev = P->cap_ev;
      P->cap_ev.clear();
      if (ok && hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0) != hipSuccess) ok = false;
      if (graph) hipGraphDestroy(graph);
      (void)hipGetLastError();
      if (!ok) {
        for (auto& e : G.ev) { hipEventDestroy(std::get<1>(e)); hipEventDestroy(std::get<2>(e)); }
        if (G.exec) hipGraphExecDestroy(G.exec);
        P->use_graphs = false;   // fall back to direct launches for this plan
      } else {
        g = &(P->graphs[key] = std::move(G));
      }
    }
  }
  for (int ch = 0; ch < nchunks; ++ch) {
    if (g) {
      HIPCHK(hipGraphLaunch(g->exec, st));
    } else {
      T* a = pold;
      T* b = pnew;
      T* ra = rold;
      T* rb = rnew;
      for (int c = 0; c < chunk; ++c) {
        body(a, b, ra, rb);
        std::swap(a, b);
        std::swap(ra, rb);
      }
    }
    const int a = count_active(P, P->st.active, sys0, nsys);
    if (a < 0) {
      g_last_error = hipGetErrorString(hipGetLastError());
      return BURA_EDEVICE;
    }
    if (g) prof_graph(P, *g);
    if (a == 0) break;
  }
  if (fx && !defer_finish) {
    // the iterate update of each system's last iteration is still pending
    ProfScope ps(P, BURA_K_UPDATE_XR);
    Launch<T>::finish_x(P->N, W.x + o, W.p + o, W.p2 + o, S.alpha, S.iters, nsys, st, ps.ctr);
  }
  HIPCHK(hipGetLastError());
  return BURA_OK;
}

int set_flags(bura_plan_t P, int* dev, size_t sys0, int nsys, int value) {
  launch_fill_int(dev + sys0, nsys, value, P->stream);
  return BURA_OK;
}

// FP64 plans without stages leave each system's last deferred iterate update
// to the combine, which reads x anyway (k_finish_x would read and write it
// once more); a later stage of a sequential form reads x itself, so staged
// plans finish it.
bool combine_finishes_x(const bura_plan_t P) {
  return P->foldxr && P->opts.precision == BURA_FP64 && P->stages.empty();
}

int solve_batch_fp64(bura_plan_t P, const double* f, int nrhs, size_t sys0, int nsys, bool preset) {
  hipStream_t st = P->stream;
  Work<double>& W = P->w64;
  const LevelDev<double> L0 = level_view<double>(P, 0);
  const size_t o = sys0 * (size_t)P->N;
  const SysState S = state_at(P, sys0);
  int rc;
  if (!preset && (rc = set_flags(P, P->st.active, sys0, nsys, 1))) return rc;
  // no deferred iterate update pending on any system of the batch (slots that
  // stay inactive keep alpha = 0, so the final update skips them)
  launch_zero(S.alpha, (size_t)nsys * sizeof(double), st);
  {
    ProfScope ps(P, BURA_K_OTHER);
    Launch<double>::copy_rhs(L0, P->dim, f, W.r + o, W.x + o, nrhs, S.active, P->partial, nsys, st);
  }
  {
    ProfScope ps(P, BURA_K_OTHER);
    launch_scalars(OP_INIT, P->partial, flat_blocks(P->N), nsys, S, P->run_tol, P->opts.max_iter, st);
  }
  return run_pcg<double>(P, W, sys0, nsys, P->run_tol, P->opts.max_iter, combine_finishes_x(P));
}

// The refinement loop of a mixed batch (the FP64 residual of every active
// system already formed and tested): FP32 inner solves on the active systems,
// x64 += e, the FP64 residual and the outer test, until no system is active.
// x_zero: x64 was not cleared (k_first_residual with zero_x false) and the
// first update assigns it (the fused update and residual pass only)
int mixed_outer_loop(bura_plan_t P, const double* f, int nrhs, size_t sys0, int nsys, bool x_zero = false) {
  hipStream_t st = P->stream;
  Work<float>& W = P->w32;
  const LevelDev<double> L0 = level_view<double>(P, 0);
  const size_t o = sys0 * (size_t)P->N;
  const SysState S = state_at(P, sys0);
  int rc;
  for (int outer = 0; outer < P->opts.max_outer + 1; ++outer) {
    const int a = count_active(P, P->st.active64, sys0, nsys);
    if (a < 0) {
      g_last_error = "device error during refinement";
      return BURA_EDEVICE;
    }
    if (a == 0) break;
    // with the folded updates, x64 += e also applies the inner solve's last
    // deferred update (k_finish_x is not launched)
    const bool fx = P->foldxr;
    if ((rc = run_pcg<float>(P, W, sys0, nsys, P->opts.inner_tol, P->opts.max_iter, fx))) return rc;
    if (residual_marches_rows(P->dim, P->n, nsys)) {
      // x64 += e and the FP64 residual in one pass where the residual marches rows
      ProfScope ps(P, BURA_K_RESIDUAL64);
      launch_update_residual64(P->dim, P->var, L0, f, P->x64 + o, W.x + o, W.r + o, P->d_shift64 + sys0, S.active64,
                               P->partial, nrhs, nsys, st, ps.ctr, fx ? W.p + o : nullptr, fx ? W.p2 + o : nullptr,
                               S.alpha, S.iters, x_zero && outer == 0);
    } else {
      {
        ProfScope ps(P, BURA_K_OTHER);
        launch_x_from_e(L0, P->dim, W.x + o, P->x64 + o, S.active64, nsys, st, fx ? W.p + o : nullptr,
                        fx ? W.p2 + o : nullptr, S.alpha, S.iters);
      }
      {
        ProfScope ps(P, BURA_K_RESIDUAL64);
        launch_residual64(P->dim, P->var, L0, f, P->x64 + o, W.x + o, W.r + o, P->d_shift64 + sys0, S.active64,
                          P->partial, nrhs, nsys, false, st, ps.ctr);
      }
    }
    {
      ProfScope ps(P, BURA_K_OTHER);
      launch_scalars(OP_OUTER, P->partial, residual_blocks(P->dim, P->n, nsys), nsys, S, P->run_tol, P->opts.max_outer,
                     st);
    }
  }
  HIPCHK(hipGetLastError());
  return BURA_OK;
}

int solve_batch_mixed(bura_plan_t P, const double* f, int nrhs, size_t sys0, int nsys, bool preset) {
  hipStream_t st = P->stream;
  Work<float>& W = P->w32;
  const LevelDev<double> L0 = level_view<double>(P, 0);
  const size_t o = sys0 * (size_t)P->N;
  const SysState S = state_at(P, sys0);
  int rc;
  if (!preset) {
    if ((rc = set_flags(P, P->st.active64, sys0, nsys, 1))) return rc;
    if ((rc = set_flags(P, P->st.active, sys0, nsys, 1))) return rc;
  } else {
    // inner flags follow the outer ones (OP_OUTER re-arms them per system)
    HIPCHK(hipMemcpyAsync(P->st.active + sys0, P->st.active64 + sys0, nsys * sizeof(int), hipMemcpyDeviceToDevice,
                          P->stream));
  }
  launch_zero(S.alpha, (size_t)nsys * sizeof(double), st);   // see solve_batch_fp64
  // with the fused update and residual pass the first update assigns x64,
  // so the first residual need not clear it
  const bool x_zero = residual_marches_rows(P->dim, P->n, nsys);
  {
    ProfScope ps(P, BURA_K_RESIDUAL64);
    launch_residual64(P->dim, P->var, L0, f, P->x64 + o, W.x + o, W.r + o, P->d_shift64 + sys0, S.active64,
                      P->partial, nrhs, nsys, true, st, ps.ctr, !x_zero);
  }
  {
    ProfScope ps(P, BURA_K_OTHER);
    launch_scalars(OP_OUTER, P->partial, flat_blocks(P->N), nsys, S, P->run_tol, P->opts.max_outer, st);
  }
  return mixed_outer_loop(P, f, nrhs, sys0, nsys, x_zero);
}

// Continue the refinement of the systems of [sys0, sys0 + nsys) flagged in
// the host array act (1 = continue) from their current x64: their FP64
// residual is formed again and tested against the current tolerances (the
// per-system ones if st.tol_outer is set).
int resume_batch_mixed(bura_plan_t P, const double* f, int nrhs, size_t sys0, int nsys, const int* act) {
  hipStream_t st = P->stream;
  Work<float>& W = P->w32;
  const LevelDev<double> L0 = level_view<double>(P, 0);
  const size_t o = sys0 * (size_t)P->N;
  const SysState S = state_at(P, sys0);
  HIPCHK(hipMemcpyAsync(P->st.active64 + sys0, act, nsys * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(P->st.active + sys0, act, nsys * sizeof(int), hipMemcpyHostToDevice, st));
  launch_zero(S.alpha, (size_t)nsys * sizeof(double), st);
  {
    ProfScope ps(P, BURA_K_RESIDUAL64);
    launch_residual64(P->dim, P->var, L0, f, P->x64 + o, W.x + o, W.r + o, P->d_shift64 + sys0, S.active64,
                      P->partial, nrhs, nsys, false, st, ps.ctr);
  }
  {
    ProfScope ps(P, BURA_K_OTHER);
    launch_scalars(OP_OUTER, P->partial, residual_blocks(P->dim, P->n, nsys), nsys, S, P->run_tol, P->opts.max_outer,
                   st);
  }
  return mixed_outer_loop(P, f, nrhs, sys0, nsys);
}

// Per-solve terms of a slot plan: rhs r has nterms[r] terms with weights
// w[r * max_terms + j], shifts s[r * max_terms + j] and tolerance tol[r].
struct SlotTerms {
  const int* nterms;
  const double* w;
  const double* s;
  const double* tol;   // nullptr: opts.tol for every rhs
};

int check_slot_terms(const bura_plan_t P, int nrhs, const SlotTerms& t) {
  if (!t.nterms || !t.w || !t.s) return BURA_EINVAL;
  const int K = P->nterms;
  for (int r = 0; r < nrhs; ++r) {
    if (t.nterms[r] < 1 || t.nterms[r] > K) return BURA_EINVAL;
    if (t.tol && !(t.tol[r] > 0.0)) return BURA_EINVAL;
    for (int j = 0; j < t.nterms[r]; ++j) {
      const double w = t.w[(size_t)r * K + j], sh = t.s[(size_t)r * K + j];
      if (!std::isfinite(w) || !(sh >= 0.0) || !std::isfinite(sh)) return BURA_EINVAL;
    }
  }
  return BURA_OK;
}

// Upload one solve's per-system weights, shifts, tolerances and active flags
// (system j * R + r is used iff r < nrhs and j < nterms[r]).
int upload_slots(bura_plan_t P, int nrhs, const SlotTerms& t) {
  const int K = P->nterms, R = P->opts.nrhs_max;
  const size_t S = (size_t)P->S;
  const bool mixed = P->opts.precision == BURA_MIXED;
  double* hw = (double*)P->h_slot;
  double* hs = hw + S;
  double* ht = hs + S;
  float* hs32 = (float*)(ht + S);
  int* hf = (int*)(hs32 + S);
  for (int j = 0; j < K; ++j) {
    for (int r = 0; r < R; ++r) {
      const size_t i = (size_t)j * R + r;
      const bool used = r < nrhs && j < t.nterms[r];
      hw[i] = used ? t.w[(size_t)r * K + j] : 0.0;
      hs[i] = used ? t.s[(size_t)r * K + j] : 0.0;
      ht[i] = used && t.tol ? t.tol[r] : P->run_tol;
      hs32[i] = (float)hs[i];
      hf[i] = used ? 1 : 0;
    }
  }
  hipStream_t st = P->stream;
  HIPCHK(hipMemcpyAsync(P->d_wsys, hw, S * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(P->d_shift64, hs, S * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(P->d_tol, ht, S * 8, hipMemcpyHostToDevice, st));
  if (mixed) {
    HIPCHK(hipMemcpyAsync(P->w32.shift, hs32, S * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(P->st.active64, hf, S * 4, hipMemcpyHostToDevice, st));
  } else {
    HIPCHK(hipMemcpyAsync(P->w64.shift, hs, S * 8, hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipMemcpyAsync(P->st.active, hf, S * 4, hipMemcpyHostToDevice, st));
  return BURA_OK;
}

int do_solve(bura_plan_t P, const double* f, double* u, int nrhs, bura_report_t* rep,
             const SlotTerms* slot = nullptr, double tol = 0.0) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!P || !f || !u || nrhs < 1 || nrhs > P->opts.nrhs_max) return BURA_EINVAL;
  if (!(tol >= 0.0) || !std::isfinite(tol)) return BURA_EINVAL;
  P->run_tol = tol > 0.0 ? tol : P->opts.tol;
  if (P->slots != (slot != nullptr)) return BURA_EINVAL;
  if (slot && check_slot_terms(P, nrhs, *slot)) return BURA_EINVAL;
  HIPCHK(hipSetDevice(P->device));
  const bool mixed = P->opts.precision == BURA_MIXED;
  const int R = P->opts.nrhs_max;
  // systems are laid out sys = j * R + r; only r < nrhs are used
  const size_t S_used = (size_t)P->nterms * R;
  int rc;
  // the plan works on its own stream, ordered after the caller's pending work
  // (a static-workspace plan runs on the caller's stream itself)
  if (P->join_ev) {
    HIPCHK(hipEventRecord(P->join_ev, P->user_stream));
    HIPCHK(hipStreamWaitEvent(P->stream, P->join_ev, 0));
  }
  if ((rc = set_flags(P, P->st.flags, 0, (int)S_used, 0))) return rc;
  if ((rc = set_flags(P, P->st.total_iters, 0, (int)S_used, 0))) return rc;
  if ((rc = set_flags(P, P->st.outer, 0, (int)S_used, 0))) return rc;
  auto batch_rhs = [&](const double* rhs, size_t sys0, int nsys, bool preset) {
    // the kernels take rhs = sys % R; pass rhs with R slots (rhs >= nrhs never active)
    return mixed ? solve_batch_mixed(P, rhs, R, sys0, nsys, preset)
                 : solve_batch_fp64(P, rhs, R, sys0, nsys, preset);
  };
  auto batch = [&](size_t sys0, int nsys, bool preset) { return batch_rhs(f, sys0, nsys, preset); };
  const double* xsol = mixed ? P->x64 : P->w64.x;
  if (slot) {
    // every rhs with its own terms, all in one batch; unused slots inactive
    if ((rc = upload_slots(P, nrhs, *slot))) return rc;
    rc = batch(0, (int)S_used, true);
  } else if (!P->stages.empty()) {
    // sequential form: each stage solves its terms against its input, then
    // combines into the stage buffer (or u for the last stage)
    rc = BURA_OK;
    for (size_t si = 0; si < P->stages.size() && rc == BURA_OK; ++si) {
      const Stage& g = P->stages[si];
      const bool last = si + 1 == P->stages.size();
      const double* in = g.input == Stage::F ? f
                         : g.input == Stage::PREV ? P->d_buf
                                                  : xsol + (size_t)g.sol_term * R * P->N;
      const size_t sys0 = (size_t)g.tb * R;
      const int nt = g.te - g.tb;
      if (nrhs == R) {
        rc = batch_rhs(in, sys0, nt * R, false);
      } else {
        launch_slot_flags(P->st.active + sys0, nt, R, nrhs, P->stream);
        if (mixed) launch_slot_flags(P->st.active64 + sys0, nt, R, nrhs, P->stream);
        rc = batch_rhs(in, sys0, nt * R, true);
      }
      if (rc) break;
      ProfScope ps(P, BURA_K_COMBINE);
      launch_combine(P->N, xsol + sys0 * P->N, P->d_w + g.tb, nt, nrhs, R, last ? u : P->d_buf, P->stream, ps.ctr,
                     g.base ? P->d_buf : nullptr, g.base_w);
    }
  } else if (P->opts.schedule == BURA_PER_POLE) {
    if (nrhs < R) {
      if ((rc = set_flags(P, P->st.active, 0, (int)S_used, 0))) return rc;
      if ((rc = set_flags(P, P->st.active64, 0, (int)S_used, 0))) return rc;
    }
    for (int j = 0; j < P->nterms && rc == BURA_OK; ++j) rc = batch((size_t)j * R, nrhs, false);
  } else if (nrhs == R) {
    rc = batch(0, (int)S_used, false);
  } else {
    // fewer rhs than slots: one batch over all systems, unused slots inactive
    launch_slot_flags(P->st.active, P->nterms, R, nrhs, P->stream);
    if (mixed) launch_slot_flags(P->st.active64, P->nterms, R, nrhs, P->stream);
    rc = batch(0, (int)S_used, true);
  }
  if (rc) return rc;
  const size_t S = (size_t)P->S;
  const size_t sb = S * (6 * 8 + 8 * 4);
  // outputs with an error bound (rows of u): every output of a plan without
  // stages, one per rhs of a slot plan
  const int rows = slot ? nrhs : (P->stages.empty() ? P->nout * nrhs : 0);
  // combine u_i = sum_{j in output i} w_j x_j (fixed order, FP64), then the
  // squared norm of every output row
  auto combine = [&]() -> int {
    const bool pend = combine_finishes_x(P);
    if (slot) {
      ProfScope ps(P, BURA_K_COMBINE);
      launch_combine(P->N, xsol, P->d_wsys, P->nterms, nrhs, R, u, P->stream, ps.ctr, nullptr, 0.0, true,
                     pend ? P->w64.p : nullptr, pend ? P->w64.p2 : nullptr, P->st.alpha, P->st.iters);
    }
    for (int i = 0; i < P->nout && P->stages.empty() && !slot; ++i) {
      ProfScope ps(P, BURA_K_COMBINE);
      const int b = P->out_begin[i], e = P->out_end[i];
      const size_t ob = (size_t)b * R;   // first system of output i
      launch_combine(P->N, xsol + ob * P->N, P->d_w + b, e - b, nrhs, R, u + (size_t)i * nrhs * P->N, P->stream,
                     ps.ctr, nullptr, 0.0, false, pend ? P->w64.p + ob * P->N : nullptr,
                     pend ? P->w64.p2 + ob * P->N : nullptr, P->st.alpha + ob, P->st.iters + ob);
    }
    if (rows > 0) launch_row_norms(u, P->N, rows, P->d_upart, P->d_unorm, P->stream);
    HIPCHK(hipGetLastError());
    return BURA_OK;
  };
  // report: one copy of the per-system scalar state (and the output norms)
  auto fetch = [&]() -> int {
    HIPCHK(hipMemcpyAsync(P->h_state, P->state_block, sb, hipMemcpyDeviceToHost, P->stream));
    HIPCHK(hipMemcpyAsync((char*)P->h_state + sb, P->st.relres64, S * 8, hipMemcpyDeviceToHost, P->stream));
    if (rows > 0)
      HIPCHK(hipMemcpyAsync((char*)P->h_state + sb + S * 8, P->d_unorm, (size_t)rows * 8, hipMemcpyDeviceToHost,
                            P->stream));
    HIPCHK(hipStreamSynchronize(P->stream));
    prof_flush(P);
    return BURA_OK;
  };
  const double* hd = (const double*)P->h_state;
  const double* rr = mixed ? (const double*)((const char*)P->h_state + sb) : hd + 4 * S;
  const double* fn2 = mixed ? hd + 5 * S : hd;   // ||f_r||^2 of each system's rhs
  const double* un2 = (const double*)((const char*)P->h_state + sb + S * 8);
  // Certified a posteriori bound (Section 2.2, eq. (16); Lemma 2.5 for
  // c_j > 0): system j stopped with residual r_j, so its error is
  // (A - d_j)^-1 r_j, of norm at most |r_j| / (lambda_min + s_j) <=
  // |r_j| / (lam_lb + s_j), and the output's distance to the exact
  // sum_j c_j (A - d_j)^-1 f is at most sum_j |c_j| |r_j| / (lam_lb + s_j).
  // Relative to |u|, the largest over the rows (and per row in *per).
  auto term = [&](int row, int t, size_t* sys, double* w, double* sh) {
    if (slot) {
      const int K = P->nterms;
      *sys = (size_t)t * R + row;
      *w = slot->w[(size_t)row * K + t];
      *sh = slot->s[(size_t)row * K + t];
    } else {
      const int a = row / nrhs, r = row % nrhs;
      const int j = P->out_begin[a] + t;
      *sys = (size_t)j * R + r;
      *w = P->w_applied[j];
      *sh = P->s[j];
    }
  };
  auto nterms_of = [&](int row) {
    return slot ? slot->nterms[row] : P->out_end[row / nrhs] - P->out_begin[row / nrhs];
  };
  auto bound = [&](std::vector<double>* per) {
    double mx = 0.0;
    if (per) per->assign(rows, 0.0);
    for (int row = 0; row < rows; ++row) {
      double acc = 0.0;
      for (int t = 0; t < nterms_of(row); ++t) {
        size_t sy;
        double w, sh;
        term(row, t, &sy, &w, &sh);
        acc += std::fabs(w) * std::sqrt(fn2[sy]) * rr[sy] / (P->lam_lb + sh);
      }
      const double un = std::sqrt(un2[row]);
      const double v = acc == 0.0 ? 0.0 : (un > 0.0 ? acc / un : HUGE_VAL);
      if (per) (*per)[row] = v;
      mx = std::max(mx, v);
    }
    return mx;
  };
  if ((rc = combine()) || (rc = fetch())) return rc;
  double eb = rows > 0 ? bound(nullptr) : -1.0;
  const double etol = P->opts.err_tol;
  if (mixed && etol > 0.0 && rows > 0) {
    // opts.err_tol: refine the terms of every row over the bound further.
    // Their target residuals share the allowed error equally among the
    // terms: |r_j| <= err_tol |u| (lam_lb + s_j) / (terms |c_j|), halved
    // against the change of |u|.
    std::vector<double> per, tolv(S);
    for (int round = 0; round < 4 && eb > etol; ++round) {
      bound(&per);
      for (size_t i = 0; i < S; ++i) {
        const int r = (int)(i % R);
        tolv[i] = slot && slot->tol && r < nrhs ? slot->tol[r] : P->run_tol;
        P->h_flags[i] = 0;
      }
      for (int row = 0; row < rows; ++row) {
        if (!(per[row] > etol)) continue;
        const int nt = nterms_of(row);
        for (int t = 0; t < nt; ++t) {
          size_t sy;
          double w, sh;
          term(row, t, &sy, &w, &sh);
          const double fnr = std::sqrt(fn2[sy]);
          if (w == 0.0 || !(fnr > 0.0)) continue;
          const double target = 0.5 * etol * std::sqrt(un2[row]) * (P->lam_lb + sh) / (nt * std::fabs(w) * fnr);
          tolv[sy] = std::min(tolv[sy], target);
          if (rr[sy] > tolv[sy]) P->h_flags[sy] = 1;
        }
      }
      HIPCHK(hipMemcpyAsync(P->d_tol_err, tolv.data(), S * 8, hipMemcpyHostToDevice, P->stream));
      HIPCHK(hipStreamSynchronize(P->stream));
      P->st.tol_outer = P->d_tol_err;
      rc = resume_batch_mixed(P, f, R, 0, (int)S_used, P->h_flags);
      P->st.tol_outer = P->slots ? P->d_tol : nullptr;
      if (rc || (rc = combine()) || (rc = fetch())) return rc;
      eb = bound(nullptr);
    }
  }
  const int* hi = (const int*)(hd + 6 * S);
  const int* it = hi + 2 * S;
  const int* flags = hi + 3 * S;
  const int* outer = hi + 5 * S;
  int status = BURA_OK;
  bura_report_t R_{};
  R_.nterms = P->nterms;
  if (slot) R_.nterms = *std::max_element(slot->nterms, slot->nterms + nrhs);
  R_.E = P->E;
  for (int j = 0; j < P->nterms && j < BURA_MAX_TERMS; ++j) {
    for (int r = 0; r < nrhs; ++r) {
      if (slot && j >= slot->nterms[r]) continue;
      const double tol = slot && slot->tol ? slot->tol[r] : P->run_tol;
      const size_t s = (size_t)j * R + r;
      R_.iters[j] = std::max(R_.iters[j], it[s]);
      R_.outer[j] = std::max(R_.outer[j], outer[s]);
      R_.relres[j] = std::max(R_.relres[j], rr[s]);
      if (flags[s] & 1) status = BURA_ENAN;
      if (status == BURA_OK && !(rr[s] <= tol)) status = BURA_ENOCONV;
    }
  }
  if (status == BURA_OK && mixed && etol > 0.0 && rows > 0 && !(eb <= etol)) status = BURA_ENOCONV;
  R_.status = status;
  R_.err_bound = eb;
  R_.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = R_;
  return status;
}

int validate_opts(const bura_opts_t* o) {
  if (!o) return BURA_EINVAL;
  if (!(o->tol > 0) || !(o->inner_tol > 0) || o->max_iter < 0 || o->nrhs_max < 1 || o->max_outer < 1)
    return BURA_EINVAL;
  if (o->precision != BURA_FP64 && o->precision != BURA_MIXED) return BURA_EINVAL;
  if (o->schedule != BURA_BATCHED && o->schedule != BURA_PER_POLE) return BURA_EINVAL;
  // the V-cycle must be symmetric for PCG (post-smoothing = pre-smoothing
  // reversed), and the per-sweep weight sets hold up to three sweeps
  if (o->nu_pre != o->nu_post || o->nu_pre < 1 || o->nu_pre > 3) return BURA_EINVAL;
  if (o->check_every < 1) return BURA_EINVAL;
  if (!(o->err_tol >= 0.0) || !std::isfinite(o->err_tol)) return BURA_EINVAL;
  if (o->err_tol > 0.0 && o->precision != BURA_MIXED) return BURA_EUNSUPPORTED;
  const int known = BURA_VARIANT_UNFUSED | BURA_VARIANT_NO_FOLDXR | BURA_VARIANT_FOLD_SCALARS | BURA_VARIANT_NO_GRAPH;
  if (o->variant & ~known) return BURA_EINVAL;
  return BURA_OK;
}

// The partial-fraction terms of a plan, u_a = sum_{j in output a} w_j (A + s_j I)^-1 f.
struct Terms {
  std::vector<double> w, s;
  std::vector<int> begin{0};   // first term of each output
  double E = 0.0;
  std::vector<Stage> stages;   // sequential form (one output), see Stage
  // fractional power approximated by each output (empty for caller-given
  // terms): with unscaled input the output is multiplied by Lambda^-alpha
  std::vector<double> out_alpha;
};

int check_terms(const Terms& t) {
  const int nterms = (int)t.w.size();
  if (nterms < 1 || nterms > BURA_MAX_TERMS || t.s.size() != t.w.size() || t.begin.empty()) return BURA_EINVAL;
  for (size_t a = 0; a < t.begin.size(); ++a) {
    const int e = a + 1 < t.begin.size() ? t.begin[a + 1] : nterms;
    if (t.begin[a] < 0 || t.begin[a] >= e || (a == 0 && t.begin[0] != 0)) return BURA_EINVAL;
  }
  for (int j = 0; j < nterms; ++j)
    if (!(t.s[j] >= 0.0) || !std::isfinite(t.w[j]) || !std::isfinite(t.s[j])) return BURA_EINVAL;
  if (!t.stages.empty()) {
    if (t.begin.size() != 1) return BURA_EINVAL;
    int next = 0;
    for (size_t i = 0; i < t.stages.size(); ++i) {
      const Stage& g = t.stages[i];
      if (g.tb != next || g.te <= g.tb || g.te > nterms) return BURA_EINVAL;
      if (i == 0 && (g.input != Stage::F || g.base)) return BURA_EINVAL;
      if (g.input == Stage::SOL && (g.sol_term < 0 || g.sol_term >= g.tb)) return BURA_EINVAL;
      if (!std::isfinite(g.base_w)) return BURA_EINVAL;
      next = g.te;
    }
    if (next != nterms) return BURA_EINVAL;
  }
  return BURA_OK;
}

// Terms that depend on the plan's spectral bound Lambda (known after the
// operator is built) are produced by `late`.
using LateTerms = std::function<int(double lambda, Terms& t)>;

// ---------------------------------------------------------------------------
// Launch-shape tuning (opts.autotune).  The knobs are the tile variant of the
// 2D stencil product and of each level's fused down and up kernels (levels
// with n >= kTuneMinN; smaller ones are launch-bound and keep the default).
// Each knob in turn (coordinate descent from the defaults, fine level first)
// takes the variant for which a whole solve of the plan -- every system, in
// the plan's schedule, a fixed pseudo-random right-hand side, to the plan's
// tolerance -- runs fastest.  Timing real solves takes in what a proxy misses: systems
// converging at different iterations (their blocks still launch and exit),
// the alternating buffers, the scalar updates.  (Timed as a few PCG iterations
// with every system active, the tuner picked a 2-row stencil product that is
// 8 % slower in the 2048-system solves.)  The variants are timed in
// interleaved rounds, each by its fastest round, and one must beat the default
// (set_default_tiles) by kTuneMargin.  The solves run without graph capture (captured graphs fix
// the launch shapes).  The choice is cached per (precision, grid,
// coefficients or not, sweeps, systems, schedule) for the life of the process.  The
// variants compute the same value at every point; only the grouping of the
// per-block partial sums of the dot products differs.
// ---------------------------------------------------------------------------
struct TileChoice {
  int spmv = 0;
  std::vector<int> down, up;
};

std::mutex g_tile_mu;
std::map<std::string, TileChoice> g_tile_cache;

// (127: the 511^2 workload's third level, 2048 systems, runs 0.5 - 1 % of
// the solve faster with the row-marching kernels, which the default rule
// keeps to levels of at least 255 points)
constexpr int kTuneMinN = 127;
// interleaved timings per variant (the minimum counts), and how much faster
// than the default a variant must be to replace it: whole solves of a
// batched plan repeat to about 0.3 %, and the shapes that win on the largest
// batches win by 1-2 % per knob (two rounds and a 1 % margin kept the default
// on the 511^2 variable-coefficient workload at 2048 systems, 2 % slower)
constexpr int kTuneRounds = 3;
constexpr float kTuneMargin = 0.005f;

// Systems that share one launch: all of them, one pole's right-hand sides
// (per-pole schedule), or the largest stage (sequential forms).
long long launch_systems(const bura_plan_t P) {
  const long long R = P->opts.nrhs_max;
  if (!P->stages.empty()) {
    long long m = 1;
    for (const Stage& g : P->stages) m = std::max(m, (long long)(g.te - g.tb) * R);
    return m;
  }
  return P->opts.schedule == BURA_PER_POLE ? R : (long long)P->S;
}

// The default launch shapes (default_spmv_tile, default_down_tile,
// default_up_tile): the row-marching kernels on large levels whose launches
// make enough workgroups with them, else the tiles.
void set_default_tiles(bura_plan_t P) {
  const long long ns = launch_systems(P);
  P->tile_spmv = default_spmv_tile(P->dim, P->n, ns);
  for (size_t l = 0; l < P->tile_down.size(); ++l) {
    P->tile_down[l] = default_down_tile(P->dim, P->lev[l].n, ns);
    P->tile_up[l] = default_up_tile(P->dim, P->lev[l].n, ns);
  }
}

int tune_tiles(bura_plan_t P) {
  if (P->dim != 2) return BURA_OK;   // the 3D kernels have one shape
  const bool mixed = P->opts.precision == BURA_MIXED;
  char key[192];
  std::snprintf(key, sizeof(key), "%d/%d/%d/%d/%d/%d/%d/%d/%d/%d", mixed ? 4 : 8, P->dim, P->n, (int)P->var,
                P->opts.nu_pre, P->opts.nu_post, P->S, (int)P->foldxr, (int)P->opts.schedule,
                (int)P->stages.size());
  {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tile_cache.find(key);
    if (it != g_tile_cache.end()) {
      P->tile_spmv = it->second.spmv;
      P->tile_down = it->second.down;
      P->tile_up = it->second.up;
      return BURA_OK;
    }
  }
  hipStream_t st = P->stream;
  // one right-hand side for every system (nrhs = 1 below): uniform in [-1, 1)
  // from a fixed 64-bit linear congruential sequence
  std::vector<double> hf((size_t)P->N);
  uint64_t state = 0x9E3779B97F4A7C15ULL;
  for (auto& v : hf) {
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    v = (double)(state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
  double* df = nullptr;
  if (hipMalloc((void**)&df, hf.size() * 8) != hipSuccess) return BURA_ENOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMemcpyAsync(df, hf.data(), hf.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    hipFree(df);
    return BURA_EDEVICE;
  }
  const bool graphs = P->use_graphs;
  P->use_graphs = false;
  bool ok = true;
  // a timed solve follows the plan's schedule (as in do_solve): stage by
  // stage, pole by pole, or every system in one batch -- a one-system launch
  // fills the chip differently from a batched one
  const int R = P->opts.nrhs_max;
  auto solve_once = [&]() {
    auto batch = [&](size_t sys0, int nsys) {
      return mixed ? solve_batch_mixed(P, df, 1, sys0, nsys, false) : solve_batch_fp64(P, df, 1, sys0, nsys, false);
    };
    int rc = BURA_OK;
    if (!P->stages.empty()) {
      for (size_t si = 0; si < P->stages.size() && rc == BURA_OK; ++si)
        rc = batch((size_t)P->stages[si].tb * R, (P->stages[si].te - P->stages[si].tb) * R);
    } else if (P->opts.schedule == BURA_PER_POLE) {
      for (int j = 0; j < P->nterms && rc == BURA_OK; ++j) rc = batch((size_t)j * R, R);
    } else {
      rc = batch(0, P->S);
    }
    return rc;
  };
  auto timed = [&]() {
    float ms = 0.0f;
    // the per-solve counters a solve starts from (as in do_solve)
    set_flags(P, P->st.flags, 0, P->S, 0);
    set_flags(P, P->st.total_iters, 0, P->S, 0);
    set_flags(P, P->st.outer, 0, P->S, 0);
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    const int rc = ok ? solve_once() : BURA_EDEVICE;
    ok = ok && rc == BURA_OK && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    return ms;
  };
  // BURA_TUNE_LOG=1 prints the timings of each knob's variants to stderr
  const char* tl_env = std::getenv("BURA_TUNE_LOG");
  const bool log = tl_env && tl_env[0] == '1';
  int knob_id = 0;
  // kind: 0 stencil product, 1 down, 2 up (variants that repeat another's
  // shape on this level are not timed)
  auto tune = [&](int* knob, int kind, int n) {
    const int def = *knob;
    float best_of[kTileVariants];
    bool timed_v[kTileVariants];
    for (int v = 0; v < kTileVariants; ++v) {
      best_of[v] = 0.0f;
      timed_v[v] = v == def || tile_variant_distinct(kind, P->dim, n, v);
    }
    for (int r = 0; r < kTuneRounds && ok; ++r) {
      for (int v = 0; v < kTileVariants && ok; ++v) {
        if (!timed_v[v]) continue;
        *knob = v;
        const float ms = timed();
        if (r == 0 || ms < best_of[v]) best_of[v] = ms;
      }
    }
    int best = def;
    for (int v = 0; v < kTileVariants; ++v)
      if (timed_v[v] && v != best && best_of[v] < best_of[best] * (best == def ? 1.0f - kTuneMargin : 1.0f))
        best = v;
    *knob = best;
    if (log) {
      std::fprintf(stderr, "[bura tune] knob %d:", knob_id);
      for (int v = 0; v < kTileVariants; ++v) std::fprintf(stderr, " %.4f", timed_v[v] ? best_of[v] : 0.0f);
      std::fprintf(stderr, " ms -> %d\n", best);
    }
    ++knob_id;
  };
  // the row-marching down and up kernels of a level together (then the up
  // kernel forms the pre-smoothed iterate again and the down kernel stores
  // none): a pair that changing one knob at a time does not reach from the
  // tiles (1023^2, 30 systems, mixed: 5.13 -> 4.89 ms per solve)
  auto tune_pair = [&](int l) {
    const int n = P->lev[l].n;
    const int d0 = P->tile_down[l], u0 = P->tile_up[l];
    const int cand[2] = {kRowsVariant, kShortRowsVariant};
    float base = 0.0f, best_ms[2] = {0.0f, 0.0f};
    bool timed_c[2];
    for (int c = 0; c < 2; ++c)
      timed_c[c] = tile_variant_distinct(1, P->dim, n, cand[c]) && !(d0 == cand[c] && u0 == cand[c]);
    if (!timed_c[0] && !timed_c[1]) return;
    for (int r = 0; r < kTuneRounds && ok; ++r) {
      P->tile_down[l] = d0;
      P->tile_up[l] = u0;
      const float mb = timed();
      if (r == 0 || mb < base) base = mb;
      for (int c = 0; c < 2 && ok; ++c) {
        if (!timed_c[c]) continue;
        P->tile_down[l] = P->tile_up[l] = cand[c];
        const float ms = timed();
        if (r == 0 || ms < best_ms[c]) best_ms[c] = ms;
      }
    }
    int best = -1;
    float best_t = base * (1.0f - kTuneMargin);
    for (int c = 0; c < 2; ++c)
      if (timed_c[c] && best_ms[c] < best_t) {
        best = c;
        best_t = best_ms[c];
      }
    P->tile_down[l] = best < 0 ? d0 : cand[best];
    P->tile_up[l] = best < 0 ? u0 : cand[best];
    if (log)
      std::fprintf(stderr, "[bura tune] level %d down+up rows: %.4f (current %d/%d) %.4f (3/3) %.4f (4/4) ms -> %d/%d\n",
                   l, base, d0, u0, timed_c[0] ? best_ms[0] : 0.0f, timed_c[1] ? best_ms[1] : 0.0f,
                   P->tile_down[l], P->tile_up[l]);
  };
  set_default_tiles(P);
  timed();   // warm-up (clocks, caches, first-touch)
  tune(&P->tile_spmv, 0, P->n);
  for (int l = 0; l < P->lc && fused_ok(P) && ok; ++l) {
    if (P->lev[l].n < kTuneMinN) continue;
    tune(&P->tile_down[l], 1, P->lev[l].n);
    tune(&P->tile_up[l], 2, P->lev[l].n);
    tune_pair(l);
  }
  P->use_graphs = graphs;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  const bool synced = hipStreamSynchronize(st) == hipSuccess;
  hipFree(df);
  if (!ok || !synced) return BURA_EDEVICE;
  TileChoice c;
  c.spmv = P->tile_spmv;
  c.down = P->tile_down;
  c.up = P->tile_up;
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tile_cache[key] = c;
  return BURA_OK;
}

int create(const bura_grid_t* g, Terms terms, const bura_opts_t* opts_in, bura_plan_t* out,
           const LateTerms& late = LateTerms(), void* ws = nullptr, size_t ws_cap = 0) {
  if (out) *out = nullptr;
  if (!g || !out) return BURA_EINVAL;
  if (!late && check_terms(terms)) return BURA_EINVAL;
  if (g->dim != 2 && g->dim != 3) return BURA_EINVAL;
  if (g->n < 1) return BURA_EINVAL;
  if (g->rhs_unscaled != 0 && g->rhs_unscaled != 1) return BURA_EINVAL;
  long long N = 1;
  for (int a = 0; a < g->dim; ++a) N *= g->n;
  if (N > 2147483647LL) return BURA_EINVAL;
  bura_opts_t o;
  if (opts_in) o = *opts_in;
  else bura_opts_default(&o);
  if (const int vr = validate_opts(&o)) return vr;
  if (o.err_tol > 0.0 && !terms.stages.empty()) return BURA_EUNSUPPORTED;   // no bound for sequential forms
  if (ws && o.autotune) return BURA_EINVAL;   // tuning times solves with its own events
  if (g->coeff) {
    const long long m = (long long)(g->n + 2);
    long long cnt = g->dim == 2 ? m * m : m * m * m;
    for (long long i = 0; i < cnt; ++i)
      if (!(g->coeff[i] > 0.0) || !std::isfinite(g->coeff[i])) return BURA_EINVAL;
  }
  auto* P = new bura_plan_s();
  P->dim = g->dim;
  P->n = g->n;
  P->N = N;
  P->var = g->coeff != nullptr;
  P->opts = o;
  P->user_stream = (hipStream_t)o.stream;
  if (ws) {
    P->ws_base = (char*)ws;
    P->ws_cap = ws_cap;
  }
  P->use_graphs = !(o.variant & BURA_VARIANT_NO_GRAPH) && !ws;
  // folding the scalar updates into the producing kernels needs a device-scope
  // fence per block, which on a multi-XCD part writes back L2; it is slower
  // than a separate launch, so it is a variant, not the default
  P->fold = (o.variant & BURA_VARIANT_FOLD_SCALARS) != 0;
  P->unfused = (o.variant & BURA_VARIANT_UNFUSED) != 0;
  int rc = build_levels(P, g);
  if (rc) { delete P; return rc; }
  P->tile_down.assign(P->lev.size(), 0);
  P->tile_up.assign(P->lev.size(), 0);
  if (late) {
    if ((rc = late(P->lambda, terms)) || (rc = check_terms(terms))) { delete P; return rc ? rc : BURA_EINVAL; }
  }
  const int nterms = (int)terms.w.size();
  // unscaled input f~ of A~^alpha u = f~ (Section 1.4, eq. (10)): u = A~^-alpha f~ =
  // Lambda^-alpha A^-alpha f~, the factor folded into the combine weights of each
  // output (for a sequential form: its last stage, whose output is u)
  std::vector<double> wdev = terms.w;
  if (g->rhs_unscaled) {
    const int nout = (int)terms.begin.size();
    if ((int)terms.out_alpha.size() != nout) { delete P; return BURA_EINVAL; }
    if (!terms.stages.empty()) {
      Stage& last = terms.stages.back();
      const double f = std::pow(P->lambda, -terms.out_alpha[0]);
      for (int j = last.tb; j < last.te; ++j) wdev[j] *= f;
      last.base_w *= f;
    } else {
      for (int a = 0; a < nout; ++a) {
        const double f = std::pow(P->lambda, -terms.out_alpha[a]);
        const int e = a + 1 < nout ? terms.begin[a + 1] : nterms;
        for (int j = terms.begin[a]; j < e; ++j) wdev[j] *= f;
      }
    }
  }
  P->nterms = nterms;
  P->w = terms.w;
  P->w_applied = wdev;
  P->s = terms.s;
  P->nout = (int)terms.begin.size();
  for (int i = 0; i < P->nout; ++i) {
    P->out_begin.push_back(terms.begin[i]);
    P->out_end.push_back(i + 1 < P->nout ? terms.begin[i + 1] : nterms);
  }
  P->E = terms.E;
  P->stages = terms.stages;
  P->S = nterms * o.nrhs_max;
  set_default_tiles(P);
  const bool mixed = o.precision == BURA_MIXED;
  choose_lds(P, mixed ? 4 : 8);
  // the folded vector updates need a multigrid level with a pre-smoothing
  // sweep (the fused down kernel in 2D, the first Jacobi sweep otherwise)
  P->foldxr = P->lc > 0 && !(o.variant & BURA_VARIANT_NO_FOLDXR);
  if (P->opts.max_iter == 0) {
    // automatic cap: multigrid-PCG needs O(1) iterations per digit; Jacobi-PCG
    // (no hierarchy) needs O(sqrt(kappa)) = O(n) per digit
    P->opts.max_iter = P->lc >= 0 ? 200 : 40 * P->n + 200;
  }
  if (o.hbm_budget > 0 && footprint(P, mixed ? 4 : 8, mixed) > o.hbm_budget) {
    delete P;
    return BURA_ENOMEM;
  }
  if (hipGetDevice(&P->device) != hipSuccess) { delete P; return BURA_EDEVICE; }
  auto fail = [&](int code) { bura_plan_destroy(P); return code; };
  if (ws) {
    // everything on the caller's stream, in order after its pending work
    P->stream = P->user_stream;
    P->owns_stream = false;
  } else {
    if (hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking) != hipSuccess) return fail(BURA_EDEVICE);
    if (hipEventCreateWithFlags(&P->join_ev, hipEventDisableTiming) != hipSuccess) return fail(BURA_EDEVICE);
  }
  if ((rc = upload_faces(P))) return fail(rc);
  if (mixed) {
    if ((rc = alloc_work<float>(P, P->w32))) return fail(rc);
    if ((rc = dev_alloc(P, (void**)&P->x64, (size_t)P->S * P->N * 8))) return fail(rc);
    if ((rc = dev_zero(P, P->x64, (size_t)P->S * P->N * 8))) return fail(rc);
  } else {
    if ((rc = alloc_work<double>(P, P->w64))) return fail(rc);
  }
  // the FP64 shift (residual kernel) exists in both modes
  if ((rc = dev_alloc(P, (void**)&P->d_shift64, (size_t)P->S * 8))) return fail(rc);
  {
    std::vector<double> sh(P->S);
    for (int i = 0; i < P->S; ++i) sh[i] = P->s[i / o.nrhs_max];
    if (hipMemcpyAsync(P->d_shift64, sh.data(), sh.size() * 8, hipMemcpyHostToDevice, P->stream) != hipSuccess ||
        hipStreamSynchronize(P->stream) != hipSuccess)
      return fail(BURA_EDEVICE);
  }
  P->partial_len = (size_t)P->S * (size_t)max_partial_blocks(P->dim, P->n, P->N);
  if ((rc = dev_alloc(P, (void**)&P->partial, P->partial_len * 8))) return fail(rc);
  if ((rc = dev_alloc(P, (void**)&P->d_w, nterms * 8))) return fail(rc);
  if (!P->stages.empty() && (rc = dev_alloc(P, (void**)&P->d_buf, (size_t)o.nrhs_max * P->N * 8))) return fail(rc);
  if (hipMemcpyAsync(P->d_w, wdev.data(), nterms * 8, hipMemcpyHostToDevice, P->stream) != hipSuccess ||
      hipStreamSynchronize(P->stream) != hipSuccess)
    return fail(BURA_EDEVICE);
  // state arrays: 6 double + 7 int arrays of length S
  const size_t S = (size_t)P->S;
  const size_t bytes = S * (6 * 8 + 8 * 4);
  if ((rc = dev_alloc(P, &P->state_block, bytes))) return fail(rc);
  if ((rc = dev_zero(P, P->state_block, bytes))) return fail(rc);
  double* dp = (double*)P->state_block;
  P->st.bnorm2 = dp; P->st.rho = dp + S; P->st.alpha = dp + 2 * S; P->st.beta = dp + 3 * S;
  P->st.relres = dp + 4 * S; P->st.fnorm2 = dp + 5 * S;
  P->st.relres64 = nullptr;
  int* ip = (int*)(dp + 6 * S);
  P->st.active = ip; P->st.iters = ip + S; P->st.total_iters = ip + 2 * S; P->st.flags = ip + 3 * S;
  P->st.active64 = ip + 4 * S; P->st.outer = ip + 5 * S;
  // relres64 needs doubles: carve from a separate allocation
  if ((rc = dev_alloc(P, (void**)&P->st.relres64, S * 8))) return fail(rc);
  if ((rc = dev_zero(P, P->st.relres64, S * 8))) return fail(rc);
  if ((rc = dev_alloc(P, (void**)&P->d_cnt, S * sizeof(unsigned int)))) return fail(rc);
  if ((rc = dev_zero(P, P->d_cnt, S * sizeof(unsigned int)))) return fail(rc);
  if ((rc = dev_alloc(P, (void**)&P->prof.d_ctr, BURA_K_COUNT * sizeof(unsigned long long)))) return fail(rc);
  if ((rc = dev_zero(P, P->prof.d_ctr, BURA_K_COUNT * sizeof(unsigned long long)))) return fail(rc);
  // output norms for the error bound (rows = outputs x rhs)
  {
    const size_t rows = (size_t)P->nout * o.nrhs_max;
    const size_t nb = (size_t)((P->N + 255) / 256);
    if ((rc = dev_alloc(P, (void**)&P->d_upart, rows * nb * 8))) return fail(rc);
    if ((rc = dev_alloc(P, (void**)&P->d_unorm, rows * 8))) return fail(rc);
    if (mixed && (rc = dev_alloc(P, (void**)&P->d_tol_err, S * 8))) return fail(rc);
  }
  if (mixed) {
    // each inner solve's tolerance, set per system by the refinement test
    // before the solve starts (every path runs OP_OUTER first)
    if ((rc = dev_alloc(P, (void**)&P->st.tol_inner, S * 8))) return fail(rc);
    P->st.inner_floor = o.inner_tol;
  }
  const size_t state_mirror = S * (6 * 8 + 8 * 4) + S * 8 + (size_t)P->nout * o.nrhs_max * 8;
  if (ws) {
    // host mirrors in ordinary memory (8-byte aligned: the state comes first)
    P->host_mirror.assign(state_mirror + S * sizeof(int) + 8, 0);
    P->h_state = P->host_mirror.data();
    P->h_flags = (int*)(P->host_mirror.data() + state_mirror);
  } else {
    if (hipHostMalloc((void**)&P->h_flags, S * sizeof(int), hipHostMallocDefault) != hipSuccess)
      return fail(BURA_ENOMEM);
    if (hipHostMalloc(&P->h_state, state_mirror, hipHostMallocDefault) != hipSuccess) return fail(BURA_ENOMEM);
  }
  if (o.autotune) {
    if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(BURA_EDEVICE);
    if ((rc = tune_tiles(P))) return fail(rc);
  }
  // only this plan's stream: a device-wide synchronisation would break graph
  // capture running on other plans' streams in other threads
  if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(BURA_EDEVICE);
  *out = P;
  return BURA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Continuous batching on a slot plan (see bura_internal.h)
// ---------------------------------------------------------------------------
namespace bura {

int serve_reset(bura_plan_t P) {
  if (!P || !P->slots || P->opts.precision != BURA_MIXED) return BURA_EUNSUPPORTED;
  const int R = P->opts.nrhs_max, K = P->nterms;
  const size_t S = (size_t)P->S;
  int rc;
  HIPCHK(hipSetDevice(P->device));
  if (!P->d_fserve && (rc = dev_alloc(P, (void**)&P->d_fserve, (size_t)R * P->N * 8))) return rc;
  if (!P->d_init && (rc = dev_alloc(P, (void**)&P->d_init, S * sizeof(int)))) return rc;
  hipStream_t st = P->stream;
  launch_zero(P->d_init, S * sizeof(int), st);
  launch_zero(P->d_wsys, S * 8, st);
  for (int* f : {P->st.active, P->st.active64, P->st.flags, P->st.total_iters, P->st.outer})
    launch_fill_int(f, (long long)S, 0, st);
  P->run_tol = P->opts.tol;
  P->st.tol_outer = P->d_tol;
  P->serve_nterms.assign(R, 0);
  P->serve_w.assign((size_t)R * K, 0.0);
  P->serve_s.assign((size_t)R * K, 0.0);
  P->serve_tol.assign(R, P->opts.tol);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return BURA_OK;
}

int serve_admit(bura_plan_t P, int slot, const double* f_dev, int nterms, const double* w, const double* s,
                double tol) {
  if (!P || !P->d_fserve || !f_dev || !w || !s) return BURA_EINVAL;
  const int R = P->opts.nrhs_max, K = P->nterms;
  if (slot < 0 || slot >= R || nterms < 1 || nterms > K || !(tol > 0.0) || P->serve_nterms[slot] != 0)
    return BURA_EINVAL;
  for (int j = 0; j < nterms; ++j)
    if (!std::isfinite(w[j]) || !(s[j] >= 0.0) || !std::isfinite(s[j])) return BURA_EINVAL;
  HIPCHK(hipSetDevice(P->device));
  hipStream_t st = P->stream;
  const size_t S = (size_t)P->S;
  HIPCHK(hipMemcpyAsync(P->d_fserve + (size_t)slot * P->N, f_dev, (size_t)P->N * 8, hipMemcpyDeviceToDevice, st));
  SlotTermsDev v{};
  v.slot = slot;
  v.R = R;
  v.K = K;
  v.nterms = nterms;
  v.tol = tol;
  for (int j = 0; j < nterms; ++j) {
    v.w[j] = w[j];
    v.s[j] = s[j];
  }
  launch_slot_terms(v, P->d_wsys, P->d_shift64, P->w32.shift, P->d_tol, P->d_init, P->st.total_iters, P->st.outer,
                    P->st.flags, P->st.active, P->st.active64, st);
  // first FP64 residual (x = 0) and outer test of the new systems only: they
  // are flagged in d_init, which stands in for active64 until merged
  SysState Si = P->st;
  Si.active64 = P->d_init;
  const LevelDev<double> L0 = level_view<double>(P, 0);
  launch_residual64(P->dim, P->var, L0, P->d_fserve, P->x64, P->w32.x, P->w32.r, P->d_shift64, P->d_init,
                    P->partial, R, (int)S, true, st, nullptr);
  launch_scalars(OP_OUTER, P->partial, flat_blocks(P->N), (int)S, Si, P->run_tol, P->opts.max_outer, st);
  launch_merge_init(P->d_init, P->st.active64, (int)S, st);
  HIPCHK(hipGetLastError());
  P->serve_nterms[slot] = nterms;
  for (int j = 0; j < K; ++j) {
    P->serve_w[(size_t)slot * K + j] = j < nterms ? w[j] : 0.0;
    P->serve_s[(size_t)slot * K + j] = j < nterms ? s[j] : 0.0;
  }
  P->serve_tol[slot] = tol;
  return BURA_OK;
}

int serve_step(bura_plan_t P) {
  if (!P || !P->d_fserve) return BURA_EINVAL;
  HIPCHK(hipSetDevice(P->device));
  const int S = P->S;
  int a = count_active(P, P->st.active64, 0, S);
  if (a < 0) return BURA_EDEVICE;
  if (a == 0) return 0;
  hipStream_t st = P->stream;
  const bool fx = P->foldxr;
  const SysState Ss = state_at(P, 0);
  const LevelDev<double> L0 = level_view<double>(P, 0);
  Work<float>& W = P->w32;
  int rc;
  if ((rc = run_pcg<float>(P, W, 0, S, P->opts.inner_tol, P->opts.max_iter, fx))) return rc;
  {
    ProfScope ps(P, BURA_K_OTHER);
    launch_x_from_e(L0, P->dim, W.x, P->x64, Ss.active64, S, st, fx ? W.p : nullptr, fx ? W.p2 : nullptr, Ss.alpha,
                    Ss.iters);
  }
  {
    ProfScope ps(P, BURA_K_RESIDUAL64);
    launch_residual64(P->dim, P->var, L0, P->d_fserve, P->x64, W.x, W.r, P->d_shift64, Ss.active64, P->partial,
                      P->opts.nrhs_max, S, false, st, ps.ctr);
  }
  {
    ProfScope ps(P, BURA_K_OTHER);
    launch_scalars(OP_OUTER, P->partial, residual_blocks(P->dim, P->n, S), S, Ss, P->run_tol, P->opts.max_outer, st);
  }
  a = count_active(P, P->st.active64, 0, S);
  return a < 0 ? BURA_EDEVICE : a;
}

int serve_slot_done(bura_plan_t P, int slot, double* u_dev, bura_report_t* rep) {
  if (!P || !P->d_fserve || !u_dev) return BURA_EINVAL;
  const int R = P->opts.nrhs_max, K = P->nterms;
  if (slot < 0 || slot >= R) return BURA_EINVAL;
  const int nt = P->serve_nterms[slot];
  if (nt == 0) return BURA_EINVAL;
  for (int j = 0; j < nt; ++j)
    if (P->h_flags[(size_t)j * R + slot]) return 0;
  HIPCHK(hipSetDevice(P->device));
  hipStream_t st = P->stream;
  const size_t S = (size_t)P->S;
  {
    ProfScope ps(P, BURA_K_COMBINE);
    launch_combine(P->N, P->x64 + (size_t)slot * P->N, P->d_wsys + slot, K, 1, R, u_dev, st, ps.ctr, nullptr, 0.0,
                   true);
  }
  launch_row_norms(u_dev, P->N, 1, P->d_upart, P->d_unorm, st);
  const size_t sb = S * (6 * 8 + 8 * 4);
  HIPCHK(hipMemcpyAsync(P->h_state, P->state_block, sb, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync((char*)P->h_state + sb, P->st.relres64, S * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync((char*)P->h_state + sb + S * 8, P->d_unorm, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double* hd = (const double*)P->h_state;
  const int* hi = (const int*)(hd + 6 * S);
  const double* rr = (const double*)((const char*)P->h_state + sb);
  const double un = std::sqrt(*(const double*)((const char*)P->h_state + sb + S * 8));
  bura_report_t R_{};
  R_.nterms = nt;
  int status = BURA_OK;
  double acc = 0.0;
  for (int j = 0; j < nt; ++j) {
    const size_t sy = (size_t)j * R + slot;
    R_.iters[j] = hi[2 * S + sy];
    R_.outer[j] = hi[5 * S + sy];
    R_.relres[j] = rr[sy];
    if (hi[3 * S + sy] & 1) status = BURA_ENAN;
    if (status == BURA_OK && !(rr[sy] <= P->serve_tol[slot])) status = BURA_ENOCONV;
    acc += std::fabs(P->serve_w[(size_t)slot * K + j]) * std::sqrt(hd[5 * S + sy]) * rr[sy] /
           (P->lam_lb + P->serve_s[(size_t)slot * K + j]);
  }
  R_.status = status;
  R_.err_bound = acc == 0.0 ? 0.0 : (un > 0.0 ? acc / un : HUGE_VAL);
  P->serve_nterms[slot] = 0;
  if (rep) *rep = R_;
  return 1;
}

}  // namespace bura

// ---------------------------------------------------------------------------
// Static device workspace of bura_solve_static: one copy per GPU, held until
// the process ends.  In host code the symbol is only a host-side stand-in;
// its device address on the current GPU comes from hipGetSymbolAddress, once
// per device, and only that address is passed to kernels and fill launches.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[BURA_STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};   // device address of `scratch`, per device ordinal

int scratch_on_current_device(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return BURA_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return BURA_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BURA_OK;
}

// Tickets of asynchronous solves, valid across plans until polled.
struct TicketRec {
  int status = BURA_PENDING;
  bura_report_t rep{};
};
std::mutex g_tk_mu;
std::condition_variable g_tk_cv;
std::unordered_map<uint64_t, TicketRec> g_tickets;
uint64_t g_next_ticket = 1;

void worker_loop(bura_plan_t P) {
  for (;;) {
    bura_plan_s::Job j;
    {
      std::unique_lock<std::mutex> lk(P->q_mu);
      P->q_cv.wait(lk, [&]() { return P->stop || !P->queue.empty(); });
      if (P->queue.empty()) return;   // stop requested and nothing left
      j = std::move(P->queue.front());
      P->queue.pop_front();
      ++P->running;
    }
    bura_report_t rep{};
    int rc;
    {
      std::lock_guard<std::mutex> ex(P->exec_mu);
      if (j.slots) {
        const SlotTerms t{j.nterms.data(), j.w.data(), j.s.data(), j.tolv.empty() ? nullptr : j.tolv.data()};
        rc = do_solve(P, j.f, j.u, j.nrhs, &rep, &t);
      } else {
        rc = do_solve(P, j.f, j.u, j.nrhs, &rep, nullptr, j.tol);
      }
    }
    rep.status = rc;
    {
      std::lock_guard<std::mutex> lk(g_tk_mu);
      TicketRec& r = g_tickets[j.ticket];
      r.status = rc;
      r.rep = rep;
    }
    g_tk_cv.notify_all();
    {
      std::lock_guard<std::mutex> lk(P->q_mu);
      --P->running;
    }
    P->q_cv.notify_all();
  }
}

uint64_t enqueue(bura_plan_t P, bura_plan_s::Job&& j) {
  uint64_t t;
  {
    std::lock_guard<std::mutex> lk(g_tk_mu);
    t = g_next_ticket++;
    g_tickets[t] = TicketRec{};
  }
  j.ticket = t;
  {
    std::lock_guard<std::mutex> lk(P->q_mu);
    P->queue.push_back(std::move(j));
    if (!P->worker.joinable()) P->worker = std::thread(worker_loop, P);
  }
  P->q_cv.notify_all();
  return t;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int bura_solve_static(const bura_grid_t* grid, int nterms, const double* weights, const double* shifts,
                      const bura_opts_t* opts, const double* f_dev, double* u_dev, int nrhs, bura_report_t* rep) {
  if (!grid || !weights || !shifts || !f_dev || !u_dev || nterms < 1 || nterms > BURA_MAX_TERMS || nrhs < 1)
    return BURA_EINVAL;
  void* ws = nullptr;
  int rc = scratch_on_current_device(&ws);
  if (rc) return rc;
  Terms t;
  t.w.assign(weights, weights + nterms);
  t.s.assign(shifts, shifts + nterms);
  bura_plan_t P = nullptr;
  if ((rc = create(grid, t, opts, &P, LateTerms(), ws, BURA_STATIC_SCRATCH_BYTES))) return rc;
  rc = do_solve(P, f_dev, u_dev, nrhs, rep);
  bura_plan_destroy(P);
  return rc;
}

int bura_device_copy(void* dst_dev, const void* src_dev, size_t bytes, void* stream) {
  if (!dst_dev || !src_dev || ((uintptr_t)dst_dev & 15) || ((uintptr_t)src_dev & 15)) return BURA_EINVAL;
  const char* d = (const char*)dst_dev;
  const char* s = (const char*)src_dev;
  if (d < s + bytes && s < d + bytes) return BURA_EINVAL;
  launch_stream_copy(dst_dev, src_dev, bytes, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return BURA_OK;
}

int bura_opts_default(bura_opts_t* o) {
  if (!o) return BURA_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-12;
  o->inner_tol = 5e-6;
  o->precision = BURA_MIXED;
  o->schedule = BURA_BATCHED;
  o->max_iter = 0;
  o->max_outer = 12;
  o->nrhs_max = 1;
  o->check_every = 4;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->omega = 0.0;
  o->stream = nullptr;
  o->hbm_budget = 0;
  o->autotune = 0;
  o->err_tol = 0.0;
  o->variant = 0;
  return BURA_OK;
}

int bura_plan_create_rational(const bura_grid_t* grid, int nterms, const double* weights, const double* shifts,
                              const bura_opts_t* opts, bura_plan_t* out) {
  if (out) *out = nullptr;
  if (!weights || !shifts || nterms < 1 || nterms > BURA_MAX_TERMS) return BURA_EINVAL;
  Terms t;
  t.w.assign(weights, weights + nterms);
  t.s.assign(shifts, shifts + nterms);
  return create(grid, t, opts, out);
}

int bura_plan_create_slots(const bura_grid_t* grid, int max_terms, const bura_opts_t* opts, bura_plan_t* out) {
  if (out) *out = nullptr;
  if (!out || max_terms < 1 || max_terms > BURA_MAX_TERMS) return BURA_EINVAL;
  if (opts && opts->schedule != BURA_BATCHED) return BURA_EUNSUPPORTED;
  Terms t;   // placeholders: every solve brings its own weights and shifts
  t.w.assign(max_terms, 0.0);
  t.s.assign(max_terms, 0.0);
  bura_plan_t P = nullptr;
  int rc = create(grid, t, opts, &P);
  if (rc) return rc;
  const size_t S = (size_t)P->S;
  if ((rc = dev_alloc(P, (void**)&P->d_wsys, S * 8)) || (rc = dev_alloc(P, (void**)&P->d_tol, S * 8))) {
    bura_plan_destroy(P);
    return rc;
  }
  if (hipHostMalloc(&P->h_slot, S * (3 * 8 + 4 + 4), hipHostMallocDefault) != hipSuccess) {
    bura_plan_destroy(P);
    return BURA_ENOMEM;
  }
  P->slots = true;
  if (P->opts.precision == BURA_MIXED) P->st.tol_outer = P->d_tol;
  else P->st.tol_pcg = P->d_tol;
  *out = P;
  return BURA_OK;
}

int bura_plan_create_rational_multi(const bura_grid_t* grid, int nout, const int* nterms, const double* weights,
                                    const double* shifts, const bura_opts_t* opts, bura_plan_t* out) {
  if (out) *out = nullptr;
  if (!nterms || !weights || !shifts || nout < 1 || nout > BURA_MAX_TERMS) return BURA_EINVAL;
  Terms t;
  t.begin.clear();
  int total = 0;
  for (int a = 0; a < nout; ++a) {
    if (nterms[a] < 1 || total + nterms[a] > BURA_MAX_TERMS) return BURA_EINVAL;
    t.begin.push_back(total);
    total += nterms[a];
  }
  t.w.assign(weights, weights + total);
  t.s.assign(shifts, shifts + total);
  return create(grid, t, opts, out);
}

int bura_plan_create_sinc(const bura_grid_t* grid, int nalpha, const double* alphas, const double* kprimes,
                          const bura_opts_t* opts, bura_plan_t* out) {
  if (out) *out = nullptr;
  if (!alphas || !kprimes || nalpha < 1 || nalpha > BURA_MAX_TERMS) return BURA_EINVAL;
  for (int a = 0; a < nalpha; ++a) {
    int cnt = 0;
    // validate and count before the operator is built
    const int rc = bura_sinc_coefficients(alphas[a], kprimes[a], 1.0, 0, nullptr, nullptr, &cnt);
    if (rc != BURA_OK && cnt == 0) return rc;
  }
  std::vector<double> al(alphas, alphas + nalpha), kp(kprimes, kprimes + nalpha);
  LateTerms late = [al, kp](double lambda, Terms& t) -> int {
    t.w.clear();
    t.s.clear();
    t.begin.clear();
    for (size_t a = 0; a < al.size(); ++a) {
      double w[BURA_MAX_TERMS], s[BURA_MAX_TERMS];
      int cnt = 0;
      const int rc = bura_sinc_coefficients(al[a], kp[a], lambda, BURA_MAX_TERMS - (int)t.w.size(), w, s, &cnt);
      if (rc) return rc;
      t.begin.push_back((int)t.w.size());
      t.w.insert(t.w.end(), w, w + cnt);
      t.s.insert(t.s.end(), s, s + cnt);
      t.out_alpha.push_back(al[a]);
    }
    return BURA_OK;
  };
  return create(grid, Terms(), opts, out, late);
}

int bura_plan_create_multistep(const bura_grid_t* grid, int nsteps, const double* alphas, const int* ks,
                               const bura_opts_t* opts, bura_plan_t* out) {
  if (out) *out = nullptr;
  if (!alphas || !ks || nsteps < 1 || nsteps > BURA_MAX_TERMS) return BURA_EINVAL;
  Terms t;
  double asum = 0.0;
  for (int i = 0; i < nsteps; ++i) {
    const int k = ks[i];
    if (!(alphas[i] > 0.0 && alphas[i] < 1.0) || k < 1 || k > 16) return BURA_EINVAL;
    asum += alphas[i];
    std::vector<double> c(k + 1), d(k + 1);
    double E = 0.0;
    const int rc = bura_coefficients(alphas[i], 1, k, c.data(), d.data(), &E);
    if (rc) return rc;
    Stage g;
    g.tb = (int)t.w.size();
    for (int j = 0; j <= k; ++j) {
      t.w.push_back(c[j]);
      t.s.push_back(-d[j]);
    }
    g.te = (int)t.w.size();
    g.input = i == 0 ? Stage::F : Stage::PREV;
    t.stages.push_back(g);
    t.E = std::max(t.E, E);
  }
  if (!(asum > 0.0) || (int)t.w.size() > BURA_MAX_TERMS) return BURA_EINVAL;
  t.out_alpha = {asum};
  return create(grid, t, opts, out);
}

int bura_plan_create_product(const bura_grid_t* grid, double alpha, int beta, int k, const bura_opts_t* opts,
                             bura_plan_t* out) {
  if (out) *out = nullptr;
  if (!(alpha > 0.0 && alpha < 1.0) || k < 1 || k > 16) return BURA_EINVAL;
  if (beta != 1) return BURA_EUNSUPPORTED;
  std::vector<double> c(k + 1), d(k + 1), zeta(k);
  double E = 0.0, C = 0.0;
  int rc = bura_coefficients(alpha, beta, k, c.data(), d.data(), &E);
  if (rc) return rc;
  if ((rc = bura_zeros(alpha, beta, k, zeta.data(), &C))) return rc;
  // v_0 = A^-1 f; v_j = (A - zeta_j)(A - d_j)^-1 v_{j-1} = v_{j-1} + (d_j - zeta_j)(A - d_j)^-1 v_{j-1};
  // u = C v_k, the constant folded into the last stage
  Terms t;
  t.w.push_back(1.0);
  t.s.push_back(0.0);
  Stage g0;
  g0.tb = 0;
  g0.te = 1;
  t.stages.push_back(g0);
  for (int j = 1; j <= k; ++j) {
    const double scale = j == k ? C : 1.0;
    t.w.push_back(scale * (d[j] - zeta[j - 1]));
    t.s.push_back(-d[j]);
    Stage g;
    g.tb = j;
    g.te = j + 1;
    g.input = Stage::PREV;
    g.base = true;
    g.base_w = scale;
    t.stages.push_back(g);
  }
  t.E = E;
  t.out_alpha = {alpha};
  return create(grid, t, opts, out);
}

int bura_plan_create_multi(const bura_grid_t* grid, int nalpha, const double* alphas, int beta, const int* ks,
                           const bura_opts_t* opts, bura_plan_t* out) {
  if (out) *out = nullptr;
  if (!alphas || !ks || nalpha < 1) return BURA_EINVAL;
  if (beta != 1) return BURA_EUNSUPPORTED;
  std::vector<double> c, s;
  std::vector<int> begin;
  double E = 0.0;
  for (int a = 0; a < nalpha; ++a) {
    const int k = ks[a];
    if (!(alphas[a] > 0.0 && alphas[a] < 1.0) || k < 1 || k > 16) return BURA_EINVAL;
    std::vector<double> cc(k + 1), dd(k + 1);
    double Ea = 0.0;
    const int rc = bura_coefficients(alphas[a], beta, k, cc.data(), dd.data(), &Ea);
    if (rc) return rc;
    begin.push_back((int)c.size());
    for (int j = 0; j <= k; ++j) {
      c.push_back(cc[j]);
      s.push_back(-dd[j]);
    }
    E = std::max(E, Ea);
  }
  if ((int)c.size() > BURA_MAX_TERMS) return BURA_EINVAL;
  Terms t;
  t.w = c;
  t.s = s;
  t.begin = begin;
  t.E = E;
  t.out_alpha.assign(alphas, alphas + nalpha);
  return create(grid, t, opts, out);
}

int bura_plan_create(const bura_grid_t* grid, double alpha, int beta, int k, const bura_opts_t* opts,
                     bura_plan_t* out) {
  if (out) *out = nullptr;
  if (!(alpha > 0.0 && alpha < 1.0) || k < 1 || k > 16) return BURA_EINVAL;
  if (beta != 1 && beta != 2) return BURA_EUNSUPPORTED;
  std::vector<double> c(k + 2), d(k + 1);
  double E = 0.0;
  int rc = bura_coefficients(alpha, beta, k, c.data(), d.data(), &E);
  if (rc) return rc;
  Terms t;
  for (int j = 0; j <= k; ++j) {
    t.w.push_back(c[j]);
    t.s.push_back(-d[j]);
  }
  t.E = E;
  if (beta == 2) {
    // eq. (25) with beta = 2: the k+1 systems of c_{0,1} A^-1 f + sum_j c_j (A - d_j)^-1 f
    // in one stage, then A^-2 f = A^-1 (A^-1 f) from the first stage's pole-0
    // solution, added with c_{0,2} (Section 4.3's chained solve)
    t.w.push_back(c[k + 1]);
    t.s.push_back(0.0);
    Stage g0;
    g0.tb = 0;
    g0.te = k + 1;
    Stage g1;
    g1.tb = k + 1;
    g1.te = k + 2;
    g1.input = Stage::SOL;
    g1.sol_term = 0;
    g1.base = true;
    g1.base_w = 1.0;
    t.stages = {g0, g1};
  }
  t.out_alpha = {alpha};
  return create(grid, t, opts, out);
}

int bura_solve(bura_plan_t plan, const double* f_dev, double* u_dev, int nrhs, bura_report_t* rep) {
  if (!plan) return BURA_EINVAL;
  std::lock_guard<std::mutex> lk(plan->exec_mu);
  return do_solve(plan, f_dev, u_dev, nrhs, rep);
}

int bura_solve_slots(bura_plan_t plan, const double* f_dev, double* u_dev, int nrhs, const int* nterms,
                     const double* weights, const double* shifts, const double* tol, bura_report_t* rep) {
  if (!plan) return BURA_EINVAL;
  const SlotTerms t{nterms, weights, shifts, tol};
  std::lock_guard<std::mutex> lk(plan->exec_mu);
  return do_solve(plan, f_dev, u_dev, nrhs, rep, &t);
}

int bura_submit_slots(bura_plan_t plan, const double* f_dev, double* u_dev, int nrhs, const int* nterms,
                      const double* weights, const double* shifts, const double* tol, bura_ticket_t* ticket) {
  if (ticket) *ticket = 0;
  if (!plan || !ticket || !plan->slots || !f_dev || !u_dev || nrhs < 1 || nrhs > plan->opts.nrhs_max)
    return BURA_EINVAL;
  const SlotTerms t{nterms, weights, shifts, tol};
  if (check_slot_terms(plan, nrhs, t)) return BURA_EINVAL;
  // the job keeps its own copies (the caller's arrays may go away)
  bura_plan_s::Job j;
  const size_t K = (size_t)plan->nterms;
  j.f = f_dev;
  j.u = u_dev;
  j.nrhs = nrhs;
  j.slots = true;
  j.nterms.assign(nterms, nterms + nrhs);
  j.w.assign(weights, weights + nrhs * K);
  j.s.assign(shifts, shifts + nrhs * K);
  if (tol) j.tolv.assign(tol, tol + nrhs);
  *ticket = enqueue(plan, std::move(j));
  return BURA_OK;
}

int bura_submit(bura_plan_t plan, const double* f_dev, double* u_dev, int nrhs, double tol, bura_ticket_t* ticket) {
  if (ticket) *ticket = 0;
  if (!plan || !ticket || plan->slots || !f_dev || !u_dev || nrhs < 1 || nrhs > plan->opts.nrhs_max)
    return BURA_EINVAL;
  if (!(tol >= 0.0) || !std::isfinite(tol)) return BURA_EINVAL;
  bura_plan_s::Job j;
  j.f = f_dev;
  j.u = u_dev;
  j.nrhs = nrhs;
  j.tol = tol;
  *ticket = enqueue(plan, std::move(j));
  return BURA_OK;
}

int bura_poll(bura_ticket_t ticket, bura_report_t* rep) {
  std::lock_guard<std::mutex> lk(g_tk_mu);
  auto it = g_tickets.find(ticket);
  if (it == g_tickets.end()) return BURA_EINVAL;
  if (it->second.status == BURA_PENDING) return BURA_PENDING;
  const int rc = it->second.status;
  if (rep) *rep = it->second.rep;
  g_tickets.erase(it);
  return rc;
}

int bura_wait(bura_ticket_t ticket, bura_report_t* rep) {
  std::unique_lock<std::mutex> lk(g_tk_mu);
  auto it = g_tickets.find(ticket);
  if (it == g_tickets.end()) return BURA_EINVAL;
  g_tk_cv.wait(lk, [&]() { return it->second.status != BURA_PENDING; });
  const int rc = it->second.status;
  if (rep) *rep = it->second.rep;
  g_tickets.erase(it);
  return rc;
}

int bura_plan_coeffs(bura_plan_t plan, int* nterms, double* c, double* d, double* E) {
  if (!plan) return BURA_EINVAL;
  if (nterms) *nterms = plan->nterms;
  for (int j = 0; j < plan->nterms; ++j) {
    if (c) c[j] = plan->w[j];
    if (d) d[j] = -plan->s[j];
  }
  if (E) *E = plan->E;
  return BURA_OK;
}

int bura_plan_outputs(bura_plan_t plan, int* nout, int* term_begin) {
  if (!plan) return BURA_EINVAL;
  if (nout) *nout = plan->nout;
  if (term_begin)
    for (int i = 0; i <= plan->nout; ++i) term_begin[i] = i < plan->nout ? plan->out_begin[i] : plan->nterms;
  return BURA_OK;
}

int bura_plan_info(bura_plan_t plan, double* lambda, int* nlevels, size_t* device_bytes) {
  if (!plan) return BURA_EINVAL;
  if (lambda) *lambda = plan->lambda;
  if (nlevels) *nlevels = (int)plan->lev.size();
  if (device_bytes) *device_bytes = plan->device_bytes;
  return BURA_OK;
}

int bura_plan_apply(bura_plan_t plan, double shift, const double* x_dev, double* y_dev, int nvec) {
  if (!plan || !x_dev || !y_dev || nvec < 1 || !(shift >= 0.0)) return BURA_EINVAL;
  HIPCHK(hipSetDevice(plan->device));
  HIPCHK(hipEventRecord(plan->join_ev, plan->user_stream));
  HIPCHK(hipStreamWaitEvent(plan->stream, plan->join_ev, 0));
  launch_apply64(plan->dim, plan->var, level_view<double>(plan, 0), x_dev, y_dev, shift, nvec, plan->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(plan->stream));
  return BURA_OK;
}

int bura_plan_profile(bura_plan_t plan, int enable) {
  if (!plan) return BURA_EINVAL;
  HIPCHK(hipSetDevice(plan->device));
  HIPCHK(hipStreamSynchronize(plan->stream));
  if (enable) {
    HIPCHK(hipMemsetAsync(plan->prof.d_ctr, 0, BURA_K_COUNT * sizeof(unsigned long long), plan->stream));
    HIPCHK(hipStreamSynchronize(plan->stream));
    plan->prof.rec.clear();
    plan->prof.used = 0;
    for (int c = 0; c < BURA_K_COUNT; ++c) {
      plan->prof.ms[c] = 0.0;
      plan->prof.launches[c] = 0;
    }
  }
  destroy_graphs(plan);   // graphs carry (or lack) the profiling events
  plan->prof.on = enable != 0;
  plan->prof.mask = (unsigned)enable == 1u ? ((1u << BURA_K_COUNT) - 1u) : ((unsigned)enable >> 1);
  return BURA_OK;
}

int bura_plan_kernel_stats(bura_plan_t plan, int kclass, long long* launches, double* total_ms, double* alg_bytes) {
  if (!plan || kclass < 0 || kclass >= BURA_K_COUNT) return BURA_EINVAL;
  HIPCHK(hipSetDevice(plan->device));
  HIPCHK(hipStreamSynchronize(plan->stream));
  prof_flush(plan);
  const long long cnt = plan->prof.launches[kclass];
  const double ms = plan->prof.ms[kclass];
  unsigned long long ctr[BURA_K_COUNT];
  HIPCHK(hipMemcpyAsync(ctr, plan->prof.d_ctr, sizeof(ctr), hipMemcpyDeviceToHost, plan->stream));
  HIPCHK(hipStreamSynchronize(plan->stream));
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = ms;
  if (alg_bytes) *alg_bytes = (double)ctr[kclass];
  return BURA_OK;
}

int bura_plan_tiles(bura_plan_t plan, int* out, int max_len, int* len) {
  if (!plan || !len) return BURA_EINVAL;
  const int nf = fused_ok(plan) ? plan->lc : 0;
  *len = plan->dim == 2 ? 1 + 2 * nf : 0;
  if (!out || *len == 0) return BURA_OK;
  if (max_len < *len) return BURA_EINVAL;
  out[0] = plan->tile_spmv;
  for (int l = 0; l < nf; ++l) {
    out[1 + 2 * l] = plan->tile_down[l];
    out[2 + 2 * l] = plan->tile_up[l];
  }
  return BURA_OK;
}

int bura_plan_set_tiles(bura_plan_t plan, const int* v, int len) {
  if (!plan || (!v && len > 0)) return BURA_EINVAL;
  const int nf = fused_ok(plan) ? plan->lc : 0;
  if (len != (plan->dim == 2 ? 1 + 2 * nf : 0)) return BURA_EINVAL;
  if (len == 0) return BURA_OK;
  for (int i = 0; i < len; ++i)
    if (v[i] < 0 || v[i] >= BURA_TILE_VARIANTS) return BURA_EINVAL;
  {
    std::lock_guard<std::mutex> q(plan->q_mu);
    if (!plan->queue.empty() || plan->running) return BURA_EBUSY;
  }
  std::lock_guard<std::mutex> lk(plan->exec_mu);
  HIPCHK(hipSetDevice(plan->device));
  HIPCHK(hipStreamSynchronize(plan->stream));
  destroy_graphs(plan);   // captured launches carry their grid shapes
  plan->tile_spmv = v[0];
  for (int l = 0; l < nf; ++l) {
    plan->tile_down[l] = v[1 + 2 * l];
    plan->tile_up[l] = v[2 + 2 * l];
  }
  return BURA_OK;
}

void bura_plan_destroy(bura_plan_t plan) {
  if (!plan) return;
  {
    // the worker finishes every queued solve, then exits
    std::lock_guard<std::mutex> q(plan->q_mu);
    plan->stop = true;
  }
  plan->q_cv.notify_all();
  if (plan->worker.joinable()) plan->worker.join();
  hipSetDevice(plan->device);
  if (plan->stream) hipStreamSynchronize(plan->stream);
  destroy_graphs(plan);
  for (hipEvent_t e : plan->prof.pool) hipEventDestroy(e);
  for (void* p : plan->allocs) hipFree(p);
  if (!plan->ws_base) {
    if (plan->h_flags) hipHostFree(plan->h_flags);
    if (plan->h_state) hipHostFree(plan->h_state);
  }
  if (plan->h_slot) hipHostFree(plan->h_slot);
  if (plan->join_ev) hipEventDestroy(plan->join_ev);
  if (plan->stream && plan->owns_stream) hipStreamDestroy(plan->stream);
  delete plan;
}

const char* bura_strerror(int status) {
  switch (status) {
    case BURA_OK: return "ok";
    case BURA_PENDING: return "pending";
    case BURA_EINVAL: return "invalid argument";
    case BURA_EUNSUPPORTED: return "unsupported";
    case BURA_EREMEZ: return "rational approximation did not converge";
    case BURA_ENOCONV: return "iteration limit reached";
    case BURA_ENOMEM: return "out of device memory or over budget";
    case BURA_EDEVICE: return "HIP runtime error";
    case BURA_ENAN: return "non-finite value";
    case BURA_EBUSY: return "plan busy";
    case BURA_ETOOBIG: return "workspace larger than the static scratch array";
    default: return "unknown status";
  }
}

}  // extern "C"
