// Internal declarations shared by the HIP kernels, the solver engine and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bura.h"
#include "bura_remez.h"

namespace bura {

constexpr int kTileX = 64;             // threads along x in a stencil tile
constexpr int kTileY = 4;              // rows per tile
constexpr int kBlock = kTileX * kTileY;
constexpr int kSlots = 2;              // reduction slots per block
constexpr int kMaxLdsLevels = 8;
// Launch-shape variants of the 2D stencil-product and fused level kernels
// (tile sizes in bura_kernels.hip); 0 is the default shape.
constexpr int kTileVariants = BURA_TILE_VARIANTS;
constexpr int tile_variant(int tv) { return tv >= 0 && tv < kTileVariants ? tv : 0; }

// One multigrid level of the scaled operator A_l + s I as seen by a kernel.
// Face weights are a_f / (Lambda h_l^2); the constant-coefficient operator has
// every face weight equal to wc (= 4^-l / (2 dim)).
template <typename T>
struct LevelDev {
  int n;              // interior points per axis
  long long N;        // n^dim
  T wc;               // constant face weight (used when wf0 == nullptr)
  const T* wf0;       // x-faces  [..][n+1]       (nullptr: constant coefficient)
  const T* wf1;       // y-faces  [..][n+1][n]
  const T* wf2;       // z-faces  [n+1][n][n]
};

// Damping weights of the smoothing sweeps of one half-cycle, in the order of
// the pre-smoothing sweeps (the post-smoothing uses them in reverse).
template <typename T>
struct Sweeps {
  T w[3];
};

// Levels solved inside one workgroup (LDS V-cycle): descriptors + LDS offsets.
template <typename T>
struct LdsHierarchy {
  int nlev;
  LevelDev<T> lev[kMaxLdsLevels];
  int off[kMaxLdsLevels];   // element offset of level l's x/b/t arrays in LDS (each N_l long)
  int cycles;               // V-cycles per coarse solve
  int nu;                   // sweeps per smoothing step
  int bottom_sweeps;        // Jacobi sweeps on the last level if it is larger than one point
  T omega;                  // bottom-level damping
  Sweeps<T> pre;            // weights of the nu pre-smoothing sweeps (post: reversed)
};

// Per-system scalar state of the PCG / refinement loops (device arrays, length S).
struct SysState {
  double* bnorm2;   // ||b||^2 of the PCG right-hand side
  double* rho;      // r.z
  double* alpha;
  double* beta;
  double* relres;   // last ||r||/||b|| seen by the PCG
  int* active;      // 1 while the PCG runs on this system
  int* iters;       // PCG iterations done (this inner solve)
  int* total_iters; // PCG iterations summed over refinement steps
  int* flags;       // bit 0: breakdown / non-finite
  // refinement (MIXED) and FP64 outer state
  double* fnorm2;
  double* relres64;
  int* active64;
  int* outer;
  // per-system stopping tolerances (nullptr: the scalar passed with the
  // operation): of the PCG (FP64 mode) and of the refinement (MIXED mode)
  const double* tol_pcg = nullptr;
  const double* tol_outer = nullptr;
  // MIXED: the stopping tolerance of each system's next inner solve, set by
  // the refinement test: the reduction its outer tolerance still needs
  // (halved for margin), but no smaller than inner_floor (opts.inner_tol)
  double* tol_inner = nullptr;
  double inner_floor = 0.0;
};

enum ScalarOp { OP_INIT = 0, OP_ALPHA = 1, OP_RESID = 2, OP_BETA = 3, OP_OUTER = 4 };

// Scalar update folded into the kernel that produces the reduction: the last
// block of each system (counted in cnt[sys]) sums the block partials in the
// fixed order and applies `op` to that system's state.  op < 0: not folded.
struct Fin {
  int op = -1;
  unsigned int* cnt = nullptr;
  SysState st{};
  double tol = 0.0;
  int max_iter = 0;
};

// ---- kernel launchers (bura_kernels.hip) ----------------------------------
template <typename T>
struct Launch {
  static void jacobi(int dim, bool var, const LevelDev<T>& L, const T* b, const T* xin, T* xout,
                     const T* shift, const int* active, T omega, bool zero_guess, double* partial,
                     int nsys, hipStream_t st, unsigned long long* ctr, Fin fin = Fin());
  // zero-guess sweep with the PCG residual update: bout = bold - alpha q,
  // xout = omega D^-1 bout, partial = |bout|^2 (see k_jacobi0_rup)
  // 3D with q == nullptr: q = (A + s) p is formed from p
  static void jacobi_rup(int dim, bool var, const LevelDev<T>& L, const T* bold, const T* q, const double* alpha,
                         T* bout, T* xout, const T* shift, const int* active, T omega, double* partial, int nsys,
                         hipStream_t st, unsigned long long* ctr, Fin fin = Fin(), const T* p = nullptr);
  static void restrict_residual(int dim, bool var, const LevelDev<T>& Lf, const LevelDev<T>& Lc,
                                const T* b, const T* x, T* bc, const T* shift, const int* active,
                                int nsys, hipStream_t st, unsigned long long* ctr);
  static void prolong_add(int dim, const LevelDev<T>& Lc, const LevelDev<T>& Lf, const T* xc, T* xf,
                          const int* active, int nsys, hipStream_t st, unsigned long long* ctr);
  static void coarse_solve(int dim, bool var, const LdsHierarchy<T>& H, const T* b, T* x,
                           const T* shift, const int* active, int nsys, size_t lds_bytes, hipStream_t st,
                           unsigned long long* ctr);
  static void update_xr(const LevelDev<T>& L, int dim, T* x, T* r, const T* p, const T* q,
                        const double* alpha, const int* active, double* partial, int nsys, hipStream_t st,
                        unsigned long long* ctr, Fin fin = Fin());
  static void update_p(const LevelDev<T>& L, int dim, T* p, const T* z, const double* beta,
                       const int* active, int nsys, hipStream_t st, unsigned long long* ctr);
  // p_new = z + beta p_old, q = (A+s) p_new, p_new.q; with x != nullptr also the
  // deferred x += alpha p_old of the previous iteration.  With x != nullptr q
  // may be nullptr (only p_new.q is formed; the fused down kernel in 2D, the
  // first fine sweep in 3D, forms the product again from p_new)
  static void spmv_p(int dim, bool var, const LevelDev<T>& L, const T* z, const T* pold, T* pnew, T* q,
                     const double* beta, const T* shift, const int* active, double* partial, int nsys,
                     hipStream_t st, unsigned long long* ctr, Fin fin = Fin(), T* x = nullptr,
                     const double* alpha = nullptr, int tv = 0);
  // the last deferred x += alpha p of each system (see k_finish_x)
  static void finish_x(long long N, T* x, const T* pa, const T* pb, const double* alpha, const int* iters,
                       int nsys, hipStream_t st, unsigned long long* ctr);
  // fused level kernels (2D); return false when not applicable.  With bout !=
  // nullptr the down kernel first forms b - alpha q, writes it to bout and its
  // squared norm to partial.
  static bool fused_down(int dim, bool var, int nu, const LevelDev<T>& Lf, const LevelDev<T>& Lc, const T* b,
                         T* xout, T* bc, const T* shift, const int* active, Sweeps<T> om, int nsys, hipStream_t st,
                         unsigned long long* ctr, const T* p = nullptr, const double* alpha = nullptr,
                         T* bout = nullptr, double* partial = nullptr, Fin fin = Fin(), int tv = 0,
                         int tv_up = 0);
  static bool fused_up(int dim, bool var, int nu, const LevelDev<T>& Lc, const LevelDev<T>& Lf, const T* xc,
                       const T* xin, const T* b, T* xout, const T* shift, const int* active, Sweeps<T> om,
                       double* partial, int nsys, hipStream_t st, unsigned long long* ctr, Fin fin = Fin(),
                       int tv = 0);
  static void copy_rhs(const LevelDev<T>& L, int dim, const double* f, T* r, T* x, int nrhs,
                       const int* active, double* partial, int nsys, hipStream_t st);
};

// FP64-only steps of the refinement loop and the combine.
void launch_residual64(int dim, bool var, const LevelDev<double>& L, const double* f, const double* x64, float* e,
                       float* r32, const double* shift, const int* active64, double* partial, int nrhs, int nsys,
                       bool first, hipStream_t st, unsigned long long* ctr, bool zero_x = true);
// whether the FP64 residual of nsys systems on a level of n points per axis
// marches whole rows (then launch_update_residual64 applies)
bool residual_marches_rows(int dim, int n, long long nsys);
// x64 += e (as launch_x_from_e) and the FP64 residual of the updated iterate
// in one pass, when the residual marches whole rows (2D wide launches);
// returns false, launching nothing, otherwise
bool launch_update_residual64(int dim, bool var, const LevelDev<double>& L, const double* f, double* x64, float* e,
                              float* r32, const double* shift, const int* active64, double* partial, int nrhs,
                              int nsys, hipStream_t st, unsigned long long* ctr, const float* pa, const float* pb,
                              const double* alpha, const int* iters, bool assign = false);
// x64 += e; with pa != nullptr e first takes the inner solve's pending update
// e + alpha p (p = pa or pb by the parity of the system's iteration count)
void launch_x_from_e(const LevelDev<double>& L, int dim, const float* e, double* x64, const int* active64,
                     int nsys, hipStream_t st, const float* pa = nullptr, const float* pb = nullptr,
                     const double* alpha = nullptr, const int* iters = nullptr);
// u_r = base_w base_r + sum_j w_j x_{j stride + r}; with w_per_system the weight
// of term j of rhs r is w[j stride + r] and zero weights skip their term.
// With pa != nullptr system s = j stride + r still has its last deferred
// update pending (alpha[s], p = pa or pb by the parity of iters[s]; arrays
// indexed from the same first system as x), applied to x_s as it is read.
void launch_combine(long long N, const double* x, const double* w, int nterms, int nrhs, int stride, double* u,
                    hipStream_t st, unsigned long long* ctr, const double* base = nullptr, double base_w = 0.0,
                    bool w_per_system = false, const double* pa = nullptr, const double* pb = nullptr,
                    const double* alpha = nullptr, const int* iters = nullptr);
// out[r] = ||u_r||_2^2 for rows r < rows of [rows][N] (partial: rows x
// ceil(N/256) doubles of scratch); fixed summation order per row
void launch_row_norms(const double* u, long long N, int rows, double* partial, double* out, hipStream_t st);
void launch_apply64(int dim, bool var, const LevelDev<double>& L, const double* x, double* y, double shift,
                    int nvec, hipStream_t st);
void launch_scalars(int op, const double* partial, int nblk, int nsys, SysState st_, double tol,
                    int max_iter, hipStream_t st);
void launch_zero(void* p, size_t bytes, hipStream_t st);
// the terms of one rhs slot of a slot plan, passed by value to a kernel
struct SlotTermsDev {
  int slot, R, K, nterms;
  double tol;
  double w[BURA_MAX_TERMS], s[BURA_MAX_TERMS];
};
void launch_slot_terms(const SlotTermsDev& v, double* w, double* s64, float* s32, double* tol, int* init,
                       int* total_iters, int* outer, int* flags, int* active, int* active64, hipStream_t st);
void launch_merge_init(int* init, int* active64, int n, hipStream_t st);
// dst = src, 16-byte aligned, non-overlapping (counter calibration)
void launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
void launch_fill_int(int* p, long long n, int v, hipStream_t st);
void launch_slot_flags(int* p, int nterms, int R, int nrhs, hipStream_t st);

int stencil_blocks(int dim, int n);   // blocks per system of a stencil launch (tile grid)
int flat_blocks(long long N);        // blocks per system of an element-wise launch
// blocks per system of the fused up kernel, of the fused down kernel (fine
// level n) and of the stencil product with the p update, in shape variant tv
int up_blocks(int dim, int n, int tv);
int down_blocks(int dim, int n, int tv);
// workgroups a launch needs to keep every CU of the chip busy (4 per CU)
constexpr long long kFillBlocks = 4 * 256;
// default launch-shape variants of a level of n points per axis, nsys systems per launch
int default_down_tile(int dim, int n, long long nsys);
int default_up_tile(int dim, int n, long long nsys);
int default_spmv_tile(int dim, int n, long long nsys);
int spmv_blocks(int dim, int n, int tv);
// false where launch-shape variant tv of a kernel kind (0 stencil product, 1 down,
// 2 up) on a level of n points per axis runs the same shape as another variant
bool tile_variant_distinct(int kind, int dim, int n, int tv);
// the launch-shape variants of the row-marching 2D kernels: segments of 128
// fine rows and of 32
constexpr int kRowsVariant = 3, kShortRowsVariant = 4;
// blocks per system of the FP64 residual (refinement step) of a batch of nsys systems
int residual_blocks(int dim, int n, long long nsys);
int max_partial_blocks(int dim, int n, long long N);   // over every launch shape

// Continuous batching on a slot plan (BURA_MIXED): right-hand sides join and
// leave a running solve at outer refinement-step boundaries, where every
// system of the plan is at the start of an inner solve, so each one goes
// through the same operations as in a solve of its own.  One host thread
// drives a plan at a time.
//   serve_reset: no slot in use.
//   serve_admit: stage f into the plan's rhs slot, set its terms and
//     tolerance, form its first FP64 residual (x = 0) and outer test.
//   serve_step: one outer step of every active system (FP32 inner solve,
//     x += e, FP64 residual, outer test); returns the systems still active
//     (or a negative status).
//   serve_slot_done: whether the slot's systems are all finished; if so its
//     combine is written to u_dev, its report filled and 1 returned.
int serve_reset(bura_plan_t P);
int serve_admit(bura_plan_t P, int slot, const double* f_dev, int nterms, const double* w, const double* s,
                double tol);
int serve_step(bura_plan_t P);
int serve_slot_done(bura_plan_t P, int slot, double* u_dev, bura_report_t* rep);

}  // namespace bura
