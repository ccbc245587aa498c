/*
 * bura.h -- C ABI of a gfx950 (MI355X) solver for A^alpha u = f, 0 < alpha < 1.
 *
 * Method: Harizanov, Lazarov, Marinov, Margenov, Vutov, "Optimal solvers for
 * linear systems with fractional powers of sparse SPD matrices"
 * (arXiv:1612.04846).  With A scaled so that its spectrum lies in (0,1]
 * (Section 1.4, eq. (10), Assumption 1.1) the solution is approximated by
 *
 *     u_r = sum_{j=0..k} c_j (A - d_j I)^{-1} f          (Section 2.2, eq. (16))
 *
 * where r(t)/t = sum_j c_j/(t - d_j) (eq. (15)), r the best uniform rational
 * approximation of t^(1-alpha) on [0,1] (Definition 2.1, eq. (11)), d_0 = 0 >
 * d_1 > ... > d_k and c_j > 0 (Lemma 2.5, Remark 2.6).  Each of the k+1 shifted
 * SPD systems is solved on the GPU by geometric-multigrid preconditioned CG;
 * the k+1 solutions are combined in FP64.
 *
 * Grids: the unit square / cube, n interior points per axis, h = 1/(n+1),
 * homogeneous Dirichlet boundary.  Vectors are FP64, interior points only, in
 * lexicographic order with x fastest (the paper's ordering, Section 5.3); a
 * batch of nrhs right-hand sides is nrhs such vectors back to back.
 *
 * Operator (before scaling): the five-point (2D) / seven-point (3D)
 * difference operator A~ = h^-2 * [flux form], (A~ x)_i = h^-2 sum_faces a_f
 * (x_i - x_nb), x_nb = 0 outside the grid; a_f = 1 (Laplacian, Section 5.3) or
 * the harmonic mean 2 a_i a_nb/(a_i + a_nb) of a caller-supplied nodal
 * coefficient a > 0 on the (n+2)^dim lattice including the boundary nodes.
 * Lambda, the upper bound of the spectrum of A~ that scales A = A~/Lambda
 * (Section 1.4, eq. (10)): for the Laplacian 4 dim/h^2 at every n (the
 * paper's scaling in Section 5.3, h^2/8 in 2D; it equals the Gershgorin bound
 * for n >= 3 and exceeds it below); with coefficients the Gershgorin bound
 * max_i sum_j |A~_ij| = max_i 2 A~_ii; or the caller's upper bound.
 *
 * Conventions: every function returns an int status (enum bura_status); none
 * throws or aborts.  Pointers named *_dev are device pointers in the current
 * HIP device's address space (e.g. from hipMalloc or a torch CUDA tensor on
 * ROCm); all other pointers are host pointers.  A plan owns every internal
 * buffer it allocates and frees them in bura_plan_destroy.  Solves on one
 * plan are serialised inside the library (synchronous solves and the plan's
 * queue of asynchronous ones), so several host threads may solve and submit
 * on one plan; creating or destroying a plan must not race with other calls
 * on it.
 */
#ifndef BURA_H
#define BURA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque plan: operator hierarchy, coefficients, device workspace. */
typedef struct bura_plan_s* bura_plan_t;

/* Handle of one asynchronous solve (bura_submit / bura_submit_slots), unique
 * in the process; released by the bura_poll or bura_wait that returns its
 * result.  0 is never a valid ticket. */
typedef uint64_t bura_ticket_t;

enum bura_status {
  BURA_OK = 0,
  BURA_PENDING = 1,          /* bura_poll: the solve is still running            */
  BURA_EINVAL = -1,          /* bad argument                                     */
  BURA_EUNSUPPORTED = -2,    /* valid but not implemented (e.g. beta != 1)       */
  BURA_EREMEZ = -3,          /* the rational approximation did not converge      */
  BURA_ENOCONV = -4,         /* iteration cap hit; u holds the last iterate      */
  BURA_ENOMEM = -5,          /* device allocation failed / over the HBM budget   */
  BURA_EDEVICE = -6,         /* HIP runtime error                                */
  BURA_ENAN = -7,            /* non-finite residual                              */
  BURA_EBUSY = -8,           /* plan has queued or running asynchronous solves   */
  BURA_ETOOBIG = -9          /* bura_solve_static: the workspace does not fit
                                BURA_STATIC_SCRATCH_BYTES                        */
};

enum bura_precision {
  BURA_FP64 = 0,   /* FP64 multigrid-PCG throughout                                 */
  BURA_MIXED = 1   /* FP32 multigrid-PCG inner solves, FP64 residual refinement,
                      FP64 dot products and FP64 combine                           */
};

enum bura_schedule {
  BURA_BATCHED = 0,  /* all (pole, rhs) systems advance together, one launch per step */
  BURA_PER_POLE = 1  /* one pole after another (all rhs of that pole together)        */
};

/* Grid / operator description. */
typedef struct {
  int dim;                 /* 2 or 3                                                    */
  int n;                   /* interior points per axis, 1 <= n; n^dim <= 2^31 - 1.
                              Multigrid coarsens while n is odd (n = 2^L - 1 gives a
                              full hierarchy); otherwise the preconditioner is Jacobi. */
  const double* coeff;     /* NULL: Laplacian.  Else host array, (n+2)^dim nodal values
                              a > 0 incl. boundary, x fastest; copied at plan time.     */
  double lambda_upper;     /* 0: the library's bound (below).  >0: caller's bound, must
                              be >= the largest eigenvalue of A~.                       */
  int rhs_unscaled;        /* 0: f is the right-hand side of the scaled problem
                              A^alpha u = f, A = A~/Lambda (Section 1.4, eq. (10)).
                              1: f is f~ of the unscaled A~^alpha u = f~, and the
                              result is u = A~^-alpha f~ = Lambda^-alpha A^-alpha f~
                              (the factor is applied in the FP64 combine).  Needs a
                              plan that knows its fractional power: the plans of
                              _rational, _rational_multi and _slots return
                              BURA_EINVAL, as does any other value.  (0 keeps a
                              zero-initialised struct on the scaled problem.)       */
} bura_grid_t;

/* Solver options.  bura_opts_default fills sensible values. */
typedef struct {
  double tol;          /* per-system stop: ||f - (A - d_j I) x_j||_2 <= tol ||f||_2 (FP64) */
  double inner_tol;    /* MIXED: the largest relative reduction asked of one FP32 inner
                          solve.  A refinement step that can finish a system asks only for
                          what its tol still needs (half of tol / its current FP64 relative
                          residual, when that is larger than inner_tol)                   */
  int precision;       /* enum bura_precision                                            */
  int schedule;        /* enum bura_schedule                                             */
  int max_iter;        /* PCG iteration cap (per inner solve in MIXED mode); 0 = automatic
                          (200 with a multigrid hierarchy, 40 n + 200 without)           */
  int max_outer;       /* MIXED: refinement-step cap                                     */
  int nrhs_max;        /* largest nrhs any solve on this plan will use (sizes buffers)   */
  int check_every;     /* PCG iterations between host convergence checks (>= 1)          */
  int nu_pre, nu_post; /* Jacobi sweeps before / after coarse-grid correction             */
  double omega;        /* Jacobi damping of every sweep; 0 = library default: 4/5 (2D)
                          or 6/7 (3D), and for the FP32 inner solves of BURA_MIXED
                          per-sweep Chebyshev weights on [0.4, 2] (2D) or [0.5, 2]
                          (3D) for nu <= 2, on [0.3, 2] for nu = 3                     */
  void* stream;        /* hipStream_t used for every launch and copy; NULL = null stream */
  size_t hbm_budget;   /* 0 = unlimited; else plan creation fails with BURA_ENOMEM if its
                          device footprint would exceed this many bytes                 */
  int autotune;        /* 2D multigrid plans: 0 = default tile shapes; 1 = plan creation
                          times every tile-shape variant of the stencil product and of
                          each level's fused kernels on the plan's buffers (whole solves
                          in the plan's schedule) and keeps the fastest (cached per shape
                          in the process; see bura_plan_tiles)                           */
  double err_tol;      /* 0: stop on the residual test (tol) alone.  > 0 (BURA_MIXED, plans
                          without stages; else BURA_EUNSUPPORTED): also require the certified
                          bound of the report (err_bound) to be <= err_tol; the refinement
                          continues on the systems of every output over it (at most four
                          more rounds, else BURA_ENOCONV)                                */
  int variant;         /* 0: the default code path.  Else a bitwise OR of enum bura_variant:
                          alternative implementations of the same steps, which give the same
                          result to rounding (bitwise for the scalar and graph variants) and
                          are kept to cross-check the default path and to measure it against
                          them; any other bit: BURA_EINVAL                               */
} bura_opts_t;

/* Alternative code paths (bura_opts_t.variant). */
enum bura_variant {
  BURA_VARIANT_UNFUSED = 1,      /* 2D multigrid: one kernel per V-cycle step (sweep, residual
                                    and restriction, prolongation) instead of the two fused
                                    LDS-tiled level kernels                                 */
  BURA_VARIANT_NO_FOLDXR = 2,    /* PCG vector updates x += alpha p, r -= alpha q in a pass of
                                    their own instead of inside the stencil product and the
                                    first fine pre-smoothing kernel                          */
  BURA_VARIANT_FOLD_SCALARS = 4, /* the per-system scalar updates by the last block of the
                                    producing kernel (device-scope fence) instead of a small
                                    kernel of their own                                      */
  BURA_VARIANT_NO_GRAPH = 8      /* launch every PCG iteration eagerly instead of replaying a
                                    captured graph per chunk of iterations                   */
};

/* Per-solve report (host struct filled by solve/poll). */
#define BURA_MAX_TERMS 64
typedef struct {
  int status;                       /* status of the solve                              */
  int nterms;                       /* k+1                                              */
  double E;                         /* E_alpha(k,k;1) of the rational approximation      */
  int iters[BURA_MAX_TERMS];        /* total PCG iterations, max over rhs, per pole      */
  int outer[BURA_MAX_TERMS];        /* refinement steps (MIXED), max over rhs, per pole  */
  double relres[BURA_MAX_TERMS];    /* final FP64 relative residual, max over rhs       */
  double seconds;                   /* wall time of the solve on the host clock          */
  double err_bound;                 /* certified bound, max over outputs and rhs, of
                                       |u - u_r| / |u|: u as computed, u_r the exact
                                       sum_j c_j (A - d_j I)^-1 f of the same terms.  Each
                                       system's error is (A - d_j I)^-1 r_j, so |u - u_r| <=
                                       sum_j |c_j| |r_j| / (lam_lb - d_j), lam_lb a guaranteed
                                       lower bound of the spectrum of A (the Laplacian's
                                       smallest eigenvalue, times the smallest face
                                       coefficient for variable coefficients); FP64 plans use
                                       the PCG's recursively updated residual, BURA_MIXED the
                                       FP64 residual of the refinement.  -1 for plans with
                                       stages (sequential forms), where it is not formed.   */
} bura_report_t;

/* Fill *o with defaults: tol 1e-12, inner_tol 5e-6, BURA_MIXED, BURA_BATCHED,
 * max_iter 0 (automatic), max_outer 12, nrhs_max 1, check_every 4, V(2,2),
 * stream NULL, err_tol 0, variant 0. */
int bura_opts_default(bura_opts_t* o);

/* Step 1-2 of Section 2.2 on the host: the (k,k) best uniform rational
 * approximation of t^(1-alpha) on [0,1] (Definition 2.1) by a Remez exchange
 * (Section 3.2) in extended precision, and its partial fractions eq. (15).
 * Writes c[0..k], d[0..k] (d[0] = 0 > d[1] > ... > d[k]) and *E.
 * beta == 2: the (k+1,k) 2-BURA of t^(2-alpha) (Section 4.1) with
 * r(t)/t^2 = c_{0,2}/t^2 + c_{0,1}/t + sum_j c_j/(t - d_j) (eq. (22), (25)):
 * c[0] = c_{0,1}, c[1..k], and c[k+1] = c_{0,2} (= -E, eq. (23)), so c needs
 * k+2 doubles.  alpha in (0,1), beta 1 or 2 (else BURA_EUNSUPPORTED),
 * 1 <= k <= 16.  Returns BURA_EREMEZ if the exchange does not level.
 * Results are cached per (alpha, beta, k) for the life of the process. */
int bura_coefficients(double alpha, int beta, int k, double* c, double* d, double* E);

/* The zeros of the same (k,k) BURA r (Lemma 2.5: real, negative, interlacing
 * with the poles, 0 > zeta[0] > d_1 > zeta[1] > ... > zeta[k-1] > d_k) and the
 * leading constant *C with r(t) = C prod_j (t - zeta_j)/(t - d_j), for the
 * zero-pole product form of the remark in Section 2.2.  zeta has room for k
 * doubles.  Same arguments, errors and caching as bura_coefficients. */
int bura_zeros(double alpha, int beta, int k, double* zeta, double* C);

/* Create a plan: operator hierarchy, coefficients (via bura_coefficients) and
 * device workspace for up to opts->nrhs_max right-hand sides.  *out receives
 * the plan on success and NULL otherwise. */
int bura_plan_create(const bura_grid_t* grid, double alpha, int beta, int k,
                     const bura_opts_t* opts, bura_plan_t* out);
/* (beta == 2 runs k+2 systems: the k+1 of c_{0,1} A^-1 f + sum_j c_j (A - d_j)^-1 f
 * together, then A^-1 applied to the pole-0 solution for the c_{0,2} A^-2 f
 * term (eq. (25); Section 4.3's chained solve).  The negative c_{0,2} makes
 * the FP64 combine subtract large terms; errors grow like E kappa(A)^(beta-1)
 * (the corollary in Section 4.3).) */

/* Same engine for a caller-given partial-fraction form
 * u = sum_{j<nterms} w[j] (A + shift[j] I)^{-1} f, shift[j] >= 0, w[j] any sign
 * (e.g. the quadrature of Section 5.3's comparison method, or coefficients
 * computed elsewhere).  1 <= nterms <= BURA_MAX_TERMS. */
int bura_plan_create_rational(const bura_grid_t* grid, int nterms, const double* weights,
                              const double* shifts, const bura_opts_t* opts, bura_plan_t* out);

/* Several caller-given partial-fraction forms in one plan: output a uses the
 * nterms[a] consecutive terms that follow those of outputs 0..a-1 in
 * weights/shifts (sum_a nterms[a] <= BURA_MAX_TERMS).  All systems advance
 * together; bura_solve writes nout * nrhs vectors, output a of right-hand side
 * r at u_dev[a * nrhs + r]. */
int bura_plan_create_rational_multi(const bura_grid_t* grid, int nout, const int* nterms, const double* weights,
                                    const double* shifts, const bura_opts_t* opts, bura_plan_t* out);

/* The sinc quadrature of Bonito and Pasciak that Section 5.3 compares against:
 * for an SPD B,
 *   B^-alpha ~= (2 k' sin(pi alpha)/pi) sum_{l=-m}^{M} e^{2(alpha-1) l k'} (e^{-2 l k'} I + B)^-1,
 *   m = ceil(pi^2/(4 alpha k'^2)), M = ceil(pi^2/(4 (1-alpha) k'^2)),
 * with step k' > 0 (Section 5.3 parametrises it by k_Q = pi^2/(4 alpha (1-alpha) k'^2)).
 * Values of the two ceiling arguments within 1e-9 (relative) of an integer are
 * taken as that integer.  The rule is applied to B = scale * A and returned as
 * weights/shifts for A that approximate A^-alpha itself:
 *   weights[l+m] = scale^(alpha-1) (2k' sin(pi alpha)/pi) e^{2(alpha-1) l k'},
 *   shifts[l+m]  = e^{-2 l k'} / scale,   l = -m..M (shifts decreasing).
 * *nterms receives m+M+1 even when it exceeds max_terms (then BURA_EINVAL and
 * nothing is written).  Host-only; alpha in (0,1), k' > 0, scale > 0. */
int bura_sinc_coefficients(double alpha, double kprime, double scale, int max_terms, double* weights,
                           double* shifts, int* nterms);

/* The step k' of the sinc quadrature for Section 5.3's parameter k_Q =
 * pi^2/(4 alpha (1-alpha) k'^2) (the nominal number of its systems):
 * *kprime = pi/(2 sqrt(alpha (1-alpha) k_Q)).  alpha in (0,1), k_Q > 0. */
int bura_sinc_kprime(double alpha, double kq, double* kprime);

/* A plan for the sinc quadrature, one output per (alphas[a], kprimes[a]).
 * As in Section 5.3's comparison the rule is applied to the unscaled operator
 * Lambda * A (scale = the plan's spectral bound Lambda, see bura_plan_info), and
 * the result is multiplied by Lambda^alpha, so that output a approximates the
 * same A^-alpha f as a BURA plan.  Total terms <= BURA_MAX_TERMS; E is 0. */
int bura_plan_create_sinc(const bura_grid_t* grid, int nalpha, const double* alphas, const double* kprimes,
                          const bura_opts_t* opts, bura_plan_t* out);

/* Multi-step BURA (Section 4.4): A^-alpha f for alpha = sum_i alphas[i] as
 * nsteps 1-BURA steps applied in order, u_i = r_{alphas[i]}(A) A^-1 u_{i-1},
 * u_0 = f, each with ks[i] + 1 shifted systems (sum <= BURA_MAX_TERMS).  The
 * steps run one after the other (each step's systems in one batch); the plan
 * holds one extra nrhs_max x N FP64 buffer between steps.  bura_solve writes
 * u_n; the report's E is the largest E_{alphas[i]}(ks[i],ks[i];1) (the error
 * of the composition depends on the condition number, eq. (29)). */
int bura_plan_create_multistep(const bura_grid_t* grid, int nsteps, const double* alphas, const int* ks,
                               const bura_opts_t* opts, bura_plan_t* out);

/* The zero-pole product form of the remark in Section 2.2:
 * u = C prod_{j=1..k} (A - zeta_j I)(A - d_j I)^-1 A^-1 f, evaluated as k+1
 * sequential solves, v_0 = A^-1 f, v_j = v_{j-1} + (d_j - zeta_j)(A - d_j I)^-1 v_{j-1},
 * u = C v_k (zeros and C from bura_zeros).  Same result as bura_plan_create
 * up to rounding; the systems cannot run concurrently (only the right-hand
 * sides of a batch do).  Extra nrhs_max x N FP64 buffer as for multistep. */
int bura_plan_create_product(const bura_grid_t* grid, double alpha, int beta, int k, const bura_opts_t* opts,
                             bura_plan_t* out);

/* Several fractional powers of the same operator in one plan: alpha[a] with
 * ks[a] poles each (a < nalpha, sum_a (ks[a]+1) <= BURA_MAX_TERMS).  All
 * shifted systems of all outputs advance together; bura_solve then writes
 * nalpha * nrhs vectors, output a of right-hand side r at u_dev[a * nrhs + r].
 * bura_plan_coeffs returns the terms of all outputs back to back and the
 * largest E. */
int bura_plan_create_multi(const bura_grid_t* grid, int nalpha, const double* alphas, int beta, const int* ks,
                           const bura_opts_t* opts, bura_plan_t* out);

/* A plan whose partial-fraction terms come with each solve (eq. (16) with
 * per-right-hand-side weights and shifts): right-hand side r of a solve is
 * mapped to u_r = sum_{j < nterms[r]} w_rj (A + s_rj I)^{-1} f_r, so requests
 * for different fractional powers, numbers of poles or tolerances on one grid
 * share one batched solve.  The plan holds max_terms * nrhs_max systems
 * (max_terms <= BURA_MAX_TERMS); a system slot that a solve leaves unused
 * costs one early exit per launch.  Only BURA_BATCHED (else
 * BURA_EUNSUPPORTED).  bura_solve / bura_submit on such a plan return
 * BURA_EINVAL; bura_plan_coeffs returns max_terms zero placeholders. */
int bura_plan_create_slots(const bura_grid_t* grid, int max_terms, const bura_opts_t* opts, bura_plan_t* out);

/* Solve on a slot plan.  f_dev, u_dev: [nrhs][N] FP64 device buffers (caller
 * owned), nrhs <= nrhs_max.  Host arrays: nterms[nrhs] (1..max_terms),
 * weights and shifts [nrhs][max_terms] (row r, entries j < nterms[r] used;
 * weights finite, shifts >= 0 and finite), tol[nrhs] the FP64 relative
 * residual tolerance of each rhs (NULL: opts.tol for all).  The report's
 * per-term entries are maxima over the rhs that use the term; its E is 0.
 * Synchronous like bura_solve; BURA_EINVAL on a plan not made by
 * bura_plan_create_slots or on invalid terms. */
int bura_solve_slots(bura_plan_t plan, const double* f_dev, double* u_dev, int nrhs, const int* nterms,
                     const double* weights, const double* shifts, const double* tol, bura_report_t* rep);

/* Asynchronous bura_solve_slots: queued like bura_submit (the host arrays are
 * copied before it returns); *ticket identifies it for bura_poll/bura_wait. */
int bura_submit_slots(bura_plan_t plan, const double* f_dev, double* u_dev, int nrhs, const int* nterms,
                      const double* weights, const double* shifts, const double* tol, bura_ticket_t* ticket);

/* Number of outputs and their term ranges: output i uses terms
 * [term_begin[i], term_begin[i+1]); term_begin has nout + 1 entries. */
int bura_plan_outputs(bura_plan_t plan, int* nout, int* term_begin);

/* u_dev[r] = sum_j c_j (A - d_j I)^{-1} f_dev[r], r < nrhs <= nrhs_max.
 * Synchronous: returns after the result is in u_dev.  rep may be NULL.
 * BURA_ENOCONV leaves the last iterate combined in u_dev. */
int bura_solve(bura_plan_t plan, const double* f_dev, double* u_dev, int nrhs, bura_report_t* rep);

/* Asynchronous variant of bura_solve: queue the solve and return at once with
 * *ticket set.  tol > 0 replaces opts.tol (the per-system FP64 relative
 * residual) for this solve only; 0 keeps opts.tol.  Any number of solves may
 * be queued on one plan: a worker thread of the plan runs them one after
 * another in submission order (they share the plan's buffers), and a
 * synchronous bura_solve on the same plan waits for the running one.
 * f_dev/u_dev of each solve must stay valid and untouched until its ticket
 * completes; solves whose u_dev overlap complete in submission order.
 * BURA_EINVAL for a slot plan, nrhs outside [1, nrhs_max], tol < 0 or a null
 * pointer (then *ticket = 0). */
int bura_submit(bura_plan_t plan, const double* f_dev, double* u_dev, int nrhs, double tol, bura_ticket_t* ticket);

/* BURA_PENDING while the ticket's solve is queued or running; then its final
 * status, with the report copied to *rep (may be NULL), and the ticket is
 * released (a second poll returns BURA_EINVAL, as does an unknown ticket).
 * Thread-safe. */
int bura_poll(bura_ticket_t ticket, bura_report_t* rep);

/* Blocking bura_poll: returns once the ticket's solve has finished. */
int bura_wait(bura_ticket_t ticket, bura_report_t* rep);

/* Introspection: the plan's c_j, d_j (arrays of nterms) and E (may be NULL). */
int bura_plan_coeffs(bura_plan_t plan, int* nterms, double* c, double* d, double* E);

/* Lambda used for the scaling A = A~/Lambda, and the number of multigrid levels. */
int bura_plan_info(bura_plan_t plan, double* lambda, int* nlevels, size_t* device_bytes);

/* y_dev = (A + shift I) x_dev in FP64 for nvec vectors (operator check). */
int bura_plan_apply(bura_plan_t plan, double shift, const double* x_dev, double* y_dev, int nvec);

/* Tile-shape variants of the 2D stencil product and fused multigrid level
 * kernels (an implementation choice, not part of the method).  Every variant
 * computes the same value at every grid point up to rounding (the grouping of
 * the per-block partial sums of the PCG dot products differs, and variant 3
 * of the down kernel sums the full weighting in another order), so results
 * of two variants agree to rounding, not bit for bit.  Variants 3 and 4
 * walk whole grid rows, in segments of 128 and of 32 fine rows per
 * workgroup (levels of up to 1023 points per axis; a larger level runs
 * variant 0). */
#define BURA_TILE_VARIANTS 5

/* The variants a 2D plan launches: out[0] for the stencil product, out[1 + 2l]
 * and out[2 + 2l] for the fused down and up kernels of level l, for each of
 * the plan's levels with fused kernels; *len = 1 + 2 * (those levels) (0 for
 * a 3D plan, whose kernels have one shape).  With out == NULL only *len is
 * written.  BURA_EINVAL if max_len < *len.  Untuned, with nsys the systems
 * that share a launch (all of them; one pole's right-hand sides in the
 * per-pole schedule; the largest stage of a sequential form): a kernel of a
 * level of 255 to 1023 points per axis takes variant 3 (whole rows) when
 * nsys times its row segments per system is at least 1024 (segments of 128
 * fine rows for the stencil product and the up kernel, of 64 coarse rows for
 * the down kernel); otherwise every entry is 0 except the down kernel of a
 * level whose default tile (64 x 6 coarse points) would give one launch fewer
 * than 1024 workgroups: that level takes variant 1 (32 x 8). */
int bura_plan_tiles(bura_plan_t plan, int* out, int max_len, int* len);

/* Set the variants (layout as bura_plan_tiles, len must equal its *len, each
 * value in [0, BURA_TILE_VARIANTS)).  Synchronises the plan's stream and
 * drops its captured graphs; BURA_EBUSY while asynchronous solves are queued
 * or running. */
int bura_plan_set_tiles(bura_plan_t plan, const int* v, int len);

/* Kernel classes for profiling. */
enum bura_kernel_class {
  BURA_K_SMOOTH_FINE = 0,    /* Jacobi sweeps on the finest level (or the Jacobi preconditioner) */
  BURA_K_SMOOTH_COARSE = 1,  /* Jacobi sweeps (or fused level kernels) on coarser global levels   */
  BURA_K_RESTRICT = 2,       /* residual + full-weighting restriction                             */
  BURA_K_PROLONG = 3,        /* interpolation + correction                                        */
  BURA_K_COARSE_LDS = 4,     /* coarse levels solved inside one workgroup per system              */
  BURA_K_SPMV = 5,           /* q = (A + s) p with p.q                                             */
  BURA_K_UPDATE_XR = 6,      /* x += a p, r -= a q with r.r                                        */
  BURA_K_UPDATE_P = 7,       /* p = z + b p                                                        */
  BURA_K_RESIDUAL64 = 8,     /* FP64 refinement residual                                           */
  BURA_K_COMBINE = 9,        /* u = sum_j c_j x_j                                                  */
  BURA_K_OTHER = 10,         /* per-system scalar updates, copies                                  */
  BURA_K_DOWN_FINE = 11,     /* finest level, fused, with the PCG residual update r -= alpha q:
                                sweeps from zero + residual + restriction                          */
  BURA_K_UP_FINE = 12,       /* finest level, fused: prolongation + sweeps + r.z                  */
  BURA_K_DOWN_FINE_PLAIN = 13, /* finest level, fused, without the residual update (the first
                                preconditioner application of each PCG solve)                    */
  BURA_K_SMOOTH_FINE_RUP = 14, /* first fine-level sweep with the PCG residual update (3D)         */
  BURA_K_COUNT = 15
};

/* Profiling of the plan's launches (for measurement, not for production use).
 * enable != 0 resets the statistics and starts counting, per block, the
 * algorithmic bytes each launch moves (each vector element read or written
 * once; blocks of systems that have already converged count zero).  Launches
 * are bracketed by a pair of HIP events on the plan's stream: all classes when
 * enable == 1, else the classes whose bit (1 << (class + 1)) is set in enable.
 * enable = 0 stops recording. */
int bura_plan_profile(bura_plan_t plan, int enable);

/* Launch count, summed event time (ms) and algorithmic bytes of one kernel
 * class since profiling was enabled.  Synchronises the plan's stream. */
int bura_plan_kernel_stats(bura_plan_t plan, int kclass, long long* launches, double* total_ms,
                           double* alg_bytes);

/* Measurement utility (not part of the method): copy `bytes` bytes from
 * src_dev to dst_dev on `stream` (NULL: the null stream) with the library's
 * plain streaming kernel (16-byte loads and stores, one pass), so that HBM
 * counters can be calibrated on a kernel of known traffic.  Both pointers
 * must be 16-byte aligned and the buffers must not overlap.  Asynchronous. */
int bura_device_copy(void* dst_dev, const void* src_dev, size_t bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Request server (continuous batching on one GPU).
 *
 * Requests for the constant-coefficient grids are queued by bura_server_submit
 * (which computes the request's BURA terms, cached per (alpha, k), and fails
 * with that status if they cannot be computed).  A dispatcher thread assigns
 * each request to the resident slot plan (bura_plan_create_slots) of its key:
 * grid, precision and a class of term counts (13 or 17 term slots per
 * right-hand side, the smaller holding k+1), creating the plan if needed.
 * Each plan has max_group right-hand-side slots and a worker thread.  With
 * BURA_MIXED the worker admits queued requests into free slots of the solve
 * that is running, at every outer refinement-step boundary, advances all
 * admitted requests one outer step at a time, and returns each result as
 * soon as that request's own systems have finished -- requests join and
 * leave a running solve.  With BURA_FP64 each solve takes up to max_group
 * queued requests of its key.  Up to max_concurrent plans have work at once,
 * each on its own stream.  New plans are admitted against hbm_budget bytes
 * (0 = unlimited), evicting idle plans least recently used first; a request
 * whose plan can never fit fails with BURA_ENOMEM.  A request's result does
 * not depend on which other requests share its plan or when they arrive.
 * f_dev / u_dev are FP64 device vectors of n^dim values; f_dev must be fully
 * written (its stream synchronised) before submit, and both must stay valid
 * until the ticket completes.  All server functions are thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct bura_server_s* bura_server_t;

typedef struct {
  int dim, n;        /* grid (Laplacian, scaled as above)                    */
  double alpha;      /* 0 < alpha < 1                                        */
  int k;             /* poles: k+1 shifted systems, 1 <= k <= 16             */
  double tol;        /* FP64 relative residual per shifted system            */
  int precision;     /* enum bura_precision                                  */
} bura_request_t;

typedef struct {
  long long submitted, completed, failed, batches, plans_created, plans_evicted;
  double unknown_pole_solves;   /* sum over successful requests of n^dim (k+1)   */
  double p50_latency_s, p99_latency_s;   /* submit -> result, completed requests */
  double mean_batch;            /* requests per solve step (mixed precision: per outer
                                   refinement step of a running solve; FP64: per solve) */
  size_t resident_bytes;        /* device bytes of resident plans                */
  long long joined_running;     /* requests admitted into a solve already running     */
} bura_server_stats_t;

int bura_server_create(size_t hbm_budget, int max_concurrent, int max_group, bura_server_t* out);
/* Queue a request; *ticket identifies it.  Returns at once. */
int bura_server_submit(bura_server_t s, const bura_request_t* req, const double* f_dev, double* u_dev,
                       uint64_t* ticket);
/* BURA_PENDING while queued or running; then the request's status (the ticket
 * is released) with its report in *rep (may be NULL). */
int bura_server_poll(bura_server_t s, uint64_t ticket, bura_report_t* rep);
/* Blocking variant of bura_server_poll. */
int bura_server_wait(bura_server_t s, uint64_t ticket, bura_report_t* rep);
int bura_server_stats(bura_server_t s, bura_server_stats_t* st);

/* Forget the latency samples collected so far (the counters stay cumulative),
 * e.g. after a warm-up pass that created the plans. */
int bura_server_reset_latency(bura_server_t s);
/* Waits for queued and running requests, then frees every plan. */
void bura_server_destroy(bura_server_t s);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code running between its
 * own allocation-free phases (a serving loop with a fixed memory pool), a
 * harness that forbids hipMalloc, work launched on a stream the caller may
 * later capture.  The same result as bura_plan_create_rational(grid, nterms,
 * weights, shifts, opts) followed by bura_solve(f_dev, u_dev, nrhs) and
 * bura_plan_destroy, but every device buffer of that plan (iterates,
 * multigrid levels, face weights, partial sums, per-system state) is carved
 * from one static device array of BURA_STATIC_SCRATCH_BYTES per GPU, held by
 * the library until the process ends.  No hipMalloc, hipFree, pinned-host
 * allocation, stream, event or graph is created; the launches and copies run
 * in order on opts->stream (NULL: the null stream) and the call returns when
 * u_dev holds the result.  Host-side bookkeeping uses ordinary host memory.
 *
 * f_dev, u_dev: [nrhs][N] FP64 device buffers (caller owned), nrhs <=
 * opts->nrhs_max.  opts->autotune must be 0 (BURA_EINVAL otherwise).  A
 * problem whose workspace exceeds the array (e.g. FP64, 2D 255^2, one
 * right-hand side and more than about 15 terms; 1023^2 at any size) returns
 * BURA_ETOOBIG before the solve starts.  Every
 * call on one GPU uses that GPU's single array and leaves its contents
 * behind (each call clears what must start at zero): calls that overlap on
 * one GPU, from several threads or streams, race and must be serialised by
 * the caller. */
#define BURA_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int bura_solve_static(const bura_grid_t* grid, int nterms, const double* weights, const double* shifts,
                      const bura_opts_t* opts, const double* f_dev, double* u_dev, int nrhs, bura_report_t* rep);

/* Release every resource of the plan.  Runs every queued asynchronous solve to
 * completion first (their tickets stay pollable). */
void bura_plan_destroy(bura_plan_t plan);

/* Static string for a status code. */
const char* bura_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* BURA_H */
