/*
 * rpf.h -- C ABI of the reduced-space power-flow derivative library for
 * AMD MI355X (gfx950), FP64 throughout.
 *
 * The library computes the quantities of the feasible reduced-space method
 * for optimal power flow (Pacaud et al., "A Feasible Reduced Space Method
 * for Real-Time Optimal Power Flow"):
 *
 *   rpf_pf_solve               Newton-Raphson power flow g(x, u) = 0
 *                              (Section III-A, eq. projection:newtonraphson;
 *                              stopping rule ||g||_2 < tol of Section V-A.1)
 *   rpf_al_objective           scaled augmented-Lagrangian value and the
 *                              operational constraints c (Section IV-A.1,
 *                              IV-A.2; c = (h, r) of eq. acopf_controlstate)
 *   rpf_reduced_gradient       reduced gradient by the adjoint method
 *                              (Proposition 1, eq. reduced_gradient)
 *   rpf_reduced_hessian_batch  reduced Hessian-vector products by the
 *                              adjoint-adjoint method (Proposition 2,
 *                              eq. hessvecprod, eq. socadjoint)
 *   rpf_reduced_hessian        the dense reduced Hessian, n_u products in
 *                              batches (Section III-C, reduced Hessian)
 *   rpf_factor_solve           Cholesky of the symmetrised, shifted reduced
 *                              Hessian and the resulting step (Section IV-B.2,
 *                              Proposition 3 and the inertia-control remark)
 *   rpf_qp_step                exact real-time step: the bounded QP of eq.
 *                              qp_rto by an interior-point method whose Newton
 *                              systems go through the Schur complement of
 *                              Proposition 3 (Section IV-B.2, IV-C)
 *   rpf_track_step_qp          one real-time tracking update with that step
 *   rpf_static_opf             static OPF by the augmented-Lagrangian method
 *                              (Section IV-B.3, tolerances of Section V-B)
 *
 * Variables and orderings (Section II-B, eq. statecontrol):
 *   u = (v_ref, v_pv, p_pv)            n_u = 1 + 2 n_pv
 *   x = (theta_pv, theta_pq, v_pq)     n_x = n_pv + 2 n_pq
 *   g rows = (P balance at PV, P balance at PQ, Q balance at PQ)
 * Buses within each group in ascending bus id; theta_ref = 0.
 *   c = (|S_f|^2 per branch, |S_t|^2 per branch, v_pq, p^g_ref,
 *        q^net_ref, q^net_pv)          m = 2 n_l + n_pq + n_pv + 2
 * with S_f, S_t the complex flows at the from/to ends (pi model, no taps),
 * p^g_ref = P_ref + p^d_ref, q^net_i = Q_i + q^d_i.  The cost is
 * f = sum_g c2 (B p_g)^2 + c1 (B p_g) + c0, B = base_mva, over all
 * generators (the slack's p_g is p^g_ref).  The AL value is
 *   phi = sigma_f f + y^T D_c (c - s) + rho/2 ||D_c (c - s)||^2,
 * D_c = diag(sigma_c).
 *
 * Conventions for every call:
 *  - Pointers marked "device" are device memory on the current HIP device;
 *    "host" pointers are read during the call only.  The caller owns all
 *    buffers it passes; the handle owns its internal workspace.
 *  - Compute calls enqueue work on `stream` and return without waiting;
 *    none of them synchronises the host or allocates, so a sequence of them
 *    can be captured into a HIP graph (rpf_profile_* timing is for eager
 *    calls only).
 *  - Dense matrices are row-major.  A batch of vectors is an [n x nbatch]
 *    row-major block with leading dimension ld >= nbatch (element (i, k) at
 *    i * ld + k).
 *  - Return value: 0 on success, a negative RPF_E* code otherwise, with a
 *    message from rpf_last_error().  Numerical outcomes (power flow not
 *    converged, tiny pivot of J_x, Cholesky failure) are reported in device
 *    status words, never as return codes.
 *  - Tiny pivot word (static pivoting, Section V-A.1): the refactorization
 *    of J_x keeps the pivots the host ordering fixed.  A sparse pivot with
 *    |u_ii| <= 1e-14 max_j |a_ij| (row i before elimination), or a zero or
 *    non-finite pivot of the dense top block, is reported as the 1-based
 *    index in x of a failing pivot (0 = all pivots passed); the solves with
 *    such a factor are not meaningful.
 *  - A handle is not thread-safe; use one handle per host thread / stream.
 *  - Tracing: with the environment variable RPF_TRACE set (not empty, not
 *    "0") when a handle is created, each compute call on it records two
 *    events on `stream` and, once they have completed, writes one line
 *    {"rpf_trace": "<call>", "ms": <device time>, "arg": <size argument>}
 *    to stderr -- polled at later calls on the handle, waited for when it is
 *    destroyed.  Calls on a stream that is capturing a graph are not traced.
 *  - Launch-shape switches, read when a handle is created: RPF_HVP_STREAMS
 *    (see rpf_reduced_hessian), RPF_PACK_TW = 8 | 16 and RPF_PACK_SV = 0 | 1
 *    (column tile of the batched pack solves, factor values staged in LDS),
 *    RPF_PACK_THREADS = 512 (512-thread workgroups for 16-column tiles: two
 *    per CU when packs are at most 512 rows), RPF_SUBTREE_MAX and
 *    RPF_TAIL_MAX (presolve: largest pack, largest dense tail).  Results
 *    agree to rounding across them.
 */
#ifndef RPF_H
#define RPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* rpf_stream_t; /* hipStream_t; NULL = default stream */

enum {
  RPF_OK = 0,
  RPF_EINVAL = -1, /* bad argument (null pointer, size out of range, bad grid) */
  RPF_ENOMEM = -2, /* device allocation failed */
  RPF_EHIP = -3,   /* a HIP runtime call failed */
  RPF_ESTATE = -4, /* call order: e.g. Hessian products before rpf_reduced_gradient */
  RPF_ESIZE = -5   /* nbatch above the max_batch given at creation */
};

typedef struct rpf_grid rpf_grid;

/* Grid description (host pointers, copied by rpf_grid_create).
 * bus_type: 0 = PQ, 1 = PV, 2 = REF (exactly one REF).  Branches are pi
 * models with series impedance br_r + j br_x and total line charging br_b
 * (half at each end), all per unit; no parallel branches.  gen_bus: one
 * generator at each PV and REF bus and none elsewhere.  Costs c2, c1, c0
 * apply to the generator's active output in MW (per-unit times base_mva). */
typedef struct {
  int32_t nb, nl, ng;
  double base_mva;
  const int32_t* bus_type; /* [nb] */
  const int32_t* br_from;  /* [nl] */
  const int32_t* br_to;    /* [nl] */
  const double* br_r;      /* [nl] */
  const double* br_x;      /* [nl] */
  const double* br_b;      /* [nl] */
  const int32_t* gen_bus;  /* [ng] */
  const double* c2;        /* [ng] */
  const double* c1;        /* [ng] */
  const double* c0;        /* [ng] */
} rpf_grid_desc;

/* Host presolve (index maps, fill-reducing ordering, symbolic LU of J_x,
 * level schedules, gather lists) and device allocations for batches of up
 * to max_batch Hessian-vector products.  Uses the current HIP device.
 * Static pivoting: the diagonal pairs P_i/theta_i, Q_i/v_i are the pivots
 * (Section V-A.1: symbolic factorization once, numeric refactorization on
 * the device).  On failure *out is NULL. */
int rpf_grid_create(const rpf_grid_desc* desc, int32_t max_batch, rpf_grid** out);
void rpf_grid_destroy(rpf_grid* grid);

/* Sizes n_x, n_u, m (eq. statecontrol, eq. acopf_controlstate). Host ints. */
int rpf_dims(const rpf_grid* grid, int32_t* nx, int32_t* nu, int32_t* m);

/* Structure figures of the presolve (host int64 [10]): nnz(J_x), nnz(L+U),
 * forward levels, backward levels, longest LU row, refactorization
 * updates, nnz(J_u), nnz(K), nnz(rank-one rows), max_batch. */
int rpf_structure(const rpf_grid* grid, int64_t* out10);

/* Newton-Raphson power flow at fixed control u and loads (Section III-A):
 * x_{k+1} = x_k - (grad_x g_k)^{-1} g_k, stopped when ||g||_2 < tol, when
 * the residual is not finite, or after max_iter steps.
 *   u [n_u], pd [nb], qd [nb]: device, read only.
 *   x [n_x]: device, in: starting point, out: last iterate.
 *   max_iter: 0 .. 100.
 *   status [3]: device int32, out: {Newton steps taken, converged (0/1),
 *   tiny pivot word of the factorizations of this call}.
 *   resid [1]: device, out: ||g(x, u)||_2 at the returned x.
 * The loop runs on the device: max_iter predicated Newton steps are
 * enqueued, and once the test is met every later kernel of the loop returns
 * at once, so the call never waits for the device.  Leaves J_x of the last
 * step factorized in the handle. */
int rpf_pf_solve(rpf_grid* grid, const double* u, const double* pd, const double* qd, double* x,
                 double tol, int32_t max_iter, int32_t* status, double* resid, rpf_stream_t stream);

/* AL value and constraints at (x, u) (Section IV-A).
 *   x [n_x], u [n_u], pd/qd [nb], s/y [m], sigma [1 + m] = (sigma_f,
 *   sigma_c): device, read only.
 *   phi [1], c [m]: device, out.  c may be NULL. */
int rpf_al_objective(rpf_grid* grid, const double* x, const double* u, const double* pd,
                     const double* qd, const double* s, const double* y, double rho,
                     const double* sigma, double* phi, double* c, rpf_stream_t stream);

/* Reduced gradient of phi (Proposition 1 applied to the AL function):
 * solves (grad_x g)^T lambda = -(d_x phi)^T with the LU of J_x refactorized
 * at x, then grad = d_u phi + lambda^T grad_u g.
 *   inputs as rpf_al_objective (device).
 *   grad [n_u], lambda [n_x] (x order): device, out.  lambda may be NULL.
 *   info [1]: device int32, out, may be NULL: tiny pivot word of J_x's
 *   factorization at x (nonzero: grad, lambda and the cached point are not
 *   meaningful).
 * Caches the point (factorized J_x, J_u, the Lagrangian Hessian of
 * l = phi + lambda^T g, rank-one constraint terms) for the Hessian calls. */
int rpf_reduced_gradient(rpf_grid* grid, const double* x, const double* u, const double* pd,
                         const double* qd, const double* s, const double* y, double rho,
                         const double* sigma, double* grad, double* lambda, int32_t* info,
                         rpf_stream_t stream);

/* Reduced Hessian-vector products at the cached point (Proposition 2):
 * for each column w of V: J_x z = -J_u w; J_x^T psi = -(K_xu w + K_xx z);
 * H w = K_uu w + K_ux z + J_u^T psi, with K the Hessian of
 * l = phi + lambda^T g in (x, u).
 *   V: device [n_u x nbatch], leading dimension ldv, read only.
 *   HV: device [n_u x nbatch], leading dimension ldhv, out.
 *   1 <= nbatch <= max_batch.  RPF_ESTATE before rpf_reduced_gradient. */
int rpf_reduced_hessian_batch(rpf_grid* grid, const double* V, int32_t nbatch, int32_t ldv,
                              double* HV, int32_t ldhv, rpf_stream_t stream);

/* The dense reduced Hessian H [n_u x n_u] (device, row-major, out) at the
 * cached point: products with the identity in batches of `batch` columns
 * (0 = the library's choice, at most max_batch).  The batches run one after
 * the other on `stream`.  With RPF_HVP_STREAMS = 2 .. 8 (read when the handle
 * is created) they run concurrently on that many streams owned by the
 * handle, each with its own workspace, forked from `stream` and joined back
 * to it by events (same results, bit for bit); while `stream` is being
 * captured into a graph they run on `stream` alone. */
int rpf_reduced_hessian(rpf_grid* grid, double* H, int32_t batch, rpf_stream_t stream);

/* The dense reduced Hessian H [n_u x n_u] and/or the reduced Jacobian of the
 * constraints J = grad_u c(x(u), u) = (d_x c) Z + d_u c [m x n_u] (Section
 * III-C, reduced Jacobian; Z = -J_x^{-1} J_u) at the cached point, both
 * row-major on the device (out), either may be NULL (not both).  J comes
 * from the same batches of directions V = I as H, with no extra sparse
 * solves; with H NULL only the first solve of each batch runs.  Batching,
 * streams and capture behaviour as rpf_reduced_hessian. */
int rpf_reduced_derivatives(rpf_grid* grid, double* H, double* J, int32_t batch, rpf_stream_t stream);

/* Dense step (Section IV-B.2): K = (H + H^T)/2 + diag(d) + delta I is
 * factorized as L L^T (Cholesky), then step = -K^{-1} rhs.
 *   n: order; Kmat [n x n]: device, in: H, out: L in the lower triangle
 *   (upper triangle left as K).  diag [n] or NULL, rhs [n]: device, read.
 *   step [n]: device, out (left unchanged when info != 0).
 *   info [1]: device int32, out: 0, or the 1-based column whose pivot was
 *   not positive, or -1 when a workgroup of the triangular solves gave up
 *   waiting for another block (the solves are spread over one workgroup per
 *   block of 64 rows that wait for each other with a bounded spin; -1 is
 *   not expected on an idle or shared device and marks step as invalid). */
int rpf_factor_solve(rpf_grid* grid, int32_t n, double* Kmat, const double* diag, double delta,
                     const double* rhs, double* step, int32_t* info, rpf_stream_t stream);

/* rpf_factor_solve without a handle and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * kernels and results as rpf_factor_solve (bit for bit), for
 * 1 <= n <= RPF_NOALLOC_MAX_N; larger n returns RPF_ESIZE.  Its scratch
 * (about 4.2 MB: inverses of the factor's diagonal blocks, the forward
 * solve vector, block flags) is a static device array, one per GPU, held
 * until the process ends; the flags are cleared by a kernel at every call.
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (concurrent streams or host threads) race and must be serialised by the
 * caller. */
#define RPF_NOALLOC_MAX_N 4096
int rpf_factor_solve_noalloc(int32_t n, double* Kmat, const double* diag, double delta, const double* rhs,
                             double* step, int32_t* info, rpf_stream_t stream);

/* One real-time tracking update at new loads (Section IV-C, steps 1-3),
 * entirely on the device with no host synchronisation (capturable in a HIP
 * graph).  The bounded QP of step 2 is replaced by one shifted Newton step:
 *   loads pd = pd0 * load_factor, qd = qd0 * load_factor (per bus);
 *   power flow at u from x (pf_iters predicated Newton steps, tol);
 *   s = clip(c + y / (rho sigma_c), s_lo, s_hi) (minimiser of the scaled
 *   AL in s); reduced gradient and Hessian at (u, s, y);
 *   d = -((H + H^T)/2 + delta I)^{-1} grad (d = 0 if the Cholesky fails);
 *   u <- clip(u + d / 2^k, u_lo, u_hi) for the first k <= max_halvings whose
 *   power flow converges (u unchanged if none);
 *   s = clip(c(u) + y / (rho sigma_c), s_lo, s_hi), y <- y + rho D_c (c - s).
 * u [n_u], x [n_x], y [m]: device, in/out.  pd0, qd0, load_factor [nb],
 * s_lo, s_hi [m], u_lo, u_hi [n_u], sigma [1 + m]: device, read.
 * status [5]: device int32 out {first power flow converged, accepted
 * halving k (-1: none), Cholesky info, Newton steps of the first power
 * flow, tiny pivot word of the factorization behind the gradient and
 * Hessian}.  Uses the handle's workspace (one step at a time per handle). */
int rpf_track_step(rpf_grid* grid, double* u, double* x, double* y, const double* pd0, const double* qd0,
                   const double* load_factor, const double* s_lo, const double* s_hi, const double* u_lo,
                   const double* u_hi, double rho, const double* sigma, double delta, int32_t pf_iters,
                   int32_t max_halvings, double tol, int32_t* status, rpf_stream_t stream);

/* Exact real-time step (Section IV-C, step 2): the bounded QP of eq.
 * (qp_rto) in w = (u, s) at the point (x, u, s, y),
 *   min_d g^T d + 1/2 d^T Hw d  subject to  w_lo - w <= d <= w_hi - w,
 *   g  = (grad_u phi, -D_c (y + rho D_c (c - s))),
 *   Hw = [[H + delta I, -rho J^T D_c^2], [-rho D_c^2 J, rho D_c^2]]
 * (eq. gradient_auglag, eq. hessian_auglag with the scaling of Section
 * IV-A.2; H the symmetrised reduced Hessian of phi at fixed s, J = grad_u c
 * the reduced Jacobian).  The call first does what rpf_reduced_gradient
 * does at (x, u, s, y), then forms H and J from the same identity batches
 * (rpf_reduced_derivatives), then runs max_iter predicated iterations of a
 * primal-dual interior-point method with Mehrotra's predictor-corrector
 * (Section IV-B.1/2, eq. ipm_kkt_reduced) in max_iter slots: start d = clip(0, lo + k, hi - k)
 * with k = 1e-2 (hi - lo), duals 1 / slack, steps stopped 0.995 of the way
 * to the boundary; it stops once the scaled KKT error max(max|Hw d + g - z_l
 * + z_u| / (1 + max|g|), max complementarity product) is below tol.  Each
 * Newton system is solved through the Schur complement of Proposition 3
 * (eq. schur_matrix): S = H_gn + Sigma_u + delta I, where H_gn is the
 * reduced Hessian with each constraint's curvature weight rho sigma_k^2
 * replaced by rho sigma_k^2 Sigma_s,k / (Sigma_s,k + rho sigma_k^2), formed
 * by the batched Hessian-vector products, then its Cholesky factor.
 * Inertia control (Section IV-B.2): the Cholesky runs on S + w I, w = 0
 * first (or max(w0, w_last / 4) after a regularised iteration), raised to
 * w0 = 1e-4 max(1, max|diag H|) and then 8 times per failed attempt, each
 * attempt one of the max_iter slots; past w = 1e30 the call gives up.
 *   x [n_x], u [n_u], pd/qd [nb], s/y [m], sigma [1 + m]: device, read.
 *   u_lo, u_hi [n_u], s_lo, s_hi [m]: device, read (lo < hi).
 *   batch: width of the Hessian batches (0 = the handle's).
 *   H [n_u x n_u] (may be NULL: handle buffer), J [m x n_u]: device, out.
 *   grad [n_u] (may be NULL): device, out: the reduced gradient.
 *   dw [n_u + m]: device, out: the step (du, ds).
 *   zw [2 (n_u + m)] (may be NULL): device, out: bound duals (z_l, z_u).
 *   kkt [1] (may be NULL): device, out: the last KKT error.
 *   wreg [1] (may be NULL): device, out: the last regularisation w.
 *   status [6]: device int32, out: {iterations, converged (0/1), Cholesky
 *   info of S once the regularisation gave up (1-based column, -1 solve
 *   wait expired, 0), raw stop word (0 out of slots, 1 converged, 2
 *   non-finite, 16 + column, -1), tiny pivot word of J_x at x,
 *   factorization attempts}.
 * Leaves the point cached as rpf_reduced_gradient does (its own
 * second-order data restored).  Uses the handle's workspace, and its
 * streams as rpf_reduced_hessian does. */
int rpf_qp_step(rpf_grid* grid, const double* x, const double* u, const double* pd, const double* qd,
                const double* s, const double* y, double rho, const double* sigma, double delta,
                const double* u_lo, const double* u_hi, const double* s_lo, const double* s_hi,
                int32_t max_iter, double tol, int32_t batch, double* H, double* J, double* grad, double* dw,
                double* zw, double* kkt, double* wreg, int32_t* status, rpf_stream_t stream);

/* One real-time tracking update with the exact step (Section IV-C, steps
 * 1-3), entirely on the device (no host synchronisation):
 *   loads pd = pd0 * load_factor, qd = qd0 * load_factor (per bus);
 *   p_pv <- p_pv * dispatch_scale (1.0: unchanged), the generators' share
 *   of a uniform load change taken before the power flow (as primary
 *   frequency response would), for load steps a single slack bus cannot
 *   absorb;
 *   power flow at u from x (pf_iters predicated Newton steps, tol);
 *   the bounded QP of eq. (qp_rto) at w = (u, s) with the multipliers y, as
 *   rpf_qp_step (qp_iters iterations at most, stopping tolerance qp_tol);
 *   w <- w + dw / 2^k for the first k <= max_halvings whose power flow
 *   converges (w unchanged if none);
 *   y <- y + rho D_c (c(u) - s).
 * u [n_u], s [m], x [n_x], y [m]: device, in/out.  pd0, qd0, load_factor
 * [nb], s_lo, s_hi [m], u_lo, u_hi [n_u], sigma [1 + m]: device, read.
 * dispatch_scale: host, > 0.  J [m x n_u]: device workspace (out: the reduced Jacobian at the step's
 * point).  batch: width of the Hessian batches (0 = the handle's).
 * status [8]: device int32, out: {first power flow converged, accepted
 * halving k (-1: none), QP iterations, QP converged, Cholesky info of the
 * Schur complement, Newton steps of the first power flow, tiny pivot word
 * of the factorization behind the QP data, QP stop word (as rpf_qp_step)}.
 * Uses the handle's workspace (one step at a time per handle). */
int rpf_track_step_qp(rpf_grid* grid, double* u, double* s, double* x, double* y, const double* pd0,
                      const double* qd0, const double* load_factor, const double* s_lo, const double* s_hi,
                      const double* u_lo, const double* u_hi, double rho, const double* sigma, double delta,
                      int32_t pf_iters, int32_t max_halvings, double tol, int32_t qp_iters, double qp_tol,
                      int32_t batch, double dispatch_scale, double* J, int32_t* status, rpf_stream_t stream);

/* Static OPF by the augmented-Lagrangian method (Section IV-B.3; the
 * bound-constrained Lagrangian method of the textbook it cites; stopping
 * tolerances of Section V-B: ||c(u) - s||_inf <= 1e-5 and projected
 * gradient <= 1e-4).  Outer iteration at multipliers y and penalty rho:
 *   the subproblem eq. (auglag_subproblem), min L_rho(w; y) over the box of
 *   w = (u, s), warm-started from the current w: repeated bounded QPs of the
 *   form eq. (qp_rto) at the current point (as rpf_qp_step, shift 0, the
 *   interior point's inertia control keeping its systems positive definite,
 *   qp_iters slots, qp_tol), each followed by a backtracking line search on
 *   L_rho (Armijo 1e-4, at most 10 halvings, a power flow from the current
 *   state at every trial point), until ||w - clip(w - grad L_rho, lo, hi)||
 *   _inf <= omega (at most max_inner QPs);
 *   theta = ||c(u) - s||_inf <= eta: stop if theta <= 1e-5 and the measure
 *   <= 1e-4, else y <- y + rho D_c (c - s), eta <- eta / rho^0.9, omega <-
 *   omega / rho; otherwise rho <- 10 rho, eta <- rho^-0.1, omega <- 1 / rho
 *   (omega = 1 / rho0, eta = rho0^-0.1 at the start).
 * x [n_x] (start: any point from which the power flow at u converges; out:
 * the power-flow state at the final u), u [n_u], s [m], y [m]: device,
 * in/out.  pd, qd [nb], sigma [1 + m], u_lo, u_hi [n_u], s_lo, s_hi [m]:
 * device, read.  J [m x n_u]: device workspace.  hist [max_outer x 8]:
 * HOST, out, per outer iteration {rho, QPs of the subproblem, theta,
 * projected-gradient measure, cost f, multipliers updated (0/1),
 * converged (0/1), L_rho}; nhist (host): outer iterations done; rho_out
 * (host, may be NULL): the final penalty.
 * Unlike the compute calls above, this driver synchronises the host after
 * every QP and every trial point to take its decisions (it is not
 * capturable); RPF_EINVAL if the power flow at the starting u fails. */
int rpf_static_opf(rpf_grid* grid, double* x, double* u, double* s, double* y, const double* pd, const double* qd,
                   double rho0, const double* sigma, const double* u_lo, const double* u_hi, const double* s_lo,
                   const double* s_hi, int32_t max_outer, int32_t max_inner, int32_t qp_iters, double qp_tol,
                   int32_t pf_iters, double tol, double* J, double* hist, int32_t* nhist, double* rho_out,
                   rpf_stream_t stream);

/* Kernel timing with HIP events recorded on the launch stream, per kernel
 * class: 0 batched triangular solves inside the independent subtree packs
 * (more than one right-hand side), 1 single right-hand-side triangular
 * solves (all parts), 2 LU refactorization, 3 sparse products of the
 * Hessian batches, 4 dense Cholesky kernels, 5 batched triangular solves of
 * the top (separator) rows (their pack contributions, the product with the
 * top block's inverse, and the pack rows' products with the solved top).
 * rpf_profile_read waits for the recorded events, returns the summed
 * milliseconds and launch counts per class (host arrays [RPF_PROF_CLASSES])
 * and clears them when reset != 0. */
#define RPF_PROF_CLASSES 6
int rpf_profile_enable(rpf_grid* grid, int32_t enable);
int rpf_profile_read(rpf_grid* grid, double* ms, int64_t* launches, int32_t reset);
/* As rpf_profile_read, and busy_ms [RPF_PROF_CLASSES] (host, out, may be
 * NULL): per class the length of the union of its launch intervals (launches
 * that overlap on concurrent streams are counted once), from the same events
 * timed against the first recorded one. */
int rpf_profile_read_busy(rpf_grid* grid, double* ms, int64_t* launches, double* busy_ms, int32_t reset);

/* Host-only presolve introspection (no device needed), for checking the
 * index maps and the symbolic factorization:
 *   rpf_presolve_info: out20 = {n_x, n_u, m, nnz(J_x), nnz(L+U), forward
 *   levels, backward levels, longest LU row, refactorization updates,
 *   nnz(J_u), nnz(K), nnz(rank-one rows), packs of independent subtrees,
 *   rows of the top part, most levels in one pack, levels of the top part,
 *   most forward / backward levels of a pack in the batched solves (dense
 *   tails taken out), rows in dense tails, tail limit (RPF_TAIL_MAX,
 *   0 .. 128, read at each call; default 128)}.
 *   rpf_presolve_pattern: perm [n_x] (internal state index -> paper x
 *   index), lu_ptr [n_x + 1], lu_col [nnz(L+U)] (internal order, sorted
 *   columns, diagonal included); any pointer may be NULL. */
int rpf_presolve_info(const rpf_grid_desc* desc, int64_t* out20);
int rpf_presolve_pattern(const rpf_grid_desc* desc, int32_t* perm, int32_t* lu_ptr, int32_t* lu_col);

/* Message for the last nonzero return on this thread. */
const char* rpf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RPF_H */
