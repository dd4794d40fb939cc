/*
 * helmholtz6 - sixth-order compact Helmholtz solver for one AMD Instinct MI355X (gfx950).
 *
 * Method: Gryazin, "Preconditioned Krylov subspace methods for sixth order
 * compact approximations of the Helmholtz equation" (arXiv:1212.1397).
 *   - Problem and faces: Section 1, eqs. (problem) and (bc).
 *   - Operator A: Section 3.1, eq. (scheme), with the Neumann closure of
 *     Section 3.2.1, eq. (3DN), and the Sommerfeld-like closure of
 *     Section 3.2.2, eq. (3DDISCS).
 *   - Preconditioner A_p: Section 3.3, eq. (3DAP).
 *   - Solvers: right-preconditioned GMRES (Section 2, eq. (AAP)), the SKS
 *     iteration (Section 2, Algorithm 1) and Chebyshev acceleration (Section 2,
 *     Theorem 2) with the closed-form spectrum bounds of eq. (3DEGV).
 *
 * Every entry point is extern "C" and never throws.  All vectors are device
 * pointers to complex128 values stored as interleaved (re, im) doubles, x
 * fastest: element (i, j, l) of an n'x x n'y x n'z grid sits at
 * i + n'x * (j + n'y * l).  n'a = n[a] + (number of Neumann/Sommerfeld faces
 * on axis a), see helmholtz6_dims.  Pointers must be 16-byte aligned.
 *
 * Ownership: the caller owns every vector buffer; the library owns a plan and
 * its device workspace (allocated by helmholtz6_setup / helmholtz6_solve,
 * released by helmholtz6_destroy).  No caller pointer is kept after a call
 * returns.  apply_* and rhs_* only enqueue work on the given HIP stream (NULL
 * means the legacy default stream); the caller keeps buffers alive until the
 * stream is synchronised.  helmholtz6_solve synchronises the stream before it
 * returns.  A plan must not be used from two host threads at once.
 *
 * Errors: a negative status means the call failed and outputs are
 * unspecified; helmholtz6_last_error(plan) gives a message.  Non-negative
 * statuses other than H6_OK (not converged, diverged) leave a valid iterate.
 */
#ifndef HELMHOLTZ6_H
#define HELMHOLTZ6_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  H6_OK = 0,
  H6_NOT_CONVERGED = 1,      /* maxit reached; U holds the last iterate */
  H6_DIVERGED = 2,           /* SKS: relative residual > 1e4 or not finite; U = last iterate */
  H6_ERR_ARG = -1,           /* invalid argument (null pointer, bad size, bad enum) */
  H6_ERR_UNSUPPORTED_BC = -2,/* face pattern without a preconditioner in Section 3.3 */
  H6_ERR_ALLOC = -3,         /* device allocation failed */
  H6_ERR_HIP = -4,           /* a HIP runtime call or kernel launch failed */
  H6_ERR_SINGULAR = -5       /* zero or non-finite pivot in a z tridiagonal of A_p:
                                k^2 lies on the spectrum of the 7-point operator */
} h6_status;

typedef enum { H6_DIRICHLET = 0, H6_NEUMANN = 1, H6_SOMMERFELD = 2 } h6_bc;
typedef enum { H6_GMRES = 0, H6_FGMRES = 1, H6_SKS = 2, H6_CHEBYSHEV = 3 } h6_method;
typedef enum { H6_FP64 = 0, H6_MIXED = 1 } h6_precision;

typedef struct h6_plan_s* h6_plan;

typedef struct {
  int n[3];        /* interior node counts nx, ny, nz (>= 1); domain length on axis a is (n[a]+1)*h */
  double h;        /* grid step, common to all axes (Section 3.3: same step in x, y, z) */
  double k_re;     /* wavenumber k = k_re + i k_im (Section 1: k may be complex) */
  double k_im;
  int bc[6];       /* h6_bc of faces x-, x+, y-, y+, z-, z+.  Section 3.3 covers x/y faces
                      as a Dirichlet or a Neumann pair; z faces may be any of the three,
                      independently.  Other patterns give H6_ERR_UNSUPPORTED_BC. */
  int precision;   /* h6_precision.  H6_MIXED runs the preconditioner's transforms and
                      tridiagonal solves in complex64 (FP32 arithmetic); the operator,
                      residuals, Arnoldi and Hessenberg stay FP64.  Use H6_FGMRES or
                      H6_SKS with it (plain GMRES assumes an exact preconditioner). */
} h6_params;

typedef struct {
  int method;        /* in: h6_method */
  int restart;       /* in: GMRES/FGMRES cycle length m (1..256); ignored by SKS */
  int maxit;         /* in: maximum number of A A_p^{-1} applications (>= 1) */
  double tol;        /* in: stop when ||F - A U||_2 / ||F||_2 <= tol (true residual) */
  int iters;         /* out: A A_p^{-1} applications made, counted across restarts */
  double rel_resid;  /* out: true FP64 relative residual of the returned U */
  double* history;   /* in (optional, host): per-iteration residual estimates (GMRES: the
                        least-squares residual; SKS: the true residual), relative to ||F|| */
  int history_len;   /* in: capacity of history; out: entries written */
  int zero_guess;    /* in: nonzero: the solve starts from U = 0 and U's contents are never
                        read (U may hold anything).  SKS then forms U_1 = A_p^{-1} F directly
                        (r_0 = F, no residual pass) with the same arithmetic as from a zeroed
                        U; the other methods clear U on the stream first.  0: U is the initial
                        guess. */
} h6_solve_info;

/* Builds a plan: validates the parameters, derives the unknown counts, the
 * complex coefficients of A (Section 3.1-3.2) and A_p (Section 3.3), the
 * transverse eigenvalue tables, transform plans, and checks every z
 * tridiagonal of A_p for a zero pivot (H6_ERR_SINGULAR).  hip_stream: the
 * stream used for table uploads.  On failure *out is NULL.  */
h6_status helmholtz6_setup(const h6_params* p, void* hip_stream, h6_plan* out);

/* Unknown counts dims = {n'x, n'y, n'z}. */
h6_status helmholtz6_dims(h6_plan plan, int dims[3]);

/* y = A x: the h^2-scaled 27-point compact operator of eq. (scheme) with the
 * Neumann (3DN) and Sommerfeld (3DDISCS) closure rows.  x and y must not
 * alias.  Enqueue only. */
h6_status helmholtz6_apply_A(h6_plan plan, const void* x, void* y, void* hip_stream);

/* z = A_p^{-1} r for the h^2-scaled 7-point operator of eq. (3DAP): forward
 * sine/cosine transforms in x and y, one tridiagonal solve per transverse
 * mode in z, inverse transforms.  r is not modified; r and z must not alias.
 * In H6_MIXED plans the arithmetic is complex64 (r and z stay complex128).
 * Enqueue only. */
h6_status helmholtz6_apply_Pinv(h6_plan plan, const void* r, void* z, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * z = A_p^{-1} r as helmholtz6_apply_Pinv (the same kernels, the same result
 * bit for bit), with the preconditioner's two intermediate vectors in a fixed
 * work space that the library holds in device memory (a file-scope array of
 * 128 MiB, one copy on every GPU the library runs on, kept until the process
 * ends) instead of the plan's workspace.  Limit: 2 vectors of n'x n'y n'z
 * values in the plan's compute precision, each rounded up to 256 bytes, must
 * fit in 128 MiB: up to 4,194,304 unknowns in H6_FP64 plans (complex128) and
 * 8,388,608 in H6_MIXED plans (complex64); larger grids give H6_ERR_ARG with
 * a message (use helmholtz6_apply_Pinv).  The call allocates nothing (no
 * hipMalloc, hipFree, event creation or library allocation; kernel timing of
 * helmholtz6_profile does not cover it).  Every call on one GPU shares that
 * GPU's work space, which keeps the last call's contents: calls whose work
 * overlaps in time on one GPU (other streams, other plans, other host threads)
 * race and give wrong results; order them on one stream or synchronise.
 * Nothing needs to start at zero.  Enqueue only. */
h6_status helmholtz6_apply_Pinv_noalloc(h6_plan plan, const void* r, void* z, void* hip_stream);

/* F = h^2-scaled compact right-hand side (eq. (scheme) right side, with the
 * mixed fourth-derivative coefficient h^4/180, plus the Neumann and
 * Sommerfeld face terms of (3DN) and (3DIMP)/(3DDISCS)) for the source
 *   f(x,y,z) = sum_s amp_s exp(-|x - c_s|^2 / (2 sigma^2)).
 * centres: host array of 3*nsrc doubles (x, y, z per source); amps: host
 * array of 2*nsrc doubles (re, im per source); nsrc in 0..64.  Enqueue only. */
h6_status helmholtz6_rhs_gaussians(h6_plan plan, int nsrc, const double* centres,
                                   const double* amps, double sigma, void* F, void* hip_stream);

/* F for a separable source (the manufactured solutions of Section 4 are of
 * this form): the same interior and face terms as helmholtz6_rhs_gaussians for
 *   f(x,y,z) = sum_{s < nterms} c_s X_s(x) Y_s(y) Z_s(z).
 * coef: host array of 2*nterms doubles (re, im of c_s).  tx, ty, tz: host
 * arrays of complex128 values (re, im interleaved) holding, for each term s
 * and derivative order o = 0..4, the o-th derivative of the axis factor at
 * the n'_a unknown nodes of that axis:
 *   tx[2 * ((s * 5 + o) * n'x + i) + {0, 1}] = d^o X_s / dx^o at x = q_i h,
 * q_i = i for a non-Dirichlet low face and i + 1 for a Dirichlet one (likewise
 * ty with n'y, tz with n'z).  Faces are unknown nodes wherever their face
 * terms apply, so node samples suffice.  nterms in 0..1024 (0 gives F = 0).
 * The tables are copied to a plan-owned device buffer (grown on demand);
 * synchronises hip_stream before returning, so the host arrays may be
 * released afterwards. */
h6_status helmholtz6_rhs_separable(h6_plan plan, int nterms, const double* coef, const double* tx,
                                   const double* ty, const double* tz, void* F, void* hip_stream);

/* Nonhomogeneous Dirichlet data on a z face (side 0: z = 0, side 1: the top
 * face), as in Table 5's problem.  The unknown plane next to the face couples
 * to the face values through the in-plane operator G of eq. (scheme)'s
 * delta_z^2 term, G = I + (1 + kappa/30)/6 (D_x + D_y) + (1/30) D_x D_y with
 * D = h^2 delta^2, so F -= G g on that plane.  g: device complex128 array of
 * n'x * n'y values (x fastest) at the face nodes above or below the
 * unknowns; on the face's own edges g is taken as 0 next to a Dirichlet x or
 * y face and mirrored next to a Neumann one (the data of a consistent
 * solution).  The face must be Dirichlet (H6_ERR_ARG otherwise).  Call after
 * building the source part of F.  Enqueue only. */
h6_status helmholtz6_rhs_dirichlet_z(h6_plan plan, int side, const void* g, void* F, void* hip_stream);

/* Nonzero Neumann data beta = du/dn on a Neumann face (face 0..5: x low,
 * x high, y low, y high, z low, z high; the derivative is taken along the
 * positive axis direction on both faces of an axis).  Eq. (3DN): the ghost
 * relation of the face carries -2h B with
 *   B = (1 - kappa/6 + kappa^2/120) beta - (h^4/180)(beta_t1t1t2t2 + beta_t1t1t1t1
 *       + beta_t2t2t2t2) - (k^2 h^4/180)(beta_t1t1 + beta_t2t2),
 * so F += 2h B on a low face and F -= 2h B on a high face (added to F, which
 * already holds the source terms).  beta = sum_{s < nterms} c_s T1_s(t1) T2_s(t2)
 * over the face's tangential axes t1 < t2 (x face: y, z; y face: x, z; z
 * face: x, y): coef as for helmholtz6_rhs_separable, t1 / t2 host complex128
 * tables [(s * 5 + o) * n' + i] of derivative orders o = 0..4 at the unknown
 * nodes of each tangential axis.  H6_ERR_ARG for a face that is not Neumann.
 * Synchronises hip_stream before returning. */
h6_status helmholtz6_rhs_neumann(h6_plan plan, int face, int nterms, const double* coef, const double* t1,
                                 const double* t2, void* F, void* hip_stream);

/* Solves A U = F.  U is the initial guess on entry (may be zero) and the
 * solution on return.  F and U must not alias.  GMRES/FGMRES: right
 * preconditioning, modified Gram-Schmidt Arnoldi, Givens least squares in FP64
 * on the host, restart every info->restart steps.  SKS: Algorithm 1 written
 * in correction form U += A_p^{-1} r (identical iterates for U0 = 0).
 * Chebyshev: the classical Chebyshev iteration on A A_p^{-1} over the exact
 * spectrum interval of helmholtz6_spectrum_bounds, one A and one A_p^{-1}
 * per iteration (all-Dirichlet faces, real k; diverged as for SKS).
 * Synchronises hip_stream before returning. */
h6_status helmholtz6_solve(h6_plan plan, const void* F, void* U, h6_solve_info* info,
                           void* hip_stream);

/* Exact bounds [lo, hi] of the spectrum of A A_p^{-1} for all-Dirichlet faces
 * and real k: the smallest and largest lambda / lambda^p of eq. (3DEGV) over
 * every sine mode of the grid (computed on the host on first use).
 * H6_ERR_ARG for other face patterns or complex k.  Chebyshev acceleration
 * (method H6_CHEBYSHEV) uses them and requires lo > 0 (H6_ERR_ARG otherwise:
 * the iteration does not apply). */
h6_status helmholtz6_spectrum_bounds(h6_plan plan, double* lo, double* hi);

/* Order estimate psi of eq. (PSI) from the first two SKS residual norms on
 * grids h and gamma h: eps = ||r_2|| / ||r_1|| on each grid,
 * psi = (ln eps^{gamma h} - ln eps^h) / ln gamma (gamma > 1; NaN if any
 * argument is not positive). */
double helmholtz6_psi_order(double r1_h, double r2_h, double r1_gh, double r2_gh, double gamma);

/* Solves count independent systems concurrently (the throughput form for many
 * right-hand sides, wavenumbers and grid sizes): solve i is
 * helmholtz6_solve(plans[i], F[i], U[i], &infos[i], s) on one of nstreams
 * library-owned HIP streams (1..16), each driven by its own host thread;
 * solves are started in decreasing order of an estimated cost (unknowns times
 * a kh-based iteration estimate), longest first.  Every plan must appear once
 * (a plan is not used by two threads).  statuses[i] receives solve i's
 * status.  Returns H6_OK when every solve returned a non-negative status,
 * otherwise the first negative one; waits for all solves. */
h6_status helmholtz6_solve_batch(h6_plan* plans, const void* const* F, void* const* U,
                                 h6_solve_info* infos, h6_status* statuses, int count, int nstreams);

/* The same many independent solves as one captured HIP graph fed by a
 * device-side work queue (flexible GMRES only).  helmholtz6_queue_create
 * groups the problems of plans[0..count-1] by grid shape (unknown counts,
 * faces, precision); each group gets up to `lanes` (1..16) lanes, a lane
 * being a library-owned plan of that shape with its own FGMRES(restart)
 * workspace, and a queue of the group's problems in decreasing order of an
 * estimated cost (unknowns times a kh-based iteration estimate); it captures
 * one graph holding every lane (allocates; synchronous).  The queue keeps
 * pointers to the plans, which must stay alive and unchanged until it is
 * destroyed.  helmholtz6_queue_solve solves problem i: plans[i] U[i] = F[i]
 * with infos[i] (method H6_FGMRES, restart equal to the queue's; tol and
 * maxit per problem): U[i] starts from zero (its contents are not read), F[i]
 * is read only; infos[i] receives iters and rel_resid (no history),
 * statuses[i] the solve's status.  A replay of the graph advances every lane
 * by one restart cycle with the Givens rotations on the device; at the start
 * of each cycle the lane tests its problem's true residual on the device, and
 * when the problem is done it copies U out, takes the next problem from its
 * queue (atomic head) and loads that problem's right-hand side and
 * wavenumber-dependent tables (stencil weights and z tridiagonal data of
 * plans[i]) into the lane.  The host replays the graph until every lane has
 * found its queue empty (one wait per replay); the call returns when all
 * solves are done, with H6_OK when every solve returned a non-negative
 * status, otherwise the first negative one (message in
 * helmholtz6_queue_last_error).  One solve at a time per queue.
 * helmholtz6_solve_batch_queue is create, solve and destroy in one call
 * (infos[0].restart sets the restart length; message in
 * helmholtz6_last_error(plans[0])). */
typedef struct h6_queue_s* h6_queue;
h6_status helmholtz6_queue_create(h6_plan* plans, int count, int restart, int lanes, h6_queue* out);
h6_status helmholtz6_queue_solve(h6_queue queue, const void* const* F, void* const* U, h6_solve_info* infos,
                                 h6_status* statuses);
const char* helmholtz6_queue_last_error(h6_queue queue);
void helmholtz6_queue_destroy(h6_queue queue);
h6_status helmholtz6_solve_batch_queue(h6_plan* plans, const void* const* F, void* const* U,
                                       h6_solve_info* infos, h6_status* statuses, int count, int lanes);

/* HIP graphs for GMRES / FGMRES solves on the plan, run on a plan-owned
 * stream ordered after hip_stream; built on first use, replayed by later
 * solves, rebuilt when the workspace, restart length or solution vector
 * changes.  enable = 1: one graph per Arnoldi step; the host applies the
 * Givens rotations and decides after every step.  enable = 2: one graph per
 * restart cycle; the rotations and the least-squares solution are computed on
 * the device, a device flag set when the estimate meets the tolerance (or
 * the step budget, or a breakdown) makes the remaining steps' kernels return
 * at once, and the host waits once per cycle (iterates equal mode 1's up to
 * rounding).  Graphs are not used while kernel timing is enabled or a learned
 * correction is attached.  enable = 0 releases them; other values give
 * H6_ERR_ARG. */
h6_status helmholtz6_set_graphs(h6_plan plan, int enable);

/* Autotuner: times the variants of the plan's kernels on the plan's own grid
 * (stencil z-chunk depth 8, 16 or 32 planes per workgroup; for n'x or n'y + 1
 * = 257 also the dense transform against the Rader transform at 4 or 8 lines
 * per workgroup along x and 8 or 16 columns along y; for an odd n + 1 up to
 * 255 the dense transform against the Bluestein (chirp-z) transform) and
 * keeps the fastest.  Untuned plans use Rader for n + 1 = 257, Bluestein
 * where 2(n + 1) - 2 fills at least 15/16 of its FFT length (256 or 512),
 * else the dense transform; with the environment variable
 * H6_DENSE_TRANSFORMS set at setup only the dense transform is built.  With
 * cache_path != NULL the choice is read from, or appended to, that text file
 * (one line per grid shape, precision and device).  Synchronous. */
h6_status helmholtz6_autotune(h6_plan plan, const char* cache_path, void* hip_stream);

/* Per-kernel timing: when enabled, the library records HIP events around
 * every kernel (or fused group of kernels) it launches on the caller's stream
 * and accumulates, per kernel class, the durations, the launch count and the
 * algorithmic HBM bytes of the timed work (the bytes the method must move:
 * each input vector read once, each output written once, in the storage
 * precision of the plan).  helmholtz6_kernel_time reads (and with reset != 0
 * clears) one class by name ("stencil", "stencil_resid", "xform_x",
 * "xform_y", "tridiag_z", "mgs_dots", "mgs_update", "norm", "axpy", "rhs"); it
 * synchronises the plan's timing events.  Any of ms, launches, bytes may be
 * NULL.  Returns H6_ERR_ARG for an unknown name. */
h6_status helmholtz6_profile(h6_plan plan, int enable);
h6_status helmholtz6_kernel_time(h6_plan plan, const char* name, int reset, double* ms,
                                 long long* launches, double* bytes);

/* Releases the plan and its workspace (NULL is accepted). */
void helmholtz6_destroy(h6_plan plan);

/* Static description of a status code. */
const char* helmholtz6_status_string(h6_status s);

/* Detail of the last failing call on this plan (empty if none); valid until
 * the next call on the plan.  With plan == NULL: the last setup failure. */
const char* helmholtz6_last_error(h6_plan plan);

#ifdef __cplusplus
}
#endif
#endif /* HELMHOLTZ6_H */
