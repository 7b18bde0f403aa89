/*
 * amg.h -- C ABI of the MI355X (gfx950) fast block-structured algebraic
 * multigrid for the Toeplitz-like-plus-Cross systems of
 * M. Chen, R. Cao, S. Serra-Capizzano, "Fast algebraic multigrid for
 * block-structured dense and Toeplitz-like-plus-Cross systems arising from
 * nonlocal diffusion problems" (arXiv 2202.11288).
 *
 * Problem (Sec. 2.2): -L_delta u = f on (0,1), u = 0 on the interaction
 * volume, L_delta u(x) = int_{|y-x|<=delta} gamma(y-x) (u(y) - u(x)) dy,
 * discretised by shifted-symmetric piecewise-quadratic collocation
 * (eq. (system1)) with N = 2^K intervals, h = 1/N.  The unknown vector has
 * 2N-1 entries in the paper's block order
 *     U_h = [u_1 .. u_{N-1} | u_{1/2} .. u_{N-1/2}]        (Sec. 2.2.1),
 * i.e. v (N-1 node values) followed by w (N midpoint values).
 *
 * Solver: the block V-cycle of Algorithm 2 (damped Jacobi, eq. (7 Jacobi);
 * simple restriction 1/4[1 2 1] and prolongation 2 R^T on the block-ordered
 * vector, Sec. 3.1; Galerkin coarse levels, eq. (block Galerkin), kept as
 * Toeplitz generators plus Cross vectors via Lemma 3.1, eq. (split01)); every
 * level's matrix-vector product uses circulant-embedded FFTs (Sec. 3.2,
 * eq. (ccs3.4)); the coarsest level is solved by LU.  The outer iteration is
 * x <- x + B_K (b - A x), stopped when ||b - A x||_2 / ||b - A x_0||_2 < tol
 * (Sec. 5).
 *
 * Conventions shared by every entry point:
 *  - Vector arguments are DEVICE pointers (e.g. torch.Tensor.data_ptr() of a
 *    cuda tensor), contiguous, 2N-1 entries in block order, owned by the
 *    caller.  Host pointers are marked "host".
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    work is enqueued on it; functions that return values to the host
 *    (amg_solve's iters/relres) synchronise that stream.
 *  - Every function returns an amg_status; nothing throws across the ABI.
 *    On error no output is written, except amg_solve, which leaves x at its
 *    last iterate for AMG_NOT_CONVERGED / AMG_DIVERGED.
 *  - A handle is not thread-safe: use one handle per concurrent stream.
 */
#ifndef AMG_H
#define AMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amg_ctx* amg_t; /* opaque; owned by the library until amg_destroy */

typedef enum {
  AMG_OK = 0,
  AMG_NOT_CONVERGED = 1, /* max_iter reached; x holds the last iterate          */
  AMG_DIVERGED = 2,      /* NaN/Inf or residual grew 1e3x over its minimum       */
  AMG_EINVAL = -1,       /* bad argument (see each function)                     */
  AMG_ENOMEM = -2,       /* device or host allocation failed                     */
  AMG_EHIP = -3,         /* a HIP runtime call failed                            */
  AMG_ENOTSUP = -4       /* valid request the library does not implement        */
} amg_status;

typedef enum {
  /* gamma(s) = c on |s| <= delta, c = 3/(2 delta^3) (int gamma s^2 = 1).
     Sec. 2.2 uses the constant kernel 3 delta^-3; the normalisation only
     rescales A and f together.                                               */
  AMG_K_CONST = 0,
  /* gamma(s) = c*wl for s = y-x < 0, c*wr for s > 0, c as above
     (non-symmetric operator; same shifted collocation rule).                 */
  AMG_K_WEIGHTED = 1,
  /* gamma(s) = c |s|^(-1-2 alpha), c = (1-alpha) delta^(2 alpha-2),
     0 < alpha < 1/2 (the product-integration weights diverge beyond 1/2).    */
  AMG_K_FRACTIONAL = 2,
  /* Caller-supplied finest-level Toeplitz blocks of eq. (blocksystem):
     gen (host) = [A | B | C | D] generators, each ordered from the lowest
     offset to the highest, T[i,j] = t_{j-i}:
       A (N-1)x(N-1): offsets -(N-2)..N-2   (2N-3 values)
       B (N-1)xN    : offsets -(N-2)..N-1   (2N-2 values)
       C Nx(N-1)    : offsets -(N-1)..N-2   (2N-2 values)
       D NxN        : offsets -(N-1)..N-1   (2N-1 values)
     8N-8 doubles in total; delta is ignored.                                */
  AMG_K_GENERATORS = 3,
  /* The weakly singular nonlocal model of Sec. 2.1 (eq. (3system)): the
     operator int_0^1 (u(x) - u(y)) |x - y|^-gamma dy on (0, 1), 0 <= gamma
     < 1, standard piecewise-quadratic collocation, Dirichlet data u(0),
     u(1).  A = D - T: D the variable diagonal int_0^1 |x - y|^-gamma dy (a
     tridiagonal band on every level: its Galerkin images), T the product-
     integration weights (Toeplitz plus Cross).  This is eq. (3system)
     divided by its factor eta_{h,gamma}.  delta and scheme are ignored; the
     Dirichlet data enter through amg_volume_rhs (reach 0: g_left[0] = u(0),
     g_right[0] = u(1)).  amg_manufactured_rhs is AMG_ENOTSUP.              */
  AMG_K_WEAKLY_SINGULAR = 4,
  /* The fractional kernel of AMG_K_FRACTIONAL for 0 < alpha < 1, with a
     near-field rule that is an extension, not in the paper: on |t| <= h/2
     around each collocation point the piecewise quadratic is replaced by the
     one quadratic through x_c - h/2, x_c, x_c + h/2, whose linear term
     cancels between the two sides (a principal value) and whose quadratic
     term is integrable for alpha < 1; the cell pieces beyond h/2 are
     integrated as for AMG_K_FRACTIONAL.  Exact on quadratics, symmetric
     positive definite; shifted rule only.  For alpha < 1/2 it is a
     different discretization from AMG_K_FRACTIONAL.                         */
  AMG_K_FRACTIONAL_NEAR = 5
} amg_kernel_kind;

typedef struct {
  int kind;          /* amg_kernel_kind                                      */
  double alpha;      /* AMG_K_FRACTIONAL, AMG_K_FRACTIONAL_NEAR only         */
  double wl, wr;     /* AMG_K_WEIGHTED only (e.g. 1.2, 0.8)                 */
  const double* gen; /* AMG_K_GENERATORS only (host, copied during setup)    */
  int scheme;        /* AMG_SCHEME_SHIFTED (default) or AMG_SCHEME_STANDARD  */
  double gamma;      /* AMG_K_WEAKLY_SINGULAR only: exponent, 0 <= gamma < 1  */
} amg_kernel_t;

/* Collocation rule (Sec. 2.2).
   AMG_SCHEME_SHIFTED: the shifted-symmetric rule of eq. (system1): every row,
   node or midpoint, uses the quadratic pieces whose end points are of its own
   type, so all rows share one stencil (SPD for the constant kernel).
   AMG_SCHEME_STANDARD: the standard collocation of eq. (ccs2.6) / eq.
   (nonsym system): every row uses the mesh cells [x_m, x_{m+1}]; midpoint rows
   get their own stencil (blocks C, D differ from B^T, A; non-symmetric).
   Constant and weighted kernels (AMG_ENOTSUP for the fractional kernel);
   ignored for AMG_K_GENERATORS. */
#define AMG_SCHEME_SHIFTED 0
#define AMG_SCHEME_STANDARD 1

typedef enum { AMG_FP64 = 0, AMG_MIXED = 1 } amg_precision;

typedef struct {
  int m1, m2;                 /* pre/post Jacobi sweeps (Algorithm 2)        */
  double omega_pre, omega_post; /* damping (eq. (7 Jacobi))                  */
  int coarsest_log2;          /* coarsest level has 2^coarsest_log2 intervals */
  int precision;              /* AMG_FP64: everything FP64.  AMG_MIXED: V-cycle
                                 FFT matvecs/smoothing/transfers in FP32; outer
                                 residual, refinement update and the coarsest
                                 inverse in FP64 (iterative refinement).      */
  int max_iter;               /* outer iterations                            */
  int flags;                  /* AMG_FLAG_* bits, 0 by default               */
  int inner;                  /* AMG_INNER_VCYCLE (default) or AMG_INNER_PCG */
  double shift, scale;        /* operator shift*I + scale*A (defaults 0, 1)  */
  int restart;                /* AMG_INNER_GMRES cycle length, 1..64 (30)    */
  int cycle;                  /* coarse visits per level: 1 = V-cycle (the
                                 paper's Algorithm 2, default), 2 = W-cycle */
} amg_opts_t;

/* W-cycle (cycle = 2): every level above the coarsest computes its coarse
   correction with two cycles on the next level, the second starting from the
   first's result with the same right-hand side (m1 smoothing sweeps from that
   iterate, then the residual); the level above the coarsest solves exactly
   once.  It keeps the stationary iteration count flat in N where the V-cycle's
   grows (the fractional kernel), at the price of 2^l visits of level l: the
   small levels, which are latency-bound, then dominate the cycle's time. */

/* Shifted operators (Sec. 5, eq. (bdf4)).  With shift = sigma and scale = s
   the handle solves (sigma I + s A) x = b, A the collocation matrix of the
   kernel: the finest level's Toeplitz generators and Cross data are
   multiplied by s and sigma is added to its diagonal (a_0, d_0, o); the
   coarse levels are the Galerkin images of that level (Lemma 3.1), so one
   hierarchy serves every time step of a fixed (sigma, s).  A BDF4 step at
   time step tau has sigma = 25/12, s = tau (times the ratio of the caller's
   kernel constant to this library's normalised one: 2 for the paper's
   3 delta^-3).  scale must be finite and > 0, shift finite (AMG_EINVAL
   otherwise).  The volume correction E g of amg_volume_rhs belongs to A:
   scale it by s. */

/* Outer iteration of amg_solve.
   AMG_INNER_VCYCLE: the stationary iteration x <- x + B_K (b - A x) of the
   paper (Algorithm 2 as the iteration operator, Sec. 5 stopping rule).
   AMG_INNER_PCG: conjugate gradients preconditioned by one V-cycle B_K per
   iteration (the Krylov acceleration of the same V-cycle), for symmetric
   positive definite operators only (constant and fractional kernels, or
   symmetric generators); Polak-Ribiere direction update, so a V-cycle run in
   FP32 (AMG_MIXED) stays a valid preconditioner.  CG's theory wants a
   symmetric V-cycle: m1 = m2 and omega_pre = omega_post (the defaults).  The
   iteration runs on the recurrence's residual r <- r - alpha A p (FP64); when
   it passes the stop test, the true residual b - A x is formed and decides
   (the recurrence drifts from it on ill-conditioned problems): below tol the
   solve ends, otherwise CG restarts from it; a true residual not below 0.9
   times the previous one ends the solve with AMG_NOT_CONVERGED (it has
   reached what FP64 resolves for this operator, about eps |A| |x| / |b|).
   relres and the history's last entry are the true residual's.  A non-positive <r, B r> or <p, A p> ends
   the solve with AMG_DIVERGED. */
#define AMG_INNER_VCYCLE 0
#define AMG_INNER_PCG 1
/* AMG_INNER_GMRES: restarted flexible GMRES right-preconditioned by one
   V-cycle per Arnoldi step, for any non-singular operator (the non-symmetric
   weighted kernel and standard collocation included).  Classical
   Gram-Schmidt applied twice; Givens rotations give the residual estimate
   |g_{j+1}| that ends a cycle (below tol, after `restart` steps, or at
   max_iter); then x += Z y, and the true residual b - A x (FP64) decides the
   stop.  Iterations count V-cycles.  The history holds the estimates, the
   last of each cycle replaced by the true value.  Device memory: 2 restart + 1
   vectors of 2N-1 doubles (amg_footprint_bytes counts them). */
#define AMG_INNER_GMRES 2

/* amg_setup builds only the host-side hierarchy (generators, Lemma 3.1
   levels, coarsest LU) and touches no GPU; amg_level_tpx, amg_num_levels and
   amg_level_size work on such a handle, every device entry point returns
   AMG_EINVAL.  Used to verify the host setup on machines without a GPU. */
#define AMG_FLAG_HOST_ONLY 1
/* Record HIP events on the caller's stream around the finest level's three
   FFT passes, the small-level V-cycle kernel, each V-cycle and each outer
   residual during amg_solve; read the totals with amg_profile_stats. */
#define AMG_FLAG_PROFILE 2
/* Launch every V-cycle kernel directly.  By default, when the hierarchy has
   at least two levels above the small-level kernel (N >= 2^13), a handle's
   second V-cycle is captured into a HIP graph on an internal stream and every
   later V-cycle replays that graph on the caller's stream (same kernels, same
   arguments, fewer launch gaps).  Set this flag when the caller captures the
   solve into a graph of its own.  Profiled handles always launch directly. */
#define AMG_FLAG_EAGER 4
/* Form the outer FP64 residual b - A x (the stopping rule's measure, and the
   refinement's right-hand side) in split form.  The finest matrix is, in the
   interleaved order of the collocation points, the row stencil W of each
   point cut to the interior columns (eq. (ccs2.6)); its entries within 64
   half-steps are applied in difference form
     sum_{0<|k|<=64} W(k) (x_{s+k} - x_s) + R_s x_s,
   R_s = the row's near entries summed, and only the entries beyond 64
   half-steps go through the FFT (their own spectra).  The own-point weight
   W(0) = int gamma (1 - l_0) equals -sum_{k != 0} W(k), the quadratic basis
   being a partition of unity on every cell (so interior rows sum to zero);
   R_s is formed from that identity in long double at setup, as minus the
   stencil's weight beyond 64 half-steps and outside the interval, so the
   operator measured is the collocation matrix with that diagonal, not its
   FP64 rounding (whose last bit alone moves b - A x by eps |W(0)| |x|).  A
   plain FP64 FFT evaluation of b - A x carries an error of about
   eps |A| |x|, which for kernels with large near-field weights (the
   fractional kernel at large N) exceeds 1e-10 |b|; the split form's error is
   that of the small far-field entries and of the differences of neighbouring
   values (about 1e-12 |b| at N = 2^22, fractional alpha = 0.4).  Constant,
   weighted and fractional kernels (AMG_ENOTSUP otherwise); no effect for
   N < 2^11, whose finest level runs in the small-level kernels.  Costs one
   near-field pass (129 terms per unknown) per outer residual and FP64
   spectra of the far field. */
#define AMG_FLAG_ACCURATE_RESIDUAL 8
/* V-cycles only: the cycle below the four-step levels (levels of 2^12 or
 * fewer intervals, when the problem has more) is formed at setup as its
 * dense matrix (up to 4095 x 4095, from the unit vectors; about 2 ms more
 * setup and 201 MB (mixed) or 134 MB (FP64) more memory at its largest) and
 * applied as one product by many workgroups, in place of the one-workgroup
 * kernel that runs those levels one after another.  The same linear map up
 * to rounding; pays off when a hierarchy serves many V-cycles. */
#define AMG_FLAG_DEEP_FOLD 16

/* Per-kernel timing accumulated while AMG_FLAG_PROFILE is set. */
typedef struct {
  char name[48];      /* e.g. "fp32_finest_sweep" (the finest level's three
                         passes, events around the sweep only), "vcycle" */
  int64_t launches;   /* launches timed since the last reset                  */
  double total_ms;    /* summed event-to-event time (ms)                      */
} amg_stat_t;

/* Fill *o with m1 = m2 = 1, omega = 2/3, coarsest_log2 = 5, FP64,
   max_iter = 200, flags = 0, inner = AMG_INNER_VCYCLE. */
void amg_default_opts(amg_opts_t* o);

/* Build the multigrid hierarchy (Sec. 3): finest generators by product
 * integration of the kernel against the quadratic basis (eq. (ccs2.1); the
 * partial last cell [r h, delta] is integrated exactly when delta/h is not an
 * integer), Galerkin levels by Lemma 3.1 down to 2^coarsest_log2 intervals,
 * per-level circulant spectra (eq. (ccs3.4)) on the device, LU of the
 * coarsest level.  The cycle below and including the largest level above the
 * coarsest with at most 255 unknowns (V-cycles), or the visits a level with
 * at most 511 unknowns receives per descent (W-cycles, below the small-level
 * kernel's first level), is a linear map of that level's right-hand side:
 * setup forms its matrix from the unit vectors (FP64, a few ms) and cycles
 * apply it as one dense product (the same operator as the recursion, to
 * rounding).  N must be a power of two with coarsest_log2 < log2 N <= 22
 * and 2 <= coarsest_log2; 0 < delta < 1/2 (ignored for AMG_K_GENERATORS).
 * *out receives the handle.  Errors: AMG_EINVAL (bad N, delta, alpha, weights,
 * null pointer, options; inner = AMG_INNER_PCG with a non-symmetric operator),
 * AMG_ENOMEM, AMG_EHIP. */
int amg_setup(const amg_kernel_t* kernel, double delta, int64_t N,
              const amg_opts_t* opts, void* stream, amg_t* out);

/* y = A x on the finest level (FP64; x, y device, 2N-1 doubles, must not
 * alias).  Errors: AMG_EINVAL (null), AMG_EHIP. */
int amg_matvec(amg_t h, const double* x, double* y, void* stream);

/* r = b - A x on the finest level in FP64, evaluated exactly as the solve's
 * outer residual (Sec. 5 stopping rule): the FFT matvec, or with
 * AMG_FLAG_ACCURATE_RESIDUAL the split form (near field in difference form,
 * far field through the FFT).  b, x, r device, 2N-1 doubles; r must alias
 * neither.  Errors: AMG_EINVAL, AMG_EHIP. */
int amg_residual(amg_t h, const double* b, const double* x, double* r, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): y = A x on the finest level, the
 * same kernels and arithmetic as amg_matvec (bitwise the same result), with
 * the FFT work buffer, the block partials and the w_o scalars taken from a
 * static device array of the library (8 MiB + 32 KiB per device, held until
 * the process ends) instead of the handle's work memory.  Calls no hipMalloc,
 * hipFree or other allocating routine.  Limit: N <= 2^18 (AMG_EINVAL above;
 * with AMG_DEBUG set the reason goes to stderr).  Every call on a device
 * shares that device's array: calls that overlap on one device (different
 * streams, threads or handles) race.  x, y device, 2N-1 doubles, must not
 * alias.  Errors: AMG_EINVAL, AMG_EHIP. */
int amg_matvec_noalloc(amg_t h, const double* x, double* y, void* stream);

/* y = A_level x for level `level` (0 = finest, amg_num_levels()-1 =
 * coarsest) in FP64; x, y device, amg_level_size(level) doubles.  Exposes
 * every level's FFT matvec for verification.  Errors: AMG_EINVAL. */
int amg_level_matvec(amg_t h, int level, const double* x, double* y, void* stream);

/* y = A_level x in FP32, with the FP32 spectra, Cross vectors and FFTs the
 * FP32 V-cycle of an AMG_MIXED handle uses (Sec. 3.2, eq. (ccs3.4)):
 * the same kernels as amg_level_matvec, instantiated for float.  x, y
 * device, amg_level_size(level) floats, must not alias.  Exposes the FP32
 * FFT matvec of every level for verification (its error grows like
 * eps_32 log2 L).  Errors: AMG_EINVAL (null, aliasing, bad level, or a
 * handle not set up with AMG_MIXED), AMG_EHIP. */
int amg_level_matvec_f32(amg_t h, int level, const float* x, float* y, void* stream);

/* e = B_K r: one V-cycle of Algorithm 2 from a zero initial guess.  With
 * AMG_FP64, r and e are double*; with AMG_MIXED they are float* (the
 * coarsest inverse is applied from FP64 entries with FP64 sums, the folded
 * bottom levels (amg_setup) from their FP32 rounding).  2N-1 entries,
 * device, must not alias. */
int amg_vcycle(amg_t h, const void* r, void* e, void* stream);

/* Solve A x = b by x <- x + B_K (b - A x) (or, with inner = AMG_INNER_PCG,
 * by V-cycle-preconditioned conjugate gradients) until the relative residual
 * ||b - A x||_2 / ||b - A x_0||_2 < tol or max_iter (Sec. 5 stopping rule).
 * b (device, 2N-1 doubles), x (device, in: initial guess, out: solution).
 * iters/relres (host, may be NULL) receive the iteration count and the final
 * relative residual (FP64, computed by the FFT matvec).  The call returns when
 * the solve is done (its work is queued on `stream`); between iterations the
 * calling thread polls (pinned host memory the stop test writes, or the
 * stream) rather than sleeping, so it keeps one CPU core busy meanwhile.
 * Returns AMG_OK, AMG_NOT_CONVERGED or AMG_DIVERGED, or an error code. */
int amg_solve(amg_t h, const double* b, double* x, double tol, void* stream,
              int* iters, double* relres);

/* Solve `count` independent problems: for each i, the same iteration as
 * amg_solve(hs[i], b[i], x[i], tol[i]) (host arrays of device pointers and
 * tolerances).  The instances run concurrently on internal streams of the
 * library, forked from and joined back into `stream` (so the work is ordered
 * after earlier work on `stream`, and later work on it sees the results);
 * their iterations advance in rounds with one host synchronisation per round.
 * Handles must be distinct and live on one device; N, kernel and precision
 * may differ.  Each instance's arithmetic is identical to its solo solve.
 * iters/relres (host arrays, may be NULL) receive per-instance results.
 * Returns AMG_OK if every instance converged, else the largest positive
 * status (AMG_NOT_CONVERGED, AMG_DIVERGED), or an error code. */
int amg_solve_batch(int count, amg_t* hs, const double* const* b, double* const* x,
                    const double* tol, void* stream, int* iters, double* relres);

/* Relative residual history of the last amg_solve: hist (host) receives
 * min(cap, iters+1) values, hist[i] = ||b - A x_i|| / ||r_0||.  Returns the
 * number written (>= 0) or an error code. */
int amg_residual_history(amg_t h, double* hist, int cap);

/* Number of levels (finest .. coarsest) and the unknown count 2 n_l + 1 of
 * level l (n_l = 2^(K-l) - 1). */
int amg_num_levels(amg_t h);
int64_t amg_level_size(amg_t h, int level);

/* Copy level `level`'s Toeplitz-plus-Cross data (eq. (split01)), as built on
 * the host by Lemma 3.1, into host arrays (any may be NULL).  The hierarchy of
 * a device handle with a constant, weighted or fractional kernel is formed
 * on the device (the same recurrences; the host keeps only the coarsest
 * level), and its other levels give AMG_ENOTSUP: set the handle up with
 * AMG_FLAG_HOST_ONLY to inspect them.  The generators
 * a, b, c, d of A, B_bar, C_bar, D_bar (2n-1 values each, offsets -(n-1)..n-1),
 * the Cross vectors p, q, xi, zeta (n values each) and o (1 value). */
int amg_level_tpx(amg_t h, int level, double* a, double* b, double* c, double* d,
                  double* p, double* q, double* xi, double* zeta, double* o);

/* Copy level `level`'s tridiagonal band (2n+1 values each, host arrays; any
   may be NULL): sub[i] couples unknown i to i-1, main[i] to i, sup[i] to i+1.
   Returns 1 if the level has a band (AMG_K_WEAKLY_SINGULAR), 0 if not (the
   arrays are then left untouched), or AMG_EINVAL. */
int amg_level_band(amg_t h, int level, double* sub, double* main, double* sup);

/* Copy up to `cap` timing records (host array) accumulated by amg_solve
 * under AMG_FLAG_PROFILE; returns the number of records (>= 0) or an error
 * code.  reset != 0 clears the totals after copying. */
int amg_profile_stats(amg_t h, amg_stat_t* out, int cap, int reset);

/* Right-hand side f(x_c) = -L_delta u(x_c) for the manufactured solution
 * u = x^2 (1-x)^2 (zero outside (0,1)) at the 2N-1 collocation points in
 * block order; host output b_host (2N-1 doubles).  Same kernel/delta/N rules
 * as amg_setup (AMG_K_GENERATORS is AMG_EINVAL).  For AMG_K_FRACTIONAL_NEAR
 * with alpha >= 1/2 the first moment of the kernel over the part of the
 * horizon inside (0, 1) is a principal value. */
int amg_manufactured_rhs(const amg_kernel_t* kernel, double delta, int64_t N, double* b_host);

/* One step of the fourth-order backward differentiation formula (Sec. 5,
   eq. (bdf4)) on a handle with shift = 25/12 and scale = tau (see above):
     b = 4 u1 - 3 u2 + (4/3) u3 - (1/4) u4 + src,   x <- u1,
   then amg_solve(h, b, x, tol, ...) from that initial guess.  u1..u4 are
   U^{k-1}..U^{k-4}, src = tau (F^k - E g^k) (NULL: zero), x receives U^k; all
   device arrays of 2N-1 doubles in block order on the handle's device.  x may
   be one of u1..u4 (b is formed before x is written); it must not be src.
   b lives in a handle-owned buffer allocated by the first call (8 (2N-1)
   bytes).  Same status, iters and relres as amg_solve. */
int amg_bdf4_step(amg_t h, const double* u1, const double* u2, const double* u3,
                  const double* u4, const double* src, double* x, double tol, void* stream,
                  int* iters, double* relres);

/* Volume data (Sec. 2.2: u = g on the interaction volume).  The rows near
 * x = 0 and x = 1 couple to the exterior collocation points x = -k h/2 and
 * x = 1 + k h/2, k = 0..S.  Returns S (>= 0) for this kernel, delta, N and
 * scheme, or an error status (< 0). */
int64_t amg_volume_reach(const amg_kernel_t* kernel, double delta, int64_t N);

/* b -= E g: carries known exterior values to the right-hand side (the
 * boundary corrections of eqs. (rightside1), (rightside2), for either
 * scheme).  g_left[k] = g(-k h/2), g_right[k] = g(1 + k h/2), k = 0..S (host,
 * S + 1 doubles each, S from amg_volume_reach); b (host, 2N-1 doubles, block
 * order) is updated in place.  Host only, FP64: direct sums for a short
 * reach, FFT convolution (O(S log S)) beyond.  Errors: AMG_EINVAL (bad
 * kernel, delta, N, null pointer), AMG_ENOTSUP, AMG_ENOMEM. */
int amg_volume_rhs(const amg_kernel_t* kernel, double delta, int64_t N, const double* g_left,
                   const double* g_right, double* b);

/* Device bytes amg_setup would allocate for this problem (spectra, Cross
 * vectors, per-level work vectors, FFT scratch); < 0 on invalid input. */
int64_t amg_footprint_bytes(const amg_kernel_t* kernel, double delta, int64_t N,
                            const amg_opts_t* opts);

/* Release every device and host resource of the handle (NULL is a no-op). */
int amg_destroy(amg_t h);

/* ---- Geometry of the level matvecs and its autotuner --------------------
 * A level of size L = 2^logL (13 <= logL <= 23; smaller levels run in
 * one-workgroup kernels) evaluates its FFT product (eq. (ccs3.4)) as a
 * four-step FFT over an L1 x L2 array (rows of L1 = 2^logL1, columns in
 * tiles of `tcols`).  Every geometry computes the same product up to FP
 * rounding order; their speed differs.  The geometry in use is
 * process-wide, per size, and read when a hierarchy is set up (hierarchies
 * keep theirs).
 * amg_autotune: for each size in [logL_min, logL_max], times the level
 * matvec (FP32 + FP64, general blocks, median of 7) in every candidate
 * geometry on the current device and stream, rejects a candidate whose FP64
 * product differs from the default geometry's by more than 1e-11 of its
 * largest entry, and selects the fastest.  Errors: AMG_EINVAL
 * (logL_min > logL_max), AMG_EHIP, AMG_ENOMEM. */
int amg_autotune(int logL_min, int logL_max, void* stream);
/* The geometry in use for size 2^logL and the autotuner's record of it
 * (host pointers, each may be NULL): log2 row length, tile width, cost of
 * the default and of the chosen geometry in microseconds (0: not tuned),
 * number of candidates and of rejected candidates.  AMG_EINVAL for logL
 * outside 13..23. */
int amg_plan_get(int logL, int* logL1, int* tcols, double* us_default, double* us_best,
                 int* candidates, int* rejected);
/* Select a candidate geometry for size 2^logL (logL1 = 0: the default).
 * AMG_EINVAL if logL is outside 13..23 or (logL1, tcols) is no candidate. */
int amg_plan_set(int logL, int logL1, int tcols);

/* ---- Serving: a request loop with continuous batching ------------------
 * A server solves independent requests (kernel, delta, N, options, b, x,
 * tol), each the same iteration as amg_solve, while requests keep arriving.
 *  - Admission: a submitted request waits until its device footprint
 *    (amg_footprint_bytes) fits in the server's memory budget, counting the
 *    requests in flight and the cached hierarchies (evicted oldest first;
 *    a set-up thread frees them, and their bytes count until it has).
 *  - Setup: worker threads build hierarchies on their own streams; a cached
 *    hierarchy of a finished request with the same problem key (kernel
 *    parameters, delta, N, options: its generator spectra for every level)
 *    is taken instead.
 *  - Rounds: amg_server_step starts the requests whose hierarchy is ready
 *    (x then holds their initial guess), runs `rounds` rounds in which every
 *    request in flight does one iteration (batched launches over all of
 *    them, as amg_solve_batch), and retires the finished ones.  A request's
 *    arithmetic is that of its solo amg_solve, whatever else is in flight.
 * Supported: constant, weighted and fractional kernels; V-cycle or CG inner
 * iteration; V-cycles (cycle = 1); one (m1, m2) per server (AMG_ENOTSUP
 * otherwise).  b and x are device arrays of 2N-1 doubles owned by the caller,
 * valid until the request is reported by amg_server_poll.  Threads:
 * amg_server_submit, amg_server_poll and amg_server_stats may run on any
 * thread, also while amg_server_step runs on another; calls of
 * amg_server_step must not overlap each other, and amg_server_destroy must
 * not overlap any call on the server. */
typedef struct amg_server* amg_server_t;
typedef struct {
  int64_t id;        /* the id amg_server_submit returned                    */
  int status;        /* amg_solve's status, or the setup's error code        */
  int iters;
  double relres;
  int cached;        /* 1: the request reused a cached hierarchy             */
} amg_server_result_t;
typedef struct {
  int64_t submitted, finished, rounds;
  int64_t cache_hits, cache_misses, evictions;
  int64_t reserved_bytes, peak_reserved_bytes, cached_hierarchies;
  /* host wall time in microseconds: amg_server_step starting requests, in
   * rebuilding the batched launch tables, and in enqueueing and waiting for
   * rounds; the set-up threads' time in amg_setup (summed over threads) */
  int64_t start_us, rebuild_us, rounds_us, setup_us, rebuilds;
} amg_server_stats_t;

/* Create a server on the current device: `workers` setup threads (1..64),
 * device memory budget in bytes, rounds enqueued on `stream` (NULL: a
 * non-blocking stream of the server's own).  A request's b and initial x
 * are read on that stream from the next amg_server_step on: work producing
 * them on another stream must have completed by then (synchronise it before
 * amg_server_submit).  Errors: AMG_EINVAL, AMG_ENOMEM, AMG_EHIP. */
int amg_server_create(int64_t mem_budget_bytes, int workers, void* stream, amg_server_t* out);
/* Queue a request; *id (host, may be NULL) receives its id.  opts may be
 * NULL (defaults).  Errors: AMG_EINVAL (bad arguments), AMG_ENOTSUP (see
 * above, or a footprint larger than the budget). */
int amg_server_submit(amg_server_t sv, const amg_kernel_t* kernel, double delta, int64_t N,
                      const amg_opts_t* opts, const double* b, double* x, double tol,
                      int64_t* id);
/* Start ready requests, run `rounds` rounds over the requests in flight,
 * retire the finished ones; returns when the rounds are done (the calling
 * thread polls the stream; with two lanes, when one lane's are, see
 * amg_server_lanes).  With rounds > 0 and no request in the rounds,
 * it first waits until a set-up (or the release of an evicted hierarchy) in
 * progress ends; it returns at once if there is none.  *in_flight / *waiting (host, may be NULL): the requests started
 * or being set up / waiting for memory. */
int amg_server_step(amg_server_t sv, int rounds, int* in_flight, int* waiting);
/* Two lanes: requests with N <= small_max_N run their rounds on a second
 * stream of the server's, small_rounds of them per amg_server_step round
 * (1..16).  The lanes advance independently: amg_server_step queues the
 * rounds of every idle lane and returns once one lane has completed (and
 * been queued again), so small requests are not paced by the large ones'
 * iterations and the two lanes' kernels overlap on the device.
 * small_max_N = 0: one lane (the default).  Only while no request is in the
 * rounds (AMG_EINVAL otherwise); not concurrently with amg_server_step.
 * A request's arithmetic is the same in either lane. */
int amg_server_lanes(amg_server_t sv, int64_t small_max_N, int small_rounds);
/* Copy up to `cap` results of requests finished since the last poll (host
 * array); returns their number. */
int amg_server_poll(amg_server_t sv, amg_server_result_t* out, int cap);
int amg_server_stats(amg_server_t sv, amg_server_stats_t* out);
/* Stop the workers and release every hierarchy (NULL is a no-op). */
int amg_server_destroy(amg_server_t sv);

/* Static description of a status code. */
const char* amg_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* AMG_H */
