/*
 * fracsolve.h -- C ABI of the MI355X (gfx950) divide-and-conquer solver for
 * the L1 time-stepping system of Caputo time-fractional equations.
 *
 * Problem (Liu, Cheng, Li, Wang, "Fast procedures for Caputo fractional
 * ordinary and partial differential equations", section 3):
 *   0<gamma<1: D_t^gamma u = u_xx + f on (x0,x1) x (0,T], u(x,0) = u0,
 *              homogeneous Dirichlet data (eq. e18), discretised by Scheme 4
 *              (eq. e19/e20);
 *   1<gamma<2: the same with u_t(x,0) = phi, discretised in time by the
 *              L1-type formula of eq. e15-e17 (source at t_{n-1/2}, spatial
 *              term at t_n).
 * With U^n the values at the M interior points x_i = x0 + i h,
 * h = (x1-x0)/(M+1), tau = T/N, both regimes give the block lower-triangular
 * Toeplitz system (time-major form of eq. e21)
 *   (a_0 I + K) U^n + sum_{j=1}^{n-1} a_{n-j} U^j = F^n - rho_n u0 + psi_n phi,
 *   n = 1..N,  K = h^-2 tridiag(-1, 2, -1),
 * with a_m, rho_n, psi_n the L1 weights of section 3 (G_k for 0<gamma<1,
 * M_k and W_j = M_{j-2} - 2 M_{j-1} + M_j for 1<gamma<2).  The library solves
 * it exactly (up to rounding) in O(M N log^2 N) work: recursive halving in
 * time, tridiagonal solves of the diagonal block, and Toeplitz-block
 * products for the off-diagonal blocks done as FFT convolutions (the
 * circulant embedding of section 3.1) or as dense products below a
 * crossover size.
 *
 * Conventions for every entry point
 *   - Arrays are float64.  Fields are time-major [N][M], row-major: element
 *     (n-1)*M + (i-1) is the value at (x_i, t_n).  u0 and phi are [M].
 *   - Field pointers (f, u0, phi, u, g, dL_df) are DEVICE pointers to memory
 *     on the current HIP device (e.g. torch tensors' data_ptr()).  Weight
 *     outputs of fracsolve_weights are HOST pointers.
 *   - A handle holds `count` independent instances (count >= 1); field
 *     arguments are host arrays of `count` device pointers, one per instance.
 *   - The caller owns every buffer passed in; the library keeps no pointer
 *     after a call returns.  The handle owns its weights, spectra, factor
 *     tables and workspace, and frees them in fracsolve_destroy.
 *   - Work is enqueued on the stream given at create time (NULL = the null
 *     stream); fracsolve_solve / fracsolve_apply / fracsolve_adjoint return
 *     after enqueueing, except where stated.  Results are valid after the
 *     stream is synchronised.  A handle must not be used from two threads at
 *     once.
 *   - Errors: every function returns FRACSOLVE_OK (0) or a negative status.
 *     Argument errors are detected before any device work.  The text of the
 *     last error is available from fracsolve_last_error(h) (or with h = NULL
 *     for errors of fracsolve_create).
 *
 * Environment (read once per process or per handle; none changes a result
 * beyond rounding order):
 *   FRACSOLVE_TUNE=0, FRACSOLVE_TUNE_CACHE   plan cache (fracsolve_plan)
 *   FRACSOLVE_PAIR=0          leaves one at a time instead of in pairs
 *   FRACSOLVE_MFMA_FROM=s     smallest dense level size on the matrix cores
 *                             (default 128)
 *   FRACSOLVE_MP_SCRATCH_MB   multi-pass FFT scratch in MiB (16..4096,
 *                             default 256)
 *   FRACSOLVE_GRAPH=1         record the recursive solve's launch
 *                             sequences as HIP graphs and replay them
 *   FRACSOLVE_ODE_GRAPH=0     launch the conjugate-gradient steps of
 *                             fracsolve_ode_cg directly instead of replaying
 *                             a recorded graph
 */
#ifndef FRACSOLVE_H
#define FRACSOLVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fracsolve_ctx *fracsolve_t;

enum {
    FRACSOLVE_OK = 0,
    FRACSOLVE_E_ARG = -1,      /* invalid argument (nothing was enqueued)   */
    FRACSOLVE_E_NOMEM = -2,    /* device or host allocation failed           */
    FRACSOLVE_E_DEVICE = -3,   /* no usable device, or a HIP call failed     */
    FRACSOLVE_E_NUMERIC = -4,  /* non-finite value found where checked       */
    FRACSOLVE_E_STATE = -5     /* call not valid in the handle's state       */
};

/* Arithmetic of the off-diagonal Toeplitz-block products.  Weights, the
 * tridiagonal solves of the diagonal blocks, the dense (small) level
 * products, the near-corner band of the FFT levels and the refinement
 * residual are float64 in every mode. */
enum {
    FRACSOLVE_FP64 = 0,   /* all products in float64                          */
    FRACSOLVE_FP32 = 1,   /* FFT level products in float32, their history
                             accumulated in float32                           */
    FRACSOLVE_BF16X3 = 2  /* reserved for split bf16 products on the matrix
                             cores; not available in this version:
                             fracsolve_create returns E_ARG for it            */
};

typedef struct {
    double gamma;   /* fractional order, in (0,1) or (1,2); 1 is rejected      */
    double T;       /* final time, > 0                                         */
    double x0, x1;  /* spatial interval, x1 > x0                               */
    int64_t M;      /* interior points, 1 <= M <= 4096                         */
    int64_t N;      /* time steps, 1 <= N <= 2^17 (padded internally to a
                       power of 2; exact, because the system is causal)       */
} fracsolve_problem;

/* Equation of every instance of a handle. */
enum {
    FRACSOLVE_DIFFUSION = 0,  /* D_t^gamma u = u_xx + f (the system above)      */
    FRACSOLVE_ADVECTION = 1,  /* D_t^gamma u + u_x = f with inflow value
                                 u(x0, t) = 0 (section 3, eq. e11-e17): Scheme 2
                                 for 0<gamma<1 (L1 formula averaged over x_i and
                                 x_{i-1}, difference (U_i - U_{i-1})/h, both at
                                 the midpoint x_i - h/2, where f is sampled, at
                                 t_n); Scheme 3 for 1<gamma<2 (the diffusion-
                                 wave weights, the same difference at x_i, f at
                                 (x_i, t_{n-1/2})).  The diagonal block is lower
                                 bidiagonal; the history keeps the scalar
                                 Toeplitz form (for Scheme 2 in W = B U,
                                 (B U)_i = U_i + U_{i-1}).  Float64 solves only. */
    FRACSOLVE_DIFFUSION_CN = 2  /* 1<gamma<2 only: the diffusion-wave equation
                                 with the spatial term averaged over t_n and
                                 t_{n-1} (Crank-Nicolson in the spatial term,
                                 the form of the Sun-Wu scheme cited with eq.
                                 e15): (a_0 I + K/2) U^n + (a_1 I + K/2) U^{n-1}
                                 + sum_{j<n-1} a_{n-j} U^j = F^n - rho_n u0
                                 + psi_n phi - [n = 1] (K/2) u0.  Float64;
                                 solve, apply, adjoint and GMRES.           */
};

typedef struct {
    int32_t precision;    /* FRACSOLVE_FP64 or FRACSOLVE_FP32 (BF16X3: E_ARG)  */
    int32_t refine_steps; /* iterative-refinement steps against the float64
                             operator for FP32 / BF16X3 (0 = none; FP64 ignores
                             it)                                               */
    int32_t leaf;         /* leaf size L (4, 8 or 16); 0 = tuned plan          */
    int32_t crossover;    /* largest half-block size s done as a dense product;
                             FFT above it.  0 = tuned plan (fracsolve_plan),
                             < 0 = FFT at every level                          */
    int32_t leaf_solver;  /* tridiagonal solve of a_0 I + K in the leaves:
                             0 = closed-form inverse by parallel scan (default),
                             1 = block Thomas + parallel cyclic reduction      */
    void *stream;         /* hipStream_t for all work; NULL = null stream      */
    int32_t equation;     /* FRACSOLVE_DIFFUSION (0), FRACSOLVE_ADVECTION (1)
                             or FRACSOLVE_DIFFUSION_CN (2); 1 and 2 need
                             precision FP64 and leaf_solver 0.  ADVECTION
                             supports fracsolve_solve and fracsolve_weights
                             only (the other entry points return E_ARG)       */
} fracsolve_options;

/*
 * Create a handle for `count` instances (probs[0..count-1]).  Validates every
 * problem (gamma in (0,1) or (1,2), T > 0, x1 > x0, 1 <= M <= 4096,
 * 1 <= N <= 2^17),
 * computes the weights (section 3: G_k / M_k in cancellation-free form),
 * the FFT spectra of the Toeplitz column for every FFT level (circulant
 * embedding, section 3.1) and the factor tables of a_0 I + K, on the device.
 * opts may be NULL (defaults).  On success *out receives the handle.
 * Errors: E_ARG (bad argument; the message names the instance and field),
 * E_DEVICE (no HIP device), E_NOMEM.
 */
int fracsolve_create(const fracsolve_problem *probs, int32_t count,
                     const fracsolve_options *opts, fracsolve_t *out);

/*
 * The plan fracsolve_create would choose for these problems and options: the
 * leaf size L and the crossover s* (largest half-block size done as a dense
 * product; -1 = FFT at every level).  Options leaf / crossover > 0 (or
 * crossover < 0) are taken as given; zeros are looked up, first in the plan
 * cache written by the tuner (paper_1710_11593_amd/tune.py: a JSON file at
 * $FRACSOLVE_TUNE_CACHE, else $XDG_CACHE_HOME/fracsolve/plan.json, else
 * ~/.cache/fracsolve/plan.json; not read when FRACSOLVE_TUNE=0), then in the
 * library's built-in table (the tuner's measurements on MI355X).  A missing,
 * unreadable or malformed cache file falls back to the built-in table.
 * *source (any output may be NULL) tells which: FRACSOLVE_PLAN_OPTIONS,
 * FRACSOLVE_PLAN_CACHE or FRACSOLVE_PLAN_BUILTIN.  Host only: no device is
 * needed.  Errors: E_ARG (as fracsolve_create's problem checks).
 */
enum { FRACSOLVE_PLAN_OPTIONS = 0, FRACSOLVE_PLAN_CACHE = 1, FRACSOLVE_PLAN_BUILTIN = 2 };

int fracsolve_plan(const fracsolve_problem *probs, int32_t count, const fracsolve_options *opts,
                   int32_t *leaf, int32_t *crossover, int32_t *source);

/*
 * Copy instance `inst`'s weights to host arrays of length N (any may be NULL):
 *   b[k]    = G_k or M_k,                    k = 0..N-1
 *   a[m]    = Toeplitz column a_m,           m = 0..N-1  (a_0 = diagonal shift)
 *   rho[n-1], psi[n-1] = u0 and phi coefficients of step n, n = 1..N
 *   da, drho, dpsi = derivatives of a, rho, psi with respect to gamma.
 * Synchronises the handle's stream.  Errors: E_ARG, E_DEVICE.
 */
int fracsolve_weights(fracsolve_t h, int32_t inst, double *b, double *a, double *rho,
                      double *psi, double *da, double *drho, double *dpsi);

/*
 * Solve every instance: u[k] <- solution U [N][M] for source f[k] [N][M]
 * (sampled at t_n for gamma<1, at t_{n-1/2} for gamma>1) and initial data
 * u0[k], phi[k] ([M]; phi is ignored for gamma<1).  u0 or phi (the outer
 * array, or any entry) may be NULL, meaning zero.  u[k] may equal f[k]
 * (in place).  u[k] is used as workspace during the call.
 * Errors: E_ARG (NULL f or u), E_DEVICE, E_NOMEM.
 */
int fracsolve_solve(fracsolve_t h, const double *const *f, const double *const *u0,
                    const double *const *phi, double *const *u);

/*
 * Operator apply in float64: y[k] <- A u[k], the left-hand side of the block
 * system (no u0/phi terms), i.e. y^n = (a_0 I + K) U^n + sum_{j<n} a_{n-j} U^j.
 * Errors: E_ARG, E_DEVICE.
 */
int fracsolve_apply(fracsolve_t h, const double *const *u, double *const *y);

/*
 * Adjoint of fracsolve_solve for a loss L(U): given g[k] = dL/dU [N][M] and
 * the forward solution u[k], writes dL_df[k] = A^{-T} g[k] [N][M] (the
 * reverse-time, block upper-triangular Toeplitz solve; f enters the
 * right-hand side with identity, so this is dL/df) and, if dL_dgamma is not
 * NULL, dL_dgamma[k] = sum_n <dL_df^n, -rho'_n u0 + psi'_n phi>
 *                       - sum_n sum_{j<=n} a'_{n-j} <dL_df^n, U^j>
 * (f, u0 and phi held fixed; primes are gamma-derivatives).  dL_dgamma is a
 * host array of `count` doubles; when it is requested the call synchronises
 * the stream before returning.  dL_df[k] may equal g[k].
 * Errors: E_ARG, E_DEVICE, E_NOMEM.
 */
int fracsolve_adjoint(fracsolve_t h, const double *const *g, const double *const *u,
                      const double *const *u0, const double *const *phi,
                      double *const *dL_df, double *dL_dgamma);

/*
 * Restarted GMRES(m) on the same system: the iterative method the paper uses
 * for Scheme 4 (section 3.1), a second solver next to fracsolve_solve.  Each
 * step applies the operator of fracsolve_apply (tridiagonal block plus the
 * Toeplitz history, the latter as circulant-embedded FFT products above the
 * crossover and dense products below it), orthogonalises against the basis
 * and updates the Givens-rotated Hessenberg matrix; after m steps (or
 * earlier, once the least-squares residual is at most rtol ||b||_2) the
 * iterate is updated and the residual recomputed from its definition.  The
 * method stops when that residual is at most rtol ||b||_2 or max_iters steps
 * were taken.  b = F - rho_n u0 + psi_n phi is the right-hand side of
 * fracsolve_solve; the arithmetic is float64 whatever the handle's precision.
 */
typedef struct {
    int32_t restart;    /* m, Krylov steps per cycle, 1..512                   */
    int32_t max_iters;  /* total Krylov steps over all cycles, >= 0            */
    double rtol;        /* relative residual target, finite and >= 0           */
    int32_t precond;    /* 0: none (the paper's method); 1: right block-
                           diagonal preconditioner diag(a_0 I + K), i.e. the
                           tridiagonal solve of every time step on its own     */
    int32_t use_guess;  /* 0: start from zero; 1: start from the contents of u */
} fracsolve_gmres_options;

typedef struct {
    int32_t iterations; /* Krylov steps taken                                  */
    int32_t cycles;     /* cycles started (restarts + 1; 0 if none was needed) */
    int32_t converged;  /* 1 if the recomputed residual reached rtol           */
    int32_t reserved;
    double relres;      /* ||b - A u||_2 / ||b||_2 recomputed at the end       */
    double relres_est;  /* the last least-squares estimate of it               */
} fracsolve_gmres_info;

/*
 * Solve every instance (one after another) by GMRES(m): u[k] <- iterate for
 * source f[k] and initial data u0[k], phi[k] (as in fracsolve_solve; NULL
 * entries mean zero).  u[k] may equal f[k].  opts NULL = {30, 1000, 1e-10, 0,
 * 0}.  info (NULL or `count` records, host) receives the outcome per
 * instance; hist (NULL or hist_cap doubles, host) receives instance 0's
 * residual history divided by ||b||_2: hist[0] for the start, hist[j] for the
 * least-squares residual after step j.  The call synchronises the stream
 * (the Hessenberg matrix lives on the host) and holds (m + 1) M N doubles of
 * basis per instance in the handle after the first call.
 * Errors: E_ARG (bad option or field; nothing enqueued), E_NOMEM, E_DEVICE,
 * E_NUMERIC (non-finite basis norm).
 */
int fracsolve_gmres(fracsolve_t h, const double *const *f, const double *const *u0,
                    const double *const *phi, double *const *u,
                    const fracsolve_gmres_options *opts, fracsolve_gmres_info *info,
                    double *hist, int32_t hist_cap);

/*
 * Scheme 1 (section 2, eq. e7): the two-sided fractional ODE
 *   D_t^gamma u + tD_1^gamma u + u = f on (0, 1), u(0) = u(1) = 0, 0<gamma<1,
 * whose matrix is symmetric Toeplitz (Theorem 1): diagonal 1 + 2 mu,
 * distance k: mu (G_k - G_{k-1}), tau = 1/N.  Solved by conjugate gradients
 * (section 2.2); each product goes through the circulant embedding of
 * eq. e10 (one forward and one inverse FFT of L >= 2N - 3 points, a power of
 * two), the paper's fast CG.  f and u are DEVICE arrays of the N - 1 values at t_i = i/N
 * (u may not alias f).  The iteration stops when |r| <= rtol |f| (residual
 * of the recurrence) or after max_iters steps.  opts NULL = {10000, 1e-10,
 * 0}; info (NULL or one record, host); hist (NULL or hist_cap doubles,
 * host): |r_k| / |f| from the recurrence, hist[0] for the start.
 * Work runs on `stream` (NULL = null stream); the call synchronises it and
 * holds its workspace only for its duration: 40 L + 32 (N - 1) bytes of
 * device memory (the spectrum and two complex arrays of L < 4N points, four
 * vectors; about 470 MB at N = 2^22).
 * 3 <= N <= 2^22 + 1.
 * Errors (text in fracsolve_last_error(NULL)): E_ARG, E_NOMEM, E_DEVICE,
 * E_NUMERIC (a direction with <p, A p> <= 0).
 */
typedef struct {
    int32_t max_iters;  /* >= 0                                                */
    double rtol;        /* relative residual target, finite and >= 0           */
    int32_t use_guess;  /* 0: start from zero; 1: from the contents of u       */
} fracsolve_cg_options;

typedef struct {
    int32_t iterations; /* CG steps taken                                      */
    int32_t converged;  /* 1 if the recurrence residual reached rtol           */
    double relres;      /* |f - A u| / |f| recomputed at the end               */
    double relres_est;  /* |r| / |f| of the recurrence                         */
} fracsolve_cg_info;

int fracsolve_ode_cg(double gamma, int64_t N, const double *f, double *u,
                     const fracsolve_cg_options *opts, fracsolve_cg_info *info,
                     double *hist, int32_t hist_cap, void *stream);

/*
 * Scheme 1 by conjugate gradients, as fracsolve_ode_cg, for callers that
 * cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid allocation).  Every workspace (the embedded
 * spectrum, the FFT work arrays, the CG vectors and scalars, the residual
 * history and the reduction partials) lives in one fixed device array of
 * 64 MiB that the library holds on each device it runs on until the process
 * ends; the call allocates nothing and creates no stream or graph (the steps
 * are launched directly on `stream`, whose device must be the current one).
 * Same arguments, results and errors as fracsolve_ode_cg, with two more
 * limits checked before any device work: N <= FRACSOLVE_ODE_NOALLOC_MAX_N and
 * hist_cap <= FRACSOLVE_ODE_NOALLOC_MAX_HIST (E_ARG beyond).  Every call on a
 * device shares that device's array and leaves its contents behind: calls
 * that overlap on one device (two threads, or two streams) race and must be
 * serialised by the caller.  The call synchronises `stream`.
 */
#define FRACSOLVE_ODE_NOALLOC_MAX_N ((int64_t)(1 << 19) + 1)
#define FRACSOLVE_ODE_NOALLOC_MAX_HIST 65536

int fracsolve_ode_cg_noalloc(double gamma, int64_t N, const double *f, double *u,
                             const fracsolve_cg_options *opts, fracsolve_cg_info *info,
                             double *hist, int32_t hist_cap, void *stream);

/*
 * Timing and plan details of the last call, for reporting.  Fields are -1
 * when not measured.  Filled only if timing was enabled with
 * fracsolve_set_timing(h, 1) before the call (it adds events and a
 * synchronisation).
 */
typedef struct {
    int32_t leaf;              /* leaf size used by instance 0                 */
    int32_t crossover;         /* dense/FFT crossover s* of instance 0         */
    int32_t levels;            /* recursion levels of instance 0               */
    int32_t kernels;           /* kernel launches of the last call             */
    double ms_total;           /* wall time of the last call (events)          */
    double ms_leaf;            /* summed leaf-kernel time                      */
    double ms_dense;           /* summed dense-update time                     */
    double ms_fft;             /* summed FFT-update time                       */
    double residual_norm;      /* max |r| of the last refinement residual      */
} fracsolve_stats;

/* on = 0: off; 1: total time and residual norm; 2: also per-kernel-group
 * times (an event pair around every launch; adds overhead). */
int fracsolve_set_timing(fracsolve_t h, int32_t on);

/* Output check (failure detection, off by default).  With on = 1, every
 * later fracsolve_solve, fracsolve_apply and fracsolve_adjoint of the handle
 * scans its output fields (u, y, dL_df; and dL_dgamma) for NaN and
 * infinities after the work and returns FRACSOLVE_E_NUMERIC, naming the
 * field, the instance and the count, if it finds any; the outputs are left
 * as computed.  The scan reads each output once more (8 bytes per unknown)
 * and synchronises the handle's stream.  on = 0 turns it off.  E_ARG for a
 * NULL handle. */
int fracsolve_set_check(fracsolve_t h, int32_t on);
int fracsolve_get_stats(fracsolve_t h, fracsolve_stats *out);

/* Per-kernel-group timing of the last call (timing level 2).  One record per
 * (kind, s): kind 0 = leaf solves (s = leaf size), 1 = dense float64 level
 * products, 2 = dense float32, 3 = FFT float64, 4 = FFT float32, 5 = the
 * near-corner band added after single-pass FFT levels (s = level
 * half-size).  bytes = algorithmic HBM bytes of those launches (reads of X
 * and of the right-hand side, read+write of Y, solution writes).  Writes at
 * most cap records to out and their number to *count. */
typedef struct {
    int32_t kind;
    int32_t s;
    int32_t launches;
    int32_t tasks;
    double ms;
    double bytes;
} fracsolve_kernel_stat;

int fracsolve_kernel_stats(fracsolve_t h, fracsolve_kernel_stat *out, int32_t cap, int32_t *count);

/* Release every device and host resource of the handle.  NULL-safe. */
void fracsolve_destroy(fracsolve_t h);

/* Text of the last error on h (or of the last failed create when h is NULL).
 * The string stays valid until the next call on the same handle. */
const char *fracsolve_last_error(fracsolve_t h);

#ifdef __cplusplus
}
#endif

#endif /* FRACSOLVE_H */
