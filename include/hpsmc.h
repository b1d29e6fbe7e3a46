/*
 * hpsmc.h -- C ABI of the MI355X hot path of the hp-version time-stepping
 * spectral Monte Carlo method for u_t = Lap u + f(u) + s on (-1,1)^d with
 * homogeneous Dirichlet data, and u_t = -(-Lap)^{alpha/2} u + f(u) + s on
 * (-1,1) with u = 0 outside (arXiv 2608.22190).
 *
 * The library estimates, at every space-time node (x_j, t_{n,l}) of an
 * interval, the residual increment eps of eq. varepsilon_1 by Monte Carlo
 * sample paths of the sphere-jump walk (Lemma 2.1, eq. indexL, eq. interIQ),
 * adds it to the nodal values (Algorithm 1, Step 3) and reconstructs the
 * space-time polynomial from the nodal values (Sec. 2.3, eq. u_N) before the
 * next iteration.  Intervals run one after another (Algorithm 1, Step 4), or
 * all together in Jacobi-in-time sweeps.
 *
 * General conventions
 *   - Every call returns hpsmc_status (0 = OK).  No exception or abort crosses
 *     the ABI; hpsmc_last_error() returns a thread-local message.
 *   - Arguments are validated before any device work.  After HPSMC_EDEVICE the
 *     plan must be destroyed.
 *   - Pointers marked "host" are host memory owned by the caller; "device"
 *     pointers are device memory owned by the caller; on_device selects which
 *     for the copy-in / copy-out calls.  The plan owns all other device memory
 *     (allocated in hpsmc_create with hipMalloc or the hpsmc_set_allocator
 *     hooks, freed in hpsmc_destroy).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     work and return; copy-out calls to host memory synchronize the stream.
 *   - Spatial nodes: the n-point Jacobi-Gauss (1,1) rule per dimension
 *     (Sec. 2.3), node index j = C-order over (j_0, ..., j_{d-1}).  Temporal
 *     nodes: the M_n+1 shifted Legendre-Gauss-Lobatto points of interval n
 *     (Sec. 2.1); l = 0 is t_{n-1}.  Nodal arrays are [instance][j][l].
 *   - Monte Carlo node id of (j, l >= 1): j + n^d (l - 1).
 *   - Random numbers: Philox4x32-10 with key (lo32(seed), hi32(seed)) and
 *     counter (node id, sample, step block, instance<<16 | interval<<8 | tag),
 *     tag = iteration (or sweep) index when fresh_per_iter, else 0.  d = 1 uses
 *     one bit per step (128 steps per block), d = 2 one word (4 steps per
 *     block), d = 3, 4 one block per step, d = 5 two blocks per step; the
 *     fractional walk (d = 1) two words per step (2 steps per block); the
 *     ball-point rule draws from step blocks with bit 31 set.
 *   - Variants of the method selected per plan (hpsmc_problem): the estimator
 *     (residual form, eq. varepsilon_1, or the Picard form, eq. uast), the
 *     update (plain, or Aitken-relaxed), the path quadrature (centre point,
 *     eq. interIQ, or the Green's-function ball point), and the order of the
 *     operator (the Laplacian, or the fractional Laplacian in 1-D).
 */
#ifndef HPSMC_H
#define HPSMC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HPSMC_OK = 0,
    HPSMC_EINVAL = -1,     /* invalid argument (nothing was enqueued)          */
    HPSMC_ENOTSUP = -2,    /* valid but unsupported (e.g. nonzero boundary data) */
    HPSMC_ENOMEM = -3,     /* device or host allocation failed                  */
    HPSMC_EDEVICE = -4,    /* a HIP call failed; the plan is poisoned           */
    HPSMC_EDIVERGED = -5,  /* tolerance mode: max|eps| non-finite, or grew in
                              three consecutive iterations; iterates readable   */
    HPSMC_ENOTCONVERGED = -6 /* tolerance mode: some interval used all `iters`
                              iterations with max|eps| >= tol (informational:
                              the results are valid)                            */
} hpsmc_status;

/* nonlinearity f(u) of eq. mainproblem */
enum { HPSMC_F_AFFINE = 0,        /* f = a u + b, f_param = {a, b} */
       HPSMC_F_U_MINUS_U3 = 1,    /* u - u^3   */
       HPSMC_F_SIN = 2,           /* sin u     */
       HPSMC_F_U2_OVER_1PU2 = 3,  /* u^2/(1+u^2) */
       HPSMC_F_NEG_U3 = 4,        /* -u^3      */
       HPSMC_F_U_SIN_U = 5 };     /* u sin u (Ex. 1) */

/* manufactured source: s = u_t - Lap u - f(u) of an exact solution u_ex */
enum { HPSMC_SRC_NONE = 0,        /* s = 0 */
       HPSMC_SRC_SIN_DECAY = 1,   /* u_ex = e^{-t} prod sin(pi x_i)   */
       HPSMC_SRC_COS_DECAY = 2,   /* u_ex = e^{-t} prod cos(pi x_i/2) */
       HPSMC_SRC_LONGTIME = 3,    /* u_ex = prod(1-x_i^2) sin(sum x_i) e^{cos t}/(1+t^2) */
       HPSMC_SRC_QUAD = 4,        /* u_ex = prod(1-x_i^2)(c0 + c1 t + c2 t^2), src_param = {c0,c1,c2} */
       /* fractional operator only (0 < alpha < 2, d = 1), u_ex = (1-x^2)_+^{alpha/2} g(x) T(t),
          source s = u_t + (-Delta)^{alpha/2} u - f(u) (Ex. 2-3): */
       HPSMC_SRC_FRAC_LONGTIME = 5, /* g = sin x, T = e^{cos t}/(1+t^2)                   */
       HPSMC_SRC_FRAC_SINGULAR = 6, /* g = cos(x^3+1)/(10x^2+1), T = t^rho, rho = src_param[0] */
       HPSMC_SRC_FRAC_POLY = 7,     /* g = p0 + p1 x + p2 x^2, T = 1 + c t,
                                       src_param = {p0, p1, p2, c}                         */
       /* a given polynomial source (the Laplacian only): per interval a tensor-Legendre
          polynomial of P = n+2 modes per dimension and degree M_n in time (src_coeffs,
          src_len); it enters the time contraction of v* = Lap u* - d_t u*, so a path
          step costs no more; no exact solution (no IC_EXACT); residual form only */
       HPSMC_SRC_POLY = 8 };

/* initial data */
enum { HPSMC_IC_EXACT = 0,        /* u_ex(x, t_0) of the source's exact solution */
       HPSMC_IC_SINGULAR = 1,     /* prod(1-x_i^2) |x_0|^a, ic_param = {a}        */
       HPSMC_IC_PHI = 2,          /* sum_p c_p prod phi_{p_i}(x_i), ic_data = c [instance][n^d] */
       HPSMC_IC_NODAL = 3 };      /* nodal values, ic_data [instance][n^d]        */

enum { HPSMC_SEQUENTIAL = 0,      /* Algorithm 1: intervals one after another     */
       HPSMC_SWEEPS = 1 };        /* every sweep updates all intervals; interval n
                                     takes its initial column from interval n-1's
                                     last column of the previous sweep            */

enum { HPSMC_EST_RESIDUAL = 0,    /* eq. varepsilon_1: the Monte Carlo estimate of the
                                     residual increment eps, added to the iterate  */
       HPSMC_EST_PICARD = 1 };    /* eq. uast: the Picard (classical Monte Carlo) form
                                     -- integrand f(u*) + s, plus the interval's
                                     initial data at the end point of paths that stay
                                     inside for all N* steps; the estimate replaces
                                     the iterate (eps = its change).  Vector-unit
                                     round kernel only; no gradient               */

enum { HPSMC_ACCEL_NONE = 0,      /* Algorithm 1's update: U += eps               */
       HPSMC_ACCEL_AITKEN = 1 };  /* the acceleration remark after Algorithm 1:
                                     Aitken's delta-squared extrapolation as a
                                     weighted average, U += w eps, per (instance,
                                     interval) vector of node values, with
                                     w = omega[0] on its first iteration, then
                                     w = -w_prev <e_prev, e - e_prev> / |e - e_prev|^2
                                     (w_prev when the denominator is 0), clipped to
                                     [omega[1], omega[2]]; e is the estimator's
                                     change (eps).  The history restarts at
                                     hpsmc_start_interval, at the start of every
                                     solve, and after hpsmc_set_nodes of the
                                     interval.  No gradient                       */

enum { HPSMC_QUAD_CENTRE = 0,     /* eq. interIQ: a walk step adds Delta * r at its
                                     ball centre X_q                               */
       HPSMC_QUAD_BALL = 1 };     /* the path-integral representation of a step in
                                     the error analysis (Sec. 3): Delta * r(Y_q) with
                                     Y_q drawn in the ball B_J(X_q) from the
                                     normalized Green's function of -Laplace with
                                     pole at X_q (Y_q = X_q + J sqrt(U_a) U_b^{1/d}
                                     theta, theta uniform; Philox counter word 2
                                     with bit 31 set, 2q and, for d >= 3, 2q+1).
                                     Y_q may lie outside Omega.  Vector-unit round
                                     kernel only; no gradient                     */

/* path lengths N* of the node times (eq. time division: N* depends on h_n and
 * on l).  A rule gives N*_{n,l} = max(nstar_min, ceil((t_{n,l} - t_{n-1}) /
 * Delta_max)) with the same Delta_max for every node time of interval n: */
enum { HPSMC_NSTAR_ARRAY = 0,     /* the `nstar` array, one entry per node time    */
       HPSMC_NSTAR_DT = 1,        /* Delta_max = dt_max                            */
       HPSMC_NSTAR_SPECTRAL = 2 };/* Delta_max = nstar_c / rho(A_h) per interval,
                                     rho the spectral radius of the interval's
                                     discrete operator A_h = d_t - Lap_h (or
                                     d_t + (-Lap)^{alpha/2}_h) on the nodal values
                                     of l >= 1 (the residual estimator scales an
                                     error mode of eigenvalue lambda by about
                                     1 - Delta lambda per iteration), computed at
                                     set-up                                       */

enum { HPSMC_FP64 = 0,            /* everything in FP64                            */
       HPSMC_FP32_SAMPLING = 1,   /* paths and basis evaluation in FP32 with
                                     compensated accumulation; reconstruction,
                                     increments, norms and stop test in FP64      */
       HPSMC_FP32_THEN_FP64 = 2 };/* hpsmc_solve samples an interval (a sweep) in
                                     FP32 until max|eps| < switch_tol, then goes on
                                     in FP64 with the same counter tags (iteration
                                     k draws the Philox words a plain FP64 solve
                                     draws at k): FP32's throughput for the early
                                     iterations, FP64's accuracy floor at the end.
                                     The host reads max|eps| after every
                                     iteration.  hpsmc_iterate / hpsmc_sweep run
                                     in FP32; residual form, no Aitken relaxation,
                                     no gradient                                  */

typedef struct {
    int32_t dim;               /* 1..5, Omega = (-1,1)^dim                      */
    int32_t n;                 /* spatial nodes per dimension, 1..32            */
    int32_t n_intervals;       /* N_h, 1..255                                   */
    int32_t n_instances;       /* independent problems sharing the grid, 1..65535 */
    const double *t_breaks;    /* host, N_h+1 strictly increasing               */
    const int32_t *degree;     /* host, N_h entries M_n in 1..31                */
    const int32_t *nstar;      /* host, sum_n M_n entries: N* of node time l>=1
                                  of interval n (eq. time division), 1..2^24-1;
                                  read only with nstar_mode HPSMC_NSTAR_ARRAY  */
    int32_t f_kind, src_kind, ic_kind, schedule;
    double f_param[4], src_param[8], ic_param[4];
    const double *ic_data;     /* host, [instance][n^d] for IC_PHI / IC_NODAL   */
    int64_t M;                 /* samples per node, >= 1                        */
    int32_t iters;             /* iterations per interval, or sweeps, 1..255    */
    int32_t fresh_per_iter;    /* 1: new samples each iteration, 0: reuse       */
    uint64_t seed;
    int32_t precision;         /* HPSMC_FP64 or HPSMC_FP32_SAMPLING            */
    int32_t estimator;         /* HPSMC_EST_RESIDUAL (default) or HPSMC_EST_PICARD */
    double tol;                /* 0: exactly `iters` iterations per interval (or
                                  sweeps), asynchronous.  > 0: Algorithm 1's loop
                                  condition -- an interval stops once max|eps| <
                                  tol (at most `iters`); the host reads max|eps|
                                  after every iteration, so hpsmc_solve runs
                                  eagerly even with the "graph" option          */
    int32_t accel;             /* HPSMC_ACCEL_NONE (default) or HPSMC_ACCEL_AITKEN */
    int32_t quad;              /* HPSMC_QUAD_CENTRE (default) or HPSMC_QUAD_BALL  */
    double omega[3];           /* Aitken: first weight, lower and upper bound;
                                  0 selects 1, 0.5, 2; need 0 < omega[1] <=
                                  omega[0] <= omega[2] after the defaults       */
    double alpha;              /* order of the operator: 0 or 2 the Laplacian;
                                  0 < alpha < 2 the fractional Laplacian
                                  (-Delta)^{alpha/2} with u = 0 outside Omega
                                  (Ex. 2-3): d = 1, spatial nodes Gauss-Jacobi
                                  (alpha/2, alpha/2), basis (1-x^2)^{alpha/2}
                                  P_p^{(alpha/2,alpha/2)}, p < n, the alpha-stable
                                  walk (jumps from the exit law of a ball whose
                                  mean exit time is Delta).  Residual or Picard
                                  form, centre-point rule, initial data IC_EXACT
                                  or IC_NODAL; no gradient, no hpsmc_eval or
                                  hpsmc_get_coeffs                              */
    int32_t nstar_mode;        /* HPSMC_NSTAR_ARRAY (default), _DT or _SPECTRAL  */
    int32_t nstar_min;         /* rules: smallest N* (0 selects 4)              */
    double nstar_c;            /* HPSMC_NSTAR_SPECTRAL: Delta_max = nstar_c/rho
                                  (0 selects 0.25)                              */
    double dt_max;             /* HPSMC_NSTAR_DT: Delta_max, > 0                 */
    const double *src_coeffs;  /* HPSMC_SRC_POLY: host, the source's tensor-Legendre
                                  coefficients, per interval n a block
                                  [k_0..k_{d-1}][q] of P^d (M_n+1) values (P = n+2
                                  modes per dimension), s(x, t) = sum c
                                  prod_i L_{k_i}(x_i) L_q(xi), xi = 2(t -
                                  t_{n-1})/h_n - 1; shared by all instances      */
    int64_t src_len;           /* HPSMC_SRC_POLY: sum_n P^d (M_n+1)             */
    double switch_tol;         /* HPSMC_FP32_THEN_FP64: max|eps| below which the
                                  solve continues in FP64, > 0                  */
} hpsmc_problem;

typedef struct hpsmc_plan hpsmc_plan;

/* Device-memory hooks (hpsmc_set_allocator): bytes >= 1; stream is the stream
 * the plan is created or used on (NULL: the default stream); ctx is passed
 * through.  alloc returns NULL on failure. */
typedef void *(*hpsmc_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*hpsmc_free_fn)(void *ptr, void *stream, void *ctx);

typedef struct {
    uint64_t path_steps;       /* residual evaluations (sum of L over paths)     */
    uint64_t lane_steps;       /* walk steps executed by all sample slots        */
    uint64_t node_samples;     /* (node, sample) estimates                       */
    int32_t n_records;         /* entries filled in max_eps                      */
    int32_t status_flags;      /* bit 0: non-finite increment seen; bit 1: max|eps|
                                  grew in three consecutive iterations of one
                                  interval (divergence, any mode)                */
    int32_t sample_launches;   /* sampling-kernel launches timed (one per round) */
    int32_t recon_launches;    /* reconstructions timed                         */
    double sample_ms;          /* summed duration of those launches (HIP events
                                  on the launching stream), milliseconds        */
    double sampling_span_ms;   /* summed span of whole sampling phases (rounds,
                                  their prep kernels and launch gaps)           */
    double recon_ms;           /* summed reconstruction time (all its kernels)   */
    double slab_ms;            /* summed time-contraction (slab) kernel time     */
    int64_t advance_launches;  /* path-advancing kernel launches, timed or not   */
    double max_eps[4096];      /* max|eps| per (interval, iteration) or sweep    */
    int64_t adjoint_launches;  /* adjoint-kernel launches timed                 */
    double adjoint_ms;         /* their summed duration (HIP events), ms         */
} hpsmc_stats_t;

/* Sampling-kernel launch shape (chosen by hpsmc_tune or set directly). */
typedef struct {
    int32_t samples_per_lane;  /* 1, 2 or 4 (4 only for dim <= 2); plans with the
                                  Picard form, the ball-point rule or the
                                  fractional operator run 1 whatever is set     */
    int32_t waves_per_block;   /* 1..4                                            */
    int32_t blocks_per_cu;     /* persistent grid = CUs * blocks_per_cu          */
    int32_t round_steps;       /* walk steps per round of the path-advancing
                                  kernel (multiple of 4 in 16..4096; 0 keeps
                                  the current value)                             */
} hpsmc_launch;

/* Install the allocator that plans created afterwards use for every device
 * workspace they own (for example a framework's caching allocator); both
 * NULL restores hipMalloc / hipFree.  A plan keeps the hooks it was created
 * with until hpsmc_destroy.  EINVAL when exactly one hook is NULL.
 * Process-wide; thread-safe. */
hpsmc_status hpsmc_set_allocator(hpsmc_alloc_fn alloc, hpsmc_free_fn free_, void *ctx);

/* Validate the problem, compute the grid and transform matrices on the host,
 * allocate device memory, and write the initial iterate (the initial column
 * replicated in time, for interval 0 or for all intervals under SWEEPS).
 * The set-up of Sec. 2.1 and 2.3: the Jacobi-Gauss nodes, the shifted Lobatto
 * nodes of every interval, the nodal-to-modal matrices of eqs. spacelag and
 * timeLag, the path lengths of eq. time division (resolved here when a rule
 * is selected), and Algorithm 1's initial guess.
 * EINVAL on any out-of-range field; ENOTSUP for unsupported combinations. */
hpsmc_status hpsmc_create(const hpsmc_problem *pb, hpsmc_plan **out);
void hpsmc_destroy(hpsmc_plan *plan);

/* Resolve the path lengths of a problem without a plan or a device (the rule
 * that hpsmc_create applies, eq. time division): nstar (host, sum_n M_n
 * entries) receives N* of every node time l >= 1 of every interval, dt_max
 * (host, n_intervals entries, may be NULL) the rule's Delta_max per interval
 * (0 for HPSMC_NSTAR_ARRAY).  Validates the problem like hpsmc_create; EINVAL
 * also when the rule gives N* >= 2^24. */
hpsmc_status hpsmc_resolve_nstar(const hpsmc_problem *pb, int32_t *nstar, double *dt_max);

/* The plan's resolved path lengths, as hpsmc_resolve_nstar returns them. */
hpsmc_status hpsmc_get_nstar(const hpsmc_plan *plan, int32_t *nstar, double *dt_max);

/* Spatial nodes (n, host) and temporal nodes of interval iv (M_iv+1, host). */
hpsmc_status hpsmc_grid(const hpsmc_plan *plan, int32_t iv, double *x_nodes, double *t_nodes);

/* Whole solve: Algorithm 1 (or the sweeps), `iters` iterations each, or with
 * tol > 0 until max|eps| < tol per interval (then EDIVERGED / ENOTCONVERGED
 * as described at hpsmc_status). */
hpsmc_status hpsmc_solve(hpsmc_plan *plan, void *stream);

/* Start interval iv (SEQUENTIAL): column 0 = initial data (iv = 0) or the last
 * column of interval iv-1 (Algorithm 1, Step 4), replicated to every column. */
hpsmc_status hpsmc_start_interval(hpsmc_plan *plan, int32_t iv, void *stream);

/* One residual iteration on interval iv with counter tag `tag`: reconstruct,
 * time-contract, sample every node, reduce, update (Algorithm 1, Steps 1-3). */
hpsmc_status hpsmc_iterate(hpsmc_plan *plan, int32_t iv, int32_t tag, void *stream);

/* One sweep over all intervals (SWEEPS) with counter tag `tag`. */
hpsmc_status hpsmc_sweep(hpsmc_plan *plan, int32_t tag, void *stream);

/* Copy nodal values of interval iv out of / into the plan, [instance][j][l]. */
hpsmc_status hpsmc_get_nodes(const hpsmc_plan *plan, int32_t iv, double *out, int32_t on_device, void *stream);
hpsmc_status hpsmc_set_nodes(hpsmc_plan *plan, int32_t iv, const double *in, int32_t on_device, void *stream);

/* Last increment of interval iv: eps and sum of S^2 per node, [instance][node id]
 * (host).  eps is the Monte Carlo average of eq. varepsilon_1 over the M sample
 * paths of each node (the per-path values S_i of eq. interIQ); sum S_i^2 gives
 * the node's standard error sqrt((sumsq/M - eps^2)/M).  Synchronizes the stream. */
hpsmc_status hpsmc_get_increment(const hpsmc_plan *plan, int32_t iv, double *eps, double *sumsq, void *stream);

/* Evaluate the current reconstruction of interval iv at npts points
 * pts[k] = (x_0..x_{d-1}, t) (host): out[k] = (u, Lap u - d_t u) (host) --
 * the approximation u* of eq. u_N built from the nodal values the last
 * iteration started from, and the operator part of the residual of eq. ufg_ep1
 * (no nonlinearity, no source).  ENOTSUP for the fractional operator.
 * Allocates two staging buffers per call (hpsmc_eval_noalloc does not). */
hpsmc_status hpsmc_eval(hpsmc_plan *plan, int32_t iv, int32_t inst, const double *pts, int64_t npts,
                        double *out, void *stream);

/* hpsmc_eval for callers that cannot allocate device memory (serving loops,
 * harnesses that forbid hipMalloc): the same arguments, layouts and results,
 * but the points and values are staged in a static 16 MiB device array
 * instead of per-call allocations -- no hipMalloc, hipFree or other
 * allocating call.  Each GPU holds its own copy of the array until the
 * process ends; the current device must be the plan's.  npts * (dim + 3)
 * doubles must fit in 16 MiB (npts <= 524288 for dim = 1, 262144 for dim = 5),
 * else EINVAL before any device work.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other threads or streams) race
 * and must be serialized by the caller.  Synchronizes the stream. */
hpsmc_status hpsmc_eval_noalloc(hpsmc_plan *plan, int32_t iv, int32_t inst, const double *pts, int64_t npts,
                                double *out, void *stream);

/* Keep the per-sample values S_i of samples i < m_probe of every node of the
 * next iterations (0 disables); read them as [instance][node id][i]. */
hpsmc_status hpsmc_set_probe(hpsmc_plan *plan, int64_t m_probe);
hpsmc_status hpsmc_get_probe(const hpsmc_plan *plan, int32_t iv, double *out, void *stream);

/* Sampling-kernel launch shape. */
hpsmc_status hpsmc_set_launch(hpsmc_plan *plan, const hpsmc_launch *l);
hpsmc_status hpsmc_get_launch(const hpsmc_plan *plan, hpsmc_launch *l);

/* Autotuner: time every candidate launch shape on one iteration of interval iv
 * with samples limited to m_tune per node, keep the fastest (and cache it in
 * the JSON file `cache_path` if not NULL). */
hpsmc_status hpsmc_tune(hpsmc_plan *plan, int32_t iv, int64_t m_tune, const char *cache_path, void *stream);

/* Counters accumulated since creation or the last reset (synchronizes): the
 * residual evaluations (the sum of the exit indices L of eq. indexL over all
 * paths), the walk steps executed, and max|eps| per iteration -- the quantity
 * of Algorithm 1's loop condition.  A solve overwrites the records it writes
 * (record iv * iters + k of a sequential solve, k of a sweep solve). */
hpsmc_status hpsmc_stats(const hpsmc_plan *plan, hpsmc_stats_t *out, void *stream);
hpsmc_status hpsmc_reset_stats(hpsmc_plan *plan, void *stream);

/* Terminal misfit of a single-interval problem with IC_PHI initial data:
 * loss[i] = 1/2 sum_j (u_i(x_j, T) - target[i][j])^2 after `iters`
 * iterations, and grad[i] = d loss[i] / d c_i (the phi-coefficients) by the
 * adjoint of the iteration with every sample path fixed (common random
 * numbers; the paths are regenerated from their Philox counters).
 * target, loss, grad: host or device per on_device.  Runs the forward solve. */
hpsmc_status hpsmc_loss_grad_c0(hpsmc_plan *plan, const double *target, double *loss, double *grad,
                                int32_t on_device, void *stream);

/* Replace the initial data by nodal values u0 [instance][n^d] at the spatial
 * nodes (host or device per on_device); the next start of interval 0 (or of
 * every interval under SWEEPS) uses them: u(x, 0) = u_0 of eq. mainproblem,
 * entering as column 0 of the first interval (Algorithm 1, Step 4 hands the
 * last column on from there).  EINVAL for IC_PHI plans (use
 * hpsmc_set_initial_coeffs there).  Synchronizes the stream. */
hpsmc_status hpsmc_set_initial_nodes(hpsmc_plan *plan, const double *u0, int32_t on_device, void *stream);

/* The current iterate of interval iv in the basis of Sec. 2.3 (eq. u_N):
 * out [instance][p_1..p_d][q] = coefficient of prod_i phi_{p_i}(x_i) L_q(xi),
 * p_i in 0..n-1, q in 0..M_iv, i.e. U x_i A x_t B with the nodal-to-modal
 * matrices of eqs. spacelag / timeLag.  out: host or device per on_device;
 * synchronizes the stream. */
hpsmc_status hpsmc_get_coeffs(hpsmc_plan *plan, int32_t iv, double *out, int32_t on_device, void *stream);

/* Replace the phi-coefficients of IC_PHI initial data, [instance][n^d] (host or
 * device per on_device); the next start of interval 0 uses them.  EINVAL
 * when the plan's initial data are not phi-coefficients. */
hpsmc_status hpsmc_set_initial_coeffs(hpsmc_plan *plan, const double *c0, int32_t on_device, void *stream);

/* Named integer options:
 *   "adjoint_mfma"      1 (default): FP32 adjoint outer products on the matrix
 *                       cores; 0: on the vector units.
 *   "sample_mfma"       1 (default): 2-D FP32 plans with P = n + 2 <= 32 and one
 *                       sample per lane run the path-advancing kernel with the
 *                       slab contraction of eq. ufg_ep1 on the matrix cores
 *                       (v_mfma_f32_32x32x2f32) -- the residual and Picard
 *                       forms, the centre-point and ball-point rules (plans of
 *                       the Picard form or the ball rule count as one sample
 *                       per lane); so do 5-D FP32 plans of the residual form
 *                       with the centre-point rule, P <= 12 and one sample per
 *                       lane (the innermost two modes of the contraction as
 *                       matrix-core products); 0: always on the vector units.
 *                       Same walks and exit steps either way; the FP32 sums
 *                       differ only by rounding order.  Changing it discards a
 *                       captured graph.
 *   "sample_split"      1 (default): in a round of the 5-D matrix-core kernel
 *                       whose live paths fit in one pass of the grid at 64
 *                       paths per block, the block's two or four waves walk the
 *                       same 64 paths and share each step's products (shorter
 *                       rounds when few long paths remain); 0: never.  The
 *                       FP32 sums differ only by rounding order.
 *   "sample_1d"         1 (default): d = 1 rounds of the residual form with
 *                       the centre-point rule run the windowed 1-D kernel (the
 *                       slabs of 32 walk steps staged in LDS per barrier, the
 *                       same walk and arithmetic as the general kernel); 0: the
 *                       general vector-unit kernel.
 *   "sample_1d_active"  read-only: 1 when the rounds run the windowed 1-D
 *                       kernel with the current launch shape.
 *   "graph"            1: hpsmc_solve captures the whole solve into a hipGraph
 *                       on its first call (on a stream of the plan) and replays
 *                       it on this and later calls; 0 (default): eager launches.
 *                       A new launch shape discards the captured graph.
 * EINVAL for an unknown name or value. */
hpsmc_status hpsmc_set_option(hpsmc_plan *plan, const char *name, int64_t value);

/* Read a named option into *value: the names above, and the read-only
 * "sample_mfma_active": 0 when the current launch shape runs no matrix-core
 * path-advancing kernel, 1 the 2-D one, 2 the 5-D one.  EINVAL for an
 * unknown name. */
hpsmc_status hpsmc_get_option(const hpsmc_plan *plan, const char *name, int64_t *value);

const char *hpsmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
