/*
 * hpsmc_oracle.h -- plain CPU FP64 oracle of the hp-version time-stepping
 * spectral Monte Carlo method (Feng, Hui, Sheng, Xu, arXiv 2608.22190).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only tests/, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no source with the GPU path.
 *
 * Every routine follows the paper's definitions in the paper's order, in FP64,
 * without blocking, fusion or reordering beyond what the definition states.
 * The readings taken where the paper is silent or garbled are listed in the
 * repository design notes (readings R1..R25) and repeated at each use.
 *
 * Conventions (shared with the GPU path only through the published problem
 * statement, never through code):
 *   - Omega = (-1,1)^d, d = 1..5, homogeneous Dirichlet data (g = 0).
 *   - spatial nodes: the n-point Jacobi-Gauss (1,1) rule per dimension
 *     (Sec. 2.3, eq. spacelag); node index j_flat = C-order over (j_0..j_{d-1}).
 *   - temporal nodes on interval n: shifted LGL, ell = 0..M_n (Sec. 2.1).
 *   - nodal array of one interval: U[j_flat*(M_n+1) + ell].
 *   - modal array (phi x Legendre): Ut[p_flat*(M_n+1) + q], p_flat C-order.
 *   - Philox counter of a path (reading R22):
 *       c0 = j_flat + n^d*(ell-1), c1 = sample, c2 = step block,
 *       c3 = (instance << 16) | (interval << 8) | iteration_tag,
 *     key = (lo32(seed), hi32(seed)).
 *
 * Status codes: 0 ok, -1 invalid argument, -2 not supported, -3 no memory.
 */
#ifndef HPSMC_ORACLE_H
#define HPSMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* nonlinearity f(u) (problem statement, eq. mainproblem) */
enum { OR_F_AFFINE = 0,        /* f = a*u + b, f_param = {a, b}        */
       OR_F_U_MINUS_U3 = 1,    /* f = u - u^3                           */
       OR_F_SIN = 2,           /* f = sin(u)                            */
       OR_F_U2_OVER_1PU2 = 3,  /* f = u^2/(1+u^2)                       */
       OR_F_NEG_U3 = 4,        /* f = -u^3                              */
       OR_F_U_SIN_U = 5 };     /* f = u*sin(u)                          */

/* manufactured source s(x,t) so that u_t = Lap u + f(u) + s holds exactly */
enum { OR_SRC_NONE = 0,        /* s = 0                                              */
       OR_SRC_SIN_DECAY = 1,   /* u_ex = exp(-t) prod sin(pi x_i)                    */
       OR_SRC_COS_DECAY = 2,   /* u_ex = exp(-t) prod cos(pi x_i / 2)                */
       OR_SRC_LONGTIME = 3,    /* u_ex = prod(1-x_i^2) sin(sum x_i) e^{cos t}/(1+t^2) */
       OR_SRC_QUAD = 4,        /* u_ex = prod(1-x_i^2) (c0 + c1 t + c2 t^2), src_param = {c0,c1,c2} */
       /* fractional operator (alpha in (0,2), d = 1), u_ex = (1-x^2)_+^{alpha/2} g(x) T(t): */
       OR_SRC_FRAC_LONGTIME = 5, /* g = sin x, T = e^{cos t}/(1+t^2) (Ex. 2)             */
       OR_SRC_FRAC_SINGULAR = 6, /* g = cos(x^3+1)/(10x^2+1), T = t^rho, rho = src_param[0] (Ex. 3) */
       OR_SRC_FRAC_POLY = 7,     /* g = p0 + p1 x + p2 x^2, T = 1 + c t, src_param = {p0,p1,p2,c} */
       OR_SRC_POLY = 8 };        /* s given per interval n by tensor-Legendre coefficients
                                    src_coeffs: block n (after the blocks of the intervals
                                    before it) holds c[k_1..k_d][q], k_i < n+2, q <= M_n, and
                                    s(x, t) = sum c prod_i L_{k_i}(x_i) L_q(xi),
                                    xi = 2 (t - t_{n-1}) / h_n - 1; no exact solution        */

/* initial data u0 */
enum { OR_IC_EXACT = 0,        /* u0 = u_ex(x, 0) of the source's exact solution     */
       OR_IC_SINGULAR = 1,     /* u0 = prod(1-x_i^2) |x_0|^a, ic_param = {a}          */
       OR_IC_PHI = 2,          /* u0 = sum_p c_p prod phi_{p_i}(x_i), ic_data = c    */
       OR_IC_NODAL = 3 };      /* u0 given at the spatial nodes, ic_data = values    */

enum { OR_SCHED_SEQUENTIAL = 0, OR_SCHED_SWEEPS = 1 };

typedef struct {
    int32_t dim, n, n_intervals, n_instances;
    const double *t_breaks;   /* n_intervals+1, strictly increasing            */
    const int32_t *degree;    /* n_intervals entries M_n >= 1                   */
    const int32_t *nstar;     /* sum_n M_n entries: N* of (interval n, ell>=1)  */
    int32_t f_kind, src_kind, ic_kind, schedule;
    double f_param[4], src_param[8], ic_param[4];
    const double *ic_data;    /* [instance][n^d] for OR_IC_PHI / OR_IC_NODAL    */
    int64_t M;                /* samples per node                               */
    int32_t iters;            /* iterations per interval (or sweeps)            */
    int32_t fresh_per_iter;   /* 1: iteration tag in the counter, 0: tag = 0    */
    uint64_t seed;
    int32_t estimator;        /* OR_EST_RESIDUAL or OR_EST_PICARD               */
    int32_t accel;            /* OR_ACCEL_NONE or OR_ACCEL_AITKEN               */
    int32_t quad;             /* OR_QUAD_CENTRE or OR_QUAD_BALL                 */
    double omega[3];          /* Aitken: first weight, lower and upper bound of
                                 the weight; a zero entry selects 1, 0.5, 2     */
    double alpha;             /* order of the operator: 2 (or 0) the Laplacian;
                                 (0,2) the fractional Laplacian (-Delta)^{alpha/2}
                                 with the alpha-stable walk, d = 1 only         */
    const double *src_coeffs; /* OR_SRC_POLY: sum_n (n+2)^d (M_n+1) coefficients  */
    int64_t src_len;
} or_problem;

/* acceleration of the fixed-point iteration (the remark after Algorithm 1):
 * none, or Aitken's delta-squared extrapolation in relaxation form */
enum { OR_ACCEL_NONE = 0, OR_ACCEL_AITKEN = 1 };

/* path quadrature of one walk step: the integrand at the ball centre X_q
 * (eq. interIQ), or at a point Y_q drawn in the ball B_r(X_q) from the
 * normalized Green's function density Q_r (the path-integral representation
 * of the error analysis, Sec. 3), with the same weight Delta = W(X_q) */
enum { OR_QUAD_CENTRE = 0, OR_QUAD_BALL = 1 };

/* estimators: eq. varepsilon_1 (the residual increment, added to the iterate)
 * or eq. uast (the Picard form: the iterate itself, replacing it) */
enum { OR_EST_RESIDUAL = 0, OR_EST_PICARD = 1 };

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* orthogonal polynomials (Sec. 2.3) */
double or_legendre(int k, double x);
double or_legendre_deriv(int k, double x);
double or_jacobi11(int p, double x);
double or_phi(int p, double x);

/* quadrature rules (Sec. 2.1, 2.3) */
int or_jg11(int n, double *x, double *w);
int or_lgl(int M, double *xi, double *w);

/* transform matrices: A[p*n+j] (eq. spacelag), B[q*(M+1)+k] (eq. timeLag) */
int or_matrix_A(int n, double *A);
int or_matrix_B(int M, double *B);

/* nodal -> modal (eq. u_N): Ut = U x_1 A ... x_d A x_t B */
int or_reconstruct(int dim, int n, int M, const double *U, double *Ut);

/* evaluate u*, d_t u*, Lap u* at (X, xi) with xi the reference time in [-1,1];
 * h is the interval length (d_t = (2/h) d_xi).  out = {u, u_t, lap u}. */
int or_eval(int dim, int n, int M, double h, const double *Ut,
            const double *X, double xi, double out[3]);

/* residual integrand r = f(u*) + s - d_t u* + Lap u* (eq. ufg_ep1) */
double or_residual(const or_problem *pb, int interval, const double *Ut,
                   const double *X, double tau);

/* nonlinearity, its derivative, the source and the exact solution */
double or_f(const or_problem *pb, double u);
double or_fprime(const or_problem *pb, double u);
double or_source(const or_problem *pb, const double *X, double t);
double or_exact(const or_problem *pb, const double *X, double t);

/* spatial nodes and the temporal nodes of an interval */
int or_grid(const or_problem *pb, int interval, double *x_nodes, double *t_nodes);

/* initial nodal values of one instance, n^d entries */
int or_ic_nodes(const or_problem *pb, int inst, double *u0);

/* fractional operator (Ex. 2-3): Gauss-Jacobi (a,a) nodes and weights
 * (weight (1-x^2)^a), the symmetric Jacobi polynomial P_p^{(a,a)}, the
 * eigenvalue of (-Delta)^{alpha/2} on the generalized Jacobi function
 * (1-x^2)_+^{alpha/2} P_p^{(alpha/2,alpha/2)}, the regularized incomplete beta
 * function and its inverse, the jump of the alpha-stable walk */
int or_gauss_jacobi(int n, double a, double *x, double *w);
double or_jacobi_aa(int p, double a, double x);
double or_frac_lambda(int p, double alpha);
double or_ibeta(double x, double a, double b);
double or_ibeta_inv(double y, double a, double b);
double or_frac_jump(double alpha, double delta, double omega);
/* nodal -> modal for the fractional basis (d = 1): Ut[p][q] with
 * u = (1-x^2)^{alpha/2} sum Ut[p][q] P_p^{(a,a)}(x) L_q(xi) */
int or_frac_reconstruct(double alpha, int n, int M, const double *U, double *Ut);
/* u*, d_t u*, -(-Delta)^{alpha/2} u* at (x, xi) */
int or_frac_eval(double alpha, int n, int M, double h, const double *Ut, double x, double xi, double out[3]);

/* the ball point of walk step q of a path as an offset in the unit ball
 * (Y_q = X_q + J * offset), OR_QUAD_BALL's law */
int or_ball_offset(const or_problem *pb, int inst, int interval, int iter_tag, int64_t node,
                   int64_t sample, int64_t q, double *offset);

/* one sample path of the residual estimator (eq. interIQ, eq. varepsilon_1):
 * returns S = Delta * sum_{q<L} r(X_q, tau_q); *L_out = L. */
double or_sample_path(const or_problem *pb, const double *Ut, int inst, int interval,
                      int iter_tag, int64_t node, int64_t sample, int64_t *L_out);

/* Monte Carlo residual at a list of nodes (node ids c0 as above; NULL = all),
 * averaged over samples [m_lo, m_hi).  eps, sumsq (sum of S^2) and steps
 * (sum of L) have n_nodes entries. */
int or_estimate(const or_problem *pb, int inst, int interval, int iter_tag,
                const double *U, const int64_t *nodes, int64_t n_nodes,
                int64_t m_lo, int64_t m_hi, double *eps, double *sumsq, int64_t *steps);

/* one residual iteration in place: U[:,ell>=1] += eps; returns max|eps| */
int or_iterate(const or_problem *pb, int inst, int interval, int iter_tag,
               double *U, double *max_eps, int64_t *steps);

/* whole solve of one instance (Algorithm 1, or the sweep schedule).
 * U_all: the nodal arrays of all intervals concatenated (sum n^d (M_n+1)).
 * max_eps: n_intervals*iters entries (sequential) or iters entries (sweeps). */
int or_solve(const or_problem *pb, int inst, double *U_all, double *max_eps);

/* One Aitken-relaxed iteration of one interval: r = the estimator's change
 * (eq. varepsilon_1's increment, or eq. uast's estimate minus the iterate),
 * weight w = w0 on the first iteration, else
 *   w = -w_prev <r_prev, r - r_prev> / |r - r_prev|^2   (w_prev if the
 * denominator is 0), clipped to [w_min, w_max]; U += w r at every node l >= 1.
 * r_prev [n^d M] and state {w_prev, have_prev} carry over between calls
 * (zero state: first iteration).  max_eps = max |r|. */
int or_iterate_aitken(const or_problem *pb, int inst, int interval, int iter_tag, double *U,
                      double *r_prev, double state[2], double *max_eps, int64_t *steps);

/* terminal misfit L = 1/2 sum_j (u(x_j,T) - target_j)^2 of a single-interval
 * solve from phi-coefficients c0, and its gradient dL/dc0 by reverse mode with
 * every sample path fixed (common random numbers). */
int or_loss_grad(const or_problem *pb, int inst, const double *c0,
                 const double *target, double *loss, double *grad);

/* the source at (X, t) on interval `interval` (OR_SRC_POLY needs the interval;
 * the other kinds ignore it) */
double or_source_iv(const or_problem *pb, int interval, const double *X, double t);

/* fraction of walks started at `starts` ([nwalk][dim]) that leave Omega within
 * nstar steps of length J = sqrt(2 d T/nstar) (Table 1 setting). */
double or_exit_fraction(int dim, double T, int nstar, const double *starts,
                        int64_t nwalk, uint64_t seed);

/* Unit jump directions of one walk (Lemma 2.1, reading R9, counter layout
 * R22): the walk of sample `sample` from node id `node` of (inst, interval,
 * iter_tag) under `seed`, steps q0 .. q0+nq-1, written to out[nq][dim]. */
int or_walk_directions(int dim, uint64_t seed, int64_t node, int64_t sample, int inst,
                       int interval, int iter_tag, int64_t q0, int64_t nq, double *out);

int or_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
