/*
 * hpsmc_oracle.c -- plain CPU FP64 oracle (test infrastructure only).
 *
 * Follows arXiv 2608.22190 step by step: quadrature and transforms of Sec. 2.3,
 * the sphere-jump walk of Lemma 2.1 with the exit index of eq. indexL and the
 * left-point path quadrature of eq. interIQ, the residual equation of
 * eq. ufg_ep1 with the Monte Carlo average of eq. varepsilon_1, the update and
 * interval loop of Algorithm 1.  Each function names the passage it follows.
 * Readings of the paper (R#) are those listed in the repository design notes.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may use
 * this file.  It shares no code with the GPU library.
 */
#include "hpsmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXD 5
#define OR_MAXN 64   /* max modes per dimension / temporal degree + 1 */

static const double OR_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11.  Ten rounds of the 4x32 Philox S-box with        */
/* multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments 0x9E3779B9,    */
/* 0xBB67AE85; the key is bumped between rounds.                              */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform on (0,1) from one 32-bit word (reading R22) */
static double or_u01(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* ------------------------------------------------------------------------ */
/* Orthogonal polynomials (Sec. 2.3).                                         */
/* ------------------------------------------------------------------------ */

/* Legendre L_k by Bonnet's recurrence (k+1)L_{k+1} = (2k+1)x L_k - k L_{k-1} */
double or_legendre(int k, double x)
{
    if (k == 0) return 1.0;
    double a = 1.0, b = x;
    for (int m = 1; m < k; ++m) {
        double c = ((2.0 * m + 1.0) * x * b - m * a) / (m + 1.0);
        a = b; b = c;
    }
    return b;
}

/* L_k, L'_k and L''_k together, for k = 0..kmax, from Bonnet's recurrence and
 * L'_{m+1} = L'_{m-1} + (2m+1) L_m,  L''_{m+1} = L''_{m-1} + (2m+1) L'_m */
static void or_legendre_all(int kmax, double x, double *L, double *dL, double *d2L)
{
    L[0] = 1.0; dL[0] = 0.0; if (d2L) d2L[0] = 0.0;
    if (kmax < 1) return;
    L[1] = x; dL[1] = 1.0; if (d2L) d2L[1] = 0.0;
    for (int m = 1; m < kmax; ++m) {
        L[m + 1] = ((2.0 * m + 1.0) * x * L[m] - m * L[m - 1]) / (m + 1.0);
        dL[m + 1] = dL[m - 1] + (2.0 * m + 1.0) * L[m];
        if (d2L) d2L[m + 1] = d2L[m - 1] + (2.0 * m + 1.0) * dL[m];
    }
}

double or_legendre_deriv(int k, double x)
{
    double L[OR_MAXN + 2], dL[OR_MAXN + 2];
    or_legendre_all(k, x, L, dL, NULL);
    return dL[k];
}

static double or_legendre_deriv2(int k, double x)
{
    double L[OR_MAXN + 2], dL[OR_MAXN + 2], d2L[OR_MAXN + 2];
    or_legendre_all(k, x, L, dL, d2L);
    return d2L[k];
}

/* Jacobi P_p^{(1,1)} by the three-term recurrence of the Jacobi family with
 * alpha = beta = 1:
 *   P_{m+1} = (2m+3)(m+2)/((m+1)(m+3)) x P_m - (m+2)/(m+3) P_{m-1},
 *   P_0 = 1, P_1 = 2x. */
double or_jacobi11(int p, double x)
{
    if (p == 0) return 1.0;
    double a = 1.0, b = 2.0 * x;
    for (int m = 1; m < p; ++m) {
        double c = (2.0 * m + 3.0) * (m + 2.0) / ((m + 1.0) * (m + 3.0)) * x * b
                 - (m + 2.0) / (m + 3.0) * a;
        a = b; b = c;
    }
    return b;
}

/* P_0..P_pmax^{(1,1)} by the same recurrence */
static void or_jacobi11_all(int pmax, double x, double *P)
{
    P[0] = 1.0;
    if (pmax < 1) return;
    P[1] = 2.0 * x;
    for (int m = 1; m < pmax; ++m)
        P[m + 1] = (2.0 * m + 3.0) * (m + 2.0) / ((m + 1.0) * (m + 3.0)) * x * P[m]
                 - (m + 2.0) / (m + 3.0) * P[m - 1];
}

/* Babuska-Shen basis as a generalized Jacobi function phi_p = (1-x^2) P_p^{(1,1)} */
double or_phi(int p, double x) { return (1.0 - x * x) * or_jacobi11(p, x); }

/* ------------------------------------------------------------------------ */
/* Quadrature (Sec. 2.1 shifted LGL in time; Sec. 2.3 JG(1,1) in space).      */
/* The JG(1,1) n-point nodes are the zeros of L'_{n+1}; they are found by     */
/* Newton's method with deflation.  Weights: the (n+2)-point LGL weight       */
/* times (1-x^2), which makes the rule exact for (1-x^2) p, deg p <= 2n-1.    */
/* ------------------------------------------------------------------------ */
static int or_zeros_dlegendre(int N, double *z) /* N-1 zeros of L'_N, ascending */
{
    int nz = N - 1;
    for (int j = 0; j < nz; ++j) {
        double x = -cos(OR_PI * (j + 1.0) / N);
        for (int it = 0; it < 100; ++it) {
            double p = or_legendre_deriv(N, x);
            double dp = or_legendre_deriv2(N, x);
            double s = 0.0;
            for (int i = 0; i < j; ++i) s += 1.0 / (x - z[i]);
            double dx = p / (dp - s * p);
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        z[j] = x;
    }
    /* ascending order (Newton from ascending guesses keeps it; enforce it) */
    for (int a = 1; a < nz; ++a)
        for (int b = a; b > 0 && z[b - 1] > z[b]; --b) { double t = z[b]; z[b] = z[b - 1]; z[b - 1] = t; }
    return 0;
}

int or_jg11(int n, double *x, double *w)
{
    if (n < 1 || n > OR_MAXN) return -1;
    or_zeros_dlegendre(n + 1, x);
    for (int j = 0; j < n; ++j) {
        double L = or_legendre(n + 1, x[j]);
        w[j] = 2.0 * (1.0 - x[j] * x[j]) / ((n + 1.0) * (n + 2.0) * L * L);
    }
    return 0;
}

int or_lgl(int M, double *xi, double *w)
{
    if (M < 1 || M + 1 > OR_MAXN) return -1;
    xi[0] = -1.0; xi[M] = 1.0;
    if (M > 1) or_zeros_dlegendre(M, xi + 1);
    for (int k = 0; k <= M; ++k) {
        double L = or_legendre(M, xi[k]);
        w[k] = 2.0 / (M * (M + 1.0) * L * L);
    }
    return 0;
}

/* eq. spacelag: a_pj = P_p(x_j) w_j / (gt_p (1 - x_j^2)), gt_p = 8(p+1)/((2p+3)(p+2)) */
int or_matrix_A(int n, double *A)
{
    double x[OR_MAXN], w[OR_MAXN];
    if (or_jg11(n, x, w)) return -1;
    for (int p = 0; p < n; ++p) {
        double gt = 8.0 * (p + 1.0) / ((2.0 * p + 3.0) * (p + 2.0));
        for (int j = 0; j < n; ++j)
            A[p * n + j] = or_jacobi11(p, x[j]) * w[j] / (gt * (1.0 - x[j] * x[j]));
    }
    return 0;
}

/* eq. timeLag: b_qk = L_q(xi_k) w_k / gamma_q, gamma_q = 2/(2q+1) for q < M and
 * gamma_M = sum_k L_M(xi_k)^2 w_k (reference-interval weights, reading R5). */
int or_matrix_B(int M, double *B)
{
    double xi[OR_MAXN], w[OR_MAXN];
    if (or_lgl(M, xi, w)) return -1;
    for (int q = 0; q <= M; ++q) {
        double g;
        if (q < M) g = 2.0 / (2.0 * q + 1.0);
        else { g = 0.0; for (int k = 0; k <= M; ++k) { double L = or_legendre(M, xi[k]); g += L * L * w[k]; } }
        for (int k = 0; k <= M; ++k) B[q * (M + 1) + k] = or_legendre(q, xi[k]) * w[k] / g;
    }
    return 0;
}

static int64_t or_ipow(int n, int d) { int64_t r = 1; for (int i = 0; i < d; ++i) r *= n; return r; }

/* ------------------------------------------------------------------------ */
/* Reconstruction (eq. u_N and the tensor-product remark): the modal          */
/* coefficients are U multiplied by A along every spatial mode and by B along */
/* time.  Applied one mode at a time (Kronecker product of the 1-D maps).     */
/* ------------------------------------------------------------------------ */
static void or_mode_product(const double *in, double *out, int64_t outer, int len,
                            int64_t inner, const double *Mat /* len x len */)
{
    for (int64_t o = 0; o < outer; ++o)
        for (int a = 0; a < len; ++a)
            for (int64_t i = 0; i < inner; ++i) {
                double s = 0.0;
                for (int b = 0; b < len; ++b)
                    s += Mat[a * len + b] * in[(o * len + b) * inner + i];
                out[(o * len + a) * inner + i] = s;
            }
}

int or_reconstruct(int dim, int n, int M, const double *U, double *Ut)
{
    if (dim < 1 || dim > OR_MAXD || n < 1 || M < 1) return -1;
    int T1 = M + 1;
    int64_t size = or_ipow(n, dim) * T1;
    double *A = malloc(sizeof(double) * n * n), *B = malloc(sizeof(double) * T1 * T1);
    double *t0 = malloc(sizeof(double) * size), *t1 = malloc(sizeof(double) * size);
    if (!A || !B || !t0 || !t1) { free(A); free(B); free(t0); free(t1); return -3; }
    or_matrix_A(n, A);
    or_matrix_B(M, B);
    memcpy(t0, U, sizeof(double) * size);
    /* layout [j_0]..[j_{d-1}][ell]; spatial mode i has outer n^i, inner n^{d-1-i}*T1 */
    for (int i = 0; i < dim; ++i) {
        or_mode_product(t0, t1, or_ipow(n, i), n, or_ipow(n, dim - 1 - i) * T1, A);
        double *t = t0; t0 = t1; t1 = t;
    }
    or_mode_product(t0, t1, or_ipow(n, dim), T1, 1, B);
    memcpy(Ut, t1, sizeof(double) * size);
    free(A); free(B); free(t0); free(t1);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Evaluation of the reconstruction (eq. u_N) at an arbitrary point, with the */
/* two corrections of readings R3 (-phi_p'' = (p+1)(p+2) P_p^{(1,1)}) and R4  */
/* (d_t u keeps the spatial basis phi_p).                                      */
/* ------------------------------------------------------------------------ */
int or_eval(int dim, int n, int M, double h, const double *Ut,
            const double *X, double xi, double out[3])
{
    double phi[OR_MAXD][OR_MAXN], jac[OR_MAXD][OR_MAXN], Lt[OR_MAXN], dLt[OR_MAXN];
    int T1 = M + 1;
    for (int i = 0; i < dim; ++i) {
        or_jacobi11_all(n - 1, X[i], jac[i]);
        for (int p = 0; p < n; ++p) phi[i][p] = (1.0 - X[i] * X[i]) * jac[i][p];
    }
    or_legendre_all(M, xi, Lt, dLt, NULL);
    int64_t np = or_ipow(n, dim);
    double u = 0.0, ut = 0.0, lap = 0.0;
    for (int64_t pf = 0; pf < np; ++pf) {
        int pi[OR_MAXD];
        int64_t r = pf;
        for (int i = dim - 1; i >= 0; --i) { pi[i] = (int)(r % n); r /= n; }
        double a = 0.0, b = 0.0;
        for (int q = 0; q < T1; ++q) { a += Ut[pf * T1 + q] * Lt[q]; b += Ut[pf * T1 + q] * dLt[q]; }
        double prodphi = 1.0;
        for (int i = 0; i < dim; ++i) prodphi *= phi[i][pi[i]];
        u += a * prodphi;
        ut += b * prodphi;
        for (int i = 0; i < dim; ++i) {
            double term = (pi[i] + 1.0) * (pi[i] + 2.0) * jac[i][pi[i]];
            for (int m = 0; m < dim; ++m) if (m != i) term *= phi[m][pi[m]];
            lap -= a * term;
        }
    }
    out[0] = u; out[1] = ut * 2.0 / h; out[2] = lap;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Fractional operator (Ex. 2-3; the remark that the method carries over with */
/* an alpha-stable walk and generalized Jacobi functions of parameter         */
/* (alpha/2, alpha/2)).  d = 1.                                                */
/* ------------------------------------------------------------------------ */
static int or_is_frac(const or_problem *pb) { return pb->alpha > 0.0 && pb->alpha < 2.0; }

/* Jacobi P_p^{(al,be)} by the standard three-term recurrence */
static double or_jacobi_ab(int p, double al, double be, double x)
{
    if (p == 0) return 1.0;
    double pm = 1.0, pc = 0.5 * (al - be) + 0.5 * (al + be + 2.0) * x;
    for (int k = 1; k < p; ++k) {
        double s2 = 2.0 * k + al + be;
        double c1 = 2.0 * (k + 1.0) * (k + al + be + 1.0) * s2;
        double c2 = (s2 + 1.0) * (al * al - be * be);
        double c3 = s2 * (s2 + 1.0) * (s2 + 2.0);
        double c4 = 2.0 * (k + al) * (k + be) * (s2 + 2.0);
        double pn = ((c2 + c3 * x) * pc - c4 * pm) / c1;
        pm = pc; pc = pn;
    }
    return pc;
}

double or_jacobi_aa(int p, double a, double x) { return or_jacobi_ab(p, a, a, x); }

/* Gauss-Jacobi rule for the weight (1-x^2)^a: zeros of P_n^{(a,a)} by Newton's
 * method with deflation (P_n' = (n+2a+1)/2 P_{n-1}^{(a+1,a+1)}), weights
 *   w_j = 2^{2a+1} Gamma(n+a+1)^2 / (n! Gamma(n+2a+1) (1-x_j^2) P_n'(x_j)^2). */
int or_gauss_jacobi(int n, double a, double *x, double *w)
{
    if (n < 1 || !(a > -1.0)) return -1;
    for (int j = 0; j < n; ++j) {
        double z = -cos(OR_PI * (j + 0.75) / (n + 0.5));
        for (int it = 0; it < 200; ++it) {
            double p = or_jacobi_ab(n, a, a, z);
            double dp = 0.5 * (n + 2.0 * a + 1.0) * or_jacobi_ab(n - 1, a + 1.0, a + 1.0, z);
            double sdef = 0.0;
            for (int i = 0; i < j; ++i) sdef += 1.0 / (z - x[i]);
            double dz = p / (dp - sdef * p);
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[j] = z;
    }
    for (int i = 1; i < n; ++i)
        for (int k = i; k > 0 && x[k - 1] > x[k]; --k) { double t = x[k]; x[k] = x[k - 1]; x[k - 1] = t; }
    double lc = (2.0 * a + 1.0) * log(2.0) + 2.0 * lgamma(n + a + 1.0) - lgamma(n + 1.0) - lgamma(n + 2.0 * a + 1.0);
    for (int j = 0; j < n; ++j) {
        double dp = 0.5 * (n + 2.0 * a + 1.0) * or_jacobi_ab(n - 1, a + 1.0, a + 1.0, x[j]);
        w[j] = exp(lc) / ((1.0 - x[j] * x[j]) * dp * dp);
    }
    return 0;
}

/* (-Delta)^{alpha/2} [(1-x^2)_+^{alpha/2} P_p^{(alpha/2,alpha/2)}] = lambda_p P_p^{(alpha/2,alpha/2)}
 * on (-1,1), lambda_p = Gamma(p+alpha+1)/p! (the operator with Fourier symbol |xi|^alpha) */
double or_frac_lambda(int p, double alpha) { return exp(lgamma(p + alpha + 1.0) - lgamma(p + 1.0)); }

/* regularized incomplete beta I_x(a,b) by the continued fraction of DLMF 8.17.22
 * (modified Lentz), with I_x(a,b) = 1 - I_{1-x}(b,a) beyond (a+1)/(a+b+2) */
double or_ibeta(double x, double a, double b)
{
    if (x <= 0.0) return 0.0;
    if (x >= 1.0) return 1.0;
    if (x > (a + 1.0) / (a + b + 2.0)) return 1.0 - or_ibeta(1.0 - x, b, a);
    double lpre = a * log(x) + b * log1p(-x) - log(a) - (lgamma(a) + lgamma(b) - lgamma(a + b));
    const double tiny = 1e-300;
    double f = 1.0, C = 1.0, D = 0.0;
    for (int j = 1; j < 2000; ++j) {
        int m = j / 2;
        double dj = (j & 1) ? -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0))
                            : m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
        D = 1.0 + dj * D;
        if (fabs(D) < tiny) D = tiny;
        C = 1.0 + dj / C;
        if (fabs(C) < tiny) C = tiny;
        D = 1.0 / D;
        double del = C * D;
        f *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return exp(lpre) / f;
}

/* inverse in x of I_x(a,b) = y by bisection on log x over [-745, 0] */
double or_ibeta_inv(double y, double a, double b)
{
    double lo = -745.0, hi = 0.0;
    for (int it = 0; it < 90; ++it) {
        double mid = 0.5 * (lo + hi);
        if (or_ibeta(exp(mid), a, b) < y) lo = mid; else hi = mid;
    }
    return exp(0.5 * (lo + hi));
}

/* Jump length of the alpha-stable walk from the centre of its ball.  The
 * ball radius r = (Delta / C_1^alpha)^{1/alpha} with C_1^alpha = 1/Gamma(1+alpha)
 * (the mean exit time of the ball is Delta).  The exit point Y of the process
 * started at the centre has P(|Y| > rho) = I_{r^2/rho^2}(alpha/2, 1 - alpha/2)
 * (the exit law of a ball for a symmetric stable process), so a uniform omega
 * gives rho = r / sqrt(I^{-1}(omega; alpha/2, 1 - alpha/2)). */
double or_frac_jump(double alpha, double delta, double omega)
{
    double r = pow(delta * exp(lgamma(1.0 + alpha)), 1.0 / alpha);
    return r / sqrt(or_ibeta_inv(omega, 0.5 * alpha, 1.0 - 0.5 * alpha));
}

/* nodal -> modal: collocation solve sum_p c_p w(x_j) P_p(x_j) = U_j (Gaussian
 * elimination with partial pivoting) for every time column, then B in time */
int or_frac_reconstruct(double alpha, int n, int M, const double *U, double *Ut)
{
    int T1 = M + 1;
    double a = 0.5 * alpha, x[OR_MAXN], w[OR_MAXN];
    if (n < 1 || n > OR_MAXN || M < 1 || or_gauss_jacobi(n, a, x, w)) return -1;
    double *Phi = malloc(sizeof(double) * n * n), *rhs = malloc(sizeof(double) * n * T1);
    double *B = malloc(sizeof(double) * T1 * T1), *C = malloc(sizeof(double) * n * T1);
    if (!Phi || !rhs || !B || !C) { free(Phi); free(rhs); free(B); free(C); return -3; }
    for (int j = 0; j < n; ++j)
        for (int p = 0; p < n; ++p) Phi[j * n + p] = pow(1.0 - x[j] * x[j], a) * or_jacobi_aa(p, a, x[j]);
    memcpy(rhs, U, sizeof(double) * n * T1);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r) if (fabs(Phi[r * n + c]) > fabs(Phi[piv * n + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < n; ++k) { double t = Phi[c * n + k]; Phi[c * n + k] = Phi[piv * n + k]; Phi[piv * n + k] = t; }
            for (int k = 0; k < T1; ++k) { double t = rhs[c * T1 + k]; rhs[c * T1 + k] = rhs[piv * T1 + k]; rhs[piv * T1 + k] = t; }
        }
        for (int r = c + 1; r < n; ++r) {
            double m = Phi[r * n + c] / Phi[c * n + c];
            for (int k = c; k < n; ++k) Phi[r * n + k] -= m * Phi[c * n + k];
            for (int k = 0; k < T1; ++k) rhs[r * T1 + k] -= m * rhs[c * T1 + k];
        }
    }
    for (int c = n - 1; c >= 0; --c)
        for (int k = 0; k < T1; ++k) {
            double s = rhs[c * T1 + k];
            for (int q = c + 1; q < n; ++q) s -= Phi[c * n + q] * C[q * T1 + k];
            C[c * T1 + k] = s / Phi[c * n + c];
        }
    or_matrix_B(M, B);
    or_mode_product(C, Ut, n, T1, 1, B);
    free(Phi); free(rhs); free(B); free(C);
    return 0;
}

int or_frac_eval(double alpha, int n, int M, double h, const double *Ut, double x, double xi, double out[3])
{
    int T1 = M + 1;
    double a = 0.5 * alpha, Lt[OR_MAXN], dLt[OR_MAXN];
    if (n > OR_MAXN || T1 > OR_MAXN) return -1;
    or_legendre_all(M, xi, Lt, dLt, NULL);
    double w = pow(1.0 - x * x, a), u = 0.0, ut = 0.0, F = 0.0;
    for (int p = 0; p < n; ++p) {
        double J = or_jacobi_aa(p, a, x), lam = or_frac_lambda(p, alpha);
        double su = 0.0, st = 0.0;
        for (int q = 0; q < T1; ++q) { su += Ut[p * T1 + q] * Lt[q]; st += Ut[p * T1 + q] * dLt[q]; }
        u += J * su;
        ut += J * st;
        F += lam * J * su;
    }
    out[0] = w * u;
    out[1] = (2.0 / h) * w * ut;
    out[2] = -F;
    return 0;
}

/* Manufactured fractional solutions u = w g T: (-Delta)^{alpha/2}(w g) =
 * sum_k a_k lambda_k P_k^{(a,a)} with a_k the Jacobi coefficients of g
 * (Gauss-Jacobi quadrature with 160 nodes).  Cached per (alpha, kind, params);
 * or_frac_prepare runs outside parallel regions. */
#define OR_FRAC_NQ 160
#define OR_FRAC_K 150
static struct { int valid, kind; double alpha, par[4]; int K; double c[OR_FRAC_K]; } or_fsrc;

static double or_frac_g(int kind, const double *par, double x)
{
    switch (kind) {
    case OR_SRC_FRAC_LONGTIME: return sin(x);
    case OR_SRC_FRAC_SINGULAR: return cos(x * x * x + 1.0) / (10.0 * x * x + 1.0);
    case OR_SRC_FRAC_POLY: return par[0] + par[1] * x + par[2] * x * x;
    }
    return 0.0;
}

static int or_frac_prepare(const or_problem *pb)
{
    int kind = pb->src_kind;
    if (kind < OR_SRC_FRAC_LONGTIME || kind > OR_SRC_FRAC_POLY) return 0;
    if (or_fsrc.valid && or_fsrc.kind == kind && or_fsrc.alpha == pb->alpha &&
        memcmp(or_fsrc.par, pb->src_param, sizeof(or_fsrc.par)) == 0) return 0;
    double a = 0.5 * pb->alpha;
    double *x = malloc(sizeof(double) * OR_FRAC_NQ), *w = malloc(sizeof(double) * OR_FRAC_NQ);
    if (!x || !w) { free(x); free(w); return -3; }
    or_gauss_jacobi(OR_FRAC_NQ, a, x, w);
    int K = kind == OR_SRC_FRAC_POLY ? 3 : kind == OR_SRC_FRAC_LONGTIME ? 40 : OR_FRAC_K;
    for (int k = 0; k < K; ++k) {
        /* ||P_k||^2 = 2^{2a+1} Gamma(k+a+1)^2 / ((2k+2a+1) k! Gamma(k+2a+1)) */
        double nrm = exp((2.0 * a + 1.0) * log(2.0) + 2.0 * lgamma(k + a + 1.0) - lgamma(k + 1.0) -
                         lgamma(k + 2.0 * a + 1.0)) / (2.0 * k + 2.0 * a + 1.0);
        double s = 0.0;
        for (int j = 0; j < OR_FRAC_NQ; ++j) s += w[j] * or_frac_g(kind, pb->src_param, x[j]) * or_jacobi_aa(k, a, x[j]);
        or_fsrc.c[k] = s / nrm * or_frac_lambda(k, pb->alpha);
    }
    free(x); free(w);
    or_fsrc.K = K;
    or_fsrc.kind = kind;
    or_fsrc.alpha = pb->alpha;
    memcpy(or_fsrc.par, pb->src_param, sizeof(or_fsrc.par));
    or_fsrc.valid = 1;
    return 0;
}

static void or_frac_exact_parts(const or_problem *pb, double x, double t, double *u, double *ut, double *lap)
{
    or_frac_prepare(pb);
    double a = 0.5 * pb->alpha, w = pow(1.0 - x * x, a), g = or_frac_g(pb->src_kind, pb->src_param, x);
    double T, Tp;
    switch (pb->src_kind) {
    case OR_SRC_FRAC_LONGTIME:
        T = exp(cos(t)) / (1.0 + t * t);
        Tp = T * (-sin(t) - 2.0 * t / (1.0 + t * t));
        break;
    case OR_SRC_FRAC_SINGULAR:
        T = pow(t, pb->src_param[0]);
        Tp = t > 0.0 ? pb->src_param[0] * pow(t, pb->src_param[0] - 1.0) : 0.0;
        break;
    default:
        T = 1.0 + pb->src_param[3] * t;
        Tp = pb->src_param[3];
        break;
    }
    double F = 0.0;
    for (int k = 0; k < or_fsrc.K; ++k) F += or_fsrc.c[k] * or_jacobi_aa(k, a, x);
    *u = w * g * T;
    *ut = w * g * Tp;
    *lap = -F * T;            /* -(-Delta)^{alpha/2} u */
}

/* spatial nodes of the problem: JG(1,1), or Gauss-Jacobi (alpha/2, alpha/2) */
static int or_space_nodes(const or_problem *pb, double *x, double *w)
{
    if (or_is_frac(pb)) return or_gauss_jacobi(pb->n, 0.5 * pb->alpha, x, w);
    return or_jg11(pb->n, x, w);
}

/* ------------------------------------------------------------------------ */
/* Problem data: f, f', manufactured sources and exact solutions.             */
/* ------------------------------------------------------------------------ */
double or_f(const or_problem *pb, double u)
{
    switch (pb->f_kind) {
    case OR_F_AFFINE: return pb->f_param[0] * u + pb->f_param[1];
    case OR_F_U_MINUS_U3: return u - u * u * u;
    case OR_F_SIN: return sin(u);
    case OR_F_U2_OVER_1PU2: return u * u / (1.0 + u * u);
    case OR_F_NEG_U3: return -u * u * u;
    case OR_F_U_SIN_U: return u * sin(u);
    }
    return NAN;
}

double or_fprime(const or_problem *pb, double u)
{
    switch (pb->f_kind) {
    case OR_F_AFFINE: return pb->f_param[0];
    case OR_F_U_MINUS_U3: return 1.0 - 3.0 * u * u;
    case OR_F_SIN: return cos(u);
    case OR_F_U2_OVER_1PU2: return 2.0 * u / ((1.0 + u * u) * (1.0 + u * u));
    case OR_F_NEG_U3: return -3.0 * u * u;
    case OR_F_U_SIN_U: return sin(u) + u * cos(u);
    }
    return NAN;
}

/* exact solution, its time derivative and Laplacian for the manufactured sources */
static void or_exact_parts(const or_problem *pb, const double *X, double t,
                           double *u, double *ut, double *lap)
{
    int d = pb->dim;
    if (pb->src_kind >= OR_SRC_FRAC_LONGTIME && pb->src_kind <= OR_SRC_FRAC_POLY) {
        or_frac_exact_parts(pb, X[0], t, u, ut, lap);
        return;
    }
    switch (pb->src_kind) {
    case OR_SRC_SIN_DECAY: {
        double p = exp(-t);
        for (int i = 0; i < d; ++i) p *= sin(OR_PI * X[i]);
        *u = p; *ut = -p; *lap = -d * OR_PI * OR_PI * p;
        return;
    }
    case OR_SRC_COS_DECAY: {
        double p = exp(-t);
        for (int i = 0; i < d; ++i) p *= cos(0.5 * OR_PI * X[i]);
        *u = p; *ut = -p; *lap = -0.25 * d * OR_PI * OR_PI * p;
        return;
    }
    case OR_SRC_LONGTIME: {
        /* u = a(x) sin(sigma) T(t), a = prod(1-x_i^2), sigma = sum x_i,
         * T = e^{cos t}/(1+t^2).  Lap u = T [ S Lap a + 2 C grad a . 1 - d a S ]. */
        double a = 1.0, sig = 0.0;
        for (int i = 0; i < d; ++i) { a *= 1.0 - X[i] * X[i]; sig += X[i]; }
        double S = sin(sig), C = cos(sig);
        double lapa = 0.0, grada = 0.0;
        for (int i = 0; i < d; ++i) {
            double rest = 1.0;
            for (int m = 0; m < d; ++m) if (m != i) rest *= 1.0 - X[m] * X[m];
            lapa += -2.0 * rest;
            grada += -2.0 * X[i] * rest;
        }
        double T = exp(cos(t)) / (1.0 + t * t);
        double Tp = T * (-sin(t) - 2.0 * t / (1.0 + t * t));
        *u = a * S * T;
        *ut = a * S * Tp;
        *lap = T * (S * lapa + 2.0 * C * grada - d * a * S);
        return;
    }
    case OR_SRC_QUAD: {
        double a = 1.0, lapa = 0.0;
        for (int i = 0; i < d; ++i) a *= 1.0 - X[i] * X[i];
        for (int i = 0; i < d; ++i) {
            double rest = 1.0;
            for (int m = 0; m < d; ++m) if (m != i) rest *= 1.0 - X[m] * X[m];
            lapa += -2.0 * rest;
        }
        double c0 = pb->src_param[0], c1 = pb->src_param[1], c2 = pb->src_param[2];
        double g = c0 + c1 * t + c2 * t * t, gp = c1 + 2.0 * c2 * t;
        *u = a * g; *ut = a * gp; *lap = lapa * g;
        return;
    }
    }
    *u = 0.0; *ut = 0.0; *lap = 0.0;
}

double or_exact(const or_problem *pb, const double *X, double t)
{
    double u, ut, lap;
    or_exact_parts(pb, X, t, &u, &ut, &lap);
    return u;
}

/* s = u_t - Lap u - f(u) at the exact solution, so that the exact solution
 * satisfies u_t = Lap u + f(u) + s (fractional kinds: -(-Delta)^{alpha/2} in
 * place of Lap) */
/* OR_SRC_POLY: the interval's tensor-Legendre polynomial evaluated term by term */
static double or_source_poly(const or_problem *pb, int interval, const double *X, double t)
{
    const int d = pb->dim, P = pb->n + 2;
    const int64_t pd = or_ipow(P, d);
    int64_t off = 0;
    for (int i = 0; i < interval; ++i) off += pd * (pb->degree[i] + 1);
    const int T1 = pb->degree[interval] + 1;
    const double t0 = pb->t_breaks[interval], h = pb->t_breaks[interval + 1] - t0;
    const double xi = 2.0 * (t - t0) / h - 1.0;
    double s = 0.0;
    for (int64_t k = 0; k < pd; ++k) {
        double sp = 1.0;
        int64_t r = k;
        for (int i = d - 1; i >= 0; --i) {
            sp *= or_legendre((int)(r % P), X[i]);
            r /= P;
        }
        for (int q = 0; q < T1; ++q) s += pb->src_coeffs[off + k * T1 + q] * sp * or_legendre(q, xi);
    }
    return s;
}

double or_source_iv(const or_problem *pb, int interval, const double *X, double t)
{
    if (pb->src_kind == OR_SRC_POLY) return or_source_poly(pb, interval, X, t);
    return or_source(pb, X, t);
}

double or_source(const or_problem *pb, const double *X, double t)
{
    if (pb->src_kind == OR_SRC_NONE) return 0.0;
    if (pb->src_kind == OR_SRC_POLY) {   /* the first interval whose closure holds t */
        int iv = 0;
        while (iv + 1 < pb->n_intervals && t > pb->t_breaks[iv + 1]) ++iv;
        return or_source_poly(pb, iv, X, t);
    }
    double u, ut, lap;
    or_exact_parts(pb, X, t, &u, &ut, &lap);
    return ut - lap - or_f(pb, u);
}

/* eq. ufg_ep1: the right-hand side of the residual equation at (X, tau),
 * r = f(u*) - d_t u* + Lap u*, plus the source term of the forced problem */
double or_residual(const or_problem *pb, int interval, const double *Ut,
                   const double *X, double tau)
{
    double t0 = pb->t_breaks[interval], h = pb->t_breaks[interval + 1] - t0;
    double xi = 2.0 * (tau - t0) / h - 1.0;
    double v[3];
    if (or_is_frac(pb)) or_frac_eval(pb->alpha, pb->n, pb->degree[interval], h, Ut, X[0], xi, v);
    else or_eval(pb->dim, pb->n, pb->degree[interval], h, Ut, X, xi, v);
    return or_f(pb, v[0]) + or_source_iv(pb, interval, X, tau) - v[1] + v[2];
}

int or_grid(const or_problem *pb, int interval, double *x_nodes, double *t_nodes)
{
    double w[OR_MAXN], xi[OR_MAXN];
    if (x_nodes && or_space_nodes(pb, x_nodes, w)) return -1;
    if (t_nodes) {
        int M = pb->degree[interval];
        if (or_lgl(M, xi, w)) return -1;
        double t0 = pb->t_breaks[interval], h = pb->t_breaks[interval + 1] - t0;
        for (int k = 0; k <= M; ++k) t_nodes[k] = t0 + 0.5 * (xi[k] + 1.0) * h;
    }
    return 0;
}

int or_ic_nodes(const or_problem *pb, int inst, double *u0)
{
    double x[OR_MAXN], w[OR_MAXN];
    int d = pb->dim, n = pb->n;
    if (or_space_nodes(pb, x, w)) return -1;
    int64_t nsp = or_ipow(n, d);
    for (int64_t jf = 0; jf < nsp; ++jf) {
        int ji[OR_MAXD];
        double X[OR_MAXD];
        int64_t r = jf;
        for (int i = d - 1; i >= 0; --i) { ji[i] = (int)(r % n); r /= n; }
        for (int i = 0; i < d; ++i) X[i] = x[ji[i]];
        double v = 0.0;
        switch (pb->ic_kind) {
        case OR_IC_EXACT: v = or_exact(pb, X, pb->t_breaks[0]); break;
        case OR_IC_SINGULAR: {
            v = pow(fabs(X[0]), pb->ic_param[0]);
            for (int i = 0; i < d; ++i) v *= 1.0 - X[i] * X[i];
            break;
        }
        case OR_IC_PHI: {
            const double *c = pb->ic_data + (int64_t)inst * nsp;
            for (int64_t pf = 0; pf < nsp; ++pf) {
                int64_t rr = pf;
                double prod = 1.0;
                for (int i = d - 1; i >= 0; --i) { prod *= or_phi((int)(rr % n), X[i]); rr /= n; }
                v += c[pf] * prod;
            }
            break;
        }
        case OR_IC_NODAL: v = pb->ic_data[(int64_t)inst * nsp + jf]; break;
        default: return -2;
        }
        u0[jf] = v;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Direction of the sphere jump (Lemma 2.1, reading R9 with the counter      */
/* layout of R22).  d=1: a fair sign from one bit; d=2: angle 2*pi*u;        */
/* d>=3: a normalized vector of Box-Muller normals.                           */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t key[2]; uint32_t c0, c1, c3; int64_t blk; uint32_t w[4]; uint32_t w2[4]; } or_stream;

static void or_stream_block(or_stream *st, int64_t blk, uint32_t out[4])
{
    uint32_t ctr[4] = { st->c0, st->c1, (uint32_t)blk, st->c3 };
    or_philox4x32_10(ctr, st->key, out);
}

static void or_direction(or_stream *st, int dim, int64_t q, double *dir)
{
    if (dim == 1) {
        int64_t blk = q >> 7;
        if (blk != st->blk) { or_stream_block(st, blk, st->w); st->blk = blk; }
        uint32_t word = st->w[(q >> 5) & 3];
        dir[0] = ((word >> (q & 31)) & 1u) ? 1.0 : -1.0;
        return;
    }
    if (dim == 2) {
        int64_t blk = q >> 2;
        if (blk != st->blk) { or_stream_block(st, blk, st->w); st->blk = blk; }
        double th = 2.0 * OR_PI * or_u01(st->w[q & 3]);
        dir[0] = cos(th); dir[1] = sin(th);
        return;
    }
    double g[8];
    uint32_t w[8];
    if (dim <= 4) {
        or_stream_block(st, q, w);
    } else {
        or_stream_block(st, 2 * q, w);
        or_stream_block(st, 2 * q + 1, w + 4);
    }
    int npairs = (dim + 1) / 2;
    for (int k = 0; k < npairs; ++k) {
        double r = sqrt(-2.0 * log(or_u01(w[2 * k])));
        double th = 2.0 * OR_PI * or_u01(w[2 * k + 1]);
        g[2 * k] = r * cos(th);
        g[2 * k + 1] = r * sin(th);
    }
    double nrm = 0.0;
    for (int i = 0; i < dim; ++i) nrm += g[i] * g[i];
    nrm = sqrt(nrm);
    for (int i = 0; i < dim; ++i) dir[i] = g[i] / nrm;
}

/* ------------------------------------------------------------------------ */
/* Ball point of a walk step (OR_QUAD_BALL).  The expected path integral over */
/* the sojourn in the ball B_r(x), r = J, equals W(x) E_{Q_r}[g(Y)] with       */
/* Q_r = G_r(x, .)/W(x) and G_r the Green's function of -Laplace on the ball  */
/* with pole at its centre (Sec. 3, the representation used for the B_1       */
/* bound).  W(x) = r^2/(2d) = Delta.  Q_r is radial: the radius rho = r s has  */
/* density proportional to s^{d-1} G(s), i.e. 2d/(d-2) (s - s^{d-1}) for      */
/* d >= 3, 4 s log(1/s) for d = 2 and 2 (1 - s) for d = 1 -- in every case    */
/* the law of the product sqrt(U_a) * U_b^{1/d} of independent uniform powers */
/* (a product of variables with densities 2a and d b^{d-1}).  The direction   */
/* is uniform.  Philox words: counter word 2 with bit 31 set, 2q (radius      */
/* from words 0 and 1, direction from words 2 and 3) and, for d >= 3, 2q+1   */
/* (more Box-Muller pairs); the walk's own counters never set bit 31.        */
/* ------------------------------------------------------------------------ */
static void or_ball_point(or_stream *st, int dim, int64_t q, double *off)
{
    uint32_t w[8];
    or_stream_block(st, (int64_t)(0x80000000u | (uint32_t)(2 * q)), w);
    double ua = or_u01(w[0]), ub = or_u01(w[1]), root;
    switch (dim) {
    case 1: root = ub; break;
    case 2: root = sqrt(ub); break;
    case 3: root = cbrt(ub); break;
    case 4: root = sqrt(sqrt(ub)); break;
    default: root = pow(ub, 0.2); break;
    }
    double s = sqrt(ua) * root;
    if (dim == 1) {
        off[0] = (w[2] & 1u) ? s : -s;
        return;
    }
    if (dim == 2) {
        double th = 2.0 * OR_PI * or_u01(w[2]);
        off[0] = s * cos(th); off[1] = s * sin(th);
        return;
    }
    or_stream_block(st, (int64_t)(0x80000000u | (uint32_t)(2 * q + 1)), w + 4);
    double g[6];
    for (int k = 0; k < 3; ++k) {
        double rr = sqrt(-2.0 * log(or_u01(w[2 + 2 * k])));
        double th = 2.0 * OR_PI * or_u01(w[3 + 2 * k]);
        g[2 * k] = rr * cos(th);
        g[2 * k + 1] = rr * sin(th);
    }
    double nrm = 0.0;
    for (int i = 0; i < dim; ++i) nrm += g[i] * g[i];
    nrm = sqrt(nrm);
    for (int i = 0; i < dim; ++i) off[i] = s * g[i] / nrm;
}

static void or_stream_init(or_stream *st, uint64_t seed, int64_t node, int64_t sample,
                           int inst, int interval, int iter_tag)
{
    st->key[0] = (uint32_t)seed; st->key[1] = (uint32_t)(seed >> 32);
    st->c0 = (uint32_t)node; st->c1 = (uint32_t)sample;
    st->c3 = ((uint32_t)inst << 16) | (((uint32_t)interval & 0xFFu) << 8) | ((uint32_t)iter_tag & 0xFFu);
    st->blk = -1;
}

/* The directions a walk draws, step by step, exactly as or_path draws them. */
int or_walk_directions(int dim, uint64_t seed, int64_t node, int64_t sample, int inst,
                       int interval, int iter_tag, int64_t q0, int64_t nq, double *out)
{
    if (dim < 1 || dim > OR_MAXD || q0 < 0 || nq < 0) return -1;
    or_stream st;
    or_stream_init(&st, seed, node, sample, inst, interval, iter_tag);
    for (int64_t k = 0; k < nq; ++k) or_direction(&st, dim, q0 + k, out + k * dim);
    return 0;
}

/* node geometry: the spatial point and (ell, span, N*) of a node id */
typedef struct { double X[OR_MAXD]; int ell; int nstar; double span; double delta; } or_node;

/* reference nodes of the interval: JG(1,1) in space, LGL in time */
typedef struct { double x[OR_MAXN]; double xi[OR_MAXN]; } or_ref;

static void or_ref_nodes(const or_problem *pb, int interval, or_ref *rf)
{
    double w[OR_MAXN];
    or_space_nodes(pb, rf->x, w);
    or_lgl(pb->degree[interval], rf->xi, w);
}

static int or_node_info(const or_problem *pb, int interval, int64_t node, const or_ref *rf, or_node *nd)
{
    int d = pb->dim, n = pb->n, M = pb->degree[interval];
    int64_t nsp = or_ipow(n, d);
    if (node < 0 || node >= nsp * M) return -1;
    int64_t jf = node % nsp;
    nd->ell = (int)(node / nsp) + 1;
    int64_t r = jf;
    for (int i = d - 1; i >= 0; --i) { nd->X[i] = rf->x[r % n]; r /= n; }
    int off = 0;
    for (int k = 0; k < interval; ++k) off += pb->degree[k];
    nd->nstar = pb->nstar[off + nd->ell - 1];
    double h = pb->t_breaks[interval + 1] - pb->t_breaks[interval];
    nd->span = 0.5 * (rf->xi[nd->ell] + 1.0) * h;      /* t_{n,ell} - t_{n-1}     */
    nd->delta = nd->span / nd->nstar;                   /* eq. time division       */
    return 0;
}

/* eq. uast, the Picard form of the iteration: the integrand is f(u*) plus the
 * source only (the linear part of the operator is carried by the walk) */
static double or_picard_integrand(const or_problem *pb, int interval, const double *Ut,
                                  const double *X, double tau)
{
    double t0 = pb->t_breaks[interval], h = pb->t_breaks[interval + 1] - t0;
    double xi = 2.0 * (tau - t0) / h - 1.0;
    double v[3];
    if (or_is_frac(pb)) or_frac_eval(pb->alpha, pb->n, pb->degree[interval], h, Ut, X[0], xi, v);
    else or_eval(pb->dim, pb->n, pb->degree[interval], h, Ut, X, xi, v);
    return or_f(pb, v[0]) + or_source_iv(pb, interval, X, tau);
}

/* One path of the estimator.  Reading R6: the time of step q runs
 * backward from the node, tau_q = t_{n,ell} - q*Delta.  eq. indexL / interIQ:
 * the jump X_{q+1} = X_q + J*dir (J = sqrt(2 d Delta), Lemma 2.1) is drawn
 * first; if X_{q+1} has left Omega the path stops (L = q) without adding the
 * last inside point, otherwise Delta*r(X_q, tau_q) is added and the walk moves.
 * Picard form (eq. uast): r = f(u*) + s, and a path still inside after all N*
 * steps (it reached t_{n-1}) adds the interval's initial data u*(X_{N*}, t_{n-1});
 * a path that left Omega adds the boundary data g = 0. */
static double or_path(const or_problem *pb, const double *Ut, int inst, int interval,
                      int iter_tag, int64_t node, const or_node *nd, int64_t sample, int64_t *L_out)
{
    int d = pb->dim;
    double t0 = pb->t_breaks[interval];
    double J = sqrt(2.0 * d * nd->delta);
    double X[OR_MAXD], Y[OR_MAXD], dir[OR_MAXD];
    or_stream st;
    or_stream_init(&st, pb->seed, node, sample, inst, interval, iter_tag);
    for (int i = 0; i < d; ++i) X[i] = nd->X[i];
    double acc = 0.0;
    int64_t q;
    for (q = 0; q < nd->nstar; ++q) {
        if (or_is_frac(pb)) {
            /* alpha-stable walk (d = 1): a uniform omega and a fair sign from the
             * Philox block q/2, words 2(q mod 2) and 2(q mod 2) + 1 */
            int64_t blk = q >> 1;
            if (blk != st.blk) { or_stream_block(&st, blk, st.w); st.blk = blk; }
            double om = or_u01(st.w[2 * (q & 1)]);
            dir[0] = (st.w[2 * (q & 1) + 1] & 1u) ? 1.0 : -1.0;
            J = or_frac_jump(pb->alpha, nd->delta, om);
        } else {
            or_direction(&st, d, q, dir);
        }
        int outside = 0;
        for (int i = 0; i < d; ++i) {
            Y[i] = fma(J, dir[i], X[i]);
            if (fabs(Y[i]) >= 1.0) outside = 1;
        }
        if (outside) break;
        double tau = t0 + (nd->span - (double)q * nd->delta);
        const double *E = X;            /* where the step's integrand is evaluated */
        double Z[OR_MAXD];
        if (pb->quad == OR_QUAD_BALL) {
            double off[OR_MAXD];
            or_ball_point(&st, d, q, off);
            for (int i = 0; i < d; ++i) Z[i] = fma(J, off[i], X[i]);
            E = Z;
        }
        if (pb->estimator == OR_EST_PICARD)
            acc += nd->delta * or_picard_integrand(pb, interval, Ut, E, tau);
        else
            acc += nd->delta * or_residual(pb, interval, Ut, E, tau);
        for (int i = 0; i < d; ++i) X[i] = Y[i];
    }
    if (pb->estimator == OR_EST_PICARD && q == nd->nstar) {
        double h = pb->t_breaks[interval + 1] - t0, v[3];
        if (or_is_frac(pb)) or_frac_eval(pb->alpha, pb->n, pb->degree[interval], h, Ut, X[0], -1.0, v);
        else or_eval(d, pb->n, pb->degree[interval], h, Ut, X, -1.0, v);   /* t = t_{n-1}: xi = -1 */
        acc += v[0];
    }
    if (L_out) *L_out = q;
    return acc;
}

static int or_iter_tag(const or_problem *pb, int k) { return pb->fresh_per_iter ? k : 0; }

int or_ball_offset(const or_problem *pb, int inst, int interval, int iter_tag, int64_t node,
                   int64_t sample, int64_t q, double *offset)
{
    if (pb->dim < 1 || pb->dim > OR_MAXD || q < 0 || q >= (1 << 24)) return -1;
    or_stream st;
    or_stream_init(&st, pb->seed, node, sample, inst, interval, iter_tag);
    or_ball_point(&st, pb->dim, q, offset);
    return 0;
}

double or_sample_path(const or_problem *pb, const double *Ut, int inst, int interval,
                      int iter_tag, int64_t node, int64_t sample, int64_t *L_out)
{
    or_node nd;
    or_ref rf;
    or_ref_nodes(pb, interval, &rf);
    if (or_node_info(pb, interval, node, &rf, &nd)) return NAN;
    return or_path(pb, Ut, inst, interval, iter_tag, node, &nd, sample, L_out);
}

/* pairwise (cascade) summation in fixed index order */
static double or_pairwise(const double *v, int64_t n)
{
    if (n <= 8) { double s = 0.0; for (int64_t i = 0; i < n; ++i) s += v[i]; return s; }
    int64_t h = n / 2;
    return or_pairwise(v, h) + or_pairwise(v + h, n - h);
}

int or_estimate(const or_problem *pb, int inst, int interval, int iter_tag,
                const double *U, const int64_t *nodes, int64_t n_nodes,
                int64_t m_lo, int64_t m_hi, double *eps, double *sumsq, int64_t *steps)
{
    int d = pb->dim, n = pb->n, M = pb->degree[interval];
    int64_t nsp = or_ipow(n, d), size = nsp * (M + 1);
    int64_t cnt = m_hi - m_lo;
    if (cnt <= 0 || m_lo < 0) return -1;
    if (or_is_frac(pb)) {
        /* the fractional form: d = 1, residual estimator, centre-point rule */
        if (d != 1 || pb->quad != OR_QUAD_CENTRE) return -2;
        int rc = or_frac_prepare(pb);
        if (rc) return rc;
    }
    double *Ut = malloc(sizeof(double) * size);
    if (!Ut) return -3;
    if (or_is_frac(pb) ? or_frac_reconstruct(pb->alpha, n, M, U, Ut) : or_reconstruct(d, n, M, U, Ut)) {
        free(Ut);
        return -1;
    }
    int64_t total = nodes ? n_nodes : nsp * M;
    int err = 0;
    or_ref rf;
    or_ref_nodes(pb, interval, &rf);
#pragma omp parallel
    {
        double *S = malloc(sizeof(double) * cnt);
        double *S2 = malloc(sizeof(double) * cnt);
        if (!S || !S2) {
#pragma omp atomic write
            err = -3;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t a = 0; a < total; ++a) {
            if (!S || !S2) continue;
            int64_t node = nodes ? nodes[a] : a;
            or_node nd;
            if (or_node_info(pb, interval, node, &rf, &nd)) {
#pragma omp atomic write
                err = -1;
                continue;
            }
            int64_t lsum = 0;
            for (int64_t i = 0; i < cnt; ++i) {
                int64_t L;
                S[i] = or_path(pb, Ut, inst, interval, iter_tag, node, &nd, m_lo + i, &L);
                S2[i] = S[i] * S[i];
                lsum += L;
            }
            eps[a] = or_pairwise(S, cnt) / (double)cnt;       /* eq. varepsilon_1 */
            if (sumsq) sumsq[a] = or_pairwise(S2, cnt);
            if (steps) steps[a] = lsum;
        }
        free(S); free(S2);
    }
    free(Ut);
    return err;
}

/* Algorithm 1, Steps 1-3 for one interval: reconstruct, estimate the residual
 * at every node (j, ell>=1), add it to the nodal values.  Picard form: the
 * estimate replaces the nodal value and max_eps is the largest change. */
int or_iterate(const or_problem *pb, int inst, int interval, int iter_tag,
               double *U, double *max_eps, int64_t *steps)
{
    int d = pb->dim, n = pb->n, M = pb->degree[interval];
    int64_t nsp = or_ipow(n, d), nn = nsp * M;
    double *eps = malloc(sizeof(double) * nn);
    int64_t *st = malloc(sizeof(int64_t) * nn);
    if (!eps || !st) { free(eps); free(st); return -3; }
    int rc = or_estimate(pb, inst, interval, iter_tag, U, NULL, nn, 0, pb->M, eps, NULL, st);
    if (rc) { free(eps); free(st); return rc; }
    double mx = 0.0;
    int64_t tot = 0;
    for (int64_t node = 0; node < nn; ++node) {
        int64_t jf = node % nsp;
        int ell = (int)(node / nsp) + 1;
        double *u = &U[jf * (M + 1) + ell], change;
        if (pb->estimator == OR_EST_PICARD) {
            change = eps[node] - *u;
            *u = eps[node];
        } else {
            change = eps[node];
            *u += eps[node];                               /* Step 3 */
        }
        if (!(fabs(change) <= mx)) mx = fabs(change);     /* NaN propagates */
        tot += st[node];
    }
    if (max_eps) *max_eps = mx;
    if (steps) *steps = tot;
    free(eps); free(st);
    return 0;
}

/* The remark after Algorithm 1: Aitken extrapolation of the iteration as a
 * weighted average of the iterate and its update.  Read as Aitken's
 * delta-squared process for vector sequences in relaxation form (Irons and
 * Tuck, 1969): u <- u + w r, with w the secant estimate of 1/(1 - G') along
 * the last two residuals r of the fixed-point map G. */
static void or_aitken_bounds(const or_problem *pb, double w[3])
{
    w[0] = pb->omega[0] != 0.0 ? pb->omega[0] : 1.0;
    w[1] = pb->omega[1] != 0.0 ? pb->omega[1] : 0.5;
    w[2] = pb->omega[2] != 0.0 ? pb->omega[2] : 2.0;
}

int or_iterate_aitken(const or_problem *pb, int inst, int interval, int iter_tag, double *U,
                      double *r_prev, double state[2], double *max_eps, int64_t *steps)
{
    int d = pb->dim, n = pb->n, M = pb->degree[interval];
    int64_t nsp = or_ipow(n, d), nn = nsp * M;
    double *r = malloc(sizeof(double) * nn);
    int64_t *st = malloc(sizeof(int64_t) * nn);
    if (!r || !st) { free(r); free(st); return -3; }
    int rc = or_estimate(pb, inst, interval, iter_tag, U, NULL, nn, 0, pb->M, r, NULL, st);
    if (rc) { free(r); free(st); return rc; }
    double mx = 0.0, num = 0.0, den = 0.0;
    int64_t tot = 0;
    for (int64_t node = 0; node < nn; ++node) {
        int64_t jf = node % nsp;
        int ell = (int)(node / nsp) + 1;
        if (pb->estimator == OR_EST_PICARD) r[node] -= U[jf * (M + 1) + ell];
        double dr = r[node] - r_prev[node];
        num += r_prev[node] * dr;
        den += dr * dr;
        if (!(fabs(r[node]) <= mx)) mx = fabs(r[node]);
        tot += st[node];
    }
    double wb[3], w;
    or_aitken_bounds(pb, wb);
    if (state[1] == 0.0) w = wb[0];
    else if (den > 0.0) w = -state[0] * num / den;
    else w = state[0];
    if (w < wb[1]) w = wb[1];
    if (w > wb[2]) w = wb[2];
    if (!(w == w)) w = wb[0];
    for (int64_t node = 0; node < nn; ++node) {
        int64_t jf = node % nsp;
        int ell = (int)(node / nsp) + 1;
        U[jf * (M + 1) + ell] += w * r[node];
        r_prev[node] = r[node];
    }
    state[0] = w;
    state[1] = 1.0;
    if (max_eps) *max_eps = mx;
    if (steps) *steps = tot;
    free(r); free(st);
    return 0;
}

static int64_t or_interval_offset(const or_problem *pb, int interval)
{
    int64_t nsp = or_ipow(pb->n, pb->dim), off = 0;
    for (int k = 0; k < interval; ++k) off += nsp * (pb->degree[k] + 1);
    return off;
}

/* Algorithm 1 (sequential intervals; Step 4 hands the last column over), or the
 * Jacobi-in-time sweep schedule of reading R18.  Initial iterate: the initial
 * column replicated in time (reading R12). */
int or_solve(const or_problem *pb, int inst, double *U_all, double *max_eps)
{
    int d = pb->dim, n = pb->n;
    int64_t nsp = or_ipow(n, d);
    double *u0 = malloc(sizeof(double) * nsp);
    if (!u0) return -3;
    int rc = or_ic_nodes(pb, inst, u0);
    if (rc) { free(u0); return rc; }
    if (pb->schedule == OR_SCHED_SEQUENTIAL) {
        for (int iv = 0; iv < pb->n_intervals; ++iv) {
            int M = pb->degree[iv];
            double *U = U_all + or_interval_offset(pb, iv);
            for (int64_t j = 0; j < nsp; ++j) {
                double c0;
                if (iv == 0) c0 = u0[j];
                else {
                    int Mp = pb->degree[iv - 1];
                    c0 = U_all[or_interval_offset(pb, iv - 1) + j * (Mp + 1) + Mp];
                }
                for (int l = 0; l <= M; ++l) U[j * (M + 1) + l] = c0;
            }
            double *rp = NULL, ast[2] = {0.0, 0.0};
            if (pb->accel == OR_ACCEL_AITKEN) {
                rp = calloc((size_t)(nsp * M), sizeof(double));
                if (!rp) { free(u0); return -3; }
            }
            for (int k = 0; k < pb->iters; ++k) {
                double mx;
                if (rp) rc = or_iterate_aitken(pb, inst, iv, or_iter_tag(pb, k), U, rp, ast, &mx, NULL);
                else rc = or_iterate(pb, inst, iv, or_iter_tag(pb, k), U, &mx, NULL);
                if (rc) { free(u0); free(rp); return rc; }
                if (max_eps) max_eps[iv * pb->iters + k] = mx;
            }
            free(rp);
        }
    } else {
        for (int iv = 0; iv < pb->n_intervals; ++iv) {
            int M = pb->degree[iv];
            double *U = U_all + or_interval_offset(pb, iv);
            for (int64_t j = 0; j < nsp; ++j)
                for (int l = 0; l <= M; ++l) U[j * (M + 1) + l] = u0[j];
        }
        double *last = malloc(sizeof(double) * nsp * (pb->n_intervals > 0 ? pb->n_intervals : 1));
        if (!last) { free(u0); return -3; }
        /* Aitken under sweeps: one weight and residual history per interval */
        double **rp = calloc((size_t)pb->n_intervals, sizeof(double *));
        double *ast = calloc((size_t)pb->n_intervals * 2, sizeof(double));
        if (!rp || !ast) { free(u0); free(last); free(rp); free(ast); return -3; }
        for (int iv = 0; iv < pb->n_intervals && pb->accel == OR_ACCEL_AITKEN; ++iv) {
            rp[iv] = calloc((size_t)(nsp * pb->degree[iv]), sizeof(double));
            if (!rp[iv]) rc = -3;
        }
        for (int s = 0; s < pb->iters && !rc; ++s) {
            /* every interval takes column 0 from the previous sweep's last column
             * of the interval before it */
            for (int iv = 0; iv < pb->n_intervals; ++iv) {
                int M = pb->degree[iv];
                const double *U = U_all + or_interval_offset(pb, iv);
                for (int64_t j = 0; j < nsp; ++j) last[iv * nsp + j] = U[j * (M + 1) + M];
            }
            for (int iv = 1; iv < pb->n_intervals; ++iv) {
                int M = pb->degree[iv];
                double *U = U_all + or_interval_offset(pb, iv);
                for (int64_t j = 0; j < nsp; ++j) U[j * (M + 1)] = last[(iv - 1) * nsp + j];
            }
            double mxs = 0.0;
            for (int iv = 0; iv < pb->n_intervals && !rc; ++iv) {
                double mx = 0.0;
                double *Ui = U_all + or_interval_offset(pb, iv);
                if (pb->accel == OR_ACCEL_AITKEN)
                    rc = or_iterate_aitken(pb, inst, iv, or_iter_tag(pb, s), Ui, rp[iv], ast + 2 * iv, &mx, NULL);
                else
                    rc = or_iterate(pb, inst, iv, or_iter_tag(pb, s), Ui, &mx, NULL);
                if (!(mx <= mxs)) mxs = mx;
            }
            if (rc) break;
            if (max_eps) max_eps[s] = mxs;
        }
        for (int iv = 0; iv < pb->n_intervals; ++iv) free(rp[iv]);
        free(rp); free(ast);
        free(last);
        if (rc) { free(u0); return rc; }
    }
    free(u0);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reverse mode of a single-interval solve (gradient with respect to the      */
/* phi-coefficients of the initial data, every path fixed).  The residual is  */
/* affine in the modal coefficients except for f(u*), so                       */
/*   d r / d Ut[p][q] = (f'(u*) L_q(xi) - (2/h) L'_q(xi)) Phi_p(X)             */
/*                      - sum_i (p_i+1)(p_i+2) P_{p_i}(X_i) prod_{m!=i} phi L_q */
/* and the adjoint of U <- U + eps(R U) is lam <- lam + R^T (d eps/d Ut)^T lam. */
/* ------------------------------------------------------------------------ */
static void or_dresidual(const or_problem *pb, int interval, const double *Ut, const double *X,
                         double tau, double weight, double *G)
{
    int dim = pb->dim, n = pb->n, M = pb->degree[interval], T1 = M + 1;
    double t0 = pb->t_breaks[interval], h = pb->t_breaks[interval + 1] - t0;
    double xi = 2.0 * (tau - t0) / h - 1.0;
    double v[3];
    or_eval(dim, n, M, h, Ut, X, xi, v);
    double fp = or_fprime(pb, v[0]);
    double phi[OR_MAXD][OR_MAXN], jac[OR_MAXD][OR_MAXN], Lt[OR_MAXN], dLt[OR_MAXN];
    for (int i = 0; i < dim; ++i) {
        or_jacobi11_all(n - 1, X[i], jac[i]);
        for (int p = 0; p < n; ++p) phi[i][p] = (1.0 - X[i] * X[i]) * jac[i][p];
    }
    or_legendre_all(M, xi, Lt, dLt, NULL);
    int64_t np = or_ipow(n, dim);
    for (int64_t pf = 0; pf < np; ++pf) {
        int pi[OR_MAXD];
        int64_t r = pf;
        for (int i = dim - 1; i >= 0; --i) { pi[i] = (int)(r % n); r /= n; }
        double prodphi = 1.0;
        for (int i = 0; i < dim; ++i) prodphi *= phi[i][pi[i]];
        double lapb = 0.0;
        for (int i = 0; i < dim; ++i) {
            double term = (pi[i] + 1.0) * (pi[i] + 2.0) * jac[i][pi[i]];
            for (int m = 0; m < dim; ++m) if (m != i) term *= phi[m][pi[m]];
            lapb += term;
        }
        for (int q = 0; q < T1; ++q)
            G[pf * T1 + q] += weight * ((fp * Lt[q] - 2.0 / h * dLt[q]) * prodphi - lapb * Lt[q]);
    }
}

static void or_transpose_mat(const double *A, double *At, int n)
{
    for (int a = 0; a < n; ++a) for (int b = 0; b < n; ++b) At[b * n + a] = A[a * n + b];
}

int or_loss_grad(const or_problem *pb, int inst, const double *c0,
                 const double *target, double *loss, double *grad)
{
    int d = pb->dim, n = pb->n, M = pb->degree[0], T1 = M + 1, K = pb->iters;
    int64_t nsp = or_ipow(n, d), size = nsp * T1, nn = nsp * M;
    if (pb->n_intervals != 1 || K < 1) return -1;
    /* the reverse mode below is that of the plain residual iteration */
    if (pb->estimator != OR_EST_RESIDUAL || pb->accel != OR_ACCEL_NONE || pb->quad != OR_QUAD_CENTRE) return -2;
    double x[OR_MAXN], w[OR_MAXN];
    or_jg11(n, x, w);
    /* Phi[j][p] = prod_i phi_{p_i}(x_{j_i}) */
    double *Phi = malloc(sizeof(double) * nsp * nsp);
    double *U = malloc(sizeof(double) * size);
    double *Uts = malloc(sizeof(double) * size * K);
    double *lam = malloc(sizeof(double) * size);
    double *G = malloc(sizeof(double) * size);
    double *t0b = malloc(sizeof(double) * size), *t1b = malloc(sizeof(double) * size);
    double *eps = malloc(sizeof(double) * nn);
    double *A = malloc(sizeof(double) * n * n), *At = malloc(sizeof(double) * n * n);
    double *B = malloc(sizeof(double) * T1 * T1), *Bt = malloc(sizeof(double) * T1 * T1);
    if (!Phi || !U || !Uts || !lam || !G || !t0b || !t1b || !eps || !A || !At || !B || !Bt) return -3;
    for (int64_t j = 0; j < nsp; ++j)
        for (int64_t pf = 0; pf < nsp; ++pf) {
            int64_t rj = j, rp = pf;
            double prod = 1.0;
            for (int i = d - 1; i >= 0; --i) { prod *= or_phi((int)(rp % n), x[rj % n]); rj /= n; rp /= n; }
            Phi[j * nsp + pf] = prod;
        }
    /* forward */
    for (int64_t j = 0; j < nsp; ++j) {
        double s = 0.0;
        for (int64_t pf = 0; pf < nsp; ++pf) s += Phi[j * nsp + pf] * c0[pf];
        for (int l = 0; l < T1; ++l) U[j * T1 + l] = s;
    }
    for (int k = 0; k < K; ++k) {
        or_reconstruct(d, n, M, U, Uts + (int64_t)k * size);
        int rc = or_estimate(pb, inst, 0, or_iter_tag(pb, k), U, NULL, nn, 0, pb->M, eps, NULL, NULL);
        if (rc) return rc;
        for (int64_t node = 0; node < nn; ++node)
            U[(node % nsp) * T1 + node / nsp + 1] += eps[node];
    }
    double L = 0.0;
    for (int64_t j = 0; j < nsp; ++j) { double e = U[j * T1 + M] - target[j]; L += 0.5 * e * e; }
    *loss = L;
    /* backward */
    memset(lam, 0, sizeof(double) * size);
    for (int64_t j = 0; j < nsp; ++j) lam[j * T1 + M] = U[j * T1 + M] - target[j];
    or_matrix_A(n, A); or_transpose_mat(A, At, n);
    or_matrix_B(M, B); or_transpose_mat(B, Bt, T1);
    int nthr = or_num_threads();
    or_ref rf;
    or_ref_nodes(pb, 0, &rf);
    double *Gt = calloc((size_t)size * nthr, sizeof(double));
    if (!Gt) return -3;
    for (int k = K - 1; k >= 0; --k) {
        const double *Ut = Uts + (int64_t)k * size;
        memset(Gt, 0, sizeof(double) * size * nthr);
#pragma omp parallel for schedule(static)
        for (int64_t node = 0; node < nn; ++node) {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double *Gl = Gt + (int64_t)tid * size;
            or_node nd;
            or_node_info(pb, 0, node, &rf, &nd);
            double lamv = lam[(node % nsp) * T1 + nd.ell];
            if (lamv == 0.0) continue;
            double wgt = lamv * nd.delta / (double)pb->M;
            double J = sqrt(2.0 * d * nd.delta);
            for (int64_t smp = 0; smp < pb->M; ++smp) {
                double X[OR_MAXD], Y[OR_MAXD], dir[OR_MAXD];
                or_stream st;
                or_stream_init(&st, pb->seed, node, smp, inst, 0, or_iter_tag(pb, k));
                for (int i = 0; i < d; ++i) X[i] = nd.X[i];
                for (int64_t q = 0; q < nd.nstar; ++q) {
                    or_direction(&st, d, q, dir);
                    int outside = 0;
                    for (int i = 0; i < d; ++i) { Y[i] = fma(J, dir[i], X[i]); if (fabs(Y[i]) >= 1.0) outside = 1; }
                    if (outside) break;
                    double tau = pb->t_breaks[0] + (nd.span - (double)q * nd.delta);
                    or_dresidual(pb, 0, Ut, X, tau, wgt, Gl);
                    for (int i = 0; i < d; ++i) X[i] = Y[i];
                }
            }
        }
        memset(G, 0, sizeof(double) * size);
        for (int t = 0; t < nthr; ++t)
            for (int64_t a = 0; a < size; ++a) G[a] += Gt[(int64_t)t * size + a];
        /* R^T G = G x_1 A^T ... x_d A^T x_t B^T */
        memcpy(t0b, G, sizeof(double) * size);
        for (int i = 0; i < d; ++i) {
            or_mode_product(t0b, t1b, or_ipow(n, i), n, or_ipow(n, d - 1 - i) * T1, At);
            double *t = t0b; t0b = t1b; t1b = t;
        }
        or_mode_product(t0b, t1b, or_ipow(n, d), T1, 1, Bt);
        for (int64_t a = 0; a < size; ++a) lam[a] += t1b[a];
    }
    for (int64_t pf = 0; pf < nsp; ++pf) {
        double s = 0.0;
        for (int64_t j = 0; j < nsp; ++j) {
            double colsum = 0.0;
            for (int l = 0; l < T1; ++l) colsum += lam[j * T1 + l];
            s += Phi[j * nsp + pf] * colsum;
        }
        grad[pf] = s;
    }
    free(Gt); free(Phi); free(U); free(Uts); free(lam); free(G); free(t0b); free(t1b);
    free(eps); free(A); free(At); free(B); free(Bt);
    return 0;
}

/* Table 1 setting: walks of nstar jumps of length sqrt(2 d T / nstar). */
double or_exit_fraction(int dim, double T, int nstar, const double *starts,
                        int64_t nwalk, uint64_t seed)
{
    double J = sqrt(2.0 * dim * T / nstar);
    int64_t exits = 0;
#pragma omp parallel for reduction(+ : exits) schedule(static)
    for (int64_t wlk = 0; wlk < nwalk; ++wlk) {
        double X[OR_MAXD], dir[OR_MAXD];
        or_stream st;
        or_stream_init(&st, seed, wlk, 0, 0, 0, 0);
        for (int i = 0; i < dim; ++i) X[i] = starts[wlk * dim + i];
        for (int q = 0; q < nstar; ++q) {
            or_direction(&st, dim, q, dir);
            int outside = 0;
            for (int i = 0; i < dim; ++i) { X[i] = fma(J, dir[i], X[i]); if (fabs(X[i]) >= 1.0) outside = 1; }
            if (outside) { exits++; break; }
        }
    }
    return (double)exits / (double)nwalk;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
