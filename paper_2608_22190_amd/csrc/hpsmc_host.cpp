// Host runtime of the spectral Monte Carlo hot path: problem validation,
// quadrature and transform set-up, device memory, node scheduling, the
// iteration / interval / sweep drivers and the C ABI of include/hpsmc.h.
#include "hpsmc_internal.h"
#include "hpsmc_lobatto_eigs.h"
#include "../../include/hpsmc.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace hpsmc {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;
// allocator installed by hpsmc_set_allocator (copied into each new plan)
static std::mutex g_alloc_mutex;
static hpsmc_alloc_fn g_alloc_fn = nullptr;
static hpsmc_free_fn g_free_fn = nullptr;
static void *g_alloc_ctx = nullptr;
static thread_local bool g_capturing = false;   // no event records inside a stream capture

static hpsmc_status fail(hpsmc_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            plan->poisoned = true;                                                           \
            return fail(HPSMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
        }                                                                                    \
    } while (0)

// ---------------------------------------------------------------------------
// Gauss rules by the Golub-Welsch route: nodes are eigenvalues of the Jacobi
// matrix of the three-term recurrence (Sturm-sequence bisection), weights are
// Christoffel numbers 1 / sum_k p_k(x)^2 of the orthonormal polynomials.
// ---------------------------------------------------------------------------
static int sturm_count(const std::vector<double> &e2, int n, double x)
{
    // zero diagonal (symmetric weights); e2[k] = beta_k, k = 1..n-1
    int cnt = 0;
    double d = -x;
    if (d < 0) ++cnt;
    for (int k = 1; k < n; ++k) {
        if (d == 0.0) d = 1e-300;
        d = -x - e2[k] / d;
        if (d < 0) ++cnt;
    }
    return cnt;
}

static void gauss_rule_e2(int n, double mu0, const std::vector<double> &e2, std::vector<double> &x,
                          std::vector<double> &w);

static void gauss_rule(int n, double mu0, double (*beta)(int), std::vector<double> &x, std::vector<double> &w)
{
    std::vector<double> e2(n + 1, 0.0);
    for (int k = 1; k < n; ++k) e2[k] = beta(k);
    gauss_rule_e2(n, mu0, e2, x, w);
}

// e2[k] = beta_k (k = 1..n-1) of the monic recurrence, mu0 = integral of the weight
static void gauss_rule_e2(int n, double mu0, const std::vector<double> &e2, std::vector<double> &x,
                          std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double lo = -1.0, hi = 1.0;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (sturm_count(e2, n, mid) > i) hi = mid; else lo = mid;
        }
        x[i] = 0.5 * (lo + hi);
    }
    for (int i = 0; i < n; ++i) {
        double pm = 0.0, pc = 1.0 / std::sqrt(mu0), s = pc * pc;
        for (int k = 0; k + 1 < n; ++k) {
            const double ek1 = std::sqrt(e2[k + 1]), ek = k > 0 ? std::sqrt(e2[k]) : 0.0;
            const double pn = (x[i] * pc - ek * pm) / ek1;
            pm = pc;
            pc = pn;
            s += pc * pc;
        }
        w[i] = 1.0 / s;
    }
}

static double beta_legendre(int k) { return double(k) * k / (4.0 * k * k - 1.0); }

// ---------------------------------------------------------------------------
// Fractional operator (Ex. 2-3), d = 1: symmetric Jacobi polynomials of
// parameter a = alpha/2 in the standard normalization,
//   P_{k+1} = A_k x P_k - C_k P_{k-1},  A_k = (2k+2a+1)(2k+2a+2) / (2(k+1)(k+2a+1)),
//   C_k = (k+a)^2 (2k+2a+2) / ((k+1)(k+2a+1)(2k+2a)),
// their Gauss rule for the weight (1-x^2)^a (monic beta_k = k(k+2a) /
// ((2k+2a+1)(2k+2a-1)), mu0 = 2^{2a+1} Gamma(a+1)^2 / Gamma(2a+2)) and norms
//   gamma_k = 2^{2a+1} Gamma(k+a+1)^2 / ((2k+2a+1) k! Gamma(k+2a+1)).
// ---------------------------------------------------------------------------
static void jacobi_rec(int kmax, double a, std::vector<double> &A, std::vector<double> &C)
{
    A.assign(kmax, 0.0);
    C.assign(kmax, 0.0);
    const double s2 = 2.0 * a;
    for (int k = 0; k < kmax; ++k) {
        A[k] = (2.0 * k + s2 + 1.0) * (2.0 * k + s2 + 2.0) / (2.0 * (k + 1.0) * (k + s2 + 1.0));
        C[k] = (k + a) * (k + a) * (2.0 * k + s2 + 2.0) / ((k + 1.0) * (k + s2 + 1.0) * (2.0 * k + s2));
    }
}

static void jacobi_values(int kmax, const std::vector<double> &A, const std::vector<double> &C, double x, double *P)
{
    double pm = 0.0, pc = 1.0;
    for (int k = 0; k < kmax; ++k) {
        P[k] = pc;
        const double pn = A[k] * x * pc - C[k] * pm;
        pm = pc;
        pc = pn;
    }
}

static void gauss_jacobi_aa(int n, double a, std::vector<double> &x, std::vector<double> &w)
{
    std::vector<double> e2(n + 1, 0.0);
    for (int k = 1; k < n; ++k) e2[k] = k * (k + 2.0 * a) / ((2.0 * k + 2.0 * a + 1.0) * (2.0 * k + 2.0 * a - 1.0));
    const double mu0 = std::exp((2.0 * a + 1.0) * std::log(2.0) + 2.0 * std::lgamma(a + 1.0) - std::lgamma(2.0 * a + 2.0));
    gauss_rule_e2(n, mu0, e2, x, w);
}

static double jacobi_norm2(int k, double a)
{
    return std::exp((2.0 * a + 1.0) * std::log(2.0) + 2.0 * std::lgamma(k + a + 1.0) - std::lgamma(k + 1.0) -
                    std::lgamma(k + 2.0 * a + 1.0)) / (2.0 * k + 2.0 * a + 1.0);
}

static bool is_frac(const hpsmc_problem &pb) { return pb.alpha > 0.0 && pb.alpha < 2.0; }

// the spatial factor g of the fractional manufactured solutions
static double frac_g(const hpsmc_problem &pb, double x)
{
    switch (pb.src_kind) {
    case HPSMC_SRC_FRAC_LONGTIME: return std::sin(x);
    case HPSMC_SRC_FRAC_SINGULAR: return std::cos(x * x * x + 1.0) / (10.0 * x * x + 1.0);
    case HPSMC_SRC_FRAC_POLY: return pb.src_param[0] + x * (pb.src_param[1] + x * pb.src_param[2]);
    }
    return 0.0;
}

static double frac_T(const hpsmc_problem &pb, double t)
{
    switch (pb.src_kind) {
    case HPSMC_SRC_FRAC_LONGTIME: return std::exp(std::cos(t)) / (1.0 + t * t);
    case HPSMC_SRC_FRAC_SINGULAR: return std::pow(t, pb.src_param[0]);
    case HPSMC_SRC_FRAC_POLY: return 1.0 + pb.src_param[3] * t;
    }
    return 0.0;
}
static double beta_jacobi11(int k) { return double(k) * (k + 2) / ((2.0 * k + 1.0) * (2.0 * k + 3.0)); }

static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) { gauss_rule(n, 2.0, beta_legendre, x, w); }
static void jacobi_gauss11(int n, std::vector<double> &x, std::vector<double> &w) { gauss_rule(n, 4.0 / 3.0, beta_jacobi11, x, w); }

// Legendre-Gauss-Lobatto on [-1,1]: end points plus the JG(1,1) nodes; the
// interior weights are the JG(1,1) Christoffel numbers divided by (1 - x^2).
static void lobatto(int M, std::vector<double> &xi, std::vector<double> &w)
{
    xi.assign(M + 1, 0.0);
    w.assign(M + 1, 0.0);
    xi[0] = -1.0;
    xi[M] = 1.0;
    w[0] = w[M] = 2.0 / (M * (M + 1.0));
    if (M > 1) {
        std::vector<double> x, wj;
        jacobi_gauss11(M - 1, x, wj);
        for (int k = 1; k < M; ++k) {
            xi[k] = x[k - 1];
            w[k] = wj[k - 1] / (1.0 - x[k - 1] * x[k - 1]);
        }
    }
}

static void legendre_values(int kmax, double x, double *L)
{
    L[0] = 1.0;
    if (kmax >= 1) L[1] = x;
    for (int m = 1; m < kmax; ++m) L[m + 1] = ((2.0 * m + 1.0) * x * L[m] - m * L[m - 1]) / (m + 1.0);
}

// Legendre coefficients (P modes) of the spatial Lagrange basis of the
// JG(1,1) nodes, l_j(x) = (1-x^2)/(1-x_j^2) prod_{m != j}(x-x_m)/(x_j-x_m)
// (eq. spacelag): G[k][j] = (2k+1)/2 int l_j L_k, by exact Gauss-Legendre.
static std::vector<double> spatial_to_legendre(const std::vector<double> &xn, int P)
{
    const int n = (int)xn.size();
    std::vector<double> xq, wq;
    gauss_legendre(n + 3, xq, wq);
    std::vector<double> G((size_t)P * n, 0.0), L(P + 1);
    for (size_t a = 0; a < xq.size(); ++a) {
        legendre_values(P, xq[a], L.data());
        for (int j = 0; j < n; ++j) {
            double lj = (1.0 - xq[a] * xq[a]) / (1.0 - xn[j] * xn[j]);
            for (int m = 0; m < n; ++m)
                if (m != j) lj *= (xq[a] - xn[m]) / (xn[j] - xn[m]);
            for (int k = 0; k < P; ++k) G[(size_t)k * n + j] += (2.0 * k + 1.0) / 2.0 * wq[a] * lj * L[k];
        }
    }
    return G;
}

// Legendre coefficients of the temporal Lagrange basis on the LGL nodes (eq. timeLag).
static std::vector<double> temporal_to_legendre(const std::vector<double> &xi)
{
    const int T1 = (int)xi.size();
    std::vector<double> xq, wq;
    gauss_legendre(T1 + 1, xq, wq);
    std::vector<double> B((size_t)T1 * T1, 0.0), L(T1 + 1);
    for (size_t a = 0; a < xq.size(); ++a) {
        legendre_values(T1, xq[a], L.data());
        for (int k = 0; k < T1; ++k) {
            double hk = 1.0;
            for (int m = 0; m < T1; ++m)
                if (m != k) hk *= (xq[a] - xi[m]) / (xi[k] - xi[m]);
            for (int q = 0; q < T1; ++q) B[(size_t)q * T1 + k] += (2.0 * q + 1.0) / 2.0 * wq[a] * hk * L[q];
        }
    }
    return B;
}

// Legendre-basis differentiation: (c')_q = (2q+1) sum_{m>q, m-q odd} c_m;
// (c'')_k = (k+1/2) sum_{m>=k+2, m-k even} (m(m+1) - k(k+1)) c_m.
static std::vector<double> legendre_d1(int N)
{
    std::vector<double> D((size_t)N * N, 0.0);
    for (int q = 0; q < N; ++q)
        for (int m = q + 1; m < N; m += 2) D[(size_t)q * N + m] = 2.0 * q + 1.0;
    return D;
}
// A[j][k] (N x N): the Chebyshev coefficients of L_k, L_k = sum_j A[j][k] T_j,
// from the Legendre recurrence and x T_j = (T_{j+1} + T_{|j-1|}) / 2
static std::vector<double> legendre_to_chebyshev(int N)
{
    std::vector<std::vector<double>> c(N, std::vector<double>(N + 1, 0.0));
    c[0][0] = 1.0;
    if (N > 1) c[1][1] = 1.0;
    for (int k = 1; k + 1 < N; ++k) {
        std::vector<double> xc(N + 1, 0.0);   // x L_k
        for (int j = 0; j <= k; ++j) {
            if (j == 0) { xc[1] += c[k][0]; continue; }
            xc[j + 1] += 0.5 * c[k][j];
            xc[j - 1] += 0.5 * c[k][j];
        }
        const double a = (2.0 * k + 1.0) / (k + 1.0), b = double(k) / (k + 1.0);
        for (int j = 0; j <= k + 1; ++j) c[k + 1][j] = a * xc[j] - b * c[k - 1][j];
    }
    std::vector<double> A((size_t)N * N);
    for (int j = 0; j < N; ++j)
        for (int k = 0; k < N; ++k) A[(size_t)j * N + k] = c[k][j];
    return A;
}

static std::vector<double> legendre_d2(int N)
{
    std::vector<double> D((size_t)N * N, 0.0);
    for (int k = 0; k < N; ++k)
        for (int m = k + 2; m < N; m += 2) D[(size_t)k * N + m] = (k + 0.5) * (m * (m + 1.0) - k * (k + 1.0));
    return D;
}

// ---------------------------------------------------------------------------
// Exact solutions of the manufactured sources and initial data.
// ---------------------------------------------------------------------------
static double exact_solution(const hpsmc_problem &pb, const double *X, double t)
{
    const int d = pb.dim;
    const double pi = 3.14159265358979323846;
    if (pb.src_kind >= HPSMC_SRC_FRAC_LONGTIME)
        return std::pow(1.0 - X[0] * X[0], 0.5 * pb.alpha) * frac_g(pb, X[0]) * frac_T(pb, t);
    switch (pb.src_kind) {
    case HPSMC_SRC_SIN_DECAY: { double p = std::exp(-t); for (int i = 0; i < d; ++i) p *= std::sin(pi * X[i]); return p; }
    case HPSMC_SRC_COS_DECAY: { double p = std::exp(-t); for (int i = 0; i < d; ++i) p *= std::cos(0.5 * pi * X[i]); return p; }
    case HPSMC_SRC_LONGTIME: {
        double a = 1.0, s = 0.0;
        for (int i = 0; i < d; ++i) { a *= 1.0 - X[i] * X[i]; s += X[i]; }
        return a * std::sin(s) * std::exp(std::cos(t)) / (1.0 + t * t);
    }
    case HPSMC_SRC_QUAD: {
        double a = 1.0;
        for (int i = 0; i < d; ++i) a *= 1.0 - X[i] * X[i];
        return a * (pb.src_param[0] + pb.src_param[1] * t + pb.src_param[2] * t * t);
    }
    }
    return 0.0;
}

// phi_p in the Legendre form 2(p+1)/(2p+3) (L_p - L_{p+2})
static double phi_legendre(int p, const double *L) { return 2.0 * (p + 1) / (2.0 * p + 3.0) * (L[p] - L[p + 2]); }

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct NodeSet {               // the nodes one sampling launch covers
    std::vector<NodeDesc> host;
    NodeDesc *dev = nullptr;
    int64_t n = 0;
    // slab groups
    int32_t n_groups = 0, max_nstar = 0;
    int64_t slab_elems = 0;
    int64_t slab_elems_row = 0;   // the row layout's extent (the slab adjoint's table)
    void *group_mem = nullptr; // coef_off, slab_off, span, delta, h2, nstar, deg
    SlabArgs slab{};
    // outputs (canonical order)
    double *eps = nullptr, *sumsq = nullptr, *probe = nullptr;
    int64_t probe_cap = 0;
    std::vector<int32_t> ivs;  // intervals covered
    // round-based sampling (slabs staged in LDS)
    bool rounds = false;
    std::vector<GroupDesc> ghost;
    GroupDesc *gdev = nullptr;
    int64_t ms = 0;            // samples per slice
    void *state[2] = {nullptr, nullptr};
    uint32_t *live = nullptr;  // [2][n_groups]
    int64_t *prefix = nullptr; // [n_groups + 1]
    double *result = nullptr;  // [n][ms]
    // Aitken-relaxed update: one vector per (interval of the set, instance)
    int32_t n_vec = 0;
    int64_t *vbeg = nullptr;   // [n_vec + 1] node ranges
    double *ait = nullptr;     // [2 n_vec] {w_prev, have_prev}, then e_prev [n]
};

}  // namespace hpsmc

struct hpsmc_plan {
    hpsmc_problem pb{};
    hpsmc_alloc_fn alloc_fn = nullptr;   // device workspaces (null: hipMalloc / hipFree)
    hpsmc_free_fn free_fn = nullptr;
    void *alloc_ctx = nullptr;
    int64_t ainv_off = 0;                // nodal -> phi-coefficient matrix A = Phi^{-1} (n x n)
    std::vector<double> t_breaks;
    std::vector<int32_t> degree, nstar;   // N* resolved at creation (explicit array or the rule)
    std::vector<double> dt_max;           // per interval: the rule's step bound (0: explicit array)
    std::vector<double> ic_data;
    int d = 0, n = 0, P = 0, PP = 0, n_iv = 0, n_inst = 0;
    int64_t nsp = 0, psp = 0;   // n^d, P^d
    std::vector<double> x;      // spatial nodes
    std::vector<std::vector<double>> xi, tnodes;   // per interval: reference LGL nodes, t_{n,l}
    bool fp32 = false, poisoned = false;
    hpsmc_plan *twin = nullptr;   // HPSMC_FP32_THEN_FP64: the FP64 plan the solve switches to
    std::vector<char> twin_last;  // per interval: its last iteration ran on the twin
    int cus = 0;
    hpsmc_launch launch{2, 4, 8, 256};
    int32_t round_steps = 256;           // walk steps per round
    size_t round_budget = (size_t)16 << 30;   // bytes for path states and per-sample results

    // device memory
    double *U = nullptr;                 // all intervals, [iv block][inst][j][l]
    std::vector<int64_t> u_off;          // per interval
    double *cu = nullptr, *cv = nullptr; // [iv block][inst][P^d][T1]
    std::vector<int64_t> c_off;          // per interval
    // 2-D plans the matrix-core kernel can serve: c^u, c^v (and a polynomial
    // source) in the Chebyshev basis of both spatial dimensions, the slab image's basis
    double *cu_ch = nullptr, *cv_ch = nullptr, *cs_ch = nullptr;
    int64_t cheb_off = -1;               // in mats: Legendre -> Chebyshev, A[j][k] = coefficient of T_j in L_k
    double *tmp0 = nullptr, *tmp1 = nullptr;
    double *ic = nullptr;                // [inst][nsp]
    double *mats = nullptr;              // G0 (P x n), D2 (P x P), then per interval Bt, D1
    std::vector<int64_t> bt_off, d1_off;
    int64_t g0t_off = 0, d2t_off = 0, phi_off = 0, phit_off = 0;   // transposes and the phi collocation
    std::vector<int64_t> btt_off, d1t_off;
    // adjoint buffers (allocated on the first gradient call)
    double *hist_u = nullptr, *hist_v = nullptr, *lam = nullptr, *cbar_u = nullptr, *cbar_v = nullptr;
    double *dtarget = nullptr, *dloss = nullptr, *dgrad = nullptr;
    void *slab_bar = nullptr;
    int32_t adj_use_mfma = 1;
    // hipGraph of a whole solve (captured on the first graph solve, replayed after)
    int32_t use_graph = 0;
    int32_t sample_mma = 1;     // FP32 round kernels on the matrix cores where eligible (2-D, 5-D)
    int32_t sample_split = 1;   // sparse rounds of the 5-D matrix-core kernel on all waves of a block
    int32_t sample_1d = 1;      // d = 1 rounds on the windowed 1-D kernel where eligible
    // fractional operator (d = 1): tables of the round kernel (see Physics)
    bool frac = false;
    double *frac_tab = nullptr;
    int32_t frac_kmax = 0, frac_K = 0, frac_nt = 0;
    // polynomial source: per interval [P^d][T1] tensor-Legendre coefficients
    double *src_poly = nullptr;
    std::vector<int64_t> src_off;
    double frac_half = 0.0, frac_lpb1 = 0.0, frac_lpb2 = 0.0;
    bool capturing = false;
    hipStream_t own_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int64_t graph_node_samples = 0;
    int32_t graph_records = 0;
    void *slab_table = nullptr;
    size_t slab_bytes = 0;
    double *part = nullptr;
    int64_t part_elems = 0;
    unsigned long long *counters = nullptr;  // [0] work, [1] evals, [2] lane steps, [3] unused
    unsigned long long *maxbits = nullptr;   // [4096]
    int64_t m_probe = 0;
    std::vector<hpsmc::NodeSet> sets;        // sequential: one per interval; sweeps: one
    int64_t node_samples = 0;
    // HIP-event timing of the sampling, slab and reconstruction kernels
    struct EvPair { hipEvent_t a = nullptr, b = nullptr; };
    std::vector<EvPair> ev_sample, ev_slab, ev_recon, ev_span, ev_adj;
    size_t n_sample = 0, n_slab = 0, n_recon = 0, n_span = 0, n_adj = 0;
    int64_t n_advance = 0;                   // advance-kernel launches (round mode)
    int32_t n_records = 0, sweep_count = 0;
};

namespace hpsmc {

static int64_t ipow(int64_t b, int e)
{
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// next event pair of a pool (created on first use); null when the pool is full
static hpsmc_plan::EvPair *next_pair(std::vector<hpsmc_plan::EvPair> &pool, size_t &used)
{
    if (used >= 16384 || g_capturing) return nullptr;
    if (used == pool.size()) {
        hpsmc_plan::EvPair e;
        if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        pool.push_back(e);
    }
    return &pool[used++];
}

static double pool_ms(const std::vector<hpsmc_plan::EvPair> &pool, size_t used)
{
    double tot = 0.0;
    for (size_t i = 0; i < used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pool[i].a, pool[i].b) == hipSuccess) tot += ms;
        else (void)hipGetLastError();
    }
    return tot;
}

// LDS chunking of a slab: the first cf dimensions fixed per chunk.  The two
// options per dimension are those the kernel is instantiated for.  Returns
// false when no option fits four 16-byte vectors per thread.
static bool pick_chunking(const hpsmc_plan *plan, int nthr, int *cf, int64_t *chunk_elems, int *n_chunks)
{
    const int d = plan->d;
    const int opts[2] = {d <= 3 ? 0 : d - 3, d <= 1 ? 0 : (d <= 3 ? 1 : d - 2)};
    const int T = plan->fp32 ? 4 : 8;
    for (int o = 0; o < 2; ++o) {
        const int c = opts[o];
        const int64_t rows = ipow(plan->P, d - 1 - c);
        const int64_t elems = rows * 2 * plan->PP;
        if (elems * T / 16 <= 4LL * nthr) {
            *cf = c;
            *chunk_elems = elems;
            *n_chunks = (int)ipow(plan->P, c);
            return true;
        }
    }
    return false;
}

// first weight and bounds of the Aitken relaxation; zeros select 1, 0.5, 2
static void aitken_weights(const hpsmc_problem *pb, double w[3])
{
    w[0] = pb->omega[0] != 0.0 ? pb->omega[0] : 1.0;
    w[1] = pb->omega[1] != 0.0 ? pb->omega[1] : 0.5;
    w[2] = pb->omega[2] != 0.0 ? pb->omega[2] : 2.0;
}

static hpsmc_status validate(const hpsmc_problem *pb)
{
    if (!pb) return fail(HPSMC_EINVAL, "problem is NULL");
    if (pb->dim < 1 || pb->dim > 5) return fail(HPSMC_EINVAL, "dim must be 1..5");
    if (pb->n < 1 || pb->n > kMaxN) return fail(HPSMC_EINVAL, "n must be 1..32");
    if (pb->n_intervals < 1 || pb->n_intervals > 255) return fail(HPSMC_EINVAL, "n_intervals must be 1..255");
    if (pb->n_instances < 1 || pb->n_instances > 65535) return fail(HPSMC_EINVAL, "n_instances must be 1..65535");
    if (pb->nstar_mode < HPSMC_NSTAR_ARRAY || pb->nstar_mode > HPSMC_NSTAR_SPECTRAL)
        return fail(HPSMC_EINVAL, "unknown nstar_mode");
    if (!pb->t_breaks || !pb->degree || (pb->nstar_mode == HPSMC_NSTAR_ARRAY && !pb->nstar))
        return fail(HPSMC_EINVAL, "t_breaks/degree/nstar is NULL");
    if (pb->nstar_mode != HPSMC_NSTAR_ARRAY && (pb->nstar_min < 0 || pb->nstar_min >= (1 << 24)))
        return fail(HPSMC_EINVAL, "nstar_min must be 0 (4) .. 2^24-1");
    if (pb->nstar_mode == HPSMC_NSTAR_DT && !(std::isfinite(pb->dt_max) && pb->dt_max > 0.0))
        return fail(HPSMC_EINVAL, "dt_max must be finite and > 0");
    if (pb->nstar_mode == HPSMC_NSTAR_SPECTRAL && !(std::isfinite(pb->nstar_c) && pb->nstar_c >= 0.0))
        return fail(HPSMC_EINVAL, "nstar_c must be finite and >= 0 (0 selects 0.25)");
    for (int i = 0; i <= pb->n_intervals; ++i)
        if (!std::isfinite(pb->t_breaks[i])) return fail(HPSMC_EINVAL, "t_breaks must be finite");
    for (int i = 0; i < pb->n_intervals; ++i) {
        if (!(pb->t_breaks[i + 1] > pb->t_breaks[i])) return fail(HPSMC_EINVAL, "t_breaks must increase strictly");
        if (pb->degree[i] < 1 || pb->degree[i] > kMaxDeg) return fail(HPSMC_EINVAL, "degree must be 1..31");
    }
    int64_t tot = 0;
    for (int i = 0; i < pb->n_intervals; ++i) tot += pb->degree[i];
    if (pb->nstar_mode == HPSMC_NSTAR_ARRAY)
        for (int64_t k = 0; k < tot; ++k)
            if (pb->nstar[k] < 1 || pb->nstar[k] >= (1 << 24)) return fail(HPSMC_EINVAL, "nstar must be 1..2^24-1");
    if (pb->M < 1 || pb->M > (int64_t)0xFFFFFFFFll) return fail(HPSMC_EINVAL, "M must be 1..2^32-1");
    if (pb->iters < 1 || pb->iters > 255) return fail(HPSMC_EINVAL, "iters must be 1..255");
    if (pb->f_kind < 0 || pb->f_kind > 5) return fail(HPSMC_EINVAL, "unknown f_kind");
    if (pb->src_kind < 0 || pb->src_kind > HPSMC_SRC_POLY) return fail(HPSMC_EINVAL, "unknown src_kind");
    if (!std::isfinite(pb->alpha) || pb->alpha < 0.0 || pb->alpha > 2.0)
        return fail(HPSMC_EINVAL, "alpha must be 0 (the Laplacian) or in (0, 2]");
    if (is_frac(*pb)) {
        if (pb->dim != 1) return fail(HPSMC_ENOTSUP, "the fractional operator is built for d = 1");
        if (pb->src_kind != HPSMC_SRC_NONE && pb->src_kind < HPSMC_SRC_FRAC_LONGTIME)
            return fail(HPSMC_EINVAL, "the Laplacian's manufactured sources do not solve the fractional problem");
        if (pb->quad != HPSMC_QUAD_CENTRE)
            return fail(HPSMC_ENOTSUP, "the fractional form takes the centre-point rule");
        if (pb->ic_kind != HPSMC_IC_EXACT && pb->ic_kind != HPSMC_IC_NODAL)
            return fail(HPSMC_ENOTSUP, "the fractional form takes IC_EXACT or IC_NODAL");
    } else if (pb->src_kind >= HPSMC_SRC_FRAC_LONGTIME && pb->src_kind <= HPSMC_SRC_FRAC_POLY) {
        return fail(HPSMC_EINVAL, "fractional sources need 0 < alpha < 2");
    }
    if (pb->src_kind == HPSMC_SRC_POLY) {
        if (is_frac(*pb)) return fail(HPSMC_ENOTSUP, "the polynomial source is built for the Laplacian");
        if (pb->estimator != HPSMC_EST_RESIDUAL)
            return fail(HPSMC_ENOTSUP, "the polynomial source enters the residual form's v* slab only");
        if (!pb->src_coeffs) return fail(HPSMC_EINVAL, "src_coeffs is NULL");
        const int64_t P = pb->n + 2;
        int64_t len = 0, pd = 1;
        for (int i = 0; i < pb->dim; ++i) pd *= P;
        for (int i = 0; i < pb->n_intervals; ++i) len += pd * (pb->degree[i] + 1);
        if (pb->src_len != len) return fail(HPSMC_EINVAL, "src_len must be sum_n (n+2)^dim (M_n+1)");
        for (int64_t k = 0; k < len; ++k)
            if (!std::isfinite(pb->src_coeffs[k])) return fail(HPSMC_EINVAL, "src_coeffs must be finite");
        if (pb->ic_kind == HPSMC_IC_EXACT) return fail(HPSMC_EINVAL, "the polynomial source has no exact solution");
    }
    if (pb->ic_kind < 0 || pb->ic_kind > 3) return fail(HPSMC_EINVAL, "unknown ic_kind");
    if (pb->schedule < 0 || pb->schedule > 1) return fail(HPSMC_EINVAL, "unknown schedule");
    if (pb->precision < 0 || pb->precision > HPSMC_FP32_THEN_FP64) return fail(HPSMC_EINVAL, "unknown precision");
    if (pb->precision == HPSMC_FP32_THEN_FP64) {
        if (!(std::isfinite(pb->switch_tol) && pb->switch_tol > 0.0))
            return fail(HPSMC_EINVAL, "switch_tol must be finite and > 0");
        if (pb->estimator != HPSMC_EST_RESIDUAL || pb->accel != HPSMC_ACCEL_NONE)
            return fail(HPSMC_ENOTSUP, "the precision switch covers the plain residual iteration");
    }
    if (!std::isfinite(pb->tol) || pb->tol < 0.0) return fail(HPSMC_EINVAL, "tol must be finite and >= 0");
    if (pb->tol > 0.0 && pb->schedule == HPSMC_SEQUENTIAL && (int64_t)pb->n_intervals * pb->iters > 4096)
        return fail(HPSMC_EINVAL, "tolerance mode keeps one max|eps| record per (interval, iteration): "
                                  "n_intervals * iters must be <= 4096");
    if (pb->estimator < 0 || pb->estimator > 1) return fail(HPSMC_EINVAL, "unknown estimator");
    if (pb->accel < 0 || pb->accel > 1) return fail(HPSMC_EINVAL, "unknown accel");
    if (pb->quad < 0 || pb->quad > 1) return fail(HPSMC_EINVAL, "unknown quad");
    if (pb->accel == HPSMC_ACCEL_AITKEN) {
        double w[3];
        aitken_weights(pb, w);
        if (!(std::isfinite(w[0]) && std::isfinite(w[1]) && std::isfinite(w[2]) && w[1] > 0.0 && w[1] <= w[0] &&
              w[0] <= w[2]))
            return fail(HPSMC_EINVAL, "Aitken weights need 0 < omega[1] <= omega[0] <= omega[2]");
    }
    if ((pb->ic_kind == HPSMC_IC_PHI || pb->ic_kind == HPSMC_IC_NODAL) && !pb->ic_data)
        return fail(HPSMC_EINVAL, "ic_data is NULL");
    if (pb->ic_kind == HPSMC_IC_EXACT && pb->src_kind == HPSMC_SRC_NONE)
        return fail(HPSMC_EINVAL, "IC_EXACT needs a source with an exact solution");
    const int P = pb->n + 2;
    if ((pb->dim == 5 && P > 12) || (pb->dim == 4 && P > 20))
        return fail(HPSMC_ENOTSUP, "too many modes for this dimension (d=5: n<=10, d=4: n<=18)");
    return HPSMC_OK;
}

// device workspaces: hipMalloc/hipFree, or the allocator installed by
// hpsmc_set_allocator when the plan was created
static hpsmc_status dalloc(hpsmc_plan *plan, void **p, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    if (plan->alloc_fn) {
        *p = plan->alloc_fn(bytes, nullptr, plan->alloc_ctx);
        if (!*p) return fail(HPSMC_ENOMEM, "allocator hook returned NULL for " + std::to_string(bytes) + " bytes");
        return HPSMC_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(HPSMC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return HPSMC_OK;
}

static void dfree(const hpsmc_plan *plan, void *p)
{
    if (!p) return;
    if (plan->free_fn) plan->free_fn(p, nullptr, plan->alloc_ctx);
    else (void)hipFree(p);
}

// Expected path length used to order work (longest first): the walk leaves
// the box after roughly min_i (1 - x_i^2)/2 time units, capped by the node's span.
static double expected_cost(const NodeDesc &nd, int d)
{
    double tex = 1.0;
    for (int i = 0; i < d; ++i) tex = std::min(tex, 0.5 * (1.0 - nd.x0[i] * nd.x0[i]));
    const double steps = std::min((double)nd.nstar, tex / nd.delta + 1.0);
    return steps;
}

// sphere radius of a walk step: sqrt(2 d Delta) (Lemma 2.1), or for the
// alpha-stable walk the ball radius whose mean exit time from the centre is
// Delta, (Delta Gamma(1+alpha))^{1/alpha} in 1-D
static double walk_radius(const hpsmc_plan *plan, double delta)
{
    if (plan->frac) return std::pow(delta * std::exp(std::lgamma(1.0 + plan->pb.alpha)), 1.0 / plan->pb.alpha);
    return std::sqrt(2.0 * plan->d * delta);
}

// whether some launch shape runs this plan's rounds on a matrix-core kernel
static bool mma_capable(const hpsmc_plan *plan)
{
    if (plan->d == 5)
        return advance_mma5_eligible(plan->fp32, 5, plan->P, plan->pb.estimator == HPSMC_EST_PICARD,
                                     plan->pb.quad == HPSMC_QUAD_BALL, 1, 4);
    return advance_mma_eligible(plan->fp32, plan->d, plan->P, 0, 1, 4);
}

static hpsmc_status build_set(hpsmc_plan *plan, NodeSet &set, const std::vector<int32_t> &ivs)
{
    const int d = plan->d;
    set.ivs = ivs;
    set.host.clear();
    std::vector<int64_t> coef_off, slab_off, slab_off_mma, src_goff;
    std::vector<double> span, delta, h2;
    std::vector<int32_t> nst, deg;
    const int64_t rows = ipow(plan->P, d - 1);
    const int64_t stride = rows * 2 * plan->PP;
    // plans a matrix-core round kernel can serve also get offsets in its slab layout
    const bool mma_ok = mma_capable(plan);
    const int extra = plan->pb.estimator == HPSMC_EST_PICARD ? 1 : 0;   // the slab of q = N* (t = t_{n-1})
    const int64_t mstride = d == 5 ? mma5_geom(plan->P).step : mma_slab_elems(plan->PP);
    int64_t slab_pos = 0, slab_pos_mma = 0, out = 0;
    // canonical output order: [iv][inst][node id]
    for (int32_t iv : ivs) {
        const int M = plan->degree[iv];
        const double h = plan->t_breaks[iv + 1] - plan->t_breaks[iv];
        int noff = 0;
        for (int k = 0; k < iv; ++k) noff += plan->degree[k];
        for (int inst = 0; inst < plan->n_inst; ++inst) {
            for (int l = 1; l <= M; ++l) {
                const int ns = plan->nstar[noff + l - 1];
                const double sp = 0.5 * (plan->xi[iv][l] + 1.0) * h;
                const double dl = sp / ns;
                const int g = (int)coef_off.size();
                coef_off.push_back(plan->c_off[iv] + (int64_t)inst * plan->psp * (M + 1));
                src_goff.push_back(plan->src_poly ? plan->src_off[iv] : 0);
                slab_off.push_back(slab_pos);
                slab_off_mma.push_back(slab_pos_mma);
                span.push_back(sp);
                delta.push_back(dl);
                h2.push_back(2.0 / h);
                nst.push_back(ns);
                deg.push_back(M);
                (void)g;
                for (int64_t j = 0; j < plan->nsp; ++j) {
                    NodeDesc nd{};
                    int64_t r = j;
                    for (int i = d - 1; i >= 0; --i) { nd.x0[i] = plan->x[r % plan->n]; r /= plan->n; }
                    nd.delta = dl;
                    nd.jump = walk_radius(plan, dl);
                    nd.span = sp;
                    nd.t_prev = plan->t_breaks[iv];
                    nd.u_index = plan->u_off[iv] + ((int64_t)inst * plan->nsp + j) * (M + 1) + l;
                    nd.slab = slab_pos;
                    nd.nstar = ns;
                    nd.c0 = (uint32_t)(j + plan->nsp * (l - 1));
                    nd.c3 = ((uint32_t)inst << 16) | ((uint32_t)iv << 8);
                    nd.out = (int32_t)(out + inst * plan->nsp * M + (int64_t)(l - 1) * plan->nsp + j);
                    set.host.push_back(nd);
                }
                slab_pos += (int64_t)(ns + extra) * stride;
                if (mma_ok) slab_pos_mma += (int64_t)(ns + extra) * mstride;
            }
        }
        out += (int64_t)plan->n_inst * plan->nsp * M;
    }
    set.n = (int64_t)set.host.size();
    if (set.n > (int64_t)0x7fffffff) return fail(HPSMC_EINVAL, "too many nodes");
    // rounds stream the slab of a step through LDS in chunks of at most 4 vectors per thread
    {
        int cf, nc;
        int64_t ce;
        set.rounds = pick_chunking(plan, 256, &cf, &ce, &nc);
    }
    if (set.rounds) {
        // group descriptors: nodes were generated group by group
        const int64_t per = plan->nsp;
        for (size_t g = 0; g < coef_off.size(); ++g) {
            GroupDesc gd{};
            gd.delta = delta[g];
            gd.jump = walk_radius(plan, delta[g]);
            gd.span = span[g];
            gd.node_begin = (int32_t)(g * per);
            gd.node_count = (int32_t)per;
            gd.t_prev = set.host[g * per].t_prev;
            gd.slab = slab_off[g];
            gd.slab_mma = slab_off_mma[g];
            gd.nstar = nst[g];
            gd.c3 = set.host[g * per].c3;
            set.ghost.push_back(gd);
        }
    } else if (plan->pb.accel != HPSMC_ACCEL_AITKEN) {
        // longest expected paths first (stable for determinism); the Aitken
        // update reads its vectors as contiguous ranges of the generation order,
        // so relaxed plans keep that order
        std::stable_sort(set.host.begin(), set.host.end(), [d](const NodeDesc &a, const NodeDesc &b) {
            return expected_cost(a, d) > expected_cost(b, d);
        });
    }
    set.n_groups = (int32_t)coef_off.size();
    set.max_nstar = *std::max_element(nst.begin(), nst.end());
    set.slab_elems = std::max(slab_pos, slab_pos_mma);   // one layout is live at a time
    set.slab_elems_row = slab_pos;
    hpsmc_status st;
    if ((st = dalloc(plan, (void **)&set.dev, sizeof(NodeDesc) * set.n))) return st;
    const size_t G = set.n_groups;
    const size_t gbytes = G * (4 * sizeof(int64_t) + 3 * sizeof(double) + 2 * sizeof(int32_t));
    if ((st = dalloc(plan, &set.group_mem, gbytes))) return st;
    std::vector<char> gh(gbytes);
    char *p = gh.data();
    auto put = [&](const void *src, size_t b) { memcpy(p, src, b); p += b; };
    put(coef_off.data(), G * 8); put(slab_off.data(), G * 8);
    put(span.data(), G * 8); put(delta.data(), G * 8); put(h2.data(), G * 8);
    put(nst.data(), G * 4); put(deg.data(), G * 4);
    put(slab_off_mma.data(), G * 8);
    put(src_goff.data(), G * 8);
    if (hipMemcpy(set.group_mem, gh.data(), gbytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(set.dev, set.host.data(), sizeof(NodeDesc) * set.n, hipMemcpyHostToDevice) != hipSuccess)
        return fail(HPSMC_EDEVICE, "upload of node descriptors failed");
    char *gb = (char *)set.group_mem;
    SlabArgs &sa = set.slab;
    sa.cu = plan->cu;
    sa.cv = plan->cv;
    sa.coef_off = (const int64_t *)gb;
    sa.slab_off = (const int64_t *)(gb + G * 8);
    sa.span = (const double *)(gb + G * 16);
    sa.delta = (const double *)(gb + G * 24);
    sa.h2 = (const double *)(gb + G * 32);
    sa.nstar = (const int32_t *)(gb + G * 40);
    sa.deg = (const int32_t *)(gb + G * 44);
    sa.slab_off_mma = mma_ok ? (const int64_t *)(gb + G * 48) : nullptr;
    sa.cs = plan->src_poly;
    sa.cs_off = (const int64_t *)(gb + G * 56);
    sa.mma_stride = mstride;
    sa.layout = 0;
    sa.extra = extra;
    sa.n_groups = set.n_groups;
    sa.P = plan->P;
    sa.PP = plan->PP;
    sa.rows = (int32_t)rows;
    sa.slab_stride = stride;
    if ((st = dalloc(plan, (void **)&set.eps, sizeof(double) * set.n))) return st;
    if ((st = dalloc(plan, (void **)&set.sumsq, sizeof(double) * set.n))) return st;
    if (plan->pb.accel == HPSMC_ACCEL_AITKEN) {
        // nodes were generated interval by interval, instance by instance
        std::vector<int64_t> vb(1, 0);
        for (int32_t iv : ivs)
            for (int inst = 0; inst < plan->n_inst; ++inst) vb.push_back(vb.back() + plan->nsp * plan->degree[iv]);
        set.n_vec = (int32_t)(vb.size() - 1);
        if ((st = dalloc(plan, (void **)&set.vbeg, sizeof(int64_t) * vb.size()))) return st;
        if ((st = dalloc(plan, (void **)&set.ait, sizeof(double) * (2 * set.n_vec + set.n)))) return st;
        if (hipMemcpy(set.vbeg, vb.data(), sizeof(int64_t) * vb.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(set.ait, 0, sizeof(double) * (2 * set.n_vec + set.n)) != hipSuccess)
            return fail(HPSMC_EDEVICE, "Aitken state upload failed");
    }
    if (set.rounds) {
        const size_t sb = path_state_bytes(plan->fp32, d);
        const int64_t per_sample = (int64_t)(2 * sb + sizeof(double));
        int64_t ms = (int64_t)(plan->round_budget / (size_t)(per_sample * set.n));
        ms = std::max<int64_t>(1, std::min<int64_t>(ms, plan->pb.M));
        set.ms = ms;
        for (size_t g = 0; g < set.ghost.size(); ++g) set.ghost[g].path_off = (int64_t)set.ghost[g].node_begin * ms;
        const size_t G = set.ghost.size();
        if ((st = dalloc(plan, (void **)&set.gdev, sizeof(GroupDesc) * G))) return st;
        if ((st = dalloc(plan, &set.state[0], sb * set.n * ms))) return st;
        if ((st = dalloc(plan, &set.state[1], sb * set.n * ms))) return st;
        if ((st = dalloc(plan, (void **)&set.live, sizeof(uint32_t) * 2 * G))) return st;
        if ((st = dalloc(plan, (void **)&set.prefix, sizeof(int64_t) * (G + 2)))) return st;
        if ((st = dalloc(plan, (void **)&set.result, sizeof(double) * set.n * ms))) return st;
        if (hipMemcpy(set.gdev, set.ghost.data(), sizeof(GroupDesc) * G, hipMemcpyHostToDevice) != hipSuccess)
            return fail(HPSMC_EDEVICE, "upload of group descriptors failed");
    }
    return HPSMC_OK;
}

static void free_set(const hpsmc_plan *plan, NodeSet &s)
{
    for (void *p : {(void *)s.dev, s.group_mem, (void *)s.eps, (void *)s.sumsq, (void *)s.probe, (void *)s.gdev,
                    s.state[0], s.state[1], (void *)s.live, (void *)s.prefix, (void *)s.result, (void *)s.vbeg,
                    (void *)s.ait})
        dfree(plan, p);
    s = NodeSet{};
}

// initial nodal values [inst][nsp], computed on the host in FP64
// nodal -> Jacobi coefficients of u/w (fractional basis): c_p = sum_j A[p][j] U_j,
// A[p][j] = P_p(x_j) w_j / ((1 - x_j^2)^a gamma_p), exact by the Gauss rule
static std::vector<double> frac_nodal_to_modal(const std::vector<double> &x, const std::vector<double> &w, double a)
{
    const int n = (int)x.size();
    std::vector<double> A, C, Pv(n), M((size_t)n * n);
    jacobi_rec(n, a, A, C);
    for (int j = 0; j < n; ++j) {
        jacobi_values(n, A, C, x[j], Pv.data());
        const double wt = std::pow(1.0 - x[j] * x[j], a);
        for (int p = 0; p < n; ++p) M[(size_t)p * n + j] = Pv[p] * w[j] / (wt * jacobi_norm2(p, a));
    }
    return M;
}

// ---------------------------------------------------------------------------
// Path lengths N* (eq. time division: N* depends on h_n and l).  The residual
// estimator weighs the node itself with Delta, so a nodal error mode of the
// interval's discrete operator A_h = d_t - Lap_h (or d_t + (-Lap)^{alpha/2}_h)
// with eigenvalue lambda is scaled by about (1 - Delta lambda) per iteration;
// the rule keeps Delta_{n,l} <= c / rho(A_h).  A_h is the Kronecker sum of the
// temporal collocation derivative (2/h) D_t on the Lobatto times l >= 1
// (column 0 is held) and d copies of the spatial collocation operator K
// (-Lap_h, or the fractional Laplacian, on the Jacobi-Gauss nodes).  Its
// eigenvalues are (2/h) mu_j + sum_i kappa_i; K has real positive eigenvalues
// and D_t eigenvalues of positive real part, so the largest modulus takes
// kappa_i = rho(K) in every dimension: rho(A_h) = max_j |(2/h) mu_j + d rho(K)|.
// rho(K) comes from Gelfand's formula (||K^m||^{1/m}, m = 2^k by repeated
// squaring; K is close enough to normal for it); the mu_j of D_t, whose
// eigen-problem is too ill-conditioned for double precision at high degree,
// come from a table computed once at 60 digits (gen_lobatto_eigs.py).
// ---------------------------------------------------------------------------
static_assert(kLobattoEigMaxDeg >= kMaxDeg, "the Lobatto eigenvalue table must cover every temporal degree");

static double spectral_radius(std::vector<double> A, int n)
{
    auto fro = [](const std::vector<double> &B) {
        double s = 0.0;
        for (double v : B) s += v * v;
        return std::sqrt(s);
    };
    double c = fro(A);
    if (!(c > 0.0) || !std::isfinite(c)) return c > 0.0 ? c : 0.0;
    for (double &v : A) v /= c;
    // A^{2^k} = prod_j c_j^{2^{k-j}} A_k with ||A_k|| = 1: log rho ~ sum_j 2^{-j} log c_j
    double logr = std::log(c), scale = 1.0;
    std::vector<double> B((size_t)n * n);
    for (int k = 1; k <= 64; ++k) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double t = 0.0;
                for (int m = 0; m < n; ++m) t += A[(size_t)i * n + m] * A[(size_t)m * n + j];
                B[(size_t)i * n + j] = t;
            }
        const double c2 = fro(B);
        if (!(c2 > 0.0)) return 0.0;   // nilpotent
        scale *= 0.5;
        const double inc = scale * std::log(c2);
        logr += inc;
        for (double &v : B) v /= c2;
        std::swap(A, B);
        if (k >= 12 && std::fabs(inc) < 1e-18) break;
    }
    return std::exp(logr);
}

// spatial collocation operator on the n nodes: -Lap_h in one dimension
// (Legendre route: nodal -> Legendre coefficients of phi-space interpolant,
// second derivative, values at the nodes), or the fractional Laplacian
// (nodal -> Jacobi coefficients of u/w, eigenvalues lambda_p, values of P_p)
static std::vector<double> spatial_operator(const hpsmc_problem &pb, const std::vector<double> &x,
                                            const std::vector<double> &w)
{
    const int n = (int)x.size();
    std::vector<double> K((size_t)n * n, 0.0);
    if (is_frac(pb)) {
        const double a = 0.5 * pb.alpha;
        const auto G = frac_nodal_to_modal(x, w, a);
        std::vector<double> A, C, Pv(n);
        jacobi_rec(n, a, A, C);
        for (int m = 0; m < n; ++m) {
            jacobi_values(n, A, C, x[m], Pv.data());
            for (int p = 0; p < n; ++p) {
                const double lp = std::exp(std::lgamma(p + pb.alpha + 1.0) - std::lgamma(p + 1.0)) * Pv[p];
                for (int j = 0; j < n; ++j) K[(size_t)m * n + j] += lp * G[(size_t)p * n + j];
            }
        }
        return K;
    }
    const int P = n + 2;
    const auto G = spatial_to_legendre(x, P);
    const auto D2 = legendre_d2(P);
    std::vector<double> DG((size_t)P * n, 0.0), L(P + 1);
    for (int k = 0; k < P; ++k)
        for (int m = 0; m < P; ++m)
            if (D2[(size_t)k * P + m] != 0.0)
                for (int j = 0; j < n; ++j) DG[(size_t)k * n + j] += D2[(size_t)k * P + m] * G[(size_t)m * n + j];
    for (int m = 0; m < n; ++m) {
        legendre_values(P, x[m], L.data());
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < n; ++j) K[(size_t)m * n + j] -= L[k] * DG[(size_t)k * n + j];
    }
    return K;
}

// N* of every node time l >= 1 of every interval, and the step bound per
// interval (0 for explicit arrays)
static hpsmc_status resolve_nstar(const hpsmc_problem &pb, std::vector<int32_t> &nstar, std::vector<double> &dt_max)
{
    const int NH = pb.n_intervals;
    int64_t tot = 0;
    for (int i = 0; i < NH; ++i) tot += pb.degree[i];
    nstar.clear();
    dt_max.assign(NH, 0.0);
    if (pb.nstar_mode == HPSMC_NSTAR_ARRAY) {
        nstar.assign(pb.nstar, pb.nstar + tot);
        return HPSMC_OK;
    }
    const int nmin = pb.nstar_min > 0 ? pb.nstar_min : 4;
    double kappa = 0.0;
    if (pb.nstar_mode == HPSMC_NSTAR_SPECTRAL) {
        std::vector<double> x, w;
        if (is_frac(pb)) gauss_jacobi_aa(pb.n, 0.5 * pb.alpha, x, w);
        else jacobi_gauss11(pb.n, x, w);
        kappa = (is_frac(pb) ? 1.0 : (double)pb.dim) * spectral_radius(spatial_operator(pb, x, w), pb.n);
    }
    for (int iv = 0; iv < NH; ++iv) {
        const int M = pb.degree[iv];
        const double h = pb.t_breaks[iv + 1] - pb.t_breaks[iv];
        std::vector<double> xi, wt;
        lobatto(M, xi, wt);
        double dt = pb.dt_max;
        if (pb.nstar_mode == HPSMC_NSTAR_SPECTRAL) {
            double rho = 0.0;
            for (int k = kLobattoEigOff[M]; k < kLobattoEigOff[M + 1]; ++k)
                rho = std::max(rho, std::hypot(2.0 / h * kLobattoEig[k][0] + kappa, 2.0 / h * kLobattoEig[k][1]));
            dt = (pb.nstar_c > 0.0 ? pb.nstar_c : 0.25) / rho;
        }
        dt_max[iv] = dt;
        for (int l = 1; l <= M; ++l) {
            // a quotient within rounding of an integer is not carried to the next one
            const double steps = std::ceil((1.0 - 1e-12) * 0.5 * (xi[l] + 1.0) * h / dt);
            if (!(steps < (double)(1 << 24))) return fail(HPSMC_EINVAL, "the path-length rule gives N* >= 2^24");
            nstar.push_back(std::max(nmin, (int32_t)steps));
        }
    }
    return HPSMC_OK;
}

// tables of the fractional round kernel: recurrence, eigenvalues, the source
// series sum_k a_k lambda_k P_k = (-Delta)^{alpha/2}(w g) (a_k the Jacobi
// coefficients of g by a 160-point Gauss rule), the series ratios of the
// inverse incomplete beta; and its branch point and constants
static hpsmc_status frac_tables(hpsmc_plan *plan)
{
    const double alpha = plan->pb.alpha, a = 0.5 * alpha, b = 1.0 - a;
    const int P = plan->P;
    int K = 0;
    switch (plan->pb.src_kind) {
    case HPSMC_SRC_FRAC_LONGTIME: K = 40; break;
    case HPSMC_SRC_FRAC_SINGULAR: K = 150; break;
    case HPSMC_SRC_FRAC_POLY: K = 3; break;
    }
    const int kmax = std::max(P, K), nt = plan->fp32 ? 26 : 60;
    std::vector<double> A, C;
    jacobi_rec(kmax, a, A, C);
    std::vector<double> tab(A);
    tab.insert(tab.end(), C.begin(), C.end());
    for (int k = 0; k < P; ++k) tab.push_back(std::exp(std::lgamma(k + alpha + 1.0) - std::lgamma(k + 1.0)));
    if (K > 0) {
        std::vector<double> xq, wq, Pv(K);
        gauss_jacobi_aa(160, a, xq, wq);
        std::vector<double> ck(K, 0.0);
        for (size_t j = 0; j < xq.size(); ++j) {
            jacobi_values(K, A, C, xq[j], Pv.data());
            const double g = frac_g(plan->pb, xq[j]);
            for (int k = 0; k < K; ++k) ck[k] += wq[j] * g * Pv[k];
        }
        for (int k = 0; k < K; ++k)
            tab.push_back(ck[k] / jacobi_norm2(k, a) * std::exp(std::lgamma(k + alpha + 1.0) - std::lgamma(k + 1.0)));
    }
    for (int k = 0; k < nt; ++k) tab.push_back((k + 1.0) / (a + 1.0 + k));
    for (int k = 0; k < nt; ++k) tab.push_back((k + 1.0) / (b + 1.0 + k));
    plan->frac_kmax = kmax;
    plan->frac_K = K;
    plan->frac_nt = nt;
    plan->frac_lpb1 = std::log(a) + std::lgamma(a) + std::lgamma(b);
    plan->frac_lpb2 = std::log(b) + std::lgamma(a) + std::lgamma(b);
    // I_{1/2}(a, b) by its series (x = 1/2): x^a (1-x)^b / (a B) sum_k t_k
    double S = 1.0, t = 1.0;
    for (int k = 0; k < 200; ++k) { t *= 0.5 * (k + 1.0) / (a + 1.0 + k); S += t; }
    plan->frac_half = std::exp(-std::log(2.0) - plan->frac_lpb1) * S;
    // start tables of the inverse per branch (p = a with log(a B), p = b with
    // log(b B)): at X0_i = i X0max / kFracTab the converged log x minus log X0_i,
    // by the kernel's Newton iteration run in FP64 with 200 series terms, where
    // X0max = e^{z0} at x = 1/2 (z0 the small-x asymptote of the branch)
    double x0max[2];
    for (int br = 0; br < 2; ++br) {
        const double p = br ? b : a, lpb = br ? plan->frac_lpb2 : plan->frac_lpb1;
        auto series = [&](double x) {
            double Ss = 1.0, tt = 1.0;
            for (int k = 0; k < 200; ++k) { tt *= x * (k + 1.0) / (p + 1.0 + k); Ss += tt; }
            return Ss;
        };
        const double lhalf = -std::log(2.0);
        const double l_half_cdf = lhalf - lpb + std::log(series(0.5));   // log I_{1/2}(p, 1-p)
        x0max[br] = std::exp((l_half_cdf + lpb) / p);
        tab.push_back(0.0);   // X0 -> 0: x / X0 -> 1
        for (int i = 1; i <= kFracTab; ++i) {
            const double lx0 = std::log(x0max[br] * i / kFracTab), ly = p * lx0 - lpb;
            double z = std::min(lx0, lhalf);
            for (int it = 0; it < 60; ++it) {
                const double x = std::exp(z), Sx = series(x);
                const double lI = p * z + (1.0 - p) * std::log1p(-x) - lpb + std::log(Sx);
                z = std::min(z - (lI - ly) * (1.0 - x) * Sx / p, lhalf);
            }
            tab.push_back(z - lx0);
        }
    }
    tab.push_back(x0max[0]);
    tab.push_back(x0max[1]);
    hpsmc_status st;
    if ((st = dalloc(plan, (void **)&plan->frac_tab, tab.size() * 8))) return st;
    if (hipMemcpy(plan->frac_tab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        return fail(HPSMC_EDEVICE, "fractional table upload failed");
    return HPSMC_OK;
}

static void initial_nodes(const hpsmc_plan *plan, std::vector<double> &u0)
{
    const int d = plan->d, n = plan->n;
    u0.assign((size_t)plan->n_inst * plan->nsp, 0.0);
    std::vector<std::vector<double>> Lx(n, std::vector<double>(n + 3));
    for (int j = 0; j < n; ++j) legendre_values(n + 2, plan->x[j], Lx[j].data());
    for (int inst = 0; inst < plan->n_inst; ++inst)
        for (int64_t jf = 0; jf < plan->nsp; ++jf) {
            int ji[kMaxDim];
            double X[kMaxDim];
            int64_t r = jf;
            for (int i = d - 1; i >= 0; --i) { ji[i] = (int)(r % n); X[i] = plan->x[ji[i]]; r /= n; }
            double v = 0.0;
            switch (plan->pb.ic_kind) {
            case HPSMC_IC_EXACT: v = exact_solution(plan->pb, X, plan->t_breaks[0]); break;
            case HPSMC_IC_SINGULAR:
                v = std::pow(std::fabs(X[0]), plan->pb.ic_param[0]);
                for (int i = 0; i < d; ++i) v *= 1.0 - X[i] * X[i];
                break;
            case HPSMC_IC_PHI: {
                const double *c = plan->ic_data.data() + (size_t)inst * plan->nsp;
                for (int64_t pf = 0; pf < plan->nsp; ++pf) {
                    int64_t rr = pf;
                    double prod = 1.0;
                    for (int i = d - 1; i >= 0; --i) { prod *= phi_legendre((int)(rr % n), Lx[ji[i]].data()); rr /= n; }
                    v += c[pf] * prod;
                }
                break;
            }
            case HPSMC_IC_NODAL: v = plan->ic_data[(size_t)inst * plan->nsp + jf]; break;
            }
            u0[(size_t)inst * plan->nsp + jf] = v;
        }
}

// ---------------------------------------------------------------------------
// Device pipeline pieces
// ---------------------------------------------------------------------------
static hpsmc_status reconstruct(hpsmc_plan *plan, int iv, hipStream_t s)
{
    const int d = plan->d, n = plan->n, P = plan->P, T1 = plan->degree[iv] + 1;
    const double h = plan->t_breaks[iv + 1] - plan->t_breaks[iv];
    const double *G0 = plan->mats, *D2 = plan->mats + (size_t)P * n;
    const double *Bt = plan->mats + plan->bt_off[iv], *D1 = plan->mats + plan->d1_off[iv];
    double *cu = plan->cu + plan->c_off[iv], *cv = plan->cv + plan->c_off[iv];
    const int64_t I = plan->n_inst;
    hpsmc_plan::EvPair *ev = next_pair(plan->ev_recon, plan->n_recon);
    if (ev) HIP_TRY(hipEventRecord(ev->a, s));
    // c^u = U x_1 G0 ... x_d G0 x_t Bt
    const double *in = plan->U + plan->u_off[iv];
    double *bufs[2] = {plan->tmp0, plan->tmp1};
    for (int i = 0; i < d; ++i) {
        double *o = bufs[i & 1];
        HIP_TRY(launch_mode_product(in, o, I * ipow(P, i), n, P, ipow(n, d - 1 - i) * T1, G0, 1.0, 0, s));
        in = o;
    }
    HIP_TRY(launch_mode_product(in, cu, I * plan->psp, T1, T1, 1, Bt, 1.0, 0, s));
    // c^v = sum_i c^u x_i D2 - (2/h) c^u x_t D1   (Lap u - d_t u)
    for (int i = 0; i < d; ++i)
        HIP_TRY(launch_mode_product(cu, cv, I * ipow(P, i), P, P, ipow(P, d - 1 - i) * T1, D2, 1.0, i > 0, s));
    HIP_TRY(launch_mode_product(cu, cv, I * plan->psp, T1, T1, 1, D1, -2.0 / h, 1, s));
    if (ev) HIP_TRY(hipEventRecord(ev->b, s));
    return HPSMC_OK;
}

static Physics physics_of(const hpsmc_plan *plan)
{
    Physics ph{};
    ph.dim = plan->d;
    ph.f_kind = plan->pb.f_kind;
    ph.src_kind = plan->pb.src_kind == HPSMC_SRC_POLY ? HPSMC_SRC_NONE : plan->pb.src_kind;   // in the v slab
    ph.picard = plan->pb.estimator == HPSMC_EST_PICARD;
    ph.ball = plan->pb.quad == HPSMC_QUAD_BALL;
    ph.frac = plan->frac ? 1 : 0;
    ph.frac_kmax = plan->frac_kmax;
    ph.frac_K = plan->frac_K;
    ph.frac_nt = plan->frac_nt;
    ph.frac_P = plan->P;
    ph.frac_a = 0.5 * plan->pb.alpha;
    ph.frac_half = plan->frac_half;
    ph.frac_lpb1 = plan->frac_lpb1;
    ph.frac_lpb2 = plan->frac_lpb2;
    ph.frac_tab = plan->frac_tab;
    memcpy(ph.f_param, plan->pb.f_param, sizeof(ph.f_param));
    memcpy(ph.src_param, plan->pb.src_param, sizeof(ph.src_param));
    return ph;
}

static bool one_sample_per_lane(const hpsmc_plan *plan)
{
    return plan->frac || plan->pb.estimator == HPSMC_EST_PICARD || plan->pb.quad == HPSMC_QUAD_BALL;
}

// Whether the rounds run the windowed 1-D kernel with ns paths per lane
static bool uses_1d(const hpsmc_plan *plan, int ns)
{
    return plan->sample_1d && advance_1d_eligible(plan->d, plan->P, plan->pb.estimator == HPSMC_EST_PICARD,
                                                  plan->pb.quad == HPSMC_QUAD_BALL, plan->frac ? 1 : 0, ns);
}

static int set_uses_mma(const hpsmc_plan *plan, const NodeSet &set);

// Whether the rounds of this set run the windowed 1-D kernel with the current
// launch shape (its slabs then hold Chebyshev coefficients)
static bool set_uses_1d(const hpsmc_plan *plan, const NodeSet &set)
{
    return set.rounds && set_uses_mma(plan, set) == 0 &&
           uses_1d(plan, one_sample_per_lane(plan) ? 1 : plan->launch.samples_per_lane);
}

// Whether the rounds of this set run a matrix-core kernel with the current
// launch shape (its slabs are then written in that kernel's layout): 1 the
// 2-D kernel, 2 the 5-D kernel, 0 neither.
static int set_uses_mma(const hpsmc_plan *plan, const NodeSet &set)
{
    if (!set.rounds || !plan->sample_mma || !set.slab.slab_off_mma) return 0;
    if (plan->d == 5)
        return advance_mma5_eligible(plan->fp32, plan->d, plan->P, plan->pb.estimator == HPSMC_EST_PICARD,
                                     plan->pb.quad == HPSMC_QUAD_BALL,
                                     one_sample_per_lane(plan) ? 1 : plan->launch.samples_per_lane,
                                     plan->launch.waves_per_block) ? 2 : 0;
    int cf, nc;
    int64_t ce;
    if (!pick_chunking(plan, 64 * plan->launch.waves_per_block, &cf, &ce, &nc)) return 0;
    return advance_mma_eligible(plan->fp32, plan->d, plan->P, cf,
                                one_sample_per_lane(plan) ? 1 : plan->launch.samples_per_lane,
                                plan->launch.waves_per_block) ? 1 : 0;
}

// Round-based sampling of one node set: slices of samples, each advanced in
// rounds of round_steps walk steps with compaction between rounds.
// reduce-kernel mode: bit 0 Picard form, bit 1 the Aitken kernel applies the update
static int update_mode(const hpsmc_plan *plan)
{
    return (plan->pb.estimator == HPSMC_EST_PICARD ? 1 : 0) | (plan->pb.accel == HPSMC_ACCEL_AITKEN ? 2 : 0);
}

static hpsmc_status aitken_update(hpsmc_plan *plan, NodeSet &set, hipStream_t s)
{
    if (plan->pb.accel != HPSMC_ACCEL_AITKEN) return HPSMC_OK;
    double w[3];
    aitken_weights(&plan->pb, w);
    HIP_TRY(launch_aitken(set.dev, set.vbeg, set.n_vec, set.eps, set.ait + 2 * set.n_vec, set.ait, w[0], w[1], w[2],
                          plan->U, s));
    return HPSMC_OK;
}

// restart the Aitken history of interval iv (every instance)
static hpsmc_status aitken_reset(hpsmc_plan *plan, int iv, hipStream_t s)
{
    if (plan->pb.accel != HPSMC_ACCEL_AITKEN) return HPSMC_OK;
    const bool seq = plan->pb.schedule == HPSMC_SEQUENTIAL;
    NodeSet &set = seq ? plan->sets[iv] : plan->sets[0];
    const int64_t v0 = (int64_t)(seq ? 0 : iv) * plan->n_inst;
    HIP_TRY(launch_fill_u64((unsigned long long *)(set.ait + 2 * v0), 2 * (int64_t)plan->n_inst, 0ull, s));
    return HPSMC_OK;
}

static hpsmc_status sample_rounds(hpsmc_plan *plan, NodeSet &set, int tag, int record, hipStream_t s)
{
    // the fractional kernel, the Picard form and the ball-point rule run one sample per lane
    const int ns = one_sample_per_lane(plan) ? 1 : plan->launch.samples_per_lane, waves = plan->launch.waves_per_block;
    const int nthr = 64 * waves;
    const int mma = set_uses_mma(plan, set);
    int cf = 0, n_chunks = 1;
    int64_t chunk_elems = 0;
    if (mma != 2 && !pick_chunking(plan, nthr, &cf, &chunk_elems, &n_chunks))
        return fail(HPSMC_EINVAL, "slab chunk too large for this block size; use more waves per block");
    const int64_t nvec = chunk_elems * (plan->fp32 ? 4 : 8) / 16;
    const bool k1d = set_uses_1d(plan, set);
    const size_t lds = k1d ? advance_1d_lds_bytes(plan->fp32, set.slab.slab_stride)
                     : mma == 2 ? advance_mma5_lds_bytes(plan->P)
                     : mma ? advance_mma_lds_bytes(plan->PP)
                     : plan->frac ? frac_lds_bytes(plan->fp32, plan->PP, plan->frac_kmax, plan->P, plan->frac_K,
                                                   plan->frac_nt)
                                  : (size_t)2 * ((nvec + 1) & ~1LL) * 16;
    const int C = plan->round_steps;
    const int R = (set.max_nstar + C - 1) / C;
    const int G = (int)set.ghost.size();
    RoundArgs a{};
    a.groups = set.gdev;
    a.nodes = set.dev;
    a.n_groups = G;
    a.steps = C;
    a.batch = nthr * ns;
    a.batch_prefix = set.prefix;
    a.result = set.result;
    a.cf = cf;
    a.n_chunks = n_chunks;
    a.chunk_elems = chunk_elems;
    a.P = plan->P;
    a.PP = plan->PP;
    a.tag = tag;
    a.key0 = (uint32_t)plan->pb.seed;
    a.key1 = (uint32_t)(plan->pb.seed >> 32);
    a.slab_table = plan->slab_table;
    a.slab_stride = mma ? set.slab.mma_stride : set.slab.slab_stride;
    a.work = plan->counters;
    a.stats = plan->counters + 1;
    a.phys = physics_of(plan);
    const int blocks = std::max(1, plan->cus * plan->launch.blocks_per_cu);
    // rounds of the 5-D matrix-core kernel whose paths fit in one pass of the
    // grid at 64 paths per block run each item on all the block's waves (two or
    // four), each taking a share of every tile's products.  (The 2-D kernel does
    // several vector instructions per product, which a split wave repeats: it
    // measured no faster.)
    const int split_batch = mma == 2 && plan->sample_split && (waves == 2 || waves == 4) ? 64 : 0;
    const int64_t split_max = blocks;
    hpsmc_plan::EvPair *ek = next_pair(plan->ev_span, plan->n_span);
    if (ek) HIP_TRY(hipEventRecord(ek->a, s));
    int first = 1;
    for (int64_t m0 = 0; m0 < plan->pb.M; m0 += set.ms) {
        const int64_t mc = std::min<int64_t>(set.ms, plan->pb.M - m0);
        a.m0 = m0;
        a.mcount = mc;
        for (int r = 0; r < R; ++r) {
            a.round = r;
            a.state_in = set.state[r & 1];
            a.state_out = set.state[(r + 1) & 1];
            a.live_in = set.live + (r & 1) * G;
            a.live_out = set.live + ((r + 1) & 1) * G;
            HIP_TRY(launch_round_prep(set.gdev, G, r, C, mc, a.batch, split_batch, split_max, a.live_in, a.live_out,
                                      set.prefix, plan->counters, s));
            hpsmc_plan::EvPair *ea = next_pair(plan->ev_sample, plan->n_sample);
            if (ea) HIP_TRY(hipEventRecord(ea->a, s));
            HIP_TRY(launch_advance(a, plan->fp32, ns, waves, blocks, lds, k1d ? 3 : mma, s));
            if (ea) HIP_TRY(hipEventRecord(ea->b, s));
        }
        HIP_TRY(launch_slice_reduce(set.result, set.n, mc, plan->part, first, s));
        if (set.probe && plan->m_probe > 0 && m0 == 0)
            HIP_TRY(hipMemcpy2DAsync(set.probe, plan->m_probe * 8, set.result, mc * 8,
                                     std::min<int64_t>(plan->m_probe, mc) * 8, set.n, hipMemcpyDeviceToDevice, s));
        first = 0;
    }
    if (ek) HIP_TRY(hipEventRecord(ek->b, s));
    plan->n_advance += (int64_t)R * ((plan->pb.M + set.ms - 1) / set.ms);
    unsigned long long *mb = plan->maxbits + std::min(record, 4095);
    HIP_TRY(launch_reduce_update(plan->part, 1, update_mode(plan), set.dev, set.n, plan->pb.M, plan->U, set.eps,
                                 set.sumsq, mb, s));
    if (hpsmc_status st = aitken_update(plan, set, s)) return st;
    plan->node_samples += set.n * plan->pb.M;
    plan->n_records = std::max(plan->n_records, std::min(record, 4095) + 1);
    return HPSMC_OK;
}

// Slab arguments for `layout`: the 2-D matrix-core image (layout 1) holds
// Chebyshev coefficients in both spatial dimensions, so c^u and c^v of the
// set's intervals are converted first (two mode products per table and
// interval) and the slab kernel reads the converted tensors.  The rows of the
// windowed 1-D kernel (cheb1d, row layout) hold Chebyshev coefficients too
// (one mode product per table and interval).
static hpsmc_status slab_args_for(hpsmc_plan *plan, const NodeSet &set, int layout, bool cheb1d, SlabArgs &sa,
                                  hipStream_t s)
{
    sa = set.slab;
    sa.slab_table = plan->slab_table;
    sa.layout = layout;
    if (layout != 1 && !cheb1d) return HPSMC_OK;
    if (!plan->cu_ch) return fail(HPSMC_EINVAL, "no Chebyshev coefficient buffers for this slab layout");
    const int P = plan->P;
    const double *A = plan->mats + plan->cheb_off;
    const int64_t I = plan->n_inst;
    for (int32_t iv : set.ivs) {
        const int T1 = plan->degree[iv] + 1;
        for (int t = 0; t < 2; ++t) {
            const double *in = (t ? plan->cv : plan->cu) + plan->c_off[iv];
            double *out = (t ? plan->cv_ch : plan->cu_ch) + plan->c_off[iv];
            if (plan->d == 1) {
                HIP_TRY(launch_mode_product(in, out, I, P, P, T1, A, 1.0, 0, s));
            } else {
                HIP_TRY(launch_mode_product(in, plan->tmp0, I, P, P, (int64_t)P * T1, A, 1.0, 0, s));
                HIP_TRY(launch_mode_product(plan->tmp0, out, I * P, P, P, T1, A, 1.0, 0, s));
            }
        }
    }
    sa.cu = plan->cu_ch;
    sa.cv = plan->cv_ch;
    if (sa.cs) sa.cs = plan->cs_ch;
    return HPSMC_OK;
}

static hpsmc_status sample_set(hpsmc_plan *plan, NodeSet &set, int tag, int record, hipStream_t s)
{
    const int ns = plan->launch.samples_per_lane;
    SlabArgs sa;
    if (hpsmc_status st = slab_args_for(plan, set, set_uses_mma(plan, set), set_uses_1d(plan, set), sa, s))
        return st;
    hpsmc_plan::EvPair *es = next_pair(plan->ev_slab, plan->n_slab);
    if (es) HIP_TRY(hipEventRecord(es->a, s));
    HIP_TRY(launch_slabs(sa, plan->fp32, set.max_nstar, s));
    if (es) HIP_TRY(hipEventRecord(es->b, s));
    if (set.rounds) return sample_rounds(plan, set, tag, record, s);
    if (plan->pb.estimator != HPSMC_EST_RESIDUAL || plan->pb.quad != HPSMC_QUAD_CENTRE)
        return fail(HPSMC_ENOTSUP, "the Picard form and the ball quadrature need the round kernel (slab too large "
                                   "for LDS chunks)");
    HIP_TRY(launch_fill_u64(plan->counters, 1, 0ull, s));
    SampleArgs a{};
    a.nodes = set.dev;
    a.n_nodes = set.n;
    a.M = plan->pb.M;
    a.chunks_per_node = (int32_t)((plan->pb.M + 64 * ns - 1) / (64 * ns));
    a.P = plan->P;
    a.PP = plan->PP;
    a.tag = tag;
    a.key0 = (uint32_t)plan->pb.seed;
    a.key1 = (uint32_t)(plan->pb.seed >> 32);
    a.slab_table = plan->slab_table;
    a.slab_stride = sa.slab_stride;
    a.part = plan->part;
    a.probe = (plan->m_probe > 0 && set.probe) ? set.probe : nullptr;
    a.m_probe = plan->m_probe;
    a.work = plan->counters;
    a.stats = plan->counters + 1;
    a.phys.dim = plan->d;
    a.phys.f_kind = plan->pb.f_kind;
    a.phys.src_kind = plan->pb.src_kind == HPSMC_SRC_POLY ? HPSMC_SRC_NONE : plan->pb.src_kind;
    memcpy(a.phys.f_param, plan->pb.f_param, sizeof(a.phys.f_param));
    memcpy(a.phys.src_param, plan->pb.src_param, sizeof(a.phys.src_param));
    const int blocks = std::max(1, plan->cus * plan->launch.blocks_per_cu);
    hpsmc_plan::EvPair *ek = next_pair(plan->ev_sample, plan->n_sample);
    if (ek) HIP_TRY(hipEventRecord(ek->a, s));
    HIP_TRY(launch_sample(a, plan->fp32, ns, plan->launch.waves_per_block, blocks, s));
    if (ek) HIP_TRY(hipEventRecord(ek->b, s));
    unsigned long long *mb = plan->maxbits + std::min(record, 4095);
    HIP_TRY(launch_reduce_update(plan->part, a.chunks_per_node, update_mode(plan), set.dev, set.n, plan->pb.M,
                                 plan->U, set.eps, set.sumsq, mb, s));
    if (hpsmc_status st = aitken_update(plan, set, s)) return st;
    plan->node_samples += set.n * plan->pb.M;
    plan->n_records = std::max(plan->n_records, std::min(record, 4095) + 1);
    return HPSMC_OK;
}

static hpsmc_status start_interval(hpsmc_plan *plan, int iv, int replicate, hipStream_t s)
{
    if (iv < (int)plan->twin_last.size()) plan->twin_last[iv] = 0;
    if (hpsmc_status st = aitken_reset(plan, iv, s)) return st;
    const int T1 = plan->degree[iv] + 1;
    const int64_t rows = (int64_t)plan->n_inst * plan->nsp;
    double *dst = plan->U + plan->u_off[iv];
    if (iv == 0) {
        HIP_TRY(launch_start_columns(dst, plan->ic, 1, 0, T1, T1, rows, replicate, s));
    } else {
        const int Tp = plan->degree[iv - 1] + 1;
        HIP_TRY(launch_start_columns(dst, plan->U + plan->u_off[iv - 1], Tp, Tp - 1, T1, T1, rows, replicate, s));
    }
    return HPSMC_OK;
}

}  // namespace hpsmc

using namespace hpsmc;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *hpsmc_last_error(void) { return g_err.c_str(); }

void hpsmc_destroy(hpsmc_plan *plan)
{
    if (!plan) return;
    if (plan->twin) hpsmc_destroy(plan->twin);
    if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->own_stream) (void)hipStreamDestroy(plan->own_stream);
    for (auto &s : plan->sets) free_set(plan, s);
    for (auto *pool : {&plan->ev_sample, &plan->ev_slab, &plan->ev_recon, &plan->ev_span, &plan->ev_adj})
        for (auto &e : *pool) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    void *ptrs[] = {plan->U, plan->cu, plan->cv, plan->tmp0, plan->tmp1, plan->ic, plan->mats,
                    plan->slab_table, plan->part, plan->counters, plan->maxbits, plan->hist_u, plan->hist_v,
                    plan->lam, plan->cbar_u, plan->cbar_v, plan->dtarget, plan->dloss, plan->dgrad, plan->slab_bar,
                    plan->frac_tab, plan->src_poly, plan->cu_ch, plan->cv_ch, plan->cs_ch};
    for (void *p : ptrs) dfree(plan, p);
    delete plan;
}

hpsmc_status hpsmc_create(const hpsmc_problem *pb, hpsmc_plan **out)
{
    if (!out) return fail(HPSMC_EINVAL, "out is NULL");
    *out = nullptr;
    hpsmc_status st = validate(pb);
    if (st) return st;
    if (pb->precision == HPSMC_FP32_THEN_FP64) {
        // an FP32 plan and its FP64 twin over the same problem
        hpsmc_problem p32 = *pb, p64 = *pb;
        p32.precision = HPSMC_FP32_SAMPLING;
        p64.precision = HPSMC_FP64;
        hpsmc_plan *main = nullptr, *twin = nullptr;
        if ((st = hpsmc_create(&p32, &main))) return st;
        if ((st = hpsmc_create(&p64, &twin))) { hpsmc_destroy(main); return st; }
        main->twin = twin;
        main->pb.precision = HPSMC_FP32_THEN_FP64;
        *out = main;
        return HPSMC_OK;
    }
    std::unique_ptr<hpsmc_plan, void (*)(hpsmc_plan *)> plan(new hpsmc_plan, hpsmc_destroy);
    {
        std::lock_guard<std::mutex> lk(g_alloc_mutex);
        plan->alloc_fn = g_alloc_fn;
        plan->free_fn = g_free_fn;
        plan->alloc_ctx = g_alloc_ctx;
    }
    plan->pb = *pb;
    plan->d = pb->dim;
    plan->n = pb->n;
    plan->frac = is_frac(*pb);
    plan->P = plan->frac ? pb->n : pb->n + 2;   // Jacobi modes p < n, or Legendre modes of phi_p, p < n
    plan->PP = (plan->P + 3) / 4 * 4;
    plan->n_iv = pb->n_intervals;
    plan->n_inst = pb->n_instances;
    plan->nsp = ipow(pb->n, pb->dim);
    plan->psp = ipow(plan->P, pb->dim);
    plan->fp32 = pb->precision == HPSMC_FP32_SAMPLING;
    plan->t_breaks.assign(pb->t_breaks, pb->t_breaks + pb->n_intervals + 1);
    plan->degree.assign(pb->degree, pb->degree + pb->n_intervals);
    std::vector<double> dtm;
    if ((st = resolve_nstar(*pb, plan->nstar, dtm))) return st;
    plan->dt_max = dtm;
    if (pb->ic_data && (pb->ic_kind == HPSMC_IC_PHI || pb->ic_kind == HPSMC_IC_NODAL))
        plan->ic_data.assign(pb->ic_data, pb->ic_data + (size_t)pb->n_instances * plan->nsp);
    plan->pb.t_breaks = plan->t_breaks.data();
    plan->pb.degree = plan->degree.data();
    plan->pb.nstar = plan->nstar.data();
    plan->pb.nstar_mode = HPSMC_NSTAR_ARRAY;   // resolved
    plan->pb.ic_data = plan->ic_data.empty() ? nullptr : plan->ic_data.data();

    // grid
    std::vector<double> wx;
    if (plan->frac) gauss_jacobi_aa(plan->n, 0.5 * pb->alpha, plan->x, wx);
    else jacobi_gauss11(plan->n, plan->x, wx);
    plan->xi.resize(plan->n_iv);
    plan->tnodes.resize(plan->n_iv);
    for (int iv = 0; iv < plan->n_iv; ++iv) {
        std::vector<double> wt;
        lobatto(plan->degree[iv], plan->xi[iv], wt);
        const double t0 = plan->t_breaks[iv], h = plan->t_breaks[iv + 1] - t0;
        for (double z : plan->xi[iv]) plan->tnodes[iv].push_back(t0 + 0.5 * (z + 1.0) * h);
    }

    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(HPSMC_EDEVICE, "no HIP device");
    }
    plan->cus = prop.multiProcessorCount;
    if (set_recurrence_tables() != hipSuccess) return fail(HPSMC_EDEVICE, "constant table upload failed");

    // device buffers
    const int64_t I = plan->n_inst;
    int64_t usz = 0, csz = 0, tmax = 0;
    for (int iv = 0; iv < plan->n_iv; ++iv) {
        const int T1 = plan->degree[iv] + 1;
        plan->u_off.push_back(usz);
        plan->c_off.push_back(csz);
        usz += I * plan->nsp * T1;
        csz += I * plan->psp * T1;
        tmax = std::max<int64_t>(tmax, I * ipow(std::max(plan->n, plan->P), plan->d) * T1);
    }
    hpsmc_plan *pl = plan.get();
    if ((st = dalloc(pl, (void **)&pl->U, usz * 8))) return st;
    if ((st = dalloc(pl, (void **)&pl->cu, csz * 8))) return st;
    if ((st = dalloc(pl, (void **)&pl->cv, csz * 8))) return st;
    if ((st = dalloc(pl, (void **)&pl->tmp0, tmax * 8))) return st;
    if ((st = dalloc(pl, (void **)&pl->tmp1, tmax * 8))) return st;
    if ((st = dalloc(pl, (void **)&pl->ic, I * plan->nsp * 8))) return st;
    if ((st = dalloc(pl, (void **)&pl->counters, 4 * 8))) return st;
    if ((st = dalloc(pl, (void **)&pl->maxbits, 4096 * 8))) return st;
    if (pl->frac && (st = frac_tables(pl))) return st;
    if (pb->src_kind == HPSMC_SRC_POLY) {
        int64_t off = 0;
        for (int iv = 0; iv < plan->n_iv; ++iv) {
            plan->src_off.push_back(off);
            off += plan->psp * (plan->degree[iv] + 1);
        }
        if ((st = dalloc(pl, (void **)&pl->src_poly, off * 8))) return st;
        if (hipMemcpy(pl->src_poly, pb->src_coeffs, off * 8, hipMemcpyHostToDevice) != hipSuccess)
            return fail(HPSMC_EDEVICE, "source coefficient upload failed");
        plan->pb.src_coeffs = nullptr;   // the caller's array is not kept
    }

    // transform matrices
    std::vector<double> mats;
    auto G0 = plan->frac ? frac_nodal_to_modal(plan->x, wx, 0.5 * pb->alpha) : spatial_to_legendre(plan->x, plan->P);
    auto D2 = plan->frac ? std::vector<double>((size_t)plan->P * plan->P, 0.0) : legendre_d2(plan->P);
    mats.insert(mats.end(), G0.begin(), G0.end());
    mats.insert(mats.end(), D2.begin(), D2.end());
    auto transpose = [](const std::vector<double> &A, int rows, int cols) {
        std::vector<double> T((size_t)rows * cols);
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c) T[(size_t)c * rows + r] = A[(size_t)r * cols + c];
        return T;
    };
    for (int iv = 0; iv < plan->n_iv; ++iv) {
        const int T1 = plan->degree[iv] + 1;
        auto Bt = temporal_to_legendre(plan->xi[iv]);
        auto D1 = legendre_d1(T1);
        plan->bt_off.push_back((int64_t)mats.size());
        mats.insert(mats.end(), Bt.begin(), Bt.end());
        plan->d1_off.push_back((int64_t)mats.size());
        mats.insert(mats.end(), D1.begin(), D1.end());
        auto BtT = transpose(Bt, T1, T1), D1T = transpose(D1, T1, T1);
        plan->btt_off.push_back((int64_t)mats.size());
        mats.insert(mats.end(), BtT.begin(), BtT.end());
        plan->d1t_off.push_back((int64_t)mats.size());
        mats.insert(mats.end(), D1T.begin(), D1T.end());
    }
    {
        auto G0T = transpose(G0, plan->P, plan->n), D2T = transpose(D2, plan->P, plan->P);
        plan->g0t_off = (int64_t)mats.size();
        mats.insert(mats.end(), G0T.begin(), G0T.end());
        plan->d2t_off = (int64_t)mats.size();
        mats.insert(mats.end(), D2T.begin(), D2T.end());
        // phi collocation Phi[j][p] = phi_p(x_j) and its transpose
        std::vector<double> Phi((size_t)plan->n * plan->n), L(plan->n + 3);
        for (int j = 0; j < plan->n; ++j) {
            legendre_values(plan->n + 2, plan->x[j], L.data());
            for (int pp = 0; pp < plan->n; ++pp) Phi[(size_t)j * plan->n + pp] = phi_legendre(pp, L.data());
        }
        plan->phi_off = (int64_t)mats.size();
        mats.insert(mats.end(), Phi.begin(), Phi.end());
        auto PhiT = transpose(Phi, plan->n, plan->n);
        plan->phit_off = (int64_t)mats.size();
        mats.insert(mats.end(), PhiT.begin(), PhiT.end());
        // A[p][j] with sum_j A[p][j] phi_q(x_j) = delta_pq: nodal values -> phi-coefficients
        const int n = plan->n;
        std::vector<double> W(Phi), Ainv((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i) Ainv[(size_t)i * n + i] = 1.0;
        // Gauss-Jordan with partial pivoting on W = Phi (rows j, columns p): Ainv becomes
        // Phi^{-1}, rows p and columns j
        for (int c = 0; c < n; ++c) {
            int piv = c;
            for (int r = c + 1; r < n; ++r)
                if (std::fabs(W[(size_t)r * n + c]) > std::fabs(W[(size_t)piv * n + c])) piv = r;
            if (piv != c)
                for (int k = 0; k < n; ++k) {
                    std::swap(W[(size_t)c * n + k], W[(size_t)piv * n + k]);
                    std::swap(Ainv[(size_t)c * n + k], Ainv[(size_t)piv * n + k]);
                }
            const double inv = 1.0 / W[(size_t)c * n + c];
            for (int k = 0; k < n; ++k) { W[(size_t)c * n + k] *= inv; Ainv[(size_t)c * n + k] *= inv; }
            for (int r = 0; r < n; ++r) {
                if (r == c) continue;
                const double f = W[(size_t)r * n + c];
                if (f == 0.0) continue;
                for (int k = 0; k < n; ++k) {
                    W[(size_t)r * n + k] -= f * W[(size_t)c * n + k];
                    Ainv[(size_t)r * n + k] -= f * Ainv[(size_t)c * n + k];
                }
            }
        }
        plan->ainv_off = (int64_t)mats.size();
        mats.insert(mats.end(), Ainv.begin(), Ainv.end());
    }
    // the basis of the 2-D matrix-core image and of the windowed 1-D kernel's rows
    const bool cheb = !plan->frac && ((plan->d == 2 && mma_capable(pl)) || plan->d == 1);
    if (cheb) {
        auto Ach = legendre_to_chebyshev(plan->P);
        plan->cheb_off = (int64_t)mats.size();
        mats.insert(mats.end(), Ach.begin(), Ach.end());
        if ((st = dalloc(pl, (void **)&pl->cu_ch, csz * 8))) return st;
        if ((st = dalloc(pl, (void **)&pl->cv_ch, csz * 8))) return st;
    }
    if ((st = dalloc(pl, (void **)&pl->mats, mats.size() * 8))) return st;
    std::vector<double> u0;
    initial_nodes(pl, u0);
    if (hipMemcpy(pl->mats, mats.data(), mats.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pl->ic, u0.data(), u0.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(pl->counters, 0, 32) != hipSuccess || hipMemset(pl->maxbits, 0, 4096 * 8) != hipSuccess ||
        hipMemset(pl->U, 0, usz * 8) != hipSuccess)
        return fail(HPSMC_EDEVICE, "initial upload failed");
    if (cheb && pl->src_poly) {   // the polynomial source in the image's basis, once
        int64_t off = 0;
        for (int iv = 0; iv < plan->n_iv; ++iv) off += plan->psp * (plan->degree[iv] + 1);
        if ((st = dalloc(pl, (void **)&pl->cs_ch, off * 8))) return st;
        const double *A = pl->mats + pl->cheb_off;
        const int P = plan->P;
        for (int iv = 0; iv < plan->n_iv; ++iv) {
            const int T1 = plan->degree[iv] + 1;
            const bool ok =
                plan->d == 1
                    ? launch_mode_product(pl->src_poly + pl->src_off[iv], pl->cs_ch + pl->src_off[iv], 1, P, P, T1, A,
                                          1.0, 0, nullptr) == hipSuccess
                    : launch_mode_product(pl->src_poly + pl->src_off[iv], pl->tmp0, 1, P, P, (int64_t)P * T1, A, 1.0,
                                          0, nullptr) == hipSuccess &&
                          launch_mode_product(pl->tmp0, pl->cs_ch + pl->src_off[iv], P, P, P, T1, A, 1.0, 0, nullptr) ==
                              hipSuccess;
            if (!ok) return fail(HPSMC_EDEVICE, "source conversion failed");
        }
    }

    // node sets and the slab table
    if (pb->schedule == HPSMC_SEQUENTIAL) {
        plan->sets.resize(plan->n_iv);
        for (int iv = 0; iv < plan->n_iv; ++iv)
            if ((st = build_set(pl, plan->sets[iv], {iv}))) return st;
    } else {
        plan->sets.resize(1);
        std::vector<int32_t> all;
        for (int iv = 0; iv < plan->n_iv; ++iv) all.push_back(iv);
        if ((st = build_set(pl, plan->sets[0], all))) return st;
    }
    int64_t slab_max = 0, nmax = 0;
    for (auto &s : plan->sets) { slab_max = std::max(slab_max, s.slab_elems); nmax = std::max(nmax, s.n); }
    plan->slab_bytes = (size_t)slab_max * (plan->fp32 ? 4 : 8);
    if ((st = dalloc(pl, &pl->slab_table, plan->slab_bytes))) return st;
    plan->part_elems = nmax * ((pb->M + 63) / 64) * 2;
    if ((st = dalloc(pl, (void **)&pl->part, plan->part_elems * 8))) return st;

    // initial iterate: the initial column replicated in time
    if (pb->schedule == HPSMC_SEQUENTIAL) {
        if ((st = start_interval(pl, 0, 1, nullptr))) return st;
    } else {
        for (int iv = 0; iv < plan->n_iv; ++iv)
            if (launch_start_columns(pl->U + pl->u_off[iv], pl->ic, 1, 0, plan->degree[iv] + 1, plan->degree[iv] + 1,
                                     I * plan->nsp, 1, nullptr) != hipSuccess)
                return fail(HPSMC_EDEVICE, "initial iterate failed");
    }
    if (hipDeviceSynchronize() != hipSuccess) return fail(HPSMC_EDEVICE, "device synchronize failed");
    *out = plan.release();
    return HPSMC_OK;
}

#define CHECK_PLAN(p)                                                            \
    do {                                                                         \
        if (!(p)) return fail(HPSMC_EINVAL, "plan is NULL");                     \
        if ((p)->poisoned) return fail(HPSMC_EDEVICE, "plan is poisoned");       \
    } while (0)

hpsmc_status hpsmc_resolve_nstar(const hpsmc_problem *pb, int32_t *nstar, double *dt_max)
{
    if (!nstar) return fail(HPSMC_EINVAL, "nstar is NULL");
    hpsmc_status st = validate(pb);
    if (st) return st;
    std::vector<int32_t> ns;
    std::vector<double> dtm;
    if ((st = resolve_nstar(*pb, ns, dtm))) return st;
    std::copy(ns.begin(), ns.end(), nstar);
    if (dt_max) std::copy(dtm.begin(), dtm.end(), dt_max);
    return HPSMC_OK;
}

hpsmc_status hpsmc_get_nstar(const hpsmc_plan *plan, int32_t *nstar, double *dt_max)
{
    CHECK_PLAN(plan);
    if (!nstar) return fail(HPSMC_EINVAL, "nstar is NULL");
    std::copy(plan->nstar.begin(), plan->nstar.end(), nstar);
    if (dt_max) std::copy(plan->dt_max.begin(), plan->dt_max.end(), dt_max);
    return HPSMC_OK;
}

hpsmc_status hpsmc_grid(const hpsmc_plan *plan, int32_t iv, double *x_nodes, double *t_nodes)
{
    if (!plan) return fail(HPSMC_EINVAL, "plan is NULL");
    if (iv < 0 || iv >= plan->n_iv) return fail(HPSMC_EINVAL, "interval out of range");
    if (x_nodes) memcpy(x_nodes, plan->x.data(), sizeof(double) * plan->n);
    if (t_nodes) memcpy(t_nodes, plan->tnodes[iv].data(), sizeof(double) * plan->tnodes[iv].size());
    return HPSMC_OK;
}

hpsmc_status hpsmc_start_interval(hpsmc_plan *plan, int32_t iv, void *stream)
{
    CHECK_PLAN(plan);
    if (iv < 0 || iv >= plan->n_iv) return fail(HPSMC_EINVAL, "interval out of range");
    if (plan->pb.schedule != HPSMC_SEQUENTIAL) return fail(HPSMC_EINVAL, "plan uses sweeps");
    return start_interval(plan, iv, 1, (hipStream_t)stream);
}

static hpsmc_status iterate_impl(hpsmc_plan *plan, int iv, int tag, int record, hipStream_t s)
{
    hpsmc_status st;
    if (iv < (int)plan->twin_last.size()) plan->twin_last[iv] = 0;
    if ((st = reconstruct(plan, iv, s))) return st;
    return sample_set(plan, plan->sets[iv], tag, record, s);
}

hpsmc_status hpsmc_iterate(hpsmc_plan *plan, int32_t iv, int32_t tag, void *stream)
{
    CHECK_PLAN(plan);
    if (iv < 0 || iv >= plan->n_iv) return fail(HPSMC_EINVAL, "interval out of range");
    if (tag < 0 || tag > 255) return fail(HPSMC_EINVAL, "tag must be 0..255");
    if (plan->pb.schedule != HPSMC_SEQUENTIAL) return fail(HPSMC_EINVAL, "plan uses sweeps");
    return iterate_impl(plan, iv, tag, plan->n_records, (hipStream_t)stream);
}

static hpsmc_status sweep_impl(hpsmc_plan *plan, int tag, int record, hipStream_t s)
{
    hpsmc_status st;
    std::fill(plan->twin_last.begin(), plan->twin_last.end(), 0);
    // every interval takes column 0 from the previous interval's last column
    // (the values of the previous sweep: the copies run before any update)
    for (int iv = 1; iv < plan->n_iv; ++iv) {
        const int T1 = plan->degree[iv] + 1, Tp = plan->degree[iv - 1] + 1;
        HIP_TRY(launch_start_columns(plan->U + plan->u_off[iv], plan->U + plan->u_off[iv - 1], Tp, Tp - 1, T1, T1,
                                     (int64_t)plan->n_inst * plan->nsp, 0, s));
    }
    for (int iv = 0; iv < plan->n_iv; ++iv)
        if ((st = reconstruct(plan, iv, s))) return st;
    return sample_set(plan, plan->sets[0], tag, record, s);
}

hpsmc_status hpsmc_sweep(hpsmc_plan *plan, int32_t tag, void *stream)
{
    CHECK_PLAN(plan);
    if (tag < 0 || tag > 255) return fail(HPSMC_EINVAL, "tag must be 0..255");
    if (plan->pb.schedule != HPSMC_SWEEPS) return fail(HPSMC_EINVAL, "plan is sequential");
    return sweep_impl(plan, tag, plan->n_records, (hipStream_t)stream);
}

// max|eps| of one record (synchronizes the stream)
static hpsmc_status read_record(hpsmc_plan *plan, int record, double *v, hipStream_t s)
{
    unsigned long long bits = 0;
    if (hipMemcpyAsync(&bits, plan->maxbits + std::min(record, 4095), 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(HPSMC_EDEVICE, "record copy failed");
    memcpy(v, &bits, 8);
    return HPSMC_OK;
}

// divergence: the latest max|eps| is not finite, or it grew in each of the last three iterations
static bool diverged(const std::vector<double> &h)
{
    const size_t n = h.size();
    if (n > 0 && !std::isfinite(h[n - 1])) return true;
    return n >= 4 && h[n - 1] > h[n - 2] && h[n - 2] > h[n - 3] && h[n - 3] > h[n - 4];
}

// Algorithm 1 (or the sweeps).  tol = 0: exactly `iters` iterations, asynchronous.
// tol > 0: after each iteration the host reads max|eps| (Algorithm 1's loop
// condition), stops the interval below tol, returns EDIVERGED on divergence and
// ENOTCONVERGED when some interval used all `iters` iterations.
static hpsmc_status solve_body(hpsmc_plan *plan, hipStream_t s)
{
    hpsmc_status st;
    const int K = plan->pb.iters;
    const double tol = plan->pb.tol;
    bool unconverged = false;
    // the records this solve writes start from zero (their maxima are taken with
    // atomics); a fill kernel rather than a memset, so a captured solve replays it
    const int64_t n_rec = std::min<int64_t>(4096, plan->pb.schedule == HPSMC_SEQUENTIAL
                                                       ? (int64_t)plan->n_iv * K : (int64_t)K);
    HIP_TRY(launch_fill_u64(plan->maxbits, n_rec, 0ull, s));
    if (plan->pb.schedule == HPSMC_SEQUENTIAL) {
        for (int iv = 0; iv < plan->n_iv; ++iv) {
            if ((st = start_interval(plan, iv, 1, s))) return st;
            std::vector<double> hist;
            int k = 0;
            for (; k < K; ++k) {
                if ((st = iterate_impl(plan, iv, plan->pb.fresh_per_iter ? k : 0, iv * K + k, s))) return st;
                if (tol > 0.0) {
                    double e;
                    if ((st = read_record(plan, iv * K + k, &e, s))) return st;
                    hist.push_back(e);
                    if (diverged(hist))
                        return fail(HPSMC_EDIVERGED, "max|eps| diverged in interval " + std::to_string(iv) +
                                                         ", iteration " + std::to_string(k));
                    if (e < tol) break;
                }
            }
            if (tol > 0.0 && k == K) unconverged = true;
        }
    } else {
        for (int iv = 0; iv < plan->n_iv; ++iv) {
            HIP_TRY(launch_start_columns(plan->U + plan->u_off[iv], plan->ic, 1, 0, plan->degree[iv] + 1,
                                         plan->degree[iv] + 1, (int64_t)plan->n_inst * plan->nsp, 1, s));
            if ((st = aitken_reset(plan, iv, s))) return st;
        }
        std::vector<double> hist;
        int k = 0;
        for (; k < K; ++k) {
            if ((st = sweep_impl(plan, plan->pb.fresh_per_iter ? k : 0, k, s))) return st;
            if (tol > 0.0) {
                double e;
                if ((st = read_record(plan, k, &e, s))) return st;
                hist.push_back(e);
                if (diverged(hist)) return fail(HPSMC_EDIVERGED, "max|eps| diverged at sweep " + std::to_string(k));
                if (e < tol) break;
            }
        }
        if (tol > 0.0 && k == K) unconverged = true;
    }
    if (unconverged) return fail(HPSMC_ENOTCONVERGED, "max|eps| stayed above tol after iters iterations");
    return HPSMC_OK;
}

// nodal values of interval iv from one plan into another of the same layout
// (a plan and its twin)
static hpsmc_status copy_interval(hpsmc_plan *dst, hpsmc_plan *src, int iv, hipStream_t s)
{
    const size_t bytes = (size_t)src->n_inst * src->nsp * (src->degree[iv] + 1) * 8;
    if (hipMemcpyAsync(dst->U + dst->u_off[iv], src->U + src->u_off[iv], bytes, hipMemcpyDeviceToDevice, s) !=
        hipSuccess) {
        dst->poisoned = true;
        return fail(HPSMC_EDEVICE, "copy between the FP32 plan and its FP64 twin failed");
    }
    return HPSMC_OK;
}

// HPSMC_FP32_THEN_FP64: Algorithm 1 (or the sweeps) as in solve_body, each
// interval (the sweep sequence) sampled by the FP32 plan until max|eps| <
// switch_tol and by the FP64 twin afterwards, with the counter tags running
// on; the twin's max|eps| records are copied into the plan's, and the final
// nodal values back into the plan.  Always eager: the switch needs the host.
static hpsmc_status mixed_solve_body(hpsmc_plan *plan, hipStream_t s)
{
    hpsmc_status st;
    hpsmc_plan *tw = plan->twin;
    const int K = plan->pb.iters;
    const double tol = plan->pb.tol, sw = plan->pb.switch_tol;
    const bool seq = plan->pb.schedule == HPSMC_SEQUENTIAL;
    const int64_t n_rec = std::min<int64_t>(4096, seq ? (int64_t)plan->n_iv * K : (int64_t)K);
    HIP_TRY(launch_fill_u64(plan->maxbits, n_rec, 0ull, s));
    HIP_TRY(launch_fill_u64(tw->maxbits, n_rec, 0ull, s));
    auto step = [&](hpsmc_plan *p, int iv, int k, int rec, double *e) -> hpsmc_status {
        const int tag = plan->pb.fresh_per_iter ? k : 0;
        hpsmc_status r = seq ? iterate_impl(p, iv, tag, rec, s) : sweep_impl(p, tag, rec, s);
        if (r || (r = read_record(p, rec, e, s))) return r;
        if (p == tw) {
            unsigned long long bits;
            memcpy(&bits, e, 8);
            if (hipMemcpyAsync(plan->maxbits + std::min(rec, 4095), &bits, 8, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                plan->poisoned = true;
                return fail(HPSMC_EDEVICE, "record copy failed");
            }
            plan->n_records = std::max(plan->n_records, std::min(rec, 4095) + 1);
        }
        return HPSMC_OK;
    };
    bool unconverged = false;
    plan->twin_last.assign(plan->n_iv, 0);
    if (seq) {
        for (int iv = 0; iv < plan->n_iv; ++iv) {
            if ((st = start_interval(plan, iv, 1, s))) return st;
            std::vector<double> hist;
            bool in64 = false;
            int k = 0;
            for (; k < K; ++k) {
                double e;
                if ((st = step(in64 ? tw : plan, iv, k, iv * K + k, &e))) return st;
                hist.push_back(e);
                if (diverged(hist))
                    return fail(HPSMC_EDIVERGED, "max|eps| diverged in interval " + std::to_string(iv) +
                                                     ", iteration " + std::to_string(k));
                if (tol > 0.0 && e < tol) break;
                if (!in64 && e < sw) {
                    if ((st = copy_interval(tw, plan, iv, s))) return st;
                    in64 = true;
                }
            }
            if (in64 && (st = copy_interval(plan, tw, iv, s))) return st;
            plan->twin_last[iv] = in64 ? 1 : 0;
            if (tol > 0.0 && k == K) unconverged = true;
        }
    } else {
        for (int iv = 0; iv < plan->n_iv; ++iv)
            HIP_TRY(launch_start_columns(plan->U + plan->u_off[iv], plan->ic, 1, 0, plan->degree[iv] + 1,
                                         plan->degree[iv] + 1, (int64_t)plan->n_inst * plan->nsp, 1, s));
        std::vector<double> hist;
        bool in64 = false;
        int k = 0;
        for (; k < K; ++k) {
            double e;
            if ((st = step(in64 ? tw : plan, 0, k, k, &e))) return st;
            hist.push_back(e);
            if (diverged(hist)) return fail(HPSMC_EDIVERGED, "max|eps| diverged at sweep " + std::to_string(k));
            if (tol > 0.0 && e < tol) break;
            if (!in64 && e < sw) {
                for (int iv = 0; iv < plan->n_iv; ++iv)
                    if ((st = copy_interval(tw, plan, iv, s))) return st;
                in64 = true;
            }
        }
        if (in64)
            for (int iv = 0; iv < plan->n_iv; ++iv) {
                if ((st = copy_interval(plan, tw, iv, s))) return st;
                plan->twin_last[iv] = 1;
            }
        if (tol > 0.0 && k == K) unconverged = true;
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (unconverged) return fail(HPSMC_ENOTCONVERGED, "max|eps| stayed above tol after iters iterations");
    return HPSMC_OK;
}

hpsmc_status hpsmc_solve(hpsmc_plan *plan, void *stream)
{
    CHECK_PLAN(plan);
    hipStream_t s = (hipStream_t)stream;
    if (plan->twin) return mixed_solve_body(plan, s);
    if (!plan->use_graph || plan->pb.tol > 0.0) return solve_body(plan, s);   // the stop test needs the host
    if (!plan->graph_exec) {
        // capture on a stream of the plan (the legacy default stream cannot be captured)
        if (!plan->own_stream) HIP_TRY(hipStreamCreateWithFlags(&plan->own_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamSynchronize(s));
        const int64_t ns0 = plan->node_samples;
        const int32_t rec0 = plan->n_records;
        HIP_TRY(hipStreamBeginCapture(plan->own_stream, hipStreamCaptureModeThreadLocal));
        g_capturing = true;
        hpsmc_status st = solve_body(plan, plan->own_stream);
        g_capturing = false;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(plan->own_stream, &graph);
        if (st) { if (graph) (void)hipGraphDestroy(graph); return st; }
        if (e != hipSuccess) { plan->poisoned = true; return fail(HPSMC_EDEVICE, std::string("capture: ") + hipGetErrorString(e)); }
        plan->graph = graph;
        HIP_TRY(hipGraphInstantiate(&plan->graph_exec, graph, nullptr, nullptr, 0));
        plan->graph_node_samples = plan->node_samples - ns0;
        plan->graph_records = plan->n_records;
        plan->node_samples = ns0;   // counted again at each launch below
        plan->n_records = rec0;
    }
    hpsmc_plan::EvPair *ek = next_pair(plan->ev_span, plan->n_span);
    if (ek) HIP_TRY(hipEventRecord(ek->a, s));
    HIP_TRY(hipGraphLaunch(plan->graph_exec, s));
    if (ek) HIP_TRY(hipEventRecord(ek->b, s));
    plan->node_samples += plan->graph_node_samples;
    plan->n_records = std::max(plan->n_records, plan->graph_records);
    return HPSMC_OK;
}

static hpsmc_status copy_nodes(const hpsmc_plan *plan, int iv, void *dst, const void *src, int on_device,
                               hipStream_t s, bool to_plan)
{
    const size_t bytes = (size_t)plan->n_inst * plan->nsp * (plan->degree[iv] + 1) * 8;
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : (to_plan ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost);
    if (hipMemcpyAsync(dst, src, bytes, kind, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return fail(HPSMC_EDEVICE, "node copy failed");
    return HPSMC_OK;
}

hpsmc_status hpsmc_get_nodes(const hpsmc_plan *plan, int32_t iv, double *out, int32_t on_device, void *stream)
{
    CHECK_PLAN(plan);
    if (iv < 0 || iv >= plan->n_iv || !out) return fail(HPSMC_EINVAL, "bad interval or output");
    return copy_nodes(plan, iv, out, plan->U + plan->u_off[iv], on_device, (hipStream_t)stream, false);
}

hpsmc_status hpsmc_set_nodes(hpsmc_plan *plan, int32_t iv, const double *in, int32_t on_device, void *stream)
{
    CHECK_PLAN(plan);
    if (iv < 0 || iv >= plan->n_iv || !in) return fail(HPSMC_EINVAL, "bad interval or input");
    if (hpsmc_status st = aitken_reset(plan, iv, (hipStream_t)stream)) return st;
    return copy_nodes(plan, iv, plan->U + plan->u_off[iv], in, on_device, (hipStream_t)stream, true);
}

static const NodeSet *set_of(const hpsmc_plan *plan, int iv, int64_t *off)
{
    if (plan->pb.schedule == HPSMC_SEQUENTIAL) { *off = 0; return &plan->sets[iv]; }
    int64_t o = 0;
    for (int k = 0; k < iv; ++k) o += (int64_t)plan->n_inst * plan->nsp * plan->degree[k];
    *off = o;
    return &plan->sets[0];
}

hpsmc_status hpsmc_get_increment(const hpsmc_plan *plan, int32_t iv, double *eps, double *sumsq, void *stream)
{
    CHECK_PLAN(plan);
    if (plan->twin && iv >= 0 && iv < (int)plan->twin_last.size() && plan->twin_last[iv])
        return hpsmc_get_increment(plan->twin, iv, eps, sumsq, stream);   // the last iteration ran in FP64
    if (iv < 0 || iv >= plan->n_iv) return fail(HPSMC_EINVAL, "interval out of range");
    int64_t off;
    const NodeSet *set = set_of(plan, iv, &off);
    const size_t cnt = (size_t)plan->n_inst * plan->nsp * plan->degree[iv];
    hipStream_t s = (hipStream_t)stream;
    if ((eps && hipMemcpyAsync(eps, set->eps + off, cnt * 8, hipMemcpyDeviceToHost, s) != hipSuccess) ||
        (sumsq && hipMemcpyAsync(sumsq, set->sumsq + off, cnt * 8, hipMemcpyDeviceToHost, s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(HPSMC_EDEVICE, "increment copy failed");
    return HPSMC_OK;
}

hpsmc_status hpsmc_eval(hpsmc_plan *plan, int32_t iv, int32_t inst, const double *pts, int64_t npts, double *out,
                        void *stream)
{
    CHECK_PLAN(plan);
    if (plan->frac) return fail(HPSMC_ENOTSUP, "hpsmc_eval covers the Laplacian's basis");
    if (iv < 0 || iv >= plan->n_iv || inst < 0 || inst >= plan->n_inst || npts < 0 || (npts && (!pts || !out)))
        return fail(HPSMC_EINVAL, "bad eval arguments");
    if (npts == 0) return HPSMC_OK;
    hipStream_t s = (hipStream_t)stream;
    double *dp = nullptr, *dout = nullptr;
    const size_t pb = (size_t)npts * (plan->d + 1) * 8, ob = (size_t)npts * 2 * 8;
    if (dalloc(plan, (void **)&dp, pb) != HPSMC_OK || dalloc(plan, (void **)&dout, ob) != HPSMC_OK) {
        dfree(plan, dp);
        return fail(HPSMC_ENOMEM, "eval buffers");
    }
    const int T1 = plan->degree[iv] + 1;
    const int64_t co = plan->c_off[iv] + (int64_t)inst * plan->psp * T1;
    hipError_t e = hipMemcpyAsync(dp, pts, pb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_eval(plan->cu + co, plan->cv + co, plan->d, plan->P, T1, plan->t_breaks[iv],
                        plan->t_breaks[iv + 1] - plan->t_breaks[iv], dp, npts, dout, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, ob, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(plan, dp);
    dfree(plan, dout);
    if (e != hipSuccess) return fail(HPSMC_EDEVICE, std::string("eval: ") + hipGetErrorString(e));
    return HPSMC_OK;
}

// ---- evaluation without allocation ----------------------------------------
// Staging of hpsmc_eval_noalloc (the points in, the values out): one copy per
// GPU, held until the process ends and shared by every call on that GPU.  In
// host code `scratch` names a host-side stand-in, so kernels and copies take
// the device address that hipGetSymbolAddress returns for the current device,
// looked up once per device on its first call.
constexpr size_t kNoAllocBytes = (size_t)16 << 20;
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double *g_scratch_dev[kMaxDevices];

static hpsmc_status scratch_of_current_device(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(HPSMC_EDEVICE, "no current device for the static scratch array");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(HPSMC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = (double *)ptr;
    }
    *out = g_scratch_dev[dev];
    return HPSMC_OK;
}

hpsmc_status hpsmc_eval_noalloc(hpsmc_plan *plan, int32_t iv, int32_t inst, const double *pts, int64_t npts,
                                double *out, void *stream)
{
    CHECK_PLAN(plan);
    if (plan->frac) return fail(HPSMC_ENOTSUP, "hpsmc_eval_noalloc covers the Laplacian's basis");
    if (iv < 0 || iv >= plan->n_iv || inst < 0 || inst >= plan->n_inst || npts < 0 || (npts && (!pts || !out)))
        return fail(HPSMC_EINVAL, "bad eval arguments");
    const int64_t per_pt = plan->d + 1 + 2;   // doubles staged per point: coordinates and time in, (u, v) out
    if (npts > (int64_t)(kNoAllocBytes / sizeof(double)) / per_pt)
        return fail(HPSMC_EINVAL, "npts exceeds the static scratch of hpsmc_eval_noalloc (" +
                                      std::to_string((kNoAllocBytes / sizeof(double)) / per_pt) + " points)");
    if (npts == 0) return HPSMC_OK;
    double *base = nullptr;
    if (hpsmc_status st = scratch_of_current_device(&base)) return st;
    hipStream_t s = (hipStream_t)stream;
    double *dp = base, *dout = base + npts * (plan->d + 1);   // both regions are written in full before any read
    const size_t pb = (size_t)npts * (plan->d + 1) * 8, ob = (size_t)npts * 2 * 8;
    const int T1 = plan->degree[iv] + 1;
    const int64_t co = plan->c_off[iv] + (int64_t)inst * plan->psp * T1;
    hipError_t e = hipMemcpyAsync(dp, pts, pb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_eval(plan->cu + co, plan->cv + co, plan->d, plan->P, T1, plan->t_breaks[iv],
                        plan->t_breaks[iv + 1] - plan->t_breaks[iv], dp, npts, dout, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, ob, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(HPSMC_EDEVICE, std::string("eval: ") + hipGetErrorString(e));
    return HPSMC_OK;
}

hpsmc_status hpsmc_set_probe(hpsmc_plan *plan, int64_t m_probe)
{
    CHECK_PLAN(plan);
    if (plan->twin)
        if (hpsmc_status st = hpsmc_set_probe(plan->twin, m_probe)) return st;
    if (m_probe < 0 || m_probe > plan->pb.M) return fail(HPSMC_EINVAL, "m_probe must be 0..M");
    if (plan->graph_exec) {   // the captured graph holds the old probe buffers
        (void)hipGraphExecDestroy(plan->graph_exec);
        (void)hipGraphDestroy(plan->graph);
        plan->graph_exec = nullptr;
        plan->graph = nullptr;
    }
    for (auto &s : plan->sets) {
        dfree(plan, s.probe);
        s.probe = nullptr;
        if (m_probe > 0) {
            hpsmc_status st = dalloc(plan, (void **)&s.probe, (size_t)s.n * m_probe * 8);
            if (st) return st;
        }
    }
    plan->m_probe = m_probe;
    return HPSMC_OK;
}

hpsmc_status hpsmc_get_probe(const hpsmc_plan *plan, int32_t iv, double *out, void *stream)
{
    CHECK_PLAN(plan);
    if (plan->twin && iv >= 0 && iv < (int)plan->twin_last.size() && plan->twin_last[iv])
        return hpsmc_get_probe(plan->twin, iv, out, stream);
    if (iv < 0 || iv >= plan->n_iv || !out || plan->m_probe == 0) return fail(HPSMC_EINVAL, "no probe");
    int64_t off;
    const NodeSet *set = set_of(plan, iv, &off);
    const size_t cnt = (size_t)plan->n_inst * plan->nsp * plan->degree[iv] * plan->m_probe;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(out, set->probe + off * plan->m_probe, cnt * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(HPSMC_EDEVICE, "probe copy failed");
    return HPSMC_OK;
}

hpsmc_status hpsmc_set_launch(hpsmc_plan *plan, const hpsmc_launch *l)
{
    CHECK_PLAN(plan);
    if (!l) return fail(HPSMC_EINVAL, "launch is NULL");
    const bool ns_ok = l->samples_per_lane == 1 || l->samples_per_lane == 2 || (l->samples_per_lane == 4 && plan->d <= 2);
    if (!ns_ok || l->waves_per_block < 1 || l->waves_per_block > 4 || l->blocks_per_cu < 1 || l->blocks_per_cu > 64)
        return fail(HPSMC_EINVAL, "launch shape out of range");
    if (l->round_steps != 0 && (l->round_steps < 16 || l->round_steps > 4096 || l->round_steps % 4 != 0))
        return fail(HPSMC_EINVAL, "round_steps must be 0 or a multiple of 4 in 16..4096");
    plan->launch = *l;
    if (l->round_steps) plan->round_steps = l->round_steps;
    if (plan->graph_exec) {   // the captured launches used the previous shape
        (void)hipGraphExecDestroy(plan->graph_exec);
        (void)hipGraphDestroy(plan->graph);
        plan->graph_exec = nullptr;
        plan->graph = nullptr;
    }
    plan->launch.round_steps = plan->round_steps;
    return HPSMC_OK;
}

hpsmc_status hpsmc_get_launch(const hpsmc_plan *plan, hpsmc_launch *l)
{
    if (!plan || !l) return fail(HPSMC_EINVAL, "NULL argument");
    *l = plan->launch;
    return HPSMC_OK;
}

hpsmc_status hpsmc_stats(const hpsmc_plan *plan, hpsmc_stats_t *out, void *stream)
{
    CHECK_PLAN(plan);
    if (!out) return fail(HPSMC_EINVAL, "out is NULL");
    memset(out, 0, sizeof(*out));
    unsigned long long c[4];
    std::vector<unsigned long long> mb(4096);
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(c, plan->counters, sizeof(c), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(mb.data(), plan->maxbits, 4096 * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(HPSMC_EDEVICE, "stats copy failed");
    out->sample_ms = pool_ms(plan->ev_sample, plan->n_sample);
    out->sampling_span_ms = pool_ms(plan->ev_span, plan->n_span);
    out->slab_ms = pool_ms(plan->ev_slab, plan->n_slab);
    out->recon_ms = pool_ms(plan->ev_recon, plan->n_recon);
    out->sample_launches = (int32_t)plan->n_sample;
    out->adjoint_ms = pool_ms(plan->ev_adj, plan->n_adj);
    out->adjoint_launches = (int64_t)plan->n_adj;
    out->advance_launches = plan->n_advance;
    out->recon_launches = (int32_t)plan->n_recon;
    out->path_steps = c[1];
    out->lane_steps = c[2];
    out->node_samples = (uint64_t)plan->node_samples;
    if (plan->twin) {   // the FP64 twin's share of the work
        hpsmc_stats_t t;
        if (hpsmc_status st = hpsmc_stats(plan->twin, &t, stream)) return st;
        out->path_steps += t.path_steps;
        out->lane_steps += t.lane_steps;
        out->node_samples += t.node_samples;
        out->sample_launches += t.sample_launches;
        out->recon_launches += t.recon_launches;
        out->sample_ms += t.sample_ms;
        out->sampling_span_ms += t.sampling_span_ms;
        out->recon_ms += t.recon_ms;
        out->slab_ms += t.slab_ms;
        out->advance_launches += t.advance_launches;
    }
    out->n_records = plan->n_records;
    const int K = std::max(1, plan->pb.iters);
    for (int r = 0; r < plan->n_records; ++r) {
        double v;
        memcpy(&v, &mb[r], 8);
        out->max_eps[r] = v;
        if (!std::isfinite(v)) out->status_flags |= 1;
        // records r-3..r of one interval (blocks of `iters` records) grew each time
        if (r % K >= 3 && out->max_eps[r] > out->max_eps[r - 1] && out->max_eps[r - 1] > out->max_eps[r - 2] &&
            out->max_eps[r - 2] > out->max_eps[r - 3])
            out->status_flags |= 2;
    }
    return HPSMC_OK;
}

hpsmc_status hpsmc_reset_stats(hpsmc_plan *plan, void *stream)
{
    CHECK_PLAN(plan);
    if (plan->twin)
        if (hpsmc_status st = hpsmc_reset_stats(plan->twin, stream)) return st;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_fill_u64(plan->counters, 4, 0ull, s));
    HIP_TRY(launch_fill_u64(plan->maxbits, 4096, 0ull, s));
    plan->node_samples = 0;
    plan->n_records = 0;
    plan->n_sample = plan->n_slab = plan->n_recon = plan->n_span = plan->n_adj = 0;
    plan->n_advance = 0;
    return HPSMC_OK;
}

// ---- autotuner ------------------------------------------------------------
// Cache file: a JSON object, one entry per line,
//   "d2_n24_P26_deg16_fp32_M1024_gfx950": [samples_per_lane, waves, blocks_per_cu, round_steps],
static std::string tune_key(const hpsmc_plan *plan, int iv, int64_t M)
{
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "gpu";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch = arch.substr(0, c);
    }
    // plans that may run the matrix-core round kernel tune separately from those that may not
    const bool picard = plan->pb.estimator == HPSMC_EST_PICARD;
    const bool ball = plan->pb.quad == HPSMC_QUAD_BALL;
    const bool mma = plan->sample_mma && mma_capable(plan);
    char buf[256];
    snprintf(buf, sizeof(buf), "d%d_n%d_P%d_deg%d_%s%s%s%s%s_M%lld_I%d_%s", plan->d, plan->n, plan->P, plan->degree[iv],
             plan->fp32 ? "fp32" : "fp64", mma ? "mma" : "", uses_1d(plan, 1) ? "_win" : "", picard ? "_picard" : "",
             ball ? "_ball" : "", (long long)M, plan->n_inst, arch.c_str());
    return buf;
}

static bool cache_lookup(const char *path, const std::string &key, hpsmc_launch &l)
{
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    const std::string pat = "\"" + key + "\"";
    while (fgets(line, sizeof(line), f)) {
        const char *k = strstr(line, pat.c_str());
        if (!k) continue;
        int a, b, c, d;
        if (sscanf(k + pat.size(), " : [%d , %d , %d , %d]", &a, &b, &c, &d) == 4) {
            l.samples_per_lane = a; l.waves_per_block = b; l.blocks_per_cu = c; l.round_steps = d;
            found = true;
        }
    }
    fclose(f);
    return found;
}

static void cache_store(const char *path, const std::string &key, const hpsmc_launch &l)
{
    std::vector<std::string> lines;
    if (FILE *f = fopen(path, "r")) {
        char line[512];
        while (fgets(line, sizeof(line), f)) {
            std::string s(line);
            while (!s.empty() && (s.back() == '\n' || s.back() == '\r' || s.back() == ',' || s.back() == ' ')) s.pop_back();
            if (s.empty() || s == "{" || s == "}" || s.find("\"" + key + "\"") != std::string::npos) continue;
            lines.push_back(s);
        }
        fclose(f);
    }
    char buf[512];
    snprintf(buf, sizeof(buf), "  \"%s\": [%d, %d, %d, %d]", key.c_str(), l.samples_per_lane, l.waves_per_block,
             l.blocks_per_cu, l.round_steps);
    lines.push_back(buf);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    for (size_t i = 0; i < lines.size(); ++i) fprintf(f, "%s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
    rename(tmp.c_str(), path);
}

hpsmc_status hpsmc_tune(hpsmc_plan *plan, int32_t iv, int64_t m_tune, const char *cache_path, void *stream)
{
    CHECK_PLAN(plan);
    if (iv < 0 || iv >= plan->n_iv) return fail(HPSMC_EINVAL, "interval out of range");
    if (m_tune < 0) return fail(HPSMC_EINVAL, "m_tune must be >= 0");
    if (plan->pb.schedule != HPSMC_SEQUENTIAL && iv != 0) return fail(HPSMC_EINVAL, "sweep plans tune interval 0");
    if (plan->twin)   // the FP64 twin tunes its own launch shape (its own cache key)
        if (hpsmc_status st = hpsmc_tune(plan->twin, iv, m_tune, cache_path, stream)) return st;
    const int64_t M_full = plan->pb.M;
    const int64_t mt = m_tune == 0 ? std::min<int64_t>(M_full, 256) : std::min<int64_t>(M_full, m_tune);
    const std::string key = tune_key(plan, iv, M_full);
    hpsmc_launch best = plan->launch;
    if (cache_path && cache_lookup(cache_path, key, best)) return hpsmc_set_launch(plan, &best);

    hipStream_t s = (hipStream_t)stream;
    NodeSet &set = plan->pb.schedule == HPSMC_SEQUENTIAL ? plan->sets[iv] : plan->sets[0];
    // keep the iterate and the counters: every trial restores them
    int64_t usz = 0;
    for (int k = 0; k < plan->n_iv; ++k) usz += (int64_t)plan->n_inst * plan->nsp * (plan->degree[k] + 1);
    double *Usave = nullptr;
    if (dalloc(plan, (void **)&Usave, usz * 8) != HPSMC_OK) return fail(HPSMC_ENOMEM, "tune buffer");
    HIP_TRY(hipMemcpyAsync(Usave, plan->U, usz * 8, hipMemcpyDeviceToDevice, s));
    const int64_t ns_save = plan->node_samples;
    const int32_t rec_save = plan->n_records;

    std::vector<hpsmc_launch> cands;
    const int nsv[3] = {1, 2, 4};
    for (int a = 0; a < 3; ++a) {
        if (nsv[a] == 4 && plan->d > 2) continue;
        if (nsv[a] != 1 && one_sample_per_lane(plan)) continue;
        if (nsv[a] == 1 && plan->sample_mma && plan->d == 5 && mma_capable(plan)) {
            // the 5-D matrix-core kernel: two LDS buffers of 2 x 32-row tiles per block
            const int fit = std::max(1, (int)((160 * 1024 - 4096) / advance_mma5_lds_bytes(plan->P)));
            for (int w : {2, 4})
                for (int b = 1; b <= std::min(fit, 4); ++b) cands.push_back(hpsmc_launch{1, w, b, plan->round_steps});
            continue;
        }
        for (int w : {2, 4}) {
            // two-wave blocks of the matrix-core kernel: 1, 1.5, 2, 3, 4 waves per SIMD
            if (w == 2 && nsv[a] == 1 && plan->sample_mma && advance_mma_eligible(plan->fp32, plan->d, plan->P, 0, 1, 2)) {
                for (int b : {2, 3, 4, 6, 8}) cands.push_back(hpsmc_launch{1, 2, b, plan->round_steps});
                continue;
            }
            // the windowed 1-D kernel: few registers, so up to 16 blocks per CU
            if (set.rounds && uses_1d(plan, nsv[a])) {
                for (int b : {2, 4, 8, 16}) cands.push_back(hpsmc_launch{nsv[a], w, b, plan->round_steps});
                continue;
            }
            // the LDS-staged slab chunk must fit 4 vectors per thread
            int cf, nc;
            int64_t ce;
            if (set.rounds && !pick_chunking(plan, 64 * w, &cf, &ce, &nc)) continue;
            for (int b : {2, 3, 4, 8}) cands.push_back(hpsmc_launch{nsv[a], w, b, plan->round_steps});
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        dfree(plan, Usave);
        return fail(HPSMC_EDEVICE, "tune events");
    }
    plan->pb.M = mt;
    const int32_t accel_save = plan->pb.accel;
    plan->pb.accel = HPSMC_ACCEL_NONE;   // trials leave the Aitken history alone
    auto trial = [&](const hpsmc_launch &l, float &ms) -> hpsmc_status {
        hpsmc_launch keep = plan->launch;
        plan->launch = l;
        plan->round_steps = l.round_steps;
        hpsmc_status st = HPSMC_OK;
        for (int rep = 0; rep < 2 && st == HPSMC_OK; ++rep) {   // a short first run may be dominated by code loading
            if (rep == 1 && ms > 200.f) break;
            if (hipEventRecord(e0, s) != hipSuccess) return fail(HPSMC_EDEVICE, "event");
            st = plan->pb.schedule == HPSMC_SEQUENTIAL ? iterate_impl(plan, iv, 0, 4095, s) : sweep_impl(plan, 0, 4095, s);
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return fail(HPSMC_EDEVICE, "event");
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return fail(HPSMC_EDEVICE, "event");
            if (hipMemcpyAsync(plan->U, Usave, usz * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return fail(HPSMC_EDEVICE, "restore");
        }
        plan->launch = keep;
        plan->round_steps = keep.round_steps;
        return st;
    };
    hpsmc_status st = HPSMC_OK;
    float best_ms = 1e30f;
    const bool verbose = getenv("HPSMC_TUNE_VERBOSE") != nullptr;
    auto report = [&](const hpsmc_launch &c, float ms) {
        if (verbose)
            fprintf(stderr, "[tune] %s ns=%d waves=%d blocks/cu=%d steps=%d: %.3f ms\n", key.c_str(), c.samples_per_lane,
                    c.waves_per_block, c.blocks_per_cu, c.round_steps, ms);
    };
    for (const auto &c : cands) {
        float ms;
        if ((st = trial(c, ms))) break;
        report(c, ms);
        if (ms < best_ms) { best_ms = ms; best = c; }
    }
    if (!st) {
        // walk steps per round: long rounds for 1-D (cheap steps), short ones from
        // 3-D on (expensive steps: compaction pays sooner)
        const int rs_d1[5] = {128, 256, 512, 1024, 128}, rs[5] = {32, 64, 128, 256, 512},
                  rs_d3[5] = {16, 32, 64, 128, 256};
        const hpsmc_launch base = best;
        for (int k = 0; k < 5; ++k) {
            hpsmc_launch c = base;
            c.round_steps = plan->d == 1 ? rs_d1[k] : plan->d == 2 ? rs[k] : rs_d3[k];
            if (c.round_steps == base.round_steps) continue;
            float ms;
            if ((st = trial(c, ms))) break;
            report(c, ms);
            if (ms < best_ms) { best_ms = ms; best = c; }
        }
    }
    plan->pb.M = M_full;
    plan->pb.accel = accel_save;
    (void)launch_fill_u64(plan->maxbits + 4095, 1, 0ull, s);
    plan->node_samples = ns_save;
    plan->n_records = rec_save;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    dfree(plan, Usave);
    (void)set;
    if (st) return st;
    st = hpsmc_set_launch(plan, &best);
    if (!st && cache_path) cache_store(cache_path, key, best);
    return st;
}

// u0 = Phi c (per instance), Phi[j][p] = prod_i phi_{p_i}(x_{j_i})
static hpsmc_status phi_apply(hpsmc_plan *plan, const double *in, double *out, int64_t mat_off, hipStream_t s)
{
    const int d = plan->d, n = plan->n;
    const int64_t I = plan->n_inst;
    const double *src = in;
    double *bufs[2] = {plan->tmp0, plan->tmp1};
    for (int i = 0; i < d; ++i) {
        double *o = (i == d - 1) ? out : bufs[i & 1];
        HIP_TRY(launch_mode_product(src, o, I * ipow(n, i), n, n, ipow(n, d - 1 - i), plan->mats + mat_off, 1.0, 0, s));
        src = o;
    }
    return HPSMC_OK;
}

hpsmc_status hpsmc_set_initial_coeffs(hpsmc_plan *plan, const double *c0, int32_t on_device, void *stream)
{
    CHECK_PLAN(plan);
    if (!c0) return fail(HPSMC_EINVAL, "c0 is NULL");
    if (plan->pb.ic_kind != HPSMC_IC_PHI) return fail(HPSMC_EINVAL, "plan's initial data are not phi-coefficients");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)plan->n_inst * plan->nsp * 8;
    // stage the coefficients in the gradient's target buffer slot (free until a gradient call)
    double *stage = nullptr;
    if (dalloc(plan, (void **)&stage, bytes) != HPSMC_OK) return fail(HPSMC_ENOMEM, "staging");
    hipError_t e = hipMemcpyAsync(stage, c0, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
    if (e != hipSuccess) { dfree(plan, stage); plan->poisoned = true; return fail(HPSMC_EDEVICE, "coefficient copy"); }
    hpsmc_status st = phi_apply(plan, stage, plan->ic, plan->phi_off, s);
    if (!st && hipStreamSynchronize(s) != hipSuccess) st = fail(HPSMC_EDEVICE, "synchronize");
    dfree(plan, stage);
    if (st) return st;
    if (!on_device) plan->ic_data.assign(c0, c0 + (size_t)plan->n_inst * plan->nsp);
    return HPSMC_OK;
}

hpsmc_status hpsmc_set_initial_nodes(hpsmc_plan *plan, const double *u0, int32_t on_device, void *stream)
{
    CHECK_PLAN(plan);
    if (!u0) return fail(HPSMC_EINVAL, "u0 is NULL");
    if (plan->pb.ic_kind == HPSMC_IC_PHI)
        return fail(HPSMC_EINVAL, "the plan's initial data are phi-coefficients: use hpsmc_set_initial_coeffs");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)plan->n_inst * plan->nsp * 8;
    if (hipMemcpyAsync(plan->ic, u0, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        plan->poisoned = true;
        return fail(HPSMC_EDEVICE, "initial node copy failed");
    }
    return HPSMC_OK;
}

hpsmc_status hpsmc_get_coeffs(hpsmc_plan *plan, int32_t iv, double *out, int32_t on_device, void *stream)
{
    CHECK_PLAN(plan);
    if (plan->frac) return fail(HPSMC_ENOTSUP, "hpsmc_get_coeffs covers the Laplacian's basis");
    if (iv < 0 || iv >= plan->n_iv || !out) return fail(HPSMC_EINVAL, "bad interval or output");
    hipStream_t s = (hipStream_t)stream;
    const int d = plan->d, n = plan->n, T1 = plan->degree[iv] + 1;
    const int64_t I = plan->n_inst;
    // U x_1 A ... x_d A x_t Bt: phi-coefficients in space, Legendre coefficients in time
    const double *in = plan->U + plan->u_off[iv];
    double *bufs[2] = {plan->tmp0, plan->tmp1};
    for (int i = 0; i < d; ++i) {
        double *o = bufs[i & 1];
        HIP_TRY(launch_mode_product(in, o, I * ipow(n, i), n, n, ipow(n, d - 1 - i) * T1, plan->mats + plan->ainv_off,
                                    1.0, 0, s));
        in = o;
    }
    double *o = bufs[d & 1];
    HIP_TRY(launch_mode_product(in, o, I * plan->nsp, T1, T1, 1, plan->mats + plan->bt_off[iv], 1.0, 0, s));
    const size_t bytes = (size_t)I * plan->nsp * T1 * 8;
    if (hipMemcpyAsync(out, o, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(HPSMC_EDEVICE, "coefficient copy failed");
    return HPSMC_OK;
}

hpsmc_status hpsmc_set_allocator(hpsmc_alloc_fn alloc, hpsmc_free_fn free_, void *ctx)
{
    if ((alloc == nullptr) != (free_ == nullptr)) return fail(HPSMC_EINVAL, "alloc and free must both be set or both NULL");
    std::lock_guard<std::mutex> lk(g_alloc_mutex);
    g_alloc_fn = alloc;
    g_free_fn = free_;
    g_alloc_ctx = ctx;
    return HPSMC_OK;
}

hpsmc_status hpsmc_set_option(hpsmc_plan *plan, const char *name, int64_t value)
{
    CHECK_PLAN(plan);
    if (!name) return fail(HPSMC_EINVAL, "option name is NULL");
    if (strcmp(name, "graph") == 0) {
        if (value != 0 && value != 1) return fail(HPSMC_EINVAL, "graph must be 0 or 1");
        plan->use_graph = (int32_t)value;
        return HPSMC_OK;
    }
    if (strcmp(name, "adjoint_mfma") == 0) {
        if (value != 0 && value != 1) return fail(HPSMC_EINVAL, "adjoint_mfma must be 0 or 1");
        plan->adj_use_mfma = (int32_t)value;
        return HPSMC_OK;
    }
    if (strcmp(name, "sample_mfma") == 0) {
        if (value != 0 && value != 1) return fail(HPSMC_EINVAL, "sample_mfma must be 0 or 1");
        if (plan->sample_mma != (int32_t)value && plan->graph_exec) {   // the captured launches used the other kernel
            (void)hipGraphExecDestroy(plan->graph_exec);
            (void)hipGraphDestroy(plan->graph);
            plan->graph_exec = nullptr;
            plan->graph = nullptr;
        }
        plan->sample_mma = (int32_t)value;
        return HPSMC_OK;
    }
    if (strcmp(name, "sample_split") == 0) {
        if (value != 0 && value != 1) return fail(HPSMC_EINVAL, "sample_split must be 0 or 1");
        if (plan->sample_split != (int32_t)value && plan->graph_exec) {   // captured with the other batching
            (void)hipGraphExecDestroy(plan->graph_exec);
            (void)hipGraphDestroy(plan->graph);
            plan->graph_exec = nullptr;
            plan->graph = nullptr;
        }
        plan->sample_split = (int32_t)value;
        return HPSMC_OK;
    }
    if (strcmp(name, "sample_1d") == 0) {
        if (value != 0 && value != 1) return fail(HPSMC_EINVAL, "sample_1d must be 0 or 1");
        if (plan->sample_1d != (int32_t)value && plan->graph_exec) {   // the captured launches used the other kernel
            (void)hipGraphExecDestroy(plan->graph_exec);
            (void)hipGraphDestroy(plan->graph);
            plan->graph_exec = nullptr;
            plan->graph = nullptr;
        }
        plan->sample_1d = (int32_t)value;
        return HPSMC_OK;
    }
    return fail(HPSMC_EINVAL, std::string("unknown option ") + name);
}

// whether the round kernel of interval iv runs on the matrix cores with the current launch shape
static int mma_active(const hpsmc_plan *plan, int iv)
{
    return set_uses_mma(plan, plan->pb.schedule == HPSMC_SEQUENTIAL ? plan->sets[iv] : plan->sets[0]);
}

hpsmc_status hpsmc_get_option(const hpsmc_plan *plan, const char *name, int64_t *value)
{
    CHECK_PLAN(plan);
    if (!name || !value) return fail(HPSMC_EINVAL, "NULL argument");
    if (strcmp(name, "graph") == 0) { *value = plan->use_graph; return HPSMC_OK; }
    if (strcmp(name, "adjoint_mfma") == 0) { *value = plan->adj_use_mfma; return HPSMC_OK; }
    if (strcmp(name, "sample_mfma") == 0) { *value = plan->sample_mma; return HPSMC_OK; }
    if (strcmp(name, "sample_split") == 0) { *value = plan->sample_split; return HPSMC_OK; }
    if (strcmp(name, "sample_1d") == 0) { *value = plan->sample_1d; return HPSMC_OK; }
    if (strcmp(name, "sample_1d_active") == 0) { *value = set_uses_1d(plan, plan->sets[0]); return HPSMC_OK; }
    if (strcmp(name, "sample_mfma_active") == 0) {
        *value = 0;
        for (int iv = 0; iv < (plan->pb.schedule == HPSMC_SEQUENTIAL ? plan->n_iv : 1); ++iv)
            *value |= mma_active(plan, iv);
        return HPSMC_OK;
    }
    return fail(HPSMC_EINVAL, std::string("unknown option ") + name);
}

// Form of the adjoint kernel: 0 vector units; 1 outer products on the matrix
// cores; 2 (d = 2, slabs in the matrix-core layout) u* on the matrix cores too.
static int adjoint_mfma_mode(const hpsmc_plan *plan, const NodeSet &set)
{
    if (!plan->fp32 || !plan->adj_use_mfma) return 0;
    return plan->d == 2 && plan->P <= 2 * kAdjMma2MaxKH && set.slab.slab_off_mma ? 2 : 1;
}

static hpsmc_status adjoint_sampling(hpsmc_plan *plan, NodeSet &set, int tag, hipStream_t s)
{
    const int G = (int)set.ghost.size();
    // the matrix-core form needs four waves: each forms one of the two weighted
    // tables over half of the block's samples, and the halves meet in LDS
    // before the atomics into the slab-adjoint table; the vector form sums one
    // wave's
    const int mfma = adjoint_mfma_mode(plan, set);
    const int waves = mfma ? 4 : 1;
    const int nthr = 64 * waves;
    const size_t lds = mfma == 2 ? adjoint_mma2_lds_bytes(plan->P, nthr)
                                 : adjoint_lds_bytes(plan->fp32, mfma, plan->d, plan->P, nthr, set.slab.slab_stride);
    const int64_t nvec = set.slab.slab_stride * (plan->fp32 ? 4 : 8) / 16;
    if ((mfma != 2 && nvec > 4LL * nthr) || lds > 65536) return fail(HPSMC_ENOTSUP, "slab too large for the adjoint kernel");
    const int C = plan->round_steps;
    const int R = (set.max_nstar + C - 1) / C;
    AdjointArgs aa{};
    RoundArgs &a = aa.r;
    a.groups = set.gdev;
    a.nodes = set.dev;
    a.n_groups = G;
    a.steps = C;
    a.batch = nthr;
    a.batch_prefix = set.prefix;
    a.P = plan->P;
    a.PP = plan->PP;
    a.tag = tag;
    a.key0 = (uint32_t)plan->pb.seed;
    a.key1 = (uint32_t)(plan->pb.seed >> 32);
    a.slab_table = plan->slab_table;
    a.slab_stride = mfma == 2 ? set.slab.mma_stride : set.slab.slab_stride;
    a.work = plan->counters;
    a.stats = plan->counters + 1;
    a.phys = physics_of(plan);
    aa.bar_stride = set.slab.slab_stride;
    aa.lambda = plan->lam;
    aa.slab_bar = plan->slab_bar;
    aa.inv_M = 1.0 / (double)plan->pb.M;
    aa.use_mfma = mfma;
    // the matrix-core form is compiled for three waves per SIMD: three
    // four-wave blocks per CU when their LDS fits in the CU's 160 KiB
    const int per_cu = mfma ? (3 * lds <= (size_t)160 * 1024 ? 3 : 2) : 8 / waves;
    const int blocks = std::max(1, plan->cus * per_cu);
    for (int64_t m0 = 0; m0 < plan->pb.M; m0 += set.ms) {
        const int64_t mc = std::min<int64_t>(set.ms, plan->pb.M - m0);
        a.m0 = m0;
        a.mcount = mc;
        for (int r = 0; r < R; ++r) {
            a.round = r;
            a.state_in = set.state[r & 1];
            a.state_out = set.state[(r + 1) & 1];
            a.live_in = set.live + (r & 1) * G;
            a.live_out = set.live + ((r + 1) & 1) * G;
            HIP_TRY(launch_round_prep(set.gdev, G, r, C, mc, a.batch, 0, 0, a.live_in, a.live_out, set.prefix,
                                      plan->counters, s));
            hpsmc_plan::EvPair *ea = next_pair(plan->ev_adj, plan->n_adj);
            if (ea) HIP_TRY(hipEventRecord(ea->a, s));
            HIP_TRY(launch_adjoint(aa, plan->fp32, waves, blocks, lds, s));
            if (ea) HIP_TRY(hipEventRecord(ea->b, s));
        }
    }
    return HPSMC_OK;
}

// the slab-adjoint table: the row layout of the set's slabs (the adjoint kernels
// accumulate in it and the slab adjoint reads it), in whole 8-byte words
static size_t bar_alloc_bytes(const hpsmc_plan *plan, const NodeSet &set)
{
    return ((size_t)set.slab_elems_row * (plan->fp32 ? 4 : 8) + 7) & ~(size_t)7;
}

hpsmc_status hpsmc_loss_grad_c0(hpsmc_plan *plan, const double *target, double *loss, double *grad,
                                int32_t on_device, void *stream)
{
    CHECK_PLAN(plan);
    if (!target || !loss || !grad) return fail(HPSMC_EINVAL, "NULL argument");
    if (plan->twin) return fail(HPSMC_ENOTSUP, "no gradient under the precision switch");
    if (plan->n_iv != 1 || plan->pb.ic_kind != HPSMC_IC_PHI || plan->pb.schedule != HPSMC_SEQUENTIAL)
        return fail(HPSMC_EINVAL, "the gradient needs one interval, phi-coefficient initial data, sequential schedule");
    if (plan->d > 2 || plan->P > 32 || !plan->sets[0].rounds)
        return fail(HPSMC_ENOTSUP, "the adjoint kernel covers dim <= 2 and n <= 30");
    if (plan->pb.estimator != HPSMC_EST_RESIDUAL) return fail(HPSMC_ENOTSUP, "the adjoint is that of the residual form");
    if (plan->pb.accel != HPSMC_ACCEL_NONE) return fail(HPSMC_ENOTSUP, "the adjoint is that of the unrelaxed iteration");
    if (plan->pb.quad != HPSMC_QUAD_CENTRE) return fail(HPSMC_ENOTSUP, "the adjoint is that of the centre-point rule");
    if (plan->frac) return fail(HPSMC_ENOTSUP, "no adjoint for the fractional operator");
    hipStream_t s = (hipStream_t)stream;
    const int d = plan->d, n = plan->n, P = plan->P, K = plan->pb.iters, T1 = plan->degree[0] + 1;
    const int64_t I = plan->n_inst, nsp = plan->nsp, psp = plan->psp;
    const int64_t usz = I * nsp * T1, csz = I * psp * T1;
    NodeSet &set = plan->sets[0];
    hpsmc_status st;
    if (!plan->lam) {
        if ((st = dalloc(plan, (void **)&plan->hist_u, (size_t)K * csz * 8)) ||
            (st = dalloc(plan, (void **)&plan->hist_v, (size_t)K * csz * 8)) ||
            (st = dalloc(plan, (void **)&plan->lam, (size_t)usz * 8)) ||
            (st = dalloc(plan, (void **)&plan->cbar_u, (size_t)csz * 8)) ||
            (st = dalloc(plan, (void **)&plan->cbar_v, (size_t)csz * 8)) ||
            (st = dalloc(plan, (void **)&plan->dtarget, (size_t)I * nsp * 8)) ||
            (st = dalloc(plan, (void **)&plan->dloss, (size_t)I * 8)) ||
            (st = dalloc(plan, (void **)&plan->dgrad, (size_t)I * nsp * 8)) ||
            (st = dalloc(plan, &plan->slab_bar, bar_alloc_bytes(plan, set))))
            return st;
    }
    HIP_TRY(hipMemcpyAsync(plan->dtarget, target, (size_t)I * nsp * 8,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    // forward, keeping every iteration's Legendre tensors
    if ((st = start_interval(plan, 0, 1, s))) return st;
    for (int k = 0; k < K; ++k) {
        if ((st = reconstruct(plan, 0, s))) return st;
        HIP_TRY(hipMemcpyAsync(plan->hist_u + (size_t)k * csz, plan->cu, csz * 8, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(plan->hist_v + (size_t)k * csz, plan->cv, csz * 8, hipMemcpyDeviceToDevice, s));
        if ((st = sample_set(plan, set, plan->pb.fresh_per_iter ? k : 0, plan->n_records, s))) return st;
    }
    // terminal misfit and its nodal adjoint
    HIP_TRY(launch_fill_u64((unsigned long long *)plan->lam, usz, 0ull, s));
    HIP_TRY(launch_loss_lambda(plan->U, plan->dtarget, (int)I, nsp, T1, plan->lam, plan->dloss, s));
    const double h = plan->t_breaks[1] - plan->t_breaks[0];
    const double *M = plan->mats;
    for (int k = K - 1; k >= 0; --k) {
        HIP_TRY(hipMemcpyAsync(plan->cu, plan->hist_u + (size_t)k * csz, csz * 8, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(plan->cv, plan->hist_v + (size_t)k * csz, csz * 8, hipMemcpyDeviceToDevice, s));
        SlabArgs sa;   // the slabs in the layout the adjoint reads
        if ((st = slab_args_for(plan, set, adjoint_mfma_mode(plan, set) == 2 ? 1 : 0, false, sa, s))) return st;
        HIP_TRY(launch_slabs(sa, plan->fp32, set.max_nstar, s));
        // the adjoint accumulates into the row layout's extent of the table
        HIP_TRY(launch_fill_u64((unsigned long long *)plan->slab_bar, (int64_t)(bar_alloc_bytes(plan, set) / 8), 0ull, s));
        if ((st = adjoint_sampling(plan, set, plan->pb.fresh_per_iter ? k : 0, s))) return st;
        SlabArgs sb = set.slab;
        sb.slab_table = plan->slab_bar;
        HIP_TRY(launch_slab_adjoint(sb, plan->degree[0], (int)I, plan->fp32, plan->cbar_u, plan->cbar_v, psp * T1, s));
        // cbar_u += (c^u -> c^v)^T cbar_v
        for (int i = 0; i < d; ++i)
            HIP_TRY(launch_mode_product(plan->cbar_v, plan->cbar_u, I * ipow(P, i), P, P, ipow(P, d - 1 - i) * T1,
                                        M + plan->d2t_off, 1.0, 1, s));
        HIP_TRY(launch_mode_product(plan->cbar_v, plan->cbar_u, I * psp, T1, T1, 1, M + plan->d1t_off[0], -2.0 / h, 1, s));
        // Ubar = cbar_u x_t Bt^T x_1 G0^T ... x_d G0^T;  lambda += Ubar
        HIP_TRY(launch_mode_product(plan->cbar_u, plan->tmp0, I * psp, T1, T1, 1, M + plan->btt_off[0], 1.0, 0, s));
        const double *in = plan->tmp0;
        double *bufs[2] = {plan->tmp1, plan->tmp0};
        for (int i = 0; i < d; ++i) {
            double *o = bufs[i & 1];
            HIP_TRY(launch_mode_product(in, o, I * ipow(n, i), P, n, ipow(P, d - 1 - i) * T1, M + plan->g0t_off, 1.0, 0, s));
            in = o;
        }
        HIP_TRY(launch_axpy(plan->lam, in, usz, s));
    }
    // dL/dc = Phi^T sum_l lambda[:, l]
    HIP_TRY(launch_column_sum(plan->lam, I * nsp, T1, plan->cbar_v, s));
    if ((st = phi_apply(plan, plan->cbar_v, plan->dgrad, plan->phit_off, s))) return st;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIP_TRY(hipMemcpyAsync(loss, plan->dloss, (size_t)I * 8, kind, s));
    HIP_TRY(hipMemcpyAsync(grad, plan->dgrad, (size_t)I * nsp * 8, kind, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HPSMC_OK;
}

}  // extern "C"
