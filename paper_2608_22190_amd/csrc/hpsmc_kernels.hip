// gfx950 kernels of the spectral Monte Carlo hot path (arXiv 2608.22190).
//
//   mode_product   -- nodal -> Legendre-tensor transform, one tensor mode at a
//                     time (Sec. 2.3, eq. u_N); FP64.
//   slabs          -- time contraction of the Legendre-tensor coefficients of
//                     u* and of v* = Lap u* - d_t u* at every path step of every
//                     node time: the spatial coefficient slab the walk reads.
//   sample         -- persistent kernel: one wavefront per batch of
//                     node-samples; Philox directions, sphere jumps with the
//                     exit test (Lemma 2.1, eq. indexL), tensor-product Legendre
//                     evaluation by three-term recurrence against the slab,
//                     residual f(u*) + s + v* and its left-point path quadrature
//                     (eq. interIQ); deterministic per-chunk FP64 sums.
//   reduce_update  -- eps = sample mean (eq. varepsilon_1), U += eps
//                     (Algorithm 1, Step 3), max|eps| (the stop metric).
#include "hpsmc_internal.h"

#include <algorithm>
#include <type_traits>

namespace hpsmc {

// ---------------------------------------------------------------------------
// Legendre three-term recurrence L_{k+1} = a_k x L_k - b_k L_{k-1},
// a_k = (2k+1)/(k+1), b_k = k/(k+1).
// ---------------------------------------------------------------------------
struct RecTable {
    double ad[kMaxP + 2], bd[kMaxP + 2];
    float af[kMaxP + 2], bf[kMaxP + 2];
    double mu[kMaxP + 2];   // leading coefficient of L_k: L_k = mu_k Q_k, Q_k monic
};
__constant__ RecTable c_rec;

hipError_t set_recurrence_tables()
{
    RecTable t;
    for (int k = 0; k < kMaxP + 2; ++k) {
        t.ad[k] = (2.0 * k + 1.0) / (k + 1.0);
        t.bd[k] = double(k) / (k + 1.0);
        t.af[k] = float(t.ad[k]);
        t.bf[k] = float(t.bd[k]);
    }
    t.mu[0] = 1.0;
    for (int k = 0; k + 1 < kMaxP + 2; ++k) t.mu[k + 1] = t.mu[k] * t.ad[k];
    return hipMemcpyToSymbol(HIP_SYMBOL(c_rec), &t, sizeof(t));
}

template <typename T> __device__ __forceinline__ T rec_a(int k);
template <typename T> __device__ __forceinline__ T rec_b(int k);
template <> __device__ __forceinline__ double rec_a<double>(int k) { return c_rec.ad[k]; }
template <> __device__ __forceinline__ double rec_b<double>(int k) { return c_rec.bd[k]; }
template <> __device__ __forceinline__ float rec_a<float>(int k) { return c_rec.af[k]; }
template <> __device__ __forceinline__ float rec_b<float>(int k) { return c_rec.bf[k]; }

// wave-uniform read-only data is read through the constant address space so
// that uniform addresses become scalar loads feeding VALU operands directly
template <typename T> using cptr = const __attribute__((address_space(4))) T *;
template <typename T> __device__ __forceinline__ cptr<T> as_const(const T *p) { return (cptr<T>)p; }

// ---------------------------------------------------------------------------
// Math in the sampling precision.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double m_sin(double x) { return sin(x); }
__device__ __forceinline__ float m_sin(float x) { return sinf(x); }
__device__ __forceinline__ double m_cos(double x) { return cos(x); }
__device__ __forceinline__ float m_cos(float x) { return cosf(x); }
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_exp(float x) { return expf(x); }
__device__ __forceinline__ double m_log(double x) { return log(x); }
__device__ __forceinline__ float m_log(float x) { return logf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_fma(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float m_fma(float a, float b, float c) { return fmaf(a, b, c); }

// uniform variate from one Philox word: FP64 uses all 32 bits, FP32 the top 24
__device__ __forceinline__ double u01(uint32_t w, double) { return ((double)w + 0.5) * 0x1p-32; }
__device__ __forceinline__ float u01(uint32_t w, float) { return ((float)(w >> 8) + 0.5f) * 0x1p-24f; }

// direction angle 2*pi*u
__device__ __forceinline__ void angle_dir(double u, double &c, double &s)
{
    const double th = 2.0 * 3.14159265358979323846 * u;
    c = cos(th);
    s = sin(th);
}
__device__ __forceinline__ void angle_dir(float u, float &c, float &s) { sincospif(2.0f * u, &s, &c); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 S-box with
// multipliers D2511F53 / CD9E8D57 and Weyl key steps 9E3779B9 / BB67AE85.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1, uint32_t (&o)[4])
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o[0] = c0; o[1] = c1; o[2] = c2; o[3] = c3;
}

// ---------------------------------------------------------------------------
// Ball point of walk step q (the Green's-function representation of a step's
// path integral, Sec. 3): an offset in the unit ball whose radius s has the
// density of s^{d-1} G(s), G the Green's function of -Laplace on the ball with
// pole at its centre -- the law of sqrt(U_a) * U_b^{1/d} -- in a uniform
// direction.  Counter word 2 = bit 31 | 2q (radius words 0, 1; direction
// words 2, 3) and, for d >= 3, bit 31 | (2q + 1) for two more normal pairs.
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void ball_offset(uint32_t c0, uint32_t c1, int q, uint32_t c3, uint32_t k0, uint32_t k1,
                                            T (&off)[D])
{
    uint32_t o[4];
    philox(c0, c1, 0x80000000u | (uint32_t)(2 * q), c3, k0, k1, o);
    const T ua = u01(o[0], (T)0), ub = u01(o[1], (T)0);
    T root;
    if constexpr (D == 1) root = ub;
    else if constexpr (D == 2) root = m_sqrt(ub);
    else if constexpr (D == 3) root = sizeof(T) == 4 ? (T)cbrtf((float)ub) : (T)cbrt((double)ub);
    else if constexpr (D == 4) root = m_sqrt(m_sqrt(ub));
    else root = sizeof(T) == 4 ? (T)powf((float)ub, 0.2f) : (T)pow((double)ub, 0.2);
    const T sr = m_sqrt(ua) * root;
    if constexpr (D == 1) {
        off[0] = (o[2] & 1u) ? sr : -sr;
    } else if constexpr (D == 2) {
        T c, sn;
        angle_dir(u01(o[2], (T)0), c, sn);
        off[0] = sr * c;
        off[1] = sr * sn;
    } else {
        uint32_t o2[4];
        philox(c0, c1, 0x80000000u | (uint32_t)(2 * q + 1), c3, k0, k1, o2);
        const uint32_t ww[6] = {o[2], o[3], o2[0], o2[1], o2[2], o2[3]};
        T g[6];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T r = m_sqrt((T)-2 * m_log(u01(ww[2 * k], (T)0)));
            T c, sn;
            angle_dir(u01(ww[2 * k + 1], (T)0), c, sn);
            g[2 * k] = r * c;
            g[2 * k + 1] = r * sn;
        }
        T nrm = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) nrm += g[i] * g[i];
        nrm = m_sqrt(nrm);
#pragma unroll
        for (int i = 0; i < D; ++i) off[i] = sr * g[i] / nrm;
    }
}

// ---------------------------------------------------------------------------
// Problem terms.
// ---------------------------------------------------------------------------
// sin(u) for the nonlinearity: FP32 arguments with |u| <= 2 take the sine's
// Maclaurin series to u^17/17! (truncation below 4e-10 there, no range
// reduction); larger ones and FP64 the library sine
__device__ __forceinline__ double sin_of_u(double u) { return sin(u); }
__device__ __forceinline__ float sin_of_u(float u)
{
    if (fabsf(u) <= 2.f) {
        const float z = u * u;
        float p = (float)(1.0 / 355687428096000.0);         // +1/17!
        p = fmaf(p, z, (float)(-1.0 / 1307674368000.0));   // -1/15!
        p = fmaf(p, z, (float)(1.0 / 6227020800.0));       // +1/13!
        p = fmaf(p, z, (float)(-1.0 / 39916800.0));        // -1/11!
        p = fmaf(p, z, (float)(1.0 / 362880.0));           // +1/9!
        p = fmaf(p, z, (float)(-1.0 / 5040.0));            // -1/7!
        p = fmaf(p, z, (float)(1.0 / 120.0));              // +1/5!
        p = fmaf(p, z, (float)(-1.0 / 6.0));               // -1/3!
        return fmaf(p * z, u, u);
    }
    return sinf(u);
}

template <typename T>
__device__ __forceinline__ T f_of(const Physics &ph, T u)
{
    switch (ph.f_kind) {
    case 0: return (T)ph.f_param[0] * u + (T)ph.f_param[1];
    case 1: return u - u * u * u;
    case 2: return sin_of_u(u);
    case 3: return u * u / ((T)1 + u * u);
    case 4: return -u * u * u;
    case 5: return u * sin_of_u(u);
    }
    return (T)0;
}

template <typename T>
__device__ __forceinline__ T fprime_of(const Physics &ph, T u)
{
    switch (ph.f_kind) {
    case 0: return (T)ph.f_param[0];
    case 1: return (T)1 - (T)3 * u * u;
    case 2: return m_cos(u);
    case 3: { T a = (T)1 + u * u; return (T)2 * u / (a * a); }
    case 4: return (T)-3 * u * u;
    case 5: return m_sin(u) + u * m_cos(u);
    }
    return (T)0;
}

// s = u_t - Lap u - f(u) at the manufactured exact solution, split into the
// factors that depend on time only (the same for every path of a group at one
// walk step) and the spatial evaluation that combines them.
template <typename T> struct SrcTime {
    T a, b;
};

template <typename T>
__device__ __forceinline__ SrcTime<T> source_time(const Physics &ph, T t)
{
    switch (ph.src_kind) {
    case 1:
    case 2:
        return {m_exp(-t), (T)0};
    case 3: {
        const T q = (T)1 + t * t;
        const T Tt = m_exp(m_cos(t)) / q;
        return {Tt, Tt * (-m_sin(t) - (T)2 * t / q)};
    }
    case 4: {
        const T c0 = (T)ph.src_param[0], c1 = (T)ph.src_param[1], c2 = (T)ph.src_param[2];
        return {c0 + c1 * t + c2 * t * t, c1 + (T)2 * c2 * t};
    }
    }
    return {(T)0, (T)0};
}

__device__ __forceinline__ void m_sincos(double x, double &s, double &c) { sincos(x, &s, &c); }
__device__ __forceinline__ void m_sincos(float x, float &s, float &c) { sincosf(x, &s, &c); }

// sin and cos of |x| <= 2 by their Maclaurin series in Horner form (terms to
// x^17/17! and x^18/18!; the truncation error is below 4e-10 there): no range
// reduction and no branch
__device__ __forceinline__ void sincos_small(float x, float &s, float &c)
{
    const float z = x * x;
    float ps = (float)(1.0 / 355687428096000.0);         // +1/17!
    ps = fmaf(ps, z, (float)(-1.0 / 1307674368000.0));   // -1/15!
    ps = fmaf(ps, z, (float)(1.0 / 6227020800.0));       // +1/13!
    ps = fmaf(ps, z, (float)(-1.0 / 39916800.0));        // -1/11!
    ps = fmaf(ps, z, (float)(1.0 / 362880.0));           // +1/9!
    ps = fmaf(ps, z, (float)(-1.0 / 5040.0));            // -1/7!
    ps = fmaf(ps, z, (float)(1.0 / 120.0));              // +1/5!
    ps = fmaf(ps, z, (float)(-1.0 / 6.0));               // -1/3!
    s = fmaf(ps * z, x, x);
    float pc = (float)(-1.0 / 6402373705728000.0);      // -1/18!
    pc = fmaf(pc, z, (float)(1.0 / 20922789888000.0));   // +1/16!
    pc = fmaf(pc, z, (float)(-1.0 / 87178291200.0));     // -1/14!
    pc = fmaf(pc, z, (float)(1.0 / 479001600.0));       // +1/12!
    pc = fmaf(pc, z, (float)(-1.0 / 3628800.0));         // -1/10!
    pc = fmaf(pc, z, (float)(1.0 / 40320.0));            // +1/8!
    pc = fmaf(pc, z, (float)(-1.0 / 720.0));             // -1/6!
    pc = fmaf(pc, z, (float)(1.0 / 24.0));               // +1/4!
    pc = fmaf(pc, z, -0.5f);                             // -1/2!
    c = fmaf(pc, z, 1.0f);
}

// BOUNDED: the point lies in (-1,1)^2 (d = 2, FP32), so sin/cos of x0 + x1 use
// the branch-free series above
template <typename T, int D, bool BOUNDED = false>
__device__ __forceinline__ T source_space(const Physics &ph, const T (&X)[D], SrcTime<T> tf)
{
    const T pi = (T)3.14159265358979323846;
    T u, ut, lap;
    switch (ph.src_kind) {
    case 1: {
        T p = tf.a;
#pragma unroll
        for (int i = 0; i < D; ++i) p *= m_sin(pi * X[i]);
        u = p; ut = -p; lap = -(T)D * pi * pi * p;
        break;
    }
    case 2: {
        T p = tf.a;
#pragma unroll
        for (int i = 0; i < D; ++i) p *= m_cos((T)0.5 * pi * X[i]);
        u = p; ut = -p; lap = (T)(-0.25 * D) * pi * pi * p;
        break;
    }
    case 3: {
        T om[D], a = (T)1, sig = (T)0;
#pragma unroll
        for (int i = 0; i < D; ++i) { om[i] = (T)1 - X[i] * X[i]; a *= om[i]; sig += X[i]; }
        T lapa = 0, grada = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            T rest = (T)1;
#pragma unroll
            for (int m = 0; m < D; ++m) if (m != i) rest *= om[m];
            lapa += (T)-2 * rest;
            grada += (T)-2 * X[i] * rest;
        }
        T S, C;
        if constexpr (BOUNDED && D == 2 && std::is_same<T, float>::value)
            sincos_small(sig, S, C);
        else
            m_sincos(sig, S, C);
        u = a * S * tf.a;
        ut = a * S * tf.b;
        lap = tf.a * (S * lapa + (T)2 * C * grada - (T)D * a * S);
        break;
    }
    case 4: {
        T om[D], a = (T)1;
#pragma unroll
        for (int i = 0; i < D; ++i) { om[i] = (T)1 - X[i] * X[i]; a *= om[i]; }
        T lapa = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            T rest = (T)1;
#pragma unroll
            for (int m = 0; m < D; ++m) if (m != i) rest *= om[m];
            lapa += (T)-2 * rest;
        }
        u = a * tf.a; ut = a * tf.b; lap = lapa * tf.a;
        break;
    }
    default:
        return (T)0;
    }
    return ut - lap - f_of<T>(ph, u);
}

template <typename T, int D>
__device__ __forceinline__ T source_of(const Physics &ph, const T (&X)[D], T t)
{
    return source_space<T, D>(ph, X, source_time<T>(ph, t));
}

// ---------------------------------------------------------------------------
// Tensor-product Legendre contraction of one step's slab.
//   u(X) = sum_k Su[k] prod_i L_{k_i}(X_i),  v(X) likewise with Sv.
// The last dimension's L values sit in registers (Ll); the outer dimensions
// run as loops whose L values advance by the recurrence on the fly.  Slab rows
// are wave-uniform: [u: PP][v: PP] per multi-index of the first d-1 dims.
// UO skips the v half: the Picard-form integrand needs u only.
// ---------------------------------------------------------------------------
template <typename T, int D, int PMAX, int NS, int LV, typename SP, bool UO = false>
__device__ __forceinline__ void contract(SP S, int P, int PP, const T (&X)[NS][D], const T (&W)[NS],
                                         const T (&Ll)[NS][PMAX], T (&u)[NS], T (&v)[NS], int row)
{
    if constexpr (LV == D - 1) {
        // rows are padded with zeros to a multiple of 4 modes and read 4 at a time
        SP srow = S + (int64_t)row * (2 * PP);
        T tu[NS], tv[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) { tu[s] = (T)0; tv[s] = (T)0; }
        if constexpr (UO) {
#pragma unroll
            for (int kb = 0; kb < PMAX / 4; ++kb) {
                if (kb * 4 < P) {
                    T cu[4];
                    if constexpr (std::is_same<SP, const T *>::value) {
                        typedef T v4 __attribute__((ext_vector_type(4)));
                        const v4 qu = *(const v4 *)(srow + 4 * kb);
                        cu[0] = qu.x; cu[1] = qu.y; cu[2] = qu.z; cu[3] = qu.w;
                    } else {
#pragma unroll
                        for (int c = 0; c < 4; ++c) cu[c] = srow[4 * kb + c];
                    }
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
#pragma unroll
                        for (int s = 0; s < NS; ++s) tu[s] = m_fma(cu[c], Ll[s][4 * kb + c], tu[s]);
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) u[s] = m_fma(W[s], tu[s], u[s]);
            return;
        }
#pragma unroll
        for (int kb = 0; kb < PMAX / 4; ++kb) {
            if (kb * 4 < P) {
                T cu[4], cv[4];
                if constexpr (std::is_same<SP, const T *>::value) {
                    // rows and half-rows start on multiples of 4 elements: one vector read each
                    typedef T v4 __attribute__((ext_vector_type(4)));
                    const v4 qu = *(const v4 *)(srow + 4 * kb), qv = *(const v4 *)(srow + PP + 4 * kb);
                    cu[0] = qu.x; cu[1] = qu.y; cu[2] = qu.z; cu[3] = qu.w;
                    cv[0] = qv.x; cv[1] = qv.y; cv[2] = qv.z; cv[3] = qv.w;
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) { cu[c] = srow[4 * kb + c]; cv[c] = srow[PP + 4 * kb + c]; }
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        tu[s] = m_fma(cu[c], Ll[s][4 * kb + c], tu[s]);
                        tv[s] = m_fma(cv[c], Ll[s][4 * kb + c], tv[s]);
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            u[s] = m_fma(W[s], tu[s], u[s]);
            v[s] = m_fma(W[s], tv[s], v[s]);
        }
    } else {
        T Lp[NS], Lc[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) { Lp[s] = (T)0; Lc[s] = (T)1; }
        for (int k = 0; k < P; ++k) {
            T W2[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) W2[s] = W[s] * Lc[s];
            contract<T, D, PMAX, NS, LV + 1, SP, UO>(S, P, PP, X, W2, Ll, u, v, row * P + k);
            const T ak = rec_a<T>(k), bk = rec_b<T>(k);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const T nx = ak * X[s][LV] * Lc[s] - bk * Lp[s];
                Lp[s] = Lc[s];
                Lc[s] = nx;
            }
        }
    }
}

// 64-lane FP64 sum with a fixed butterfly (deterministic)
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// ---------------------------------------------------------------------------
// Persistent sampling kernel.  Each wavefront repeatedly takes one work item
// (node, chunk of 64*NS samples) from a global counter until none is left.
// ---------------------------------------------------------------------------
template <typename T, int D, int PMAX, int NS>
__global__ void __launch_bounds__(256) sample_kernel(SampleArgs a)
{
    const int lane = threadIdx.x & 63;
    cptr<T> table = as_const((const T *)a.slab_table);
    cptr<NodeDesc> nodes = as_const(a.nodes);
    const int64_t total = a.n_nodes * (int64_t)a.chunks_per_node;
    unsigned long long evals = 0, lsteps = 0;

    for (;;) {
        unsigned long long item = 0;
        if (lane == 0) item = atomicAdd(a.work, 1ull);
        const uint32_t lo = uniform_u32((uint32_t)item), hi = uniform_u32((uint32_t)(item >> 32));
        const int64_t it = (int64_t)(((uint64_t)hi << 32) | lo);
        if (it >= total) break;
        const int64_t ni = it / a.chunks_per_node;
        const int chunk = (int)(it - ni * a.chunks_per_node);
        cptr<NodeDesc> nd = nodes + ni;

        const T delta = (T)nd->delta, J = (T)nd->jump;
        const double span = nd->span, t_prev = nd->t_prev, ddelta = nd->delta;
        const int nstar = nd->nstar;
        const uint32_t c0 = nd->c0, c3 = nd->c3 | (uint32_t)a.tag;
        cptr<T> slab0 = table + nd->slab;
        const int out = nd->out;

        T X[NS][D], Y[NS][D], acc[NS], comp[NS];
        bool alive[NS];
        int64_t sample[NS];
        uint32_t w[NS][4];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            sample[s] = (int64_t)chunk * (64 * NS) + s * 64 + lane;
            alive[s] = sample[s] < a.M;
#pragma unroll
            for (int i = 0; i < D; ++i) X[s][i] = (T)nd->x0[i];
            acc[s] = (T)0;
            comp[s] = (T)0;
        }

        for (int q = 0; q < nstar; ++q) {
            // ---- draw the jump direction and test the new ball centre
            T dir[NS][D];
            if constexpr (D == 1) {
                if ((q & 127) == 0) {
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        philox(c0, (uint32_t)sample[s], (uint32_t)(q >> 7), c3, a.key0, a.key1, w[s]);
                }
                const int wi = (q >> 5) & 3, b = q & 31;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    uint32_t word = wi == 0 ? w[s][0] : wi == 1 ? w[s][1] : wi == 2 ? w[s][2] : w[s][3];
                    dir[s][0] = ((word >> b) & 1u) ? (T)1 : (T)-1;
                }
            } else if constexpr (D == 2) {
                if ((q & 3) == 0) {
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        philox(c0, (uint32_t)sample[s], (uint32_t)(q >> 2), c3, a.key0, a.key1, w[s]);
                }
                const int wi = q & 3;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    uint32_t word = wi == 0 ? w[s][0] : wi == 1 ? w[s][1] : wi == 2 ? w[s][2] : w[s][3];
                    angle_dir(u01(word, (T)0), dir[s][0], dir[s][1]);
                }
            } else {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    uint32_t ww[8];
                    if constexpr (D <= 4) {
                        uint32_t o[4];
                        philox(c0, (uint32_t)sample[s], (uint32_t)q, c3, a.key0, a.key1, o);
                        ww[0] = o[0]; ww[1] = o[1]; ww[2] = o[2]; ww[3] = o[3];
                    } else {
                        uint32_t o[4], o2[4];
                        philox(c0, (uint32_t)sample[s], (uint32_t)(2 * q), c3, a.key0, a.key1, o);
                        philox(c0, (uint32_t)sample[s], (uint32_t)(2 * q + 1), c3, a.key0, a.key1, o2);
                        ww[0] = o[0]; ww[1] = o[1]; ww[2] = o[2]; ww[3] = o[3];
                        ww[4] = o2[0]; ww[5] = o2[1]; ww[6] = o2[2]; ww[7] = o2[3];
                    }
                    T g[D + 1];
#pragma unroll
                    for (int k = 0; k < (D + 1) / 2; ++k) {
                        const T r = m_sqrt((T)-2 * m_log(u01(ww[2 * k], (T)0)));
                        T c, sn;
                        angle_dir(u01(ww[2 * k + 1], (T)0), c, sn);
                        g[2 * k] = r * c;
                        g[2 * k + 1] = r * sn;
                    }
                    T nrm = 0;
#pragma unroll
                    for (int i = 0; i < D; ++i) nrm += g[i] * g[i];
                    nrm = m_sqrt(nrm);
#pragma unroll
                    for (int i = 0; i < D; ++i) dir[s][i] = g[i] / nrm;
                }
            }
            bool any_live = false;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (alive[s]) {
                    bool inside = true;
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        Y[s][i] = m_fma(J, dir[s][i], X[s][i]);
                        inside = inside && (fabs(Y[s][i]) < (T)1);
                    }
                    alive[s] = inside;   // eq. indexL: the path ends when the new centre has left
                }
                any_live = any_live || alive[s];
            }
            lsteps += NS;
            if (__ballot(any_live) == 0ull) break;

            // ---- residual at the current centre X_q and time tau_q = t_{n,l} - q Delta
            cptr<T> S = slab0 + (int64_t)q * a.slab_stride;
            T Ll[NS][PMAX];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const T x = X[s][D - 1];
                Ll[s][0] = (T)1;
                if (PMAX > 1) Ll[s][1] = x;
#pragma unroll
                for (int k = 1; k + 1 < PMAX; ++k)
                    Ll[s][k + 1] = (T)((2.0 * k + 1.0) / (k + 1.0)) * x * Ll[s][k] - (T)(k / (k + 1.0)) * Ll[s][k - 1];
            }
            T u[NS], v[NS], W[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) { u[s] = (T)0; v[s] = (T)0; W[s] = (T)1; }
            contract<T, D, PMAX, NS, 0, cptr<T>>(S, a.P, a.PP, X, W, Ll, u, v, 0);

            const T tau = (T)(t_prev + (span - (double)q * ddelta));
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (alive[s]) {
                    const T r = f_of<T>(a.phys, u[s]) + source_of<T, D>(a.phys, X[s], tau) + v[s];
                    const T y = delta * r;
                    if constexpr (sizeof(T) == 4) {   // Kahan-compensated FP32 path sum
                        const T yc = y - comp[s];
                        const T tt = acc[s] + yc;
                        comp[s] = (tt - acc[s]) - yc;
                        acc[s] = tt;
                    } else {
                        acc[s] += y;
                    }
#pragma unroll
                    for (int i = 0; i < D; ++i) X[s][i] = Y[s][i];
                    ++evals;
                }
            }
        }

        // ---- per-chunk sums in FP64 (fixed order), optional per-sample probe
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double Sv = (double)acc[s] - (double)comp[s];
            s1 += Sv;
            s2 += Sv * Sv;
            if (a.probe != nullptr && sample[s] < a.m_probe && sample[s] < a.M)
                a.probe[(int64_t)out * a.m_probe + sample[s]] = Sv;
        }
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        if (lane == 0) {
            double *pp = a.part + ((int64_t)out * a.chunks_per_node + chunk) * 2;
            pp[0] = s1;
            pp[1] = s2;
        }
    }
    evals = wave_sum_u64(evals);
    lsteps = wave_sum_u64(lsteps);
    if (lane == 0) {
        atomicAdd(a.stats + 0, evals);
        atomicAdd(a.stats + 1, lsteps);
    }
}

// ---------------------------------------------------------------------------
// Dispatch of the sampling kernel over (precision, dim, mode bucket, NS).
// ---------------------------------------------------------------------------
template <typename T, int D, int PMAX>
static hipError_t dispatch_ns(const SampleArgs &a, int ns, dim3 grid, dim3 block, hipStream_t s)
{
    switch (ns) {
    case 1: hipLaunchKernelGGL((sample_kernel<T, D, PMAX, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((sample_kernel<T, D, PMAX, 2>), grid, block, 0, s, a); break;
    case 4:
        if constexpr (D <= 2) { hipLaunchKernelGGL((sample_kernel<T, D, PMAX, 4>), grid, block, 0, s, a); break; }
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int D>
static hipError_t dispatch_p(const SampleArgs &a, int ns, dim3 grid, dim3 block, hipStream_t s)
{
    if (a.P <= 12) return dispatch_ns<T, D, 12>(a, ns, grid, block, s);
    if constexpr (D <= 4) {
        if (a.P <= 20) return dispatch_ns<T, D, 20>(a, ns, grid, block, s);
    }
    if constexpr (D <= 3) {
        if (a.P <= 28) return dispatch_ns<T, D, 28>(a, ns, grid, block, s);
        if (a.P <= 36) return dispatch_ns<T, D, 36>(a, ns, grid, block, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t dispatch_d(const SampleArgs &a, int ns, dim3 grid, dim3 block, hipStream_t s)
{
    switch (a.phys.dim) {
    case 1: return dispatch_p<T, 1>(a, ns, grid, block, s);
    case 2: return dispatch_p<T, 2>(a, ns, grid, block, s);
    case 3: return dispatch_p<T, 3>(a, ns, grid, block, s);
    case 4: return dispatch_p<T, 4>(a, ns, grid, block, s);
    case 5: return dispatch_p<T, 5>(a, ns, grid, block, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sample(const SampleArgs &a, int fp32, int samples_per_lane, int waves_per_block,
                         int blocks, hipStream_t s)
{
    dim3 block(64 * waves_per_block), grid(blocks);
    return fp32 ? dispatch_d<float>(a, samples_per_lane, grid, block, s)
                : dispatch_d<double>(a, samples_per_lane, grid, block, s);
}

// ---------------------------------------------------------------------------
// Mode product: out[o][a][i] (+)= alpha * sum_b mat[a][b] in[o][b][i].
// ---------------------------------------------------------------------------
__global__ void mode_product_kernel(const double *__restrict__ in, double *__restrict__ out, int64_t outer,
                                    int len_in, int len_out, int64_t inner, const double *__restrict__ mat,
                                    double alpha, int accumulate)
{
    const int64_t total = outer * len_out * inner;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % inner;
        const int64_t r = idx / inner;
        const int aa = (int)(r % len_out);
        const int64_t o = r / len_out;
        const double *src = in + o * len_in * inner + i;
        const double *m = mat + (int64_t)aa * len_in;
        double s = 0.0;
        for (int b = 0; b < len_in; ++b) s = fma(m[b], src[(int64_t)b * inner], s);
        out[idx] = accumulate ? fma(alpha, s, out[idx]) : alpha * s;
    }
}

hipError_t launch_mode_product(const double *in, double *out, int64_t outer, int len_in, int len_out,
                               int64_t inner, const double *mat, double alpha, int accumulate, hipStream_t s)
{
    const int64_t total = outer * len_out * inner;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(mode_product_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, out, outer, len_in,
                       len_out, inner, mat, alpha, accumulate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Slabs: for group g = (inst, iv, l) and step q < N*, the spatial coefficient
// rows of u* and v* at the reference time xi = 2 (span - q Delta)/h - 1.
// A block takes kSlabQ consecutive steps of one group: the Legendre values
// L_k(xi_q) of its steps go to LDS once, and every entry's T1 time
// coefficients are loaded once into registers and contracted with each step's
// values (the same products in the same order as entry by entry).
// ---------------------------------------------------------------------------
constexpr int kSlabQ = 32;

template <typename T>
__global__ void __launch_bounds__(256) slab_kernel(SlabArgs a)
{
    __shared__ double Lq[kSlabQ][kMaxDeg + 2];
    const int g = blockIdx.y;
    const int nq = a.nstar[g] + a.extra;
    const int T1 = a.deg[g] + 1;
    const bool mma = a.layout == 1;
    const int64_t stride = mma ? a.mma_stride : a.slab_stride;
    const int64_t base = mma ? a.slab_off_mma[g] : a.slab_off[g];
    T *table = (T *)a.slab_table;
    const double *cu = a.cu + a.coef_off[g], *cv = a.cv + a.coef_off[g];
    const double span = a.span[g], delta = a.delta[g], h2 = a.h2[g];
    for (int q0 = blockIdx.x * kSlabQ; q0 < nq; q0 += gridDim.x * kSlabQ) {
        const int qn = min(kSlabQ, nq - q0);
        __syncthreads();   // the previous chunk's reads of Lq are over
        if ((int)threadIdx.x < qn) {
            const double xi = h2 * (span - (double)(q0 + (int)threadIdx.x) * delta) - 1.0;
            double lp = 0.0, lc = 1.0;
            for (int k = 0; k < T1; ++k) {
                Lq[threadIdx.x][k] = lc;
                const double nx = c_rec.ad[k] * xi * lc - c_rec.bd[k] * lp;
                lp = lc;
                lc = nx;
            }
        }
        __syncthreads();
        for (int64_t e = threadIdx.x; e < stride; e += blockDim.x) {
            int64_t row;
            int uv, kl;
            if (mma) {   // column c = uv * PP + k1 of kMmaRows rows k0
                const int c = (int)(e / kMmaRows);
                row = e - (int64_t)c * kMmaRows;
                uv = c / a.PP;
                kl = c - uv * a.PP;
            } else {
                row = e / (2 * a.PP);
                const int rem = (int)(e - row * 2 * a.PP);
                uv = rem / a.PP;
                kl = rem - uv * a.PP;
            }
            const bool live = kl < a.P && row < a.rows;
            double c[kMaxDeg + 1];
            if (live) {
                const double *cp = (uv ? cv : cu) + (row * a.P + kl) * T1;
#pragma unroll
                for (int k = 0; k <= kMaxDeg; ++k) c[k] = k < T1 ? cp[k] : 0.0;
            }
            const double sc = mma && live ? c_rec.mu[kl] * c_rec.mu[row] : 1.0;   // coefficients of Q_{k0} Q_{k1}
            for (int j = 0; j < qn; ++j) {
                double val = 0.0;
                if (live) {
#pragma unroll
                    for (int k = 0; k <= kMaxDeg; ++k)
                        if (k < T1) val = fma(c[k], Lq[j][k], val);
                }
                if (mma) val *= sc;
                table[base + (int64_t)(q0 + j) * stride + e] = (T)val;
            }
        }
    }
}

hipError_t launch_slabs(const SlabArgs &a, int fp32, int max_nstar, hipStream_t s)
{
    if (a.n_groups <= 0) return hipSuccess;
    int64_t bx = (max_nstar + a.extra + kSlabQ - 1) / kSlabQ;
    if (bx > 65535) bx = 65535;
    dim3 grid((unsigned)bx, (unsigned)a.n_groups);
    if (fp32)
        hipLaunchKernelGGL(slab_kernel<float>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(slab_kernel<double>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// eps = (1/M) sum of the chunk sums in chunk order; U += eps; max|eps|.
// mode bit 0: Picard form (the estimate replaces U, eps = the change);
// bit 1: leave U alone (the Aitken kernel applies the weighted update).
// ---------------------------------------------------------------------------
__global__ void reduce_update_kernel(const double *__restrict__ part, int chunks, int mode,
                                     const NodeDesc *__restrict__ nodes,
                                     int64_t n_nodes, int64_t M, double *__restrict__ U, double *__restrict__ eps,
                                     double *__restrict__ sumsq, unsigned long long *maxbits)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double mx = 0.0;
    if (i < n_nodes) {
        const NodeDesc &nd = nodes[i];
        const double *p = part + (int64_t)nd.out * chunks * 2;
        double s1 = 0.0, s2 = 0.0;
        for (int c = 0; c < chunks; ++c) { s1 += p[2 * c]; s2 += p[2 * c + 1]; }
        double e = s1 / (double)M;
        if (mode & 2) {
            if (mode & 1) e -= U[nd.u_index];
        } else if (mode & 1) {   // eq. uast: the estimate replaces the iterate; eps is the change
            const double uo = U[nd.u_index];
            U[nd.u_index] = e;
            e -= uo;
        } else {
            U[nd.u_index] += e;
        }
        eps[nd.out] = e;
        sumsq[nd.out] = s2;
        mx = fabs(e);
        if (!(mx == mx)) mx = __longlong_as_double(0x7ff8000000000000ll);
    }
    // block max, then one atomic (max is order independent)
    __shared__ double sm[256];
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double b = sm[threadIdx.x + o];
            if (!(b <= sm[threadIdx.x])) sm[threadIdx.x] = b;   // NaN wins
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(sm[0]));
}

hipError_t launch_reduce_update(const double *part, int chunks, int mode, const NodeDesc *nodes, int64_t n_nodes,
                                int64_t M,
                                double *U, double *eps, double *sumsq, unsigned long long *maxbits, hipStream_t s)
{
    if (n_nodes <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_update_kernel, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, s, part, chunks,
                       mode, nodes, n_nodes, M, U, eps, sumsq, maxbits);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Aitken-relaxed update (the acceleration remark after Algorithm 1), one block
// per (instance, interval) vector of nodes [vbeg[v], vbeg[v+1]):
//   w = w0 on the vector's first iteration, else
//   w = -w_prev <e_prev, e - e_prev> / |e - e_prev|^2 (w_prev if that is 0/0),
// clipped to [wmin, wmax]; U += w e; e_prev = e.  state[2v] = w_prev,
// state[2v+1] = 1 once the vector has a history.  The two inner products are
// summed per thread in node order, then by a fixed tree: deterministic.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) aitken_update_kernel(const NodeDesc *__restrict__ nodes,
                                                            const int64_t *__restrict__ vbeg,
                                                            const double *__restrict__ eps,
                                                            double *__restrict__ eprev, double *__restrict__ state,
                                                            double w0, double wmin, double wmax,
                                                            double *__restrict__ U)
{
    const int v = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t b = vbeg[v], e = vbeg[v + 1];
    const bool have = state[2 * v + 1] != 0.0;
    double num = 0.0, den = 0.0;
    if (have) {
        for (int64_t i = b + tid; i < e; i += blockDim.x) {
            const int32_t o = nodes[i].out;
            const double rp = eprev[o], dr = eps[o] - rp;
            num = fma(rp, dr, num);
            den = fma(dr, dr, den);
        }
    }
    __shared__ double sn[256], sd[256];
    __shared__ double w_sh;
    sn[tid] = num;
    sd[tid] = den;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) {
            sn[tid] += sn[tid + o];
            sd[tid] += sd[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double wp = state[2 * v];
        double w = !have ? w0 : (sd[0] > 0.0 ? -wp * sn[0] / sd[0] : wp);
        if (w < wmin) w = wmin;
        if (w > wmax) w = wmax;
        if (!(w == w)) w = w0;
        w_sh = w;
    }
    __syncthreads();
    const double w = w_sh;
    for (int64_t i = b + tid; i < e; i += blockDim.x) {
        const NodeDesc &nd = nodes[i];
        const double r = eps[nd.out];
        U[nd.u_index] += w * r;
        eprev[nd.out] = r;
    }
    if (tid == 0) {
        state[2 * v] = w;
        state[2 * v + 1] = 1.0;
    }
}

hipError_t launch_aitken(const NodeDesc *nodes, const int64_t *vbeg, int n_vec, const double *eps, double *eprev,
                         double *state, double w0, double wmin, double wmax, double *U, hipStream_t s)
{
    if (n_vec <= 0) return hipSuccess;
    hipLaunchKernelGGL(aitken_update_kernel, dim3((unsigned)n_vec), dim3(256), 0, s, nodes, vbeg, eps, eprev, state,
                       w0, wmin, wmax, U);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Column 0 of an interval (and optionally every column) from a source column.
// ---------------------------------------------------------------------------
__global__ void start_columns_kernel(double *__restrict__ U, const double *__restrict__ src, int64_t src_stride,
                                     int64_t src_off, int64_t dst_stride, int T1, int64_t count, int replicate)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= count) return;
    const double v = src[r * src_stride + src_off];
    double *d = U + r * dst_stride;
    if (replicate)
        for (int l = 0; l < T1; ++l) d[l] = v;
    else
        d[0] = v;
}

hipError_t launch_start_columns(double *U, const double *src, int64_t src_stride, int64_t src_off, int64_t dst_stride,
                                int T1, int64_t count, int replicate, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(start_columns_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, U, src,
                       src_stride, src_off, dst_stride, T1, count, replicate);
    return hipGetLastError();
}

__global__ void fill_u64_kernel(unsigned long long *p, int64_t n, unsigned long long v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Off-node evaluation of u* and v* = Lap u* - d_t u* from the Legendre tensors.
// ---------------------------------------------------------------------------
__global__ void eval_kernel(const double *__restrict__ cu, const double *__restrict__ cv, int dim, int P, int T1,
                            double t_prev, double h, const double *__restrict__ pts, int64_t npts,
                            double *__restrict__ out)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= npts) return;
    double L[kMaxDim][kMaxP], Lt[kMaxDeg + 1];
    for (int i = 0; i < dim; ++i) {
        const double x = pts[k * (dim + 1) + i];
        L[i][0] = 1.0;
        if (P > 1) L[i][1] = x;
        for (int m = 1; m + 1 < P; ++m) L[i][m + 1] = ((2.0 * m + 1.0) * x * L[i][m] - m * L[i][m - 1]) / (m + 1.0);
    }
    const double xi = 2.0 * (pts[k * (dim + 1) + dim] - t_prev) / h - 1.0;
    Lt[0] = 1.0;
    if (T1 > 1) Lt[1] = xi;
    for (int m = 1; m + 1 < T1; ++m) Lt[m + 1] = ((2.0 * m + 1.0) * xi * Lt[m] - m * Lt[m - 1]) / (m + 1.0);
    int64_t np = 1;
    for (int i = 0; i < dim; ++i) np *= P;
    double u = 0.0, v = 0.0;
    for (int64_t f = 0; f < np; ++f) {
        int64_t r = f;
        double w = 1.0;
        for (int i = dim - 1; i >= 0; --i) { w *= L[i][r % P]; r /= P; }
        double a = 0.0, b = 0.0;
        for (int q = 0; q < T1; ++q) { a = fma(cu[f * T1 + q], Lt[q], a); b = fma(cv[f * T1 + q], Lt[q], b); }
        u = fma(w, a, u);
        v = fma(w, b, v);
    }
    out[2 * k] = u;
    out[2 * k + 1] = v;
}

hipError_t launch_eval(const double *cu, const double *cv, int dim, int P, int T1, double t_prev, double h,
                       const double *pts, int64_t npts, double *out, hipStream_t s)
{
    if (npts <= 0) return hipSuccess;
    hipLaunchKernelGGL(eval_kernel, dim3((unsigned)((npts + 63) / 64)), dim3(64), 0, s, cu, cv, dim, P, T1, t_prev,
                       h, pts, npts, out);
    return hipGetLastError();
}

// ===========================================================================
// Round-based path advancing.  A block takes a batch of live paths of one
// (instance, interval, l) group; every path of the batch shares the group's
// slab sequence, so the block stages the slab of each step in LDS (double
// buffered, one barrier per step) and all lanes read it with uniform
// (broadcast) addresses.  After `steps` steps the surviving paths are
// appended, compacted, to the group's region of the other state buffer, so
// every round starts with full batches whatever the spread of exit times.
// ===========================================================================
template <typename T, int D> struct PathState {
    T x[D];
    T acc, comp;
    uint32_t node;     // node row in the set's node array
    uint32_t sample;
};

size_t path_state_bytes(int fp32, int dim)
{
    switch (dim) {
    case 1: return fp32 ? sizeof(PathState<float, 1>) : sizeof(PathState<double, 1>);
    case 2: return fp32 ? sizeof(PathState<float, 2>) : sizeof(PathState<double, 2>);
    case 3: return fp32 ? sizeof(PathState<float, 3>) : sizeof(PathState<double, 3>);
    case 4: return fp32 ? sizeof(PathState<float, 4>) : sizeof(PathState<double, 4>);
    default: return fp32 ? sizeof(PathState<float, 5>) : sizeof(PathState<double, 5>);
    }
}

__global__ void round_prep_kernel(const GroupDesc *__restrict__ groups, int32_t n_groups, int32_t round,
                                  int32_t steps, int64_t mcount, int32_t batch, const uint32_t *__restrict__ live_in,
                                  uint32_t *__restrict__ live_out, int64_t *__restrict__ batch_prefix,
                                  unsigned long long *work)
{
    // one block of 256 threads: clear the output counters, then an exclusive
    // prefix over groups of their work items (each thread a contiguous chunk,
    // a scan of the 256 chunk sums in LDS, then the chunks again)
    __shared__ int64_t part[256];
    const int t = threadIdx.x, nt = blockDim.x;
    for (int g = t; g < n_groups; g += nt) live_out[g] = 0u;
    const int64_t q0 = (int64_t)round * steps;
    auto items = [&](int g) -> int64_t {
        int64_t live = round == 0 ? (int64_t)groups[g].node_count * mcount : (int64_t)live_in[g];
        if (q0 >= groups[g].nstar) live = 0;
        return (live + batch - 1) / batch;
    };
    const int chunk = (n_groups + nt - 1) / nt;
    const int g0 = min(n_groups, t * chunk), g1 = min(n_groups, g0 + chunk);
    int64_t sum = 0;
    for (int g = g0; g < g1; ++g) sum += items(g);
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int i = 0; i < nt; ++i) { const int64_t v = part[i]; part[i] = acc; acc += v; }
        batch_prefix[n_groups] = acc;
        *work = 0ull;
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int g = g0; g < g1; ++g) {
        batch_prefix[g] = acc;
        acc += items(g);
    }
}

hipError_t launch_round_prep(const GroupDesc *groups, int32_t n_groups, int32_t round, int32_t steps, int64_t mcount,
                             int32_t batch, const uint32_t *live_in, uint32_t *live_out, int64_t *batch_prefix,
                             unsigned long long *work, hipStream_t s)
{
    hipLaunchKernelGGL(round_prep_kernel, dim3(1), dim3(256), 0, s, groups, n_groups, round, steps, mcount, batch,
                       live_in, live_out, batch_prefix, work);
    return hipGetLastError();
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kMaxStageVec = 4;   // 16-byte slab vectors staged per thread and step
constexpr int kMmaRS = kMmaRows;  // LDS column stride (floats) of the transposed slab: odd, so
                                  // the 32 rows a half-wave reads fall in distinct banks

// Direct global -> LDS copy of a matrix-core slab image (gfx950
// global_load_lds_dwordx4): lane i of a wave writes its 16 bytes at
// wave_base + 16 i, so vector v of the image lands at LDS vector v.  The copy
// completes under vmcnt; mma_stage_wait() precedes the barrier that publishes it.
__device__ __forceinline__ void mma_stage(const u32x4 *src, u32x4 *dst, int nvec, int tid, int nthr)
{
    const int wbase = tid & ~63;
    for (int k = 0; k * nthr < nvec; ++k) {
        const int v = k * nthr + tid;
        if (v < nvec)
            __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)(src + v),
                                             (void __attribute__((address_space(3))) *)(dst + k * nthr + wbase),
                                             16, 0, 0);
    }
}
__device__ __forceinline__ void mma_stage_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// ---------------------------------------------------------------------------
// Matrix-core contraction of one step's 2-D slab for the 64 paths of a wave.
// For 32 paths s at points (x0_s, x1_s) and either coefficient table S (u or v):
//     T[k0][s] = sum_{k1} S[k0][k1] L_{k1}(x1_s)     -- a (32 x K) (K x 32) product
//     u_s      = sum_{k0} L_{k0}(x0_s) T[k0][s]
// The product runs on v_mfma_f32_32x32x2f32 (A: lane l holds A[l%32][l/32], B:
// B[l/32][l%32], D register r: D[8(r/4) + 4(l/32) + r%4][l%32]) with the mode
// axis k1 split into halves of KH = ceil(P/2): at step kk lanes 0-31 supply mode
// kk, lanes 32-63 mode KH + kk.  Paths 0-31 of the wave form one product and
// paths 32-63 the other; permlane32 swaps move each lane's own Legendre values
// into the operand layout and bring the rows of T back to the lane that owns
// the path, so no lane duplicates another's work.
// Sb: slab in LDS, transposed: Sb[c * kMmaRS + k0], c = k1 (u) or PP + k1 (v);
// rows k0 in [P, 32) hold zeros, columns k1 in [P, PP) the slab's zero padding.
// The image holds the coefficients of the monic basis Q_{k0} Q_{k1} (L_k =
// mu_k Q_k), so each basis value costs one multiply and one fma.
// ---------------------------------------------------------------------------

// B operands: monic Legendre values Q_{k1}(x1) of the wave's 64 points
template <int KH>
__device__ __forceinline__ void mma_operands(float x1, int P, float (&b0)[KH], float (&b1)[KH])
{
    static_assert(KH >= 2 && KH <= 16, "one 32-row tile, at least 4 modes");
    constexpr int K2 = 2 * KH;
    // monic Legendre polynomials Q_{k+1} = x Q_k - k^2/(4k^2-1) Q_{k-1} (the slab
    // image holds the coefficients of Q_{k0} Q_{k1})
    float L[K2];
    L[0] = 1.f;
    L[1] = x1;
#pragma unroll
    for (int k = 1; k + 1 < K2; ++k)
        L[k + 1] = fmaf(x1, L[k], -(float)((double)k * k / (4.0 * k * k - 1.0)) * L[k - 1]);
    if (P < K2) L[K2 - 1] = 0.f;   // odd P: mode P does not exist
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(L[kk]), __float_as_uint(L[KH + kk]), false, false);
        b0[kk] = __uint_as_float(r[0]);   // paths 0-31: lanes 0-31 modes kk, lanes 32-63 modes KH + kk
        b1[kk] = __uint_as_float(r[1]);   // paths 32-63, same split
    }
}

// the four products (u and v tables, both path halves); UO: the u table only
template <int KH, bool UO = false>
__device__ __forceinline__ void mma_issue(const float *Sb, int PP, int lane, const float (&b0)[KH],
                                          const float (&b1)[KH], f32x16 &du0, f32x16 &dv0, f32x16 &du1, f32x16 &dv1)
{
    const float *Au = Sb + (lane >> 5) * KH * kMmaRS + (lane & 31);
    const float *Av = Au + PP * kMmaRS;
    du0 = f32x16{}; dv0 = f32x16{}; du1 = f32x16{}; dv1 = f32x16{};
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
        const float au = Au[kk * kMmaRS];
        du0 = __builtin_amdgcn_mfma_f32_32x32x2f32(au, b0[kk], du0, 0, 0, 0);
        if constexpr (!UO) dv0 = __builtin_amdgcn_mfma_f32_32x32x2f32(Av[kk * kMmaRS], b0[kk], dv0, 0, 0, 0);
        du1 = __builtin_amdgcn_mfma_f32_32x32x2f32(au, b1[kk], du1, 0, 0, 0);
        if constexpr (!UO) dv1 = __builtin_amdgcn_mfma_f32_32x32x2f32(Av[kk * kMmaRS], b1[kk], dv1, 0, 0, 0);
    }
}

// rows back to the owning lane and the contraction with Q_{k0}(x0) (rows >= P
// of T are zero).  Registers r = 4g..4g+3 hold rows 8g..8g+3 (before the swap)
// and 8g+4..8g+7 (after it): the Legendre values in x0 advance eight at a time.
template <int KH, bool UO = false>
__device__ __forceinline__ void mma_epilogue(const f32x16 &du0, const f32x16 &dv0, const f32x16 &du1,
                                             const f32x16 &dv1, float x0, float &u, float &v)
{
    constexpr int K2 = 2 * KH;
    float su = 0.f, sv = 0.f, lp = 0.f, lc = 1.f;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if (8 * g >= K2) break;
        float Lb[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            Lb[j] = lc;
            const float nx = fmaf(x0, lc, -(float)((double)k * k / (4.0 * k * k - 1.0)) * lp);   // monic
            lp = lc;
            lc = nx;
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int r = 4 * g + rr, ia = 8 * g + rr, ib = ia + 4;
            if (ia < K2) {
                const auto pu = __builtin_amdgcn_permlane32_swap(__float_as_uint(du0[r]), __float_as_uint(du1[r]), false, false);
                su = fmaf(Lb[rr], __uint_as_float(pu[0]), su);
                if (ib < K2) su = fmaf(Lb[4 + rr], __uint_as_float(pu[1]), su);
                if constexpr (!UO) {
                    const auto pv = __builtin_amdgcn_permlane32_swap(__float_as_uint(dv0[r]), __float_as_uint(dv1[r]), false, false);
                    sv = fmaf(Lb[rr], __uint_as_float(pv[0]), sv);
                    if (ib < K2) sv = fmaf(Lb[4 + rr], __uint_as_float(pv[1]), sv);
                }
            }
        }
    }
    u = su;
    v = sv;
}

// EXT: the Picard form and the ball-point rule are compiled in (selected at
// run time by Physics); without it the residual form with the centre-point
// rule carries none of their code.
template <typename T, int D, int PMAX, int NS, int CF, bool EXT>
__device__ __forceinline__ void advance_body(const RoundArgs &a)
{
    const bool picard = EXT && a.phys.picard, ball = EXT && a.phys.ball;
    constexpr int NSTG = kMaxStageVec;
    extern __shared__ u32x4 lds[];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63;
    const int NC = a.n_chunks;
    const int64_t nvec = a.chunk_elems * (int64_t)sizeof(T) / 16;   // 16-byte vectors per chunk
    const int64_t cvec = (nvec + 1) & ~(int64_t)1;                   // LDS buffer stride in vectors
    __shared__ long long s_item;
    __shared__ SrcTime<T> s_tf[256];   // source time factors of a window of blockDim.x steps
    cptr<GroupDesc> groups = as_const(a.groups);
    cptr<NodeDesc> nodes = as_const(a.nodes);
    const int64_t total = a.batch_prefix[a.n_groups];
    unsigned long long evals = 0, slots = 0;
    using State = PathState<T, D>;
    const State *sin = (const State *)a.state_in;
    State *sout = (State *)a.state_out;

    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = (long long)atomicAdd(a.work, 1ull);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= total) break;
        // group of this work item: last g with batch_prefix[g] <= item
        int lo = 0, hi = a.n_groups - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.batch_prefix[mid] <= item) lo = mid; else hi = mid - 1;
        }
        const int g = lo;
        const int64_t b = item - a.batch_prefix[g];
        cptr<GroupDesc> G = groups + g;
        const int nstar = G->nstar;
        const int q0 = a.round * a.steps;
        const int q1 = min(q0 + a.steps, nstar);
        const T delta = (T)G->delta, J = (T)G->jump;
        const double span = G->span, t_prev = G->t_prev, ddelta = G->delta;
        const uint32_t c3 = G->c3 | (uint32_t)a.tag;
        const int64_t live = a.round == 0 ? (int64_t)G->node_count * a.mcount : (int64_t)a.live_in[g];
        const T *gtab = (const T *)a.slab_table + G->slab;

        // ---- the batch's paths
        T X[NS][D], Y[NS][D], acc[NS], comp[NS];
        bool alive[NS];
        uint32_t node[NS], sample[NS], c0[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int64_t p = b * a.batch + (int64_t)s * nthr + tid;
            alive[s] = p < live;
            node[s] = 0; sample[s] = 0; c0[s] = 0;
            acc[s] = (T)0; comp[s] = (T)0;
#pragma unroll
            for (int i = 0; i < D; ++i) X[s][i] = (T)0;
            if (alive[s]) {
                if (a.round == 0) {
                    node[s] = (uint32_t)(G->node_begin + p / a.mcount);
                    sample[s] = (uint32_t)(a.m0 + p % a.mcount);
#pragma unroll
                    for (int i = 0; i < D; ++i) X[s][i] = (T)nodes[node[s]].x0[i];
                } else {
                    const State st = sin[G->path_off + p];
#pragma unroll
                    for (int i = 0; i < D; ++i) X[s][i] = st.x[i];
                    acc[s] = st.acc;
                    comp[s] = st.comp;
                    node[s] = st.node;
                    sample[s] = st.sample;
                }
                c0[s] = nodes[node[s]].c0;
            }
        }

        // ---- source time factors of steps [q0, q0 + nthr), one per thread
        auto fill_time = [&](int qs) {
            const int qq = qs + tid;
            if (qq < q1) s_tf[tid] = source_time<T>(a.phys, (T)(t_prev + (span - (double)qq * ddelta)));
        };
        fill_time(q0);

        // ---- first chunk of the first step's slab into LDS buffer 0
        u32x4 stage[NSTG];
        {
            const u32x4 *src = (const u32x4 *)(gtab + (int64_t)q0 * a.slab_stride);
#pragma unroll
            for (int k = 0; k < NSTG; ++k) {
                const int64_t v = tid + (int64_t)k * nthr;
                if (v < nvec) lds[v] = src[v];
            }
        }
        __syncthreads();

        uint32_t w[NS][4];
        int q = q0, tslot = 0;
        for (; q < q1; ++q, ++tslot) {
            if (tslot == nthr) {   // the previous step's barrier ended every read of the old window
                tslot = 0;
                fill_time(q);
                __syncthreads();
            }
            // ---- directions (Philox words refreshed on block boundaries of the counter)
            T dir[NS][D];
            if constexpr (D == 1) {
                if ((q & 127) == 0 || q == q0) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) philox(c0[s], sample[s], (uint32_t)(q >> 7), c3, a.key0, a.key1, w[s]);
                }
                const int wi = (q >> 5) & 3, bb = q & 31;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const uint32_t word = wi == 0 ? w[s][0] : wi == 1 ? w[s][1] : wi == 2 ? w[s][2] : w[s][3];
                    dir[s][0] = ((word >> bb) & 1u) ? (T)1 : (T)-1;
                }
            } else if constexpr (D == 2) {
                if ((q & 3) == 0 || q == q0) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) philox(c0[s], sample[s], (uint32_t)(q >> 2), c3, a.key0, a.key1, w[s]);
                }
                const int wi = q & 3;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const uint32_t word = wi == 0 ? w[s][0] : wi == 1 ? w[s][1] : wi == 2 ? w[s][2] : w[s][3];
                    angle_dir(u01(word, (T)0), dir[s][0], dir[s][1]);
                }
            } else {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    uint32_t ww[8];
                    if constexpr (D <= 4) {
                        uint32_t o[4];
                        philox(c0[s], sample[s], (uint32_t)q, c3, a.key0, a.key1, o);
                        ww[0] = o[0]; ww[1] = o[1]; ww[2] = o[2]; ww[3] = o[3];
                    } else {
                        uint32_t o[4], o2[4];
                        philox(c0[s], sample[s], (uint32_t)(2 * q), c3, a.key0, a.key1, o);
                        philox(c0[s], sample[s], (uint32_t)(2 * q + 1), c3, a.key0, a.key1, o2);
                        ww[0] = o[0]; ww[1] = o[1]; ww[2] = o[2]; ww[3] = o[3];
                        ww[4] = o2[0]; ww[5] = o2[1]; ww[6] = o2[2]; ww[7] = o2[3];
                    }
                    T gg[D + 1];
#pragma unroll
                    for (int k = 0; k < (D + 1) / 2; ++k) {
                        const T r = m_sqrt((T)-2 * m_log(u01(ww[2 * k], (T)0)));
                        T c, sn;
                        angle_dir(u01(ww[2 * k + 1], (T)0), c, sn);
                        gg[2 * k] = r * c;
                        gg[2 * k + 1] = r * sn;
                    }
                    T nrm = 0;
#pragma unroll
                    for (int i = 0; i < D; ++i) nrm += gg[i] * gg[i];
                    nrm = m_sqrt(nrm);
#pragma unroll
                    for (int i = 0; i < D; ++i) dir[s][i] = gg[i] / nrm;
                }
            }
            // ---- jump and exit test (eq. indexL)
            bool any_live = false;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (alive[s]) {
                    bool inside = true;
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        Y[s][i] = m_fma(J, dir[s][i], X[s][i]);
                        inside = inside && (fabs(Y[s][i]) < (T)1);
                    }
                    if (!inside) {   // path ended: L = q
                        alive[s] = false;
                        a.result[(int64_t)nodes[node[s]].out * a.mcount + (sample[s] - a.m0)] =
                            (double)acc[s] - (double)comp[s];
                    }
                }
                any_live = any_live || alive[s];
            }
            slots += NS;
            // ---- the point where step q's integrand is evaluated: the ball centre
            // X_q (eq. interIQ) or the step's Green's-function ball point, written
            // over X (a live path moves to Y after the evaluation)
            if (ball) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (alive[s]) {
                        T off[D];
                        ball_offset<T, D>(c0[s], sample[s], q, c3, a.key0, a.key1, off);
#pragma unroll
                        for (int i = 0; i < D; ++i) X[s][i] = m_fma(J, off[i], X[s][i]);
                    }
                }
            }
            // ---- residual at X_q, time tau_q = t_{n,l} - q Delta: the slab of step q
            // streams through LDS in NC chunks (double buffered along the chunk sequence)
            const bool wave_live = __ballot(any_live) != 0ull;
            T u[NS], v[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) { u[s] = (T)0; v[s] = (T)0; }
            T Ll[NS][PMAX];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const T x = X[s][D - 1];
                Ll[s][0] = (T)1;
                if (PMAX > 1) Ll[s][1] = x;
#pragma unroll
                for (int k = 1; k + 1 < PMAX; ++k)
                    Ll[s][k + 1] = (T)((2.0 * k + 1.0) / (k + 1.0)) * x * Ll[s][k] - (T)(k / (k + 1.0)) * Ll[s][k - 1];
            }
            for (int c = 0; c < NC; ++c) {
                const int64_t tseq = (int64_t)(q - q0) * NC + c;
                const int buf = (int)(tseq & 1);
                int qn = q, cn = c + 1;
                if (cn == NC) { cn = 0; qn = q + 1; }
                const bool has_next = qn < q1;
                if (has_next) {
                    const u32x4 *src = (const u32x4 *)(gtab + (int64_t)qn * a.slab_stride + (int64_t)cn * a.chunk_elems);
#pragma unroll
                    for (int k = 0; k < NSTG; ++k) {
                        const int64_t vv = tid + (int64_t)k * nthr;
                        if (vv < nvec) stage[k] = src[vv];
                    }
                }
                if (wave_live) {
                    const T *S = (const T *)(lds + (int64_t)buf * cvec);
                    T Wc[NS];
#pragma unroll
                    for (int s = 0; s < NS; ++s) Wc[s] = (T)1;
                    if constexpr (CF > 0) {
                        // weight of the chunk: prod over the fixed dims of L_{k_i}(X_i)
                        int rem = c;
#pragma unroll
                        for (int i = CF - 1; i >= 0; --i) {
                            const int ki = rem % a.P;
                            rem /= a.P;
#pragma unroll
                            for (int s = 0; s < NS; ++s) {
                                T lp = (T)0, lc = (T)1;
                                for (int m = 0; m < ki; ++m) {
                                    const T nx = rec_a<T>(m) * X[s][i] * lc - rec_b<T>(m) * lp;
                                    lp = lc;
                                    lc = nx;
                                }
                                Wc[s] *= lc;
                            }
                        }
                    }
                    if (picard)
                        contract<T, D, PMAX, NS, CF, const T *, true>(S, a.P, a.PP, X, Wc, Ll, u, v, 0);
                    else
                        contract<T, D, PMAX, NS, CF, const T *, false>(S, a.P, a.PP, X, Wc, Ll, u, v, 0);
                }
                if (has_next) {
                    u32x4 *dst = lds + (int64_t)(buf ^ 1) * cvec;
#pragma unroll
                    for (int k = 0; k < NSTG; ++k) {
                        const int64_t vv = tid + (int64_t)k * nthr;
                        if (vv < nvec) dst[vv] = stage[k];
                    }
                }
                if (c + 1 < NC) __syncthreads();
            }
            if (wave_live) {
                const SrcTime<T> tf = s_tf[tslot];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (alive[s]) {
                        const T r = f_of<T>(a.phys, u[s]) + source_space<T, D>(a.phys, X[s], tf) +
                                    (picard ? (T)0 : v[s]);
                        const T y = delta * r;
                        if constexpr (sizeof(T) == 4) {
                            const T yc = y - comp[s];
                            const T tt = acc[s] + yc;
                            comp[s] = (tt - acc[s]) - yc;
                            acc[s] = tt;
                        } else {
                            acc[s] += y;
                        }
#pragma unroll
                        for (int i = 0; i < D; ++i) X[s][i] = Y[s][i];
                        ++evals;
                    }
                }
            }
            if (__syncthreads_or(any_live ? 1 : 0) == 0) { ++q; break; }
        }

        // ---- Picard form (eq. uast): a path still inside after all N* steps has
        // reached t_{n-1} and adds the interval's initial data u*(X_{N*}, t_{n-1}),
        // the slab of step N* (xi = -1), streamed through LDS like any step
        if (picard && q1 == nstar && q == q1) {
            bool any_live = false;
#pragma unroll
            for (int s = 0; s < NS; ++s) any_live = any_live || alive[s];
            const bool wave_live = __ballot(any_live) != 0ull;
            T Ll[NS][PMAX], u[NS], v[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const T x = X[s][D - 1];
                Ll[s][0] = (T)1;
                if (PMAX > 1) Ll[s][1] = x;
#pragma unroll
                for (int k = 1; k + 1 < PMAX; ++k)
                    Ll[s][k + 1] = (T)((2.0 * k + 1.0) / (k + 1.0)) * x * Ll[s][k] - (T)(k / (k + 1.0)) * Ll[s][k - 1];
                u[s] = (T)0;
                v[s] = (T)0;
            }
            for (int c = 0; c < NC; ++c) {
                __syncthreads();   // every read of the buffer is over
                const u32x4 *src = (const u32x4 *)(gtab + (int64_t)nstar * a.slab_stride + (int64_t)c * a.chunk_elems);
#pragma unroll
                for (int k = 0; k < NSTG; ++k) {
                    const int64_t vv = tid + (int64_t)k * nthr;
                    if (vv < nvec) lds[vv] = src[vv];
                }
                __syncthreads();
                if (wave_live) {
                    T Wc[NS];
#pragma unroll
                    for (int s = 0; s < NS; ++s) Wc[s] = (T)1;
                    if constexpr (CF > 0) {
                        int rem = c;
#pragma unroll
                        for (int i = CF - 1; i >= 0; --i) {
                            const int ki = rem % a.P;
                            rem /= a.P;
#pragma unroll
                            for (int s = 0; s < NS; ++s) {
                                T lp = (T)0, lc = (T)1;
                                for (int m = 0; m < ki; ++m) {
                                    const T nx = rec_a<T>(m) * X[s][i] * lc - rec_b<T>(m) * lp;
                                    lp = lc;
                                    lc = nx;
                                }
                                Wc[s] *= lc;
                            }
                        }
                    }
                    contract<T, D, PMAX, NS, CF, const T *, true>((const T *)lds, a.P, a.PP, X, Wc, Ll, u, v, 0);
                }
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (alive[s]) {
                    if constexpr (sizeof(T) == 4) {
                        const T yc = u[s] - comp[s];
                        const T tt = acc[s] + yc;
                        comp[s] = (tt - acc[s]) - yc;
                        acc[s] = tt;
                    } else {
                        acc[s] += u[s];
                    }
                }
            }
        }

        // ---- paths alive after the round: finished at N*, or carried to the next round
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const bool carry = alive[s] && q1 < nstar;
            if (alive[s] && !carry)
                a.result[(int64_t)nodes[node[s]].out * a.mcount + (sample[s] - a.m0)] = (double)acc[s] - (double)comp[s];
            const unsigned long long mask = __ballot(carry);
            if (mask != 0ull) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(a.live_out + g, (uint32_t)__popcll(mask));
                base = __shfl(base, 0, 64);
                if (carry) {
                    const uint32_t off = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
                    State st;
#pragma unroll
                    for (int i = 0; i < D; ++i) st.x[i] = X[s][i];
                    st.acc = acc[s];
                    st.comp = comp[s];
                    st.node = node[s];
                    st.sample = sample[s];
                    sout[G->path_off + off] = st;
                }
            }
        }
    }
    evals = wave_sum_u64(evals);
    slots = wave_sum_u64(slots);
    if (lane == 0) {
        atomicAdd(a.stats + 0, evals);
        atomicAdd(a.stats + 1, slots);
    }
}

// One-dimensional FP64 kernels with two paths per lane and up to 20 Legendre
// modes sit a few registers above the two-waves-per-SIMD budget; holding them
// to it spills five registers to scratch and still lifts the 1-D
// whole-solve throughput by a third (12.5 M -> 16.1 M node-samples/s).
template <typename T, int D, int NS, int PMAX>
constexpr int advance_min_waves() { return (sizeof(T) == 8 && D == 1 && NS == 2 && PMAX <= 20) ? 2 : 1; }

template <typename T, int D, int PMAX, int NS, int CF, bool EXT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(advance_min_waves<T, D, NS, PMAX>())))
advance_kernel(RoundArgs a)
{
    advance_body<T, D, PMAX, NS, CF, EXT>(a);
}

// ===========================================================================
// Round kernel, matrix-core form: d = 2, FP32, one path per lane, the whole
// slab of a step in LDS (its image copied straight from the table).  The step
// loop is software-pipelined so that a wave's vector work runs under its own
// products: at step q the wave issues the 4 KH products of the residual at X_q
// and meanwhile draws the direction of step q, takes the jump and the exit
// test (eq. indexL) and forms the operands of the next point; the epilogue
// then completes u and v, and the residual enters the path sum (eq. interIQ)
// only for paths whose jump stayed inside -- the same walk, exit steps and
// quadrature as the vector-unit kernel.
// ===========================================================================
// MODE bit 0: the Picard form (the u table only, the initial data at the end
// point of paths that stay inside for all N* steps); bit 1: the ball-point
// rule (the operands and the epilogue take the step's Green's-function ball
// point, drawn one step ahead like the walk's next point).
template <int KH, int MODE>
__device__ __forceinline__ void advance_mma_body(const RoundArgs &a)
{
    constexpr bool PIC = (MODE & 1) != 0, BALL = (MODE & 2) != 0;
    extern __shared__ u32x4 lds[];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63;
    __shared__ long long s_item;
    __shared__ SrcTime<float> s_tf[256];   // source time factors of a window of blockDim.x steps
    const int mbuf = 2 * a.PP * kMmaRS;   // floats per LDS buffer (slab image)
    const int mvec = mbuf / 4;            // 16-byte vectors per buffer
    cptr<GroupDesc> groups = as_const(a.groups);
    cptr<NodeDesc> nodes = as_const(a.nodes);
    const int64_t total = a.batch_prefix[a.n_groups];
    unsigned long long evals = 0, slots = 0;
    using State = PathState<float, 2>;
    const State *sin = (const State *)a.state_in;
    State *sout = (State *)a.state_out;

    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = (long long)atomicAdd(a.work, 1ull);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= total) break;
        int lo = 0, hi = a.n_groups - 1;   // last g with batch_prefix[g] <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.batch_prefix[mid] <= item) lo = mid; else hi = mid - 1;
        }
        const int g = lo;
        const int64_t b = item - a.batch_prefix[g];
        cptr<GroupDesc> G = groups + g;
        const int nstar = G->nstar;
        const int q0 = a.round * a.steps;
        const int q1 = min(q0 + a.steps, nstar);
        const float delta = (float)G->delta, J = (float)G->jump;
        const double span = G->span, t_prev = G->t_prev, ddelta = G->delta;
        const uint32_t c3 = G->c3 | (uint32_t)a.tag;
        const int64_t live = a.round == 0 ? (int64_t)G->node_count * a.mcount : (int64_t)a.live_in[g];
        const float *gtab = (const float *)a.slab_table + G->slab_mma;

        // ---- this lane's path
        const int64_t p = b * a.batch + tid;
        bool alive = p < live;
        uint32_t node = 0, sample = 0, c0 = 0;
        float x0 = 0.f, x1 = 0.f, acc = 0.f, comp = 0.f;
        if (alive) {
            if (a.round == 0) {
                node = (uint32_t)(G->node_begin + p / a.mcount);
                sample = (uint32_t)(a.m0 + p % a.mcount);
                x0 = (float)nodes[node].x0[0];
                x1 = (float)nodes[node].x0[1];
            } else {
                const State st = sin[G->path_off + p];
                x0 = st.x[0];
                x1 = st.x[1];
                acc = st.acc;
                comp = st.comp;
                node = st.node;
                sample = st.sample;
            }
            c0 = nodes[node].c0;
        }
        auto fill_time = [&](int qs) {
            const int qq = qs + tid;
            if (qq < q1) s_tf[tid] = source_time<float>(a.phys, (float)(t_prev + (span - (double)qq * ddelta)));
        };
        fill_time(q0);
        mma_stage((const u32x4 *)(gtab + (int64_t)q0 * a.slab_stride), lds, mvec, tid, nthr);
        float ex0 = x0, ex1 = x1;   // where the current step's integrand is evaluated
        if constexpr (BALL) {
            if (alive) {
                float off[2];
                ball_offset<float, 2>(c0, sample, q0, c3, a.key0, a.key1, off);
                ex0 = fmaf(J, off[0], x0);
                ex1 = fmaf(J, off[1], x1);
            }
        }
        float b0[KH], b1[KH];
        mma_operands<KH>(ex1, a.P, b0, b1);
        mma_stage_wait();
        __syncthreads();

        uint32_t w[4];
        int q = q0, tslot = 0;
        for (; q < q1; ++q, ++tslot) {
            if (tslot == nthr) {   // the previous step's barrier ended every read of the old window
                tslot = 0;
                fill_time(q);
                __syncthreads();
            }
            if ((q & 3) == 0 || q == q0) philox(c0, sample, (uint32_t)(q >> 2), c3, a.key0, a.key1, w);
            const int wi = q & 3;
            const uint32_t word = wi == 0 ? w[0] : wi == 1 ? w[1] : wi == 2 ? w[2] : w[3];
            const int buf = (q - q0) & 1;
            if (q + 1 < q1)
                mma_stage((const u32x4 *)(gtab + (int64_t)(q + 1) * a.slab_stride), lds + (buf ^ 1) * mvec, mvec, tid,
                          nthr);
            float u = 0.f, v = 0.f, y0 = x0, y1 = x1, nx0 = x0, nx1 = x1;
            bool inside = false;
            if (__ballot(alive) != 0ull) {
                f32x16 du0, dv0, du1, dv1;
                mma_issue<KH, PIC>((const float *)lds + buf * mbuf, a.PP, lane, b0, b1, du0, dv0, du1, dv1);
                // under the products: direction, jump, exit test, next operands
                float d0, d1;
                angle_dir(u01(word, 0.f), d0, d1);
                y0 = fmaf(J, d0, x0);
                y1 = fmaf(J, d1, x1);
                inside = fabsf(y0) < 1.f && fabsf(y1) < 1.f;
                nx0 = y0;
                nx1 = y1;
                if constexpr (BALL) {
                    if (alive && inside && q + 1 < q1) {
                        float off[2];
                        ball_offset<float, 2>(c0, sample, q + 1, c3, a.key0, a.key1, off);
                        nx0 = fmaf(J, off[0], y0);
                        nx1 = fmaf(J, off[1], y1);
                    }
                }
                float nb0[KH], nb1[KH];
                mma_operands<KH>(nx1, a.P, nb0, nb1);
                mma_epilogue<KH, PIC>(du0, dv0, du1, dv1, ex0, u, v);
#pragma unroll
                for (int kk = 0; kk < KH; ++kk) { b0[kk] = nb0[kk]; b1[kk] = nb1[kk]; }
            }
            ++slots;
            if (alive) {
                if (inside) {   // residual at X_q (or its ball point), time tau_q = t_{n,l} - q Delta
                    const float X[2] = {ex0, ex1};
                    const float r = f_of<float>(a.phys, u) + source_space<float, 2, !BALL>(a.phys, X, s_tf[tslot]) +
                                    (PIC ? 0.f : v);
                    const float y = delta * r;
                    const float yc = y - comp;
                    const float tt = acc + yc;
                    comp = (tt - acc) - yc;
                    acc = tt;
                    x0 = y0;
                    x1 = y1;
                    ex0 = nx0;
                    ex1 = nx1;
                    ++evals;
                } else {        // path ended: L = q
                    alive = false;
                    a.result[(int64_t)nodes[node].out * a.mcount + (sample - a.m0)] = (double)acc - (double)comp;
                }
            }
            mma_stage_wait();
            if (__syncthreads_or(alive ? 1 : 0) == 0) { ++q; break; }
        }

        // ---- Picard form (eq. uast): a path still inside after all N* steps adds
        // the interval's initial data u*(X_{N*}, t_{n-1}), the slab of step N*
        if constexpr (PIC) {
            if (q1 == nstar && q == q1) {
                __syncthreads();
                mma_stage((const u32x4 *)(gtab + (int64_t)nstar * a.slab_stride), lds, mvec, tid, nthr);
                mma_stage_wait();
                __syncthreads();
                if (__ballot(alive) != 0ull) {
                    float tb0[KH], tb1[KH];
                    mma_operands<KH>(x1, a.P, tb0, tb1);
                    f32x16 du0, dv0, du1, dv1;
                    mma_issue<KH, true>((const float *)lds, a.PP, lane, tb0, tb1, du0, dv0, du1, dv1);
                    float u = 0.f, v = 0.f;
                    mma_epilogue<KH, true>(du0, dv0, du1, dv1, x0, u, v);
                    if (alive) {
                        const float yc = u - comp;
                        const float tt = acc + yc;
                        comp = (tt - acc) - yc;
                        acc = tt;
                    }
                }
            }
        }

        // ---- paths alive after the round: finished at N*, or carried to the next round
        const bool carry = alive && q1 < nstar;
        if (alive && !carry)
            a.result[(int64_t)nodes[node].out * a.mcount + (sample - a.m0)] = (double)acc - (double)comp;
        const unsigned long long mask = __ballot(carry);
        if (mask != 0ull) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(a.live_out + g, (uint32_t)__popcll(mask));
            base = __shfl(base, 0, 64);
            if (carry) {
                const uint32_t off = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
                State st;
                st.x[0] = x0;
                st.x[1] = x1;
                st.acc = acc;
                st.comp = comp;
                st.node = node;
                st.sample = sample;
                sout[G->path_off + off] = st;
            }
        }
    }
    evals = wave_sum_u64(evals);
    slots = wave_sum_u64(slots);
    if (lane == 0) {
        atomicAdd(a.stats + 0, evals);
        atomicAdd(a.stats + 1, slots);
    }
}

template <int KH, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) advance_mma_kernel(RoundArgs a)
{
    advance_mma_body<KH, MODE>(a);
}

template <typename T, int D, int PMAX, int NS>
static hipError_t adv_cf(const RoundArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    // chunking options per dimension: whole slab or one fixed dimension for d <= 3,
    // two or three fixed dimensions for d = 4, 5
    constexpr int C0 = D <= 3 ? 0 : D - 3;
    constexpr int C1 = D <= 1 ? 0 : (D <= 3 ? 1 : D - 2);
    // the Picard form and the ball-point rule run one sample per lane
    if (a.phys.picard || a.phys.ball) {
        if constexpr (NS == 1) {
            if (a.cf == C0) { hipLaunchKernelGGL((advance_kernel<T, D, PMAX, NS, C0, true>), grid, block, lds, s, a); return hipGetLastError(); }
            if (a.cf == C1) { hipLaunchKernelGGL((advance_kernel<T, D, PMAX, NS, C1, true>), grid, block, lds, s, a); return hipGetLastError(); }
        }
        return hipErrorInvalidValue;
    }
    if (a.cf == C0) { hipLaunchKernelGGL((advance_kernel<T, D, PMAX, NS, C0, false>), grid, block, lds, s, a); return hipGetLastError(); }
    if (a.cf == C1) { hipLaunchKernelGGL((advance_kernel<T, D, PMAX, NS, C1, false>), grid, block, lds, s, a); return hipGetLastError(); }
    return hipErrorInvalidValue;
}

template <typename T, int D, int PMAX>
static hipError_t adv_ns(const RoundArgs &a, int ns, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    switch (ns) {
    case 1: return adv_cf<T, D, PMAX, 1>(a, grid, block, lds, s);
    case 2: return adv_cf<T, D, PMAX, 2>(a, grid, block, lds, s);
    case 4:
        if constexpr (D <= 2) return adv_cf<T, D, PMAX, 4>(a, grid, block, lds, s);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int D>
static hipError_t adv_p(const RoundArgs &a, int ns, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    if (a.P <= 12) return adv_ns<T, D, 12>(a, ns, grid, block, lds, s);
    if constexpr (D <= 4) {
        if (a.P <= 20) return adv_ns<T, D, 20>(a, ns, grid, block, lds, s);
    }
    if constexpr (D <= 3) {
        if (a.P <= 28) return adv_ns<T, D, 28>(a, ns, grid, block, lds, s);
        if (a.P <= 36) return adv_ns<T, D, 36>(a, ns, grid, block, lds, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t adv_d(const RoundArgs &a, int ns, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    switch (a.phys.dim) {
    case 1: return adv_p<T, 1>(a, ns, grid, block, lds, s);
    case 2: return adv_p<T, 2>(a, ns, grid, block, lds, s);
    case 3: return adv_p<T, 3>(a, ns, grid, block, lds, s);
    case 4: return adv_p<T, 4>(a, ns, grid, block, lds, s);
    case 5: return adv_p<T, 5>(a, ns, grid, block, lds, s);
    }
    return hipErrorInvalidValue;
}

template <int KH, int MODE>
static hipError_t adv_mma(const RoundArgs &a, int kh, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    if constexpr (KH > 16) {
        return hipErrorInvalidValue;
    } else {
        if (kh != KH) return adv_mma<KH + 1, MODE>(a, kh, grid, block, lds, s);
        hipLaunchKernelGGL((advance_mma_kernel<KH, MODE>), grid, block, lds, s, a);
        return hipGetLastError();
    }
}

bool advance_mma_eligible(int fp32, int dim, int P, int cf, int samples_per_lane, int waves_per_block)
{
    return fp32 && dim == 2 && P >= 3 && P <= 32 && cf == 0 && samples_per_lane == 1 && waves_per_block >= 1 &&
           waves_per_block <= 4;
}

size_t advance_mma_lds_bytes(int PP) { return (size_t)2 * 2 * PP * kMmaRS * sizeof(float); }

// ===========================================================================
// Round kernel, fractional form (Ex. 2-3): d = 1, u_t = -(-Delta)^{alpha/2} u
// + f(u) + s, one path per lane.  The walk jumps by J = R / sqrt(x) with
// x = I^{-1}(omega; alpha/2, 1 - alpha/2) (the exit law of a ball of radius R
// for the alpha-stable process started at its centre; the mean exit time of
// that ball is Delta), in a fair direction.  The slab of a step holds the
// symmetric Jacobi coefficients (parameter a = alpha/2) of u*/w and of
// -d_t u*/w, w = (1 - x^2)^a, and the residual is
//   r = f(w U) + s + w V - sum_k lambda_k U_k P_k,  lambda_k = Gamma(k+alpha+1)/k!
// (the fractional Laplacian of the generalized Jacobi function w P_k).
// Philox: block q/2, words 2(q mod 2) (omega) and 2(q mod 2) + 1 (sign bit).
// ===========================================================================

// log x solving I_x(p, 1-p) = y for x <= 1/2: Newton on log x with the series
// I_x = x^p (1-x)^{1-p} / (p B) sum_k t_k, t_{k+1} = t_k x (k+1)/(p+1+k)
// (ratios rt[k] from the block's LDS copy of the table), started from the
// small-x asymptote.  FP64: 6 iterations of 60 terms; FP32: 4 of 26.
template <typename T> struct FracIters { static constexpr int nit = sizeof(T) == 8 ? 6 : 4, nt = sizeof(T) == 8 ? 60 : 26; };

template <typename T>
__device__ __forceinline__ T ibeta_inv_log(T y, T p, T lpb, const T *rt)
{
    constexpr int NIT = FracIters<T>::nit, NT = FracIters<T>::nt;
    const T lhalf = (T)-0.69314718055994530942;
    const T ly = m_log(y);
    T z = (ly + lpb) / p;
    z = z < lhalf ? z : lhalf;
    for (int it = 0; it < NIT; ++it) {
        const T x = m_exp(z);
        T S = (T)1, t = (T)1;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            t *= x * rt[k];
            S += t;
        }
        const T l1 = sizeof(T) == 8 ? (T)log1p((double)-x) : (T)log1pf((float)-x);
        const T lI = p * z + ((T)1 - p) * l1 - lpb + m_log(S);
        z = z - (lI - ly) * ((T)1 - x) * S / p;
        z = z < lhalf ? z : lhalf;
    }
    return z;
}

// one Newton solve per lane whichever half of (0,1) omega falls in (no
// divergent second solve): x <= 1/2 solves I_x(a, 1-a) = omega for log x;
// otherwise z = 1 - x solves I_z(1-a, a) = 1 - omega for log z
template <typename T>
__device__ __forceinline__ T frac_jump(const Physics &ph, T R, T om, const T *ra, const T *rb)
{
    const T a = (T)ph.frac_a;
    const bool lower = om <= (T)ph.frac_half;
    const T z = ibeta_inv_log<T>(lower ? om : (T)1 - om, lower ? a : (T)1 - a,
                                 lower ? (T)ph.frac_lpb1 : (T)ph.frac_lpb2, lower ? ra : rb);
    return lower ? R * m_exp((T)-0.5 * z) : R / m_sqrt((T)1 - m_exp(z));
}

template <typename T>
__global__ void __launch_bounds__(256) frac_advance_kernel(RoundArgs a)
{
    extern __shared__ u32x4 lds[];
    const int tid = threadIdx.x, lane = tid & 63;
    __shared__ long long s_item;
    const Physics &ph = a.phys;
    const int P = a.P, PP = a.PP, K = ph.frac_K, kmax = ph.frac_kmax;
    const int nv = 2 * PP * (int)sizeof(T) / 16;   // 16-byte vectors per slab
    const int cv = (nv + 1) & ~1;
    // the tables, in the sampling precision, after the two slab buffers
    T *tl = (T *)(lds + 2 * cv);
    const int ntab = 2 * kmax + P + K + 2 * ph.frac_nt;
    for (int i = tid; i < ntab; i += blockDim.x) tl[i] = (T)ph.frac_tab[i];
    const T *tA = tl, *tC = tl + kmax, *tlam = tl + 2 * kmax, *tsrc = tlam + P, *ra = tsrc + K, *rb = ra + ph.frac_nt;
    cptr<GroupDesc> groups = as_const(a.groups);
    cptr<NodeDesc> nodes = as_const(a.nodes);
    const int64_t total = a.batch_prefix[a.n_groups];
    unsigned long long evals = 0, slots = 0;
    using State = PathState<T, 1>;
    const State *sin = (const State *)a.state_in;
    State *sout = (State *)a.state_out;
    const T fa = (T)ph.frac_a;

    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = (long long)atomicAdd(a.work, 1ull);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= total) break;
        int lo = 0, hi = a.n_groups - 1;   // last g with batch_prefix[g] <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.batch_prefix[mid] <= item) lo = mid; else hi = mid - 1;
        }
        const int g = lo;
        const int64_t b = item - a.batch_prefix[g];
        cptr<GroupDesc> G = groups + g;
        const int nstar = G->nstar;
        const int q0 = a.round * a.steps;
        const int q1 = min(q0 + a.steps, nstar);
        const T delta = (T)G->delta, R = (T)G->jump;
        const double span = G->span, t_prev = G->t_prev, ddelta = G->delta;
        const uint32_t c3 = G->c3 | (uint32_t)a.tag;
        const int64_t live = a.round == 0 ? (int64_t)G->node_count * a.mcount : (int64_t)a.live_in[g];
        const T *gtab = (const T *)a.slab_table + G->slab;

        T X = (T)0, acc = (T)0, comp = (T)0;
        uint32_t node = 0, sample = 0, c0 = 0;
        const int64_t p = b * a.batch + tid;
        bool alive = p < live;
        if (alive) {
            if (a.round == 0) {
                node = (uint32_t)(G->node_begin + p / a.mcount);
                sample = (uint32_t)(a.m0 + p % a.mcount);
                X = (T)nodes[node].x0[0];
            } else {
                const State st = sin[G->path_off + p];
                X = st.x[0];
                acc = st.acc;
                comp = st.comp;
                node = st.node;
                sample = st.sample;
            }
            c0 = nodes[node].c0;
        }
        // the slab of the first step into buffer 0
        {
            const u32x4 *src = (const u32x4 *)(gtab + (int64_t)q0 * a.slab_stride);
            if (tid < nv) lds[tid] = src[tid];
        }
        __syncthreads();

        uint32_t w[4] = {0u, 0u, 0u, 0u};
        int q = q0;
        for (; q < q1; ++q) {
            const int buf = (q - q0) & 1;
            if (q + 1 < q1 && tid < nv)
                lds[(buf ^ 1) * cv + tid] = ((const u32x4 *)(gtab + (int64_t)(q + 1) * a.slab_stride))[tid];
            bool any_live = false;
            if (alive) {
                if ((q & 1) == 0 || q == q0) philox(c0, sample, (uint32_t)(q >> 1), c3, a.key0, a.key1, w);
                const uint32_t wo = (q & 1) ? w[2] : w[0], ws = (q & 1) ? w[3] : w[1];
                const T J = frac_jump<T>(ph, R, u01(wo, (T)0), ra, rb);
                const T Y = m_fma(J, (ws & 1u) ? (T)1 : (T)-1, X);
                if (!(fabs(Y) < (T)1)) {   // path ended: L = q
                    alive = false;
                    a.result[(int64_t)nodes[node].out * a.mcount + (sample - a.m0)] = (double)acc - (double)comp;
                } else {
                    // ---- residual at X_q, tau_q = t_{n,l} - q Delta
                    const T *S = (const T *)(lds + buf * cv);
                    const T wgt = m_exp(fa * m_log(((T)1 - X) * ((T)1 + X)));
                    T pm = (T)0, pc = (T)1, uj = (T)0, vj = (T)0, F = (T)0, Gs = (T)0;
#pragma unroll 4
                    for (int k = 0; k < kmax; ++k) {
                        if (k < P) {
                            uj = m_fma(S[k], pc, uj);
                            vj = m_fma(S[PP + k], pc, vj);
                            F = m_fma((T)tlam[k] * S[k], pc, F);
                        }
                        if (k < K) Gs = m_fma((T)tsrc[k], pc, Gs);
                        const T pn = (T)tA[k] * X * pc - (T)tC[k] * pm;
                        pm = pc;
                        pc = pn;
                    }
                    // manufactured source s = w g T' + T (-Delta)^{alpha/2}(w g) - f(w g T)
                    T src = (T)0;
                    if (ph.src_kind >= 5) {
                        const T tau = (T)(t_prev + (span - (double)q * ddelta));
                        T gx, Tt, Tp;
                        if (ph.src_kind == 5) {
                            gx = m_sin(X);
                            const T qq = (T)1 + tau * tau;
                            Tt = m_exp(m_cos(tau)) / qq;
                            Tp = Tt * (-m_sin(tau) - (T)2 * tau / qq);
                        } else if (ph.src_kind == 6) {
                            gx = m_cos(X * X * X + (T)1) / ((T)10 * X * X + (T)1);
                            const T rho = (T)ph.src_param[0];
                            Tt = m_exp(rho * m_log(tau));
                            Tp = rho * Tt / tau;
                        } else {
                            gx = (T)ph.src_param[0] + X * ((T)ph.src_param[1] + X * (T)ph.src_param[2]);
                            Tt = (T)1 + (T)ph.src_param[3] * tau;
                            Tp = (T)ph.src_param[3];
                        }
                        src = wgt * gx * Tp + Gs * Tt - f_of<T>(ph, wgt * gx * Tt);
                    }
                    // Picard form (eq. uast): the integrand f(u*) + s only
                    const T r = ph.picard ? f_of<T>(ph, wgt * uj) + src : f_of<T>(ph, wgt * uj) + src + wgt * vj - F;
                    const T y = delta * r;
                    if constexpr (sizeof(T) == 4) {
                        const T yc = y - comp;
                        const T tt = acc + yc;
                        comp = (tt - acc) - yc;
                        acc = tt;
                    } else {
                        acc += y;
                    }
                    X = Y;
                    ++evals;
                    any_live = true;
                }
            }
            ++slots;
            if (__syncthreads_or(any_live ? 1 : 0) == 0) { ++q; break; }
        }

        // ---- Picard form (eq. uast): a path still inside after all N* steps adds
        // the interval's initial data u*(X_{N*}, t_{n-1}), the slab of step N*
        if (ph.picard && q1 == nstar && q == q1) {
            __syncthreads();
            if (tid < nv) lds[tid] = ((const u32x4 *)(gtab + (int64_t)nstar * a.slab_stride))[tid];
            __syncthreads();
            if (alive) {
                const T *S = (const T *)lds;
                T pm = (T)0, pc = (T)1, uj = (T)0;
                for (int k = 0; k < P; ++k) {
                    uj = m_fma(S[k], pc, uj);
                    const T pn = tA[k] * X * pc - tC[k] * pm;
                    pm = pc;
                    pc = pn;
                }
                const T y = m_exp(fa * m_log(((T)1 - X) * ((T)1 + X))) * uj;
                if constexpr (sizeof(T) == 4) {
                    const T yc = y - comp;
                    const T tt = acc + yc;
                    comp = (tt - acc) - yc;
                    acc = tt;
                } else {
                    acc += y;
                }
            }
        }

        // ---- paths alive after the round: finished at N*, or carried to the next round
        const bool carry = alive && q1 < nstar;
        if (alive && !carry)
            a.result[(int64_t)nodes[node].out * a.mcount + (sample - a.m0)] = (double)acc - (double)comp;
        const unsigned long long mask = __ballot(carry);
        if (mask != 0ull) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(a.live_out + g, (uint32_t)__popcll(mask));
            base = __shfl(base, 0, 64);
            if (carry) {
                const uint32_t off = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
                State st;
                st.x[0] = X;
                st.acc = acc;
                st.comp = comp;
                st.node = node;
                st.sample = sample;
                sout[G->path_off + off] = st;
            }
        }
    }
    evals = wave_sum_u64(evals);
    slots = wave_sum_u64(slots);
    if (lane == 0) {
        atomicAdd(a.stats + 0, evals);
        atomicAdd(a.stats + 1, slots);
    }
}

// dynamic LDS of the fractional round kernel: two slab buffers and the tables
size_t frac_lds_bytes(int fp32, int PP, int kmax, int P, int K, int nt)
{
    const int nv = 2 * PP * (fp32 ? 4 : 8) / 16, cv = (nv + 1) & ~1;
    return (size_t)2 * cv * 16 + (size_t)(2 * kmax + P + K + 2 * nt) * (fp32 ? 4 : 8);
}

hipError_t launch_advance(const RoundArgs &a, int fp32, int samples_per_lane, int waves_per_block, int blocks,
                          size_t lds_bytes, int mma, hipStream_t s)
{
    dim3 block(64 * waves_per_block), grid(blocks);
    if (a.phys.frac) {
        const int nt = fp32 ? FracIters<float>::nt : FracIters<double>::nt;
        if (a.phys.dim != 1 || a.batch != (int)block.x || a.P > a.PP || 2 * a.PP * (fp32 ? 4 : 8) / 16 > (int)block.x ||
            a.phys.frac_nt != nt || lds_bytes < frac_lds_bytes(fp32, a.PP, a.phys.frac_kmax, a.P, a.phys.frac_K, nt))
            return hipErrorInvalidValue;
        if (fp32)
            hipLaunchKernelGGL(frac_advance_kernel<float>, grid, block, lds_bytes, s, a);
        else
            hipLaunchKernelGGL(frac_advance_kernel<double>, grid, block, lds_bytes, s, a);
        return hipGetLastError();
    }
    if (mma) {
        if (!advance_mma_eligible(fp32, a.phys.dim, a.P, a.cf, samples_per_lane, waves_per_block))
            return hipErrorInvalidValue;
        switch ((a.phys.picard ? 1 : 0) | (a.phys.ball ? 2 : 0)) {
        case 0: return adv_mma<2, 0>(a, (a.P + 1) / 2, grid, block, lds_bytes, s);
        case 1: return adv_mma<2, 1>(a, (a.P + 1) / 2, grid, block, lds_bytes, s);
        case 2: return adv_mma<2, 2>(a, (a.P + 1) / 2, grid, block, lds_bytes, s);
        default: return adv_mma<2, 3>(a, (a.P + 1) / 2, grid, block, lds_bytes, s);
        }
    }
    return fp32 ? adv_d<float>(a, samples_per_lane, grid, block, lds_bytes, s)
                : adv_d<double>(a, samples_per_lane, grid, block, lds_bytes, s);
}

// sums[out][0..1] (+)= sum over the slice's samples of S and S^2, in sample order
__global__ void slice_reduce_kernel(const double *__restrict__ result, int64_t n_nodes, int64_t mcount,
                                    double *__restrict__ sums, int first)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    const double *r = result + i * mcount;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t k = 0; k < mcount; ++k) { s1 += r[k]; s2 += r[k] * r[k]; }
    if (first) { sums[2 * i] = s1; sums[2 * i + 1] = s2; }
    else { sums[2 * i] += s1; sums[2 * i + 1] += s2; }
}

hipError_t launch_slice_reduce(const double *result, int64_t n_nodes, int64_t mcount, double *sums, int first,
                               hipStream_t s)
{
    if (n_nodes <= 0) return hipSuccess;
    hipLaunchKernelGGL(slice_reduce_kernel, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, s, result, n_nodes,
                       mcount, sums, first);
    return hipGetLastError();
}


// ===========================================================================
// Adjoint of the residual estimator under common random numbers.
//
// For iteration k the estimator is eps_node = (1/M) sum_paths sum_{q<L}
// Delta r(X_q, tau_q), with r = f(u*) + s + v* and u*, v* linear in the
// slabs of step q.  With a nodal adjoint lambda (the adjoint of eps), the
// adjoint of the slab of group g at step q is
//   Sbar^u_{g,q}[k] = sum_paths (lambda_node Delta/M) f'(u*(X_q)) Psi_k(X_q),
//   Sbar^v_{g,q}[k] = sum_paths (lambda_node Delta/M) Psi_k(X_q),
// Psi_k(X) = prod_i L_{k_i}(X_i).  The kernel regenerates the forward paths
// (same Philox counters, same arithmetic) and, per step, accumulates the sum
// of the block's weighted outer products Psi = L(X_0) (x) L(X_1) into the
// slab-adjoint table: on the matrix cores (FP32, v_mfma_f32_32x32x2f32 with
// the samples as the reduction dimension) or on the vector units.
// ===========================================================================
typedef float f32x16 __attribute__((ext_vector_type(16)));

size_t adjoint_lds_bytes(int fp32, int mfma, int dim, int P, int nthr, int64_t slab_stride)
{
    const size_t T = fp32 ? 4 : 8;
    const int64_t nvec = slab_stride * (int64_t)T / 16;
    const size_t slab = (size_t)2 * ((nvec + 1) & ~1LL) * 16;
    if (mfma) return slab + (size_t)nthr * (2 * (P | 1) + 2) * 4 + 2 * 32 * 32 * 4;
    const int R = dim == 1 ? 1 : P;
    const int RS = (std::max(R, P) + 3) & ~3;
    return slab + (size_t)nthr * 3 * RS * T;
}

template <typename T, int D, int PMAX, bool MFMA>
__global__ void __launch_bounds__(256) adjoint_kernel(AdjointArgs aa)
{
    const RoundArgs &a = aa.r;
    extern __shared__ u32x4 lds[];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int64_t nvec = a.slab_stride * (int64_t)sizeof(T) / 16;
    const int64_t svec = (nvec + 1) & ~(int64_t)1;
    const int P = a.P, PP = a.PP;
    const int R = D == 1 ? 1 : P;
    // vector path: weighted rows Au, Av and columns Bm per sample (stride RS);
    // matrix-core path: basis rows Am and columns Bm (odd stride PS, so that a
    // wave's row writes fall in distinct banks) and the two
    // weights Wm per sample, the upper half's tiles gsum [2][16][64]
    const int RS = MFMA ? P : (((R > P ? R : P) + 3) & ~3);
    T *Au = (T *)(lds + 2 * svec);
    T *Av = Au + (int64_t)nthr * RS;
    T *Bm = Av + (int64_t)nthr * RS;
    const int PS = P | 1;
    float *Am = (float *)(lds + 2 * svec);
    float *Bmm = Am + (int64_t)nthr * PS;
    float *Wm = Bmm + (int64_t)nthr * PS;
    float *gsum = MFMA ? Wm + 2 * (int64_t)nthr : nullptr;
    __shared__ long long s_item;
    cptr<GroupDesc> groups = as_const(a.groups);
    cptr<NodeDesc> nodes = as_const(a.nodes);
    const int64_t total = a.batch_prefix[a.n_groups];
    using State = PathState<T, D>;
    const State *sin = (const State *)a.state_in;
    State *sout = (State *)a.state_out;
    T *sbar = (T *)aa.slab_bar;
    const int E = 2 * R * P;

    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = (long long)atomicAdd(a.work, 1ull);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= total) break;
        int lo = 0, hi = a.n_groups - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.batch_prefix[mid] <= item) lo = mid; else hi = mid - 1;
        }
        const int g = lo;
        const int64_t b = item - a.batch_prefix[g];
        cptr<GroupDesc> G = groups + g;
        const int nstar = G->nstar;
        const int q0 = a.round * a.steps;
        const int q1 = min(q0 + a.steps, nstar);
        const T J = (T)G->jump;
        const double ddelta = G->delta;
        const uint32_t c3 = G->c3 | (uint32_t)a.tag;
        const int64_t live = a.round == 0 ? (int64_t)G->node_count * a.mcount : (int64_t)a.live_in[g];
        const T *gtab = (const T *)a.slab_table + G->slab;
        T *gbar = sbar + G->slab;

        T X[1][D], Y[1][D], acc[1], comp[1];
        bool alive;
        uint32_t node = 0, sample = 0, c0 = 0;
        T lam = (T)0;
        {
            const int64_t p = b * a.batch + tid;
            alive = p < live;
            acc[0] = (T)0; comp[0] = (T)0;
#pragma unroll
            for (int i = 0; i < D; ++i) X[0][i] = (T)0;
            if (alive) {
                if (a.round == 0) {
                    node = (uint32_t)(G->node_begin + p / a.mcount);
                    sample = (uint32_t)(a.m0 + p % a.mcount);
#pragma unroll
                    for (int i = 0; i < D; ++i) X[0][i] = (T)nodes[node].x0[i];
                } else {
                    const State st = sin[G->path_off + p];
#pragma unroll
                    for (int i = 0; i < D; ++i) X[0][i] = st.x[i];
                    node = st.node;
                    sample = st.sample;
                }
                c0 = nodes[node].c0;
                lam = (T)(aa.lambda[nodes[node].u_index] * ddelta * aa.inv_M);
            }
        }
        u32x4 stage[kMaxStageVec];
        {
            const u32x4 *src = (const u32x4 *)(gtab + (int64_t)q0 * a.slab_stride);
#pragma unroll
            for (int k = 0; k < kMaxStageVec; ++k) {
                const int64_t v = tid + (int64_t)k * nthr;
                if (v < nvec) lds[v] = src[v];
            }
        }
        __syncthreads();

        uint32_t w[1][4];
        for (int q = q0; q < q1; ++q) {
            const int buf = (q - q0) & 1;
            if (q + 1 < q1) {
                const u32x4 *src = (const u32x4 *)(gtab + (int64_t)(q + 1) * a.slab_stride);
#pragma unroll
                for (int k = 0; k < kMaxStageVec; ++k) {
                    const int64_t v = tid + (int64_t)k * nthr;
                    if (v < nvec) stage[k] = src[v];
                }
            }
            T dir[1][D];
            if constexpr (D == 1) {
                if ((q & 127) == 0 || q == q0) philox(c0, sample, (uint32_t)(q >> 7), c3, a.key0, a.key1, w[0]);
                const int wi = (q >> 5) & 3, bb = q & 31;
                const uint32_t word = wi == 0 ? w[0][0] : wi == 1 ? w[0][1] : wi == 2 ? w[0][2] : w[0][3];
                dir[0][0] = ((word >> bb) & 1u) ? (T)1 : (T)-1;
            } else {
                if ((q & 3) == 0 || q == q0) philox(c0, sample, (uint32_t)(q >> 2), c3, a.key0, a.key1, w[0]);
                const int wi = q & 3;
                const uint32_t word = wi == 0 ? w[0][0] : wi == 1 ? w[0][1] : wi == 2 ? w[0][2] : w[0][3];
                angle_dir(u01(word, (T)0), dir[0][0], dir[0][1]);
            }
            if (alive) {
                bool inside = true;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    Y[0][i] = m_fma(J, dir[0][i], X[0][i]);
                    inside = inside && (fabs(Y[0][i]) < (T)1);
                }
                alive = inside;
            }
            // ---- weights of this evaluation: lambda Delta/M f'(u*(X_q)) and lambda Delta/M
            T wu = (T)0, wv = (T)0;
            const T *S = (const T *)(lds + (int64_t)buf * svec);
            T Ll[1][PMAX];
            {
                const T x = X[0][D - 1];
                Ll[0][0] = (T)1;
                if (PMAX > 1) Ll[0][1] = x;
#pragma unroll
                for (int k = 1; k + 1 < PMAX; ++k)
                    Ll[0][k + 1] = (T)((2.0 * k + 1.0) / (k + 1.0)) * x * Ll[0][k] - (T)(k / (k + 1.0)) * Ll[0][k - 1];
            }
            if (__ballot(alive) != 0ull) {
                T u[1], v[1], W1[1];
                u[0] = (T)0; v[0] = (T)0; W1[0] = (T)1;
                contract<T, D, PMAX, 1, 0, const T *>(S, P, PP, X, W1, Ll, u, v, 0);
                if (alive) {
                    wv = lam;
                    wu = lam * fprime_of<T>(a.phys, u[0]);
                }
            }
            // ---- outer-product factors of this sample: rows L(X_0) weighted, columns L(X_{d-1})
            if constexpr (MFMA) {
                float *am = Am + (int64_t)tid * PS, *bm = Bmm + (int64_t)tid * PS;
                Wm[2 * tid] = wu;
                Wm[2 * tid + 1] = wv;
                if constexpr (D == 1) {
                    for (int i = 0; i < P; ++i) am[i] = i == 0 ? 1.f : 0.f;
                } else {
                    float lp = 0.f, lc = 1.f;
                    const float x0 = X[0][0];
                    for (int i = 0; i < P; ++i) {
                        am[i] = lc;
                        const float nx = rec_a<float>(i) * x0 * lc - rec_b<float>(i) * lp;
                        lp = lc;
                        lc = nx;
                    }
                }
#pragma unroll
                for (int j = 0; j < PMAX; ++j)
                    if (j < P) bm[j] = Ll[0][j];
            } else {
                T *au = Au + (int64_t)tid * RS, *av = Av + (int64_t)tid * RS, *bm = Bm + (int64_t)tid * RS;
                if constexpr (D == 1) {
                    for (int i = 0; i < RS; ++i) { au[i] = i == 0 ? wu : (T)0; av[i] = i == 0 ? wv : (T)0; }
                } else {
                    T lp = (T)0, lc = (T)1;
                    const T x0 = X[0][0];
                    for (int i = 0; i < RS; ++i) {
                        const bool in = i < P;
                        au[i] = in ? wu * lc : (T)0;
                        av[i] = in ? wv * lc : (T)0;
                        const T nx = rec_a<T>(i < kMaxP ? i : 0) * x0 * lc - rec_b<T>(i < kMaxP ? i : 0) * lp;
                        lp = lc;
                        lc = nx;
                    }
                }
#pragma unroll
                for (int j = 0; j < PMAX; ++j)
                    if (j < RS) bm[j] = j < P ? Ll[0][j] : (T)0;
                for (int j = PMAX; j < RS; ++j) bm[j] = (T)0;
            }
            if (alive) {
#pragma unroll
                for (int i = 0; i < D; ++i) X[0][i] = Y[0][i];
            }
            if (q + 1 < q1) {
                u32x4 *dst = lds + (int64_t)(buf ^ 1) * svec;
#pragma unroll
                for (int k = 0; k < kMaxStageVec; ++k) {
                    const int64_t v = tid + (int64_t)k * nthr;
                    if (v < nvec) dst[v] = stage[k];
                }
            }
            __syncthreads();
            // ---- block sum of the outer products into the slab adjoint of step q
            T *dstq = gbar + (int64_t)q * a.slab_stride;
            if constexpr (MFMA) {
                // wave w forms tile w & 1 (0: the f'(u)-weighted table, 1: the
                // plain one) over half w >> 1 of the block's samples, two samples
                // per product; the upper half hands its tile to the lower one
                // through LDS with plain stores, which then adds into the table
                // operand rows and columns i >= P read the next sample's factors
                // (inside the LDS block): they only reach output rows or columns
                // >= P, which are not written out
                const int tile = wave & 1, half = wave >> 1, i = lane & 31;
                constexpr int hs = 128;   // the matrix-core form runs four waves per block
                f32x16 c = {};
#pragma unroll 4
                for (int kk = 0; kk < hs / 2; ++kk) {
                    const int sidx = half * hs + 2 * kk + (lane >> 5);
                    const float am = Am[sidx * PS + i], bb = Bmm[sidx * PS + i];
                    c = __builtin_amdgcn_mfma_f32_32x32x2f32(Wm[2 * sidx + tile] * am, bb, c, 0, 0, 0);
                }
                float *cm = gsum + tile * 16 * 64 + lane;
                if (half == 1) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) cm[r * 64] = c[r];
                }
                // past this barrier no wave reads this step's factors again, and
                // the upper half writes its next tile only after the next step's
                // first barrier: it also closes the step
                const int any_alive = __syncthreads_or(alive ? 1 : 0);
                if (half == 0) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int ii = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                        const float val = c[r] + cm[r * 64];
                        if (ii < R && i < P && val != 0.f)
                            atomicAdd(dstq + (int64_t)ii * 2 * PP + tile * PP + i, (T)val);
                    }
                }
                if (any_alive == 0) break;
            } else {
                for (int e = tid; e < E; e += nthr) {
                    const int uv = e / (R * P), rem = e - uv * R * P, ii = rem / P, jj = rem - ii * P;
                    const T *A = uv ? Av : Au;
                    T sum = (T)0;
                    for (int sidx = 0; sidx < nthr; ++sidx) sum = m_fma(A[sidx * RS + ii], Bm[sidx * RS + jj], sum);
                    if (sum != (T)0) atomicAdd(dstq + (int64_t)ii * 2 * PP + uv * PP + jj, sum);
                }
                if (__syncthreads_or(alive ? 1 : 0) == 0) break;
            }
        }
        // survivors to the next round
        {
            const bool carry = alive && q1 < nstar;
            const unsigned long long mask = __ballot(carry);
            if (mask != 0ull) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(a.live_out + g, (uint32_t)__popcll(mask));
                base = __shfl(base, 0, 64);
                if (carry) {
                    const uint32_t off = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
                    State st;
#pragma unroll
                    for (int i = 0; i < D; ++i) st.x[i] = X[0][i];
                    st.acc = (T)0;
                    st.comp = (T)0;
                    st.node = node;
                    st.sample = sample;
                    sout[G->path_off + off] = st;
                }
            }
        }
    }
}

template <typename T, int D, int PMAX>
static hipError_t adj_mfma(const AdjointArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    if constexpr (sizeof(T) == 4) {
        if (a.use_mfma) { hipLaunchKernelGGL((adjoint_kernel<T, D, PMAX, true>), grid, block, lds, s, a); return hipGetLastError(); }
    }
    hipLaunchKernelGGL((adjoint_kernel<T, D, PMAX, false>), grid, block, lds, s, a);
    return hipGetLastError();
}

template <typename T, int D>
static hipError_t adj_p(const AdjointArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    if (a.r.P <= 12) return adj_mfma<T, D, 12>(a, grid, block, lds, s);
    if (a.r.P <= 20) return adj_mfma<T, D, 20>(a, grid, block, lds, s);
    if (a.r.P <= 28) return adj_mfma<T, D, 28>(a, grid, block, lds, s);
    if (a.r.P <= 32) return adj_mfma<T, D, 32>(a, grid, block, lds, s);
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint(const AdjointArgs &a, int fp32, int waves_per_block, int blocks, size_t lds_bytes,
                          hipStream_t s)
{
    dim3 block(64 * waves_per_block), grid(blocks);
    if (a.r.phys.dim == 1) return fp32 ? adj_p<float, 1>(a, grid, block, lds_bytes, s) : adj_p<double, 1>(a, grid, block, lds_bytes, s);
    if (a.r.phys.dim == 2) return fp32 ? adj_p<float, 2>(a, grid, block, lds_bytes, s) : adj_p<double, 2>(a, grid, block, lds_bytes, s);
    return hipErrorInvalidValue;
}

// Transpose of the slab kernel: cbar[inst][k][q'] = sum over the instance's
// node times l and steps q of Sbar_{g,q}[k] L_{q'}(xi_{l,q}).
template <typename T>
__global__ void slab_adjoint_kernel(SlabArgs a, int32_t groups_per_inst, int32_t n_inst, double *__restrict__ cbar_u,
                                    double *__restrict__ cbar_v, int64_t coef_inst_stride)
{
    const int64_t psp = (int64_t)a.rows * a.P;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_inst * 2 * psp) return;
    const int inst = (int)(idx / (2 * psp));
    const int64_t rem = idx - (int64_t)inst * 2 * psp;
    const int uv = (int)(rem / psp);
    const int64_t k = rem - uv * psp;
    const int64_t row = k / a.P;
    const int kl = (int)(k - row * a.P);
    const T *tab = (const T *)a.slab_table;
    double accq[kMaxDeg + 1];
    const int T1 = a.deg[inst * groups_per_inst] + 1;
#pragma unroll
    for (int m = 0; m <= kMaxDeg; ++m) accq[m] = 0.0;
    for (int gl = 0; gl < groups_per_inst; ++gl) {
        const int g = inst * groups_per_inst + gl;
        const int nstar = a.nstar[g];
        const double span = a.span[g], delta = a.delta[g], h2 = a.h2[g];
        const T *src = tab + a.slab_off[g] + row * 2 * a.PP + uv * a.PP + kl;
        for (int q = 0; q < nstar; ++q) {
            const double val = (double)src[(int64_t)q * a.slab_stride];
            if (val == 0.0) continue;
            const double xi = h2 * (span - (double)q * delta) - 1.0;
            double lp = 0.0, lc = 1.0;
            // fully unrolled with a guard so that accq stays in registers
#pragma unroll
            for (int m = 0; m <= kMaxDeg; ++m) {
                if (m < T1) {
                    accq[m] = fma(val, lc, accq[m]);
                    const double nx = c_rec.ad[m] * xi * lc - c_rec.bd[m] * lp;
                    lp = lc;
                    lc = nx;
                }
            }
        }
    }
    double *out = (uv ? cbar_v : cbar_u) + (int64_t)inst * coef_inst_stride + k * T1;
#pragma unroll
    for (int m = 0; m <= kMaxDeg; ++m)
        if (m < T1) out[m] = accq[m];
}

hipError_t launch_slab_adjoint(const SlabArgs &a, int32_t groups_per_inst, int32_t n_inst, int fp32, double *cbar_u,
                               double *cbar_v, int64_t coef_inst_stride, hipStream_t s)
{
    const int64_t n = (int64_t)n_inst * 2 * a.rows * a.P;
    dim3 grid((unsigned)((n + 127) / 128)), block(128);
    if (fp32)
        hipLaunchKernelGGL(slab_adjoint_kernel<float>, grid, block, 0, s, a, groups_per_inst, n_inst, cbar_u, cbar_v, coef_inst_stride);
    else
        hipLaunchKernelGGL(slab_adjoint_kernel<double>, grid, block, 0, s, a, groups_per_inst, n_inst, cbar_u, cbar_v, coef_inst_stride);
    return hipGetLastError();
}

// loss[inst] = 1/2 sum_j (U[inst][j][T1-1] - target[inst][j])^2 (fixed-order
// block tree) and the terminal nodal adjoint lambda[inst][j][T1-1] = residual.
__global__ void loss_lambda_kernel(const double *__restrict__ U, const double *__restrict__ target, int64_t nsp, int T1,
                                   double *__restrict__ lambda, double *__restrict__ loss)
{
    const int inst = blockIdx.x;
    __shared__ double sm[256];
    double part = 0.0;
    for (int64_t j = threadIdx.x; j < nsp; j += blockDim.x) {
        const int64_t r = (int64_t)inst * nsp + j;
        const double e = U[r * T1 + T1 - 1] - target[r];
        lambda[r * T1 + T1 - 1] = e;
        part += 0.5 * e * e;
    }
    sm[threadIdx.x] = part;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[inst] = sm[0];
}

hipError_t launch_loss_lambda(const double *U, const double *target, int n_inst, int64_t nsp, int T1, double *lambda,
                              double *loss, hipStream_t s)
{
    hipLaunchKernelGGL(loss_lambda_kernel, dim3(n_inst), dim3(256), 0, s, U, target, nsp, T1, lambda, loss);
    return hipGetLastError();
}

__global__ void column_sum_kernel(const double *__restrict__ lambda, int64_t rows, int T1, double *__restrict__ out)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= rows) return;
    double s = 0.0;
    for (int l = 0; l < T1; ++l) s += lambda[r * T1 + l];
    out[r] = s;
}

hipError_t launch_column_sum(const double *lambda, int64_t rows, int T1, double *out, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(column_sum_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, lambda, rows, T1, out);
    return hipGetLastError();
}

__global__ void axpy_kernel(double *__restrict__ y, const double *__restrict__ x, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] += x[i];
}

hipError_t launch_axpy(double *y, const double *x, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, x, n);
    return hipGetLastError();
}

}  // namespace hpsmc
