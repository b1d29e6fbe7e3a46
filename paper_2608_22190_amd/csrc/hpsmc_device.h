// Device-side helpers shared by the gfx950 kernel translation units of the
// spectral Monte Carlo hot path (arXiv 2608.22190): the Legendre recurrence
// tables, math in the sampling precision, Philox4x32-10, the jump direction and
// ball point of a walk step, the problem terms, the tensor-product Legendre
// contraction, the path state of the round kernels and the matrix-core
// operand helpers.  Not part of the C ABI.
#pragma once
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
};
// every translation unit holds its own copy, uploaded by its own setter
static __constant__ RecTable c_rec;

static hipError_t upload_recurrence_tables()
{
    RecTable t;
    for (int k = 0; k < kMaxP + 2; ++k) {
        t.ad[k] = (2.0 * k + 1.0) / (k + 1.0);
        t.bd[k] = double(k) / (k + 1.0);
        t.af[k] = float(t.ad[k]);
        t.bf[k] = float(t.bd[k]);
    }
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
__device__ __forceinline__ void m_sincos(double x, double &s, double &c) { sincos(x, &s, &c); }
__device__ __forceinline__ void m_sincos(float x, float &s, float &c) { sincosf(x, &s, &c); }
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

// ---------------------------------------------------------------------------
// sin(pi y) and cos(pi y), branch-free, for |y| < 2^30: y = n/2 + f with
// n = rint(2y), so |f| <= 1/4 and f = y - n/2 is exact; the Maclaurin series of
// sin(pi f) and cos(pi f) (|pi f| <= pi/4), truncated where the next term is
// below 1e-17 (FP64: through f^17 and f^16) or 2e-9 (FP32: through f^9 and
// f^10); then n quarter turns.  Coefficients (-1)^k pi^(2k+1)/(2k+1)! and
// (-1)^k pi^(2k)/(2k)!, rounded from 60-digit values.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincospi_series(double y, double &s, double &c)
{
    const double n = rint(y + y);
    const double f = fma(n, -0.5, y);
    const double z = f * f;
    double ps = 0x1.aaec32af93359p-21;
    ps = fma(ps, z, -0x1.6fadb9f155744p-16);
    ps = fma(ps, z, 0x1.e8f434d018d63p-12);
    ps = fma(ps, z, -0x1.e3074fde8871fp-8);
    ps = fma(ps, z, 0x1.50783487ee782p-4);
    ps = fma(ps, z, -0x1.32d2cce62bd86p-1);
    ps = fma(ps, z, 0x1.466bc6775aae2p+1);
    ps = fma(ps, z, -0x1.4abbce625be53p+2);
    ps = fma(ps, z, 0x1.921fb54442d18p+1);
    double pc = 0x1.20c62c2f2d7f5p-18;
    pc = fma(pc, z, -0x1.b6e24f44b128fp-14);
    pc = fma(pc, z, 0x1.f9d38a3763cc3p-10);
    pc = fma(pc, z, -0x1.a6d1f2a204a8cp-6);
    pc = fma(pc, z, 0x1.e1f506891babbp-3);
    pc = fma(pc, z, -0x1.55d3c7e3cbffap+0);
    pc = fma(pc, z, 0x1.03c1f081b5ac4p+2);
    pc = fma(pc, z, -0x1.3bd3cc9be45dep+2);
    const double sn = ps * f, cs = fma(pc, z, 1.0);
    const int q = (int)n;
    const double a = (q & 1) ? cs : sn, b = (q & 1) ? sn : cs;
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}
__device__ __forceinline__ void sincospi_series(float y, float &s, float &c)
{
    const float n = rintf(y + y);
    const float f = fmaf(n, -0.5f, y);
    const float z = f * f;
    float ps = (float)0x1.50783487ee782p-4;
    ps = fmaf(ps, z, (float)-0x1.32d2cce62bd86p-1);
    ps = fmaf(ps, z, (float)0x1.466bc6775aae2p+1);
    ps = fmaf(ps, z, (float)-0x1.4abbce625be53p+2);
    ps = fmaf(ps, z, (float)0x1.921fb54442d18p+1);
    float pc = (float)-0x1.a6d1f2a204a8cp-6;
    pc = fmaf(pc, z, (float)0x1.e1f506891babbp-3);
    pc = fmaf(pc, z, (float)-0x1.55d3c7e3cbffap+0);
    pc = fmaf(pc, z, (float)0x1.03c1f081b5ac4p+2);
    pc = fmaf(pc, z, (float)-0x1.3bd3cc9be45dep+2);
    const float sn = ps * f, cs = fmaf(pc, z, 1.0f);
    const int q = (int)n;
    const float a = (q & 1) ? cs : sn, b = (q & 1) ? sn : cs;
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}

// direction (cos, sin) of the angle 2*pi*u, u in (0, 1)
template <typename T> __device__ __forceinline__ void angle_dir(T u, T &c, T &s) { sincospi_series(u + u, s, c); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 S-box with
// multipliers D2511F53 / CD9E8D57 and Weyl key steps 9E3779B9 / BB67AE85.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1, uint32_t (&o)[4])
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32 x 32 -> 64-bit product in one v_mad_u64_u32 (not a mul_hi and a mul_lo)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        c0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        c1 = (uint32_t)p1;
        c2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c3 = (uint32_t)p0;
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
// Uniform direction on the unit sphere of R^D, D >= 3, for walk step q
// (Lemma 2.1): Philox blocks q (D <= 4) or 2q and 2q + 1 (D = 5), Box-Muller
// pairs of words (2k, 2k + 1), the first D normals normalised.
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void sphere_dir(uint32_t c0, uint32_t c1, int q, uint32_t c3, uint32_t k0, uint32_t k1,
                                           T (&dir)[D])
{
    static_assert(D >= 3 && D <= 5, "Gaussian directions for d = 3..5");
    uint32_t ww[8];
    if constexpr (D <= 4) {
        uint32_t o[4];
        philox(c0, c1, (uint32_t)q, c3, k0, k1, o);
        ww[0] = o[0]; ww[1] = o[1]; ww[2] = o[2]; ww[3] = o[3];
    } else {
        uint32_t o[4], o2[4];
        philox(c0, c1, (uint32_t)(2 * q), c3, k0, k1, o);
        philox(c0, c1, (uint32_t)(2 * q + 1), c3, k0, k1, o2);
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
    for (int i = 0; i < D; ++i) dir[i] = gg[i] / nrm;
}

// ---------------------------------------------------------------------------
// Problem terms.
// ---------------------------------------------------------------------------
// sin(u) for the nonlinearity: arguments with |u| <= 2 take the sine's
// Maclaurin series, no range reduction (FP32 to u^17/17!, truncation below
// 4e-10; FP64 to u^27/27!, below 1e-20), larger ones the library sine
__device__ __forceinline__ double sin_of_u(double u)
{
    if (fabs(u) <= 2.0) {
        const double z = u * u;
        double p = 1.0 / 10888869450418352160768000000.0;   // +1/27!
        p = fma(p, z, -1.0 / 15511210043330985984000000.0);  // -1/25!
        p = fma(p, z, 1.0 / 25852016738884976640000.0);      // +1/23!
        p = fma(p, z, -1.0 / 51090942171709440000.0);        // -1/21!
        p = fma(p, z, 1.0 / 121645100408832000.0);           // +1/19!
        p = fma(p, z, -1.0 / 355687428096000.0);             // -1/17!
        p = fma(p, z, 1.0 / 1307674368000.0);                // +1/15!
        p = fma(p, z, -1.0 / 6227020800.0);                  // -1/13!
        p = fma(p, z, 1.0 / 39916800.0);                     // +1/11!
        p = fma(p, z, -1.0 / 362880.0);                      // -1/9!
        p = fma(p, z, 1.0 / 5040.0);                         // +1/7!
        p = fma(p, z, -1.0 / 120.0);                         // -1/5!
        p = fma(p, z, 1.0 / 6.0);                            // +1/3!
        return fma(-p * z, u, u);
    }
    return sin(u);
}
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

// The two sine kinds share one call: with a call in each case the compiler
// hoists the sine's common range reduction above the switch, and every kind
// pays for it at every walk step.
template <typename T>
__device__ __forceinline__ T f_of(const Physics &ph, T u)
{
    switch (ph.f_kind) {
    case 0: return (T)ph.f_param[0] * u + (T)ph.f_param[1];
    case 1: return u - u * u * u;
    case 2:
    case 5: {
        const T sn = sin_of_u(u);
        return ph.f_kind == 2 ? sn : u * sn;
    }
    case 3: return u * u / ((T)1 + u * u);
    case 4: return -u * u * u;
    }
    return (T)0;
}

template <typename T>
__device__ __forceinline__ T fprime_of(const Physics &ph, T u)
{
    switch (ph.f_kind) {
    case 0: return (T)ph.f_param[0];
    case 1: return (T)1 - (T)3 * u * u;
    case 2:
    case 5: {   // one sine-cosine call for both kinds (as in f_of)
        T sn, cs;
        m_sincos(u, sn, cs);
        return ph.f_kind == 2 ? cs : sn + u * cs;
    }
    case 3: { T a = (T)1 + u * u; return (T)2 * u / (a * a); }
    case 4: return (T)-3 * u * u;
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
        for (int i = 0; i < D; ++i) {   // sin(pi x)
            T sn, cs;
            sincospi_series(X[i], sn, cs);
            p *= sn;
        }
        u = p; ut = -p; lap = -(T)D * pi * pi * p;
        break;
    }
    case 2: {
        T p = tf.a;
#pragma unroll
        for (int i = 0; i < D; ++i) {   // cos(pi x / 2)
            T sn, cs;
            sincospi_series((T)0.5 * X[i], sn, cs);
            p *= cs;
        }
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
        else   // |sig| <= d: sin and cos of pi (sig / pi)
            sincospi_series(sig * (T)0.31830988618379067154, S, C);
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
// The image holds coefficients in the Chebyshev basis T_{k0} T_{k1} (converted
// from the Legendre tensors on the host side), whose recurrence T_{k+1} =
// 2x T_k - T_{k-1} has constant coefficients: one fma per basis value.
// ---------------------------------------------------------------------------

// B operands: Chebyshev values T_{k1}(x1) of the wave's 64 points
template <int KH>
__device__ __forceinline__ void mma_operands(float x1, int P, float (&b0)[KH], float (&b1)[KH])
{
    static_assert(KH >= 2 && KH <= 16, "one 32-row tile, at least 4 modes");
    constexpr int K2 = 2 * KH;
    float L[K2];
    const float x2 = x1 + x1;
    L[0] = 1.f;
    L[1] = x1;
#pragma unroll
    for (int k = 1; k + 1 < K2; ++k) L[k + 1] = fmaf(x2, L[k], -L[k - 1]);
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

// rows back to the owning lane and the contraction with T_{k0}(x0) (rows >= P
// of T are zero).  Registers r = 4g..4g+3 hold rows 8g..8g+3 (before the swap)
// and 8g+4..8g+7 (after it): the Chebyshev values in x0 advance eight at a time.
template <int KH, bool UO = false>
__device__ __forceinline__ void mma_epilogue(const f32x16 &du0, const f32x16 &dv0, const f32x16 &du1,
                                             const f32x16 &dv1, float x0, float &u, float &v)
{
    constexpr int K2 = 2 * KH;
    const float x02 = x0 + x0;
    float su = 0.f, sv = 0.f, lp = 0.f, lc = 1.f;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if (8 * g >= K2) break;
        float Lb[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            Lb[j] = lc;
            const float nx = k == 0 ? x0 : fmaf(x02, lc, -lp);   // T_1 = x, T_{k+1} = 2x T_k - T_{k-1}
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

// per-unit launchers of the round kernels (hpsmc_kern_*.hip)
hipError_t launch_adv_valu_f32(const RoundArgs &a, int ns, dim3 grid, dim3 block, size_t lds, hipStream_t s);
hipError_t launch_adv_valu_f64(const RoundArgs &a, int ns, dim3 grid, dim3 block, size_t lds, hipStream_t s);
hipError_t launch_adv_mma(const RoundArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s);
hipError_t launch_adv_mma5(const RoundArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s);
hipError_t launch_adv_frac(const RoundArgs &a, int fp32, dim3 grid, dim3 block, size_t lds, hipStream_t s);
hipError_t launch_adv_1d(const RoundArgs &a, int fp32, int ns, dim3 grid, dim3 block, size_t lds, hipStream_t s);
// each unit's copy of the recurrence tables
hipError_t set_rec_tables_main();
hipError_t set_rec_tables_valu_f32();
hipError_t set_rec_tables_valu_f64();
hipError_t set_rec_tables_mma();
hipError_t set_rec_tables_mma5();
hipError_t set_rec_tables_frac();
hipError_t set_rec_tables_adjoint();

}  // namespace hpsmc
