// Fractional form of the round kernel (Ex. 2-3, d = 1).
#include "hpsmc_device.h"

namespace hpsmc {

hipError_t set_rec_tables_frac() { return upload_recurrence_tables(); }

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
// (ratios rt[k] from the block's LDS copy of the table).  The small-x
// asymptote z0 = (log y + log(p B)) / p gives X0 = e^{z0}; the solution is
// x = X0 e^{-h(x)/p}, h(x) = (1-p) log(1-x) + log sum_k t_k, an analytic
// function of X0 on [0, X0max] (X0max the asymptote at x = 1/2), so the start
// is z0 plus log(x / X0) interpolated linearly in a table of kFracTab
// intervals (the host runs the same Newton to convergence at each grid
// point); from there one Newton step (FP32: 26 terms, FP64: 60) reaches the
// iteration's fixed point to rounding.
template <typename T> struct FracIters { static constexpr int nit = 1, nt = sizeof(T) == 8 ? 60 : 26; };

template <typename T>
__device__ __forceinline__ T ibeta_inv_log(T y, T p, T lpb, const T *rt, const T *dtab, T x0max)
{
    constexpr int NIT = FracIters<T>::nit, NT = FracIters<T>::nt;
    const T lhalf = (T)-0.69314718055994530942;
    const T ly = m_log(y);
    const T z0 = (ly + lpb) / p;
    const T f = m_exp(z0) * ((T)kFracTab / x0max);
    T z = lhalf;
    if (f < (T)kFracTab) {
        const int i = (int)f;
        const T w = f - (T)i;
        z = z0 + m_fma(w, dtab[i + 1] - dtab[i], dtab[i]);
    }
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
// otherwise z = 1 - x solves I_z(1-a, a) = 1 - omega for log z.  The start
// tables follow the series ratios: [ra | rb | da | db | X0max_a, X0max_b].
template <typename T>
__device__ __forceinline__ T frac_jump(const Physics &ph, T R, T om, const T *ra, const T *rb)
{
    const T a = (T)ph.frac_a;
    const bool lower = om <= (T)ph.frac_half;
    const T *da = rb + ph.frac_nt, *db = da + kFracTab + 1, *xm = db + kFracTab + 1;
    const T z = ibeta_inv_log<T>(lower ? om : (T)1 - om, lower ? a : (T)1 - a,
                                 lower ? (T)ph.frac_lpb1 : (T)ph.frac_lpb2, lower ? ra : rb, lower ? da : db,
                                 lower ? xm[0] : xm[1]);
    return lower ? R * m_exp((T)-0.5 * z) : R / m_sqrt((T)1 - m_exp(z));
}

template <typename T>
__global__ void __launch_bounds__(256) frac_advance_kernel(RoundArgs a)
{
    extern __shared__ u32x4 lds[];
    const int tid = threadIdx.x, lane = tid & 63, nthr = blockDim.x;
    __shared__ long long s_item;
    __shared__ T s_tt[256], s_tp[256];   // source time factors of a window of blockDim.x steps
    const Physics &ph = a.phys;
    const int P = a.P, PP = a.PP, K = ph.frac_K, kmax = ph.frac_kmax;
    const int nv = 2 * PP * (int)sizeof(T) / 16;   // 16-byte vectors per slab
    const int cv = (nv + 1) & ~1;
    // the tables, in the sampling precision, after the two slab buffers
    T *tl = (T *)(lds + 2 * cv);
    const int ntab = 2 * kmax + P + K + 2 * ph.frac_nt + 2 * (kFracTab + 1) + 2;
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
        // time factors T(tau_q), T'(tau_q) of the manufactured source for a window
        // of blockDim.x steps (the same for every lane of the item), one step a thread
        auto fill_time = [&](int qs) {
            const int qq = qs + tid;
            if (ph.src_kind < 5 || qq >= q1) return;
            const T tau = (T)(t_prev + (span - (double)qq * ddelta));
            T Tt, Tp;
            if (ph.src_kind == 5) {
                const T qd = (T)1 + tau * tau;
                Tt = m_exp(m_cos(tau)) / qd;
                Tp = Tt * (-m_sin(tau) - (T)2 * tau / qd);
            } else if (ph.src_kind == 6) {
                const T rho = (T)ph.src_param[0];
                Tt = m_exp(rho * m_log(tau));
                Tp = rho * Tt / tau;
            } else {
                Tt = (T)1 + (T)ph.src_param[3] * tau;
                Tp = (T)ph.src_param[3];
            }
            s_tt[tid] = Tt;
            s_tp[tid] = Tp;
        };
        fill_time(q0);
        // the slab of the first step into buffer 0
        {
            const u32x4 *src = (const u32x4 *)(gtab + (int64_t)q0 * a.slab_stride);
            if (tid < nv) lds[tid] = src[tid];
        }
        __syncthreads();

        uint32_t w[4] = {0u, 0u, 0u, 0u};
        int q = q0, tslot = 0;
        for (; q < q1; ++q, ++tslot) {
            if (tslot == nthr) {   // the previous step's barrier ended every read of the old window
                tslot = 0;
                fill_time(q);
                __syncthreads();
            }
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
                    // manufactured source s = w g T' + T (-Delta)^{alpha/2}(w g) - f(w g T),
                    // the step's time factors T, T' from the block's window table
                    T src = (T)0;
                    if (ph.src_kind >= 5) {
                        const T Tt = s_tt[tslot], Tp = s_tp[tslot];
                        T gx;
                        if (ph.src_kind == 5)
                            gx = m_sin(X);
                        else if (ph.src_kind == 6)
                            gx = m_cos(X * X * X + (T)1) / ((T)10 * X * X + (T)1);
                        else
                            gx = (T)ph.src_param[0] + X * ((T)ph.src_param[1] + X * (T)ph.src_param[2]);
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
    return (size_t)2 * cv * 16 + (size_t)(2 * kmax + P + K + 2 * nt + 2 * (kFracTab + 1) + 2) * (fp32 ? 4 : 8);
}

hipError_t launch_adv_frac(const RoundArgs &a, int fp32, dim3 grid, dim3 block, size_t lds_bytes, hipStream_t s)
{
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

}  // namespace hpsmc
