// One-dimensional round kernel (vector units, FP64 or FP32): the residual form
// with the centre-point rule, the path-advancing step of eq. varepsilon_1 on a
// line, where a step's slab is only the 2 P coefficients of u* and v* at the
// step's time.
#include "hpsmc_device.h"

namespace hpsmc {

// ===========================================================================
// The general round kernel stages one step's slab per barrier and holds the
// Legendre values of every mode in registers; on a line the slab is a few
// hundred bytes and the per-step work is the walk itself, so both costs
// dominate.  Here a block copies the slabs of a window of k1dWin steps into
// LDS at once (straight from the table, double buffered: the next window
// lands while the current one is walked), computes the window's source time
// factors one per thread, and meets at a barrier once per window.  The rows
// hold the coefficients of u* and v* in the Chebyshev basis (converted from
// the Legendre tensors by one mode product per table before the time
// contraction), whose recurrence T_{k+1} = 2x T_k - T_{k-1} has constant
// coefficients: one fma per basis value, run interleaved with the two dot
// products, so a path keeps two basis values instead of P.  The walk (Philox
// words, +-J jumps, the exit test of eq. indexL) and the residual (eq.
// interIQ) are those of the general kernel.
// ===========================================================================
constexpr int k1dWin = 32;

template <typename T, int NS, int PM>
__device__ __forceinline__ void advance_1d_body(const RoundArgs &a)
{
    extern __shared__ u32x4 lds[];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63;
    __shared__ long long s_item;
    __shared__ SrcTime<T> s_tf[2][k1dWin];
    const int64_t sstride = a.slab_stride;                       // elements per step: [u: PP][v: PP]
    const int wvec = (int)(k1dWin * sstride * (int64_t)sizeof(T) / 16);   // 16-byte vectors per window buffer
    cptr<GroupDesc> groups = as_const(a.groups);
    cptr<NodeDesc> nodes = as_const(a.nodes);
    const int64_t total = a.batch_prefix[a.n_groups];
    unsigned long long evals = 0, slots = 0;
    using State = PathState<T, 1>;
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
        const T delta = (T)G->delta, J = (T)G->jump;
        const double span = G->span, t_prev = G->t_prev, ddelta = G->delta;
        const uint32_t c3 = G->c3 | (uint32_t)a.tag;
        const int64_t live = a.round == 0 ? (int64_t)G->node_count * a.mcount : (int64_t)a.live_in[g];
        const T *gtab = (const T *)a.slab_table + G->slab;

        // ---- the batch's paths
        T X[NS], acc[NS], comp[NS];
        bool alive[NS];
        uint32_t node[NS], sample[NS], c0[NS], w[NS][4], bits[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int64_t p = b * a.batch + (int64_t)s * nthr + tid;
            alive[s] = p < live;
            node[s] = 0; sample[s] = 0; c0[s] = 0;
            X[s] = (T)0; acc[s] = (T)0; comp[s] = (T)0;
            if (alive[s]) {
                if (a.round == 0) {
                    node[s] = (uint32_t)(G->node_begin + p / a.mcount);
                    sample[s] = (uint32_t)(a.m0 + p % a.mcount);
                    X[s] = (T)nodes[node[s]].x0[0];
                } else {
                    const State st = sin[G->path_off + p];
                    X[s] = st.x[0];
                    acc[s] = st.acc;
                    comp[s] = st.comp;
                    node[s] = st.node;
                    sample[s] = st.sample;
                }
                c0[s] = nodes[node[s]].c0;
            }
        }

        // ---- window [qw, qe) of steps into LDS buffer wb: the slabs (contiguous in
        // the table) by direct global -> LDS copies, the source time factors one per thread
        auto stage = [&](int qw, int wb) {
            const int n = min(k1dWin, q1 - qw);
            mma_stage((const u32x4 *)(gtab + (int64_t)qw * sstride), lds + wb * wvec,
                      (int)(n * sstride * (int64_t)sizeof(T) / 16), tid, nthr);
            if (tid < n)
                s_tf[wb][tid] = source_time<T>(a.phys, (T)(t_prev + (span - (double)(qw + tid) * ddelta)));
        };
        stage(q0, 0);
        mma_stage_wait();
        __syncthreads();

        int q = q0, wb = 0;
#pragma unroll 1
        for (int qw = q0; qw < q1; qw += k1dWin, wb ^= 1) {
            const int qe = min(qw + k1dWin, q1);
            if (qe < q1) stage(qe, wb ^ 1);   // the other buffer: its last readers passed the previous barrier
            const T *Sw = (const T *)(lds + wb * wvec);
            bool any_live = false;
#pragma unroll 1
            for (q = qw; q < qe; ++q) {
                // ---- directions: bit q % 32 of word (q / 32) % 4 of the Philox block
                // q / 128 (the general kernel's counter layout), read by shifting
                // the current word one bit per step
                if ((q & 127) == 0 || q == q0) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) philox(c0[s], sample[s], (uint32_t)(q >> 7), c3, a.key0, a.key1, w[s]);
                }
                if ((q & 31) == 0 || q == q0) {
                    const int wi = (q >> 5) & 3;
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        bits[s] = (wi == 0 ? w[s][0] : wi == 1 ? w[s][1] : wi == 2 ? w[s][2] : w[s][3]) >> (q & 31);
                }
                T Y[NS];
                any_live = false;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const T dir = (bits[s] & 1u) ? (T)1 : (T)-1;
                    bits[s] >>= 1;
                    Y[s] = m_fma(J, dir, X[s]);
                    if (alive[s] && !(fabs(Y[s]) < (T)1)) {   // path ended: L = q
                        alive[s] = false;
                        a.result[(int64_t)nodes[node[s]].out * a.mcount + (sample[s] - a.m0)] =
                            (double)acc[s] - (double)comp[s];
                    }
                    any_live = any_live || alive[s];
                }
                slots += NS;
                if (__ballot(any_live) == 0ull) continue;
                // ---- residual at X_q, time tau_q = t_{n,l} - q Delta: u*, v* by the
                // Chebyshev recurrence, each value entering both sums as it is formed
                const T *S = Sw + (int64_t)(q - qw) * sstride;
                T tu[NS], tv[NS], lp[NS], lc[NS], x2[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    tu[s] = (T)0; tv[s] = (T)0; lp[s] = (T)1; lc[s] = X[s]; x2[s] = X[s] + X[s];
                }
                typedef T v4 __attribute__((ext_vector_type(4)));
#pragma unroll
                for (int kb = 0; kb < PM / 4; ++kb) {
                    if (kb * 4 < a.P) {
                        const v4 qu = *(const v4 *)(S + 4 * kb), qv = *(const v4 *)(S + a.PP + 4 * kb);
                        const T cu[4] = {qu.x, qu.y, qu.z, qu.w}, cv[4] = {qv.x, qv.y, qv.z, qv.w};
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const int k = 4 * kb + c;   // mode of this term
#pragma unroll
                            for (int s = 0; s < NS; ++s) {
                                // T_k: 1, x, then 2x T_{k-1} - T_{k-2}
                                T Lk;
                                if (k == 0) Lk = (T)1;
                                else if (k == 1) Lk = X[s];
                                else {
                                    Lk = m_fma(x2[s], lc[s], -lp[s]);
                                    lp[s] = lc[s];
                                    lc[s] = Lk;
                                }
                                tu[s] = m_fma(cu[c], Lk, tu[s]);
                                tv[s] = m_fma(cv[c], Lk, tv[s]);
                            }
                        }
                    }
                }
                const SrcTime<T> tf = s_tf[wb][q - qw];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (alive[s]) {
                        const T u = m_fma((T)1, tu[s], (T)0), v = m_fma((T)1, tv[s], (T)0);
                        const T Xs[1] = {X[s]};
                        const T r = f_of<T>(a.phys, u) + source_space<T, 1>(a.phys, Xs, tf) + v;
                        const T y = delta * r;
                        if constexpr (sizeof(T) == 4) {
                            const T yc = y - comp[s];
                            const T tt = acc[s] + yc;
                            comp[s] = (tt - acc[s]) - yc;
                            acc[s] = tt;
                        } else {
                            acc[s] += y;
                        }
                        X[s] = Y[s];
                        ++evals;
                    }
                }
            }
            mma_stage_wait();   // the next window's slabs have landed
            if (__syncthreads_or(any_live ? 1 : 0) == 0) { q = qe; break; }
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
                    st.x[0] = X[s];
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

template <typename T, int NS, int PM>
__global__ void __launch_bounds__(256) advance_1d_kernel(RoundArgs a)
{
    advance_1d_body<T, NS, PM>(a);
}

template <typename T, int NS>
static hipError_t adv_1d_p(const RoundArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    if (a.P <= 12) hipLaunchKernelGGL((advance_1d_kernel<T, NS, 12>), grid, block, lds, s, a);
    else if (a.P <= 20) hipLaunchKernelGGL((advance_1d_kernel<T, NS, 20>), grid, block, lds, s, a);
    else if (a.P <= 36) hipLaunchKernelGGL((advance_1d_kernel<T, NS, 36>), grid, block, lds, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
static hipError_t adv_1d_t(const RoundArgs &a, int ns, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    switch (ns) {
    case 1: return adv_1d_p<T, 1>(a, grid, block, lds, s);
    case 2: return adv_1d_p<T, 2>(a, grid, block, lds, s);
    case 4: return adv_1d_p<T, 4>(a, grid, block, lds, s);
    }
    return hipErrorInvalidValue;
}

bool advance_1d_eligible(int dim, int P, int picard, int ball, int frac, int samples_per_lane)
{
    return dim == 1 && P >= 1 && P <= 36 && !picard && !ball && !frac &&
           (samples_per_lane == 1 || samples_per_lane == 2 || samples_per_lane == 4);
}

size_t advance_1d_lds_bytes(int fp32, int64_t slab_stride)
{
    return (size_t)2 * k1dWin * (size_t)slab_stride * (fp32 ? 4 : 8);
}

hipError_t launch_adv_1d(const RoundArgs &a, int fp32, int ns, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    if (a.slab_stride * (fp32 ? 4 : 8) % 16 != 0) return hipErrorInvalidValue;   // whole 16-byte vectors per step
    return fp32 ? adv_1d_t<float>(a, ns, grid, block, lds, s) : adv_1d_t<double>(a, ns, grid, block, lds, s);
}

}  // namespace hpsmc
