// The vector-unit round kernel of the path-advancing step (advance_kernel)
// and its dispatch over dimension, mode tier, samples per lane and LDS
// chunking; instantiated once per sampling precision (hpsmc_kern_valu_f32.hip,
// hpsmc_kern_valu_f64.hip).
#pragma once
#include "hpsmc_device.h"

namespace hpsmc {

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
                for (int s = 0; s < NS; ++s) sphere_dir<T, D>(c0[s], sample[s], q, c3, a.key0, a.key1, dir[s]);
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

}  // namespace hpsmc
