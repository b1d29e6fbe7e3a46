// Matrix-core form of the 2-D FP32 round kernel (v_mfma_f32_32x32x2f32).
#include "hpsmc_device.h"

namespace hpsmc {

hipError_t set_rec_tables_mma() { return upload_recurrence_tables(); }

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

hipError_t launch_adv_mma(const RoundArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    switch ((a.phys.picard ? 1 : 0) | (a.phys.ball ? 2 : 0)) {
    case 0: return adv_mma<2, 0>(a, (a.P + 1) / 2, grid, block, lds, s);
    case 1: return adv_mma<2, 1>(a, (a.P + 1) / 2, grid, block, lds, s);
    case 2: return adv_mma<2, 2>(a, (a.P + 1) / 2, grid, block, lds, s);
    default: return adv_mma<2, 3>(a, (a.P + 1) / 2, grid, block, lds, s);
    }
}

}  // namespace hpsmc
