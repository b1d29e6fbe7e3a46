// Adjoint of the residual estimator (gradient with respect to the initial data).
#include "hpsmc_device.h"

namespace hpsmc {

hipError_t set_rec_tables_adjoint() { return upload_recurrence_tables(); }

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
size_t adjoint_lds_bytes(int fp32, int mfma, int dim, int P, int nthr, int64_t slab_stride)
{
    const size_t T = fp32 ? 4 : 8;
    const int64_t nvec = slab_stride * (int64_t)T / 16;
    const size_t slab = (size_t)2 * ((nvec + 1) & ~1LL) * 16;
    if (mfma) return slab + ((size_t)2 * P * (nthr + 4) + 2 * nthr) * 4 + 2 * 32 * 32 * 4;
    const int R = dim == 1 ? 1 : P;
    const int RS = (std::max(R, P) + 3) & ~3;
    return slab + (size_t)nthr * 3 * RS * T;
}

template <typename T, int D, int PMAX, bool MFMA>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MFMA ? 3 : 1))) adjoint_kernel(AdjointArgs aa)
{
    const RoundArgs &a = aa.r;
    extern __shared__ u32x4 lds[];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int64_t nvec = a.slab_stride * (int64_t)sizeof(T) / 16;
    const int64_t svec = (nvec + 1) & ~(int64_t)1;
    const int P = a.P, PP = a.PP;
    const int R = D == 1 ? 1 : P;
    // vector path: weighted rows Au, Av and columns Bm per sample (stride RS);
    // matrix-core path: the basis values L_i(x_0) (Am) and L_j(x_{d-1}) (Bm)
    // as [i][sample] tables of row stride NST = nthr + 4 (rows start four banks
    // apart, so the 16-byte reads of a half-wave, one row per lane, are free of
    // bank conflicts), the two weights Wm [2][sample], and the upper half's
    // tiles gsum [2][16][64]
    const int RS = MFMA ? P : (((R > P ? R : P) + 3) & ~3);
    T *Au = (T *)(lds + 2 * svec);
    T *Av = Au + (int64_t)nthr * RS;
    T *Bm = Av + (int64_t)nthr * RS;
    const int NST = nthr + 4;
    float *Am = (float *)(lds + 2 * svec);
    float *Bmm = Am + (int64_t)P * NST;
    float *Wm = Bmm + (int64_t)P * NST;
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
                Wm[tid] = wu;
                Wm[nthr + tid] = wv;
                if constexpr (D == 1) {
                    for (int i = 0; i < P; ++i) Am[(int64_t)i * NST + tid] = i == 0 ? 1.f : 0.f;
                } else {
                    float lp = 0.f, lc = 1.f;
                    const float x0 = X[0][0];
#pragma unroll
                    for (int i = 0; i < PMAX; ++i) {
                        if (i < P) Am[(int64_t)i * NST + tid] = lc;
                        const float nx = rec_a<float>(i) * x0 * lc - rec_b<float>(i) * lp;
                        lp = lc;
                        lc = nx;
                    }
                }
#pragma unroll
                for (int j = 0; j < PMAX; ++j)
                    if (j < P) Bmm[(int64_t)j * NST + tid] = Ll[0][j];
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
            T *dstq = gbar + (int64_t)q * aa.bar_stride;
            if constexpr (MFMA) {
                // wave w forms tile w & 1 (0: the f'(u)-weighted table, 1: the
                // plain one) over half w >> 1 of the block's samples, two samples
                // per product (the reduction index k of a product is the lane
                // half: lanes 0-31 take samples base .. base + 63, lanes 32-63 the
                // next 64, four at a time from one 16-byte read per table); the
                // upper half hands its tile to the lower one through LDS with
                // plain stores, which then adds into the table.  Lanes of rows
                // i >= P read row P - 1: they only reach output rows or columns
                // >= P, which are not written out
                const int tile = wave & 1, half = wave >> 1, i = lane & 31;
                constexpr int hs = 128;   // the matrix-core form runs four waves per block
                const int ri = i < P ? i : P - 1;
                const int base = half * hs + (lane >> 5) * (hs / 2);
                const float4 *ap = (const float4 *)(Am + (int64_t)ri * NST + base);
                const float4 *bp = (const float4 *)(Bmm + (int64_t)ri * NST + base);
                const float4 *wp = (const float4 *)(Wm + (int64_t)tile * nthr + base);
                f32x16 c = {};
#pragma unroll
                for (int m = 0; m < hs / 8; ++m) {
                    const float4 a4 = ap[m], b4 = bp[m], w4 = wp[m];
                    c = __builtin_amdgcn_mfma_f32_32x32x2f32(w4.x * a4.x, b4.x, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_32x32x2f32(w4.y * a4.y, b4.y, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_32x32x2f32(w4.z * a4.z, b4.z, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_32x32x2f32(w4.w * a4.w, b4.w, c, 0, 0, 0);
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

// ===========================================================================
// Two-dimensional FP32 form with u* on the matrix cores as well: the lanes
// read the u-table operands of the forward kernel's contraction (32 rows k0
// per column k1, Chebyshev basis) straight from the slab image in the matrix-core
// layout (coalesced 128-byte rows, L2-resident: every block of a group reads
// the same image), and run its products and epilogue in the same order
// -- so u*(X_q), and with it f'(u*), is bit for bit the forward kernel's.  No
// slab passes through LDS.  The weighted outer products stack the u and v
// factors as one set of rows in 16 x 16 tiles (P = 18: six tiles of 256 sums
// where two 32 x 32 tiles hold 1024 each), with the samples as the reduction
// dimension as above.
// Templated on KH = ceil(P/2): every per-sample loop has a fixed trip count.
// ===========================================================================
typedef float f32x4 __attribute__((ext_vector_type(4)));
size_t adjoint_mma2_lds_bytes(int P, int nthr)
{
    const int K2 = 2 * ((P + 1) / 2);
    return ((size_t)2 * K2 * (nthr + 4) + 2 * nthr) * 4 + 2 * 16 * 64 * 4;
}

template <int KH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) adjoint_mma2_kernel(AdjointArgs aa)
{
    constexpr int K2 = 2 * KH;
    constexpr int MT = (2 * K2 + 15) / 16;   // 16-row tiles of the stacked factors (2P <= 2 K2 rows)
    constexpr int NT = (K2 + 15) / 16;       // 16-column tiles of L(X_1)
    constexpr int TP = MT * NT, TW = (TP + 1) / 2;   // tile pairs; at most TW per wave
    static_assert(NT <= 2 && TW <= 4, "the upper half's tiles fit the LDS sum buffer");
    const RoundArgs &a = aa.r;
    extern __shared__ u32x4 lds[];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int P = a.P, PP = a.PP;
    // [i][sample] tables of the basis values L_i(x_0) (Am) and L_j(x_1) (Bm),
    // rows NST = nthr + 4 floats apart, the two weights Wm [2][sample], and
    // the upper half's tiles gsum [2][16][64]
    const int NST = nthr + 4;
    float *Am = (float *)lds;
    float *Bm = Am + K2 * NST;
    float *Wm = Bm + K2 * NST;
    float *gsum = Wm + 2 * nthr;
    __shared__ long long s_item;
    cptr<GroupDesc> groups = as_const(a.groups);
    cptr<NodeDesc> nodes = as_const(a.nodes);
    const int64_t total = a.batch_prefix[a.n_groups];
    using State = PathState<float, 2>;
    const State *sin = (const State *)a.state_in;
    State *sout = (State *)a.state_out;
    float *sbar = (float *)aa.slab_bar;
    // this lane's u-table operands in a step's image: column (lane / 32) KH + kk, row lane % 32
    const int aoff = (lane >> 5) * KH * kMmaRS + (lane & 31);

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
        const float J = (float)G->jump;
        const double ddelta = G->delta;
        const uint32_t c3 = G->c3 | (uint32_t)a.tag;
        const int64_t live = a.round == 0 ? (int64_t)G->node_count * a.mcount : (int64_t)a.live_in[g];
        const float *gtab = (const float *)a.slab_table + G->slab_mma;
        float *gbar = sbar + G->slab;

        float x0 = 0.f, x1 = 0.f, lam = 0.f;
        uint32_t node = 0, sample = 0, c0 = 0;
        const int64_t p = b * a.batch + tid;
        bool alive = p < live;
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
                node = st.node;
                sample = st.sample;
            }
            c0 = nodes[node].c0;
            lam = (float)(aa.lambda[nodes[node].u_index] * ddelta * aa.inv_M);
        }
        uint32_t w[4];
        for (int q = q0; q < q1; ++q) {
            // this step's operands, in flight under the walk step
            const float *gq = gtab + (int64_t)q * a.slab_stride;   // uniform: lanes add a 32-bit offset
            float au[KH];
#pragma unroll
            for (int kk = 0; kk < KH; ++kk) au[kk] = gq[aoff + kk * kMmaRS];
            if ((q & 3) == 0 || q == q0) philox(c0, sample, (uint32_t)(q >> 2), c3, a.key0, a.key1, w);
            const int wi = q & 3;
            const uint32_t word = wi == 0 ? w[0] : wi == 1 ? w[1] : wi == 2 ? w[2] : w[3];
            float d0, d1, y0 = x0, y1 = x1;
            angle_dir(u01(word, 0.f), d0, d1);
            if (alive) {
                y0 = fmaf(J, d0, x0);
                y1 = fmaf(J, d1, x1);
                alive = fabsf(y0) < 1.f && fabsf(y1) < 1.f;
            }
            // ---- weights of this evaluation: lambda Delta/M f'(u*(X_q)) and lambda Delta/M
            float wu = 0.f, wv = 0.f;
            if (__ballot(alive) != 0ull) {
                float b0[KH], b1[KH];
                mma_operands<KH>(x1, P, b0, b1);
                f32x16 du0 = {}, du1 = {}, dv = {};
#pragma unroll
                for (int kk = 0; kk < KH; ++kk) {
                    du0 = __builtin_amdgcn_mfma_f32_32x32x2f32(au[kk], b0[kk], du0, 0, 0, 0);
                    du1 = __builtin_amdgcn_mfma_f32_32x32x2f32(au[kk], b1[kk], du1, 0, 0, 0);
                }
                float u = 0.f, v = 0.f;
                mma_epilogue<KH, true>(du0, dv, du1, dv, x0, u, v);
                if (alive) {
                    wv = lam;
                    wu = lam * fprime_of<float>(a.phys, u);
                }
            }
            // ---- outer-product factors of this sample: rows L(X_0) weighted, columns L(X_1)
            Wm[tid] = wu;
            Wm[nthr + tid] = wv;
            {
                float lp = 0.f, lc = 1.f, mp = 0.f, mc = 1.f;
#pragma unroll
                for (int i = 0; i < K2; ++i) {
                    Am[i * NST + tid] = lc;
                    Bm[i * NST + tid] = mc;
                    const float ai = (float)((2.0 * i + 1.0) / (i + 1.0)), bi = (float)(i / (i + 1.0));
                    const float nx = ai * x0 * lc - bi * lp, ny = ai * x1 * mc - bi * mp;
                    lp = lc;
                    lc = nx;
                    mp = mc;
                    mc = ny;
                }
            }
            if (alive) {
                x0 = y0;
                x1 = y1;
            }
            __syncthreads();
            // ---- block sum of the outer products into the slab adjoint of step q.
            // The two weighted factors are stacked as rows R < 2P (R < P: wu L_R(X_0),
            // else wv L_{R-P}(X_0)) against the columns L_j(X_1), in 16 x 16 tiles on
            // v_mfma_f32_16x16x4f32 with four samples per product (A: lane l holds
            // A[l % 16][l / 16], B: B[l / 16][l % 16], D register r: D[4 (l / 16) + r][l % 16]).
            // Tile pairs t = mt NT + nt alternate between the waves w & 1, the waves
            // w >> 1 take half of the samples each, and the upper half's tiles are added
            // in LDS.  Rows R >= 2P and columns >= P hold finite values never written out.
            float *dstq = gbar + (int64_t)q * aa.bar_stride;
            const int ts = wave & 1, half = wave >> 1, li = lane & 15, ks = lane >> 4;
            const int base = half * 128 + ks * 32;   // this lane's samples: base + m, m < 32
            const float4 *bp = (const float4 *)(Bm + min(16 * (ts % NT) + li, K2 - 1) * NST + base);
            const float4 *ap[TW], *wp[TW];
#pragma unroll
            for (int j = 0; j < TW; ++j) {
                const int R = 16 * ((2 * j + ts) / NT) + li;
                const int tab = R < P ? 0 : 1;
                ap[j] = (const float4 *)(Am + min(R - tab * P, K2 - 1) * NST + base);
                wp[j] = (const float4 *)(Wm + tab * nthr + base);
            }
            f32x4 c[TW];
            float4 b4 = bp[0], a4[TW], w4[TW];
#pragma unroll
            for (int j = 0; j < TW; ++j) {
                c[j] = f32x4{};
                a4[j] = ap[j][0];
                w4[j] = wp[j][0];
            }
            // operands one group of four samples ahead of the products; the fence
            // keeps the scheduler from hoisting every group's reads
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                float4 b4n = b4, a4n[TW], w4n[TW];
#pragma unroll
                for (int j = 0; j < TW; ++j) { a4n[j] = a4[j]; w4n[j] = w4[j]; }
                if (m + 1 < 8) {
                    b4n = bp[m + 1];
#pragma unroll
                    for (int j = 0; j < TW; ++j) { a4n[j] = ap[j][m + 1]; w4n[j] = wp[j][m + 1]; }
                }
                // the weighted operands first, then the products round-robin over the
                // tile pairs: no product waits on the one just issued
                float wa[TW][4];
#pragma unroll
                for (int j = 0; j < TW; ++j) {
                    wa[j][0] = w4[j].x * a4[j].x;
                    wa[j][1] = w4[j].y * a4[j].y;
                    wa[j][2] = w4[j].z * a4[j].z;
                    wa[j][3] = w4[j].w * a4[j].w;
                }
                const float bb[4] = {b4.x, b4.y, b4.z, b4.w};
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
#pragma unroll
                    for (int j = 0; j < TW; ++j)
                        if (2 * j + ts < TP) c[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[j][k4], bb[k4], c[j], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
                b4 = b4n;
#pragma unroll
                for (int j = 0; j < TW; ++j) { a4[j] = a4n[j]; w4[j] = w4n[j]; }
            }
            float *cm = gsum + ts * 16 * 64 + lane;
            if (half == 1) {
#pragma unroll
                for (int j = 0; j < TW; ++j)
                    if (2 * j + ts < TP) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) cm[(4 * j + r) * 64] = c[j][r];
                    }
            }
            const int any_alive = __syncthreads_or(alive ? 1 : 0);
            if (half == 0) {
                const int col = 16 * (ts % NT) + li;
#pragma unroll
                for (int j = 0; j < TW; ++j) {
                    if (2 * j + ts >= TP || col >= P) continue;
                    const int R0 = 16 * ((2 * j + ts) / NT) + 4 * ks;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int R = R0 + r;
                        const float val = c[j][r] + cm[(4 * j + r) * 64];
                        if (R < 2 * P && val != 0.f) {
                            const int tab = R < P ? 0 : 1;
                            atomicAdd(dstq + ((R - tab * P) * 2 * PP + tab * PP + col), val);
                        }
                    }
                }
            }
            if (any_alive == 0) break;
        }
        // survivors to the next round
        const bool carry = alive && q1 < nstar;
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
                st.acc = 0.f;
                st.comp = 0.f;
                st.node = node;
                st.sample = sample;
                sout[G->path_off + off] = st;
            }
        }
    }
}

template <int KH>
static hipError_t adj_mma2(const AdjointArgs &a, int kh, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    if constexpr (KH > kAdjMma2MaxKH) {
        return hipErrorInvalidValue;
    } else {
        if (kh != KH) return adj_mma2<KH + 1>(a, kh, grid, block, lds, s);
        if (block.x != 256 || lds < adjoint_mma2_lds_bytes(a.r.P, 256)) return hipErrorInvalidValue;
        hipLaunchKernelGGL((adjoint_mma2_kernel<KH>), grid, block, lds, s, a);
        return hipGetLastError();
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
    if (a.use_mfma == 2) {
        if (!fp32 || a.r.phys.dim != 2 || a.r.P < 3 || a.r.P > 2 * kAdjMma2MaxKH) return hipErrorInvalidValue;
        return adj_mma2<2>(a, (a.r.P + 1) / 2, grid, block, lds_bytes, s);
    }
    if (a.r.phys.dim == 1) return fp32 ? adj_p<float, 1>(a, grid, block, lds_bytes, s) : adj_p<double, 1>(a, grid, block, lds_bytes, s);
    if (a.r.phys.dim == 2) return fp32 ? adj_p<float, 2>(a, grid, block, lds_bytes, s) : adj_p<double, 2>(a, grid, block, lds_bytes, s);
    return hipErrorInvalidValue;
}

}  // namespace hpsmc
