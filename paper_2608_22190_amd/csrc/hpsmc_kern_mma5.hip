// Matrix-core form of the 5-D FP32 round kernel (v_mfma_f32_32x32x2f32).
#include "hpsmc_device.h"

namespace hpsmc {

hipError_t set_rec_tables_mma5() { return upload_recurrence_tables(); }

// ===========================================================================
// The residual of a walk step needs u and v at the path's point X, each a
// contraction of the step's slab S[k0..k4] with the tensor product of the
// Legendre values L_{k_i}(X_i) (eq. interIQ, the tensor-product basis of the
// discrete space).  Over the 64 paths of a wave the innermost two modes form
// a dense product: with B[(k3,k4)][s] = L_{k3}(X3_s) L_{k4}(X4_s),
//     T[(k0,k1,k2)][s] = sum_{k3,k4} S[k0,k1,k2,k3,k4] B[(k3,k4)][s],
// a (rows x P^2)(P^2 x 64) product, then per path
//     u_s = sum_{k0,k1,k2} L_{k0} L_{k1} L_{k2} T[(k0,k1,k2)][s],
// P^3 multiply-adds on the vector unit.  The product takes 4 P^5 of the 4 P^5
// + O(P^3) operations of a residual evaluation; it runs on the matrix cores in
// 32-row tiles (the slab layout of mma5_geom) streamed through LDS.
//
// Operands of v_mfma_f32_32x32x2f32 (A: lane l holds A[l%32][l/32]; B:
// B[l/32][l%32]; D register r: D[8(r/4) + 4(l/32) + r%4][l%32]).  Paths 0-31
// form product "A", paths 32-63 product "B", the u and v tables each take
// both: four independent accumulators.  K-step j = (k3, m) feeds k4 = 2m on
// lanes 0-31 and k4 = 2m + 1 on lanes 32-63, so a lane needs L_{k3} and
// L_{k4} of its own path and of the path 32 lanes away -- one permlane32 swap
// per value, once per step -- and forms each B entry with one multiply.
// ===========================================================================
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int P>
__device__ __forceinline__ void legendre_row(float x, float (&L)[P])
{
    L[0] = 1.f;
    if (P > 1) L[1] = x;
#pragma unroll
    for (int k = 1; k + 1 < P; ++k)
        L[k + 1] = (float)((2.0 * k + 1.0) / (k + 1.0)) * x * L[k] - (float)(k / (k + 1.0)) * L[k - 1];
}

// B-operand factors of the wave's 64 points: a3/a4 for product A (paths 0-31),
// b3/b4 for product B (paths 32-63), in the lane-half split of the K-steps
template <int P>
__device__ __forceinline__ void mma5_operands(float x3, float x4, float (&a3)[P], float (&b3)[P],
                                              float (&a4)[(P + 1) / 2], float (&b4)[(P + 1) / 2])
{
    constexpr int HK = (P + 1) / 2;
    float L3[P], L4[P];
    legendre_row<P>(x3, L3);
    legendre_row<P>(x4, L4);
#pragma unroll
    for (int k = 0; k < P; ++k) {
        // lanes 0-31 keep their own value and take the upper lane's, lanes 32-63 the reverse
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(L3[k]), __float_as_uint(L3[k]), false, false);
        a3[k] = __uint_as_float(r[0]);
        b3[k] = __uint_as_float(r[1]);
    }
#pragma unroll
    for (int m = 0; m < HK; ++m) {
        const float lo = L4[2 * m], hi = 2 * m + 1 < P ? L4[2 * m + 1] : 0.f;   // odd P: mode P is zero
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
        a4[m] = __uint_as_float(r[0]);   // lanes 0-31: own L_{2m}; lanes 32-63: L_{2m+1} of lane - 32
        b4[m] = __uint_as_float(r[1]);   // lanes 0-31: L_{2m} of lane + 32; lanes 32-63: own L_{2m+1}
    }
}

// the four products of one tile over k-steps [J0, J1) (S: the chunk's u tile,
// its v tile 32 RS floats on)
template <int P, int J0, int J1>
__device__ __forceinline__ void mma5_tile(const float *S, int lane, const float (&a3)[P], const float (&b3)[P],
                                          const float (&a4)[(P + 1) / 2], const float (&b4)[(P + 1) / 2],
                                          f32x16 &uA, f32x16 &vA, f32x16 &uB, f32x16 &vB)
{
    constexpr Mma5Geom g = mma5_geom(P);
    static_assert(0 <= J0 && J0 < J1 && J1 <= g.KJ, "k-step range");
    constexpr int JB = J0 & ~3;   // first 16-byte group
    const float *Au = S + (lane & 31) * g.RS + (lane >> 5) * g.KH2;
    const float *Av = Au + 32 * g.RS;
    uA = f32x16{}; vA = f32x16{}; uB = f32x16{}; vB = f32x16{};
    // the B entries are formed next to their products: hoisted out of the tile
    // and k0 loops, all KJ pairs of them would stay live
    float f3[P], g3[P], f4[(P + 1) / 2], g4[(P + 1) / 2];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        f3[k] = a3[k];
        g3[k] = b3[k];
        asm volatile("" : "+v"(f3[k]), "+v"(g3[k]));
    }
#pragma unroll
    for (int m = 0; m < (P + 1) / 2; ++m) {
        f4[m] = a4[m];
        g4[m] = b4[m];
        asm volatile("" : "+v"(f4[m]), "+v"(g4[m]));
    }
    // A operands four k-steps at a time, one group ahead of the products; the
    // scheduling fence keeps later groups from being hoisted (their registers
    // would push the kernel past two waves per SIMD)
    f32x4 xu = *(const f32x4 *)(Au + JB), xv = *(const f32x4 *)(Av + JB);
#pragma unroll
    for (int jj = JB; jj < J1; jj += 4) {
        f32x4 nu = xu, nv = xv;
        if (jj + 4 < J1) {
            nu = *(const f32x4 *)(Au + jj + 4);
            nv = *(const f32x4 *)(Av + jj + 4);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int j = jj + s;
            if (j >= J0 && j < J1) {
                const int k3 = j / g.HK, m = j - k3 * g.HK;
                const float bA = f3[k3] * f4[m], bB = g3[k3] * g4[m];
                uA = __builtin_amdgcn_mfma_f32_32x32x2f32(xu[s], bA, uA, 0, 0, 0);
                vA = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[s], bA, vA, 0, 0, 0);
                uB = __builtin_amdgcn_mfma_f32_32x32x2f32(xu[s], bB, uB, 0, 0, 0);
                vB = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[s], bB, vB, 0, 0, 0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        xu = nu;
        xv = nv;
    }
}

// the products of part `part` of `nparts` (1, 2 or 4: the waves that share
// one item in a sparse round) -- k-steps [KJ part / nparts, KJ (part + 1) / nparts)
template <int P>
__device__ __forceinline__ void mma5_tile_part(int part, int nparts, const float *S, int lane, const float (&a3)[P],
                                               const float (&b3)[P], const float (&a4)[(P + 1) / 2],
                                               const float (&b4)[(P + 1) / 2], f32x16 &uA, f32x16 &vA, f32x16 &uB,
                                               f32x16 &vB)
{
    constexpr int KJ = mma5_geom(P).KJ;
    if (nparts == 1) {
        mma5_tile<P, 0, KJ>(S, lane, a3, b3, a4, b4, uA, vA, uB, vB);
    } else if (nparts == 2) {
        if (part == 0) mma5_tile<P, 0, KJ / 2>(S, lane, a3, b3, a4, b4, uA, vA, uB, vB);
        else mma5_tile<P, KJ / 2, KJ>(S, lane, a3, b3, a4, b4, uA, vA, uB, vB);
    } else {
        switch (part) {
        case 0: mma5_tile<P, 0, KJ / 4>(S, lane, a3, b3, a4, b4, uA, vA, uB, vB); break;
        case 1: mma5_tile<P, KJ / 4, KJ / 2>(S, lane, a3, b3, a4, b4, uA, vA, uB, vB); break;
        case 2: mma5_tile<P, KJ / 2, 3 * KJ / 4>(S, lane, a3, b3, a4, b4, uA, vA, uB, vB); break;
        default: mma5_tile<P, 3 * KJ / 4, KJ>(S, lane, a3, b3, a4, b4, uA, vA, uB, vB); break;
        }
    }
}

// Rows of a tile back to the lane that owns the path: register r holds rows
// 8(r/4) + r%4 (from the lane's own half) and 8(r/4) + 4 + r%4 (from the other
// half) of the path's column after one swap of the A and B products.
// Main tile t of a k0: rows f = 32 t + i = (k1, k2); au[k1] += L_{k2} T.
template <int P>
__device__ __forceinline__ void mma5_fold_main(int t, const f32x16 &uA, const f32x16 &vA, const f32x16 &uB,
                                               const f32x16 &vB, const float (&L2)[P], float (&au)[P], float (&av)[P])
{
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int ia = 8 * (r >> 2) + (r & 3), ib = ia + 4;
        const int fa = 32 * t + ia, fb = 32 * t + ib;
        const auto pu = __builtin_amdgcn_permlane32_swap(__float_as_uint(uA[r]), __float_as_uint(uB[r]), false, false);
        const auto pv = __builtin_amdgcn_permlane32_swap(__float_as_uint(vA[r]), __float_as_uint(vB[r]), false, false);
        au[fa / P] = fmaf(L2[fa % P], __uint_as_float(pu[0]), au[fa / P]);
        au[fb / P] = fmaf(L2[fb % P], __uint_as_float(pu[1]), au[fb / P]);
        av[fa / P] = fmaf(L2[fa % P], __uint_as_float(pv[0]), av[fa / P]);
        av[fb / P] = fmaf(L2[fb % P], __uint_as_float(pv[1]), av[fb / P]);
    }
}

// Remainder tile t: rows rr = 32 t + i hold (k0, f) = (rr / B, 32 A + rr % B),
// weight L_{k0} L_{k1} L_{k2}; rows past B P are zero and skipped.
template <int P>
__device__ __forceinline__ void mma5_fold_rem(int t, const f32x16 &uA, const f32x16 &vA, const f32x16 &uB,
                                              const f32x16 &vB, const float (&L0)[P], const float (&L1)[P],
                                              const float (&L2)[P], float &u, float &v)
{
    constexpr Mma5Geom g = mma5_geom(P);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int ia = 8 * (r >> 2) + (r & 3), ib = ia + 4;
        const int ra = 32 * t + ia, rb = 32 * t + ib;
        if (ra >= g.B * P) continue;   // rb > ra
        const auto pu = __builtin_amdgcn_permlane32_swap(__float_as_uint(uA[r]), __float_as_uint(uB[r]), false, false);
        const auto pv = __builtin_amdgcn_permlane32_swap(__float_as_uint(vA[r]), __float_as_uint(vB[r]), false, false);
        {
            const int k0 = ra / g.B, f = 32 * g.A + ra % g.B;
            const float w = L0[k0] * (L1[f / P] * L2[f % P]);
            u = fmaf(w, __uint_as_float(pu[0]), u);
            v = fmaf(w, __uint_as_float(pv[0]), v);
        }
        if (rb < g.B * P) {
            const int k0 = rb / g.B, f = 32 * g.A + rb % g.B;
            const float w = L0[k0] * (L1[f / P] * L2[f % P]);
            u = fmaf(w, __uint_as_float(pu[1]), u);
            v = fmaf(w, __uint_as_float(pv[1]), v);
        }
    }
}

// ===========================================================================
// Round kernel, matrix-core form: d = 5, FP32, residual form with the
// centre-point rule, one path per lane.  The walk (directions from two
// Philox blocks per step, jump, exit test of eq. indexL, left-point
// quadrature of eq. interIQ with compensated summation) is the vector-unit
// kernel's, so both take the same exit steps and differ in u, v only by the
// order of the FP32 sums.  A step's NCH chunks stream through two LDS buffers
// along one sequence that runs on into the next step: while a chunk's
// products run, the next chunk is in flight (global_load_lds), and one
// barrier per chunk publishes it.
// ===========================================================================
template <int P>
__device__ __forceinline__ void advance_mma5_body(const RoundArgs &a)
{
    constexpr Mma5Geom g5 = mma5_geom(P);
    constexpr int HK = g5.HK, A = g5.A, R = g5.R, NCH = g5.NCH;
    constexpr int CF = (int)g5.chunk, CV = CF / 4;   // floats, 16-byte vectors per chunk
    extern __shared__ u32x4 lds[];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6;
    __shared__ long long s_item;
    __shared__ SrcTime<float> s_tf[256];   // source time factors of a window of blockDim.x steps
    __shared__ float s_red[2][4][64];      // sparse rounds: each wave's share of u and v
    cptr<GroupDesc> groups = as_const(a.groups);
    cptr<NodeDesc> nodes = as_const(a.nodes);
    const int64_t total = a.batch_prefix[a.n_groups];
    // Sparse rounds (few live paths, set by the round's prep kernel): an item is
    // 64 paths that every wave of the block walks alike; wave w runs its share
    // of each tile's k-steps, the shares are summed in wave order, and wave 0
    // alone writes results, state and counts.
    const int bsz = (int)a.batch_prefix[a.n_groups + 1];
    const bool split = bsz < nthr;
    const int nparts = split ? nthr >> 6 : 1, part = split ? wave : 0;
    const bool writer = !split || wave == 0;
    unsigned long long evals = 0, slots = 0;
    using State = PathState<float, 5>;
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
        const int64_t p = b * bsz + (split ? lane : tid);
        bool alive = p < live;
        uint32_t node = 0, sample = 0, c0 = 0;
        float X[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, acc = 0.f, comp = 0.f;
        if (alive) {
            if (a.round == 0) {
                node = (uint32_t)(G->node_begin + p / a.mcount);
                sample = (uint32_t)(a.m0 + p % a.mcount);
#pragma unroll
                for (int i = 0; i < 5; ++i) X[i] = (float)nodes[node].x0[i];
            } else {
                const State st = sin[G->path_off + p];
#pragma unroll
                for (int i = 0; i < 5; ++i) X[i] = st.x[i];
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
        // chunk 0 of the first step into buffer 0; buf: the buffer of the current chunk
        mma_stage((const u32x4 *)(gtab + (int64_t)q0 * a.slab_stride), lds, CV, tid, nthr);
        mma_stage_wait();
        __syncthreads();
        int buf = 0;

        int q = q0, tslot = 0;
        for (; q < q1; ++q, ++tslot) {
            if (tslot == nthr) {   // the previous step's barrier ended every read of the old window
                tslot = 0;
                fill_time(q);
                __syncthreads();
            }
            // ---- direction (Philox blocks 2q, 2q + 1), jump and exit test (eq. indexL)
            float Y[5];
            if (alive) {
                float dir[5];
                sphere_dir<float, 5>(c0, sample, q, c3, a.key0, a.key1, dir);
                bool inside = true;
#pragma unroll
                for (int i = 0; i < 5; ++i) {
                    Y[i] = m_fma(J, dir[i], X[i]);
                    inside = inside && (fabsf(Y[i]) < 1.f);
                }
                if (!inside) {   // path ended: L = q
                    alive = false;
                    if (writer)
                        a.result[(int64_t)nodes[node].out * a.mcount + (sample - a.m0)] = (double)acc - (double)comp;
                }
            }
            if (writer) ++slots;
            // ---- u and v at X_q: the step's chunks, the next one always in flight
            const bool wave_live = __ballot(alive) != 0ull;
            float a3[P], b3[P], a4[HK], b4[HK], L1[P], L2[P];
            mma5_operands<P>(X[3], X[4], a3, b3, a4, b4);
            legendre_row<P>(X[1], L1);
            legendre_row<P>(X[2], L2);
            const float *step_src = gtab + (int64_t)q * a.slab_stride;
            const bool more = q + 1 < q1;
            auto stage_next = [&](int c) {   // chunk c + 1 of this step, or chunk 0 of the next
                const float *src = c + 1 < NCH ? step_src + (int64_t)(c + 1) * CF : (more ? step_src + a.slab_stride : nullptr);
                if (src) mma_stage((const u32x4 *)src, lds + (buf ^ 1) * CV, CV, tid, nthr);
            };
            float u = 0.f, v = 0.f;
            if constexpr (A > 0) {
                float l0p = 0.f, l0c = 1.f;   // L_{k0}(X0)
                for (int k0 = 0; k0 < P; ++k0) {
                    float au[P], av[P];
#pragma unroll
                    for (int k = 0; k < P; ++k) { au[k] = 0.f; av[k] = 0.f; }
#pragma unroll
                    for (int t = 0; t < A; ++t) {
                        stage_next(k0 * A + t);
                        if (wave_live) {
                            f32x16 uA, vA, uB, vB;
                            mma5_tile_part<P>(part, nparts, (const float *)(lds + buf * CV), lane, a3, b3, a4, b4,
                                              uA, vA, uB, vB);
                            mma5_fold_main<P>(t, uA, vA, uB, vB, L2, au, av);
                        }
                        mma_stage_wait();
                        __syncthreads();
                        buf ^= 1;
                    }
                    float su = 0.f, sv = 0.f;
#pragma unroll
                    for (int k = 0; k < P; ++k) {
                        su = fmaf(L1[k], au[k], su);
                        sv = fmaf(L1[k], av[k], sv);
                    }
                    u = fmaf(l0c, su, u);
                    v = fmaf(l0c, sv, v);
                    const float nx = (float)((2.0 * k0 + 1.0) / (k0 + 1.0)) * X[0] * l0c - (float)(k0 / (k0 + 1.0)) * l0p;
                    l0p = l0c;
                    l0c = nx;
                }
            }
            if constexpr (R > 0) {
                float L0[P];
                legendre_row<P>(X[0], L0);
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    stage_next(P * A + t);
                    if (wave_live) {
                        f32x16 uA, vA, uB, vB;
                        mma5_tile_part<P>(part, nparts, (const float *)(lds + buf * CV), lane, a3, b3, a4, b4, uA, vA,
                                          uB, vB);
                        mma5_fold_rem<P>(t, uA, vA, uB, vB, L0, L1, L2, u, v);
                    }
                    mma_stage_wait();
                    __syncthreads();
                    buf ^= 1;
                }
            }
            if (split) {   // the waves' shares of u and v, summed in wave order
                s_red[0][wave][lane] = u;
                s_red[1][wave][lane] = v;
                __syncthreads();
                u = 0.f;
                v = 0.f;
                for (int k = 0; k < nparts; ++k) {
                    u += s_red[0][k][lane];
                    v += s_red[1][k][lane];
                }
            }
            if (alive) {   // residual at X_q, time tau_q = t_{n,l} - q Delta
                const float r = f_of<float>(a.phys, u) + source_space<float, 5>(a.phys, X, s_tf[tslot]) + v;
                const float y = delta * r;
                const float yc = y - comp;
                const float tt = acc + yc;
                comp = (tt - acc) - yc;
                acc = tt;
#pragma unroll
                for (int i = 0; i < 5; ++i) X[i] = Y[i];
                if (writer) ++evals;
            }
            if (__syncthreads_or(alive ? 1 : 0) == 0) { ++q; break; }
        }

        // ---- paths alive after the round: finished at N*, or carried to the next round
        const bool carry = writer && alive && q1 < nstar;
        if (writer && alive && !carry)
            a.result[(int64_t)nodes[node].out * a.mcount + (sample - a.m0)] = (double)acc - (double)comp;
        const unsigned long long mask = __ballot(carry);
        if (mask != 0ull) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(a.live_out + g, (uint32_t)__popcll(mask));
            base = __shfl(base, 0, 64);
            if (carry) {
                const uint32_t off = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
                State st;
#pragma unroll
                for (int i = 0; i < 5; ++i) st.x[i] = X[i];
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

template <int P>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) advance_mma5_kernel(RoundArgs a)
{
    advance_mma5_body<P>(a);
}

bool advance_mma5_eligible(int fp32, int dim, int P, int picard, int ball, int samples_per_lane, int waves_per_block)
{
    return fp32 && dim == 5 && P >= 3 && P <= 12 && !picard && !ball && samples_per_lane == 1 &&
           waves_per_block >= 1 && waves_per_block <= 4;
}

size_t advance_mma5_lds_bytes(int P) { return (size_t)2 * mma5_geom(P).chunk * sizeof(float); }

template <int P>
static hipError_t adv_mma5(const RoundArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    if constexpr (P > 12) {
        return hipErrorInvalidValue;
    } else {
        if (a.P != P) return adv_mma5<P + 1>(a, grid, block, lds, s);
        if (lds < advance_mma5_lds_bytes(P) || a.slab_stride != mma5_geom(P).step) return hipErrorInvalidValue;
        hipLaunchKernelGGL((advance_mma5_kernel<P>), grid, block, lds, s, a);
        return hipGetLastError();
    }
}

hipError_t launch_adv_mma5(const RoundArgs &a, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    if (a.phys.dim != 5 || a.phys.picard || a.phys.ball || a.P < 3 || block.x > 256 || block.x % 64 != 0)
        return hipErrorInvalidValue;
    return adv_mma5<3>(a, grid, block, lds, s);
}

}  // namespace hpsmc
