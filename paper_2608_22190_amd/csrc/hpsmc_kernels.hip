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
//                     (Algorithm 1, Step 3), max|eps| (the stop metric).//   (the round kernels live in hpsmc_kern_valu_f32/f64.hip, hpsmc_kern_mma.hip
//   and hpsmc_kern_frac.hip, the adjoint in hpsmc_kern_adjoint.hip)
#include "hpsmc_device.h"

namespace hpsmc {

// Element-wise kernels stride over their range from a grid of at most kGridCap
// blocks: a dispatch counts its work-items in 32 bits, so a grid of one
// thread per element wraps past 2^32 elements (a c5 slab-adjoint table holds
// 10.7 G 8-byte words).
constexpr int64_t kGridCap = 1 << 20;
// a grid's y and z extents are at most 65536 blocks: counts past that run over y and z
constexpr int kGridYZ = 65535;
static inline unsigned grid_blocks(int64_t n, int block) { return (unsigned)std::min<int64_t>((n + block - 1) / block, kGridCap); }


hipError_t set_rec_tables_main() { return upload_recurrence_tables(); }

hipError_t set_recurrence_tables()
{
    for (hipError_t (*f)() : {set_rec_tables_main, set_rec_tables_valu_f32, set_rec_tables_valu_f64,
                              set_rec_tables_mma, set_rec_tables_mma5, set_rec_tables_frac,
                              set_rec_tables_adjoint})
        if (hipError_t e = f(); e != hipSuccess) return e;
    return hipSuccess;
}

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
// L_k(xi_q) of its steps go to LDS once (one row per degree k, the steps
// contiguous), and every entry runs over its T1 time coefficients once,
// each feeding the kSlabQ independent step sums -- the same products in the
// same order as entry by entry, with no per-degree branch in the loop.
// ---------------------------------------------------------------------------
constexpr int kSlabQ = 32;

template <typename T>
__global__ void __launch_bounds__(256) slab_kernel(SlabArgs a)
{
    __shared__ __align__(16) double Lt[kMaxDeg + 1][kSlabQ];
    const int g = blockIdx.z * kGridYZ + blockIdx.y;   // groups over y and z (y at most 65535)
    if (g >= a.n_groups) return;
    const int nq = a.nstar[g] + a.extra;
    const int T1 = a.deg[g] + 1;
    const bool mma = a.layout == 1, mma5 = a.layout == 2;
    const Mma5Geom g5 = mma5_geom(a.P);
    const int64_t stride = a.layout ? a.mma_stride : a.slab_stride;
    const int64_t base = a.layout ? a.slab_off_mma[g] : a.slab_off[g];
    T *table = (T *)a.slab_table;
    const double *cu = a.cu + a.coef_off[g], *cv = a.cv + a.coef_off[g];
    const double *cs = a.cs ? a.cs + a.cs_off[g] : nullptr;   // polynomial source, folded into v
    const double span = a.span[g], delta = a.delta[g], h2 = a.h2[g];
    for (int q0 = blockIdx.x * kSlabQ; q0 < nq; q0 += gridDim.x * kSlabQ) {
        const int qn = min(kSlabQ, nq - q0);
        __syncthreads();   // the previous chunk's reads of Lt are over
        if ((int)threadIdx.x < kSlabQ) {   // steps past the chunk's end get zeros (never stored)
            const int j = threadIdx.x;
            const double xi = h2 * (span - (double)(q0 + j) * delta) - 1.0;
            double lp = 0.0, lc = 1.0;
            for (int k = 0; k < T1; ++k) {
                Lt[k][j] = j < qn ? lc : 0.0;
                const double nx = c_rec.ad[k] * xi * lc - c_rec.bd[k] * lp;
                lp = lc;
                lc = nx;
            }
        }
        __syncthreads();
        for (int64_t e = threadIdx.x; e < stride; e += blockDim.x) {
            int64_t row = 0;
            int uv = 0, kl = 0;
            bool live;
            if (mma5) {  // 32-row tiles over (k0, k1, k2), columns (k3, k4)
                live = mma5_source(g5, e, uv, row, kl);
            } else {
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
                live = kl < a.P && row < a.rows;
            }
            double acc[kSlabQ];
#pragma unroll
            for (int j = 0; j < kSlabQ; ++j) acc[j] = 0.0;
            if (live) {
                const double *cp = (uv ? cv : cu) + (row * a.P + kl) * T1;
                const double *sp = uv && cs ? cs + (row * a.P + kl) * T1 : nullptr;
                for (int k = 0; k < T1; ++k) {
                    const double ck = sp ? cp[k] + sp[k] : cp[k];
                    const double2 *lk = (const double2 *)Lt[k];
#pragma unroll
                    for (int j = 0; j < kSlabQ / 2; ++j) {
                        const double2 l2 = lk[j];
                        acc[2 * j] = fma(ck, l2.x, acc[2 * j]);
                        acc[2 * j + 1] = fma(ck, l2.y, acc[2 * j + 1]);
                    }
                }
            }
            T *dst = table + base + (int64_t)q0 * stride + e;
#pragma unroll
            for (int j = 0; j < kSlabQ; ++j)
                if (j < qn) dst[(int64_t)j * stride] = (T)acc[j];
        }
    }
}

hipError_t launch_slabs(const SlabArgs &a, int fp32, int max_nstar, hipStream_t s)
{
    if (a.n_groups <= 0) return hipSuccess;
    int64_t bx = (max_nstar + a.extra + kSlabQ - 1) / kSlabQ;
    if (bx > 65535) bx = 65535;
    dim3 grid((unsigned)bx, (unsigned)std::min<int64_t>(a.n_groups, kGridYZ),
              (unsigned)((a.n_groups + kGridYZ - 1) / kGridYZ));
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
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < count; r += (int64_t)gridDim.x * blockDim.x) {
        const double v = src[r * src_stride + src_off];
        double *d = U + r * dst_stride;
        if (replicate)
            for (int l = 0; l < T1; ++l) d[l] = v;
        else
            d[0] = v;
    }
}

hipError_t launch_start_columns(double *U, const double *src, int64_t src_stride, int64_t src_off, int64_t dst_stride,
                                int T1, int64_t count, int replicate, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(start_columns_kernel, dim3(grid_blocks(count, 256)), dim3(256), 0, s, U, src,
                       src_stride, src_off, dst_stride, T1, count, replicate);
    return hipGetLastError();
}

__global__ void fill_u64_kernel(unsigned long long *p, int64_t n, unsigned long long v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_blocks(n, 256)), dim3(256), 0, s, p, n, v);
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
    // one thread per point, in launches of at most kGridCap blocks
    for (int64_t k0 = 0; k0 < npts; k0 += kGridCap * 64) {
        const int64_t n = std::min<int64_t>(npts - k0, kGridCap * 64);
        hipLaunchKernelGGL(eval_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, cu, cv, dim, P, T1, t_prev,
                           h, pts + k0 * (dim + 1), n, out + 2 * k0);
        if (hipError_t e = hipGetLastError()) return e;
    }
    return hipSuccess;
}

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
                                  int32_t steps, int64_t mcount, int32_t batch, int32_t batch_split,
                                  int64_t split_max, const uint32_t *__restrict__ live_in,
                                  uint32_t *__restrict__ live_out, int64_t *__restrict__ batch_prefix,
                                  unsigned long long *work)
{
    // one block of 256 threads: clear the output counters, then an exclusive
    // prefix over groups of their work items (each thread a contiguous chunk,
    // an inclusive scan of the 256 chunk sums in LDS in eight doubling steps,
    // then the chunks again).  With batch_split > 0 a round whose paths fit in
    // at most split_max items of batch_split paths takes that batch instead;
    // batch_prefix[n_groups + 1] holds the paths per item the round kernel is
    // to use.
    __shared__ int64_t part[256], part_s[256];
    __shared__ int32_t s_split;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int g = t; g < n_groups; g += nt) live_out[g] = 0u;
    const int64_t q0 = (int64_t)round * steps;
    auto items = [&](int g, int32_t bsz) -> int64_t {
        int64_t live = round == 0 ? (int64_t)groups[g].node_count * mcount : (int64_t)live_in[g];
        if (q0 >= groups[g].nstar) live = 0;
        return (live + bsz - 1) / bsz;
    };
    const int chunk = (n_groups + nt - 1) / nt;
    const int g0 = min(n_groups, t * chunk), g1 = min(n_groups, g0 + chunk);
    int64_t sum = 0, sum_s = 0;
    for (int g = g0; g < g1; ++g) {
        sum += items(g, batch);
        if (batch_split > 0) sum_s += items(g, batch_split);
    }
    part[t] = sum;
    part_s[t] = sum_s;
    __syncthreads();
    for (int o = 1; o < nt; o <<= 1) {   // inclusive scans of both sets of chunk sums
        const int64_t v = t >= o ? part[t - o] : 0, v_s = t >= o ? part_s[t - o] : 0;
        __syncthreads();
        part[t] += v;
        part_s[t] += v_s;
        __syncthreads();
    }
    if (t == 0) {
        const bool split = batch_split > 0 && part_s[nt - 1] <= split_max;
        batch_prefix[n_groups] = split ? part_s[nt - 1] : part[nt - 1];
        batch_prefix[n_groups + 1] = split ? batch_split : batch;
        s_split = split ? 1 : 0;
        *work = 0ull;
    }
    __syncthreads();
    const bool split = s_split != 0;
    const int32_t bsz = split ? batch_split : batch;
    int64_t acc = split ? part_s[t] - sum_s : part[t] - sum;   // this chunk's exclusive prefix
    for (int g = g0; g < g1; ++g) {
        batch_prefix[g] = acc;
        acc += items(g, bsz);
    }
}

hipError_t launch_round_prep(const GroupDesc *groups, int32_t n_groups, int32_t round, int32_t steps, int64_t mcount,
                             int32_t batch, int32_t batch_split, int64_t split_max, const uint32_t *live_in,
                             uint32_t *live_out, int64_t *batch_prefix, unsigned long long *work, hipStream_t s)
{
    hipLaunchKernelGGL(round_prep_kernel, dim3(1), dim3(256), 0, s, groups, n_groups, round, steps, mcount, batch,
                       batch_split, split_max, live_in, live_out, batch_prefix, work);
    return hipGetLastError();
}

hipError_t launch_advance(const RoundArgs &a, int fp32, int samples_per_lane, int waves_per_block, int blocks,
                          size_t lds_bytes, int kern, hipStream_t s)
{
    dim3 block(64 * waves_per_block), grid(blocks);
    if (a.phys.frac) return launch_adv_frac(a, fp32, grid, block, lds_bytes, s);
    const int mma = kern;
    if (kern == 3) {
        if (!advance_1d_eligible(a.phys.dim, a.P, a.phys.picard, a.phys.ball, a.phys.frac, samples_per_lane))
            return hipErrorInvalidValue;
        return launch_adv_1d(a, fp32, samples_per_lane, grid, block, lds_bytes, s);
    }
    if (mma == 2) {
        if (!advance_mma5_eligible(fp32, a.phys.dim, a.P, a.phys.picard, a.phys.ball, samples_per_lane, waves_per_block))
            return hipErrorInvalidValue;
        return launch_adv_mma5(a, grid, block, lds_bytes, s);
    }
    if (mma) {
        if (!advance_mma_eligible(fp32, a.phys.dim, a.P, a.cf, samples_per_lane, waves_per_block))
            return hipErrorInvalidValue;
        return launch_adv_mma(a, grid, block, lds_bytes, s);
    }
    return fp32 ? launch_adv_valu_f32(a, samples_per_lane, grid, block, lds_bytes, s)
                : launch_adv_valu_f64(a, samples_per_lane, grid, block, lds_bytes, s);
}

// sums[out][0..1] (+)= sum over the slice's samples of S and S^2: one wave per
// node (nodes strided over a capped grid), lane l summing samples l, l + 64,
// ... in order from coalesced loads, then a fixed xor butterfly over the lanes
// (every lane ends with the same sums, the same way every run)
__global__ void __launch_bounds__(256) slice_reduce_kernel(const double *__restrict__ result, int64_t n_nodes,
                                                           int64_t mcount, double *__restrict__ sums, int first)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; i < n_nodes; i += nwaves) {
        const double *r = result + i * mcount;
        double s1 = 0.0, s2 = 0.0;
        for (int64_t k = lane; k < mcount; k += 64) {
            const double v = r[k];
            s1 += v;
            s2 = fma(v, v, s2);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            s1 += __shfl_xor(s1, o, 64);
            s2 += __shfl_xor(s2, o, 64);
        }
        if (lane == 0) {
            if (first) { sums[2 * i] = s1; sums[2 * i + 1] = s2; }
            else { sums[2 * i] += s1; sums[2 * i + 1] += s2; }
        }
    }
}

hipError_t launch_slice_reduce(const double *result, int64_t n_nodes, int64_t mcount, double *sums, int first,
                               hipStream_t s)
{
    if (n_nodes <= 0) return hipSuccess;
    hipLaunchKernelGGL(slice_reduce_kernel, dim3(grid_blocks(n_nodes, 4)), dim3(256), 0, s, result, n_nodes, mcount,
                       sums, first);
    return hipGetLastError();
}

// Transpose of the slab kernel: cbar[inst][k][m] = sum over the instance's
// node times l and steps q of Sbar_{g,q}[k] L_m(xi_{l,q}).  A block takes one
// instance and 256 consecutive entries e of the row layout ([row][u: PP][v:
// PP]) and streams their columns over every step of every group of the
// instance: one coalesced 1 KiB row per step, a chunk of kSlabQ steps' loads
// in flight per thread (a half or a quarter of it past degree 15), the Legendre values of
// those steps in LDS (computed once per block, one row per degree with the
// steps contiguous).  Each entry's sums run over (l, q) in order, with the
// recurrence of the slab kernel.  The degree loop has a fixed trip count T1P
// (T1 rounded up to a multiple of 4): the degrees past T1 sum finite values
// that are never stored, and steps past a chunk's end meet zero Legendre rows.
template <typename T, int T1P>
__device__ __forceinline__ void slab_adjoint_body(const SlabArgs &a, int32_t groups_per_inst, double *cbar_u,
                                                  double *cbar_v, int64_t coef_inst_stride,
                                                  double (*Lt)[kSlabQ])
{
    constexpr int QB = T1P <= 16 ? kSlabQ : T1P <= 20 ? kSlabQ / 2 : kSlabQ / 4;   // loads in flight per thread
    const int inst = blockIdx.z * kGridYZ + blockIdx.y;   // instances over y and z (y at most 65535)
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t row = e / (2 * a.PP);
    const int rem = (int)(e - row * 2 * a.PP), uv = rem / a.PP, kl = rem - uv * a.PP;
    const bool live = e < a.slab_stride && kl < a.P;
    const T *tab = (const T *)a.slab_table;
    const int T1 = a.deg[inst * groups_per_inst] + 1;
    double acc[T1P];
#pragma unroll
    for (int m = 0; m < T1P; ++m) acc[m] = 0.0;
    for (int gl = 0; gl < groups_per_inst; ++gl) {
        const int g = inst * groups_per_inst + gl;
        const int nstar = a.nstar[g];
        const double span = a.span[g], delta = a.delta[g], h2 = a.h2[g];
        const T *src = tab + a.slab_off[g] + (live ? e : 0);
        for (int q0 = 0; q0 < nstar; q0 += kSlabQ) {
            const int qn = min(kSlabQ, nstar - q0);
            __syncthreads();   // the previous chunk's reads of Lt are over
            if ((int)threadIdx.x < kSlabQ) {
                const int j = threadIdx.x;
                const double xi = h2 * (span - (double)(q0 + j) * delta) - 1.0;
                double lp = 0.0, lc = 1.0;
#pragma unroll 1
                for (int m = 0; m < T1P; ++m) {   // rolled: the recurrence constants stay out of registers
                    Lt[m][j] = j < qn ? lc : 0.0;
                    const double nx = c_rec.ad[m] * xi * lc - c_rec.bd[m] * lp;
                    lp = lc;
                    lc = nx;
                }
            }
            __syncthreads();
            if (!live) continue;
#pragma unroll
            for (int j0 = 0; j0 < kSlabQ; j0 += QB) {
                double v[QB];
#pragma unroll
                for (int j = 0; j < QB; ++j)   // past the chunk's end: a finite entry against zero rows of Lt
                    v[j] = (double)src[(int64_t)(q0 + min(j0 + j, qn - 1)) * a.slab_stride];
#pragma unroll
                for (int m = 0; m < T1P; ++m) {
                    const double2 *lm = (const double2 *)(Lt[m] + j0);
#pragma unroll
                    for (int jj = 0; jj < QB / 2; ++jj) {
                        const double2 l2 = lm[jj];
                        acc[m] = fma(v[2 * jj], l2.x, acc[m]);
                        acc[m] = fma(v[2 * jj + 1], l2.y, acc[m]);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);   // the next batch's loads after this batch's sums
            }
        }
    }
    if (!live) return;
    double *out = (uv ? cbar_v : cbar_u) + (int64_t)inst * coef_inst_stride + (row * a.P + kl) * T1;
#pragma unroll
    for (int m = 0; m < T1P; ++m)
        if (m < T1) out[m] = acc[m];
}

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
slab_adjoint_kernel(SlabArgs a, int32_t groups_per_inst, int32_t n_inst,
                                                           double *__restrict__ cbar_u, double *__restrict__ cbar_v,
                                                           int64_t coef_inst_stride)
{
    __shared__ __align__(16) double Lt[kMaxDeg + 1][kSlabQ];
    if ((int)(blockIdx.z * kGridYZ + blockIdx.y) >= n_inst) return;
    switch ((a.deg[(blockIdx.z * kGridYZ + blockIdx.y) * groups_per_inst] + 4) >> 2) {   // ceil(T1 / 4), T1 <= 32
    case 1: slab_adjoint_body<T, 4>(a, groups_per_inst, cbar_u, cbar_v, coef_inst_stride, Lt); break;
    case 2: slab_adjoint_body<T, 8>(a, groups_per_inst, cbar_u, cbar_v, coef_inst_stride, Lt); break;
    case 3: slab_adjoint_body<T, 12>(a, groups_per_inst, cbar_u, cbar_v, coef_inst_stride, Lt); break;
    case 4: slab_adjoint_body<T, 16>(a, groups_per_inst, cbar_u, cbar_v, coef_inst_stride, Lt); break;
    case 5: slab_adjoint_body<T, 20>(a, groups_per_inst, cbar_u, cbar_v, coef_inst_stride, Lt); break;
    case 6: slab_adjoint_body<T, 24>(a, groups_per_inst, cbar_u, cbar_v, coef_inst_stride, Lt); break;
    case 7: slab_adjoint_body<T, 28>(a, groups_per_inst, cbar_u, cbar_v, coef_inst_stride, Lt); break;
    default: slab_adjoint_body<T, 32>(a, groups_per_inst, cbar_u, cbar_v, coef_inst_stride, Lt); break;
    }
}

hipError_t launch_slab_adjoint(const SlabArgs &a, int32_t groups_per_inst, int32_t n_inst, int fp32, double *cbar_u,
                               double *cbar_v, int64_t coef_inst_stride, hipStream_t s)
{
    if (n_inst <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.slab_stride + 255) / 256), (unsigned)std::min<int32_t>(n_inst, kGridYZ),
              (unsigned)((n_inst + kGridYZ - 1) / kGridYZ)), block(256);
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
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int l = 0; l < T1; ++l) s += lambda[r * T1 + l];
        out[r] = s;
    }
}

hipError_t launch_column_sum(const double *lambda, int64_t rows, int T1, double *out, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(column_sum_kernel, dim3(grid_blocks(rows, 256)), dim3(256), 0, s, lambda, rows, T1, out);
    return hipGetLastError();
}

__global__ void axpy_kernel(double *__restrict__ y, const double *__restrict__ x, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += x[i];
}

hipError_t launch_axpy(double *y, const double *x, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(axpy_kernel, dim3(grid_blocks(n, 256)), dim3(256), 0, s, y, x, n);
    return hipGetLastError();
}

}  // namespace hpsmc
