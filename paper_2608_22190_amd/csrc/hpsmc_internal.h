// Internal declarations shared by the host runtime (hpsmc_host.cpp) and the
// gfx950 kernels (hpsmc_kernels.hip).  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hpsmc {

constexpr int kMaxDim = 5;
constexpr int kMaxN = 32;            // spatial nodes per dimension
constexpr int kMaxP = kMaxN + 2;     // Legendre modes per dimension (phi_p has degree p+2)
constexpr int kMaxDeg = 31;          // temporal degree M_n

// One Monte Carlo node (instance, interval, l >= 1, spatial node j).
struct NodeDesc {
    double x0[kMaxDim];   // spatial node
    double delta;         // Delta_{n,l} = (t_{n,l} - t_{n-1}) / N*
    double jump;          // J = sqrt(2 d Delta)
    double span;          // t_{n,l} - t_{n-1}
    double t_prev;        // t_{n-1}
    int64_t u_index;      // offset of U[inst][iv][j][l] in the nodal buffer
    int64_t slab;         // offset of the q = 0 slab of (inst, iv, l) in the slab table
    int32_t nstar;        // N*
    uint32_t c0;          // Philox counter word 0: j + n^d (l - 1)
    uint32_t c3;          // Philox counter word 3 without the tag: inst<<16 | iv<<8
    int32_t out;          // row of this node in the per-launch output arrays
};

// One (instance, interval, l) group: its nodes share the slab sequence, N*,
// Delta and J, so a block can advance any mix of their paths in lockstep.
struct GroupDesc {
    double delta, jump, span, t_prev;
    int64_t slab;          // offset of the q = 0 slab in the slab table (row layout)
    int64_t slab_mma;      // the same in the matrix-core layout (d = 2, FP32)
    int64_t path_off;      // first path slot of the group in the state buffers
    int32_t nstar;
    int32_t node_begin;    // the group's nodes are [node_begin, node_begin + node_count)
    int32_t node_count;
    uint32_t c3;           // Philox counter word 3 without the tag
};

// intervals of the start tables of the fractional walk's inverse incomplete
// beta (da, db: kFracTab + 1 values each)
constexpr int kFracTab = 256;

// Problem constants every sampling lane needs.
struct Physics {
    int32_t dim, f_kind, src_kind;
    int32_t picard;              // 1: Picard-form estimator (eq. uast)
    int32_t ball;                // 1: integrand at the step's Green's-function ball point
    int32_t frac;                // 1: fractional operator (d = 1, alpha-stable walk)
    int32_t frac_kmax, frac_K, frac_nt;  // recurrence length, source series terms, series terms of the inverse
    int32_t frac_P;              // Jacobi modes of the slab
    double frac_a;               // alpha / 2
    double frac_half;            // I_{1/2}(a, 1 - a): the branch of the inverse
    double frac_lpb1, frac_lpb2; // log(a B(a, 1-a)), log((1-a) B(1-a, a))
    const double *frac_tab;      // A[kmax], C[kmax], lambda[P], src[K], ra[nt], rb[nt], da, db, X0max[2]
    double f_param[4];
    double src_param[8];
};

// Arguments of the persistent sampling kernel.
struct SampleArgs {
    const NodeDesc *nodes;       // all nodes of this launch, in scheduling order
    int64_t n_nodes;
    int64_t M;                   // samples per node
    int32_t chunks_per_node;     // ceil(M / (64 * samples_per_lane))
    int32_t P;                   // Legendre modes per dimension
    int32_t PP;                  // padded row length of the slab (>= P, multiple of 4)
    int32_t tag;                 // iteration / sweep tag of the counter
    uint32_t key0, key1;
    const void *slab_table;      // T, rows of [u: PP][v: PP]
    int64_t slab_stride;         // elements per (inst, iv, l, q) slab
    double *part;                // [node out][chunk][2]: sum S, sum S^2
    double *probe;               // [node out][m_probe] or null
    int64_t m_probe;
    unsigned long long *work;    // work-item counter (zeroed before launch)
    unsigned long long *stats;   // [0] residual evaluations, [1] lane steps
    Physics phys;
};

// Arguments of one round of the path-advancing kernel: every live path of
// every group advances by up to `steps` walk steps, the survivors are
// compacted into the other state buffer.
struct RoundArgs {
    const GroupDesc *groups;
    const NodeDesc *nodes;
    int32_t n_groups;
    int32_t round, steps;        // steps [round*steps, (round+1)*steps)
    int32_t batch;               // paths per block work item (64 * waves * NS)
    int64_t m0, mcount;          // sample slice [m0, m0 + mcount)
    const void *state_in;
    void *state_out;
    const uint32_t *live_in;     // per group, paths in state_in (round > 0)
    uint32_t *live_out;          // per group, survivors appended to state_out
    const int64_t *batch_prefix; // [n_groups + 2] work items per group, prefix; [n_groups + 1] paths per item
    double *result;              // [node out][mcount] path value S of each sample
    int32_t n_chunks;            // LDS chunks per slab: P^cf, the first cf dimensions fixed per chunk
    int32_t cf;
    int64_t chunk_elems;         // slab elements per chunk (P^{d-1-cf} rows)
    int32_t P, PP, tag;
    uint32_t key0, key1;
    const void *slab_table;
    int64_t slab_stride;
    unsigned long long *work;    // block work counter (zeroed by the prep kernel)
    unsigned long long *stats;   // [0] residual evaluations, [1] slot steps
    Physics phys;
};

// Arguments of one round of the adjoint kernel: the forward paths of one
// iteration are regenerated and every residual evaluation scatters its
// weighted basis values into the slab-adjoint table.
struct AdjointArgs {
    RoundArgs r;                 // paths, slabs, counters (result unused)
    const double *lambda;        // nodal adjoint, U layout
    void *slab_bar;              // slab-adjoint table, slab layout, type T
    double inv_M;                // 1/M
    int32_t use_mfma;            // FP32 only: 1 outer products on the matrix cores; 2 (d = 2) u* too, from
                                 // the slabs in the matrix-core layout (r.slab_stride, GroupDesc::slab_mma)
    int64_t bar_stride;          // elements per step of the slab-adjoint table (row layout, GroupDesc::slab)
};

// Time contraction of the modal coefficients into per-step spatial slabs.
// One group = one (instance, interval, node time l).
struct SlabArgs {
    const double *cu, *cv;       // Legendre tensors, blocks of [P^d][T1]
    const double *cs;            // polynomial source, blocks of [P^d][T1] per interval (null: none);
                                 // added to v in the contraction
    const int64_t *cs_off;       // per group: offset of its interval's source block
    const int64_t *coef_off;     // per group: offset of its (inst, iv) coefficient block
    const int64_t *slab_off;     // per group: offset of its q = 0 slab in the table (row layout)
    const int64_t *slab_off_mma; // the same in the matrix-core layout (null when not available)
    int64_t mma_stride;          // elements per slab in the matrix-core layout
    int32_t layout;              // 0: rows [k0][u: PP][v: PP]; 1: matrix-core layout
    int32_t extra;               // slabs past N* per group (1 for the Picard form: q = N*, t_{n-1})
    const double *span;          // per group: t_{n,l} - t_{n-1}
    const double *delta;         // per group: Delta_{n,l}
    const double *h2;            // per group: 2 / h_n
    const int32_t *nstar;        // per group: N*
    const int32_t *deg;          // per group: M_n
    int32_t n_groups;
    int32_t P, PP, rows;         // rows = P^{d-1}
    int64_t slab_stride;         // rows * 2 * PP
    void *slab_table;
};

// Launch wrappers (hpsmc_kernels.hip).
hipError_t launch_mode_product(const double *in, double *out, int64_t outer, int len_in, int len_out,
                               int64_t inner, const double *mat, double alpha, int accumulate,
                               hipStream_t s);
hipError_t launch_slabs(const SlabArgs &a, int fp32, int max_nstar, hipStream_t s);
hipError_t launch_sample(const SampleArgs &a, int fp32, int samples_per_lane, int waves_per_block,
                         int blocks, hipStream_t s);
hipError_t launch_reduce_update(const double *part, int chunks, int mode, const NodeDesc *nodes, int64_t n_nodes,
                                int64_t M, double *U, double *eps, double *sumsq,
                                unsigned long long *maxbits, hipStream_t s);
// Aitken-relaxed update of the vectors [vbeg[v], vbeg[v+1]) of a node set
hipError_t launch_aitken(const NodeDesc *nodes, const int64_t *vbeg, int n_vec, const double *eps, double *eprev,
                         double *state, double w0, double wmin, double wmax, double *U, hipStream_t s);
hipError_t launch_start_columns(double *U, const double *src, int64_t src_stride, int64_t src_off,
                                int64_t dst_stride, int T1, int64_t count, int replicate, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s);
size_t frac_lds_bytes(int fp32, int PP, int kmax, int P, int K, int nt);
hipError_t launch_eval(const double *cu, const double *cv, int dim, int P, int T1, double t_prev, double h,
                       const double *pts, int64_t npts, double *out, hipStream_t s);
// batch_prefix: [n_groups + 2]; batch_split > 0 lets a round that fits in at
// most split_max items of batch_split paths use that batch (the 5-D
// matrix-core kernel then splits each item's products over the block's waves)
hipError_t launch_round_prep(const GroupDesc *groups, int32_t n_groups, int32_t round, int32_t steps,
                             int64_t mcount, int32_t batch, int32_t batch_split, int64_t split_max,
                             const uint32_t *live_in, uint32_t *live_out, int64_t *batch_prefix,
                             unsigned long long *work, hipStream_t s);
// kern: 0 the vector-unit kernel, 1 the 2-D matrix-core kernel, 2 the 5-D one,
// 3 the windowed 1-D kernel
hipError_t launch_advance(const RoundArgs &a, int fp32, int samples_per_lane, int waves_per_block, int blocks,
                          size_t lds_bytes, int kern, hipStream_t s);
// windowed 1-D round kernel: residual form, centre-point rule, P <= 36, 1, 2 or
// 4 paths per lane; LDS: two windows of slabs
bool advance_1d_eligible(int dim, int P, int picard, int ball, int frac, int samples_per_lane);
size_t advance_1d_lds_bytes(int fp32, int64_t slab_stride);
// matrix-core form of the round kernel: FP32, d = 2, P <= 32, whole slab per
// LDS buffer, one path per lane
bool advance_mma_eligible(int fp32, int dim, int P, int cf, int samples_per_lane, int waves_per_block);
size_t advance_mma_lds_bytes(int PP);
// matrix-core slab layout: 2 PP columns (u modes k1, then v modes k1) of
// kMmaRows rows k0 (zeros past P), stored as the kernel's LDS image; the
// coefficients are those of the Chebyshev basis T_{k0} T_{k1}
constexpr int kMmaRows = 33;
inline int64_t mma_slab_elems(int PP) { return (int64_t)2 * PP * kMmaRows; }

// Five-dimensional matrix-core slab layout.  A step's image is a sequence of
// NCH chunks, each a 32-row tile of the u coefficients followed by the same
// tile of the v coefficients.  Tile rows run over (k0, k1, k2); the
// contraction index over (k3, k4) in k-steps j = k3 HK + m, k4 = 2m + h, where
// h is the half of the wave that feeds k4's parity to the 32x32x2 product.
// Row i of a tile holds [h = 0: j < KH2][h = 1: j < KH2][4 floats pad]: RS is
// an odd multiple of 4 floats, so eight rows read as 16-byte vectors hit
// distinct bank quads.  The rows f = k1 P + k2 < 32 A of each k0 fill A main
// tiles per k0, k0-major; the B = P^2 - 32 A remaining rows of every k0 are
// gathered, k0-major, into R tiles at the end, so every P in 3..12 wastes at
// most 3% of the rows.  Entries past P (k4 of odd P) and past the last row are zero.
struct Mma5Geom {
    int P, HK, KJ, KH2, RS, A, B, R, NCH;
    int64_t chunk;   // floats per chunk (u tile, v tile)
    int64_t step;    // floats per step
};
constexpr Mma5Geom mma5_geom(int P)
{
    const int HK = (P + 1) / 2, KJ = P * HK, KH2 = (KJ + 3) & ~3, RS = 2 * KH2 + 4;
    const int A = P * P / 32, B = P * P - 32 * A, R = (B * P + 31) / 32;
    return Mma5Geom{P, HK, KJ, KH2, RS, A, B, R, P * A + R, (int64_t)64 * RS, (int64_t)(P * A + R) * 64 * RS};
}
// Element e of a step's image: false for padding, else its table (0 u, 1 v),
// the flat index row4 = ((k0 P + k1) P + k2) P + k3 of the first four modes, and k4.
__host__ __device__ inline bool mma5_source(const Mma5Geom &g, int64_t e, int &uv, int64_t &row4, int &k4)
{
    const int c = (int)(e / g.chunk);
    int r = (int)(e - (int64_t)c * g.chunk);
    uv = r / (32 * g.RS);
    r -= uv * 32 * g.RS;
    const int i = r / g.RS, col = r - i * g.RS;
    const int h = col / g.KH2, j = col - h * g.KH2;
    if (h > 1 || j >= g.KJ) return false;
    const int k3 = j / g.HK, m = j - k3 * g.HK;
    k4 = 2 * m + h;
    if (k4 >= g.P) return false;
    int k0, f;
    if (c < g.P * g.A) {
        k0 = c / g.A;
        f = 32 * (c - k0 * g.A) + i;
    } else {
        const int rr = 32 * (c - g.P * g.A) + i;
        if (rr >= g.B * g.P) return false;
        k0 = rr / g.B;
        f = 32 * g.A + (rr - k0 * g.B);
    }
    row4 = ((int64_t)k0 * g.P * g.P + f) * g.P + k3;
    return true;
}
// matrix-core form of the 5-D round kernel: FP32, 3 <= P <= 12, residual form
// with the centre-point rule, one path per lane
bool advance_mma5_eligible(int fp32, int dim, int P, int picard, int ball, int samples_per_lane, int waves_per_block);
size_t advance_mma5_lds_bytes(int P);
hipError_t launch_slice_reduce(const double *result, int64_t n_nodes, int64_t mcount, double *sums, int first,
                               hipStream_t s);
size_t path_state_bytes(int fp32, int dim);
hipError_t launch_adjoint(const AdjointArgs &a, int fp32, int waves_per_block, int blocks, size_t lds_bytes,
                          hipStream_t s);
size_t adjoint_lds_bytes(int fp32, int mfma, int dim, int P, int nthr, int64_t slab_stride);
size_t adjoint_mma2_lds_bytes(int P, int nthr);
// the 2-D adjoint with u* on the matrix cores covers KH = ceil(P/2) <= 10 (past
// that its registers spill; larger P keep u* on the vector units)
constexpr int kAdjMma2MaxKH = 10;
hipError_t launch_slab_adjoint(const SlabArgs &a, int32_t groups_per_inst, int32_t n_inst, int fp32, double *cbar_u,
                               double *cbar_v, int64_t coef_inst_stride, hipStream_t s);
hipError_t launch_loss_lambda(const double *U, const double *target, int n_inst, int64_t nsp, int T1, double *lambda,
                              double *loss, hipStream_t s);
hipError_t launch_column_sum(const double *lambda, int64_t rows, int T1, double *out, hipStream_t s);
hipError_t launch_axpy(double *y, const double *x, int64_t n, hipStream_t s);
hipError_t set_recurrence_tables();

}  // namespace hpsmc
