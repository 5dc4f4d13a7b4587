// FP64 kernels of the plain single-query path.
//
// Local phase (Algorithm 3's queue phase, run level-synchronously): the
// frontier S^(j) (Section 4.2) is pushed simultaneously.  A snapshot kernel
// takes every frontier residue x_v (r(v) <- 0, pi(v) += alpha x_v); a push
// kernel then adds (1-alpha) x_v / d_v to every out-neighbour with FP64
// atomics.  Residues only grow during the push, so exactly one atomic add
// carries r(u) across the activity threshold d_u * rmax (strict >, Section
// 3.2); that lane appends u to S^(j+1) with a wave-aggregated append
// (ballot, popcount, one atomic per wave, mbcnt for the lane's slot).
//
// Global phase: pull-form sweeps over the in-edge lists.  With rmax = 0 every
// node pushes (Simultaneous Forward Push, Eq. 7): r'(u) = sum_{v in N_in(u)}
// y(v) with y(v) = (1-alpha) r(v) / d_v, and pi(u) += alpha r(u).  A sweep can
// fold the alpha-part of the *next* push into pi right away (pi(u) +=
// alpha r'(u)), so consecutive sweeps need not store r at all: a run of K
// sweeps is ENTRY|FOLD, FOLD x (K-2), WRITE_R, and adds exactly
// sum_{k<K} alpha r^(k) to pi.
#include "ppr_internal.h"

namespace ppr {
namespace k {

namespace {

constexpr int kBlock = 256;
constexpr int kPartsFixed = 1024;   // fixed grid of the n-wide reductions (deterministic)

__device__ inline double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum: wave sums, then wave 0 adds the wave results in order.
__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        int nw = blockDim.x >> 6;
        for (int i = 0; i < nw; ++i) t += sh[i];
    }
    __syncthreads();
    return t;   // valid in thread 0
}

__global__ void init_kernel(double* __restrict__ r, double* __restrict__ pi, int32_t n, int32_t s,
                            int32_t* __restrict__ F) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        r[i] = (i == s) ? 1.0 : 0.0;
        pi[i] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) F[0] = s;
}

__global__ void snapshot_kernel(const int32_t* __restrict__ F, int32_t nf, const int32_t* __restrict__ deg,
                                double alpha, double* __restrict__ r, double* __restrict__ pi,
                                double* __restrict__ X, int64_t* __restrict__ degF,
                                double* __restrict__ partials) {
    __shared__ double sh[kBlock / 64];
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    double taken = 0.0;
    if (i < nf) {
        int32_t v = F[i];
        // exchange rather than read-then-zero: a node listed twice would push once
        double x = atomicExch(&r[v], 0.0);
        pi[v] += alpha * x;
        taken = alpha * x;
        int32_t d = deg[v];
        X[i] = ((1.0 - alpha) * x) / (double)d;
        degF[i] = d;
    }
    double t = block_sum(taken, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// First index i in [0, len) with a[i] > key, minus one (a ascending, a[0] = 0 <= key).
__device__ inline int32_t find_owner(const int64_t* __restrict__ a, int32_t len, int64_t key) {
    int32_t lo = 0, hi = len;   // invariant: a[lo] <= key < a[hi] (a[len] = total > key)
    while (hi - lo > 1) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= key) lo = mid; else hi = mid;
    }
    return lo;
}

// First index i in [lo, hi] with a[i] <= key < a[i+1], given a[lo] <= key and
// key < a[hi + 1].
__device__ inline int64_t find_owner_between(const int64_t* __restrict__ a, int64_t lo, int64_t hi, int64_t key) {
    int64_t h = hi + 1;
    while (h - lo > 1) {
        int64_t mid = lo + ((h - lo) >> 1);
        if (a[mid] <= key) lo = mid; else h = mid;
    }
    return lo;
}

// Edge slot t of the frontier's out-edges: r(u) += X (FP64 atomic); the lane
// whose add carries r(u) across d_u rmax appends u.  Persistent blocks take
// 256 consecutive slots per round; a round's appended nodes are counted in
// LDS and reserve their entries with one global atomic per block and round,
// and the appended volume reaches ctr[1] once per block (global atomics per
// wave serialize on the two counter addresses when most waves append).
__global__ __launch_bounds__(kBlock) void push_kernel(
        const int32_t* __restrict__ F, const int64_t* __restrict__ off, int32_t nf, int64_t vol,
        const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
        const int32_t* __restrict__ deg, const double* __restrict__ X, double rmax,
        double* __restrict__ r, int32_t* __restrict__ F_next, unsigned long long* __restrict__ ctr) {
    __shared__ int64_t s_lo, s_hi;
    __shared__ unsigned long long s_base, s_vol;
    __shared__ unsigned int s_n;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x == 0) {
        s_n = 0u;
        s_vol = 0ull;
    }
    if (off[nf] < vol) vol = off[nf];   // never address past the frontier's last out-edge
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t0 = (int64_t)blockIdx.x * kBlock; t0 < vol; t0 += stride) {   // uniform per block
        if (threadIdx.x == 0) s_lo = find_owner(off, nf, t0);
        if (threadIdx.x == 64) s_hi = find_owner(off, nf, min(t0 + kBlock, vol) - 1);
        __syncthreads();
        const int64_t lo = s_lo, hi = s_hi;
        const int64_t t = t0 + threadIdx.x;
        bool crossed = false;
        int32_t u = 0;
        int32_t du = 0;
        if (t < vol) {
            const int64_t i = find_owner_between(off, lo, hi, t);
            int32_t v = F[i];
            int64_t e = row_ptr[v] + (t - off[i]);
            u = col[e];
            double x = X[i];
            double old = atomicAdd(&r[u], x);
            double now = old + x;
            du = deg[u];
            double thr = (double)du * rmax;
            crossed = (old <= thr) && (now > thr);
        }
        const uint64_t mask = __ballot(crossed);
        const int leader = mask ? __ffsll((unsigned long long)mask) - 1 : 0;
        unsigned int woff = 0u;
        if (mask) {
            // sum of out-degrees of the appended nodes (volume of S^(j+1))
            int64_t myvol = crossed ? du : 0;
            for (int o = 32; o >= 1; o >>= 1) myvol += __shfl_xor(myvol, o, 64);
            if (lane == leader) {
                woff = atomicAdd(&s_n, (unsigned int)__popcll(mask));
                atomicAdd(&s_vol, (unsigned long long)myvol);
            }
        }
        __syncthreads();                             // the round's appended nodes are counted
        if (threadIdx.x == 0) {
            const unsigned int tot = s_n;
            s_n = 0u;
            s_base = tot ? atomicAdd(&ctr[0], (unsigned long long)tot) : 0ull;
        }
        __syncthreads();                             // s_base: the round's first entry
        if (mask) {
            woff = __shfl(woff, leader, 64);
            unsigned int below = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
            if (crossed) F_next[s_base + woff + below] = u;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_vol) atomicAdd(&ctr[1], s_vol);
}

__global__ void prep_kernel(const double* __restrict__ r, const int32_t* __restrict__ deg, double alpha,
                            int32_t n, double* __restrict__ y, double* __restrict__ partials) {
    __shared__ double sh[kBlock / 64];
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double x = r[i];
        s += x;
        y[i] = ((1.0 - alpha) * x) / (double)deg[i];
    }
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// Epoch scan snapshot: the active test is the oracle's, r(v) > d_v * rmax in FP64.
__global__ void threshold_kernel(const int32_t* __restrict__ deg, int32_t n, double alpha, double rmax,
                                 double* __restrict__ r, double* __restrict__ pi, double* __restrict__ y,
                                 double* __restrict__ partials) {
    __shared__ double sh[kBlock / 64];
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double vol = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double x = r[i];
        const int32_t d = deg[i];
        if (x > (double)d * rmax) {
            r[i] = 0.0;
            pi[i] += alpha * x;
            y[i] = ((1.0 - alpha) * x) / (double)d;
            vol += (double)d;
        } else {
            y[i] = 0.0;
        }
    }
    double t = block_sum(vol, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void reduce_kernel(const double* __restrict__ partials, int nparts, double* __restrict__ out) {
    __shared__ double sh[1024 / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += partials[i];
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = t;
}

// ---- pull sweep (FP64, one query)
// Block b of the schedule covers rows [r0, r1).  Leading blocks (b < n_long)
// hold one long row each: all threads stride its in-edges and a fixed-order
// tree adds the partial sums.  Other blocks stage the gathered values of all
// their in-edges in LDS (the row_idx reads are coalesced), then T threads per
// row add the row's slice (T = the largest power of two with T * rows <= 256,
// at most 64, so a row's threads sit in one wave).
constexpr int kNnzCap = 2048;
constexpr int kRowCap = 256;
constexpr int kPer = kNnzCap / kBlock;

// Every thread first issues all of its index loads, then all of its gathers,
// so a wave keeps kPer independent requests in flight per lane.
__device__ inline void stage_gather(const int32_t* __restrict__ row_idx, int64_t e0, int32_t ne,
                                    const double* __restrict__ x, double* lds) {
    int32_t idx[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        int32_t i = threadIdx.x + k * kBlock;
        idx[k] = (i < ne) ? row_idx[e0 + i] : -1;
    }
    double val[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) val[k] = (idx[k] >= 0) ? x[idx[k]] : 0.0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        int32_t i = threadIdx.x + k * kBlock;
        if (i < ne) lds[i] = val[k];
    }
}

// Sum of x over the in-edges [e0, e1) of one long row by the whole block:
// four independent load chains per thread, combined in a fixed order.
__device__ inline double long_row_sum(const int32_t* __restrict__ row_idx, int64_t e0, int64_t e1,
                                      const double* __restrict__ x, double* sh) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t e = e0 + threadIdx.x;
    for (; e + 3 * kBlock < e1; e += 4 * kBlock) {
        int32_t i0 = row_idx[e], i1 = row_idx[e + kBlock], i2 = row_idx[e + 2 * kBlock],
                i3 = row_idx[e + 3 * kBlock];
        a0 += x[i0];
        a1 += x[i1];
        a2 += x[i2];
        a3 += x[i3];
    }
    for (; e < e1; e += kBlock) a0 += x[row_idx[e]];
    return block_sum((a0 + a1) + (a2 + a3), sh);
}

// Row sums sum_{v in N_in(u)} x(v) for the rows of schedule block b.  On
// return, exactly one thread per row holds (u, acc); other threads have u = -1.
template <typename OffT>
__device__ inline void pull_rows(const OffT* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
                                 const RowBlock b, bool is_long, const double* __restrict__ x,
                                 double* lds, double* sh, int32_t& u, double& acc) {
    u = -1;
    acc = 0.0;
    if (is_long) {
        acc = long_row_sum(row_idx, b.e0, b.e0 + b.ne, x, sh);
        if (threadIdx.x == 0) u = b.r0;
        return;
    }
    const int32_t r0 = b.r0, r1 = b.r1;
    const int32_t R = r1 - r0;
    int T = 64;
    while (T * R > kBlock) T >>= 1;
    const int32_t row = threadIdx.x / T;
    const int32_t sub = threadIdx.x % T;
    const int64_t e0 = b.e0;
    const int32_t ne = b.ne;
    int32_t s0 = 0, s1 = 0;
    if (row < R) {              // row bounds loaded before the gathers are waited on
        s0 = (int32_t)((int64_t)col_ptr[r0 + row] - e0);
        s1 = (int32_t)((int64_t)col_ptr[r0 + row + 1] - e0);
    }
    stage_gather(row_idx, e0, ne, x, lds);
    __syncthreads();
    for (int32_t i = s0 + sub; i < s1; i += T) acc += lds[i];
    for (int o = T >> 1; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (row < R && sub == 0) u = r0 + row;
}

// acc_in (nullable): the row sums of the earlier source slices, added first
// and reset to 0 for the next sweep (the last slice's pass of a sliced sweep).
template <typename OffT, int FLAGS>
__global__ __launch_bounds__(kBlock) void sweep_kernel(
        const OffT* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
        const int32_t* __restrict__ deg, const RowBlock* __restrict__ blocks, int32_t n_long,
        const double* __restrict__ y_in, double* __restrict__ y_out, double* __restrict__ pi,
        const double* r_in, double* r_out, double alpha,   // r_in and r_out may alias
        double* __restrict__ partials, double* __restrict__ acc_in) {
    __shared__ double lds[kNnzCap];
    __shared__ double sh[kBlock / 64];
    const double oma = 1.0 - alpha;
    int32_t u;
    double acc;
    pull_rows<OffT>(col_ptr, row_idx, blocks[blockIdx.x], (int32_t)blockIdx.x < n_long, y_in, lds, sh, u,
                    acc);
    double contrib = 0.0;
    if (u >= 0) {
        if (acc_in) {
            acc = acc_in[u] + acc;
            acc_in[u] = 0.0;
        }
        if (FLAGS & SW_ENTRY) pi[u] += alpha * r_in[u];
        if (FLAGS & SW_FOLD) pi[u] += alpha * acc;
        if (FLAGS & SW_ACCUM) {
            const double nr = r_in[u] + acc;
            r_out[u] = nr;
            contrib = nr;
        } else {
            if (FLAGS & SW_WRITE_R) r_out[u] = acc;
            y_out[u] = (oma * acc) / (double)deg[u];
            contrib = acc;
        }
    }
    double t = block_sum(contrib, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// One source slice's pass of a sliced sweep (not the last): over the slice's
// listed rows (those with in-edges in it; list position k holds row rows[k]),
// each row's sum over its in-edges in the slice added to acc[row].  acc is 0
// at the start of a sweep (the last pass resets it).  A zero sum is not added
// (every y is >= 0, so that changes no bit).
template <typename OffT>
__global__ __launch_bounds__(kBlock) void slice_pass_kernel(
        const OffT* __restrict__ col_ptr, const int32_t* __restrict__ row_idx, const int32_t* __restrict__ rows,
        const RowBlock* __restrict__ blocks, int32_t n_long, const double* __restrict__ y_in,
        double* __restrict__ acc) {
    __shared__ double lds[kNnzCap];
    __shared__ double sh[kBlock / 64];
    int32_t k;
    double a;
    pull_rows<OffT>(col_ptr, row_idx, blocks[blockIdx.x], (int32_t)blockIdx.x < n_long, y_in, lds, sh, k, a);
    if (k < 0 || a == 0.0) return;
    acc[rows[k]] += a;
}

// ---- residual certificate (FP64): q(v) = pi(v) / d_v gathered over in-edges,
// rt(u) = e_s(u) - (pi(u) - (1-alpha) sum_{v in N_in(u)} q(v)) / alpha, and
// per-block sums of |rt|.  Same block structure as the sweep.
__global__ void q_kernel(const double* __restrict__ pi, const int32_t* __restrict__ deg, int32_t n,
                         double* __restrict__ q) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        q[i] = pi[i] / (double)deg[i];
}

template <typename OffT>
__global__ __launch_bounds__(kBlock) void cert_kernel(
        const OffT* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
        const RowBlock* __restrict__ blocks, int32_t n_long, const double* __restrict__ q,
        const double* __restrict__ pi, int32_t src, double alpha, double* __restrict__ rt_out,
        double* __restrict__ partials) {
    __shared__ double lds[kNnzCap];
    __shared__ double sh[kBlock / 64];
    int32_t u;
    double acc;
    pull_rows<OffT>(col_ptr, row_idx, blocks[blockIdx.x], (int32_t)blockIdx.x < n_long, q, lds, sh, u, acc);
    double contrib = 0.0;
    if (u >= 0) {
        double rt = (u == src ? 1.0 : 0.0) - (pi[u] - (1.0 - alpha) * acc) / alpha;
        if (rt_out) rt_out[u] = rt;
        contrib = fabs(rt);
    }
    double t = block_sum(contrib, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename OffT>
void launch_sweep(const Graph& g, const Schedule& sch, int flags, double alpha, const double* y_in,
                  double* y_out, double* pi, const double* r_in, double* r_out, double* partials,
                  hipStream_t s, double* acc) {
    const bool sliced = acc != nullptr && g.fp64_slices > 1;
    const OffT* cp = g.col_ptr.as<const OffT>();
    const int32_t* ri = g.row_idx.as<int32_t>();
    const Schedule* fin = &sch;
    if (sliced) {
        // passes over the source slices but the last, each gathering from its
        // S-th of y_in, the row sums collected in acc
        const int32_t S = g.fp64_slices;
        ri = g.sl_idx.as<int32_t>();
        for (int32_t sl = 0; sl + 1 < S; ++sl) {
            const Schedule& ss = *g.sl_sched[(size_t)sl];
            if (ss.n_blocks == 0) continue;                 // no in-edge has its source in the slice
            const int64_t f = g.sl_first[(size_t)sl];
            hipLaunchKernelGGL((slice_pass_kernel<OffT>), dim3((unsigned)ss.n_blocks), dim3(kBlock), 0, s,
                               g.sl_cptr.as<const OffT>() + f, ri, g.sl_rows.as<const int32_t>() + f,
                               ss.blocks.as<const RowBlock>(), ss.n_long, y_in, acc);
        }
        fin = g.sl_sched.back().get();
        cp = g.sl_last.as<const OffT>();
    }
    const RowBlock* bl = fin->blocks.as<const RowBlock>();
    double* acc_in = sliced ? acc : nullptr;
    dim3 grid((unsigned)fin->n_blocks), blk(kBlock);
#define PPR_SWEEP_CASE(F)                                                                        \
    case F:                                                                                      \
        hipLaunchKernelGGL((sweep_kernel<OffT, F>), grid, blk, 0, s, cp, ri,                      \
                           g.deg.as<int32_t>(), bl, fin->n_long, y_in, y_out, pi, r_in, r_out,    \
                           alpha, partials, acc_in);                                             \
        break;
    switch (flags) {
        PPR_SWEEP_CASE(0)
        PPR_SWEEP_CASE(SW_FOLD)
        PPR_SWEEP_CASE(SW_ENTRY | SW_FOLD)
        PPR_SWEEP_CASE(SW_WRITE_R)
        PPR_SWEEP_CASE(SW_ENTRY | SW_WRITE_R)
        PPR_SWEEP_CASE(SW_ACCUM)
        default:
            fail(PPR_ERR_ARG, "unsupported sweep flags");
    }
#undef PPR_SWEEP_CASE
    HIPCHECK(hipGetLastError());
}

inline unsigned grid_for(int64_t items) {
    int64_t g = (items + kBlock - 1) / kBlock;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

int32_t sweep_nnz_cap() { return kNnzCap; }
int32_t sweep_row_cap() { return kRowCap; }

void query_init(double* r, double* pi, int32_t n, int32_t s_node, int32_t* F, hipStream_t st) {
    unsigned g = grid_for(n);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(init_kernel, dim3(g), dim3(kBlock), 0, st, r, pi, n, s_node, F);
    HIPCHECK(hipGetLastError());
}

void frontier_snapshot(const int32_t* F, int32_t nf, const int32_t* deg, double alpha, double* r,
                       double* pi, double* X, int64_t* degF, double* partials, int* nparts,
                       hipStream_t s) {
    unsigned g = grid_for(nf);
    hipLaunchKernelGGL(snapshot_kernel, dim3(g), dim3(kBlock), 0, s, F, nf, deg, alpha, r, pi, X, degF,
                       partials);
    HIPCHECK(hipGetLastError());
    *nparts = (int)g;
}

void frontier_push(const int32_t* F, const int64_t* off, int32_t nf, int64_t vol,
                   const int64_t* row_ptr, const int32_t* col, const int32_t* deg, const double* X,
                   double rmax, double* r, int32_t* F_next, int64_t* ctr, hipStream_t s) {
    if (vol <= 0) return;
    unsigned g = grid_for(vol);
    if (g > 2048) g = 2048;             // persistent: 8 blocks per CU of a 256-CU device
    hipLaunchKernelGGL(push_kernel, dim3(g), dim3(kBlock), 0, s, F, off, nf, vol, row_ptr, col, deg, X,
                       rmax, r, F_next, reinterpret_cast<unsigned long long*>(ctr));
    HIPCHECK(hipGetLastError());
}

void prep_y(const double* r, const int32_t* deg, double alpha, int32_t n, double* y, double* partials,
            int* nparts, hipStream_t s) {
    hipLaunchKernelGGL(prep_kernel, dim3(kPartsFixed), dim3(kBlock), 0, s, r, deg, alpha, n, y, partials);
    HIPCHECK(hipGetLastError());
    *nparts = kPartsFixed;
}

void threshold_snapshot(const int32_t* deg, int32_t n, double alpha, double rmax, double* r, double* pi,
                        double* y, double* partials, int* nparts, hipStream_t s) {
    hipLaunchKernelGGL(threshold_kernel, dim3(kPartsFixed), dim3(kBlock), 0, s, deg, n, alpha, rmax, r, pi, y,
                       partials);
    HIPCHECK(hipGetLastError());
    *nparts = kPartsFixed;
}

void reduce_sum(const double* partials, int nparts, double* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, s, partials, nparts, out);
    HIPCHECK(hipGetLastError());
}

void sweep_f64(const Graph& g, const Schedule& sch, int flags, double alpha, const double* y_in,
               double* y_out, double* pi, const double* r_in, double* r_out, double* partials,
               hipStream_t s, double* acc) {
    if (g.off64)
        launch_sweep<int64_t>(g, sch, flags, alpha, y_in, y_out, pi, r_in, r_out, partials, s, acc);
    else
        launch_sweep<uint32_t>(g, sch, flags, alpha, y_in, y_out, pi, r_in, r_out, partials, s, acc);
}

int sweep_parts(const Schedule& sch) { return sch.n_blocks; }
int sweep_parts(const Graph& g, const Schedule& sch, const double* acc) {
    return (acc != nullptr && g.fp64_slices > 1) ? g.sl_sched.back()->n_blocks : sch.n_blocks;
}

void cert_f64(const Graph& g, const Schedule& sch, double alpha, int32_t src, const double* pi,
              double* q, double* rt_out, double* partials, hipStream_t s) {
    unsigned gq = grid_for(g.n);
    if (gq > 4096) gq = 4096;
    hipLaunchKernelGGL(q_kernel, dim3(gq), dim3(kBlock), 0, s, pi, g.deg.as<int32_t>(), g.n, q);
    dim3 grid((unsigned)sch.n_blocks), blk(kBlock);
    if (g.off64)
        hipLaunchKernelGGL((cert_kernel<int64_t>), grid, blk, 0, s, g.col_ptr.as<int64_t>(),
                           g.row_idx.as<int32_t>(), sch.blocks.as<RowBlock>(), sch.n_long, q, pi, src,
                           alpha, rt_out, partials);
    else
        hipLaunchKernelGGL((cert_kernel<uint32_t>), grid, blk, 0, s, g.col_ptr.as<uint32_t>(),
                           g.row_idx.as<int32_t>(), sch.blocks.as<RowBlock>(), sch.n_long, q, pi, src,
                           alpha, rt_out, partials);
    HIPCHECK(hipGetLastError());
}

}  // namespace k
}  // namespace ppr
