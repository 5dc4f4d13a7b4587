// Approximate SSPPR: SpeedPPR (Section 6, Algorithm 4) on the FP64 path.
//
//   W       = 2 (2 eps / 3 + 2) ln n / (eps^2 mu)                    (Eq. 8)
//   phase 1: PowerPush to lambda = m / W (the high-precision path), then the
//            refinement: no node active w.r.t. rmax = 1 / W, taken
//            level-synchronously with the local phase's frontier kernels
//            (every active node pushes at once; a node joins the next level
//            when an atomic add carries it across d_u rmax);
//   phase 2: every v with r(v) > 0 runs W_v = ceil(r(v) W) alpha-random walks
//            (at most d_v after the refinement; capped at d_v for the rounding
//            of r(v) W), and a walk that stops at u adds r(v) / W_v to
//            pi_hat(u)                                                  (Eqs. 9-10).
//
// Walks are counter-based: walk j from v draws from SplitMix64 seeded with
// b = splitmix(seed ^ splitmix(v << 32 | j)); step t uses draw 2t for the stop
// test (top 53 bits as a uniform in [0, 1), stop when < alpha) and draw 2t + 1
// for the next node (index (top 32 bits * d) >> 32 among the out-edges).  A
// walk therefore depends only on (seed, v, j): one thread per walk in any
// order, and the index of pre-computed walks (walk j of v for every j < d_v,
// m in all, stored at CSR offset row_ptr[v] + j) reproduces exactly the walks
// an index-free query would take with the same seed.
#include <chrono>
#include <cmath>

#include "ppr_internal.h"

namespace ppr {

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ inline uint64_t splitmix(uint64_t z) {
    z += kGamma;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline int32_t walk_from(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                    double alpha, uint64_t seed, int32_t v, uint32_t j) {
    const uint64_t b = splitmix(seed ^ splitmix(((uint64_t)(uint32_t)v << 32) | (uint64_t)j));
    int32_t cur = v;
    for (int32_t t = 0; t < kMaxWalkSteps; ++t) {
        const uint64_t x = splitmix(b + (uint64_t)(2 * t) * kGamma);
        if ((double)(x >> 11) * 0x1p-53 < alpha) break;
        const uint64_t y = splitmix(b + (uint64_t)(2 * t + 1) * kGamma);
        const int64_t e0 = row_ptr[cur];
        const uint64_t d = (uint64_t)(row_ptr[cur + 1] - e0);
        cur = col[e0 + (int64_t)(((y >> 32) * d) >> 32)];
    }
    return cur;
}

// Largest i in [0, len) with a[i] <= key (a ascending, a[0] = 0 <= key < a[len]).
__device__ inline int32_t owner_of(const int64_t* __restrict__ a, int32_t len, int64_t key) {
    int32_t lo = 0, hi = len;
    while (hi - lo > 1) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= key) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Frontier of the refinement: every v with r(v) > d_v rmax, in node order.
// Two passes over fixed node ranges (kCompactBlocks blocks): count the
// active nodes and their volume per block, scan, then write each block's
// nodes at its offset (wave ballots and a block prefix in LDS; no atomics).
constexpr int kCompactBlocks = 1024;

__device__ inline void compact_range(int32_t n, int64_t& lo, int64_t& hi) {
    const int64_t per = ((int64_t)n + kCompactBlocks - 1) / kCompactBlocks;
    lo = std::min<int64_t>((int64_t)blockIdx.x * per, n);
    hi = std::min<int64_t>(lo + per, n);
}

__global__ __launch_bounds__(kBlock) void active_count_kernel(const double* __restrict__ r,
                                                              const int32_t* __restrict__ deg, int32_t n,
                                                              double rmax, int64_t* __restrict__ cnt,
                                                              int64_t* __restrict__ vol) {
    __shared__ int64_t sc[kBlock / 64], sv[kBlock / 64];
    int64_t lo, hi;
    compact_range(n, lo, hi);
    int64_t c = 0, w = 0;
    for (int64_t v = lo + threadIdx.x; v < hi; v += kBlock) {
        const int32_t d = deg[v];
        if (r[v] > (double)d * rmax) {
            c += 1;
            w += d;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        w += __shfl_xor(w, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sc[threadIdx.x >> 6] = c;
        sv[threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tc = 0, tw = 0;
        for (int i = 0; i < kBlock / 64; ++i) {
            tc += sc[i];
            tw += sv[i];
        }
        cnt[blockIdx.x] = tc;
        vol[blockIdx.x] = tw;
    }
}

__global__ __launch_bounds__(kBlock) void active_write_kernel(const double* __restrict__ r,
                                                              const int32_t* __restrict__ deg, int32_t n,
                                                              double rmax, const int64_t* __restrict__ off,
                                                              int32_t* __restrict__ F) {
    __shared__ int64_t wcount[kBlock / 64];
    int64_t lo, hi;
    compact_range(n, lo, hi);
    int64_t base = off[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t v0 = lo; v0 < hi; v0 += kBlock) {         // uniform for the block
        const int64_t v = v0 + threadIdx.x;
        const bool act = v < hi && r[v] > (double)deg[v] * rmax;
        const uint64_t mask = __ballot(act);
        if (lane == 0) wcount[wave] = __popcll(mask);
        __syncthreads();
        int64_t before = 0, total = 0;
        for (int i = 0; i < kBlock / 64; ++i) {
            if (i < wave) before += wcount[i];
            total += wcount[i];
        }
        const unsigned below = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
        if (act) F[base + before + below] = (int32_t)v;
        base += total;
        __syncthreads();                                     // wcount is rewritten next round
    }
}

// W_v = min(ceil(r(v) W), d_v) for r(v) > 0, else 0.
__global__ void walk_count_kernel(const double* __restrict__ r, const int32_t* __restrict__ deg, int32_t n, double W,
                                  int64_t* __restrict__ cnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const double x = r[v];
        int64_t c = 0;
        if (x > 0.0) {
            const double w = ceil(x * W);
            const double d = (double)deg[v];
            c = (int64_t)(w > d ? d : w);
        }
        cnt[v] = c;
    }
}

// One thread per walk t < off[n]: its node v (off[v] <= t < off[v + 1]), its
// index j = t - off[v], its stop node (walked, or read from the index), and
// pi(u) += r(v) / W_v.
__global__ __launch_bounds__(kBlock) void walk_kernel(const int64_t* __restrict__ off, int32_t n,
                                                      const double* __restrict__ r,
                                                      const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, double alpha, uint64_t seed,
                                                      const int32_t* __restrict__ index, double* __restrict__ pi) {
    const int64_t total = off[n];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int32_t v = owner_of(off, n, t);
        const int64_t j = t - off[v];
        const int64_t wv = off[v + 1] - off[v];
        const int32_t u = index ? index[row_ptr[v] + j] : walk_from(row_ptr, col, alpha, seed, v, (uint32_t)j);
        atomicAdd(&pi[u], r[v] / (double)wv);
    }
}

// The index: walk j of v for every j < d_v, at CSR offset row_ptr[v] + j.
__global__ __launch_bounds__(kBlock) void index_kernel(const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col, int32_t n, int64_t m,
                                                       double alpha, uint64_t seed, int32_t* __restrict__ index) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += stride) {
        const int32_t v = owner_of(row_ptr, n, t);
        index[t] = walk_from(row_ptr, col, alpha, seed, v, (uint32_t)(t - row_ptr[v]));
    }
}

unsigned grid_for(int64_t items) {
    int64_t g = (items + kBlock - 1) / kBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

struct Lease {
    Graph& g;
    std::unique_ptr<QueryCtx> c;
    explicit Lease(Graph& gg) : g(gg), c(ctx_acquire(gg)) {}
    ~Lease() {
        if (c) {
            (void)hipStreamSynchronize(c->stream);
            ctx_release(g, std::move(c));
        }
    }
};

// A level whose frontier moves more than m / kPullRatio edges runs in pull
// form: one threshold scan over the in-edge lists (every active node pushes
// at once, as in the push form, with no atomics; about one sweep of time),
// then the next frontier by compaction.  Smaller frontiers push along their
// out-edges with FP64 atomics.  On the 4M/70M graph (eps = 0.5) the
// refinement took 25.8 / 17.1 / 21.0 ms with ratios 8 / 32 / 128.
constexpr int64_t kPullRatio = 32;

// Refinement in place on c.r / c.pi (device): level-synchronous pushes of the
// active nodes until none is active.
void refine(Graph& g, QueryCtx& c, double alpha, double rmax, int32_t* levels_out, int64_t* edges_out) {
    hipStream_t ss = c.stream;
    int64_t* hctr = c.host.as<int64_t>();
    auto* ctr = c.ctr.as<int64_t>();
    int32_t* F = c.F0.as<int32_t>();
    int32_t* Fn = c.F1.as<int32_t>();
    auto frontier = [&](int32_t* out) { active_set(g, c, rmax, out, &hctr[0], &hctr[1]); };
    frontier(F);
    int64_t nf = hctr[0], vol = hctr[1];
    int32_t levels = 0;
    int64_t edges = 0;
    const Schedule& sch = g.schedule(k::sweep_nnz_cap(), k::sweep_row_cap());
    // pull levels sweep over the source slices (if the graph has them): their
    // row sums start from 0
    if (c.acc.p) HIPCHECK(hipMemsetAsync(c.acc.p, 0, c.acc.bytes, ss));
    while (nf > 0) {
        if (vol * kPullRatio > g.m) {
            int np = 0;
            k::threshold_snapshot(g.deg.as<int32_t>(), g.n, alpha, rmax, c.r.as<double>(), c.pi.as<double>(),
                                  c.y0.as<double>(), c.partials.as<double>(), &np, ss);
            k::sweep_f64(g, sch, k::SW_ACCUM, alpha, c.y0.as<double>(), nullptr, c.pi.as<double>(),
                         c.r.as<double>(), c.r.as<double>(), c.partials.as<double>(), ss, c.acc.as<double>());
            edges += vol;
            ++levels;
            frontier(F);
            nf = hctr[0];
            vol = hctr[1];
            continue;
        }
        int np = 0;
        k::frontier_snapshot(F, (int32_t)nf, g.deg.as<int32_t>(), alpha, c.r.as<double>(), c.pi.as<double>(),
                             c.X.as<double>(), c.degF.as<int64_t>(), c.partials.as<double>(), &np, ss);
        k::exclusive_scan_i64(c.degF.as<int64_t>(), c.off.as<int64_t>(), nf, c.scan_tmp.p, ss);
        HIPCHECK(hipMemsetAsync(c.ctr.p, 0, 16, ss));
        k::frontier_push(F, c.off.as<int64_t>(), (int32_t)nf, vol, g.row_ptr.as<int64_t>(), g.col.as<int32_t>(),
                         g.deg.as<int32_t>(), c.X.as<double>(), rmax, c.r.as<double>(), Fn, ctr, ss);
        HIPCHECK(hipMemcpyAsync(hctr, ctr, 16, hipMemcpyDeviceToHost, ss));
        HIPCHECK(hipStreamSynchronize(ss));
        edges += vol;
        nf = hctr[0];
        vol = hctr[1];
        std::swap(F, Fn);
        ++levels;
    }
    if (levels_out) *levels_out = levels;
    if (edges_out) *edges_out = edges;
}

// Monte Carlo phase on c.r (device) into c.pi (device).  Returns the walks.
int64_t walks(Graph& g, QueryCtx& c, double alpha, double W, uint64_t seed, const int32_t* index) {
    hipStream_t ss = c.stream;
    int64_t* cnt = c.degF.as<int64_t>();     // int64[n]
    int64_t* off = c.off.as<int64_t>();      // int64[n + 1]
    hipLaunchKernelGGL(walk_count_kernel, dim3(grid_for(g.n)), dim3(kBlock), 0, ss, c.r.as<double>(),
                       g.deg.as<int32_t>(), g.n, W, cnt);
    HIPCHECK(hipGetLastError());
    k::exclusive_scan_i64(cnt, off, g.n, c.scan_tmp.p, ss);
    int64_t* hctr = c.host.as<int64_t>();
    HIPCHECK(hipMemcpyAsync(hctr, off + g.n, 8, hipMemcpyDeviceToHost, ss));
    HIPCHECK(hipStreamSynchronize(ss));
    const int64_t total = hctr[0];
    if (total > 0) {
        hipLaunchKernelGGL(walk_kernel, dim3(grid_for(total)), dim3(kBlock), 0, ss, off, g.n, c.r.as<double>(),
                           g.row_ptr.as<int64_t>(), g.col.as<int32_t>(), alpha, seed, index, c.pi.as<double>());
        HIPCHECK(hipGetLastError());
    }
    HIPCHECK(hipStreamSynchronize(ss));
    return total;
}

const int32_t* index_for(const Graph& g, double alpha, uint64_t seed, bool use) {
    if (!use) return nullptr;
    if (!g.walk_index.p) fail(PPR_ERR_ARG, "no walk index: build one with ppr_walk_index_build");
    if (g.walk_alpha != alpha || g.walk_seed != seed)
        fail(PPR_ERR_ARG, "the walk index was built for another alpha or seed");
    return g.walk_index.as<int32_t>();
}

}  // namespace

void active_set(const Graph& g, QueryCtx& c, double rmax, int32_t* out, int64_t* count, int64_t* vol) {
    hipStream_t ss = c.stream;
    // per-block counts and volumes, then their scans
    static_assert(4 * (kCompactBlocks + 1) <= kAuxLen, "compaction scratch");
    int64_t* bc = c.aux.as<int64_t>();
    int64_t* bv = bc + kCompactBlocks;
    int64_t* oc = bv + kCompactBlocks;
    int64_t* ov = oc + kCompactBlocks + 1;
    hipLaunchKernelGGL(active_count_kernel, dim3(kCompactBlocks), dim3(kBlock), 0, ss, c.r.as<double>(),
                       g.deg.as<int32_t>(), g.n, rmax, bc, bv);
    HIPCHECK(hipGetLastError());
    k::exclusive_scan_i64(bc, oc, kCompactBlocks, c.scan_tmp.p, ss);
    k::exclusive_scan_i64(bv, ov, kCompactBlocks, c.scan_tmp.p, ss);
    if (out) {
        hipLaunchKernelGGL(active_write_kernel, dim3(kCompactBlocks), dim3(kBlock), 0, ss, c.r.as<double>(),
                           g.deg.as<int32_t>(), g.n, rmax, oc, out);
        HIPCHECK(hipGetLastError());
    }
    int64_t* h = c.host.as<int64_t>() + 6;
    HIPCHECK(hipMemcpyAsync(h, oc + kCompactBlocks, 8, hipMemcpyDeviceToHost, ss));
    HIPCHECK(hipMemcpyAsync(h + 1, ov + kCompactBlocks, 8, hipMemcpyDeviceToHost, ss));
    HIPCHECK(hipStreamSynchronize(ss));
    *count = h[0];
    *vol = h[1];
}

double walk_budget(int32_t n, double eps, double mu) {
    return 2.0 * (2.0 * eps / 3.0 + 2.0) * std::log((double)n) / (eps * eps * mu);
}

void run_approx_query(Graph& g, int32_t s, double alpha, double eps, double mu, uint64_t seed, bool use_index,
                      const ppr_options& opt, double* pi_out, ppr_approx_stats* st) {
    const auto t0 = std::chrono::steady_clock::now();
    HIPCHECK(hipSetDevice(g.device));
    const int32_t* index = index_for(g, alpha, seed, use_index);
    const double W = walk_budget(g.n, eps, mu);
    const double lambda = std::min(1.0, (double)g.m / W);
    Lease lease(g);
    QueryCtx& c = *lease.c;
    // phase 1: PowerPush to lambda = m / W (pi and r land in this context)
    ppr_stats pst;
    run_fp64_query(g, s, alpha, lambda, opt, c.pi.as<double>(), c.r.as<double>(), &pst);
    const double ms_push = ms_since(t0);
    const auto t1 = std::chrono::steady_clock::now();
    int32_t levels = 0;
    int64_t redges = 0;
    refine(g, c, alpha, 1.0 / W, &levels, &redges);
    const double ms_refine = ms_since(t1);
    // residue mass handed to the walks
    int np = 0;
    k::prep_y(c.r.as<double>(), g.deg.as<int32_t>(), alpha, g.n, c.y0.as<double>(), c.partials.as<double>(), &np,
              c.stream);
    k::reduce_sum(c.partials.as<double>(), np, c.dsum.as<double>(), c.stream);
    double* hd = c.host.as<double>();
    HIPCHECK(hipMemcpyAsync(hd + 2, c.dsum.p, 8, hipMemcpyDeviceToHost, c.stream));
    HIPCHECK(hipStreamSynchronize(c.stream));
    const double r_sum = hd[2];
    const auto t2 = std::chrono::steady_clock::now();
    const int64_t nw = walks(g, c, alpha, W, seed, index);
    const double ms_walks = ms_since(t2);
    HIPCHECK(hipMemcpyAsync(pi_out, c.pi.p, 8 * (size_t)g.n, hipMemcpyDefault, c.stream));
    HIPCHECK(hipStreamSynchronize(c.stream));
    if (st) {
        st->source = s;
        st->local_levels = pst.local_levels;
        st->sweeps = pst.sweeps;
        st->refine_levels = levels;
        st->refine_edge_pushes = redges;
        st->walks = nw;
        st->W = W;
        st->lambda = lambda;
        st->r_sum = r_sum;
        st->ms_push = ms_push;
        st->ms_refine = ms_refine;
        st->ms_walks = ms_walks;
        st->ms = ms_since(t0);
        st->used_index = index ? 1 : 0;
        st->reserved = 0;
    }
}

void build_walk_index(Graph& g, double alpha, uint64_t seed, double* ms) {
    HIPCHECK(hipSetDevice(g.device));
    const auto t0 = std::chrono::steady_clock::now();
    Lease lease(g);
    hipStream_t ss = lease.c->stream;
    if (!g.walk_index.p || g.walk_index.bytes < 4 * (size_t)g.m) g.walk_index.alloc(4 * (size_t)g.m);
    g.walk_alpha = -1.0;      // invalid until the kernel has run
    hipLaunchKernelGGL(index_kernel, dim3(grid_for(g.m)), dim3(kBlock), 0, ss, g.row_ptr.as<int64_t>(),
                       g.col.as<int32_t>(), g.n, g.m, alpha, seed, g.walk_index.as<int32_t>());
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(ss));
    g.walk_alpha = alpha;
    g.walk_seed = seed;
    if (ms) *ms = ms_since(t0);
}

void copy_walk_index(const Graph& g, int32_t* out) {
    if (!g.walk_index.p) fail(PPR_ERR_ARG, "no walk index");
    HIPCHECK(hipSetDevice(g.device));
    HIPCHECK(hipMemcpy(out, g.walk_index.p, 4 * (size_t)g.m, hipMemcpyDefault));
}

void debug_refine(Graph& g, double alpha, double rmax, double* pi, double* r, int32_t* levels, int64_t* edges) {
    HIPCHECK(hipSetDevice(g.device));
    Lease lease(g);
    QueryCtx& c = *lease.c;
    HIPCHECK(hipMemcpyAsync(c.pi.p, pi, 8 * (size_t)g.n, hipMemcpyDefault, c.stream));
    HIPCHECK(hipMemcpyAsync(c.r.p, r, 8 * (size_t)g.n, hipMemcpyDefault, c.stream));
    refine(g, c, alpha, rmax, levels, edges);
    HIPCHECK(hipMemcpyAsync(pi, c.pi.p, 8 * (size_t)g.n, hipMemcpyDefault, c.stream));
    HIPCHECK(hipMemcpyAsync(r, c.r.p, 8 * (size_t)g.n, hipMemcpyDefault, c.stream));
    HIPCHECK(hipStreamSynchronize(c.stream));
}

void debug_walks(Graph& g, double alpha, double W, uint64_t seed, bool use_index, const double* r, double* pi,
                 int64_t* nwalks) {
    HIPCHECK(hipSetDevice(g.device));
    const int32_t* index = index_for(g, alpha, seed, use_index);
    Lease lease(g);
    QueryCtx& c = *lease.c;
    HIPCHECK(hipMemcpyAsync(c.r.p, r, 8 * (size_t)g.n, hipMemcpyDefault, c.stream));
    HIPCHECK(hipMemcpyAsync(c.pi.p, pi, 8 * (size_t)g.n, hipMemcpyDefault, c.stream));
    const int64_t nw = walks(g, c, alpha, W, seed, index);
    HIPCHECK(hipMemcpyAsync(pi, c.pi.p, 8 * (size_t)g.n, hipMemcpyDefault, c.stream));
    HIPCHECK(hipStreamSynchronize(c.stream));
    if (nwalks) *nwalks = nw;
}

}  // namespace ppr
