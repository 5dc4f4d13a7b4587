// Batched mixed-precision path: B sources as the columns of an n x B block.
//
// State (node-major, the B values of one node contiguous, so that one edge's
// gather reads one contiguous B*4-byte row):
//   Y[n][B]       FP32, y = (1 - alpha) r / d_u, the residue still to be pushed
//   Shi, Slo[n][B] FP32 pair, S = Shi + Slo accumulated with TwoSum (Knuth),
//                 a compensated FP32 reserve in the "y domain":
//                 pi_hat(u) = alpha d_u S(u) / (1 - alpha).
// Every edge read serves all B columns.
//
// Per batch:
//  1. local phase in FP64, all columns at once: the iteration sets S^(j) of
//     Section 4.2 (one frontier list of (node, column) keys), pushed
//     simultaneously with FP64 atomics into a dense FP64 n x B scratch;
//  2. conversion of the FP64 state into the FP32 block (the alpha-part of the
//     remaining residue is folded into S at the same time);
//  3. stages of FP32 pull sweeps, y'(u) = (1-alpha)/d_u sum_{v in N_in(u)} y(v);
//     the alpha-part of the next push is folded in at once (as in the FP64
//     path) into a per-stage FP32 accumulator T(u) += y'(u), which is added
//     into the compensated reserve (S += T, TwoSum) before each refresh, so a
//     sweep moves 8 bytes of reserve state per (node, column) instead of 16;
//  4. after each stage an FP64 residual refresh recomputes, from S alone, the
//     exact residual of the current estimate (Eq. 1):
//        rt(u) = e_s(u) - d_u S(u) / (1-alpha) + sum_{v in N_in(u)} S(v)
//     (this is e_s - pi_hat (I - (1-alpha) P) / alpha in the y domain); its
//     l1 norm certifies ||pi_hat - pi_s||_1 <= ||rt||_1 and it replaces the
//     drifting FP32 residue.  A column whose certificate is <= lambda is done:
//     its residue is set to zero, so later sweeps leave its S unchanged;
//  5. export of pi_hat in FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "ppr_internal.h"

namespace ppr {

namespace mk {

constexpr int kBlock = 256;
constexpr int kLdsBytes = 32768;        // staging budget of the sweep / refresh blocks
constexpr int kGridRed = 2048;          // persistent grid of the refresh (fixed -> deterministic)

__device__ inline double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Knuth's TwoSum: s + e == a + b exactly.
__device__ inline void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    float bp = s - a;
    float ap = s - bp;
    e = (a - ap) + (b - bp);
}

// (hi, lo) += y, compensated: the error of hi + y is carried into lo, and the
// pair is renormalised so that |lo| <= ulp(hi) / 2.
__device__ inline void comp_add(float& hi, float& lo, float y) {
    float s, e;
    two_sum(hi, y, s, e);
    float t = lo + e;
    float h = s + t;               // Fast2Sum (|s| >= |t|)
    lo = t - (h - s);
    hi = h;
}

__device__ inline void split_double(double x, float& hi, float& lo) {
    hi = (float)x;
    lo = (float)(x - (double)hi);
}

// ---------------------------------------------------------------- local phase
__global__ void init_sources(const int32_t* __restrict__ src, int32_t Bw, int shift,
                             double* __restrict__ r64, int64_t* __restrict__ F) {
    int b = threadIdx.x;
    if (b < Bw) {
        int32_t s = src[b];
        if (s >= 0) {
            int64_t key = ((int64_t)s << shift) + b;
            r64[key] = 1.0;
        }
    }
}

// entry i of the frontier: key = (node << shift) | column.  Columns whose
// local phase has ended (active[b] == 0) are skipped: their residue stays.
__global__ void snapshot_b(const int64_t* __restrict__ F, int64_t nf, int shift,
                           const uint8_t* __restrict__ active, const int32_t* __restrict__ deg,
                           double alpha, double* __restrict__ r64, double* __restrict__ pi64,
                           double* __restrict__ X, int64_t* __restrict__ degF,
                           double* __restrict__ taken) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    int64_t key = F[i];
    int32_t b = (int32_t)(key & ((1 << shift) - 1));
    int32_t v = (int32_t)(key >> shift);
    if (!active[b]) {
        X[i] = 0.0;
        degF[i] = 0;
        return;
    }
    double x = atomicExch(&r64[key], 0.0);
    pi64[key] += alpha * x;
    atomicAdd(&taken[b], alpha * x);
    int32_t d = deg[v];
    X[i] = ((1.0 - alpha) * x) / (double)d;
    degF[i] = d;
}

__device__ inline int64_t find_owner64(const int64_t* __restrict__ a, int64_t len, int64_t key) {
    int64_t lo = 0, hi = len;
    while (hi - lo > 1) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= key) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void push_b(
        const int64_t* __restrict__ F, const int64_t* __restrict__ off, int64_t nf, int64_t vol,
        int shift, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
        const int32_t* __restrict__ deg, const double* __restrict__ X, double rmax,
        double* __restrict__ r64, int64_t* __restrict__ F_next, int64_t cap,
        unsigned long long* __restrict__ tail, unsigned long long* __restrict__ cnt_b,
        unsigned long long* __restrict__ vol_b) {
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (off[nf] < vol) vol = off[nf];
    for (int64_t wb = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); wb < vol; wb += stride) {
        int64_t t = wb + lane;
        bool crossed = false;
        int64_t tkey = 0;
        if (t < vol) {
            int64_t i = find_owner64(off, nf, t);
            int64_t key = F[i];
            int32_t b = (int32_t)(key & ((1 << shift) - 1));
            int32_t v = (int32_t)(key >> shift);
            int64_t e = row_ptr[v] + (t - off[i]);
            int32_t u = col[e];
            tkey = ((int64_t)u << shift) + b;
            double x = X[i];
            double old = atomicAdd(&r64[tkey], x);
            double now = old + x;
            int32_t du = deg[u];
            double thr = (double)du * rmax;
            crossed = (old <= thr) && (now > thr);
            if (crossed) {
                atomicAdd(&cnt_b[b], 1ull);
                atomicAdd(&vol_b[b], (unsigned long long)du);
            }
        }
        uint64_t mask = __ballot(crossed);
        if (mask) {
            int leader = __ffsll((unsigned long long)mask) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(tail, (unsigned long long)__popcll(mask));
            base = __shfl(base, leader, 64);
            unsigned int below = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
            // the host sizes F_next for the worst case; the guard keeps a
            // violation of that bound from writing out of bounds (the host
            // sees tail > cap and fails the call)
            if (crossed && (int64_t)(base + below) < cap) F_next[base + below] = tkey;
        }
    }
}

// FP64 state -> FP32 block, dense over (u, b); the FP64 scratch is cleared
// for the next batch.  S = (1-alpha) pi / (alpha d) + y (the alpha-part of
// the remaining residue folded in), y = (1-alpha) r / d.
__global__ void convert_b(int32_t n, int shift, const int32_t* __restrict__ deg, double alpha,
                          double* __restrict__ r64, double* __restrict__ pi64, float* __restrict__ Y,
                          float* __restrict__ Shi, float* __restrict__ Slo, float* __restrict__ T,
                          double* __restrict__ partials) {
    // partials[blockIdx][B]: per-column sum of r (thread's column is fixed: B | blockDim)
    __shared__ double sh[kBlock];
    const int B = 1 << shift;
    const int64_t total = (int64_t)n << shift;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        double r = r64[i];
        double p = pi64[i];
        int32_t u = (int32_t)(i >> shift);
        double d = (double)deg[u];
        double y = ((1.0 - alpha) * r) / d;
        double S = ((1.0 - alpha) * p) / (alpha * d) + y;
        Y[i] = (float)y;
        float h, l;
        split_double(S, h, l);
        Shi[i] = h;
        Slo[i] = l;
        T[i] = 0.f;
        r64[i] = 0.0;
        pi64[i] = 0.0;
        acc += r;
    }
    // column of this thread is threadIdx.x % B (stride is a multiple of B)
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < B) {
        double t = 0.0;
        for (int j = threadIdx.x; j < kBlock; j += B) t += sh[j];
        partials[(int64_t)blockIdx.x * B + threadIdx.x] = t;
    }
}

__global__ void reduce_cols(const double* __restrict__ partials, int nparts, int B, double* __restrict__ out) {
    // one thread per column, fixed order
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double t = 0.0;
    for (int i = 0; i < nparts; ++i) t += partials[(int64_t)i * B + b];
    out[b] = t;
}

__global__ void scale_kernel(const int32_t* __restrict__ deg, int32_t n, double alpha, float* __restrict__ scale) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        scale[i] = (float)((1.0 - alpha) / (double)deg[i]);
}

// ---------------------------------------------------------------- sweep
// Schedule blocks hold <= kLdsBytes / (16 C) in-edges (C = B/4 float4 chunks)
// and <= 256 / C rows, or one long row.  Stream phase: item (edge e, chunk c)
// gathers the float4 Y[v][4c..4c+3] of the edge's source into LDS; every
// thread has 8 items in flight.  Reduce phase: T threads per (row, chunk)
// add the row's slice from LDS.  Long rows: 256 / C slots stride the row's
// edges, then the slots are added in a fixed order through LDS.
template <int C>
struct Sw {
    static constexpr int kNnz = kLdsBytes / (16 * C);     // edges per block
    static constexpr int kRows = kBlock / C;              // rows per block
    static constexpr int kItems = kNnz * C / kBlock;      // items per thread (= 8)
    static constexpr int kSlots = kBlock / C;
};

__device__ inline float4 f4_add(float4 a, float4 b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
__device__ inline float4 f4_shfl_xor(float4 a, int o) {
    return make_float4(__shfl_xor(a.x, o, 64), __shfl_xor(a.y, o, 64), __shfl_xor(a.z, o, 64), __shfl_xor(a.w, o, 64));
}

__device__ inline float4 f4_mul(float4 a, float4 m) { return make_float4(a.x * m.x, a.y * m.y, a.z * m.z, a.w * m.w); }

// Per-column activity in the current stage: column b runs kb[b] sweeps, the
// device counter *step counts the sweeps done.  A column whose budget is
// spent gets y' = 0 (its pending residue is dropped; the next FP64 refresh
// recomputes the exact residual from S), so its S no longer changes.
__device__ inline float4 active4(const int32_t* __restrict__ kb, int32_t step, int c) {
    int4 k = reinterpret_cast<const int4*>(kb)[c];
    return make_float4(step < k.x ? 1.f : 0.f, step < k.y ? 1.f : 0.f, step < k.z ? 1.f : 0.f,
                       step < k.w ? 1.f : 0.f);
}

// ENTRY: the first sweep after a refresh also folds the alpha-part of the
// refreshed residue (still in Y_in) into S.
//
// Latency: all loads that do not depend on the gathered data (row bounds,
// the reserve pair, the scale, the own residue) are issued before the
// index loads, so a block waits for about two memory round trips (indices,
// then gathers) instead of four.
template <typename OffT, int C, bool ENTRY>
__global__ __launch_bounds__(kBlock) void sweep_b(
        const OffT* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
        const RowBlock* __restrict__ blocks, int32_t n_long, const float* __restrict__ scale,
        const float4* __restrict__ Y_in, float4* __restrict__ Y_out, float4* __restrict__ T,
        const int32_t* __restrict__ kb, const int32_t* __restrict__ step_p) {
    using P = Sw<C>;
    __shared__ float4 lds[kLdsBytes / 16];
    const RowBlock b = blocks[blockIdx.x];
    const int32_t step = *step_p;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int32_t u = -1;
    int c = 0;
    if ((int32_t)blockIdx.x < n_long) {
        // one long row: 256 / C slots stride its edges, then a fixed-order sum
        const int slot = threadIdx.x / C;
        c = threadIdx.x % C;
        const int64_t e0 = b.e0, e1 = b.e0 + b.ne;
        float4 a0 = acc, a1 = acc, a2 = acc, a3 = acc;
        int64_t e = e0 + slot;
        for (; e + 3 * P::kSlots < e1; e += 4 * P::kSlots) {
            int32_t v0 = row_idx[e], v1 = row_idx[e + P::kSlots], v2 = row_idx[e + 2 * P::kSlots],
                    v3 = row_idx[e + 3 * P::kSlots];
            float4 g0 = Y_in[(int64_t)v0 * C + c], g1 = Y_in[(int64_t)v1 * C + c];
            float4 g2 = Y_in[(int64_t)v2 * C + c], g3 = Y_in[(int64_t)v3 * C + c];
            a0 = f4_add(a0, g0);
            a1 = f4_add(a1, g1);
            a2 = f4_add(a2, g2);
            a3 = f4_add(a3, g3);
        }
        for (; e < e1; e += P::kSlots) a0 = f4_add(a0, Y_in[(int64_t)row_idx[e] * C + c]);
        lds[threadIdx.x] = f4_add(f4_add(a0, a1), f4_add(a2, a3));
        __syncthreads();
        if (threadIdx.x < C) {
            float4 t = lds[threadIdx.x];
            for (int s2 = 1; s2 < P::kSlots; ++s2) t = f4_add(t, lds[s2 * C + threadIdx.x]);
            acc = t;
            u = b.r0;
        }
    } else {
        const int32_t r0 = b.r0;
        const int32_t R = b.r1 - r0;
        const int32_t ne = b.ne;
        const int64_t e0 = b.e0;
        int T = 64 / C < 1 ? 1 : 64 / C;                // (row, chunk) groups stay inside a wave
        while (T > 1 && T * R * C > kBlock) T >>= 1;
        const int32_t grp = threadIdx.x / T;
        const int sub = threadIdx.x % T;
        const int32_t row = grp / C;
        c = grp % C;
        // independent loads first: row bounds, then the index loads
        int32_t s0 = 0, s1 = 0;
        if (row < R) {
            s0 = (int32_t)((int64_t)col_ptr[r0 + row] - e0);
            s1 = (int32_t)((int64_t)col_ptr[r0 + row + 1] - e0);
        }
        int32_t vv[P::kItems];
#pragma unroll
        for (int k = 0; k < P::kItems; ++k) {
            int32_t it = threadIdx.x + k * kBlock;
            vv[k] = (it / C < ne) ? row_idx[e0 + it / C] : -1;
        }
        float4 gv[P::kItems];
#pragma unroll
        for (int k = 0; k < P::kItems; ++k) {
            int32_t it = threadIdx.x + k * kBlock;
            gv[k] = (vv[k] >= 0) ? Y_in[(int64_t)vv[k] * C + (it % C)] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < P::kItems; ++k) {
            int32_t it = threadIdx.x + k * kBlock;
            if (it / C < ne) lds[it] = gv[k];
        }
        __syncthreads();
        for (int32_t e = s0 + sub; e < s1; e += T) acc = f4_add(acc, lds[e * C + c]);
        for (int o = T >> 1; o >= 1; o >>= 1) acc = f4_add(acc, f4_shfl_xor(acc, o));
        if (row < R && sub == 0) u = r0 + row;
    }
    if (u < 0) return;
    const int64_t at = (int64_t)u * C + c;
    float4 t = T[at];
    const float sc = scale[u];
    const float4 m = active4(kb, step, c);
    if (ENTRY) t = f4_add(t, f4_mul(Y_in[at], m));
    acc = f4_mul(acc, m);
    float4 y = make_float4(sc * acc.x, sc * acc.y, sc * acc.z, sc * acc.w);
    Y_out[at] = y;
    T[at] = f4_add(t, y);
}

// S += T with the compensated add, T = 0 (dense over n x B); run before each
// refresh so that the refresh and the export see the whole reserve.
__global__ void flush_b(int64_t total, float* __restrict__ Shi, float* __restrict__ Slo, float* __restrict__ T) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        float t = T[i];
        if (t != 0.f) {
            float h = Shi[i], l = Slo[i];
            comp_add(h, l, t);
            Shi[i] = h;
            Slo[i] = l;
            T[i] = 0.f;
        }
    }
}

__global__ void bump_step(int32_t* step) { step[0] += 1; }

// ---------------------------------------------------------------- refresh (FP64)
// rt(u) = e_s(u) - d_u S(u) / (1-alpha) + sum_{v in N_in(u)} S(v), all in
// FP64 from the exact values S = Shi + Slo.  Writes y~ = (1-alpha) rt / d_u
// (FP32) as the residue still to be pushed, and per-column sums of |rt|.
// Persistent grid: block k handles schedule blocks k, k + G, ...; thread t
// always works on chunk t % C (one thread per (row, chunk), rows <= 256 / C),
// so the per-column sums are fixed-order and deterministic.
template <int C>
struct Rf {
    static constexpr int kNnz = kLdsBytes / (32 * C);
    static constexpr int kItems = kNnz * C / kBlock;      // = 4
    static constexpr int kRows = kBlock / C;
};

template <typename OffT, int C>
__global__ __launch_bounds__(kBlock) void refresh_b(
        const OffT* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
        const RowBlock* __restrict__ blocks, int32_t n_blocks, int32_t n_long,
        const int32_t* __restrict__ deg, const float4* __restrict__ Shi, const float4* __restrict__ Slo,
        const int32_t* __restrict__ src, double alpha, float4* __restrict__ Y_out,
        double* __restrict__ rt_out, int32_t n, double* __restrict__ partials) {
    using P = Rf<C>;
    __shared__ float4 lds_h[P::kNnz * C];
    __shared__ float4 lds_l[P::kNnz * C];
    __shared__ double red[kBlock * 4];
    const int c = threadIdx.x % C;
    const int32_t myrow = threadIdx.x / C;
    double cs0 = 0.0, cs1 = 0.0, cs2 = 0.0, cs3 = 0.0;   // |rt| of columns 4c..4c+3
    const double inv_oma = 1.0 / (1.0 - alpha);
    const double oma = 1.0 - alpha;
    int32_t srcs[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) srcs[j] = src[4 * c + j];
    for (int32_t bi = blockIdx.x; bi < n_blocks; bi += gridDim.x) {
        const RowBlock b = blocks[bi];
        int32_t u = -1;
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
        if (bi < n_long) {
            // one long row: slots stride the edges, FP64 partials through LDS
            const int slot = threadIdx.x / C;
            const int64_t e0 = b.e0, e1 = b.e0 + b.ne;
            for (int64_t e = e0 + slot; e < e1; e += kBlock / C) {
                int64_t v = row_idx[e];
                float4 h = Shi[v * C + c], l = Slo[v * C + c];
                g0 += (double)h.x + (double)l.x;
                g1 += (double)h.y + (double)l.y;
                g2 += (double)h.z + (double)l.z;
                g3 += (double)h.w + (double)l.w;
            }
            red[threadIdx.x * 4 + 0] = g0;
            red[threadIdx.x * 4 + 1] = g1;
            red[threadIdx.x * 4 + 2] = g2;
            red[threadIdx.x * 4 + 3] = g3;
            __syncthreads();
            if (threadIdx.x < C) {
                g0 = g1 = g2 = g3 = 0.0;
                for (int s = 0; s < kBlock / C; ++s) {
                    int t = s * C + threadIdx.x;
                    g0 += red[t * 4 + 0];
                    g1 += red[t * 4 + 1];
                    g2 += red[t * 4 + 2];
                    g3 += red[t * 4 + 3];
                }
                u = b.r0;
            }
            __syncthreads();
        } else {
            const int32_t r0 = b.r0, r1 = b.r1;
            const int64_t e0 = b.e0;
            const int32_t ne = b.ne;
            int32_t s0 = 0, s1 = 0;
            const bool has = myrow < r1 - r0;
            if (has) {
                s0 = (int32_t)((int64_t)col_ptr[r0 + myrow] - e0);
                s1 = (int32_t)((int64_t)col_ptr[r0 + myrow + 1] - e0);
            }
            int32_t vv[P::kItems];
#pragma unroll
            for (int k = 0; k < P::kItems; ++k) {
                int32_t it = threadIdx.x + k * kBlock;
                vv[k] = (it / C < ne) ? row_idx[e0 + it / C] : -1;
            }
            float4 hv[P::kItems], lv[P::kItems];
#pragma unroll
            for (int k = 0; k < P::kItems; ++k) {
                int32_t it = threadIdx.x + k * kBlock;
                if (vv[k] >= 0) {
                    hv[k] = Shi[(int64_t)vv[k] * C + (it % C)];
                    lv[k] = Slo[(int64_t)vv[k] * C + (it % C)];
                } else {
                    hv[k] = lv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                }
            }
#pragma unroll
            for (int k = 0; k < P::kItems; ++k) {
                int32_t it = threadIdx.x + k * kBlock;
                if (it / C < ne) {
                    lds_h[it] = hv[k];
                    lds_l[it] = lv[k];
                }
            }
            __syncthreads();
            for (int32_t e = s0; e < s1; ++e) {
                float4 h = lds_h[e * C + c], l = lds_l[e * C + c];
                g0 += (double)h.x + (double)l.x;
                g1 += (double)h.y + (double)l.y;
                g2 += (double)h.z + (double)l.z;
                g3 += (double)h.w + (double)l.w;
            }
            if (has) u = r0 + myrow;
            __syncthreads();
        }
        if (u >= 0) {
            const int64_t at = (int64_t)u * C + c;
            const double d = (double)deg[u];
            float4 h = Shi[at], l = Slo[at];
            double S0 = (double)h.x + (double)l.x, S1 = (double)h.y + (double)l.y;
            double S2 = (double)h.z + (double)l.z, S3 = (double)h.w + (double)l.w;
            double t0 = (srcs[0] == u ? 1.0 : 0.0) - d * S0 * inv_oma + g0;
            double t1 = (srcs[1] == u ? 1.0 : 0.0) - d * S1 * inv_oma + g1;
            double t2 = (srcs[2] == u ? 1.0 : 0.0) - d * S2 * inv_oma + g2;
            double t3 = (srcs[3] == u ? 1.0 : 0.0) - d * S3 * inv_oma + g3;
            cs0 += fabs(t0);
            cs1 += fabs(t1);
            cs2 += fabs(t2);
            cs3 += fabs(t3);
            Y_out[at] = make_float4((float)(oma * t0 / d), (float)(oma * t1 / d), (float)(oma * t2 / d),
                                    (float)(oma * t3 / d));
            if (rt_out) {   // column-major FP64 residual [B][n]
                rt_out[(int64_t)(4 * c + 0) * n + u] = t0;
                rt_out[(int64_t)(4 * c + 1) * n + u] = t1;
                rt_out[(int64_t)(4 * c + 2) * n + u] = t2;
                rt_out[(int64_t)(4 * c + 3) * n + u] = t3;
            }
        }
    }
    // per-column sums: threads with the same chunk hold columns 4c..4c+3
    red[threadIdx.x * 4 + 0] = cs0;
    red[threadIdx.x * 4 + 1] = cs1;
    red[threadIdx.x * 4 + 2] = cs2;
    red[threadIdx.x * 4 + 3] = cs3;
    __syncthreads();
    if (threadIdx.x < C) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int t = threadIdx.x; t < kBlock; t += C) {
            a0 += red[t * 4 + 0];
            a1 += red[t * 4 + 1];
            a2 += red[t * 4 + 2];
            a3 += red[t * 4 + 3];
        }
        double* out = partials + (int64_t)blockIdx.x * (4 * C) + 4 * threadIdx.x;
        out[0] = a0;
        out[1] = a1;
        out[2] = a2;
        out[3] = a3;
    }
}

// ---------------------------------------------------------------- export
// pi_hat(u, b) = alpha d_u (Shi + Slo) / (1 - alpha), written row-major
// [Breal][n] through an LDS transpose of 64 nodes x B columns.
template <int C>
struct Ex {
    static constexpr int kNodes = (4 * C >= 128) ? 32 : 64;   // tile of kNodes x (B+1) doubles
};

template <int C>
__global__ __launch_bounds__(kBlock) void export_b(int32_t n, int32_t Breal, const int32_t* __restrict__ deg,
                                                   double alpha, const float* __restrict__ Shi,
                                                   const float* __restrict__ Slo, double* __restrict__ out) {
    constexpr int B = 4 * C;
    constexpr int kNodes = Ex<C>::kNodes;
    __shared__ double tile[kNodes * (B + 1)];
    const int64_t u0 = (int64_t)blockIdx.x * kNodes;
    const double f = alpha / (1.0 - alpha);
    for (int i = threadIdx.x; i < kNodes * B; i += kBlock) {
        int du = i / B, b = i % B;
        int64_t u = u0 + du;
        double v = 0.0;
        if (u < n) v = f * (double)deg[u] * ((double)Shi[u * B + b] + (double)Slo[u * B + b]);
        tile[du * (B + 1) + b] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNodes * B; i += kBlock) {
        int b = i / kNodes, du = i % kNodes;
        int64_t u = u0 + du;
        if (b < Breal && u < n) out[(int64_t)b * n + u] = tile[du * (B + 1) + b];
    }
}

}  // namespace mk

// ======================================================================== host

struct MixedCtx {
    hipStream_t stream = nullptr;
    int32_t n = 0;
    int Bw = 0, shift = 0;
    double alpha = -1.0;
    int64_t fcap = 0;                 // frontier capacity (entries)
    DevBuf r64, pi64;                 // double[n][Bw]
    DevBuf F0, F1, X, degF, off;      // frontier (int64 keys), increments, degrees, prefix
    DevBuf scan_tmp;
    DevBuf Y0, Y1, Shi, Slo;          // float[n][Bw]
    DevBuf T;                         // float[n][Bw] per-stage reserve accumulator
    DevBuf scale;                     // float[n]
    DevBuf partials;                  // double[kGridRed][Bw]
    DevBuf colsum;                    // double[Bw]
    DevBuf ctr;                       // tail + per-column counts + vols
    DevBuf taken;                     // double[Bw]
    DevBuf active;                    // uint8[Bw]
    DevBuf src;                       // int32[Bw]
    DevBuf kb;                        // int32[Bw] per-column sweep budget of the stage
    DevBuf step;                      // int32[1] sweeps done in the stage
    DevBuf stage;                     // double[Bw][n], host-output staging (lazy)
    PinnedBuf host;
    hipGraphExec_t chunk = nullptr;   // captured plain sweeps Y1->Y0->Y1 ...
    int chunk_sweeps = 0;
    ~MixedCtx() {
        if (chunk) (void)hipGraphExecDestroy(chunk);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

void MixedCtxDeleter::operator()(MixedCtx* c) const { delete c; }

namespace {

int ilog2(int x) {
    int s = 0;
    while ((1 << s) < x) ++s;
    return s;
}


template <int C>
const Schedule& sweep_schedule(Graph& g) { return g.schedule(mk::Sw<C>::kNnz, mk::Sw<C>::kRows); }
template <int C>
const Schedule& refresh_schedule(Graph& g) { return g.schedule(mk::Rf<C>::kNnz, mk::Rf<C>::kRows); }

MixedCtxPtr mixed_acquire(Graph& g, int Bw, int64_t fcap) {
    {
        std::lock_guard<std::mutex> lk(g.pool_mu);
        for (auto it = g.mixed_pool.begin(); it != g.mixed_pool.end(); ++it) {
            if ((*it)->Bw == Bw && (*it)->fcap >= fcap) {
                MixedCtxPtr c = std::move(*it);
                g.mixed_pool.erase(it);
                return c;
            }
        }
    }
    MixedCtxPtr c(new MixedCtx());
    const size_t n = (size_t)g.n, nb = n * (size_t)Bw;
    c->n = g.n;
    c->Bw = Bw;
    c->shift = ilog2(Bw);
    c->fcap = fcap;
    HIPCHECK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->r64.alloc(8 * nb);
    c->pi64.alloc(8 * nb);
    HIPCHECK(hipMemsetAsync(c->r64.p, 0, 8 * nb, c->stream));
    HIPCHECK(hipMemsetAsync(c->pi64.p, 0, 8 * nb, c->stream));
    c->F0.alloc(8 * (size_t)fcap);
    c->F1.alloc(8 * (size_t)fcap);
    c->X.alloc(8 * (size_t)fcap);
    c->degF.alloc(8 * (size_t)fcap);
    c->off.alloc(8 * ((size_t)fcap + 1));
    c->scan_tmp.alloc(k::scan_tmp_bytes(fcap));
    c->Y0.alloc(4 * nb);
    c->Y1.alloc(4 * nb);
    c->Shi.alloc(4 * nb);
    c->Slo.alloc(4 * nb);
    c->T.alloc(4 * nb);
    c->scale.alloc(4 * n);
    c->partials.alloc(8 * (size_t)mk::kGridRed * Bw);
    c->colsum.alloc(8 * (size_t)Bw);
    c->ctr.alloc(8 * (1 + 2 * (size_t)Bw));
    c->taken.alloc(8 * (size_t)Bw);
    c->active.alloc((size_t)Bw);
    c->src.alloc(4 * (size_t)Bw);
    c->kb.alloc(4 * (size_t)Bw);
    c->step.alloc(64);
    c->host.alloc(64 + 48 * (size_t)Bw);
    HIPCHECK(hipStreamSynchronize(c->stream));
    return c;
}

void mixed_release(Graph& g, MixedCtxPtr c) {
    std::lock_guard<std::mutex> lk(g.pool_mu);
    g.mixed_pool.push_back(std::move(c));
}

template <typename OffT, int C, bool ENTRY>
void launch_sweep_b3(Graph& g, MixedCtx& c, const Schedule& sch, const float4* Y4i, float4* Y4o) {
    hipLaunchKernelGGL((mk::sweep_b<OffT, C, ENTRY>), dim3((unsigned)sch.n_blocks), dim3(mk::kBlock), 0,
                       c.stream, g.col_ptr.as<OffT>(), g.row_idx.as<int32_t>(), sch.blocks.as<RowBlock>(),
                       sch.n_long, c.scale.as<float>(), Y4i, Y4o, c.T.as<float4>(),
                       c.kb.as<int32_t>(), c.step.as<int32_t>());
    hipLaunchKernelGGL(mk::bump_step, dim3(1), dim3(1), 0, c.stream, c.step.as<int32_t>());
}

template <int C>
void launch_sweep_b(Graph& g, MixedCtx& c, bool entry, const float* yin, float* yout) {
    const Schedule& sch = sweep_schedule<C>(g);
    auto Y4i = reinterpret_cast<const float4*>(yin);
    auto Y4o = reinterpret_cast<float4*>(yout);
    if (g.off64) {
        if (entry) launch_sweep_b3<int64_t, C, true>(g, c, sch, Y4i, Y4o);
        else launch_sweep_b3<int64_t, C, false>(g, c, sch, Y4i, Y4o);
    } else {
        if (entry) launch_sweep_b3<uint32_t, C, true>(g, c, sch, Y4i, Y4o);
        else launch_sweep_b3<uint32_t, C, false>(g, c, sch, Y4i, Y4o);
    }
    HIPCHECK(hipGetLastError());
}

template <int C>
void launch_refresh_b(Graph& g, MixedCtx& c, float* yout, double* rt_out) {
    hipLaunchKernelGGL(mk::flush_b, dim3(2048), dim3(mk::kBlock), 0, c.stream, (int64_t)g.n * c.Bw,
                       c.Shi.as<float>(), c.Slo.as<float>(), c.T.as<float>());
    HIPCHECK(hipGetLastError());
    const Schedule& sch = refresh_schedule<C>(g);
    dim3 grid((unsigned)std::min(sch.n_blocks, mk::kGridRed)), blk(mk::kBlock);
    auto H = c.Shi.as<float4>();
    auto L = c.Slo.as<float4>();
    const RowBlock* bl = sch.blocks.as<RowBlock>();
    if (g.off64)
        hipLaunchKernelGGL((mk::refresh_b<int64_t, C>), grid, blk, 0, c.stream, g.col_ptr.as<int64_t>(),
                           g.row_idx.as<int32_t>(), bl, sch.n_blocks, sch.n_long, g.deg.as<int32_t>(), H, L,
                           c.src.as<int32_t>(), c.alpha, reinterpret_cast<float4*>(yout), rt_out, g.n,
                           c.partials.as<double>());
    else
        hipLaunchKernelGGL((mk::refresh_b<uint32_t, C>), grid, blk, 0, c.stream, g.col_ptr.as<uint32_t>(),
                           g.row_idx.as<int32_t>(), bl, sch.n_blocks, sch.n_long, g.deg.as<int32_t>(), H, L,
                           c.src.as<int32_t>(), c.alpha, reinterpret_cast<float4*>(yout), rt_out, g.n,
                           c.partials.as<double>());
    HIPCHECK(hipGetLastError());
    hipLaunchKernelGGL(mk::reduce_cols, dim3(1), dim3(256), 0, c.stream, c.partials.as<double>(),
                       (int)grid.x, c.Bw, c.colsum.as<double>());
    HIPCHECK(hipGetLastError());
}

template <int C>
void launch_export_b(Graph& g, MixedCtx& c, int Breal, double* out) {
    constexpr int kNodes = mk::Ex<C>::kNodes;
    unsigned grid = (unsigned)((g.n + kNodes - 1) / kNodes);
    hipLaunchKernelGGL((mk::export_b<C>), dim3(grid), dim3(mk::kBlock), 0, c.stream, g.n, Breal,
                       g.deg.as<int32_t>(), c.alpha, c.Shi.as<float>(), c.Slo.as<float>(), out);
    HIPCHECK(hipGetLastError());
}

struct Dispatch {
    void (*sweep)(Graph&, MixedCtx&, bool, const float*, float*);
    void (*refresh)(Graph&, MixedCtx&, float*, double*);
    void (*exportf)(Graph&, MixedCtx&, int, double*);
};

template <int C>
Dispatch make_dispatch() { return {&launch_sweep_b<C>, &launch_refresh_b<C>, &launch_export_b<C>}; }

Dispatch dispatch_for(int Bw) {
    switch (Bw) {
        case 4: return make_dispatch<1>();
        case 8: return make_dispatch<2>();
        case 16: return make_dispatch<4>();
        case 32: return make_dispatch<8>();
        case 64: return make_dispatch<16>();
        case 128: return make_dispatch<32>();
        default: fail(PPR_ERR_ARG, "batch width must be a power of two in [4, 128]");
    }
}

// Batched form of the switch rule.  Edge rule: a column keeps pushing locally
// while switch_param * kBatchRef * vol_b <= m, so one level of a block of
// kBatchRef columns moves at most about m / switch_param edges, the bound of
// the single-query path.  The rule does not depend on the block width, so a
// column's schedule is the same whichever block it runs in.
constexpr double kBatchRef = 32.0;

bool continue_local(const ppr_options& opt, int64_t nf, int64_t vol, int32_t n, int64_t m) {
    if (opt.switch_rule == PPR_SWITCH_NODES) return 4 * nf <= (int64_t)n;
    return opt.switch_param * kBatchRef * (double)vol <= (double)m;
}

constexpr int kChunkSweeps = 16;

void run_mixed_chunk(Graph& g, MixedCtx& c, const int32_t* sources, int Breal, double alpha, double lambda,
                     const ppr_options& opt, double* pi_out, double* r_out, ppr_stats* st) {
    auto t0 = std::chrono::steady_clock::now();
    const int Bw = c.Bw;
    const int32_t n = g.n;
    hipStream_t ss = c.stream;
    Dispatch D = dispatch_for(Bw);
    char* hb = c.host.as<char>();
    // ---- per-column parameters
    std::vector<int32_t> hsrc(Bw, -1);
    for (int b = 0; b < Breal; ++b) hsrc[b] = sources[b];
    HIPCHECK(hipMemcpyAsync(c.src.p, hsrc.data(), 4 * (size_t)Bw, hipMemcpyHostToDevice, ss));
    if (c.alpha != alpha) {
        hipLaunchKernelGGL(mk::scale_kernel, dim3(1024), dim3(256), 0, ss, g.deg.as<int32_t>(), n, alpha,
                           c.scale.as<float>());
        HIPCHECK(hipGetLastError());
        if (c.chunk) {
            (void)hipGraphExecDestroy(c.chunk);
            c.chunk = nullptr;
        }
        c.alpha = alpha;
    }

    // ---- local phase, all columns together (FP64)
    std::vector<int64_t> nf_b(Bw, 0), vol_b(Bw, 0);
    std::vector<double> rsum_b(Bw, 0.0);
    std::vector<int32_t> levels_b(Bw, 0);
    std::vector<int64_t> edges_b(Bw, 0);
    std::vector<uint8_t> act(Bw, 0);
    std::vector<int64_t> hF;
    for (int b = 0; b < Breal; ++b) {
        nf_b[b] = 1;
        vol_b[b] = g.h_deg[sources[b]];
        rsum_b[b] = 1.0;
        hF.push_back(((int64_t)sources[b] << c.shift) + b);
    }
    HIPCHECK(hipMemcpyAsync(c.F0.p, hF.data(), 8 * hF.size(), hipMemcpyHostToDevice, ss));
    hipLaunchKernelGGL(mk::init_sources, dim3(1), dim3(128), 0, ss, c.src.as<int32_t>(), Bw, c.shift,
                       c.r64.as<double>(), c.F0.as<int64_t>());
    HIPCHECK(hipGetLastError());
    int64_t nf = (int64_t)hF.size();
    int64_t* F = c.F0.as<int64_t>();
    int64_t* Fn = c.F1.as<int64_t>();
    const double rmax = lambda / (double)g.m;
    for (;;) {
        int64_t vol = 0;
        bool any = false;
        for (int b = 0; b < Bw; ++b) {
            // a column's next frontier holds at most vol_b entries: it must fit
            // the per-column share of the frontier capacity
            act[b] = (b < Breal && nf_b[b] > 0 && rsum_b[b] > lambda &&
                      continue_local(opt, nf_b[b], vol_b[b], n, g.m) &&
                      vol_b[b] <= c.fcap / Bw) ? 1 : 0;
            if (act[b]) {
                vol += vol_b[b];
                any = true;
            }
        }
        if (!any || nf == 0) break;
        HIPCHECK(hipMemcpyAsync(c.active.p, act.data(), (size_t)Bw, hipMemcpyHostToDevice, ss));
        HIPCHECK(hipMemsetAsync(c.ctr.p, 0, 8 * (1 + 2 * (size_t)Bw), ss));
        HIPCHECK(hipMemsetAsync(c.taken.p, 0, 8 * (size_t)Bw, ss));
        unsigned gs = (unsigned)((nf + 255) / 256);
        hipLaunchKernelGGL(mk::snapshot_b, dim3(gs), dim3(256), 0, ss, F, nf, c.shift, c.active.as<uint8_t>(),
                           g.deg.as<int32_t>(), alpha, c.r64.as<double>(), c.pi64.as<double>(), c.X.as<double>(),
                           c.degF.as<int64_t>(), c.taken.as<double>());
        HIPCHECK(hipGetLastError());
        k::exclusive_scan_i64(c.degF.as<int64_t>(), c.off.as<int64_t>(), nf, c.scan_tmp.p, ss);
        if (vol > 0) {
            unsigned gp = (unsigned)std::min<int64_t>((vol + 255) / 256, 16384);
            auto* ctr = reinterpret_cast<unsigned long long*>(c.ctr.p);
            hipLaunchKernelGGL(mk::push_b, dim3(gp), dim3(256), 0, ss, F, c.off.as<int64_t>(), nf, vol, c.shift,
                               g.row_ptr.as<int64_t>(), g.col.as<int32_t>(), g.deg.as<int32_t>(), c.X.as<double>(),
                               rmax, c.r64.as<double>(), Fn, c.fcap, ctr, ctr + 1, ctr + 1 + Bw);
            HIPCHECK(hipGetLastError());
        }
        HIPCHECK(hipMemcpyAsync(hb, c.ctr.p, 8 * (1 + 2 * (size_t)Bw), hipMemcpyDeviceToHost, ss));
        HIPCHECK(hipMemcpyAsync(hb + 8 * (1 + 2 * (size_t)Bw), c.taken.p, 8 * (size_t)Bw, hipMemcpyDeviceToHost, ss));
        HIPCHECK(hipStreamSynchronize(ss));
        const uint64_t* hc = reinterpret_cast<const uint64_t*>(hb);
        const double* ht = reinterpret_cast<const double*>(hb + 8 * (1 + 2 * (size_t)Bw));
        nf = (int64_t)hc[0];
        for (int b = 0; b < Bw; ++b) {
            if (!act[b]) {
                nf_b[b] = 0;       // this column's local phase is over
                continue;
            }
            edges_b[b] += vol_b[b];
            levels_b[b] += 1;
            rsum_b[b] -= ht[b];
            nf_b[b] = (int64_t)hc[1 + b];
            vol_b[b] = (int64_t)hc[1 + Bw + b];
        }
        if (nf > c.fcap) fail(PPR_ERR_OOM, "frontier capacity exceeded");
        std::swap(F, Fn);
    }

    // ---- FP64 -> FP32 block (alpha-part of the residue folded into S)
    {
        unsigned gc = 1024;
        hipLaunchKernelGGL(mk::convert_b, dim3(gc), dim3(256), 0, ss, n, c.shift, g.deg.as<int32_t>(), alpha,
                           c.r64.as<double>(), c.pi64.as<double>(), c.Y0.as<float>(), c.Shi.as<float>(),
                           c.Slo.as<float>(), c.T.as<float>(), c.partials.as<double>());
        HIPCHECK(hipGetLastError());
        hipLaunchKernelGGL(mk::reduce_cols, dim3(1), dim3(256), 0, ss, c.partials.as<double>(), (int)gc, Bw,
                           c.colsum.as<double>());
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemcpyAsync(hb, c.colsum.p, 8 * (size_t)Bw, hipMemcpyDeviceToHost, ss));
        HIPCHECK(hipStreamSynchronize(ss));
    }
    const double* hcol = reinterpret_cast<const double*>(hb);
    // err_b: bound on ||pi_hat - pi_s||_1 as the sweeps go (exact after a refresh)
    std::vector<double> err(Bw, 0.0), cert(Bw, -1.0);
    std::vector<int32_t> sweeps_b(Bw, 0), refresh_b(Bw, 0);
    std::vector<uint8_t> done(Bw, 1);
    for (int b = 0; b < Breal; ++b) {
        err[b] = (1.0 - alpha) * hcol[b];
        done[b] = 0;
    }
    const float* yc = c.Y0.as<float>();
    float* yn = c.Y1.as<float>();
    auto advance = [&](bool entry) {
        D.sweep(g, c, entry, yc, yn);
        float* t = const_cast<float*>(yc);
        yc = yn;
        yn = t;
    };
    bool entry = false;       // the converted state has its alpha-part folded
    EventPair ev;
    double sweep_ms = 0.0;
    int32_t total_sweeps = 0, total_refresh = 0;
    const double oma = 1.0 - alpha;
    std::vector<int32_t> hkb(Bw, 0);
    for (;;) {
        // per-column budget: sweeps until err_b has fallen by refresh_factor
        // (or to lambda / 2); a column's schedule depends on its own error only
        int K = 0;
        for (int b = 0; b < Bw; ++b) {
            hkb[b] = 0;
            if (done[b]) continue;
            double target = std::max(err[b] / opt.refresh_factor, 0.5 * lambda);
            int k = 0;
            for (double x = err[b]; x > target; x *= oma) ++k;
            hkb[b] = k;
            K = std::max(K, k);
        }
        if (total_sweeps + K > opt.max_sweeps) {
            K = std::max(0, opt.max_sweeps - total_sweeps);
            for (int b = 0; b < Bw; ++b) hkb[b] = std::min(hkb[b], K);
        }
        if (K > 0) {
            HIPCHECK(hipMemcpyAsync(c.kb.p, hkb.data(), 4 * (size_t)Bw, hipMemcpyHostToDevice, ss));
            HIPCHECK(hipMemsetAsync(c.step.p, 0, 4, ss));
            ev.start(ss);
            advance(entry);
            entry = false;
            int rest = K - 1;
            // replay captured chunks of plain sweeps when the buffers line up
            if (rest >= kChunkSweeps && yc == c.Y1.as<float>()) {
                if (!c.chunk) {
                    hipGraph_t graph = nullptr;
                    HIPCHECK(hipStreamBeginCapture(ss, hipStreamCaptureModeThreadLocal));
                    const float* a = c.Y1.as<float>();
                    float* bb = c.Y0.as<float>();
                    try {
                        for (int i = 0; i < kChunkSweeps; ++i) {
                            D.sweep(g, c, false, a, bb);
                            float* t = const_cast<float*>(a);
                            a = bb;
                            bb = t;
                        }
                    } catch (...) {
                        (void)hipStreamEndCapture(ss, &graph);
                        if (graph) (void)hipGraphDestroy(graph);
                        throw;
                    }
                    HIPCHECK(hipStreamEndCapture(ss, &graph));
                    hipError_t e = hipGraphInstantiate(&c.chunk, graph, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(graph);
                    HIPCHECK(e);
                    c.chunk_sweeps = kChunkSweeps;
                }
                while (rest >= kChunkSweeps) {     // even count: yc stays Y1
                    HIPCHECK(hipGraphLaunch(c.chunk, ss));
                    rest -= kChunkSweeps;
                }
            }
            for (int i = 0; i < rest; ++i) advance(false);
            ev.stop(ss);
            total_sweeps += K;
            for (int b = 0; b < Bw; ++b)
                if (!done[b]) {
                    sweeps_b[b] += hkb[b];
                    err[b] *= std::pow(oma, hkb[b]);
                }
        }
        // FP64 refresh: exact residual of the current estimate, and its l1 norm
        D.refresh(g, c, yn, nullptr);
        {
            float* t = const_cast<float*>(yc);
            yc = yn;
            yn = t;
        }
        entry = true;
        ++total_refresh;
        HIPCHECK(hipMemcpyAsync(hb, c.colsum.p, 8 * (size_t)Bw, hipMemcpyDeviceToHost, ss));
        HIPCHECK(hipStreamSynchronize(ss));
        if (K > 0) sweep_ms += ev.elapsed_ms();
        bool all = true;
        for (int b = 0; b < Breal; ++b) {
            if (done[b]) continue;
            refresh_b[b] += 1;
            cert[b] = hcol[b];
            err[b] = hcol[b];
            if (hcol[b] <= lambda) done[b] = 1;
            else all = false;
        }
        if (all) break;
        if (total_sweeps >= opt.max_sweeps) break;
    }
    // ---- output: the export kernel writes device memory only; a host
    // destination is filled through a device staging buffer
    if (is_device_ptr(pi_out, g.device)) {
        D.exportf(g, c, Breal, pi_out);
    } else {
        if (c.stage.bytes < 8 * (size_t)Bw * n) c.stage.alloc(8 * (size_t)Bw * n);
        D.exportf(g, c, Breal, c.stage.as<double>());
        HIPCHECK(hipMemcpyAsync(pi_out, c.stage.p, 8 * (size_t)Breal * n, hipMemcpyDefault, ss));
    }
    if (r_out) {
        // residual of the exported estimate (FP64, row-major [Breal][n])
        DevBuf rt((size_t)Bw * n * 8);
        D.refresh(g, c, yn, rt.as<double>());
        HIPCHECK(hipMemcpyAsync(r_out, rt.p, 8 * (size_t)Breal * n, hipMemcpyDefault, ss));
        HIPCHECK(hipStreamSynchronize(ss));
    }
    HIPCHECK(hipStreamSynchronize(ss));
    // clear the block for the next batch is not needed (conversion rewrites it)
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    bool failed = false;
    for (int b = 0; b < Breal; ++b) {
        if (!done[b]) failed = true;
        if (st) {
            ppr_stats& s = st[b];
            s.local_levels = levels_b[b];
            s.sweeps = sweeps_b[b];
            s.refreshes = refresh_b[b];
            s.source = sources[b];
            s.edge_pushes = edges_b[b] + (int64_t)(sweeps_b[b] + refresh_b[b]) * g.m;
            s.r_sum = cert[b];
            s.cert_l1 = cert[b];
            s.ms = ms;
            s.sweep_ms = sweep_ms;
            s.sweep_launches = total_sweeps;
            s.batch_cols = Bw;
        }
    }
    (void)total_refresh;
    if (failed) fail(PPR_ERR_NOT_CONVERGED, "max_sweeps reached before the certificate fell to lambda");
}

}  // namespace

namespace {

int64_t frontier_capacity(const Graph& g, const ppr_options& opt, int Bw) {
    // a level runs only if the column's next frontier (at most vol_b entries)
    // fits its share of the capacity
    int64_t per_col = g.n;
    if (opt.switch_rule == PPR_SWITCH_EDGES && opt.switch_param > 0)
        per_col = std::min<int64_t>(per_col, (int64_t)((double)g.m / (opt.switch_param * kBatchRef)) + 1);
    per_col = std::max<int64_t>(per_col, 1 + g.max_out);
    return per_col * Bw;
}

size_t mixed_footprint(const Graph& g, int Bw, int64_t fcap) {
    const size_t nb = (size_t)g.n * (size_t)Bw;
    return 16 * nb          // FP64 local-phase scratch
           + 20 * nb        // Y0, Y1, Shi, Slo, T
           + 40 * (size_t)fcap + 4 * (size_t)g.n + ((size_t)1 << 20);
}

}  // namespace

void autotune_width(Graph& g, double alpha, const int32_t* widths, int32_t count, int32_t* best,
                    double* cost_us) {
    HIPCHECK(hipSetDevice(g.device));
    static const int32_t kDefault[5] = {8, 16, 32, 64, 128};
    if (!widths) {
        widths = kDefault;
        count = 5;
    }
    if (count < 1) fail(PPR_ERR_ARG, "no candidate widths");
    ppr_options opt;
    ppr_options_default(&opt);
    size_t free_b = 0, total_b = 0;
    HIPCHECK(hipMemGetInfo(&free_b, &total_b));
    double best_cost = 1e300;
    int best_w = 0;
    for (int32_t i = 0; i < count; ++i) {
        int W = widths[i];
        if (W < 4 || W > 128 || (W & (W - 1))) fail(PPR_ERR_ARG, "candidate widths must be powers of two in [4, 128]");
        int64_t fcap = frontier_capacity(g, opt, W);
        // contexts already pooled for this width cost nothing new
        bool pooled = false;
        {
            std::lock_guard<std::mutex> lk(g.pool_mu);
            for (auto& c : g.mixed_pool) pooled |= (c->Bw == W && c->fcap >= fcap);
        }
        if (!pooled && mixed_footprint(g, W, fcap) > free_b / 2) {
            if (cost_us) cost_us[i] = -1.0;
            continue;
        }
        MixedCtxPtr c = mixed_acquire(g, W, fcap);
        hipStream_t ss = c->stream;
        const size_t nb = (size_t)g.n * W;
        HIPCHECK(hipMemsetAsync(c->Y0.p, 0, 4 * nb, ss));
        HIPCHECK(hipMemsetAsync(c->Y1.p, 0, 4 * nb, ss));
        HIPCHECK(hipMemsetAsync(c->Shi.p, 0, 4 * nb, ss));
        HIPCHECK(hipMemsetAsync(c->Slo.p, 0, 4 * nb, ss));
        HIPCHECK(hipMemsetAsync(c->T.p, 0, 4 * nb, ss));
        std::vector<int32_t> kb(W, 1 << 30);
        HIPCHECK(hipMemcpyAsync(c->kb.p, kb.data(), 4 * (size_t)W, hipMemcpyHostToDevice, ss));
        HIPCHECK(hipMemsetAsync(c->step.p, 0, 4, ss));
        if (c->alpha != alpha) {
            hipLaunchKernelGGL(mk::scale_kernel, dim3(1024), dim3(256), 0, ss, g.deg.as<int32_t>(), g.n, alpha,
                               c->scale.as<float>());
            HIPCHECK(hipGetLastError());
            if (c->chunk) {
                (void)hipGraphExecDestroy(c->chunk);
                c->chunk = nullptr;
            }
            c->alpha = alpha;
        }
        Dispatch D = dispatch_for(W);
        const int reps = 4;
        D.sweep(g, *c, false, c->Y0.as<float>(), c->Y1.as<float>());     // warm-up
        EventPair ev;
        ev.start(ss);
        for (int r = 0; r < reps; ++r)
            D.sweep(g, *c, false, (r & 1) ? c->Y1.as<float>() : c->Y0.as<float>(),
                    (r & 1) ? c->Y0.as<float>() : c->Y1.as<float>());
        ev.stop(ss);
        HIPCHECK(hipStreamSynchronize(ss));
        double us = ev.elapsed_ms() * 1e3 / reps / W;
        if (cost_us) cost_us[i] = us;
        // the narrower block wins ties (within 1%): less memory, lower latency
        if (best_w == 0 || us < best_cost * 0.99) {
            best_cost = us;
            best_w = W;
        }
        mixed_release(g, std::move(c));
    }
    if (best_w == 0) fail(PPR_ERR_OOM, "no candidate width fits the device memory budget");
    g.tuned_width = best_w;
    if (best) *best = best_w;
}

int default_batch_width(int32_t B) {
    int w = 4;
    while (w < B && w < 32) w <<= 1;
    return w;
}

void run_mixed_batch(Graph& g, const int32_t* sources, int32_t B, double alpha, double lambda,
                     const ppr_options& opt, double* pi_out, double* r_out, ppr_stats* st) {
    HIPCHECK(hipSetDevice(g.device));
    int Bw = opt.batch_cols > 0 ? opt.batch_cols : (g.tuned_width > 0 ? g.tuned_width : default_batch_width(B));
    if (Bw < 4 || Bw > 128 || (Bw & (Bw - 1))) fail(PPR_ERR_ARG, "batch_cols must be a power of two in [4, 128]");
    // frontier capacity: a column's frontier never exceeds n, nor (edge rule)
    // m / switch_param + 1 entries
    int64_t fcap = frontier_capacity(g, opt, Bw);
    auto c = mixed_acquire(g, Bw, fcap);
    ppr_status first = PPR_OK;
    std::string msg;
    try {
        for (int32_t b0 = 0; b0 < B; b0 += Bw) {
            int Breal = std::min<int32_t>(Bw, B - b0);
            try {
                run_mixed_chunk(g, *c, sources + b0, Breal, alpha, lambda, opt, pi_out + (size_t)b0 * g.n,
                                r_out ? r_out + (size_t)b0 * g.n : nullptr, st ? st + b0 : nullptr);
            } catch (const Failure& e) {
                // not converged: the FP64 scratch was already cleared by the conversion
                if (e.status != PPR_ERR_NOT_CONVERGED) throw;
                if (first == PPR_OK) { first = e.status; msg = e.msg; }
            }
        }
    } catch (...) {
        // any other failure may leave the FP64 scratch dirty: drop the context
        (void)hipStreamSynchronize(c->stream);
        c.reset();
        throw;
    }
    HIPCHECK(hipStreamSynchronize(c->stream));
    mixed_release(g, std::move(c));
    if (first != PPR_OK) fail(first, msg);
}

}  // namespace ppr
