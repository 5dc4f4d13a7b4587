// Kernels of the batched mixed-precision path: B sources as the columns of an
// n x B block.
//
// State (node-major: the B values of one node are contiguous, so one edge's
// gather reads one contiguous row of B residues):
//   Y[n][B]         y = (1 - alpha) r / d_u, the residue still to push, stored
//                   as FP32 or as bf16 (half the gather bytes); arithmetic is
//                   FP32 either way, and what a row stores is exactly what its
//                   out-neighbours pull and what T accumulates, so the storage
//                   rounding only leaves residual that the next FP64 refresh
//                   measures
//   S[n][B]         FP64 reserve in the y domain: pi_hat(u) = alpha d_u S(u) / (1 - alpha)
//   AS[n][B]        FP64 running sum_{v in N_in(u)} S(v), kept up to date by each refresh
//   T[n][B]         FP32 per-stage accumulator of reserve increments

// Columns are independent: each one is a query with its own source, its own
// alpha, its own lambda and its own schedule.  The per-node scale table holds
// (1 - alpha) / d_u for the block's reference alpha; a column with another
// alpha_b multiplies it by the FP32 factor (1 - alpha_b) / (1 - alpha), which
// is exactly 1 for the reference alpha, and every FP64 step (local phase,
// conversion, refresh, export) takes alpha_b itself from the per-column
// coefficients acoef = [alpha_b | 1 - alpha_b | 1 / (1 - alpha_b) |
// alpha_b / (1 - alpha_b)] (each Bw long).
//  - local phase (FP64): the iteration sets S^(j) of Section 4.2 pushed
//    simultaneously, one frontier list of (node << log2 B | column) keys, FP64
//    atomics into a dense FP64 scratch; then conversion into the block (the
//    alpha-part of the remaining residue folded into S at once);
//  - sweeps (FP32): y'(u) = (1-alpha)/d_u sum_{v in N_in(u)} y(v) (Eq. 7 in the
//    y domain), over row chunks in block Gauss-Seidel order (the rows of a
//    chunk see the residues earlier chunks produced in the same sweep, as the
//    in-place scan of Algorithm 3 does); the alpha-part of the new residue
//    goes into T (two sweeps' residues at a time, by the odd step).  Per
//    column a budget kb[b]: the column runs sweeps while step < kb[b], then
//    gets y' = 0 (its pending residue is dropped: the next refresh recomputes
//    the exact residual from S) and its reserve stops changing;
//  - refresh (FP64): the exact residual of the estimate S + T (Eq. 1
//    rearranged)
//        rt(u) = e_s(u) - d_u S'(u) / (1 - alpha) + sum_{v in N_in(u)} S'(v),
//    S' = S + T, whose l1 norm certifies ||pi_hat - pi_s||_1 <= ||rt||_1.  The
//    in-neighbour sum is AS(u) + sum_{v in N_in(u)} T(v): only the FP32 stage
//    accumulator is gathered (exactly, in FP64), not the whole reserve.  For
//    the columns being refreshed AS takes the new sum, y~ = (1-alpha) rt / d
//    replaces the drifting residue, and S += T; the first sweep after that
//    starts T afresh with y~'s alpha-part (entry flag 2).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "mixed_internal.h"

namespace ppr {
namespace mk {

namespace {

// ---------------------------------------------------------------- helpers
__device__ inline float4 f4_add(float4 a, float4 b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
__device__ inline float4 f4_mul(float4 a, float4 m) { return make_float4(a.x * m.x, a.y * m.y, a.z * m.z, a.w * m.w); }
__device__ inline float4 f4_shfl_xor(float4 a, int o) {
    return make_float4(__shfl_xor(a.x, o, 64), __shfl_xor(a.y, o, 64), __shfl_xor(a.z, o, 64), __shfl_xor(a.w, o, 64));
}
__device__ inline float4 flag4(int4 f) {
    return make_float4(f.x ? 1.f : 0.f, f.y ? 1.f : 0.f, f.z ? 1.f : 0.f, f.w ? 1.f : 0.f);
}

// K consecutive columns of one node, in FP32 registers.
template <int K>
struct Vec {
    float4 q[K / 4];
};
template <int K>
__device__ inline Vec<K> v_zero() {
    Vec<K> r;
#pragma unroll
    for (int i = 0; i < K / 4; ++i) r.q[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    return r;
}
template <int K>
__device__ inline Vec<K> v_add(Vec<K> a, const Vec<K>& b) {
#pragma unroll
    for (int i = 0; i < K / 4; ++i) a.q[i] = f4_add(a.q[i], b.q[i]);
    return a;
}
template <int K>
__device__ inline Vec<K> v_mul(Vec<K> a, const Vec<K>& b) {
#pragma unroll
    for (int i = 0; i < K / 4; ++i) a.q[i] = f4_mul(a.q[i], b.q[i]);
    return a;
}
template <int K>
__device__ inline Vec<K> v_shfl_xor(Vec<K> a, int o) {
#pragma unroll
    for (int i = 0; i < K / 4; ++i) a.q[i] = f4_shfl_xor(a.q[i], o);
    return a;
}

// Residue storage.  A sweep lane gathers one 16-byte vector V of K columns
// and stages it in LDS as it was stored, so that bf16 storage doubles the
// in-edges a block keeps in flight; the refresh writes 4 columns at a time
// (value4 / pack4).
//
// bf16: the upper half of an FP32 word; packing rounds to nearest, ties to
// even (the residues are finite).  Column k of a vector sits in half k of its
// words, low half first, i.e. bf16 element order in memory.  bf16_bits rounds
// on the bits; bf16_pair converts two values with the FP32 -> bf16 conversion
// instruction of gfx950 (one instruction per pair; the same rounding, denormal
// inputs included).
__device__ inline uint32_t bf16_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ inline float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ inline uint32_t bf16_pair(float a, float b) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

struct StoreF32 {                       // 4 FP32 columns
    static constexpr int K = 4;
    using V = float4;
    __device__ static V zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ static Vec<4> value(V v) { Vec<4> r; r.q[0] = v; return r; }
    __device__ static V pack(const Vec<4>& v) { return v.q[0]; }
    __device__ static float4 value4(V v) { return v; }
    __device__ static V pack4(float4 v) { return v; }
};
struct StoreBF16 {                      // 4 bf16 columns: the refresh's view
    static constexpr int K = 4;
    using V = uint2;
    __device__ static float4 value4(V w) { return make_float4(bf16_lo(w.x), bf16_hi(w.x), bf16_lo(w.y), bf16_hi(w.y)); }
    __device__ static V pack4(float4 v) { return make_uint2(bf16_pair(v.x, v.y), bf16_pair(v.z, v.w)); }
};
struct StoreBF16x8 {                    // 8 bf16 columns: the sweep's view
    static constexpr int K = 8;
    using V = uint4;
    __device__ static V zero() { return make_uint4(0u, 0u, 0u, 0u); }
    __device__ static Vec<8> value(V w) {
        Vec<8> r;
        r.q[0] = make_float4(bf16_lo(w.x), bf16_hi(w.x), bf16_lo(w.y), bf16_hi(w.y));
        r.q[1] = make_float4(bf16_lo(w.z), bf16_hi(w.z), bf16_lo(w.w), bf16_hi(w.w));
        return r;
    }
    __device__ static V pack(const Vec<8>& v) {
        return make_uint4(bf16_pair(v.q[0].x, v.q[0].y), bf16_pair(v.q[0].z, v.q[0].w),
                          bf16_pair(v.q[1].x, v.q[1].y), bf16_pair(v.q[1].z, v.q[1].w));
    }
};

// Non-temporal loads and stores.  The sweep uses them for what it streams
// once (a row's own input residue, new residue and stage accumulator, the
// in-edge indices), so that these do not push the gathered residue rows, which
// many in-edges reuse, out of the caches.  The gathers themselves keep the
// default policy: they depend on those cache hits.
template <typename V>
__device__ inline V nt_ld(const V* p) {
    using W = unsigned int __attribute__((ext_vector_type(sizeof(V) / 4)));
    const W w = __builtin_nontemporal_load(reinterpret_cast<const W*>(p));
    V v;
    __builtin_memcpy(&v, &w, sizeof(V));
    return v;
}
template <typename V>
__device__ inline void nt_st(const V& v, V* p) {
    using W = unsigned int __attribute__((ext_vector_type(sizeof(V) / 4)));
    W w;
    __builtin_memcpy(&w, &v, sizeof(V));
    __builtin_nontemporal_store(w, reinterpret_cast<W*>(p));
}

// 16 bytes per lane from global memory straight into LDS: lane l of the wave
// writes vector l after dst (dst is the same for the whole wave).  Device
// pass only (the builtin has no host form; the host pass needs only the
// kernel's signature).
__device__ inline void lds_dma16(const void* src, void* dst) {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
#endif
}

// In-edge indices of one round of a row-tile block: item k of thread t is
// edge (t + 256 k) / C of the round (C lanes per edge, one per 16-byte vector
// of the row).  A wave's 64 lanes then need only 64 / C distinct edges per
// item.  When all G kItems of them (G = 64 / C) fit the wave, lane
// L = j + G k loads edge (wave's first) + j + k 256 / C once and the lanes
// take their kItems indices from it with shuffles, instead of every lane
// loading each of its kItems indices.  -1 marks an item beyond the round's
// nr edges.  NT: the index loads are non-temporal.
template <int C, int kItems>
struct ShuffledIndices {
    static constexpr int G = (C <= 64) ? 64 / C : 0;      // distinct edges per item per wave
    static constexpr bool value = G > 0 && G * kItems <= 64;
};

// The shuffled form in two steps: the loader lanes' loads (issued early by a
// caller that has other work to overlap them with), then the shuffles.
template <int C, int kItems, bool NT>
__device__ inline int32_t round_index_load(const int32_t* __restrict__ row_idx, int64_t first, int32_t nr) {
    constexpr int G = ShuffledIndices<C, kItems>::G;
    const int lane = threadIdx.x & 63;
    const int32_t w0 = (int32_t)(threadIdx.x >> 6) * G;   // the wave's first edge of item 0
    // loader lane L = j + G k holds edge w0 + j + k (256 / C)
    const int j = lane % G, kk = lane / G;
    const int32_t el = w0 + j + kk * (kBlock / C);
    int32_t mine = -1;
    if (lane < G * kItems && el < nr) mine = NT ? __builtin_nontemporal_load(&row_idx[first + el]) : row_idx[first + el];
    return mine;
}

template <int C, int kItems>
__device__ inline void round_index_spread(int32_t mine, int32_t (&vv)[kItems]) {
    constexpr int G = ShuffledIndices<C, kItems>::G;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < kItems; ++k) vv[k] = __shfl(mine, (lane / C) + G * k, 64);
}

template <int C, int kItems, bool NT>
__device__ inline void round_indices(const int32_t* __restrict__ row_idx, int64_t first, int32_t nr,
                                     int32_t (&vv)[kItems]) {
    if constexpr (ShuffledIndices<C, kItems>::value) {
        round_index_spread<C, kItems>(round_index_load<C, kItems, NT>(row_idx, first, nr), vv);
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int32_t it = threadIdx.x + k * kBlock;
            vv[k] = (it / C < nr) ? row_idx[first + it / C] : -1;
        }
    }
}

// ---------------------------------------------------------------- local phase
__global__ void init_sources_k(const int32_t* __restrict__ src, const int32_t* __restrict__ cmask, int32_t Bw,
                               int shift, double* __restrict__ r64) {
    int b = threadIdx.x;
    if (b < Bw && cmask[b]) {
        int32_t s = src[b];
        if (s >= 0) r64[((int64_t)s << shift) + b] = 1.0;
    }
}

// Frontier entry i: key = (node << shift) | column.  Columns whose local
// phase is over (active[b] == 0) are skipped; their residue stays in place.
// The reserve taken per column is summed in LDS first: one global atomic per
// block and column.
__global__ __launch_bounds__(kBlock) void snapshot_k(const int64_t* __restrict__ F, int64_t nf, int shift,
                           const uint8_t* __restrict__ active, const int32_t* __restrict__ deg,
                           const double* __restrict__ alpha_b,
                           double* __restrict__ r64, double* __restrict__ pi64, double* __restrict__ X,
                           int64_t* __restrict__ degF, double* __restrict__ taken) {
    __shared__ double s_taken[128];
    const int Bw = 1 << shift;
    if ((int)threadIdx.x < 128) s_taken[threadIdx.x] = 0.0;
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nf) {
        int64_t key = F[i];
        int32_t b = (int32_t)(key & (Bw - 1));
        int32_t v = (int32_t)(key >> shift);
        if (!active[b]) {
            X[i] = 0.0;
            degF[i] = 0;
        } else {
            const double alpha = alpha_b[b];
            double x = atomicExch(&r64[key], 0.0);      // a key listed twice would push once
            pi64[key] += alpha * x;
            if (x != 0.0) atomicAdd(&s_taken[b], alpha * x);
            int32_t d = deg[v];
            X[i] = ((1.0 - alpha) * x) / (double)d;
            degF[i] = d;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < Bw && s_taken[threadIdx.x] != 0.0) atomicAdd(&taken[threadIdx.x], s_taken[threadIdx.x]);
}

// First index i with a[i] <= key < a[i+1] (a ascending, a[0] = 0 <= key < a[len]).
__device__ inline int64_t find_owner64(const int64_t* __restrict__ a, int64_t len, int64_t key) {
    int64_t lo = 0, hi = len;
    while (hi - lo > 1) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= key) lo = mid; else hi = mid;
    }
    return lo;
}

// First index i in [lo, hi] with a[i] <= key < a[i+1], given a[lo] <= key and
// key < a[hi + 1].
__device__ inline int64_t find_owner_in(const int64_t* __restrict__ a, int64_t lo, int64_t hi, int64_t key) {
    int64_t h = hi + 1;
    while (h - lo > 1) {
        int64_t mid = lo + ((h - lo) >> 1);
        if (a[mid] <= key) lo = mid; else h = mid;
    }
    return lo;
}

// Edge slot t of the frontier's out-edges: r(u) += X (FP64 atomic).  Residues
// only grow here, so exactly one add carries r(u) across d_u * rmax; that
// lane appends (u, column) to the next frontier.  Persistent blocks take 256
// consecutive slots per round.  A round's crossings are counted in LDS: one
// global atomic per block and round reserves their next-frontier entries,
// and the per-column counts and volumes reach the global counters once per
// block and column at the end (a global atomic per crossing serialized on
// the few counter addresses).  A slot's owner (frontier entry) is searched
// between the owners of the round's first and last slot.
__global__ __launch_bounds__(kBlock) void push_k(
        const int64_t* __restrict__ F, const int64_t* __restrict__ off, int64_t nf, int64_t vol, int shift,
        const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const int32_t* __restrict__ deg,
        const double* __restrict__ X, const double* __restrict__ rmaxb, double* __restrict__ r64,
        int64_t* __restrict__ F_next,
        int64_t cap, unsigned long long* __restrict__ tail, unsigned long long* __restrict__ cnt_b,
        unsigned long long* __restrict__ vol_b) {
    __shared__ unsigned long long s_cnt[128], s_vol[128];
    __shared__ int64_t s_lo, s_hi;
    __shared__ unsigned long long s_base;
    __shared__ unsigned int s_n;
    const int lane = threadIdx.x & 63;
    const int Bw = 1 << shift;
    if ((int)threadIdx.x < 128) s_cnt[threadIdx.x] = s_vol[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) s_n = 0u;
    if (off[nf] < vol) vol = off[nf];
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t0 = (int64_t)blockIdx.x * kBlock; t0 < vol; t0 += stride) {
        if (threadIdx.x == 0) s_lo = find_owner64(off, nf, t0);
        if (threadIdx.x == 64) s_hi = find_owner64(off, nf, min(t0 + kBlock, vol) - 1);
        __syncthreads();
        const int64_t lo = s_lo, hi = s_hi;
        const int64_t t = t0 + threadIdx.x;
        bool crossed = false;
        int64_t tkey = 0;
        if (t < vol) {
            int64_t i = find_owner_in(off, lo, hi, t);
            int64_t key = F[i];
            int32_t b = (int32_t)(key & (Bw - 1));
            int32_t v = (int32_t)(key >> shift);
            int64_t e = row_ptr[v] + (t - off[i]);
            int32_t u = col[e];
            tkey = ((int64_t)u << shift) + b;
            double x = X[i];
            double old = atomicAdd(&r64[tkey], x);
            double now = old + x;
            int32_t du = deg[u];
            double thr = (double)du * rmaxb[b];     // rmax = lambda_b / m of this column
            crossed = (old <= thr) && (now > thr);
            if (crossed) {
                atomicAdd(&s_cnt[b], 1ull);
                atomicAdd(&s_vol[b], (unsigned long long)du);
            }
        }
        const uint64_t mask = __ballot(crossed);
        const int leader = mask ? __ffsll((unsigned long long)mask) - 1 : 0;
        unsigned int woff = 0u;
        if (mask && lane == leader) woff = atomicAdd(&s_n, (unsigned int)__popcll(mask));
        __syncthreads();                             // the round's counts are in s_n
        if (threadIdx.x == 0) {
            const unsigned int tot = s_n;
            s_n = 0u;
            s_base = tot ? atomicAdd(tail, (unsigned long long)tot) : 0ull;
        }
        __syncthreads();                             // s_base holds the round's first entry
        if (mask) {
            woff = __shfl(woff, leader, 64);
            const unsigned int below = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                         __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
            // the host sizes F_next for the worst case; the guard keeps a
            // violation of that bound from writing out of bounds (the host
            // then sees tail > cap and fails the call)
            const unsigned long long slot = s_base + woff + below;
            if (crossed && (int64_t)slot < cap) F_next[slot] = tkey;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < Bw && s_cnt[threadIdx.x]) {
        atomicAdd(&cnt_b[threadIdx.x], s_cnt[threadIdx.x]);
        atomicAdd(&vol_b[threadIdx.x], s_vol[threadIdx.x]);
    }
}

// FP64 scratch -> block for the columns with cmask = 1, dense over (u, b):
// y = (1-alpha) r / d; the local phase's reserve (1-alpha) pi / (alpha d)
// enters through the stage accumulator T (FP32), with S = AS = 0 (not
// written here: the column's first refresh runs with rmask 2 and takes both
// as 0), so that the first refresh gathers it like any stage's increments
// (its FP32 rounding is residual that refresh measures); the scratch of
// those columns is cleared.  The residue is fresh (nobody has
// pulled it), so the first sweep of the column runs with its entry flag:
// it folds the alpha-part into T and pulls y along every in-edge.
// partials[block][B]: per-column sums of r.
// Each thread takes four consecutive elements (one node, columns 4j .. 4j + 3;
// j fixed, since the grid's thread count is a multiple of B / 4) per step:
// two 32-byte loads of each FP64 array and one vector store of each output
// when all four columns convert, one element at a time otherwise.
__device__ inline void convert_one(int64_t i, double alpha, double d, double* __restrict__ r64,
                                   double* __restrict__ pi64, void* __restrict__ Y, int y_bf16,
                                   float* __restrict__ T, double& acc) {
    const double r = r64[i];
    const double p = pi64[i];
    const double y = ((1.0 - alpha) * r) / d;
    if (y_bf16)
        reinterpret_cast<uint16_t*>(Y)[i] = (uint16_t)bf16_bits((float)y);
    else
        reinterpret_cast<float*>(Y)[i] = (float)y;
    T[i] = (float)(((1.0 - alpha) * p) / (alpha * d));
    if (r != 0.0) r64[i] = 0.0;        // the scratch is mostly zero already
    if (p != 0.0) pi64[i] = 0.0;
    acc += r;
}

__global__ __launch_bounds__(kBlock) void convert_k(int32_t n, int shift, const int32_t* __restrict__ deg,
                                                    const double* __restrict__ alpha_b,
                                                    const int32_t* __restrict__ cmask, double* __restrict__ r64,
                                                    double* __restrict__ pi64, void* __restrict__ Y, int y_bf16,
                                                    float* __restrict__ T, double* __restrict__ partials) {
    __shared__ double sh[kBlock * 4];
    const int B = 1 << shift;
    const int Q = B >> 2;
    const int j = threadIdx.x & (Q - 1);
    const int b0 = 4 * j;
    const bool m0 = cmask[b0] != 0, m1 = cmask[b0 + 1] != 0, m2 = cmask[b0 + 2] != 0, m3 = cmask[b0 + 3] != 0;
    const double a0 = alpha_b[b0], a1 = alpha_b[b0 + 1], a2 = alpha_b[b0 + 2], a3 = alpha_b[b0 + 3];
    double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
    const int64_t quads = (int64_t)n << (shift - 2);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (m0 && m1 && m2 && m3) {
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < quads; q += stride) {
            const double d = (double)deg[q >> (shift - 2)];
            double2* r2 = reinterpret_cast<double2*>(r64) + 2 * q;
            double2* p2 = reinterpret_cast<double2*>(pi64) + 2 * q;
            const double2 ra = r2[0], rb = r2[1], pa = p2[0], pb = p2[1];
            const float y0 = (float)(((1.0 - a0) * ra.x) / d), y1 = (float)(((1.0 - a1) * ra.y) / d);
            const float y2 = (float)(((1.0 - a2) * rb.x) / d), y3 = (float)(((1.0 - a3) * rb.y) / d);
            if (y_bf16)
                reinterpret_cast<uint2*>(Y)[q] = make_uint2(bf16_bits(y0) | (bf16_bits(y1) << 16),
                                                            bf16_bits(y2) | (bf16_bits(y3) << 16));
            else
                reinterpret_cast<float4*>(Y)[q] = make_float4(y0, y1, y2, y3);
            reinterpret_cast<float4*>(T)[q] = make_float4((float)(((1.0 - a0) * pa.x) / (a0 * d)),
                                                          (float)(((1.0 - a1) * pa.y) / (a1 * d)),
                                                          (float)(((1.0 - a2) * pb.x) / (a2 * d)),
                                                          (float)(((1.0 - a3) * pb.y) / (a3 * d)));
            const double2 z = make_double2(0.0, 0.0);
            if (ra.x != 0.0 || ra.y != 0.0) r2[0] = z;
            if (rb.x != 0.0 || rb.y != 0.0) r2[1] = z;
            if (pa.x != 0.0 || pa.y != 0.0) p2[0] = z;
            if (pb.x != 0.0 || pb.y != 0.0) p2[1] = z;
            c0 += ra.x;
            c1 += ra.y;
            c2 += rb.x;
            c3 += rb.y;
        }
    } else if (m0 || m1 || m2 || m3) {
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < quads; q += stride) {
            const double d = (double)deg[q >> (shift - 2)];
            if (m0) convert_one(4 * q, a0, d, r64, pi64, Y, y_bf16, T, c0);
            if (m1) convert_one(4 * q + 1, a1, d, r64, pi64, Y, y_bf16, T, c1);
            if (m2) convert_one(4 * q + 2, a2, d, r64, pi64, Y, y_bf16, T, c2);
            if (m3) convert_one(4 * q + 3, a3, d, r64, pi64, Y, y_bf16, T, c3);
        }
    }
    sh[4 * threadIdx.x + 0] = c0;
    sh[4 * threadIdx.x + 1] = c1;
    sh[4 * threadIdx.x + 2] = c2;
    sh[4 * threadIdx.x + 3] = c3;
    __syncthreads();
    if ((int)threadIdx.x < Q) {
        double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
        for (int t = threadIdx.x; t < kBlock; t += Q) {
            t0 += sh[4 * t + 0];
            t1 += sh[4 * t + 1];
            t2 += sh[4 * t + 2];
            t3 += sh[4 * t + 3];
        }
        double* out = partials + (int64_t)blockIdx.x * B + b0;
        out[0] = t0;
        out[1] = t1;
        out[2] = t2;
        out[3] = t3;
    }
}
__global__ __launch_bounds__(kBlock) void reduce_cols_k(const double* __restrict__ partials, int nparts, int B,
                                                        double* __restrict__ out) {
    __shared__ double sh[kBlock];
    const int b = blockIdx.x;
    double t = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) t += partials[(int64_t)i * B + b];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int s = kBlock / 2; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = sh[0];
}

__global__ void scale_k(const int32_t* __restrict__ deg, int32_t n, double alpha, float* __restrict__ scale) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        scale[i] = (float)((1.0 - alpha) / (double)deg[i]);
}

// ---------------------------------------------------------------- sweep
// One launch handles one row chunk [lo, ...) of the sweep.  Row u of the
// chunk reads the residue of in-neighbour v from Y_out (produced earlier in
// this sweep) when v < lo, else from Y_in (the previous sweep): block
// Gauss-Seidel order, every residue increment still pulled exactly once by
// each out-neighbour.  With one chunk (lo = 0) this is the plain Eq. 7 step.
// On the first sweep of a sequence (step == 0) a column with its entry flag
// set holds a fresh residue in Y_in that nobody has pulled yet: its rows pull
// it along every in-edge, in addition to the new values of earlier chunks.
//
// Schedule blocks: up to Sw<C, L>::kRows whole rows with <= Sw<C, L>::kNnz in-edges
// (one round), or one long row of up to kLongRounds rounds of Sw<C, L>::kNnz
// in-edges, or one piece (kLongRounds rounds) of a longer row.  C is the
// number of 16-byte vectors per row (B / 4 in FP32, B / 8 in bf16).  Per
// round, indices are loaded first, then every thread has kItems 16-byte
// gathers in flight, staged in LDS as stored; T2 threads per (row, vector)
// add the row's slice in FP32.
// A piece writes its raw sum to a partial slot; combine_k adds a long row's
// pieces in slot order and finishes the row.  Y_out is read (rows < lo) and written
// (rows >= lo) in the same launch, so it carries no __restrict__.
// An entry sweep of a later chunk: what a source in an earlier chunk hands
// over is its new value plus the fresh residue nobody has pulled yet (exact in
// FP32; one more rounding in bf16), for the fresh columns (enf = 1); a source
// in this or a later chunk hands over its fresh residue.
// fm: bit j set when column j of the vector is fresh; the residue of a
// column that is not fresh is multiplied by 0 (so the sum has the same bits
// as with a 0/1 factor per column).
__device__ inline float fresh_part(float x, uint32_t fm, int j) { return ((fm >> j) & 1u) ? x : x * 0.f; }

template <typename ST>
__device__ inline typename ST::V entry_value(typename ST::V y_out, typename ST::V y_in, uint32_t fm) {
    if (fm == 0u) return y_out;
    Vec<ST::K> r = ST::value(y_in);
#pragma unroll
    for (int i = 0; i < ST::K / 4; ++i)
        r.q[i] = make_float4(fresh_part(r.q[i].x, fm, 4 * i), fresh_part(r.q[i].y, fm, 4 * i + 1),
                             fresh_part(r.q[i].z, fm, 4 * i + 2), fresh_part(r.q[i].w, fm, 4 * i + 3));
    return ST::pack(v_add(ST::value(y_out), r));
}

// y'(u) = scale(u) * acc for the columns inside their sweep budget (0 for the
// others).  T collects, per column, the fresh residue of an entry sweep and
// every residue a sweep stores (what the out-neighbours pull).  Sweeps go in
// pairs: an odd step adds its input (the stored output of the even step
// before it) and its own output, and an even step leaves T alone, except the
// last step of a sequence, which adds its output whatever its parity.  A
// column past its budget stores 0, so the odd step after its last sweep still
// adds that sweep's output.  Entry flag 2 marks a column whose T the refresh
// has already moved into S: its entry sweep overwrites T instead of adding.
// SOR: the node holds p = q + scale(u) * acc, where q is what it kept back
// last sweep, pushes y' = omega p and keeps (1 - omega) p.  What it kept back
// is (1 - omega) / omega times what it pushed, i.e. y' = omega scale(u) acc +
// (1 - omega) y_prev(u) with y_prev(u) = Y_in(u), its previous push; a fresh
// residue (entry sweep) has kept nothing back.  A column leaves its budget
// only at the end of a stage, and the refresh that follows forms a new
// residue, so no kept-back part outlives a stage.
// Lane c holds columns K c .. K c + K - 1: vector c of row u in Y, float4s
// (u C + c) K/4 + i of T, int4s / float4s c K/4 + i of kb, entry, omega.
template <int C, bool SOR, typename ST, bool AF>
__device__ inline void finish_row(int32_t u, int c, Vec<ST::K> acc, int32_t step, int32_t last,
                                  const float* __restrict__ scale, const float* __restrict__ afac,
                                  const typename ST::V* __restrict__ Y_in, typename ST::V* Y_out,
                                  float4* __restrict__ T, const int32_t* __restrict__ kb,
                                  const int32_t* __restrict__ entry, const float* __restrict__ omega) {
    constexpr int K = ST::K, Q = K / 4;
    const int64_t at = (int64_t)u * C + c;
    const float sc = scale[u];
    Vec<K> m, en = v_zero<K>(), keep;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int4 kb4 = reinterpret_cast<const int4*>(kb)[c * Q + i];
        m.q[i] = make_float4(step < kb4.x ? 1.f : 0.f, step < kb4.y ? 1.f : 0.f, step < kb4.z ? 1.f : 0.f,
                             step < kb4.w ? 1.f : 0.f);
    }
    bool any_en = false;
    if (step == 0) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int4 e4 = reinterpret_cast<const int4*>(entry)[c * Q + i];
            en.q[i] = flag4(e4);
            keep.q[i] = make_float4(e4.x == 2 ? 0.f : 1.f, e4.y == 2 ? 0.f : 1.f, e4.z == 2 ? 0.f : 1.f,
                                    e4.w == 2 ? 0.f : 1.f);
            any_en |= (en.q[i].x + en.q[i].y + en.q[i].z + en.q[i].w) != 0.f;
        }
    }
    const bool odd = (step & 1) != 0;
    // the row's own input residue: the previous push (over-relaxation), the
    // even step's output (odd steps), the fresh residue (entry sweep)
    Vec<K> yin = v_zero<K>();
    if (SOR || odd || any_en) yin = ST::value(nt_ld(&Y_in[at]));
    acc = v_mul(acc, m);
    if constexpr (AF) {
        // the column's alpha factor on the scale table (instantiated only while
        // some column has another alpha than the block's reference alpha)
        Vec<K> f;
#pragma unroll
        for (int i = 0; i < Q; ++i) f.q[i] = reinterpret_cast<const float4*>(afac)[c * Q + i];
        acc = v_mul(acc, f);
    }
    Vec<K> y;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        y.q[i] = make_float4(sc * acc.q[i].x, sc * acc.q[i].y, sc * acc.q[i].z, sc * acc.q[i].w);
    if (SOR) {
        const Vec<K> yp = yin;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float4 w = reinterpret_cast<const float4*>(omega)[c * Q + i];
            const float4 mi = m.q[i], ei = en.q[i];
            const float4 k = make_float4(mi.x * (1.f - ei.x) * (1.f - w.x), mi.y * (1.f - ei.y) * (1.f - w.y),
                                         mi.z * (1.f - ei.z) * (1.f - w.z), mi.w * (1.f - ei.w) * (1.f - w.w));
            const float4 yi = y.q[i], pi = yp.q[i];
            y.q[i] = make_float4(w.x * yi.x + k.x * pi.x, w.y * yi.y + k.y * pi.y, w.z * yi.z + k.z * pi.z,
                                 w.w * yi.w + k.w * pi.w);
        }
    }
    const typename ST::V yq = ST::pack(y);
    nt_st(yq, &Y_out[at]);
    const Vec<K> ys = ST::value(yq);             // what the out-neighbours will pull
    if (odd) {
#pragma unroll
        for (int i = 0; i < Q; ++i) nt_st(f4_add(f4_add(nt_ld(&T[at * Q + i]), yin.q[i]), ys.q[i]), &T[at * Q + i]);
    } else if (any_en || step == last) {
        Vec<K> t;
#pragma unroll
        for (int i = 0; i < Q; ++i) t.q[i] = T[at * Q + i];
        if (any_en) t = v_add(v_mul(t, keep), v_mul(v_mul(yin, en), m));
        if (step == last) t = v_add(t, ys);
#pragma unroll
        for (int i = 0; i < Q; ++i) T[at * Q + i] = t.q[i];
    }
}

template <typename OffT, int C, bool SOR, typename ST, int L, bool AF>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void sweep_k(
        const OffT* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
        const RowBlock* __restrict__ blocks, int32_t lo, const float* __restrict__ scale,
        const float* __restrict__ afac,
        const typename ST::V* __restrict__ Y_in, typename ST::V* Y_out, float4* __restrict__ T,
        const int32_t* __restrict__ kb, const int32_t* __restrict__ entry, const int32_t* __restrict__ step_p,
        Vec<ST::K>* __restrict__ partials, const float* __restrict__ omega,
        const char* ybase, uint32_t oin, uint32_t oout, int32_t off32) {
    using P = Sw<C, L>;
    constexpr int K = ST::K, Q = K / 4;
    static_assert(sizeof(typename ST::V) == 16, "a staged vector is 16 bytes");
    __shared__ typename ST::V lds[L / 16];
    const RowBlock b = blocks[blockIdx.x];
    const int32_t step = step_p[0];
    const bool entry_gs = step == 0 && lo > 0;     // a first sweep of a later chunk
    const bool whole = b.piece == -1;              // whole rows, one round
    const int32_t r0 = b.r0;
    const int32_t R = whole ? b.r1 - r0 : 1;
    const int32_t ne = b.ne;
    const int64_t e0 = b.e0;
    // (row, chunk) groups of T2 consecutive lanes (inside one wave)
    int T2 = 1;
    while (T2 < 64 && 2 * T2 * R * C <= kBlock) T2 <<= 1;
    const int32_t grp = threadIdx.x / T2;
    const int sub = threadIdx.x % T2;
    const int32_t row = grp / C;
    const int c = grp % C;
    int32_t s0 = 0, s1 = 0;
    if (whole && row < R) {
        s0 = (int32_t)((int64_t)col_ptr[r0 + row] - e0);
        s1 = (int32_t)((int64_t)col_ptr[r0 + row + 1] - e0);
    }
    Vec<K> acc = v_zero<K>();
    // the wave's part of the stage (wave-uniform, so the DMA's LDS base is scalar)
    typename ST::V* const ldsw = lds + __builtin_amdgcn_readfirstlane(threadIdx.x & ~63u);
    const uint32_t lane16 = (threadIdx.x % C) * 16u;
    // a long row (or piece) runs rounds of P::kNnz in-edges through LDS
    for (int32_t base = 0; base < ne; base += P::kNnz) {
        const int32_t nr = min(P::kNnz, ne - base);
        int32_t vv[P::kItems];
        round_indices<C, P::kItems, true>(row_idx, e0 + base, nr, vv);
        if (!entry_gs) {
            // the gathers land in the stage directly (LDS DMA: 16 bytes per lane,
            // a wave's 64 lanes fill 64 consecutive vectors, exactly the layout
            // lds[t + 256 k]); they may only start once the previous round's
            // stage has been read
            if (base > 0) __syncthreads();
            if (off32) {
                // both residue blocks in one buffer of < 4 GiB: a 32-bit offset
                // from its base (the input block at oin, the output block at oout)
                const uint32_t lin = lane16 + oin, dout = oout - oin;   // mod 2^32
#pragma unroll
                for (int k = 0; k < P::kItems; ++k) {
                    if (vv[k] >= 0) {
                        const uint32_t o = (uint32_t)vv[k] * (uint32_t)(C * 16) + lin + (vv[k] < lo ? dout : 0u);
                        lds_dma16(ybase + o, ldsw + k * kBlock);
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < P::kItems; ++k) {
                    if (vv[k] >= 0) {
                        const int64_t i = (int64_t)vv[k] * C + (threadIdx.x % C);
                        const typename ST::V* src = vv[k] >= lo ? Y_in + i : Y_out + i;
                        lds_dma16(src, ldsw + k * kBlock);
                    }
                }
            }
        } else {
            // an entry sweep of a later chunk: every source's fresh residue
            // lands in the stage by DMA; a source in an earlier chunk also hands
            // over its new value, loaded into registers first and then combined
            // into this lane's own stage slot (lds[t + 256 k], where the DMA put
            // the residue)
            const int tc = threadIdx.x % C;
            typename ST::V yo[P::kItems];
#pragma unroll
            for (int k = 0; k < P::kItems; ++k)
                if (vv[k] >= 0 && vv[k] < lo) yo[k] = Y_out[(int64_t)vv[k] * C + tc];
            if (base > 0) __syncthreads();             // the previous round's LDS reads are done
#pragma unroll
            for (int k = 0; k < P::kItems; ++k)
                if (vv[k] >= 0) lds_dma16(Y_in + (int64_t)vv[k] * C + tc, ldsw + k * kBlock);
            // the entry flags of this thread's columns (every item of the thread
            // belongs to column chunk tc), read while the gathers are in flight
            uint32_t fm = 0u;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int4 e4 = reinterpret_cast<const int4*>(entry)[tc * Q + i];
                fm |= ((e4.x ? 1u : 0u) | (e4.y ? 2u : 0u) | (e4.z ? 4u : 0u) | (e4.w ? 8u : 0u)) << (4 * i);
            }
#pragma unroll
            for (int k = 0; k < P::kItems; ++k) {
                if (vv[k] >= 0 && vv[k] < lo) {
                    typename ST::V* slot = lds + threadIdx.x + k * kBlock;
                    *slot = entry_value<ST>(yo[k], *slot, fm);
                }
            }
        }
        __syncthreads();
        if (!whole && row == 0) { s0 = 0; s1 = nr; }
        for (int32_t e = s0 + sub; e < s1; e += T2) acc = v_add(acc, ST::value(lds[e * C + c]));
    }
    for (int o = T2 >> 1; o >= 1; o >>= 1) acc = v_add(acc, v_shfl_xor(acc, o));
    if (row >= R || sub != 0) return;
    if (b.piece >= 0) {
        partials[(int64_t)b.piece * C + c] = acc;
        return;
    }
    finish_row<C, SOR, ST, AF>(r0 + row, c, acc, step, step_p[1], scale, afac, Y_in, Y_out, T, kb, entry, omega);
}

// Long rows of one chunk: the pieces' partial sums added in slot order.
template <int C, bool SOR, typename ST, bool AF>
__global__ __launch_bounds__(kBlock) void combine_k(
        const LongRow* __restrict__ rows, int32_t count, const Vec<ST::K>* __restrict__ partials,
        const int32_t* __restrict__ step_p, const float* __restrict__ scale, const float* __restrict__ afac,
        const typename ST::V* __restrict__ Y_in, typename ST::V* Y_out, float4* __restrict__ T,
        const int32_t* __restrict__ kb, const int32_t* __restrict__ entry, const float* __restrict__ omega) {
    const int32_t i = (int32_t)blockIdx.x * (kBlock / C) + (int32_t)threadIdx.x / C;
    const int c = threadIdx.x % C;
    if (i >= count) return;
    const LongRow L = rows[i];
    const Vec<ST::K>* part = partials + (int64_t)L.first * C + c;
    Vec<ST::K> acc = v_zero<ST::K>();
    // eight pieces' loads in flight at a time; the sums still go in slot order
    int32_t p = 0;
    for (; p + 8 <= L.npieces; p += 8) {
        Vec<ST::K> v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = part[(int64_t)(p + k) * C];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc = v_add(acc, v[k]);
    }
    for (; p < L.npieces; ++p) acc = v_add(acc, part[(int64_t)p * C]);
    finish_row<C, SOR, ST, AF>(L.row, c, acc, step_p[0], step_p[1], scale, afac, Y_in, Y_out, T, kb, entry, omega);
}

__global__ void bump_step_k(int32_t* step) { step[0] += 1; }

// Element-wise format conversions of a residue block (used by the one-sweep
// test entry point).
__global__ void to_bf16_k(int64_t count, const float* __restrict__ src, uint16_t* __restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        dst[i] = (uint16_t)bf16_bits(src[i]);
}

__global__ void from_bf16_k(int64_t count, const uint16_t* __restrict__ src, float* __restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        dst[i] = __uint_as_float((uint32_t)src[i] << 16);
}

// ---------------------------------------------------------------- refresh (FP64)
// Persistent grid: block k handles schedule blocks k, k + G, ...  A schedule
// block is up to Rf<C>::kRows whole rows with <= Rf<C>::kNnz in-edges, or one
// long row, which the block runs in rounds of Rf<C>::kNnz in-edges.  Per
// round the in-neighbours' T rows are staged in LDS and T2 threads per (row,
// chunk) add them in FP64, then a shuffle tree.  The per-column sums of |rt|
// are deterministic: after each schedule block the threads c < C add that
// block's rows in row order into their own accumulators (columns 4c..4c+3),
// which go to partials[block][B].  S, AS: double[n][B], read as double2 pairs.
// A refreshed column (rmask) also moves its stage accumulator into the
// reserve, S += T: every access to S is the row's own, so this is safe while
// other blocks still gather T; the column's T is then stale, and its next
// entry sweep overwrites it (entry flag 2).  rmask 2 marks a column's first
// refresh after its conversion: its S and AS are taken as 0 (the conversion
// does not clear them).  The per-column values every row reads (source,
// rmask, 1 - alpha_b, 1 / (1 - alpha_b)) are copied into LDS once per block;
// the |rt| reduction reuses the LDS stage after a barrier.
// Threads per (row, column group) of a refresh block of R rows: the largest
// power of two up to 64 with 2 T2 R C <= 256 (1 for a long row).
template <int C>
__device__ inline int rf_threads(int32_t R) {
    int T2 = 1;
    while (T2 < 64 && 2 * T2 * R * C <= kBlock) T2 <<= 1;
    return T2;
}

// The loads a refresh block needs before its first gathers: its rows' in-edge
// bounds and, in the shuffled index form, the loader lanes' indices of its
// first round.  Every lane loads bounds (its own row's, or the block's first
// row's when it has none), and the values are used only by the block's own
// iteration, so that nothing here waits for them.
template <typename OffT, int C, int kItems, bool kPre>
__device__ inline void rf_prefetch(const OffT* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
                                   const RowBlock& b, OffT& p0, OffT& p1, int32_t& mine) {
    const bool whole = b.piece == -1;
    const int32_t R = whole ? b.r1 - b.r0 : 1;
    const int32_t row = (int32_t)(threadIdx.x / rf_threads<C>(R)) / C;
    const int32_t at = (whole && row < R) ? b.r0 + row : b.r0;
    p0 = col_ptr[at];
    p1 = col_ptr[at + 1];
    if constexpr (kPre) mine = round_index_load<C, kItems, false>(row_idx, b.e0, min(Rf<C>::kNnz, b.ne));
}

template <int B>
struct RfParams {
    int32_t src[B], rmask[B];
    double oma[B], inv[B];
};

template <typename OffT, int C, typename ST>
__global__ __launch_bounds__(kBlock) void refresh_k(
        const OffT* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
        const RowBlock* __restrict__ blocks, int32_t n_blocks,
        const int32_t* __restrict__ deg, const float4* __restrict__ T, double2* __restrict__ S,
        double2* __restrict__ AS, const int32_t* __restrict__ src, const int32_t* __restrict__ rmask,
        const double* __restrict__ acoef, int32_t Bw,
        typename ST::V* __restrict__ Y, double* __restrict__ rt_out, int32_t n,
        double* __restrict__ partials) {
    using P = Rf<C>;
    __shared__ float4 lds[P::kNnz * C];
    static_assert(sizeof(lds) >= kBlock * 4 * sizeof(double), "the |rt| reduction fits the stage");
    double* red = reinterpret_cast<double*>(lds);
    __shared__ RfParams<4 * C> rp;
    if ((int)threadIdx.x < 4 * C) {
        rp.src[threadIdx.x] = src[threadIdx.x];
        rp.rmask[threadIdx.x] = rmask[threadIdx.x];
        rp.oma[threadIdx.x] = acoef[Bw + threadIdx.x];        // 1 - alpha_b
        rp.inv[threadIdx.x] = acoef[2 * Bw + threadIdx.x];    // 1 / (1 - alpha_b)
    }
    __syncthreads();
    double cs0 = 0.0, cs1 = 0.0, cs2 = 0.0, cs3 = 0.0;   // threads c < C: |rt| of columns 4c..4c+3
    // Software pipeline over the schedule blocks: the next block's descriptor
    // is loaded during this block's gathers, and its rows' in-edge bounds and
    // (shuffled form) its first round's indices before this block's row
    // finish, so that those loads overlap this block's instead of waiting in
    // front of the next block's gathers.
    constexpr bool kPre = ShuffledIndices<C, P::kItems>::value;
    RowBlock b{};
    OffT p0 = 0, p1 = 0;
    int32_t mine = -1;
    if ((int32_t)blockIdx.x < n_blocks) {
        b = blocks[blockIdx.x];
        rf_prefetch<OffT, C, P::kItems, kPre>(col_ptr, row_idx, b, p0, p1, mine);
    }
    for (int32_t bi = blockIdx.x; bi < n_blocks; bi += gridDim.x) {
        const int32_t bn = bi + (int32_t)gridDim.x;
        RowBlock nb = b;
        const bool whole = b.piece == -1;
        const int32_t r0 = b.r0;
        const int32_t R = whole ? b.r1 - r0 : 1;
        const int32_t ne = b.ne;
        const int64_t e0 = b.e0;
        const int T2 = rf_threads<C>(R);
        const int32_t grp = threadIdx.x / T2;
        const int sub = threadIdx.x % T2;
        const int32_t row = grp / C;
        const int c = grp % C;
        int32_t s0 = 0, s1 = 0;
        if (whole && row < R) {
            s0 = (int32_t)((int64_t)p0 - e0);
            s1 = (int32_t)((int64_t)p1 - e0);
        }
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
        for (int32_t base = 0; base < ne; base += P::kNnz) {
            const int32_t nr = min(P::kNnz, ne - base);
            int32_t vv[P::kItems];
            if (kPre && base == 0) round_index_spread<C, P::kItems>(mine, vv);
            else round_indices<C, P::kItems, false>(row_idx, e0 + base, nr, vv);
            __syncthreads();                       // the previous LDS reads are done
            if (base == 0 && bn < n_blocks) nb = blocks[bn];
            // the in-neighbours' accumulator rows land in the stage by DMA (16
            // bytes per lane at the stage's wave layout lds[t + 256 k])
#pragma unroll
            for (int k = 0; k < P::kItems; ++k)
                if (vv[k] >= 0) lds_dma16(T + (int64_t)vv[k] * C + (threadIdx.x % C), lds + (threadIdx.x & ~63u) + k * kBlock);
            __syncthreads();
            if (!whole && row == 0) { s0 = 0; s1 = nr; }
            for (int32_t e = s0 + sub; e < s1; e += T2) {
                const float4 t = lds[e * C + c];
                g0 += (double)t.x;
                g1 += (double)t.y;
                g2 += (double)t.z;
                g3 += (double)t.w;
            }
        }
        if (ne <= 0 && bn < n_blocks) nb = blocks[bn];     // a block of rows without in-edges
        OffT np0 = 0, np1 = 0;
        int32_t nmine = -1;
        if (bn < n_blocks) rf_prefetch<OffT, C, P::kItems, kPre>(col_ptr, row_idx, nb, np0, np1, nmine);
        for (int o = T2 >> 1; o >= 1; o >>= 1) {
            g0 += __shfl_xor(g0, o, 64);
            g1 += __shfl_xor(g1, o, 64);
            g2 += __shfl_xor(g2, o, 64);
            g3 += __shfl_xor(g3, o, 64);
        }
        double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
        if (row < R && sub == 0) {
            const int32_t u = r0 + row;
            const int64_t at = (int64_t)u * C + c;
            const double d = (double)deg[u];
            const float4 t = T[at];
            const int4 s4 = reinterpret_cast<const int4*>(rp.src)[c];
            const int4 w4 = reinterpret_cast<const int4*>(rp.rmask)[c];
            double2 sa = S[2 * at], sb = S[2 * at + 1];
            double2 aa = AS[2 * at], ab = AS[2 * at + 1];
            if (w4.x == 2) sa.x = aa.x = 0.0;    // first refresh after the conversion
            if (w4.y == 2) sa.y = aa.y = 0.0;
            if (w4.z == 2) sb.x = ab.x = 0.0;
            if (w4.w == 2) sb.y = ab.y = 0.0;
            // the in-neighbour sums of S + T
            const double a0 = aa.x + g0, a1 = aa.y + g1, a2 = ab.x + g2, a3 = ab.y + g3;
            const double2 i01 = reinterpret_cast<const double2*>(rp.inv)[2 * c];
            const double2 i23 = reinterpret_cast<const double2*>(rp.inv)[2 * c + 1];
            t0 = (s4.x == u ? 1.0 : 0.0) - d * (sa.x + (double)t.x) * i01.x + a0;
            t1 = (s4.y == u ? 1.0 : 0.0) - d * (sa.y + (double)t.y) * i01.y + a1;
            t2 = (s4.z == u ? 1.0 : 0.0) - d * (sb.x + (double)t.z) * i23.x + a2;
            t3 = (s4.w == u ? 1.0 : 0.0) - d * (sb.y + (double)t.w) * i23.y + a3;
            if (w4.x | w4.y | w4.z | w4.w) {     // the refreshed columns keep the new sums
                AS[2 * at] = make_double2(w4.x ? a0 : aa.x, w4.y ? a1 : aa.y);
                AS[2 * at + 1] = make_double2(w4.z ? a2 : ab.x, w4.w ? a3 : ab.y);
                S[2 * at] = make_double2(w4.x ? sa.x + (double)t.x : sa.x, w4.y ? sa.y + (double)t.y : sa.y);
                S[2 * at + 1] = make_double2(w4.z ? sb.x + (double)t.z : sb.x, w4.w ? sb.y + (double)t.w : sb.y);
            }
            if (w4.x | w4.y | w4.z | w4.w) {     // other columns keep their bits (exact round trip)
                float4 y = ST::value4(Y[at]);
                const double2 o01 = reinterpret_cast<const double2*>(rp.oma)[2 * c];
                const double2 o23 = reinterpret_cast<const double2*>(rp.oma)[2 * c + 1];
                if (w4.x) y.x = (float)(o01.x * t0 / d);
                if (w4.y) y.y = (float)(o01.y * t1 / d);
                if (w4.z) y.z = (float)(o23.x * t2 / d);
                if (w4.w) y.w = (float)(o23.y * t3 / d);
                Y[at] = ST::pack4(y);
            }
            if (rt_out) {   // column-major FP64 residual [B][n]
                rt_out[(int64_t)(4 * c + 0) * n + u] = t0;
                rt_out[(int64_t)(4 * c + 1) * n + u] = t1;
                rt_out[(int64_t)(4 * c + 2) * n + u] = t2;
                rt_out[(int64_t)(4 * c + 3) * n + u] = t3;
            }
        }
        // |rt| of this block's rows into the accumulators of threads c < C, in row
        // order; red aliases the stage, so every thread must be done reading it
        __syncthreads();
        red[threadIdx.x * 4 + 0] = fabs(t0);
        red[threadIdx.x * 4 + 1] = fabs(t1);
        red[threadIdx.x * 4 + 2] = fabs(t2);
        red[threadIdx.x * 4 + 3] = fabs(t3);
        __syncthreads();
        if ((int)threadIdx.x < C) {
            for (int32_t rr = 0; rr < R; ++rr) {
                const int t = T2 * (rr * C + (int)threadIdx.x);
                cs0 += red[t * 4 + 0];
                cs1 += red[t * 4 + 1];
                cs2 += red[t * 4 + 2];
                cs3 += red[t * 4 + 3];
            }
        }
        __syncthreads();                           // red and the LDS stage are reused
        b = nb;
        p0 = np0;
        p1 = np1;
        mine = nmine;
    }
    if ((int)threadIdx.x < C) {
        double* out = partials + (int64_t)blockIdx.x * (4 * C) + 4 * threadIdx.x;
        out[0] = cs0;
        out[1] = cs1;
        out[2] = cs2;
        out[3] = cs3;
    }
}

// ---------------------------------------------------------------- export
// pi_hat(u, b) = alpha_b d_u S / (1 - alpha_b) for columns [b0, b0 +
// count), written row-major [count][n] through an LDS transpose of
// kNodes nodes x B columns (f: alpha_b / (1 - alpha_b) per column).
template <int C>
struct Ex {
    static constexpr int kNodes = (4 * C >= 128) ? 32 : 64;
};

template <int C>
__global__ __launch_bounds__(kBlock) void export_k(int32_t n, int32_t b0, int32_t count,
                                                   const int32_t* __restrict__ deg, const double* __restrict__ f,
                                                   const double* __restrict__ S, double* __restrict__ out) {
    constexpr int B = 4 * C;
    constexpr int kNodes = Ex<C>::kNodes;
    __shared__ double tile[kNodes * (B + 1)];
    const int64_t u0 = (int64_t)blockIdx.x * kNodes;
    // reserve pairs in (16-byte loads), the output streamed out (nobody
    // reads it back here)
    for (int i = threadIdx.x; i < kNodes * B / 2; i += kBlock) {
        const int du = (2 * i) / B, b = (2 * i) % B;
        const int64_t u = u0 + du;
        double2 v = make_double2(0.0, 0.0);
        if (u < n) {
            const double d = (double)deg[u];
            const double2 sv = reinterpret_cast<const double2*>(S)[(u * B + b) >> 1];
            v = make_double2(f[b] * d * sv.x, f[b + 1] * d * sv.y);
        }
        tile[du * (B + 1) + b] = v.x;
        tile[du * (B + 1) + b + 1] = v.y;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNodes * B; i += kBlock) {
        int b = i / kNodes, du = i % kNodes;
        int64_t u = u0 + du;
        if (b >= b0 && b < b0 + count && u < n)
            __builtin_nontemporal_store(tile[du * (B + 1) + b], &out[(int64_t)(b - b0) * n + u]);
    }
}

__global__ void export_col_k(int32_t n, int shift, int32_t b, const int32_t* __restrict__ deg,
                             const double* __restrict__ fb, const double* __restrict__ S, double* __restrict__ out) {
    const double f = fb[b];
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        int64_t i = (u << shift) + b;
        out[u] = f * (double)deg[u] * S[i];
    }
}

// ---------------------------------------------------------------- launch helpers
template <int C, int L>
const Schedule& sweep_schedule(Graph& g, int chunks) {
    return g.schedule(Sw<C, L>::kNnz, Sw<C, L>::kRows, chunks, kLongRounds);
}
// f(std::integral_constant<int, L>) for the context's sweep stage L
template <typename F>
void by_tile(int tile, F&& f) {
    switch (tile) {
        case kTiles[0]: f(std::integral_constant<int, kTiles[0]>{}); break;
        case kTiles[1]: f(std::integral_constant<int, kTiles[1]>{}); break;
        case kTiles[2]: f(std::integral_constant<int, kTiles[2]>{}); break;
        default: fail(PPR_ERR_ARG, "unsupported sweep tile");
    }
}
template <int C>
const Schedule& refresh_schedule(Graph& g) {
    return g.schedule(Rf<C>::kNnz, Rf<C>::kRows, 1, kRefreshRounds);   // long rows whole, in rounds
}

template <int C, bool SOR, typename ST, int L, bool AF>
void sweep_launch(MixedCtx& c, Graph& g, const void* yin, void* yout) {
    const Schedule& sch = sweep_schedule<C, L>(g, c.chunks);
    auto Y4i = reinterpret_cast<const typename ST::V*>(yin);
    auto Y4o = reinterpret_cast<typename ST::V*>(yout);
    const RowBlock* blocks = sch.blocks.as<RowBlock>();
    const LongRow* lrows = sch.longrows.as<LongRow>();
    auto part = c.piece_part.as<Vec<ST::K>>();
    const float* om = SOR ? c.omega.as<float>() : nullptr;
    const float* af = AF ? c.afac.as<float>() : nullptr;
    // 32-bit gather offsets when both blocks lie in the joint buffer and it is < 4 GiB
    const char* yb = c.Y01.as<const char>();
    const auto inside = [&](const void* y) {
        return static_cast<const char*>(y) >= yb && static_cast<const char*>(y) < yb + c.Y01.bytes;
    };
    const int32_t off32 = (yb && c.Y01.bytes <= 0xffffffffull && inside(yin) && inside(yout)) ? 1 : 0;
    const uint32_t oin = off32 ? (uint32_t)(static_cast<const char*>(yin) - yb) : 0u;
    const uint32_t oout = off32 ? (uint32_t)(static_cast<const char*>(yout) - yb) : 0u;
    for (int j = 0; j < sch.chunks; ++j) {      // chunk j sees the output of chunks < j
        const int32_t nb = sch.first[j + 1] - sch.first[j];
        if (nb == 0) continue;
        dim3 grid((unsigned)nb), blk(kBlock);
        const RowBlock* bj = blocks + sch.first[j];
        if (g.off64)
            hipLaunchKernelGGL((sweep_k<int64_t, C, SOR, ST, L, AF>), grid, blk, 0, c.stream, g.col_ptr.as<int64_t>(),
                               g.row_idx.as<int32_t>(), bj, sch.lo[j], c.scale.as<float>(), af, Y4i, Y4o,
                               c.T.as<float4>(), c.kb.as<int32_t>(), c.entry.as<int32_t>(), c.step.as<int32_t>(),
                               part, om, yb, oin, oout, off32);
        else
            hipLaunchKernelGGL((sweep_k<uint32_t, C, SOR, ST, L, AF>), grid, blk, 0, c.stream, g.col_ptr.as<uint32_t>(),
                               g.row_idx.as<int32_t>(), bj, sch.lo[j], c.scale.as<float>(), af, Y4i, Y4o,
                               c.T.as<float4>(), c.kb.as<int32_t>(), c.entry.as<int32_t>(), c.step.as<int32_t>(),
                               part, om, yb, oin, oout, off32);
        const int32_t nl = sch.lr_first[j + 1] - sch.lr_first[j];
        if (nl > 0) {
            const int per = kBlock / C;
            hipLaunchKernelGGL((combine_k<C, SOR, ST, AF>), dim3((unsigned)((nl + per - 1) / per)), dim3(kBlock), 0,
                               c.stream, lrows + sch.lr_first[j], nl, part, c.step.as<int32_t>(),
                               c.scale.as<float>(), af, Y4i, Y4o, c.T.as<float4>(), c.kb.as<int32_t>(),
                               c.entry.as<int32_t>(), om);
        }
    }
    hipLaunchKernelGGL(bump_step_k, dim3(1), dim3(1), 0, c.stream, c.step.as<int32_t>());
    HIPCHECK(hipGetLastError());
}

// C = B / 4; bf16 sweeps run C / 2 vectors of 8 columns per row
template <int C>
void sweep_c(MixedCtx& c, Graph& g, const void* yin, void* yout) {
    by_tile(c.tile, [&](auto tl) {
        constexpr int L = decltype(tl)::value;
        auto go = [&](auto af) {
            constexpr bool AF = decltype(af)::value;
            if (c.bf16) {
                if constexpr (C >= 2) {
                    if (c.sor) sweep_launch<C / 2, true, StoreBF16x8, L, AF>(c, g, yin, yout);
                    else sweep_launch<C / 2, false, StoreBF16x8, L, AF>(c, g, yin, yout);
                } else {
                    fail(PPR_ERR_ARG, "bf16 residues need a block of at least 8 columns");
                }
            } else {
                if (c.sor) sweep_launch<C, true, StoreF32, L, AF>(c, g, yin, yout);
                else sweep_launch<C, false, StoreF32, L, AF>(c, g, yin, yout);
            }
        };
        if (c.af) go(std::true_type{});
        else go(std::false_type{});
    });
}

template <int C, typename ST>
void refresh_launch(MixedCtx& c, Graph& g, void* y, double* rt_out) {
    const Schedule& sch = refresh_schedule<C>(g);
    dim3 grid((unsigned)std::min(sch.n_blocks, kGridRed)), blk(kBlock);
    auto T4 = c.T.as<float4>();
    auto S2 = c.S.as<double2>();
    auto A2 = c.AS.as<double2>();
    auto Y4 = reinterpret_cast<typename ST::V*>(y);
    if (g.off64)
        hipLaunchKernelGGL((refresh_k<int64_t, C, ST>), grid, blk, 0, c.stream, g.col_ptr.as<int64_t>(),
                           g.row_idx.as<int32_t>(), sch.blocks.as<RowBlock>(), sch.n_blocks,
                           g.deg.as<int32_t>(), T4, S2, A2, c.src.as<int32_t>(), c.rmask.as<int32_t>(), c.acoef.as<double>(), c.Bw, Y4,
                           rt_out, g.n, c.partials.as<double>());
    else
        hipLaunchKernelGGL((refresh_k<uint32_t, C, ST>), grid, blk, 0, c.stream, g.col_ptr.as<uint32_t>(),
                           g.row_idx.as<int32_t>(), sch.blocks.as<RowBlock>(), sch.n_blocks,
                           g.deg.as<int32_t>(), T4, S2, A2, c.src.as<int32_t>(), c.rmask.as<int32_t>(), c.acoef.as<double>(), c.Bw, Y4,
                           rt_out, g.n, c.partials.as<double>());
    hipLaunchKernelGGL(reduce_cols_k, dim3((unsigned)c.Bw), dim3(kBlock), 0, c.stream, c.partials.as<double>(), (int)grid.x, c.Bw,
                       c.colsum.as<double>());
    HIPCHECK(hipGetLastError());
}

template <int C>
void refresh_c(MixedCtx& c, Graph& g, void* y, double* rt_out) {
    if (c.bf16) refresh_launch<C, StoreBF16>(c, g, y, rt_out);
    else refresh_launch<C, StoreF32>(c, g, y, rt_out);
}

template <int C>
void export_c(MixedCtx& c, Graph& g, int b0, int count, double* out) {
    constexpr int kNodes = Ex<C>::kNodes;
    unsigned grid = (unsigned)((g.n + kNodes - 1) / kNodes);
    hipLaunchKernelGGL((export_k<C>), dim3(grid), dim3(kBlock), 0, c.stream, g.n, b0, count, g.deg.as<int32_t>(),
                       c.acoef.as<double>() + 3 * c.Bw, c.S.as<double>(), out);
    HIPCHECK(hipGetLastError());
}

template <class F>
void by_width(int Bw, F&& f) {
    switch (Bw) {
        case 4: f(std::integral_constant<int, 1>()); break;
        case 8: f(std::integral_constant<int, 2>()); break;
        case 16: f(std::integral_constant<int, 4>()); break;
        case 32: f(std::integral_constant<int, 8>()); break;
        case 64: f(std::integral_constant<int, 16>()); break;
        case 128: f(std::integral_constant<int, 32>()); break;
        default: fail(PPR_ERR_ARG, "block width must be a power of two in [4, 128]");
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers
void set_scale(Graph& g, MixedCtx& c, double alpha) {
    hipLaunchKernelGGL(scale_k, dim3(1024), dim3(kBlock), 0, c.stream, g.deg.as<int32_t>(), g.n, alpha,
                       c.scale.as<float>());
    HIPCHECK(hipGetLastError());
}

void init_sources(MixedCtx& c) {
    hipLaunchKernelGGL(init_sources_k, dim3(1), dim3(128), 0, c.stream, c.src.as<int32_t>(), c.cmask.as<int32_t>(),
                       c.Bw, c.shift, c.r64.as<double>());
    HIPCHECK(hipGetLastError());
}

void snapshot(MixedCtx& c, const Graph& g, const int64_t* F, int64_t nf) {
    unsigned gs = (unsigned)((nf + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(snapshot_k, dim3(gs), dim3(kBlock), 0, c.stream, F, nf, c.shift, c.active.as<uint8_t>(),
                       g.deg.as<int32_t>(), c.acoef.as<double>(), c.r64.as<double>(), c.pi64.as<double>(), c.X.as<double>(),
                       c.degF.as<int64_t>(), c.taken.as<double>());
    HIPCHECK(hipGetLastError());
}

void push(MixedCtx& c, const Graph& g, const int64_t* F, int64_t nf, int64_t vol, int64_t* F_next) {
    if (vol <= 0) return;
    // persistent: 8 blocks per CU of a 256-CU device
    unsigned gp = (unsigned)std::min<int64_t>((vol + kBlock - 1) / kBlock, 2048);
    auto* ctr = reinterpret_cast<unsigned long long*>(c.ctr.p);
    hipLaunchKernelGGL(push_k, dim3(gp), dim3(kBlock), 0, c.stream, F, c.off.as<int64_t>(), nf, vol, c.shift,
                       g.row_ptr.as<int64_t>(), g.col.as<int32_t>(), g.deg.as<int32_t>(), c.X.as<double>(),
                       c.rmaxb.as<double>(), c.r64.as<double>(), F_next, c.fcap, ctr, ctr + 1, ctr + 1 + c.Bw);
    HIPCHECK(hipGetLastError());
}

void convert(MixedCtx& c, const Graph& g) {
    const unsigned gc = kGridRed;       // partials hold kGridRed rows
    hipLaunchKernelGGL(convert_k, dim3(gc), dim3(kBlock), 0, c.stream, g.n, c.shift, g.deg.as<int32_t>(),
                       c.acoef.as<double>(),
                       c.cmask.as<int32_t>(), c.r64.as<double>(), c.pi64.as<double>(),
                       const_cast<void*>(c.ycur), c.bf16 ? 1 : 0, c.T.as<float>(), c.partials.as<double>());
    hipLaunchKernelGGL(reduce_cols_k, dim3((unsigned)c.Bw), dim3(kBlock), 0, c.stream, c.partials.as<double>(), (int)gc, c.Bw,
                       c.colsum.as<double>());
    HIPCHECK(hipGetLastError());
}

void prepare(MixedCtx& c, const Graph& g) {
    Graph& gg = const_cast<Graph&>(g);
    by_width(c.Bw, [&](auto cc) {
        constexpr int C = decltype(cc)::value;
        int32_t n_pieces = 0;
        by_tile(c.tile, [&](auto tl) {
            constexpr int L = decltype(tl)::value;
            if (c.bf16) {
                if constexpr (C >= 2) n_pieces = sweep_schedule<C / 2, L>(gg, c.chunks).n_pieces;
                else fail(PPR_ERR_ARG, "bf16 residues need a block of at least 8 columns");
            } else {
                n_pieces = sweep_schedule<C, L>(gg, c.chunks).n_pieces;
            }
        });
        const size_t need = (size_t)std::max(n_pieces, 1) * (size_t)c.Bw * 4;   // FP32 per piece and column
        if (c.piece_part.bytes < need) {
            c.drop_chunks();                   // a captured chunk holds the old buffer
            c.piece_part.alloc(need);
        }
        (void)refresh_schedule<decltype(cc)::value>(gg);
    });
}

void sweep(MixedCtx& c, const Graph& g, const void* y_in, void* y_out) {
    Graph& gg = const_cast<Graph&>(g);
    by_width(c.Bw, [&](auto cc) { sweep_c<decltype(cc)::value>(c, gg, y_in, y_out); });
}

void store_from_f32(MixedCtx& c, const float* src, void* dst, int64_t count) {
    if (!c.bf16) {
        HIPCHECK(hipMemcpyAsync(dst, src, 4 * (size_t)count, hipMemcpyDeviceToDevice, c.stream));
        return;
    }
    hipLaunchKernelGGL(to_bf16_k, dim3(1024), dim3(kBlock), 0, c.stream, count, src,
                       reinterpret_cast<uint16_t*>(dst));
    HIPCHECK(hipGetLastError());
}

void store_to_f32(MixedCtx& c, const void* src, float* dst, int64_t count) {
    if (!c.bf16) {
        HIPCHECK(hipMemcpyAsync(dst, src, 4 * (size_t)count, hipMemcpyDeviceToDevice, c.stream));
        return;
    }
    hipLaunchKernelGGL(from_bf16_k, dim3(1024), dim3(kBlock), 0, c.stream, count,
                       reinterpret_cast<const uint16_t*>(src), dst);
    HIPCHECK(hipGetLastError());
}

void refresh(MixedCtx& c, const Graph& g, void* y, double* rt_out) {
    Graph& gg = const_cast<Graph&>(g);
    by_width(c.Bw, [&](auto cc) { refresh_c<decltype(cc)::value>(c, gg, y, rt_out); });
}

void export_cols(MixedCtx& c, const Graph& g, int b0, int count, double* out) {
    Graph& gg = const_cast<Graph&>(g);
    by_width(c.Bw, [&](auto cc) { export_c<decltype(cc)::value>(c, gg, b0, count, out); });
}

void export_col(MixedCtx& c, const Graph& g, int b, double* out) {
    hipLaunchKernelGGL(export_col_k, dim3(2048), dim3(kBlock), 0, c.stream, g.n, c.shift, b, g.deg.as<int32_t>(),
                       c.acoef.as<double>() + 3 * c.Bw, c.S.as<double>(), out);
    HIPCHECK(hipGetLastError());
}

}  // namespace mk
}  // namespace ppr
