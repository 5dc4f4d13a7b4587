// Device construction of the in-edge lists (CSC) from the CSR out-edges.
//
// The pull form of a global sweep needs, for every node u, the list of nodes
// v with an edge (v, u).  The paper pushes over the CSR (Section 5, global
// sequential scan); on the GPU each destination gathers from its in-list, so
// the transpose is built once per graph:
//   count in-degrees -> exclusive scan -> scatter -> sort every in-list.
// The scatter uses atomics (order inside a list is arbitrary); the sort makes
// every list ascending by source id, which is the order a counting-sort
// transpose produces, so the result is the same bit for bit on every run.
#include "ppr_internal.h"

namespace ppr {
namespace k {

namespace {

constexpr int kBlock = 256;

__global__ void deg_kernel(const int64_t* __restrict__ row_ptr, int32_t* __restrict__ deg, int32_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) deg[i] = (int32_t)(row_ptr[i + 1] - row_ptr[i]);
}

__global__ void count_kernel(const int32_t* __restrict__ col, int64_t m,
                             unsigned long long* __restrict__ cnt) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride)
        atomicAdd(&cnt[col[e]], 1ull);
}

// ---- exclusive scan of int64 (three passes: tile sums, scan of tile sums, tiles)
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;      // 4096 elements per tile
constexpr int kScanTopThreads = 1024;
constexpr int kScanTopItems = 64;                   // scan_top takes up to 65536 tiles (larger scans recurse)

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
    // Hillis-Steele over the block (kBlock threads) in shared memory
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int64_t add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t incl = sh[t];
    *total = sh[kBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ void scan_tiles_reduce(const int64_t* __restrict__ in, int64_t len, int64_t* __restrict__ tile_sums) {
    __shared__ int64_t sh[kBlock];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
        if (idx < len) s += in[idx];
    }
    int64_t tot;
    block_exclusive_scan(s, sh, &tot);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanTopThreads) void scan_top(int64_t* __restrict__ tile_sums, int64_t ntiles) {
    // single workgroup: exclusive scan in place, kScanTopThreads tile sums per
    // round (one load and one store per thread) with a running carry; no
    // per-thread arrays, so nothing spills and a small scan is two memory
    // round trips (it sits on the critical path of every frontier level)
    __shared__ int64_t sh[kScanTopThreads];
    const int t = threadIdx.x;
    int64_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += kScanTopThreads) {
        const int64_t idx = base + t;
        const int64_t v = (idx < ntiles) ? tile_sums[idx] : 0;
        sh[t] = v;
        __syncthreads();
        for (int off = 1; off < kScanTopThreads; off <<= 1) {
            const int64_t add = (t >= off) ? sh[t - off] : 0;
            __syncthreads();
            sh[t] += add;
            __syncthreads();
        }
        const int64_t incl = sh[t];
        const int64_t total = sh[kScanTopThreads - 1];
        if (idx < ntiles) tile_sums[idx] = carry + incl - v;
        carry += total;
        __syncthreads();                           // sh is rewritten by the next round
    }
}

__global__ void scan_tiles_apply(const int64_t* __restrict__ in, int64_t len,
                                 const int64_t* __restrict__ tile_sums, int64_t* __restrict__ out) {
    __shared__ int64_t sh[kBlock];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t vals[kScanItems];
    int64_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        vals[i] = (idx < len) ? in[idx] : 0;
        s += vals[i];
    }
    int64_t tot;
    int64_t run = block_exclusive_scan(s, sh, &tot) + tile_sums[blockIdx.x];
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        if (idx < len) out[idx] = run;
        run += vals[i];
    }
    // the grand total goes to out[len]
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) out[len] = tile_sums[blockIdx.x] + tot;
}

// ---- scatter: one wave per source row, lanes stride over the row
__global__ void scatter_kernel(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                               int32_t n, unsigned long long* __restrict__ fill,
                               int32_t* __restrict__ row_idx) {
    int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    int lane = threadIdx.x & 63;
    int64_t nwaves = (int64_t)gridDim.x * blockDim.x / 64;
    for (int64_t v = wave; v < n; v += nwaves) {
        int64_t e0 = row_ptr[v], e1 = row_ptr[v + 1];
        for (int64_t e = e0 + lane; e < e1; e += 64) {
            int32_t u = col[e];
            unsigned long long pos = atomicAdd(&fill[u], 1ull);
            row_idx[pos] = (int32_t)v;
        }
    }
}

// ---- segmented sort
// Bitonic network in the formulation where every comparator puts the smaller
// key at the lower index: merge stage k (blocks of size 2^k) first compares
// i with its mirror inside the block, then i with i ^ 2^j for j < k-1.  With
// all comparators ascending, positions past the end of a segment behave as
// +infinity and never move, so a segment of any length sorts in place as if
// padded to the next power of two.

__global__ void sort_small(const int64_t* __restrict__ col_ptr, int32_t* __restrict__ row_idx,
                           int32_t n, int32_t small_max, int32_t* __restrict__ mid_list,
                           int32_t* __restrict__ big_list, unsigned int* __restrict__ counts,
                           int32_t mid_max) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int64_t a = col_ptr[u], b = col_ptr[u + 1];
    int64_t len = b - a;
    if (len <= 1) return;
    if (len <= small_max) {
        int32_t* x = row_idx + a;
        for (int64_t i = 1; i < len; ++i) {       // insertion sort
            int32_t key = x[i];
            int64_t j = i - 1;
            while (j >= 0 && x[j] > key) { x[j + 1] = x[j]; --j; }
            x[j + 1] = key;
        }
    } else if (len <= mid_max) {
        unsigned int p = atomicAdd(&counts[0], 1u);
        mid_list[p] = (int32_t)u;
    } else {
        unsigned int p = atomicAdd(&counts[1], 1u);
        big_list[p] = (int32_t)u;
    }
}

constexpr int kMidMax = 4096;

__global__ __launch_bounds__(kBlock) void sort_mid(const int64_t* __restrict__ col_ptr,
                                                   int32_t* __restrict__ row_idx,
                                                   const int32_t* __restrict__ list) {
    __shared__ int32_t sh[kMidMax];
    int32_t u = list[blockIdx.x];
    int64_t a = col_ptr[u];
    int len = (int)(col_ptr[u + 1] - a);
    int P = 1;
    while (P < len) P <<= 1;
    for (int i = threadIdx.x; i < P; i += kBlock) sh[i] = (i < len) ? row_idx[a + i] : INT32_MAX;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < P / 2; t += kBlock) {
                // pair t: lower index i, partner p
                int blk = t / j, off = t % j;
                int i = blk * 2 * j + off;
                int p;
                if (j == (k >> 1)) {            // mirror inside the block of size k
                    int base = i & ~(k - 1);
                    p = base + (k - 1 - (i - base));
                } else {
                    p = i + j;
                }
                int x = sh[i], y = sh[p];
                if (x > y) { sh[i] = y; sh[p] = x; }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < len; i += kBlock) row_idx[a + i] = sh[i];
}

__global__ __launch_bounds__(1024) void sort_big(const int64_t* __restrict__ col_ptr,
                                                 int32_t* __restrict__ row_idx,
                                                 const int32_t* __restrict__ list) {
    int32_t u = list[blockIdx.x];
    int64_t a = col_ptr[u];
    int64_t len = col_ptr[u + 1] - a;
    int32_t* x = row_idx + a;
    int64_t P = 1;
    while (P < len) P <<= 1;
    for (int64_t k = 2; k <= P; k <<= 1) {
        for (int64_t j = k >> 1; j > 0; j >>= 1) {
            for (int64_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                int64_t blk = t / j, off = t % j;
                int64_t i = blk * 2 * j + off;
                int64_t p;
                if (j == (k >> 1)) {
                    int64_t base = i & ~(k - 1);
                    p = base + (k - 1 - (i - base));
                } else {
                    p = i + j;
                }
                if (p < len) {                    // positions >= len act as +infinity
                    int32_t xi = x[i], xp = x[p];
                    if (xi > xp) { x[i] = xp; x[p] = xi; }
                }
            }
            __syncthreads();
        }
    }
}

__global__ void narrow_kernel(const int64_t* __restrict__ in, uint32_t* __restrict__ out, int64_t len) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) out[i] = (uint32_t)in[i];
}

inline unsigned grid_for(int64_t items, int per_block = kBlock) {
    int64_t g = (items + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

void deg_from_rowptr(const int64_t* row_ptr, int32_t* deg, int32_t n, hipStream_t s) {
    hipLaunchKernelGGL(deg_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, row_ptr, deg, n);
    HIPCHECK(hipGetLastError());
}

void count_in(const int32_t* col, int64_t m, int64_t* cnt, hipStream_t s) {
    unsigned g = grid_for(m);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(count_kernel, dim3(g), dim3(kBlock), 0, s, col, m,
                       reinterpret_cast<unsigned long long*>(cnt));
    HIPCHECK(hipGetLastError());
}

size_t scan_tmp_bytes(int64_t len) {
    // level sizes t1 = ceil(len / tile), then recursively for the tile sums
    size_t total = 0;
    int64_t cur = len;
    for (int lvl = 0; lvl < 4; ++lvl) {
        int64_t tiles = (cur + kScanTile - 1) / kScanTile;
        if (tiles < 1) tiles = 1;
        total += 2 * (size_t)tiles + 2;
        if (tiles <= (int64_t)kScanTopThreads * kScanTopItems) break;
        cur = tiles;
    }
    return sizeof(int64_t) * total;
}

void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t len, void* tmp, hipStream_t s) {
    // tile sums -> (recursive) exclusive scan of the tile sums -> tiles
    int64_t tiles = (len + kScanTile - 1) / kScanTile;
    if (tiles < 1) tiles = 1;
    int64_t* ts = static_cast<int64_t*>(tmp);
    hipLaunchKernelGGL(scan_tiles_reduce, dim3((unsigned)tiles), dim3(kBlock), 0, s, in, len, ts);
    if (tiles <= (int64_t)kScanTopThreads * kScanTopItems) {
        hipLaunchKernelGGL(scan_top, dim3(1), dim3(kScanTopThreads), 0, s, ts, tiles);
    } else {
        // scan the tile sums into the space after them, then copy back in place
        int64_t* ts_out = ts + tiles + 1;
        exclusive_scan_i64(ts, ts_out, tiles, ts_out + tiles + 1, s);
        HIPCHECK(hipMemcpyAsync(ts, ts_out, sizeof(int64_t) * (size_t)tiles, hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL(scan_tiles_apply, dim3((unsigned)tiles), dim3(kBlock), 0, s, in, len, ts, out);
    HIPCHECK(hipGetLastError());
}

void scatter_in(const int64_t* row_ptr, const int32_t* col, int32_t n, const int64_t* col_ptr,
                int64_t* fill, int32_t* row_idx, hipStream_t s) {
    (void)col_ptr;
    unsigned g = grid_for((int64_t)n * 64);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(scatter_kernel, dim3(g), dim3(kBlock), 0, s, row_ptr, col, n,
                       reinterpret_cast<unsigned long long*>(fill), row_idx);
    HIPCHECK(hipGetLastError());
}

void sort_segments(const int64_t* col_ptr, int32_t* row_idx, int32_t n, int32_t max_len,
                   hipStream_t s) {
    (void)max_len;
    DevBuf lists(sizeof(int32_t) * 2 * (size_t)n + 64);
    int32_t* mid = lists.as<int32_t>();
    int32_t* big = mid + n;
    unsigned int* counts = reinterpret_cast<unsigned int*>(big + n);
    HIPCHECK(hipMemsetAsync(counts, 0, 16, s));
    hipLaunchKernelGGL(sort_small, dim3(grid_for(n)), dim3(kBlock), 0, s, col_ptr, row_idx, n, 32,
                       mid, big, counts, kMidMax);
    HIPCHECK(hipGetLastError());
    unsigned int h[2] = {0, 0};
    HIPCHECK(hipMemcpyAsync(h, counts, 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (h[0]) hipLaunchKernelGGL(sort_mid, dim3(h[0]), dim3(kBlock), 0, s, col_ptr, row_idx, mid);
    if (h[1]) hipLaunchKernelGGL(sort_big, dim3(h[1]), dim3(1024), 0, s, col_ptr, row_idx, big);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
}

// ---- source slices of the FP64 sweep
// The first node of slice s of S: ceil(s n / S) (node v is in slice floor(v S / n)).
__device__ inline int32_t slice_first(int32_t s, int32_t n, int32_t S) {
    return (int32_t)(((int64_t)s * n + S - 1) / S);
}
// First position in the ascending list row_idx[a, b) whose source is >= v.
__device__ inline int64_t lower_src(const int32_t* __restrict__ row_idx, int64_t a, int64_t b, int32_t v) {
    while (a < b) {
        const int64_t mid = a + (b - a) / 2;
        if (row_idx[mid] < v) a = mid + 1;
        else b = mid;
    }
    return a;
}
__global__ void slice_count_kernel(const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
                                   int32_t n, int32_t S, int64_t* __restrict__ cnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        const int64_t b = col_ptr[u + 1];
        int64_t lo = col_ptr[u];
        for (int32_t s = 0; s < S; ++s) {
            const int64_t hi = (s + 1 < S) ? lower_src(row_idx, lo, b, slice_first(s + 1, n, S)) : b;
            cnt[(int64_t)s * n + u] = hi - lo;
            lo = hi;
        }
    }
}
__global__ void slice_scatter_kernel(const int64_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
                                     int32_t n, int32_t S, const int64_t* __restrict__ off,
                                     int32_t* __restrict__ sl_idx) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        const int64_t b = col_ptr[u + 1];
        int64_t lo = col_ptr[u];
        for (int32_t s = 0; s < S; ++s) {
            const int64_t hi = (s + 1 < S) ? lower_src(row_idx, lo, b, slice_first(s + 1, n, S)) : b;
            int64_t o = off[(int64_t)s * n + u];
            for (int64_t e = lo; e < hi; ++e) sl_idx[o++] = row_idx[e];
            lo = hi;
        }
    }
}

__global__ void nonzero_flags_kernel(const int64_t* __restrict__ cnt, int64_t len, int64_t* __restrict__ f) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) f[i] = cnt[i] > 0 ? 1 : 0;
}
__global__ void slice_compact_kernel(const int64_t* __restrict__ cnt, const int64_t* __restrict__ pos,
                                     const int64_t* __restrict__ off, int64_t len, int32_t n,
                                     int32_t* __restrict__ rows, int64_t* __restrict__ cptr) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
        if (cnt[i] > 0) {
            rows[pos[i]] = (int32_t)(i % n);
            cptr[pos[i]] = off[i];
        }
    }
}

void nonzero_flags(const int64_t* cnt, int64_t len, int64_t* flags, hipStream_t s) {
    unsigned g = grid_for(len);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(nonzero_flags_kernel, dim3(g), dim3(kBlock), 0, s, cnt, len, flags);
    HIPCHECK(hipGetLastError());
}

void slice_compact(const int64_t* cnt, const int64_t* pos, const int64_t* off, int64_t len, int32_t n,
                   int32_t* rows, int64_t* cptr, hipStream_t s) {
    unsigned g = grid_for(len);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(slice_compact_kernel, dim3(g), dim3(kBlock), 0, s, cnt, pos, off, len, n, rows, cptr);
    HIPCHECK(hipGetLastError());
}

void slice_count(const int64_t* col_ptr, const int32_t* row_idx, int32_t n, int32_t S, int64_t* cnt,
                 hipStream_t s) {
    unsigned g = grid_for(n);
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(slice_count_kernel, dim3(g), dim3(kBlock), 0, s, col_ptr, row_idx, n, S, cnt);
    HIPCHECK(hipGetLastError());
}

void slice_scatter(const int64_t* col_ptr, const int32_t* row_idx, int32_t n, int32_t S, const int64_t* off,
                   int32_t* sl_idx, hipStream_t s) {
    unsigned g = grid_for(n);
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(slice_scatter_kernel, dim3(g), dim3(kBlock), 0, s, col_ptr, row_idx, n, S, off, sl_idx);
    HIPCHECK(hipGetLastError());
}

void narrow_offsets(const int64_t* in, uint32_t* out, int64_t len, hipStream_t s) {
    hipLaunchKernelGGL(narrow_kernel, dim3(grid_for(len)), dim3(kBlock), 0, s, in, out, len);
    HIPCHECK(hipGetLastError());
}

}  // namespace k
}  // namespace ppr
