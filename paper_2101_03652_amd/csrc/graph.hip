// Host side of graph creation: CSR validation, device upload, CSC build,
// sweep schedules, and the common helpers (errors, buffers).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <thread>

#include "ppr_internal.h"

namespace ppr {

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

[[noreturn]] void fail(ppr_status st, const std::string& msg) { throw Failure{st, msg}; }

void check_hip(hipError_t e, const char* what, const char* file, int line) {
    if (e == hipSuccess) return;
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    fail(e == hipErrorOutOfMemory ? PPR_ERR_OOM : PPR_ERR_DEVICE, buf);
}

bool is_device_ptr(const void* p, int device) {
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof a);
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();      // plain pageable host memory
        return false;
    }
    if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) {
        if (a.device != device) fail(PPR_ERR_ARG, "output buffer lives on another device than the graph");
        return true;
    }
    return false;
}

EventPair::EventPair() {
    HIPCHECK(hipEventCreate(&a));
    HIPCHECK(hipEventCreate(&b));
}
EventPair::~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
}
void EventPair::start(hipStream_t s) { HIPCHECK(hipEventRecord(a, s)); }
void EventPair::stop(hipStream_t s) { HIPCHECK(hipEventRecord(b, s)); }
double EventPair::elapsed_ms() const {
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, a, b));
    return (double)ms;
}

// ---------------------------------------------------------------- buffers
void DevBuf::alloc(size_t b) {
    release();
    if (b == 0) b = 8;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        char buf[160];
        snprintf(buf, sizeof buf, "hipMalloc of %zu bytes failed: %s", b, hipGetErrorString(e));
        fail(PPR_ERR_OOM, buf);
    }
    bytes = b;
}

void DevBuf::view(void* base, size_t b) {
    release();
    p = base;
    bytes = b;
    owned = false;
}

void DevBuf::release() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    owned = true;
}

void PinnedBuf::alloc(size_t b) {
    release();
    hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        fail(PPR_ERR_OOM, "hipHostMalloc failed");
    }
    bytes = b;
}

void PinnedBuf::release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
}

// ---------------------------------------------------------------- validation
// O(n + m) checks of the CSR, split over host threads by row range.  The
// failure reported is the one at the smallest node id.
void graph_validate(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t m) {
    if (row_ptr[0] != 0) fail(PPR_ERR_CSR, "row_ptr[0] must be 0");
    if (row_ptr[n] != m) fail(PPR_ERR_CSR, "row_ptr[n] must equal m");
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v])
            fail(PPR_ERR_CSR, "row_ptr is not monotone at node " + std::to_string(v));
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 65536) nt = 1;
    struct Found { ppr_status st = PPR_OK; int32_t at = -1; };
    std::vector<Found> found(nt);
    auto work = [&](unsigned t, int32_t a, int32_t b) {
        std::vector<int32_t> tmp;
        for (int32_t v = a; v < b; ++v) {
            int64_t e0 = row_ptr[v], e1 = row_ptr[v + 1];
            if (e1 == e0) { found[t] = {PPR_ERR_DANGLING, v}; return; }
            bool sorted = true;
            for (int64_t e = e0; e < e1; ++e) {
                int32_t u = col[e];
                if (u < 0 || u >= n) { found[t] = {PPR_ERR_CSR, v}; return; }
                if (e > e0 && col[e - 1] >= u) sorted = false;
            }
            if (!sorted) {
                tmp.assign(col + e0, col + e1);
                std::sort(tmp.begin(), tmp.end());
                if (std::adjacent_find(tmp.begin(), tmp.end()) != tmp.end()) {
                    found[t] = {PPR_ERR_DUPLICATE, v};
                    return;
                }
            }
        }
    };
    std::vector<std::thread> th;
    int32_t chunk = (int32_t)((n + (int64_t)nt - 1) / nt);
    for (unsigned t = 0; t < nt; ++t) {
        int32_t a = (int32_t)std::min<int64_t>((int64_t)t * chunk, n);
        int32_t b = (int32_t)std::min<int64_t>((int64_t)a + chunk, n);
        if (a < b) th.emplace_back(work, t, a, b);
    }
    for (auto& x : th) x.join();
    for (const Found& f : found) {      // threads cover ascending row ranges
        if (f.st == PPR_OK) continue;
        std::string at = std::to_string(f.at);
        if (f.st == PPR_ERR_CSR) fail(PPR_ERR_CSR, "column index out of range in the out-list of node " + at);
        if (f.st == PPR_ERR_DANGLING) fail(PPR_ERR_DANGLING, "node " + at + " has out-degree 0 (dead end)");
        fail(PPR_ERR_DUPLICATE, "duplicate edge in the out-list of node " + at);
    }
}

// ---------------------------------------------------------------- graph
Graph::~Graph() {
    // contexts first: their streams and captured graphs reference this graph
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    mixed_pool.clear();
    pool.clear();
}

// Source slices of the FP64 sweep: enough that a slice of the FP64 residue
// vector (8 bytes per node) is at most kSliceBytes, at most kMaxSlices; graphs
// whose vector already fits get none.  Gathers from a smaller part of the
// vector hit the caches more often (the in-edge gathers alone of one sweep of
// the 4M-node graph: 0.85 ms from the whole 32 MB vector, 0.44 ms in 8 passes
// over 4 MB slices), but every pass also visits the rows with in-edges in its
// slice (offsets, the row sums read and written).  Measured per FP64 sweep
// (ms; slices 1 / 2 / 3 / 4 / 8 / 16): 4M nodes, 70M edges 0.89 / 0.79 / 0.75
// / 0.79 / 0.96; 16M, 300M 4.83 / 4.45 / - / 3.96 / 3.80; 40M, 1.4B 23.3 / - /
// 19.9 / - / 16.6 / 16.1.
constexpr size_t kSliceBytes = size_t(12) << 20;
constexpr int32_t kMaxSlices = 16;

int32_t fp64_slice_count(int32_t n, uint32_t flags) {
    const int32_t forced = (int32_t)((flags >> 8) & 0xffu);
    if (forced > 0) return std::min(forced, n);
    const size_t want = (8 * (size_t)n + kSliceBytes - 1) / kSliceBytes;
    return (int32_t)std::max<size_t>(1, std::min<size_t>(want, (size_t)kMaxSlices));
}

size_t graph_footprint(int32_t n, int64_t m) {
    const size_t nn = (size_t)n, mm = (size_t)m;
    const size_t off = (m >= (int64_t)UINT32_MAX) ? 8 : 4;  // CSC offsets: uint32 below 2^32 - 1 edges
    const size_t S = (size_t)fp64_slice_count(n, 0);
    // source slices: the in-edges, the listed (slice, row) pairs of all slices
    // but the last (at most (S - 1) n and at most m of them: row and offset
    // each) and the last slice's offsets; an upper bound (the pairs depend on
    // the graph)
    const size_t K = S > 1 ? std::min((S - 1) * nn, mm) : 0;
    return 8 * (nn + 1) + 4 * mm            // CSR: row_ptr, col
           + off * (nn + 1) + 4 * mm        // CSC: col_ptr, row_idx
           + 4 * nn                         // out-degrees
           + (S > 1 ? 4 * mm + (4 + off) * K + off + off * (nn + 1) : 0);
}

size_t Graph::device_bytes() const {
    size_t b = row_ptr.bytes + col.bytes + col_ptr.bytes + row_idx.bytes + deg.bytes + walk_index.bytes +
               sl_idx.bytes + sl_rows.bytes + sl_cptr.bytes + sl_last.bytes;
    return b;
}

const Schedule* Graph::find_schedule(int32_t nnz_cap, int32_t row_cap, int32_t chunks, int32_t rounds) {
    std::lock_guard<std::mutex> lk(sched_mu);
    chunks = std::max<int32_t>(1, std::min<int32_t>(chunks, n));
    const bool split = rounds > 0;
    for (auto& s : schedules)
        if (s->nnz_cap == nnz_cap && s->row_cap == row_cap && s->chunks == chunks && s->split == split &&
            s->rounds == std::max(rounds, 1))
            return s.get();
    return nullptr;
}

const Schedule& Graph::schedule(int32_t nnz_cap, int32_t row_cap, int32_t chunks, int32_t rounds) {
    std::lock_guard<std::mutex> lk(sched_mu);
    chunks = std::max<int32_t>(1, std::min<int32_t>(chunks, n));
    const bool split = rounds > 0;
    for (auto& s : schedules)
        if (s->nnz_cap == nnz_cap && s->row_cap == row_cap && s->chunks == chunks && s->split == split &&
            s->rounds == std::max(rounds, 1))
            return *s;
    schedules.push_back(make_schedule(h_col_ptr.data(), n, nnz_cap, row_cap, chunks, rounds));
    return *schedules.back();
}

std::unique_ptr<Schedule> make_schedule(const int64_t* cp, int32_t n, int32_t nnz_cap, int32_t row_cap,
                                        int32_t chunks, int32_t rounds) {
    chunks = std::max<int32_t>(1, std::min<int32_t>(chunks, n));
    const bool split = rounds > 0;
    // Row chunks: contiguous row ranges of about m / chunks in-edges each
    // (boundaries depend on the graph alone).  Inside a chunk, contiguous row
    // ranges with at most nnz_cap in-edges and row_cap rows.  A row with more
    // in-edges than nnz_cap gets a block of its own, listed first; with
    // rounds > 0 that block runs up to `rounds` rounds of nnz_cap in-edges,
    // and a row longer than that is cut into pieces of rounds * nnz_cap
    // in-edges whose partial sums are added afterwards.
    std::vector<int32_t> lo(chunks + 1, n);
    lo[0] = 0;
    const int64_t e_first = cp[0], e_all = cp[n] - cp[0];   // (an edge range of its own for a slice)
    for (int32_t j = 1; j < chunks; ++j) {
        const int64_t want = e_first + e_all * (int64_t)j / chunks;      // floor(m j / chunks) past cp[0]
        int32_t r = (int32_t)(std::lower_bound(cp, cp + n + 1, want) - cp);
        lo[j] = std::max(lo[j - 1], std::min(r, n));
    }
    std::vector<RowBlock> all;
    std::vector<LongRow> lrows;
    std::vector<int32_t> first(chunks + 1, 0), nlong(chunks, 0), lr_first(chunks + 1, 0);
    int32_t slot = 0;
    for (int32_t j = 0; j < chunks; ++j) {
        std::vector<RowBlock> longb, normal;
        lr_first[j] = (int32_t)lrows.size();
        int32_t r = lo[j];
        const int32_t rend = lo[j + 1];
        while (r < rend) {
            int64_t d = cp[r + 1] - cp[r];
            if (d > nnz_cap) {
                const int64_t piece_cap = (int64_t)nnz_cap * rounds;
                if (split && d <= piece_cap) {
                    longb.push_back({r, r + 1, (int32_t)d, -2, cp[r]});
                } else if (split) {
                    const int32_t np = (int32_t)((d + piece_cap - 1) / piece_cap);
                    lrows.push_back({r, slot, np, 0});
                    for (int32_t p = 0; p < np; ++p) {
                        const int64_t e = cp[r] + (int64_t)p * piece_cap;
                        longb.push_back({r, r + 1, (int32_t)std::min<int64_t>(piece_cap, cp[r + 1] - e), slot++, e});
                    }
                } else {
                    longb.push_back({r, r + 1, 0, -1, 0});
                }
                ++r;
                continue;
            }
            int32_t r0 = r;
            int64_t e = 0;
            while (r < rend && r - r0 < row_cap) {
                int64_t dd = cp[r + 1] - cp[r];
                if (dd > nnz_cap || e + dd > nnz_cap) break;
                e += dd;
                ++r;
            }
            normal.push_back({r0, r, 0, -1, 0});
        }
        first[j] = (int32_t)all.size();
        nlong[j] = split ? 0 : (int32_t)longb.size();
        all.insert(all.end(), longb.begin(), longb.end());
        all.insert(all.end(), normal.begin(), normal.end());
    }
    first[chunks] = (int32_t)all.size();
    lr_first[chunks] = (int32_t)lrows.size();
    auto s = std::make_unique<Schedule>();
    s->nnz_cap = nnz_cap;
    s->row_cap = row_cap;
    s->chunks = chunks;
    s->split = split;
    s->rounds = std::max(rounds, 1);
    s->n_long = nlong[0];
    s->n_blocks = (int32_t)all.size();
    s->n_pieces = slot;
    s->first = first;
    s->nlong = nlong;
    s->lo = lo;
    s->lr_first = lr_first;
    for (RowBlock& b : all) {
        if (b.piece != -1) continue;        // long rows and pieces carry their own edge range
        b.e0 = cp[b.r0];
        b.ne = (int32_t)std::min<int64_t>(cp[b.r1] - cp[b.r0], INT32_MAX);
    }
    s->blocks.alloc(sizeof(RowBlock) * std::max<size_t>(all.size(), 1));
    if (!all.empty())
        HIPCHECK(hipMemcpy(s->blocks.p, all.data(), sizeof(RowBlock) * all.size(), hipMemcpyHostToDevice));
    s->longrows.alloc(sizeof(LongRow) * std::max<size_t>(lrows.size(), 1));
    if (!lrows.empty())
        HIPCHECK(hipMemcpy(s->longrows.p, lrows.data(), sizeof(LongRow) * lrows.size(), hipMemcpyHostToDevice));
    return s;
}

Graph* graph_create(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t m, uint32_t flags) {
    auto t0 = std::chrono::steady_clock::now();
    if (!row_ptr || !col) fail(PPR_ERR_ARG, "row_ptr and col must not be NULL");
    if (n < 1) fail(PPR_ERR_ARG, "n must be >= 1");
    if (m < n) fail(PPR_ERR_DANGLING, "m < n: some node has out-degree 0");
    if (flags & ~(PPR_GRAPH_TRUST_INPUT | PPR_GRAPH_WIDE_OFFSETS | PPR_GRAPH_FP64_SLICES(0xffu)))
        fail(PPR_ERR_ARG, "unknown graph flags");
    if (((flags >> 8) & 0xffu) > 64u) fail(PPR_ERR_ARG, "at most 64 source slices");
    if (!(flags & PPR_GRAPH_TRUST_INPUT)) graph_validate(row_ptr, col, n, m);
    else if (row_ptr[0] != 0 || row_ptr[n] != m) fail(PPR_ERR_CSR, "row_ptr[0] must be 0 and row_ptr[n] = m");

    int ndev = 0;
    hipError_t de = hipGetDeviceCount(&ndev);
    if (de != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        fail(PPR_ERR_DEVICE, "no HIP device available");
    }
    auto g = std::make_unique<Graph>();
    HIPCHECK(hipGetDevice(&g->device));
    g->n = n;
    g->m = m;
    g->off64 = m >= (int64_t)UINT32_MAX || (flags & PPR_GRAPH_WIDE_OFFSETS) != 0;
    hipStream_t s;
    HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct StreamGuard { hipStream_t s; ~StreamGuard() { (void)hipStreamDestroy(s); } } sg{s};

    g->row_ptr.alloc(sizeof(int64_t) * ((size_t)n + 1));
    g->col.alloc(sizeof(int32_t) * (size_t)m);
    HIPCHECK(hipMemcpyAsync(g->row_ptr.p, row_ptr, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(g->col.p, col, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, s));
    g->deg.alloc(sizeof(int32_t) * (size_t)n);
    k::deg_from_rowptr(g->row_ptr.as<int64_t>(), g->deg.as<int32_t>(), n, s);

    // in-degree counts -> offsets -> scatter -> per-list sort
    DevBuf cnt(sizeof(int64_t) * ((size_t)n + 1));
    DevBuf cp64(sizeof(int64_t) * ((size_t)n + 1));
    DevBuf tmp(k::scan_tmp_bytes(n));
    HIPCHECK(hipMemsetAsync(cnt.p, 0, sizeof(int64_t) * ((size_t)n + 1), s));
    k::count_in(g->col.as<int32_t>(), m, cnt.as<int64_t>(), s);
    k::exclusive_scan_i64(cnt.as<int64_t>(), cp64.as<int64_t>(), n, tmp.p, s);
    HIPCHECK(hipMemcpyAsync(cnt.p, cp64.p, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    g->row_idx.alloc(sizeof(int32_t) * (size_t)m);
    k::scatter_in(g->row_ptr.as<int64_t>(), g->col.as<int32_t>(), n, cp64.as<int64_t>(), cnt.as<int64_t>(),
                  g->row_idx.as<int32_t>(), s);
    k::sort_segments(cp64.as<int64_t>(), g->row_idx.as<int32_t>(), n, 0, s);
    if (g->off64) {
        g->col_ptr.alloc(sizeof(int64_t) * ((size_t)n + 1));
        HIPCHECK(hipMemcpyAsync(g->col_ptr.p, cp64.p, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s));
    } else {
        g->col_ptr.alloc(sizeof(uint32_t) * ((size_t)n + 1));
        k::narrow_offsets(cp64.as<int64_t>(), g->col_ptr.as<uint32_t>(), (int64_t)n + 1, s);
    }
    // source slices of the FP64 sweep: counts per (slice, row), one scan over
    // them in slice-major order (so slice s's offsets are entries s n .. s n + n),
    // the in-edges copied to their places; then the non-empty (slice, row) pairs
    // of all slices but the last listed with their offsets (the run of a listed
    // pair ends where the next listed one starts, the last one where the last
    // slice starts)
    g->fp64_slices = fp64_slice_count(n, flags);
    if (g->fp64_slices > 1) {
        const int32_t S = g->fp64_slices;
        const int64_t len = (int64_t)S * n;
        const int64_t head = (int64_t)(S - 1) * n;       // pairs of the listed slices
        DevBuf scnt(sizeof(int64_t) * ((size_t)len + 1));
        DevBuf soff(sizeof(int64_t) * ((size_t)len + 1));
        DevBuf stmp(k::scan_tmp_bytes(len));
        k::slice_count(cp64.as<int64_t>(), g->row_idx.as<int32_t>(), n, S, scnt.as<int64_t>(), s);
        k::exclusive_scan_i64(scnt.as<int64_t>(), soff.as<int64_t>(), len, stmp.p, s);
        g->sl_idx.alloc(sizeof(int32_t) * (size_t)m);
        k::slice_scatter(cp64.as<int64_t>(), g->row_idx.as<int32_t>(), n, S, soff.as<int64_t>(),
                         g->sl_idx.as<int32_t>(), s);
        DevBuf flag(sizeof(int64_t) * ((size_t)head + 1));
        DevBuf pos(sizeof(int64_t) * ((size_t)head + 1));
        k::nonzero_flags(scnt.as<int64_t>(), head, flag.as<int64_t>(), s);
        k::exclusive_scan_i64(flag.as<int64_t>(), pos.as<int64_t>(), head, stmp.p, s);
        // slice starts among the listed pairs: pos[s n], and the total K = pos[head]
        std::vector<int64_t> first((size_t)S);
        for (int32_t sl = 0; sl < S; ++sl)
            HIPCHECK(hipMemcpyAsync(&first[(size_t)sl], pos.as<int64_t>() + (int64_t)sl * n, sizeof(int64_t),
                                    hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        const int64_t K = first[(size_t)S - 1];
        DevBuf cp_list(sizeof(int64_t) * ((size_t)K + 1));
        g->sl_rows.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(K, 1));
        k::slice_compact(scnt.as<int64_t>(), pos.as<int64_t>(), soff.as<int64_t>(), head, n,
                         g->sl_rows.as<int32_t>(), cp_list.as<int64_t>(), s);
        HIPCHECK(hipMemcpyAsync(cp_list.as<int64_t>() + K, soff.as<int64_t>() + head, sizeof(int64_t),
                                hipMemcpyDeviceToDevice, s));
        const size_t ob = g->off64 ? 8 : 4;
        g->sl_cptr.alloc(ob * ((size_t)K + 1));
        g->sl_last.alloc(ob * ((size_t)n + 1));
        if (g->off64) {
            HIPCHECK(hipMemcpyAsync(g->sl_cptr.p, cp_list.p, 8 * ((size_t)K + 1), hipMemcpyDeviceToDevice, s));
            HIPCHECK(hipMemcpyAsync(g->sl_last.p, soff.as<int64_t>() + head, 8 * ((size_t)n + 1),
                                    hipMemcpyDeviceToDevice, s));
        } else {
            k::narrow_offsets(cp_list.as<int64_t>(), g->sl_cptr.as<uint32_t>(), K + 1, s);
            k::narrow_offsets(soff.as<int64_t>() + head, g->sl_last.as<uint32_t>(), (int64_t)n + 1, s);
        }
        g->sl_first = first;
        g->sl_first.push_back(K);
        // one FP64 sweep schedule per slice: over the listed rows of the first
        // S - 1 slices (their offsets are consecutive entries of the list), over
        // all rows for the last
        std::vector<int64_t> hoff;
        for (int32_t sl = 0; sl < S; ++sl) {
            const bool last = sl + 1 == S;
            const int64_t rows = last ? n : g->sl_first[(size_t)sl + 1] - g->sl_first[(size_t)sl];
            hoff.resize((size_t)rows + 1);
            const int64_t* src = last ? soff.as<int64_t>() + head : cp_list.as<int64_t>() + g->sl_first[(size_t)sl];
            HIPCHECK(hipMemcpyAsync(hoff.data(), src, sizeof(int64_t) * ((size_t)rows + 1), hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            if (last && hoff[(size_t)n] != m) fail(PPR_ERR_DEVICE, "source slices hold a wrong edge count");
            g->sl_sched.push_back(make_schedule(hoff.data(), (int32_t)rows, k::sweep_nnz_cap(), k::sweep_row_cap(), 1, 0));
        }
    }
    g->h_col_ptr.resize((size_t)n + 1);
    HIPCHECK(hipMemcpyAsync(g->h_col_ptr.data(), cp64.p, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, s));
    g->h_deg.resize((size_t)n);
    for (int32_t v = 0; v < n; ++v) g->h_deg[v] = (int32_t)(row_ptr[v + 1] - row_ptr[v]);
    HIPCHECK(hipStreamSynchronize(s));
    if (g->h_col_ptr[n] != m) fail(PPR_ERR_DEVICE, "CSC build produced a wrong edge count");
    int32_t mi = 0, mo = 0;
    for (int32_t v = 0; v < n; ++v) {
        mi = std::max<int32_t>(mi, (int32_t)(g->h_col_ptr[v + 1] - g->h_col_ptr[v]));
        mo = std::max<int32_t>(mo, g->h_deg[v]);
    }
    g->max_in = mi;
    g->max_out = mo;
    (void)g->schedule(k::sweep_nnz_cap(), k::sweep_row_cap());   // the FP64 sweep's, used by every query path
    g->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return g.release();
}

void graph_copy_csc(const Graph& g, int64_t* col_ptr, int32_t* row_idx, int32_t* deg) {
    HIPCHECK(hipSetDevice(g.device));
    if (col_ptr) {   // the device offsets themselves, widened when stored as uint32
        if (g.off64) {
            HIPCHECK(hipMemcpy(col_ptr, g.col_ptr.p, sizeof(int64_t) * ((size_t)g.n + 1), hipMemcpyDeviceToHost));
        } else {
            std::vector<uint32_t> narrow((size_t)g.n + 1);
            HIPCHECK(hipMemcpy(narrow.data(), g.col_ptr.p, sizeof(uint32_t) * ((size_t)g.n + 1),
                               hipMemcpyDeviceToHost));
            for (size_t i = 0; i < narrow.size(); ++i) col_ptr[i] = (int64_t)narrow[i];
        }
    }
    if (row_idx) HIPCHECK(hipMemcpy(row_idx, g.row_idx.p, sizeof(int32_t) * (size_t)g.m, hipMemcpyDeviceToHost));
    if (deg) HIPCHECK(hipMemcpy(deg, g.deg.p, sizeof(int32_t) * (size_t)g.n, hipMemcpyDeviceToHost));
}

}  // namespace ppr
