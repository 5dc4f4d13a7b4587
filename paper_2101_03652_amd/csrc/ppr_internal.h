// Internal declarations of libppr (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ppr.h"

namespace ppr {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
const char* last_error_cstr();
struct Failure {
    ppr_status status;
    std::string msg;
};
[[noreturn]] void fail(ppr_status st, const std::string& msg);
void check_hip(hipError_t e, const char* what, const char* file, int line);
#define HIPCHECK(x) ::ppr::check_hip((x), #x, __FILE__, __LINE__)

// Runs f and turns every failure (Failure, std::bad_alloc, other exceptions)
// into a status code and the thread-local message: nothing throws across the
// C ABI.
template <class F>
ppr_status guarded_call(F&& f) {
    try {
        f();
        set_error("");
        return PPR_OK;
    } catch (const Failure& e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return PPR_ERR_OOM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return PPR_ERR_DEVICE;
    } catch (...) {
        set_error("unknown failure");
        return PPR_ERR_DEVICE;
    }
}

// True if p is device (or managed) memory of `device`; false for host memory
// (pageable, pinned or unregistered).  Device memory of another device is an
// argument error.
bool is_device_ptr(const void* p, int device);

// A pair of HIP events bracketing work on one stream; elapsed() after a sync.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair();
    ~EventPair();
    EventPair(const EventPair&) = delete;
    EventPair& operator=(const EventPair&) = delete;
    void start(hipStream_t s);
    void stop(hipStream_t s);
    double elapsed_ms() const;   // requires the stop event to have completed
};

// ---------------------------------------------------------------- device buffers
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool owned = true;         // false: a view into another buffer (not freed here)
    DevBuf() = default;
    explicit DevBuf(size_t b) { alloc(b); }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    void alloc(size_t b);
    void view(void* base, size_t b);   // b bytes at base, owned by another buffer
    void release();
    template <class T> T* as() const { return static_cast<T*>(p); }
};

struct PinnedBuf {
    void* p = nullptr;
    size_t bytes = 0;
    PinnedBuf() = default;
    ~PinnedBuf() { release(); }
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;
    void alloc(size_t b);
    void release();
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// A contiguous range of destination rows processed by one workgroup of a
// pull sweep.  Long rows (more in-edges than the block's edge budget) get a
// block of their own, listed first, or are cut into pieces (split schedules).
struct RowBlock {
    int32_t r0, r1;      // rows [r0, r1)
    int32_t ne;          // in-edges of the block
    int32_t piece;       // -1: whole rows [r0, r1) with at most one round of in-edges;
                         // -2: the whole long row r0, in several rounds;
                         // >= 0: one piece of the long row r0, whose sum goes to
                         // partial slot `piece`
    int64_t e0;          // offset of the first in-edge (= col_ptr[r0] unless a piece)
};

// A long row of a split schedule: its pieces' partial sums are slots
// [first, first + npieces), added in slot order.
struct LongRow {
    int32_t row, first, npieces, pad;
};

// Sweep schedule for one edge budget.
struct Schedule {
    int32_t nnz_cap = 0;       // edge budget per block
    int32_t row_cap = 0;       // row budget per block
    int32_t chunks = 1;        // row chunks (contiguous row ranges of about m / chunks in-edges)
    bool split = false;        // long rows in rounds / pieces (else one block per long row)
    int32_t rounds = 1;        // split: edge rounds (of nnz_cap) one block may run
    int32_t n_long = 0;        // leading blocks that hold a single long row (chunks == 1, !split)
    int32_t n_blocks = 0;
    int32_t n_pieces = 0;      // partial slots of a split schedule
    // chunk j: blocks [first[j], first[j+1]), of which the first nlong[j] hold
    // one long row each (!split); rows [lo[j], lo[j+1]); long rows
    // [lr_first[j], lr_first[j+1]) of `longrows` (split)
    std::vector<int32_t> first, nlong, lo, lr_first;
    DevBuf blocks;             // RowBlock[n_blocks]
    DevBuf longrows;           // LongRow[...] (split)
};

struct QueryCtx;
struct MixedCtx;
struct MixedCtxDeleter {
    void operator()(MixedCtx* c) const;
};
using MixedCtxPtr = std::unique_ptr<MixedCtx, MixedCtxDeleter>;

// Device graph: CSR (out-edges, for the frontier push), CSC (in-edges, for
// the pull sweeps), out-degrees, schedules.
struct Graph {
    int device = 0;
    int32_t n = 0;
    int64_t m = 0;
    bool off64 = false;        // CSC offsets int64 (else uint32)
    int32_t max_in = 0, max_out = 0;
    double build_ms = 0;
    DevBuf row_ptr;            // int64[n+1]
    DevBuf col;                // int32[m]
    DevBuf col_ptr;            // uint32 or int64 [n+1]
    DevBuf row_idx;            // int32[m]
    DevBuf deg;                // int32[n] out-degree
    // Source slices of the FP64 sweep: the in-edges regrouped by the slice of
    // their source, slice s = sources [ceil(s n / S), ceil((s + 1) n / S)), so
    // that one pass gathers from an S-th of the residue vector only (it stays
    // in the caches).  sl_idx: int32[m], slice-major: slice s's in-edges of
    // row u form one run, rows ascending, runs of slice s before those of s + 1.
    // Slices s < S - 1 list only their rows with in-edges: the K such (slice,
    // row) pairs in that order are sl_rows (int32[K], the row) and sl_cptr
    // (OffT[K + 1], the run's start in sl_idx; entry K is the start of the last
    // slice), slice s being positions [sl_first[s], sl_first[s + 1]).  The last
    // slice, whose pass finishes every row, keeps full CSC offsets sl_last
    // (OffT[n + 1]).  S = 1: none.
    int32_t fp64_slices = 1;
    DevBuf sl_idx, sl_rows, sl_cptr, sl_last;
    std::vector<int64_t> sl_first;                     // S entries: slice starts in sl_rows, then K
    std::vector<std::unique_ptr<Schedule>> sl_sched;   // the FP64 sweep's schedule of each slice
    std::vector<int64_t> h_col_ptr;   // host copy of the CSC offsets (schedules)
    std::vector<int32_t> h_deg;       // host copy of the out-degrees
    std::mutex sched_mu;
    std::vector<std::unique_ptr<Schedule>> schedules;
    // Query state pools.  They belong to the graph: their captured HIP graphs
    // hold this graph's device pointers, so they must die with it.
    std::mutex pool_mu;
    std::vector<std::unique_ptr<QueryCtx>> pool;       // idle FP64 query contexts
    std::vector<MixedCtxPtr> mixed_pool;               // idle batched contexts (any width)
    // autotuner's choices (ppr_autotune; atomics: a query may read them while it
    // runs): the block width (0 = not tuned) and the sweep stage bytes per
    // residue format (0 FP32, 1 bf16) and log2(width) (0 = default)
    std::atomic<int> tuned_width{0};
    std::atomic<int> tuned_tile[2][8] = {};
    std::atomic<int> tuned_fmt[8] = {};                // residue format + 1 per log2(width) (0 = not tuned)
    DevBuf walk_index;                                 // int32[m]: stop nodes of d_v walks per node
    double walk_alpha = -1.0;                          // the index's alpha (-1: none)
    uint64_t walk_seed = 0;                            // the index's seed
    int live_blocks = 0;                               // serving blocks on this graph (pool_mu)
    ~Graph();
    size_t device_bytes() const;
    const Schedule& schedule(int32_t nnz_cap, int32_t row_cap, int32_t chunks = 1, int32_t rounds = 0);
    // The schedule if it has been built, else nullptr (allocates nothing).
    const Schedule* find_schedule(int32_t nnz_cap, int32_t row_cap, int32_t chunks = 1, int32_t rounds = 0);
};

Graph* graph_create(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t m,
                    uint32_t flags);
// The schedule of row blocks over CSC offsets cp[0..n] (Graph::schedule's rules).
std::unique_ptr<Schedule> make_schedule(const int64_t* cp, int32_t n, int32_t nnz_cap, int32_t row_cap,
                                        int32_t chunks, int32_t rounds);
// Source slices of the FP64 sweep for n nodes: the count the library picks
// (flags without PPR_GRAPH_FP64_SLICES), or the forced count of the flags.
int32_t fp64_slice_count(int32_t n, uint32_t flags);
void graph_validate(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t m);
void graph_copy_csc(const Graph& g, int64_t* col_ptr, int32_t* row_idx, int32_t* deg);

// ---------------------------------------------------------------- FP64 query context
constexpr int64_t kAuxLen = 4 * 1024 + 16;

struct QueryCtx {
    hipStream_t stream = nullptr;   // work stream: `own`, or the caller's stream during a query on it
    hipStream_t own = nullptr;      // the context's own stream (HIP graphs are captured here)
    int32_t n = 0;
    DevBuf r;          // double[n]  residue
    DevBuf pi;         // double[n]  reserve
    DevBuf y0, y1;     // double[n]  scaled residue (1-alpha) r / d, ping-pong
    DevBuf F0, F1;     // int32[n]   frontier lists
    DevBuf X;          // double[n]  per-frontier-entry push increment
    DevBuf degF;       // int64[n]   out-degrees of the frontier entries
    DevBuf off;        // int64[n+1] degree prefix of the frontier
    DevBuf partials;   // double[max blocks]
    DevBuf acc;        // double[n]  row sums across the source slices of a sweep (graphs with slices)
    DevBuf scan_tmp;   // scan scratch
    DevBuf ctr;        // int64[8] counters: [0] |F'|, [1] vol(F'), [2..] spare
    DevBuf dsum;       // double[8]: [0] reduced sum
    DevBuf aux;        // int64[kAuxLen]: per-block counts and their scans (frontier compaction)
    PinnedBuf host;    // 64 bytes readback
    hipGraphExec_t chunk_exec = nullptr;   // captured FOLD sweep pairs
    int chunk_pairs = 0;
    double chunk_alpha = -1;
    ~QueryCtx();
};

std::unique_ptr<QueryCtx> ctx_acquire(Graph& g);
void ctx_release(Graph& g, std::unique_ptr<QueryCtx> c);

// ---------------------------------------------------------------- kernels (launchers)
namespace k {
void deg_from_rowptr(const int64_t* row_ptr, int32_t* deg, int32_t n, hipStream_t s);
void count_in(const int32_t* col, int64_t m, int64_t* cnt, hipStream_t s);
// exclusive scan of int64 counts (len entries) into out[len+1]
size_t scan_tmp_bytes(int64_t len);
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t len, void* tmp, hipStream_t s);
void scatter_in(const int64_t* row_ptr, const int32_t* col, int32_t n, const int64_t* col_ptr,
                int64_t* fill, int32_t* row_idx, hipStream_t s);
void sort_segments(const int64_t* col_ptr, int32_t* row_idx, int32_t n, int32_t max_len,
                   hipStream_t s);
void narrow_offsets(const int64_t* in, uint32_t* out, int64_t len, hipStream_t s);
// source slices: per (slice, row) in-edge counts cnt[s n + u], then the edges
// copied to their slice-major places (off: the exclusive scan of cnt); the
// non-empty pairs of the first len pairs listed (flags: 1 per non-empty pair,
// pos: their exclusive scan): rows[pos[i]] = i mod n, cptr[pos[i]] = off[i]
void slice_count(const int64_t* col_ptr, const int32_t* row_idx, int32_t n, int32_t S, int64_t* cnt,
                 hipStream_t s);
void slice_scatter(const int64_t* col_ptr, const int32_t* row_idx, int32_t n, int32_t S, const int64_t* off,
                   int32_t* sl_idx, hipStream_t s);
void nonzero_flags(const int64_t* cnt, int64_t len, int64_t* flags, hipStream_t s);
void slice_compact(const int64_t* cnt, const int64_t* pos, const int64_t* off, int64_t len, int32_t n,
                   int32_t* rows, int64_t* cptr, hipStream_t s);

// local phase (FP64, one query)
void query_init(double* r, double* pi, int32_t n, int32_t s_node, int32_t* F, hipStream_t st);
void frontier_snapshot(const int32_t* F, int32_t nf, const int32_t* deg, double alpha, double* r,
                       double* pi, double* X, int64_t* degs_of_F, double* partials, int* nparts,
                       hipStream_t s);
void frontier_push(const int32_t* F, const int64_t* off, int32_t nf, int64_t vol,
                   const int64_t* row_ptr, const int32_t* col, const int32_t* deg, const double* X,
                   double rmax, double* r, int32_t* F_next, int64_t* ctr, hipStream_t s);
// y = (1-alpha) r / d for all nodes, with per-block partial sums of r
void prep_y(const double* r, const int32_t* deg, double alpha, int32_t n, double* y,
            double* partials, int* nparts, hipStream_t s);
void reduce_sum(const double* partials, int nparts, double* out, hipStream_t s);

// Epoch scans: every node with r(v) > d_v rmax pushes now (pi += alpha r,
// r = 0, y = (1-alpha) r / d_v), the others get y = 0; per-block partial sums
// of the pushed nodes' out-degrees (the scan's edge pushes)
void threshold_snapshot(const int32_t* deg, int32_t n, double alpha, double rmax, double* r, double* pi,
                        double* y, double* partials, int* nparts, hipStream_t s);

// FP64 pull sweep: flags (SW_ACCUM: r_out = r_in + the pulled sum, no y_out).
// With acc (double[n] scratch) and a graph with source slices, the sweep runs
// one pass per slice (the row sums collected in acc) and the last pass
// finishes the rows; acc = nullptr: one pass over the whole CSC.  The sweep's
// partial sums are then sweep_parts(g, sch, acc) values.
enum : int { SW_ENTRY = 1, SW_FOLD = 2, SW_WRITE_R = 4, SW_ACCUM = 8 };
void sweep_f64(const Graph& g, const Schedule& sch, int flags, double alpha, const double* y_in,
               double* y_out, double* pi, const double* r_in, double* r_out, double* partials,
               hipStream_t s, double* acc = nullptr);
int sweep_parts(const Schedule& sch);
int sweep_parts(const Graph& g, const Schedule& sch, const double* acc);
int32_t sweep_nnz_cap();
int32_t sweep_row_cap();
// certificate pass: q(v) = pi(v) / d_v, then rt(u) = e_s(u) - (pi(u) - (1-alpha) sum q) / alpha;
// partials receive sum |rt| per block; rt_out (nullable) receives rt
void cert_f64(const Graph& g, const Schedule& sch, double alpha, int32_t src, const double* pi,
              double* q, double* rt_out, double* partials, hipStream_t s);
}  // namespace k

// ---------------------------------------------------------------- runtime
// Convergence trace of one FP64 query: a point per local iteration and per
// global sweep or scan, written while there is room, counted always.
struct TraceSink {
    ppr_trace_point* out = nullptr;
    int32_t cap = 0;
    int32_t count = 0;
    std::chrono::steady_clock::time_point t0;
    void note(int32_t phase, int32_t index, int64_t edge_pushes, double r_sum) {
        if (count < cap) {
            ppr_trace_point& p = out[count];
            p.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            p.r_sum = r_sum;
            p.edge_pushes = edge_pushes;
            p.phase = phase;
            p.index = index;
        }
        ++count;
    }
};

void run_fp64_query(Graph& g, int32_t s, double alpha, double lambda, const ppr_options& opt,
                    double* pi_out, double* r_out, ppr_stats* st, TraceSink* trace = nullptr);
// The same query with the default options, its state in a static device
// array (no allocation); pi: device memory.
void run_fp64_query_noalloc(Graph& g, int32_t s, double alpha, double lambda, hipStream_t stream, double* pi,
                            ppr_stats* st);

// Approximate SSPPR (SpeedPPR).  A walk alive after kMaxWalkSteps steps stops
// where it is (probability (1 - alpha)^4096).
constexpr int32_t kMaxWalkSteps = 4096;
double walk_budget(int32_t n, double eps, double mu);
// The active nodes of c.r w.r.t. rmax (r(v) > d_v rmax), in node order, into
// out (nullable: count only), with their number and edge volume.
void active_set(const Graph& g, QueryCtx& c, double rmax, int32_t* out, int64_t* count, int64_t* vol);
void run_approx_query(Graph& g, int32_t s, double alpha, double eps, double mu, uint64_t seed, bool use_index,
                      const ppr_options& opt, double* pi_out, ppr_approx_stats* st);
void build_walk_index(Graph& g, double alpha, uint64_t seed, double* ms);
void copy_walk_index(const Graph& g, int32_t* out);
void debug_refine(Graph& g, double alpha, double rmax, double* pi, double* r, int32_t* levels, int64_t* edges);
void debug_walks(Graph& g, double alpha, double W, uint64_t seed, bool use_index, const double* r, double* pi,
                 int64_t* nwalks);
void run_mixed_batch(Graph& g, const int32_t* sources, int32_t B, double alpha, double lambda,
                     const ppr_options& opt, double* pi_out, double* r_out, ppr_stats* st);
void autotune_width(Graph& g, double alpha, double lambda, const int32_t* widths, int32_t count, int32_t* best,
                    double* cost_us);

void debug_sweeps_mixed(Graph& g, double alpha, int32_t B, int32_t chunks, int32_t sweeps, const float* y_in,
                        const int32_t* entry, const int32_t* budget, const float* t_in, float* y_out,
                        float* t_out, const float* omega, int32_t residue_format, int32_t sweep_tile,
                        bool wide_gather);

// serving blocks (continuous batching); the handle is an opaque Block*
void* serve_block_create(Graph& g, int32_t slots, double alpha, const ppr_options& opt);
void serve_block_destroy(void* blk);
int32_t serve_admit(void* blk, int32_t s, double alpha, double lambda);
void serve_step(void* blk, int32_t max_sweeps);
void serve_poll(void* blk, int wait, uint8_t* done, int32_t* n_done, int32_t* n_busy, int32_t* ready);
void serve_retire(void* blk, int32_t slot, double* pi_out, ppr_stats* st);
// device bytes of a serving block of `slots` columns on a graph of n nodes and
// m edges (default options), and of one FP64 query context on n nodes; both
// depend on the sizes only
size_t serve_footprint(int32_t n, int64_t m, int32_t slots);
size_t fp64_ctx_footprint(int32_t n);
// device bytes of a graph's CSR, CSC and degree table (its row schedules not counted)
size_t graph_footprint(int32_t n, int64_t m);

}  // namespace ppr
