/*
 * ppr.h -- C ABI of the MI355X high-precision single-source PPR library
 * (libppr.so).
 *
 * The library answers High-Precision SSPPR queries (Section 2 of Wu, Gan, Wei,
 * Zhang, "Unifying the Global and Local Approaches: An Efficient Power
 * Iteration with Forward Push", SIGMOD 2021): given a directed graph G, a
 * source s, the stop probability alpha of the alpha-random walk and an l1
 * error threshold lambda in (0, 1], it returns pi_hat with
 *     || pi_hat - pi_s ||_1 <= lambda,
 * where pi_s solves the linear system of Eq. 1,
 *     pi_s = alpha e_s + (1 - alpha) pi_s P,   P = D^-1 A (Section 2).
 *
 * Method (PowerPush, Algorithm 3, run level-synchronously on the GPU): a
 * forward-push local phase over frontiers (the iteration sets S^(j) of
 * Section 4.2, pushed simultaneously), then global push sweeps over every
 * edge with rmax = 0 (Simultaneous Forward Push, Eq. 7, identical to power
 * iteration by Lemma 1), until the residue sum r_sum <= lambda.
 *
 * Conventions
 *  - Every function returns a ppr_status; no C++ exception crosses the ABI.
 *    On failure ppr_last_error() returns a thread-local message.
 *  - Inputs are borrowed: the library copies what it keeps; the caller keeps
 *    ownership of every buffer it passes.
 *  - Output buffers are caller-owned and may be host or device memory (the
 *    library detects which with hipPointerGetAttributes).  A device output
 *    must be on the device the graph was created on.
 *  - A ppr_graph's structure is immutable after creation; queries on one
 *    graph from different threads are safe (each call takes its own state
 *    slot and HIP stream from the graph's pool).  ppr_autotune changes the
 *    graph's defaults (block width, row tiles) and must not run while other
 *    calls use the graph.  A ppr_block is used from one thread.
 *  - Streams: by default every call runs on a stream of its own state slot.
 *    With ppr_options.use_stream = 1 a query (ppr_query_ex, ppr_query_trace)
 *    or a serving block runs every launch and copy on the caller's HIP stream
 *    ppr_options.stream instead (NULL: the null stream), after the work the
 *    caller enqueued there earlier; a PyTorch stream's handle passes straight
 *    through.  HIP graphs the library replays are captured on its own streams
 *    and launched on the caller's.
 *  - Node ids are 0..n-1 (int32).  Edge counts and offsets are int64.
 *  - All calls are synchronous unless stated: they return once results are
 *    in the caller's buffer.
 */
#ifndef PPR_H
#define PPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ppr_graph ppr_graph;   /* opaque, library-owned, device resident */
typedef struct ppr_block ppr_block;   /* opaque serving block: query slots on one graph */

typedef enum {
    PPR_OK = 0,
    PPR_ERR_ARG = -1,            /* bad argument (null pointer, out of range, NaN) */
    PPR_ERR_CSR = -2,            /* CSR malformed: offsets not monotone, row_ptr[0] != 0,
                                    row_ptr[n] != m, or a column index outside [0, n) */
    PPR_ERR_DANGLING = -3,       /* a node has out-degree 0 (Section 2 assumes d_v >= 1) */
    PPR_ERR_DUPLICATE = -4,      /* an edge appears twice (A is a 0/1 matrix, Section 2) */
    PPR_ERR_OOM = -5,            /* device or host allocation failed, or over budget */
    PPR_ERR_DEVICE = -6,         /* a HIP runtime call failed, or no GPU is present */
    PPR_ERR_NOT_CONVERGED = -7,  /* max_sweeps reached before r_sum <= lambda */
    PPR_ERR_BUSY = -8            /* no free slot in a serving block */
} ppr_status;

typedef enum {
    PPR_FP64 = 0,    /* plain path: residues, reserves and sums in double precision */
    PPR_MIXED = 1    /* FP32 arithmetic on FP32 or bf16 residues (block Gauss-Seidel,
                        over-relaxed push sweeps) with an FP32 stage accumulator;
                        FP64 reserves; every stage ends with an FP64 residual
                        refresh that certifies the result */
} ppr_precision;

/* Storage of the batched path's residue block (arithmetic is FP32 either way). */
typedef enum {
    PPR_RESIDUE_F32 = 0,   /* 4 bytes per residue */
    PPR_RESIDUE_BF16 = 1,  /* 2 bytes: half the bytes each sweep gathers; the rounding a
                              stored residue takes is residual that the next FP64 refresh
                              measures, so stages are shorter (refresh factor 40).  Blocks
                              of at least 8 columns (a sweep lane holds 8) */
    PPR_RESIDUE_AUTO = 2   /* the storage ppr_autotune chose for the block's width; on a
                              graph not tuned at that width, bf16 for blocks of at least
                              32 columns, else FP32 (default) */
} ppr_residue_format;

/* Rule that ends the local (frontier) phase and starts the global sweeps. */
typedef enum {
    PPR_SWITCH_NODES = 0,  /* continue while 4 |S^(j)| <= n: Algorithm 3's
                              scanThreshold = n/4 */
    PPR_SWITCH_EDGES = 1   /* continue while switch_param * sum_{v in S^(j)} d_v <= m:
                              edge volume, the GPU cost model (default) */
} ppr_switch_rule;

/* Per-query statistics. */
typedef struct {
    int32_t local_levels;   /* frontier iterations S^(j) run by the local phase */
    int32_t sweeps;         /* global sweeps (each reads every edge once) */
    int32_t refreshes;      /* FP64 residual refresh passes (mixed path) */
    int32_t source;         /* the query's source node */
    int64_t edge_pushes;    /* residue updates: sum of d_v over local pushes + sweeps * m */
    double r_sum;           /* residue sum when the query stopped (FP64) */
    double cert_l1;         /* ||e_s - pi_hat (I - (1-alpha) P) / alpha||_1 computed in FP64
                               (always for PPR_MIXED; for PPR_FP64 only when certify = 1,
                               else -1).  An upper bound on ||pi_hat - pi_s||_1. */
    double ms;              /* wall time of the call (whole batch for batched calls) */
    double sweep_ms;        /* GPU time of the global sweep kernels of this query's block, measured
                               with HIP events on the library's stream (whole block for batched
                               calls; refresh passes excluded) */
    int32_t sweep_launches; /* sweep kernel launches that sweep_ms covers */
    int32_t batch_cols;     /* block width used (1 for PPR_FP64) */
    int32_t sweep_chunks;   /* row chunks per global sweep (1 = Eq. 7 order) */
    double sor_omega;       /* over-relaxation factor of the query's last stage (1 = none) */
    int32_t residue_format; /* storage of the residues the query swept: PPR_RESIDUE_F32 or
                               PPR_RESIDUE_BF16 (PPR_FP64: F32, though it sweeps in double) */
    int32_t push_scans;     /* PPR_GLOBAL_EPOCHS: scans taken in push form (the rest of
                               `sweeps` in pull form); 0 otherwise */
    int32_t sweep_tile_bytes; /* LDS stage of a batched sweep block (its row tile: in-edges
                               and rows per block), chosen per width by ppr_autotune;
                               0 for PPR_FP64 */
    double refresh_ms;      /* PPR_MIXED: GPU time of the FP64 refresh passes of the query's block
                               (HIP events on the library's stream, whole block); 0 for PPR_FP64 */
    int32_t refresh_launches; /* refresh passes that refresh_ms covers */
    int32_t reserved;
} ppr_stats;

/* Global phase of the PPR_FP64 path. */
typedef enum {
    PPR_GLOBAL_SWEEPS = 0,  /* threshold-0 sweeps: every sweep is one Eq. 7 step (default) */
    PPR_GLOBAL_EPOCHS = 1   /* Algorithm 3's epochs: rmax_i = lambda^(i/8) / m, i = 1..8,
                               scans while r_sum > m rmax_i; each scan pushes, at once,
                               the nodes active at its start (r(v) > d_v rmax_i) */
} ppr_global_rule;

/* Form of a thresholded scan of PPR_GLOBAL_EPOCHS (both push, at once, every
 * node active at the scan's start: the same scan, the same result up to FP64
 * rounding order). */
typedef enum {
    PPR_SCAN_AUTO = 0,  /* push form when switch_param * vol <= m for the active set's
                           out-edge volume vol, pull form otherwise (direction-optimizing;
                           default) */
    PPR_SCAN_PULL = 1,  /* pull form: a threshold pass over all nodes, then every in-edge
                           list reads the pushing nodes' shares (no atomics; reads all m
                           edges) */
    PPR_SCAN_PUSH = 2   /* push form: the active nodes, listed, add their shares along
                           their out-edges with FP64 atomics (reads vol edges); the next
                           scan's active nodes are the ones such an add carried across
                           their threshold */
} ppr_scan_form;

/* Query options (ppr_options_default fills the defaults). */
typedef struct {
    int32_t precision;      /* ppr_precision */
    int32_t switch_rule;    /* ppr_switch_rule; default PPR_SWITCH_EDGES */
    double switch_param;    /* PPR_SWITCH_EDGES: continue while param * vol <= m; default 32 */
    int32_t max_sweeps;     /* cap on the global sweeps of each query; default 4096 */
    int32_t certify;        /* PPR_FP64: also compute cert_l1; default 0 */
    double refresh_factor;  /* PPR_MIXED: refresh the residual in FP64 whenever r_sum has
                               fallen by this factor since the last refresh; 0 = chosen by
                               the residue format (1e3 for FP32, 40 for bf16; default) */
    int32_t batch_cols;     /* PPR_MIXED batched: columns per block (multiple of 4, or 0 =
                               autotuned); default 0 */
    int32_t sweep_chunks;   /* PPR_MIXED: row chunks per global sweep.  1 = every sweep is
                               one Eq. 7 step (Jacobi order); G > 1 = block Gauss-Seidel
                               order: the rows of chunk j see the residues that chunks
                               0..j-1 produced in the same sweep, as the in-place scan of
                               Algorithm 3 does; 0 = chosen from m (default) */
    int32_t global_rule;    /* PPR_FP64: ppr_global_rule; default PPR_GLOBAL_SWEEPS */
    double sor_omega;       /* PPR_MIXED, block Gauss-Seidel order (more than one chunk):
                               over-relaxation factor of the sweeps (each node pushes omega
                               times the residue it holds and keeps 1 - omega of it);
                               0 = automatic: 1.2 when a sweep has more than one chunk
                               (default); 1 = off; or a factor in (1, 1.9].  A column whose
                               measured contraction shows no gain falls back to 1; the FP64
                               certificate bounds the result either way */
    int32_t residue_format; /* PPR_MIXED: ppr_residue_format; default PPR_RESIDUE_AUTO */
    int32_t scan_form;      /* PPR_FP64 with PPR_GLOBAL_EPOCHS: ppr_scan_form; default
                               PPR_SCAN_AUTO */
    int32_t sweep_tile;     /* PPR_MIXED: LDS stage (row tile) of a sweep block in bytes,
                               12288, 16384 or 24576; 0 = the tile ppr_autotune chose for
                               the block width on this graph, else 16384 (default).  Any
                               other value: PPR_ERR_ARG */
    int32_t use_stream;     /* 1: run on `stream` (below); 0: on the library's own streams
                               (default) */
    void* stream;           /* hipStream_t of the caller when use_stream = 1 (NULL: the null
                               stream).  Synchronous calls still return only once their
                               results are in the caller's buffers; a serving block's steps
                               are enqueued there and collected by ppr_block_poll */
} ppr_options;

/* Read-only facts about a created graph. */
typedef struct {
    int32_t n;
    int32_t max_in_degree;
    int64_t m;
    int32_t max_out_degree;
    int32_t offsets_64bit;  /* 1 if the device CSC offsets are int64 (m >= 2^32) */
    double build_ms;        /* wall time of ppr_graph_create */
    size_t device_bytes;    /* device memory held by the graph */
    int32_t fp64_slices;    /* source slices of the FP64 sweep (1: none) */
    int32_t reserved;
} ppr_graph_info;

/* Default options. */
void ppr_options_default(ppr_options* opt);

/*
 * Create a device-resident graph from CSR out-edges (the storage the paper's
 * global scan assumes: nodes sorted by id, adjacency lists concatenated,
 * Section 5).
 *   row_ptr: host int64[n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = m.
 *   col:     host int32[m], col[row_ptr[v] .. row_ptr[v+1]) = out-neighbours of v.
 *   n >= 1, m >= n (every node needs an out-edge).
 *   flags:   PPR_GRAPH_TRUST_INPUT skips the O(n + m) host validation;
 *            PPR_GRAPH_WIDE_OFFSETS stores the device CSC offsets as int64 even
 *            when m < 2^32 (they are int64 whenever m >= 2^32);
 *            PPR_GRAPH_FP64_SLICES(S), S in [1, 64], sets the number of source
 *            slices of the FP64 sweep (see below; 0 or absent: the library's
 *            choice, one slice per 12 MiB of FP64 residue vector, at most 16).
 * Validation (unless skipped): PPR_ERR_CSR, PPR_ERR_DANGLING, PPR_ERR_DUPLICATE.
 * Self-loops are allowed.  The library builds on the current HIP device the
 * in-edge lists (CSC, each list ascending by source id), the out-degree
 * table and the sweep schedule.  With S > 1 source slices it also keeps a
 * copy of the in-edges grouped by the slice of their source (slice s holds
 * the sources [ceil(s n / S), ceil((s + 1) n / S))): an FP64 sweep (Eq. 7)
 * then makes one pass per slice, each gathering from an S-th of the residue
 * vector, which stays in the GPU's caches, and the last pass finishes the
 * rows.  The sum over a row's in-edges is then taken slice by slice (the
 * rounding of FP64 sums changes, nothing else); ppr_graph_info.fp64_slices
 * reports S and device_bytes includes the copy.  *out receives the handle.
 */
#define PPR_GRAPH_TRUST_INPUT 1u
#define PPR_GRAPH_WIDE_OFFSETS 2u
#define PPR_GRAPH_FP64_SLICES(S) ((uint32_t)(S) << 8)
ppr_status ppr_graph_create(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t m,
                            uint32_t flags, ppr_graph** out);

/* Release the graph and everything it owns.  NULL is accepted. */
ppr_status ppr_graph_destroy(ppr_graph* g);

/* Facts about the graph. */
ppr_status ppr_graph_get_info(const ppr_graph* g, ppr_graph_info* info);

/*
 * Copy the device CSC to host buffers (for verification): col_ptr int64[n+1],
 * row_idx int32[m] (in-list of u is row_idx[col_ptr[u] .. col_ptr[u+1]),
 * ascending), deg_out int32[n].  Any pointer may be NULL to skip it.
 */
ppr_status ppr_graph_copy_csc(const ppr_graph* g, int64_t* col_ptr, int32_t* row_idx,
                              int32_t* deg_out);

/*
 * One HP-SSPPR query.  alpha in (0, 1), lambda in (0, 1], 0 <= s < n.
 * pi_out: double[n] (host or device), receives pi_hat.  stats nullable.
 * Uses the default options with the given precision.
 */
ppr_status ppr_query(ppr_graph* g, int32_t s, double alpha, double lambda,
                     ppr_precision precision, double* pi_out, ppr_stats* stats);

/*
 * B queries on the same graph.  sources int32[B] (host), pi_out double[B*n]
 * row-major (row b is the answer for sources[b]), stats ppr_stats[B] or NULL.
 * PPR_FP64 runs the plain path once per source; PPR_MIXED runs the sources as
 * columns of an n x B block so that every edge read serves all columns.
 */
ppr_status ppr_query_batch(ppr_graph* g, const int32_t* sources, int32_t B, double alpha,
                           double lambda, ppr_precision precision, double* pi_out,
                           ppr_stats* stats);

/*
 * General form of the two calls above.  opt NULL means defaults.
 * r_out (nullable, double[B*n]) receives the final residue of each query
 * (PPR_FP64: the pushed residue r; PPR_MIXED: the FP64 residual of the flush).
 */
ppr_status ppr_query_ex(ppr_graph* g, const int32_t* sources, int32_t B, double alpha,
                        double lambda, const ppr_options* opt, double* pi_out, double* r_out,
                        ppr_stats* stats);

/* ------------------------------------------------------------------ */
/* Approximate SSPPR: SpeedPPR (Section 6, Algorithm 4).               */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t source;
    int32_t local_levels;        /* PowerPush local iterations (phase 1) */
    int32_t sweeps;              /* PowerPush global sweeps (phase 1) */
    int32_t refine_levels;       /* refinement iterations (every active node pushes at once) */
    int64_t refine_edge_pushes;  /* residue updates of the refinement */
    int64_t walks;               /* alpha-random walks of the Monte Carlo phase (index entries
                                    read when the index is used) */
    double W;                    /* Eq. 8 */
    double lambda;               /* phase 1 threshold m / W (at most 1) */
    double r_sum;                /* residue mass the walks distribute */
    double ms_push, ms_refine, ms_walks, ms;   /* host wall time per phase and in all */
    int32_t used_index;
    int32_t reserved;
} ppr_approx_stats;

/*
 * One approximate query (Algorithm 4): with W = 2 (2 eps / 3 + 2) ln n /
 * (eps^2 mu) (Eq. 8), PowerPush to lambda = min(m / W, 1), the refinement
 * until no node is active w.r.t. rmax = 1 / W, then for every v with r(v) > 0
 * W_v = ceil(r(v) W) <= d_v alpha-random walks from v, each adding
 * r(v) / W_v to pi_hat at its stop node (Eqs. 9-10).  The estimate has
 * |pi_hat(v) - pi_s(v)| <= eps pi_s(v) for every v with pi_s(v) >= mu with
 * probability 1 - 1/n (Section 2's Approx-SSPPR).
 *   eps in (0, 1]; mu in (0, 1] (the literature's 1/n is the usual choice).
 *   seed: the walks' generator seed (walk j from v is a function of seed, v, j
 *   and the graph; see ppr_walk_index_build).
 *   use_index: 1 = read the walks from the graph's index (built with the same
 *   alpha and seed, else PPR_ERR_ARG); the result is then the same as
 *   without the index.
 *   opt: options of the phase-1 PowerPush (NULL = defaults with
 *   PPR_GLOBAL_EPOCHS, Algorithm 3's own thresholds, which leave fewer nodes
 *   active for the refinement than threshold-0 sweeps; it runs the PPR_FP64
 *   path whatever opt->precision says).
 *   pi_out: double[n], host or device.
 */
ppr_status ppr_query_approx(ppr_graph* g, int32_t s, double alpha, double eps, double mu, uint64_t seed,
                            int32_t use_index, const ppr_options* opt, double* pi_out, ppr_approx_stats* stats);

/*
 * The SpeedPPR index (Section 6): walk j from v for every j < d_v, m walks in
 * all, independent of eps; stored on the device beside the graph (4 m bytes)
 * until the graph is destroyed or the index rebuilt.  Walk j from v draws
 * from SplitMix64 seeded with splitmix(seed ^ splitmix(v << 32 | j)) (output
 * k of SplitMix64 seeded with b being mix(b + (k + 1) 0x9E3779B97F4A7C15));
 * step t stops when (draw 2t >> 11) 2^-53 < alpha, else moves along out-edge
 * ((draw 2t+1 >> 32) d_v) >> 32 of the CSR; a walk alive after 4096 steps
 * stops where it is.  *ms (nullable) receives the build time.
 */
ppr_status ppr_walk_index_build(ppr_graph* g, double alpha, uint64_t seed, double* ms);
/* Host copy of the index: int32[m], entry row_ptr[v] + j = stop node of walk j from v. */
ppr_status ppr_walk_index_copy(const ppr_graph* g, int32_t* out);

/*
 * The two phases on caller data, for tests (pi, r: double[n] in device
 * memory).  ppr_debug_refine: the refinement w.r.t. rmax in place (levels,
 * edge_pushes nullable).  ppr_debug_walks: the Monte Carlo phase for budget W
 * on residue r, adding into pi; W_v = min(ceil(r(v) W), d_v); *walks
 * (nullable) receives the number of walks.
 */
ppr_status ppr_debug_refine(ppr_graph* g, double alpha, double rmax, double* pi, double* r, int32_t* levels,
                            int64_t* edge_pushes);
ppr_status ppr_debug_walks(ppr_graph* g, double alpha, double W, uint64_t seed, int32_t use_index,
                           const double* r, double* pi, int64_t* walks);

/* One point of a convergence trace (see ppr_query_trace). */
typedef struct {
    double ms;              /* host time since the call started, taken once the iteration has
                               completed on the device */
    double r_sum;           /* residue sum after the iteration (FP64).  The residues of the
                               PPR_FP64 path stay >= 0, so this is ||pi_hat - pi_s||_1 exactly
                               (Section 2: pi_s = pi_hat + sum_v r(v) pi_v, ||pi_v||_1 = 1) */
    int64_t edge_pushes;    /* residue updates so far: sum of d_v over pushed nodes (a
                               threshold-0 sweep counts m) */
    int32_t phase;          /* 0: local iteration S^(j); 1: global sweep or scan */
    int32_t index;          /* 1-based iteration number within its phase */
} ppr_trace_point;

/*
 * One PPR_FP64 query that records how its l1 error falls against time and
 * against residue updates (the quantities of Section 8's convergence
 * figures): a point after every local iteration and every global sweep or
 * scan.  Local points carry the running r_sum the switch test uses; global
 * points the exact sum after that sweep.  The traced run synchronises with
 * the device after every iteration (an untraced query replays its threshold-0
 * sweeps from a captured graph), so its times run a few percent above an
 * untraced query's.  With switch_param = 1e30 the query is power iteration
 * (Eqs. 3-6), with switch_param = 0 the level-synchronous forward push
 * (Algorithm 2), with global_rule = PPR_GLOBAL_EPOCHS Algorithm 3's epochs.
 *   opt: NULL = defaults; opt->precision must be PPR_FP64.
 *   pi_out: double[n], host or device.
 *   trace: host array of `capacity` points; *count (host) receives the number
 *   of iterations run; points beyond capacity are not written.
 *   Errors as ppr_query_ex; PPR_ERR_ARG if trace or count is NULL while
 *   capacity > 0, or capacity < 0.
 */
ppr_status ppr_query_trace(ppr_graph* g, int32_t s, double alpha, double lambda, const ppr_options* opt,
                           double* pi_out, ppr_trace_point* trace, int32_t capacity, int32_t* count,
                           ppr_stats* stats);

/*
 * One global sweep on caller data, for verification of the sweep kernel:
 * r_out = (1 - alpha) r_in P and pi += alpha r_in (Simultaneous Forward Push,
 * Eq. 7), all double[n] in device memory; *r_sum_out (host) receives
 * sum(r_out) in FP64.  The sweep of the FP64 queries: one pass per source
 * slice when the graph has them.
 */
ppr_status ppr_debug_sweep_fp64(ppr_graph* g, double alpha, const double* r_in, double* r_out,
                                double* pi, double* r_sum_out);

/*
 * One global sweep of the batched mixed path, for tests: the block
 * Gauss-Seidel sweep over `chunks` row chunks of about m / chunks in-edges
 * (chunk j starts at the first row whose CSC offset reaches floor(m j /
 * chunks)); with chunks = 1 it is the Eq. 7 step.  Row u of chunk j gets
 *   y_out(u) = (1-alpha)/d_u * ( sum_{v in N_in(u), v <  lo_j} y_out(v)
 *                              + sum_{v in N_in(u), v >= lo_j} y_in(v)
 *                              + fresh * sum_{v in N_in(u), v < lo_j} y_in(v) )
 * per column, i.e. Algorithm 3's in-place scan taken a chunk at a time in the
 * y domain (y(v) = (1-alpha) r(v) / d_v).  t_out (nullable) receives the
 * stage accumulator: y_out, plus y_in for the fresh columns.
 * With omega (host float[B], nullable) the sweep is over-relaxed: row u
 * pushes y_out(u) = omega * (the value above) + (1 - omega) * y_in(u) in the
 * columns that are not fresh, omega * (the value above) in the fresh ones.
 * This is a node that holds p = q + the value above, pushes omega p and keeps
 * q' = (1 - omega) p, with q = (1 - omega) / omega * y_in(u) (what it kept
 * when it pushed y_in(u)); a fresh residue has kept nothing back.
 * residue_format: ppr_residue_format (PPR_RESIDUE_AUTO: bf16 when B >= 32).
 * With bf16 storage (B >= 8) the block is stored in bf16: y_in is
 * rounded to bf16 (nearest, ties to even) on the way in, every y_out value
 * is the bf16 value the row stored (its out-neighbours pull exactly that),
 * and t_out adds those stored values; on an entry sweep a fresh column's row
 * pulls an earlier chunk's new value plus the fresh residue as one bf16
 * value.
 *   B: power of two in [4, 128]; chunks in [1, 64].
 *   y_in, y_out, t_out: float[n][B] (node-major), host or device memory.
 *   fresh: host int32[B] (1: the column's y_in is a residue nobody has
 *   received yet).
 */
ppr_status ppr_debug_sweep_mixed(ppr_graph* g, double alpha, int32_t B, int32_t chunks,
                                 const float* y_in, const int32_t* fresh, float* y_out,
                                 float* t_out, const float* omega, int32_t residue_format);

/*
 * Test entry point: one launch sequence of `sweeps` consecutive batched
 * global sweeps, each the sweep of ppr_debug_sweep_mixed (Algorithm 3's
 * global phase, Section 4.1, in block Gauss-Seidel order), with the stage
 * accumulator carried through the sequence as a query carries it between
 * refreshes.  ppr_debug_sweep_mixed is this with sweeps = 1, every budget 1
 * and T starting at 0.  Over-relaxed sweeps derive what a row kept back
 * from its previous push, so only the first sweep of a fresh column starts
 * from nothing kept.
 *   sweeps: in [1, 64].
 *   entry: host int32[B]: 0 the column continues (its y_in is already in
 *     T), 1 its y_in is a fresh residue (the first sweep adds it to T and
 *     its rows pull it along every in-edge), 2 the same with T restarting
 *     from y_in (t_in ignored for the column: a refresh has moved it into
 *     the reserve).
 *   budget: host int32[B] in [0, sweeps] (NULL: all `sweeps`): the sweeps
 *     the column runs; after them it stores 0 and its T stops growing.
 *   t_in: float[n][B], host or device, the accumulator at the start (NULL:
 *     0).  y_out: the residue after the last sweep; t_out (nullable): the
 *     accumulator after the sequence, i.e. t_in (unless entry 2), plus y_in
 *     for entry columns with a budget of at least one sweep, plus every
 *     residue the column's sweeps stored.
 *   sweep_tile: the LDS stage of a sweep block as ppr_options.sweep_tile
 *     (0: the graph's choice for width B).
 *   flags: 0, or PPR_DEBUG_WIDE_GATHER: the sweeps run on two residue
 *     buffers allocated apart, so that the gathers take full 64-bit addresses
 *     (the form used when a block's two residue buffers do not fit one
 *     4 GiB buffer; otherwise they gather at 32-bit offsets from its base).
 *     The results are the same bit for bit.
 *   Other arguments as ppr_debug_sweep_mixed; PPR_ERR_ARG for values out of
 *   range.
 */
#define PPR_DEBUG_WIDE_GATHER 1
ppr_status ppr_debug_sweeps_mixed(ppr_graph* g, double alpha, int32_t B, int32_t chunks, int32_t sweeps,
                                  const float* y_in, const int32_t* entry, const int32_t* budget,
                                  const float* t_in, float* y_out, float* t_out, const float* omega,
                                  int32_t residue_format, int32_t sweep_tile, int32_t flags);

/*
 * Autotuner of the batched path.  For each candidate block width (a power of
 * two in [4, 128]; widths NULL = {8, 16, 32, 64, 128}) and each residue
 * storage (FP32; bf16 from 8 columns) whose state fits half of the free
 * device memory: first the row tile of the sweep (an LDS stage of 12, 16 or
 * 24 KB per block, which sets the in-edges and rows a block takes) by timing
 * a few global sweeps with HIP events (16 KB unless another is more than 1%
 * faster); then, at that tile, the same Q queries for every width (Q the
 * largest candidate width; sources spread over the ids, this alpha and
 * lambda) answered end to end in Q / width batches after a warm-up batch:
 * local phase, sweeps, refreshes.  Each width keeps the storage with
 * the lower time per query, and the width with the lowest time per query
 * wins (a narrower width within 1%: less memory, lower latency).  The
 * choices are kept in the graph: the tile per (width, storage) for every
 * later batched block (queries and serving blocks), the storage per width
 * for queries with residue_format PPR_RESIDUE_AUTO, and the width for
 * ppr_options.batch_cols = 0.  Must not run while other calls use the graph.
 *   alpha in (0, 1), lambda in (0, 1]: the workload the batch times.
 *   widths: host int32[count] or NULL.  best_width: out.  cost_us: out,
 *   host double[count] (or [5] when widths is NULL), microseconds per query
 *   at the width's chosen storage and tile, -1 for a width skipped for
 *   memory; nullable.
 */
ppr_status ppr_autotune(ppr_graph* g, double alpha, double lambda, const int32_t* widths, int32_t count,
                        int32_t* best_width, double* cost_us);

/*
 * Serving: continuous batching of mixed-precision queries on one graph.
 *
 * A block holds `slots` query slots (the columns of one n x slots state in
 * device memory).  Each slot answers one single-source query with its own
 * source, alpha and lambda, by the same computation as ppr_query_ex with
 * PPR_MIXED: a frontier local phase over the iteration sets S^(j) of
 * Section 4.2 in FP64, global push sweeps in FP32 arithmetic (block
 * Gauss-Seidel order over row chunks, over-relaxed, residues stored in bf16
 * from 32 slots up), and FP64 refreshes whose residual (Eq. 1 rearranged)
 * certifies ||pi_hat - pi_s||_1 <= lambda.  A slot's schedule depends on its
 * own source, alpha and lambda only, so a query's result is the same
 * whichever other queries share the block (up to FP32 summation order).
 * Slots free up and refill while the others run.
 *
 * A block is used by one host thread at a time.  Blocks must be destroyed
 * before their graph (ppr_graph_destroy returns PPR_ERR_BUSY otherwise).
 */

/* Create a block.  slots: power of two in [4, 128].  alpha in (0, 1): the
 * block's reference stop probability, the default of ppr_slot_admit (the
 * per-node scale table of the FP32 sweeps holds (1 - alpha) / d_u; a slot
 * admitted with another alpha_b multiplies it by the FP32 factor
 * (1 - alpha_b) / (1 - alpha), one more rounding in its sweeps, which its FP64
 * refresh measures like any other).  opt (nullable): switch rule, max_sweeps
 * (a cap on each query's sweeps), refresh_factor, use_stream / stream (the
 * stream that carries every step of the block); opt->precision must be
 * PPR_MIXED (a block is the batched mixed path; PPR_FP64 queries go through
 * ppr_query_ex), else PPR_ERR_ARG.  PPR_ERR_OOM if the device memory
 * (ppr_block_footprint) cannot be allocated. */
ppr_status ppr_block_create(ppr_graph* g, int32_t slots, double alpha, const ppr_options* opt,
                            ppr_block** out);

/* Destroy a block (waits for its enqueued work).  NULL is a no-op. */
ppr_status ppr_block_destroy(ppr_block* blk);

/* Device bytes a block of `slots` slots allocates on this graph (for
 * admission against a memory budget); equal to ppr_footprint_bytes's
 * state_bytes for the graph's n and m. */
ppr_status ppr_block_footprint(const ppr_graph* g, int32_t slots, size_t* bytes);

/* Device memory before any graph exists (admission of a graph and its
 * queries against a budget), from the sizes alone:
 *   graph_bytes (nullable): what ppr_graph_create keeps for n nodes and m
 *     edges (CSR, CSC with uint32 offsets below 2^32 - 1 edges, degrees; the
 *     row schedules, a few percent more, are built on demand);
 *   state_bytes (nullable): PPR_MIXED: a serving block of `slots` columns
 *     (power of two in [4, 128]) with the default options, exactly what
 *     ppr_block_create allocates and ppr_block_footprint reports; PPR_FP64:
 *     an upper bound on `slots` (>= 1) concurrent PPR_FP64 queries, one
 *     pooled context each.
 * n >= 1 and n <= m <= n^2, else PPR_ERR_ARG. */
ppr_status ppr_footprint_bytes(int32_t n, int64_t m, int32_t slots, ppr_precision precision, size_t* graph_bytes,
                               size_t* state_bytes);

/* Put a query into a free slot; *slot receives its index.  The query starts
 * at the next ppr_block_step.  alpha: the query's stop probability in (0, 1)
 * (0: the block's reference alpha); each slot has its own alpha and lambda.
 * PPR_ERR_BUSY if every slot is taken, PPR_ERR_ARG for a source outside
 * [0, n), alpha outside (0, 1) and not 0, or lambda outside (0, 1]. */
ppr_status ppr_slot_admit(ppr_block* blk, int32_t source, double alpha, double lambda, int32_t* slot);

/* Advance the block: collect the previous step's results (waiting for them),
 * run the local phase of newly admitted slots, then enqueue up to max_sweeps
 * (>= 1) global sweeps and the FP64 refresh of every slot whose stage ends.
 * Returns once the work is enqueued; ppr_block_poll collects it. */
ppr_status ppr_block_step(ppr_block* blk, int32_t max_sweeps);

/* Collect the enqueued work if it has finished (wait = 1: wait for it).
 * done: host uint8[slots] (nullable), 1 for slots holding a finished query
 * (certified, or at its sweep cap); n_done, n_busy (admitted, not yet retired), ready (1 if nothing
 * is in flight): nullable outputs. */
ppr_status ppr_block_poll(ppr_block* blk, int32_t wait, uint8_t* done, int32_t* n_done,
                          int32_t* n_busy, int32_t* ready);

/* Copy a finished query's result out and free the slot.  pi_out: double[n],
 * host or device memory of the graph's device.  stats (nullable): the
 * query's statistics, ms = time from admission to retirement.  PPR_ERR_BUSY
 * if the slot holds no finished query.  PPR_ERR_NOT_CONVERGED if the query
 * reached max_sweeps with its certificate above lambda: pi_out and stats
 * still receive its estimate and certificate, and the slot is freed. */
ppr_status ppr_slot_retire(ppr_block* blk, int32_t slot, double* pi_out, ppr_stats* stats);

/* ------------------------------------------------------------------ */
/* Allocation-free query.                                              */
/* ------------------------------------------------------------------ */
/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * computation as ppr_query with PPR_FP64 and the default options (the local
 * phase over the iteration sets S^(j), then threshold-0 sweeps of Eq. 7
 * until r_sum <= lambda; the same kernels), but its working state lives in a
 * fixed device array of PPR_NOALLOC_SCRATCH_BYTES that the library holds on
 * every device it runs on until the process ends, and the reserve is written
 * straight into pi_out.  The call allocates no device or pinned memory and
 * creates no stream, event or HIP graph.
 *   Limits: n <= PPR_NOALLOC_MAX_NODES and at most
 *   PPR_NOALLOC_MAX_SWEEP_BLOCKS blocks in the graph's FP64 sweep schedule
 *   (about n / 256 + 3 m / 2048; m up to about 80M edges at the node limit);
 *   larger graphs give PPR_ERR_ARG and nothing runs.
 *   hip_stream: the caller's hipStream_t (NULL: the null stream); every
 *   kernel and copy of the call goes there, after the stream's earlier work.
 *   The call synchronises the stream before it returns.
 *   pi_out: double[n], device memory of the graph's device (host memory:
 *   PPR_ERR_ARG).  stats nullable; cert_l1 and sweep_ms are -1 (no
 *   certificate pass, no timing events).
 * The array is shared by every call on one device and keeps the last call's
 * contents; each call first writes everything it later reads.  Calls on one
 * device are serialised by a lock inside the library (one at a time per
 * device in this process); callers that overlap calls on one device wait.
 * Errors as ppr_query, plus PPR_ERR_ARG for the limits above.
 */
#define PPR_NOALLOC_MAX_NODES (1 << 20)
#define PPR_NOALLOC_MAX_SWEEP_BLOCKS (1 << 17)
#define PPR_NOALLOC_SCRATCH_BYTES 43057920u   /* 41.1 MiB per device */
ppr_status ppr_query_fp64_noalloc(ppr_graph* g, int32_t s, double alpha, double lambda, void* hip_stream,
                                  double* pi_out, ppr_stats* stats);

/* Library version string. */
const char* ppr_version(void);

/* Message of the last failure on the calling thread ("" if none). */
const char* ppr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PPR_H */
