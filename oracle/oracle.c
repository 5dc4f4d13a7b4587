/*
 * FP64 CPU oracle for high-precision single-source Personalized PageRank
 * (Wu, Gan, Wei, Zhang: "Unifying the Global and Local Approaches: An
 * Efficient Power Iteration with Forward Push", SIGMOD 2021).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  It shares no code, header, table or
 * helper with the GPU library; every routine is a plain, sequential, obviously
 * correct restatement of a definition or algorithm of the paper, in double
 * precision, with no blocking, fusion or reordering beyond what that passage
 * states.
 *
 * Graph: CSR of out-edges (Section 2): row_ptr[n+1] (int64), col[m] (int32);
 * d_v = row_ptr[v+1] - row_ptr[v] >= 1 (no dead ends, Section 2).  The
 * transition matrix P has row v equal to A_v / d_v (Section 2).
 *
 * Readings of points the paper leaves open (each is repeated in the design
 * notes of the repository):
 *  - a push snapshots x = r(v), sets r(v) = 0, then distributes; the printed
 *    order (distribute, then zero) loses mass on a self-loop (Section 3.2);
 *  - "u is active" is the strict test r(u) > d_u * rmax with rmax = lambda / m
 *    and the product taken in double precision (Section 3.2, Algorithm 3);
 *  - "Q.size() <= scanThreshold = n/4" is the integer test 4 |Q| <= n at the
 *    head of the local loop (Algorithm 3);
 *  - r_sum is maintained incrementally inside the local loop and recomputed
 *    exactly (Neumaier summation) after the local phase and after every scan
 *    or sweep; termination uses the recomputed value (Algorithm 3);
 *  - an epoch whose condition already fails runs zero scans (Algorithm 3);
 *  - the epoch loop condition of Algorithm 3, r_sum > m * rmax', is taken
 *    literally (so epoch i stops at an l1 error of lambda^(i/8)).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct {
    int64_t pushes;          /* push operations performed */
    int64_t edge_pushes;     /* residue updates: sum of d_v over pushes (Section 8) */
    int32_t local_levels;    /* iterations S^(j) processed by the local phase (Section 4.2) */
    int32_t sweeps;          /* global scans (Algorithm 3) or simultaneous sweeps (Eq. 7) */
    int32_t scans_per_epoch[8];
    int32_t switched;        /* 1 if the global phase ran */
    int32_t pad;
    double r_sum;            /* exact residue sum at return */
} oracle_stats;

/* ------------------------------------------------------------------ */
/* Compensated (Neumaier) summation of a vector.                        */
/* ------------------------------------------------------------------ */
double oracle_sum(int64_t len, const double* x) {
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double t = s + x[i];
        if (fabs(s) >= fabs(x[i])) c += (s - t) + x[i];
        else c += (x[i] - t) + s;
        s = t;
    }
    return s + c;
}

static double sum_abs(int64_t len, const double* x) {
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double a = fabs(x[i]);
        double t = s + a;
        if (s >= a) c += (s - t) + a; else c += (a - t) + s;
        s = t;
    }
    return s + c;
}

/* ------------------------------------------------------------------ */
/* In-edge lists (CSC) by counting sort: for every edge (v, u) of the   */
/* CSR, v is appended to the in-list of u while v runs 0..n-1, so each  */
/* in-list is ascending.  Also the out-degree table d_v (Section 2).    */
/* ------------------------------------------------------------------ */
int oracle_csc(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
               int64_t* col_ptr, int32_t* row_idx, int32_t* deg_out) {
    if (row_ptr[n] != m) return -1;
    for (int32_t u = 0; u <= n; ++u) col_ptr[u] = 0;
    for (int64_t e = 0; e < m; ++e) col_ptr[col[e] + 1]++;
    for (int32_t u = 0; u < n; ++u) col_ptr[u + 1] += col_ptr[u];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!fill) return -2;
    for (int32_t u = 0; u < n; ++u) fill[u] = col_ptr[u];
    for (int32_t v = 0; v < n; ++v) {
        deg_out[v] = (int32_t)(row_ptr[v + 1] - row_ptr[v]);
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) row_idx[fill[col[e]]++] = v;
    }
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Shared objects of the push-based methods (Sections 3.2, 4 and 5).    */
/* ------------------------------------------------------------------ */

/* Out-degree d_v of the CSR (Section 2). */
static int64_t out_degree(const int64_t* row_ptr, int32_t v) { return row_ptr[v + 1] - row_ptr[v]; }

/* Activity (Section 3.2): u is active w.r.t. rmax when r(u) > d_u * rmax,
   strict, with the product taken in double precision. */
static int is_active(const int64_t* row_ptr, const double* r, int32_t u, double rmax) {
    return r[u] > (double)out_degree(row_ptr, u) * rmax;
}

/* The queue of the forward-push methods (Algorithms 2 and 3): first in,
   first out, with a membership flag per node ("u not in Q" is a flag that is
   set on append and cleared on pop), so a node is held at most once and n
   places suffice.  Each entry also carries the iteration j of Section 4.2
   it belongs to: the source is in S^(0), and a node appended while a node
   of S^(j) is processed belongs to S^(j+1). */
typedef struct {
    int32_t* node;
    int32_t* iter;
    uint8_t* member;
    int64_t cap, head, size;
} push_queue;

static int queue_open(push_queue* q, int32_t n) {
    q->cap = n > 0 ? n : 1;
    q->node = (int32_t*)malloc(sizeof(int32_t) * (size_t)q->cap);
    q->iter = (int32_t*)malloc(sizeof(int32_t) * (size_t)q->cap);
    q->member = (uint8_t*)calloc((size_t)q->cap, 1);
    q->head = 0;
    q->size = 0;
    return q->node && q->iter && q->member;
}

static void queue_close(push_queue* q) {
    free(q->node);
    free(q->iter);
    free(q->member);
}

static void queue_append(push_queue* q, int32_t u, int32_t j) {
    int64_t at = (q->head + q->size) % q->cap;
    q->node[at] = u;
    q->iter[at] = j;
    q->member[u] = 1;
    q->size++;
}

static int32_t queue_pop(push_queue* q, int32_t* j) {
    int32_t v = q->node[q->head];
    *j = q->iter[q->head];
    q->head = (q->head + 1) % q->cap;
    q->size--;
    q->member[v] = 0;
    return v;
}

/* The push operation on v (Section 3.2): the residue x = r(v) is taken
   first (r(v) = 0, so that a self-loop's share is not lost), alpha x goes to
   the reserve of v, and each out-neighbour u receives (1 - alpha) x / d_v.
   With a queue, every out-neighbour that is active w.r.t. rmax after its
   share arrived and is not queued yet is appended, in iteration j + 1 (the
   forward-push methods); without one (q = NULL) the push only moves mass
   (the scans of the global phase).  Returns x. */
static double push_node(const int64_t* row_ptr, const int32_t* col, double alpha, double* pi, double* r,
                        int32_t v, push_queue* q, double rmax, int32_t j) {
    const double x = r[v];
    const int64_t d = out_degree(row_ptr, v);
    r[v] = 0.0;
    pi[v] += alpha * x;
    const double share = (1.0 - alpha) * x / (double)d;
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        const int32_t u = col[e];
        r[u] += share;
        if (q && !q->member[u] && is_active(row_ptr, r, u, rmax)) queue_append(q, u, j + 1);
    }
    return x;
}

/* Exported form of the push operation (Section 3.2). */
void oracle_push(const int64_t* row_ptr, const int32_t* col, double alpha,
                 double* pi, double* r, int32_t v) {
    (void)push_node(row_ptr, col, alpha, pi, r, v, NULL, 0.0, 0);
}

/* Start of every query: pi_hat = 0, r = e_s (Section 3.2). */
static void start_query(int32_t n, int32_t s, double* pi, double* r) {
    for (int32_t v = 0; v < n; ++v) { pi[v] = 0.0; r[v] = 0.0; }
    r[s] = 1.0;
}

/* ------------------------------------------------------------------ */
/* Forward Push in queue order (Algorithm 2): start from the source      */
/* queued, pop and push until the queue is empty; a pushed node queues   */
/* the out-neighbours it made active.  The iteration sets S^(j) of       */
/* Section 4.2 are the entries' iteration numbers.  trace_nodes /        */
/* trace_levels (nullable, trace_cap entries) receive each popped node   */
/* and its iteration j, in pop order.                                    */
/* Returns the number of pushes, or -2 if memory runs out.               */
/* ------------------------------------------------------------------ */
int64_t oracle_fifo_fwdpush(int32_t n, const int64_t* row_ptr, const int32_t* col,
                            int32_t s, double alpha, double rmax, double* pi, double* r,
                            int32_t* trace_nodes, int32_t* trace_levels, int64_t trace_cap,
                            oracle_stats* st) {
    push_queue q;
    if (!queue_open(&q, n)) { queue_close(&q); return -2; }
    start_query(n, s, pi, r);
    queue_append(&q, s, 0);
    int64_t pushes = 0, edges = 0;
    int32_t last_iter = 0;
    while (q.size > 0) {
        int32_t j;
        const int32_t v = queue_pop(&q, &j);
        if (trace_nodes && pushes < trace_cap) { trace_nodes[pushes] = v; trace_levels[pushes] = j; }
        if (j > last_iter) last_iter = j;
        (void)push_node(row_ptr, col, alpha, pi, r, v, &q, rmax, j);
        pushes++;
        edges += out_degree(row_ptr, v);
    }
    if (st) {
        memset(st, 0, sizeof(*st));
        st->pushes = pushes; st->edge_pushes = edges; st->local_levels = last_iter + 1;
        st->r_sum = oracle_sum(n, r);
    }
    queue_close(&q);
    return pushes;
}

/* ------------------------------------------------------------------ */
/* Power Iteration with Forward Push (Section 5, Algorithm 3) is two     */
/* phases over one state (pi_hat, r):                                    */
/*  - a local phase of queue-ordered forward pushes at rmax = lambda / m */
/*    that lasts while the queue is non-empty and small, and the residue */
/*    sum is above lambda (the queue is left once the active nodes are   */
/*    many: random access then costs more than a scan);                  */
/*  - if the residue sum is still above lambda, a global phase of        */
/*    sequential scans in id order, in epochs whose l1 error target      */
/*    lambda^(i/E) falls towards lambda (the dynamic l1 threshold, E = 8 */
/*    epochs).                                                           */
/* ------------------------------------------------------------------ */

/* Number of epochs of the global phase, and the queue-size bound of the
   local phase as a fraction of n (Algorithm 3's two constants). */
#define PP_EPOCHS 8
#define PP_QUEUE_FRACTION 4      /* the queue stays while |Q| <= n / 4 */

/* The local phase continues while these hold; "|Q| <= n/4" is read as the
   integer test 4 |Q| <= n, taken before each pop. */
static int local_phase_continues(const push_queue* q, int32_t n, double r_sum, double lambda) {
    return q->size > 0 && PP_QUEUE_FRACTION * q->size <= (int64_t)n && r_sum > lambda;
}

/* rmax' of epoch i: the residue mass per edge that still allows l1 error
   lambda^(i/E). */
static double epoch_rmax(double lambda, int i, int64_t m) {
    return pow(lambda, (double)i / (double)PP_EPOCHS) / (double)m;
}

/* One sequential scan: every node that is active w.r.t. rmax when the scan
   reaches it pushes in place, so it already holds what nodes earlier in the
   scan sent it (asynchronous pushes).  Adds the pushes and sum of d_v to st;
   returns the number of pushes. */
static int64_t sequential_scan(int32_t n, const int64_t* row_ptr, const int32_t* col, double alpha,
                               double rmax, double* pi, double* r, oracle_stats* st) {
    int64_t pushed = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (!is_active(row_ptr, r, v, rmax)) continue;
        (void)push_node(row_ptr, col, alpha, pi, r, v, NULL, 0.0, 0);
        pushed++;
        st->edge_pushes += out_degree(row_ptr, v);
    }
    st->pushes += pushed;
    return pushed;
}

/* The local phase; the residue sum is kept incrementally (a push removes
   alpha x from it).  Records the iterations reached in st. */
static int powerpush_local_phase(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                                 int32_t s, double alpha, double lambda, double* pi, double* r,
                                 oracle_stats* st) {
    push_queue q;
    if (!queue_open(&q, n)) { queue_close(&q); return -2; }
    const double rmax = lambda / (double)m;
    double r_sum = 1.0;
    int32_t last_iter = 0;
    queue_append(&q, s, 0);
    while (local_phase_continues(&q, n, r_sum, lambda)) {
        int32_t j;
        const int32_t v = queue_pop(&q, &j);
        if (j > last_iter) last_iter = j;
        r_sum -= alpha * push_node(row_ptr, col, alpha, pi, r, v, &q, rmax, j);
        st->pushes++;
        st->edge_pushes += out_degree(row_ptr, v);
    }
    st->local_levels = last_iter + 1;
    queue_close(&q);
    return 0;
}

/* The global phase: in epoch i, scans at rmax' = lambda^(i/E) / m repeat
   while the residue sum exceeds m rmax' (an epoch whose target is already
   met runs no scan); the sum is recomputed exactly after every scan, and a
   scan that pushes nothing ends its epoch. */
static void powerpush_global_phase(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                                   double alpha, double lambda, double* pi, double* r, double* r_sum,
                                   oracle_stats* st, double* rsum_trace, int32_t trace_cap, int* ntr) {
    for (int i = 1; i <= PP_EPOCHS; ++i) {
        const double rmax_i = epoch_rmax(lambda, i, m);
        while (*r_sum > (double)m * rmax_i) {
            const int64_t pushed = sequential_scan(n, row_ptr, col, alpha, rmax_i, pi, r, st);
            st->sweeps++;
            st->scans_per_epoch[i - 1]++;
            *r_sum = oracle_sum(n, r);
            if (rsum_trace && *ntr < trace_cap) rsum_trace[(*ntr)++] = *r_sum;
            if (pushed == 0) break;
        }
    }
}

/* ------------------------------------------------------------------ */
/* PowerPush (Algorithm 3): the local phase, the exact residue sum, and  */
/* the global phase if that sum is still above lambda.                   */
/* rsum_trace (nullable, trace_cap entries): exact r_sum after the local */
/* phase and after each scan.  Returns the number of trace entries       */
/* written, or -2 if memory runs out.                                    */
/* ------------------------------------------------------------------ */
int oracle_powerpush(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                     int32_t s, double alpha, double lambda, double* pi, double* r,
                     oracle_stats* st, double* rsum_trace, int32_t trace_cap) {
    oracle_stats S;
    memset(&S, 0, sizeof(S));
    int ntr = 0;
    start_query(n, s, pi, r);
    if (powerpush_local_phase(n, m, row_ptr, col, s, alpha, lambda, pi, r, &S) != 0) return -2;
    double r_sum = oracle_sum(n, r);
    if (rsum_trace && ntr < trace_cap) rsum_trace[ntr++] = r_sum;
    if (r_sum > lambda) {
        S.switched = 1;
        powerpush_global_phase(n, m, row_ptr, col, alpha, lambda, pi, r, &r_sum, &S, rsum_trace, trace_cap, &ntr);
    }
    S.r_sum = r_sum;
    if (st) *st = S;
    return ntr;
}

/* ------------------------------------------------------------------ */
/* One Simultaneous Forward Push iteration (Section 4.1, Eq. 7): every  */
/* node with non-zero residue pushes its residue r_in(v) at once, so    */
/* r_out = (1 - alpha) r_in P and pi += alpha r_in.  Pushes run over    */
/* v = 0..n-1 and each node's out-list in CSR order.                    */
/* ------------------------------------------------------------------ */
void oracle_sim_sweep(int32_t n, const int64_t* row_ptr, const int32_t* col, double alpha,
                      const double* r_in, double* r_out, double* pi) {
    for (int32_t u = 0; u < n; ++u) r_out[u] = 0.0;
    for (int32_t v = 0; v < n; ++v) {
        double x = r_in[v];
        if (x == 0.0) continue;
        int64_t d = row_ptr[v + 1] - row_ptr[v];
        pi[v] += alpha * x;
        double inc = (1.0 - alpha) * x / (double)d;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) r_out[col[e]] += inc;
    }
}

/* ------------------------------------------------------------------ */
/* One global sweep in block Gauss-Seidel order, written in the y       */
/* domain: y(v) = (1 - alpha) r(v) / d_v is what each out-neighbour of  */
/* v receives when v pushes r(v) (the push of Section 3.2).  The rows   */
/* are cut into chunks [lo[j], lo[j+1]); chunk j is handled after       */
/* chunks 0..j-1, and node u of chunk j pushes everything it received   */
/* since its previous push:                                             */
/*   y_new(u) = (1-alpha)/d_u * ( sum_{v in N_in(u), v <  lo[j]} y_new(v) */
/*                              + sum_{v in N_in(u), v >= lo[j]} y_old(v) */
/*                              + fresh * sum_{v in N_in(u), v < lo[j]} y_old(v) ) */
/* i.e. the in-place scan of Algorithm 3's global phase taken one chunk  */
/* at a time (a node sees the pushes of earlier chunks made in the same  */
/* scan).  y_old holds the previous sweep's pushes, of which nodes in    */
/* later chunks already received their share; with fresh = 1 it holds a  */
/* residue nobody has received yet (the first sweep after a residue is   */
/* formed), which every out-neighbour receives in this sweep.  One chunk */
/* (lo = {0, n}) is Eq. 7.  Uses the CSC of oracle_csc.                  */
/* ------------------------------------------------------------------ */
void oracle_block_gs_sweep(int32_t n, const int64_t* col_ptr, const int32_t* row_idx, const int32_t* deg,
                           double alpha, int32_t chunks, const int32_t* lo, const double* y_old, int fresh,
                           double* y_new) {
    for (int32_t j = 0; j < chunks; ++j) {
        for (int32_t u = lo[j]; u < lo[j + 1]; ++u) {
            double acc = 0.0;
            for (int64_t e = col_ptr[u]; e < col_ptr[u + 1]; ++e) {
                int32_t v = row_idx[e];
                if (v < lo[j]) {
                    acc += y_new[v];
                    if (fresh) acc += y_old[v];
                } else {
                    acc += y_old[v];
                }
            }
            y_new[u] = (1.0 - alpha) / (double)deg[u] * acc;
        }
    }
}

/* ------------------------------------------------------------------ */
/* The same sweep over-relaxed: node u of chunk j holds                  */
/*   p(u) = q_in(u) + (the block Gauss-Seidel value above)               */
/* (q_in: what u kept back at its previous push), pushes                 */
/* y_new(u) = omega p(u) and keeps q_out(u) = (1 - omega) p(u).  In the  */
/* reserve domain (S = the sum of a node's pushes y) this is successive  */
/* over-relaxation of the block Gauss-Seidel iteration for Eq. 1;        */
/* omega = 1 is oracle_block_gs_sweep with q_out = 0.                   */
/* ------------------------------------------------------------------ */
void oracle_block_sor_sweep(int32_t n, const int64_t* col_ptr, const int32_t* row_idx, const int32_t* deg,
                            double alpha, int32_t chunks, const int32_t* lo, const double* y_old, int fresh,
                            double omega, const double* q_in, double* q_out, double* y_new) {
    for (int32_t j = 0; j < chunks; ++j) {
        for (int32_t u = lo[j]; u < lo[j + 1]; ++u) {
            double acc = 0.0;
            for (int64_t e = col_ptr[u]; e < col_ptr[u + 1]; ++e) {
                int32_t v = row_idx[e];
                if (v < lo[j]) {
                    acc += y_new[v];
                    if (fresh) acc += y_old[v];
                } else {
                    acc += y_old[v];
                }
            }
            double p = q_in[u] + (1.0 - alpha) / (double)deg[u] * acc;
            y_new[u] = omega * p;
            q_out[u] = (1.0 - omega) * p;
        }
    }
}

/* ------------------------------------------------------------------ */
/* The level-synchronous schedule that the GPU path runs, stated with   */
/* the paper's objects:                                                 */
/*  - local phase: the iterations S^(j) of Section 4.2, each performed  */
/*    simultaneously (every node of S^(j) pushes the residue it held at */
/*    the start of the iteration; Section 4.1); S^(j+1) is the set of   */
/*    nodes whose residue became active during iteration j.  The phase  */
/*    runs while S^(j) is non-empty, r_sum > lambda and the switch rule */
/*    allows it;                                                        */
/*  - global phase (global_rule 0): Simultaneous Forward Push with      */
/*    rmax = 0 (Eq. 7), identical to power iteration by Lemma 1, until  */
/*    r_sum <= lambda; (global_rule 1): Algorithm 3's epochs with each  */
/*    scan taken simultaneously over the nodes active at its start.     */
/* Switch rule 0: continue while 4 |S^(j)| <= n (Algorithm 3's          */
/* scanThreshold = n/4).  Rule 1: continue while                        */
/* switch_param * sum_{v in S^(j)} d_v <= m (edge volume).              */
/* The local r_sum is updated as r_sum - alpha * sum_{v in S^(j)} x_v   */
/* per iteration (Eq. 8) and recomputed exactly when the phase ends;    */
/* the global phase recomputes it exactly after every sweep.            */
/* Per iteration j (nullable arrays of level_cap entries): level_sizes  */
/* receives |S^(j)|, level_vols sum_{v in S^(j)} d_v, level_rsum the    */
/* r_sum at the start of iteration j (used to check Eq. 9).             */
/* Returns 0, or -2 if memory runs out.                                 */
/* ------------------------------------------------------------------ */
int oracle_powerpush_sync(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                          int32_t s, double alpha, double lambda, int switch_rule,
                          double switch_param, int global_rule, double* pi, double* r, oracle_stats* st,
                          double* rsum_trace, int32_t trace_cap,
                          int32_t* level_sizes, int64_t* level_vols, double* level_rsum,
                          int32_t level_cap) {
    int32_t* F = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* F2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    double* x = (double*)malloc(sizeof(double) * (size_t)n);
    double* r2 = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!F || !F2 || !x || !r2 || !mark) { free(F); free(F2); free(x); free(r2); free(mark); return -2; }
    oracle_stats S;
    memset(&S, 0, sizeof(S));
    int ntr = 0;
    for (int32_t v = 0; v < n; ++v) { pi[v] = 0.0; r[v] = 0.0; mark[v] = -1; }
    r[s] = 1.0;
    double r_sum = 1.0;
    double rmax = lambda / (double)m;
    int64_t nf = 1;
    F[0] = s;
    int32_t level = 0;
    for (;;) {
        if (nf == 0 || !(r_sum > lambda)) break;
        int64_t vol = 0;
        for (int64_t i = 0; i < nf; ++i) vol += row_ptr[F[i] + 1] - row_ptr[F[i]];
        if (switch_rule == 0 && !(4 * nf <= (int64_t)n)) break;
        if (switch_rule == 1 && !(switch_param * (double)vol <= (double)m)) break;
        if (level < level_cap) {
            if (level_sizes) level_sizes[level] = (int32_t)nf;
            if (level_vols) level_vols[level] = vol;
            if (level_rsum) level_rsum[level] = r_sum;
        }
        /* snapshot: every node of S^(j) pushes the residue it holds now */
        double taken = 0.0;
        for (int64_t i = 0; i < nf; ++i) {
            int32_t v = F[i];
            x[i] = r[v];
            r[v] = 0.0;
            pi[v] += alpha * x[i];
            taken += alpha * x[i];
        }
        /* distribute; a node joins S^(j+1) the first time its residue is active */
        int64_t nf2 = 0;
        for (int64_t i = 0; i < nf; ++i) {
            int32_t v = F[i];
            int64_t d = row_ptr[v + 1] - row_ptr[v];
            double inc = (1.0 - alpha) * x[i] / (double)d;
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int32_t u = col[e];
                r[u] += inc;
                double du = (double)(row_ptr[u + 1] - row_ptr[u]);
                if (mark[u] != level + 1 && r[u] > du * rmax) { mark[u] = level + 1; F2[nf2++] = u; }
            }
        }
        S.pushes += nf;
        S.edge_pushes += vol;
        r_sum -= taken;
        int32_t* t = F; F = F2; F2 = t;
        nf = nf2;
        level++;
    }
    S.local_levels = level;
    r_sum = oracle_sum(n, r);
    if (rsum_trace && ntr < trace_cap) rsum_trace[ntr++] = r_sum;
    if (r_sum > lambda) S.switched = 1;
    if (global_rule == 0) {
        while (r_sum > lambda) {
            oracle_sim_sweep(n, row_ptr, col, alpha, r, r2, pi);
            memcpy(r, r2, sizeof(double) * (size_t)n);
            S.sweeps++;
            S.edge_pushes += m;
            S.pushes += n;
            r_sum = oracle_sum(n, r);
            if (rsum_trace && ntr < trace_cap) rsum_trace[ntr++] = r_sum;
        }
    } else {
        /* Algorithm 3's epochs (rmax_i = lambda^(i/8) / m, scans while
           r_sum > m rmax_i, taken literally), each scan taken simultaneously: every
           node active at the start of the scan (r(v) > d_v rmax_i) pushes the
           residue it holds then (Simultaneous Forward Push of Section 4.1 with
           threshold rmax_i).  A scan with no active node ends the epoch; scans
           at rmax_8 = lambda / m continue while rounding leaves r_sum above
           lambda. */
        for (int i = 1; i <= 9; ++i) {
            const int last = (i == 9);
            double rmax_i = pow(lambda, (double)(last ? 8 : i) / 8.0) / (double)m;
            for (;;) {
                if (last ? !(r_sum > lambda) : !(r_sum > (double)m * rmax_i)) break;
                int64_t nact = 0, vol = 0;
                for (int32_t v = 0; v < n; ++v) {
                    int64_t d = row_ptr[v + 1] - row_ptr[v];
                    if (r[v] > (double)d * rmax_i) {
                        x[v] = r[v];
                        r[v] = 0.0;
                        pi[v] += alpha * x[v];
                        nact++;
                        vol += d;
                    } else {
                        x[v] = 0.0;
                    }
                }
                if (nact == 0) break;
                for (int32_t v = 0; v < n; ++v) {
                    if (x[v] == 0.0) continue;
                    int64_t d = row_ptr[v + 1] - row_ptr[v];
                    double inc = (1.0 - alpha) * x[v] / (double)d;
                    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) r[col[e]] += inc;
                }
                S.sweeps++;
                S.edge_pushes += vol;
                S.pushes += nact;
                r_sum = oracle_sum(n, r);
                if (rsum_trace && ntr < trace_cap) rsum_trace[ntr++] = r_sum;
            }
        }
    }
    S.r_sum = r_sum;
    if (st) *st = S;
    free(F); free(F2); free(x); free(r2); free(mark);
    return ntr;
}

/* ------------------------------------------------------------------ */
/* Power iteration (Section 3.1, Eqs. 3-5): gamma^(0) = e_s,            */
/* gamma^(j+1) = (1 - alpha) gamma^(j) P, and the estimate after K      */
/* iterations is sum_{k<K} alpha gamma^(k), whose l1 error is exactly   */
/* (1 - alpha)^K (Eq. 6).  The estimate is accumulated with Neumaier    */
/* compensation so that it serves as the converged truth.               */
/* ------------------------------------------------------------------ */
int oracle_powitr(int32_t n, const int64_t* row_ptr, const int32_t* col, int32_t s,
                  double alpha, int32_t K, double* pi_out) {
    double* g = (double*)calloc((size_t)n, sizeof(double));
    double* g2 = (double*)malloc(sizeof(double) * (size_t)n);
    double* comp = (double*)calloc((size_t)n, sizeof(double));
    if (!g || !g2 || !comp) { free(g); free(g2); free(comp); return -2; }
    for (int32_t v = 0; v < n; ++v) pi_out[v] = 0.0;
    g[s] = 1.0;
    for (int32_t j = 0; j < K; ++j) {
        for (int32_t v = 0; v < n; ++v) {
            double a = alpha * g[v];
            double t = pi_out[v] + a;
            if (fabs(pi_out[v]) >= fabs(a)) comp[v] += (pi_out[v] - t) + a;
            else comp[v] += (a - t) + pi_out[v];
            pi_out[v] = t;
        }
        for (int32_t u = 0; u < n; ++u) g2[u] = 0.0;
        for (int32_t v = 0; v < n; ++v) {
            if (g[v] == 0.0) continue;
            int64_t d = row_ptr[v + 1] - row_ptr[v];
            double inc = (1.0 - alpha) * g[v] / (double)d;
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) g2[col[e]] += inc;
        }
        double* t = g; g = g2; g2 = t;
    }
    for (int32_t v = 0; v < n; ++v) pi_out[v] += comp[v];
    free(g); free(g2); free(comp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Residual certificate, from the linear system of Eq. 1:               */
/*   rt = e_s - (pi_hat - (1 - alpha) pi_hat P) / alpha.                */
/* Since the PPR vectors pi_v are the rows of alpha (I - (1-alpha)P)^-1,*/
/* pi_s - pi_hat = sum_v rt(v) pi_v, and with ||pi_v||_1 = 1            */
/* (Section 2), ||pi_hat - pi_s||_1 <= ||rt||_1, with equality when     */
/* rt >= 0.  Returns ||rt||_1 (compensated); rt is written if non-null. */
/* ------------------------------------------------------------------ */
double oracle_certificate(int32_t n, const int64_t* row_ptr, const int32_t* col, int32_t s,
                          double alpha, const double* pi_hat, double* rt_out) {
    double* q = (double*)calloc((size_t)n, sizeof(double));   /* q = pi_hat P */
    double* rt = rt_out ? rt_out : (double*)malloc(sizeof(double) * (size_t)n);
    if (!q || !rt) { free(q); if (!rt_out) free(rt); return -1.0; }
    for (int32_t v = 0; v < n; ++v) {
        if (pi_hat[v] == 0.0) continue;
        int64_t d = row_ptr[v + 1] - row_ptr[v];
        double inc = pi_hat[v] / (double)d;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) q[col[e]] += inc;
    }
    for (int32_t u = 0; u < n; ++u)
        rt[u] = (u == s ? 1.0 : 0.0) - (pi_hat[u] - (1.0 - alpha) * q[u]) / alpha;
    double l1 = sum_abs(n, rt);
    free(q);
    if (!rt_out) free(rt);
    return l1;
}

/* ------------------------------------------------------------------ */
/* Several independent queries of Algorithm 3, one per thread; used to  */
/* time the oracle on the host's cores.  pi_out / r_out hold count rows */
/* of n doubles.  Returns 0, or -2 if a query ran out of memory.        */
/* ------------------------------------------------------------------ */
int oracle_powerpush_many(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                          const int32_t* sources, int32_t count, double alpha, double lambda,
                          double* pi_out, double* r_out, oracle_stats* st, int32_t threads) {
    int rc = 0;
    #pragma omp parallel for schedule(dynamic, 1) num_threads(threads) reduction(min:rc)
    for (int32_t i = 0; i < count; ++i) {
        int k = oracle_powerpush(n, m, row_ptr, col, sources[i], alpha, lambda,
                                 pi_out + (int64_t)i * n, r_out + (int64_t)i * n,
                                 st ? st + i : NULL, NULL, 0);
        if (k < 0) rc = k;
    }
    return rc;
}

/* ================================================================== */
/* Approximate SSPPR: SpeedPPR (Section 6, Algorithm 4).              */
/* ================================================================== */

/* W of Eq. 8: the number of alpha-random walks from s that the Monte  */
/* Carlo method needs for relative error eps on every node with        */
/* pi(s, v) >= mu, with probability 1 - 1/n (Chernoff bound).  Reading: */
/* "log" is the natural logarithm.                                      */
double oracle_walk_budget(int32_t n, double eps, double mu) {
    return 2.0 * (2.0 * eps / 3.0 + 2.0) * log((double)n) / (eps * eps * mu);
}

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the output for state z */
/* is mix(z + gamma).  Used as a counter-based generator: draw k of the  */
/* generator seeded with b is oracle_splitmix64(b + k * gamma).          */
#define ORACLE_GAMMA 0x9E3779B97F4A7C15ULL
uint64_t oracle_splitmix64(uint64_t z) {
    z += ORACLE_GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Stop node of walk j from v (an alpha-random walk, Section 2: at each   */
/* node it stops with probability alpha, else moves to an out-neighbour   */
/* chosen uniformly).  The walk's draws come from SplitMix64 seeded with  */
/* b = splitmix64(seed ^ splitmix64(v << 32 | j)); step t uses draw 2t    */
/* for the stop test (top 53 bits as a uniform in [0, 1): stop when it is */
/* < alpha) and draw 2t + 1 for the neighbour (index = (top 32 bits * d)  */
/* >> 32, i.e. floor of a uniform times d).  A walk still alive after     */
/* max_steps steps stops where it is (probability (1 - alpha)^max_steps). */
int32_t oracle_walk_endpoint(const int64_t* row_ptr, const int32_t* col, double alpha, uint64_t seed,
                             int32_t v, uint32_t j, int32_t max_steps) {
    uint64_t b = oracle_splitmix64(seed ^ oracle_splitmix64(((uint64_t)(uint32_t)v << 32) | (uint64_t)j));
    int32_t cur = v;
    for (int32_t t = 0; t < max_steps; ++t) {
        uint64_t x = oracle_splitmix64(b + (uint64_t)(2 * t) * ORACLE_GAMMA);
        double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);   /* 2^-53 */
        if (u < alpha) break;
        uint64_t y = oracle_splitmix64(b + (uint64_t)(2 * t + 1) * ORACLE_GAMMA);
        uint64_t d = (uint64_t)(row_ptr[cur + 1] - row_ptr[cur]);
        uint64_t idx = ((y >> 32) * d) >> 32;
        cur = col[row_ptr[cur] + (int64_t)idx];
    }
    return cur;
}

/* The refinement of Algorithm 4 (no node active w.r.t. rmax), taken       */
/* level-synchronously: S = { v : r(v) > d_v rmax }; every node of S pushes */
/* at once the residue it holds (x = r(v), r(v) = 0, pi(v) += alpha x, each */
/* out-neighbour gets (1 - alpha) x / d_v); the next S holds the nodes      */
/* active after the distribution; until S is empty.  Returns the number of  */
/* levels; *edge_pushes (nullable) receives sum of d_v over the pushes.      */
int32_t oracle_refine_sync(int32_t n, const int64_t* row_ptr, const int32_t* col, double alpha, double rmax,
                           double* pi, double* r, int64_t* edge_pushes) {
    double* x = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* S = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!x || !S) { free(x); free(S); return -2; }
    int32_t levels = 0;
    int64_t pushes = 0;
    for (;;) {
        int32_t ns = 0;
        for (int32_t v = 0; v < n; ++v) {
            double d = (double)(row_ptr[v + 1] - row_ptr[v]);
            if (r[v] > d * rmax) S[ns++] = v;
        }
        if (ns == 0) break;
        for (int32_t i = 0; i < ns; ++i) {
            int32_t v = S[i];
            x[i] = r[v];
            r[v] = 0.0;
            pi[v] += alpha * x[i];
        }
        for (int32_t i = 0; i < ns; ++i) {
            int32_t v = S[i];
            int64_t d = row_ptr[v + 1] - row_ptr[v];
            double inc = (1.0 - alpha) * x[i] / (double)d;
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) r[col[e]] += inc;
            pushes += d;
        }
        levels++;
    }
    free(x);
    free(S);
    if (edge_pushes) *edge_pushes = pushes;
    return levels;
}

/* The Monte Carlo phase of Algorithm 4 (FORA's second phase, Eqs. 9-10):  */
/* for every v with r(v) > 0, W_v = ceil(r(v) W) walks from v (capped at   */
/* d_v, which a refined residue meets up to rounding: r(v) <= d_v / W);    */
/* each walk that stops at u adds r(v) / W_v to pi(u).  Walk j of v is     */
/* oracle_walk_endpoint(.., v, j, ..).  Returns the number of walks.        */
int64_t oracle_mc_phase(int32_t n, const int64_t* row_ptr, const int32_t* col, double alpha, double W,
                        uint64_t seed, int32_t max_steps, const double* r, double* pi) {
    int64_t walks = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (!(r[v] > 0.0)) continue;
        int64_t d = row_ptr[v + 1] - row_ptr[v];
        int64_t wv = (int64_t)ceil(r[v] * W);
        if (wv > d) wv = d;
        double share = r[v] / (double)wv;
        for (int64_t j = 0; j < wv; ++j) {
            int32_t u = oracle_walk_endpoint(row_ptr, col, alpha, seed, v, (uint32_t)j, max_steps);
            pi[u] += share;
        }
        walks += wv;
    }
    return walks;
}
