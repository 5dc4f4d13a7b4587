// The plain FP64 single-query path: local phase over frontiers, then global
// pull sweeps, with the sweep loop replayed from a captured HIP graph.
#include <chrono>
#include <cmath>
#include <cstring>

#include "ppr_internal.h"

namespace ppr {

QueryCtx::~QueryCtx() {
    if (chunk_exec) (void)hipGraphExecDestroy(chunk_exec);
    if (own) (void)hipStreamDestroy(own);
}

std::unique_ptr<QueryCtx> ctx_acquire(Graph& g) {
    {
        std::lock_guard<std::mutex> lk(g.pool_mu);
        if (!g.pool.empty()) {
            auto c = std::move(g.pool.back());
            g.pool.pop_back();
            return c;
        }
    }
    auto c = std::make_unique<QueryCtx>();
    const size_t n = (size_t)g.n;
    c->n = g.n;
    HIPCHECK(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
    c->stream = c->own;
    c->r.alloc(8 * n);
    c->pi.alloc(8 * n);
    c->y0.alloc(8 * n);
    c->y1.alloc(8 * n);
    c->F0.alloc(4 * n);
    c->F1.alloc(4 * n);
    c->X.alloc(8 * n);
    c->degF.alloc(8 * n);
    c->off.alloc(8 * (n + 1));
    const Schedule& sch = g.schedule(k::sweep_nnz_cap(), k::sweep_row_cap());
    size_t parts = std::max<size_t>({(size_t)sch.n_blocks, 4096, (n + 255) / 256});
    for (const auto& ss : g.sl_sched) parts = std::max(parts, (size_t)ss->n_blocks);
    c->partials.alloc(8 * parts);
    if (g.fp64_slices > 1) {
        c->acc.alloc(8 * n);
        HIPCHECK(hipMemset(c->acc.p, 0, 8 * n));   // a sliced sweep starts from 0 and leaves 0
    }
    c->scan_tmp.alloc(k::scan_tmp_bytes(std::max<int64_t>(g.n, 4096)));
    c->aux.alloc(8 * (size_t)kAuxLen);
    c->ctr.alloc(64);
    c->dsum.alloc(64);
    c->host.alloc(64);
    return c;
}

void ctx_release(Graph& g, std::unique_ptr<QueryCtx> c) {
    std::lock_guard<std::mutex> lk(g.pool_mu);
    g.pool.push_back(std::move(c));
}

// Upper bound on what ctx_acquire allocates for n nodes: eight n-vectors of
// 8 bytes and two of 4 (state, frontier lists, increments, degrees, prefix,
// the row sums across source slices), per-block partials (a sweep schedule
// has at most one block per row), the scan scratch, the compaction counters
// and the readback area.
size_t fp64_ctx_footprint(int32_t n) {
    const size_t nn = (size_t)n;
    return 8 * 8 * nn + 4 * 2 * nn + 8 + 8 * std::max<size_t>({nn, 4096, (nn + 255) / 256}) +
           k::scan_tmp_bytes(std::max<int64_t>(n, 4096)) + 8 * (size_t)kAuxLen + 192;
}

namespace {

// A pooled context for one query; with the caller's stream (options
// use_stream) every launch and copy of the query goes there.
struct CtxLease {
    Graph& g;
    std::unique_ptr<QueryCtx> c;
    CtxLease(Graph& gg, const ppr_options& opt) : g(gg), c(ctx_acquire(gg)) {
        if (opt.use_stream) c->stream = static_cast<hipStream_t>(opt.stream);
    }
    ~CtxLease() {
        if (c) {
            (void)hipStreamSynchronize(c->stream);
            c->stream = c->own;
            ctx_release(g, std::move(c));
        }
    }
};

constexpr int kChunkPairs = 8;   // a captured chunk is 16 FOLD sweeps

// Capture [FOLD y1 -> y0, FOLD y0 -> y1] x kChunkPairs on the context's own
// stream (the work stream may be the caller's null stream, which cannot be
// captured); the work stream launches the instantiated graph.
void ensure_chunk(Graph& g, QueryCtx& c, const Schedule& sch, double alpha) {
    if (c.chunk_exec && c.chunk_alpha == alpha) return;
    if (c.chunk_exec) {
        (void)hipGraphExecDestroy(c.chunk_exec);
        c.chunk_exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    HIPCHECK(hipStreamBeginCapture(c.own, hipStreamCaptureModeThreadLocal));
    try {
        for (int p = 0; p < kChunkPairs; ++p) {
            k::sweep_f64(g, sch, k::SW_FOLD, alpha, c.y1.as<double>(), c.y0.as<double>(), c.pi.as<double>(),
                         nullptr, nullptr, c.partials.as<double>(), c.own, c.acc.as<double>());
            k::sweep_f64(g, sch, k::SW_FOLD, alpha, c.y0.as<double>(), c.y1.as<double>(), c.pi.as<double>(),
                         nullptr, nullptr, c.partials.as<double>(), c.own, c.acc.as<double>());
        }
    } catch (...) {
        (void)hipStreamEndCapture(c.own, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    HIPCHECK(hipStreamEndCapture(c.own, &graph));
    hipError_t e = hipGraphInstantiate(&c.chunk_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHECK(e);
    c.chunk_pairs = kChunkPairs;
    c.chunk_alpha = alpha;
}

bool continue_local(const ppr_options& opt, int64_t nf, int64_t vol, int32_t n, int64_t m) {
    if (opt.switch_rule == PPR_SWITCH_NODES) return 4 * nf <= (int64_t)n;
    return opt.switch_param * (double)vol <= (double)m;
}

}  // namespace

void run_fp64_query(Graph& g, int32_t s, double alpha, double lambda, const ppr_options& opt,
                    double* pi_out, double* r_out, ppr_stats* st, TraceSink* trace) {
    auto t0 = std::chrono::steady_clock::now();
    HIPCHECK(hipSetDevice(g.device));
    CtxLease lease(g, opt);
    QueryCtx& c = *lease.c;
    hipStream_t ss = c.stream;
    const Schedule& sch = g.schedule(k::sweep_nnz_cap(), k::sweep_row_cap());
    double* r = c.r.as<double>();
    double* pi = c.pi.as<double>();
    double* partials = c.partials.as<double>();
    double* acc = c.acc.as<double>();          // row sums across source slices (nullptr: none)
    if (acc) HIPCHECK(hipMemsetAsync(acc, 0, 8 * (size_t)g.n, ss));   // whatever an earlier query left
    int64_t* hctr = c.host.as<int64_t>();
    double* hd = c.host.as<double>();
    const int32_t* deg = g.deg.as<int32_t>();

    // ---- local phase: iterations S^(j) pushed simultaneously
    k::query_init(r, pi, g.n, s, c.F0.as<int32_t>(), ss);
    int32_t* F = c.F0.as<int32_t>();
    int32_t* Fn = c.F1.as<int32_t>();
    int64_t nf = 1, vol = g.h_deg[s];
    double r_sum = 1.0;
    const double rmax = lambda / (double)g.m;
    int32_t levels = 0;
    int64_t edge_pushes = 0;
    while (nf > 0 && r_sum > lambda && continue_local(opt, nf, vol, g.n, g.m)) {
        int np = 0;
        k::frontier_snapshot(F, (int32_t)nf, deg, alpha, r, pi, c.X.as<double>(), c.degF.as<int64_t>(),
                             partials, &np, ss);
        k::reduce_sum(partials, np, c.dsum.as<double>(), ss);
        k::exclusive_scan_i64(c.degF.as<int64_t>(), c.off.as<int64_t>(), nf, c.scan_tmp.p, ss);
        HIPCHECK(hipMemsetAsync(c.ctr.p, 0, 16, ss));
        k::frontier_push(F, c.off.as<int64_t>(), (int32_t)nf, vol, g.row_ptr.as<int64_t>(), g.col.as<int32_t>(),
                         deg, c.X.as<double>(), rmax, r, Fn, c.ctr.as<int64_t>(), ss);
        HIPCHECK(hipMemcpyAsync(hctr, c.ctr.p, 16, hipMemcpyDeviceToHost, ss));
        HIPCHECK(hipMemcpyAsync(hd + 2, c.dsum.p, 8, hipMemcpyDeviceToHost, ss));
        HIPCHECK(hipStreamSynchronize(ss));
        edge_pushes += vol;
        r_sum -= hd[2];
        nf = hctr[0];
        vol = hctr[1];
        std::swap(F, Fn);
        ++levels;
        if (trace) trace->note(0, levels, edge_pushes, r_sum);
    }

    // ---- exact r_sum, and y = (1-alpha) r / d for the first sweep
    {
        int np = 0;
        k::prep_y(r, deg, alpha, g.n, c.y0.as<double>(), partials, &np, ss);
        k::reduce_sum(partials, np, c.dsum.as<double>(), ss);
        HIPCHECK(hipMemcpyAsync(hd, c.dsum.p, 8, hipMemcpyDeviceToHost, ss));
        HIPCHECK(hipStreamSynchronize(ss));
        r_sum = hd[0];
    }

    int32_t sweeps = 0;
    double sweep_ms = 0.0;
    int32_t timed_sweeps = 0;
    EventPair ev;
    int32_t push_scans = 0;
    if (opt.global_rule == PPR_GLOBAL_EPOCHS && r_sum > lambda) {
        // ---- global phase, Algorithm 3's epochs: rmax_i = lambda^(i/8) / m,
        // scans while r_sum > m rmax_i (as printed); each scan pushes at once the
        // nodes active at its start.  A scan with no active node ends the epoch;
        // scans at rmax_8 continue while rounding leaves r_sum above lambda.
        // A scan runs in push form over the listed active set when that set's
        // out-edge volume is small (scan_form), else in pull form over all
        // in-edges.  After a push scan the next active set is the list of
        // nodes its atomic adds carried across the threshold (every other
        // node is below it and unchanged); a new epoch lowers the threshold,
        // and a pull scan leaves no list, so the set is then listed afresh:
        // under PPR_SCAN_AUTO only when the last pull scan's volume was within
        // twice the push bound (sizing the set costs a pass over all nodes and
        // a host round trip), and counted before it is listed.
        ev.start(ss);
        double* y = c.y0.as<double>();
        bool capped = false;
        int32_t* F = c.F0.as<int32_t>();
        int32_t* Fn = c.F1.as<int32_t>();
        const auto push_pays = [&](int64_t v) {
            return opt.scan_form == PPR_SCAN_PUSH ||
                   (opt.scan_form == PPR_SCAN_AUTO && opt.switch_param * (double)v <= (double)g.m);
        };
        for (int i = 1; i <= 9 && !capped; ++i) {
            const bool last = (i == 9);
            const double rmax_i = std::pow(lambda, (double)(last ? 8 : i) / 8.0) / (double)g.m;
            bool listed = false;         // F holds exactly the nodes active w.r.t. rmax_i
            int64_t nfa = 0, vola = 0;
            double last_pull = -1.0;     // volume of the last pull scan of this epoch
            for (;;) {
                if (last ? !(r_sum > lambda) : !(r_sum > (double)g.m * rmax_i)) break;
                if (sweeps >= opt.max_sweeps) {
                    capped = true;
                    break;
                }
                if (opt.scan_form == PPR_SCAN_PUSH && !listed) {
                    active_set(g, c, rmax_i, F, &nfa, &vola);
                    if (nfa == 0) break;      // nothing is active: the scan would move nothing
                    listed = true;
                } else if (opt.scan_form == PPR_SCAN_AUTO && !listed &&
                           (last_pull < 0.0 || push_pays((int64_t)(last_pull / 2.0)))) {
                    active_set(g, c, rmax_i, nullptr, &nfa, &vola);
                    if (nfa == 0) break;
                    if (push_pays(vola)) {
                        active_set(g, c, rmax_i, F, &nfa, &vola);
                        listed = true;
                    }
                }
                if (listed && push_pays(vola)) {
                    if (nfa == 0) break;
                    int np = 0;
                    k::frontier_snapshot(F, (int32_t)nfa, deg, alpha, r, pi, c.X.as<double>(),
                                         c.degF.as<int64_t>(), partials, &np, ss);
                    k::exclusive_scan_i64(c.degF.as<int64_t>(), c.off.as<int64_t>(), nfa, c.scan_tmp.p, ss);
                    HIPCHECK(hipMemsetAsync(c.ctr.p, 0, 16, ss));
                    k::frontier_push(F, c.off.as<int64_t>(), (int32_t)nfa, vola, g.row_ptr.as<int64_t>(),
                                     g.col.as<int32_t>(), deg, c.X.as<double>(), rmax_i, r, Fn,
                                     c.ctr.as<int64_t>(), ss);
                    // the exact residue sum after the scan
                    k::prep_y(r, deg, alpha, g.n, y, partials, &np, ss);
                    k::reduce_sum(partials, np, c.dsum.as<double>(), ss);
                    HIPCHECK(hipMemcpyAsync(hctr, c.ctr.p, 16, hipMemcpyDeviceToHost, ss));
                    HIPCHECK(hipMemcpyAsync(hd + 2, c.dsum.p, 8, hipMemcpyDeviceToHost, ss));
                    HIPCHECK(hipStreamSynchronize(ss));
                    ++sweeps;
                    ++push_scans;
                    edge_pushes += vola;
                    r_sum = hd[2];
                    nfa = hctr[0];
                    vola = hctr[1];
                    std::swap(F, Fn);
                    if (trace) trace->note(1, sweeps, edge_pushes, r_sum);
                    continue;
                }
                listed = false;                // a pull scan leaves no list
                int np = 0;
                k::threshold_snapshot(deg, g.n, alpha, rmax_i, r, pi, y, partials, &np, ss);
                k::reduce_sum(partials, np, c.dsum.as<double>() + 1, ss);
                k::sweep_f64(g, sch, k::SW_ACCUM, alpha, y, nullptr, pi, r, r, partials, ss, acc);
                k::reduce_sum(partials, k::sweep_parts(g, sch, acc), c.dsum.as<double>(), ss);
                HIPCHECK(hipMemcpyAsync(hd, c.dsum.p, 16, hipMemcpyDeviceToHost, ss));
                HIPCHECK(hipStreamSynchronize(ss));
                if (hd[1] == 0.0) break;      // nothing was active: the scan moved nothing
                ++sweeps;
                last_pull = hd[1];
                edge_pushes += (int64_t)hd[1];
                r_sum = hd[0];
                if (trace) trace->note(1, sweeps, edge_pushes, r_sum);
            }
        }
        ev.stop(ss);
        HIPCHECK(hipStreamSynchronize(ss));
        sweep_ms = ev.elapsed_ms();
        timed_sweeps = sweeps;
    } else if (r_sum > lambda) {
        // ---- global phase: threshold-0 sweeps contract r_sum by exactly (1 - alpha)
        ev.start(ss);
        int32_t K = 0;
        for (double x = r_sum; x > lambda && K < opt.max_sweeps; x *= (1.0 - alpha)) ++K;
        double* y0 = c.y0.as<double>();
        double* y1 = c.y1.as<double>();
        auto sweep = [&](int flags, const double* yi, double* yo) {
            k::sweep_f64(g, sch, flags, alpha, yi, yo, pi, r, r, partials, ss, acc);
        };
        const double* yc = y0;   // buffer holding the current y
        double* yn = y1;
        auto advance = [&](int flags) {
            sweep(flags, yc, yn);
            double* t = const_cast<double*>(yc);
            yc = yn;
            yn = t;
        };
        if (trace) {
            // the same flag sequence one sweep at a time, each followed by its
            // exact r_sum (the sweep's partials hold the new residues' sums)
            for (int32_t j = 1; j <= K; ++j) {
                advance((j == 1 ? k::SW_ENTRY : 0) | (j == K ? k::SW_WRITE_R : k::SW_FOLD));
                k::reduce_sum(partials, k::sweep_parts(g, sch, acc), c.dsum.as<double>(), ss);
                HIPCHECK(hipMemcpyAsync(hd, c.dsum.p, 8, hipMemcpyDeviceToHost, ss));
                HIPCHECK(hipStreamSynchronize(ss));
                trace->note(1, j, edge_pushes + (int64_t)j * g.m, hd[0]);
            }
        } else if (K == 1) {
            advance(k::SW_ENTRY | k::SW_WRITE_R);
        } else {
            advance(k::SW_ENTRY | k::SW_FOLD);            // now yc == y1
            int32_t mid = K - 2;
            int32_t chunks = mid / (2 * kChunkPairs);
            if (chunks > 0) {                              // an even number of sweeps: yc stays y1
                ensure_chunk(g, c, sch, alpha);
                for (int32_t i = 0; i < chunks; ++i) HIPCHECK(hipGraphLaunch(c.chunk_exec, ss));
            }
            for (int32_t i = chunks * 2 * kChunkPairs; i < mid; ++i) advance(k::SW_FOLD);
            advance(k::SW_WRITE_R);
        }
        sweeps = K;
        ev.stop(ss);
        k::reduce_sum(partials, k::sweep_parts(g, sch, acc), c.dsum.as<double>(), ss);
        HIPCHECK(hipMemcpyAsync(hd, c.dsum.p, 8, hipMemcpyDeviceToHost, ss));
        HIPCHECK(hipStreamSynchronize(ss));
        r_sum = hd[0];
        sweep_ms = ev.elapsed_ms();
        timed_sweeps = K;
        // rounding can leave r_sum a hair above lambda: one more plain sweep each time
        while (r_sum > lambda && sweeps < opt.max_sweeps) {
            advance(k::SW_ENTRY | k::SW_WRITE_R);
            ++sweeps;
            k::reduce_sum(partials, k::sweep_parts(g, sch, acc), c.dsum.as<double>(), ss);
            HIPCHECK(hipMemcpyAsync(hd, c.dsum.p, 8, hipMemcpyDeviceToHost, ss));
            HIPCHECK(hipStreamSynchronize(ss));
            r_sum = hd[0];
            if (trace) trace->note(1, sweeps, edge_pushes + (int64_t)sweeps * g.m, r_sum);
        }
    }
    if (opt.global_rule != PPR_GLOBAL_EPOCHS) edge_pushes += (int64_t)sweeps * g.m;

    // ---- optional certificate
    double cert = -1.0;
    if (opt.certify) {
        k::cert_f64(g, sch, alpha, s, pi, c.y0.as<double>(), nullptr, partials, ss);
        k::reduce_sum(partials, k::sweep_parts(sch), c.dsum.as<double>(), ss);
        HIPCHECK(hipMemcpyAsync(hd + 4, c.dsum.p, 8, hipMemcpyDeviceToHost, ss));
    }
    // ---- output
    HIPCHECK(hipMemcpyAsync(pi_out, pi, 8 * (size_t)g.n, hipMemcpyDefault, ss));
    if (r_out) HIPCHECK(hipMemcpyAsync(r_out, r, 8 * (size_t)g.n, hipMemcpyDefault, ss));
    HIPCHECK(hipStreamSynchronize(ss));
    if (opt.certify) cert = hd[4];
    if (st) {
        st->sweep_ms = sweep_ms;
        st->sweep_launches = timed_sweeps;
        st->batch_cols = 1;
        st->sweep_chunks = 1;
        st->sor_omega = 1.0;
        st->residue_format = PPR_RESIDUE_F32;
        st->push_scans = push_scans;
        st->sweep_tile_bytes = 0;
        st->refresh_ms = 0.0;
        st->refresh_launches = 0;
        st->reserved = 0;
        st->local_levels = levels;
        st->sweeps = sweeps;
        st->refreshes = 0;
        st->source = s;
        st->edge_pushes = edge_pushes;
        st->r_sum = r_sum;
        st->cert_l1 = cert;
        st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (r_sum > lambda) fail(PPR_ERR_NOT_CONVERGED, "max_sweeps reached before r_sum <= lambda");
}

}  // namespace ppr
