// Host side of the batched mixed-precision path: the block engine (one n x B
// block of independent query slots on one graph), the synchronous batch
// driver (ppr_query_batch with PPR_MIXED), the width autotuner, and the
// serving mechanism (admit / step / poll / retire on a block).
//
// A slot's life: FREE -> PENDING (admitted; local phase not run) -> RUNNING
// (stages of sweeps, each ended by an FP64 refresh of that slot) -> DONE (its
// FP64 certificate is <= its lambda; its reserve no longer changes) ->
// retired (exported) -> FREE.  A slot's schedule (local levels, stage
// lengths, refresh points) depends on its own source, alpha and lambda only,
// so a query's result is the same whichever other slots share the block, up
// to the FP32 summation order of the block width.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "mixed_internal.h"

namespace ppr {

// ======================================================================== contexts

void MixedCtx::drop_chunks() {
    for (auto& ch : chunk) {
        if (ch) (void)hipGraphExecDestroy(ch);
        ch = nullptr;
    }
}

MixedCtx::~MixedCtx() {
    drop_chunks();
    if (own) (void)hipStreamDestroy(own);
}

void MixedCtxDeleter::operator()(MixedCtx* c) const { delete c; }

namespace {
int ilog2(int x) {
    int s = 0;
    while ((1 << s) < x) ++s;
    return s;
}

// Batched switch rule.  Edge rule: a column keeps pushing locally while
// switch_param * kBatchRef * vol_b <= m, so one level of a block of kBatchRef
// columns moves at most about m / switch_param edges, the single-query bound.
// It does not depend on the block width, so a column's schedule is the same
// whichever block it runs in.
constexpr double kBatchRef = 32.0;

bool continue_local(const ppr_options& opt, int64_t nf, int64_t vol, int32_t n, int64_t m) {
    if (opt.switch_rule == PPR_SWITCH_NODES) return 4 * nf <= (int64_t)n;
    return opt.switch_param * kBatchRef * (double)vol <= (double)m;
}

// Row chunks per sweep: about 2M in-edges per chunk keep each launch filling
// the device; at most 8 (beyond that the launches cost more than the few
// sweeps they save).
int sweep_chunks(const Graph& g, const ppr_options& opt) {
    if (opt.sweep_chunks > 0) return opt.sweep_chunks;
    return (int)std::max<int64_t>(1, std::min<int64_t>(8, g.m >> 21));
}

// LDS stage (row tile) of the sweep blocks at width Bw: the autotuner's
// choice for this graph and width, else the default.
int sweep_tile(const Graph& g, int Bw, bool bf16) {
    const int t = g.tuned_tile[bf16 ? 1 : 0][ilog2(Bw) & 7].load();
    return t > 0 ? t : mk::kLdsBytes;
}

// Automatic over-relaxation factor of block Gauss-Seidel sweeps.  On
// Chung-Lu power-law graphs (n = 4M, m = 70M, 8 chunks, lambda = 1e-8) the
// sweeps per query go 46.6 -> 34.5 -> 31.6 -> 38.9 -> 52.0 for omega = 1,
// 1.15, 1.2, 1.25, 1.3; beyond the optimum the residual oscillates.  Graphs
// where it does not pay (a directed cycle) fall back to 1 after one stage.
constexpr double kAutoOmega = 1.2;

// Residue storage of a block of Bw columns under these options.  bf16 pays
// where a residue row spans several cache lines: on the 4M/70M graph at
// lambda = 1e-8, B = 8: 147 against 164 queries/s in FP32, B = 32: 420
// against 402, B = 128: 585 against 454.
bool residues_bf16(const ppr_options& o, int Bw) {
    return o.residue_format == PPR_RESIDUE_BF16 || (o.residue_format == PPR_RESIDUE_AUTO && Bw >= 32);
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kChunkSweeps = 16;
enum SlotState : int { FREE = 0, PENDING = 1, RUNNING = 2, DONE = 3 };
}  // namespace

int64_t frontier_capacity(int32_t n, int64_t m, const ppr_options& opt, int Bw) {
    // A level runs only if the column's next frontier (at most vol_b entries,
    // at most n) fits its share of the capacity.  Under the edge rule a level
    // runs only while switch_param * kBatchRef * vol_b <= m, so that share
    // never stops a level the rule allows; it depends on (n, m, options) only,
    // so the footprint is known before the graph exists.
    int64_t per_col = n;
    if (opt.switch_rule == PPR_SWITCH_EDGES && opt.switch_param > 0)
        per_col = std::min<int64_t>(per_col, (int64_t)((double)m / (opt.switch_param * kBatchRef)) + 1);
    return std::max<int64_t>(per_col, 1) * Bw;
}

size_t mixed_footprint(int32_t n, int64_t m, int Bw, int64_t fcap, bool bf16) {
    const size_t nb = (size_t)n * (size_t)Bw;
    // long-row pieces: each holds piece_cap = kLongRounds L / (4 Bw) in-edges
    // of a row with more than piece_cap (L the sweep stage, at least
    // kMinTile), so there are fewer than 2 m / piece_cap
    const size_t piece_cap = (size_t)mk::kLongRounds * mk::kMinTile / (4 * (size_t)Bw);
    const size_t pieces = 2 * (size_t)m / piece_cap + 1;
    return 16 * nb                       // FP64 local-phase scratch
           + (bf16 ? 24 : 28) * nb       // Y0, Y1 (4 or 2 bytes), S, AS (8), T (4)
           + 4 * (size_t)Bw * pieces     // partial sums of the pieces
           + 8 * (size_t)mk::kGridRed * Bw   // per-block column sums of the refresh
           + 40 * (size_t)fcap + 4 * (size_t)n + ((size_t)1 << 20);
}

MixedCtxPtr mixed_acquire(Graph& g, int Bw, int64_t fcap, bool bf16) {
    {
        std::lock_guard<std::mutex> lk(g.pool_mu);
        for (auto it = g.mixed_pool.begin(); it != g.mixed_pool.end(); ++it) {
            if ((*it)->Bw == Bw && (*it)->fcap >= fcap && (*it)->bf16 == bf16) {
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
    c->bf16 = bf16;
    HIPCHECK(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
    c->stream = c->own;
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
    c->Y01.alloc(2 * (bf16 ? 2 : 4) * nb);
    c->Y0.view(c->Y01.p, (bf16 ? 2 : 4) * nb);
    c->Y1.view(static_cast<char*>(c->Y01.p) + (bf16 ? 2 : 4) * nb, (bf16 ? 2 : 4) * nb);
    c->S.alloc(8 * nb);
    c->AS.alloc(8 * nb);
    c->T.alloc(4 * nb);
    for (DevBuf* b : {&c->Y0, &c->Y1, &c->S, &c->AS, &c->T}) HIPCHECK(hipMemsetAsync(b->p, 0, b->bytes, c->stream));
    c->scale.alloc(4 * n);
    c->partials.alloc(8 * (size_t)mk::kGridRed * Bw);
    c->colsum.alloc(8 * (size_t)Bw);
    c->ctr.alloc(8 * (1 + 2 * (size_t)Bw));
    c->taken.alloc(8 * (size_t)Bw);
    c->active.alloc((size_t)Bw);
    for (DevBuf* b : {&c->src, &c->kb, &c->entry, &c->rmask, &c->cmask}) b->alloc(4 * (size_t)Bw);
    c->rmaxb.alloc(8 * (size_t)Bw);
    c->omega.alloc(4 * (size_t)Bw);
    c->acoef.alloc(32 * (size_t)Bw);
    c->afac.alloc(4 * (size_t)Bw);
    {
        std::vector<float> ones(Bw, 1.0f);
        HIPCHECK(hipMemcpyAsync(c->omega.p, ones.data(), 4 * (size_t)Bw, hipMemcpyHostToDevice, c->stream));
        HIPCHECK(hipStreamSynchronize(c->stream));
    }
    std::vector<int32_t> neg(Bw, -1), zero(Bw, 0);
    HIPCHECK(hipMemcpyAsync(c->src.p, neg.data(), 4 * (size_t)Bw, hipMemcpyHostToDevice, c->stream));
    for (DevBuf* b : {&c->kb, &c->entry, &c->rmask, &c->cmask})
        HIPCHECK(hipMemcpyAsync(b->p, zero.data(), 4 * (size_t)Bw, hipMemcpyHostToDevice, c->stream));
    c->step.alloc(64);
    c->host.alloc(64 + 48 * (size_t)Bw);
    c->ycur = c->Y0.p;
    HIPCHECK(hipStreamSynchronize(c->stream));
    return c;
}

void mixed_release(Graph& g, MixedCtxPtr c) {
    std::lock_guard<std::mutex> lk(g.pool_mu);
    g.mixed_pool.push_back(std::move(c));
}

// ======================================================================== block engine

struct Block {
    struct Slot {
        int state = FREE;
        int32_t src = -1;
        double alpha = 0.0;          // the query's stop probability
        double lambda = 0.0;
        double err = 0.0;            // bound on ||pi_hat - pi_s||_1 (exact right after a refresh)
        int32_t stage_left = 0;      // sweeps left in the current stage
        bool entry = false;          // the residue is fresh: the next sweep folds its alpha-part
                                     // and pulls it along every in-edge
        bool t_moved = false;        // the last refresh moved T into S: the entry sweep restarts T
        bool s_unset = false;        // converted, not refreshed yet: S and AS hold another query's values
        bool refreshing = false;     // in the refresh whose result is in flight
        bool failed = false;         // reached max_sweeps with a certificate above lambda
        double cert = -1.0;
        double omega = 1.0;          // over-relaxation factor of this column's sweeps
        double rho = 0.0;            // per-sweep contraction of err the stage lengths assume
        double stage_err0 = 0.0;     // err when the current stage started
        int32_t stage_sweeps = 0;    // sweeps run in the current stage
        int32_t levels = 0, sweeps = 0, refreshes = 0;
        int64_t edges = 0;
        double t_admit = 0.0;
    };

    Graph& g;
    MixedCtxPtr c;
    int Bw;
    double alpha;                    // reference alpha: the scale table's, and the default of a slot
    ppr_options opt;
    std::vector<Slot> slots;
    bool scratch_dirty = false;      // the FP64 scratch holds a local phase's values
    bool inflight = false;           // results of enqueued work are on their way
    hipEvent_t ev_ready = nullptr;
    EventPair ev_sweep;
    bool sweep_timed = false;        // ev_sweep brackets the last launch sequence
    int32_t seq_sweeps = 0;
    double sweep_ms = 0.0;           // accumulated GPU time of the sweeps
    int32_t sweep_launches = 0;
    EventPair ev_refresh;
    bool refresh_timed = false;      // ev_refresh brackets the last refresh pass
    double refresh_ms = 0.0;         // accumulated GPU time of the refresh passes
    int32_t refresh_launches = 0;
    double refresh_factor;           // drop of err that ends a stage

    Block(Graph& gg, int width, double a, const ppr_options& o) : g(gg), Bw(width), alpha(a), opt(o) {
        // a bf16 residue carries ~2^-9 relative rounding per push, so a stage
        // stalls near 1e-2 of the residual it started from (1e-6 with FP32,
        // where the first stage also carries the local phase's reserve in the
        // FP32 accumulator).  Fastest factors on the 4M/70M graph at B = 128:
        // bf16 30 / 40 / 50 / 70: 606 / 660 / 635 / 612 queries/s; FP32
        // 300 / 1e3 / 2e3 / 1e4: 463 / 491 / 468 / 415
        refresh_factor = opt.refresh_factor > 0.0 ? opt.refresh_factor
                                                  : (residues_bf16(opt, Bw) ? 40.0 : 1e3);
        if (Bw < 4 || Bw > 128 || (Bw & (Bw - 1))) fail(PPR_ERR_ARG, "block width must be a power of two in [4, 128]");
        if (opt.residue_format == PPR_RESIDUE_BF16 && Bw < 8)
            fail(PPR_ERR_ARG, "bf16 residues need a block of at least 8 columns");
        int tile = sweep_tile(g, Bw, residues_bf16(opt, Bw));
        if (opt.sweep_tile != 0) {
            bool known = false;
            for (int t : mk::kTiles) known |= (t == opt.sweep_tile);
            if (!known) fail(PPR_ERR_ARG, "sweep_tile must be 0, 12288, 16384 or 24576");
            tile = opt.sweep_tile;
        }
        c = mixed_acquire(g, Bw, frontier_capacity(g.n, g.m, opt, Bw), residues_bf16(opt, Bw));
        // the caller's stream, if it gave one, carries every launch and copy of
        // this block; HIP graphs are still captured on the context's own stream
        if (opt.use_stream) c->stream = static_cast<hipStream_t>(opt.stream);
        const int chunks = sweep_chunks(g, opt);
        if (c->chunks != chunks) {
            c->drop_chunks();
            c->chunks = chunks;
        }
        if (c->tile != tile) {
            c->drop_chunks();
            c->tile = tile;
        }
        mk::prepare(*c, g);
        c->sor = false;              // set per launch sequence by step()
        if (c->af) {                 // a pooled context may carry another block's choice
            c->drop_chunks();
            c->af = false;
        }
        slots.resize(Bw);
        HIPCHECK(hipEventCreateWithFlags(&ev_ready, hipEventDisableTiming));
        if (c->alpha != alpha) {
            mk::set_scale(g, *c, alpha);
            c->drop_chunks();
            c->alpha = alpha;
        }
        upload_alphas();
    }

    ~Block() {
        if (c) release();
        if (ev_ready) (void)hipEventDestroy(ev_ready);
    }

    // Hand the device state back to the graph's pool, or destroy it when the
    // FP64 scratch may hold values (an interrupted local phase).  Stale values
    // in the other arrays are harmless: a column is written by its conversion
    // before it is used, and unused columns have zero budgets.
    void release() {
        if (!c) return;
        hipError_t e = hipStreamSynchronize(c->stream);
        c->stream = c->own;
        if (!scratch_dirty && e == hipSuccess) mixed_release(g, std::move(c));
        else c.reset();
    }

    int admit(int32_t s, double a, double lambda) {
        for (int b = 0; b < Bw; ++b) {
            if (slots[b].state != FREE) continue;
            Slot& sl = slots[b];
            sl = Slot();
            sl.state = PENDING;
            sl.src = s;
            sl.alpha = a;
            sl.lambda = lambda;
            sl.t_admit = now_ms();
            return b;
        }
        return -1;
    }

    // Per-column alpha coefficients (acoef, afac) of every slot; a free slot
    // takes the reference alpha.  Running columns keep their values.
    void upload_alphas() {
        std::vector<double> co(4 * (size_t)Bw);
        std::vector<float> fac(Bw);
        for (int b = 0; b < Bw; ++b) {
            const double a = slots[b].state == FREE ? alpha : slots[b].alpha;
            co[b] = a;
            co[Bw + b] = 1.0 - a;
            co[2 * Bw + b] = 1.0 / (1.0 - a);
            co[3 * Bw + b] = a / (1.0 - a);
            fac[b] = a == alpha ? 1.0f : (float)((1.0 - a) / (1.0 - alpha));
        }
        HIPCHECK(hipMemcpyAsync(c->acoef.p, co.data(), 32 * (size_t)Bw, hipMemcpyHostToDevice, c->stream));
        HIPCHECK(hipMemcpyAsync(c->afac.p, fac.data(), 4 * (size_t)Bw, hipMemcpyHostToDevice, c->stream));
        // the host vectors die here: wait for the copies
        HIPCHECK(hipStreamSynchronize(c->stream));
    }

    // Sweeps of one stage: until err has fallen by refresh_factor, or to
    // 0.8 lambda (the margin covers the FP32 rounding a stage adds and a rate
    // estimate slightly too optimistic; a stage that still ends above lambda
    // is followed by another).
    int32_t stage_length(const Slot& sl) const {
        double target = std::max(sl.err / refresh_factor, 0.8 * sl.lambda);
        int32_t k = 0;
        for (double x = sl.err; x > target && k < (1 << 20); x *= sl.rho) ++k;
        return std::max<int32_t>(k, 1);
    }

    // A stage starts (after the conversion or a refresh) with err known exactly.
    void start_stage(Slot& sl) {
        sl.stage_err0 = sl.err;
        sl.stage_sweeps = 0;
        sl.stage_left = stage_length(sl);
    }

    // Contraction the first stage assumes: exactly 1 - alpha for Jacobi
    // sweeps; for block Gauss-Seidel sweeps a prior of (1 - alpha)^1.4 (on
    // power-law graphs they contract like (1 - alpha)^1.5 .. (1 - alpha)^1.7);
    // a stage that falls short is simply followed by another.
    double first_rate(const Slot& sl) const {
        if (c->chunks <= 1) return 1.0 - sl.alpha;
        return std::pow(1.0 - sl.alpha, sl.omega > 1.0 ? 1.8 : 1.4);
    }

    // Contraction for the next stage's length.  A Jacobi sweep (one chunk)
    // contracts the residue mass by exactly 1 - alpha (Eq. 6, Lemma 1).  In
    // block Gauss-Seidel order every pending unit of mass is pushed at least
    // once per sweep, so 1 - alpha still bounds the contraction; the measured
    // rate of the stage just ended (rounded towards 1 - alpha) sets the next
    // stage's length, and a stage that falls short is followed by another.
    //
    // Over-relaxation (omega > 1) is kept only while it pays: a stage whose
    // measured rate is no better than (1 - alpha)^1.4, the rate plain block
    // Gauss-Seidel order starts from, switches the column back to omega = 1
    // (over-relaxed pushes can grow the residue on graphs with periodic
    // structure; the refresh that ends the stage measures it exactly).
    void update_rate(Slot& sl, double cert) const {
        if (c->chunks <= 1 || sl.stage_sweeps <= 0 || !(sl.stage_err0 > 0.0) || !(cert > 0.0)) return;
        double r = std::pow(cert / sl.stage_err0, 1.0 / sl.stage_sweeps);
        if (sl.omega > 1.0 && !(r < std::pow(1.0 - sl.alpha, 1.4))) {
            sl.omega = 1.0;
            sl.rho = first_rate(sl);
            return;
        }
        r = std::pow(r, 0.95);
        r = std::ceil(r * 1024.0) / 1024.0;
        sl.rho = std::min(1.0 - sl.alpha, std::max(0.05, r));
    }

    void upload_i32(DevBuf& d, const std::vector<int32_t>& h) {
        HIPCHECK(hipMemcpyAsync(d.p, h.data(), 4 * (size_t)Bw, hipMemcpyHostToDevice, c->stream));
    }

    // A launch sequence starts at step 0; its step `last` adds its output to T
    // whatever the step's parity.
    void set_steps(int32_t last) {
        const int32_t h[2] = {0, last};
        HIPCHECK(hipMemcpyAsync(c->step.p, h, sizeof(h), hipMemcpyHostToDevice, c->stream));
    }

    // Local phase (FP64) of every PENDING slot, all in one frontier list, and
    // the conversion of those columns into the block.
    void run_local_phase() {
        std::vector<int> cols;
        for (int b = 0; b < Bw; ++b)
            if (slots[b].state == PENDING) cols.push_back(b);
        if (cols.empty()) return;
        hipStream_t ss = c->stream;
        std::vector<int32_t> hsrc(Bw), hc(Bw, 0);
        std::vector<double> hrmax(Bw, 0.0);
        for (int b = 0; b < Bw; ++b) {
            hsrc[b] = (slots[b].state == FREE) ? -1 : slots[b].src;
            hrmax[b] = slots[b].lambda / (double)g.m;     // rmax = lambda / m (Algorithm 3)
        }
        for (int b : cols) hc[b] = 1;
        upload_i32(c->src, hsrc);
        upload_i32(c->cmask, hc);
        upload_alphas();
        HIPCHECK(hipMemcpyAsync(c->rmaxb.p, hrmax.data(), 8 * (size_t)Bw, hipMemcpyHostToDevice, ss));
        scratch_dirty = true;
        mk::init_sources(*c);
        std::vector<int64_t> nf_b(Bw, 0), vol_b(Bw, 0);
        std::vector<double> rsum_b(Bw, 0.0);
        std::vector<int64_t> hF;
        for (int b : cols) {
            nf_b[b] = 1;
            vol_b[b] = g.h_deg[slots[b].src];
            rsum_b[b] = 1.0;
            hF.push_back(((int64_t)slots[b].src << c->shift) + b);
        }
        HIPCHECK(hipMemcpyAsync(c->F0.p, hF.data(), 8 * hF.size(), hipMemcpyHostToDevice, ss));
        int64_t nf = (int64_t)hF.size();
        int64_t* F = c->F0.as<int64_t>();
        int64_t* Fn = c->F1.as<int64_t>();
        std::vector<uint8_t> act(Bw, 0);
        char* hb = c->host.as<char>();
        const size_t nctr = 1 + 2 * (size_t)Bw;
        for (;;) {
            int64_t vol = 0;
            bool any = false;
            for (int b = 0; b < Bw; ++b) {
                const Slot& sl = slots[b];
                // a column's next frontier holds at most vol_b entries: it must
                // fit the per-column share of the frontier capacity
                act[b] = (sl.state == PENDING && nf_b[b] > 0 && rsum_b[b] > sl.lambda &&
                          continue_local(opt, nf_b[b], vol_b[b], g.n, g.m) && vol_b[b] <= c->fcap / Bw) ? 1 : 0;
                if (act[b]) {
                    vol += vol_b[b];
                    any = true;
                }
            }
            if (!any || nf == 0) break;
            HIPCHECK(hipMemcpyAsync(c->active.p, act.data(), (size_t)Bw, hipMemcpyHostToDevice, ss));
            HIPCHECK(hipMemsetAsync(c->ctr.p, 0, 8 * nctr, ss));
            HIPCHECK(hipMemsetAsync(c->taken.p, 0, 8 * (size_t)Bw, ss));
            mk::snapshot(*c, g, F, nf);
            k::exclusive_scan_i64(c->degF.as<int64_t>(), c->off.as<int64_t>(), nf, c->scan_tmp.p, ss);
            mk::push(*c, g, F, nf, vol, Fn);
            HIPCHECK(hipMemcpyAsync(hb, c->ctr.p, 8 * nctr, hipMemcpyDeviceToHost, ss));
            HIPCHECK(hipMemcpyAsync(hb + 8 * nctr, c->taken.p, 8 * (size_t)Bw, hipMemcpyDeviceToHost, ss));
            HIPCHECK(hipStreamSynchronize(ss));
            const uint64_t* hcnt = reinterpret_cast<const uint64_t*>(hb);
            const double* ht = reinterpret_cast<const double*>(hb + 8 * nctr);
            nf = (int64_t)hcnt[0];
            if (nf > c->fcap) fail(PPR_ERR_OOM, "frontier capacity exceeded");
            for (int b = 0; b < Bw; ++b) {
                if (!act[b]) {
                    nf_b[b] = 0;   // this column's local phase is over
                    continue;
                }
                slots[b].edges += vol_b[b];
                slots[b].levels += 1;
                rsum_b[b] -= ht[b];
                nf_b[b] = (int64_t)hcnt[1 + b];
                vol_b[b] = (int64_t)hcnt[1 + Bw + b];
            }
            std::swap(F, Fn);
        }
        // FP64 -> block for these columns (alpha-part of the residue folded in)
        mk::convert(*c, g);
        HIPCHECK(hipMemcpyAsync(hb, c->colsum.p, 8 * (size_t)Bw, hipMemcpyDeviceToHost, ss));
        HIPCHECK(hipStreamSynchronize(ss));
        scratch_dirty = false;
        const double* hcol = reinterpret_cast<const double*>(hb);
        for (int b : cols) {
            Slot& sl = slots[b];
            sl.state = RUNNING;
            sl.err = (1.0 - sl.alpha) * hcol[b];
            sl.entry = true;
            sl.t_moved = false;          // T holds the local phase's reserve
            sl.s_unset = true;           // the first refresh takes S = AS = 0 (rmask 2)
            const double w = opt.sor_omega == 0.0 ? kAutoOmega : opt.sor_omega;
            sl.omega = (c->chunks > 1 && w > 1.0) ? w : 1.0;
            sl.rho = first_rate(sl);
            start_stage(sl);
        }
    }

    // Capture on the context's own stream (never the caller's, which may be
    // the null stream); the work stream only launches the instantiated graph.
    void capture_chunk() {
        hipStream_t ss = c->own;
        hipGraph_t graph = nullptr;
        const hipStream_t work = c->stream;
        c->stream = ss;
        HIPCHECK(hipStreamBeginCapture(ss, hipStreamCaptureModeThreadLocal));
        const void* a = c->Y1.p;
        void* bb = c->Y0.p;
        try {
            for (int i = 0; i < kChunkSweeps; ++i) {
                mk::sweep(*c, g, a, bb);
                void* t = const_cast<void*>(a);
                a = bb;
                bb = t;
            }
        } catch (...) {
            (void)hipStreamEndCapture(ss, &graph);
            c->stream = work;
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        c->stream = work;
        HIPCHECK(hipStreamEndCapture(ss, &graph));
        hipError_t e = hipGraphInstantiate(&c->chunk[c->sor ? 1 : 0], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHECK(e);
    }

    void* other(const void* y) const { return y == c->Y0.p ? c->Y1.p : c->Y0.p; }

    // Collect the results of the enqueued work (blocking when wait).  Returns
    // false if they are not ready yet.
    bool collect(bool wait) {
        if (!inflight) return true;
        if (!wait) {
            hipError_t q = hipEventQuery(ev_ready);
            if (q == hipErrorNotReady) {
                (void)hipGetLastError();
                return false;
            }
            HIPCHECK(q);
        } else {
            HIPCHECK(hipEventSynchronize(ev_ready));
        }
        if (sweep_timed) {
            sweep_ms += ev_sweep.elapsed_ms();
            sweep_launches += seq_sweeps;
            sweep_timed = false;
        }
        if (refresh_timed) {
            refresh_ms += ev_refresh.elapsed_ms();
            refresh_launches += 1;
            refresh_timed = false;
        }
        const double* hcol = c->host.as<double>();
        for (int b = 0; b < Bw; ++b) {
            Slot& sl = slots[b];
            if (!sl.refreshing) continue;
            sl.refreshing = false;
            sl.refreshes += 1;
            sl.cert = hcol[b];
            update_rate(sl, hcol[b]);
            sl.err = hcol[b];
            if (hcol[b] <= sl.lambda) {
                sl.state = DONE;
            } else if (out_of_sweeps(sl)) {
                sl.state = DONE;
                sl.failed = true;
            } else {
                sl.entry = true;
                start_stage(sl);
            }
        }
        inflight = false;
        return true;
    }

    // per-query cap on global sweeps (opt.max_sweeps)
    int32_t sweeps_left(const Slot& sl) const { return std::max(0, opt.max_sweeps - sl.sweeps); }
    bool out_of_sweeps(const Slot& sl) const { return sl.sweeps >= opt.max_sweeps; }

    // Enqueue up to max_sweeps sweeps and the refreshes of the slots whose
    // stage ends; their results are taken by collect().
    void step(int32_t max_sweeps) {
        collect(true);
        run_local_phase();
        hipStream_t ss = c->stream;
        int32_t K = 0;
        for (const Slot& sl : slots)
            if (sl.state == RUNNING) K = std::max(K, std::min(sl.stage_left, sweeps_left(sl)));
        K = std::min(K, max_sweeps);
        if (K > 0) {
            std::vector<int32_t> hkb(Bw, 0), hen(Bw, 0);
            for (int b = 0; b < Bw; ++b) {
                Slot& sl = slots[b];
                if (sl.state != RUNNING) continue;
                hkb[b] = std::min(std::min(sl.stage_left, sweeps_left(sl)), K);
                hen[b] = (sl.entry && hkb[b] > 0) ? (sl.t_moved ? 2 : 1) : 0;
            }
            upload_i32(c->kb, hkb);
            upload_i32(c->entry, hen);
            // over-relaxation factors of this sequence (1 for plain columns)
            std::vector<float> hom(Bw, 1.0f);
            bool any_sor = false;
            for (int b = 0; b < Bw; ++b)
                if (slots[b].state == RUNNING && slots[b].omega != 1.0) {
                    hom[b] = (float)slots[b].omega;
                    any_sor = true;
                }
            if (any_sor) HIPCHECK(hipMemcpyAsync(c->omega.p, hom.data(), 4 * (size_t)Bw, hipMemcpyHostToDevice, ss));
            c->sor = any_sor;
            // per-column alpha factors only while a running slot has another alpha
            // than the block's (the captured chunks hold the choice)
            bool any_af = false;
            for (const Slot& sl : slots) any_af |= (sl.state == RUNNING && sl.alpha != alpha);
            if (any_af != c->af) {
                c->drop_chunks();
                c->af = any_af;
            }
            set_steps(K - 1);
            ev_sweep.start(ss);
            int rest = K;
            while (rest > 0) {
                if (rest >= kChunkSweeps && c->ycur == c->Y1.p) {
                    if (!c->chunk[c->sor ? 1 : 0]) capture_chunk();
                    HIPCHECK(hipGraphLaunch(c->chunk[c->sor ? 1 : 0], ss));    // even count: ycur stays Y1
                    rest -= kChunkSweeps;
                } else {
                    void* yo = other(c->ycur);
                    mk::sweep(*c, g, c->ycur, yo);
                    c->ycur = yo;
                    rest -= 1;
                }
            }
            ev_sweep.stop(ss);
            sweep_timed = true;
            seq_sweeps = K;
            for (int b = 0; b < Bw; ++b) {
                Slot& sl = slots[b];
                if (sl.state != RUNNING) continue;
                sl.sweeps += hkb[b];
                sl.stage_sweeps += hkb[b];
                sl.stage_left -= hkb[b];
                sl.err *= std::pow(sl.rho, hkb[b]);
                if (hkb[b] > 0) {
                    sl.entry = false;
                    sl.t_moved = false;
                }
            }
        }
        // refresh the slots whose stage has ended, and those out of sweeps
        // (their final certificate)
        std::vector<int32_t> hr(Bw, 0);
        bool any = false;
        for (int b = 0; b < Bw; ++b) {
            Slot& sl = slots[b];
            if (sl.state == RUNNING && (sl.stage_left <= 0 || out_of_sweeps(sl))) {
                // T holds this stage's increments unless a refresh already moved it
                if (sl.t_moved) fail(PPR_ERR_DEVICE, "internal: refresh of a column without a stage");
                hr[b] = sl.s_unset ? 2 : 1;
                sl.t_moved = true;
                sl.s_unset = false;
                sl.refreshing = true;
                any = true;
            }
        }
        if (any) {
            upload_i32(c->rmask, hr);
            ev_refresh.start(ss);
            mk::refresh(*c, g, const_cast<void*>(c->ycur), nullptr);
            ev_refresh.stop(ss);
            refresh_timed = true;
            HIPCHECK(hipMemcpyAsync(c->host.p, c->colsum.p, 8 * (size_t)Bw, hipMemcpyDeviceToHost, ss));
        }
        if (any || sweep_timed) {
            HIPCHECK(hipEventRecord(ev_ready, ss));
            inflight = true;
        }
    }

    bool settled() const {
        for (const Slot& sl : slots)
            if (sl.state == PENDING || sl.state == RUNNING) return false;
        return true;
    }

    void fill_stats(int b, ppr_stats* st, double ms) const {
        const Slot& sl = slots[b];
        st->local_levels = sl.levels;
        st->sweeps = sl.sweeps;
        st->refreshes = sl.refreshes;
        st->source = sl.src;
        st->edge_pushes = sl.edges + (int64_t)(sl.sweeps + sl.refreshes) * g.m;
        st->r_sum = sl.cert;
        st->cert_l1 = sl.cert;
        st->ms = ms;
        st->sweep_ms = sweep_ms;
        st->sweep_launches = sweep_launches;
        st->batch_cols = Bw;
        st->sweep_chunks = c->chunks;
        st->sor_omega = sl.omega;
        st->residue_format = c->bf16 ? PPR_RESIDUE_BF16 : PPR_RESIDUE_F32;
        st->push_scans = 0;
        st->sweep_tile_bytes = c->tile;
        st->refresh_ms = refresh_ms;
        st->refresh_launches = refresh_launches;
        st->reserved = 0;
    }

    // Export slot b (DONE) into out[n] (host or device) and free the slot;
    // a slot that ended at its sweep cap is exported too, then reported.
    void retire(int b, double* out, ppr_stats* st) {
        if (b < 0 || b >= Bw) fail(PPR_ERR_ARG, "slot out of range");
        if (slots[b].state != DONE) fail(PPR_ERR_BUSY, "slot has no certified result yet");
        hipStream_t ss = c->stream;
        if (is_device_ptr(out, g.device)) {
            mk::export_col(*c, g, b, out);
        } else {
            if (c->stage.bytes < 8 * (size_t)g.n) c->stage.alloc(8 * (size_t)g.n);
            mk::export_col(*c, g, b, c->stage.as<double>());
            HIPCHECK(hipMemcpyAsync(out, c->stage.p, 8 * (size_t)g.n, hipMemcpyDefault, ss));
        }
        HIPCHECK(hipStreamSynchronize(ss));
        if (st) fill_stats(b, st, now_ms() - slots[b].t_admit);
        const bool failed = slots[b].failed;
        slots[b] = Slot();
        if (failed) fail(PPR_ERR_NOT_CONVERGED, "max_sweeps reached before the certificate fell to lambda");
    }
};

// ======================================================================== batch driver

namespace {

void run_mixed_chunk(Block& blk, const int32_t* sources, int Breal, double lambda, double* pi_out, double* r_out,
                     ppr_stats* st) {
    const double t0 = now_ms();
    Graph& g = blk.g;
    MixedCtx& c = *blk.c;
    for (int b = 0; b < Breal; ++b)
        if (blk.admit(sources[b], blk.alpha, lambda) != b) fail(PPR_ERR_ARG, "internal: batch slot order");
    while (!blk.settled()) {     // each slot ends: certified, or at its sweep cap
        blk.step(1 << 30);
        blk.collect(true);
    }
    // ---- output: the export kernel writes device memory only; a host
    // destination is filled through a device staging buffer
    hipStream_t ss = c.stream;
    if (is_device_ptr(pi_out, g.device)) {
        mk::export_cols(c, g, 0, Breal, pi_out);
    } else {
        if (c.stage.bytes < 8 * (size_t)blk.Bw * g.n) c.stage.alloc(8 * (size_t)blk.Bw * g.n);
        mk::export_cols(c, g, 0, Breal, c.stage.as<double>());
        HIPCHECK(hipMemcpyAsync(pi_out, c.stage.p, 8 * (size_t)Breal * g.n, hipMemcpyDefault, ss));
    }
    if (r_out) {
        // FP64 residual of the exported estimates, row-major [Breal][n]
        std::vector<int32_t> none(blk.Bw, 0);
        blk.upload_i32(c.rmask, none);
        // every column's last refresh moved its T into S
        HIPCHECK(hipMemsetAsync(c.T.p, 0, c.T.bytes, ss));
        DevBuf rt((size_t)blk.Bw * g.n * 8);
        mk::refresh(c, g, const_cast<void*>(c.ycur), rt.as<double>());
        HIPCHECK(hipMemcpyAsync(r_out, rt.p, 8 * (size_t)Breal * g.n, hipMemcpyDefault, ss));
        HIPCHECK(hipStreamSynchronize(ss));
    }
    HIPCHECK(hipStreamSynchronize(ss));
    const double ms = now_ms() - t0;
    bool failed = false;
    for (int b = 0; b < Breal; ++b) {
        if (blk.slots[b].failed) failed = true;
        if (st) blk.fill_stats(b, st + b, ms);
        blk.slots[b] = Block::Slot();
    }
    if (failed) fail(PPR_ERR_NOT_CONVERGED, "max_sweeps reached before the certificate fell to lambda");
}

int default_batch_width(int32_t B) {
    int w = 4;
    while (w < B && w < 32) w <<= 1;
    return w;
}

}  // namespace

void run_mixed_batch(Graph& g, const int32_t* sources, int32_t B, double alpha, double lambda,
                     const ppr_options& opt, double* pi_out, double* r_out, ppr_stats* st) {
    HIPCHECK(hipSetDevice(g.device));
    const int tw = g.tuned_width.load();
    int Bw = opt.batch_cols > 0 ? opt.batch_cols : (tw > 0 ? tw : default_batch_width(B));
    if (opt.batch_cols == 0 && opt.residue_format == PPR_RESIDUE_BF16) Bw = std::max(Bw, 8);   // 8-column vectors
    if (Bw < 4 || Bw > 128 || (Bw & (Bw - 1))) fail(PPR_ERR_ARG, "batch_cols must be a power of two in [4, 128]");
    // the autotuner's residue format for this width, unless the caller chose one
    ppr_options o = opt;
    const int tf = g.tuned_fmt[ilog2(Bw) & 7].load();
    if (o.residue_format == PPR_RESIDUE_AUTO && tf > 0) o.residue_format = tf - 1;
    ppr_status first = PPR_OK;
    std::string msg;
    for (int32_t b0 = 0; b0 < B; b0 += Bw) {
        int Breal = std::min<int32_t>(Bw, B - b0);
        Block blk(g, Bw, alpha, o);
        try {
            run_mixed_chunk(blk, sources + b0, Breal, lambda, pi_out + (size_t)b0 * g.n,
                            r_out ? r_out + (size_t)b0 * g.n : nullptr, st ? st + b0 : nullptr);
        } catch (const Failure& e) {
            // not converged: the FP64 scratch was already cleared by the conversion
            if (e.status != PPR_ERR_NOT_CONVERGED) throw;
            if (first == PPR_OK) {
                first = e.status;
                msg = e.msg;
            }
        }
    }
    if (first != PPR_OK) fail(first, msg);
}

// ======================================================================== autotuner

namespace {

// Sources of a tuning batch of W queries: ids spread by a multiplicative hash.
std::vector<int32_t> tuning_sources(int32_t n, int W) {
    std::vector<int32_t> s(W);
    for (int k = 0; k < W; ++k) s[k] = (int32_t)(((uint64_t)(k + 1) * 2654435761ull + 12345ull) % (uint64_t)n);
    return s;
}

// The sweep tile of this block's width and residue format: time a few
// sweeps at each candidate LDS stage; the default stage stays unless another
// is more than 1% faster.  Leaves the block at that tile, its state cleared.
int tune_tile(Graph& g, Block& blk) {
    MixedCtx& c = *blk.c;
    hipStream_t ss = c.stream;
    const int W = blk.Bw;
    // every column active for the timing; the cost of a sweep does not
    // depend on the values it moves
    std::vector<int32_t> kb(W, 1 << 30), zero(W, 0);
    blk.upload_i32(c.kb, kb);
    blk.upload_i32(c.entry, zero);
    blk.set_steps(1 << 30);              // odd and even steps alternate, as in a query
    const int reps = 4;
    double tile_us[mk::kTileCount];
    for (int ti = 0; ti < mk::kTileCount; ++ti) {
        c.drop_chunks();
        c.tile = mk::kTiles[ti];
        mk::prepare(c, g);                   // the tile's schedule and piece buffer
        mk::sweep(c, g, c.Y0.p, c.Y1.p);     // warm-up
        EventPair ev;
        ev.start(ss);
        for (int r = 0; r < reps; ++r) mk::sweep(c, g, (r & 1) ? c.Y1.p : c.Y0.p, (r & 1) ? c.Y0.p : c.Y1.p);
        ev.stop(ss);
        HIPCHECK(hipStreamSynchronize(ss));
        tile_us[ti] = ev.elapsed_ms() * 1e3 / reps;
    }
    int tile = mk::kLdsBytes;
    double us = 0.0;
    for (int ti = 0; ti < mk::kTileCount; ++ti)
        if (mk::kTiles[ti] == mk::kLdsBytes) us = tile_us[ti];
    const double us_default = us;
    for (int ti = 0; ti < mk::kTileCount; ++ti)
        if (tile_us[ti] < us_default * 0.99 && tile_us[ti] < us) {
            us = tile_us[ti];
            tile = mk::kTiles[ti];
        }
    c.drop_chunks();
    c.tile = tile;
    mk::prepare(c, g);
    blk.upload_i32(c.kb, zero);
    for (DevBuf* b : {&c.Y0, &c.Y1, &c.T}) HIPCHECK(hipMemsetAsync(b->p, 0, b->bytes, ss));
    HIPCHECK(hipStreamSynchronize(ss));
    c.ycur = c.Y0.p;
    return tile;
}

// Wall time (ms) of one batch of queries answered by the block, from
// admission to the last certificate (no export).
double time_batch(Block& blk, const std::vector<int32_t>& src, double lambda) {
    HIPCHECK(hipStreamSynchronize(blk.c->stream));
    const double t0 = now_ms();
    for (size_t b = 0; b < src.size(); ++b)
        if (blk.admit(src[b], blk.alpha, lambda) != (int)b) fail(PPR_ERR_ARG, "internal: tuning slot order");
    while (!blk.settled()) {
        blk.step(1 << 30);
        blk.collect(true);
    }
    const double ms = now_ms() - t0;
    for (auto& sl : blk.slots) sl = Block::Slot();
    return ms;
}

}  // namespace

void autotune_width(Graph& g, double alpha, double lambda, const int32_t* widths, int32_t count, int32_t* best,
                    double* cost_us) {
    HIPCHECK(hipSetDevice(g.device));
    static const int32_t kDefault[5] = {8, 16, 32, 64, 128};
    if (!widths) {
        widths = kDefault;
        count = 5;
    }
    if (count < 1) fail(PPR_ERR_ARG, "no candidate widths");
    size_t free_b = 0, total_b = 0;
    HIPCHECK(hipMemGetInfo(&free_b, &total_b));
    int qmax = 0;
    for (int32_t i = 0; i < count; ++i) {
        const int W = widths[i];
        if (W < 4 || W > 128 || (W & (W - 1))) fail(PPR_ERR_ARG, "candidate widths must be powers of two in [4, 128]");
        qmax = std::max(qmax, W);
    }
    double best_cost = 1e300;
    int best_w = 0;
    for (int32_t i = 0; i < count; ++i) {
        int W = widths[i];
        if (cost_us) cost_us[i] = -1.0;
        double w_cost = 1e300;
        int w_fmt = -1;
        for (int fmt : {PPR_RESIDUE_F32, PPR_RESIDUE_BF16}) {
            if (fmt == PPR_RESIDUE_BF16 && W < 8) continue;       // bf16 vectors hold 8 columns
            ppr_options opt;
            ppr_options_default(&opt);
            opt.precision = PPR_MIXED;
            opt.residue_format = fmt;
            const bool bf = fmt == PPR_RESIDUE_BF16;
            const int64_t fcap = frontier_capacity(g.n, g.m, opt, W);
            bool pooled = false;
            {
                std::lock_guard<std::mutex> lk(g.pool_mu);
                for (auto& cc : g.mixed_pool) pooled |= (cc->Bw == W && cc->fcap >= fcap && cc->bf16 == bf);
            }
            if (!pooled && mixed_footprint(g.n, g.m, W, fcap, bf) > free_b / 2) continue;
            opt.sweep_tile = mk::kLdsBytes;
            Block blk(g, W, alpha, opt);
            const int tile = tune_tile(g, blk);
            g.tuned_tile[bf ? 1 : 0][ilog2(W) & 7].store(tile);
            // end to end: local phase, sweeps and refreshes (the refresh
            // count depends on the residue format, the sweeps per query on
            // the width), after one warm-up batch; every width answers the
            // same qmax queries, in qmax / W batches, so that the widths are
            // compared on one workload
            const std::vector<int32_t> src = tuning_sources(g.n, qmax);
            (void)time_batch(blk, std::vector<int32_t>(src.begin(), src.begin() + W), lambda);
            double ms = 0.0;
            for (int q0 = 0; q0 < qmax; q0 += W)
                ms += time_batch(blk, std::vector<int32_t>(src.begin() + q0, src.begin() + q0 + W), lambda);
            const double us = ms * 1e3 / qmax;
            if (us < w_cost * 0.99 || (us < w_cost && fmt == PPR_RESIDUE_F32)) {
                w_cost = us;
                w_fmt = fmt;
            }
        }
        if (w_fmt < 0) continue;                                    // no format fits the memory
        g.tuned_fmt[ilog2(W) & 7].store(w_fmt + 1);
        if (cost_us) cost_us[i] = w_cost;
        // the narrower block wins ties (within 1%): less memory, lower latency
        if (best_w == 0 || w_cost < best_cost * 0.99) {
            best_cost = w_cost;
            best_w = W;
        }
    }
    if (best_w == 0) fail(PPR_ERR_OOM, "no candidate width fits the device memory budget");
    g.tuned_width = best_w;
    if (best) *best = best_w;
}

// ======================================================================== sweep sequences (tests)

void debug_sweeps_mixed(Graph& g, double alpha, int32_t B, int32_t chunks, int32_t sweeps, const float* y_in,
                        const int32_t* entry, const int32_t* budget, const float* t_in, float* y_out,
                        float* t_out, const float* omega, int32_t residue_format, int32_t sweep_tile,
                        bool wide_gather) {
    HIPCHECK(hipSetDevice(g.device));
    ppr_options opt;
    ppr_options_default(&opt);
    opt.sweep_chunks = chunks;
    opt.residue_format = residue_format;
    opt.sweep_tile = sweep_tile;
    Block blk(g, B, alpha, opt);
    MixedCtx& c = *blk.c;
    hipStream_t ss = c.stream;
    const int64_t count = (int64_t)g.n * B;
    const size_t bytes = 4 * (size_t)count;
    DevBuf stage(bytes);                    // FP32 copy of the residue block on the device
    HIPCHECK(hipMemcpyAsync(stage.p, y_in, bytes, hipMemcpyDefault, ss));
    mk::store_from_f32(c, stage.as<float>(), c.Y0.p, count);
    if (t_in) HIPCHECK(hipMemcpyAsync(c.T.p, t_in, bytes, hipMemcpyDefault, ss));
    else HIPCHECK(hipMemsetAsync(c.T.p, 0, bytes, ss));
    std::vector<int32_t> kb(B, sweeps), en(entry, entry + B), zero(B, 0);
    if (budget) kb.assign(budget, budget + B);
    blk.upload_i32(c.kb, kb);
    blk.upload_i32(c.entry, en);
    blk.set_steps(sweeps - 1);
    if (omega) {
        HIPCHECK(hipMemcpyAsync(c.omega.p, omega, 4 * (size_t)B, hipMemcpyHostToDevice, ss));
        c.sor = true;
    }
    void* a = c.Y0.p;
    void* o = c.Y1.p;
    DevBuf w0, w1;                          // residue buffers apart from the joint one (64-bit gathers)
    if (wide_gather) {
        w0.alloc(c.Y0.bytes);
        w1.alloc(c.Y1.bytes);
        HIPCHECK(hipMemcpyAsync(w0.p, c.Y0.p, c.Y0.bytes, hipMemcpyDeviceToDevice, ss));
        HIPCHECK(hipMemsetAsync(w1.p, 0, w1.bytes, ss));
        a = w0.p;
        o = w1.p;
    }
    for (int32_t k = 0; k < sweeps; ++k) {
        mk::sweep(c, g, a, o);
        std::swap(a, o);
    }
    c.sor = false;
    mk::store_to_f32(c, a, stage.as<float>(), count);
    HIPCHECK(hipMemcpyAsync(y_out, stage.p, bytes, hipMemcpyDefault, ss));
    if (t_out) HIPCHECK(hipMemcpyAsync(t_out, c.T.p, bytes, hipMemcpyDefault, ss));
    if (omega) {
        std::vector<float> ones(B, 1.0f);
        HIPCHECK(hipMemcpyAsync(c.omega.p, ones.data(), 4 * (size_t)B, hipMemcpyHostToDevice, ss));
    }
    blk.upload_i32(c.kb, zero);
    blk.upload_i32(c.entry, zero);
    for (DevBuf* d : {&c.Y0, &c.Y1, &c.T}) HIPCHECK(hipMemsetAsync(d->p, 0, d->bytes, ss));
    HIPCHECK(hipStreamSynchronize(ss));
    c.ycur = c.Y0.p;
}

// ======================================================================== serving mechanism

void* serve_block_create(Graph& g, int32_t slots, double alpha, const ppr_options& opt) {
    HIPCHECK(hipSetDevice(g.device));
    Block* b = new Block(g, slots, alpha, opt);
    std::lock_guard<std::mutex> lk(g.pool_mu);
    g.live_blocks += 1;
    return b;
}

void serve_block_destroy(void* h) {
    Block* b = static_cast<Block*>(h);
    if (!b) return;
    Graph& g = b->g;
    (void)hipSetDevice(g.device);
    try {
        b->collect(true);
    } catch (...) {
    }
    delete b;
    std::lock_guard<std::mutex> lk(g.pool_mu);
    g.live_blocks -= 1;
}

int32_t serve_admit(void* h, int32_t s, double alpha, double lambda) {
    Block* blk = static_cast<Block*>(h);
    HIPCHECK(hipSetDevice(blk->g.device));
    if (s < 0 || s >= blk->g.n) fail(PPR_ERR_ARG, "source outside [0, n)");
    if (alpha == 0.0) alpha = blk->alpha;          // the block's reference alpha
    if (!(alpha > 0.0 && alpha < 1.0)) fail(PPR_ERR_ARG, "alpha must lie in (0, 1), or be 0 for the block's");
    if (!(lambda > 0.0 && lambda <= 1.0)) fail(PPR_ERR_ARG, "lambda must lie in (0, 1]");
    int b = blk->admit(s, alpha, lambda);
    if (b < 0) fail(PPR_ERR_BUSY, "no free slot in the block");
    return b;
}

void serve_step(void* h, int32_t max_sweeps) {
    Block* blk = static_cast<Block*>(h);
    HIPCHECK(hipSetDevice(blk->g.device));
    if (max_sweeps < 1) fail(PPR_ERR_ARG, "max_sweeps must be >= 1");
    blk->step(max_sweeps);
}

void serve_poll(void* h, int wait, uint8_t* done, int32_t* n_done, int32_t* n_busy, int32_t* ready) {
    Block* blk = static_cast<Block*>(h);
    HIPCHECK(hipSetDevice(blk->g.device));
    bool r = blk->collect(wait != 0);
    int32_t nd = 0, nb = 0;
    for (int b = 0; b < blk->Bw; ++b) {
        int st = blk->slots[b].state;
        if (done) done[b] = (st == DONE) ? 1 : 0;
        if (st == DONE) ++nd;
        if (st != FREE) ++nb;
    }
    if (n_done) *n_done = nd;
    if (n_busy) *n_busy = nb;
    if (ready) *ready = r ? 1 : 0;
}

void serve_retire(void* h, int32_t slot, double* pi_out, ppr_stats* st) {
    Block* blk = static_cast<Block*>(h);
    HIPCHECK(hipSetDevice(blk->g.device));
    if (!pi_out) fail(PPR_ERR_ARG, "pi_out is NULL");
    blk->retire(slot, pi_out, st);
}

size_t serve_footprint(int32_t n, int64_t m, int32_t slots) {
    ppr_options opt;
    ppr_options_default(&opt);
    return mixed_footprint(n, m, slots, frontier_capacity(n, m, opt, slots), residues_bf16(opt, slots));
}

}  // namespace ppr
