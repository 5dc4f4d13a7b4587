// C ABI entry points of libppr.  Every function converts internal failures
// (ppr::Failure, std::bad_alloc, other exceptions) into a status code and a
// thread-local message; nothing throws across the boundary.
#include <cmath>
#include <cstring>
#include <new>
#include <utility>

#include "ppr_internal.h"

using namespace ppr;

namespace {

template <class F>
ppr_status guarded(F&& f) {
    return guarded_call(std::forward<F>(f));
}

void check_query_args(const Graph* g, const int32_t* sources, int32_t B, double alpha, double lambda,
                      const void* pi_out) {
    if (!g) fail(PPR_ERR_ARG, "graph is NULL");
    if (!sources) fail(PPR_ERR_ARG, "sources is NULL");
    if (!pi_out) fail(PPR_ERR_ARG, "pi_out is NULL");
    if (B < 1) fail(PPR_ERR_ARG, "batch size must be >= 1");
    if (!(alpha > 0.0 && alpha < 1.0)) fail(PPR_ERR_ARG, "alpha must lie in (0, 1)");
    if (!(lambda > 0.0 && lambda <= 1.0)) fail(PPR_ERR_ARG, "lambda must lie in (0, 1]");
    for (int32_t b = 0; b < B; ++b)
        if (sources[b] < 0 || sources[b] >= g->n)
            fail(PPR_ERR_ARG, "source " + std::to_string(sources[b]) + " is outside [0, n)");
}

void check_options(const ppr_options& o) {
    if (o.precision != PPR_FP64 && o.precision != PPR_MIXED) fail(PPR_ERR_ARG, "unknown precision");
    if (o.switch_rule != PPR_SWITCH_NODES && o.switch_rule != PPR_SWITCH_EDGES)
        fail(PPR_ERR_ARG, "unknown switch rule");
    if (!(o.switch_param >= 0.0) || std::isinf(o.switch_param)) fail(PPR_ERR_ARG, "switch_param must be finite and >= 0");
    if (o.max_sweeps < 0) fail(PPR_ERR_ARG, "max_sweeps must be >= 0");
    if (!(o.refresh_factor == 0.0 || o.refresh_factor > 1.0)) fail(PPR_ERR_ARG, "refresh_factor must be 0 or > 1");
    if (o.residue_format != PPR_RESIDUE_F32 && o.residue_format != PPR_RESIDUE_BF16 &&
        o.residue_format != PPR_RESIDUE_AUTO)
        fail(PPR_ERR_ARG, "unknown residue format");
    if (o.scan_form != PPR_SCAN_AUTO && o.scan_form != PPR_SCAN_PULL && o.scan_form != PPR_SCAN_PUSH)
        fail(PPR_ERR_ARG, "unknown scan form");
    if (o.batch_cols < 0 || (o.batch_cols % 4) != 0) fail(PPR_ERR_ARG, "batch_cols must be 0 or a multiple of 4");
    if (o.sweep_chunks < 0 || o.sweep_chunks > 64) fail(PPR_ERR_ARG, "sweep_chunks must lie in [0, 64]");
    if (!(o.sor_omega == 0.0 || (o.sor_omega >= 1.0 && o.sor_omega <= 1.9)))
        fail(PPR_ERR_ARG, "sor_omega must be 0 (automatic), 1 (off) or lie in (1, 1.9]");
    if (o.global_rule != PPR_GLOBAL_SWEEPS && o.global_rule != PPR_GLOBAL_EPOCHS)
        fail(PPR_ERR_ARG, "unknown global rule");
    if (o.global_rule == PPR_GLOBAL_EPOCHS && o.precision != PPR_FP64)
        fail(PPR_ERR_ARG, "the epoch global phase is a PPR_FP64 option");
    if (o.use_stream != 0 && o.use_stream != 1) fail(PPR_ERR_ARG, "use_stream must be 0 or 1");
}

}  // namespace

extern "C" {

void ppr_options_default(ppr_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = PPR_FP64;
    o->switch_rule = PPR_SWITCH_EDGES;
    o->switch_param = 32.0;
    o->max_sweeps = 4096;
    o->certify = 0;
    o->refresh_factor = 0.0;
    o->batch_cols = 0;
    o->residue_format = PPR_RESIDUE_AUTO;
    o->scan_form = PPR_SCAN_AUTO;
    o->use_stream = 0;
    o->stream = NULL;
}

const char* ppr_version(void) { return "libppr 0.1 (gfx950)"; }

const char* ppr_last_error(void) { return last_error_cstr(); }

ppr_status ppr_graph_create(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t m,
                            uint32_t flags, ppr_graph** out) {
    return guarded([&] {
        if (!out) fail(PPR_ERR_ARG, "out is NULL");
        *out = nullptr;
        Graph* g = graph_create(row_ptr, col, n, m, flags);
        *out = reinterpret_cast<ppr_graph*>(g);
    });
}

ppr_status ppr_graph_destroy(ppr_graph* gh) {
    return guarded([&] {
        Graph* g = reinterpret_cast<Graph*>(gh);
        if (!g) return;
        {
            std::lock_guard<std::mutex> lk(g->pool_mu);
            if (g->live_blocks > 0) fail(PPR_ERR_BUSY, "serving blocks still use this graph");
        }
        (void)hipSetDevice(g->device);
        (void)hipDeviceSynchronize();
        delete g;
    });
}

ppr_status ppr_graph_get_info(const ppr_graph* gh, ppr_graph_info* info) {
    return guarded([&] {
        const Graph* g = reinterpret_cast<const Graph*>(gh);
        if (!g || !info) fail(PPR_ERR_ARG, "NULL argument");
        info->n = g->n;
        info->m = g->m;
        info->max_in_degree = g->max_in;
        info->max_out_degree = g->max_out;
        info->offsets_64bit = g->off64 ? 1 : 0;
        info->build_ms = g->build_ms;
        info->device_bytes = g->device_bytes();
        info->fp64_slices = g->fp64_slices;
        info->reserved = 0;
    });
}

ppr_status ppr_graph_copy_csc(const ppr_graph* gh, int64_t* col_ptr, int32_t* row_idx, int32_t* deg_out) {
    return guarded([&] {
        const Graph* g = reinterpret_cast<const Graph*>(gh);
        if (!g) fail(PPR_ERR_ARG, "graph is NULL");
        graph_copy_csc(*g, col_ptr, row_idx, deg_out);
    });
}

ppr_status ppr_query_ex(ppr_graph* gh, const int32_t* sources, int32_t B, double alpha, double lambda,
                        const ppr_options* opt, double* pi_out, double* r_out, ppr_stats* stats) {
    return guarded([&] {
        Graph* g = reinterpret_cast<Graph*>(gh);
        check_query_args(g, sources, B, alpha, lambda, pi_out);
        ppr_options o;
        if (opt) o = *opt; else ppr_options_default(&o);
        check_options(o);
        HIPCHECK(hipSetDevice(g->device));
        (void)is_device_ptr(pi_out, g->device);            // rejects another device's memory
        if (r_out) (void)is_device_ptr(r_out, g->device);
        if (o.precision == PPR_FP64) {
            ppr_status first = PPR_OK;
            std::string msg;
            for (int32_t b = 0; b < B; ++b) {
                try {
                    run_fp64_query(*g, sources[b], alpha, lambda, o, pi_out + (size_t)b * g->n,
                                   r_out ? r_out + (size_t)b * g->n : nullptr, stats ? stats + b : nullptr);
                } catch (const Failure& e) {
                    if (e.status != PPR_ERR_NOT_CONVERGED) throw;
                    if (first == PPR_OK) { first = e.status; msg = e.msg; }
                }
            }
            if (first != PPR_OK) fail(first, msg);
        } else {
            run_mixed_batch(*g, sources, B, alpha, lambda, o, pi_out, r_out, stats);
        }
    });
}

ppr_status ppr_query_trace(ppr_graph* gh, int32_t s, double alpha, double lambda, const ppr_options* opt,
                           double* pi_out, ppr_trace_point* trace, int32_t capacity, int32_t* count,
                           ppr_stats* stats) {
    return guarded([&] {
        Graph* g = reinterpret_cast<Graph*>(gh);
        check_query_args(g, &s, 1, alpha, lambda, pi_out);
        ppr_options o;
        if (opt) o = *opt; else ppr_options_default(&o);
        check_options(o);
        if (o.precision != PPR_FP64) fail(PPR_ERR_ARG, "a traced query runs the PPR_FP64 path");
        if (capacity < 0 || !count || (capacity > 0 && !trace)) fail(PPR_ERR_ARG, "bad trace buffer");
        HIPCHECK(hipSetDevice(g->device));
        (void)is_device_ptr(pi_out, g->device);
        TraceSink sink;
        sink.out = trace;
        sink.cap = capacity;
        sink.t0 = std::chrono::steady_clock::now();
        *count = 0;
        try {
            run_fp64_query(*g, s, alpha, lambda, o, pi_out, nullptr, stats, &sink);
        } catch (...) {
            *count = sink.count;
            throw;
        }
        *count = sink.count;
    });
}

ppr_status ppr_query(ppr_graph* g, int32_t s, double alpha, double lambda, ppr_precision precision,
                     double* pi_out, ppr_stats* stats) {
    ppr_options o;
    ppr_options_default(&o);
    o.precision = precision;
    return ppr_query_ex(g, &s, 1, alpha, lambda, &o, pi_out, nullptr, stats);
}

ppr_status ppr_query_batch(ppr_graph* g, const int32_t* sources, int32_t B, double alpha, double lambda,
                           ppr_precision precision, double* pi_out, ppr_stats* stats) {
    ppr_options o;
    ppr_options_default(&o);
    o.precision = precision;
    return ppr_query_ex(g, sources, B, alpha, lambda, &o, pi_out, nullptr, stats);
}

ppr_status ppr_autotune(ppr_graph* gh, double alpha, double lambda, const int32_t* widths, int32_t count,
                        int32_t* best_width, double* cost_us) {
    return guarded([&] {
        Graph* g = reinterpret_cast<Graph*>(gh);
        if (!g) fail(PPR_ERR_ARG, "graph is NULL");
        if (!(alpha > 0.0 && alpha < 1.0)) fail(PPR_ERR_ARG, "alpha must lie in (0, 1)");
        if (!(lambda > 0.0 && lambda <= 1.0)) fail(PPR_ERR_ARG, "lambda must lie in (0, 1]");
        if (widths && count < 1) fail(PPR_ERR_ARG, "count must be >= 1");
        autotune_width(*g, alpha, lambda, widths, count, best_width, cost_us);
    });
}

ppr_status ppr_debug_sweep_mixed(ppr_graph* gh, double alpha, int32_t B, int32_t chunks, const float* y_in,
                                 const int32_t* fresh, float* y_out, float* t_out, const float* omega,
                                 int32_t residue_format) {
    if (!fresh || B < 4 || B > 128) return ppr_debug_sweeps_mixed(gh, alpha, B, chunks, 1, y_in, fresh, nullptr,
                                                                  nullptr, y_out, t_out, omega, residue_format, 0, 0);
    std::vector<int32_t> en(B);
    for (int32_t b = 0; b < B; ++b) en[b] = fresh[b] ? 1 : 0;
    return ppr_debug_sweeps_mixed(gh, alpha, B, chunks, 1, y_in, en.data(), nullptr, nullptr, y_out, t_out, omega,
                                  residue_format, 0, 0);
}

ppr_status ppr_debug_sweeps_mixed(ppr_graph* gh, double alpha, int32_t B, int32_t chunks, int32_t sweeps,
                                  const float* y_in, const int32_t* entry, const int32_t* budget,
                                  const float* t_in, float* y_out, float* t_out, const float* omega,
                                  int32_t residue_format, int32_t sweep_tile, int32_t flags) {
    return guarded([&] {
        Graph* g = reinterpret_cast<Graph*>(gh);
        if (!g || !y_in || !entry || !y_out) fail(PPR_ERR_ARG, "NULL argument");
        if (!(alpha > 0.0 && alpha < 1.0)) fail(PPR_ERR_ARG, "alpha must lie in (0, 1)");
        if (B < 4 || B > 128 || (B & (B - 1))) fail(PPR_ERR_ARG, "B must be a power of two in [4, 128]");
        if (chunks < 1 || chunks > 64) fail(PPR_ERR_ARG, "chunks must lie in [1, 64]");
        if (sweeps < 1 || sweeps > 64) fail(PPR_ERR_ARG, "sweeps must lie in [1, 64]");
        for (int32_t b = 0; b < B; ++b) {
            if (entry[b] < 0 || entry[b] > 2) fail(PPR_ERR_ARG, "entry flags must be 0, 1 or 2");
            if (budget && (budget[b] < 0 || budget[b] > sweeps)) fail(PPR_ERR_ARG, "budgets must lie in [0, sweeps]");
        }
        HIPCHECK(hipSetDevice(g->device));
        (void)is_device_ptr(y_in, g->device);              // rejects another device's memory
        (void)is_device_ptr(y_out, g->device);
        if (t_out) (void)is_device_ptr(t_out, g->device);
        if (t_in) (void)is_device_ptr(t_in, g->device);
        if (omega)
            for (int32_t b = 0; b < B; ++b)
                if (!(omega[b] > 0.0f && omega[b] < 2.0f)) fail(PPR_ERR_ARG, "omega must lie in (0, 2)");
        if (residue_format != PPR_RESIDUE_F32 && residue_format != PPR_RESIDUE_BF16 &&
            residue_format != PPR_RESIDUE_AUTO)
            fail(PPR_ERR_ARG, "unknown residue format");
        if (flags & ~PPR_DEBUG_WIDE_GATHER) fail(PPR_ERR_ARG, "unknown debug flags");
        debug_sweeps_mixed(*g, alpha, B, chunks, sweeps, y_in, entry, budget, t_in, y_out, t_out, omega,
                           residue_format, sweep_tile, (flags & PPR_DEBUG_WIDE_GATHER) != 0);
    });
}

// ---------------------------------------------------------------- approximate SSPPR

ppr_status ppr_query_approx(ppr_graph* gh, int32_t s, double alpha, double eps, double mu, uint64_t seed,
                            int32_t use_index, const ppr_options* opt, double* pi_out, ppr_approx_stats* stats) {
    return guarded([&] {
        Graph* g = reinterpret_cast<Graph*>(gh);
        check_query_args(g, &s, 1, alpha, 1.0, pi_out);
        if (!(eps > 0.0 && eps <= 1.0)) fail(PPR_ERR_ARG, "eps must lie in (0, 1]");
        if (!(mu > 0.0 && mu <= 1.0)) fail(PPR_ERR_ARG, "mu must lie in (0, 1]");
        if (use_index != 0 && use_index != 1) fail(PPR_ERR_ARG, "use_index must be 0 or 1");
        ppr_options o;
        if (opt) {
            o = *opt;
        } else {
            ppr_options_default(&o);
            o.global_rule = PPR_GLOBAL_EPOCHS;      // Algorithm 3's thresholds: fewer refinement levels
        }
        o.precision = PPR_FP64;
        check_options(o);
        HIPCHECK(hipSetDevice(g->device));
        (void)is_device_ptr(pi_out, g->device);
        run_approx_query(*g, s, alpha, eps, mu, seed, use_index == 1, o, pi_out, stats);
    });
}

ppr_status ppr_walk_index_build(ppr_graph* gh, double alpha, uint64_t seed, double* ms) {
    return guarded([&] {
        Graph* g = reinterpret_cast<Graph*>(gh);
        if (!g) fail(PPR_ERR_ARG, "graph is NULL");
        if (!(alpha > 0.0 && alpha < 1.0)) fail(PPR_ERR_ARG, "alpha must lie in (0, 1)");
        build_walk_index(*g, alpha, seed, ms);
    });
}

ppr_status ppr_walk_index_copy(const ppr_graph* gh, int32_t* out) {
    return guarded([&] {
        const Graph* g = reinterpret_cast<const Graph*>(gh);
        if (!g || !out) fail(PPR_ERR_ARG, "NULL argument");
        copy_walk_index(*g, out);
    });
}

ppr_status ppr_debug_refine(ppr_graph* gh, double alpha, double rmax, double* pi, double* r, int32_t* levels,
                            int64_t* edge_pushes) {
    return guarded([&] {
        Graph* g = reinterpret_cast<Graph*>(gh);
        if (!g || !pi || !r) fail(PPR_ERR_ARG, "NULL argument");
        if (!(alpha > 0.0 && alpha < 1.0)) fail(PPR_ERR_ARG, "alpha must lie in (0, 1)");
        if (!(rmax > 0.0)) fail(PPR_ERR_ARG, "rmax must be > 0");
        HIPCHECK(hipSetDevice(g->device));
        if (!is_device_ptr(pi, g->device) || !is_device_ptr(r, g->device))
            fail(PPR_ERR_ARG, "pi and r must be device memory");
        debug_refine(*g, alpha, rmax, pi, r, levels, edge_pushes);
    });
}

ppr_status ppr_debug_walks(ppr_graph* gh, double alpha, double W, uint64_t seed, int32_t use_index,
                           const double* r, double* pi, int64_t* walks) {
    return guarded([&] {
        Graph* g = reinterpret_cast<Graph*>(gh);
        if (!g || !pi || !r) fail(PPR_ERR_ARG, "NULL argument");
        if (!(alpha > 0.0 && alpha < 1.0)) fail(PPR_ERR_ARG, "alpha must lie in (0, 1)");
        if (!(W >= 1.0) || std::isinf(W)) fail(PPR_ERR_ARG, "W must be finite and >= 1");
        if (use_index != 0 && use_index != 1) fail(PPR_ERR_ARG, "use_index must be 0 or 1");
        HIPCHECK(hipSetDevice(g->device));
        if (!is_device_ptr(pi, g->device) || !is_device_ptr(r, g->device))
            fail(PPR_ERR_ARG, "pi and r must be device memory");
        debug_walks(*g, alpha, W, seed, use_index == 1, r, pi, walks);
    });
}

// ---------------------------------------------------------------- serving

ppr_status ppr_block_create(ppr_graph* gh, int32_t slots, double alpha, const ppr_options* opt, ppr_block** out) {
    return guarded([&] {
        Graph* g = reinterpret_cast<Graph*>(gh);
        if (!g || !out) fail(PPR_ERR_ARG, "NULL argument");
        *out = nullptr;
        if (!(alpha > 0.0 && alpha < 1.0)) fail(PPR_ERR_ARG, "alpha must lie in (0, 1)");
        if (slots < 4 || slots > 128 || (slots & (slots - 1))) fail(PPR_ERR_ARG, "slots must be a power of two in [4, 128]");
        ppr_options o;
        if (opt) {
            o = *opt;
            if (o.precision != PPR_MIXED)
                fail(PPR_ERR_ARG, "a serving block runs the batched PPR_MIXED path (PPR_FP64 queries: ppr_query_ex)");
        } else {
            ppr_options_default(&o);
            o.precision = PPR_MIXED;
        }
        check_options(o);
        *out = reinterpret_cast<ppr_block*>(serve_block_create(*g, slots, alpha, o));
    });
}

ppr_status ppr_block_destroy(ppr_block* blk) {
    return guarded([&] { serve_block_destroy(blk); });
}

ppr_status ppr_block_footprint(const ppr_graph* gh, int32_t slots, size_t* bytes) {
    return guarded([&] {
        const Graph* g = reinterpret_cast<const Graph*>(gh);
        if (!g || !bytes) fail(PPR_ERR_ARG, "NULL argument");
        if (slots < 4 || slots > 128 || (slots & (slots - 1))) fail(PPR_ERR_ARG, "slots must be a power of two in [4, 128]");
        *bytes = serve_footprint(g->n, g->m, slots);
    });
}

ppr_status ppr_footprint_bytes(int32_t n, int64_t m, int32_t slots, ppr_precision precision, size_t* graph_bytes,
                               size_t* state_bytes) {
    return guarded([&] {
        if (n < 1 || m < n) fail(PPR_ERR_ARG, "need n >= 1 and m >= n (every node has an out-edge)");
        if ((double)m > (double)n * (double)n) fail(PPR_ERR_ARG, "m exceeds n^2 (A is a 0/1 matrix)");
        if (precision == PPR_MIXED) {
            if (slots < 4 || slots > 128 || (slots & (slots - 1)))
                fail(PPR_ERR_ARG, "slots must be a power of two in [4, 128]");
        } else if (precision == PPR_FP64) {
            if (slots < 1) fail(PPR_ERR_ARG, "slots must be >= 1");
        } else {
            fail(PPR_ERR_ARG, "unknown precision");
        }
        if (graph_bytes) *graph_bytes = graph_footprint(n, m);
        if (state_bytes)
            *state_bytes = precision == PPR_MIXED ? serve_footprint(n, m, slots) : (size_t)slots * fp64_ctx_footprint(n);
    });
}

ppr_status ppr_slot_admit(ppr_block* blk, int32_t source, double alpha, double lambda, int32_t* slot) {
    return guarded([&] {
        if (!blk || !slot) fail(PPR_ERR_ARG, "NULL argument");
        *slot = -1;
        *slot = serve_admit(blk, source, alpha, lambda);
    });
}

ppr_status ppr_block_step(ppr_block* blk, int32_t max_sweeps) {
    return guarded([&] {
        if (!blk) fail(PPR_ERR_ARG, "block is NULL");
        serve_step(blk, max_sweeps);
    });
}

ppr_status ppr_block_poll(ppr_block* blk, int32_t wait, uint8_t* done, int32_t* n_done, int32_t* n_busy,
                          int32_t* ready) {
    return guarded([&] {
        if (!blk) fail(PPR_ERR_ARG, "block is NULL");
        serve_poll(blk, wait, done, n_done, n_busy, ready);
    });
}

ppr_status ppr_slot_retire(ppr_block* blk, int32_t slot, double* pi_out, ppr_stats* stats) {
    return guarded([&] {
        if (!blk) fail(PPR_ERR_ARG, "block is NULL");
        serve_retire(blk, slot, pi_out, stats);
    });
}

ppr_status ppr_debug_sweep_fp64(ppr_graph* gh, double alpha, const double* r_in, double* r_out, double* pi,
                                double* r_sum_out) {
    return guarded([&] {
        Graph* g = reinterpret_cast<Graph*>(gh);
        if (!g || !r_in || !r_out || !pi) fail(PPR_ERR_ARG, "NULL argument");
        if (!(alpha > 0.0 && alpha < 1.0)) fail(PPR_ERR_ARG, "alpha must lie in (0, 1)");
        HIPCHECK(hipSetDevice(g->device));
        if (!is_device_ptr(r_in, g->device) || !is_device_ptr(r_out, g->device) || !is_device_ptr(pi, g->device))
            fail(PPR_ERR_ARG, "ppr_debug_sweep_fp64 takes device buffers");
        const Schedule& sch = g->schedule(k::sweep_nnz_cap(), k::sweep_row_cap());
        DevBuf y((size_t)g->n * 8), yo((size_t)g->n * 8), acc((size_t)g->n * 8);
        int32_t nb = std::max(sch.n_blocks, 1024);
        for (const auto& ss : g->sl_sched) nb = std::max(nb, ss->n_blocks);
        DevBuf parts(8 * (size_t)nb), sum(8);
        int np = 0;
        hipStream_t s = nullptr;
        HIPCHECK(hipMemsetAsync(acc.p, 0, acc.bytes, s));
        k::prep_y(r_in, g->deg.as<int32_t>(), alpha, g->n, y.as<double>(), parts.as<double>(), &np, s);
        k::sweep_f64(*g, sch, k::SW_ENTRY | k::SW_WRITE_R, alpha, y.as<double>(), yo.as<double>(), pi, r_in,
                     r_out, parts.as<double>(), s, acc.as<double>());
        k::reduce_sum(parts.as<double>(), k::sweep_parts(*g, sch, acc.as<double>()), sum.as<double>(), s);
        double h = 0;
        HIPCHECK(hipMemcpy(&h, sum.p, 8, hipMemcpyDeviceToHost));
        if (r_sum_out) *r_sum_out = h;
    });
}

}  // extern "C"
