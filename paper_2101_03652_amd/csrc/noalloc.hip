// Allocation-free form of the plain FP64 query, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// It runs the kernels of the FP64 path (the local phase over the iteration
// sets S^(j) of Section 4.2, then threshold-0 global sweeps of Eq. 7 until
// r_sum <= lambda) in the same order as ppr_query with default options, but
// its working state (residue, the two scaled-residue buffers, the frontier
// lists, the degree prefix, the per-block partial sums, the scan scratch and
// the counters) lives in one file-scope device array instead of a pooled,
// hipMalloc'ed context, and the reserve pi_hat is written straight into the
// caller's output.  The sweeps are launched one by one (no captured HIP
// graph: instantiating one allocates).
//
// The array exists once per device (each device's copy of the code object
// holds its own); its address comes from hipGetSymbolAddress, taken once per
// device with that device current.  A per-device lock serialises the calls
// of this process on one device, and every call synchronises its stream
// before it returns, so calls from several threads wait for each other
// rather than share the array at the same time.
#include <chrono>
#include <mutex>

#include "ppr_internal.h"

namespace {

constexpr int32_t kMaxNodes = PPR_NOALLOC_MAX_NODES;
constexpr int64_t kMaxParts = PPR_NOALLOC_MAX_SWEEP_BLOCKS;
constexpr size_t kAlign = 256;
constexpr size_t kScanBytes = 64 * 1024;

constexpr size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Layout of the array (byte offsets), sized for kMaxNodes nodes.
constexpr size_t kOffR = 0;                                                  // double[n]  residue r
constexpr size_t kOffY0 = kOffR + align_up(8 * (size_t)kMaxNodes);           // double[n]  y, or X in the local phase
constexpr size_t kOffY1 = kOffY0 + align_up(8 * (size_t)kMaxNodes);          // double[n]  y, or degF (int64)
constexpr size_t kOffOff = kOffY1 + align_up(8 * (size_t)kMaxNodes);         // int64[n+1] degree prefix of the frontier
constexpr size_t kOffF0 = kOffOff + align_up(8 * ((size_t)kMaxNodes + 1));   // int32[n]   frontier
constexpr size_t kOffF1 = kOffF0 + align_up(4 * (size_t)kMaxNodes);          // int32[n]   next frontier
constexpr size_t kOffParts = kOffF1 + align_up(4 * (size_t)kMaxNodes);       // double[kMaxParts]
constexpr size_t kOffScan = kOffParts + align_up(8 * (size_t)kMaxParts);     // exclusive-scan scratch
constexpr size_t kOffCtr = kOffScan + kScanBytes;                            // int64[2]: |S^(j+1)|, vol
constexpr size_t kOffSum = kOffCtr + kAlign;                                 // double[1]: reduced sum
constexpr size_t kScratchBytes = kOffSum + kAlign;
static_assert(kScratchBytes == PPR_NOALLOC_SCRATCH_BYTES, "the header states the array's size");

constexpr int kMaxDevices = 64;

}  // namespace

// The working state of every call on a device (see above).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct DeviceSlot {
    std::mutex mu;            // serialises the calls on this device
    unsigned char* base = nullptr;
};
DeviceSlot g_dev[kMaxDevices];

// Device address of this device's copy of `scratch`, looked up on the
// device's first call (the device is current).  Called with slot.mu held.
unsigned char* scratch_base(int device) {
    DeviceSlot& slot = g_dev[device];
    if (!slot.base) {
        void* p = nullptr;
        HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) ppr::fail(PPR_ERR_DEVICE, "hipGetSymbolAddress returned no address for the query scratch");
        slot.base = static_cast<unsigned char*>(p);
    }
    return slot.base;
}

}  // namespace

namespace ppr {

void run_fp64_query_noalloc(Graph& g, int32_t s, double alpha, double lambda, hipStream_t ss, double* pi,
                            ppr_stats* st) {
    const auto t0 = std::chrono::steady_clock::now();
    if (g.n > kMaxNodes)
        fail(PPR_ERR_ARG, "the allocation-free query takes graphs of at most " + std::to_string(kMaxNodes) +
                              " nodes (this one has " + std::to_string(g.n) + ")");
    if (g.device < 0 || g.device >= kMaxDevices) fail(PPR_ERR_DEVICE, "device index beyond the supported range");
    const Schedule* schp = g.find_schedule(k::sweep_nnz_cap(), k::sweep_row_cap());
    if (!schp) fail(PPR_ERR_DEVICE, "internal: the graph has no FP64 sweep schedule");
    const Schedule& sch = *schp;
    if (sch.n_blocks > kMaxParts)
        fail(PPR_ERR_ARG, "the allocation-free query takes graphs whose FP64 sweep has at most " +
                              std::to_string(kMaxParts) + " blocks (this one has " + std::to_string(sch.n_blocks) + ")");
    HIPCHECK(hipSetDevice(g.device));
    std::lock_guard<std::mutex> lk(g_dev[g.device].mu);
    unsigned char* base = scratch_base(g.device);
    double* r = reinterpret_cast<double*>(base + kOffR);
    double* y0 = reinterpret_cast<double*>(base + kOffY0);
    double* y1 = reinterpret_cast<double*>(base + kOffY1);
    int64_t* off = reinterpret_cast<int64_t*>(base + kOffOff);
    int32_t* F = reinterpret_cast<int32_t*>(base + kOffF0);
    int32_t* Fn = reinterpret_cast<int32_t*>(base + kOffF1);
    double* partials = reinterpret_cast<double*>(base + kOffParts);
    void* scan_tmp = base + kOffScan;
    int64_t* ctr = reinterpret_cast<int64_t*>(base + kOffCtr);
    double* dsum = reinterpret_cast<double*>(base + kOffSum);
    if (k::scan_tmp_bytes(g.n) > kScanBytes) fail(PPR_ERR_DEVICE, "internal: scan scratch too small");
    const int32_t* deg = g.deg.as<int32_t>();
    auto readback = [&](void* dst, const void* src, size_t bytes) {
        HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ss));
    };

    // ---- local phase: iterations S^(j) pushed simultaneously (every array
    // the phase reads is written first: r and pi by the init kernel, the
    // counters by the memset of each level)
    k::query_init(r, pi, g.n, s, F, ss);
    int64_t nf = 1, vol = g.h_deg[s];
    double r_sum = 1.0;
    const double rmax = lambda / (double)g.m;
    constexpr double kSwitch = 32.0;     // ppr_options_default's switch_param, edge rule
    int32_t levels = 0;
    int64_t edge_pushes = 0;
    int64_t hctr[2] = {0, 0};
    double hsum = 0.0;
    while (nf > 0 && r_sum > lambda && kSwitch * (double)vol <= (double)g.m) {
        int np = 0;
        k::frontier_snapshot(F, (int32_t)nf, deg, alpha, r, pi, y0, reinterpret_cast<int64_t*>(y1), partials, &np,
                             ss);
        k::reduce_sum(partials, np, dsum, ss);
        k::exclusive_scan_i64(reinterpret_cast<int64_t*>(y1), off, nf, scan_tmp, ss);
        HIPCHECK(hipMemsetAsync(ctr, 0, 16, ss));
        k::frontier_push(F, off, (int32_t)nf, vol, g.row_ptr.as<int64_t>(), g.col.as<int32_t>(), deg, y0, rmax, r,
                         Fn, ctr, ss);
        readback(hctr, ctr, 16);
        readback(&hsum, dsum, 8);
        HIPCHECK(hipStreamSynchronize(ss));
        edge_pushes += vol;
        r_sum -= hsum;
        nf = hctr[0];
        vol = hctr[1];
        std::swap(F, Fn);
        ++levels;
    }

    // ---- exact r_sum, y = (1 - alpha) r / d for the first sweep
    {
        int np = 0;
        k::prep_y(r, deg, alpha, g.n, y0, partials, &np, ss);
        k::reduce_sum(partials, np, dsum, ss);
        readback(&hsum, dsum, 8);
        HIPCHECK(hipStreamSynchronize(ss));
        r_sum = hsum;
    }

    // ---- global phase: threshold-0 sweeps contract r_sum by exactly 1 - alpha
    int32_t sweeps = 0;
    constexpr int32_t kMaxSweeps = 4096;   // ppr_options_default's max_sweeps
    if (r_sum > lambda) {
        int32_t K = 0;
        for (double x = r_sum; x > lambda && K < kMaxSweeps; x *= (1.0 - alpha)) ++K;
        const double* yc = y0;
        double* yn = y1;
        auto advance = [&](int flags) {
            k::sweep_f64(g, sch, flags, alpha, yc, yn, pi, r, r, partials, ss);
            double* t = const_cast<double*>(yc);
            yc = yn;
            yn = t;
        };
        if (K == 1) {
            advance(k::SW_ENTRY | k::SW_WRITE_R);
        } else {
            advance(k::SW_ENTRY | k::SW_FOLD);
            for (int32_t i = 0; i < K - 2; ++i) advance(k::SW_FOLD);
            advance(k::SW_WRITE_R);
        }
        sweeps = K;
        k::reduce_sum(partials, k::sweep_parts(sch), dsum, ss);
        readback(&hsum, dsum, 8);
        HIPCHECK(hipStreamSynchronize(ss));
        r_sum = hsum;
        // rounding can leave r_sum a hair above lambda: one more plain sweep each time
        while (r_sum > lambda && sweeps < kMaxSweeps) {
            advance(k::SW_ENTRY | k::SW_WRITE_R);
            ++sweeps;
            k::reduce_sum(partials, k::sweep_parts(sch), dsum, ss);
            readback(&hsum, dsum, 8);
            HIPCHECK(hipStreamSynchronize(ss));
            r_sum = hsum;
        }
    }
    edge_pushes += (int64_t)sweeps * g.m;
    HIPCHECK(hipStreamSynchronize(ss));
    if (st) {
        st->local_levels = levels;
        st->sweeps = sweeps;
        st->refreshes = 0;
        st->source = s;
        st->edge_pushes = edge_pushes;
        st->r_sum = r_sum;
        st->cert_l1 = -1.0;
        st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        st->sweep_ms = -1.0;                 // not timed: timing events would be created here
        st->sweep_launches = sweeps;
        st->batch_cols = 1;
        st->sweep_chunks = 1;
        st->sor_omega = 1.0;
        st->residue_format = PPR_RESIDUE_F32;
        st->push_scans = 0;
        st->sweep_tile_bytes = 0;
        st->refresh_ms = 0.0;
        st->refresh_launches = 0;
        st->reserved = 0;
    }
    if (r_sum > lambda) fail(PPR_ERR_NOT_CONVERGED, "max_sweeps reached before r_sum <= lambda");
}

}  // namespace ppr

extern "C" ppr_status ppr_query_fp64_noalloc(ppr_graph* gh, int32_t s, double alpha, double lambda,
                                             void* hip_stream, double* pi_out, ppr_stats* stats) {
    return ppr::guarded_call([&] {
        ppr::Graph* g = reinterpret_cast<ppr::Graph*>(gh);
        if (!g) ppr::fail(PPR_ERR_ARG, "graph is NULL");
        if (!pi_out) ppr::fail(PPR_ERR_ARG, "pi_out is NULL");
        if (!(alpha > 0.0 && alpha < 1.0)) ppr::fail(PPR_ERR_ARG, "alpha must lie in (0, 1)");
        if (!(lambda > 0.0 && lambda <= 1.0)) ppr::fail(PPR_ERR_ARG, "lambda must lie in (0, 1]");
        if (s < 0 || s >= g->n) ppr::fail(PPR_ERR_ARG, "source " + std::to_string(s) + " is outside [0, n)");
        HIPCHECK(hipSetDevice(g->device));
        if (!ppr::is_device_ptr(pi_out, g->device))
            ppr::fail(PPR_ERR_ARG, "pi_out must be device memory of the graph's device");
        ppr::run_fp64_query_noalloc(*g, s, alpha, lambda, static_cast<hipStream_t>(hip_stream), pi_out, stats);
    });
}
