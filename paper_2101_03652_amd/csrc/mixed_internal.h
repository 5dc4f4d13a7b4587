// Internal declarations of the batched mixed-precision path (n x B block).
#pragma once

#include "ppr_internal.h"

namespace ppr {

namespace mk {
constexpr int kBlock = 256;
constexpr int kLdsBytes = 16384;   // default LDS stage of a sweep block (its row tile)
// Sweep stages the autotuner tries per block width (3, 4 or 6 gathers of 16
// bytes in flight per thread); the smallest bounds the long-row piece count.
constexpr int kTileCount = 3;
constexpr int kTiles[kTileCount] = {12288, 16384, 24576};
constexpr int kMinTile = 12288;
// Persistent grid of the refresh and the conversion (fixed, so that the
// per-column sums come out the same every run).  Block k of the refresh
// takes schedule blocks k, k + G, ...: with G well above the blocks a device
// holds at once, the rows in progress stay close together and a block's
// share is short (refresh at B = 128 on 4M nodes, 70M edges: 9.78 / 9.44 /
// 9.04 / 8.93 / 8.93 ms for G = 2048 / 4096 / 8192 / 16384 / 32768).
constexpr int kGridRed = 16384;
constexpr int kLongRounds = 8;     // edge rounds one sweep block runs on a long row
constexpr int kRefreshRounds = 1 << 20;   // a refresh block runs a long row whole

// Sweep blocks with an L-byte LDS stage: <= kNnz in-edges (C 16-byte vectors
// per row) and <= kRows rows.
template <int C, int L = kLdsBytes>
struct Sw {
    static constexpr int kNnz = L / (16 * C);
    static constexpr int kRows = kBlock / C;
    static constexpr int kItems = kNnz * C / kBlock;   // 3, 4 or 6
    static constexpr int kSlots = kBlock / C;
    static_assert(kItems * kBlock == kNnz * C, "a stage holds a whole number of gathers per thread");
};
// Refresh blocks gather the in-neighbours' stage accumulator rows (16 C bytes
// per edge) through a 32 KB stage per round.
constexpr int kRfLdsBytes = 32768;
template <int C>
struct Rf {
    static constexpr int kNnz = kRfLdsBytes / (16 * C);
    static constexpr int kItems = kNnz * C / kBlock;   // = 8
    static constexpr int kRows = kBlock / C;
};
}  // namespace mk

// Device state of one block of Bw columns on one graph.
struct MixedCtx {
    hipStream_t stream = nullptr;     // work stream: `own`, or the caller's stream while a block uses it
    hipStream_t own = nullptr;        // the context's own stream (created with it; HIP graphs are captured here)
    int32_t n = 0;
    int Bw = 0, shift = 0;
    int chunks = 1;                   // row chunks per sweep (block Gauss-Seidel order when > 1)
    int tile = mk::kLdsBytes;         // LDS stage of a sweep block, one of mk::kTiles
    double alpha = -1.0;              // alpha the scale table holds (the block's reference alpha)
    int64_t fcap = 0;                 // frontier capacity (entries)
    DevBuf r64, pi64;                 // double[n][Bw]  local-phase scratch, zero between uses
    DevBuf F0, F1, X, degF, off;      // frontier (int64 keys), increments, degrees, prefix
    DevBuf scan_tmp;
    DevBuf Y01;                       // Y0 and Y1 back to back (a sweep gathers both at 32-bit offsets)
    DevBuf Y0, Y1;                    // [n][Bw] FP32 or bf16: residue still to push, y = (1-alpha) r / d (views of Y01)
    DevBuf S;                         // double[n][Bw]  reserve (y domain)
    DevBuf AS;                        // double[n][Bw]  sum of S over each node's in-neighbours
    DevBuf T;                         // float[n][Bw]   per-stage reserve accumulator
    DevBuf scale;                     // float[n]       (1-alpha) / d_u
    DevBuf partials;                  // double[kGridRed][Bw]
    DevBuf colsum;                    // double[Bw]
    DevBuf ctr;                       // tail + per-column counts + per-column volumes
    DevBuf taken;                     // double[Bw]
    DevBuf active;                    // uint8[Bw]  local phase: column pushes this level
    DevBuf src;                       // int32[Bw]  source per column (-1: free)
    DevBuf kb;                        // int32[Bw]  sweeps each column runs in this launch sequence
    DevBuf entry;                     // int32[Bw]  1: fold the fresh residue into T on the first sweep,
                                      //            2: the same, restarting T (the refresh moved it into S)
    DevBuf rmask;                     // int32[Bw]  1: refresh writes this column's residue (and S, AS),
                                      //            2: the same, its S and AS taken as 0 (first refresh)
    DevBuf cmask;                     // int32[Bw]  1: conversion writes this column
    DevBuf rmaxb;                     // double[Bw] lambda_b / m: activity threshold per column
    DevBuf step;                      // int32[2]   sweeps done in the current sequence, its last step
    DevBuf stage;                     // double[Bw][n] host-output staging (lazy)
    DevBuf piece_part;                // float[pieces][Bw]: partial sums of long-row pieces
    DevBuf omega;                     // float[Bw]      over-relaxation factor per column
    DevBuf acoef;                     // double[4][Bw]  per column: alpha_b, 1 - alpha_b, 1 / (1 - alpha_b),
                                      //                alpha_b / (1 - alpha_b)
    DevBuf afac;                      // float[Bw]      (1 - alpha_b) / (1 - alpha): the column's factor on
                                      //                the scale table (exactly 1 when alpha_b = alpha)
    bool sor = false;                 // the next sweeps run the over-relaxed update
    bool af = false;                  // the next sweeps apply the per-column alpha factors (afac)
    PinnedBuf host;                   // readback area
    hipGraphExec_t chunk[2] = {nullptr, nullptr};   // captured sweep chunks Y1 -> Y0 -> ... -> Y1
                                                     // (plain, over-relaxed)
    const void* ycur = nullptr;       // buffer holding the current residue rows
    bool bf16 = false;                // residues stored as bf16 (else FP32)
    void drop_chunks();
    ~MixedCtx();
};

MixedCtxPtr mixed_acquire(Graph& g, int Bw, int64_t fcap, bool bf16);
void mixed_release(Graph& g, MixedCtxPtr c);
int64_t frontier_capacity(int32_t n, int64_t m, const ppr_options& opt, int Bw);
size_t mixed_footprint(int32_t n, int64_t m, int Bw, int64_t fcap, bool bf16);

// Launchers (mixed_kernels.hip).  All run on c.stream.
namespace mk {
void set_scale(Graph& g, MixedCtx& c, double alpha);
// r64 = e_s for the columns with cmask = 1
void init_sources(MixedCtx& c);
// per-column alpha: c.acoef
void snapshot(MixedCtx& c, const Graph& g, const int64_t* F, int64_t nf);
// rmax per column: c.rmaxb (lambda_b / m)
void push(MixedCtx& c, const Graph& g, const int64_t* F, int64_t nf, int64_t vol, int64_t* F_next);
// FP64 scratch -> block for the columns with cmask = 1 (others untouched); per-column sums of r -> colsum
void convert(MixedCtx& c, const Graph& g);
// build the graph's sweep and refresh schedules for this width (they allocate,
// so this runs before any stream capture)
void prepare(MixedCtx& c, const Graph& g);
// allocate (zeroed) the state of the over-relaxed sweeps
// one sweep Y_in -> Y_out (budgets kb, entry flags, device step counter), then step += 1
void sweep(MixedCtx& c, const Graph& g, const void* y_in, void* y_out);
// residue block <-> FP32 copy (device memory, count = n * Bw values)
void store_from_f32(MixedCtx& c, const float* src, void* dst, int64_t count);
void store_to_f32(MixedCtx& c, const void* src, float* dst, int64_t count);
// S += T, T = 0; then for columns with rmask = 1 write y~ into `y` (in place);
// per-column sums of |rt| (all columns) -> colsum; rt_out (nullable): column-major FP64 residual
void refresh(MixedCtx& c, const Graph& g, void* y, double* rt_out);
void export_cols(MixedCtx& c, const Graph& g, int b0, int count, double* out);   // out[count][n]
void export_col(MixedCtx& c, const Graph& g, int b, double* out);                // out[n]
}  // namespace mk

}  // namespace ppr
