// Host-side view of the workspace and the kernel launchers of the LST pipeline.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lst.h"
#include "lst_device.h"

namespace lst {

// Work-item counts used to size grids; they depend only on capacities, never
// on data, so a whole build can be captured into a HIP graph.
constexpr int kBlock = 256;
constexpr int kScanBlocks = 1024;
constexpr int kEvalBlocks = 8192;     // compaction blocks (256 CUs x 32), default
constexpr int kMaxStride = 8192;      // grid cap of grid-stride kernels
constexpr int kMaxRecBytes = 48;      // largest per-candidate record a stage compacts
constexpr int kBinRangesMax = 1024;   // sensor ranges per event in hit binning, at most
constexpr int kBinRangeSensors = 512; // sensor ids of one binning range, at most
constexpr int kBinSplitMax = 256;     // largest tuned count of binning ranges per event
constexpr int kBinTileHits = 4096;     // hits of one binning tile

// Launch shapes (never change results: outputs are in candidate order for any
// tiling). Stage order: MD, LS, T3, T5 pre-cuts, T5 fit.
constexpr int kStages = 5;
// candidates per thread in a 256-thread tile that each stage is compiled for
// (bit v set = value v allowed; values are powers of two)
constexpr int kPerMask[kStages] = {2 | 4 | 8, 2 | 4 | 8, 1 | 2 | 4, 1 | 2 | 4, 1 | 2};
struct Tuning {
    int32_t bin_split;                // sensor ranges (blocks) per event in hit binning, 1..64
    int32_t per[kStages];
    int32_t eval_blocks;              // persistent blocks of the compaction kernels
    int32_t t3_masks;                 // pass masks kept per wavefront in the T3 stage, 1..kT3MaxMasks
};
constexpr int kT3MaxMasks = 8;
constexpr Tuning kDefaultTuning = {4, {4, 8, 2, 2, 1}, kEvalBlocks, kT3MaxMasks};
inline bool tuning_valid(const Tuning &t) {
    if (t.bin_split < 1 || t.bin_split > kBinSplitMax) return false;
    if (t.eval_blocks < 256 || t.eval_blocks > kMaxStride) return false;
    if (t.t3_masks < 1 || t.t3_masks > kT3MaxMasks) return false;
    for (int i = 0; i < kStages; ++i) {
        const int v = t.per[i];
        if (v < 1 || v > 8 || (v & (v - 1)) || !(kPerMask[i] & v)) return false;
    }
    return true;
}

struct Work {
    // capacities
    int64_t cap_hits, cap_ev, cap_md, cap_ls, cap_t3, cap_t5, cap_cand, max_tiles;
    int64_t n_anchor_cap;             // largest anchor count of any stage + 1
    // hits binned by (event, sensor)
    int64_t *bin_off;                 // [cap_ev * n_sens + 1]
    float4 *bin_hit;                  // [cap_hits] x, y, z, input index (bits)
    int64_t max_bin_tiles, max_bin_entries;
    int64_t *bin_tbase;               // [cap_ev + 1] first coarse tile of each event
    int64_t *bin_nent;                // [1] coarse (event, range, tile) entries
    int32_t *bin_cnt;                 // [max_bin_entries] hits per entry
    int64_t *bin_cpos;                // [max_bin_entries + 1] their exclusive scan
    float4 *bin_tmp;                  // [cap_hits] hits partitioned by (event, range)
    int32_t *bin_tsens;               // [cap_hits] their sensor ids
    // per-stage scratch
    int64_t *cand_off;                // [n_anchor_cap + 1]
    int64_t *scan_part;               // [kScanBlocks + 1]
    int32_t *tile_anchor;             // [max_tiles + 1]
    int32_t *tile_cnt;                // [max_tiles] survivors per tile
    int64_t *tile_pre;                // [max_tiles + 1] their exclusive scan
    int64_t *ntiles;                  // [1] tiles of the current stage
    void *rec_scratch;                // [max_tiles * kMinTile] records of kMaxRecBytes
    // MD
    float4 *md_a;                     // [cap_md] anchor x, y, z, global module (bits)
    float2 *md_o;                     // [cap_md] other hit x, y
    float2 *md_rq;                    // [cap_md] radius and resolution term (sign: endcap) for the pair cuts
    int64_t *md_mod_off;              // [cap_ev * n_mod + 1]
    // LS
    int64_t *ls_off;                  // [cap_md + 1] CSR by inner MD (exclusive scan of ls_cnt)
    int32_t *ls_cnt;                  // [cap_md] LS per inner MD
    int4 *ls_chunk;                   // [cap_ls] (A, B, rank of B among A's segments) before placement
    unsigned long long *ls_top;       // [1] records written
    // T3
    int4 *t3_mds;                     // [cap_t3] MDs (A, B, C)
    int32_t *t3_wcnt;                 // [cap_ls / 64 + 1] T3 per wavefront of inner LSs
    int64_t *t3_woff;                 // [cap_ls / 64 + 2] their exclusive scan
    unsigned long long *t3_bits;      // [(cap_ls / 64 + 1) * kT3MaxMasks] pass masks
    int64_t *t3_nw;                   // [1] wavefronts of the build
    int64_t *t3_pos;                  // [cap_ls + 1] first T3 position of every inner LS
    int2 *t3_cn;                      // [cap_ls] candidate range of every inner LS
    int32_t *t3_ovf;                  // [cap_ls / 64 + 1] wavefronts beyond the kept masks
    unsigned long long *t3_n_ovf;     // [1] their number

    int64_t *t3i_off;                 // [cap_md + 1] T3 by inner MD (they are sorted by it)
    // T5
    int64_t cap_t5pre;
    int2 *t5_pre;                     // [cap_t5pre] T3 pairs passing the FP32 cuts
    float *t5_fitf;                   // [cap_t5][8] fit outputs and chi2s of each T5
    int64_t *ev_off;                  // [2] event offsets of a single-event call
};

struct Outputs {
    int2 *md_hits, *ls_md, *t3_ls, *t5_t3;
    float *t5_score, *t5_chi2_rphi, *t5_chi2_rz, *t5_feat;
    int64_t *counts;
};

struct RunArgs {
    GeomDev g;
    CutParams p;
    ModelDev m;
    const float *x, *y, *z;
    const int32_t *sensor;
    int64_t n_hits;
    const int64_t *ev_off;            // device [n_ev + 1]
    int32_t n_ev;
    int32_t mode, precision;
    float score_min;
    int64_t *ev_obj_off;              // device [4][n_ev + 1] or null
    hipEvent_t *timing;               // null, or kTimingEvents events recorded around the stages
    Tuning tune;
    int32_t stop_before;              // 1..kFailStages: enqueue only the stages before this one
};

// Pipeline stages for failure injection: 1 hit binning, 2 MD, 3 LS, 4 T3,
// 5 T5, 6 T5-DNN scoring.
constexpr int32_t kFailStages = 6;

// Timing windows (pairs of events): 0 whole build, 1 binning, 2 MD, 3 LS,
// 4 T3 (2-4: the stage's eval kernel alone), 5 T5 compaction kernels, 6 T5
// features + DNN scoring, then the whole MD, LS and T3 stages (7, 8, 9): for
// MD and T3 the candidate-count scan, eval, tile-count scan, copy and CSR
// fill; for LS the eval, the scan of the per-MD counts and the placement.
constexpr int kTimingWindows = 10;
constexpr int kTimingEvents = 2 * kTimingWindows;

struct GnnDev {
    const uint4 *frag;                // BF16 fragments of every MFMA layer
    int64_t foff[kGnnLayers];         // first fragment of each layer
    const float *bias;                // FP32 biases of every layer
    int64_t boff[kGnnLayers];
    const float *wh2;                 // head output weights [32] (vector ALU)
    float bh2;
};
struct GnnWork {
    float *h0, *h1;                   // [n_nodes][64] node states
    float *e1;                        // [n_edges][64] edge states after step 0
    float *msg;                       // [n_nodes][64] sums of the incoming edge states
    int64_t *in_off;                  // [n_nodes + 1] incoming-edge ranges
    int64_t *err;                     // [1] bit 0: invalid graph
};
hipError_t run_gnn(const GnnDev &m, const float *x, int64_t n_nodes, const int32_t *src, const int32_t *dst,
                   int64_t n_edges, float *score, const GnnWork &w, hipStream_t stream);

// Enqueue the whole object-building pipeline on `stream`.
hipError_t run_pipeline(const RunArgs &a, const Work &w, const Outputs &o, hipStream_t stream);
// Enqueue standalone scoring of n rows (f32 or bf16 input).
hipError_t run_score(const ModelDev &m, const void *X, int dtype, int64_t n, float *out,
                     int precision, hipStream_t stream);
// Fill a two-entry event-offset array {0, n} on the device.
hipError_t set_single_event(int64_t *ev_off, int64_t n, hipStream_t stream);

}  // namespace lst
