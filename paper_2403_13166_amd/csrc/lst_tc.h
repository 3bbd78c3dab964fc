// Host-side view of track-candidate selection (lst_tc.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lst.h"

namespace lst {

constexpr int kTcPhiBins = 256;           // phi0 bins per event of the object index
constexpr int kTcEtaBins = 32;            // asinh(cot) bins per event (uniform over +-kTcEtaMax)
constexpr double kTcEtaMax = 2.6;
constexpr int kTcBinsPerEvent = kTcPhiBins * kTcEtaBins;
constexpr int kTcPT5 = 0, kTcT5 = 1, kTcPT3 = 2, kTcPLS = 3, kTcT3 = 4;   // kTcT3: MD list of a T3
constexpr int kTcCounts = 8;              // out counts: kept per kind (0-3), kept, before removal
constexpr int kTcCountKept = 4, kTcCountBefore = 5;

struct TcArgs {
    const float *x, *y, *z;
    const int2 *md_hits, *ls_md, *t3_ls, *t5_t3;
    const float *t5_score, *t5_chi2_rphi;
    int64_t n_md, n_ls, n3, n5;
    const int64_t *ev_obj;                // [4][n_ev + 1] per-event object starts (null: one event)
    int32_t n_ev;
    const float *seeds;                   // [ns][8]
    const int64_t *seed_off;              // [n_ev + 1]
    int64_t ns;
    lst_tc_options opt;
};

struct TcSizes {
    int64_t n_md, n3, n5, ns;
    int32_t n_ev;
};

struct TcWork {
    double4 *par;                         // [n5 + n3] kappa, phi0, cot, z0 (cot NaN: none)
    int32_t *okey;                        // [n5 + n3] (kind, event, phi0 bin) or -1
    uint64_t *obj_best;                   // [n5 + n3] best (chi2, seed) offered
    int32_t *obj_pair;                    // [n5 + n3] paired seed or -1
    int32_t *bin_cnt, *bin_off, *bin_cur; // [2 n_ev kTcBinsPerEvent (+1)] (kind, event, eta bin, phi0 bin)
    int32_t *bin_obj;                     // [n5 + n3] objects by bin
    uint64_t *seed_best;                  // [ns] best (chi2, object) of the current pass
    int32_t *seed_pair, *seed_kind;       // [ns] paired object (T5 or T3 index) or -1, its kind
    float *seed_chi2;                     // [ns] chi2 of the pair (FP32)
    int32_t *t3_used;                     // [n3] T3 of a pT5's T5
    int32_t *c_kind, *c_seed, *c_obj;     // [n5 + n3 + ns] TCs before duplicate removal
    int64_t *c_key;                       //   [2] priority key: quality bits, kind << 32 | object
    int32_t *c_md;                        //   [8] MDs (-1 padded)
    int32_t *c_drop;                      //   removed as a duplicate
    int32_t *md_cnt, *md_cur;             // [n_md] TCs per MD
    int64_t *md_off;                      // [n_md] their list starts
    int32_t *md_tc;                       // [5 (n5 + n3 + ns)] MD -> TC lists
    int64_t *blk;                         // block sums of the compaction scans
    int64_t *n_cand;                      // [1] TCs before duplicate removal
    int64_t *ev_single;                   // [4][2] offsets of a single-event call
    int32_t *out_kind, *out_seed, *out_obj;
    int64_t *out_counts;                  // [kTcCounts]
    int64_t cap_tc;
};

size_t tc_layout(const TcSizes &z, char *base, TcWork *w);
hipError_t run_tc(const TcArgs &a, const TcWork &w, hipStream_t stream);

}  // namespace lst
