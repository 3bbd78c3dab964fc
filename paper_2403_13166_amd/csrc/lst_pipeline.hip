// LST object-building pipeline on gfx950: hit binning, mini-doublets, line
// segments, triplets, quintuplets (paper Table 1 steps 1-4), each stage one
// compaction kernel over its candidate pairs.
//
// Every stage has the same shape:
//   * anchors (a module for MD and LS, the inner LS for T3, the inner T3 for
//     T5) own a contiguous
//     range of candidate pairs (left list x right list); a device-wide
//     exclusive scan of the per-anchor counts gives the ranges and, for every
//     tile of candidates, the anchor its first candidate belongs to;
//   * an eval kernel walks the tiles (grid-stride). The block first stages the
//     tile's window of anchor offsets and per-anchor list bases in LDS (for
//     LS also the module-map tables of those modules), so decoding a
//     candidate into its (left, right) pair is LDS work; each thread then
//     applies the cuts to kPer candidates and the block compacts the
//     survivors with wavefront ballots into the tile's scratch slot. No block
//     ever waits for another: a scan of the tile counts and a copy kernel
//     place the survivors. Output is in candidate order (deterministic)
//     without per-object global atomics;
//   * CSR offsets the next stage needs are filled from the sorted outputs.
// Grid shapes depend only on capacities, never on data, so a whole build can be
// captured into a HIP graph.
#include <hip/hip_runtime.h>

#include "lst_internal.h"
#include "lst_mlp_tile.h"

namespace lst {

// ------------------------------------------------------------- utilities

__device__ __forceinline__ int64_t grid_tid() {
    return (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
}
__device__ __forceinline__ int64_t grid_stride() { return (int64_t)gridDim.x * blockDim.x; }

__device__ __forceinline__ int64_t dev_count(const int64_t *p, int64_t cap) {
    int64_t v = *p;
    return v < cap ? v : cap;
}

static inline int grid_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > kMaxStride) g = kMaxStride;
    return (int)g;
}

// XCD-aware tile walk. Workgroups are dispatched round-robin over the 8
// accelerator dies (XCDs), each with its own L2; neighbouring tiles share
// their inputs (MDs of adjacent modules, the same event's hits), so each XCD
// takes one contiguous range of tiles and its blocks stride through it. With
// a grid that is not a multiple of 8 this is a plain grid-stride walk.
constexpr int kXcds = 8;
struct TileWalk {
    int64_t first, end, step;
    __device__ TileWalk(int64_t ntiles) {
        if (gridDim.x % kXcds == 0) {
            const int64_t x = blockIdx.x % kXcds, per = gridDim.x / kXcds;
            const int64_t chunk = (ntiles + kXcds - 1) / kXcds;
            const int64_t t0 = x * chunk;
            first = t0 + blockIdx.x / kXcds;
            end = t0 + chunk < ntiles ? t0 + chunk : ntiles;
            step = per;
        } else {
            first = blockIdx.x;
            end = ntiles;
            step = gridDim.x;
        }
    }
};

static inline int round_up_xcd(int nb) { return nb < kXcds ? nb : (nb + kXcds - 1) / kXcds * kXcds; }

__global__ void k_fill_i32_dev(int32_t *p, const int64_t *n_dev, int64_t cap, int32_t v) {
    int64_t n = dev_count(n_dev, cap);
    for (int64_t i = grid_tid(); i < n; i += grid_stride()) p[i] = v;
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
    for (int64_t i = grid_tid(); i < n; i += grid_stride()) p[i] = v;
}

__global__ void k_set_single_event(int64_t *ev, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) { ev[0] = 0; ev[1] = n; }
}

// wave64 inclusive scan of a 64-bit value
__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// block (256 threads) inclusive scan; returns inclusive value, total in *tot
__device__ __forceinline__ int64_t block_incl_scan(int64_t v, int64_t *tot) {
    __shared__ int64_t s_w[kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan(v);
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    int64_t off = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) {
        if (k < wv) off += s_w[k];
        all += s_w[k];
    }
    __syncthreads();
    *tot = all;
    return inc + off;
}

// ------------------------------------------------------------------ scan
// Exclusive scan of count(i), i < n (n from device or host), into out[0..n],
// out[n] = total. With tile_anchor != null also records, for every tile of
// `tile` scanned positions, the index i whose range holds the tile's start.

template <class F>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(F f, const int64_t *n_dev, int64_t n_cap,
                                                        int64_t *part) {
    int64_t n = n_dev ? dev_count(n_dev, n_cap) : n_cap;
    int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
    int64_t s = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kBlock) s += f(i);
    int64_t tot;
    block_incl_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <class F>
__global__ __launch_bounds__(kBlock) void k_scan_down(F f, const int64_t *n_dev, int64_t n_cap,
                                                      const int64_t *part, int64_t *out,
                                                      int32_t *tile_anchor, int64_t max_tiles, int tile) {
    int64_t n = n_dev ? dev_count(n_dev, n_cap) : n_cap;
    int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
    // this block's offset: the sum of the totals of the blocks before it (and,
    // for the last block, the grand total)
    int64_t pre = 0, all = 0;
    for (int k = threadIdx.x; k < (int)gridDim.x; k += kBlock) {
        const int64_t v = part[k];
        all += v;
        if (k < (int)blockIdx.x) pre += v;
    }
    int64_t pre_tot, all_tot;
    block_incl_scan(pre, &pre_tot);
    block_incl_scan(all, &all_tot);
    int64_t run = pre_tot;
    for (int64_t base = b0; base < b1; base += kBlock) {
        int64_t i = base + threadIdx.x;
        int64_t c = i < b1 ? f(i) : 0;
        int64_t tot;
        int64_t inc = block_incl_scan(c, &tot);
        int64_t o = run + inc - c;
        if (i < b1) {
            out[i] = o;
            if (tile_anchor && c > 0) {
                int64_t t0 = (o + tile - 1) / tile, t1 = (o + c - 1) / tile;
                for (int64_t t = t0; t <= t1 && t < max_tiles; ++t) tile_anchor[t] = (int32_t)i;
            }
        }
        run += tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = all_tot;
}

template <class F>
static void scan(F f, const int64_t *n_dev, int64_t n_cap, const Work &w, int64_t *out,
                 int32_t *tile_anchor, hipStream_t st, int tile = 256) {
    int nb = (int)((n_cap + kBlock - 1) / kBlock);
    if (nb < 1) nb = 1;
    if (nb > kScanBlocks) nb = kScanBlocks;
    hipLaunchKernelGGL(k_scan_reduce<F>, dim3(nb), dim3(kBlock), 0, st, f, n_dev, n_cap, w.scan_part);
    hipLaunchKernelGGL(k_scan_down<F>, dim3(nb), dim3(kBlock), 0, st, f, n_dev, n_cap, w.scan_part,
                       out, tile_anchor, w.max_tiles, tile);
}

// ------------------------------------------------ compaction (one stage)

struct CntF {
    const int32_t *c;
    __device__ int64_t operator()(int64_t i) const { return c[i]; }
};

// LDS of one tile: the anchor offsets and per-anchor list bases of the tile's
// window (at most kWin anchors), and (LS only) the module-map tables of the
// window's modules.
template <int kEnt, int kWin>
struct TileLds {
    int64_t off[kWin + 1];
    int32_t info[kWin][4];
    int32_t ebase[kEnt > 0 ? kWin : 1];   // first table entry of each window anchor
    int32_t ek0[kEnt > 0 ? kWin : 1];     // its first module-map entry
    int32_t ent_rp[kEnt > 0 ? kEnt : 1];
    int32_t ent_md[kEnt > 0 ? kEnt : 1];  // first MD of the entry's target, bit 31: endcap target
};

// Two-phase stages split their cuts: phase 1 runs on every candidate, and the
// survivors of each wavefront are queued in LDS, so that phase 2 (the costlier
// remainder of the cuts) runs on dense batches of 64 instead of wave-wide on
// every sub-round. Results return to the candidate's slot, so the outcome and
// the output order are those of a single-phase evaluation.
constexpr int kQCap = 128;            // queued survivors per wavefront (flushed at 64)

template <class S, int kPer, bool kOn>
struct PhaseQ { };
template <class S, int kPer>
struct PhaseQ<S, kPer, true> {
    typename S::Mid e[kBlock / 64][kQCap];     // phase-1 survivors
    uint16_t slot[kBlock / 64][kQCap];
    uint8_t res[kBlock / 64][kPer * 64];       // outcome of phase 2, per slot
};

// copy of a record of whole 32-bit words (keeps LDS <-> register copies out of
// private memory)
template <class T>
__device__ __forceinline__ void copy_words(T &dst, const T &src) {
    static_assert(sizeof(T) % 4 == 0, "records are whole words");
    const uint32_t *ps = reinterpret_cast<const uint32_t *>(&src);
    uint32_t *pd = reinterpret_cast<uint32_t *>(&dst);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) pd[k] = ps[k];
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// run phase 2 on queue entries [0, n) (n <= 64), then move entries [n, qn) to the front
template <class S, class Q>
__device__ __forceinline__ void phase2_flush(const S &st, Q &q, int wv, int lane, int n, int qn) {
    wave_sync_lds();
    if (lane < n) q.res[wv][q.slot[wv][lane]] = st.eval2(q.e[wv][lane]) ? 1 : 0;
    const int rest = qn - n;
    if (rest > 0) {                    // wavefront-uniform
        wave_sync_lds();
        const int src = n + (lane < rest ? lane : 0);
        typename S::Mid te;
        copy_words(te, q.e[wv][src]);
        const uint16_t ts = q.slot[wv][src];
        wave_sync_lds();
        if (lane < rest) {
            copy_words(q.e[wv][lane], te);
            q.slot[wv][lane] = ts;
        }
    }
    wave_sync_lds();
}

// Compaction of one stage in three steps, none of which waits on another
// block: (1) the eval kernel takes tiles of kBlock * kPer candidates
// (grid-stride), stages the tile's anchor window in LDS, applies the cuts and
// compacts each tile's survivors, in candidate order, into that tile's slot of
// a scratch buffer, with the tile's count; (2) an exclusive scan of the tile
// counts gives every tile its output offset; (3) a copy kernel moves each
// tile's survivors to their final position. Output order = candidate order.
template <class S, int kPer>
__global__ __launch_bounds__(kBlock, S::kMinBlocks) void k_stage_eval(S st, const int64_t *cand_off,
                                                       const int64_t *n_dev, int64_t n_cap,
                                                       const int32_t *tile_anchor, int64_t max_tiles,
                                                       int32_t *tile_cnt, typename S::Rec *scratch,
                                                       int64_t *ntiles_out, int64_t *counts, int64_t cap_cand) {
    constexpr int kWaves = kBlock / 64;
    constexpr int kTileC = kBlock * kPer;
    constexpr int kSeg = kPer * kWaves;     // output segments, in candidate order
    constexpr int kWin = S::kWin;
    __shared__ TileLds<S::kEnt, (S::kUnitCount ? 1 : S::kWin)> L;
    __shared__ int s_cnt[kSeg];
    __shared__ PhaseQ<S, kPer, (S::kPhases > 1)> Q;
    __shared__ uint16_t s_anc[S::kUnitCount ? 1 : kTileC];   // window anchor of each tile candidate
    __shared__ int s_wmax[kWaves];
    const int64_t na = n_dev ? dev_count(n_dev, n_cap) : n_cap;
    // unit-count stages: candidate g is anchor g (no offsets, no decode)
    const int64_t total = S::kUnitCount ? na : cand_off[na];
    int64_t ntiles = (total + kTileC - 1) / kTileC;
    // max_tiles counts tiles of kMinTile candidates (the scratch size)
    const int64_t max_t = max_tiles * kMinTile / kTileC;
    if (ntiles > max_t) ntiles = max_t;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *ntiles_out = ntiles;
        atomicMax((unsigned long long *)&counts[LST_COUNT_MAXCAND], (unsigned long long)total);
        if (total > cap_cand) atomicOr((unsigned long long *)&counts[LST_COUNT_ERR], 2ull);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const TileWalk walk(ntiles);
    // a tile's first and last anchors, read as uniform scalar loads (the tile
    // anchors are read-only here); the next tile's are fetched a tile ahead
    auto tile_lo = [&](int64_t t) -> int64_t { return ld_scalar(tile_anchor + t); };
    auto tile_hi = [&](int64_t t) -> int64_t { return t + 1 < ntiles ? tile_lo(t + 1) : na - 1; };
    int64_t alo_n = 0, ahi_n = 0;
    if constexpr (!S::kUnitCount)
        if (walk.first < walk.end) { alo_n = tile_lo(walk.first); ahi_n = tile_hi(walk.first); }
    for (int64_t tile = walk.first; tile < walk.end; tile += walk.step) {
        const int64_t alo = alo_n, ahi = ahi_n;
        if constexpr (!S::kUnitCount)
            if (tile + walk.step < walk.end) { alo_n = tile_lo(tile + walk.step); ahi_n = tile_hi(tile + walk.step); }
        const int nw = (int)(ahi - alo + 1 < (int64_t)kWin + 1 ? ahi - alo + 1 : (int64_t)kWin + 1);
        const bool staged = !S::kUnitCount && nw <= kWin;
        if constexpr (!S::kUnitCount) {
            if (staged) {
                for (int i = threadIdx.x; i <= nw; i += kBlock) {
                    L.off[i] = cand_off[alo + i];
                    if (i < nw) st.info(alo + i, L.info[i]);
                }
                for (int q = threadIdx.x; q < kTileC; q += kBlock) s_anc[q] = 0;
                __syncthreads();
                // anchor map: each non-empty window anchor marks its first
                // candidate in the tile; a running maximum then gives every
                // candidate the last anchor that starts at or before it
                const int64_t g0 = tile * kTileC;
                for (int w = threadIdx.x; w < nw; w += kBlock) {
                    const int64_t o = L.off[w];
                    if (L.off[w + 1] > o && o > g0 && o < g0 + kTileC) s_anc[o - g0] = (uint16_t)w;
                }
                __syncthreads();
                int v[kPer], m = 0;
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    const int a = s_anc[threadIdx.x * kPer + k];
                    m = a > m ? a : m;
                    v[k] = m;
                }
                int incl = m;               // inclusive running maximum over the wavefront
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int o = __shfl_up(incl, d, 64);
                    if (lane >= d && o > incl) incl = o;
                }
                if (lane == 63) s_wmax[wv] = incl;
                int carry = __shfl_up(incl, 1, 64);
                if (lane == 0) carry = 0;
                __syncthreads();
                for (int k = 0; k < wv; ++k) carry = s_wmax[k] > carry ? s_wmax[k] : carry;
#pragma unroll
                for (int k = 0; k < kPer; ++k) s_anc[threadIdx.x * kPer + k] = (uint16_t)(v[k] > carry ? v[k] : carry);
                __syncthreads();
                st.prepare(L, alo, nw);
            }
        }
        // candidate g = tile * kTileC + i * kBlock + tid: each sub-round i is a
        // contiguous run of kBlock candidates (coalesced reads)
        typename S::Rec rec[kPer];
        bool pass[kPer];
        int64_t glo = alo;           // anchor index (global search)
        int qn = 0;                  // queued phase-2 entries of this wavefront
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int64_t g = tile * kTileC + i * kBlock + threadIdx.x;
            pass[i] = false;
            typename S::Mid mid_i;
            if (g < total) {
                if constexpr (S::kUnitCount) {
                    int32_t f[4];
                    st.info(g, f);
                    pass[i] = st.eval(g, 0, f, L, rec[i], mid_i);
                } else if (staged) {
                    const int wlo = s_anc[i * kBlock + threadIdx.x];
                    pass[i] = st.eval(alo + wlo, (int32_t)(g - L.off[wlo]), L.info[wlo], L, rec[i], mid_i);
                } else {
                    int64_t hi = ahi + 1;
                    while (hi - glo > 1) {
                        int64_t mid = (glo + hi) >> 1;
                        if (cand_off[mid] <= g) glo = mid; else hi = mid;
                    }
                    int32_t f[4];
                    st.info(glo, f);
                    f[2] = S::kEnt > 0 ? -1 : f[2];
                    pass[i] = st.eval(glo, (int32_t)(g - cand_off[glo]), f, L, rec[i], mid_i);
                }
            }
            if constexpr (S::kPhases > 1) {
                const unsigned long long m = __ballot(pass[i]);
                const int rk = __popcll(m & ((1ull << lane) - 1ull));
                if (pass[i]) {
                    copy_words(Q.e[wv][qn + rk], mid_i);
                    Q.slot[wv][qn + rk] = (uint16_t)(i * 64 + lane);
                }
                qn += __popcll(m);
                if (qn >= 64) {
                    phase2_flush(st, Q, wv, lane, 64, qn);
                    qn -= 64;
                }
            }
        }
        if constexpr (S::kPhases > 1) {
            if (qn > 0) phase2_flush(st, Q, wv, lane, qn, qn);
#pragma unroll
            for (int i = 0; i < kPer; ++i)
                if (pass[i]) pass[i] = Q.res[wv][i * 64 + lane] != 0;
        }
        int rank[kPer];
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const unsigned long long m = __ballot(pass[i]);
            rank[i] = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) s_cnt[i * kWaves + wv] = __popcll(m);
        }
        __syncthreads();
        // segment offsets: every wavefront scans the kSeg (<= 64) counts itself
        static_assert(kSeg <= 64, "one wavefront scans the segment counts");
        const int cseg = lane < kSeg ? s_cnt[lane] : 0;
        int incl = cseg;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        const int excl = incl - cseg, tcnt = __shfl(incl, kSeg - 1, 64);
        typename S::Rec *slot = scratch + tile * kTileC;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int off = __shfl(excl, i * kWaves + wv, 64);
            if (pass[i]) slot[off + rank[i]] = rec[i];
        }
        if (threadIdx.x == 0) tile_cnt[tile] = tcnt;
        __syncthreads();
    }
}

template <class S, int kPer>
__global__ __launch_bounds__(kBlock) void k_stage_copy(S st, const typename S::Rec *scratch,
                                                       const int32_t *tile_cnt, const int64_t *tile_pre,
                                                       const int64_t *ntiles_dev, int64_t *out_count,
                                                       int64_t cap_out) {
    constexpr int kTileC = kBlock * kPer;
    const int64_t ntiles = *ntiles_dev;
    if (blockIdx.x == 0 && threadIdx.x == 0) *out_count = tile_pre[ntiles];
    const TileWalk walk(ntiles);
    // a tile's count and output base as uniform scalar loads, one tile ahead
    auto cnt_of = [&](int64_t t) -> int { return ld_scalar(tile_cnt + t); };
    auto pre_of = [&](int64_t t) -> int64_t { return ld_scalar(tile_pre + t); };
    int n_n = 0;
    int64_t base_n = 0;
    if (walk.first < walk.end) { n_n = cnt_of(walk.first); base_n = pre_of(walk.first); }
    for (int64_t tile = walk.first; tile < walk.end; tile += walk.step) {
        const int n = n_n;
        const int64_t base = base_n;
        if (tile + walk.step < walk.end) { n_n = cnt_of(tile + walk.step); base_n = pre_of(tile + walk.step); }
        const typename S::Rec *slot = scratch + tile * kTileC;
        for (int i = threadIdx.x; i < n; i += kBlock) {
            const int64_t pos = base + i;
            if (pos < cap_out) st.write(pos, slot[i]);
        }
    }
}

template <class S>
struct StageCount {
    S s;
    __device__ int64_t operator()(int64_t a) const { return s.count(a); }
};

static inline void mark(hipEvent_t *ev, int k, hipStream_t st) {
    if (ev) (void)hipEventRecord(ev[k], st);
}

template <class S, int kPer>
static void run_stage_p(const S &s, const int64_t *n_dev, int64_t n_cap, const Work &w, int64_t *out_count,
                        int64_t cap_out, int64_t *counts, hipStream_t st, hipEvent_t *ev, int win,
                        int eval_blocks) {
    static_assert(sizeof(typename S::Rec) <= kMaxRecBytes, "scratch record too large");
    static_assert((kPerMask[S::kStage] & kPer) != 0, "tile size not offered for this stage");
    const int tile = kBlock * kPer;
    if constexpr (!S::kUnitCount) scan(StageCount<S>{s}, n_dev, n_cap, w, w.cand_off, w.tile_anchor, st, tile);
    int nb = (int)(w.max_tiles < eval_blocks ? w.max_tiles : eval_blocks);
    if (nb < 1) nb = 1;
    nb = round_up_xcd(nb);
    typename S::Rec *scratch = (typename S::Rec *)w.rec_scratch;
    mark(ev, 2 * win, st);
    hipLaunchKernelGGL((k_stage_eval<S, kPer>), dim3(nb), dim3(kBlock), 0, st, s, w.cand_off, n_dev, n_cap,
                       w.tile_anchor, w.max_tiles, w.tile_cnt, scratch, w.ntiles, counts, w.cap_cand);
    mark(ev, 2 * win + 1, st);
    scan(CntF{w.tile_cnt}, w.ntiles, w.max_tiles, w, w.tile_pre, nullptr, st);
    hipLaunchKernelGGL((k_stage_copy<S, kPer>), dim3(nb), dim3(kBlock), 0, st, s, scratch, w.tile_cnt, w.tile_pre,
                       w.ntiles, out_count, cap_out);
}

// Run a stage with the tile size chosen at run time among those compiled for
// it (the host validated `per` against kPerMask).
template <class S>
static void run_stage(const S &s, const int64_t *n_dev, int64_t n_cap, const Work &w, int64_t *out_count,
                      int64_t cap_out, int64_t *counts, hipStream_t st, hipEvent_t *ev, int win,
                      const Tuning &tn) {
    constexpr int m = kPerMask[S::kStage];
    const int per = tn.per[S::kStage], nb = tn.eval_blocks;
    if constexpr ((m & 1) != 0) if (per == 1) return run_stage_p<S, 1>(s, n_dev, n_cap, w, out_count, cap_out, counts, st, ev, win, nb);
    if constexpr ((m & 2) != 0) if (per == 2) return run_stage_p<S, 2>(s, n_dev, n_cap, w, out_count, cap_out, counts, st, ev, win, nb);
    if constexpr ((m & 4) != 0) if (per == 4) return run_stage_p<S, 4>(s, n_dev, n_cap, w, out_count, cap_out, counts, st, ev, win, nb);
    if constexpr ((m & 8) != 0) if (per == 8) return run_stage_p<S, 8>(s, n_dev, n_cap, w, out_count, cap_out, counts, st, ev, win, nb);
}

// ------------------------------------------------------------- binning
// Hits are sorted by (event, sensor), and by input index within a sensor, in
// two deterministic passes without device-wide atomics.
//  * Coarse pass: each event's hits are cut into tiles of kBinTile; a tile
//    counts its hits per sensor range (ranges of at most kFineRange sensor
//    ids); an exclusive scan over (event, range, tile) gives every tile's
//    output base per range; the tile then scatters its hits, each ranked
//    among the tile's earlier hits of its range, so each range keeps the
//    input order.
//  * Fine pass: one block per (event, range) ranks that range's hits by
//    sensor the same way, writes the bin offsets and moves every hit to its
//    binned position.
// Ranks come from ballots: the lanes holding the same key are found with one
// ballot per key bit, and per-wavefront running counters in LDS carry the
// count of earlier rounds, so the order within a key is the input order
// without atomics or sorting.
// Hits with an out-of-range sensor id set error bit 0 and are dropped.

constexpr int kBinTile = kBinTileHits;  // hits of one coarse tile
constexpr int kBinThreads = 256;        // threads of a coarse count block
constexpr int kScatterThreads = 512;    // threads of a coarse scatter block: eight wavefronts of 512 hits
constexpr int kFineRange = kBinRangeSensors;   // sensor ids of one range, at most
constexpr int kMaxRanges = kBinRangesMax;
constexpr int kFineThreads = 512;       // threads of a fine-pass block
constexpr int kFineSrcCap = 12224;      // hits of a range gathered through LDS (16-bit indices; four blocks fit one CU's LDS)

// q = v / d for 0 <= v < 2^24, d >= 1: FP32 reciprocal estimate, made exact
__device__ __forceinline__ int div_small(int v, int d, float inv) {
    int q = (int)((float)v * inv);
    int r = v - q * d;
    while (r < 0) { --q; r += d; }
    while (r >= d) { ++q; r -= d; }
    return q;
}

// tbase[e] = first coarse tile of event e; tbase[n_ev] = all tiles; *nent = tiles * nr
__global__ __launch_bounds__(1024) void k_bin_tiles(const int64_t *ev_off, int n_ev, int nr, int64_t *tbase,
                                                    int64_t *nent) {
    __shared__ int64_t s_w[16];
    __shared__ int64_t s_carry;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < n_ev; base += 1024) {
        const int e = base + threadIdx.x;
        const int64_t v = e < n_ev ? (ev_off[e + 1] - ev_off[e] + kBinTile - 1) / kBinTile : 0;
        const int64_t inc = wave_incl_scan(v);
        if (lane == 63) s_w[wv] = inc;
        __syncthreads();
        int64_t off = 0, all = 0;
        for (int k = 0; k < 16; ++k) { if (k < wv) off += s_w[k]; all += s_w[k]; }
        if (e < n_ev) tbase[e] = s_carry + off + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) s_carry += all;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tbase[n_ev] = s_carry;
        *nent = s_carry * nr;
    }
}

// block -> (event, tile of that event); false past the last tile
__device__ __forceinline__ bool bin_tile_of(const int64_t *tbase, int n_ev, int &e, int64_t &t, int64_t &nt) {
    const int64_t b = blockIdx.x;
    if (b >= ld_scalar(tbase + n_ev)) return false;
    int lo = 0, hi = n_ev;                       // largest e with tbase[e] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ld_scalar(tbase + mid) <= b) lo = mid; else hi = mid;
    }
    e = lo;
    const int64_t t0 = ld_scalar(tbase + e);
    t = b - t0;
    nt = ld_scalar(tbase + e + 1) - t0;
    return true;
}

__global__ __launch_bounds__(kBinThreads) void k_bin_count(const int32_t *sensor, const int64_t *ev_off, int n_ev,
                                                           int n_sens, int nr, int rw, const int64_t *tbase,
                                                           int32_t *cnt, int64_t *counts) {
    __shared__ int32_t s_c[kMaxRanges];
    int e;
    int64_t t, nt;
    if (!bin_tile_of(tbase, n_ev, e, t, nt)) return;
    const int64_t h0 = ld_scalar(ev_off + e) + t * kBinTile, he = ld_scalar(ev_off + e + 1);
    const int64_t h1 = h0 + kBinTile < he ? h0 + kBinTile : he;
    for (int r = threadIdx.x; r < nr; r += kBinThreads) s_c[r] = 0;
    __syncthreads();
    const float inv = 1.0f / (float)rw;
    bool bad = false;
    constexpr int kU = kBinTile / kBinThreads;      // all of the tile's loads in flight
    int sv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int64_t h = h0 + threadIdx.x + (int64_t)u * kBinThreads;
        sv[u] = h < h1 ? sensor[h] : 0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int64_t h = h0 + threadIdx.x + (int64_t)u * kBinThreads;
        if (h >= h1) continue;
        const int v = sv[u];
        if (v < 0 || v >= n_sens) { bad = true; continue; }
        atomicAdd(&s_c[div_small(v, rw, inv)], 1);
    }
    if (bad) atomicOr((unsigned long long *)&counts[LST_COUNT_ERR], 1ull);
    __syncthreads();
    const int64_t base = tbase[e] * nr + t;
    for (int r = threadIdx.x; r < nr; r += kBinThreads) cnt[base + (int64_t)r * nt] = s_c[r];
}

// Lanes of the wavefront whose key equals this lane's key (key in [0, 2^nbits),
// valid lanes only): one ballot per key bit.
__device__ __forceinline__ unsigned long long match_key(int key, bool valid, int nbits) {
    unsigned long long m = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (key >> b) & 1;
        const unsigned long long bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// Stable rank of this lane's key among the wavefront's earlier keys, counting
// the earlier rounds through the wavefront's running counters wc[key]. Every
// lane of the wavefront calls it (uniform control flow).
__device__ __forceinline__ int wave_rank(int32_t *wc, int key, bool valid, int nbits) {
    const int lane = threadIdx.x & 63;
    const unsigned long long m = match_key(key, valid, nbits);
    const unsigned long long below = m & ((1ull << lane) - 1ull);
    const int prev = valid ? wc[key] : 0;
    wave_sync_lds();
    if (valid && below == 0) wc[key] = prev + __popcll(m);   // the group's first lane
    wave_sync_lds();
    return prev + __popcll(below);
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));   // native vector (copies stay in registers)

__device__ __forceinline__ int key_bits(int n) { return n > 1 ? 32 - __clz(n - 1) : 0; }

// Wait for every outstanding vector-memory access of this wavefront. Stores
// count in the same counter as loads; after a branch the compiler can lose
// track of which loads are done and then waits for all, including the stores
// just issued, before each later use of a loaded value. Waiting once for the
// loads of a batch before its stores avoids that serialisation.
__device__ __forceinline__ void vmem_wait_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }   // vmcnt(0)

// Coarse pass: wavefront w of a tile takes the tile's hits [w * 512, (w + 1) * 512)
// in 8 rounds of 64, all loaded up front, and ranks each hit among the
// wavefront's hits of the same range (running counters per wavefront); the
// wavefronts' counts then give every hit its position in input order.
__global__ __launch_bounds__(kScatterThreads) void k_bin_scatter(const float *x, const float *y, const float *z,
                                                             const int32_t *sensor, const int64_t *ev_off, int n_ev,
                                                             int n_sens, int nr, int rw, const int64_t *tbase,
                                                             const int64_t *cpos, float4 *tmp, int32_t *tsens) {
    constexpr int kWaves = kScatterThreads / 64;
    constexpr int kRounds = kBinTile / kScatterThreads;
    __shared__ int64_t s_base[kMaxRanges];
    __shared__ int32_t s_wc[kWaves][kMaxRanges];
    int e;
    int64_t t, nt;
    if (!bin_tile_of(tbase, n_ev, e, t, nt)) return;
    const int64_t h0 = ld_scalar(ev_off + e) + t * kBinTile, he = ld_scalar(ev_off + e + 1);
    const int64_t h1 = h0 + kBinTile < he ? h0 + kBinTile : he;
    const int64_t ebase = tbase[e] * nr + t;
    for (int r = threadIdx.x; r < nr; r += kScatterThreads) {
        s_base[r] = cpos[ebase + (int64_t)r * nt];
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s_wc[w][r] = 0;
    }
    const float inv = 1.0f / (float)rw;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nbits = key_bits(nr);
    const int64_t hw = h0 + (int64_t)wv * (kRounds * 64) + lane;
    int sv[kRounds];
    float4 hv[kRounds];
#pragma unroll
    for (int j = 0; j < kRounds; ++j) {
        const int64_t h = hw + j * 64;
        sv[j] = -1;
        if (h < h1) {
            sv[j] = sensor[h];
            hv[j] = make_float4(x[h], y[h], z[h], __int_as_float((int)h));
        }
    }
    __syncthreads();
    int dr[kRounds];           // range << 16 | rank within the wavefront's hits of that range
#pragma unroll
    for (int j = 0; j < kRounds; ++j) {
        const bool ok = sv[j] >= 0 && sv[j] < n_sens;
        const int d = ok ? div_small(sv[j], rw, inv) : 0;
        const int rk = wave_rank(s_wc[wv], d, ok, nbits);
        dr[j] = ok ? (d << 16) | rk : -1;
    }
    __syncthreads();
    // exclusive prefix over the wavefronts, per range
    for (int r = threadIdx.x; r < nr; r += kScatterThreads) {
        int run = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const int c = s_wc[w][r];
            s_wc[w][r] = run;
            run += c;
        }
    }
    __syncthreads();
    vmem_wait_all();
#pragma unroll
    for (int j = 0; j < kRounds; ++j) {
        if (dr[j] < 0) continue;
        const int d = dr[j] >> 16;
        const int64_t pos = s_base[d] + s_wc[wv][d] + (dr[j] & 0xffff);
        tmp[pos] = hv[j];
        tsens[pos] = sv[j];
    }
}

// Fine pass, one block per (event, range): wavefront w takes the range's hits
// [w * chunk, (w + 1) * chunk) and counts them per sensor (counters per
// wavefront and sensor); per sensor, the counts of the wavefronts give their
// offsets and the sensor totals the bin offsets, which turn the counters into
// output cursors; ranking the same hits in order then yields each hit's
// binned position directly.
__global__ __launch_bounds__(kFineThreads) void k_bin_fine(const float4 *tmp, const int32_t *tsens, const int64_t *tbase,
                                                          const int64_t *cpos, const int64_t *nent, int n_ev, int n_sens,
                                                          int nr, int rw, int xcd_map, int64_t *bin_off, float4 *bin_hit) {
    constexpr int kW = kFineThreads / 64;
    __shared__ int32_t s_wc[kW][kFineRange];
    __shared__ uint16_t s_src[kFineSrcCap];
    __shared__ int64_t s_w[kW];
    int e, r;
    if (xcd_map) {
        const int xx = blockIdx.x % kXcds, k = blockIdx.x / kXcds;
        e = (k / nr) * kXcds + xx;
        r = k % nr;
        if (e >= n_ev) return;
    } else {
        e = blockIdx.x / nr;
        r = blockIdx.x - e * nr;
    }
    const int64_t tb = ld_scalar(tbase + e), nt = ld_scalar(tbase + e + 1) - tb;
    const int64_t cs = ld_scalar(cpos + tb * nr + (int64_t)r * nt), ce = ld_scalar(cpos + tb * nr + (int64_t)(r + 1) * nt);
    const int64_t cnt = ce - cs;
    const int lo = r * rw < n_sens ? r * rw : n_sens;
    const int hi = lo + rw < n_sens ? lo + rw : n_sens;
    const int nb = hi - lo;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < nb; k += kFineThreads)
#pragma unroll
        for (int w = 0; w < kW; ++w) s_wc[w][k] = 0;
    __syncthreads();
    const int64_t chunk = (cnt + kW * 64 - 1) / (kW * 64) * 64;
    const int64_t j0 = wv * chunk, j1 = j0 + chunk < cnt ? j0 + chunk : cnt;
    const int nbits = key_bits(nb);
    constexpr int kFU = 4;                           // rounds loaded ahead
    for (int64_t jb = j0; jb < j1; jb += 64 * kFU) {
        // loads from a clamped index, so none sits behind a branch (each
        // would then be waited for on its own)
        int kv[kFU];
#pragma unroll
        for (int u = 0; u < kFU; ++u) {
            const int64_t j = jb + u * 64 + lane;
            kv[u] = tsens[cs + (j < j1 ? j : j1 - 1)];
        }
#pragma unroll
        for (int u = 0; u < kFU; ++u) kv[u] = jb + u * 64 + lane < j1 ? kv[u] - lo : -1;
        // counts only: their order does not matter
#pragma unroll
        for (int u = 0; u < kFU; ++u)
            if (kv[u] >= 0) atomicAdd(&s_wc[wv][kv[u]], 1);
    }
    __syncthreads();
    // per sensor: the wavefronts' offsets, then the sensors' exclusive scan
    // (thread t owns sensors 2t and 2t + 1); counters become output cursors
    int tot[2] = {0, 0};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int k = 2 * threadIdx.x + q;
        if (k >= nb) continue;
        int run = 0;
#pragma unroll
        for (int w = 0; w < kW; ++w) {
            const int c = s_wc[w][k];
            s_wc[w][k] = run;
            run += c;
        }
        tot[q] = run;
    }
    const int64_t inc = wave_incl_scan((int64_t)(tot[0] + tot[1]));
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    int64_t acc = inc - tot[0] - tot[1];
    for (int k = 0; k < wv; ++k) acc += s_w[k];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int k = 2 * threadIdx.x + q;
        if (k < nb) {
            bin_off[(int64_t)e * n_sens + lo + k] = cs + acc;
#pragma unroll
            for (int w = 0; w < kW; ++w) s_wc[w][k] += (int32_t)acc;
        }
        acc += tot[q];
    }
    if (e == n_ev - 1 && r == nr - 1 && threadIdx.x == 0) bin_off[(int64_t)n_ev * n_sens] = cpos[*nent];
    __syncthreads();
    if (cnt <= kFineSrcCap) {
        // ranks give, for every binned position, its source hit (LDS); the
        // hits are then gathered into place with coalesced stores
        for (int64_t jb = j0; jb < j1; jb += 64 * kFU) {
            int kv[kFU];
#pragma unroll
            for (int u = 0; u < kFU; ++u) {
                const int64_t j = jb + u * 64 + lane;
                kv[u] = tsens[cs + (j < j1 ? j : j1 - 1)];
            }
#pragma unroll
            for (int u = 0; u < kFU; ++u) kv[u] = jb + u * 64 + lane < j1 ? kv[u] - lo : -1;
#pragma unroll
            for (int u = 0; u < kFU; ++u) {
                if (jb + u * 64 < j1) {              // wavefront-uniform
                    const bool ok = kv[u] >= 0;
                    const int p = wave_rank(s_wc[wv], ok ? kv[u] : 0, ok, nbits);
                    if (ok) s_src[p] = (uint16_t)(jb + u * 64 + lane);
                }
            }
        }
        __syncthreads();
        const int n = (int)cnt;
        for (int pb = 0; pb < n; pb += kFineThreads * kFU) {
            f32x4_t hv[kFU];
#pragma unroll
            for (int u = 0; u < kFU; ++u) {
                const int p = pb + u * kFineThreads + threadIdx.x;
                hv[u] = reinterpret_cast<const f32x4_t *>(tmp)[cs + s_src[p < n ? p : n - 1]];
            }
#pragma unroll
            for (int u = 0; u < kFU; ++u) {
                const int p = pb + u * kFineThreads + threadIdx.x;
                if (p < n) reinterpret_cast<f32x4_t *>(bin_hit)[cs + p] = hv[u];
            }
        }
        return;
    }
    // larger ranges: each hit is stored at its binned position directly
    for (int64_t jb = j0; jb < j1; jb += 64 * kFU) {
        int kv[kFU];
        f32x4_t hv[kFU];
#pragma unroll
        for (int u = 0; u < kFU; ++u) {
            const int64_t j = jb + u * 64 + lane, jc = j < j1 ? j : j1 - 1;
            kv[u] = tsens[cs + jc];
            hv[u] = reinterpret_cast<const f32x4_t *>(tmp)[cs + jc];
        }
        vmem_wait_all();
#pragma unroll
        for (int u = 0; u < kFU; ++u) kv[u] = jb + u * 64 + lane < j1 ? kv[u] - lo : -1;
#pragma unroll
        for (int u = 0; u < kFU; ++u) {
            if (jb + u * 64 < j1) {                  // wavefront-uniform
                const bool ok = kv[u] >= 0;
                const int p = wave_rank(s_wc[wv], ok ? kv[u] : 0, ok, nbits);
                if (ok) reinterpret_cast<f32x4_t *>(bin_hit)[cs + p] = hv[u];
            }
        }
    }
}

// ------------------------------------------------------------ MD stage
// Anchor: (event, module). Left = hits on the anchor sensor, right = hits on
// the other sensor. info = {first left hit, n left, n right, module}.

struct MDStage {
    const int64_t *bin_off;
    const float4 *bin_hit;
    const ModConst *mod;
    const ModBox *box;
    int64_t *counts;
    CutParams p;
    int32_t n_mod, n_sens;
    int2 *md_hits;
    float4 *md_a;
    float2 *md_o;
    float2 *md_rq;
    static constexpr int kEnt = 0;
    static constexpr int kStage = 0;
    static constexpr int kWin = 512;             // anchors staged per tile
    static constexpr bool kUnitCount = false;
    static constexpr int kMinBlocks = 1;       // resident blocks per CU the register budget must allow
    static constexpr int kPhases = 1;            // cut phases (later ones on queued survivors)
    struct Rec { float4 a; float2 o; int hl, hu; };
    struct Mid {};

    __device__ int64_t count(int64_t gm) const {
        int64_t e = gm / n_mod, m = gm - e * n_mod;
        int64_t b = e * n_sens + 2 * m;
        return (bin_off[b + 1] - bin_off[b]) * (bin_off[b + 2] - bin_off[b + 1]);
    }
    __device__ void info(int64_t gm, int32_t *f) const {
        int64_t e = gm / n_mod, m = gm - e * n_mod;
        int64_t b = e * n_sens + 2 * m;
        int64_t b0 = bin_off[b], b1 = bin_off[b + 1], b2 = bin_off[b + 2];
        f[0] = (int32_t)b0; f[1] = (int32_t)(b1 - b0); f[2] = (int32_t)(b2 - b1); f[3] = (int32_t)m;
    }
    template <class LDS>
    __device__ void prepare(LDS &, int64_t, int) const {}
    template <class LDS>
    __device__ bool eval(int64_t gm, int32_t local, const int32_t *f, const LDS &, Rec &r, Mid &) const {
        const int nR = f[2];
        const int l = local / nR, rr = local - l * nR;
        float4 hi = bin_hit[f[0] + l];
        float4 hj = bin_hit[f[0] + f[1] + rr];
        bool ok = md_pass(mod[f[3]], p, P3{hi.x, hi.y, hi.z}, P3{hj.x, hj.y, hj.z});
        r.hl = __float_as_int(hi.w); r.hu = __float_as_int(hj.w);
        r.a = make_float4(hi.x, hi.y, hi.z, __int_as_float((int)gm));
        r.o = make_float2(hj.x, hj.y);
        return ok;
    }
    __device__ void write(int64_t pos, const Rec &r) const {
        const int m = __float_as_int(r.a.w) % n_mod;
        md_hits[pos] = make_int2(r.hl, r.hu);
        md_a[pos] = r.a;
        md_o[pos] = r.o;
        const float2 rq = make_md_rq(p, r.a.x, r.a.y, mod[m].kind != 0);
        md_rq[pos] = rq;
        // the anchor must lie on its sensor: the line-segment windows rely on it
        const ModBox bx = box[m];
        float ph = atan2f(r.a.y, r.a.x);
        if (ph < 0.0f) ph += 6.2831853f;
        const bool phi_ok = (ph >= bx.phi_lo && ph <= bx.phi_hi) || ph + 6.2831853f <= bx.phi_hi ||
                            ph - 6.2831853f >= bx.phi_lo;
        const bool on = rq.x >= bx.r_lo && rq.x <= bx.r_hi && r.a.z >= bx.z_lo && r.a.z <= bx.z_hi && phi_ok;
        if (!on) atomicOr((unsigned long long *)&counts[LST_COUNT_ERR], 8ull);
    }
};

// CSR offsets from a key column sorted ascending: off[k] = first i < n with
// key(i) >= k (n if none), for k = 0..K. Element i owns the run of keys
// key(i-1) < k <= key(i) (with key(-1) = -1 and key(n) = K), so the runs
// partition 0..K, every entry is written once and the key column is read
// once, coalesced. A lane writes a short run itself; runs longer than
// kRunLane (modules or events without objects) are written by the whole
// wavefront, 64 entries a step.
constexpr int kRunLane = 8;

template <class KF>
__global__ __launch_bounds__(kBlock) void k_fill_offsets(KF key, const int64_t *n_dev, int64_t n_cap,
                                                         const int64_t *K_dev, int64_t K_cap, int64_t *off) {
    const int64_t n = n_dev ? dev_count(n_dev, n_cap) : n_cap;
    const int64_t K = K_dev ? dev_count(K_dev, K_cap) : K_cap;
    const int lane = threadIdx.x & 63;
    // base is uniform per wavefront, so whole wavefronts run the loop
    for (int64_t base = grid_tid() - lane; base <= n; base += grid_stride()) {
        const int64_t i = base + lane;
        int64_t lo = 1, hi = 0;   // empty run
        if (i <= n) {
            const int64_t kp = i > 0 ? (int64_t)key(i - 1) : -1;
            const int64_t kc = i < n ? (int64_t)key(i) : K;
            lo = kp < 0 ? 0 : (kp < K ? kp : K) + 1;
            hi = kc < K ? kc : K;
        }
        const bool wide = hi - lo >= kRunLane;
        if (!wide)
            for (int64_t k = lo; k <= hi; ++k) off[k] = i;
        unsigned long long m = __ballot(wide);
        while (m) {
            const int l = __ffsll(m) - 1;
            m &= m - 1;
            const int64_t rlo = __shfl(lo, l, 64), rhi = __shfl(hi, l, 64);
            for (int64_t k = rlo + lane; k <= rhi; k += 64) off[k] = base + l;
        }
    }
}

// ------------------------------------------------------------ LS stage
// Line segments (Table 1 step 2): pairs of MDs (A, B) with B on a module of
// A's module-map row (LS0), passing the curvature (LS1), z0 (LS2) and, for
// barrel MDs, direction (LS3) cuts.
//
// One lane per inner MD A: a wavefront takes 64 consecutive MDs (sorted by
// event and module) and each lane walks its own candidates B, in ascending B,
// so no candidate is ever decoded from a flat index. A's map row is stored as
// runs (consecutive target modules of one detector row, adjacent in phi), and
// for this A every run gets windows that contain every B the cuts can accept:
//  * s ordering: LS2 needs s_B > s_A, i.e. r_B > r_A, so a run whose rows lie
//    below r_A is skipped;
//  * phi: on a circle through the beam line with signed half-curvature k the
//    points at radii r_A < r_B are g(k, r_B) = asin(k r_B) - asin(k r_A) apart
//    in phi, and g grows with k. LS1 bounds |k| by c_lim (with |B - A| >=
//    r_B,min - r_A and the row's largest resolution term). For a barrel A,
//    LS3 on A compares the MD's own chord direction alpha (angle from the
//    radial direction at the chord midpoint M) with sgn asin(c' |M|),
//    c' = min(c, c_max), so sgn c' lies in [sin(alpha - tol), sin(alpha +
//    tol)] / |M|; when that interval reaches +-c_max the pair's k may run on
//    to +-c_lim. The k interval maps to a phi window [g(k_lo), g(k_hi)] over
//    the row's radii, which trims the run's modules and is tested on every B
//    (two cross products with the window's edge directions);
//  * z0, barrel to barrel: z_B = z_A + (z_A - z0) rho with
//    rho = s_B / s_A - 1 between its values at c = 0 and c_max and
//    |z0| <= z_lum + n_sigma sigma_z0 bounds z_B; runs outside are skipped and
//    every barrel B of the run is tested against the window.
// Every bound is widened well beyond FP32 rounding, and anchors are known to
// lie on their sensors (checked when MDs are written), so the windows never
// remove a pair that the cuts would accept.
//
// Candidates inside the windows are queued in LDS; LS1 and LS2 run on dense
// batches of 64 queue entries (the anchor of each entry is shuffled from its
// owner lane), and the pairs passing both are queued again for LS3, also run
// on dense batches. The queues keep each A's candidate order, so an LS3
// survivor gets its rank among the segments of its A. Survivors collect in an
// LDS list that is written out, a few hundred at a time, as (A, B, rank)
// records to a scratch array (one atomic add per write-out). A scan of the
// per-A counts gives the CSR offsets of LS by inner MD, and a placement kernel
// stores each record at offset[A] + rank.

constexpr int kLsWaves = 1;             // wavefronts per block of the eval kernel (one tile each)
constexpr int kLsBlock = 64 * kLsWaves;
constexpr int kLsRunsPerRound = 2;      // trimmed runs staged per lane at a time (even)
constexpr int kLsQCap = 128;            // queue entries per wavefront (up to 63 waiting + 64 new)
constexpr int kLsOutCap = 256;          // survivors held per wavefront before a write-out
constexpr int kLsBlocks = 32768;        // blocks of the eval kernel (one per tile of 64 MDs at the benchmark's sizes)
constexpr float kLsCrossMargin = 1e-3f; // cm: slack of the phi-window cross products
// queue entry tag: bits 0-5 owner lane, 6 bends positive, 7 / 8 direction cut
// on A / on B (barrel MDs)
constexpr int kTagPos = 64, kTagDirA = 128, kTagDirB = 256;

struct LsLds {
    int2 rng[kLsWaves][kLsRunsPerRound][64];     // trimmed MD ranges [j, je) of each lane
    float4 win[kLsWaves][kLsRunsPerRound][64];   // their phi-window edge directions (all 0: no window)
    float2 zw[kLsWaves][kLsRunsPerRound][64];    // their z windows
    int pb[kLsWaves][kLsQCap];                   // window survivors: B
    int po[kLsWaves][kLsQCap];                   //                   owner lane
    int qb[kLsWaves][kLsQCap];                   // LS1 + LS2 survivors: B
    float qc[kLsWaves][kLsQCap];                 //                      clamped curvature
    int qt[kLsWaves][kLsQCap];                   //                      tag
    int ob[kLsWaves][kLsOutCap];                 // LS3 survivors: B
    int ot[kLsWaves][kLsOutCap];                 //                owner lane | rank << 6
    int cnt[kLsWaves][64];                       // survivors per owner lane
};

struct LsArgs {
    const float4 *md_a;
    const float2 *md_o;
    const float2 *md_rq;
    const int64_t *md_mod_off;
    GeomDev g;
    CutParams p;
    int32_t *ls_cnt;                 // [cap_md] LS per inner MD
    int4 *chunk;                     // [cap_chunk] (A, B, rank of B among A's segments, 0)
    int64_t cap_chunk;
    unsigned long long *top;         // records written (zeroed before the eval kernel)
    int64_t *counts;
    int64_t cap_md;
};

// The anchor MD of one lane.
struct LsAnchor {
    float x, y, z, r, q, phi;   // q: resolution term |rq.y|; phi in [0, 2 pi)
    float ux, uy;               // radial unit vector
    float klo, khi;             // LS3 interval of sgn * min(c, c_max) (barrel, when hask)
    bool end;                   // endcap MD
    bool hask, none;            // k interval in use; no B can pass (empty interval)
    int64_t ebase;              // event * n_mod
    int32_t r0, r1;             // runs of the module's map row
};

__device__ __forceinline__ LsAnchor ls_anchor(const LsArgs &a, int64_t A) {
    LsAnchor s;
    const float4 p = a.md_a[A];
    const float2 rq = a.md_rq[A];
    const int32_t gm = __float_as_int(p.w);
    const int32_t e = gm / a.g.n_mod, m = gm - e * a.g.n_mod;
    s.x = p.x; s.y = p.y; s.z = p.z;
    s.r = rq.x;
    s.q = fabsf(rq.y);
    s.end = signbit(rq.y);
    float ph = atan2f(p.y, p.x);
    s.phi = ph < 0.0f ? ph + 6.2831853f : ph;
    s.ux = p.x / s.r;
    s.uy = p.y / s.r;
    s.ebase = (int64_t)e * a.g.n_mod;
    s.r0 = a.g.run_off[m];
    s.r1 = a.g.run_off[m + 1];
    s.hask = s.none = false;
    s.klo = s.khi = 0.0f;
    if (!s.end) {
        // LS3 on A: the chord d from the anchor to the other hit, at angle
        // alpha from the radial direction of the chord midpoint M; the
        // interval ends are sin(alpha -+ tol) / |M| with alpha -+ tol clipped
        // to [-pi/2, pi/2] (taken from sin and cos of alpha, no angles)
        const float2 o = a.md_o[A];
        const float dx = o.x - p.x, dy = o.y - p.y;
        const float mx = 0.5f * (p.x + o.x), my = 0.5f * (p.y + o.y);
        const float mm = sqrtf(mx * mx + my * my), dl = sqrtf(dx * dx + dy * dy);
        const float inv = 1.0f / (mm * dl);
        const float sa = (mx * dy - my * dx) * inv, ca = (mx * dx + my * dy) * inv;
        const float tol = (a.p.nsig * 1.41421356f * a.p.srphi / dl + a.p.ls3slack) * 1.001f + 2e-5f;
        if (tol < 0.5f) {
            s.hask = true;
            float st, ct;
            __sincosf(tol, &st, &ct);
            const float sp = sa * ct + ca * st, cp = ca * ct - sa * st;   // alpha + tol
            const float sm = sa * ct - ca * st, cm = ca * ct + sa * st;   // alpha - tol
            float shi = sp, slo = sm;
            if (cp < 0.0f) {
                if (sp > 0.0f) shi = 1.0f;
                else s.none = true;
            }
            if (cm < 0.0f) {
                if (sm < 0.0f) slo = -1.0f;
                else s.none = true;
            }
            s.klo = slo / mm;
            s.khi = shi / mm;
            if (s.khi < -a.p.cmax || s.klo > a.p.cmax) s.none = true;
        }
    }
    return s;
}

// z window of barrel MDs at radii [r_lo, r_hi] for barrel anchor s (see the
// stage comment): rho0 at c = 0 and r_B = r_lo, rho1 at c = c_max and
// r_B = r_hi bound rho; sigma_z0 = sigma_z sqrt(1 + (1 + rho)^2) / rho is
// bounded with rho1 above and rho0 below.
__device__ __forceinline__ void ls_zwindow(const CutParams &p, float za, float ra, float r_lo, float r_hi,
                                           float &lo, float &hi) {
    const float rho0 = r_lo / ra - 1.0f;
    const float rho1 = arc_len_f(p.cmax, r_hi) / arc_len_f(p.cmax, ra) - 1.0f;
    const float zt = p.zlum + p.nsig * p.sz * sqrtf(1.0f + (1.0f + rho1) * (1.0f + rho1)) / rho0;
    const float a0 = (za - zt) * rho0, a1 = (za - zt) * rho1;
    const float b0 = (za + zt) * rho0, b1 = (za + zt) * rho1;
    lo = za + fminf(a0, a1);
    hi = za + fmaxf(b0, b1);
    const float m = 1e-3f * (hi - lo) + 1e-2f;
    lo -= m;
    hi += m;
}

// asin(x) for |x| <= 0.8 from the arc-length polynomial (relative error below
// 1e-7, far inside the windows' slack)
__device__ __forceinline__ float ls_asin(float x) { return x * asin_over_x_f(x * x); }

// Kept target modules i0 .. i1 of run rr for anchor s (i1 < i0: none), with
// the phi window every candidate must pass (edge directions e_lo, e_hi; all
// zero: no window) and its z window.
__device__ __forceinline__ int2 ls_run_trim(const CutParams &p, const LsAnchor &s, const RunRec &rr, float4 &win,
                                            float2 &zw) {
    int i0 = 0, i1 = rr.n - 1;
    win = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    zw = make_float2(-INFINITY, INFINITY);
    // s ordering: every anchor of the row is below r_A
    bool keep = !s.none && !(rr.r_hi * (1.0f + 2e-5f) < s.r);
    // barrel to barrel: z window
    if (keep && !s.end && !(rr.flags & kRunEndcap) && rr.r_lo > s.r * 1.0001f) {
        ls_zwindow(p, s.z, s.r, rr.r_lo, rr.r_hi, zw.x, zw.y);
        if (rr.z_hi < zw.x || rr.z_lo > zw.y) keep = false;
    }
    // curvature (and, for a barrel A, its direction): phi window
    if (keep && !(rr.flags & kRunNoTrim)) {
        const float dmin = rr.r_lo - s.r * (1.0f + 1e-6f);
        if (dmin > 0.05f) {
            const float clim = 1.001f * (p.cmax + p.nsig * sqrtf(s.q + rr.qb_max) / dmin);
            const float xh = clim * rr.r_hi;
            if (xh < 0.8f) {
                // every |k r| below is at most xh < 0.8, where asin(x) =
                // x asin_over_x(x^2) holds to 1e-7
                float dlo, dhi;
                if (s.hask) {
                    const float kl = s.klo <= -p.cmax ? -clim : fmaxf(s.klo, -clim);
                    const float kh = s.khi >= p.cmax ? clim : fminf(s.khi, clim);
                    dlo = ls_asin(kl * (kl >= 0.0f ? rr.r_lo : rr.r_hi)) - ls_asin(kl * s.r);
                    dhi = ls_asin(kh * (kh >= 0.0f ? rr.r_hi : rr.r_lo)) - ls_asin(kh * s.r);
                } else {
                    dhi = ls_asin(xh) - ls_asin(clim * s.r);
                    dlo = -dhi;
                }
                dlo -= 1e-4f;
                dhi += 1e-4f;
                // window [phi + dlo, phi + dhi] against the run [phi_start,
                // phi_start + n dphi], at shifts of -2 pi, 0, 2 pi; the hull of
                // the overlaps is kept
                int lo = rr.n, hi = -1;
#pragma unroll
                for (int sh = -1; sh <= 1; ++sh) {
                    const float c = s.phi + (float)sh * 6.2831853f - rr.phi_start;
                    const float u0 = (c + dlo) * rr.inv_dphi - 1e-4f, u1 = (c + dhi) * rr.inv_dphi + 1e-4f;
                    if (u1 >= 0.0f && u0 < (float)rr.n) {
                        const int v0 = u0 < 0.0f ? 0 : (int)u0;
                        const int v1 = u1 >= (float)(rr.n - 1) ? rr.n - 1 : (int)u1;
                        lo = v0 < lo ? v0 : lo;
                        hi = v1 > hi ? v1 : hi;
                    }
                }
                i0 = lo;
                i1 = hi;
                float sl, cl, sh, ch;
                __sincosf(dlo, &sl, &cl);
                __sincosf(dhi, &sh, &ch);
                win = make_float4(cl * s.ux - sl * s.uy, sl * s.ux + cl * s.uy, ch * s.ux - sh * s.uy,
                                  sh * s.ux + ch * s.uy);
            }
        }
    }
    if (!keep) i1 = i0 - 1;
    return make_int2(i0, i1);
}

// Window test of candidate B: between the edge directions (the window spans
// less than pi) and inside the z window.
__device__ __forceinline__ bool ls_window_pass(const float4 &w, const float2 &zw, const float4 &PB) {
    return w.x * PB.y - w.y * PB.x >= -kLsCrossMargin && PB.x * w.w - PB.y * w.z >= -kLsCrossMargin &&
           PB.z >= zw.x && PB.z <= zw.y;
}

__device__ __forceinline__ unsigned long long lanes_below(int lane) { return (1ull << lane) - 1ull; }

// Write the wavefront's LDS list of survivors [0, outn) to the scratch array
// as (A, B, rank) records.
__device__ void ls_spill(const LsArgs &a, LsLds &L, int wv, int lane, int64_t wbase, int &outn) {
    wave_sync_lds();
    unsigned long long b0 = 0;
    if (lane == 0) b0 = atomicAdd(a.top, (unsigned long long)outn);
    const long long base = (long long)__shfl((long long)b0, 0, 64);
    for (int i = lane; i < outn; i += 64) {
        if (base + i < a.cap_chunk) {
            const int t = L.ot[wv][i];
            a.chunk[base + i] = make_int4((int)(wbase + (t & 63)), L.ob[wv][i], t >> 6, 0);
        }
    }
    outn = 0;
    wave_sync_lds();
}

// LS3 on queue entries [0, n) (n <= 64); survivors go to the output list
// with their rank among their owner's survivors, the remaining entries move
// to the front.
__device__ void ls_flush(const LsArgs &a, LsLds &L, int wv, int lane, int64_t wbase, int n, int &qn, int &outn) {
    if (outn > kLsOutCap - 64) ls_spill(a, L, wv, lane, wbase, outn);
    wave_sync_lds();
    bool ok = false;
    int b = 0, owner = 0;
    if (lane < n) {
        b = L.qb[wv][lane];
        const float cp = L.qc[wv][lane];
        const int tg = L.qt[wv][lane];
        owner = tg & 63;
        const float sg = (tg & kTagPos) ? 1.0f : -1.0f;
        const int64_t A = wbase + owner;
        const int64_t ia = (tg & kTagDirA) ? A : b, ib = (tg & kTagDirB) ? b : ia;
        const float4 PA = a.md_a[ia], PB = a.md_a[ib];
        const float2 oa = a.md_o[ia], ob = a.md_o[ib];
        ok = true;
        if (tg & kTagDirA) ok = md_dir_pass(a.p, P3{PA.x, PA.y, PA.z}, oa.x, oa.y, cp, sg);
        if (ok && (tg & kTagDirB)) ok = md_dir_pass(a.p, P3{PB.x, PB.y, PB.z}, ob.x, ob.y, cp, sg);
    }
    const int rest = qn - n;
    if (rest > 0) {
        wave_sync_lds();
        const int src = n + (lane < rest ? lane : 0);
        const int tb = L.qb[wv][src];
        const float tc = L.qc[wv][src];
        const int tt = L.qt[wv][src];
        wave_sync_lds();
        if (lane < rest) { L.qb[wv][lane] = tb; L.qc[wv][lane] = tc; L.qt[wv][lane] = tt; }
    }
    qn = rest;
    // lanes of the same owner: equal in all six owner bits
    unsigned long long same = __ballot(ok);
#pragma unroll
    for (int bit = 0; bit < 6; ++bit) {
        const bool v = (owner >> bit) & 1;
        const unsigned long long m = __ballot(ok && v);
        same &= v ? m : ~m;
    }
    if (!ok) same = 0;
    const int rank = __popcll(same & lanes_below(lane));
    wave_sync_lds();
    const int base = ok ? L.cnt[wv][owner] : 0;
    wave_sync_lds();
    if (ok && rank == 0) L.cnt[wv][owner] = base + __popcll(same);
    const unsigned long long mo = __ballot(ok);
    const int pos = outn + __popcll(mo & lanes_below(lane));
    if (ok) {
        L.ob[wv][pos] = b;
        L.ot[wv][pos] = owner | ((base + rank) << 6);
    }
    outn += __popcll(mo);
    wave_sync_lds();
}

// LS1 and LS2 on window-survivor entries [0, n) (n <= 64), the anchor of
// each taken from its owner lane; passing pairs join the LS3 queue, the
// remaining entries move to the front. Called with every lane active.
__device__ void ls_dense(const LsArgs &a, LsLds &L, int wv, int lane, int64_t wbase, const LsAnchor &s, int n,
                         int &pn, int &qn, int &outn) {
    wave_sync_lds();
    int b = 0, o = 0;
    if (lane < n) {
        b = L.pb[wv][lane];
        o = L.po[wv][lane];
    }
    const float ax = __shfl(s.x, o, 64), ay = __shfl(s.y, o, 64), az = __shfl(s.z, o, 64);
    const float ar = __shfl(s.r, o, 64), aq = __shfl(s.end ? -s.q : s.q, o, 64);
    bool pass = false;
    float cp = 0.0f;
    int tag = 0;
    if (lane < n) {
        const float4 PB = a.md_a[b];
        const float2 qb = a.md_rq[b];
        const P3 PA{ax, ay, az}, PBp{PB.x, PB.y, PB.z};
        const float2 qa = make_float2(ar, aq);
        float c, sg;
        if (pair_curv_pass(a.p, PA, qa, PBp, qb, c, sg)) {
            cp = fminf(c, a.p.cmax);
            if (pair_z0_pass(a.p, PA, qa, PBp, qb, cp)) {
                pass = true;
                tag = o | (sg > 0.0f ? kTagPos : 0) | (signbit(aq) ? 0 : kTagDirA) | (signbit(qb.y) ? 0 : kTagDirB);
            }
        }
    }
    const int rest = pn - n;
    if (rest > 0) {
        wave_sync_lds();
        const int src = n + (lane < rest ? lane : 0);
        const int tb = L.pb[wv][src], to = L.po[wv][src];
        wave_sync_lds();
        if (lane < rest) { L.pb[wv][lane] = tb; L.po[wv][lane] = to; }
    }
    pn = rest;
    const unsigned long long m = __ballot(pass);
    if (pass) {
        const int pos = qn + __popcll(m & lanes_below(lane));
        L.qb[wv][pos] = b;
        L.qc[wv][pos] = cp;
        L.qt[wv][pos] = tag;
    }
    qn += __popcll(m);
    if (qn >= 64) ls_flush(a, L, wv, lane, wbase, 64, qn, outn);
}

// Stage the trimmed MD ranges of runs [rbeg, rbeg + kLsRunsPerRound) of each
// lane's anchor in LDS with their windows, two runs at a time (their records,
// then their four module offsets, in flight together); returns the number of
// non-empty ranges of this lane and adds their candidates to *cands.
__device__ __forceinline__ int ls_stage_round(const LsArgs &a, LsLds &L, int wv, int lane, const LsAnchor &s,
                                              bool act, int rbeg, int rmax, int &cands) {
    int nr = 0;
    const int last = s.r1 - 1 >= s.r0 ? s.r1 - 1 : s.r0;   // clamped run index (valid: the table is never empty)
    for (int r = rbeg; r < rbeg + kLsRunsPerRound && r < rmax; r += 2) {
        const bool h0 = act && s.r0 + r < s.r1, h1 = act && s.r0 + r + 1 < s.r1;
        const int k0 = s.r0 + r < last ? s.r0 + r : last;
        const int k1 = s.r0 + r + 1 < last ? s.r0 + r + 1 : last;
        const RunRec ra = a.g.runs[k0], rb = a.g.runs[k1];
        int2 ta = make_int2(0, -1), tb = make_int2(0, -1);
        float4 wa, wb;
        float2 za, zb;
        if (h0) ta = ls_run_trim(a.p, s, ra, wa, za);
        if (h1) tb = ls_run_trim(a.p, s, rb, wb, zb);
        const int64_t ea = s.ebase + ra.t_first, eb = s.ebase + rb.t_first;
        const int64_t ia0 = ta.y >= ta.x ? ea + ta.x : s.ebase, ia1 = ta.y >= ta.x ? ea + ta.y + 1 : s.ebase;
        const int64_t ib0 = tb.y >= tb.x ? eb + tb.x : s.ebase, ib1 = tb.y >= tb.x ? eb + tb.y + 1 : s.ebase;
        const int ja = (int)a.md_mod_off[ia0], jae = (int)a.md_mod_off[ia1];
        const int jb = (int)a.md_mod_off[ib0], jbe = (int)a.md_mod_off[ib1];
        if (jae > ja) {
            L.rng[wv][nr][lane] = make_int2(ja, jae);
            L.win[wv][nr][lane] = wa;
            L.zw[wv][nr][lane] = za;
            cands += jae - ja;
            ++nr;
        }
        if (jbe > jb) {
            L.rng[wv][nr][lane] = make_int2(jb, jbe);
            L.win[wv][nr][lane] = wb;
            L.zw[wv][nr][lane] = zb;
            cands += jbe - jb;
            ++nr;
        }
    }
    return nr;
}

// A lane's walk over its staged ranges: next() returns the next candidate
// index with its range's windows, and whether there is one.
struct LsCursor {
    int ri, nr, j, je;
    bool on;
    float4 w;
    float2 zw;
    __device__ __forceinline__ void load(const LsLds &L, int wv, int lane) {
        const int2 g = L.rng[wv][ri][lane];
        j = g.x;
        je = g.y;
        w = L.win[wv][ri][lane];
        zw = L.zw[wv][ri][lane];
    }
    __device__ __forceinline__ void start(const LsLds &L, int wv, int lane, int n) {
        ri = 0;
        nr = n;
        on = n > 0;
        j = je = 0;
        w = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        zw = make_float2(0.0f, 0.0f);
        if (on) load(L, wv, lane);
    }
    __device__ __forceinline__ bool next(const LsLds &L, int wv, int lane, int &b, float4 &wo, float2 &zo) {
        if (!on) return false;
        b = j++;
        wo = w;
        zo = zw;
        if (j >= je) {
            if (++ri < nr) load(L, wv, lane);
            else on = false;
        }
        return true;
    }
};

__global__ __launch_bounds__(kLsBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_ls_eval(LsArgs a) {
    __shared__ LsLds L;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t n_md = dev_count(a.counts + LST_COUNT_MD, a.cap_md);
    const int64_t nwaves = (n_md + 63) / 64;
    const int64_t ntiles = (nwaves + kLsWaves - 1) / kLsWaves;
    const TileWalk walk(ntiles);
    for (int64_t tile = walk.first; tile < walk.end; tile += walk.step) {
        const int64_t w = tile * kLsWaves + wv;
        if (w >= nwaves) continue;             // wavefront-uniform
        const int64_t wbase = w * 64, A = wbase + lane;
        const bool act = A < n_md;
        const int a_safe = (int)(act ? A : n_md - 1);
        const LsAnchor s = ls_anchor(a, a_safe);
        L.cnt[wv][lane] = 0;
        int pn = 0, qn = 0, outn = 0, cands = 0;
        // runs of the wavefront's longest map row
        int nrun = act ? s.r1 - s.r0 : 0;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const int o = __shfl_xor(nrun, d, 64);
            nrun = o > nrun ? o : nrun;
        }
        for (int rbeg = 0; rbeg < nrun; rbeg += kLsRunsPerRound) {
            const int nr = ls_stage_round(a, L, wv, lane, s, act, rbeg, nrun, cands);
            wave_sync_lds();
            LsCursor cu;
            cu.start(L, wv, lane, nr);
            // Two register sets take alternate candidates; a set is reloaded
            // right after its candidate is tested, so every load has the
            // other set's test to complete in.
            int bA = a_safe, bB = a_safe;
            float4 wA, wB;
            float2 zA, zB;
            bool vA = cu.next(L, wv, lane, bA, wA, zA);
            float4 PBa = a.md_a[bA];
            bool vB = cu.next(L, wv, lane, bB, wB, zB);
            float4 PBb = a.md_a[bB];
            auto step = [&](bool v, int b, const float4 &PB, const float4 &wn, const float2 &zn) {
                const bool pass = v && ls_window_pass(wn, zn, PB);
                const unsigned long long m = __ballot(pass);
                if (pass) {
                    const int pos = pn + __popcll(m & lanes_below(lane));
                    L.pb[wv][pos] = b;
                    L.po[wv][pos] = lane;
                }
                pn += __popcll(m);
                if (pn >= 64) ls_dense(a, L, wv, lane, wbase, s, 64, pn, qn, outn);
            };
            while (__ballot(vA) != 0ull) {
                step(vA, bA, PBa, wA, zA);
                bA = a_safe;
                vA = cu.next(L, wv, lane, bA, wA, zA);
                PBa = a.md_a[bA];
                if (__ballot(vB) == 0ull) break;
                step(vB, bB, PBb, wB, zB);
                bB = a_safe;
                vB = cu.next(L, wv, lane, bB, wB, zB);
                PBb = a.md_a[bB];
            }
        }
        // drain the queues
        while (pn > 0) ls_dense(a, L, wv, lane, wbase, s, pn < 64 ? pn : 64, pn, qn, outn);
        while (qn > 0) ls_flush(a, L, wv, lane, wbase, qn < 64 ? qn : 64, qn, outn);
        if (outn > 0) ls_spill(a, L, wv, lane, wbase, outn);
        wave_sync_lds();
        if (act) a.ls_cnt[A] = L.cnt[wv][lane];
        int cs = cands;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) cs += __shfl_xor(cs, d, 64);
        if (lane == 0) atomicAdd((unsigned long long *)&a.counts[LST_COUNT_LSCAND], (unsigned long long)cs);
        wave_sync_lds();
    }
}

// Place every record at offset[A] + rank (ls_off = exclusive scan of the
// per-A counts). When more segments were found than the scratch holds (the
// build then reports a capacity overflow), the list is filled with valid
// indices instead, for the stages that still read it.
__global__ __launch_bounds__(kBlock) void k_ls_place(LsArgs a, const int64_t *ls_off, int2 *ls_md, int64_t cap_ls) {
    const int64_t n_md = dev_count(a.counts + LST_COUNT_MD, a.cap_md);
    const int64_t tot = ls_off[n_md];
    if (blockIdx.x == 0 && threadIdx.x == 0) a.counts[LST_COUNT_LS] = tot;
    const int64_t top = (int64_t)*a.top;
    if (top > a.cap_chunk) {
        const int64_t n = tot < cap_ls ? tot : cap_ls;
        for (int64_t i = grid_tid(); i < n; i += grid_stride()) ls_md[i] = make_int2(0, 0);
        return;
    }
    for (int64_t i = grid_tid(); i < top; i += grid_stride()) {
        const int4 r = a.chunk[i];
        const int64_t pos = ls_off[r.x] + r.z;
        if (pos < cap_ls) ls_md[pos] = make_int2(r.x, r.y);
    }
}

// the LS stage's record counter and the T3 stage's list counter (one launch
// for both stages)
__global__ void k_zero_counters(unsigned long long *p, unsigned long long *q) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *p = 0ull;
        *q = 0ull;
    }
}

// ------------------------------------------------------------ T3 stage
// T3 come out sorted by inner LS, hence by inner MD A: the next stage reads
// the T3 starting at an MD as one contiguous range.
//
// T3 stage without the tile compaction. A wavefront takes 64 consecutive
// inner LSs (A, B); the candidates of LS l are the LSs starting at B, a
// contiguous range of the LS list, and the wavefront's candidates, numbered
// in (inner LS, candidate) order through an inclusive scan of the per-LS
// counts, go 64 at a time to its lanes (a lane finds its inner LS by binary
// search of the scan held in registers). The first kernel counts survivors
// per wavefront, keeps its first pass masks (a tuning) and every LS's candidate
// range, and lists the wavefronts with more candidates than the masks cover.
// After a scan of the counts over wavefronts the second kernel writes every
// survivor of the other wavefronts at its final place (the wavefront's offset
// plus the survivors before it) from the masks alone, with every inner LS's
// first T3 position; a third does the listed wavefronts, evaluating the
// candidates beyond the masks again; the last turns the positions into the
// CSR of T3 by inner MD.
constexpr int kT3Blocks = 4096;           // grid of the count and write kernels (more than the resident blocks)
constexpr int kT3OvfBlocks = 64;          // grid of the kernel for the listed wavefronts

struct T3Direct {
    const int2 *ls_md;
    const int64_t *ls_off;        // CSR of LS by inner MD (entries may exceed cap_ls after an overflow)
    int64_t cap_ls;
    const float4 *md_a;
    const float2 *md_o;
    const float2 *md_rq;
    CutParams p;
    int32_t *wcnt;                // [cap_ls / 64 + 1] survivors per wavefront
    int64_t *woff;                // [cap_ls / 64 + 2] their exclusive scan
    unsigned long long *bits;     // [(cap_ls / 64 + 1) * kT3MaxMasks] pass masks
    int masks;                    // masks kept per wavefront (1..kT3MaxMasks)
    int64_t *nw;                  // [1] wavefronts of this build
    int2 *cn;                     // [cap_ls] first candidate and candidate count of every inner LS
    int32_t *ovf;                 // [cap_ls / 64 + 1] wavefronts with more than 64 masks candidates
    unsigned long long *n_ovf;    // [1] their number (zeroed before the count kernel)
    int64_t *pos;                 // [cap_ls + 1] first T3 position of every inner LS
    int2 *t3_ls;
    int4 *t3_mds;
    int64_t cap_t3;
    int64_t *counts;
};

__device__ __forceinline__ int64_t t3_lsoff(const T3Direct &d, int64_t md) {
    const int64_t v = d.ls_off[md];
    return v < d.cap_ls ? v : d.cap_ls;
}

// One wavefront's inner LSs: per lane its MDs, first candidate, candidate
// count and the inclusive scan of the counts.
struct T3Wave {
    int64_t l1;
    bool act;
    int2 lm;
    int c0, n, incl, tot;
    float ax, ay, az, qax, qay, bx, by, bz, obx, oby, qby;
};

// kCn: the candidate ranges kept by the count kernel instead of the CSR
template <bool kCn>
__device__ __forceinline__ T3Wave t3_wave(const T3Direct &d, int64_t w, int64_t n_ls, int lane) {
    T3Wave v;
    v.l1 = w * 64 + lane;
    v.act = v.l1 < n_ls;
    const int64_t li = v.act ? v.l1 : n_ls - 1;
    v.lm = d.ls_md[li];
    if constexpr (kCn) {
        const int2 cn = d.cn[li];
        v.c0 = cn.x;
        v.n = v.act ? cn.y : 0;
    } else {
        const int64_t c0 = t3_lsoff(d, v.lm.y);
        v.c0 = (int)c0;
        v.n = v.act ? (int)(t3_lsoff(d, v.lm.y + 1) - c0) : 0;
    }
    int incl = v.n;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const int o = __shfl_up(incl, s, 64);
        if (lane >= s) incl += o;
    }
    v.incl = incl;
    v.tot = __shfl(incl, 63, 64);
    return v;
}

// the MD coordinates the cuts need (read only where candidates are evaluated)
__device__ __forceinline__ void t3_wave_pts(const T3Direct &d, T3Wave &v) {
    const float4 a = d.md_a[v.lm.x], b = d.md_a[v.lm.y];
    const float2 qa = d.md_rq[v.lm.x], qb = d.md_rq[v.lm.y], ob = d.md_o[v.lm.y];
    v.ax = a.x; v.ay = a.y; v.az = a.z; v.qax = qa.x; v.qay = qa.y;
    v.bx = b.x; v.by = b.y; v.bz = b.z; v.obx = ob.x; v.oby = ob.y; v.qby = qb.y;
}

// the lane whose candidate range holds candidate j (j < tot): the first lane
// with inclusive count above j
__device__ __forceinline__ int t3_owner(int incl, int j) {
    int pos = 0;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        const int v = __shfl(incl, pos + s - 1, 64);
        if (v <= j) pos += s;
    }
    return pos;
}

// Candidate j0 + lane of the wavefront (all lanes call): its outer LS, the
// lane of its inner LS and that LS's MD coordinates.
struct T3Cand {
    bool has;
    int lo, own;
    float ax, ay, az, qax, qay, bx, by, bz, obx, oby, qby;
};

__device__ __forceinline__ T3Cand t3_cand(const T3Wave &v, int j0, int lane) {
    T3Cand c;
    const int j = j0 + lane;
    c.has = j < v.tot;
    c.own = t3_owner(v.incl, c.has ? j : v.tot - 1);
    const int excl = __shfl(v.incl - v.n, c.own, 64), c0 = __shfl(v.c0, c.own, 64);
    c.lo = c0 + ((c.has ? j : v.tot - 1) - excl);
    c.ax = __shfl(v.ax, c.own, 64); c.ay = __shfl(v.ay, c.own, 64); c.az = __shfl(v.az, c.own, 64);
    c.qax = __shfl(v.qax, c.own, 64); c.qay = __shfl(v.qay, c.own, 64);
    c.bx = __shfl(v.bx, c.own, 64); c.by = __shfl(v.by, c.own, 64); c.bz = __shfl(v.bz, c.own, 64);
    c.obx = __shfl(v.obx, c.own, 64); c.oby = __shfl(v.oby, c.own, 64); c.qby = __shfl(v.qby, c.own, 64);
    return c;
}

// the T3 cuts of a candidate with its outer MD C loaded: beam-line pair cuts
// on (A, C), then the direction cut of a barrel middle MD B
__device__ __forceinline__ bool t3_cuts(const T3Direct &d, const T3Cand &k, const float4 &c, const float2 &qc) {
    float cv, sg;
    bool pass = pair_pass_rq(d.p, P3{k.ax, k.ay, k.az}, make_float2(k.qax, k.qay), P3{c.x, c.y, c.z}, qc, cv, sg);
    if (pass && !signbit(k.qby)) pass = md_dir_pass(d.p, P3{k.bx, k.by, k.bz}, k.obx, k.oby, fminf(cv, d.p.cmax), sg);
    return k.has && pass;
}

// pass mask of the candidates j0 + lane (one window of 64)
__device__ __forceinline__ unsigned long long t3_eval(const T3Direct &d, const T3Wave &v, int j0, int lane,
                                                      int *lo_out, int *own_out) {
    const T3Cand k = t3_cand(v, j0, lane);
    *lo_out = k.lo;
    *own_out = k.own;
    const int C = d.ls_md[k.lo].y;
    return __ballot(t3_cuts(d, k, d.md_a[C], d.md_rq[C]));
}

// pass masks of two windows, their loads issued together
__device__ __forceinline__ void t3_eval2(const T3Direct &d, const T3Wave &v, int j0, int lane,
                                         unsigned long long *m0, unsigned long long *m1) {
    const T3Cand k0 = t3_cand(v, j0, lane), k1 = t3_cand(v, j0 + 64, lane);
    const int C0 = d.ls_md[k0.lo].y, C1 = d.ls_md[k1.lo].y;
    const float4 c0 = d.md_a[C0], c1 = d.md_a[C1];
    const float2 q0 = d.md_rq[C0], q1 = d.md_rq[C1];
    *m0 = __ballot(t3_cuts(d, k0, c0, q0));
    *m1 = __ballot(t3_cuts(d, k1, c1, q1));
}

__global__ __launch_bounds__(kBlock) void k_t3_count(T3Direct d) {
    // wavefront index made uniform, so that per-wavefront values load as scalars
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t n_ls = dev_count(d.counts + LST_COUNT_LS, d.cap_ls);
    const int64_t nwaves = (n_ls + 63) / 64;
    if (blockIdx.x == 0 && threadIdx.x == 0) *d.nw = nwaves;
    const int64_t ntiles = (nwaves + kBlock / 64 - 1) / (kBlock / 64);
    const TileWalk walk(ntiles);
    for (int64_t tile = walk.first; tile < walk.end; tile += walk.step) {
        const int64_t w = tile * (kBlock / 64) + wv;
        if (w >= nwaves) continue;                 // wavefront-uniform
        T3Wave v = t3_wave<false>(d, w, n_ls, lane);
        if (v.act) d.cn[v.l1] = make_int2(v.c0, v.n);
        t3_wave_pts(d, v);
        int cnt = 0;
        for (int j0 = 0, it = 0; j0 < v.tot; j0 += 128, it += 2) {
            unsigned long long m0, m1 = 0ull;
            if (j0 + 64 < v.tot) {
                t3_eval2(d, v, j0, lane, &m0, &m1);
            } else {
                int lo, own;
                m0 = t3_eval(d, v, j0, lane, &lo, &own);
            }
            cnt += __popcll(m0) + __popcll(m1);
            if (lane == 0) {
                if (it < d.masks) d.bits[w * kT3MaxMasks + it] = m0;
                if (it + 1 < d.masks) d.bits[w * kT3MaxMasks + it + 1] = m1;
            }
        }
        if (lane == 0) {
            d.wcnt[w] = cnt;
            if (v.tot > 64 * d.masks) d.ovf[atomicAdd(d.n_ovf, 1ull)] = (int32_t)w;
        }
    }
}

// Write the T3 of wavefront w at their final places and the first T3
// position of each of its inner LSs. kEval: candidates beyond the kept masks
// are evaluated again (the listed wavefronts); otherwise there are none.
template <bool kEval>
__device__ __forceinline__ void t3_write_wave(const T3Direct &d, T3Wave &v, int64_t w, int lane) {
    const unsigned long long lt = (1ull << lane) - 1;
    const int64_t base = d.woff[w];
    const int mine = v.incl - v.n;                 // the lane's first candidate
    int64_t run = 0, before = 0;
    for (int j0 = 0, it = 0; j0 < v.tot; j0 += 64, ++it) {
        int lo, own;
        unsigned long long m;
        if (!kEval || it < d.masks) {
            m = d.bits[w * kT3MaxMasks + it];
            const int j = j0 + lane < v.tot ? j0 + lane : v.tot - 1;
            own = t3_owner(v.incl, j);
            const int excl = __shfl(v.incl - v.n, own, 64), c0 = __shfl(v.c0, own, 64);
            lo = c0 + (j - excl);
        } else {
            if (it == d.masks) t3_wave_pts(d, v);
            m = t3_eval(d, v, j0, lane, &lo, &own);
        }
        const int k = mine - j0;                   // the lane's candidates before this window
        before += __popcll(k <= 0 ? 0ull : (k >= 64 ? m : m & ((1ull << k) - 1)));
        const int A = __shfl(v.lm.x, own, 64), B = __shfl(v.lm.y, own, 64);
        if ((m >> lane) & 1ull) {
            const int64_t p = base + run + __popcll(m & lt);
            if (p < d.cap_t3) {
                d.t3_ls[p] = make_int2((int)(w * 64 + own), lo);
                d.t3_mds[p] = make_int4(A, B, d.ls_md[lo].y, 0);
            }
        }
        run += __popcll(m);
    }
    if (v.act) {
        const int64_t p = base + before;
        d.pos[v.l1] = p < d.cap_t3 ? p : d.cap_t3;
    }
}

__global__ __launch_bounds__(kBlock) void k_t3_write(T3Direct d) {
    // wavefront index made uniform, so that per-wavefront values load as scalars
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t n_ls = dev_count(d.counts + LST_COUNT_LS, d.cap_ls);
    const int64_t nwaves = (n_ls + 63) / 64;
    const int64_t total = d.woff[nwaves];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d.counts[LST_COUNT_T3] = total;
        d.pos[n_ls] = total < d.cap_t3 ? total : d.cap_t3;
    }
    const int64_t ntiles = (nwaves + kBlock / 64 - 1) / (kBlock / 64);
    const TileWalk walk(ntiles);
    for (int64_t tile = walk.first; tile < walk.end; tile += walk.step) {
        const int64_t w = tile * (kBlock / 64) + wv;
        if (w >= nwaves) continue;                 // wavefront-uniform
        T3Wave v = t3_wave<true>(d, w, n_ls, lane);
        if (v.tot > 64 * d.masks) continue;        // a listed wavefront
        t3_write_wave<false>(d, v, w, lane);
    }
}

__global__ __launch_bounds__(kBlock) void k_t3_write_listed(T3Direct d) {
    const int lane = threadIdx.x & 63;
    const int64_t n_ls = dev_count(d.counts + LST_COUNT_LS, d.cap_ls);
    const int64_t n = (int64_t)*d.n_ovf;
    const int64_t step = (int64_t)gridDim.x * (kBlock / 64);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / 64) + wv; i < n; i += step) {
        const int64_t w = d.ovf[i];
        T3Wave v = t3_wave<true>(d, w, n_ls, lane);
        t3_write_wave<true>(d, v, w, lane);
    }
}

// CSR of T3 by inner MD: the T3 of MD m start at the first T3 of its first LS
__global__ __launch_bounds__(kBlock) void k_t3_md_off(T3Direct d, const int64_t *n_md_dev, int64_t cap_md,
                                                      int64_t *t3i_off) {
    const int64_t n_md = dev_count(n_md_dev, cap_md);
    const int64_t n_ls = dev_count(d.counts + LST_COUNT_LS, d.cap_ls);
    for (int64_t m = grid_tid(); m <= n_md; m += grid_stride()) {
        const int64_t l = t3_lsoff(d, m);
        t3i_off[m] = d.pos[l < n_ls ? l : n_ls];
    }
}

// ------------------------------------------------------------ T5 stage
// In two passes so that the FP64 fits run on dense lanes:
//  (a) anchor: the inner T3 (A, B, C); candidates: every T3 starting at C
//      (contiguous in the T3 output); the FP32 beam-line cuts on (A, E)
//      select pre-candidates (T3 pairs) in candidate order;
//  (b) anchor: one pre-candidate each; both fits, the chi2 cuts and, with a
//      score threshold, the T5-DNN cut. T5 come out sorted by inner T3.

// The quintuplet pre-cuts also screen the r-z chi2 in FP32: a candidate is
// dropped only when its FP32 estimate exceeds the cut by a factor kScreen.
// Where it is finite, the estimate agrees with the FP64 chi2 to well under one
// percent, so every decision near the cut is left to the FP64 fits; a
// degenerate estimate (NaN) drops nothing.
struct T5PreStage {
    const int4 *t3_mds;
    const int64_t *t3i_off;
    const float4 *md_a;
    const float2 *md_rq;
    const ModConst *mod;
    CutParams p;
    int32_t n_mod;
    int2 *pre;
    static constexpr int kEnt = 0;
    static constexpr int kStage = 3;
    static constexpr int kWin = 512;             // anchors staged per tile
    static constexpr bool kUnitCount = false;
    static constexpr int kMinBlocks = 6;       // resident blocks per CU the register budget must allow
    static constexpr int kPhases = 1;            // cut phases (later ones on queued survivors)
    static constexpr float kScreen = 2.0f;
    struct Rec { int u, v; };
    struct Mid {};

    __device__ int64_t count(int64_t u) const {
        const int C = t3_mds[u].z;
        return t3i_off[C + 1] - t3i_off[C];
    }
    __device__ void info(int64_t u, int32_t *f) const {
        const int4 m1 = t3_mds[u];
        const int64_t o0 = t3i_off[m1.z];
        f[0] = (int32_t)o0; f[1] = (int32_t)(t3i_off[m1.z + 1] - o0); f[2] = m1.x; f[3] = 0;
    }
    template <class LDS>
    __device__ void prepare(LDS &, int64_t, int) const {}
    template <class LDS>
    __device__ bool eval(int64_t u, int32_t local, const int32_t *f, const LDS &, Rec &r, Mid &) const {
        const int v = f[0] + local;
        r.u = (int)u; r.v = v;
        const int4 m2 = t3_mds[v];
        const float4 a = md_a[f[2]], e = md_a[m2.z];
        float cv, sg;
        if (!pair_pass_rq(p, P3{a.x, a.y, a.z}, md_rq[f[2]], P3{e.x, e.y, e.z}, md_rq[m2.z], cv, sg)) return false;
        // FP32 screen of the r-z chi2 (see kScreen)
        const int4 m1 = t3_mds[u];
        const int ids[5] = {m1.x, m1.y, m1.z, m2.y, m2.z};
        float x[5], y[5], z[5], rt[5];
        bool en[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const float4 h = k == 0 ? a : k == 4 ? e : md_a[ids[k]];
            const float2 rq = md_rq[ids[k]];
            x[k] = h.x; y[k] = h.y; z[k] = h.z; rt[k] = rq.x;
            en[k] = signbit(rq.y);
        }
        return !(t5_chi2rz_f32(p, x, y, z, rt, en) > kScreen * p.chi2rz);
    }
    __device__ void write(int64_t pos, const Rec &r) const { pre[pos] = make_int2(r.u, r.v); }
};

// anchors of a T5 candidate, FP64, with module kinds and layers
struct T5Anchors {
    double x[5], y[5], z[5];
    bool endc[5];
    int lay[5];
};

__device__ __forceinline__ void load_t5_anchors(const int4 *t3_mds, const float4 *md_a, const ModConst *mod,
                                                int32_t n_mod, int u, int v, T5Anchors &t) {
    const int4 m1 = t3_mds[u], m2 = t3_mds[v];
    const int ids[5] = {m1.x, m1.y, m1.z, m2.y, m2.z};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const float4 a = md_a[ids[k]];
        const ModConst &mc = mod[__float_as_int(a.w) % n_mod];
        t.x[k] = a.x; t.y[k] = a.y; t.z[k] = a.z; t.endc[k] = mc.kind != 0; t.lay[k] = mc.layer;
    }
}

template <bool kScoreCut>
struct T5FitStage {
    const int2 *pre;
    const int4 *t3_mds;
    const float4 *md_a;
    const ModConst *mod;
    CutParams p;
    ModelDev mdl;
    int32_t n_mod, mode;
    float score_min;
    int2 *t5_t3;
    float *chi2_rphi, *chi2_rz;
    float *fitf;                  // [n_t5][8]: the fit outputs of each written T5
    static constexpr int kEnt = 0;
    static constexpr int kStage = 4;
    static constexpr int kWin = 512;             // anchors staged per tile
    static constexpr bool kUnitCount = true;
    static constexpr int kMinBlocks = 3;       // resident blocks per CU the register budget must allow
    static constexpr int kPhases = 1;            // cut phases (later ones on queued survivors)
    struct Rec { int u, v; float cr, cz; float fo[kNFitOut]; };
    struct Mid {};

    __device__ int64_t count(int64_t) const { return 1; }
    __device__ void info(int64_t, int32_t *f) const { f[0] = f[1] = f[2] = f[3] = 0; }
    template <class LDS>
    __device__ void prepare(LDS &, int64_t, int) const {}
    template <class LDS>
    __device__ bool eval(int64_t q, int32_t, const int32_t *, const LDS &, Rec &r, Mid &) const {
        const int2 uv = pre[q];
        r.u = uv.x; r.v = uv.y;
        T5Anchors t;
        load_t5_anchors(t3_mds, md_a, mod, n_mod, uv.x, uv.y, t);
        Fit5 fit;
        t5_fit(p, t.x, t.y, t.z, t.endc, fit);
        r.cr = (float)fit.chi2_rphi; r.cz = (float)fit.chi2_rz;
        if (!(fit.chi2_rz <= (double)p.chi2rz)) return false;
        if (mode == 1 && !(fit.chi2_rphi <= (double)p.chi2rphi)) return false;
        t5_fit_outputs(t.x, t.y, fit, r.fo);
        if (kScoreCut) {
            float ff[kNFitFeat], ft[kNFeat];
            t5_fit_features_from(p, r.fo, (double)r.cr, (double)r.cz, ff);
            t5_features_from(p, t.x, t.y, t.z, t.lay, t.endc, ff, ft);
            if (!(score_min <= mlp_f32(mdl, ft))) return false;
        }
        return true;
    }
    __device__ void write(int64_t pos, const Rec &r) const {
        t5_t3[pos] = make_int2(r.u, r.v);
        chi2_rphi[pos] = r.cr;
        chi2_rz[pos] = r.cz;
        float4 *f4 = reinterpret_cast<float4 *>(fitf + pos * 8);
        f4[0] = make_float4(r.fo[0], r.fo[1], r.fo[2], r.fo[3]);
        f4[1] = make_float4(r.fo[4], r.fo[5], r.cr, r.cz);
    }
};

// T5 features (from the anchors and the fit features stored by the fit stage)
// and the T5-DNN score, one thread per T5 (FP32 vector ALU).
__global__ __launch_bounds__(kBlock) void k_t5_score_f32(T5FitStage<false> s, const int64_t *n_dev, int64_t cap,
                                                         float *score, float *feat, int do_mlp) {
    int64_t n = dev_count(n_dev, cap);
    for (int64_t i = grid_tid(); i < n; i += grid_stride()) {
        const int2 uv = s.t5_t3[i];
        T5Anchors t;
        load_t5_anchors(s.t3_mds, s.md_a, s.mod, s.n_mod, uv.x, uv.y, t);
        const float4 a = reinterpret_cast<const float4 *>(s.fitf)[2 * i];
        const float4 b = reinterpret_cast<const float4 *>(s.fitf)[2 * i + 1];
        const float fo[kNFitOut] = {a.x, a.y, a.z, a.w, b.x, b.y};
        float ff[kNFitFeat], ft[kNFeat];
        t5_fit_features_from(s.p, fo, (double)b.z, (double)b.w, ff);
        t5_features_from(s.p, t.x, t.y, t.z, t.lay, t.endc, ff, ft);
        if (feat) {
#pragma unroll
            for (int k = 0; k < kNFeat; ++k) feat[i * kNFeat + k] = ft[k];
        }
        if (do_mlp) score[i] = s.mode == 0 ? mlp_f32(s.mdl, ft) : __builtin_nanf("");
    }
}

// T5 features and the T5-DNN score on the matrix cores: each thread computes
// one T5's features into the block's LDS tile (standardised BF16), then the
// block scores the tile with MFMA; feature rows go to HBM only when asked for.
__global__ __launch_bounds__(kTileRows, 3) void k_t5_score_mfma(T5FitStage<false> s, const int64_t *n_dev,
                                                             int64_t cap, float *score, float *feat) {
    __shared__ __align__(16) uint16_t tile[kTileRows * kRowStride];
    __shared__ MlpFrags fr;
    mlp_tile_init(&fr, tile, s.mdl);
    const int64_t n = dev_count(n_dev, cap);
    for (int64_t row0 = (int64_t)blockIdx.x * kTileRows; row0 < n; row0 += (int64_t)gridDim.x * kTileRows) {
        const int nrows = n - row0 < kTileRows ? (int)(n - row0) : kTileRows;
        const int64_t i = row0 + threadIdx.x;
        __syncthreads();                               // the previous tile is consumed
        if (threadIdx.x < nrows) {
            const int2 uv = s.t5_t3[i];
            T5Anchors t;
            load_t5_anchors(s.t3_mds, s.md_a, s.mod, s.n_mod, uv.x, uv.y, t);
            const float4 a = reinterpret_cast<const float4 *>(s.fitf)[2 * i];
            const float4 b = reinterpret_cast<const float4 *>(s.fitf)[2 * i + 1];
            const float fo[kNFitOut] = {a.x, a.y, a.z, a.w, b.x, b.y};
            float ff[kNFitFeat], ft[kNFeat];
            t5_fit_features_from(s.p, fo, (double)b.z, (double)b.w, ff);
            t5_features_from(s.p, t.x, t.y, t.z, t.lay, t.endc, ff, ft);
            if (feat) {
#pragma unroll
                for (int k = 0; k < kNFeat; ++k) feat[i * kNFeat + k] = ft[k];
            }
            mlp_tile_store_row(tile, threadIdx.x, ft, s.mdl);
        }
        __syncthreads();
        mlp_tile_score(tile, &fr, nrows, s.mdl, score + row0);
    }
}

// One resident wave of blocks (3 per CU on 256 CUs) that walk the tiles, so
// each block stages the weights once for several tiles and no second round of
// blocks waits behind the first.
constexpr int kScoreGrid = 3 * 256;

static inline int grid_for_tiles(int64_t n) {
    int64_t g = (n + kTileRows - 1) / kTileRows;
    if (g < 1) g = 1;
    if (g > kScoreGrid) g = kScoreGrid;
    return (int)g;
}

// ---------------------------------------------------- per-event offsets

// Per-event first indices: MD from the module offsets, LS from the LS CSR by
// inner MD, T3 from the T3 CSR by inner MD (T3 are sorted by it), T5 by a
// search over their inner T3 (T5 are sorted by it).
__global__ __launch_bounds__(64) void k_event_offsets(const int64_t *md_mod_off, const int64_t *ls_off,
                                                      const int64_t *t3i_off, const int2 *t5_t3,
                                                      const int64_t *counts, int64_t cap_md, int64_t cap_t5,
                                                      int32_t n_mod, int32_t n_ev, int64_t *out) {
    // one wavefront per event boundary e = 0..n_ev
    const int e = blockIdx.x, lane = threadIdx.x;
    const int64_t nmd = dev_count(counts + 0, cap_md), nt5 = dev_count(counts + 3, cap_t5);
    int64_t md0 = md_mod_off[(int64_t)e * n_mod];
    if (md0 > nmd) md0 = nmd;
    const int64_t ls0 = ls_off[md0], t30 = t3i_off[md0];
    // first T5 whose inner T3 is >= t30, by a 64-way search: the answer
    // stays in [lo, hi]; each step probes 64 evenly spaced entries and keeps
    // the gap between the last probe below t30 and the first one not below
    int64_t lo = 0, hi = nt5;
    while (hi - lo > 64) {
        const int64_t step = (hi - lo + 63) / 64;
        const int64_t p = lo + lane * step;
        const bool below = p < hi && t5_t3[p].x < t30;
        const int c = __popcll(__ballot(below));   // the probes below t30 are a prefix
        const int64_t l0 = lo;
        if (c == 0) {
            hi = lo;
        } else {
            lo = l0 + (int64_t)(c - 1) * step + 1;
            const int64_t pc = l0 + (int64_t)c * step;
            if (pc < hi) hi = pc;
        }
    }
    int64_t t50 = lo;
    if (hi > lo) {
        const int64_t q = lo + lane;
        const bool below = q < hi && t5_t3[q].x < t30;
        t50 = lo + __popcll(__ballot(below));
    }
    if (lane == 0) {
        out[0 * (n_ev + 1) + e] = md0;
        out[1 * (n_ev + 1) + e] = ls0;
        out[2 * (n_ev + 1) + e] = t30;
        out[3 * (n_ev + 1) + e] = t50;
    }
}

// ------------------------------------------------------------- pipeline

struct GmKey {
    const float4 *md_a;
    __device__ int operator()(int64_t i) const { return __float_as_int(md_a[i].w); }
};
struct T3InKey {
    const int4 *t;
    __device__ int operator()(int64_t i) const { return t[i].x; }
};

hipError_t set_single_event(int64_t *ev_off, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_set_single_event, dim3(1), dim3(64), 0, st, ev_off, n);
    return hipGetLastError();
}

hipError_t run_pipeline(const RunArgs &a, const Work &w, const Outputs &o, hipStream_t st) {
    const int32_t n_mod = a.g.n_mod, n_sens = a.g.n_sens;
    const int64_t ngm = (int64_t)a.n_ev * n_mod;
    int64_t *cnt = o.counts;

    hipEvent_t *ev = a.timing;
    mark(ev, 0, st);
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, st, cnt, (int64_t)LST_COUNTS_LEN, (int64_t)0);
    if (a.stop_before == 1) return hipGetLastError();
    // a1: bin hits by (event, sensor)
    mark(ev, 2, st);
    {
        int nr = (n_sens + kFineRange - 1) / kFineRange;
        if (a.tune.bin_split > nr) nr = a.tune.bin_split;
        const int rw = (n_sens + nr - 1) / nr;
        const int grid_t = (int)w.max_bin_tiles;
        hipLaunchKernelGGL(k_bin_tiles, dim3(1), dim3(1024), 0, st, a.ev_off, a.n_ev, nr, w.bin_tbase, w.bin_nent);
        hipLaunchKernelGGL(k_bin_count, dim3(grid_t), dim3(kBinThreads), 0, st, a.sensor, a.ev_off, a.n_ev, n_sens, nr,
                           rw, (const int64_t *)w.bin_tbase, w.bin_cnt, cnt);
        scan(CntF{w.bin_cnt}, w.bin_nent, w.max_bin_entries, w, w.bin_cpos, nullptr, st);
        hipLaunchKernelGGL(k_bin_scatter, dim3(grid_t), dim3(kScatterThreads), 0, st, a.x, a.y, a.z, a.sensor, a.ev_off,
                           a.n_ev, n_sens, nr, rw, (const int64_t *)w.bin_tbase, (const int64_t *)w.bin_cpos,
                           w.bin_tmp, w.bin_tsens);
        const int xcd_map = a.n_ev >= kXcds ? 1 : 0;
        const int grid_f = xcd_map ? (a.n_ev + kXcds - 1) / kXcds * kXcds * nr : a.n_ev * nr;
        hipLaunchKernelGGL(k_bin_fine, dim3(grid_f), dim3(kFineThreads), 0, st, (const float4 *)w.bin_tmp,
                           (const int32_t *)w.bin_tsens, (const int64_t *)w.bin_tbase, (const int64_t *)w.bin_cpos,
                           (const int64_t *)w.bin_nent, a.n_ev, n_sens, nr, rw, xcd_map, w.bin_off, w.bin_hit);
    }
    mark(ev, 3, st);

    if (a.stop_before == 2) return hipGetLastError();
    // a2: mini-doublets, anchored on (event, module)
    MDStage md{w.bin_off, w.bin_hit, a.g.mod, a.g.box, o.counts, a.p, n_mod, n_sens, o.md_hits, w.md_a, w.md_o,
               w.md_rq};
    mark(ev, 14, st);
    run_stage(md, nullptr, ngm, w, cnt + LST_COUNT_MD, w.cap_md, cnt, st, ev, 2, a.tune);
    hipLaunchKernelGGL(k_fill_offsets<GmKey>, dim3(grid_for(w.cap_md + 1)), dim3(kBlock), 0, st, GmKey{w.md_a},
                       cnt + LST_COUNT_MD, w.cap_md, nullptr, ngm, w.md_mod_off);
    mark(ev, 15, st);

    if (a.stop_before == 3) return hipGetLastError();
    // a3: line segments, one inner MD per lane over the trimmed runs of its
    // module-map row; CSR offsets by inner MD from the per-MD counts
    mark(ev, 16, st);
    LsArgs la{w.md_a, w.md_o, w.md_rq, w.md_mod_off, a.g, a.p, w.ls_cnt, w.ls_chunk, w.cap_ls, w.ls_top, cnt,
              w.cap_md};
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, w.ls_top, w.t3_n_ovf);
    {
        const int64_t tiles = (w.cap_md + 64 * kLsWaves - 1) / (64 * kLsWaves);
        int nb = (int)(tiles < kLsBlocks ? tiles : kLsBlocks);
        nb = round_up_xcd(nb < 1 ? 1 : nb);
        mark(ev, 6, st);
        hipLaunchKernelGGL(k_ls_eval, dim3(nb), dim3(kLsBlock), 0, st, la);
        mark(ev, 7, st);
        scan(CntF{w.ls_cnt}, cnt + LST_COUNT_MD, w.cap_md, w, w.ls_off, nullptr, st);
        hipLaunchKernelGGL(k_ls_place, dim3(grid_for(w.cap_ls)), dim3(kBlock), 0, st, la, (const int64_t *)w.ls_off,
                           (int2 *)o.ls_md, w.cap_ls);
    }
    mark(ev, 17, st);

    if (a.stop_before == 4) return hipGetLastError();
    // a4: triplets, anchored on the inner LS
    T3Direct t3{o.ls_md, w.ls_off, w.cap_ls, w.md_a, w.md_o, w.md_rq, a.p, w.t3_wcnt, w.t3_woff, w.t3_bits,
                a.tune.t3_masks, w.t3_nw, w.t3_cn, w.t3_ovf, w.t3_n_ovf, w.t3_pos, o.t3_ls, w.t3_mds, w.cap_t3,
                cnt};
    mark(ev, 18, st);
    {
        const int64_t tiles = (w.cap_ls + kBlock - 1) / kBlock;
        int nb = (int)(tiles < kT3Blocks ? tiles : kT3Blocks);
        nb = round_up_xcd(nb < 1 ? 1 : nb);
        mark(ev, 8, st);
        hipLaunchKernelGGL(k_t3_count, dim3(nb), dim3(kBlock), 0, st, t3);
        mark(ev, 9, st);
        scan(CntF{w.t3_wcnt}, w.t3_nw, w.cap_ls / 64 + 1, w, w.t3_woff, nullptr, st);
        hipLaunchKernelGGL(k_t3_write, dim3(nb), dim3(kBlock), 0, st, t3);
        hipLaunchKernelGGL(k_t3_write_listed, dim3(kT3OvfBlocks), dim3(kBlock), 0, st, t3);
        hipLaunchKernelGGL(k_t3_md_off, dim3(grid_for(w.cap_md + 1)), dim3(kBlock), 0, st, t3,
                           (const int64_t *)(cnt + LST_COUNT_MD), w.cap_md, w.t3i_off);
    }
    mark(ev, 19, st);

    if (a.stop_before == 5) return hipGetLastError();
    // a5: quintuplets, anchored on the inner T3: FP32 beam-line cuts, then the
    // FP64 fits on the dense list of pre-candidates
    const bool score_cut = a.mode == 0 && a.score_min == a.score_min;
    T5PreStage t5p{w.t3_mds, w.t3i_off, w.md_a, w.md_rq, a.g.mod, a.p, n_mod, w.t5_pre};
    mark(ev, 10, st);
    run_stage(t5p, cnt + LST_COUNT_T3, w.cap_t3, w, cnt + LST_COUNT_T5PRE, w.cap_t5pre, cnt, st, nullptr, 0, a.tune);
    T5FitStage<false> t5{w.t5_pre, w.t3_mds, w.md_a, a.g.mod, a.p, a.m, n_mod, a.mode, a.score_min, o.t5_t3,
                         o.t5_chi2_rphi, o.t5_chi2_rz, w.t5_fitf};
    if (score_cut) {
        T5FitStage<true> t5c{w.t5_pre, w.t3_mds, w.md_a, a.g.mod, a.p, a.m, n_mod, a.mode, a.score_min, o.t5_t3,
                             o.t5_chi2_rphi, o.t5_chi2_rz, w.t5_fitf};
        run_stage(t5c, cnt + LST_COUNT_T5PRE, w.cap_t5pre, w, cnt + LST_COUNT_T5, w.cap_t5, cnt, st, nullptr, 0, a.tune);
    } else {
        run_stage(t5, cnt + LST_COUNT_T5PRE, w.cap_t5pre, w, cnt + LST_COUNT_T5, w.cap_t5, cnt, st, nullptr, 0, a.tune);
    }
    mark(ev, 11, st);

    if (a.stop_before == 6) return hipGetLastError();
    // a6: features and T5-DNN scores (BF16 MFMA runs over the feature rows;
    // a score cut forces the FP32 path, which the T5 stage itself applied)
    bool mfma = a.mode == 0 && a.precision == 1 && !score_cut;
    mark(ev, 12, st);
    if (mfma)
        hipLaunchKernelGGL(k_t5_score_mfma, dim3(grid_for_tiles(w.cap_t5)), dim3(kTileRows), 0, st, t5,
                           cnt + LST_COUNT_T5, w.cap_t5, o.t5_score, o.t5_feat);
    else
        hipLaunchKernelGGL(k_t5_score_f32, dim3(grid_for(w.cap_t5)), dim3(kBlock), 0, st, t5,
                           cnt + LST_COUNT_T5, w.cap_t5, o.t5_score, o.t5_feat, 1);
    mark(ev, 13, st);
    if (a.ev_obj_off) {
        hipLaunchKernelGGL(k_event_offsets, dim3(a.n_ev + 1), dim3(64), 0, st, w.md_mod_off, w.ls_off,
                           w.t3i_off, o.t5_t3, cnt, w.cap_md, w.cap_t5, n_mod, a.n_ev, a.ev_obj_off);
    }
    mark(ev, 1, st);
    return hipGetLastError();
}

}  // namespace lst
