// C ABI of the LST object builder: context, geometry / model loading,
// workspace layout and the build / score entry points declared in lst.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lst.h"
#include "lst_internal.h"
#include "lst_tc.h"
#include "lst_graph.h"

using namespace lst;

// Device scratch of the allocation-free build (lst_build_objects_noalloc):
// one copy per GPU, allocated with the library's code object and held until
// the process ends. Host code never passes `scratch` itself to a kernel: its
// device address on each GPU comes from hipGetSymbolAddress, taken once per
// device when a context is created there.
constexpr size_t kNoAllocScratchBytes = (size_t)LST_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device `device` (null on failure).
static hipError_t scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

struct lst_ctx {
    int device = 0;
    std::string err;
    // geometry
    bool geom_loaded = false;
    int32_t n_mod = 0, n_barrel = 0, n_map = 0;
    CutParams cp{};
    ModConst *d_mod = nullptr;
    int32_t *d_map_off = nullptr, *d_map_tgt = nullptr;
    ModBox *d_box = nullptr;
    int32_t *d_run_off = nullptr;
    RunRec *d_runs = nullptr;
    int32_t n_runs = 0;
    // model
    bool model_loaded = false;
    float *d_model = nullptr;
    ModelDev md{};
    // stage timing
    bool timing = false, events_made = false;
    hipEvent_t tev[kTimingEvents];
    // launch shapes
    Tuning tune = kDefaultTuning;
    // edge classifier
    bool gnn_loaded = false;
    void *d_gnn = nullptr;
    GnnDev gnn{};
    // this device's address of the static scratch of lst_build_objects_noalloc
    void *noalloc_ws = nullptr;
    // failure injection: builds stop before this pipeline stage and fail (0: off)
    int32_t fail_stage = 0;
};

static lst_status fail(lst_ctx *c, lst_status s, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIP_TRY(ctx, expr)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(ctx, LST_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

extern "C" {

const char *lst_status_string(lst_status s) {
    switch (s) {
        case LST_OK: return "ok";
        case LST_E_INVAL: return "invalid argument";
        case LST_E_STATE: return "geometry or model not loaded";
        case LST_E_CAPACITY: return "capacity exceeded";
        case LST_E_HIP: return "HIP runtime error";
        case LST_E_NOMEM: return "out of device memory";
        default: return "unknown status";
    }
}

const char *lst_last_error(const lst_ctx *c) { return c ? c->err.c_str() : "null context"; }

lst_status lst_create(int device, lst_ctx **out) {
    if (!out) return LST_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LST_E_INVAL;
    if (device >= kMaxDevices) return LST_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return LST_E_HIP;
    lst_ctx *c = new lst_ctx();
    c->device = device;
    if (const char *fs = getenv("LST_FAIL_AT_STAGE")) {
        const int k = atoi(fs);
        c->fail_stage = k >= 1 && k <= kFailStages ? k : 0;
    }
    if (scratch_address(device, &c->noalloc_ws) != hipSuccess) {
        delete c;
        return LST_E_HIP;
    }
    *out = c;
    return LST_OK;
}

static void free_geom(lst_ctx *c) {
    if (c->d_mod) (void)hipFree(c->d_mod);
    if (c->d_map_off) (void)hipFree(c->d_map_off);
    if (c->d_map_tgt) (void)hipFree(c->d_map_tgt);
    if (c->d_box) (void)hipFree(c->d_box);
    if (c->d_run_off) (void)hipFree(c->d_run_off);
    if (c->d_runs) (void)hipFree(c->d_runs);
    c->d_mod = nullptr; c->d_map_off = c->d_map_tgt = nullptr;
    c->d_box = nullptr; c->d_run_off = nullptr; c->d_runs = nullptr;
    c->geom_loaded = false;
}

void lst_destroy(lst_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    free_geom(c);
    if (c->d_model) (void)hipFree(c->d_model);
    if (c->d_gnn) (void)hipFree(c->d_gnn);
    if (c->events_made)
        for (int i = 0; i < kTimingEvents; ++i) (void)hipEventDestroy(c->tev[i]);
    delete c;
}

lst_status lst_load_geometry(lst_ctx *c, const void *blob, size_t nbytes) {
    if (!c || !blob) return LST_E_INVAL;
    GeomHost g;
    std::string err;
    if (!parse_geometry(blob, nbytes, g, err)) return fail(c, LST_E_INVAL, "%s", err.c_str());
    // hit binning sorts at most kBinRangesMax ranges of kBinRangeSensors sensors per event
    if (2 * (int64_t)g.n_mod > (int64_t)kBinRangeSensors * kBinRangesMax)
        return fail(c, LST_E_INVAL, "geometry blob: %d modules, at most %d supported", g.n_mod,
                    kBinRangeSensors / 2 * kBinRangesMax);
    const size_t nm = (size_t)g.n_mod;
    const std::vector<ModConst> &mods = g.mods;
    const std::vector<ModBox> &boxes = g.boxes;
    const std::vector<int32_t> &moff = g.map_off, &mtgt = g.map_tgt, &run_off = g.run_off;
    const std::vector<RunRec> &runs = g.runs;
    HIP_TRY(c, hipSetDevice(c->device));
    free_geom(c);
    if (hipMalloc(&c->d_mod, sizeof(ModConst) * nm) != hipSuccess ||
        hipMalloc(&c->d_map_off, sizeof(int32_t) * (nm + 1)) != hipSuccess ||
        hipMalloc(&c->d_map_tgt, sizeof(int32_t) * mtgt.size()) != hipSuccess ||
        hipMalloc(&c->d_box, sizeof(ModBox) * nm) != hipSuccess ||
        hipMalloc(&c->d_run_off, sizeof(int32_t) * (nm + 1)) != hipSuccess ||
        hipMalloc(&c->d_runs, sizeof(RunRec) * runs.size()) != hipSuccess) {
        free_geom(c);
        return fail(c, LST_E_NOMEM, "geometry tables");
    }
    HIP_TRY(c, hipMemcpy(c->d_mod, mods.data(), sizeof(ModConst) * nm, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_map_off, moff.data(), sizeof(int32_t) * (nm + 1), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_map_tgt, mtgt.data(), sizeof(int32_t) * mtgt.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_box, boxes.data(), sizeof(ModBox) * nm, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_run_off, run_off.data(), sizeof(int32_t) * (nm + 1), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_runs, runs.data(), sizeof(RunRec) * runs.size(), hipMemcpyHostToDevice));
    c->n_runs = (int32_t)run_off[nm];
    c->n_mod = g.n_mod; c->n_barrel = g.n_barrel; c->n_map = g.n_map;
    c->cp = g.cp;
    c->geom_loaded = true;
    return LST_OK;
}

lst_status lst_load_model(lst_ctx *c, const void *blob, size_t nbytes) {
    if (!c || !blob) return LST_E_INVAL;
    ModelHost mh;
    std::string err;
    if (!parse_model(blob, nbytes, mh, err)) return fail(c, LST_E_INVAL, "%s", err.c_str());
    const std::vector<float> &w = mh.w;
    const size_t nf = w.size();
    HIP_TRY(c, hipSetDevice(c->device));
    if (c->d_model) { (void)hipFree(c->d_model); c->d_model = nullptr; c->model_loaded = false; }
    if (hipMalloc(&c->d_model, 4 * nf) != hipSuccess) return fail(c, LST_E_NOMEM, "model");
    HIP_TRY(c, hipMemcpy(c->d_model, w.data(), 4 * nf, hipMemcpyHostToDevice));
    float *d = c->d_model;
    ModelDev m{};
    m.mu = d; d += kNFeat;
    m.sd = d; d += kNFeat;
    m.W1 = d; d += kH1 * kNFeat;
    m.b1 = d; d += kH1;
    m.W2 = d; d += kH2 * kH1;
    m.b2 = d; d += kH2;
    m.w3 = d; d += kH2;
    m.b3 = w[nf - 1];
    c->md = m;
    c->model_loaded = true;
    return LST_OK;
}

// Carve the workspace; with base == nullptr only the size is computed.
static size_t layout(const lst_ctx *c, const lst_caps *k, char *base, Work *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const int64_t nsens = 2 * (int64_t)c->n_mod, nmod = c->n_mod;
    const int64_t ev = k->events > 0 ? k->events : 1;
    const int64_t md = k->md > 0 ? k->md : 1;
    // tiles of kMinTile candidates, with room for the largest tile's rounding
    const int64_t max_tiles = (k->cand + kMinTile - 1) / kMinTile + 8;
    // anchors: modules (MD, LS), LS (T3), T3 (T5 pre-cuts), pre-candidates (T5 fits)
    int64_t anchors = ev * nmod;
    for (int64_t v : {md, k->ls, k->t3, k->cand})
        if (v > anchors) anchors = v;
    Work x{};
    x.cap_hits = k->hits; x.cap_ev = ev; x.cap_md = md; x.cap_ls = k->ls; x.cap_t3 = k->t3;
    x.cap_t5 = k->t5; x.cap_cand = k->cand; x.max_tiles = max_tiles; x.n_anchor_cap = anchors;
    const int64_t hits = k->hits > 0 ? k->hits : 1;
    x.bin_off = (int64_t *)take(8 * (ev * nsens + 1));
    x.bin_hit = (float4 *)take(16 * hits);
    // coarse binning tiles: every event adds at most one partial tile
    x.max_bin_tiles = hits / kBinTileHits + ev + 1;
    // ranges per event: enough for kBinRangeSensors sensor ids each, or the largest bin_split
    const int64_t nr_need = (nsens + kBinRangeSensors - 1) / kBinRangeSensors;
    const int64_t nr_max = nr_need > kBinSplitMax ? nr_need : kBinSplitMax;
    x.max_bin_entries = x.max_bin_tiles * nr_max;
    x.bin_tbase = (int64_t *)take(8 * (ev + 1));
    x.bin_nent = (int64_t *)take(8);
    x.bin_cnt = (int32_t *)take(4 * x.max_bin_entries);
    x.bin_cpos = (int64_t *)take(8 * (x.max_bin_entries + 1));
    x.bin_tmp = (float4 *)take(16 * hits);
    x.bin_tsens = (int32_t *)take(4 * hits);
    x.cand_off = (int64_t *)take(8 * (anchors + 1));
    x.scan_part = (int64_t *)take(8 * (kScanBlocks + 1));
    x.tile_anchor = (int32_t *)take(4 * (max_tiles + 1));
    x.tile_cnt = (int32_t *)take(4 * max_tiles);
    x.tile_pre = (int64_t *)take(8 * (max_tiles + 1));
    x.ntiles = (int64_t *)take(8);
    x.rec_scratch = (void *)take((size_t)kMaxRecBytes * kMinTile * max_tiles);
    x.md_a = (float4 *)take(16 * md);
    x.md_o = (float2 *)take(8 * md);
    x.md_rq = (float2 *)take(8 * md);
    x.md_mod_off = (int64_t *)take(8 * (ev * nmod + 1));
    x.ls_off = (int64_t *)take(8 * (md + 1));
    x.ls_cnt = (int32_t *)take(4 * md);
    x.ls_chunk = (int4 *)take(16 * (k->ls > 0 ? k->ls : 1));
    x.ls_top = (unsigned long long *)take(8);
    x.t3_mds = (int4 *)take(16 * (k->t3 > 0 ? k->t3 : 1));
    x.t3_wcnt = (int32_t *)take(4 * (k->ls / 64 + 1));
    x.t3_woff = (int64_t *)take(8 * (k->ls / 64 + 2));
    x.t3_nw = (int64_t *)take(8);
    x.t3_pos = (int64_t *)take(8 * (k->ls + 1));
    x.t3_bits = (unsigned long long *)take(8 * kT3MaxMasks * (k->ls / 64 + 1));
    x.t3_cn = (int2 *)take(8 * (k->ls > 0 ? k->ls : 1));
    x.t3_ovf = (int32_t *)take(4 * (k->ls / 64 + 1));
    x.t3_n_ovf = (unsigned long long *)take(8);

    x.t3i_off = (int64_t *)take(8 * (md + 1));
    x.cap_t5pre = k->cand;
    x.t5_pre = (int2 *)take(8 * (k->cand > 0 ? k->cand : 1));
    x.t5_fitf = (float *)take(4 * 8 * (k->t5 > 0 ? k->t5 : 1));
    x.ev_off = (int64_t *)take(16);
    if (w) *w = x;
    return off;
}

static lst_status check_caps(lst_ctx *c, const lst_caps *k) {
    if (!k) return fail(c, LST_E_INVAL, "null caps");
    if (k->hits < 0 || k->events < 1 || k->md < 1 || k->ls < 1 || k->t3 < 1 || k->t5 < 1 || k->cand < 1)
        return fail(c, LST_E_INVAL, "capacities must be positive");
    const int64_t lim = (int64_t)1 << 31;
    if (k->hits >= lim || k->md >= lim || k->ls >= lim || k->t3 >= lim || k->t5 >= lim ||
        k->events * 2 * (int64_t)c->n_mod >= lim || k->cand > ((int64_t)1 << 40))
        return fail(c, LST_E_INVAL, "capacity beyond the 32-bit object index range");
    return LST_OK;
}

lst_status lst_workspace_size(const lst_ctx *c, const lst_caps *k, size_t *bytes) {
    if (!c || !bytes) return LST_E_INVAL;
    if (!c->geom_loaded) return LST_E_STATE;
    lst_status s = check_caps(const_cast<lst_ctx *>(c), k);
    if (s != LST_OK) return s;
    *bytes = layout(c, k, nullptr, nullptr);
    return LST_OK;
}

static lst_status build_common(lst_ctx *c, const lst_hits *h, const int64_t *ev_off, int32_t n_ev,
                               const lst_options *opt, const lst_caps *k, lst_objects *out,
                               int64_t *ev_obj_off, void *ws, size_t ws_bytes, void *stream, bool single) {
    if (!c) return LST_E_INVAL;
    if (!c->geom_loaded || !c->model_loaded) return fail(c, LST_E_STATE, "load geometry and model first");
    if (!h || !opt || !out || !ws) return fail(c, LST_E_INVAL, "null argument");
    lst_status s = check_caps(c, k);
    if (s != LST_OK) return s;
    if (h->n < 0 || h->n > k->hits) return fail(c, LST_E_INVAL, "hit count %lld exceeds caps.hits", (long long)h->n);
    if (h->n > 0 && (!h->x || !h->y || !h->z || !h->sensor)) return fail(c, LST_E_INVAL, "null hit array");
    if (n_ev < 1 || n_ev > k->events) return fail(c, LST_E_INVAL, "event count %d outside [1, caps.events]", n_ev);
    if (!single && !ev_off) return fail(c, LST_E_INVAL, "null event offsets");
    if (!out->md_hits || !out->ls_md || !out->t3_ls || !out->t5_t3 || !out->t5_score || !out->t5_chi2_rphi ||
        !out->t5_chi2_rz || !out->counts_dev)
        return fail(c, LST_E_INVAL, "null output array");
    if (opt->mode != LST_MODE_DNN && opt->mode != LST_MODE_PRE_DNN) return fail(c, LST_E_INVAL, "bad mode");
    if (opt->precision != LST_PREC_F32 && opt->precision != LST_PREC_BF16)
        return fail(c, LST_E_INVAL, "bad precision");
    if (((uintptr_t)ws & 255) != 0) return fail(c, LST_E_INVAL, "workspace must be 256-byte aligned");
    size_t need = layout(c, k, nullptr, nullptr);
    if (ws_bytes < need) return fail(c, LST_E_INVAL, "workspace %zu bytes, need %zu", ws_bytes, need);
    HIP_TRY(c, hipSetDevice(c->device));
    Work w{};
    layout(c, k, (char *)ws, &w);
    hipStream_t st = (hipStream_t)stream;
    if (single) {
        HIP_TRY(c, set_single_event(w.ev_off, h->n, st));
        ev_off = w.ev_off;
    }
    RunArgs a{};
    a.g.mod = c->d_mod; a.g.map_off = c->d_map_off; a.g.map_tgt = c->d_map_tgt;
    a.g.box = c->d_box; a.g.run_off = c->d_run_off; a.g.runs = c->d_runs;
    a.g.n_mod = c->n_mod; a.g.n_sens = 2 * c->n_mod; a.g.n_map = c->n_map;
    a.p = c->cp; a.m = c->md;
    a.x = h->x; a.y = h->y; a.z = h->z; a.sensor = h->sensor; a.n_hits = h->n;
    a.ev_off = ev_off; a.n_ev = n_ev;
    a.mode = opt->mode; a.precision = opt->precision; a.score_min = opt->score_min;
    a.ev_obj_off = ev_obj_off;
    a.timing = c->timing ? c->tev : nullptr;
    a.tune = c->tune;
    a.stop_before = c->fail_stage;
    Outputs o{};
    o.md_hits = (int2 *)out->md_hits; o.ls_md = (int2 *)out->ls_md; o.t3_ls = (int2 *)out->t3_ls;
    o.t5_t3 = (int2 *)out->t5_t3; o.t5_score = out->t5_score; o.t5_chi2_rphi = out->t5_chi2_rphi;
    o.t5_chi2_rz = out->t5_chi2_rz; o.t5_feat = out->t5_feat; o.counts = out->counts_dev;
    HIP_TRY(c, run_pipeline(a, w, o, st));
    if (c->fail_stage) {
        // the stages before it ran; leave the stream idle before reporting
        HIP_TRY(c, hipStreamSynchronize(st));
        return fail(c, LST_E_HIP, "injected failure before pipeline stage %d (failure injection is on)",
                    c->fail_stage);
    }
    if (opt->flags & LST_ASYNC) return LST_OK;
    int64_t cnt[LST_COUNTS_LEN];
    HIP_TRY(c, hipMemcpyAsync(cnt, out->counts_dev, sizeof(cnt), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    out->n_md = cnt[0]; out->n_ls = cnt[1]; out->n_t3 = cnt[2]; out->n_t5 = cnt[3];
    if (cnt[LST_COUNT_ERR] & 1) return fail(c, LST_E_INVAL, "sensor id out of range in the hits");
    if (cnt[LST_COUNT_ERR] & 8) return fail(c, LST_E_INVAL, "a mini-doublet's anchor hit lies off its sensor");
    if ((cnt[LST_COUNT_ERR] & 2) || cnt[0] > k->md || cnt[1] > k->ls || cnt[2] > k->t3 || cnt[3] > k->t5 ||
        cnt[LST_COUNT_T5PRE] > k->cand)
        return fail(c, LST_E_CAPACITY, "capacity exceeded: md %lld/%lld ls %lld/%lld t3 %lld/%lld t5 %lld/%lld cand %lld/%lld",
                    (long long)cnt[0], (long long)k->md, (long long)cnt[1], (long long)k->ls, (long long)cnt[2],
                    (long long)k->t3, (long long)cnt[3], (long long)k->t5, (long long)cnt[LST_COUNT_MAXCAND],
                    (long long)k->cand);
    return LST_OK;
}

lst_status lst_build_objects(lst_ctx *c, const lst_hits *h, const lst_options *opt, const lst_caps *k,
                             lst_objects *out, void *ws, size_t ws_bytes, void *stream) {
    return build_common(c, h, nullptr, 1, opt, k, out, nullptr, ws, ws_bytes, stream, true);
}

lst_status lst_build_objects_batched(lst_ctx *c, const lst_hits *h, const int64_t *ev_off, int32_t n_ev,
                                     const lst_options *opt, const lst_caps *k, lst_objects *out,
                                     int64_t *ev_obj_off, void *ws, size_t ws_bytes, void *stream) {
    return build_common(c, h, ev_off, n_ev, opt, k, out, ev_obj_off, ws, ws_bytes, stream, false);
}

// lst_build_objects with the static per-device scratch as its workspace: the
// same kernels, no allocation. Every stage initialises what it reads of the
// workspace, so the previous call's contents do no harm.
lst_status lst_build_objects_noalloc(lst_ctx *c, const lst_hits *h, const lst_options *opt, const lst_caps *k,
                                     lst_objects *out, void *stream) {
    if (!c) return LST_E_INVAL;
    if (!c->geom_loaded) return fail(c, LST_E_STATE, "load geometry and model first");
    lst_status s = check_caps(c, k);
    if (s != LST_OK) return s;
    const size_t need = layout(c, k, nullptr, nullptr);
    if (need > kNoAllocScratchBytes)
        return fail(c, LST_E_INVAL, "these capacities need %zu bytes of workspace; the allocation-free build "
                    "has %zu (LST_NOALLOC_SCRATCH_MIB MiB): use lst_build_objects with a workspace",
                    need, kNoAllocScratchBytes);
    if (!c->noalloc_ws) return fail(c, LST_E_STATE, "no static scratch address on this device");
    return build_common(c, h, nullptr, 1, opt, k, out, nullptr, c->noalloc_ws, kNoAllocScratchBytes, stream, true);
}

lst_status lst_set_fail_stage(lst_ctx *c, int32_t stage) {
    if (!c) return LST_E_INVAL;
    if (stage < 0 || stage > kFailStages) return fail(c, LST_E_INVAL, "fail stage %d outside [0, %d]", stage, kFailStages);
    c->fail_stage = stage;
    return LST_OK;
}

lst_status lst_set_timing(lst_ctx *c, int32_t enable) {
    if (!c) return LST_E_INVAL;
    HIP_TRY(c, hipSetDevice(c->device));
    if (enable && !c->events_made) {
        for (int i = 0; i < kTimingEvents; ++i) HIP_TRY(c, hipEventCreate(&c->tev[i]));
        c->events_made = true;
    }
    c->timing = enable != 0;
    return LST_OK;
}

lst_status lst_stage_times(lst_ctx *c, float *ms, int32_t n) {
    if (!c || !ms || n < 0) return LST_E_INVAL;
    if (!c->events_made) return fail(c, LST_E_STATE, "timing was never enabled");
    for (int i = 0; i < n && i < kTimingWindows; ++i)
        HIP_TRY(c, hipEventElapsedTime(&ms[i], c->tev[2 * i], c->tev[2 * i + 1]));
    return LST_OK;
}

// ------------------------------------------------------ edge classifier


lst_status lst_load_gnn(lst_ctx *c, const void *blob, size_t nbytes) {
    if (!c || !blob) return LST_E_INVAL;
    GnnHost gh;
    std::string err;
    if (!parse_gnn(blob, nbytes, gh, err)) return fail(c, LST_E_INVAL, "%s", err.c_str());
    const std::vector<uint16_t> &frag = gh.frag;
    const std::vector<float> &bias = gh.bias;
    GnnDev g{};
    for (int l = 0; l < kGnnLayers; ++l) { g.foff[l] = gh.foff[l]; g.boff[l] = gh.boff[l]; }
    const float bh2 = gh.bh2;
    const size_t fbytes = frag.size() * 2, bbytes = bias.size() * 4;
    HIP_TRY(c, hipSetDevice(c->device));
    if (c->d_gnn) { (void)hipFree(c->d_gnn); c->d_gnn = nullptr; c->gnn_loaded = false; }
    if (hipMalloc(&c->d_gnn, fbytes + bbytes) != hipSuccess) return fail(c, LST_E_NOMEM, "edge classifier");
    HIP_TRY(c, hipMemcpy(c->d_gnn, frag.data(), fbytes, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy((char *)c->d_gnn + fbytes, bias.data(), bbytes, hipMemcpyHostToDevice));
    g.frag = (const uint4 *)c->d_gnn;
    g.bias = (const float *)((char *)c->d_gnn + fbytes);
    g.wh2 = g.bias + (bias.size() - 32);
    g.bh2 = bh2;
    c->gnn = g;
    c->gnn_loaded = true;
    return LST_OK;
}

static size_t gnn_layout(int64_t n_nodes, int64_t n_edges, char *base, GnnWork *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    char *h0 = take((size_t)n_nodes * 64 * 4), *h1 = take((size_t)n_nodes * 64 * 4);
    char *e1 = take((size_t)n_edges * 64 * 4), *io = take((size_t)(n_nodes + 1) * 8), *er = take(8);
    char *mg = take((size_t)n_nodes * 64 * 4);
    if (w) {
        w->h0 = (float *)h0; w->h1 = (float *)h1; w->e1 = (float *)e1; w->msg = (float *)mg;
        w->in_off = (int64_t *)io; w->err = (int64_t *)er;
    }
    return off;
}

lst_status lst_gnn_workspace_size(const lst_ctx *c, int64_t n_nodes, int64_t n_edges, size_t *bytes) {
    if (!c || !bytes || n_nodes < 0 || n_edges < 0 || n_nodes > INT32_MAX) return LST_E_INVAL;
    *bytes = gnn_layout(n_nodes, n_edges, nullptr, nullptr);
    return LST_OK;
}

lst_status lst_gnn_score(lst_ctx *c, const float *x, int64_t n_nodes, const int32_t *src, const int32_t *dst,
                         int64_t n_edges, float *scores, void *ws, size_t ws_bytes, int32_t flags, void *stream) {
    if (!c) return LST_E_INVAL;
    if (!c->gnn_loaded) return fail(c, LST_E_STATE, "load an edge classifier first");
    if (n_nodes < 0 || n_edges < 0 || n_nodes > INT32_MAX) return fail(c, LST_E_INVAL, "bad graph size");
    if (n_edges > 0 && n_nodes == 0) return fail(c, LST_E_INVAL, "edges without nodes");
    if ((n_nodes > 0 && !x) || (n_edges > 0 && (!src || !dst || !scores)) || !ws)
        return fail(c, LST_E_INVAL, "null argument");
    if (((uintptr_t)ws & 255) != 0) return fail(c, LST_E_INVAL, "workspace must be 256-byte aligned");
    const size_t need = gnn_layout(n_nodes, n_edges, nullptr, nullptr);
    if (ws_bytes < need) return fail(c, LST_E_INVAL, "workspace %zu bytes, need %zu", ws_bytes, need);
    if (n_nodes == 0) return LST_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    GnnWork w{};
    gnn_layout(n_nodes, n_edges, (char *)ws, &w);
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, run_gnn(c->gnn, x, n_nodes, src, dst, n_edges, scores, w, st));
    if (flags & LST_ASYNC) return LST_OK;
    int64_t err = 0;
    HIP_TRY(c, hipMemcpyAsync(&err, w.err, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (err & 1) return fail(c, LST_E_INVAL, "graph: node id out of range or edges not sorted by dst");
    return LST_OK;
}

lst_status lst_get_tuning(const lst_ctx *c, lst_tuning *t) {
    if (!c || !t) return LST_E_INVAL;
    t->bin_split = c->tune.bin_split;
    for (int i = 0; i < kStages; ++i) t->tile_per[i] = c->tune.per[i];
    t->eval_blocks = c->tune.eval_blocks;
    t->t3_masks = c->tune.t3_masks;
    return LST_OK;
}

lst_status lst_set_tuning(lst_ctx *c, const lst_tuning *t) {
    if (!c) return LST_E_INVAL;
    Tuning n = kDefaultTuning;
    if (t) {
        n.bin_split = t->bin_split;
        for (int i = 0; i < kStages; ++i) n.per[i] = t->tile_per[i];
        n.eval_blocks = t->eval_blocks;
        n.t3_masks = t->t3_masks;
    }
    if (!tuning_valid(n))
        return fail(c, LST_E_INVAL,
                    "unsupported tuning (bin_split %d, tiles %d %d %d %d %d, eval_blocks %d, t3_masks %d)",
                    n.bin_split, n.per[0], n.per[1], n.per[2], n.per[3], n.per[4], n.eval_blocks, n.t3_masks);
    c->tune = n;
    return LST_OK;
}

lst_status lst_score(lst_ctx *c, const void *X, int32_t x_dtype, int64_t n, float *scores, int32_t precision,
                     void *stream) {
    if (!c) return LST_E_INVAL;
    if (!c->model_loaded) return fail(c, LST_E_STATE, "load a model first");
    if (n < 0 || (n > 0 && (!X || !scores))) return fail(c, LST_E_INVAL, "bad score arguments");
    if (x_dtype != LST_DTYPE_F32 && x_dtype != LST_DTYPE_BF16) return fail(c, LST_E_INVAL, "bad x_dtype");
    if (precision != LST_PREC_F32 && precision != LST_PREC_BF16) return fail(c, LST_E_INVAL, "bad precision");
    if (n == 0) return LST_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, run_score(c->md, X, x_dtype, n, scores, precision, (hipStream_t)stream));
    return LST_OK;
}

static bool tc_sizes(lst_ctx *c, const lst_objects *o, int64_t n_seeds, int32_t n_ev, TcSizes *z) {
    if (!o || n_seeds < 0 || n_ev < 1) return false;
    if (o->n_md < 0 || o->n_ls < 0 || o->n_t3 < 0 || o->n_t5 < 0) return false;
    if (o->n_md > INT32_MAX || o->n_t3 > INT32_MAX || o->n_t5 > INT32_MAX || n_seeds > INT32_MAX) return false;
    if ((int64_t)n_ev * kTcPhiBins * 2 > INT32_MAX) return false;
    z->n_md = o->n_md; z->n3 = o->n_t3; z->n5 = o->n_t5; z->ns = n_seeds; z->n_ev = n_ev;
    (void)c;
    return true;
}

lst_status lst_tc_workspace_size(const lst_ctx *c, const lst_objects *o, int64_t n_seeds, int32_t n_events,
                                 size_t *bytes) {
    if (!c || !bytes) return LST_E_INVAL;
    TcSizes z{};
    if (!tc_sizes(nullptr, o, n_seeds, n_events, &z)) return LST_E_INVAL;
    *bytes = tc_layout(z, nullptr, nullptr);
    return LST_OK;
}

lst_status lst_select_tcs(lst_ctx *c, const lst_hits *h, const lst_objects *o, const int64_t *ev_obj, int32_t n_ev,
                          const lst_seeds *s, const lst_tc_options *opt, lst_tcs *out, void *ws, size_t ws_bytes,
                          void *stream) {
    if (!c) return LST_E_INVAL;
    if (!h || !o || !s || !opt || !out) return fail(c, LST_E_INVAL, "null argument");
    TcSizes z{};
    if (!tc_sizes(c, o, s->n, n_ev, &z)) return fail(c, LST_E_INVAL, "bad object / seed / event counts");
    if (n_ev > 1 && !ev_obj) return fail(c, LST_E_INVAL, "several events need the event object offsets");
    if (!s->event_off) return fail(c, LST_E_INVAL, "null seed event offsets");
    if (s->n > 0 && !s->params) return fail(c, LST_E_INVAL, "null seed parameters");
    const bool has_obj = o->n_t3 > 0 || o->n_t5 > 0;
    if (has_obj && (!h->x || !h->y || !h->z || !o->md_hits || !o->ls_md || !o->t3_ls))
        return fail(c, LST_E_INVAL, "null hit or object array");
    if (o->n_t5 > 0 && (!o->t5_t3 || !o->t5_score || !o->t5_chi2_rphi)) return fail(c, LST_E_INVAL, "null T5 array");
    const float f[6] = {opt->chi2_max, opt->sigma_kappa_abs, opt->sigma_kappa_rel, opt->sigma_phi0, opt->sigma_cot,
                        opt->sigma_z0};
    if (!(f[0] > 0.0f) || !isfinite(f[0])) return fail(c, LST_E_INVAL, "chi2_max must be positive");
    for (int i = 1; i < 6; ++i)
        if (!(f[i] >= 0.0f) || !isfinite(f[i])) return fail(c, LST_E_INVAL, "object widths must be finite, >= 0");
    if (out->cap < 0 || (out->cap > 0 && (!out->kind || !out->seed || !out->obj)) || !out->counts_dev)
        return fail(c, LST_E_INVAL, "bad TC output arrays");
    if (((uintptr_t)ws & 255) != 0) return fail(c, LST_E_INVAL, "workspace must be 256-byte aligned");
    const size_t need = tc_layout(z, nullptr, nullptr);
    if (ws_bytes < need) return fail(c, LST_E_INVAL, "workspace %zu bytes, need %zu", ws_bytes, need);
    HIP_TRY(c, hipSetDevice(c->device));
    TcWork w{};
    tc_layout(z, (char *)ws, &w);
    w.out_kind = out->kind; w.out_seed = out->seed; w.out_obj = out->obj;
    w.out_counts = out->counts_dev; w.cap_tc = out->cap;
    TcArgs a{};
    a.x = h->x; a.y = h->y; a.z = h->z;
    a.md_hits = (const int2 *)o->md_hits; a.ls_md = (const int2 *)o->ls_md; a.t3_ls = (const int2 *)o->t3_ls;
    a.t5_t3 = (const int2 *)o->t5_t3; a.t5_score = o->t5_score; a.t5_chi2_rphi = o->t5_chi2_rphi;
    a.n_md = o->n_md; a.n_ls = o->n_ls; a.n3 = o->n_t3; a.n5 = o->n_t5;
    a.ev_obj = ev_obj;                    // null for one event: offsets {0, n} are made on the device
    a.n_ev = n_ev;
    a.seeds = s->params; a.seed_off = s->event_off; a.ns = s->n;
    a.opt = *opt;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, run_tc(a, w, st));
    int64_t cnt[kTcCounts];
    HIP_TRY(c, hipMemcpyAsync(cnt, out->counts_dev, sizeof(int64_t) * 6, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    out->n = cnt[kTcCountKept];
    if (out->n > out->cap)
        return fail(c, LST_E_CAPACITY, "%lld track candidates kept, capacity %lld", (long long)out->n,
                    (long long)out->cap);
    return LST_OK;
}

lst_status lst_md_graph(lst_ctx *c, const lst_hits *h, const lst_objects *o, float *features, int32_t *src,
                        int32_t *dst, void *stream) {
    if (!c) return LST_E_INVAL;
    if (!c->geom_loaded) return fail(c, LST_E_STATE, "load a geometry first");
    if (!h || !o) return fail(c, LST_E_INVAL, "null argument");
    if (o->n_md < 0 || o->n_ls < 0 || o->n_md > INT32_MAX || o->n_ls > INT32_MAX)
        return fail(c, LST_E_INVAL, "bad object counts");
    if (o->n_md > 0 && (!h->x || !h->y || !h->z || !h->sensor || !o->md_hits || !features))
        return fail(c, LST_E_INVAL, "null hit, MD or feature array");
    if (o->n_ls > 0 && (!o->ls_md || !src || !dst)) return fail(c, LST_E_INVAL, "null LS or edge array");
    if (o->n_md == 0 && o->n_ls == 0) return LST_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    GraphArgs a{};
    a.x = h->x; a.y = h->y; a.z = h->z; a.sensor = h->sensor;
    a.md_hits = (const int2 *)o->md_hits; a.ls_md = (const int2 *)o->ls_md; a.mod = c->d_mod;
    a.n_md = o->n_md; a.n_ls = o->n_ls;
    a.feat = features; a.src = src; a.dst = dst;
    HIP_TRY(c, run_md_graph(a, (hipStream_t)stream));
    return LST_OK;
}

lst_status lst_graph_components_workspace_size(const lst_ctx *c, int64_t n_nodes, size_t *bytes) {
    if (!c || !bytes || n_nodes < 0 || n_nodes > INT32_MAX) return LST_E_INVAL;
    *bytes = components_workspace(n_nodes);
    return LST_OK;
}

lst_status lst_graph_components(lst_ctx *c, int64_t n_nodes, const int32_t *src, const int32_t *dst,
                                const float *scores, int64_t n_edges, float threshold, int32_t min_mds,
                                int32_t *labels, int64_t *n_tc, void *ws, size_t ws_bytes, void *stream) {
    if (!c) return LST_E_INVAL;
    if (n_nodes < 0 || n_nodes > INT32_MAX || n_edges < 0) return fail(c, LST_E_INVAL, "bad graph size");
    if (!n_tc || (n_nodes > 0 && !labels) || (n_edges > 0 && (!src || !dst || !scores)))
        return fail(c, LST_E_INVAL, "null graph array");
    if (!isfinite(threshold)) return fail(c, LST_E_INVAL, "threshold must be finite");
    if (min_mds < 1) return fail(c, LST_E_INVAL, "min_mds must be at least 1");
    if (((uintptr_t)ws & 255) != 0) return fail(c, LST_E_INVAL, "workspace must be 256-byte aligned");
    const size_t need = components_workspace(n_nodes);
    if (ws_bytes < need) return fail(c, LST_E_INVAL, "workspace %zu bytes, need %zu", ws_bytes, need);
    HIP_TRY(c, hipSetDevice(c->device));
    ComponentsArgs a = components_layout((char *)ws, n_nodes);
    a.src = src; a.dst = dst; a.scores = scores; a.n_nodes = n_nodes; a.n_edges = n_edges;
    a.threshold = threshold; a.min_mds = min_mds; a.labels = labels; a.n_tc = n_tc;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, run_components(a, st));
    int64_t err = 0;
    HIP_TRY(c, hipMemcpyAsync(&err, a.err, sizeof(err), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (err) return fail(c, LST_E_INVAL, "an edge's node id is out of range (those edges were skipped)");
    return LST_OK;
}

}  // extern "C"
