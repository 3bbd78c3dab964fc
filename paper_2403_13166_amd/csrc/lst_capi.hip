// C ABI of the LST object builder: context, geometry / model loading,
// workspace layout and the build / score entry points declared in lst.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lst.h"
#include "lst_internal.h"

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
    RowConst *d_rows = nullptr;
    int32_t n_runs = 0, n_rows = 0;
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
    if (c->d_rows) (void)hipFree(c->d_rows);
    c->d_mod = nullptr; c->d_map_off = c->d_map_tgt = nullptr;
    c->d_box = nullptr; c->d_run_off = nullptr; c->d_runs = nullptr; c->d_rows = nullptr;
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

static uint32_t rd32(const unsigned char *b) {
    uint32_t v;
    memcpy(&v, b, 4);
    return v;
}

// transverse arc length from the beam line to radius r at half-curvature c
static double arc_len(double c, double r) {
    double x = c * r;
    if (x < 1e-4) return r * (1.0 + x * x / 6.0);
    if (x >= 1.0) x = 1.0;
    return asin(x) / c;
}

// Tolerances of the on-sensor check of MD anchor hits, which every window of
// the line-segment stage builds on (FP32 rounding of hit coordinates is a few
// 1e-6 cm and 1e-7 rad).
constexpr double kTolPos = 2e-3;   // cm
constexpr double kTolPhi = 2e-5;   // rad
constexpr double kTwoPi = 6.283185307179586;
constexpr double kPi = 3.141592653589793;
// Largest phi separation at which the line-segment stage trims a run: a pair
// whose curvature passes the curvature cut lies either within the window
// asin(c r_B) - asin(c r_A) of the near side of its circle, or beyond
// pi - 2 asin(0.85) = 1.1096 rad on the far side (the device trims only while
// c r_B < 0.85); runs that reach 1.10 rad from their source module are
// therefore never trimmed in phi.
constexpr double kFarSidePhi = 1.10;

struct HostMod {
    int32_t kind, layer, side, nphi;
    double p[6];
};

// circular |u| in [0, pi]
static double circ_abs(double u) {
    double d = fmod(fabs(u), kTwoPi);
    return d > kPi ? kTwoPi - d : d;
}

// Largest angular distance between a point of [a0, a1] and a point of
// [b0, b1]: the differences x - y fill [a0 - b1, a1 - b0]; if that interval
// holds pi (mod 2 pi) the answer is pi, otherwise the distance peaks at an end.
static double max_phi_sep(double a0, double a1, double b0, double b1) {
    const double lo = a0 - b1, hi = a1 - b0;
    if (hi - lo >= kTwoPi) return kPi;
    const double k = ceil((lo - kPi) / kTwoPi);
    if (kPi + k * kTwoPi <= hi) return kPi;
    return std::max(circ_abs(lo), circ_abs(hi));
}

static ModBox module_box(const HostMod &m) {
    ModBox b{};
    if (m.kind == 0) {
        b.r_lo = (float)(m.p[0] - kTolPos); b.r_hi = (float)(m.p[0] + kTolPos);
        b.z_lo = (float)(m.p[2] - kTolPos); b.z_hi = (float)(m.p[3] + kTolPos);
    } else {
        b.r_lo = (float)(m.p[2] - kTolPos); b.r_hi = (float)(m.p[3] + kTolPos);
        b.z_lo = (float)(m.p[0] - kTolPos); b.z_hi = (float)(m.p[0] + kTolPos);
    }
    b.phi_lo = (float)(m.p[4] - kTolPhi); b.phi_hi = (float)(m.p[5] + kTolPhi);
    return b;
}

// Runs of every module's map row (sorted, duplicates removed): maximal
// sequences of consecutive target ids that lie in one detector row and are
// adjacent in phi. Rows are keyed by module type, layer, side, phi count,
// anchor surface and extent.
static void build_runs(const std::vector<HostMod> &mods, const std::vector<int32_t> &moff,
                       const std::vector<int32_t> &mtgt, double cmax, double srphi, double sr,
                       std::vector<int32_t> &run_off, std::vector<RunRec> &runs, std::vector<RowConst> &rows) {
    const size_t nm = mods.size();
    std::map<std::array<double, 7>, int32_t> row_of_key;
    std::vector<int32_t> row_id(nm);
    for (size_t m = 0; m < nm; ++m) {
        const HostMod &h = mods[m];
        const std::array<double, 7> key{(double)h.kind, (double)h.layer, (double)h.side, (double)h.nphi,
                                        h.p[0], h.p[2], h.p[3]};
        auto it = row_of_key.find(key);
        if (it == row_of_key.end()) {
            const ModBox b = module_box(h);
            RowConst rc{};
            rc.r_lo = b.r_lo; rc.r_hi = b.r_hi; rc.z_lo = b.z_lo; rc.z_hi = b.z_hi;
            const double w = h.p[5] - h.p[4];
            rc.dphi = (float)w;
            rc.inv_dphi = (float)(1.0 / w);
            const double rl = h.kind == 0 ? h.p[0] - kTolPos : h.p[2] - kTolPos;
            double q = srphi * srphi / (rl * rl);
            if (h.kind != 0) q += cmax * cmax * sr * sr;
            rc.qb_max = (float)(q * (1.0 + 1e-6));
            rc.kind = h.kind;
            it = row_of_key.emplace(key, (int32_t)rows.size()).first;
            rows.push_back(rc);
        }
        row_id[m] = it->second;
    }
    run_off.assign(nm + 1, 0);
    std::vector<int32_t> row;
    for (size_t m = 0; m < nm; ++m) {
        row.assign(mtgt.begin() + moff[m], mtgt.begin() + moff[m + 1]);
        std::sort(row.begin(), row.end());
        row.erase(std::unique(row.begin(), row.end()), row.end());
        const HostMod &src = mods[m];
        size_t i = 0;
        while (i < row.size()) {
            size_t k = i + 1;
            while (k < row.size()) {
                const HostMod &a = mods[row[k - 1]], &b = mods[row[k]];
                const bool adj = row[k] == row[k - 1] + 1 && row_id[row[k]] == row_id[row[k - 1]] &&
                                 fabs(b.p[4] - a.p[5]) < 1e-9 && fabs((b.p[5] - b.p[4]) - (a.p[5] - a.p[4])) < 1e-9;
                if (!adj) break;
                ++k;
            }
            RunRec rr{};
            rr.t_first = row[i];
            rr.n = (int32_t)(k - i);
            rr.row = row_id[row[i]];
            rr.phi_start = (float)mods[row[i]].p[4];
            const double sep = max_phi_sep(src.p[4] - kTolPhi, src.p[5] + kTolPhi,
                                           mods[row[i]].p[4] - kTolPhi, mods[row[k - 1]].p[5] + kTolPhi);
            if (sep >= kFarSidePhi) rr.row |= kRunNoTrim;
            runs.push_back(rr);
            i = k;
        }
        run_off[m + 1] = (int32_t)runs.size();
    }
}

lst_status lst_load_geometry(lst_ctx *c, const void *blob, size_t nbytes) {
    if (!c || !blob) return LST_E_INVAL;
    const unsigned char *b = (const unsigned char *)blob;
    if (nbytes < 152 || memcmp(b, "LSTG", 4) != 0 || rd32(b + 4) != 1)
        return fail(c, LST_E_INVAL, "geometry blob: bad magic or version");
    uint32_t nm = rd32(b + 8), nb = rd32(b + 12), nmap = rd32(b + 16), npar = rd32(b + 20);
    if (npar != 16) return fail(c, LST_E_INVAL, "geometry blob: expected 16 parameters");
    size_t need = 152 + (size_t)nm * 64 + ((size_t)nm + 1) * 4 + (size_t)nmap * 4;
    if (nbytes != need || nm == 0 || nm > (1u << 24))
        return fail(c, LST_E_INVAL, "geometry blob: size %zu, expected %zu", nbytes, need);
    // hit binning sorts at most kBinRangesMax ranges of 1024 sensors per event
    if (2 * (uint64_t)nm > 1024ull * kBinRangesMax)
        return fail(c, LST_E_INVAL, "geometry blob: %u modules, at most %d supported", nm, 512 * kBinRangesMax);
    double prm[16];
    memcpy(prm, b + 24, sizeof(prm));
    // parameters: k_b, pt_min, z_lum, n_sigma, sigma_rphi, sigma_z, sigma_r, gap,
    //             chi2_rz_max, chi2_rphi_max, md_e2_slack, ls3_slack
    const double kb = prm[0], cmax = kb / (2.0 * prm[1]), ns = prm[3], srphi = prm[4];
    CutParams p{};
    p.kb = (float)kb; p.cmax = (float)cmax; p.zlum = (float)prm[2]; p.nsig = (float)ns;
    p.srphi = (float)srphi; p.sz = (float)prm[5]; p.sr = (float)prm[6]; p.e2slack = (float)prm[10];
    p.ls3slack = (float)prm[11]; p.chi2rz = (float)prm[8]; p.chi2rphi = (float)prm[9];
    p.kb_d = kb; p.cmax_d = cmax; p.zlum_d = prm[2]; p.nsig_d = ns; p.srphi_d = srphi;
    p.sz_d = prm[5]; p.sr_d = prm[6];
    if (!(srphi > 0) || !(prm[5] > 0) || !(prm[6] > 0))
        return fail(c, LST_E_INVAL, "geometry blob: resolutions must be positive");
    p.isrphi_d = 1.0 / srphi; p.isr_d = 1.0 / prm[6]; p.isz_d = 1.0 / prm[5];
    std::vector<ModConst> mods(nm);
    std::vector<HostMod> hmods(nm);
    std::vector<ModBox> boxes(nm);
    const unsigned char *r = b + 152;
    for (uint32_t m = 0; m < nm; ++m, r += 64) {
        int32_t kind, layer;
        double pp[6];
        memcpy(&kind, r, 4);
        memcpy(&layer, r + 4, 4);
        memcpy(pp, r + 16, 48);
        HostMod &hm = hmods[m];
        hm.kind = kind; hm.layer = layer;
        memcpy(&hm.side, r + 8, 4);
        memcpy(&hm.nphi, r + 12, 4);
        memcpy(hm.p, pp, sizeof(pp));
        if (!(pp[4] >= 0.0 && pp[5] > pp[4] && pp[5] <= kTwoPi + 1e-9))
            return fail(c, LST_E_INVAL, "geometry blob: module %u phi range outside [0, 2 pi]", m);
        boxes[m] = module_box(hm);
        ModConst mc{};
        mc.kind = kind; mc.layer = layer;
        mc.gap = (float)fabs(pp[1] - pp[0]);
        if (kind == 0) {
            // barrel MD thresholds: largest bend of a beam-line track with
            // |c| <= c_max between the two sensors, plus resolution; r-z ratios
            const double rlo = pp[0], rup = pp[1];
            mc.b1_t = (float)(asin(cmax * rup) - asin(cmax * rlo)
                              + ns * srphi * sqrt(1.0 / (rlo * rlo) + 1.0 / (rup * rup)));
            mc.rho0 = (float)((rup - rlo) / rlo);
            const double slo = arc_len(cmax, rlo);
            mc.rho1 = (float)((arc_len(cmax, rup) - slo) / slo);
        } else if (kind != 1) {
            return fail(c, LST_E_INVAL, "geometry blob: module %u has kind %d", m, kind);
        }
        mods[m] = mc;
    }
    std::vector<int32_t> moff(nm + 1), mtgt(nmap ? nmap : 1);
    for (uint32_t i = 0; i <= nm; ++i) moff[i] = (int32_t)rd32(r + 4 * i);
    const unsigned char *t = r + 4 * ((size_t)nm + 1);
    for (uint32_t i = 0; i < nmap; ++i) {
        mtgt[i] = (int32_t)rd32(t + 4 * i);
        if (mtgt[i] < 0 || (uint32_t)mtgt[i] >= nm) return fail(c, LST_E_INVAL, "module map target out of range");
    }
    if ((uint32_t)moff[nm] != nmap) return fail(c, LST_E_INVAL, "module map offsets inconsistent");
    for (uint32_t i = 0; i < nm; ++i)
        if (moff[i + 1] < moff[i]) return fail(c, LST_E_INVAL, "module map offsets not monotone");
    std::vector<int32_t> run_off;
    std::vector<RunRec> runs;
    std::vector<RowConst> rows;
    build_runs(hmods, moff, mtgt, cmax, srphi, prm[6], run_off, runs, rows);
    if (runs.empty()) runs.push_back(RunRec{});
    HIP_TRY(c, hipSetDevice(c->device));
    free_geom(c);
    if (hipMalloc(&c->d_mod, sizeof(ModConst) * nm) != hipSuccess ||
        hipMalloc(&c->d_map_off, sizeof(int32_t) * (nm + 1)) != hipSuccess ||
        hipMalloc(&c->d_map_tgt, sizeof(int32_t) * mtgt.size()) != hipSuccess ||
        hipMalloc(&c->d_box, sizeof(ModBox) * nm) != hipSuccess ||
        hipMalloc(&c->d_run_off, sizeof(int32_t) * (nm + 1)) != hipSuccess ||
        hipMalloc(&c->d_runs, sizeof(RunRec) * runs.size()) != hipSuccess ||
        hipMalloc(&c->d_rows, sizeof(RowConst) * rows.size()) != hipSuccess) {
        free_geom(c);
        return fail(c, LST_E_NOMEM, "geometry tables");
    }
    HIP_TRY(c, hipMemcpy(c->d_mod, mods.data(), sizeof(ModConst) * nm, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_map_off, moff.data(), sizeof(int32_t) * (nm + 1), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_map_tgt, mtgt.data(), sizeof(int32_t) * mtgt.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_box, boxes.data(), sizeof(ModBox) * nm, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_run_off, run_off.data(), sizeof(int32_t) * (nm + 1), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_runs, runs.data(), sizeof(RunRec) * runs.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_rows, rows.data(), sizeof(RowConst) * rows.size(), hipMemcpyHostToDevice));
    c->n_runs = (int32_t)run_off[nm];
    c->n_rows = (int32_t)rows.size();
    c->n_mod = (int32_t)nm; c->n_barrel = (int32_t)nb; c->n_map = (int32_t)nmap;
    c->cp = p;
    c->geom_loaded = true;
    return LST_OK;
}

lst_status lst_load_model(lst_ctx *c, const void *blob, size_t nbytes) {
    if (!c || !blob) return LST_E_INVAL;
    const unsigned char *b = (const unsigned char *)blob;
    if (nbytes < 24 || memcmp(b, "LSTM", 4) != 0 || rd32(b + 4) != 1)
        return fail(c, LST_E_INVAL, "model blob: bad magic or version");
    if (rd32(b + 8) != kNFeat || rd32(b + 12) != kH1 || rd32(b + 16) != kH2)
        return fail(c, LST_E_INVAL, "model blob: expected a %d-%d-%d-1 network", kNFeat, kH1, kH2);
    const size_t nf = 2 * kNFeat + kH1 * kNFeat + kH1 + kH2 * kH1 + kH2 + kH2 + 1;
    if (nbytes != 24 + 4 * nf) return fail(c, LST_E_INVAL, "model blob: size %zu", nbytes);
    std::vector<float> w(nf);
    memcpy(w.data(), b + 24, 4 * nf);
    for (int k = 0; k < kNFeat; ++k)
        if (!(w[kNFeat + k] > 0.0f)) return fail(c, LST_E_INVAL, "model blob: non-positive scale");
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
    // ranges per event: enough for 1024 sensor ids each, or the largest bin_split
    const int64_t nr_max = (nsens + 1023) / 1024 > 64 ? (nsens + 1023) / 1024 : 64;
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
    x.ls_chunk = (int2 *)take(8 * (k->ls > 0 ? k->ls : 1));
    x.ls_wave = (int64_t *)take(8 * (md / 64 + 2));
    x.ls_top = (unsigned long long *)take(8);
    x.t3_mds = (int4 *)take(16 * (k->t3 > 0 ? k->t3 : 1));
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
    a.g.box = c->d_box; a.g.run_off = c->d_run_off; a.g.runs = c->d_runs; a.g.rows = c->d_rows;
    a.g.n_mod = c->n_mod; a.g.n_sens = 2 * c->n_mod; a.g.n_map = c->n_map;
    a.p = c->cp; a.m = c->md;
    a.x = h->x; a.y = h->y; a.z = h->z; a.sensor = h->sensor; a.n_hits = h->n;
    a.ev_off = ev_off; a.n_ev = n_ev;
    a.mode = opt->mode; a.precision = opt->precision; a.score_min = opt->score_min;
    a.ev_obj_off = ev_obj_off;
    a.timing = c->timing ? c->tev : nullptr;
    a.tune = c->tune;
    Outputs o{};
    o.md_hits = (int2 *)out->md_hits; o.ls_md = (int2 *)out->ls_md; o.t3_ls = (int2 *)out->t3_ls;
    o.t5_t3 = (int2 *)out->t5_t3; o.t5_score = out->t5_score; o.t5_chi2_rphi = out->t5_chi2_rphi;
    o.t5_chi2_rz = out->t5_chi2_rz; o.t5_feat = out->t5_feat; o.counts = out->counts_dev;
    HIP_TRY(c, run_pipeline(a, w, o, st));
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

namespace {

struct GLayer { int out, in; };
// layer shapes in blob order (index = GnnLayer)
constexpr GLayer kGShape[kGnnLayers] = {{64, 7},   {64, 64},  {64, 128}, {64, 192}, {64, 64}, {64, 128}, {64, 64},
                                        {64, 192}, {64, 64},  {64, 128}, {64, 64},  {32, 64}, {1, 32}};

uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// K index carried by slot i of lane group g in K chunk ks: 64-wide inputs use
// the accumulator-compatible order of the kernels, the 7-wide input is padded
int gnn_kidx(int in, int ks, int g, int i) {
    if (in % 64 != 0) return 8 * g + i < in ? 8 * g + i : -1;
    const int seg = ks / 2, ksl = ks % 2;
    return seg * 64 + 32 * ksl + 16 * (i >> 2) + 4 * g + (i & 3);
}

}  // namespace

lst_status lst_load_gnn(lst_ctx *c, const void *blob, size_t nbytes) {
    if (!c || !blob) return LST_E_INVAL;
    const unsigned char *b = (const unsigned char *)blob;
    if (nbytes < 24 || memcmp(b, "LSTE", 4) != 0 || rd32(b + 4) != 1)
        return fail(c, LST_E_INVAL, "edge-classifier blob: bad magic or version");
    if (rd32(b + 8) != 7 || rd32(b + 12) != 64 || rd32(b + 16) != 32 || rd32(b + 20) != 2)
        return fail(c, LST_E_INVAL, "edge-classifier blob: expected 7 inputs, hidden 64, head 32, 2 steps");
    size_t nf = 0;
    for (int l = 0; l < kGnnLayers; ++l) nf += (size_t)kGShape[l].out * kGShape[l].in + kGShape[l].out;
    if (nbytes != 24 + 4 * nf) return fail(c, LST_E_INVAL, "edge-classifier blob: size %zu", nbytes);
    std::vector<float> w(nf);
    memcpy(w.data(), b + 24, 4 * nf);
    // fragments (A operand order) for the MFMA layers, biases for all
    std::vector<uint16_t> frag;
    std::vector<float> bias;
    GnnDev g{};
    size_t at = 0;
    const float *wh2 = nullptr;
    float bh2 = 0.0f;
    for (int l = 0; l < kGnnLayers; ++l) {
        const int O = kGShape[l].out, I = kGShape[l].in;
        const float *W = w.data() + at;
        const float *B = W + (size_t)O * I;
        at += (size_t)O * I + O;
        g.boff[l] = (int64_t)bias.size();
        bias.insert(bias.end(), B, B + O);
        g.foff[l] = (int64_t)(frag.size() / 8);
        if (l == kGHead2) { wh2 = W; bh2 = B[0]; continue; }
        // K chunks of 32: the 7-wide input is one padded chunk
        const int MB = O / 16, ks_n = I % 64 == 0 ? I / 32 : 1;
        for (int mb = 0; mb < MB; ++mb)
            for (int ks = 0; ks < ks_n; ++ks)
                for (int lane = 0; lane < 64; ++lane) {
                    const int gg = lane >> 4, cc = lane & 15;
                    for (int i = 0; i < 8; ++i) {
                        const int k = gnn_kidx(I, ks, gg, i);
                        frag.push_back(f32_to_bf16_rne(k >= 0 ? W[(size_t)(mb * 16 + cc) * I + k] : 0.0f));
                    }
                }
    }
    bias.insert(bias.end(), wh2, wh2 + 32);      // head output weights after the biases
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
    return LST_OK;
}

lst_status lst_set_tuning(lst_ctx *c, const lst_tuning *t) {
    if (!c) return LST_E_INVAL;
    Tuning n = kDefaultTuning;
    if (t) {
        n.bin_split = t->bin_split;
        for (int i = 0; i < kStages; ++i) n.per[i] = t->tile_per[i];
        n.eval_blocks = t->eval_blocks;
    }
    if (!tuning_valid(n))
        return fail(c, LST_E_INVAL, "unsupported tuning (bin_split %d, tiles %d %d %d %d %d, eval_blocks %d)",
                    n.bin_split, n.per[0], n.per[1], n.per[2], n.per[3], n.per[4], n.eval_blocks);
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

}  // extern "C"
