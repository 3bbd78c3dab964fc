// Host-side parsing of the library's input blobs into the plain tables the
// device code reads (see lst_host.h).
#include "lst_host.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <string>
#include <vector>

namespace lst {
namespace {

bool bad(std::string &err, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return false;
}

uint32_t rd32(const unsigned char *b) {
    uint32_t v;
    memcpy(&v, b, 4);
    return v;
}

// transverse arc length from the beam line to radius r at half-curvature c
double arc_len(double c, double r) {
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
// pi - 2 asin(0.8) = 1.287 rad on the far side (the device trims only while
// c r_B < 0.8); runs that reach 1.25 rad from their source module are
// therefore never trimmed in phi.
constexpr double kFarSidePhi = 1.25;

// Constants of one detector row, copied into every run of the row.
struct RowConst {
    float r_lo, r_hi, z_lo, z_hi, inv_dphi, qb_max;
    int32_t kind;
};

struct HostMod {
    int32_t kind, layer, side, nphi;
    double p[6];
};

// circular |u| in [0, pi]
double circ_abs(double u) {
    double d = fmod(fabs(u), kTwoPi);
    return d > kPi ? kTwoPi - d : d;
}

// Largest angular distance between a point of [a0, a1] and a point of
// [b0, b1]: the differences x - y fill [a0 - b1, a1 - b0]; if that interval
// holds pi (mod 2 pi) the answer is pi, otherwise the distance peaks at an end.
double max_phi_sep(double a0, double a1, double b0, double b1) {
    const double lo = a0 - b1, hi = a1 - b0;
    if (hi - lo >= kTwoPi) return kPi;
    const double k = ceil((lo - kPi) / kTwoPi);
    if (kPi + k * kTwoPi <= hi) return kPi;
    return std::max(circ_abs(lo), circ_abs(hi));
}

ModBox module_box(const HostMod &m) {
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
void build_runs(const std::vector<HostMod> &mods, const std::vector<int32_t> &moff,
                const std::vector<int32_t> &mtgt, double cmax, double srphi, double sr,
                std::vector<int32_t> &run_off, std::vector<RunRec> &runs) {
    std::vector<RowConst> rows;
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
            rc.inv_dphi = (float)(1.0 / (h.p[5] - h.p[4]));
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
            const RowConst &rc = rows[row_id[row[i]]];
            RunRec rr{};
            rr.t_first = row[i];
            rr.n = (int32_t)(k - i);
            rr.flags = rc.kind != 0 ? kRunEndcap : 0;
            rr.phi_start = (float)mods[row[i]].p[4];
            rr.inv_dphi = rc.inv_dphi;
            rr.r_lo = rc.r_lo; rr.r_hi = rc.r_hi; rr.z_lo = rc.z_lo; rr.z_hi = rc.z_hi;
            rr.qb_max = rc.qb_max;
            const double sep = max_phi_sep(src.p[4] - kTolPhi, src.p[5] + kTolPhi,
                                           mods[row[i]].p[4] - kTolPhi, mods[row[k - 1]].p[5] + kTolPhi);
            if (sep >= kFarSidePhi) rr.flags |= kRunNoTrim;
            runs.push_back(rr);
            i = k;
        }
        run_off[m + 1] = (int32_t)runs.size();
    }
}

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

bool parse_geometry(const void *blob, size_t nbytes, GeomHost &g, std::string &err) {
    if (!blob) return bad(err, "null blob");
    const unsigned char *b = (const unsigned char *)blob;
    if (nbytes < 152 || memcmp(b, "LSTG", 4) != 0 || rd32(b + 4) != 1)
        return bad(err, "geometry blob: bad magic or version");
    uint32_t nm = rd32(b + 8), nb = rd32(b + 12), nmap = rd32(b + 16), npar = rd32(b + 20);
    if (npar != 16) return bad(err, "geometry blob: expected 16 parameters");
    if (nb > nm) return bad(err, "geometry blob: more barrel modules than modules");
    size_t need = 152 + (size_t)nm * 64 + ((size_t)nm + 1) * 4 + (size_t)nmap * 4;
    if (nbytes != need || nm == 0 || nm > (1u << 24))
        return bad(err, "geometry blob: size %zu, expected %zu", nbytes, need);
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
        return bad(err, "geometry blob: resolutions must be positive");
    if (!(kb > 0) || !(prm[1] > 0) || !(prm[2] >= 0) || !(ns >= 0) || !isfinite(cmax) || !isfinite(prm[2]) ||
        !isfinite(ns))
        return bad(err, "geometry blob: field, pT threshold, luminous region and n_sigma must be finite and positive");
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
            return bad(err, "geometry blob: module %u phi range outside [0, 2 pi]", m);
        // anchor surface, other surface and extent: barrel (r, r', z0 < z1), endcap (z, z', r0 < r1)
        const bool box_ok = kind == 0 ? (pp[0] > 10 * kTolPos && pp[1] > pp[0] && pp[3] > pp[2] && isfinite(pp[2]) &&
                                         isfinite(pp[3]) && isfinite(pp[1]))
                                      : (pp[2] > 10 * kTolPos && pp[3] > pp[2] && isfinite(pp[3]) && isfinite(pp[0]) &&
                                         isfinite(pp[1]) && pp[0] != pp[1]);
        if (!box_ok) return bad(err, "geometry blob: module %u has an empty or non-finite extent", m);
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
            return bad(err, "geometry blob: module %u has kind %d", m, kind);
        }
        mods[m] = mc;
    }
    std::vector<int32_t> moff(nm + 1), mtgt(nmap ? nmap : 1);
    for (uint32_t i = 0; i <= nm; ++i) moff[i] = (int32_t)rd32(r + 4 * i);
    const unsigned char *t = r + 4 * ((size_t)nm + 1);
    for (uint32_t i = 0; i < nmap; ++i) {
        mtgt[i] = (int32_t)rd32(t + 4 * i);
        if (mtgt[i] < 0 || (uint32_t)mtgt[i] >= nm) return bad(err, "module map target out of range");
    }
    if (moff[0] != 0 || (uint32_t)moff[nm] != nmap) return bad(err, "module map offsets inconsistent");
    for (uint32_t i = 0; i < nm; ++i)
        if (moff[i + 1] < moff[i]) return bad(err, "module map offsets not monotone");
    std::vector<int32_t> run_off;
    std::vector<RunRec> runs;
    build_runs(hmods, moff, mtgt, cmax, srphi, prm[6], run_off, runs);
    if (runs.empty()) runs.push_back(RunRec{});
    g.n_mod = (int32_t)nm;
    g.n_barrel = (int32_t)nb;
    g.n_map = (int32_t)nmap;
    g.cp = p;
    g.mods = std::move(mods);
    g.boxes = std::move(boxes);
    g.map_off = std::move(moff);
    g.map_tgt = std::move(mtgt);
    g.run_off = std::move(run_off);
    g.runs = std::move(runs);
    return true;
}

bool parse_model(const void *blob, size_t nbytes, ModelHost &mh, std::string &err) {
    if (!blob) return bad(err, "null blob");
    const unsigned char *b = (const unsigned char *)blob;
    if (nbytes < 24 || memcmp(b, "LSTM", 4) != 0 || rd32(b + 4) != 1)
        return bad(err, "model blob: bad magic or version");
    if (rd32(b + 8) != kNFeat || rd32(b + 12) != kH1 || rd32(b + 16) != kH2)
        return bad(err, "model blob: expected a %d-%d-%d-1 network", kNFeat, kH1, kH2);
    const size_t nf = 2 * kNFeat + kH1 * kNFeat + kH1 + kH2 * kH1 + kH2 + kH2 + 1;
    if (nbytes != 24 + 4 * nf) return bad(err, "model blob: size %zu", nbytes);
    std::vector<float> w(nf);
    memcpy(w.data(), b + 24, 4 * nf);
    for (int k = 0; k < kNFeat; ++k)
        if (!(w[kNFeat + k] > 0.0f)) return bad(err, "model blob: non-positive scale");
    mh.w = std::move(w);
    return true;
}

bool parse_gnn(const void *blob, size_t nbytes, GnnHost &gh, std::string &err) {
    if (!blob) return bad(err, "null blob");
    const unsigned char *b = (const unsigned char *)blob;
    if (nbytes < 24 || memcmp(b, "LSTE", 4) != 0 || rd32(b + 4) != 1)
        return bad(err, "edge-classifier blob: bad magic or version");
    if (rd32(b + 8) != 7 || rd32(b + 12) != 64 || rd32(b + 16) != 32 || rd32(b + 20) != 2)
        return bad(err, "edge-classifier blob: expected 7 inputs, hidden 64, head 32, 2 steps");
    size_t nf = 0;
    for (int l = 0; l < kGnnLayers; ++l) nf += (size_t)kGShape[l].out * kGShape[l].in + kGShape[l].out;
    if (nbytes != 24 + 4 * nf) return bad(err, "edge-classifier blob: size %zu", nbytes);
    std::vector<float> w(nf);
    memcpy(w.data(), b + 24, 4 * nf);
    // fragments (A operand order) for the MFMA layers, biases for all
    std::vector<uint16_t> frag;
    std::vector<float> bias;
    size_t at = 0;
    const float *wh2 = nullptr;
    float bh2 = 0.0f;
    for (int l = 0; l < kGnnLayers; ++l) {
        const int O = kGShape[l].out, I = kGShape[l].in;
        const float *W = w.data() + at;
        const float *B = W + (size_t)O * I;
        at += (size_t)O * I + O;
        gh.boff[l] = (int64_t)bias.size();
        bias.insert(bias.end(), B, B + O);
        gh.foff[l] = (int64_t)(frag.size() / 8);
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
    gh.frag = std::move(frag);
    gh.bias = std::move(bias);
    gh.bh2 = bh2;
    return true;
}

}  // namespace lst
