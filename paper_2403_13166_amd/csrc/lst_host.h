// Host-side parsing of the library's input blobs (geometry and module map,
// T5-DNN model, edge classifier) into the plain tables the device code reads.
// Plain C++ without HIP, so that the parsers build and run on any CPU (the
// tests run them under AddressSanitizer and UndefinedBehaviorSanitizer on
// malformed blobs).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace lst {

constexpr int kNFeat = 42;
constexpr int kH1 = 32;
constexpr int kH2 = 32;

// ------------------------------------------------------------------ layout

// Per-module constants, derived on the host from the FP64 geometry.
struct ModConst {
    int32_t kind;      // 0 barrel, 1 endcap
    int32_t layer;     // 1..6 barrel, 7..11 disks
    float b1_t;        // barrel: MD bend threshold (envelope + resolution)
    float rho0;        // barrel: (r_up - r_lo) / r_lo
    float rho1;        // barrel: (S(r_up) - S(r_lo)) / S(r_lo) at c_max
    float gap;         // sensor separation
    float pad0, pad1;
};

struct CutParams {
    float kb, cmax, zlum, nsig, srphi, sz, sr, e2slack, ls3slack, chi2rz, chi2rphi;
    double kb_d, cmax_d, zlum_d, nsig_d, srphi_d, sz_d, sr_d;
    double isrphi_d, isr_d, isz_d;        // 1 / sigma, so the fits multiply instead of divide
};


// Where a module's anchor hits lie (nominal sensor extent widened by a small
// tolerance): transverse radius, z and azimuth ranges (phi in [0, 2 pi)).
// Hits off their sensor are rejected as invalid input, so these boxes bound
// every MD anchor of the module.
struct ModBox {
    float r_lo, r_hi, z_lo, z_hi, phi_lo, phi_hi, pad0, pad1;
};

// A run of a module's map row: n consecutive target modules t_first ..
// t_first + n - 1 of one detector row (one barrel z tile or endcap ring),
// adjacent in phi from phi_start, each 1 / inv_dphi wide, with the row's
// anchor extent (ModBox ranges) and the largest per-MD resolution term q of
// an anchor in the row.
struct RunRec {
    int32_t t_first, n;
    int32_t flags;                  // kRun* bits
    int32_t pad0;
    float phi_start, inv_dphi;
    float r_lo, r_hi, z_lo, z_hi;
    float qb_max, pad1;
};
constexpr int32_t kRunEndcap = 1;     // the row is an endcap ring
constexpr int32_t kRunNoTrim = 2;     // no phi trimming: the run reaches phi separations where a circle
                                      // through the beam line could pass the curvature cut on its far side

// Edge classifier: layers in model-blob order; all but the last are run on
// MFMA from fragments in A-operand order (see lst_gnn.hip).
enum GnnLayer {
    kGEnc1, kGEnc2, kGInit, kGEdgeA0, kGEdgeB0, kGNodeA0, kGNodeB0, kGEdgeA1, kGEdgeB1, kGNodeA1, kGNodeB1,
    kGHead1, kGHead2, kGnnLayers
};

// Everything the device needs from a geometry blob.
struct GeomHost {
    int32_t n_mod = 0, n_barrel = 0, n_map = 0;
    CutParams cp{};
    std::vector<ModConst> mods;        // [n_mod]
    std::vector<ModBox> boxes;         // [n_mod]
    std::vector<int32_t> map_off;      // [n_mod + 1]
    std::vector<int32_t> map_tgt;      // [max(n_map, 1)]
    std::vector<int32_t> run_off;      // [n_mod + 1]
    std::vector<RunRec> runs;          // [max(runs, 1)]
};

// The T5-DNN weights and standardisation, in blob order.
struct ModelHost {
    std::vector<float> w;
};

// Edge-classifier weights: BF16 fragments of the MFMA layers, FP32 biases
// followed by the head's output weights, and each layer's first fragment and
// first bias.
struct GnnHost {
    std::vector<uint16_t> frag;
    std::vector<float> bias;
    int64_t foff[kGnnLayers] = {}, boff[kGnnLayers] = {};
    float bh2 = 0.0f;
};

// Each parser returns false with a message in err on a malformed blob (bad
// magic, version, sizes, counts, indices or values); it never reads outside
// [blob, blob + nbytes).
bool parse_geometry(const void *blob, size_t nbytes, GeomHost &g, std::string &err);
bool parse_model(const void *blob, size_t nbytes, ModelHost &m, std::string &err);
bool parse_gnn(const void *blob, size_t nbytes, GnnHost &g, std::string &err);

}  // namespace lst
