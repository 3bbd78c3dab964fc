// Track-candidate selection (Table 1 steps 5-8) and duplicate removal (named
// in Sec. 2), on the objects of a build and a list of pixel seeds.
//
// The paper describes these steps in words only; the rules implemented here:
//  * every T5 and T3 gets helix parameters (kappa = signed half-curvature,
//    phi0, cot(theta), z0) from its first and last anchor hits on a circle
//    through the beam line, in FP64;
//  * a seed and an object match when the chi2 of their parameter differences
//    (widths of seed and object in quadrature) is at most chi2_max;
//  * pT5: seed and T5 that are each other's best match (smallest chi2 rounded
//    to FP32, ties to the smaller index); T5: the other T5s; pT3: the same
//    mutual best match between the seeds left and the T3s that are in no
//    pT5's T5; pLS: the seeds left;
//  * duplicate removal: two TCs with outer-tracker MDs are duplicates when
//    they share more than half of the smaller one's MDs; a TC with a duplicate
//    of higher priority (kind, then quality, then index) is removed.
//
// Layout: objects are binned per (event, phi0 bin) with a counting sort, so a
// seed (one thread) visits only the bins its chi2_max window in phi0 reaches.
// Best matches are kept as 64-bit (chi2 bits, index) words: per seed in a
// register, per object with a 64-bit atomicMin. Candidate lists are compacted
// in index order with a block-sum / scan / scatter sequence, so every output
// is deterministic.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lst_tc.h"

namespace lst {
namespace {

constexpr int kTcBlock = 256;
constexpr int kScanItems = 1024;          // items per block of the compaction scans (4 per thread)
constexpr int kTcMaxGrid = 8192;
constexpr uint64_t kNone = ~0ull;
constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 6.283185307179586;

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

inline int grid_of(int64_t n, int block = kTcBlock) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > kTcMaxGrid) g = kTcMaxGrid;
    return (int)g;
}

__device__ __forceinline__ double wrap_pi(double a) {
    // (-pi, pi]
    a = fmod(a + kPi, kTwoPi);
    if (a < 0.0) a += kTwoPi;
    return a - kPi;
}

// largest e in [0, n] with off[e] <= i (off ascending, off[0] = 0)
__device__ __forceinline__ int event_of(const int64_t *off, int n, int64_t i) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int phi_bin(double phi) {
    const int b = (int)floor((phi + kPi) * (kTcPhiBins / kTwoPi));
    return b < 0 ? 0 : (b >= kTcPhiBins ? kTcPhiBins - 1 : b);
}

// bin of asinh(cot) = pseudorapidity; values beyond +-kTcEtaMax go to the edge bins
__device__ __forceinline__ int eta_bin(double eta) {
    const double f = (eta + kTcEtaMax) * (kTcEtaBins / (2.0 * kTcEtaMax));
    if (!(f >= 0.0)) return 0;
    return f >= kTcEtaBins ? kTcEtaBins - 1 : (int)f;
}

__device__ __forceinline__ uint64_t pack(float chi2, int32_t idx) {
    return ((uint64_t)__float_as_uint(chi2) << 32) | (uint32_t)idx;
}

// First and last MD of an object: T5 i < n5, else T3 i - n5.
__device__ __forceinline__ int2 obj_ends(const TcArgs &a, int64_t i) {
    if (i < a.n5) {
        const int2 t = a.t5_t3[i];
        return make_int2(a.ls_md[a.t3_ls[t.x].x].x, a.ls_md[a.t3_ls[t.y].y].y);
    }
    const int2 t = a.t3_ls[i - a.n5];
    return make_int2(a.ls_md[t.x].x, a.ls_md[t.y].y);
}

// MDs of an object (5 for a T5, 3 for a T3); returns the count.
__device__ __forceinline__ int obj_mds(const TcArgs &a, int kind, int32_t o, int32_t *m) {
    if (kind == kTcT3) {
        const int2 t = a.t3_ls[o];
        const int2 l0 = a.ls_md[t.x], l1 = a.ls_md[t.y];
        m[0] = l0.x; m[1] = l0.y; m[2] = l1.y; m[3] = m[4] = -1;
        return 3;
    }
    const int2 t = a.t5_t3[o];
    const int2 i0 = a.t3_ls[t.x], i1 = a.t3_ls[t.y];
    const int2 a0 = a.ls_md[i0.x], a1 = a.ls_md[i0.y], b0 = a.ls_md[i1.x], b1 = a.ls_md[i1.y];
    m[0] = a0.x; m[1] = a0.y; m[2] = a1.y; m[3] = b0.y; m[4] = b1.y;
    return 5;
}

// ------------------------------------------------------------ parameters

__global__ void k_tc_params(TcArgs a, TcWork w) {
    const int64_t n = a.n5 + a.n3;
    for (int64_t i = gtid(); i < n; i += gstride()) {
        const int2 ends = obj_ends(a, i);
        const int32_t ha = a.md_hits[ends.x].x, he = a.md_hits[ends.y].x;
        const double xa = a.x[ha], ya = a.y[ha], za = a.z[ha];
        const double xe = a.x[he], ye = a.y[he], ze = a.z[he];
        const double ra = sqrt(xa * xa + ya * ya), re = sqrt(xe * xe + ye * ye);
        const double cr = xa * ye - ya * xe;
        const double dl = sqrt((xe - xa) * (xe - xa) + (ye - ya) * (ye - ya));
        const double c = fabs(cr) / (ra * re * dl);
        const double sgn = cr < 0.0 ? -1.0 : 1.0;
        double4 P = make_double4(0.0, 0.0, NAN, 0.0);
        int key = -1;
        if (c * ra < 1.0 && c * re < 1.0) {
            const double sa = c > 0.0 ? asin(c * ra) / c : ra;
            const double se = c > 0.0 ? asin(c * re) / c : re;
            if (se > sa) {
                const double cot = (ze - za) / (se - sa);
                const double phi0 = wrap_pi(atan2(ya, xa) - sgn * asin(c * ra));
                P = make_double4(sgn * c, phi0, cot, za - sa * cot);
                const bool t5 = i < a.n5;
                const int64_t *off = t5 ? a.ev_obj + 3 * (a.n_ev + 1) : a.ev_obj + 2 * (a.n_ev + 1);
                const int e = event_of(off, a.n_ev, t5 ? i : i - a.n5);
                key = (t5 ? 0 : a.n_ev * kTcBinsPerEvent) + e * kTcBinsPerEvent +
                      eta_bin(asinh(cot)) * kTcPhiBins + phi_bin(phi0);
                atomicAdd(&w.bin_cnt[key], 1);
            }
        }
        w.par[i] = P;
        w.okey[i] = key;
        w.obj_best[i] = kNone;
        w.obj_pair[i] = -1;
    }
}

__global__ void k_tc_bin_scatter(TcArgs a, TcWork w) {
    const int64_t n = a.n5 + a.n3;
    for (int64_t i = gtid(); i < n; i += gstride()) {
        const int key = w.okey[i];
        if (key < 0) continue;
        const int32_t pos = w.bin_off[key] + atomicAdd(&w.bin_cur[key], 1);
        w.bin_obj[pos] = (int32_t)i;
    }
}

// ------------------------------------------------------------ matching

// One seed per thread: best object of the seed, and the seed offered to every
// matching object (atomicMin of (chi2, seed)). T3 = false: T5s, every seed;
// true: T3s in no pT5's T5, seeds in no pT5.
template <bool T3>
__global__ void k_tc_match(TcArgs a, TcWork w) {
    for (int64_t s = gtid(); s < a.ns; s += gstride()) {
        uint64_t best = kNone;
        if (!T3 || w.seed_pair[s] < 0) {
            const float *sp = a.seeds + 8 * s;
            const double sk = sp[0], sphi = sp[1], sc = sp[2], sz = sp[3];
            const double wk = (double)sp[4] * sp[4], wphi = (double)sp[5] * sp[5];
            const double wc = (double)sp[6] * sp[6], wz = (double)sp[7] * sp[7];
            const double ophi = (double)a.opt.sigma_phi0 * a.opt.sigma_phi0;
            const double oc = (double)a.opt.sigma_cot * a.opt.sigma_cot;
            const double oz = (double)a.opt.sigma_z0 * a.opt.sigma_z0;
            const double cmax = a.opt.chi2_max;
            const int e = event_of(a.seed_off, a.n_ev, s);
            // windows in phi0 and cot: chi2 >= d^2 / (sigma_p^2 + sigma_o^2) for each parameter
            const double hw = sqrt(cmax * (wphi + ophi)) * (1.0 + 1e-9) + 1e-12;
            const double hc = sqrt(cmax * (wc + oc)) * (1.0 + 1e-9) + 1e-12;
            int b0 = 0, nb = kTcPhiBins;
            if (hw < kPi) {
                b0 = (int)floor((sphi - hw + kPi) * (kTcPhiBins / kTwoPi));
                const int b1 = (int)floor((sphi + hw + kPi) * (kTcPhiBins / kTwoPi));
                nb = b1 - b0 + 1;
                if (nb > kTcPhiBins) nb = kTcPhiBins;
            }
            const int c0 = eta_bin(asinh(sc - hc)), c1 = eta_bin(asinh(sc + hc));
            const int ebase = (T3 ? a.n_ev * kTcBinsPerEvent : 0) + e * kTcBinsPerEvent;
            for (int cb = c0; cb <= c1; ++cb)
            for (int j = 0; j < nb; ++j) {
                int b = (b0 + j) % kTcPhiBins;
                if (b < 0) b += kTcPhiBins;
                const int key = ebase + cb * kTcPhiBins + b;
                for (int32_t q = w.bin_off[key]; q < w.bin_off[key + 1]; ++q) {
                    const int32_t o = w.bin_obj[q];
                    if (T3 && w.t3_used[o - a.n5]) continue;
                    const double4 P = w.par[o];
                    const double ok = (double)a.opt.sigma_kappa_rel * fabs(P.x) + a.opt.sigma_kappa_abs;
                    double dp = sphi - P.y;   // both in (-pi, pi]: one turn at most
                    if (dp > kPi) dp -= kTwoPi;
                    else if (dp <= -kPi) dp += kTwoPi;
                    const double dk = sk - P.x, dc = sc - P.z, dz = sz - P.w;
                    const double chi2 = dk * dk / (wk + ok * ok) + dp * dp / (wphi + ophi) + dc * dc / (wc + oc) +
                                        dz * dz / (wz + oz);
                    if (!(chi2 <= cmax)) continue;
                    const float cf = (float)chi2;
                    const int32_t local = T3 ? o - (int32_t)a.n5 : o;
                    const uint64_t mine = pack(cf, local);
                    best = mine < best ? mine : best;
                    atomicMin((unsigned long long *)&w.obj_best[o], (unsigned long long)pack(cf, (int32_t)s));
                }
            }
        }
        w.seed_best[s] = best;
    }
}

template <bool T3>
__global__ void k_tc_mutual(TcArgs a, TcWork w) {
    for (int64_t s = gtid(); s < a.ns; s += gstride()) {
        const uint64_t b = w.seed_best[s];
        if (b == kNone) continue;
        const int32_t local = (int32_t)(uint32_t)b;
        const int64_t o = T3 ? a.n5 + local : local;
        const uint64_t ob = w.obj_best[o];
        if ((int32_t)(uint32_t)ob == (int32_t)s) {
            w.seed_pair[s] = local;
            w.seed_kind[s] = T3 ? kTcPT3 : kTcPT5;
            w.seed_chi2[s] = __uint_as_float((uint32_t)(b >> 32));
            w.obj_pair[o] = (int32_t)s;
        }
    }
}

__global__ void k_tc_mark_t3(TcArgs a, TcWork w) {
    for (int64_t t = gtid(); t < a.n5; t += gstride()) {
        if (w.obj_pair[t] < 0) continue;
        const int2 p = a.t5_t3[t];
        w.t3_used[p.x] = 1;
        w.t3_used[p.y] = 1;
    }
}

__global__ void k_tc_seed_init(TcArgs a, TcWork w) {
    for (int64_t s = gtid(); s < a.ns; s += gstride()) {
        w.seed_pair[s] = -1;
        w.seed_kind[s] = kTcPLS;
        w.seed_chi2[s] = 0.0f;
    }
    for (int64_t t = gtid(); t < a.n3; t += gstride()) w.t3_used[t] = 0;
}

__global__ void k_tc_reset_best(TcArgs a, TcWork w) {
    for (int64_t i = gtid(); i < a.n3; i += gstride()) w.obj_best[a.n5 + i] = kNone;
}

// ------------------------------------------------------------ compaction

// Candidate u of the TC list before duplicate removal, in output order:
// [0, n5) pT5 by T5, [n5, 2 n5) T5, [2 n5, 2 n5 + n3) pT3 by T3, then pLS by seed.
struct TcCand {
    TcArgs a;
    TcWork w;
    __device__ __forceinline__ int64_t size() const { return 2 * a.n5 + a.n3 + a.ns; }
    __device__ __forceinline__ bool get(int64_t u, int &kind, int32_t &seed, int32_t &obj) const {
        if (u < a.n5) {
            kind = kTcPT5; obj = (int32_t)u; seed = w.obj_pair[u];
            return seed >= 0;
        }
        if (u < 2 * a.n5) {
            kind = kTcT5; obj = (int32_t)(u - a.n5); seed = -1;
            return w.obj_pair[obj] < 0;
        }
        if (u < 2 * a.n5 + a.n3) {
            kind = kTcPT3; obj = (int32_t)(u - 2 * a.n5); seed = w.obj_pair[a.n5 + obj];
            return seed >= 0;
        }
        kind = kTcPLS; seed = (int32_t)(u - 2 * a.n5 - a.n3); obj = -1;
        return w.seed_pair[seed] < 0;
    }
    __device__ __forceinline__ int value(int64_t u) const {
        int k; int32_t s, o;
        return get(u, k, s, o) ? 1 : 0;
    }
    __device__ __forceinline__ void put(int64_t u, int64_t pos) const {
        int kind; int32_t seed, obj;
        if (!get(u, kind, seed, obj)) return;
        w.c_kind[pos] = kind;
        w.c_seed[pos] = seed;
        w.c_obj[pos] = obj;
        double q = 0.0;
        if (kind == kTcPT3) {
            q = (double)w.seed_chi2[seed];
        } else if (kind != kTcPLS) {
            const float sc = a.t5_score[obj];
            q = isfinite(sc) ? -(double)sc : (double)a.t5_chi2_rphi[obj];
        }
        *(int4 *)&w.c_key[2 * pos] = make_int4(__double2loint(q), __double2hiint(q), obj, kind);
        int32_t m[5] = {-1, -1, -1, -1, -1};
        const int nm = kind == kTcPLS ? 0 : obj_mds(a, kind == kTcPT3 ? kTcT3 : kTcT5, obj, m);
        *(int4 *)&w.c_md[8 * pos] = make_int4(m[0], nm > 1 ? m[1] : -1, nm > 2 ? m[2] : -1, nm > 3 ? m[3] : -1);
        *(int4 *)&w.c_md[8 * pos + 4] = make_int4(nm > 4 ? m[4] : -1, -1, -1, -1);
        w.c_drop[pos] = 0;
        for (int k = 0; k < nm; ++k) atomicAdd(&w.md_cnt[m[k]], 1);
    }
};

// Kept TCs, in list order.
struct TcKept {
    TcWork w;
    __device__ __forceinline__ int64_t size() const { return w.n_cand[0]; }
    __device__ __forceinline__ int value(int64_t u) const { return w.c_drop[u] ? 0 : 1; }
    __device__ __forceinline__ void put(int64_t u, int64_t pos) const {
        if (w.c_drop[u]) return;
        if (pos < w.cap_tc) {
            w.out_kind[pos] = w.c_kind[u];
            w.out_seed[pos] = w.c_seed[u];
            w.out_obj[pos] = w.c_obj[u];
        }
    }
};

// Offsets of the object bins (and the end entry).
struct BinOff {
    TcWork w;
    int64_t n;
    __device__ __forceinline__ int64_t size() const { return n; }
    __device__ __forceinline__ int value(int64_t i) const { return w.bin_cnt[i]; }
    __device__ __forceinline__ void put(int64_t i, int64_t pos) const {
        w.bin_off[i] = (int32_t)pos;
        w.bin_cur[i] = 0;
        if (i == n - 1) w.bin_off[n] = (int32_t)(pos + w.bin_cnt[i]);
    }
};

// Offsets of the MD -> TC incidence lists.
struct MdOff {
    TcArgs a;
    TcWork w;
    __device__ __forceinline__ int64_t size() const { return a.n_md; }
    __device__ __forceinline__ int value(int64_t m) const { return w.md_cnt[m]; }
    __device__ __forceinline__ void put(int64_t m, int64_t pos) const {
        w.md_off[m] = pos;
        w.md_cur[m] = 0;
    }
};

// Sums of 1024 consecutive item values per block.
template <class F>
__global__ __launch_bounds__(kTcBlock) void k_blk_sum(F f, int64_t *blk) {
    __shared__ int64_t red[kTcBlock / 64];
    const int64_t n = f.size();
    const int64_t nblk = (n + kScanItems - 1) / kScanItems;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int64_t i0 = b * kScanItems + 4 * threadIdx.x;
        int64_t s = 0;
        for (int k = 0; k < 4; ++k)
            if (i0 + k < n) s += f.value(i0 + k);
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t t = 0;
            for (int k = 0; k < kTcBlock / 64; ++k) t += red[k];
            blk[b] = t;
        }
        __syncthreads();
    }
}

// Exclusive scan of the block sums in one block; total in blk[nblk] and *total.
template <class F>
__global__ void k_blk_scan(F f, int64_t *blk, int64_t *total) {
    __shared__ int64_t part[1024];
    const int64_t n = f.size();
    const int64_t nblk = (n + kScanItems - 1) / kScanItems;
    const int t = threadIdx.x;
    const int64_t per = (nblk + 1023) / 1024;
    const int64_t b0 = t * per, b1 = b0 + per < nblk ? b0 + per : nblk;
    int64_t s = 0;
    for (int64_t i = b0; i < b1; ++i) s += blk[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int i = 0; i < 1024; ++i) {
            const int64_t v = part[i];
            part[i] = run;
            run += v;
        }
        blk[nblk] = run;
        if (total) *total = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int64_t i = b0; i < b1; ++i) {
        const int64_t v = blk[i];
        blk[i] = run;
        run += v;
    }
}

// Every item gets its exclusive prefix: f.put(i, prefix).
template <class F>
__global__ __launch_bounds__(kTcBlock) void k_blk_apply(F f, const int64_t *blk) {
    __shared__ int64_t wsum[kTcBlock / 64];
    const int64_t n = f.size();
    const int64_t nblk = (n + kScanItems - 1) / kScanItems;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int64_t i0 = b * kScanItems + 4 * threadIdx.x;
        int v[4];
        int64_t s = 0;
        for (int k = 0; k < 4; ++k) {
            v[k] = i0 + k < n ? f.value(i0 + k) : 0;
            s += v[k];
        }
        int64_t incl = s;
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        int64_t base = blk[b];
        for (int k = 0; k < wv; ++k) base += wsum[k];
        int64_t pos = base + incl - s;
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < n) f.put(i0 + k, pos);
            pos += v[k];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ duplicates

__global__ void k_tc_incidence(TcWork w) {
    const int64_t n = w.n_cand[0];
    for (int64_t u = gtid(); u < n; u += gstride()) {
        for (int k = 0; k < 5; ++k) {
            const int32_t m = w.c_md[8 * u + k];
            if (m < 0) break;
            const int32_t p = atomicAdd(&w.md_cur[m], 1);
            w.md_tc[w.md_off[m] + p] = (int32_t)u;
        }
    }
}

// priority key of a TC: (quality, kind << 32 | object index) in 16 bytes
__device__ __forceinline__ void tc_key(const TcWork &w, int64_t i, double &q, int64_t &ko) {
    const int4 v = *(const int4 *)&w.c_key[2 * i];
    q = __hiloint2double(v.y, v.x);
    ko = ((int64_t)v.w << 32) | (uint32_t)v.z;
}

// priority of key j over key i: kind, then quality, then object index
__device__ __forceinline__ bool key_before(double qj, int64_t koj, double qi, int64_t koi) {
    const int64_t kj = koj >> 32, ki = koi >> 32;
    if (kj != ki) return kj < ki;
    if (qj != qi) return qj < qi;
    return koj < koi;
}

// 16 lanes per TC walk the incidence lists of its MDs together; a candidate
// j is compared only when it has priority over i.
constexpr int kDupLanes = 16;
__global__ __launch_bounds__(kTcBlock) void k_tc_dups(TcWork w) {
    const int64_t n = w.n_cand[0];
    const int lane = threadIdx.x & 63, gl = threadIdx.x & (kDupLanes - 1);
    const int64_t g0 = ((int64_t)blockIdx.x * kTcBlock + threadIdx.x) / kDupLanes;
    const int64_t gs = (int64_t)gridDim.x * kTcBlock / kDupLanes;
    for (int64_t i = g0; i < n; i += gs) {
        const int4 ma = *(const int4 *)&w.c_md[8 * i], mb = *(const int4 *)&w.c_md[8 * i + 4];
        const int32_t mi[5] = {ma.x, ma.y, ma.z, ma.w, mb.x};
        const int ni = (ma.x >= 0) + (ma.y >= 0) + (ma.z >= 0) + (ma.w >= 0) + (mb.x >= 0);
        // the incidence lists of MDs 0..4 as one sequence of tot entries
        // (MD slots are filled from the front: a -1 ends the list)
        const int64_t o0 = ma.x >= 0 ? w.md_off[ma.x] : 0, o1 = ma.y >= 0 ? w.md_off[ma.y] : 0;
        const int64_t o2 = ma.z >= 0 ? w.md_off[ma.z] : 0, o3 = ma.w >= 0 ? w.md_off[ma.w] : 0;
        const int64_t o4 = mb.x >= 0 ? w.md_off[mb.x] : 0;
        const int e1 = ma.x >= 0 ? w.md_cnt[ma.x] : 0;
        const int e2 = e1 + (ma.y >= 0 ? w.md_cnt[ma.y] : 0);
        const int e3 = e2 + (ma.z >= 0 ? w.md_cnt[ma.z] : 0);
        const int e4 = e3 + (ma.w >= 0 ? w.md_cnt[ma.w] : 0);
        int tot = e4 + (mb.x >= 0 ? w.md_cnt[mb.x] : 0);
        double qi;
        int64_t koi;
        tc_key(w, i, qi, koi);
        // a TC only loses to a kind at least as long: a pT5 / T5 (5 MDs) to
        // one sharing 3 of them, so to one in the lists of its first 3 MDs; a
        // pT3 (3 MDs) to one sharing 2, so to one in the lists of its first 2
        tot = (koi >> 32) <= kTcT5 ? e3 : e2;
        bool drop = false;
        for (int t = gl; t < tot && !drop; t += kDupLanes) {
            const int64_t src = t < e1 ? o0 + t : t < e2 ? o1 + (t - e1) : t < e3 ? o2 + (t - e2)
                              : t < e4 ? o3 + (t - e3) : o4 + (t - e4);
            const int32_t j = w.md_tc[src];
            if (j == i) continue;
            double qj;
            int64_t koj;
            tc_key(w, j, qj, koj);
            if (!key_before(qj, koj, qi, koi)) continue;
            const int4 ja = *(const int4 *)&w.c_md[8 * (int64_t)j], jb = *(const int4 *)&w.c_md[8 * (int64_t)j + 4];
            const int32_t mj[5] = {ja.x, ja.y, ja.z, ja.w, jb.x};
            int nj = 0, shared = 0;
            for (int l = 0; l < 5; ++l) {
                if (mj[l] < 0) continue;
                ++nj;
                for (int q = 0; q < ni; ++q) shared += mj[l] == mi[q];
            }
            const int nmin = ni < nj ? ni : nj;
            if (2 * shared > nmin) drop = true;
        }
        const unsigned long long bal = __ballot(drop);
        const unsigned long long gmask = ((1ull << kDupLanes) - 1) << (lane & ~(kDupLanes - 1));
        if (gl == 0) w.c_drop[i] = (bal & gmask) ? 1 : 0;
    }
}

// Kept TCs per kind: block sums, one atomic add per block and kind.
__global__ __launch_bounds__(kTcBlock) void k_tc_kind_counts(TcWork w) {
    __shared__ unsigned long long cnt[4];
    if (threadIdx.x < 4) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t n = w.n_cand[0];
    unsigned long long c[4] = {0, 0, 0, 0};
    for (int64_t u = gtid(); u < n; u += gstride())
        if (!w.c_drop[u]) ++c[w.c_kind[u] & 3];
    for (int k = 0; k < 4; ++k) {
        unsigned long long v = c[k];
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd(&cnt[k], v);
    }
    __syncthreads();
    if (threadIdx.x < 4 && cnt[threadIdx.x])
        atomicAdd((unsigned long long *)&w.out_counts[threadIdx.x], cnt[threadIdx.x]);
}

__global__ void k_tc_zero(TcWork w, int64_t n_md) {
    for (int64_t m = gtid(); m < n_md; m += gstride()) w.md_cnt[m] = 0;
    if (gtid() == 0) {
        for (int k = 0; k < kTcCounts; ++k) w.out_counts[k] = 0;
    }
}

__global__ void k_tc_zero_bins(TcWork w, int64_t nbins) {
    for (int64_t i = gtid(); i < nbins; i += gstride()) w.bin_cnt[i] = 0;
}

__global__ void k_tc_single_off(int64_t *ev_obj, int64_t n_md, int64_t n_ls, int64_t n3, int64_t n5) {
    if (gtid() == 0) {
        ev_obj[0] = 0; ev_obj[1] = n_md;
        ev_obj[2] = 0; ev_obj[3] = n_ls;
        ev_obj[4] = 0; ev_obj[5] = n3;
        ev_obj[6] = 0; ev_obj[7] = n5;
    }
}

__global__ void k_tc_totals(TcWork w) {
    if (gtid() == 0) {
        w.out_counts[kTcCountKept] = w.out_counts[0] + w.out_counts[1] + w.out_counts[2] + w.out_counts[3];
        w.out_counts[kTcCountBefore] = w.n_cand[0];
    }
}

template <class F>
void compact(F f, int64_t n_max, int64_t *blk, int64_t *total, hipStream_t st) {
    const int64_t nblk = (n_max + kScanItems - 1) / kScanItems;
    const int g = (int)(nblk < 1 ? 1 : (nblk > kTcMaxGrid ? kTcMaxGrid : nblk));
    hipLaunchKernelGGL(k_blk_sum<F>, dim3(g), dim3(kTcBlock), 0, st, f, blk);
    hipLaunchKernelGGL(k_blk_scan<F>, dim3(1), dim3(1024), 0, st, f, blk, total);
    hipLaunchKernelGGL(k_blk_apply<F>, dim3(g), dim3(kTcBlock), 0, st, f, (const int64_t *)blk);
}

}  // namespace

size_t tc_layout(const TcSizes &z, char *base, TcWork *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const int64_t no = z.n5 + z.n3, nc = z.n5 + z.n3 + z.ns, nbins = 2 * (int64_t)z.n_ev * kTcBinsPerEvent;
    int64_t nscan = 2 * z.n5 + z.n3 + z.ns > z.n_md ? 2 * z.n5 + z.n3 + z.ns : z.n_md;
    nscan = nscan > nbins ? nscan : nbins;
    TcWork x{};
    x.par = (double4 *)take(sizeof(double4) * (no + 1));
    x.okey = (int32_t *)take(4 * (no + 1));
    x.obj_best = (uint64_t *)take(8 * (no + 1));
    x.obj_pair = (int32_t *)take(4 * (no + 1));
    x.bin_cnt = (int32_t *)take(4 * (nbins + 1));
    x.bin_off = (int32_t *)take(4 * (nbins + 1));
    x.bin_cur = (int32_t *)take(4 * (nbins + 1));
    x.bin_obj = (int32_t *)take(4 * (no + 1));
    x.seed_best = (uint64_t *)take(8 * (z.ns + 1));
    x.seed_pair = (int32_t *)take(4 * (z.ns + 1));
    x.seed_kind = (int32_t *)take(4 * (z.ns + 1));
    x.seed_chi2 = (float *)take(4 * (z.ns + 1));
    x.t3_used = (int32_t *)take(4 * (z.n3 + 1));
    x.c_kind = (int32_t *)take(4 * (nc + 1));
    x.c_seed = (int32_t *)take(4 * (nc + 1));
    x.c_obj = (int32_t *)take(4 * (nc + 1));
    x.c_key = (int64_t *)take(16 * (nc + 1));
    x.c_md = (int32_t *)take(32 * (nc + 1));
    x.c_drop = (int32_t *)take(4 * (nc + 1));
    x.md_cnt = (int32_t *)take(4 * (z.n_md + 1));
    x.md_off = (int64_t *)take(8 * (z.n_md + 1));
    x.md_cur = (int32_t *)take(4 * (z.n_md + 1));
    x.md_tc = (int32_t *)take(20 * (nc + 1));
    x.blk = (int64_t *)take(8 * (nscan / kScanItems + 2));
    x.n_cand = (int64_t *)take(8 * 2);
    x.ev_single = (int64_t *)take(8 * 8);
    if (w) *w = x;
    return off;
}

hipError_t run_tc(const TcArgs &a0, const TcWork &w0, hipStream_t st) {
    TcArgs a = a0;
    TcWork w = w0;
    if (!a.ev_obj) {
        hipLaunchKernelGGL(k_tc_single_off, dim3(1), dim3(64), 0, st, w.ev_single, a.n_md, a.n_ls, a.n3, a.n5);
        a.ev_obj = w.ev_single;
    }
    const int64_t no = a.n5 + a.n3, nbins = 2 * (int64_t)a.n_ev * kTcBinsPerEvent;
    hipLaunchKernelGGL(k_tc_zero_bins, dim3(grid_of(nbins)), dim3(kTcBlock), 0, st, w, nbins);
    hipLaunchKernelGGL(k_tc_zero, dim3(grid_of(a.n_md)), dim3(kTcBlock), 0, st, w, a.n_md);
    hipLaunchKernelGGL(k_tc_seed_init, dim3(grid_of(a.ns > a.n3 ? a.ns : a.n3)), dim3(kTcBlock), 0, st, a, w);
    hipLaunchKernelGGL(k_tc_params, dim3(grid_of(no)), dim3(kTcBlock), 0, st, a, w);
    compact(BinOff{w, nbins}, nbins, w.blk, nullptr, st);
    hipLaunchKernelGGL(k_tc_bin_scatter, dim3(grid_of(no)), dim3(kTcBlock), 0, st, a, w);
    // steps 5 and 7: pT5, then pT3 among what is left
    hipLaunchKernelGGL(k_tc_match<false>, dim3(grid_of(a.ns, 64)), dim3(64), 0, st, a, w);
    hipLaunchKernelGGL(k_tc_mutual<false>, dim3(grid_of(a.ns)), dim3(kTcBlock), 0, st, a, w);
    hipLaunchKernelGGL(k_tc_mark_t3, dim3(grid_of(a.n5)), dim3(kTcBlock), 0, st, a, w);
    hipLaunchKernelGGL(k_tc_reset_best, dim3(grid_of(a.n3)), dim3(kTcBlock), 0, st, a, w);
    hipLaunchKernelGGL(k_tc_match<true>, dim3(grid_of(a.ns, 64)), dim3(64), 0, st, a, w);
    hipLaunchKernelGGL(k_tc_mutual<true>, dim3(grid_of(a.ns)), dim3(kTcBlock), 0, st, a, w);
    // TC list (steps 5-8), then duplicate removal
    compact(TcCand{a, w}, 2 * a.n5 + a.n3 + a.ns, w.blk, w.n_cand, st);
    compact(MdOff{a, w}, a.n_md, w.blk, nullptr, st);
    const int64_t nc = a.n5 + a.n3 + a.ns;
    hipLaunchKernelGGL(k_tc_incidence, dim3(grid_of(nc)), dim3(kTcBlock), 0, st, w);
    hipLaunchKernelGGL(k_tc_dups, dim3(grid_of(nc * kDupLanes)), dim3(kTcBlock), 0, st, w);
    compact(TcKept{w}, nc, w.blk, nullptr, st);
    hipLaunchKernelGGL(k_tc_kind_counts, dim3(grid_of(nc < 262144 ? nc : 262144)), dim3(kTcBlock), 0, st, w);
    hipLaunchKernelGGL(k_tc_totals, dim3(1), dim3(64), 0, st, w);
    return hipGetLastError();
}

}  // namespace lst
