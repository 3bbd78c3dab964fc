// Device-side data layout and arithmetic of the LST object builder (gfx950).
//
// Cuts (paper Sec. 1: each object is kept only if its hits are compatible
// with one helix from the beam line) are evaluated in FP32; the paper gives no
// formulas, so they follow this project's reading, derived from the helix of a
// track from the beam line: half-curvature c = 1 / (2R), radius along the arc
// r(s) = sin(c s) / c, z linear in s. Every cut is "pass iff v <= t" written
// as !(v <= t) -> reject, so NaN rejects. The quintuplet fits and the T5-DNN
// features (Sec. 2) are evaluated in FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lst_host.h"

namespace lst {

constexpr int kMinTile = 256;       // smallest compaction tile (candidates)

struct ModelDev {
    const float *mu, *sd, *W1, *b1, *W2, *b2, *w3;
    float b3;
};

// Batch-wide geometry handles.
struct GeomDev {
    const ModConst *mod;
    const int32_t *map_off;   // [n_mod + 1]
    const int32_t *map_tgt;   // [n_map]
    const ModBox *box;        // [n_mod]
    const int32_t *run_off;   // [n_mod + 1] runs of each module's map row
    const RunRec *runs;       // [n_runs]
    int32_t n_mod, n_sens, n_map;
};

// ------------------------------------------------------------ small helpers

// Read-only value at a wavefront-uniform address, through the constant
// address space so that it is a scalar load (for data written by an earlier
// launch, or by the host, and not written by the reading kernel).
template <class T>
__device__ __forceinline__ T ld_scalar(const T *p) { return *(const __attribute__((address_space(4))) T *)p; }

__device__ __forceinline__ float kahan_det(float a, float b, float c, float d) {
    // a*d - b*c with Kahan's FMA compensation (error ~1 ulp of the result)
    float w = b * c;
    float e = __builtin_fmaf(-b, c, w);
    float f = __builtin_fmaf(a, d, -w);
    return f + e;
}

__device__ __forceinline__ float cross2(float ax, float ay, float bx, float by) {
    return kahan_det(ax, ay, bx, by);
}

// asin(x) / x for 0 <= x <= 0.8 as a degree-10 polynomial in t = x^2 (Horner),
// relative error below 8e-8 in FP32; coefficients from csrc/fit_arc_poly.py
__device__ __forceinline__ float asin_over_x_f(float t) {
    float g = 6.152549386e-01f;
    g = __builtin_fmaf(g, t, -1.530246854e+00f);
    g = __builtin_fmaf(g, t, 1.748290539e+00f);
    g = __builtin_fmaf(g, t, -1.095079780e+00f);
    g = __builtin_fmaf(g, t, 4.514038861e-01f);
    g = __builtin_fmaf(g, t, -8.377703279e-02f);
    g = __builtin_fmaf(g, t, 4.629246891e-02f);
    g = __builtin_fmaf(g, t, 4.326621071e-02f);
    g = __builtin_fmaf(g, t, 7.506076992e-02f);
    g = __builtin_fmaf(g, t, 1.666656137e-01f);
    return __builtin_fmaf(g, t, 1.0f);
}

// arc length asin(c r) / c (half-curvature c >= 0): r * asin(x) / x below
// x = c r = 0.8, which also covers c -> 0 without a division
__device__ __forceinline__ float arc_len_f(float c, float r) {
    float x = c * r;
    if (x <= 0.8f) return r * asin_over_x_f(x * x);
    if (x >= 1.0f) x = 1.0f;
    return asinf(x) / c;
}

__device__ __forceinline__ double arc_len_d(double c, double r) {
    double x = c * r;
    if (x < 1e-4) return r * (1.0 + x * x / 6.0);
    if (x >= 1.0) x = 1.0;
    return asin(x) / c;
}

struct P3 { float x, y, z; };

// ------------------------------------------------------------ MD cuts (FP32)
// anchor hit i, other hit j on module mc.
__device__ __forceinline__ bool md_pass(const ModConst &mc, const CutParams &p, P3 hi, P3 hj) {
    float cr = cross2(hi.x, hi.y, hj.x, hj.y);
    float dt = hi.x * hj.x + hi.y * hj.y;
    float ang = fabsf(atan2f(cr, dt));
    if (mc.kind == 0) {
        if (!(ang <= mc.b1_t)) return false;
        float a0 = (hi.z - p.zlum) * mc.rho0, a1 = (hi.z + p.zlum) * mc.rho0;
        float b0 = (hi.z - p.zlum) * mc.rho1, b1 = (hi.z + p.zlum) * mc.rho1;
        float lo = fminf(fminf(a0, a1), fminf(b0, b1));
        float hv = fmaxf(fmaxf(a0, a1), fmaxf(b0, b1));
        float v = fabsf((hj.z - hi.z) - 0.5f * (lo + hv));
        float t = 0.5f * (hv - lo) + p.nsig * 1.41421356f * p.sz;
        return v <= t;
    }
    float ri = sqrtf(hi.x * hi.x + hi.y * hi.y), rj = sqrtf(hj.x * hj.x + hj.y * hj.y);
    float az = fabsf(hi.z);
    float xm = fminf(p.cmax * ri, 1.0f);
    float asx = asinf(xm);
    float cxm = sqrtf(1.0f - xm * xm);
    float t1 = mc.gap * asx / (az - p.zlum)
             + p.nsig * (p.srphi * sqrtf(1.0f / (ri * ri) + 1.0f / (rj * rj))
                         + mc.gap * p.cmax * p.sr / ((az - p.zlum) * cxm));
    if (!(ang <= t1)) return false;
    float dr = ((hj.x - hi.x) * (hj.x + hi.x) + (hj.y - hi.y) * (hj.y + hi.y)) / (ri + rj);
    float f = (xm < 1e-8f) ? 1.0f : cxm * asx / xm;
    float lo = mc.gap * ri * f / (az + p.zlum), hv = mc.gap * ri / (az - p.zlum);
    float v = fabsf(dr - 0.5f * (lo + hv));
    float t = 0.5f * (hv - lo) + p.nsig * 1.41421356f * p.sr + p.e2slack;
    return v <= t;
}

// ---------------------------------------------- anchor-pair cuts (FP32)
// Beam-line circle through anchors X (inner) and Y (outer): curvature within
// c_max plus resolution, ordering s_X < s_Y, and z0 pointing into the
// luminous region. Returns pass; c_out = curvature, sgn_out = bending side.
__device__ __forceinline__ bool pair_pass(const CutParams &p, P3 X, bool endX, P3 Y, bool endY,
                                          float &c_out, float &sgn_out) {
    float rX = sqrtf(X.x * X.x + X.y * X.y), rY = sqrtf(Y.x * Y.x + Y.y * Y.y);
    float dx = Y.x - X.x, dy = Y.y - X.y;
    float dl = sqrtf(dx * dx + dy * dy);
    float cr = cross2(X.x, X.y, Y.x, Y.y);
    float c = fabsf(cr) / (rX * rY * dl);
    float srX = endX ? p.sr : 0.0f, srY = endY ? p.sr : 0.0f;
    float szX = endX ? 0.0f : p.sz, szY = endY ? 0.0f : p.sz;
    float sc = sqrtf(p.srphi * p.srphi * (1.0f / (rX * rX) + 1.0f / (rY * rY))
                     + p.cmax * p.cmax * (srX * srX + srY * srY)) / dl;
    c_out = c;
    sgn_out = cr < 0.0f ? -1.0f : 1.0f;
    if (!(c <= p.cmax + p.nsig * sc)) return false;
    float cp = fminf(c, p.cmax);
    float sX = arc_len_f(cp, rX), sY = arc_len_f(cp, rY);
    if (!(sX < sY)) return false;
    float ds = sY - sX;
    float k = (Y.z - X.z) / ds;
    float z0 = X.z - sX * k;
    float a = sY * szX, b = sX * szY, e = sY * srX, f = sX * srY;
    float var = (a * a + b * b + k * k * (e * e + f * f)) / (ds * ds);
    return fabsf(z0) <= p.zlum + p.nsig * sqrtf(var);
}

// Per-MD quantities the pair cuts use, computed once per MD: rq = {r, q}
// with r the transverse radius of the anchor hit and q = srphi^2 / r^2 (plus
// cmax^2 sr^2 for an endcap MD); the sign bit of q marks an endcap MD.
__device__ __forceinline__ float2 make_md_rq(const CutParams &p, float x, float y, bool endcap) {
    const float r = sqrtf(x * x + y * y);
    float q = p.srphi * p.srphi / (r * r);
    if (endcap) q += p.cmax * p.cmax * p.sr * p.sr;
    return make_float2(r, endcap ? -q : q);
}

// pair_pass with the per-MD radii and resolution terms precomputed (md_rq),
// in two parts: the curvature cut, then the ordering and z0 cuts at the
// clamped curvature cp = min(c, cmax).
__device__ __forceinline__ bool pair_curv_pass(const CutParams &p, P3 X, float2 rqX, P3 Y, float2 rqY,
                                               float &c_out, float &sgn_out) {
    const float rX = rqX.x, rY = rqY.x;
    float dx = Y.x - X.x, dy = Y.y - X.y;
    float dl = sqrtf(dx * dx + dy * dy);
    float cr = cross2(X.x, X.y, Y.x, Y.y);
    float c = fabsf(cr) / (rX * rY * dl);
    float sc = sqrtf(fabsf(rqX.y) + fabsf(rqY.y)) / dl;
    c_out = c;
    sgn_out = cr < 0.0f ? -1.0f : 1.0f;
    return c <= p.cmax + p.nsig * sc;
}

__device__ __forceinline__ bool pair_z0_pass(const CutParams &p, P3 X, float2 rqX, P3 Y, float2 rqY, float cp) {
    const float rX = rqX.x, rY = rqY.x;
    const bool endX = signbit(rqX.y), endY = signbit(rqY.y);
    float srX = endX ? p.sr : 0.0f, srY = endY ? p.sr : 0.0f;
    float szX = endX ? 0.0f : p.sz, szY = endY ? 0.0f : p.sz;
    float sX = arc_len_f(cp, rX), sY = arc_len_f(cp, rY);
    if (!(sX < sY)) return false;
    float ds = sY - sX;
    float k = (Y.z - X.z) / ds;
    float z0 = X.z - sX * k;
    float a = sY * szX, b = sX * szY, e = sY * srX, f = sX * srY;
    float var = (a * a + b * b + k * k * (e * e + f * f)) / (ds * ds);
    return fabsf(z0) <= p.zlum + p.nsig * sqrtf(var);
}

__device__ __forceinline__ bool pair_pass_rq(const CutParams &p, P3 X, float2 rqX, P3 Y, float2 rqY,
                                             float &c_out, float &sgn_out) {
    if (!pair_curv_pass(p, X, rqX, Y, rqY, c_out, sgn_out)) return false;
    return pair_z0_pass(p, X, rqX, Y, rqY, fminf(c_out, p.cmax));
}

// MD direction: the chord between the MD's hits follows the track direction at
// the chord midpoint (angle asin(c'|M|) from radial, toward the bending side).
__device__ __forceinline__ bool md_dir_pass(const CutParams &p, P3 hi, float ox, float oy, float cp,
                                            float sgn) {
    float dx = ox - hi.x, dy = oy - hi.y;
    float mx = 0.5f * (hi.x + ox), my = 0.5f * (hi.y + oy);
    float m = sqrtf(mx * mx + my * my);
    float ux = mx / m, uy = my / m;
    float s = fminf(cp * m, 1.0f);
    float cb = sqrtf(1.0f - s * s);
    float tx = cb * ux - sgn * s * uy;
    float ty = cb * uy + sgn * s * ux;
    float v = fabsf(atan2f(tx * dy - ty * dx, tx * dx + ty * dy));
    float t = p.nsig * 1.41421356f * p.srphi / sqrtf(dx * dx + dy * dy) + p.ls3slack;
    return v <= t;
}

// --------------------------------------------------- quintuplet fits (FP64)

struct Fit5 {
    double xm, ym, A, B, C, D;    // natural-form circle over centred coordinates, B^2+C^2-4AD = 1
    double R, chi2_rphi;
    double t, z0, chi2_rz;
};

__device__ __forceinline__ double circle_distance(double A, double B, double C, double D, double u,
                                                  double v) {
    double P = A * (u * u + v * v) + B * u + C * v + D;
    return 2.0 * P / (1.0 + sqrt(1.0 + 4.0 * A * P));
}

// Weighted Taubin (1991) circle fit of 5 points in the frame of the chord from
// the first to the last point: smallest root of the characteristic cubic of
// the generalised eigenproblem by Newton from 0, null vector as the largest
// cross product of two rows; straight lines give A = 0.
// isig[i] = 1 / sigma_i of point i (weights 1 / sigma^2).
__device__ inline void circle_fit5(const double *x, const double *y, const double *isig, Fit5 &f) {
    double W = 0, xm = 0, ym = 0;
    double w[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) { w[i] = isig[i] * isig[i]; W += w[i]; xm += w[i] * x[i]; ym += w[i] * y[i]; }
    const double iW = 1.0 / W;
    xm *= iW; ym *= iW;
#pragma unroll
    for (int i = 0; i < 5; ++i) w[i] *= iW;
    double cx = x[4] - x[0], cy = y[4] - y[0], cl = sqrt(cx * cx + cy * cy);
    double ca = cl > 0 ? cx / cl : 1.0, sa = cl > 0 ? cy / cl : 0.0;
    double u[5], v[5];
    double Mxx = 0, Myy = 0, Mxy = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double wi = w[i];
        double u0 = x[i] - xm, v0 = y[i] - ym;
        u[i] = ca * u0 + sa * v0; v[i] = -sa * u0 + ca * v0;
        Mxx += wi * u[i] * u[i]; Myy += wi * v[i] * v[i]; Mxy += wi * u[i] * v[i];
    }
    double Mz = Mxx + Myy;
    double Mxz = 0, Myz = 0, varz = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double wi = w[i];
        double zt = u[i] * u[i] + v[i] * v[i] - Mz;
        Mxz += wi * u[i] * zt; Myz += wi * v[i] * zt; varz += wi * zt * zt;
    }
    double cov = Mxx * Myy - Mxy * Mxy;
    double c3 = 4.0 * Mz;
    double c2 = -4.0 * Mz * Mz - varz;
    double c1 = varz * Mz + 4.0 * cov * Mz - Mxz * Mxz - Myz * Myz;
    double c0 = Mxz * (Mxz * Myy - Myz * Mxy) + Myz * (Myz * Mxx - Mxz * Mxy) - varz * cov;
    double eta = 0.0, fprev = __builtin_huge_val();
    for (int it = 0; it < 32; ++it) {
        double fv = c0 + eta * (c1 + eta * (c2 + eta * c3));
        if (fabs(fv) >= fabs(fprev)) break;
        fprev = fv;
        double df = c1 + eta * (2.0 * c2 + eta * 3.0 * c3);
        double nx = eta - fv / df;
        if (!(nx >= 0.0)) { eta = 0.0; break; }
        if (fabs(nx - eta) <= 1e-14 * fabs(nx)) { eta = nx; break; }
        eta = nx;
    }
    double k1[3] = {varz - 4.0 * Mz * eta, Mxz, Myz};
    double k2[3] = {Mxz, Mxx - eta, Mxy};
    double k3[3] = {Myz, Mxy, Myy - eta};
    double bA = 0, bB = 0, bC = 0, bn = -1.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double *a = c == 0 ? k2 : c == 1 ? k3 : k1;
        const double *b = c == 0 ? k3 : c == 1 ? k1 : k2;
        double v0 = a[1] * b[2] - a[2] * b[1], v1 = a[2] * b[0] - a[0] * b[2], v2 = a[0] * b[1] - a[1] * b[0];
        double nn = v0 * v0 + v1 * v1 + v2 * v2;
        if (nn > bn) { bn = nn; bA = v0; bB = v1; bC = v2; }
    }
    double A = bA, B = bB, C = bC, D = -A * Mz;
    const double iS = 1.0 / sqrt(B * B + C * C - 4.0 * A * D);
    A *= iS; D *= iS;
    double Br = (ca * B - sa * C) * iS, Cr = (sa * B + ca * C) * iS;
    f.xm = xm; f.ym = ym; f.A = A; f.B = Br; f.C = Cr; f.D = D;
    f.R = A != 0.0 ? 0.5 / fabs(A) : __builtin_huge_val();
    double chi2 = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double d = circle_distance(A, Br, Cr, D, x[i] - xm, y[i] - ym) * isig[i];
        chi2 += d * d;
    }
    f.chi2_rphi = chi2;
}

// Both fits of a quintuplet from its five anchors (x, y, z) and endcap flags.
__device__ inline void t5_fit(const CutParams &p, const double *x, const double *y, const double *z,
                              const bool *endc, Fit5 &f) {
    double isg[5], r[5], s[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) { isg[i] = endc[i] ? p.isr_d : p.isrphi_d; r[i] = sqrt(x[i] * x[i] + y[i] * y[i]); }
    circle_fit5(x, y, isg, f);
    double cf = fabs(f.A);
#pragma unroll
    for (int i = 0; i < 5; ++i) s[i] = arc_len_d(cf, r[i]);
    if (!(s[4] > s[0])) { f.t = __builtin_nan(""); f.z0 = __builtin_nan(""); f.chi2_rz = __builtin_huge_val(); return; }
    double kAE = fabs((z[4] - z[0]) / (s[4] - s[0]));
    // endcap points: sigma_r times the r-z slope (floored at 0.1); barrel: sigma_z
    const double ike = p.isr_d / (kAE > 0.1 ? kAE : 0.1);
    double wz[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) { const double iv = endc[i] ? ike : p.isz_d; wz[i] = iv * iv; }
    double Wt = 0, sm = 0, zm = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) { Wt += wz[i]; sm += wz[i] * s[i]; zm += wz[i] * z[i]; }
    const double iWt = 1.0 / Wt;
    sm *= iWt; zm *= iWt;
    double Sss = 0, Ssz = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        Sss += wz[i] * (s[i] - sm) * (s[i] - sm); Ssz += wz[i] * (s[i] - sm) * (z[i] - zm);
    }
    if (!(Sss > 0)) { f.t = __builtin_nan(""); f.z0 = __builtin_nan(""); f.chi2_rz = __builtin_huge_val(); return; }
    double t = Ssz / Sss, z0 = zm - t * sm, chi2 = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) { double d = z[i] - z0 - t * s[i]; chi2 += d * d * wz[i]; }
    f.t = t; f.z0 = z0; f.chi2_rz = chi2;
}

// FP32 estimate of a quintuplet's r-z chi2 from its anchors (x, y, z, transverse
// radius r): the steps of circle_fit5 and t5_fit in single precision (moments
// in the chord frame, Taubin root by Newton from 0, arc lengths at the fitted
// curvature, weighted line fit).
// NaN when a step degenerates (zero chord, non-increasing arc length, no
// spread in s), where the FP64 fit decides alone.
__device__ inline float t5_chi2rz_f32(const CutParams &p, const float *x, const float *y, const float *z,
                                      const float *r, const bool *endc) {
    const float isrphi = 1.0f / p.srphi, isr = 1.0f / p.sr, isz = 1.0f / p.sz;
    float w[5], W = 0.0f, xm = 0.0f, ym = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const float is = endc[i] ? isr : isrphi;
        w[i] = is * is; W += w[i]; xm += w[i] * x[i]; ym += w[i] * y[i];
    }
    const float iW = 1.0f / W;
    xm *= iW; ym *= iW;
    const float cx = x[4] - x[0], cy = y[4] - y[0], cl = sqrtf(cx * cx + cy * cy);
    if (!(cl > 0.0f)) return __builtin_nanf("");
    const float ca = cx / cl, sa = cy / cl;
    float u[5], v[5], Mxx = 0.0f, Myy = 0.0f, Mxy = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const float wi = w[i] * iW, u0 = x[i] - xm, v0 = y[i] - ym;
        u[i] = ca * u0 + sa * v0; v[i] = -sa * u0 + ca * v0;
        Mxx += wi * u[i] * u[i]; Myy += wi * v[i] * v[i]; Mxy += wi * u[i] * v[i];
    }
    const float Mz = Mxx + Myy;
    float Mxz = 0.0f, Myz = 0.0f, varz = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const float wi = w[i] * iW, zt = u[i] * u[i] + v[i] * v[i] - Mz;
        Mxz += wi * u[i] * zt; Myz += wi * v[i] * zt; varz += wi * zt * zt;
    }
    const float cov = Mxx * Myy - Mxy * Mxy;
    const float c3 = 4.0f * Mz, c2 = -4.0f * Mz * Mz - varz;
    const float c1 = varz * Mz + 4.0f * cov * Mz - Mxz * Mxz - Myz * Myz;
    const float c0 = Mxz * (Mxz * Myy - Myz * Mxy) + Myz * (Myz * Mxx - Mxz * Mxy) - varz * cov;
    float eta = 0.0f, fprev = __builtin_huge_valf();
    for (int it = 0; it < 16; ++it) {
        const float fv = c0 + eta * (c1 + eta * (c2 + eta * c3));
        if (fabsf(fv) >= fabsf(fprev)) break;
        fprev = fv;
        const float df = c1 + eta * (2.0f * c2 + eta * 3.0f * c3);
        const float nx = eta - fv / df;
        if (!(nx >= 0.0f)) { eta = 0.0f; break; }
        if (fabsf(nx - eta) <= 1e-6f * fabsf(nx)) { eta = nx; break; }
        eta = nx;
    }
    const float k1[3] = {varz - 4.0f * Mz * eta, Mxz, Myz};
    const float k2[3] = {Mxz, Mxx - eta, Mxy};
    const float k3[3] = {Myz, Mxy, Myy - eta};
    float bA = 0.0f, bB = 0.0f, bC = 0.0f, bn = -1.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float *a = c == 0 ? k2 : c == 1 ? k3 : k1;
        const float *b = c == 0 ? k3 : c == 1 ? k1 : k2;
        const float v0 = a[1] * b[2] - a[2] * b[1], v1 = a[2] * b[0] - a[0] * b[2], v2 = a[0] * b[1] - a[1] * b[0];
        const float nn = v0 * v0 + v1 * v1 + v2 * v2;
        if (nn > bn) { bn = nn; bA = v0; bB = v1; bC = v2; }
    }
    const float cf = fabsf(bA) / sqrtf(bB * bB + bC * bC + 4.0f * bA * bA * Mz);
    float sv[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) sv[i] = arc_len_f(cf, r[i]);
    if (!(sv[4] > sv[0])) return __builtin_nanf("");
    const float kAE = fabsf((z[4] - z[0]) / (sv[4] - sv[0]));
    const float ike = isr / (kAE > 0.1f ? kAE : 0.1f);
    float wz[5], Wt = 0.0f, sm = 0.0f, zm = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const float iv = endc[i] ? ike : isz;
        wz[i] = iv * iv; Wt += wz[i]; sm += wz[i] * sv[i]; zm += wz[i] * z[i];
    }
    sm /= Wt; zm /= Wt;
    float Sss = 0.0f, Ssz = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) { Sss += wz[i] * (sv[i] - sm) * (sv[i] - sm); Ssz += wz[i] * (sv[i] - sm) * (z[i] - zm); }
    if (!(Sss > 0.0f)) return __builtin_nanf("");
    const float t = Ssz / Sss, z0 = zm - t * sm;
    float chi2 = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) { const float d = z[i] - z0 - t * sv[i]; chi2 += d * d * wz[i]; }
    return chi2;
}

// Circumradius |AB| |BC| |CA| / (2 |cross|), with one square root of the
// product of the squared sides.
__device__ __forceinline__ double circumradius_d(double ax, double ay, double bx, double by, double cx,
                                                 double cy) {
    double ab2 = (bx - ax) * (bx - ax) + (by - ay) * (by - ay);
    double bc2 = (cx - bx) * (cx - bx) + (cy - by) * (cy - by);
    double ca2 = (ax - cx) * (ax - cx) + (ay - cy) * (ay - cy);
    double cr = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
    return sqrt(ab2 * bc2 * ca2) / (2.0 * fabs(cr));
}

// Beam-line curvature |A x B| / (rA rB |B - A|), one square root.
__device__ __forceinline__ double beam_curv_d(double ax, double ay, double bx, double by) {
    double rA2 = ax * ax + ay * ay, rB2 = bx * bx + by * by;
    double dl2 = (bx - ax) * (bx - ax) + (by - ay) * (by - ay);
    return fabs(ax * by - ay * bx) / sqrt(rA2 * rB2 * dl2);
}

// log of v clamped to [1e-3, 1e6] (NaN -> 1e6), in FP32
__device__ __forceinline__ float clamp_logf(double vd) {
    float v = (float)vd;
    if (!(v >= 1e-3f)) v = (vd != vd) ? 1e6f : 1e-3f;
    if (v > 1e6f) v = 1e6f;
    return logf(v);
}

// The 42 DNN inputs (Sec. 2 list plus this project's additions), FP64 -> FP32,
// before standardisation.
// What the feature row needs from the fits, kept as FP32 by the fit stage:
// R, tan(lambda), z0, |d0| and the (unnormalised) direction at the point of
// closest approach, oriented toward the first anchor.
constexpr int kNFitOut = 6;
__device__ inline void t5_fit_outputs(const double *x, const double *y, const Fit5 &f, float *fo) {
    double u0 = -f.xm, v0 = -f.ym;
    double d0 = circle_distance(f.A, f.B, f.C, f.D, u0, v0);
    double gx = 2.0 * f.A * u0 + f.B, gy = 2.0 * f.A * v0 + f.C;
    double dx = -gy, dy = gx;
    if (x[0] * dx + y[0] * dy < 0) { dx = -dx; dy = -dy; }
    fo[0] = (float)f.R;
    fo[1] = (float)f.t;
    fo[2] = (float)f.z0;
    fo[3] = (float)fabs(d0);
    fo[4] = (float)dx;
    fo[5] = (float)dy;
}

// The seven features that come from the fits (indices 34, 35, 36, 38, 39, 40,
// 41 of the feature row), from the fit outputs and the two chi2 values.
constexpr int kNFitFeat = 7;
__device__ inline void t5_fit_features_from(const CutParams &p, const float *fo, double chi2_rphi,
                                            double chi2_rz, float *ff) {
    ff[0] = clamp_logf(p.kb_d * (double)fo[0]);
    ff[1] = asinhf(fo[1]);
    ff[2] = atan2f(fo[5], fo[4]);
    ff[3] = log1pf((float)chi2_rphi);
    ff[4] = log1pf((float)chi2_rz);
    ff[5] = fo[3];
    ff[6] = fo[2];
}

// The feature row from the anchors and the fit features above.
__device__ inline void t5_features_from(const CutParams &p, const double *x, const double *y, const double *z,
                                        const int *layer, const bool *endc, const float *ff, float *ft) {
    // per-anchor features in FP32 (the anchors are FP32 positions); the
    // three-point radii and curvatures below keep FP64 (near-collinear
    // triplets cancel badly in FP32)
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const float xf = (float)x[i], yf = (float)y[i], zf = (float)z[i];
        const float r = sqrtf(xf * xf + yf * yf);
        ft[6 * i + 0] = r;
        ft[6 * i + 1] = atan2f(yf, xf);
        ft[6 * i + 2] = zf;
        ft[6 * i + 3] = asinhf(zf / r);
        ft[6 * i + 4] = (float)layer[i];
        ft[6 * i + 5] = endc[i] ? 1.0f : 0.0f;
    }
    double cin = beam_curv_d(x[0], y[0], x[2], y[2]);
    double cou = beam_curv_d(x[2], y[2], x[4], y[4]);
    ft[30] = clamp_logf(p.kb_d / (2.0 * cin));
    ft[31] = clamp_logf(circumradius_d(x[0], y[0], x[1], y[1], x[2], y[2]));
    ft[32] = clamp_logf(p.kb_d / (2.0 * cou));
    ft[33] = clamp_logf(circumradius_d(x[2], y[2], x[3], y[3], x[4], y[4]));
    ft[34] = ff[0];
    ft[35] = ff[1];
    ft[36] = ff[2];
    ft[37] = clamp_logf(circumradius_d(x[1], y[1], x[2], y[2], x[3], y[3]));
    ft[38] = ff[3];
    ft[39] = ff[4];
    ft[40] = ff[5];
    ft[41] = ff[6];
}

__device__ inline void t5_features(const CutParams &p, const double *x, const double *y,
                                   const double *z, const int *layer, const bool *endc,
                                   const Fit5 &f, float *ft) {
    float fo[kNFitOut], ff[kNFitFeat];
    t5_fit_outputs(x, y, f, fo);
    t5_fit_features_from(p, fo, f.chi2_rphi, f.chi2_rz, ff);
    t5_features_from(p, x, y, z, layer, endc, ff, ft);
}

// T5-DNN forward pass, FP32 vector ALU (weights read with wave-uniform
// addresses, i.e. through the scalar cache).

__device__ inline float mlp_f32(const ModelDev &m, const float *x) {
    // weights read as uniform constants (scalar loads)
    float xs[kNFeat];
#pragma unroll
    for (int k = 0; k < kNFeat; ++k) xs[k] = (x[k] - ld_scalar(m.mu + k)) / ld_scalar(m.sd + k);
    float h1[kH1];
#pragma unroll 4
    for (int j = 0; j < kH1; ++j) {
        float a = ld_scalar(m.b1 + j);
#pragma unroll
        for (int k = 0; k < kNFeat; ++k) a = __builtin_fmaf(ld_scalar(m.W1 + j * kNFeat + k), xs[k], a);
        h1[j] = fmaxf(a, 0.0f);
    }
    float o = m.b3;
#pragma unroll 4
    for (int j = 0; j < kH2; ++j) {
        float a = ld_scalar(m.b2 + j);
#pragma unroll
        for (int k = 0; k < kH1; ++k) a = __builtin_fmaf(ld_scalar(m.W2 + j * kH1 + k), h1[k], a);
        o = __builtin_fmaf(ld_scalar(m.w3 + j), fmaxf(a, 0.0f), o);
    }
    return 1.0f / (1.0f + expf(-o));
}

}  // namespace lst
