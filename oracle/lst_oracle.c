/*
 * Line-segment-tracking object building: plain FP64 reference (the oracle).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline of the benchmark load this library. It shares no code, header or
 * table with the GPU library; it parses the geometry and model blobs itself.
 *
 * What it computes (paper Sec. 1, Table 1 steps 1-4; Sec. 2 for the T5-DNN),
 * written as the plain definition, without blocking or reordering:
 *
 *   MD = { (i, j) : i on the anchor sensor, j on the other sensor of the same
 *          module, every mini-doublet cut passes }                (step 1)
 *   LS = { (a, b) in MD x MD : module(b) in Map(module(a)), every line-segment
 *          cut passes }                                            (step 2)
 *   T3 = { (l1, l2) in LS x LS : outer MD of l1 == inner MD of l2, every
 *          triplet cut passes }                                    (step 3)
 *   T5 = { (t1, t2) in T3 x T3 : outer MD of t1 == inner MD of t2, every
 *          quintuplet cut passes }                                 (step 4)
 *   score(T5) = sigmoid(w3 . relu(W2 relu(W1 x + b1) + b2) + b3)   (Sec. 2)
 *
 * The paper states the structure but no cut formula; the cuts below are this
 * project's reading, derived from the helix of a track from the beam line
 * (half-curvature c = 1 / (2R), r(s) = sin(cs)/c, z linear in s). Every cut is
 * "pass iff v <= t" (equality passes, NaN fails) unless marked strict.
 *
 * Enumeration uses per-module and per-MD lists, which is exact because map
 * membership and MD sharing are themselves part of the definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- geometry */

enum { P_KB, P_PTMIN, P_ZLUM, P_NSIG, P_SRPHI, P_SZ, P_SR, P_GAP, P_CHI2RZ, P_CHI2RPHI,
       P_E2SLACK, P_LS3SLACK, P_NPARAM = 16 };

typedef struct {
    int32_t n_mod, n_barrel, n_map;
    double prm[P_NPARAM];
    int32_t *kind, *layer;
    double *p;               /* [n_mod][6] */
    uint32_t *map_off, *map_tgt;
} orc_geom;

static uint32_t rd_u32(const unsigned char *b) {
    return (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) | ((uint32_t)b[3] << 24);
}

void orc_geom_free(orc_geom *g) {
    if (!g) return;
    free(g->kind); free(g->layer); free(g->p); free(g->map_off); free(g->map_tgt); free(g);
}

orc_geom *orc_geom_load(const void *blob, size_t nbytes) {
    const unsigned char *b = (const unsigned char *)blob;
    if (nbytes < 152 || memcmp(b, "LSTG", 4) != 0 || rd_u32(b + 4) != 1) return NULL;
    uint32_t nm = rd_u32(b + 8), nb = rd_u32(b + 12), nmap = rd_u32(b + 16), npar = rd_u32(b + 20);
    if (npar != P_NPARAM) return NULL;
    size_t need = 152 + (size_t)nm * 64 + ((size_t)nm + 1) * 4 + (size_t)nmap * 4;
    if (nbytes != need) return NULL;
    orc_geom *g = (orc_geom *)calloc(1, sizeof(orc_geom));
    g->n_mod = (int32_t)nm; g->n_barrel = (int32_t)nb; g->n_map = (int32_t)nmap;
    memcpy(g->prm, b + 24, sizeof(double) * P_NPARAM);
    g->kind = (int32_t *)malloc(sizeof(int32_t) * nm);
    g->layer = (int32_t *)malloc(sizeof(int32_t) * nm);
    g->p = (double *)malloc(sizeof(double) * 6 * nm);
    const unsigned char *r = b + 152;
    for (uint32_t m = 0; m < nm; ++m, r += 64) {
        memcpy(&g->kind[m], r, 4);
        memcpy(&g->layer[m], r + 4, 4);
        memcpy(&g->p[6 * m], r + 16, 48);
    }
    g->map_off = (uint32_t *)malloc(sizeof(uint32_t) * (nm + 1));
    g->map_tgt = (uint32_t *)malloc(sizeof(uint32_t) * (nmap ? nmap : 1));
    memcpy(g->map_off, r, 4 * ((size_t)nm + 1));
    memcpy(g->map_tgt, r + 4 * ((size_t)nm + 1), 4 * (size_t)nmap);
    /* a map row per module, in order, and targets that are modules */
    int ok = g->map_off[0] == 0 && g->map_off[nm] == nmap && nm > 0 && nb <= nm;
    for (uint32_t m = 0; ok && m < nm; ++m) ok = g->map_off[m] <= g->map_off[m + 1];
    for (uint32_t i = 0; ok && i < nmap; ++i) ok = g->map_tgt[i] < nm;
    for (uint32_t m = 0; ok && m < nm; ++m) ok = g->kind[m] == 0 || g->kind[m] == 1;
    if (!ok) { orc_geom_free(g); return NULL; }
    return g;
}

/* ------------------------------------------------------------------- model */

typedef struct {
    int n_in, n_h1, n_h2;
    double *mu, *sd, *W1, *b1, *W2, *b2, *w3, b3;
} orc_model;

void orc_model_free(orc_model *m) {
    if (!m) return;
    free(m->mu); free(m->sd); free(m->W1); free(m->b1); free(m->W2); free(m->b2); free(m->w3);
    free(m);
}

static double *rd_f32_array(const unsigned char **pp, int n) {
    double *a = (double *)malloc(sizeof(double) * (size_t)n);
    for (int i = 0; i < n; ++i) { float f; memcpy(&f, *pp + 4 * i, 4); a[i] = (double)f; }
    *pp += 4 * (size_t)n;
    return a;
}

orc_model *orc_model_load(const void *blob, size_t nbytes) {
    const unsigned char *b = (const unsigned char *)blob;
    if (nbytes < 24 || memcmp(b, "LSTM", 4) != 0 || rd_u32(b + 4) != 1) return NULL;
    int ni = (int)rd_u32(b + 8), h1 = (int)rd_u32(b + 12), h2 = (int)rd_u32(b + 16);
    /* the forward pass keeps each layer in a 64-entry array */
    if (ni < 1 || ni > 64 || h1 < 1 || h1 > 64 || h2 < 1 || h2 > 64) return NULL;
    size_t nf = (size_t)2 * ni + (size_t)h1 * ni + h1 + (size_t)h2 * h1 + h2 + h2 + 1;
    if (nbytes != 24 + 4 * nf) return NULL;
    orc_model *m = (orc_model *)calloc(1, sizeof(orc_model));
    m->n_in = ni; m->n_h1 = h1; m->n_h2 = h2;
    const unsigned char *p = b + 24;
    m->mu = rd_f32_array(&p, ni); m->sd = rd_f32_array(&p, ni);
    m->W1 = rd_f32_array(&p, h1 * ni); m->b1 = rd_f32_array(&p, h1);
    m->W2 = rd_f32_array(&p, h2 * h1); m->b2 = rd_f32_array(&p, h2);
    m->w3 = rd_f32_array(&p, h2);
    double *b3 = rd_f32_array(&p, 1); m->b3 = b3[0]; free(b3);
    return m;
}

/* Sec. 2: two hidden layers (ReLU), sigmoid output; x is the transformed
 * feature vector before standardisation. */
double orc_mlp_one(const orc_model *m, const double *x) {
    double xs[64], h1[64], h2[64];
    for (int k = 0; k < m->n_in; ++k) xs[k] = (x[k] - m->mu[k]) / m->sd[k];
    for (int j = 0; j < m->n_h1; ++j) {
        double a = m->b1[j];
        for (int k = 0; k < m->n_in; ++k) a += m->W1[j * m->n_in + k] * xs[k];
        h1[j] = a > 0 ? a : 0;
    }
    for (int j = 0; j < m->n_h2; ++j) {
        double a = m->b2[j];
        for (int k = 0; k < m->n_h1; ++k) a += m->W2[j * m->n_h1 + k] * h1[k];
        h2[j] = a > 0 ? a : 0;
    }
    double o = m->b3;
    for (int k = 0; k < m->n_h2; ++k) o += m->w3[k] * h2[k];
    return 1.0 / (1.0 + exp(-o));
}

void orc_mlp(const orc_model *m, const float *X, int64_t n, double *out) {
    double x[64];
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < m->n_in; ++k) x[k] = (double)X[i * m->n_in + k];
        out[i] = orc_mlp_one(m, x);
    }
}

/* ----------------------------------------------------------------- helpers */

typedef struct { double x, y, z; int32_t module, which; } hit_t;

typedef struct { double v, t; int strict; } cutv;   /* pass iff v <= t (v < t if strict) */

static int cut_pass(cutv c) { return c.strict ? (c.v < c.t) : (c.v <= c.t); }

static double cmax_of(const orc_geom *g) { return g->prm[P_KB] / (2.0 * g->prm[P_PTMIN]); }

/* transverse arc length from the beam line to radius r at half-curvature c */
static double arc_len(double c, double r) {
    double x = c * r;
    if (x < 1e-4) return r * (1.0 + x * x / 6.0);
    if (x >= 1.0) x = 1.0;
    return asin(x) / c;
}

static double hypot2(double a, double b) { return sqrt(a * a + b * b); }

/* angle between two transverse position vectors */
static double opening_angle(const hit_t *a, const hit_t *b) {
    double cr = a->x * b->y - a->y * b->x;
    double dt = a->x * b->x + a->y * b->y;
    return fabs(atan2(cr, dt));
}

/* ----------------------------------------------------------- MD cuts (step 1) */

/* Barrel bend: the track from the beam line at |c| <= c_max turns by at most
 * asin(c_max r_up) - asin(c_max r_lo) between the sensors; plus resolution.
 * Barrel r-z: dz = (z_i - z_v) * rho(c), rho = (S(r_up) - S(r_lo)) / S(r_lo),
 * monotone in c, z_v in [-Z, Z]; window is the hull of the four corners.
 * Endcap bend: dphi = g asin(c r_i) / |z_i - z_v|; endcap radial step:
 * dr = g r_i f(c r_i) / |z_i - z_v|, f(x) = sqrt(1 - x^2) asin(x) / x. */
static int md_cuts(const orc_geom *g, const hit_t *hi, const hit_t *hj, cutv *out) {
    const double *pr = g->prm;
    const double cm = cmax_of(g), ns = pr[P_NSIG], Z = pr[P_ZLUM];
    const double *p = &g->p[6 * hi->module];
    if (g->kind[hi->module] == 0) {
        double rlo = p[0], rup = p[1];
        out[0].v = opening_angle(hi, hj);
        out[0].t = asin(cm * rup) - asin(cm * rlo)
                 + ns * pr[P_SRPHI] * sqrt(1.0 / (rlo * rlo) + 1.0 / (rup * rup));
        out[0].strict = 0;
        double rho0 = (rup - rlo) / rlo;
        double slo = arc_len(cm, rlo);
        double rho1 = (arc_len(cm, rup) - slo) / slo;
        double c4[4] = {(hi->z - Z) * rho0, (hi->z + Z) * rho0, (hi->z - Z) * rho1, (hi->z + Z) * rho1};
        double lo = c4[0], hiv = c4[0];
        for (int k = 1; k < 4; ++k) { if (c4[k] < lo) lo = c4[k]; if (c4[k] > hiv) hiv = c4[k]; }
        out[1].v = fabs((hj->z - hi->z) - 0.5 * (lo + hiv));
        out[1].t = 0.5 * (hiv - lo) + ns * sqrt(2.0) * pr[P_SZ];
        out[1].strict = 0;
    } else {
        double gap = fabs(p[1] - p[0]);
        double ri = hypot2(hi->x, hi->y), rj = hypot2(hj->x, hj->y);
        double az = fabs(hi->z);
        double xm = cm * ri; if (xm > 1.0) xm = 1.0;
        out[0].v = opening_angle(hi, hj);
        out[0].t = gap * asin(xm) / (az - Z)
                 + ns * (pr[P_SRPHI] * sqrt(1.0 / (ri * ri) + 1.0 / (rj * rj))
                         + gap * cm * pr[P_SR] / ((az - Z) * sqrt(1.0 - xm * xm)));
        out[0].strict = 0;
        double dr = ((hj->x - hi->x) * (hj->x + hi->x) + (hj->y - hi->y) * (hj->y + hi->y)) / (ri + rj);
        double f = (xm < 1e-8) ? 1.0 : sqrt(1.0 - xm * xm) * asin(xm) / xm;
        double lo = gap * ri * f / (az + Z), hiv = gap * ri / (az - Z);
        out[1].v = fabs(dr - 0.5 * (lo + hiv));
        out[1].t = 0.5 * (hiv - lo) + ns * sqrt(2.0) * pr[P_SR] + pr[P_E2SLACK];
        out[1].strict = 0;
    }
    return 2;
}

/* ------------------------------------------- anchor-pair cuts (LS, T3, T5) */

/* For anchors X (inner) and Y (outer):
 *   curvature of the beam-line circle through X and Y, c = |X x Y| / (rX rY |Y - X|),
 *     must not exceed c_max plus n_sigma of its resolution;
 *   with c' = min(c, c_max) and s = S_c'(r), the straight line in (s, z) through
 *     X and Y must point back to |z0| <= Z plus n_sigma of its resolution
 *     (ordering s_X < s_Y is required first). */
static void pair_cuts(const orc_geom *g, const hit_t *X, const hit_t *Y, double *c_out, cutv *out) {
    const double *pr = g->prm;
    const double cm = cmax_of(g), ns = pr[P_NSIG], Z = pr[P_ZLUM];
    int ex = g->kind[X->module] != 0, ey = g->kind[Y->module] != 0;
    double rX = hypot2(X->x, X->y), rY = hypot2(Y->x, Y->y);
    double dl = hypot2(Y->x - X->x, Y->y - X->y);
    double cr = X->x * Y->y - X->y * Y->x;
    double c = fabs(cr) / (rX * rY * dl);
    double srX = ex ? pr[P_SR] : 0.0, srY = ey ? pr[P_SR] : 0.0;
    double szX = ex ? 0.0 : pr[P_SZ], szY = ey ? 0.0 : pr[P_SZ];
    double sc = sqrt(pr[P_SRPHI] * pr[P_SRPHI] * (1.0 / (rX * rX) + 1.0 / (rY * rY))
                     + cm * cm * (srX * srX + srY * srY)) / dl;
    out[0].v = c; out[0].t = cm + ns * sc; out[0].strict = 0;
    double cp = c < cm ? c : cm;
    double sX = arc_len(cp, rX), sY = arc_len(cp, rY);
    out[1].v = sX; out[1].t = sY; out[1].strict = 1;
    double k = (Y->z - X->z) / (sY - sX);
    double z0 = X->z - sX * k;
    double var = ((sY * szX) * (sY * szX) + (sX * szY) * (sX * szY)
                  + k * k * ((sY * srX) * (sY * srX) + (sX * srY) * (sX * srY)))
                 / ((sY - sX) * (sY - sX));
    out[2].v = fabs(z0); out[2].t = Z + ns * sqrt(var); out[2].strict = 0;
    if (c_out) *c_out = c;
}

/* Mini-doublet direction: the chord between the MD hits must follow the
 * track direction at the chord midpoint M, which for the beam-line circle of
 * half-curvature c' makes the angle asin(c' |M|) with the radial direction,
 * turned toward the bending side sgn. */
static cutv md_direction_cut(const orc_geom *g, const hit_t *hi, const hit_t *hj, double cp, double sgn) {
    const double *pr = g->prm;
    double dx = hj->x - hi->x, dy = hj->y - hi->y;
    double mx = 0.5 * (hi->x + hj->x), my = 0.5 * (hi->y + hj->y);
    double m = hypot2(mx, my);
    double ux = mx / m, uy = my / m;
    double s = cp * m; if (s > 1.0) s = 1.0;
    double be = asin(s);
    double tx = cos(be) * ux - sgn * sin(be) * uy;
    double ty = cos(be) * uy + sgn * sin(be) * ux;
    cutv o;
    o.v = fabs(atan2(tx * dy - ty * dx, tx * dx + ty * dy));
    o.t = pr[P_NSIG] * sqrt(2.0) * pr[P_SRPHI] / hypot2(dx, dy) + pr[P_LS3SLACK];
    o.strict = 0;
    return o;
}

static double bend_sign(const hit_t *X, const hit_t *Y) {
    double cr = X->x * Y->y - X->y * Y->x;
    return cr < 0 ? -1.0 : 1.0;
}

/* LS (step 2): MDs a = (A, a'), b = (B, b'); anchors A, B. */
static int ls_cuts(const orc_geom *g, const hit_t *A, const hit_t *A2, const hit_t *B, const hit_t *B2,
                   cutv *out) {
    double c;
    int n = 0;
    int member = 0;
    for (uint32_t e = g->map_off[A->module]; e < g->map_off[A->module + 1]; ++e)
        if ((int32_t)g->map_tgt[e] == B->module) { member = 1; break; }
    out[n].v = member ? 0.0 : 1.0; out[n].t = 0.5; out[n].strict = 0; ++n;
    pair_cuts(g, A, B, &c, out + n); n += 3;
    double cm = cmax_of(g), cp = c < cm ? c : cm, sg = bend_sign(A, B);
    if (g->kind[A->module] == 0) out[n++] = md_direction_cut(g, A, A2, cp, sg);
    if (g->kind[B->module] == 0) out[n++] = md_direction_cut(g, B, B2, cp, sg);
    return n;
}

/* T3 (step 3): LS (MD_A, MD_B) + LS (MD_B, MD_C); anchors A, B, C. */
static int t3_cuts(const orc_geom *g, const hit_t *A, const hit_t *B, const hit_t *B2, const hit_t *C,
                   cutv *out) {
    double c;
    int n = 0;
    pair_cuts(g, A, C, &c, out); n += 3;
    double cm = cmax_of(g), cp = c < cm ? c : cm;
    if (g->kind[B->module] == 0) out[n++] = md_direction_cut(g, B, B2, cp, bend_sign(A, C));
    return n;
}

/* --------------------------------------------------- T5 fits (step 4, Sec. 2) */

typedef struct {
    /* circle in natural form A (u^2 + v^2) + B u + C v + D = 0 over coordinates
     * centred on (xm, ym), scaled so that B^2 + C^2 - 4AD = 1; A = 0 is a line */
    double xm, ym, A, B, C, D;
    double R;                 /* 1 / (2 |A|), +inf for a line */
    double chi2_rphi;
    double t, z0, chi2_rz;    /* r-z line z = z0 + t s */
} t5fit;

/* Signed geometric distance of centred point (u, v) from the normalised
 * natural-form circle; exact, and finite as A -> 0. */
static double circle_distance(double A, double B, double C, double D, double u, double v) {
    double P = A * (u * u + v * v) + B * u + C * v + D;
    return 2.0 * P / (1.0 + sqrt(1.0 + 4.0 * A * P));
}

/* Weighted algebraic circle fit of Taubin (1991): minimise
 *   sum w (A z + B u + C v + D)^2,  z = u^2 + v^2,
 * subject to the weighted mean squared gradient 4 A^2 mean(z) + B^2 + C^2 = 1.
 * On weight-centred data D = -A mean(z); the remaining 3x3 generalised
 * eigenproblem M p = eta N p is solved for its smallest root eta of the
 * characteristic cubic by Newton's method from eta = 0. Unlike the simpler
 * Kasa fit it is nearly unbiased on short arcs and reaches straight lines
 * continuously (A = 0). res: xm, ym, A, B, C, D (normalised), R, chi2. */
void orc_circle_fit(const double *x, const double *y, const double *sig, int n, double *res) {
    double W = 0, xm = 0, ym = 0;
    for (int i = 0; i < n; ++i) { double w = 1.0 / (sig[i] * sig[i]); W += w; xm += w * x[i]; ym += w * y[i]; }
    xm /= W; ym /= W;
    /* work in the frame of the chord from the first to the last point, which
     * keeps the moment products of short arcs well conditioned */
    double cx = x[n - 1] - x[0], cy = y[n - 1] - y[0], cl = hypot2(cx, cy);
    double ca = cl > 0 ? cx / cl : 1.0, sa = cl > 0 ? cy / cl : 0.0;
    double Mxx = 0, Myy = 0, Mxy = 0;
    for (int i = 0; i < n; ++i) {
        double w = 1.0 / (sig[i] * sig[i]) / W;
        double u0 = x[i] - xm, v0 = y[i] - ym;
        double u = ca * u0 + sa * v0, v = -sa * u0 + ca * v0;
        Mxx += w * u * u; Myy += w * v * v; Mxy += w * u * v;
    }
    double Mz = Mxx + Myy;
    double Mxz = 0, Myz = 0, varz = 0;
    for (int i = 0; i < n; ++i) {
        double w = 1.0 / (sig[i] * sig[i]) / W;
        double u0 = x[i] - xm, v0 = y[i] - ym;
        double u = ca * u0 + sa * v0, v = -sa * u0 + ca * v0;
        double zt = u * u + v * v - Mz;
        Mxz += w * u * zt; Myz += w * v * zt; varz += w * zt * zt;
    }
    double cov = Mxx * Myy - Mxy * Mxy;
    /* det(M - eta N) = c0 + c1 eta + c2 eta^2 + c3 eta^3 */
    double c3 = 4.0 * Mz;
    double c2 = -4.0 * Mz * Mz - varz;
    double c1 = varz * Mz + 4.0 * cov * Mz - Mxz * Mxz - Myz * Myz;
    double c0 = Mxz * (Mxz * Myy - Myz * Mxy) + Myz * (Myz * Mxx - Mxz * Mxy) - varz * cov;
    double eta = 0.0, fprev = INFINITY;
    for (int it = 0; it < 32; ++it) {
        double f = c0 + eta * (c1 + eta * (c2 + eta * c3));
        if (fabs(f) >= fabs(fprev)) break;          /* no further progress */
        fprev = f;
        double df = c1 + eta * (2.0 * c2 + eta * 3.0 * c3);
        double nx = eta - f / df;
        if (!(nx >= 0.0)) { eta = 0.0; break; }
        if (fabs(nx - eta) <= 1e-14 * fabs(nx)) { eta = nx; break; }
        eta = nx;
    }
    /* null vector (A, B, C) of K = M - eta N: the largest cross product of
     * two of its rows (K is singular at the eigenvalue); D = -A Mz */
    double k1[3] = {varz - 4.0 * Mz * eta, Mxz, Myz};
    double k2[3] = {Mxz, Mxx - eta, Mxy};
    double k3[3] = {Myz, Mxy, Myy - eta};
    const double *ra[3] = {k2, k3, k1}, *rb[3] = {k3, k1, k2};
    double best[3] = {0, 0, 0}, bn = -1.0;
    for (int c = 0; c < 3; ++c) {
        const double *a = ra[c], *b = rb[c];
        double v[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
        double nn = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        if (nn > bn) { bn = nn; best[0] = v[0]; best[1] = v[1]; best[2] = v[2]; }
    }
    double A = best[0], B = best[1], C = best[2];
    double D = -A * Mz;
    double S = sqrt(B * B + C * C - 4.0 * A * D);
    A /= S; D /= S;
    double Br = (ca * B - sa * C) / S, Cr = (sa * B + ca * C) / S;   /* back to x, y axes */
    B = Br; C = Cr;
    double chi2 = 0;
    for (int i = 0; i < n; ++i) {
        double d = circle_distance(A, B, C, D, x[i] - xm, y[i] - ym) / sig[i];
        chi2 += d * d;
    }
    res[0] = xm; res[1] = ym; res[2] = A; res[3] = B; res[4] = C; res[5] = D;
    res[6] = A != 0.0 ? 0.5 / fabs(A) : INFINITY;
    res[7] = chi2;
}

/* Weighted least-squares line z = z0 + t s (centred form); returns chi2. */
void orc_line_fit(const double *s, const double *z, const double *sig, int n, double *res) {
    double W = 0, sm = 0, zm = 0;
    for (int i = 0; i < n; ++i) { double w = 1.0 / (sig[i] * sig[i]); W += w; sm += w * s[i]; zm += w * z[i]; }
    sm /= W; zm /= W;
    double Sss = 0, Ssz = 0;
    for (int i = 0; i < n; ++i) {
        double w = 1.0 / (sig[i] * sig[i]);
        Sss += w * (s[i] - sm) * (s[i] - sm); Ssz += w * (s[i] - sm) * (z[i] - zm);
    }
    if (!(Sss > 0)) { res[0] = NAN; res[1] = NAN; res[2] = INFINITY; return; }
    double t = Ssz / Sss, z0 = zm - t * sm, chi2 = 0;
    for (int i = 0; i < n; ++i) {
        double d = z[i] - z0 - t * s[i];
        chi2 += d * d / (sig[i] * sig[i]);
    }
    res[0] = t; res[1] = z0; res[2] = chi2;
}

static void t5_fit(const orc_geom *g, const hit_t *const an[5], t5fit *f) {
    const double *pr = g->prm;
    double x[5], y[5], z[5], r[5], sg[5], s[5], res[8];
    for (int i = 0; i < 5; ++i) {
        x[i] = an[i]->x; y[i] = an[i]->y; z[i] = an[i]->z; r[i] = hypot2(x[i], y[i]);
        sg[i] = g->kind[an[i]->module] == 0 ? pr[P_SRPHI] : pr[P_SR];
    }
    orc_circle_fit(x, y, sg, 5, res);
    f->xm = res[0]; f->ym = res[1]; f->A = res[2]; f->B = res[3]; f->C = res[4]; f->D = res[5];
    f->R = res[6]; f->chi2_rphi = res[7];
    double cf = fabs(f->A);          /* half-curvature 1 / (2R) */
    for (int i = 0; i < 5; ++i) s[i] = arc_len(cf, r[i]);
    if (!(s[4] > s[0])) { f->t = NAN; f->z0 = NAN; f->chi2_rz = INFINITY; return; }
    double kAE = fabs((z[4] - z[0]) / (s[4] - s[0]));
    for (int i = 0; i < 5; ++i)
        sg[i] = g->kind[an[i]->module] == 0 ? pr[P_SZ] : pr[P_SR] * (kAE > 0.1 ? kAE : 0.1);
    orc_line_fit(s, z, sg, 5, res);
    f->t = res[0]; f->z0 = res[1]; f->chi2_rz = res[2];
}

static double circumradius(const hit_t *a, const hit_t *b, const hit_t *c) {
    double ab = hypot2(b->x - a->x, b->y - a->y), bc = hypot2(c->x - b->x, c->y - b->y);
    double ca = hypot2(a->x - c->x, a->y - c->y);
    double cr = (b->x - a->x) * (c->y - a->y) - (b->y - a->y) * (c->x - a->x);
    return ab * bc * ca / (2.0 * fabs(cr));
}

static double clamp_log(double v) {
    if (!(v >= 1e-3)) v = (v != v) ? 1e6 : 1e-3;   /* NaN -> upper clamp */
    if (v > 1e6) v = 1e6;
    return log(v);
}

/* 42 T5-DNN inputs (Sec. 2 lists the T3 pT and radius estimates, the anchor
 * coordinates, eta and layer, the T5 pT/eta/phi and the bridge-T3 radius;
 * this project adds is_endcap per anchor, both chi2 values, |d0| and z0). */
static void t5_features(const orc_geom *g, const hit_t *const an[5], const t5fit *f, double *ft) {
    const double kb = g->prm[P_KB];
    for (int i = 0; i < 5; ++i) {
        double r = hypot2(an[i]->x, an[i]->y);
        ft[6 * i + 0] = r;
        ft[6 * i + 1] = atan2(an[i]->y, an[i]->x);
        ft[6 * i + 2] = an[i]->z;
        ft[6 * i + 3] = asinh(an[i]->z / r);
        ft[6 * i + 4] = g->layer[an[i]->module];
        ft[6 * i + 5] = g->kind[an[i]->module] != 0;
    }
    double cin, cout_;
    cutv tmp[3];
    pair_cuts(g, an[0], an[2], &cin, tmp);
    pair_cuts(g, an[2], an[4], &cout_, tmp);
    ft[30] = clamp_log(kb / (2.0 * cin));
    ft[31] = clamp_log(circumradius(an[0], an[1], an[2]));
    ft[32] = clamp_log(kb / (2.0 * cout_));
    ft[33] = clamp_log(circumradius(an[2], an[3], an[4]));
    ft[34] = clamp_log(kb * f->R);
    ft[35] = asinh(f->t);
    /* closest approach to the beam line: signed distance of the origin from
     * the circle; the track direction there is perpendicular to the gradient
     * of the natural form at the origin, oriented toward the first anchor */
    double u0 = -f->xm, v0 = -f->ym;
    double d0 = circle_distance(f->A, f->B, f->C, f->D, u0, v0);
    double gx = 2.0 * f->A * u0 + f->B, gy = 2.0 * f->A * v0 + f->C;
    double dx = -gy, dy = gx;
    if (an[0]->x * dx + an[0]->y * dy < 0) { dx = -dx; dy = -dy; }
    ft[36] = atan2(dy, dx);
    ft[37] = clamp_log(circumradius(an[1], an[2], an[3]));
    ft[38] = log1p(f->chi2_rphi);
    ft[39] = log1p(f->chi2_rz);
    ft[40] = fabs(d0);
    ft[41] = f->z0;
}

/* T5 (step 4): anchors A..E (an[0..4]). Cuts: beam-line pair cuts on (A, E),
 * r-z line-fit chi2, and (pre-DNN mode only) the r-phi circle-fit chi2 which
 * the DNN replaces (Sec. 2). */
static int t5_cuts(const orc_geom *g, const orc_model *mdl, const hit_t *const an[5], int mode,
                   double score_min, cutv *out, t5fit *f, double *feat, double *score) {
    int n = 0;
    pair_cuts(g, an[0], an[4], NULL, out); n += 3;
    t5_fit(g, an, f);
    out[n].v = f->chi2_rz; out[n].t = g->prm[P_CHI2RZ]; out[n].strict = 0; ++n;
    if (mode == 1) { out[n].v = f->chi2_rphi; out[n].t = g->prm[P_CHI2RPHI]; out[n].strict = 0; ++n; }
    *score = NAN;
    int ok = 1;
    for (int k = 0; k < n; ++k) ok &= cut_pass(out[k]);
    if (feat && ok) t5_features(g, an, f, feat);
    if (mode == 0 && mdl && ok) {
        *score = orc_mlp_one(mdl, feat);
        if (score_min == score_min) {       /* pass iff score >= score_min */
            out[n].v = score_min; out[n].t = *score; out[n].strict = 0; ++n;
        }
    }
    return n;
}

/* ------------------------------------------------------------ build driver */

typedef struct { void *p; int64_t n, cap; size_t el; } vec;

static void *vpush(vec *v) {
    if (v->n == v->cap) {
        v->cap = v->cap ? 2 * v->cap : 1024;
        v->p = realloc(v->p, v->el * (size_t)v->cap);
    }
    return (char *)v->p + v->el * (size_t)(v->n++);
}

typedef struct {
    int64_t n_md, n_ls, n_t3, n_t5;
    int32_t *md;          /* [n_md][2] hit (anchor, other) */
    int32_t *ls;          /* [n_ls][2] md (inner, outer) */
    int32_t *t3;          /* [n_t3][2] ls (inner, outer) */
    int32_t *t5;          /* [n_t5][2] t3 (inner, outer) */
    double *chi2_rphi, *chi2_rz, *score;   /* [n_t5] */
    double *feat;         /* [n_t5][42] transformed features (before standardisation) */
} orc_result;

void orc_result_free(orc_result *r) {
    if (!r) return;
    free(r->md); free(r->ls); free(r->t3); free(r->t5);
    free(r->chi2_rphi); free(r->chi2_rz); free(r->score); free(r->feat);
    free(r);
}

static int all_pass(const cutv *c, int n) {
    for (int k = 0; k < n; ++k) if (!cut_pass(c[k])) return 0;
    return 1;
}

static hit_t *load_hits(const orc_geom *g, const float *x, const float *y, const float *z,
                        const int32_t *sensor, int64_t n) {
    hit_t *h = (hit_t *)malloc(sizeof(hit_t) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        if (sensor[i] < 0 || sensor[i] >= 2 * g->n_mod) { free(h); return NULL; }
        h[i].x = x[i]; h[i].y = y[i]; h[i].z = z[i];
        h[i].module = sensor[i] / 2; h[i].which = sensor[i] % 2;
    }
    return h;
}

/* mode: 0 DNN (score every T5), 1 PRE_DNN (chi2_rphi cut, no score).
 * Returns 0 on success, -1 bad input. */
int orc_build(const orc_geom *g, const orc_model *mdl, const float *x, const float *y, const float *z,
              const int32_t *sensor, int64_t n, int mode, double score_min, orc_result **out) {
    hit_t *h = load_hits(g, x, y, z, sensor, n);
    if (!h) return -1;
    const int32_t nm = g->n_mod, ns = 2 * nm;
    /* hits grouped by sensor, ascending input index */
    int64_t *soff = (int64_t *)calloc((size_t)ns + 1, sizeof(int64_t));
    int64_t *sidx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; ++i) soff[sensor[i] + 1]++;
    for (int s = 0; s < ns; ++s) soff[s + 1] += soff[s];
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)ns);
    memcpy(cur, soff, sizeof(int64_t) * (size_t)ns);
    for (int64_t i = 0; i < n; ++i) sidx[cur[sensor[i]]++] = i;
    free(cur);

    cutv cv[16];
    /* step 1: MD per module */
    vec md = {0, 0, 0, 2 * sizeof(int32_t)};
    int64_t *md_mod = (int64_t *)calloc((size_t)nm + 1, sizeof(int64_t));
    for (int32_t m = 0; m < nm; ++m) {
        md_mod[m] = md.n;
        for (int64_t a = soff[2 * m]; a < soff[2 * m + 1]; ++a)
            for (int64_t b = soff[2 * m + 1]; b < soff[2 * m + 2]; ++b) {
                int64_t i = sidx[a], j = sidx[b];
                int nc = md_cuts(g, &h[i], &h[j], cv);
                if (all_pass(cv, nc)) { int32_t *e = (int32_t *)vpush(&md); e[0] = (int32_t)i; e[1] = (int32_t)j; }
            }
    }
    md_mod[nm] = md.n;
    int32_t *MD = (int32_t *)md.p;

    /* step 2: LS per MD over the mapped modules */
    vec ls = {0, 0, 0, 2 * sizeof(int32_t)};
    int64_t *ls_start = (int64_t *)calloc((size_t)md.n + 1, sizeof(int64_t));
    for (int64_t a = 0; a < md.n; ++a) {
        ls_start[a] = ls.n;
        const hit_t *A = &h[MD[2 * a]], *A2 = &h[MD[2 * a + 1]];
        for (uint32_t e = g->map_off[A->module]; e < g->map_off[A->module + 1]; ++e) {
            int32_t mb = (int32_t)g->map_tgt[e];
            for (int64_t b = md_mod[mb]; b < md_mod[mb + 1]; ++b) {
                const hit_t *B = &h[MD[2 * b]], *B2 = &h[MD[2 * b + 1]];
                int nc = ls_cuts(g, A, A2, B, B2, cv);
                if (all_pass(cv, nc)) { int32_t *o = (int32_t *)vpush(&ls); o[0] = (int32_t)a; o[1] = (int32_t)b; }
            }
        }
    }
    ls_start[md.n] = ls.n;
    int32_t *LS = (int32_t *)ls.p;

    /* step 3: T3 = LS pairs chained at an MD */
    vec t3 = {0, 0, 0, 2 * sizeof(int32_t)};
    for (int64_t l1 = 0; l1 < ls.n; ++l1) {
        int32_t a = LS[2 * l1], b = LS[2 * l1 + 1];
        for (int64_t l2 = ls_start[b]; l2 < ls_start[b + 1]; ++l2) {
            int32_t c = LS[2 * l2 + 1];
            int nc = t3_cuts(g, &h[MD[2 * a]], &h[MD[2 * b]], &h[MD[2 * b + 1]], &h[MD[2 * c]], cv);
            if (all_pass(cv, nc)) { int32_t *o = (int32_t *)vpush(&t3); o[0] = (int32_t)l1; o[1] = (int32_t)l2; }
        }
    }
    int32_t *T3 = (int32_t *)t3.p;
    /* T3s are produced in inner-LS order, hence grouped by inner MD */
    int64_t *t3_start = (int64_t *)calloc((size_t)md.n + 1, sizeof(int64_t));
    for (int64_t k = 0; k < t3.n; ++k) t3_start[LS[2 * T3[2 * k]] + 1]++;
    for (int64_t a = 0; a < md.n; ++a) t3_start[a + 1] += t3_start[a];

    /* step 4: T5 = T3 pairs chained at an MD, fits, features, score */
    vec t5 = {0, 0, 0, 2 * sizeof(int32_t)};
    vec vr = {0, 0, 0, sizeof(double)}, vz = {0, 0, 0, sizeof(double)}, vs = {0, 0, 0, sizeof(double)};
    vec vf = {0, 0, 0, 42 * sizeof(double)};
    double feat[42];
    for (int64_t k1 = 0; k1 < t3.n; ++k1) {
        int32_t A = LS[2 * T3[2 * k1]], B = LS[2 * T3[2 * k1] + 1], C = LS[2 * T3[2 * k1 + 1] + 1];
        for (int64_t k2 = t3_start[C]; k2 < t3_start[C + 1]; ++k2) {
            int32_t D = LS[2 * T3[2 * k2] + 1], E = LS[2 * T3[2 * k2 + 1] + 1];
            const hit_t *an[5] = {&h[MD[2 * A]], &h[MD[2 * B]], &h[MD[2 * C]], &h[MD[2 * D]], &h[MD[2 * E]]};
            t5fit f; double score;
            int nc = t5_cuts(g, mdl, an, mode, score_min, cv, &f, feat, &score);
            if (all_pass(cv, nc)) {
                int32_t *o = (int32_t *)vpush(&t5); o[0] = (int32_t)k1; o[1] = (int32_t)k2;
                *(double *)vpush(&vr) = f.chi2_rphi;
                *(double *)vpush(&vz) = f.chi2_rz;
                *(double *)vpush(&vs) = score;
                memcpy(vpush(&vf), feat, sizeof(feat));
            }
        }
    }
    orc_result *r = (orc_result *)calloc(1, sizeof(orc_result));
    r->n_md = md.n; r->n_ls = ls.n; r->n_t3 = t3.n; r->n_t5 = t5.n;
    r->md = (int32_t *)md.p; r->ls = (int32_t *)ls.p; r->t3 = (int32_t *)t3.p; r->t5 = (int32_t *)t5.p;
    r->chi2_rphi = (double *)vr.p; r->chi2_rz = (double *)vz.p; r->score = (double *)vs.p;
    r->feat = (double *)vf.p;
    *out = r;
    free(h); free(soff); free(sidx); free(md_mod); free(ls_start); free(t3_start);
    return 0;
}

/* Cut values of one candidate, for classifying GPU/oracle disagreements.
 * stage 1: hits[0..1] = MD (anchor, other)
 * stage 2: hits[0..3] = MD_A, MD_B
 * stage 3: hits[0..5] = MD_A, MD_B, MD_C
 * stage 4: hits[0..9] = MD_A .. MD_E
 * Writes v[k], t[k], strict[k] for every cut of that stage (not of earlier
 * stages) and returns their number, or -1 on bad input. For stage 4 also
 * fills detail[0..6] = chi2_rphi, chi2_rz, R, t, z0, xc, yc, feat[42] and
 * score (NaN unless mode 0 with a model). */
static int cut_values_impl(const orc_geom *g, const orc_model *mdl, hit_t *H, int stage,
                           int mode, double score_min, double *v, double *t, int32_t *strict,
                           double *detail, double *feat_out, double *score_out);

int orc_cut_values(const orc_geom *g, const orc_model *mdl, const float *x, const float *y,
                   const float *z, const int32_t *sensor, int64_t n, int stage, const int64_t *hits,
                   int mode, double score_min, double *v, double *t, int32_t *strict,
                   double *detail, double *feat_out, double *score_out) {
    hit_t H[10];
    int nh = stage == 1 ? 2 : stage == 2 ? 4 : stage == 3 ? 6 : stage == 4 ? 10 : 0;
    if (!nh) return -1;
    for (int k = 0; k < nh; ++k) {
        int64_t i = hits[k];
        if (i < 0 || i >= n || sensor[i] < 0 || sensor[i] >= 2 * g->n_mod) return -1;
        H[k].x = x[i]; H[k].y = y[i]; H[k].z = z[i]; H[k].module = sensor[i] / 2; H[k].which = sensor[i] % 2;
    }
    return cut_values_impl(g, mdl, H, stage, mode, score_min, v, t, strict, detail, feat_out, score_out);
}

/* Same, with the candidate's hits given directly in FP64 (x, y, z, sensor per
 * hit, in candidate order); used to evaluate exact helix points. */
int orc_cut_values_d(const orc_geom *g, const orc_model *mdl, const double *x, const double *y,
                     const double *z, const int32_t *sensor, int stage, int mode, double score_min,
                     double *v, double *t, int32_t *strict, double *detail, double *feat_out,
                     double *score_out) {
    hit_t H[10];
    int nh = stage == 1 ? 2 : stage == 2 ? 4 : stage == 3 ? 6 : stage == 4 ? 10 : 0;
    if (!nh) return -1;
    for (int k = 0; k < nh; ++k) {
        if (sensor[k] < 0 || sensor[k] >= 2 * g->n_mod) return -1;
        H[k].x = x[k]; H[k].y = y[k]; H[k].z = z[k]; H[k].module = sensor[k] / 2; H[k].which = sensor[k] % 2;
    }
    return cut_values_impl(g, mdl, H, stage, mode, score_min, v, t, strict, detail, feat_out, score_out);
}

static int cut_values_impl(const orc_geom *g, const orc_model *mdl, hit_t *H, int stage,
                           int mode, double score_min, double *v, double *t, int32_t *strict,
                           double *detail, double *feat_out, double *score_out) {
    cutv cv[16];
    int nc = 0;
    if (stage == 1) {
        if (H[0].module != H[1].module || H[0].which != 0 || H[1].which != 1) return -1;
        nc = md_cuts(g, &H[0], &H[1], cv);
    } else if (stage == 2) {
        nc = ls_cuts(g, &H[0], &H[1], &H[2], &H[3], cv);
    } else if (stage == 3) {
        nc = t3_cuts(g, &H[0], &H[2], &H[3], &H[4], cv);
    } else {
        const hit_t *an[5] = {&H[0], &H[2], &H[4], &H[6], &H[8]};
        t5fit f; double score; double feat[42];
        nc = t5_cuts(g, mdl, an, mode, score_min, cv, &f, feat, &score);
        if (detail) {
            detail[0] = f.chi2_rphi; detail[1] = f.chi2_rz; detail[2] = f.R; detail[3] = f.t;
            detail[4] = f.z0; detail[5] = f.xm - 0.5 * f.B / f.A; detail[6] = f.ym - 0.5 * f.C / f.A;
        }
        if (feat_out) { t5_features(g, an, &f, feat); memcpy(feat_out, feat, sizeof(feat)); }
        if (score_out) {
            if (mdl && feat_out) *score_out = orc_mlp_one(mdl, feat_out);
            else *score_out = score;
        }
    }
    for (int k = 0; k < nc; ++k) { v[k] = cv[k].v; t[k] = cv[k].t; strict[k] = cv[k].strict; }
    return nc;
}

/* accessors for ctypes */
int64_t orc_result_count(const orc_result *r, int stage) {
    return stage == 1 ? r->n_md : stage == 2 ? r->n_ls : stage == 3 ? r->n_t3 : stage == 4 ? r->n_t5 : -1;
}

void orc_result_copy(const orc_result *r, int32_t *md, int32_t *ls, int32_t *t3, int32_t *t5,
                     double *chi2_rphi, double *chi2_rz, double *score, double *feat) {
    if (md) memcpy(md, r->md, sizeof(int32_t) * 2 * (size_t)r->n_md);
    if (ls) memcpy(ls, r->ls, sizeof(int32_t) * 2 * (size_t)r->n_ls);
    if (t3) memcpy(t3, r->t3, sizeof(int32_t) * 2 * (size_t)r->n_t3);
    if (t5) memcpy(t5, r->t5, sizeof(int32_t) * 2 * (size_t)r->n_t5);
    if (chi2_rphi) memcpy(chi2_rphi, r->chi2_rphi, sizeof(double) * (size_t)r->n_t5);
    if (chi2_rz) memcpy(chi2_rz, r->chi2_rz, sizeof(double) * (size_t)r->n_t5);
    if (score) memcpy(score, r->score, sizeof(double) * (size_t)r->n_t5);
    if (feat) memcpy(feat, r->feat, sizeof(double) * 42 * (size_t)r->n_t5);
}
