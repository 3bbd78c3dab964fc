/* CPU driver of the oracle for the sanitizer test (built with
 * AddressSanitizer and UndefinedBehaviorSanitizer):
 *   oracle_fuzz build <geom> <model> <hits>      one build, prints the counts
 *   oracle_fuzz fuzz <geom> <model> <hits> <seed> <mutations>
 *       mutated geometry and model blobs (truncated, extended, bytes and
 *       header words changed) must load or be rejected without touching
 *       memory outside the blob; mutated blobs that load are used for a build
 *       of the event, and hits with out-of-range sensor ids must be rejected.
 * The hits file holds n, then x, y, z (float32) and sensor (int32) arrays. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc_geom orc_geom;
typedef struct orc_model orc_model;
typedef struct orc_result orc_result;
orc_geom *orc_geom_load(const void *blob, size_t nbytes);
void orc_geom_free(orc_geom *g);
orc_model *orc_model_load(const void *blob, size_t nbytes);
void orc_model_free(orc_model *m);
int orc_build(const orc_geom *g, const orc_model *mdl, const float *x, const float *y, const float *z,
              const int32_t *sensor, int64_t n, int mode, double score_min, orc_result **out);
int64_t orc_result_count(const orc_result *r, int stage);
void orc_result_free(orc_result *r);

static unsigned char *slurp(const char *path, size_t *n) {
    FILE *f = fopen(path, "rb");
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    long len = ftell(f);
    fseek(f, 0, SEEK_SET);
    unsigned char *b = (unsigned char *)malloc(len ? (size_t)len : 1);
    *n = fread(b, 1, (size_t)len, f);
    fclose(f);
    return b;
}

static uint64_t rng_state;
static uint64_t rnd(void) {   /* splitmix64 */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static unsigned char *mutate(const unsigned char *b, size_t n, size_t *out_n) {
    size_t m = n;
    const int op = (int)(rnd() % 4);
    if (op == 0) m = rnd() % (n + 1);
    else if (op == 1) m = n + 1 + rnd() % 64;
    unsigned char *c = (unsigned char *)malloc(m ? m : 1);
    memcpy(c, b, m < n ? m : n);
    for (size_t i = n; i < m; ++i) c[i] = (unsigned char)rnd();
    if (op == 2 && m) for (int k = 0; k < 1 + (int)(rnd() % 4); ++k) c[rnd() % m] = (unsigned char)rnd();
    if (op == 3 && m >= 24) {
        const uint32_t v = (rnd() % 2) ? (uint32_t)rnd() : (uint32_t)(rnd() % 64);
        memcpy(c + 4 * (1 + rnd() % 5), &v, 4);
    }
    *out_n = m;
    return c;
}

int main(int argc, char **argv) {
    if (argc < 5) return 2;
    size_t ng, nmd, nh;
    unsigned char *gb = slurp(argv[2], &ng), *mb = slurp(argv[3], &nmd), *hb = slurp(argv[4], &nh);
    if (!gb || !mb || !hb || nh < 8) return 2;
    int64_t n;
    memcpy(&n, hb, 8);
    if (nh != 8 + 16 * (size_t)n) return 2;
    const float *x = (const float *)(hb + 8), *y = x + n, *z = y + n;
    const int32_t *sensor = (const int32_t *)(z + n);
    orc_geom *g = orc_geom_load(gb, ng);
    orc_model *md = orc_model_load(mb, nmd);
    if (!g || !md) { fprintf(stderr, "valid blobs rejected\n"); return 1; }
    orc_result *r = NULL;
    if (orc_build(g, md, x, y, z, sensor, n, 0, 0.0 / 0.0, &r) != 0) { fprintf(stderr, "build failed\n"); return 1; }
    printf("counts %lld %lld %lld %lld\n", (long long)orc_result_count(r, 1), (long long)orc_result_count(r, 2),
           (long long)orc_result_count(r, 3), (long long)orc_result_count(r, 4));
    orc_result_free(r);
    if (strcmp(argv[1], "fuzz") == 0 && argc == 7) {
        rng_state = strtoull(argv[5], NULL, 10);
        const long iters = strtol(argv[6], NULL, 10);
        long acc = 0, rej = 0, built = 0;
        for (long it = 0; it < iters; ++it) {
            size_t m;
            unsigned char *c = mutate(gb, ng, &m);
            orc_geom *gg = orc_geom_load(c, m);
            free(c);
            if (gg) {
                ++acc;
                /* hits on sensors of this geometry only, so the build runs */
                orc_result *rr = NULL;
                if (orc_build(gg, md, x, y, z, sensor, n, 0, 0.0 / 0.0, &rr) == 0) { ++built; orc_result_free(rr); }
                orc_geom_free(gg);
            } else {
                ++rej;
            }
            c = mutate(mb, nmd, &m);
            orc_model *mm = orc_model_load(c, m);
            free(c);
            if (mm) orc_model_free(mm);
        }
        /* sensor ids outside the geometry are rejected */
        int32_t *bad = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
        memcpy(bad, sensor, sizeof(int32_t) * (size_t)n);
        if (n) bad[n / 2] = 1 << 30;
        orc_result *rb = NULL;
        const int st = orc_build(g, md, x, y, z, bad, n, 0, 0.0 / 0.0, &rb);
        free(bad);
        if (n && st == 0) { fprintf(stderr, "bad sensor id accepted\n"); return 1; }
        printf("fuzz: %ld geometry mutations, %ld loaded (%ld built), %ld rejected\n", iters, acc, built, rej);
    }
    orc_geom_free(g);
    orc_model_free(md);
    free(gb); free(mb); free(hb);
    return 0;
}
