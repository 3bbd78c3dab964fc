// CPU driver of the library's blob parsers for the sanitizer test: parses a
// valid blob, then many mutated copies of it (truncated, extended, single
// bytes changed, header counts and map entries overwritten), and checks that
// every call either succeeds or reports an error, without touching memory
// outside the blob (the test builds this file with AddressSanitizer and
// UndefinedBehaviorSanitizer).
//
//   blob_fuzz <geom|model|gnn> <blob file> <seed> <mutations>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <random>
#include <string>
#include <vector>

#include "lst_host.h"

using namespace lst;

static bool parse(const std::string &kind, const std::vector<unsigned char> &b, std::string &err) {
    // the parser gets a buffer of exactly the blob's length, so that any read
    // past its end is caught
    unsigned char *p = (unsigned char *)malloc(b.size() ? b.size() : 1);
    if (!b.empty()) memcpy(p, b.data(), b.size());
    bool ok = false;
    if (kind == "geom") {
        GeomHost g;
        ok = parse_geometry(p, b.size(), g, err);
        if (ok && (g.map_off.size() != (size_t)g.n_mod + 1 || g.run_off.back() > (int32_t)g.runs.size())) {
            fprintf(stderr, "inconsistent tables\n");
            exit(3);
        }
    } else if (kind == "model") {
        ModelHost m;
        ok = parse_model(p, b.size(), m, err);
    } else {
        GnnHost g;
        ok = parse_gnn(p, b.size(), g, err);
    }
    free(p);
    return ok;
}

int main(int argc, char **argv) {
    if (argc != 5) {
        fprintf(stderr, "usage: blob_fuzz <geom|model|gnn> <blob> <seed> <mutations>\n");
        return 2;
    }
    const std::string kind = argv[1];
    FILE *f = fopen(argv[2], "rb");
    if (!f) return 2;
    std::vector<unsigned char> blob;
    unsigned char buf[65536];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) blob.insert(blob.end(), buf, buf + n);
    fclose(f);
    std::string err;
    if (!parse(kind, blob, err)) {
        fprintf(stderr, "valid blob rejected: %s\n", err.c_str());
        return 1;
    }
    std::mt19937_64 rng(strtoull(argv[3], nullptr, 10));
    const long iters = strtol(argv[4], nullptr, 10);
    long accepted = 0, rejected = 0;
    // geometry blobs: the module-map offsets follow the 64-byte module records
    uint32_t nm = 0;
    if (kind == "geom" && blob.size() >= 12) memcpy(&nm, &blob[8], 4);
    const size_t off0 = 152 + 64 * (size_t)nm;
    for (long it = 0; it < iters; ++it) {
        std::vector<unsigned char> b = blob;
        const int op = (int)(rng() % (kind == "geom" ? 7 : 6));
        if (op == 0) {                       // truncate
            b.resize(rng() % (b.size() + 1));
        } else if (op == 1) {                // extend
            b.resize(b.size() + 1 + rng() % 64, (unsigned char)rng());
        } else if (op == 2) {                // change a few bytes anywhere
            for (int k = 0; k < 1 + (int)(rng() % 4); ++k) b[rng() % b.size()] = (unsigned char)rng();
        } else if (op == 3) {                // overwrite a header word (counts, version)
            const size_t w = 4 * (1 + rng() % 5);
            const uint32_t v = (rng() % 2) ? (uint32_t)rng() : (uint32_t)(rng() % 64);
            if (w + 4 <= b.size()) memcpy(&b[w], &v, 4);
        } else if (op == 4) {                // overwrite a word in the last quarter (map offsets and targets)
            const size_t lo = b.size() * 3 / 4 / 4 * 4;
            const size_t w = lo + 4 * (rng() % ((b.size() - lo) / 4 ? (b.size() - lo) / 4 : 1));
            const uint32_t v = (uint32_t)rng();
            if (w + 4 <= b.size()) memcpy(&b[w], &v, 4);
        } else if (op == 6) {                // overwrite a map offset (often the first), small or huge
            const size_t k = (rng() % 4 == 0) ? 0 : rng() % ((size_t)nm + 1);
            const uint32_t v = (rng() % 2) ? (uint32_t)rng() : (uint32_t)-(int32_t)(1 + rng() % 64);
            if (off0 + 4 * k + 4 <= b.size()) memcpy(&b[off0 + 4 * k], &v, 4);
        } else {                             // overwrite a double anywhere with a special value
            const double sp[] = {0.0, -1.0, 1e300, -1e300, 0.0 / 0.0, 1.0 / 0.0};
            const size_t w = 8 * (rng() % (b.size() / 8 ? b.size() / 8 : 1));
            if (w + 8 <= b.size()) memcpy(&b[w], &sp[rng() % 6], 8);
        }
        if (parse(kind, b, err)) ++accepted;
        else ++rejected;
    }
    printf("%s: %ld mutations, %ld accepted, %ld rejected\n", kind.c_str(), iters, accepted, rejected);
    return 0;
}
