// Host build of the LDS hash sets of hwpm_hash.h (the kernels compile the
// same header with device qualifiers and an LDS compare-and-swap).  Checks
// that every loop ends on full, near-full and duplicate-key tables and that
// lookups return exactly what was inserted.  Prints "ok" and exits 0, or
// names the failed check and exits 1.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <set>
#include <vector>

#define HWPM_HD inline
#include "hwpm_hash.h"

using namespace hwpm;

static int fails = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond); \
            ++fails;                                                  \
        }                                                             \
    } while (0)

struct Cas32 {
    int32_t operator()(int32_t* p, int32_t e, int32_t d) const {
        const int32_t old = *p;
        if (old == e) *p = d;
        return old;
    }
};
static void test_plain(uint32_t size, uint32_t fill, uint32_t seed) {
    const uint32_t mask = size - 1;
    std::vector<int32_t> hk(size, -1), hv(size, 0);
    std::mt19937 rng(seed);
    std::set<int32_t> keys;
    while (keys.size() < fill) keys.insert((int32_t)(rng() & 0x7fffffff));
    int32_t x = 0;
    for (int32_t c : keys) CHECK(hash_insert(hk.data(), hv.data(), c, x++, mask, Cas32{}));
    x = 0;
    for (int32_t c : keys) CHECK(hash_find(hk.data(), hv.data(), c, mask) == x++);
    // absent keys end at an empty slot, or after size probes in a full table
    for (int t = 0; t < 1000; ++t) {
        const int32_t c = (int32_t)(rng() & 0x7fffffff);
        if (!keys.count(c)) CHECK(hash_find(hk.data(), hv.data(), c, mask) == -1);
    }
    // a key already present is refused and keeps its value
    if (!keys.empty()) {
        const int32_t c = *keys.begin();
        CHECK(!hash_insert(hk.data(), hv.data(), c, 12345, mask, Cas32{}));
        CHECK(hash_find(hk.data(), hv.data(), c, mask) == 0);
    }
    // a full table refuses a new key
    if (fill == size) {
        int32_t c = 0;
        while (keys.count(c)) ++c;
        CHECK(!hash_insert(hk.data(), hv.data(), c, 7, mask, Cas32{}));
        CHECK(hash_find(hk.data(), hv.data(), c, mask) == -1);
    }
}

int main() {
    // half full (the kernels' bound), near full, full, and empty tables
    for (uint32_t seed = 0; seed < 4; ++seed) {
        test_plain(64, 32, seed);
        test_plain(1024, 512, seed);
        test_plain(4096, 2048, seed);
        test_plain(64, 63, seed);
        test_plain(256, 256, seed);
        test_plain(256, 0, seed);
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("ok\n");
    return 0;
}
