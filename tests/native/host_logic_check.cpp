// Checks of the library's host-side planning (fc_host.hpp), built by the CPU
// tests with the address and undefined-behaviour sanitizers and run as a
// program: it exits with status 0 when every check holds, and prints the
// first failed check otherwise.
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <random>
#include <vector>

#include "fc_host.hpp"

using namespace fc;

static int failures = 0;
#define CHECK(cond)                                                  \
    do {                                                             \
        if (!(cond)) {                                               \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                              \
        }                                                            \
    } while (0)

static std::vector<int64_t> row_ptr_of(const std::vector<int64_t> &lens) {
    std::vector<int64_t> rp(lens.size() + 1, 0);
    for (size_t i = 0; i < lens.size(); ++i)
        rp[i + 1] = rp[i] + lens[i];
    return rp;
}

static void check_row_ptr_cases() {
    std::vector<int64_t> good = {0, 2, 2, 5, 9};
    int64_t bad = -1;
    CHECK(check_row_ptr(good.data(), 4, 9, &bad) == RP_OK);
    std::vector<int64_t> first = {1, 2, 2, 5, 9};
    CHECK(check_row_ptr(first.data(), 4, 9, &bad) == RP_FIRST);
    std::vector<int64_t> dec = {0, 3, 2, 5, 9};
    CHECK(check_row_ptr(dec.data(), 4, 9, &bad) == RP_DECREASING && bad == 1);
    std::vector<int64_t> last = {0, 2, 2, 5, 8};
    CHECK(check_row_ptr(last.data(), 4, 9, &bad) == RP_LAST && bad == 4);
    // a huge entry in the middle (it would send a row range past nnz)
    std::vector<int64_t> spike = {0, 2, 1000000000000ll, 5, 9};
    CHECK(check_row_ptr(spike.data(), 4, 9, &bad) == RP_DECREASING && bad == 2);
    std::vector<int64_t> neg = {0, -4, 2, 5, 9};
    CHECK(check_row_ptr(neg.data(), 4, 9, &bad) == RP_DECREASING && bad == 0);
    std::vector<int64_t> empty = {0};
    CHECK(check_row_ptr(empty.data(), 0, 0, &bad) == RP_OK);
}

// Every row longer than SPMM_LIGHT_MAX is in exactly one of the two lists, in
// row order, and the chunks of a heavy row cover its entries once, in order,
// each at most HEAVY_CHUNK long.
static void check_heavy_plan(const std::vector<int64_t> &lens) {
    const std::vector<int64_t> rp = row_ptr_of(lens);
    const int64_t n = (int64_t)lens.size();
    const HeavyRows p = plan_heavy_rows(rp.data(), n);
    size_t im = 0, ih = 0;
    CHECK(p.chunk_ptr.size() == p.rows.size() + 1);
    CHECK(p.chunk_row.size() == p.chunk_beg.size() && p.chunk_len.size() == p.chunk_beg.size());
    for (int64_t i = 0; i < n; ++i) {
        const int64_t len = lens[i];
        if (len <= SPMM_LIGHT_MAX)
            continue;
        if (len <= HEAVY_THR) {
            CHECK(im < p.med.size() && p.med[im] == i);
            ++im;
            continue;
        }
        CHECK(ih < p.rows.size() && p.rows[ih] == i);
        if (ih >= p.rows.size())
            return;
        int64_t next = rp[i];
        for (int32_t q = p.chunk_ptr[ih]; q < p.chunk_ptr[ih + 1]; ++q) {
            CHECK(p.chunk_row[q] == i);
            CHECK(p.chunk_beg[q] == next);
            CHECK(p.chunk_len[q] >= 1 && p.chunk_len[q] <= HEAVY_CHUNK);
            next += p.chunk_len[q];
        }
        CHECK(next == rp[i + 1]);
        ++ih;
    }
    CHECK(im == p.med.size() && ih == p.rows.size());
}

static void check_fused_grid() {
    for (int cus : {32, 38, 80, 256, 304}) {
        int64_t prev = 0;
        for (int64_t n : {1ll, 63ll, 64ll, 65ll, 1000ll, 262144ll, 262145ll, 1000000ll, 70000000ll,
                          2000000000ll}) {
            const int64_t g = fused_grid(n, cus);
            CHECK(g >= 1);
            CHECK(g <= (n + 63) / 64);                         // never an idle workgroup
            CHECK(g <= (int64_t)cus * 32);
            CHECK(g >= std::min<int64_t>((n + 63) / 64, (int64_t)cus * 2));
            CHECK(g >= prev);                                  // grows with n
            prev = g;
        }
    }
}

static void check_permutation_cases(std::mt19937_64 &rng) {
    int64_t bad = -1;
    CHECK(check_permutation(nullptr, 0, &bad) == PERM_OK);
    for (int trial = 0; trial < 20; ++trial) {
        const int64_t n = 1 + (int64_t)(rng() % 5000);
        std::vector<int32_t> perm(n);
        for (int64_t i = 0; i < n; ++i)
            perm[i] = (int32_t)i;
        std::shuffle(perm.begin(), perm.end(), rng);
        CHECK(check_permutation(perm.data(), n, &bad) == PERM_OK);
        if (n < 2)
            continue;
        const int64_t a = (int64_t)(rng() % n), b = (a + 1 + (int64_t)(rng() % (n - 1))) % n;
        const uint64_t h0 = order_fingerprint(perm.data(), n);
        std::swap(perm[a], perm[b]);
        CHECK(check_permutation(perm.data(), n, &bad) == PERM_OK);
        CHECK(order_fingerprint(perm.data(), n) != h0);     // the order, not the set
        std::swap(perm[a], perm[b]);
        CHECK(order_fingerprint(perm.data(), n) == h0);
        std::vector<int32_t> rep = perm;                   // a row twice, one missing
        rep[std::max(a, b)] = rep[std::min(a, b)];
        CHECK(check_permutation(rep.data(), n, &bad) == PERM_REPEAT && bad == std::max(a, b));
        std::vector<int32_t> out = perm;
        out[a] = (int32_t)n;
        CHECK(check_permutation(out.data(), n, &bad) == PERM_RANGE && bad == a);
        out[a] = -1;
        CHECK(check_permutation(out.data(), n, &bad) == PERM_RANGE && bad == a);
    }
    // FNV-1a's offset basis is the hash of no bytes
    CHECK(order_fingerprint(nullptr, 0) == 0xcbf29ce484222325ull);
    // one entry hashes its four little-endian bytes
    const int32_t one = 0x04030201;
    uint64_t h = 0xcbf29ce484222325ull;
    for (int b = 1; b <= 4; ++b) {
        h ^= (uint64_t)b;
        h *= 0x100000001b3ull;
    }
    CHECK(order_fingerprint(&one, 1) == h);
}

int main() {
    check_row_ptr_cases();
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 40; ++trial) {
        const int64_t n = 1 + (int64_t)(rng() % 3000);
        std::vector<int64_t> lens(n);
        for (auto &l : lens) {
            const uint64_t r = rng() % 100;
            l = r < 70 ? (int64_t)(rng() % 65) : r < 95 ? 65 + (int64_t)(rng() % 2000)
                                                        : 2040 + (int64_t)(rng() % 9000);
        }
        check_heavy_plan(lens);
    }
    check_heavy_plan({0, 64, 65, 2048, 2049, 3072, 3073, 0});
    check_fused_grid();
    check_permutation_cases(rng);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host logic: all checks passed\n");
    return 0;
}
