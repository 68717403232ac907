// fc_host.hpp -- host-side planning of the fuzzy-clustering solver, in plain
// C++17 with no HIP dependency: the structural check of a CSR row-pointer
// array, the check and fingerprint of a caller-given article order, the plan
// of the sparse product's long rows, and the launch-grid rule of the fused
// kernel that single solves and served instances share.  The
// library includes it; the CPU tests compile it alone, under the address and
// undefined-behaviour sanitizers.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace fc {

// Row classes of the sparse product: rows of at most SPMM_LIGHT_MAX stored
// nonzeros are summed by small teams of lanes, rows of up to HEAVY_THR by a
// whole wave (the medium-row list), longer rows in chunks of HEAVY_CHUNK
// nonzeros whose sums are combined per row in chunk order.
constexpr int SPMM_LIGHT_MAX = 64;
constexpr int64_t HEAVY_THR = 2048;
constexpr int64_t HEAVY_CHUNK = 1024;

// Structural check of a CSR row-pointer array of n rows holding nnz stored
// entries: it must start at 0, never decrease and end at nnz.  Returns
// RP_OK, or the first violation found (and its row in *bad_row when given).
enum { RP_OK = 0, RP_FIRST = 1, RP_DECREASING = 2, RP_LAST = 3 };
inline int check_row_ptr(const int64_t *rp, int64_t n, int64_t nnz, int64_t *bad_row) {
    if (bad_row)
        *bad_row = 0;
    if (rp[0] != 0)
        return RP_FIRST;
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) {
            if (bad_row)
                *bad_row = i;
            return RP_DECREASING;
        }
    if (rp[n] != nnz) {
        if (bad_row)
            *bad_row = n;
        return RP_LAST;
    }
    return RP_OK;
}

// Check of a caller-given article order: perm[i] is the caller's row placed
// at internal row i, so perm must hold every row of 0..n-1 exactly once.
// Returns PERM_OK, or the first violation in index order: PERM_RANGE (an entry
// outside 0..n-1) or PERM_REPEAT (an entry seen before), with its index i in
// *bad_index when given.
enum { PERM_OK = 0, PERM_RANGE = 1, PERM_REPEAT = 2 };
inline int check_permutation(const int32_t *perm, int64_t n, int64_t *bad_index) {
    if (bad_index)
        *bad_index = 0;
    std::vector<uint8_t> seen((size_t)std::max<int64_t>(n, 0), 0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t p = perm[i];
        if (p < 0 || p >= n || seen[(size_t)p]) {
            if (bad_index)
                *bad_index = i;
            return p < 0 || p >= n ? PERM_RANGE : PERM_REPEAT;
        }
        seen[(size_t)p] = 1;
    }
    return PERM_OK;
}

// 64-bit FNV-1a hash of an order's bytes (entries little-endian, in index
// order): a checkpoint records it, so a state is resumed only under the order
// it was taken with.
inline uint64_t order_fingerprint(const int32_t *perm, int64_t n) {
    uint64_t h = 0xcbf29ce484222325ull;   // FNV offset basis
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t v = (uint32_t)perm[i];
        for (int b = 0; b < 4; ++b) {
            h ^= (v >> (8 * b)) & 0xffu;
            h *= 0x100000001b3ull;            // FNV prime
        }
    }
    return h;
}

// The plan of the rows longer than SPMM_LIGHT_MAX, in row order: medium rows
// are listed; heavy rows are cut into chunks, chunk_ptr[h] .. chunk_ptr[h+1]-1
// being the chunks of heavy row rows[h].  Expects a checked row_ptr.
struct HeavyRows {
    std::vector<int32_t> med;
    std::vector<int32_t> rows, chunk_ptr, chunk_row, chunk_len;
    std::vector<int64_t> chunk_beg;
};

inline HeavyRows plan_heavy_rows(const int64_t *rp, int64_t n) {
    HeavyRows p;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t len = rp[i + 1] - rp[i];
        if (len <= SPMM_LIGHT_MAX)
            continue;
        if (len <= HEAVY_THR) {
            p.med.push_back((int32_t)i);
            continue;
        }
        p.rows.push_back((int32_t)i);
        p.chunk_ptr.push_back((int32_t)p.chunk_beg.size());
        for (int64_t b = rp[i]; b < rp[i + 1]; b += HEAVY_CHUNK) {
            const int64_t l = std::min<int64_t>(rp[i + 1] - b, HEAVY_CHUNK);
            p.chunk_row.push_back((int32_t)i);
            p.chunk_beg.push_back(b);
            p.chunk_len.push_back((int32_t)l);
        }
    }
    p.chunk_ptr.push_back((int32_t)p.chunk_beg.size());
    return p;
}

// Workgroups of the fused kernel for an instance of n rows on a device with
// `cus` compute units: one 64-row tile per workgroup up to two workgroups per
// CU; larger instances up to 32 per CU while each workgroup keeps at least
// eight tiles (n = 7e7, c = 32: 8.6 ms for the fused pass and 0.13 ms for
// reducing its partials, against 8.9 and 0.05 ms at 12 per CU).  The count
// fixes how the instance's partial sums are grouped, so single solves and
// served instances use this same rule: a served request then sums exactly as
// it does alone.
inline int64_t fused_grid(int64_t n, int cus) {
    const int64_t cap = std::min<int64_t>((int64_t)cus * 32, std::max<int64_t>((int64_t)cus * 2, n / 512));
    const int64_t tiles = (n + 63) / 64;
    return std::max<int64_t>(1, std::min<int64_t>(tiles, cap));
}

}  // namespace fc
