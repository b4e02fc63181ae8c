// Open-addressing hash sets of columns, the GPU form of the mark array of
// the marking trick (arXiv 1801.09809, Section 4): the row list of m_j is
// inserted once, and every probe m_i is one lookup.
//
// Every loop here is bounded by the table size, so a full table or a key
// inserted twice makes an insert report failure instead of spinning; the
// callers then search that root another way.  With distinct keys and at
// most half of the slots used (the sizes the kernels choose) no insert
// fails and every lookup ends at an empty slot after a few probes.
//
// The includer defines HWPM_HD (the function qualifiers: a device inline in
// the kernels, a plain inline in the host unit test) and passes the
// compare-and-swap to use on a slot (an LDS atomic in the kernels).
#pragma once

#include <stdint.h>

namespace hwpm {

// Fibonacci hash of a column into a power-of-two table.
HWPM_HD uint32_t hash_col(int32_t c, uint32_t mask) { return ((uint32_t)c * 0x9E3779B1u >> 12) & mask; }

// Table of int32 keys (empty = -1) with an int32 value per key, size
// mask + 1, linear probing.  Insert key c >= 0 with value x; returns false
// if no slot took it (the table is full, or c is already in it).
// cas(slot, expected, desired) returns the slot's previous key.
template <class Cas>
HWPM_HD bool hash_insert(int32_t* hk, int32_t* hv, int32_t c, int32_t x, uint32_t mask, Cas cas) {
    uint32_t h = hash_col(c, mask);
    for (uint32_t t = 0; t <= mask; ++t) {
        const int32_t prev = cas(hk + h, -1, c);
        if (prev == -1) {
            hv[h] = x;
            return true;
        }
        if (prev == c) return false;
        h = (h + 1) & mask;
    }
    return false;
}

// The value stored with key c, or -1.
HWPM_HD int32_t hash_find(const int32_t* hk, const int32_t* hv, int32_t c, uint32_t mask) {
    uint32_t h = hash_col(c, mask);
    for (uint32_t t = 0; t <= mask; ++t) {
        const int32_t key = hk[h];
        if (key == c) return hv[h];
        if (key == -1) return -1;
        h = (h + 1) & mask;
    }
    return -1;
}

}  // namespace hwpm
