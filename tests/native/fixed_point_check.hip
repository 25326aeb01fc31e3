// Host-side check of the library's exact fixed-point helpers against
// unsigned __int128 arithmetic: U = ceil(C * 2^64 / W) for 0 <= C < W, the
// Moller-Granlund reciprocal (over the whole normalised range), and the partial-sum recovery floor(U W / 2^64) = C.
#include <stdio.h>
#include <stdlib.h>

#include "../../paper_1901_05423_amd/csrc/rtf_internal.h"

typedef unsigned __int128 u128;

static uint64_t state = 0x243F6A8885A308D3ull;
static uint64_t next64() {  // splitmix64
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int check_reciprocal(uint64_t d) {
    const uint64_t v = rtf::reciprocal_2by1(d);
    const u128 vref = (~(u128)0) / d - ((u128)1 << 64);
    if ((u128)v != vref) {
        printf("reciprocal mismatch d=%llx\n", (unsigned long long)d);
        return 1;
    }
    return 0;
}

static int check(uint64_t C, uint64_t W) {
    const uint32_t s = (uint32_t)rtf::clz64(W);
    const uint64_t d = W << s;
    const uint64_t v = rtf::reciprocal_2by1(d);
    const u128 vref = (~(u128)0) / d - ((u128)1 << 64);
    if ((u128)v != vref) {
        printf("reciprocal mismatch d=%llx\n", (unsigned long long)d);
        return 1;
    }
    const uint64_t U = rtf::fixed_point_key(C, d, v, s);
    const u128 ref = (((u128)C << 64) + (W - 1)) / W;
    if ((u128)U != ref) {
        printf("key mismatch C=%llu W=%llu\n", (unsigned long long)C, (unsigned long long)W);
        return 1;
    }
    if (rtf::mulhi64(U, W) != C) {
        printf("recovery mismatch C=%llu W=%llu\n", (unsigned long long)C, (unsigned long long)W);
        return 1;
    }
    return 0;
}

int main() {
    int bad = 0;
    const uint64_t special[] = {1, 2, 3, 7, 113, 1ull << 20, (1ull << 32) - 1, 1ull << 32,
                                (1ull << 62) + 1, (1ull << 63) - 1, 1000000007ull};
    for (uint64_t W : special) {
        const uint64_t cs[] = {0, 1, W / 2, W - 1, W / 3, (W - 1) / 7};
        for (uint64_t C : cs)
            if (C < W) bad += check(C, W);
    }
    // the reciprocal over the whole normalised range: both ends, values next
    // to powers of two and to the FP64 grid, and random full-width divisors
    const uint64_t top = 1ull << 63;
    for (uint64_t k = 0; k < 4096; ++k) {
        bad += check_reciprocal(top + k);
        bad += check_reciprocal(~0ull - k);
        bad += check_reciprocal(top + (k << 11));
        bad += check_reciprocal(top + (k << 11) - 1 + (k == 0));
        bad += check_reciprocal(top | (1ull << (k % 63)));
        bad += check_reciprocal(top | ((1ull << (k % 64)) - 1));
    }
    for (int it = 0; it < 4000000 && bad == 0; ++it) bad += check_reciprocal(next64() | top);
    for (int it = 0; it < 2000000 && bad == 0; ++it) {
        uint64_t W = next64() >> (1 + next64() % 63);  // W < 2^63, many magnitudes
        if (W == 0) W = 1;
        uint64_t C = next64() % W;
        bad += check(C, W);
    }
    printf(bad ? "FAIL\n" : "OK\n");
    return bad ? 1 : 0;
}
