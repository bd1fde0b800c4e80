// Host check of the multiply-and-shift division used by the kernels' index
// arithmetic: every quotient and remainder against the C++ operators, for
// every divisor up to 4096, the divisors around each power of two, the
// largest divisor and pseudo-random ones, each with the dividends at the
// edges (0, multiples of d and their neighbours, 2^31 - 1) and random ones.
// Prints the number of checks and of mismatches.
#include <stdint.h>
#include <stdio.h>

#include "fastdiv.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint32_t rnd31() {
    // splitmix64, top 31 bits
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (uint32_t)(z >> 33);
}

static long checks = 0, bad = 0;

static void check(uint32_t n, const lqcd::FastDiv &f) {
    if (n >= (1u << 31)) return;
    ++checks;
    const uint32_t q = lqcd::fdiv(n, f);
    if (q != n / f.d || n - q * f.d != n % f.d) {
        if (bad < 10) printf("mismatch n=%u d=%u q=%u\n", n, f.d, q);
        ++bad;
    }
}

static void divisor(uint32_t d) {
    const lqcd::FastDiv f = lqcd::make_fastdiv(d);
    if (f.d != d) {
        printf("no constants for d=%u\n", d);
        ++bad;
        return;
    }
    const uint32_t top = (1u << 31) - 1;
    check(0, f);
    check(1, f);
    check(top, f);
    check(top - 1, f);
    const uint32_t kmax = top / d;
    const uint32_t ks[] = {1, 2, 3, 7, 1000, kmax - 1, kmax};
    for (uint32_t k : ks) {
        if (k == 0 || k > kmax) continue;
        const uint64_t m = (uint64_t)k * d;
        check((uint32_t)(m - 1), f);
        check((uint32_t)m, f);
        if (m + 1 <= top) check((uint32_t)(m + 1), f);
    }
    for (int i = 0; i < 64; ++i) check(rnd31(), f);
}

int main() {
    for (uint32_t d = 1; d <= 4096; ++d) divisor(d);
    for (int k = 12; k <= 31; ++k) {
        const uint64_t p = 1ull << k;
        if (p - 1 < (1u << 31)) divisor((uint32_t)(p - 1));
        if (p < (1u << 31)) divisor((uint32_t)p);
        if (p + 1 < (1u << 31)) divisor((uint32_t)(p + 1));
    }
    for (int i = 0; i < 4096; ++i) divisor(rnd31() | 1u);
    // 0 and 2^31 are outside the range and get no constants
    if (lqcd::make_fastdiv(0).d != 0 || lqcd::make_fastdiv(1u << 31).d != 0) ++bad;
    printf("checks %ld bad %ld\n", checks, bad);
    return bad != 0;
}
