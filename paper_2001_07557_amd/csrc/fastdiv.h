// Division by a divisor fixed at launch time as one multiply and one shift.
//
// For a divisor 1 <= d < 2^31 let l = ceil(log2 d) and m = ceil(2^(31+l) / d).
// Then 2^(31+l) <= m d < 2^(31+l) + d <= 2^(31+l) + 2^l, and by Theorem 4.2 of
// Granlund and Montgomery, "Division by invariant integers using
// multiplication" (PLDI 1994), with N = 31:
//     floor(n / d) = floor(n m / 2^(31+l))   for every 0 <= n < 2^31.
// m < 2^32 (d > 2^(l-1) for l > 0, m = 2^31 for d = 1), so m fits 32 bits and
// n m fits 63.  The host computes (m, 31 + l) once per geometry; a kernel
// then divides site and tile indices with a 32 x 32 -> 64-bit multiply and a
// shift instead of the reciprocal-and-correct sequence of a run-time integer
// division (about twenty dependent instructions per quotient).
#pragma once

#include <stdint.h>

namespace lqcd {

struct FastDiv {
    uint32_t d;   // divisor
    uint32_t m;   // multiplier ceil(2^sh / d)
    uint32_t sh;  // 31 + ceil(log2 d)
};

// Host side: the constants for divisor d (1 <= d < 2^31; other values give
// d = 0, which callers reject before launching).
inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f{0, 0, 0};
    if (d < 1 || d >= (1u << 31)) return f;
    uint32_t l = 0;
    while (((uint64_t)1 << l) < d) ++l;
    const uint64_t p = (uint64_t)1 << (31 + l);
    f.d = d;
    f.m = (uint32_t)((p + d - 1) / d);
    f.sh = 31 + l;
    return f;
}

// floor(n / f.d) for 0 <= n < 2^31.
__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f) {
    return (uint32_t)(((uint64_t)n * f.m) >> f.sh);
}

}  // namespace lqcd
