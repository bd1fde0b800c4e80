// Host check of the hop kernels' tile traversal: the plans that brick_plan
// and make_brick / make_region_brick build for a set of lattices, precisions
// and launch kinds visit every tile of a half lattice exactly once, and the
// y-bands of a both-parity plan are whole rows whose three t-slices of both
// halves fit the band budget.  The visiting order is written out here from
// its definition (z-brick, y-band, t, z-group in brick, tile in band) over
// the plan's divisors and again with the plan's multiply-and-shift divisors
// as the kernels compute it; the GPU tests compare the kernels' results
// against even-odd launches, which walk whole slabs, bit for bit.
// Prints "cases N bad B" and the band count chosen for each case.
#include "lqcd_internal.h"
#include "hop_common.h"

#include <cstdio>
#include <vector>

using namespace lqcd;

static Geom geom(int lx, int ly, int lz, int lt) {
    Geom g{};
    g.L[0] = lx;
    g.L[1] = ly;
    g.L[2] = lz;
    g.L[3] = lt;
    for (int m = 0; m < 4; ++m) g.bc[m] = m == 3 ? -1 : 1;
    g.lxh = lx / 2;
    g.vh = (int64_t)lx * ly * lz * lt / 2;
    g.ntiles = (g.vh + TILE - 1) / TILE;
    g.sy = g.lxh;
    g.sz = g.sy * ly;
    g.st = g.sz * lz;
    return g;
}

// tile visited by logical block b: the order's definition
static int64_t visit(uint32_t b, const Brick &k) {
    const uint32_t ptb = k.pt.d, bz = k.bz.d, lt = k.lt.d, ny = k.nyb.d;
    const uint32_t tile = b % ptb, r1 = b / ptb;
    const uint32_t zi = r1 % bz, r2 = r1 / bz;
    const uint32_t t = k.t0 + (r2 % lt) * k.tstep, r3 = r2 / lt;
    const uint32_t band = r3 % ny, zc = r3 / ny;
    return (int64_t)(t * (uint32_t)k.lz + zc * bz + zi) * k.ptg + band * ptb + tile;
}

// the same order with the plan's multiply-and-shift divisors, as the kernels
// compute it
static int64_t visit_fixed(uint32_t b, const Brick &k) {
    const uint32_t r1 = fdiv(b, k.pt), r2 = fdiv(r1, k.bz), r3 = fdiv(r2, k.lt), zc = fdiv(r3, k.nyb);
    const uint32_t tile = b - r1 * k.pt.d, zi = r1 - r2 * k.bz.d;
    const uint32_t t = k.t0 + (r2 - r3 * k.lt.d) * k.tstep, band = r3 - zc * k.nyb.d;
    return (int64_t)((t * k.lz + zc * k.bz.d + zi) * k.ptg + band * k.pt.d + tile);
}

static int bad = 0, cases = 0;

static void fail(const char *what, const int *L, int prec, int halves) {
    ++bad;
    printf("FAIL %s: %dx%dx%dx%d prec %d halves %d\n", what, L[0], L[1], L[2], L[3], prec, halves);
}

// every tile of the half lattice once, in the plan's order
static void check_cover(const Geom &g, const Brick &k, int64_t nblocks, std::vector<int> &seen) {
    for (int64_t b = 0; b < nblocks; ++b) {
        const int64_t t = visit((uint32_t)b, k);
        if (t < 0 || t >= g.ntiles) {
            fail("tile out of range", g.L, -1, -1);
            return;
        }
        // the order agrees with its fixed-point form
        if (visit_fixed((uint32_t)b, k) != t) {
            fail("fixed-point order differs", g.L, -1, -1);
            return;
        }
        seen[t] += 1;
    }
}

static void check_plan(int lx, int ly, int lz, int lt, int prec, int halves, int want_ny) {
    ++cases;
    const Geom g = geom(lx, ly, lz, lt);
    const BrickPlan p = brick_plan(g, prec, halves);
    const Brick k = make_brick(g, p);
    printf("%dx%dx%dx%d prec %d halves %d: pt %d bz %d ny %d\n", lx, ly, lz, lt, prec, halves, p.pt,
           p.bz, p.ny);
    if (want_ny >= 0 && p.ny != want_ny) fail("band count", g.L, prec, halves);
    if (p.ny > 1) {
        const int64_t per_band = (int64_t)(p.pt / p.ny) * TILE;
        if (p.pt % p.ny != 0 || per_band % g.lxh != 0) fail("band is not whole rows", g.L, prec, halves);
        const int64_t fp = (int64_t)halves * 3 * p.bz * p.pt * spinor_tile_bytes(prec) / p.ny;
        if (fp > ((int64_t)LQCD_BRICK_BAND_KB << 10)) fail("band over budget", g.L, prec, halves);
    }
    std::vector<int> seen(g.ntiles, 0);
    check_cover(g, k, g.ntiles, seen);
    for (int64_t t = 0; t < g.ntiles; ++t)
        if (seen[t] != 1) {
            fail("tile not visited exactly once", g.L, prec, halves);
            break;
        }
    // t decomposition: the interior slices 1 .. Lt-2 and the boundary
    // slices 0, Lt-1 together visit every tile once
    if (g.st % TILE == 0 && lt > 2) {
        ++cases;
        std::vector<int> s2(g.ntiles, 0);
        const int64_t per = g.st / TILE;
        const Brick in = make_region_brick(g, p, 1, 1, lt - 2);
        const Brick bd = make_region_brick(g, p, 0, lt - 1, 2);
        check_cover(g, in, (int64_t)(lt - 2) * per, s2);
        check_cover(g, bd, 2 * per, s2);
        for (int64_t t = 0; t < g.ntiles; ++t)
            if (s2[t] != 1) {
                fail("t regions do not cover the lattice once", g.L, prec, halves);
                break;
            }
    }
}

int main() {
    const int F64 = LQCD_F64, F32 = LQCD_F32, F16 = LQCD_F16;
    // both-parity launches: bands where three t-slices of both halves of a
    // slab exceed the budget and a z-group is one plane
    check_plan(48, 48, 48, 96, F64, 2, 6);
    check_plan(48, 48, 48, 96, F32, 2, 3);
    check_plan(48, 48, 48, 96, F16, 2, 1);
    check_plan(32, 32, 32, 32, F64, 2, 2);
    check_plan(32, 32, 32, 32, F32, 2, 1);
    check_plan(32, 32, 36, 16, F64, 2, 4);
    check_plan(32, 32, 36, 16, F32, 2, 2);
    check_plan(24, 24, 24, 24, F64, 2, 1);  // two-plane z-groups: no bands
    check_plan(48, 48, 48, 12, F64, 2, 6);
    // even-odd launches: whole slabs; the ablation's one-half footprint
    for (int prec : {F64, F32, F16}) {
        check_plan(48, 48, 48, 96, prec, 0, 1);
        check_plan(32, 32, 32, 32, prec, 0, 1);
        check_plan(24, 24, 24, 24, prec, 0, 1);
        check_plan(32, 32, 36, 16, prec, 0, 1);
        check_plan(16, 16, 16, 16, prec, 0, 1);   // plain order (small lattice)
        check_plan(18, 18, 42, 40, prec, 0, 1);   // plain order, ragged last tile
        check_plan(18, 18, 42, 40, prec, 2, 1);
    }
    check_plan(48, 48, 48, 96, F64, 1, 3);
    check_plan(48, 48, 48, 96, F32, 1, 2);
    printf("cases %d bad %d\n", cases, bad);
    return bad == 0 ? 0 : 1;
}
