// The per-site hopping term shared by the operator and the solver kernels.
#pragma once

#include "lqcd_internal.h"

namespace lqcd {

// Kernel shapes.  Both give a block 64 output sites (one tile):
//   4-way: 256 threads, wave w computes the two hops of direction w and the
//          partial spinors meet in LDS (FP64 and binary16 storage);
//   8-way: 512 threads, wave w computes hop w alone and stages the two colour
//          vectors of its multiplied half-spinor in LDS, where wave 0 rebuilds
//          the four spin rows (FP32 storage).
// Measured on gfx950 against one thread per site doing all eight hops in
// registers without LDS (shape 1, kept for ablation builds): the split
// shapes win at every size (more waves in flight, shorter dependent load
// chains), 8-way is ahead for FP32 and 4-way for FP64 and binary16 (fewer
// LDS bytes per hop).  The LQCD_HOP_SHAPE_* macros (1, 4 or 8) select the
// shape per precision in ablation builds.
#ifndef LQCD_HOP_SHAPE_F64
#define LQCD_HOP_SHAPE_F64 4
#endif
#ifndef LQCD_HOP_SHAPE_F32
#define LQCD_HOP_SHAPE_F32 8
#endif
#ifndef LQCD_HOP_SHAPE_F16
#define LQCD_HOP_SHAPE_F16 4
#endif
// XCD-aware block numbering (ablation switch)
#ifndef LQCD_HOP_XCD
#define LQCD_HOP_XCD 1
#endif
// brick traversal for FP64 (ablation switch)
#ifndef LQCD_HOP_BRICK
#define LQCD_HOP_BRICK 1
#endif

constexpr int HOP_SITES = 64;  // output sites per block

// Brick traversal.  Tiles are visited brick by brick (bz z-planes, t-major
// inside a brick) so the three input t-slices an output slice touches stay in
// the L2 of the XCD that works on them.  Rule 1 (default) takes bz = Lz/8:
// with the XCD renumbering every XCD then owns one z-slab of the lattice and
// walks it in t order (Lz/4 where Lz/8 does not fit whole tiles: two XCDs
// per slab, each with half of its t range).  Rule 0 takes the largest bz
// whose three t-slices of input fit LQCD_BRICK_BUDGET_KB.  Measured
// (fraction of 8 TB/s, plain order -> rule 1): 32^4 FP64-18 73.2 -> 78.3,
// FP32-12 70.4 -> 83.9; 48^3x96 FP64-18 60.6 -> 68.6, FP32-12 65.2 -> 72.2;
// 24^4 (two-plane groups, four slabs) FP64-18 66.3 -> 77.5, FP32-12 68 -> 73;
// binary16 60.7 -> 63.6 at 48^3x96 and 1-2 points at 32^4.
#ifndef LQCD_BRICK_BUDGET_KB
#define LQCD_BRICK_BUDGET_KB 3072
#endif
constexpr int64_t BRICK_L2_BUDGET = (int64_t)LQCD_BRICK_BUDGET_KB << 10;
#ifndef LQCD_BRICK_MODE
#define LQCD_BRICK_MODE 1
#endif
#ifndef LQCD_BRICK_MIN_LOG2
#define LQCD_BRICK_MIN_LOG2 17
#endif
// y-bands of an FP64 or FP32 both-parity launch (full-lattice D_hop and M).
// Such a launch keeps both halves of psi and its links in play, so the three
// t-slices of a z-slab that rule 1 keeps in an XCD's L2 are twice the
// even-odd footprint (48^3x96 FP64: 8 MB).  Where they exceed
// LQCD_BRICK_BAND_KB, each slab is cut into y-bands of whole rows (z-groups
// of one plane only), walked in t one after the other.  Measured
// (full-lattice M, TB/s, slab -> bands, four and two runs): 48^3x96 FP64-18
// 4.87-4.94 -> 5.11-5.23 (six bands), FP32-18 5.02-5.16 -> 5.15-5.31
// (three); 32^4 FP64-18 4.78-4.93 -> 4.95-5.04 (two); fetched bytes over
// algorithmic 1.58x -> 1.16x and 1.41x -> 1.12x (FP64).  Bands on the
// even-odd hop cut its 48^3x96 FP64 fetch from 1.27-1.35x to 1.06-1.08x yet
// run 1.5-3.2 points slower (the slices whole slabs fetch again come from
// the Infinity Cache), and bands across a two-plane z-group (24^4) lose 5%,
// so neither is done.  0 switches the bands off; LQCD_BRICK_BAND_EO = 1
// gives the even-odd launches bands too (ablation).
#ifndef LQCD_BRICK_BAND_KB
#define LQCD_BRICK_BAND_KB 1536
#endif
#ifndef LQCD_BRICK_BAND_EO
#define LQCD_BRICK_BAND_EO 0
#endif
// number of z-bricks rule 1 aims for with FP64 fields (ablation switch; 8
// gives every XCD one slab, 16 two thinner ones walked one after the other)
#ifndef LQCD_BRICK_NB_F64
#define LQCD_BRICK_NB_F64 8
#endif
// precisions that use the brick order: bit p set for precision p (F64, F32,
// F16)
#ifndef LQCD_BRICK_PRECS
#define LQCD_BRICK_PRECS 7
#endif

// Ends one hop: the values carried to the next hop are pinned in registers (an empty asm that
// reads and writes it) and the scheduler may not move instructions across.
// Without this the compiler sinks all hop arithmetic below the last load, so
// every loaded spinor and link stays live at once, the register demand
// exceeds the file and occupancy collapses to one wave per SIMD.
template <typename T, int N>
__device__ __forceinline__ void hop_fence(cplx<T> acc[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k) asm volatile("" : "+v"(acc[k].re), "+v"(acc[k].im));
    __builtin_amdgcn_sched_barrier(0);
}

// Cache-blocked tile order: tiles per z-group, z-groups per brick, Lt and
// z-groups in Lz.  The plain order is the same formula with pt = bz = lz = 1
// and lt larger than any tile index, so the traversal needs no branch on the
// mode.
struct Brick {
    FastDiv pt, bz, lt;
    int lz;
    FastDiv nyb;    // y-bands per z-group, walked one after the other
    uint32_t ptg;   // tiles per z-group (pt = ptg / nyb tiles per band)
    // t-slices visited: t0, t0 + tstep, ... (lt of them); a whole-lattice
    // launch has t0 = 0, tstep = 1, a region launch (interior or boundary
    // slices of a t decomposition) other values
    uint32_t t0, tstep;
};

struct HopArgs {
    // what the site index needs comes first, so that a block reads it with
    // one wide scalar load
    int64_t bpp;          // blocks per parity
    int par0;             // parity of the first bpp blocks
    int paired;           // both parities: block 2i / 2i + 1 = even / odd tile i
    uint32_t nblk;        // blocks in the grid
    Brick brick;          // cache-blocked tile order (identity: plain order)
    Geom g;
    char *out[2];         // output half field for output parity p
    const char *in[2];    // input half field (opposite parity) read by output parity p
    const char *y[2];     // optional beta * y term, parity p
    const char *U;        // gauge field
    double alpha, beta;
    double *partial;      // optional per-block |out|^2
    int stream;           // non-temporal hints: bit 0 output stores, bit 1 link loads
    int rows;             // 8-way shape: waves 0-3 rebuild one spin row each
    // boundary-slice launches: the t-hops that cross the t boundary read
    // face[0] (projected half-spinors of the forward neighbours) and face[1]
    // (U^dag times the projected backward neighbours) instead of `in`
    const char *face[2];
    // CG-update launches (cg_x set): the result A p is not stored; the
    // epilogue does x += alpha p, r -= alpha A p on out = r and writes the
    // block partial of |r|^2, alpha read from the device (read late: the
    // sixth line of the arguments)
    char *cg_x;
    const char *cg_p;
    const double *cg_alpha;
    // host side: dynamic LDS bytes added to each 4-way block (limits the
    // blocks in flight per CU; not read by the kernels)
    uint32_t lds_extra;
    // t-march launches: t-slices per block (0: one tile per block)
    int tseg;
};

// Tile visited by logical block b (within one parity).  With bricks of bz
// z-groups the order is (z-brick, y-band, t, z-group in brick, tile in band):
// the three t-slices of a brick that one output slice touches stay in the
// XCD's L2, where the plain order would revisit each input slice from memory
// for the t-neighbours of the slices before and after it.
__device__ __forceinline__ int64_t brick_order(uint32_t b, const Brick &k) {
    const uint32_t r1 = fdiv(b, k.pt);    // (z-group, t) in traversal order
    const uint32_t r2 = fdiv(r1, k.bz);   // (brick, band, t)
    const uint32_t r3 = fdiv(r2, k.lt);   // (brick, band)
    const uint32_t zc = fdiv(r3, k.nyb);  // brick
    const uint32_t tile = b - r1 * k.pt.d;
    const uint32_t zi = r1 - r2 * k.bz.d;
    const uint32_t t = k.t0 + (r2 - r3 * k.lt.d) * k.tstep;
    const uint32_t band = r3 - zc * k.nyb.d;
    return (int64_t)((t * k.lz + zc * k.bz.d + zi) * k.ptg + band * k.pt.d + tile);
}

__device__ __forceinline__ int64_t brick_tile(const HopArgs &a, uint32_t b) {
    return brick_order(b, a.brick);
}

// Blocked traversal plan: the tiles of a z-group (the fewest consecutive
// z-planes whose sites fill whole tiles, usually one plane) form a unit; a
// brick is bz z-groups and all t.  bz = 0: plain order.
struct BrickPlan {
    int pt;      // tiles per z-group
    int bz;      // z-groups per brick
    int lz;      // z-groups in Lz
    int ny = 1;  // y-bands per z-group
};

// See the rules next to LQCD_BRICK_MODE.  Rule 1 cuts Lz into 8 bricks (one
// per XCD), or into 4 when the z-groups do not divide by 8 (two XCDs then
// share a brick, each taking half of its t range).  `halves`: 2 for the plan
// of a both-parity launch, which may add y-bands (LQCD_BRICK_BAND_KB); 1 for
// an even-odd launch of an ablation build that bands those too; 0 no bands.
inline BrickPlan brick_plan(const Geom &g, int prec, int halves = 0) {
    BrickPlan k{0, 0, 0};
    if (!LQCD_HOP_BRICK || !((LQCD_BRICK_PRECS >> prec) & 1)) return k;
    // small lattices live in the caches anyway: only half-lattices of at
    // least 2^LQCD_BRICK_MIN_LOG2 sites take the blocked order
    if (g.vh < ((int64_t)1 << LQCD_BRICK_MIN_LOG2) || g.vh % TILE != 0) return k;
    const int64_t plane = (int64_t)g.lxh * g.L[1];
    int gz = 1;
    while (gz <= g.L[2] && (g.L[2] % gz != 0 || (plane * gz) % TILE != 0)) ++gz;
    if (gz > g.L[2]) return k;
    const int lz = g.L[2] / gz;
    const int64_t pt = plane * gz / TILE;
    if (LQCD_BRICK_MODE == 1) {
        const int nb0 = prec == LQCD_F64 ? LQCD_BRICK_NB_F64 : 8;
        for (int nb : {nb0, nb0 / 2}) {
            if (lz % nb == 0 && lz / nb >= 2) {
                k = {(int)pt, lz / nb, lz};
                // three t-slices of the slab, of each half the launch reads
                const int64_t fp = halves * 3 * (int64_t)k.bz * pt * spinor_tile_bytes(prec);
                if (halves > 0 && prec != LQCD_F16 && gz == 1 &&
                    fp > ((int64_t)LQCD_BRICK_BAND_KB << 10))
                    for (int ny = 2; ny <= pt; ++ny)
                        if (pt % ny == 0 && (pt / ny * TILE) % g.lxh == 0 &&
                            fp / ny <= ((int64_t)LQCD_BRICK_BAND_KB << 10)) {
                            k.ny = ny;
                            break;
                        }
                return k;
            }
        }
    }
    const int64_t group_bytes = pt * spinor_tile_bytes(prec);
    for (int bz = lz - 1; bz >= 1; --bz) {
        if (lz % bz == 0 && 3 * bz * group_bytes <= BRICK_L2_BUDGET) {
            k = {(int)pt, bz, lz};
            return k;
        }
    }
    return k;
}

// Traversal constants of a plan.
inline Brick make_brick(const Geom &g, const BrickPlan &b) {
    Brick k;
    if (b.bz == 0) {
        k.pt = make_fastdiv(1);
        k.bz = make_fastdiv(1);
        k.lt = make_fastdiv((1u << 31) - 1);
        k.lz = 1;
        k.nyb = make_fastdiv(1);
        k.ptg = 1;
    } else {
        k.pt = make_fastdiv((uint32_t)(b.pt / b.ny));
        k.bz = make_fastdiv((uint32_t)b.bz);
        k.lt = make_fastdiv((uint32_t)g.L[3]);
        k.lz = b.lz;
        k.nyb = make_fastdiv((uint32_t)b.ny);
        k.ptg = (uint32_t)b.pt;
    }
    k.t0 = 0;
    k.tstep = 1;
    return k;
}

// Traversal of the t-slices t0, t0 + tstep, ... (nt of them) only, each a
// whole number of tiles: the lattice's blocked order restricted to those
// slices, or slice by slice in tile order where the lattice has no blocked
// order.
inline Brick make_region_brick(const Geom &g, const BrickPlan &b, int t0, int tstep, int nt) {
    Brick k = make_brick(g, b);
    if (b.bz == 0) {
        k.pt = make_fastdiv((uint32_t)(g.st / TILE));
        k.bz = make_fastdiv(1);
        k.lz = 1;
        k.ptg = (uint32_t)(g.st / TILE);
    }
    k.lt = make_fastdiv((uint32_t)nt);
    k.t0 = (uint32_t)t0;
    k.tstep = (uint32_t)tstep;
    return k;
}

// region: -1 the whole half lattice; 0 the interior t-slices 1 .. Lt-2;
// 1 the boundary slices 0 and Lt-1, whose t-hops across the boundary read
// a.face (slices must be whole tiles for regions 0 and 1)
int hop_launch(const HopArgs &a, int prec, int link, bool dag, int nparity, hipStream_t st,
               int region = -1);
int64_t hop_partials(const Geom &g, int nparity);

// Spin projection (1 + S g_mu): with the unit constants of the chiral basis,
//   h0 = psi_0 + S c0 psi_a0,   h1 = psi_1 + S c1 psi_a1,
// and the full four-row result is rebuilt from the two colour vectors
// chi = U h as  row 0 = chi0, row 1 = chi1, row a0 = S conj(c0) chi0,
// row a1 = S conj(c1) chi1  (the projector has rank two).
// Unit codes: 0 -> 1, 1 -> -1, 2 -> i, 3 -> -i.
template <int MU> struct Proj;
template <> struct Proj<0> { static constexpr int a0 = 3, c0 = 2, a1 = 2, c1 = 2; };
template <> struct Proj<1> { static constexpr int a0 = 3, c0 = 1, a1 = 2, c1 = 0; };
template <> struct Proj<2> { static constexpr int a0 = 2, c0 = 2, a1 = 3, c1 = 3; };
template <> struct Proj<3> { static constexpr int a0 = 2, c0 = 0, a1 = 3, c1 = 0; };

__host__ __device__ constexpr int neg_code(int c) { return c ^ 1; }
__host__ __device__ constexpr int conj_code(int c) { return c < 2 ? c : (c ^ 1); }

// Rows 0 and 1 of (1 + S g_mu) psi.
template <int MU, int S, typename T>
__device__ __forceinline__ void project_half(const cplx<T> psi[12], cplx<T> h0[3], cplx<T> h1[3]) {
    using PR = Proj<MU>;
    constexpr int k0 = S > 0 ? PR::c0 : neg_code(PR::c0);
    constexpr int k1 = S > 0 ? PR::c1 : neg_code(PR::c1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h0[c] = psi[c] + mul_unit<k0>(psi[PR::a0 * 3 + c]);
        h1[c] = psi[3 + c] + mul_unit<k1>(psi[PR::a1 * 3 + c]);
    }
}

// Project with (1 + S g_mu) and apply the boundary sign: rows 0 and 1 of the
// half-spinor of one hop (FP64 and FP32 storage).
template <int MU, int S, typename T>
__device__ __forceinline__ void hop_half(const cplx<T> psi[12], T sign, cplx<T> h0[3], cplx<T> h1[3]) {
    using PR = Proj<MU>;
    constexpr int k0 = S > 0 ? PR::c0 : neg_code(PR::c0);
    constexpr int k1 = S > 0 ? PR::c1 : neg_code(PR::c1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h0[c] = scale(sign, psi[c] + mul_unit<k0>(psi[PR::a0 * 3 + c]));
        h1[c] = scale(sign, psi[3 + c] + mul_unit<k1>(psi[PR::a1 * 3 + c]));
    }
}

// chi = U h (or U^dag h) for the two colour vectors of a half-spinor.
template <bool UDAG, typename T>
__device__ __forceinline__ void half_mul(const cplx<T> u[9], const cplx<T> h0[3],
                                         const cplx<T> h1[3], cplx<T> x0[3], cplx<T> x1[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (UDAG) {
            x0[a] = cdot3c(u[a], h0[0], u[3 + a], h0[1], u[6 + a], h0[2]);
            x1[a] = cdot3c(u[a], h1[0], u[3 + a], h1[1], u[6 + a], h1[2]);
        } else {
            x0[a] = cdot3(u[3 * a], h0[0], u[3 * a + 1], h0[1], u[3 * a + 2], h0[2]);
            x1[a] = cdot3(u[3 * a], h1[0], u[3 * a + 1], h1[1], u[3 * a + 2], h1[2]);
        }
    }
}

// Hops on binary16 storage run in packed binary16 arithmetic where it can be
// exact or is one rounding, and in FP32 elsewhere:
//  * the projected half-spinor h = a + k b (k a unit) of the stored values
//    of the neighbour site is one v_pk_add_f16 per complex component, which
//    rounds the exact sum to binary16 once (ties to even);
//  * U h with rows 0 and 1 of the link as stored: two-term binary16 dot
//    products accumulated in FP32 (v_dot2_f32_f16, products exact); row 2 =
//    conj(row0 x row1) is rebuilt in FP32 and enters by mixed-precision FMAs;
//  * the neighbour's scale times the boundary sign multiplies the result.
// Each complex component of h is held in the two packed forms its products
// need, produced directly by the operand selects and negations of the add:
// F = 0 (re h, -im h), 1 (im h, re h) for U h and 2 (re h, im h),
// 3 (im h, -re h) for U^dag h.  Against the FP32 arithmetic it replaces, 12%
// fewer vector instructions per site.
template <int K, int F>
__device__ __forceinline__ v2h pk_form(v2h a, v2h b);
#define LQCD_PK_FORM(K, F, MODS)                                         \
    template <>                                                          \
    __device__ __forceinline__ v2h pk_form<K, F>(v2h a, v2h b) {         \
        v2h r;                                                           \
        asm("v_pk_add_f16 %0, %1, %2 " MODS : "=v"(r) : "v"(a), "v"(b)); \
        return r;                                                        \
    }
LQCD_PK_FORM(0, 0, "neg_hi:[1,1]")
LQCD_PK_FORM(1, 0, "neg_lo:[0,1] neg_hi:[1,0]")
LQCD_PK_FORM(2, 0, "op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,1] neg_hi:[1,1]")
LQCD_PK_FORM(3, 0, "op_sel:[0,1] op_sel_hi:[1,0] neg_hi:[1,0]")
LQCD_PK_FORM(0, 1, "op_sel:[1,1] op_sel_hi:[0,0]")
LQCD_PK_FORM(1, 1, "op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,1] neg_hi:[0,1]")
LQCD_PK_FORM(2, 1, "op_sel:[1,0] op_sel_hi:[0,1] neg_hi:[0,1]")
LQCD_PK_FORM(3, 1, "op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,1]")
LQCD_PK_FORM(0, 2, "")
LQCD_PK_FORM(1, 2, "neg_lo:[0,1] neg_hi:[0,1]")
LQCD_PK_FORM(2, 2, "op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,1]")
LQCD_PK_FORM(3, 2, "op_sel:[0,1] op_sel_hi:[1,0] neg_hi:[0,1]")
LQCD_PK_FORM(0, 3, "op_sel:[1,1] op_sel_hi:[0,0] neg_hi:[1,1]")
LQCD_PK_FORM(1, 3, "op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,1] neg_hi:[1,0]")
LQCD_PK_FORM(2, 3, "op_sel:[1,0] op_sel_hi:[0,1] neg_hi:[1,0]")
LQCD_PK_FORM(3, 3, "op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,1] neg_hi:[1,1]")
#undef LQCD_PK_FORM

// a.x b.x + a.y b.y + c, products exact, FP32 accumulation
__device__ __forceinline__ float dot2h(v2h a, v2h b, float c) {
    return __builtin_amdgcn_fdot2(a, b, c, false);
}
// the first product of a chain: the three-operand form with an inline zero
// (the two-operand form would need its accumulator cleared by a move)
__device__ __forceinline__ float dot2h0(v2h a, v2h b) {
    float r;
    asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
// a b rounded on its own: not fused into a later addition, so a hop's result
// is the same whether the caller adds it to the other hop straight away or
// after a branch (a boundary launch reading faces)
__device__ __forceinline__ float mul_nc(float a, float b) {
#pragma clang fp contract(off)
    return a * b;
}
// r.re v.x + r.im v.y + c with v binary16 (mixed-precision FMAs)
__device__ __forceinline__ float mix2(cplx<float> r, v2h v, float c) {
    return fmaf(r.re, (float)v.x, fmaf(r.im, (float)v.y, c));
}

// conj(a b - c d) of binary16 complex numbers in FP32, every product a
// mixed-precision FMA on the stored halves (no separate conversion)
__device__ __forceinline__ cplx<float> conj_cross_h(v2h a, v2h b, v2h c, v2h d) {
    float re = fmaf((float)c.y, (float)d.y, 0.f);
    re = fmaf(-(float)c.x, (float)d.x, re);
    re = fmaf(-(float)a.y, (float)b.y, re);
    re = fmaf((float)a.x, (float)b.x, re);
    float im = fmaf((float)c.x, (float)d.y, 0.f);
    im = fmaf((float)c.y, (float)d.x, im);
    im = fmaf(-(float)a.x, (float)b.y, im);
    im = fmaf(-(float)a.y, (float)b.x, im);
    return {re, im};
}

// A binary16 12-real link: rows 0 and 1 as stored (re, im pairs), row 2 =
// conj(row0 x row1) in FP32.
template <bool NT>
__device__ __forceinline__ void load_link_h(const char *__restrict__ U, int64_t ntiles, int p,
                                            int64_t s, int mu, v2h u[6], cplx<float> r2[3]) {
    const int lane = (int)(s & (TILE - 1));
    // the parity's links from a 64-bit base (p is the same across a block),
    // the tile and lane within it by a 32-bit offset (F16_MAX_TILES)
    const char *up = U + (int64_t)p * ntiles * 4 * link_tile_bytes(LQCD_F16, 12);
    const uint32_t toff = ((uint32_t)(s >> TILE_SHIFT) * 4u + (uint32_t)mu) * (uint32_t)link_tile_bytes(LQCD_F16, 12);
    const v4u q = stream_load<NT>(reinterpret_cast<const v4u *>(up + (uint64_t)(toff + (uint32_t)lane * WORD)));
    const v2u q2 = stream_load<NT>(
        reinterpret_cast<const v2u *>(up + (uint64_t)(toff + TILE * WORD + (uint32_t)lane * 8u)));
    const uint32_t w[6] = {q.x, q.y, q.z, q.w, q2.x, q2.y};
#pragma unroll
    for (int j = 0; j < 6; ++j) u[j] = __builtin_bit_cast(v2h, w[j]);
    r2[0] = conj_cross_h(u[1], u[5], u[2], u[4]);
    r2[1] = conj_cross_h(u[2], u[3], u[0], u[5]);
    r2[2] = conj_cross_h(u[0], u[4], u[1], u[3]);
}

// The projected half-spinor of one hop, rows 0 and 1 of (1 + S g_mu) psi,
// in the packed forms of U h (UDAG false) or U^dag h: hr[c], hi[c] for
// colour c of row 0 and hr[3 + c], hi[3 + c] for row 1.
template <int MU, int S, bool UDAG>
__device__ __forceinline__ void half_forms_h(const cplx<_Float16> psi[12], v2h hr[6], v2h hi[6]) {
    using PR = Proj<MU>;
    constexpr int k0 = S > 0 ? PR::c0 : neg_code(PR::c0);
    constexpr int k1 = S > 0 ? PR::c1 : neg_code(PR::c1);
    constexpr int FR = UDAG ? 2 : 0;
    constexpr int FI = UDAG ? 3 : 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const v2h a0 = v2h{psi[c].re, psi[c].im};
        const v2h b0 = v2h{psi[PR::a0 * 3 + c].re, psi[PR::a0 * 3 + c].im};
        const v2h a1 = v2h{psi[3 + c].re, psi[3 + c].im};
        const v2h b1 = v2h{psi[PR::a1 * 3 + c].re, psi[PR::a1 * 3 + c].im};
        hr[c] = pk_form<k0, FR>(a0, b0);
        hi[c] = pk_form<k0, FI>(a0, b0);
        hr[3 + c] = pk_form<k1, FR>(a1, b1);
        hi[3 + c] = pk_form<k1, FI>(a1, b1);
    }
}

// factor (U h) or factor (U^dag h) for the two colour vectors of a
// half-spinor in packed forms: x0 from row 0, x1 from row 1 (SCALE false:
// U h or U^dag h, the caller applies the factor).
template <bool UDAG, bool SCALE = true>
__device__ __forceinline__ void half_mul_h(const v2h hr[6], const v2h hi[6], const v2h u[6],
                                           const cplx<float> r2[3], float factor,
                                           cplx<float> x0[3], cplx<float> x1[3]) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const v2h *fr = hr + 3 * r, *fi = hi + 3 * r;
        cplx<float> *x = r == 0 ? x0 : x1;
        if constexpr (!UDAG) {
            // U[a][b] = u[3a + b] (a = 0, 1), row 2 from r2
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const float re = dot2h(u[3 * a + 2], fr[2], dot2h(u[3 * a + 1], fr[1], dot2h0(u[3 * a], fr[0])));
                const float im = dot2h(u[3 * a + 2], fi[2], dot2h(u[3 * a + 1], fi[1], dot2h0(u[3 * a], fi[0])));
                x[a] = SCALE ? cplx<float>{mul_nc(factor, re), mul_nc(factor, im)} : cplx<float>{re, im};
            }
            const float re = mix2(r2[2], fr[2], mix2(r2[1], fr[1], mix2(r2[0], fr[0], 0.f)));
            const float im = mix2(r2[2], fi[2], mix2(r2[1], fi[1], mix2(r2[0], fi[0], 0.f)));
            x[2] = SCALE ? cplx<float>{mul_nc(factor, re), mul_nc(factor, im)} : cplx<float>{re, im};
        } else {
            // U^dag[a][b] = conj(U[b][a]): u[a], u[3 + a] and r2[a]
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float re = dot2h(u[3 + a], fr[1], dot2h(u[a], fr[0], mix2(r2[a], fr[2], 0.f)));
                const float im = dot2h(u[3 + a], fi[1], dot2h(u[a], fi[0], mix2(r2[a], fi[2], 0.f)));
                x[a] = SCALE ? cplx<float>{mul_nc(factor, re), mul_nc(factor, im)} : cplx<float>{re, im};
            }
        }
    }
}

// One hop on binary16 storage: the two colour vectors chi0, chi1.
template <int MU, int S, bool UDAG, bool SCALE = true>
__device__ __forceinline__ void hop_chi_h(const cplx<_Float16> psi[12], const v2h u[6],
                                          const cplx<float> r2[3], float factor,
                                          cplx<float> x0[3], cplx<float> x1[3]) {
    v2h hr[6], hi[6];
    half_forms_h<MU, S, UDAG>(psi, hr, hi);
    half_mul_h<UDAG, SCALE>(hr, hi, u, r2, factor, x0, x1);
}

// Project with (1 + S g_mu), apply the boundary sign and multiply by U (or
// U^dag): the two colour vectors chi0, chi1 of one hop.
template <int MU, int S, bool UDAG, typename T>
__device__ __forceinline__ void hop_chi(const cplx<T> psi[12], const cplx<T> u[9], T sign,
                                        cplx<T> x0[3], cplx<T> x1[3]) {
    cplx<T> h0[3], h1[3];
    hop_half<MU, S>(psi, sign, h0, h1);
    half_mul<UDAG>(u, h0, h1, x0, x1);
}

// Load the link of direction MU at parity q, site y, and form the two colour
// vectors of one hop from the neighbour spinor psi (binary16 storage: the
// packed path above; factor = boundary sign, times the site scale for
// binary16).
template <int MU, int S, bool UDAG, int P, int LK, bool LNT, bool SCALE = true>
__device__ __forceinline__ void link_chi(const char *__restrict__ U, int64_t ntiles, int q,
                                         int64_t y, const cplx<typename hop_elem<P>::type> psi[12],
                                         typename real_of<P>::type factor,
                                         cplx<typename real_of<P>::type> x0[3],
                                         cplx<typename real_of<P>::type> x1[3]) {
    if constexpr (P == LQCD_F16) {
        v2h u[6];
        cplx<float> r2[3];
        load_link_h<LNT>(U, ntiles, q, y, MU, u, r2);
        hop_chi_h<MU, S, UDAG, SCALE>(psi, u, r2, factor, x0, x1);
    } else {
        cplx<typename real_of<P>::type> u[9];
        load_link<P, LK, LNT>(U, ntiles, q, y, MU, u);
        hop_chi<MU, S, UDAG>(psi, u, factor, x0, x1);
    }
}

// Face buffers of a t decomposition: per site of one t-slice (index j within
// the slice, tiles of 64 sites) two colour vectors (six complex numbers) in
// the arithmetic precision, as 16-byte words: FP64 six words of one complex,
// FP32 three words of two.
template <typename T>
__device__ __forceinline__ void load_face(const char *__restrict__ f, int64_t j, cplx<T> v[6]) {
    const int lane = (int)(j & (TILE - 1));
    if constexpr (sizeof(T) == 8) {
        const v2d *w = reinterpret_cast<const v2d *>(f + (j >> TILE_SHIFT) * (6 * TILE * WORD)) + lane;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const v2d d = w[k * TILE];
            v[k] = {d.x, d.y};
        }
    } else {
        const v4f *w = reinterpret_cast<const v4f *>(f + (j >> TILE_SHIFT) * (3 * TILE * WORD)) + lane;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const v4f d = w[k * TILE];
            v[2 * k] = {d.x, d.y};
            v[2 * k + 1] = {d.z, d.w};
        }
    }
}

template <typename T>
__device__ __forceinline__ void store_face(char *__restrict__ f, int64_t j, const cplx<T> v[6]) {
    const int lane = (int)(j & (TILE - 1));
    if constexpr (sizeof(T) == 8) {
        v2d *w = reinterpret_cast<v2d *>(f + (j >> TILE_SHIFT) * (6 * TILE * WORD)) + lane;
#pragma unroll
        for (int k = 0; k < 6; ++k) w[k * TILE] = v2d{v[k].re, v[k].im};
    } else {
        v4f *w = reinterpret_cast<v4f *>(f + (j >> TILE_SHIFT) * (3 * TILE * WORD)) + lane;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            w[k * TILE] = v4f{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im};
    }
}

// binary16 storage: 52 bytes per site, tiles of 64 sites of three 16-byte
// words and then 64 FP32 numbers.  The forward face holds the half-spinor in
// the packed forms of U h (hr[0..5], hi[0..5], four per word) and the
// neighbour's scale times the boundary sign; the backward face holds six FP32
// complex numbers in the three words, as for FP32.
constexpr int FACE_H_TILE = 3 * TILE * WORD + TILE * 4;

__device__ __forceinline__ void store_face_forms(char *__restrict__ f, int64_t j, const v2h hr[6],
                                                 const v2h hi[6], float factor) {
    const int lane = (int)(j & (TILE - 1));
    char *t = f + (j >> TILE_SHIFT) * FACE_H_TILE;
    v4u *w = reinterpret_cast<v4u *>(t) + lane;
    const v2h v[12] = {hr[0], hr[1], hr[2], hr[3], hr[4], hr[5], hi[0], hi[1], hi[2], hi[3], hi[4], hi[5]};
#pragma unroll
    for (int k = 0; k < 3; ++k)
        w[k * TILE] = v4u{__builtin_bit_cast(uint32_t, v[4 * k]), __builtin_bit_cast(uint32_t, v[4 * k + 1]),
                          __builtin_bit_cast(uint32_t, v[4 * k + 2]), __builtin_bit_cast(uint32_t, v[4 * k + 3])};
    reinterpret_cast<float *>(t + 3 * TILE * WORD)[lane] = factor;
}

__device__ __forceinline__ void load_face_forms(const char *__restrict__ f, int64_t j, v2h hr[6],
                                                v2h hi[6], float &factor) {
    const int lane = (int)(j & (TILE - 1));
    const char *t = f + (j >> TILE_SHIFT) * FACE_H_TILE;
    const v4u *w = reinterpret_cast<const v4u *>(t) + lane;
    v2h v[12];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // through a plain array: a bit cast of a vector element (q.y) reads
        // the vector's first element with this compiler
        const v4u q = w[k * TILE];
        const uint32_t e[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) v[4 * k + i] = __builtin_bit_cast(v2h, e[i]);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        hr[c] = v[c];
        hi[c] = v[6 + c];
    }
    factor = reinterpret_cast<const float *>(t + 3 * TILE * WORD)[lane];
}

__device__ __forceinline__ void store_face_h(char *__restrict__ f, int64_t j, const cplx<float> v[6],
                                             float factor) {
    const int lane = (int)(j & (TILE - 1));
    char *t = f + (j >> TILE_SHIFT) * FACE_H_TILE;
    v4f *w = reinterpret_cast<v4f *>(t) + lane;
#pragma unroll
    for (int k = 0; k < 3; ++k) w[k * TILE] = v4f{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im};
    reinterpret_cast<float *>(t + 3 * TILE * WORD)[lane] = factor;
}

__device__ __forceinline__ void load_face_h(const char *__restrict__ f, int64_t j, cplx<float> v[6],
                                            float &factor) {
    const int lane = (int)(j & (TILE - 1));
    const char *t = f + (j >> TILE_SHIFT) * FACE_H_TILE;
    const v4f *w = reinterpret_cast<const v4f *>(t) + lane;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const v4f d = w[k * TILE];
        v[2 * k] = {d.x, d.y};
        v[2 * k + 1] = {d.z, d.w};
    }
    factor = reinterpret_cast<const float *>(t + 3 * TILE * WORD)[lane];
}

// Bytes of one face buffer (one t-slice of one parity) for storage precision prec.
inline size_t face_bytes(const Geom &g, int prec) {
    if (prec == LQCD_F16) return (size_t)(g.st / TILE) * FACE_H_TILE;
    return (size_t)g.st * 6 * (prec == LQCD_F64 ? 16 : 8);
}

// Add one hop's chi0, chi1 into the four spin rows of acc.
template <int MU, int S, typename T>
__device__ __forceinline__ void chi_accumulate(const cplx<T> x0[3], const cplx<T> x1[3],
                                               cplx<T> acc[12]) {
    using PR = Proj<MU>;
    constexpr int r0 = S > 0 ? conj_code(PR::c0) : neg_code(conj_code(PR::c0));
    constexpr int r1 = S > 0 ? conj_code(PR::c1) : neg_code(conj_code(PR::c1));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[a] = acc[a] + x0[a];
        acc[3 + a] = acc[3 + a] + x1[a];
        acc[PR::a0 * 3 + a] = acc[PR::a0 * 3 + a] + mul_unit<r0>(x0[a]);
        acc[PR::a1 * 3 + a] = acc[PR::a1 * 3 + a] + mul_unit<r1>(x1[a]);
    }
}

// Neighbour index and boundary sign of one hop (FWD: x + mu, else x - mu).
template <int MU, bool FWD>
__device__ __forceinline__ int64_t hop_neighbour(const Geom &g, int64_t s, const Coord &c, bool &flip) {
    if constexpr (MU == 0) {
        const int64_t row = s - (c.x >> 1);
        if constexpr (FWD) {
            flip = c.x == g.L[0] - 1 && g.bc[0] < 0;
            return row + ((c.x + 1 == g.L[0] ? 0 : c.x + 1) >> 1);
        } else {
            flip = c.x == 0 && g.bc[0] < 0;
            return row + ((c.x == 0 ? g.L[0] - 1 : c.x - 1) >> 1);
        }
    } else {
        const int xm = MU == 1 ? c.y : MU == 2 ? c.z : c.t;
        const int L = g.L[MU];
        const int64_t st = MU == 1 ? g.sy : MU == 2 ? g.sz : g.st;
        if constexpr (FWD) {
            flip = xm == L - 1 && g.bc[MU] < 0;
            return xm == L - 1 ? s - (int64_t)(L - 1) * st : s + st;
        } else {
            flip = xm == 0 && g.bc[MU] < 0;
            return xm == 0 ? s + (int64_t)(L - 1) * st : s - st;
        }
    }
}

// chi of the single hop H (0..7: direction H/2, forward for even H) of site s.
// HALO: the t-hops that cross the t boundary take their half-spinor (forward)
// or its product with U^dag (backward) from the face buffers.
template <int H, int P, int LK, bool DAG, bool LNT, bool HALO = false>
__device__ __forceinline__ void hop_single(const Geom &g, const char *__restrict__ in,
                                           const char *__restrict__ U, int p, int64_t s,
                                           const Coord &c, cplx<typename real_of<P>::type> x0[3],
                                           cplx<typename real_of<P>::type> x1[3],
                                           const char *const *face = nullptr) {
    using T = typename real_of<P>::type;
    constexpr int MU = H >> 1;
    constexpr bool FWD = (H & 1) == 0;
    constexpr int S = FWD ? (DAG ? 1 : -1) : (DAG ? -1 : 1);
    if constexpr (HALO && MU == 3) {
        if (FWD ? c.t == g.L[3] - 1 : c.t == 0) {
            if constexpr (FWD && P == LQCD_F16) {
                v2h hr[6], hi[6], u[6];
                cplx<float> r2[3];
                float fac;
                load_face_forms(face[0], s - (int64_t)(g.L[3] - 1) * g.st, hr, hi, fac);
                load_link_h<LNT>(U, g.ntiles, p, s, MU, u, r2);
                half_mul_h<false>(hr, hi, u, r2, fac, x0, x1);
                return;
            }
            cplx<T> h[6];
            if constexpr (P == LQCD_F16) {
                float fb;
                load_face_h(face[1], s, h, fb);
#pragma unroll
                for (int k = 0; k < 6; ++k) h[k] = {mul_nc(fb, h[k].re), mul_nc(fb, h[k].im)};
            } else {
                load_face<T>(face[FWD ? 0 : 1], FWD ? s - (int64_t)(g.L[3] - 1) * g.st : s, h);
            }
            if constexpr (FWD) {
                cplx<T> u[9];
                load_link<P, LK, LNT>(U, g.ntiles, p, s, MU, u);
                half_mul<false>(u, h, h + 3, x0, x1);
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    x0[a] = h[a];
                    x1[a] = h[3 + a];
                }
            }
            return;
        }
    }
    bool flip;
    const int64_t nb = hop_neighbour<MU, FWD>(g, s, c, flip);
    cplx<typename hop_elem<P>::type> psi[12];
    T sgn = flip ? T(-1) : T(1);
    load_spinor_hop<P>(in, nb, psi, sgn);
    link_chi<MU, S, !FWD, P, LK, LNT>(U, g.ntiles, FWD ? p : p ^ 1, FWD ? s : nb, psi, sgn, x0, x1);
}

// Sign S of the projector of hop H.
template <int H, bool DAG>
struct HopSign {
    static constexpr int value = (H & 1) == 0 ? (DAG ? 1 : -1) : (DAG ? -1 : 1);
};

// Forward and backward hops in direction MU for the site s of parity p.  The
// two hops use the projectors (1 -/+ g_mu) (swapped for the adjoint), so they
// share rows 0 and 1 of the rebuild and differ by a sign in rows a0 and a1:
//   rows 0,1 = chi_f + chi_b,   rows a0,a1 = (unit of the forward hop) (chi_f - chi_b).
// Only the forward hop's two colour vectors (6 complex numbers) stay live
// while the backward hop loads, instead of a full 12-row accumulator.
template <int MU, int P, int LK, bool DAG, bool LNT, bool HALO = false>
__device__ __forceinline__ void hop_direction(const Geom &g, const char *__restrict__ in,
                                              const char *__restrict__ U, int p, int64_t s,
                                              const Coord &c, cplx<typename real_of<P>::type> acc[12],
                                              const char *const *face = nullptr) {
    using T = typename real_of<P>::type;
    using PR = Proj<MU>;
    constexpr int SF = DAG ? 1 : -1;
    constexpr int SB = -SF;
    constexpr int r0 = SF > 0 ? conj_code(PR::c0) : neg_code(conj_code(PR::c0));
    constexpr int r1 = SF > 0 ? conj_code(PR::c1) : neg_code(conj_code(PR::c1));
    // HALO (boundary-slice launches): a t-hop that crosses the t boundary
    // reads the face buffers instead of `in`
    constexpr bool TFACE = HALO && MU == 3;
    const bool face_f = TFACE && c.t == g.L[3] - 1;
    const bool face_b = TFACE && c.t == 0;
    bool flip_f, flip_b;
    const int64_t fwd = hop_neighbour<MU, true>(g, s, c, flip_f);
    const int64_t bwd = hop_neighbour<MU, false>(g, s, c, flip_b);
    cplx<T> f[6];
    if (face_f) {
        if constexpr (P == LQCD_F16) {
            v2h hr[6], hi[6], u[6];
            cplx<float> r2[3];
            float fac;
            load_face_forms(face[0], s - (int64_t)(g.L[3] - 1) * g.st, hr, hi, fac);
            load_link_h<LNT>(U, g.ntiles, p, s, MU, u, r2);
            half_mul_h<false>(hr, hi, u, r2, fac, f, f + 3);
        } else {
            cplx<T> h[6], u[9];
            load_face<T>(face[0], s - (int64_t)(g.L[3] - 1) * g.st, h);
            load_link<P, LK, LNT>(U, g.ntiles, p, s, MU, u);
            half_mul<false>(u, h, h + 3, f, f + 3);
        }
    } else {
        T sgn = flip_f ? T(-1) : T(1);
        cplx<typename hop_elem<P>::type> psi[12];
        load_spinor_hop<P>(in, fwd, psi, sgn);
        link_chi<MU, SF, false, P, LK, LNT>(U, g.ntiles, p, s, psi, sgn, f, f + 3);
    }
    hop_fence<T, 6>(f);
    {
        // binary16: the backward colour vectors stay unscaled and the
        // neighbour's factor enters the sums as an FMA
        cplx<T> b[6];
        T fb = T(1);
        if (face_b) {
            if constexpr (P == LQCD_F16) load_face_h(face[1], s, b, fb);
            else load_face<T>(face[1], s, b);
        } else {
            T sgn = flip_b ? T(-1) : T(1);
            cplx<typename hop_elem<P>::type> psi[12];
            load_spinor_hop<P>(in, bwd, psi, sgn);
            link_chi<MU, SB, true, P, LK, LNT, P != LQCD_F16>(U, g.ntiles, p ^ 1, bwd, psi, sgn, b, b + 3);
            if constexpr (P == LQCD_F16) fb = sgn;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if constexpr (P == LQCD_F16) {
                const cplx<T> s0 = {fmaf(fb, b[a].re, f[a].re), fmaf(fb, b[a].im, f[a].im)};
                const cplx<T> s1 = {fmaf(fb, b[3 + a].re, f[3 + a].re), fmaf(fb, b[3 + a].im, f[3 + a].im)};
                const cplx<T> d0 = {fmaf(-fb, b[a].re, f[a].re), fmaf(-fb, b[a].im, f[a].im)};
                const cplx<T> d1 = {fmaf(-fb, b[3 + a].re, f[3 + a].re), fmaf(-fb, b[3 + a].im, f[3 + a].im)};
                acc[a] = s0;
                acc[3 + a] = s1;
                acc[PR::a0 * 3 + a] = mul_unit<r0>(d0);
                acc[PR::a1 * 3 + a] = mul_unit<r1>(d1);
            } else {
                acc[a] = f[a] + b[a];
                acc[3 + a] = f[3 + a] + b[3 + a];
                acc[PR::a0 * 3 + a] = mul_unit<r0>(f[a] - b[a]);
                acc[PR::a1 * 3 + a] = mul_unit<r1>(f[3 + a] - b[3 + a]);
            }
        }
    }
    hop_fence<T, 12>(acc);
}

}  // namespace lqcd
