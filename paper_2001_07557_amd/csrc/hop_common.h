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
};

// Tile visited by logical block b (within one parity).  With bricks of bz
// z-groups the order is (z-brick, t, z-group in brick, tile in group): the
// three t-slices of a brick that one output slice touches stay in the XCD's L2,
// where the plain order would revisit each input slice from memory for the
// t-neighbours of the slices before and after it.
__device__ __forceinline__ int64_t brick_order(uint32_t b, const Brick &k) {
    const uint32_t r1 = fdiv(b, k.pt);   // (z-group, t) in traversal order
    const uint32_t r2 = fdiv(r1, k.bz);  // (brick, t)
    const uint32_t zc = fdiv(r2, k.lt);  // brick
    const uint32_t tile = b - r1 * k.pt.d;
    const uint32_t zi = r1 - r2 * k.bz.d;
    const uint32_t t = k.t0 + (r2 - zc * k.lt.d) * k.tstep;
    return (int64_t)((t * k.lz + zc * k.bz.d + zi) * k.pt.d + tile);
}

__device__ __forceinline__ int64_t brick_tile(const HopArgs &a, uint32_t b) {
    return brick_order(b, a.brick);
}

// Blocked traversal plan: the tiles of a z-group (the fewest consecutive
// z-planes whose sites fill whole tiles, usually one plane) form a unit; a
// brick is bz z-groups and all t.  bz = 0: plain order.
struct BrickPlan {
    int pt;  // tiles per z-group
    int bz;  // z-groups per brick
    int lz;  // z-groups in Lz
};

// See the rules next to LQCD_BRICK_MODE.  Rule 1 cuts Lz into 8 bricks (one
// per XCD), or into 4 when the z-groups do not divide by 8 (two XCDs then
// share a brick, each taking half of its t range).
inline BrickPlan brick_plan(const Geom &g, int prec) {
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
    } else {
        k.pt = make_fastdiv((uint32_t)b.pt);
        k.bz = make_fastdiv((uint32_t)b.bz);
        k.lt = make_fastdiv((uint32_t)g.L[3]);
        k.lz = b.lz;
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

// a + k b for a unit k (code as for mul_unit) in the arithmetic type T, from
// inputs of element type E, as fused multiply-adds by +-one (exact).  With
// binary16 inputs each component is one mixed-precision FMA that reads the
// stored halves directly; `one` must then be a register value the compiler
// cannot see is 1, or it turns the FMA back into an addition of two
// converted values.
template <int K, typename T, typename E>
__device__ __forceinline__ cplx<T> add_unit(cplx<E> a, cplx<E> b, T one) {
    const T ar = (T)a.re, ai = (T)a.im, br = (T)b.re, bi = (T)b.im;
    if constexpr (K == 0) return {fmad(br, one, ar), fmad(bi, one, ai)};
    else if constexpr (K == 1) return {fmad(br, -one, ar), fmad(bi, -one, ai)};
    else if constexpr (K == 2) return {fmad(bi, -one, ar), fmad(br, one, ai)};
    else return {fmad(bi, one, ar), fmad(br, -one, ai)};
}

// Project with (1 + S g_mu) and apply the boundary sign: rows 0 and 1 of the
// half-spinor of one hop.
template <int MU, int S, typename T, typename E>
__device__ __forceinline__ void hop_half(const cplx<E> psi[12], T sign, cplx<T> h0[3],
                                         cplx<T> h1[3]) {
    using PR = Proj<MU>;
    constexpr int k0 = S > 0 ? PR::c0 : neg_code(PR::c0);
    constexpr int k1 = S > 0 ? PR::c1 : neg_code(PR::c1);
    T one = 1;
    if constexpr (sizeof(E) == 2) asm volatile("" : "+v"(one));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h0[c] = scale(sign, add_unit<k0, T>(psi[c], psi[PR::a0 * 3 + c], one));
        h1[c] = scale(sign, add_unit<k1, T>(psi[3 + c], psi[PR::a1 * 3 + c], one));
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

// Project with (1 + S g_mu), apply the boundary sign and multiply by U (or
// U^dag): the two colour vectors chi0, chi1 of one hop.
template <int MU, int S, bool UDAG, typename T, typename E>
__device__ __forceinline__ void hop_chi(const cplx<E> psi[12], const cplx<T> u[9], T sign,
                                        cplx<T> x0[3], cplx<T> x1[3]) {
    cplx<T> h0[3], h1[3];
    hop_half<MU, S>(psi, sign, h0, h1);
    half_mul<UDAG>(u, h0, h1, x0, x1);
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

// Bytes of one face buffer (one t-slice of one parity) for storage precision prec.
inline size_t face_bytes(const Geom &g, int prec) {
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
            cplx<T> h[6];
            load_face<T>(face[FWD ? 0 : 1], FWD ? s - (int64_t)(g.L[3] - 1) * g.st : s, h);
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
    cplx<T> u[9];
    T sgn = flip ? T(-1) : T(1);
    load_spinor_hop<P>(in, nb, psi, sgn);
    if constexpr (FWD) load_link<P, LK, LNT>(U, g.ntiles, p, s, MU, u);
    else load_link<P, LK, LNT>(U, g.ntiles, p ^ 1, nb, MU, u);
    hop_chi<MU, S, !FWD>(psi, u, sgn, x0, x1);
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
        cplx<T> h[6], u[9];
        load_face<T>(face[0], s - (int64_t)(g.L[3] - 1) * g.st, h);
        load_link<P, LK, LNT>(U, g.ntiles, p, s, MU, u);
        half_mul<false>(u, h, h + 3, f, f + 3);
    } else {
        T sgn = flip_f ? T(-1) : T(1);
        cplx<typename hop_elem<P>::type> psi[12];
        cplx<T> u[9];
        load_spinor_hop<P>(in, fwd, psi, sgn);
        load_link<P, LK, LNT>(U, g.ntiles, p, s, MU, u);
        hop_chi<MU, SF, false>(psi, u, sgn, f, f + 3);
    }
    hop_fence<T, 6>(f);
    {
        cplx<T> b[6];
        if (face_b) {
            load_face<T>(face[1], s, b);
        } else {
            T sgn = flip_b ? T(-1) : T(1);
            cplx<typename hop_elem<P>::type> psi[12];
            cplx<T> u[9];
            load_spinor_hop<P>(in, bwd, psi, sgn);
            load_link<P, LK, LNT>(U, g.ntiles, p ^ 1, bwd, MU, u);
            hop_chi<MU, SB, true>(psi, u, sgn, b, b + 3);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc[a] = f[a] + b[a];
            acc[3 + a] = f[3 + a] + b[3 + a];
            acc[PR::a0 * 3 + a] = mul_unit<r0>(f[a] - b[a]);
            acc[PR::a1 * 3 + a] = mul_unit<r1>(f[3 + a] - b[3 + a]);
        }
    }
    hop_fence<T, 12>(acc);
}

}  // namespace lqcd
