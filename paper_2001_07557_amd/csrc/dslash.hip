// Wilson hopping term on gfx950: one thread per output site, eight
// neighbour hops with spin projection to half-spinors, SU(3) x half-spinor
// products and reconstruction into the four spin rows, boundary signs applied
// in the kernel, fused alpha*D + beta*y epilogue and an optional fused |out|^2
// block partial for the solver.
//
// The operator is the one the paper benchmarks in Sec. 3.3 (Fig. 4d); its
// definition (hopping form, DeGrand-Rossi basis) is spelled out in lqcd.h.
// The paper's kernels vectorise over sites packed into long vector registers
// (Sec. 3.1) and need lane permutations at sublattice boundaries; here each
// lane owns one site and neighbours are plain indexed loads, so no lane
// permutation exists.

#include "lqcd_internal.h"
#include "reduce.h"
#include "hop_common.h"

namespace lqcd {

// Cache hints of the hop kernels:
//  * output stores are non-temporal: the output is not read again by the same
//    launch, and a later launch reads it on other XCDs, whose L2s do not
//    share it, so keeping it in this XCD's L2 only evicts the neighbour
//    spinors held there for reuse;
//  * link loads are non-temporal when the links plus the input spinor exceed
//    the 256 MB Infinity Cache in front of HBM; when they fit, plain loads
//    leave them cached for the next application.  A launch over both
//    parities uses every link twice and always loads them plainly (48^3x96
//    full-lattice M, FP32-18: 4.4 -> 5.1 TB/s).
// Measured (fraction of 8 TB/s, alternating D_eo / D_oe): streaming the
// output takes FP64-18 from 67.0 to 78.3 at 32^4 and from 64.0 to 68.6 at
// 48^3x96; cached rather than streamed links take FP32-12 from 75.4 to 83.9
// at 32^4 (201 MB of links) and FP64-18 from 56.6 to 66.7 at 16^4.  The same
// hint on the spinor loads would destroy the L2 reuse (LQCD_SPINOR_NT,
// FP64-18 at 32^4: 51%).  LQCD_OUT_NT / LQCD_LINK_NT = 0 switch a hint off,
// LQCD_HOP_STREAM = 0..3 forces the mode (ablations).
#ifndef LQCD_HOP_STREAM
#define LQCD_HOP_STREAM -1
#endif
// row-parallel rebuild of the FP32 hop on small lattices (ablation switch)
#ifndef LQCD_HOP_ROWS
#define LQCD_HOP_ROWS 1
#endif
// both-parity launches pair the even and odd tile of a region (ablation switch)
#ifndef LQCD_HOP_ARGS_TOUCH
#define LQCD_HOP_ARGS_TOUCH 1
#endif
#ifndef LQCD_HOP_PAIRED
#define LQCD_HOP_PAIRED 1
#endif
// Blocks in flight of the FP64 4-way kernel on large lattices.  With ~120
// VGPRs four blocks fit a CU, so an XCD's 32 CUs keep 128 tiles in flight,
// more than one t-slice of its z-slab, and the three input t-slices the
// brick order relies on no longer fit its 4 MB L2 beside them.  From
// V/2 >= 2^20 sites (48^3x96 and up) the launch adds LQCD_HOP_F64_LDS_EXTRA
// bytes of dynamic LDS per block (36 + 18 KB: two blocks per CU).  Measured
// in two sessions (fraction of 8 TB/s, four -> two blocks per CU): 48^3x96
// FP64-18 68.6 -> 70.7 and 68.6 -> 69.5, FP64-12 65.6 -> 67.7 and 65.5 ->
// 67.1, full-lattice FP64-18 M 4.39 -> 4.88 TB/s; at 32^4 FP64-18 78.4 ->
// 79.8 and 78.3 -> 77.9, FP64-12 73.9 -> 72.7 and 73.8 -> 73.0 (not taken);
// three blocks per CU +0.6 at 48^3x96, one block 57%; binary16 storage
// (also 4-way) loses 8 points with it and keeps four.  A both-parity launch
// (full-lattice D_hop and M) keeps two tiles' links and both halves of psi
// in play and takes the limit from V/2 >= 2^17: full-lattice FP64-18 M at
// 24^4 4.82 -> 5.15 TB/s and at 32^4 4.67-4.73 -> 4.74-4.91 TB/s (two runs
// each).  LQCD_HOP_EXTRA_LDS forces a value for every 4-way launch
// (ablations).
#ifndef LQCD_HOP_F64_LDS_EXTRA
#define LQCD_HOP_F64_LDS_EXTRA 18432
#endif
#ifndef LQCD_HOP_F64_LDS_MIN_LOG2
#define LQCD_HOP_F64_LDS_MIN_LOG2 20
#endif
#ifndef LQCD_HOP_F64_PAIRED_LDS_MIN_LOG2
#define LQCD_HOP_F64_PAIRED_LDS_MIN_LOG2 17
#endif
#ifndef LQCD_HOP_EXTRA_LDS
#define LQCD_HOP_EXTRA_LDS -1
#endif
// t-march form of the 4-way shape: t-slices per block (0 = off), used from
// V/2 >= 2^LQCD_HOP_TMARCH_MIN_LOG2 sites
#ifndef LQCD_HOP_TMARCH
#define LQCD_HOP_TMARCH 0
#endif
#ifndef LQCD_HOP_TMARCH_MIN_LOG2
#define LQCD_HOP_TMARCH_MIN_LOG2 17
#endif
constexpr int64_t INFINITY_CACHE_BYTES = (int64_t)256 << 20;

// Epilogue shared by the kernel shapes: out = alpha acc + beta y; NORM = 1
// also returns |out|^2 of the site; NORM = 2 (the solver's last hop, with a y
// term) stores nothing of out = A p but updates the CG iterate in place,
// x += c p and r -= c A p (c the device's CG alpha, r at a.out), and returns
// |r|^2 of the site.
template <int P, bool HASY, int NORM, bool NT>
__device__ __forceinline__ double hop_epilogue(const HopArgs &a, int p, int64_t s,
                                               cplx<typename real_of<P>::type> acc[12]) {
    using T = typename real_of<P>::type;
    const T alpha = (T)a.alpha;
    if constexpr (HASY) {
        cplx<T> y[12];
        load_spinor<P>(a.y[p], s, y);
        const T beta = (T)a.beta;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            acc[k] = {alpha * acc[k].re + beta * y[k].re, alpha * acc[k].im + beta * y[k].im};
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = scale(alpha, acc[k]);
    }
    if constexpr (NORM == 2 && P == LQCD_F64 && !LQCD_LAYOUT_AOS) {
        // FP64: four words of p, x and r at a time, so that the three
        // vectors are never live together (occupancy of the 4-way shape)
        const T c = (T)*a.cg_alpha;
        const int64_t toff = (s >> TILE_SHIFT) * spinor_tile_bytes(P);
        const int lane = (int)(s & (TILE - 1));
        v2d *xw = reinterpret_cast<v2d *>(a.cg_x + toff) + lane;
        v2d *rw = reinterpret_cast<v2d *>(a.out[p] + toff) + lane;
        const v2d *pw = reinterpret_cast<const v2d *>(a.cg_p + toff) + lane;
        T nr = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            cplx<T> vx[4], vr[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 4 * q + j;
                const v2d dp = pw[k * TILE], dx = xw[k * TILE], dr = rw[k * TILE];
                vx[j] = {dx.x + c * dp.x, dx.y + c * dp.y};
                vr[j] = {dr.x - c * acc[k].re, dr.y - c * acc[k].im};
                nr += norm2(vr[j]);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 4 * q + j;
                xw[k * TILE] = v2d{vx[j].re, vx[j].im};
                rw[k * TILE] = v2d{vr[j].re, vr[j].im};
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        return (double)nr;
    } else if constexpr (NORM == 2) {
        const T c = (T)*a.cg_alpha;
        cplx<T> vx[12], vr[12], vp[12];
        load_spinor<P>(a.cg_p, s, vp);
        load_spinor<P>(a.cg_x, s, vx);
        load_spinor<P>(a.out[p], s, vr);
        T nr = 0;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            vx[k] = {vx[k].re + c * vp[k].re, vx[k].im + c * vp[k].im};
            vr[k] = {vr[k].re - c * acc[k].re, vr[k].im - c * acc[k].im};
            nr += norm2(vr[k]);
        }
        store_spinor<P>(a.cg_x, s, vx);
        store_spinor<P>(a.out[p], s, vr);
        return (double)nr;
    }
    double nrm = 0.0;
    if constexpr (NORM == 1) {
        T t = 0;
#pragma unroll
        for (int k = 0; k < 12; ++k) t += norm2(acc[k]);
        nrm = (double)t;
    }
    store_spinor<P, NT>(a.out[p], s, acc);
    return nrm;
}

// The five fields read first lie on the five 64-byte lines of the arguments.
static_assert(offsetof(HopArgs, cg_x) <= 5 * 64 && sizeof(HopArgs) <= 6 * 64,
              "the fields read first span five lines, the CG-update fields a sixth");
static_assert(offsetof(HopArgs, bpp) / 64 == 0 &&
                  (offsetof(HopArgs, g) + offsetof(Geom, lxh)) / 64 == 1 &&
                  (offsetof(HopArgs, g) + offsetof(Geom, vh)) / 64 == 2 &&
                  offsetof(HopArgs, in) / 64 == 3 && offsetof(HopArgs, stream) / 64 == 4,
              "one touched field per line of the launch arguments");

// Output parity and checkerboard site of this thread (block = one 64-site
// tile).  A launch over both parities gives consecutive blocks the even and
// the odd tile of one region: each reads the links and spinors of the other,
// so both are fetched into the same XCD's L2 once.
__device__ __forceinline__ int64_t hop_site_index(const HopArgs &a, int lane, int &p, int64_t &blk) {
    // selects, not branches: every launch argument is read up front
#if LQCD_HOP_ARGS_TOUCH
    // one field from each 64-byte line of the arguments, needed before
    // anything else: the lines come in with one scalar-cache miss instead of
    // one after each dependent step
    asm volatile("" ::"s"(a.bpp), "s"(a.g.lxh), "s"(a.g.vh), "s"(a.in[0]), "s"(a.stream));
#endif
    const uint32_t bx = blockIdx.x;
    blk = LQCD_HOP_XCD ? xcd_block(bx, a.nblk) : (int64_t)bx;
    // paired: blocks 2i / 2i + 1 take the even / odd tile i; otherwise the
    // first bpp blocks take parity par0 and the rest the other parity
    const int q = blk >= a.bpp ? 1 : 0;
    const uint32_t lb = (uint32_t)(a.paired ? blk >> 1 : blk - q * a.bpp);
    p = a.paired ? (int)(blk & 1) : a.par0 ^ q;
    return brick_tile(a, lb) * HOP_SITES + lane;
}

// 4-way shape: wave w computes both hops of direction w; waves 1..3 leave
// their partial spinors in LDS and wave 0 adds them up.
template <int P, int LK, bool DAG, bool HASY, int NORM, int NTM, bool HALO>
__global__ __launch_bounds__(256) void hop4_kernel(HopArgs a) {
    using T = typename real_of<P>::type;
    __shared__ cplx<T> part[3][12][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    int p;
    int64_t blk;
    const int64_t s = hop_site_index(a, lane, p, blk);
    const Geom &g = a.g;
    const bool active = s < g.vh;
    // (coordinates of a padding site are never used, and s < 2^31 anyway)
    const Coord c = cb_coords(g, p, s);
    cplx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {0, 0};
    if (active) {
        constexpr bool LNT = (NTM & 2) != 0;
        switch (w) {
            case 0: hop_direction<0, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, acc); break;
            case 1: hop_direction<1, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, acc); break;
            case 2: hop_direction<2, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, acc); break;
            default: hop_direction<3, P, LK, DAG, LNT, HALO>(g, a.in[p], a.U, p, s, c, acc, a.face); break;
        }
    }
    if (w > 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) part[w - 1][k][lane] = acc[k];
    }
    __syncthreads();
    double nrm[1] = {0.0};
    if (w == 0 && active) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = acc[k] + part[j][k][lane];
        nrm[0] = hop_epilogue<P, HASY, NORM, (NTM & 1) != 0>(a, p, s, acc);
    }
    if constexpr (NORM) {
        // wave 0 holds every site of the tile: a wave reduction suffices and
        // the other waves leave after the staging barrier
        if (w == 0) {
            const double t = wave_sum(nrm[0]);
            if (lane == 0) a.partial[blk] = t;
        }
    }
}

// t-march form of the 4-way shape (LQCD_HOP_TMARCH = t-slices per block):
// a block walks one tile column, the same 64 in-slice sites of tseg
// consecutive t-slices.  The t-neighbours of a tile are the same lanes of
// the tiles one slice up and one down, so the wave of direction t loads each
// input t-slice of its column once: the load of input slice t + 1 gives the
// forward hop of output slice t and the backward hop of output slice t + 2,
// whose two colour vectors wait two steps in a lane-private LDS ring (the
// 4-way form loads that input again two output slices later, from the L2
// if it is still there).  Waves 0-2 read their neighbours as in the 4-way
// shape; XCD x of 8 takes columns [x K/8, (x + 1) K/8) of every segment, so
// the blocks of one XCD walk its z-slab side by side.  Same arithmetic, in
// the same order, as the 4-way shape: the results are bit-identical.
template <int P, int LK, bool DAG, bool HASY, int NORM, int NTM>
__global__ __launch_bounds__(256) void hop4t_kernel(HopArgs a) {
    using T = typename real_of<P>::type;
    using E = typename hop_elem<P>::type;
    using PR = Proj<3>;
    constexpr bool LNT = (NTM & 2) != 0;
    constexpr int SF = DAG ? 1 : -1;
    constexpr int SB = -SF;
    constexpr int r0 = SF > 0 ? conj_code(PR::c0) : neg_code(conj_code(PR::c0));
    constexpr int r1 = SF > 0 ? conj_code(PR::c1) : neg_code(conj_code(PR::c1));
    __shared__ cplx<T> part[3][12][64];
    __shared__ cplx<T> ring[2][6][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const Geom &g = a.g;
    const int p = a.par0;
    const int lt = g.L[3];
    const uint32_t kx = (uint32_t)(g.st >> TILE_SHIFT) / 8;  // columns per XCD
    const uint32_t b = blockIdx.x;
    const uint32_t j = b >> 3;
    const uint32_t seg = j / kx;
    const uint32_t col = (b & 7) * kx + (j - seg * kx);
    const int t0 = (int)seg * a.tseg;
    const int t1 = t0 + a.tseg < lt ? t0 + a.tseg : lt;
    const int64_t s0 = (int64_t)col * TILE + lane;  // this lane's site of slice 0
    const char *in = a.in[p];
    // backward t-hop of output slice t from input slice t - 1 (wrapping, with
    // the boundary sign), as the 4-way shape forms it
    auto bwd_half = [&](int t, cplx<T> bh[6]) {
        const bool wrap = t == 0;
        const int64_t nb = (int64_t)(wrap ? lt - 1 : t - 1) * g.st + s0;
        T sgn = wrap && g.bc[3] < 0 ? T(-1) : T(1);
        cplx<E> psi[12];
        load_spinor_hop<P>(in, nb, psi, sgn);
        link_chi<3, SB, true, P, LK, LNT>(a.U, g.ntiles, p ^ 1, nb, psi, sgn, bh, bh + 3);
    };
    if (w == 3) {
        for (int t = t0; t < t0 + 2 && t < t1; ++t) {
            cplx<T> bh[6];
            bwd_half(t, bh);
#pragma unroll
            for (int k = 0; k < 6; ++k) ring[t & 1][k][lane] = bh[k];
        }
    }
    for (int t = t0; t < t1; ++t) {
        const int64_t s = (int64_t)t * g.st + s0;
        const Coord c = cb_coords(g, p, s);
        cplx<T> acc[12];
        switch (w) {
            case 0: hop_direction<0, P, LK, DAG, LNT>(g, in, a.U, p, s, c, acc); break;
            case 1: hop_direction<1, P, LK, DAG, LNT>(g, in, a.U, p, s, c, acc); break;
            case 2: hop_direction<2, P, LK, DAG, LNT>(g, in, a.U, p, s, c, acc); break;
            default: {
                // forward hop: input slice t + 1 (wrapping), link U_t(s)
                const bool wrap = t == lt - 1;
                const int64_t nb = (int64_t)(wrap ? 0 : t + 1) * g.st + s0;
                T sgn = wrap && g.bc[3] < 0 ? T(-1) : T(1);
                cplx<E> psi[12];
                cplx<T> f[6];
                load_spinor_hop<P>(in, nb, psi, sgn);
                link_chi<3, SF, false, P, LK, LNT>(a.U, g.ntiles, p, s, psi, sgn, f, f + 3);
                hop_fence<T, 6>(f);
                cplx<T> bh[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) bh[k] = ring[t & 1][k][lane];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    acc[q] = f[q] + bh[q];
                    acc[3 + q] = f[3 + q] + bh[3 + q];
                    acc[PR::a0 * 3 + q] = mul_unit<r0>(f[q] - bh[q]);
                    acc[PR::a1 * 3 + q] = mul_unit<r1>(f[3 + q] - bh[3 + q]);
                }
                hop_fence<T, 12>(acc);
                // the same input gives the backward hop of output slice t + 2
                // (never across the boundary inside a segment, so the sign
                // factor is the forward hop's: 1, times the binary16 scale)
                if (t + 2 < t1) {
                    link_chi<3, SB, true, P, LK, LNT>(a.U, g.ntiles, p ^ 1, nb, psi, sgn, bh, bh + 3);
#pragma unroll
                    for (int k = 0; k < 6; ++k) ring[t & 1][k][lane] = bh[k];
                }
            }
        }
        __syncthreads();  // wave 0 has read the partials of the step before
        if (w > 0) {
#pragma unroll
            for (int k = 0; k < 12; ++k) part[w - 1][k][lane] = acc[k];
        }
        __syncthreads();
        if (w == 0) {
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = acc[k] + part[q][k][lane];
            const double nrm = hop_epilogue<P, HASY, NORM, (NTM & 1) != 0>(a, p, s, acc);
            if constexpr (NORM != 0) {
                const double tot = wave_sum(nrm);
                if (lane == 0) a.partial[s >> TILE_SHIFT] = tot;
            }
        }
    }
}

// 1-way shape (ablation builds, LQCD_HOP_SHAPE_* = 1): one wave per block,
// every thread computes all eight hops of its site in registers, no LDS.
// The four directions are added in the 4-way shape's order.
template <int P, int LK, bool DAG, bool HASY, int NORM, int NTM, bool HALO>
__global__ __launch_bounds__(64) void hop1_kernel(HopArgs a) {
    using T = typename real_of<P>::type;
    const int lane = threadIdx.x & 63;
    int p;
    int64_t blk;
    const int64_t s = hop_site_index(a, lane, p, blk);
    const Geom &g = a.g;
    const bool active = s < g.vh;
    const Coord c = cb_coords(g, p, s);
    cplx<T> acc[12], d[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {0, 0};
    double nrm[1] = {0.0};
    if (active) {
        constexpr bool LNT = (NTM & 2) != 0;
        hop_direction<0, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, acc);
        hop_direction<1, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, d);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = acc[k] + d[k];
        hop_direction<2, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, d);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = acc[k] + d[k];
        hop_direction<3, P, LK, DAG, LNT, HALO>(g, a.in[p], a.U, p, s, c, d, a.face);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = acc[k] + d[k];
        nrm[0] = hop_epilogue<P, HASY, NORM, (NTM & 1) != 0>(a, p, s, acc);
    }
    if constexpr (NORM) {
        const double t = wave_sum(nrm[0]);
        if (lane == 0) a.partial[blk] = t;
    }
}

template <int H, int P, bool DAG>
__device__ __forceinline__ void add_staged(const cplx<typename real_of<P>::type> (*chi)[6][64],
                                           int lane, cplx<typename real_of<P>::type> acc[12]) {
    using T = typename real_of<P>::type;
    cplx<T> x0[3], x1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        x0[a] = chi[H][a][lane];
        x1[a] = chi[H][3 + a][lane];
    }
    chi_accumulate<H / 2, HopSign<H, DAG>::value>(x0, x1, acc);
}

// Spin row R of the output from the eight staged half-spinors: every hop
// adds its chi0 to row 0, its chi1 to row 1 and a unit times one of them to
// row a0 or a1 of its direction.
template <int R, int H, int P, bool DAG>
__device__ __forceinline__ void row_staged(const cplx<typename real_of<P>::type> (*chi)[6][64],
                                           int lane, cplx<typename real_of<P>::type> row[3]) {
    using PR = Proj<H / 2>;
    constexpr int S = HopSign<H, DAG>::value;
    constexpr int r0 = S > 0 ? conj_code(PR::c0) : neg_code(conj_code(PR::c0));
    constexpr int r1 = S > 0 ? conj_code(PR::c1) : neg_code(conj_code(PR::c1));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (R == 0) row[a] = row[a] + chi[H][a][lane];
        else if constexpr (R == 1) row[a] = row[a] + chi[H][3 + a][lane];
        else if constexpr (R == PR::a0) row[a] = row[a] + mul_unit<r0>(chi[H][a][lane]);
        else row[a] = row[a] + mul_unit<r1>(chi[H][3 + a][lane]);
    }
}

// Row-parallel rebuild (FP32 storage, out = alpha D in): wave R builds and
// stores spin row R, i.e. complexes 3R .. 3R + 2 of the site, which straddle
// the 16-byte words of the tile, so they are stored as three 8-byte halves.
template <int R, int P, bool DAG, bool NT>
__device__ __forceinline__ void rebuild_row(const HopArgs &a, int p, int64_t s,
                                            const cplx<typename real_of<P>::type> (*chi)[6][64],
                                            int lane) {
    static_assert(P == LQCD_F32, "row stores assume the FP32 tile layout");
    using T = typename real_of<P>::type;
    cplx<T> row[3] = {{0, 0}, {0, 0}, {0, 0}};
    row_staged<R, 0, P, DAG>(chi, lane, row);
    row_staged<R, 1, P, DAG>(chi, lane, row);
    row_staged<R, 2, P, DAG>(chi, lane, row);
    row_staged<R, 3, P, DAG>(chi, lane, row);
    row_staged<R, 4, P, DAG>(chi, lane, row);
    row_staged<R, 5, P, DAG>(chi, lane, row);
    row_staged<R, 6, P, DAG>(chi, lane, row);
    row_staged<R, 7, P, DAG>(chi, lane, row);
    const T alpha = (T)a.alpha;
    char *t = a.out[p] + (s >> TILE_SHIFT) * spinor_tile_bytes(P) + (s & (TILE - 1)) * WORD;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int c = 3 * R + k;
        v2f *d = reinterpret_cast<v2f *>(t + (c / 2) * TILE * WORD + (c % 2) * 8);
        put<NT>(d, v2f{alpha * row[k].re, alpha * row[k].im});
    }
}

// 8-way shape: wave w computes hop w (direction w/2, forward for even w) and
// stages the two colour vectors of its multiplied half-spinor in LDS; wave 0
// rebuilds the four spin rows from the eight staged half-spinors.
template <int P, int LK, bool DAG, bool HASY, int NORM, int NTM, bool ROWS, bool HALO>
__global__ __launch_bounds__(512) void hop8_kernel(HopArgs a) {
    using T = typename real_of<P>::type;
    __shared__ cplx<T> chi[8][6][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    int p;
    int64_t blk;
    const int64_t s = hop_site_index(a, lane, p, blk);
    const Geom &g = a.g;
    const bool active = s < g.vh;
    // (coordinates of a padding site are never used, and s < 2^31 anyway)
    const Coord c = cb_coords(g, p, s);
    if (active) {
        cplx<T> x0[3], x1[3];
        constexpr bool LNT = (NTM & 2) != 0;
        switch (w) {
            case 0: hop_single<0, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, x0, x1); break;
            case 1: hop_single<1, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, x0, x1); break;
            case 2: hop_single<2, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, x0, x1); break;
            case 3: hop_single<3, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, x0, x1); break;
            case 4: hop_single<4, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, x0, x1); break;
            case 5: hop_single<5, P, LK, DAG, LNT>(g, a.in[p], a.U, p, s, c, x0, x1); break;
            case 6: hop_single<6, P, LK, DAG, LNT, HALO>(g, a.in[p], a.U, p, s, c, x0, x1, a.face); break;
            default: hop_single<7, P, LK, DAG, LNT, HALO>(g, a.in[p], a.U, p, s, c, x0, x1, a.face); break;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            chi[w][k][lane] = x0[k];
            chi[w][3 + k][lane] = x1[k];
        }
    }
    __syncthreads();
    if constexpr (ROWS) {
        static_assert(!HASY && !NORM, "the row-parallel rebuild has no y term and no norm");
        if (active) {
            switch (w) {
                case 0: rebuild_row<0, P, DAG, (NTM & 1) != 0>(a, p, s, chi, lane); break;
                case 1: rebuild_row<1, P, DAG, (NTM & 1) != 0>(a, p, s, chi, lane); break;
                case 2: rebuild_row<2, P, DAG, (NTM & 1) != 0>(a, p, s, chi, lane); break;
                case 3: rebuild_row<3, P, DAG, (NTM & 1) != 0>(a, p, s, chi, lane); break;
                default: break;
            }
        }
        return;
    }
    double nrm[1] = {0.0};
    if (w == 0 && active) {
        cplx<T> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {0, 0};
        add_staged<0, P, DAG>(chi, lane, acc);
        add_staged<1, P, DAG>(chi, lane, acc);
        add_staged<2, P, DAG>(chi, lane, acc);
        add_staged<3, P, DAG>(chi, lane, acc);
        add_staged<4, P, DAG>(chi, lane, acc);
        add_staged<5, P, DAG>(chi, lane, acc);
        add_staged<6, P, DAG>(chi, lane, acc);
        add_staged<7, P, DAG>(chi, lane, acc);
        nrm[0] = hop_epilogue<P, HASY, NORM, (NTM & 1) != 0>(a, p, s, acc);
    }
    if constexpr (NORM) {
        // wave 0 holds every site of the tile: a wave reduction suffices and
        // the other waves leave after the staging barrier
        if (w == 0) {
            const double t = wave_sum(nrm[0]);
            if (lane == 0) a.partial[blk] = t;
        }
    }
}

constexpr int hop_shape(int prec) {
    return prec == LQCD_F64 ? LQCD_HOP_SHAPE_F64 : prec == LQCD_F32 ? LQCD_HOP_SHAPE_F32
                                                                     : LQCD_HOP_SHAPE_F16;
}

template <int P, int LK, bool DAG, bool HASY, int NORM, int NTM, bool HALO>
static void launch_halo(const HopArgs &a, dim3 grid, hipStream_t st) {
    if constexpr (hop_shape(P) == 1) {
        hop1_kernel<P, LK, DAG, HASY, NORM, NTM, HALO><<<grid, 64, 0, st>>>(a);
    } else if constexpr (hop_shape(P) == 8) {
        if constexpr (P == LQCD_F32 && !HASY && !NORM) {
            if (a.rows) {
                hop8_kernel<P, LK, DAG, HASY, NORM, NTM, true, HALO><<<grid, 512, 0, st>>>(a);
                return;
            }
        }
        hop8_kernel<P, LK, DAG, HASY, NORM, NTM, false, HALO><<<grid, 512, 0, st>>>(a);
    } else {
        if constexpr (!HALO && LQCD_HOP_TMARCH > 0) {
            if (a.tseg > 0) {
                hop4t_kernel<P, LK, DAG, HASY, NORM, NTM><<<grid, 256, a.lds_extra, st>>>(a);
                return;
            }
        }
        hop4_kernel<P, LK, DAG, HASY, NORM, NTM, HALO><<<grid, 256, a.lds_extra, st>>>(a);
    }
}

// Boundary-slice launches (faces given) have no norm partial; the face
// variants exist only for the other combinations.
template <int P, int LK, bool DAG, bool HASY, int NORM, int NTM>
static void launch_nt(const HopArgs &a, dim3 grid, hipStream_t st) {
    if constexpr (!NORM) {
        if (a.face[0] != nullptr) {
            launch_halo<P, LK, DAG, HASY, NORM, NTM, true>(a, grid, st);
            return;
        }
    }
    launch_halo<P, LK, DAG, HASY, NORM, NTM, false>(a, grid, st);
}

// The cache hints are template arguments: a run-time choice between two
// otherwise identical load or store sequences gets merged by the compiler,
// which then drops the hint.
template <int P, int LK, bool DAG, bool HASY, int NORM>
static void launch_shape(const HopArgs &a, dim3 grid, hipStream_t st) {
    switch (a.stream) {
        case 0: launch_nt<P, LK, DAG, HASY, NORM, 0>(a, grid, st); break;
        case 1: launch_nt<P, LK, DAG, HASY, NORM, 1>(a, grid, st); break;
        case 2: launch_nt<P, LK, DAG, HASY, NORM, 2>(a, grid, st); break;
        default: launch_nt<P, LK, DAG, HASY, NORM, 3>(a, grid, st); break;
    }
}

// norm: 0 none, 1 |out|^2 block partials, 2 CG update (needs the y term; the
// solver applies it on the adjoint hop only)
template <int P, int LK, bool DAG>
static void launch_p(const HopArgs &a, bool hasy, int norm, dim3 grid, hipStream_t st) {
    if (hasy) {
        if (norm == 1) launch_shape<P, LK, DAG, true, 1>(a, grid, st);
        else if constexpr (DAG) {
            if (norm == 2) launch_shape<P, LK, DAG, true, 2>(a, grid, st);
            else launch_shape<P, LK, DAG, true, 0>(a, grid, st);
        } else {
            launch_shape<P, LK, DAG, true, 0>(a, grid, st);
        }
    } else {
        if (norm == 1) launch_shape<P, LK, DAG, false, 1>(a, grid, st);
        else launch_shape<P, LK, DAG, false, 0>(a, grid, st);
    }
}

template <int P, int LK>
static void launch_l(const HopArgs &a, bool dag, bool hasy, int norm, dim3 grid, hipStream_t st) {
    if (dag) launch_p<P, LK, true>(a, hasy, norm, grid, st);
    else launch_p<P, LK, false>(a, hasy, norm, grid, st);
}

int hop_launch(const HopArgs &a0, int prec, int link, bool dag, int nparity, hipStream_t st,
               int region) {
    if (prec == LQCD_F16 && a0.g.ntiles > F16_MAX_TILES) return LQCD_EINVAL;
    HopArgs a = a0;
    if (region < 0) {
        a.bpp = (a.g.vh + HOP_SITES - 1) / HOP_SITES;
        a.brick = make_brick(a.g, brick_plan(a.g, prec,
                                             nparity == 2 && LQCD_HOP_PAIRED ? 2
                                             : nparity == 1 && LQCD_BRICK_BAND_EO ? 1 : 0));
        a.face[0] = a.face[1] = nullptr;
    } else {
        // interior slices 1 .. Lt-2, or boundary slices 0 and Lt-1
        const int lt = a.g.L[3];
        const int nt = region == 0 ? lt - 2 : 2;
        if (nt <= 0) return LQCD_OK;
        a.bpp = (int64_t)nt * (a.g.st / TILE);
        a.brick = make_region_brick(a.g, brick_plan(a.g, prec), region == 0 ? 1 : 0,
                                    region == 0 ? 1 : lt - 1, nt);
        if (region == 0) a.face[0] = a.face[1] = nullptr;
        nparity = 1;
    }
    a.paired = nparity == 2 && LQCD_HOP_PAIRED;
    // row-parallel rebuild only where a launch is latency-bound (V/2 < 2^17:
    // 16^4 and smaller); from 24^4 up the single-wave rebuild is 0.5-2.5
    // points faster
    a.rows = LQCD_HOP_ROWS && a.g.vh < ((int64_t)1 << 17) && a.y[0] == nullptr &&
             a.y[1] == nullptr && a.partial == nullptr && a.cg_x == nullptr;
    const int64_t spinors = (int64_t)(nparity * half_spinor_bytes(a.g, prec));
    const int64_t links = (int64_t)gauge_bytes(a.g, prec, link);
    const bool out_nt = OUT_NT;
    // a both-parity launch reads every link twice (forward from its own site,
    // backward from the paired tile), so it keeps them cached
    const bool link_nt = LQCD_LINK_NT && !a.paired && spinors + links > INFINITY_CACHE_BYTES;
    a.stream = LQCD_HOP_STREAM >= 0 ? LQCD_HOP_STREAM : (out_nt ? 1 : 0) | (link_nt ? 2 : 0);
    a.lds_extra = LQCD_HOP_EXTRA_LDS >= 0 ? (uint32_t)LQCD_HOP_EXTRA_LDS
                  : prec == LQCD_F64 && a.g.vh >= ((int64_t)1 << (a.paired ? LQCD_HOP_F64_PAIRED_LDS_MIN_LOG2
                                                                               : LQCD_HOP_F64_LDS_MIN_LOG2))
                      ? (uint32_t)LQCD_HOP_F64_LDS_EXTRA
                      : 0u;
    dim3 grid((unsigned)(a.bpp * nparity));
    // t-march launches (4-way shape, one parity, whole lattice, whole tiles
    // per t-slice in a multiple of 8 columns): one block per column and
    // segment of tseg slices
    a.tseg = 0;
    if (LQCD_HOP_TMARCH > 0 && hop_shape(prec) == 4 && nparity == 1 && region < 0 &&
        a.g.vh >= ((int64_t)1 << LQCD_HOP_TMARCH_MIN_LOG2) && a.g.st % TILE == 0 &&
        (a.g.st / TILE) % 8 == 0) {
        a.tseg = LQCD_HOP_TMARCH;
        const int64_t nseg = (a.g.L[3] + a.tseg - 1) / a.tseg;
        grid = dim3((unsigned)((a.g.st / TILE) * nseg));
        a.lds_extra = LQCD_HOP_EXTRA_LDS >= 0 ? (uint32_t)LQCD_HOP_EXTRA_LDS : 0u;
    }
    a.nblk = grid.x;
    const bool hasy = a.y[0] != nullptr || a.y[1] != nullptr;
    const int norm = a.cg_x != nullptr ? 2 : a.partial != nullptr ? 1 : 0;
    if (norm == 2 && (!hasy || !dag || !a.partial || !a.cg_p || !a.cg_alpha)) return LQCD_EINVAL;
    if (prec == LQCD_F64) {
        if (link == 18) launch_l<LQCD_F64, 18>(a, dag, hasy, norm, grid, st);
        else launch_l<LQCD_F64, 12>(a, dag, hasy, norm, grid, st);
    } else if (prec == LQCD_F32) {
        if (link == 18) launch_l<LQCD_F32, 18>(a, dag, hasy, norm, grid, st);
        else launch_l<LQCD_F32, 12>(a, dag, hasy, norm, grid, st);
    } else {
        launch_l<LQCD_F16, 12>(a, dag, hasy, norm, grid, st);
    }
    return check_launch();
}

int64_t hop_partials(const Geom &g, int nparity) {
    return ((g.vh + HOP_SITES - 1) / HOP_SITES) * nparity;
}

}  // namespace lqcd

using namespace lqcd;

static int validate_hop(const lqcd_geom_t *gg, Geom *g, const void *out, const void *in,
                        const void *U, int prec, int link) {
    if (!make_geom(gg, g)) return LQCD_EINVAL;
    if (!valid_link(prec, link)) return LQCD_EINVAL;
    if (!out || !in || !U) return LQCD_EINVAL;
    if (((uintptr_t)out | (uintptr_t)in | (uintptr_t)U) & 15) return LQCD_EINVAL;
    if (out == in) return LQCD_EINVAL;
    return LQCD_OK;
}

static int full_hop(const lqcd_geom_t *gg, void *out, const void *in, const void *y, const void *U,
                    double alpha, double beta, int prec, int link, bool dag, void *stream) {
    Geom g;
    int rc = validate_hop(gg, &g, out, in, U, prec, link);
    if (rc) return rc;
    if (y && ((uintptr_t)y & 15)) return LQCD_EINVAL;
    const size_t hb = half_spinor_bytes(g, prec);
    HopArgs a{};
    a.g = g;
    a.U = (const char *)U;
    a.alpha = alpha;
    a.beta = beta;
    a.par0 = 0;
    // output parity p reads the other parity's half of the input
    a.out[0] = (char *)out;
    a.out[1] = (char *)out + hb;
    a.in[0] = (const char *)in + hb;
    a.in[1] = (const char *)in;
    a.y[0] = y ? (const char *)y : nullptr;
    a.y[1] = y ? (const char *)y + hb : nullptr;
    a.partial = nullptr;
    return hop_launch(a, prec, link, dag, 2, (hipStream_t)stream);
}

extern "C" int lqcd_dslash(const lqcd_geom_t *g, void *out, const void *in, const void *y,
                           const void *U, double alpha, double beta, int prec, int link,
                           void *stream) {
    return full_hop(g, out, in, y, U, alpha, beta, prec, link, false, stream);
}

extern "C" int lqcd_dslash_dagger(const lqcd_geom_t *g, void *out, const void *in,
                                  const void *y, const void *U, double alpha, double beta,
                                  int prec, int link, void *stream) {
    return full_hop(g, out, in, y, U, alpha, beta, prec, link, true, stream);
}

static int eo_hop(const lqcd_geom_t *gg, int out_par, void *out, const void *in, const void *y,
                  const void *U, double alpha, double beta, int dagger, int prec, int link,
                  void *stream) {
    Geom g;
    int rc = validate_hop(gg, &g, out, in, U, prec, link);
    if (rc) return rc;
    if (y && ((uintptr_t)y & 15)) return LQCD_EINVAL;
    HopArgs a{};
    a.g = g;
    a.U = (const char *)U;
    a.alpha = alpha;
    a.beta = beta;
    a.par0 = out_par;
    a.out[out_par] = (char *)out;
    a.in[out_par] = (const char *)in;
    a.y[out_par] = (const char *)y;
    a.partial = nullptr;
    return hop_launch(a, prec, link, dagger != 0, 1, (hipStream_t)stream);
}

extern "C" int lqcd_meo(const lqcd_geom_t *g, void *out_e, const void *in_o, const void *y_e,
                        const void *U, double alpha, double beta, int dagger, int prec, int link,
                        void *stream) {
    return eo_hop(g, LQCD_EVEN, out_e, in_o, y_e, U, alpha, beta, dagger, prec, link, stream);
}

extern "C" int lqcd_moe(const lqcd_geom_t *g, void *out_o, const void *in_e, const void *y_o,
                        const void *U, double alpha, double beta, int dagger, int prec, int link,
                        void *stream) {
    return eo_hop(g, LQCD_ODD, out_o, in_e, y_o, U, alpha, beta, dagger, prec, link, stream);
}

extern "C" int lqcd_hop_region(const lqcd_geom_t *gg, int out_par, int region, void *out,
                               const void *in, const void *y, const void *U,
                               const void *face_fwd, const void *face_bwd, double alpha,
                               double beta, int dagger, int prec, int link, void *stream) {
    Geom g;
    int rc = validate_hop(gg, &g, out, in, U, prec, link);
    if (rc) return rc;
    if (out_par != LQCD_EVEN && out_par != LQCD_ODD) return LQCD_EINVAL;
    if (region != 0 && region != 1) return LQCD_EINVAL;
    if (g.st % TILE != 0) return LQCD_EINVAL;  // t-slices must be whole tiles
    if (y && ((uintptr_t)y & 15)) return LQCD_EINVAL;
    if (region == 1 && (!face_fwd || !face_bwd || (((uintptr_t)face_fwd | (uintptr_t)face_bwd) & 15)))
        return LQCD_EINVAL;
    HopArgs a{};
    a.g = g;
    a.U = (const char *)U;
    a.alpha = alpha;
    a.beta = beta;
    a.par0 = out_par;
    a.out[out_par] = (char *)out;
    a.in[out_par] = (const char *)in;
    a.y[out_par] = (const char *)y;
    a.partial = nullptr;
    a.face[0] = (const char *)face_fwd;
    a.face[1] = (const char *)face_bwd;
    return hop_launch(a, prec, link, dagger != 0, 1, (hipStream_t)stream, region);
}

extern "C" int lqcd_mhat(const lqcd_geom_t *g, void *out_e, const void *in_e, void *tmp_o,
                         const void *U, double kappa, int dagger, int prec, int link,
                         void *stream) {
    if (!tmp_o || tmp_o == in_e || tmp_o == out_e) return LQCD_EINVAL;
    // Mhat      = 1 - k^2 D_eo D_oe:              tmp = D_oe in,        out = in - k^2 D_eo tmp
    // Mhat^dag  = 1 - k^2 (D_oe)^dag (D_eo)^dag:  tmp = (D_eo)^dag in,  out = in - k^2 (D_oe)^dag tmp
    int rc = lqcd_moe(g, tmp_o, in_e, nullptr, U, 1.0, 0.0, dagger, prec, link, stream);
    if (rc) return rc;
    return lqcd_meo(g, out_e, tmp_o, in_e, U, -kappa * kappa, 1.0, dagger, prec, link, stream);
}
