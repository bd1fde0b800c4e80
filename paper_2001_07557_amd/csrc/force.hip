// Link derivative of c0 Re(Y^dag D_hop X): for every link U_mu(x) (owner
// computes: one thread per link, no atomics)
//   W = c0 s+_mu(x) [ X(x+mu) (x) ((1-g_mu) Y(x))^dag + ((1+g_mu) Y(x+mu)) (x) X(x)^dag ].
// Because (1 -+ g_mu)/2 is a rank-two hermitian projector, each spin sum
// reduces to two colour outer products of projected half-spinors:
//   sum_s a_s (x) ((1-g) b)_s^dag = sum_{u=0,1} h_u[(1-g) a] (x) h_u[(1-g) b]^dag.
// Output: mode 1 the raw gradient G = W^dag, mode 2 (12-real links) that
// gradient carried through the row-2 rebuild onto the stored rows 0 and 1,
// mode 0 the su(3) force F = TA(G U^dag) = -TA(U W),
// TA(A) = (A - A^dag)/2 - tr(A - A^dag)/6.

#include "lqcd_internal.h"
#include "hop_common.h"

namespace lqcd {

// staged kernel shape (ablation switch: 0 = every wave reads every spinor)
#ifndef LQCD_FORCE_STAGE
#define LQCD_FORCE_STAGE 1
#endif

struct ForceArgs {
    Geom g;
    char *F;
    const char *X, *Y, *U;
    int64_t hb;   // bytes of one parity half of X and Y
    int64_t bpp;  // blocks per parity
    double coeff;
    int mode, accumulate;
    Brick brick;  // tile traversal
};

template <typename T>
__device__ __forceinline__ void outer_add(cplx<T> w[9], const cplx<T> a[3], const cplx<T> b[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) w[3 * i + j] = w[3 * i + j] + cmul_conj(b[j], a[i]);
}

// Forward neighbour x + mu of site s (parity p) and whether the hop crosses
// the last slice (where the boundary sign applies).
template <int MU>
__device__ __forceinline__ int64_t force_neighbour(const Geom &g, int64_t s, const Coord &c,
                                                   bool &at_last) {
    if constexpr (MU == 0) {
        const int64_t row = s - (c.x >> 1);
        const int xp = c.x + 1 == g.L[0] ? 0 : c.x + 1;
        at_last = c.x == g.L[0] - 1;
        return row + (xp >> 1);
    } else {
        const int xm = MU == 1 ? c.y : MU == 2 ? c.z : c.t;
        const int L = g.L[MU];
        const int64_t st = MU == 1 ? g.sy : MU == 2 ? g.sz : g.st;
        at_last = xm == L - 1;
        return at_last ? s - (int64_t)(L - 1) * st : s + st;
    }
}

// Scale W by the coefficient and boundary sign, form G = W^dag (mode 1; mode
// 2 carries it onto the stored rows of a 12-real link) or F = -TA(U W)
// (mode 0), optionally add the old output, store.
template <int MU, int P, int LK>
__device__ __forceinline__ void force_store(const ForceArgs &a, int p, int64_t s, bool flip,
                                            cplx<typename real_of<P>::type> w[9]) {
    using T = typename real_of<P>::type;
    const Geom &g = a.g;
    const T cs = (T)(flip ? -a.coeff : a.coeff);
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = scale(cs, w[k]);

    cplx<T> out[9];
    if (a.mode != 0) {
        // G = W^dag
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) out[3 * i + j] = conj(w[3 * j + i]);
        if (a.mode == 2) {
            // gradient with respect to the stored rows 0, 1 of a 12-real link:
            // row 2 = conj(row0 x row1) chains G_2 into them,
            //   row0 += conj(row1 x G_2),  row1 += conj(G_2 x row0),  row2 = 0
            cplx<T> u[9];
            load_link<P, LK>(a.U, g.ntiles, p, s, MU, u);
            const cplx<T> d0[3] = {conj_cross(u[4], out[8], u[5], out[7]),
                                   conj_cross(u[5], out[6], u[3], out[8]),
                                   conj_cross(u[3], out[7], u[4], out[6])};
            const cplx<T> d1[3] = {conj_cross(out[7], u[2], out[8], u[1]),
                                   conj_cross(out[8], u[0], out[6], u[2]),
                                   conj_cross(out[6], u[1], out[7], u[0])};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                out[j] = out[j] + d0[j];
                out[3 + j] = out[3 + j] + d1[j];
                out[6 + j] = {0, 0};
            }
        }
    } else {
        cplx<T> u[9];
        load_link<P, LK>(a.U, g.ntiles, p, s, MU, u);
        cplx<T> m[9];  // U W
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                m[3 * i + j] = u[3 * i] * w[j] + u[3 * i + 1] * w[3 + j] + u[3 * i + 2] * w[6 + j];
        // F = -TA(m) = (m^dag - m)/2 + tr(m - m^dag)/6
        const T tr_im = (m[0].im + m[4].im + m[8].im) / (T)3;  // tr(m - m^dag)/6 = i Im tr(m)/3
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const cplx<T> d = conj(m[3 * j + i]) - m[3 * i + j];
                out[3 * i + j] = {(T)0.5 * d.re, (T)0.5 * d.im + (i == j ? tr_im : (T)0)};
            }
    }
    if (a.accumulate) {
        cplx<T> old[9];
        load_link<P, 18>(a.F, g.ntiles, p, s, MU, old);
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = out[k] + old[k];
    }
    store_link<P, 18, OUT_NT>(a.F, g.ntiles, p, s, MU, out);
}

// Link of direction MU at site s, every spinor read from memory.
template <int MU, int P, int LK>
__device__ __forceinline__ void force_direction(const ForceArgs &a, int p, int64_t s, const Coord &c) {
    using T = typename real_of<P>::type;
    bool at_last;
    const int64_t fwd = force_neighbour<MU>(a.g, s, c, at_last);
    cplx<T> w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = {0, 0};
    {
        // X(x+mu) (x) ((1-g) Y(x))^dag
        cplx<T> v[12], a0[3], a1[3], b0[3], b1[3];
        load_spinor<P>(a.X + (p ^ 1) * a.hb, fwd, v);
        project_half<MU, -1>(v, a0, a1);
        load_spinor<P>(a.Y + p * a.hb, s, v);
        project_half<MU, -1>(v, b0, b1);
        outer_add(w, a0, b0);
        outer_add(w, a1, b1);
    }
    {
        // ((1+g) Y(x+mu)) (x) X(x)^dag
        cplx<T> v[12], a0[3], a1[3], b0[3], b1[3];
        load_spinor<P>(a.Y + (p ^ 1) * a.hb, fwd, v);
        project_half<MU, 1>(v, a0, a1);
        load_spinor<P>(a.X + p * a.hb, s, v);
        project_half<MU, 1>(v, b0, b1);
        outer_add(w, a0, b0);
        outer_add(w, a1, b1);
    }
    force_store<MU, P, LK>(a, p, s, at_last && a.g.bc[MU] < 0, w);
}

// One 64-site tile per block; wave w computes the link of direction w for
// every site of the tile (each link is owned by exactly one thread).
template <int P, int LK>
__global__ __launch_bounds__(256) void force_plain_k(ForceArgs a) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int p = blk >= a.bpp ? 1 : 0;
    const int64_t s = (blk - p * a.bpp) * 64 + lane;
    if (s >= a.g.vh) return;
    const Coord c = cb_coords(a.g, p, s);
    switch (w) {
        case 0: force_direction<0, P, LK>(a, p, s, c); break;
        case 1: force_direction<1, P, LK>(a, p, s, c); break;
        case 2: force_direction<2, P, LK>(a, p, s, c); break;
        default: force_direction<3, P, LK>(a, p, s, c); break;
    }
}

// Spin rows 2h and 2h + 1 (complexes 6h .. 6h + 5) of the FP64 or FP32
// spinor at site s: the words of one half of the site in the tile layout.
template <int P>
__device__ __forceinline__ void load_spinor_half(const char *__restrict__ base, int64_t s, int h,
                                                 cplx<typename real_of<P>::type> v[6]) {
    const int lane = (int)(s & (TILE - 1));
    const char *t = base + (s >> TILE_SHIFT) * spinor_tile_bytes(P);
    if constexpr (P == LQCD_F64) {
        const v2d *w = reinterpret_cast<const v2d *>(t) + lane;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const v2d d = w[(6 * h + k) * TILE];
            v[k] = {d.x, d.y};
        }
    } else {
        const v4f *w = reinterpret_cast<const v4f *>(t) + lane;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const v4f f = w[(3 * h + k) * TILE];
            v[2 * k] = {f.x, f.y};
            v[2 * k + 1] = {f.z, f.w};
        }
    }
}

// Neighbour spinors of direction MU, read and projected to the halves that
// enter the link's W; returns whether the link carries the boundary sign.
template <int MU, int P>
__device__ __forceinline__ bool force_neighbours(const ForceArgs &a, int p, int64_t s,
                                                 cplx<typename real_of<P>::type> hx[6],
                                                 cplx<typename real_of<P>::type> hy[6]) {
    using T = typename real_of<P>::type;
    bool at_last;
    const int64_t fwd = force_neighbour<MU>(a.g, s, cb_coords(a.g, p, s), at_last);
    cplx<T> v[12];
    load_spinor<P>(a.X + (p ^ 1) * a.hb, fwd, v);
    project_half<MU, -1>(v, hx, hx + 3);
    load_spinor<P>(a.Y + (p ^ 1) * a.hb, fwd, v);
    project_half<MU, 1>(v, hy, hy + 3);
    return at_last && a.g.bc[MU] < 0;
}

// The link of direction MU at site s: W = X(x+mu) (x) ((1-g) Y(x))^dag +
// ((1+g) Y(x+mu)) (x) X(x)^dag from the projected neighbour halves
// hx = h[(1-g) X(x+mu)], hy = h[(1+g) Y(x+mu)] and the site's own Y, then X,
// read from the block's LDS copy one at a time (fewer live registers).
template <int MU, int P, int LK>
__device__ __forceinline__ void force_staged(const ForceArgs &a, int p, int64_t s, int lane, bool flip,
                                             const cplx<typename real_of<P>::type> hx[6],
                                             const cplx<typename real_of<P>::type> hy[6],
                                             const cplx<typename real_of<P>::type> (*xs)[64],
                                             const cplx<typename real_of<P>::type> (*ys)[64]) {
    using T = typename real_of<P>::type;
    cplx<T> v[12], b0[3], b1[3], w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = {0, 0};
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = ys[k][lane];
    project_half<MU, -1>(v, b0, b1);
    outer_add(w, hx, b0);
    outer_add(w, hx + 3, b1);
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = xs[k][lane];
    project_half<MU, 1>(v, b0, b1);
    outer_add(w, hy, b0);
    outer_add(w, hy + 3, b1);
    force_store<MU, P, LK>(a, p, s, flip, w);
}

// Staged shape.  Consecutive blocks take the even and the odd tile of one
// region (their neighbours are each other's sites, so both parities of X
// and Y are fetched into the same XCD's L2), regions are walked in the hop
// kernels' brick order, and the tile's own X and Y are loaded once by the
// four waves together and read from LDS by all of them (every wave needs
// them; the neighbour spinors are per direction).
template <int P, int LK>
__global__ __launch_bounds__(256) void force_k(ForceArgs a) {
    using T = typename real_of<P>::type;
    __shared__ cplx<T> xs[12][64], ys[12][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int p = (int)(blk & 1);
    const int64_t s = brick_order((uint32_t)(blk >> 1), a.brick) * 64 + lane;
    const bool active = s < a.g.vh;
    if (active) {
        // wave q stages spin rows 2(q & 1) and 2(q & 1) + 1 of X (q < 2) or Y
        const char *src = (w < 2 ? a.X : a.Y) + p * a.hb;
        cplx<T> v[6];
        load_spinor_half<P>(src, s, w & 1, v);
        cplx<T>(*dst)[64] = w < 2 ? xs : ys;
        const int k0 = 6 * (w & 1);
#pragma unroll
        for (int k = 0; k < 6; ++k) dst[k0 + k][lane] = v[k];
    }
    // each wave reads and projects the neighbours of its own direction while
    // the staged words arrive; the branch rejoins before the barrier, which
    // every thread of the block reaches
    cplx<T> hx[6], hy[6];
    bool flip = false;
    if (active) {
        switch (w) {
            case 0: flip = force_neighbours<0, P>(a, p, s, hx, hy); break;
            case 1: flip = force_neighbours<1, P>(a, p, s, hx, hy); break;
            case 2: flip = force_neighbours<2, P>(a, p, s, hx, hy); break;
            default: flip = force_neighbours<3, P>(a, p, s, hx, hy); break;
        }
    }
    __syncthreads();
    if (!active) return;
    switch (w) {
        case 0: force_staged<0, P, LK>(a, p, s, lane, flip, hx, hy, xs, ys); break;
        case 1: force_staged<1, P, LK>(a, p, s, lane, flip, hx, hy, xs, ys); break;
        case 2: force_staged<2, P, LK>(a, p, s, lane, flip, hx, hy, xs, ys); break;
        default: force_staged<3, P, LK>(a, p, s, lane, flip, hx, hy, xs, ys); break;
    }
}

}  // namespace lqcd

using namespace lqcd;

extern "C" int lqcd_fermion_force(const lqcd_geom_t *gg, void *F_out, const void *X, const void *Y,
                                  const void *U, double coeff, int mode, int accumulate, int prec,
                                  int link, void *stream) {
    Geom g;
    if (!make_geom(gg, &g)) return LQCD_EINVAL;
    if (prec != LQCD_F64 && prec != LQCD_F32) return LQCD_EINVAL;
    if (!valid_link(prec, link)) return LQCD_EINVAL;
    if (mode != 0 && mode != 1 && !(mode == 2 && link == 12)) return LQCD_EINVAL;
    if (!F_out || !X || !Y || !U) return LQCD_EINVAL;
    if (((uintptr_t)F_out | (uintptr_t)X | (uintptr_t)Y | (uintptr_t)U) & 15) return LQCD_EINVAL;
    if (F_out == X || F_out == Y || F_out == U) return LQCD_EINVAL;
    ForceArgs a{};
    a.g = g;
    a.F = (char *)F_out;
    a.X = (const char *)X;
    a.Y = (const char *)Y;
    a.U = (const char *)U;
    a.hb = (int64_t)half_spinor_bytes(g, prec);
    a.coeff = coeff;
    a.mode = mode;
    a.accumulate = accumulate ? 1 : 0;
    a.bpp = (g.vh + 63) / 64;
    a.brick = make_brick(g, brick_plan(g, prec));
    dim3 grid((unsigned)(2 * a.bpp)), block(256);
    hipStream_t st = (hipStream_t)stream;
#define LQCD_FORCE(P, LK)                                                       \
    if (LQCD_FORCE_STAGE) force_k<P, LK><<<grid, block, 0, st>>>(a);           \
    else force_plain_k<P, LK><<<grid, block, 0, st>>>(a);
    if (prec == LQCD_F64) {
        if (link == 18) { LQCD_FORCE(LQCD_F64, 18) }
        else { LQCD_FORCE(LQCD_F64, 12) }
    } else {
        if (link == 18) { LQCD_FORCE(LQCD_F32, 18) }
        else { LQCD_FORCE(LQCD_F32, 12) }
    }
#undef LQCD_FORCE
    return check_launch();
}
