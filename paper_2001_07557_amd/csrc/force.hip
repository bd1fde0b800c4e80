// Link derivative of c0 Re(Y^dag D_hop X): for every link U_mu(x) (owner
// computes: one thread per link, no atomics)
//   W = c0 s+_mu(x) [ X(x+mu) (x) ((1-g_mu) Y(x))^dag + ((1+g_mu) Y(x+mu)) (x) X(x)^dag ].
// Because (1 -+ g_mu)/2 is a rank-two hermitian projector, each spin sum
// reduces to two colour outer products of projected half-spinors:
//   sum_s a_s (x) ((1-g) b)_s^dag = sum_{u=0,1} h_u[(1-g) a] (x) h_u[(1-g) b]^dag.
// Output: mode 1 the raw gradient G = W^dag, mode 0 the su(3) force
// F = TA(G U^dag) = -TA(U W), TA(A) = (A - A^dag)/2 - tr(A - A^dag)/6.

#include "lqcd_internal.h"
#include "hop_common.h"

namespace lqcd {

struct ForceArgs {
    Geom g;
    char *F;
    const char *X, *Y, *U;
    int64_t hb;   // bytes of one parity half of X and Y
    int64_t bpp;  // blocks per parity
    double coeff;
    int mode, accumulate;
};

template <typename T>
__device__ __forceinline__ void outer_add(cplx<T> w[9], const cplx<T> a[3], const cplx<T> b[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) w[3 * i + j] = w[3 * i + j] + cmul_conj(b[j], a[i]);
}

template <int MU, int P, int LK>
__device__ __forceinline__ void force_direction(const ForceArgs &a, int p, int64_t s, const Coord &c) {
    using T = typename real_of<P>::type;
    const Geom &g = a.g;
    int64_t fwd;
    bool at_last;
    if constexpr (MU == 0) {
        const int64_t row = s - (c.x >> 1);
        const int xp = c.x + 1 == g.L[0] ? 0 : c.x + 1;
        fwd = row + (xp >> 1);
        at_last = c.x == g.L[0] - 1;
    } else {
        const int xm = MU == 1 ? c.y : MU == 2 ? c.z : c.t;
        const int L = g.L[MU];
        const int64_t st = MU == 1 ? g.sy : MU == 2 ? g.sz : g.st;
        at_last = xm == L - 1;
        fwd = at_last ? s - (int64_t)(L - 1) * st : s + st;
    }
    const double sgn = (at_last && g.bc[MU] < 0) ? -a.coeff : a.coeff;
    const char *Xh = a.X + p * a.hb, *Yh = a.Y + p * a.hb;
    const char *Xn = a.X + (p ^ 1) * a.hb, *Yn = a.Y + (p ^ 1) * a.hb;

    cplx<T> w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = {0, 0};
    {
        // X(x+mu) (x) ((1-g) Y(x))^dag
        cplx<T> v[12], hx0[3], hx1[3], hy0[3], hy1[3];
        load_spinor<P>(Xn, fwd, v);
        project_half<MU, -1>(v, hx0, hx1);
        load_spinor<P>(Yh, s, v);
        project_half<MU, -1>(v, hy0, hy1);
        outer_add(w, hx0, hy0);
        outer_add(w, hx1, hy1);
    }
    {
        // ((1+g) Y(x+mu)) (x) X(x)^dag
        cplx<T> v[12], hy0[3], hy1[3], hx0[3], hx1[3];
        load_spinor<P>(Yn, fwd, v);
        project_half<MU, 1>(v, hy0, hy1);
        load_spinor<P>(Xh, s, v);
        project_half<MU, 1>(v, hx0, hx1);
        outer_add(w, hy0, hx0);
        outer_add(w, hy1, hx1);
    }
    const T cs = (T)sgn;
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = scale(cs, w[k]);

    cplx<T> out[9];
    if (a.mode == 1) {
        // G = W^dag
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) out[3 * i + j] = conj(w[3 * j + i]);
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

// One 64-site tile per block; wave w computes the link of direction w for
// every site of the tile (each link is owned by exactly one thread).
template <int P, int LK>
__global__ __launch_bounds__(256) void force_k(ForceArgs a) {
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

}  // namespace lqcd

using namespace lqcd;

extern "C" int lqcd_fermion_force(const lqcd_geom_t *gg, void *F_out, const void *X, const void *Y,
                                  const void *U, double coeff, int mode, int accumulate, int prec,
                                  int link, void *stream) {
    Geom g;
    if (!make_geom(gg, &g)) return LQCD_EINVAL;
    if (prec != LQCD_F64 && prec != LQCD_F32) return LQCD_EINVAL;
    if (!valid_link(prec, link)) return LQCD_EINVAL;
    if (mode != 0 && mode != 1) return LQCD_EINVAL;
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
    dim3 grid((unsigned)(2 * a.bpp)), block(256);
    hipStream_t st = (hipStream_t)stream;
    if (prec == LQCD_F64) {
        if (link == 18) force_k<LQCD_F64, 18><<<grid, block, 0, st>>>(a);
        else force_k<LQCD_F64, 12><<<grid, block, 0, st>>>(a);
    } else {
        if (link == 18) force_k<LQCD_F32, 18><<<grid, block, 0, st>>>(a);
        else force_k<LQCD_F32, 12><<<grid, block, 0, st>>>(a);
    }
    return check_launch();
}
