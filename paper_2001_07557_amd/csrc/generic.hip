// The hopping term composed from generic lattice operations, the counterpart
// of the fused kernels in dslash.hip: the paper compares Grid's generic
// Wilson kernel, built on its shift/stencil machinery, with a hand-unrolled
// one (Sec. 3.3, Fig. 4d; stencils built from shifts, Sec. 3.1).  Here the
// generic operator is a sequence of three library kernels per hop, each a
// full pass over the lattice:
//
//   forward hop mu:   t1 = cshift(in, mu, +1);  t2 = U_mu t1;      out += (1 - g_mu) t2
//   backward hop mu:  t1 = U_mu^dag in;         t2 = cshift(t1, mu, -1);  out += (1 + g_mu) t2
//
// (projector signs exchanged for the adjoint), 24 launches per application
// against one fused launch; the first projection overwrites `out`.

#include "lqcd_internal.h"
#include "hop_common.h"

namespace lqcd {

constexpr int GEN_BLOCK = 256;

// out(x) = U_mu(x) in(x) (ADJ: U_mu(x)^dag in(x)) for every spin, full fields.
template <int P, int LK, bool ADJ>
__global__ __launch_bounds__(GEN_BLOCK) void colour_mul_k(Geom g, char *out, const char *in,
                                                          const char *U, int64_t hb, int mu,
                                                          int64_t bpp) {
    using T = typename real_of<P>::type;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int p = blk >= bpp ? 1 : 0;
    const int64_t s = (blk - p * bpp) * GEN_BLOCK + threadIdx.x;
    if (s >= g.vh) return;
    cplx<T> u[9], v[12], w[12];
    load_link<P, LK, false>(U, g.ntiles, p, s, mu, u);
    load_spinor<P>(in + p * hb, s, v);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
        const cplx<T> *c = v + 3 * sp;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if constexpr (ADJ) w[3 * sp + a] = cdot3c(u[a], c[0], u[3 + a], c[1], u[6 + a], c[2]);
            else w[3 * sp + a] = cdot3(u[3 * a], c[0], u[3 * a + 1], c[1], u[3 * a + 2], c[2]);
        }
    }
    store_spinor<P>(out + p * hb, s, w);
}

// FP64: one spin of one site per thread, a block = the four spins of one
// 64-site tile (wave = spin); the four waves read the same link words, the
// later ones from the L2, and each holds a third of the spinor registers.
template <int LK, bool ADJ>
__global__ __launch_bounds__(GEN_BLOCK) void colour_mul_f64_k(Geom g, char *out, const char *in,
                                                              const char *U, int64_t hb, int mu,
                                                              int64_t tpp) {
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int p = blk >= tpp ? 1 : 0;
    const int lane = threadIdx.x & 63;
    const int sp = threadIdx.x >> 6;
    const int64_t s = (blk - p * tpp) * TILE + lane;
    if (s >= g.vh) return;
    cplx<double> u[9];
    load_link<LQCD_F64, LK, false>(U, g.ntiles, p, s, mu, u);
    const int64_t toff = (s >> TILE_SHIFT) * spinor_tile_bytes(LQCD_F64);
    const v2d *w = reinterpret_cast<const v2d *>(in + p * hb + toff) + lane;
    v2d *o = reinterpret_cast<v2d *>(out + p * hb + toff) + lane;
    cplx<double> c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const v2d d = w[(3 * sp + a) * TILE];
        c[a] = {d.x, d.y};
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cplx<double> r = ADJ ? cdot3c(u[a], c[0], u[3 + a], c[1], u[6 + a], c[2])
                                   : cdot3(u[3 * a], c[0], u[3 * a + 1], c[1], u[3 * a + 2], c[2]);
        o[(3 * sp + a) * TILE] = v2d{r.re, r.im};
    }
}

// acc(x) (+)= (1 + S g_mu) in(x): rows 0 and 1 of the projection and the two
// rows that follow from them (the projector has rank two).
template <int P, int MU, int S>
__device__ __forceinline__ void project_site(char *acc, const char *in, int64_t s, bool add) {
    using T = typename real_of<P>::type;
    cplx<T> v[12], h0[3], h1[3], r[12];
    load_spinor<P>(in, s, v);
    project_half<MU, S>(v, h0, h1);
    if (add) {
        load_spinor<P>(acc, s, r);
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) r[k] = {0, 0};
    }
    chi_accumulate<MU, S>(h0, h1, r);
    store_spinor<P>(acc, s, r);
}

template <int P>
__global__ __launch_bounds__(GEN_BLOCK) void spin_project_k(Geom g, char *acc, const char *in,
                                                            int64_t hb, int mu_sign, int add,
                                                            int64_t bpp) {
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int p = blk >= bpp ? 1 : 0;
    const int64_t s = (blk - p * bpp) * GEN_BLOCK + threadIdx.x;
    if (s >= g.vh) return;
    char *a = acc + p * hb;
    const char *x = in + p * hb;
    switch (mu_sign) {
        case 0: project_site<P, 0, -1>(a, x, s, add != 0); break;
        case 1: project_site<P, 0, 1>(a, x, s, add != 0); break;
        case 2: project_site<P, 1, -1>(a, x, s, add != 0); break;
        case 3: project_site<P, 1, 1>(a, x, s, add != 0); break;
        case 4: project_site<P, 2, -1>(a, x, s, add != 0); break;
        case 5: project_site<P, 2, 1>(a, x, s, add != 0); break;
        case 6: project_site<P, 3, -1>(a, x, s, add != 0); break;
        default: project_site<P, 3, 1>(a, x, s, add != 0); break;
    }
}

}  // namespace lqcd

using namespace lqcd;

static bool al16(const void *p) { return p && ((uintptr_t)p & 15) == 0; }

extern "C" int lqcd_colour_mul(const lqcd_geom_t *gg, void *out, const void *in, const void *U,
                               int mu, int adjoint, int prec, int link, void *stream) {
    Geom g;
    if (!make_geom(gg, &g)) return LQCD_EINVAL;
    if ((prec != LQCD_F64 && prec != LQCD_F32) || !valid_link(prec, link)) return LQCD_EINVAL;
    if (mu < 0 || mu > 3 || !al16(out) || !al16(in) || !al16(U) || out == in) return LQCD_EINVAL;
    const int64_t hb = (int64_t)half_spinor_bytes(g, prec);
    const int64_t bpp = (g.vh + GEN_BLOCK - 1) / GEN_BLOCK;
    dim3 grid((unsigned)(2 * bpp)), block(GEN_BLOCK);
    hipStream_t st = (hipStream_t)stream;
    char *o = (char *)out;
    const char *i = (const char *)in, *u = (const char *)U;
#define LQCD_CMUL(PR, LK)                                                                        \
    if (adjoint) colour_mul_k<PR, LK, true><<<grid, block, 0, st>>>(g, o, i, u, hb, mu, bpp);    \
    else colour_mul_k<PR, LK, false><<<grid, block, 0, st>>>(g, o, i, u, hb, mu, bpp);
    if (prec == LQCD_F64 && !LQCD_LAYOUT_AOS) {
        const int64_t tpp = g.ntiles;
        dim3 g4((unsigned)(2 * tpp)), b4(GEN_BLOCK);
        if (link == 18) {
            if (adjoint) colour_mul_f64_k<18, true><<<g4, b4, 0, st>>>(g, o, i, u, hb, mu, tpp);
            else colour_mul_f64_k<18, false><<<g4, b4, 0, st>>>(g, o, i, u, hb, mu, tpp);
        } else {
            if (adjoint) colour_mul_f64_k<12, true><<<g4, b4, 0, st>>>(g, o, i, u, hb, mu, tpp);
            else colour_mul_f64_k<12, false><<<g4, b4, 0, st>>>(g, o, i, u, hb, mu, tpp);
        }
    } else if (prec == LQCD_F64) {
        if (link == 18) { LQCD_CMUL(LQCD_F64, 18) }
        else { LQCD_CMUL(LQCD_F64, 12) }
    } else {
        if (link == 18) { LQCD_CMUL(LQCD_F32, 18) }
        else { LQCD_CMUL(LQCD_F32, 12) }
    }
#undef LQCD_CMUL
    return check_launch();
}

extern "C" int lqcd_spin_project(const lqcd_geom_t *gg, void *acc, const void *in, int mu,
                                 int sign, int accumulate, int prec, void *stream) {
    Geom g;
    if (!make_geom(gg, &g)) return LQCD_EINVAL;
    if (prec != LQCD_F64 && prec != LQCD_F32) return LQCD_EINVAL;
    if (mu < 0 || mu > 3 || (sign != 1 && sign != -1)) return LQCD_EINVAL;
    if (!al16(acc) || !al16(in) || acc == in) return LQCD_EINVAL;
    const int64_t hb = (int64_t)half_spinor_bytes(g, prec);
    const int64_t bpp = (g.vh + GEN_BLOCK - 1) / GEN_BLOCK;
    dim3 grid((unsigned)(2 * bpp)), block(GEN_BLOCK);
    hipStream_t st = (hipStream_t)stream;
    const int ms = 2 * mu + (sign > 0 ? 1 : 0);
    if (prec == LQCD_F64)
        spin_project_k<LQCD_F64><<<grid, block, 0, st>>>(g, (char *)acc, (const char *)in, hb, ms,
                                                         accumulate ? 1 : 0, bpp);
    else
        spin_project_k<LQCD_F32><<<grid, block, 0, st>>>(g, (char *)acc, (const char *)in, hb, ms,
                                                         accumulate ? 1 : 0, bpp);
    return check_launch();
}

extern "C" int lqcd_dslash_generic(const lqcd_geom_t *gg, void *out, const void *in,
                                   const void *U, void *tmp1, void *tmp2, int dagger, int prec,
                                   int link, void *stream) {
    Geom g;
    if (!make_geom(gg, &g)) return LQCD_EINVAL;
    if ((prec != LQCD_F64 && prec != LQCD_F32) || !valid_link(prec, link)) return LQCD_EINVAL;
    if (!al16(out) || !al16(in) || !al16(U) || !al16(tmp1) || !al16(tmp2)) return LQCD_EINVAL;
    const void *p[4] = {out, in, tmp1, tmp2};
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b)
            if (p[a] == p[b]) return LQCD_EINVAL;
    // forward hops project with (1 - g_mu), backward with (1 + g_mu); the
    // adjoint exchanges them
    const int sf = dagger ? 1 : -1;
    int rc = LQCD_OK;
    for (int mu = 0; mu < 4 && rc == LQCD_OK; ++mu) {
        rc = lqcd_cshift(gg, tmp1, in, mu, 1, prec, stream);
        if (!rc) rc = lqcd_colour_mul(gg, tmp2, tmp1, U, mu, 0, prec, link, stream);
        if (!rc) rc = lqcd_spin_project(gg, out, tmp2, mu, sf, mu > 0, prec, stream);
        if (!rc) rc = lqcd_colour_mul(gg, tmp1, in, U, mu, 1, prec, link, stream);
        if (!rc) rc = lqcd_cshift(gg, tmp2, tmp1, mu, -1, prec, stream);
        if (!rc) rc = lqcd_spin_project(gg, out, tmp2, mu, -sf, 1, prec, stream);
    }
    return rc;
}
