// Lattice SU(3) matrix product W_mu(x) = op(U_mu(x)) op(V_mu(x)) for all 4V
// links (op = identity or hermitian conjugate): the per-link SU(3) matrix
// product whose hand-written kernel the paper benchmarks on the vector
// engine (Sec. 3.3, Fig. 4a-c).  Pure streaming: 198 flop per link against three
// links of traffic, one thread per link, a block = one 64-site tile with
// wave w on direction w.  12-real storage rebuilds row 2 of the inputs and
// stores rows 0 and 1 of the product (the product of SU(3) matrices is SU(3)).

#include "lqcd_internal.h"

namespace lqcd {

template <int P, int LK, bool AU, bool AV>
__global__ __launch_bounds__(256) void su3_mul_k(Geom g, char *W, const char *U, const char *V,
                                                 int64_t bpp) {
    using T = typename real_of<P>::type;
    const int lane = threadIdx.x & 63;
    const int mu = threadIdx.x >> 6;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int p = blk >= bpp ? 1 : 0;
    const int64_t s = (blk - p * bpp) * 64 + lane;
    if (s >= g.vh) return;
    cplx<T> u[9], v[9], w[9];
    load_link<P, LK>(U, g.ntiles, p, s, mu, u);
    load_link<P, LK>(V, g.ntiles, p, s, mu, v);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cplx<T> acc = {0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const cplx<T> a = AU ? conj(u[3 * k + i]) : u[3 * i + k];
                const cplx<T> b = AV ? conj(v[3 * j + k]) : v[3 * k + j];
                acc = acc + a * b;
            }
            w[3 * i + j] = acc;
        }
    store_link<P, LK>(W, g.ntiles, p, s, mu, w);
}

template <int P, int LK>
static void launch_su3(const Geom &g, char *W, const char *U, const char *V, bool au, bool av,
                       hipStream_t st) {
    const int64_t bpp = g.ntiles;
    dim3 grid((unsigned)(2 * bpp)), block(256);
    if (au) {
        if (av) su3_mul_k<P, LK, true, true><<<grid, block, 0, st>>>(g, W, U, V, bpp);
        else su3_mul_k<P, LK, true, false><<<grid, block, 0, st>>>(g, W, U, V, bpp);
    } else {
        if (av) su3_mul_k<P, LK, false, true><<<grid, block, 0, st>>>(g, W, U, V, bpp);
        else su3_mul_k<P, LK, false, false><<<grid, block, 0, st>>>(g, W, U, V, bpp);
    }
}

}  // namespace lqcd

using namespace lqcd;

extern "C" int lqcd_su3_mul(const lqcd_geom_t *gg, void *W, const void *U, const void *V,
                            int adj_u, int adj_v, int prec, int link, void *stream) {
    Geom g;
    if (!make_geom(gg, &g)) return LQCD_EINVAL;
    if ((prec != LQCD_F64 && prec != LQCD_F32) || !valid_link(prec, link)) return LQCD_EINVAL;
    if (!W || !U || !V || (((uintptr_t)W | (uintptr_t)U | (uintptr_t)V) & 15)) return LQCD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const bool au = adj_u != 0, av = adj_v != 0;
    if (prec == LQCD_F64) {
        if (link == 18) launch_su3<LQCD_F64, 18>(g, (char *)W, (const char *)U, (const char *)V, au, av, st);
        else launch_su3<LQCD_F64, 12>(g, (char *)W, (const char *)U, (const char *)V, au, av, st);
    } else {
        if (link == 18) launch_su3<LQCD_F32, 18>(g, (char *)W, (const char *)U, (const char *)V, au, av, st);
        else launch_su3<LQCD_F32, 12>(g, (char *)W, (const char *)U, (const char *)V, au, av, st);
    }
    return check_launch();
}
