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

template <int P, int LK, bool DAG, bool HASY, bool NORM>
__global__ __launch_bounds__(256) void hop_kernel(HopArgs a) {
    using T = typename real_of<P>::type;
    const int64_t nblk = gridDim.x;
    const int64_t blk = a.xcd ? xcd_block(blockIdx.x, nblk) : (int64_t)blockIdx.x;
    const int q = blk >= a.bpp ? 1 : 0;
    const int p = a.par0 ^ q;
    const int64_t s = (blk - q * a.bpp) * blockDim.x + threadIdx.x;
    const Geom &g = a.g;

    double nrm[1] = {0.0};
    if (s < g.vh) {
        cplx<T> acc[12];
        hop_site<P, LK, DAG>(g, a.in[p], a.U, p, s, acc);
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
        if constexpr (NORM) {
            T t = 0;
#pragma unroll
            for (int k = 0; k < 12; ++k) t += norm2(acc[k]);
            nrm[0] = (double)t;
        }
        store_spinor<P>(a.out[p], s, acc);
    }
    if constexpr (NORM) {
        block_sum<1>(nrm);
        if (threadIdx.x == 0) a.partial[blk] = nrm[0];
    }
}

template <int P, int LK, bool DAG>
static void launch_p(const HopArgs &a, bool hasy, bool norm, dim3 grid, dim3 block, hipStream_t st) {
    if (hasy) {
        if (norm) hop_kernel<P, LK, DAG, true, true><<<grid, block, 0, st>>>(a);
        else hop_kernel<P, LK, DAG, true, false><<<grid, block, 0, st>>>(a);
    } else {
        if (norm) hop_kernel<P, LK, DAG, false, true><<<grid, block, 0, st>>>(a);
        else hop_kernel<P, LK, DAG, false, false><<<grid, block, 0, st>>>(a);
    }
}

template <int P, int LK>
static void launch_l(const HopArgs &a, bool dag, bool hasy, bool norm, dim3 grid, dim3 block,
                     hipStream_t st) {
    if (dag) launch_p<P, LK, true>(a, hasy, norm, grid, block, st);
    else launch_p<P, LK, false>(a, hasy, norm, grid, block, st);
}

int hop_launch(const HopArgs &a0, int prec, int link, bool dag, int nparity, hipStream_t st) {
    HopArgs a = a0;
    const int bs = HOP_BLOCK;
    a.bpp = (a.g.vh + bs - 1) / bs;
    dim3 grid((unsigned)(a.bpp * nparity)), block(bs);
    const bool hasy = a.y[0] != nullptr || a.y[1] != nullptr;
    const bool norm = a.partial != nullptr;
    if (prec == LQCD_F64) {
        if (link == 18) launch_l<LQCD_F64, 18>(a, dag, hasy, norm, grid, block, st);
        else launch_l<LQCD_F64, 12>(a, dag, hasy, norm, grid, block, st);
    } else if (prec == LQCD_F32) {
        if (link == 18) launch_l<LQCD_F32, 18>(a, dag, hasy, norm, grid, block, st);
        else launch_l<LQCD_F32, 12>(a, dag, hasy, norm, grid, block, st);
    } else {
        launch_l<LQCD_F16, 12>(a, dag, hasy, norm, grid, block, st);
    }
    return check_launch();
}

int64_t hop_partials(const Geom &g, int nparity) {
    return ((g.vh + HOP_BLOCK - 1) / HOP_BLOCK) * nparity;
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
    a.xcd = 1;
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
    a.xcd = 1;
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
