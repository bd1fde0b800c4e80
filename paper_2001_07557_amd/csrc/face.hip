// Faces of a decomposition in t, the one-GPU part of the multi-GPU shift: the
// paper's multi-node shift splits Grid's arrays at the domain boundary and
// sends the pieces to the neighbouring node (Sec. 3.1); for the even-odd hop
// the pieces are, per site of the boundary t-slice of the input parity,
//   forward face:  s (1 + S_f g_t) in(y), y on slice 0, rows 0 and 1 (the
//                  receiver multiplies by its own U_t),
//   backward face: s U_t(y)^dag (1 + S_b g_t) in(y), y on slice Lt-1 (the
//                  sender applies the link it owns, so links never move),
// with S_f = -1, S_b = +1 (exchanged for the adjoint) and s = bc[3], the
// phase of a hop across the t boundary.  The half-spinors are formed with the
// same code and the same arithmetic as inside the fused hop, so a boundary
// launch that reads them reproduces the unsplit hop bit for bit (binary16
// storage: the forward face holds the packed binary16 half-spinor and the
// neighbour's scale times s, which the receiver applies after its link; the
// backward face holds U^dag times the half-spinor and, apart, the same kind
// of factor, which the receiver folds into its sums as the unsplit hop does).

#include "lqcd_internal.h"
#include "hop_common.h"

namespace lqcd {

constexpr int FACE_BLOCK = 256;

template <int P, int LK, bool DAG>
__global__ __launch_bounds__(FACE_BLOCK) void face_pack_k(Geom g, char *fwd_face, char *bwd_face,
                                                          const char *in, const char *U, int q,
                                                          int64_t bps) {
    using T = typename real_of<P>::type;
    using E = typename hop_elem<P>::type;
    constexpr int SF = DAG ? 1 : -1;
    const int64_t b = blockIdx.x;
    const bool bwd = b >= bps;
    const int64_t j = (bwd ? b - bps : b) * FACE_BLOCK + threadIdx.x;  // site within the slice
    if (j >= g.st) return;
    // the t boundary carries bc[3]; binary16 storage multiplies in the site scale
    T sgn = g.bc[3] < 0 ? T(-1) : T(1);
    cplx<E> psi[12];
    cplx<T> h[6];
    if (!bwd) {
        // receiver: site j of slice Lt-1, forward neighbour j of slice 0
        load_spinor_hop<P>(in, j, psi, sgn);
        if constexpr (P == LQCD_F16) {
            v2h hr[6], hi[6];
            half_forms_h<3, SF, false>(psi, hr, hi);
            store_face_forms(fwd_face, j, hr, hi, sgn);
        } else {
            hop_half<3, SF>(psi, sgn, h, h + 3);
            store_face<T>(fwd_face, j, h);
        }
    } else {
        // receiver: site j of slice 0, backward neighbour y on slice Lt-1,
        // whose link U_t(y) (parity q) the sender owns
        const int64_t y = (int64_t)(g.L[3] - 1) * g.st + j;
        cplx<T> x[6];
        load_spinor_hop<P>(in, y, psi, sgn);
        link_chi<3, -SF, true, P, LK, false, P != LQCD_F16>(U, g.ntiles, q, y, psi, sgn, x, x + 3);
        if constexpr (P == LQCD_F16) store_face_h(bwd_face, j, x, sgn);
        else store_face<T>(bwd_face, j, x);
    }
}

}  // namespace lqcd

using namespace lqcd;

extern "C" size_t lqcd_face_bytes(const lqcd_geom_t *gg, int prec) {
    Geom g;
    if (!make_geom(gg, &g) || !valid_prec(prec) || g.st % TILE != 0) return 0;
    return face_bytes(g, prec);
}

extern "C" int lqcd_face_pack(const lqcd_geom_t *gg, void *face_fwd, void *face_bwd,
                              const void *in, const void *U, int out_par, int dagger, int prec,
                              int link, void *stream) {
    Geom g;
    if (!make_geom(gg, &g) || !valid_link(prec, link)) return LQCD_EINVAL;
    if (g.st % TILE != 0) return LQCD_EINVAL;
    if (prec == LQCD_F16 && g.ntiles > F16_MAX_TILES) return LQCD_EINVAL;
    if (out_par != LQCD_EVEN && out_par != LQCD_ODD) return LQCD_EINVAL;
    if (!face_fwd || !face_bwd || !in || !U || face_fwd == face_bwd) return LQCD_EINVAL;
    if (((uintptr_t)face_fwd | (uintptr_t)face_bwd | (uintptr_t)in | (uintptr_t)U) & 15)
        return LQCD_EINVAL;
    const int q = 1 - out_par;  // parity of the input half field
    const int64_t bps = (g.st + FACE_BLOCK - 1) / FACE_BLOCK;
    dim3 grid((unsigned)(2 * bps)), block(FACE_BLOCK);
    hipStream_t st = (hipStream_t)stream;
    char *ff = (char *)face_fwd, *fb = (char *)face_bwd;
    const char *i = (const char *)in, *u = (const char *)U;
#define LQCD_FACE(PR, LK)                                                                       \
    if (dagger) face_pack_k<PR, LK, true><<<grid, block, 0, st>>>(g, ff, fb, i, u, q, bps);     \
    else face_pack_k<PR, LK, false><<<grid, block, 0, st>>>(g, ff, fb, i, u, q, bps);
    if (prec == LQCD_F64) {
        if (link == 18) { LQCD_FACE(LQCD_F64, 18) }
        else { LQCD_FACE(LQCD_F64, 12) }
    } else if (prec == LQCD_F32) {
        if (link == 18) { LQCD_FACE(LQCD_F32, 18) }
        else { LQCD_FACE(LQCD_F32, 12) }
    } else {
        LQCD_FACE(LQCD_F16, 12)
    }
#undef LQCD_FACE
    return check_launch();
}
