// Library information, geometry validation, size queries and the conversions
// between the canonical lexicographic arrays and the tiled internal layout.

#include <string.h>

#include "lqcd_internal.h"

namespace lqcd {

static thread_local char g_hip_error[256] = "";

void set_hip_error(hipError_t e) {
    const char *s = hipGetErrorString(e);
    strncpy(g_hip_error, s ? s : "unknown HIP error", sizeof(g_hip_error) - 1);
    g_hip_error[sizeof(g_hip_error) - 1] = 0;
}

int check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_hip_error(e);
        return LQCD_EHIP;
    }
    return LQCD_OK;
}

bool make_geom(const lqcd_geom_t *g, Geom *out) {
    if (!g || !out) return false;
    int64_t v = 1;
    for (int mu = 0; mu < 4; ++mu) {
        const int L = g->dims[mu];
        if (L < 2 || (L & 1) || L > (1 << 16)) return false;
        if (g->bc[mu] != 1 && g->bc[mu] != -1) return false;
        out->L[mu] = L;
        out->bc[mu] = g->bc[mu];
        v *= L;
    }
    if (v > ((int64_t)1 << 31)) return false;  // grid of one thread per site fits 32 bits
    out->lxh = g->dims[0] / 2;
    out->vh = v / 2;
    out->ntiles = (out->vh + TILE - 1) / TILE;
    out->sy = out->lxh;
    out->sz = out->sy * g->dims[1];
    out->st = out->sz * g->dims[2];
    out->dx = make_fastdiv((uint32_t)out->lxh);
    out->dy = make_fastdiv((uint32_t)g->dims[1]);
    out->dz = make_fastdiv((uint32_t)g->dims[2]);
    return true;
}

// ---------------------------------------------------------------------------
// pack / unpack kernels
// ---------------------------------------------------------------------------

struct LexSite {
    int par;
    int64_t cb;
};

__device__ __forceinline__ LexSite lex_site(const Geom &g, int64_t lex) {
    int64_t r = lex;
    const int x = (int)(r % g.L[0]);
    r /= g.L[0];
    const int y = (int)(r % g.L[1]);
    r /= g.L[1];
    const int z = (int)(r % g.L[2]);
    const int t = (int)(r / g.L[2]);
    return {(x + y + z + t) & 1, lex >> 1};
}

template <typename CT, int P>
__global__ void pack_spinor_k(Geom g, char *dst, const CT *src, int subset, int64_t hb) {
    using T = typename real_of<P>::type;
    const int64_t lex = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lex >= 2 * g.vh) return;
    const LexSite ls = lex_site(g, lex);
    if (subset != LQCD_FULL && ls.par != subset) return;
    cplx<T> v[12];
    const CT *s = src + lex * 24;
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = {(T)s[2 * k], (T)s[2 * k + 1]};
    char *base = dst + (subset == LQCD_FULL ? ls.par * hb : 0);
    store_spinor<P>(base, ls.cb, v);
}

template <typename CT, int P>
__global__ void unpack_spinor_k(Geom g, CT *dst, const char *src, int subset, int64_t hb) {
    using T = typename real_of<P>::type;
    const int64_t lex = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lex >= 2 * g.vh) return;
    const LexSite ls = lex_site(g, lex);
    if (subset != LQCD_FULL && ls.par != subset) return;
    cplx<T> v[12];
    const char *base = src + (subset == LQCD_FULL ? ls.par * hb : 0);
    load_spinor<P>(base, ls.cb, v);
    CT *d = dst + lex * 24;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        d[2 * k] = (CT)v[k].re;
        d[2 * k + 1] = (CT)v[k].im;
    }
}

template <typename CT, int P, int LK>
__global__ void pack_gauge_k(Geom g, char *dst, const CT *src) {
    using T = typename real_of<P>::type;
    const int64_t lex = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lex >= 2 * g.vh) return;
    const LexSite ls = lex_site(g, lex);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        cplx<T> u[9];
        const CT *s = src + (lex * 4 + mu) * 18;
#pragma unroll
        for (int k = 0; k < 9; ++k) u[k] = {(T)s[2 * k], (T)s[2 * k + 1]};
        store_link<P, LK>(dst, g.ntiles, ls.par, ls.cb, mu, u);
    }
}

template <typename CT, int P, int LK>
__global__ void unpack_gauge_k(Geom g, CT *dst, const char *src) {
    using T = typename real_of<P>::type;
    const int64_t lex = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lex >= 2 * g.vh) return;
    const LexSite ls = lex_site(g, lex);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        cplx<T> u[9];
        load_link<P, LK>(src, g.ntiles, ls.par, ls.cb, mu, u);
        CT *d = dst + (lex * 4 + mu) * 18;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            d[2 * k] = (CT)u[k].re;
            d[2 * k + 1] = (CT)u[k].im;
        }
    }
}

}  // namespace lqcd

using namespace lqcd;

// ---------------------------------------------------------------------------
// library information and sizes
// ---------------------------------------------------------------------------

extern "C" int lqcd_version(void) { return 10000; }

extern "C" const char *lqcd_strerror(int status) {
    switch (status) {
        case LQCD_OK: return "ok";
        case LQCD_EINVAL: return "invalid argument (geometry, pointer, alignment or precision/link combination)";
        case LQCD_EHIP: return "HIP runtime or launch error";
        case LQCD_ENOCONV: return "solver did not converge within maxiter";
        case LQCD_ENAN: return "non-finite residual";
        case LQCD_ESMALL: return "workspace (or static scratch) too small";
        default: return "unknown status";
    }
}

extern "C" const char *lqcd_last_hip_error(void) { return g_hip_error; }

extern "C" size_t lqcd_spinor_bytes(const lqcd_geom_t *gg, int prec, int subset) {
    Geom g;
    if (!make_geom(gg, &g) || !valid_prec(prec)) return 0;
    if (subset != LQCD_EVEN && subset != LQCD_ODD && subset != LQCD_FULL) return 0;
    return half_spinor_bytes(g, prec) * (subset == LQCD_FULL ? 2 : 1);
}

extern "C" size_t lqcd_gauge_bytes(const lqcd_geom_t *gg, int prec, int link) {
    Geom g;
    if (!make_geom(gg, &g) || !valid_link(prec, link)) return 0;
    return gauge_bytes(g, prec, link);
}

// ---------------------------------------------------------------------------
// pack / unpack entry points
// ---------------------------------------------------------------------------

static bool aligned16(const void *p) { return p && (((uintptr_t)p) & 15) == 0; }

template <typename CT>
static void launch_pack_spinor(const Geom &g, void *dst, const void *src, int prec, int subset,
                               hipStream_t st) {
    const int64_t n = 2 * g.vh;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    const int64_t hb = (int64_t)half_spinor_bytes(g, prec);
    if (prec == LQCD_F64)
        pack_spinor_k<CT, LQCD_F64><<<grid, block, 0, st>>>(g, (char *)dst, (const CT *)src, subset, hb);
    else if (prec == LQCD_F32)
        pack_spinor_k<CT, LQCD_F32><<<grid, block, 0, st>>>(g, (char *)dst, (const CT *)src, subset, hb);
    else
        pack_spinor_k<CT, LQCD_F16><<<grid, block, 0, st>>>(g, (char *)dst, (const CT *)src, subset, hb);
}

template <typename CT>
static void launch_unpack_spinor(const Geom &g, void *dst, const void *src, int prec, int subset,
                                 hipStream_t st) {
    const int64_t n = 2 * g.vh;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    const int64_t hb = (int64_t)half_spinor_bytes(g, prec);
    if (prec == LQCD_F64)
        unpack_spinor_k<CT, LQCD_F64><<<grid, block, 0, st>>>(g, (CT *)dst, (const char *)src, subset, hb);
    else if (prec == LQCD_F32)
        unpack_spinor_k<CT, LQCD_F32><<<grid, block, 0, st>>>(g, (CT *)dst, (const char *)src, subset, hb);
    else
        unpack_spinor_k<CT, LQCD_F16><<<grid, block, 0, st>>>(g, (CT *)dst, (const char *)src, subset, hb);
}

static int spinor_args(const lqcd_geom_t *gg, Geom *g, const void *a, const void *b,
                       int canon_prec, int prec, int subset) {
    if (!make_geom(gg, g)) return LQCD_EINVAL;
    if (!valid_prec(prec)) return LQCD_EINVAL;
    if (canon_prec != LQCD_F64 && canon_prec != LQCD_F32) return LQCD_EINVAL;
    if (subset != LQCD_EVEN && subset != LQCD_ODD && subset != LQCD_FULL) return LQCD_EINVAL;
    if (!aligned16(a) || !aligned16(b)) return LQCD_EINVAL;
    return LQCD_OK;
}

extern "C" int lqcd_pack_spinor(const lqcd_geom_t *gg, void *dst, const void *src_canon,
                                int canon_prec, int prec, int subset, void *stream) {
    Geom g;
    int rc = spinor_args(gg, &g, dst, src_canon, canon_prec, prec, subset);
    if (rc) return rc;
    if (canon_prec == LQCD_F64) launch_pack_spinor<double>(g, dst, src_canon, prec, subset, (hipStream_t)stream);
    else launch_pack_spinor<float>(g, dst, src_canon, prec, subset, (hipStream_t)stream);
    return check_launch();
}

extern "C" int lqcd_unpack_spinor(const lqcd_geom_t *gg, void *dst_canon, const void *src,
                                  int canon_prec, int prec, int subset, void *stream) {
    Geom g;
    int rc = spinor_args(gg, &g, dst_canon, src, canon_prec, prec, subset);
    if (rc) return rc;
    if (canon_prec == LQCD_F64) launch_unpack_spinor<double>(g, dst_canon, src, prec, subset, (hipStream_t)stream);
    else launch_unpack_spinor<float>(g, dst_canon, src, prec, subset, (hipStream_t)stream);
    return check_launch();
}

template <typename CT, bool PACK>
static void launch_gauge(const Geom &g, void *dst, const void *src, int prec, int link,
                         hipStream_t st) {
    const int64_t n = 2 * g.vh;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
#define LQCD_GAUGE_CASE(P, LK)                                                                   \
    if (prec == P && link == LK) {                                                              \
        if (PACK) pack_gauge_k<CT, P, LK><<<grid, block, 0, st>>>(g, (char *)dst, (const CT *)src); \
        else unpack_gauge_k<CT, P, LK><<<grid, block, 0, st>>>(g, (CT *)dst, (const char *)src);    \
        return;                                                                                 \
    }
    LQCD_GAUGE_CASE(LQCD_F64, 18)
    LQCD_GAUGE_CASE(LQCD_F64, 12)
    LQCD_GAUGE_CASE(LQCD_F32, 18)
    LQCD_GAUGE_CASE(LQCD_F32, 12)
    LQCD_GAUGE_CASE(LQCD_F16, 12)
#undef LQCD_GAUGE_CASE
}

extern "C" int lqcd_pack_gauge(const lqcd_geom_t *gg, void *dst, const void *src_canon,
                               int canon_prec, int prec, int link, void *stream) {
    Geom g;
    if (!make_geom(gg, &g) || !valid_link(prec, link)) return LQCD_EINVAL;
    if (canon_prec != LQCD_F64 && canon_prec != LQCD_F32) return LQCD_EINVAL;
    if (!aligned16(dst) || !aligned16(src_canon)) return LQCD_EINVAL;
    if (canon_prec == LQCD_F64) launch_gauge<double, true>(g, dst, src_canon, prec, link, (hipStream_t)stream);
    else launch_gauge<float, true>(g, dst, src_canon, prec, link, (hipStream_t)stream);
    return check_launch();
}

extern "C" int lqcd_unpack_gauge(const lqcd_geom_t *gg, void *dst_canon, const void *src,
                                 int canon_prec, int prec, int link, void *stream) {
    Geom g;
    if (!make_geom(gg, &g) || !valid_link(prec, link)) return LQCD_EINVAL;
    if (canon_prec != LQCD_F64 && canon_prec != LQCD_F32) return LQCD_EINVAL;
    if (!aligned16(dst_canon) || !aligned16(src)) return LQCD_EINVAL;
    if (canon_prec == LQCD_F64) launch_gauge<double, false>(g, dst_canon, src, prec, link, (hipStream_t)stream);
    else launch_gauge<float, false>(g, dst_canon, src, prec, link, (hipStream_t)stream);
    return check_launch();
}
