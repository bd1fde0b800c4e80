// BLAS-1 on internal spinor fields: inner products and norms with
// deterministic wave64 -> block -> grid reductions (FP64 from the block level
// up), y = a x + b y, and precision conversion.  One thread per site; a
// FULL field is the even half followed by the odd half.

#include <mutex>

#include "lqcd_internal.h"
#include "reduce.h"
#include "blas.h"

namespace lqcd {

constexpr int RED_BLOCK = 256;

// Ablation switch: 1 replaces the wave64 -> block -> fixed-order grid
// reduction by one FP64 atomic add per thread into the result (which is then
// order-dependent, i.e. not reproducible bit for bit).
#ifndef LQCD_REDUCE_ATOMIC
#define LQCD_REDUCE_ATOMIC 0
#endif

int64_t reduce_blocks(const Geom &g, int nhalf) { return (g.vh * nhalf + RED_BLOCK - 1) / RED_BLOCK; }

template <int P, bool DOT>
__global__ __launch_bounds__(RED_BLOCK) void reduce_k(const char *a, const char *b, int64_t vh,
                                                      int nhalf, int64_t hb, double *partial) {
    using T = typename real_of<P>::type;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (s < vh * nhalf) {
        const int64_t off = s >= vh ? hb : 0;
        if (s >= vh) s -= vh;
        cplx<T> va[12];
        load_spinor<P>(a + off, s, va);
        T re = 0, im = 0;
        if constexpr (DOT) {
            cplx<T> vb[12];
            load_spinor<P>(b + off, s, vb);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const cplx<T> z = cmul_conj(va[k], vb[k]);
                re += z.re;
                im += z.im;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) re += norm2(va[k]);
        }
        acc[0] = (double)re;
        acc[1] = (double)im;
    }
#if LQCD_REDUCE_ATOMIC
    atomicAdd(partial, acc[0]);
    atomicAdd(partial + 1, acc[1]);
#else
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = acc[0];
        partial[2 * blockIdx.x + 1] = acc[1];
    }
#endif
}

// Fixed-order sum of n partial records of NV doubles into out[0..NV).
template <int NV>
__global__ __launch_bounds__(RED_BLOCK) void finalize_k(const double *partial, int64_t n, double *out) {
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += partial[i * NV + k];
    }
    block_sum<NV>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] = v[k];
    }
}

void launch_finalize(const double *partial, int64_t n, int nv, double *out, hipStream_t st) {
    if (nv == 1) finalize_k<1><<<1, RED_BLOCK, 0, st>>>(partial, n, out);
    else finalize_k<2><<<1, RED_BLOCK, 0, st>>>(partial, n, out);
}

template <int P>
__global__ __launch_bounds__(RED_BLOCK) void axpby_k(double a, const char *x, double b, char *y,
                                                     int64_t vh, int nhalf, int64_t hb) {
    using T = typename real_of<P>::type;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= vh * nhalf) return;
    const int64_t off = s >= vh ? hb : 0;
    if (s >= vh) s -= vh;
    cplx<T> vx[12], vy[12];
    load_spinor<P>(x + off, s, vx);
    load_spinor<P>(y + off, s, vy);
    const T ta = (T)a, tb = (T)b;
#pragma unroll
    for (int k = 0; k < 12; ++k)
        vy[k] = {ta * vx[k].re + tb * vy[k].re, ta * vx[k].im + tb * vy[k].im};
    store_spinor<P>(y + off, s, vy);
}

template <int PD, int PS>
__global__ __launch_bounds__(RED_BLOCK) void convert_k(char *dst, const char *src, int64_t vh,
                                                       int nhalf, int64_t hbd, int64_t hbs) {
    using TD = typename real_of<PD>::type;
    using TS = typename real_of<PS>::type;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= vh * nhalf) return;
    const bool hi = s >= vh;
    if (hi) s -= vh;
    cplx<TS> v[12];
    load_spinor<PS>(src + (hi ? hbs : 0), s, v);
    cplx<TD> w[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = {(TD)v[k].re, (TD)v[k].im};
    store_spinor<PD>(dst + (hi ? hbd : 0), s, w);
}

// Same storage precision: the layouts agree byte for byte, so the copy is one
// 16-byte word per thread (a thread per site moving all its words measured
// 5.3 TB/s on a 4 GB copy against 6.2 TB/s for one word per thread).
__global__ __launch_bounds__(RED_BLOCK) void copy_words_k(v4u *dst, const v4u *src, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

void launch_convert(const Geom &g, int nhalf, char *dst, int pd, const char *src, int ps,
                    hipStream_t st) {
    if (pd == ps) {
        const int64_t words = (int64_t)half_spinor_bytes(g, pd) * nhalf / 16;
        dim3 grid((unsigned)((words + RED_BLOCK - 1) / RED_BLOCK)), block(RED_BLOCK);
        copy_words_k<<<grid, block, 0, st>>>((v4u *)dst, (const v4u *)src, words);
        return;
    }
    const int64_t n = g.vh * nhalf;
    dim3 grid((unsigned)((n + RED_BLOCK - 1) / RED_BLOCK)), block(RED_BLOCK);
    const int64_t hbd = (int64_t)half_spinor_bytes(g, pd), hbs = (int64_t)half_spinor_bytes(g, ps);
#define LQCD_CONV(A, B) \
    if (pd == A && ps == B) { convert_k<A, B><<<grid, block, 0, st>>>(dst, src, g.vh, nhalf, hbd, hbs); return; }
    LQCD_CONV(LQCD_F64, LQCD_F32)
    LQCD_CONV(LQCD_F64, LQCD_F16)
    LQCD_CONV(LQCD_F32, LQCD_F64)
    LQCD_CONV(LQCD_F32, LQCD_F16)
    LQCD_CONV(LQCD_F16, LQCD_F64)
    LQCD_CONV(LQCD_F16, LQCD_F32)
#undef LQCD_CONV
}

void launch_reduce(const Geom &g, int nhalf, const char *a, const char *b, int prec,
                   double *partial, hipStream_t st) {
    const int64_t nb = reduce_blocks(g, nhalf);
    const int64_t hb = (int64_t)half_spinor_bytes(g, prec);
    dim3 grid((unsigned)nb), block(RED_BLOCK);
    const bool dot = b != nullptr;
#define LQCD_RED(P)                                                                             \
    if (prec == P) {                                                                            \
        if (dot) reduce_k<P, true><<<grid, block, 0, st>>>(a, b, g.vh, nhalf, hb, partial);     \
        else reduce_k<P, false><<<grid, block, 0, st>>>(a, b, g.vh, nhalf, hb, partial);        \
        return;                                                                                 \
    }
    LQCD_RED(LQCD_F64)
    LQCD_RED(LQCD_F32)
    LQCD_RED(LQCD_F16)
#undef LQCD_RED
}

}  // namespace lqcd

using namespace lqcd;

static int subset_halves(int subset) {
    return subset == LQCD_FULL ? 2 : (subset == LQCD_EVEN || subset == LQCD_ODD) ? 1 : 0;
}

static bool al16(const void *p) { return p && ((uintptr_t)p & 15) == 0; }

extern "C" size_t lqcd_reduce_workspace_bytes(const lqcd_geom_t *gg, int subset) {
    Geom g;
    const int nh = subset_halves(subset);
    if (!make_geom(gg, &g) || !nh) return 0;
    return (size_t)(2 * reduce_blocks(g, nh) + 2) * sizeof(double);
}

static int reduce_entry(const lqcd_geom_t *gg, int subset, const void *a, const void *b,
                        int prec, void *ws, double *result, void *stream) {
    Geom g;
    const int nh = subset_halves(subset);
    if (!make_geom(gg, &g) || !nh || !valid_prec(prec)) return LQCD_EINVAL;
    if (!al16(a) || (b && !al16(b)) || !al16(ws) || !result) return LQCD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    double *partial = (double *)ws;
    const int64_t nb = reduce_blocks(g, nh);
    double *out = partial + 2 * nb;
#if LQCD_REDUCE_ATOMIC
    out = partial;
    hipError_t ez = hipMemsetAsync(out, 0, 2 * sizeof(double), st);
    if (ez != hipSuccess) {
        set_hip_error(ez);
        return LQCD_EHIP;
    }
    launch_reduce(g, nh, (const char *)a, (const char *)b, prec, partial, st);
#else
    launch_reduce(g, nh, (const char *)a, (const char *)b, prec, partial, st);
    launch_finalize(partial, nb, 2, out, st);
#endif
    int rc = check_launch();
    if (rc) return rc;
    double host[2];
    hipError_t e = hipMemcpyAsync(host, out, sizeof(host), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_hip_error(e);
        return LQCD_EHIP;
    }
    result[0] = host[0];
    if (b) result[1] = host[1];
    return LQCD_OK;
}

extern "C" int lqcd_dot(const lqcd_geom_t *g, int subset, const void *a, const void *b, int prec,
                        void *workspace, double *result, void *stream) {
    if (!b) return LQCD_EINVAL;
    return reduce_entry(g, subset, a, b, prec, workspace, result, stream);
}

// ---------------------------------------------------------------------------
// allocation-free inner product: the block partials live in a static device
// array instead of caller workspace
// ---------------------------------------------------------------------------

// Doubles of the static scratch: two per reduction block plus the two-double
// result, 1 MiB in all (every GPU the library runs on keeps its own copy until
// the process ends).
constexpr int64_t NOALLOC_DOUBLES = (int64_t)1 << 17;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEVICES = 64;
static std::mutex scratch_mutex;
static double *scratch_ptr[MAX_DEVICES] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the host-side name of the array is not a device
// address and must never reach a kernel).
static int scratch_address(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_hip_error(e);
        return LQCD_EHIP;
    }
    if (dev < 0 || dev >= MAX_DEVICES) return LQCD_EINVAL;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return LQCD_EHIP;
        }
        scratch_ptr[dev] = (double *)p;
    }
    *out = scratch_ptr[dev];
    return LQCD_OK;
}

// two doubles per block of RED_BLOCK sites, plus the result
static_assert((NOALLOC_DOUBLES - 2) / 2 * RED_BLOCK == LQCD_DOT_NOALLOC_MAX_SITES,
              "the header's site limit matches the static scratch");

extern "C" int lqcd_dot_noalloc(const lqcd_geom_t *gg, int subset, const void *a, const void *b,
                                int prec, double *result, void *stream) {
    Geom g;
    const int nh = subset_halves(subset);
    if (!b || !make_geom(gg, &g) || !nh || !valid_prec(prec)) return LQCD_EINVAL;
    if (!al16(a) || !al16(b) || !result) return LQCD_EINVAL;
    const int64_t nb = reduce_blocks(g, nh);
    if (2 * nb + 2 > NOALLOC_DOUBLES) return LQCD_ESMALL;
    double *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc) return rc;
    // every partial is written by the reduction before the final sum reads
    // it, so nothing left over from an earlier call needs clearing
    return reduce_entry(gg, subset, a, b, prec, ws, result, stream);
}

extern "C" int lqcd_norm2(const lqcd_geom_t *g, int subset, const void *a, int prec,
                          void *workspace, double *result, void *stream) {
    return reduce_entry(g, subset, a, nullptr, prec, workspace, result, stream);
}

extern "C" int lqcd_axpby(const lqcd_geom_t *gg, int subset, double a, const void *x, double b,
                          void *y, int prec, void *stream) {
    Geom g;
    const int nh = subset_halves(subset);
    if (!make_geom(gg, &g) || !nh || !valid_prec(prec)) return LQCD_EINVAL;
    if (!al16(x) || !al16(y)) return LQCD_EINVAL;
    const int64_t n = g.vh * nh;
    const int64_t hb = (int64_t)half_spinor_bytes(g, prec);
    dim3 grid((unsigned)((n + RED_BLOCK - 1) / RED_BLOCK)), block(RED_BLOCK);
    hipStream_t st = (hipStream_t)stream;
    if (prec == LQCD_F64) axpby_k<LQCD_F64><<<grid, block, 0, st>>>(a, (const char *)x, b, (char *)y, g.vh, nh, hb);
    else if (prec == LQCD_F32) axpby_k<LQCD_F32><<<grid, block, 0, st>>>(a, (const char *)x, b, (char *)y, g.vh, nh, hb);
    else axpby_k<LQCD_F16><<<grid, block, 0, st>>>(a, (const char *)x, b, (char *)y, g.vh, nh, hb);
    return check_launch();
}

extern "C" int lqcd_convert(const lqcd_geom_t *gg, int subset, void *dst, int dst_prec,
                            const void *src, int src_prec, void *stream) {
    Geom g;
    const int nh = subset_halves(subset);
    if (!make_geom(gg, &g) || !nh || !valid_prec(dst_prec) || !valid_prec(src_prec)) return LQCD_EINVAL;
    if (!al16(dst) || !al16(src) || dst == src) return LQCD_EINVAL;
    launch_convert(g, nh, (char *)dst, dst_prec, (const char *)src, src_prec, (hipStream_t)stream);
    return check_launch();
}
