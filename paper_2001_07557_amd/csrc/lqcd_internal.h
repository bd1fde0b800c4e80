// Internal definitions shared by the HIP translation units of liblqcd.so:
// geometry, the tiled structure-of-arrays layouts, complex arithmetic and the
// per-site loaders/stores for every storage precision.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/lqcd.h"
#include "fastdiv.h"

namespace lqcd {

// Sites per tile: one wavefront reads one 16-byte word of 64 sites at once.
constexpr int TILE = 64;
constexpr int TILE_SHIFT = 6;
constexpr int WORD = 16;

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------

struct Geom {
    int L[4];      // Lx, Ly, Lz, Lt
    int bc[4];     // +1 / -1
    int lxh;       // Lx / 2
    int64_t vh;    // sites per parity
    int64_t ntiles;
    // checkerboard-index strides of one step in y, z, t
    int64_t sy, sz, st;
    // divisors lxh, Ly, Lz of a checkerboard index (site -> coordinates)
    FastDiv dx, dy, dz;
};

bool make_geom(const lqcd_geom_t *g, Geom *out);

// ---------------------------------------------------------------------------
// internal layout sizes
// ---------------------------------------------------------------------------

// Spinor tile: F64 12 words (one double2 complex each), F32 6 words (two
// complexes per float4), F16 3 words (four complexes per 8 halves) followed
// by 64 FP32 scales (256 bytes).
__host__ __device__ constexpr int spinor_tile_bytes(int prec) {
    return prec == LQCD_F64 ? 12 * TILE * WORD
         : prec == LQCD_F32 ? 6 * TILE * WORD
                            : 3 * TILE * WORD + TILE * 4;
}

// Link tile (one direction): F64 18 -> 9 words, F64 12 -> 6 words,
// F32 18 -> 4 words + one 8-byte half word, F32 12 -> 3 words,
// F16 12 -> 1 word + one 8-byte half word.
__host__ __device__ constexpr int link_tile_bytes(int prec, int link) {
    return prec == LQCD_F64 ? (link == 18 ? 9 : 6) * TILE * WORD
         : prec == LQCD_F32 ? (link == 18 ? 4 * TILE * WORD + TILE * 8 : 3 * TILE * WORD)
                            : TILE * WORD + TILE * 8;
}

// binary16 hops address a parity's links and a half spinor field by 32-bit
// offsets, so each must stay below 4 GB: at most this many tiles per parity
// (V/2 <= 44.7M sites); larger binary16 hop launches return LQCD_EINVAL
constexpr int64_t F16_MAX_TILES = 0xffffffffLL / (4 * link_tile_bytes(LQCD_F16, 12));
static_assert(F16_MAX_TILES * spinor_tile_bytes(LQCD_F16) <= 0xffffffffLL, "binary16 spinor offsets");

inline bool valid_prec(int p) { return p == LQCD_F64 || p == LQCD_F32 || p == LQCD_F16; }
inline bool valid_link(int prec, int link) {
    if (link != 18 && link != 12) return false;
    if (prec == LQCD_F16 && link != 12) return false;
    return valid_prec(prec);
}

inline size_t half_spinor_bytes(const Geom &g, int prec) {
    return (size_t)g.ntiles * spinor_tile_bytes(prec);
}
inline size_t gauge_bytes(const Geom &g, int prec, int link) {
    return (size_t)2 * g.ntiles * 4 * link_tile_bytes(prec, link);
}

// ---------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------

template <typename T>
struct cplx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> scale(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename T>
__device__ __forceinline__ cplx<T> cmul_conj(cplx<T> a, cplx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }

template <typename T>
__device__ __forceinline__ T fmad(T a, T b, T c) {
    if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
    else return __builtin_fmaf(a, b, c);
}

// a0 b0 + a1 b1 + a2 b2 as two chains of fused multiply-adds (one product
// and five FMAs per component; the operator form costs two more additions
// per term).
template <typename T>
__device__ __forceinline__ cplx<T> cdot3(cplx<T> a0, cplx<T> b0, cplx<T> a1, cplx<T> b1,
                                         cplx<T> a2, cplx<T> b2) {
    T re = a0.re * b0.re, im = a0.re * b0.im;
    re = fmad(-a0.im, b0.im, re);
    im = fmad(a0.im, b0.re, im);
    re = fmad(a1.re, b1.re, re);
    im = fmad(a1.re, b1.im, im);
    re = fmad(-a1.im, b1.im, re);
    im = fmad(a1.im, b1.re, im);
    re = fmad(a2.re, b2.re, re);
    im = fmad(a2.re, b2.im, im);
    re = fmad(-a2.im, b2.im, re);
    im = fmad(a2.im, b2.re, im);
    return {re, im};
}

// conj(a0) b0 + conj(a1) b1 + conj(a2) b2, the same way.
template <typename T>
__device__ __forceinline__ cplx<T> cdot3c(cplx<T> a0, cplx<T> b0, cplx<T> a1, cplx<T> b1,
                                          cplx<T> a2, cplx<T> b2) {
    T re = a0.re * b0.re, im = a0.re * b0.im;
    re = fmad(a0.im, b0.im, re);
    im = fmad(-a0.im, b0.re, im);
    re = fmad(a1.re, b1.re, re);
    im = fmad(a1.re, b1.im, im);
    re = fmad(a1.im, b1.im, re);
    im = fmad(-a1.im, b1.re, im);
    re = fmad(a2.re, b2.re, re);
    im = fmad(a2.re, b2.im, im);
    re = fmad(a2.im, b2.im, re);
    im = fmad(-a2.im, b2.re, im);
    return {re, im};
}

// conj(a b - c d) with fused multiply-adds.
template <typename T>
__device__ __forceinline__ cplx<T> conj_cross(cplx<T> a, cplx<T> b, cplx<T> c, cplx<T> d) {
    T re = a.re * b.re, im = -(a.re * b.im);
    re = fmad(-a.im, b.im, re);
    im = fmad(-a.im, b.re, im);
    re = fmad(-c.re, d.re, re);
    im = fmad(c.re, d.im, im);
    re = fmad(c.im, d.im, re);
    im = fmad(c.im, d.re, im);
    return {re, im};
}

// Multiply by one of {1, -1, i, -i}, coded as 0, 1, 2, 3.
template <int C, typename T>
__device__ __forceinline__ cplx<T> mul_unit(cplx<T> a) {
    if constexpr (C == 0) return a;
    else if constexpr (C == 1) return {-a.re, -a.im};
    else if constexpr (C == 2) return {-a.im, a.re};
    else return {a.im, -a.re};
}

// Native vector types for 16- and 8-byte accesses.
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));

// Ablation switch: 1 stores FP64/FP32 fields site-major as arrays of complex
// {re, im} pairs (the layout of the paper's CPU/VE kernels) instead of the
// 64-site tiles; buffer sizes are identical.  binary16 always uses tiles.
#ifndef LQCD_LAYOUT_AOS
#define LQCD_LAYOUT_AOS 0
#endif

// The stencil kernels (hop, force) store their results with the non-temporal
// hint: nothing in the launch reads them again, and plain stores would evict
// the neighbour spinors that the L2 holds for reuse (ablation switch, 0 =
// plain stores).  Pure streaming kernels have no such reuse to protect and
// use plain stores.
#ifndef LQCD_OUT_NT
#define LQCD_OUT_NT 1
#endif
constexpr bool OUT_NT = LQCD_OUT_NT != 0;

// Links are read once per application: by default they are loaded with the
// non-temporal hint (the hop kernels choose per launch; 0 switches it off).
#ifndef LQCD_LINK_NT
#define LQCD_LINK_NT 1
#endif
template <bool NT, typename V>
__device__ __forceinline__ V stream_load(const V *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <int P> struct real_of { using type = float; };
template <> struct real_of<LQCD_F64> { using type = double; };

// ---------------------------------------------------------------------------
// per-site loads and stores, spinors (12 complexes, index spin*3 + colour)
// ---------------------------------------------------------------------------

// non-temporal spinor loads (ablation switch; off: the hop kernels rely on the
// L2 keeping neighbour spinors between the eight hops that read each one)
#ifndef LQCD_SPINOR_NT
#define LQCD_SPINOR_NT 0
#endif
template <int P, bool NT = (LQCD_SPINOR_NT != 0)>
__device__ __forceinline__ void load_spinor(const char *__restrict__ base, int64_t s,
                                            cplx<typename real_of<P>::type> v[12]) {
    const int64_t tile = s >> TILE_SHIFT;
    const int lane = (int)(s & (TILE - 1));
    const char *t = base + tile * spinor_tile_bytes(P);
    if constexpr (LQCD_LAYOUT_AOS && P == LQCD_F64) {
        const v2d *w = reinterpret_cast<const v2d *>(base + s * 192);
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = {w[k].x, w[k].y};
    } else if constexpr (LQCD_LAYOUT_AOS && P == LQCD_F32) {
        const v2f *w = reinterpret_cast<const v2f *>(base + s * 96);
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = {w[k].x, w[k].y};
    } else if constexpr (P == LQCD_F64) {
        const v2d *w = reinterpret_cast<const v2d *>(t) + lane;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            v2d d = stream_load<NT>(&w[k * TILE]);
            v[k] = {d.x, d.y};
        }
    } else if constexpr (P == LQCD_F32) {
        const v4f *w = reinterpret_cast<const v4f *>(t) + lane;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            v4f f = stream_load<NT>(&w[k * TILE]);
            v[2 * k] = {f.x, f.y};
            v[2 * k + 1] = {f.z, f.w};
        }
    } else {
        const v4u *w = reinterpret_cast<const v4u *>(t) + lane;
        const float sc = stream_load<NT>(reinterpret_cast<const float *>(t + 3 * TILE * WORD) + lane);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v4u q = stream_load<NT>(&w[k * TILE]);
            uint32_t u[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                __half2 h = *reinterpret_cast<__half2 *>(&u[j]);
                float2 f = __half22float2(h);
                v[4 * k + j] = {f.x * sc, f.y * sc};
            }
        }
    }
}

// Element type a hop reads spinors in: the arithmetic type, except binary16
// storage, whose stored values go unconverted into the hop's packed binary16
// projection.
template <int P> struct hop_elem { using type = typename real_of<P>::type; };
template <> struct hop_elem<LQCD_F16> { using type = _Float16; };
typedef _Float16 v2h __attribute__((ext_vector_type(2)));

// Load for a hop: binary16 storage returns the stored (unscaled) values and
// multiplies `factor` by the site's scale, which the hop then applies to the
// projected half-spinor (12 products instead of 24).
template <int P>
__device__ __forceinline__ void load_spinor_hop(const char *__restrict__ base, int64_t s,
                                                cplx<typename hop_elem<P>::type> v[12],
                                                typename real_of<P>::type &factor) {
    if constexpr (P == LQCD_F16) {
        // 32-bit offsets from the field's base (binary16 hop launches are
        // limited to fields below 4 GB): the loads take the base from
        // scalar registers and need no 64-bit address arithmetic
        const int lane = (int)(s & (TILE - 1));
        const uint32_t toff = (uint32_t)(s >> TILE_SHIFT) * (uint32_t)spinor_tile_bytes(P);
        const v4u *w = reinterpret_cast<const v4u *>(base + (uint64_t)(toff + (uint32_t)lane * WORD));
        factor *= *reinterpret_cast<const float *>(base + (uint64_t)(toff + 3u * TILE * WORD + (uint32_t)lane * 4u));
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v4u q = w[k * TILE];
            uint32_t u[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const v2h h = __builtin_bit_cast(v2h, u[j]);
                v[4 * k + j] = {h.x, h.y};
            }
        }
    } else {
        load_spinor<P>(base, s, v);
    }
}

// Store of one word; NT marks it non-temporal (a result that no later work of
// the same kernel reads).
template <bool NT, typename V>
__device__ __forceinline__ void put(V *p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <int P, bool NT = false>
__device__ __forceinline__ void store_spinor(char *__restrict__ base, int64_t s,
                                             const cplx<typename real_of<P>::type> v[12]) {
    const int64_t tile = s >> TILE_SHIFT;
    const int lane = (int)(s & (TILE - 1));
    char *t = base + tile * spinor_tile_bytes(P);
    if constexpr (LQCD_LAYOUT_AOS && P == LQCD_F64) {
        v2d *w = reinterpret_cast<v2d *>(base + s * 192);
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] = v2d{v[k].re, v[k].im};
    } else if constexpr (LQCD_LAYOUT_AOS && P == LQCD_F32) {
        v2f *w = reinterpret_cast<v2f *>(base + s * 96);
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] = v2f{v[k].re, v[k].im};
    } else if constexpr (P == LQCD_F64) {
        v2d *w = reinterpret_cast<v2d *>(t) + lane;
#pragma unroll
        for (int k = 0; k < 12; ++k) put<NT>(&w[k * TILE], v2d{v[k].re, v[k].im});
    } else if constexpr (P == LQCD_F32) {
        v4f *w = reinterpret_cast<v4f *>(t) + lane;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            put<NT>(&w[k * TILE], v4f{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im});
    } else {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        // stored value = binary16(real * (1/m)), the reciprocal rounded once in FP32
        const float inv = 1.f / (m > 0.f ? m : 1.f);
        v4u *w = reinterpret_cast<v4u *>(t) + lane;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint32_t u[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                __half2 h = __floats2half2_rn(v[4 * k + j].re * inv, v[4 * k + j].im * inv);
                u[j] = *reinterpret_cast<uint32_t *>(&h);
            }
            put<NT>(&w[k * TILE], v4u{u[0], u[1], u[2], u[3]});
        }
        put<NT>(reinterpret_cast<float *>(t + 3 * TILE * WORD) + lane, m);
    }
}

// ---------------------------------------------------------------------------
// per-site loads and stores, links (9 complexes, index row*3 + col)
// ---------------------------------------------------------------------------

// Row 2 of an SU(3) matrix from rows 0 and 1: conj(row0 x row1).
template <typename T>
__device__ __forceinline__ void reconstruct_row2(cplx<T> u[9]) {
    u[6] = conj_cross(u[1], u[5], u[2], u[4]);
    u[7] = conj_cross(u[2], u[3], u[0], u[5]);
    u[8] = conj_cross(u[0], u[4], u[1], u[3]);
}

// Address of the link tile of direction mu for parity p and site tile `tile`.
template <int P, int LK>
__device__ __forceinline__ const char *link_tile(const char *U, int64_t ntiles, int p,
                                                 int64_t tile, int mu) {
    return U + (((int64_t)p * ntiles + tile) * 4 + mu) * (int64_t)link_tile_bytes(P, LK);
}

template <int P, int LK, bool NT = (LQCD_LINK_NT != 0)>
__device__ __forceinline__ void load_link(const char *__restrict__ U, int64_t ntiles, int p,
                                          int64_t s, int mu,
                                          cplx<typename real_of<P>::type> u[9]) {
    const int lane = (int)(s & (TILE - 1));
    const char *t = link_tile<P, LK>(U, ntiles, p, s >> TILE_SHIFT, mu);
    if constexpr (LQCD_LAYOUT_AOS && P != LQCD_F16) {
        // site-major: [parity][site][mu][complex]
        constexpr int n = LK == 18 ? 9 : 6;
        using T = typename real_of<P>::type;
        const char *l = U + (((int64_t)p * ntiles * TILE + s) * 4 + mu) * (int64_t)(n * 2 * sizeof(T));
#pragma unroll
        for (int k = 0; k < n; ++k) {
            if constexpr (P == LQCD_F64) {
                v2d d = stream_load<NT>(reinterpret_cast<const v2d *>(l) + k);
                u[k] = {d.x, d.y};
            } else {
                v2f d = stream_load<NT>(reinterpret_cast<const v2f *>(l) + k);
                u[k] = {d.x, d.y};
            }
        }
    } else if constexpr (P == LQCD_F64) {
        const v2d *w = reinterpret_cast<const v2d *>(t) + lane;
        constexpr int n = LK == 18 ? 9 : 6;
#pragma unroll
        for (int k = 0; k < n; ++k) {
            v2d d = stream_load<NT>(&w[k * TILE]);
            u[k] = {d.x, d.y};
        }
    } else if constexpr (P == LQCD_F32) {
        const v4f *w = reinterpret_cast<const v4f *>(t) + lane;
        constexpr int n4 = LK == 18 ? 4 : 3;
#pragma unroll
        for (int k = 0; k < n4; ++k) {
            v4f f = stream_load<NT>(&w[k * TILE]);
            u[2 * k] = {f.x, f.y};
            u[2 * k + 1] = {f.z, f.w};
        }
        if constexpr (LK == 18) {
            const v2f *w2 = reinterpret_cast<const v2f *>(t + 4 * TILE * WORD) + lane;
            v2f f = stream_load<NT>(w2);
            u[8] = {f.x, f.y};
        }
    } else {
        const v4u *w = reinterpret_cast<const v4u *>(t) + lane;
        v4u q = stream_load<NT>(w);
        const v2u *w2 = reinterpret_cast<const v2u *>(t + TILE * WORD) + lane;
        v2u q2 = stream_load<NT>(w2);
        uint32_t a[6] = {q.x, q.y, q.z, q.w, q2.x, q2.y};
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            __half2 h = *reinterpret_cast<__half2 *>(&a[j]);
            float2 f = __half22float2(h);
            u[j] = {f.x, f.y};
        }
    }
    if constexpr (LK == 12) reconstruct_row2(u);
}

// Store a link in the layout (rows 0, 1 only for LINK12).
template <int P, int LK, bool NT = false>
__device__ __forceinline__ void store_link(char *__restrict__ U, int64_t ntiles, int p,
                                           int64_t s, int mu,
                                           const cplx<typename real_of<P>::type> u[9]) {
    const int lane = (int)(s & (TILE - 1));
    char *t = const_cast<char *>(link_tile<P, LK>(U, ntiles, p, s >> TILE_SHIFT, mu));
    if constexpr (LQCD_LAYOUT_AOS && P != LQCD_F16) {
        constexpr int n = LK == 18 ? 9 : 6;
        using T = typename real_of<P>::type;
        char *l = U + (((int64_t)p * ntiles * TILE + s) * 4 + mu) * (int64_t)(n * 2 * sizeof(T));
#pragma unroll
        for (int k = 0; k < n; ++k) {
            if constexpr (P == LQCD_F64) reinterpret_cast<v2d *>(l)[k] = v2d{u[k].re, u[k].im};
            else reinterpret_cast<v2f *>(l)[k] = v2f{u[k].re, u[k].im};
        }
    } else if constexpr (P == LQCD_F64) {
        v2d *w = reinterpret_cast<v2d *>(t) + lane;
        constexpr int n = LK == 18 ? 9 : 6;
#pragma unroll
        for (int k = 0; k < n; ++k) put<NT>(&w[k * TILE], v2d{u[k].re, u[k].im});
    } else if constexpr (P == LQCD_F32) {
        v4f *w = reinterpret_cast<v4f *>(t) + lane;
        constexpr int n4 = LK == 18 ? 4 : 3;
#pragma unroll
        for (int k = 0; k < n4; ++k)
            put<NT>(&w[k * TILE], v4f{u[2 * k].re, u[2 * k].im, u[2 * k + 1].re, u[2 * k + 1].im});
        if constexpr (LK == 18) {
            v2f *w2 = reinterpret_cast<v2f *>(t + 4 * TILE * WORD) + lane;
            put<NT>(w2, v2f{u[8].re, u[8].im});
        }
    } else {
        uint32_t a[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            __half2 h = __floats2half2_rn(u[j].re, u[j].im);
            a[j] = *reinterpret_cast<uint32_t *>(&h);
        }
        v4u *w = reinterpret_cast<v4u *>(t) + lane;
        put<NT>(w, v4u{a[0], a[1], a[2], a[3]});
        v2u *w2 = reinterpret_cast<v2u *>(t + TILE * WORD) + lane;
        put<NT>(w2, v2u{a[4], a[5]});
    }
}

// ---------------------------------------------------------------------------
// checkerboard coordinates
// ---------------------------------------------------------------------------

struct Coord {
    int x, y, z, t;
};

// Site s (checkerboard index) of parity p -> coordinates (s < 2^30, so the
// quotients are 32-bit multiply-and-shift divisions).
__device__ __forceinline__ Coord cb_coords(const Geom &g, int p, int64_t s) {
    Coord c;
    const uint32_t si = (uint32_t)s;
    const uint32_t r1 = fdiv(si, g.dx);  // (y, z, t) row index
    const uint32_t r2 = fdiv(r1, g.dy);  // (z, t) plane index
    const uint32_t t = fdiv(r2, g.dz);
    const int xh = (int)(si - r1 * g.dx.d);
    c.y = (int)(r1 - r2 * g.dy.d);
    c.z = (int)(r2 - t * g.dz.d);
    c.t = (int)t;
    c.x = 2 * xh + ((p + c.y + c.z + c.t) & 1);
    return c;
}

// Logical block index for an XCD-aware launch: the hardware hands
// consecutive workgroups to the 8 XCDs in turn, so block b runs on XCD b % 8;
// renumbering gives every XCD one contiguous range of tiles (its own L2 then
// sees the neighbouring sites of its range).  A bijection for any nblocks.
__device__ __forceinline__ int64_t xcd_block(uint32_t b, uint32_t nblocks) {
    constexpr uint32_t NX = 8;
    const uint32_t q = nblocks / NX, r = nblocks % NX;
    const uint32_t x = b % NX, k = b / NX;
    return (int64_t)(x * q + (x < r ? x : r) + k);
}

// HIP error bookkeeping shared by the entry points.
void set_hip_error(hipError_t e);
int check_launch();

}  // namespace lqcd
