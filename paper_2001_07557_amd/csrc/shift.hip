// Shifts.
//
// lqcd_cshift: out(x) = bc_mu^[crossing] in(x + dir mu) on a full spinor field,
// the shift the paper's stencils are built from (Sec. 3.1).  With one site per
// lane a shift is an indexed load of the neighbour, so the lane
// rearrangement the paper needs at sublattice boundaries never arises; the
// boundary phase is applied on the way.
//
// lqcd_split_rotate: the paper's lane permutation (Sec. 3.1) as a primitive on
// arrays of vectors: each vector of VL elements is split into s blocks of
// w = VL/s elements and every block is rotated left by r.  When VL divides the
// wavefront (64) the permutation happens in registers (ds_bpermute through
// __shfl) between a coalesced load and a coalesced store; otherwise each lane
// gathers its source element.

#include "lqcd_internal.h"
#include "hop_common.h"

namespace lqcd {

template <int P, int MU, bool FWD>
__device__ __forceinline__ void shift_site(const Geom &g, char *out, const char *in, int64_t hb,
                                           int p, int64_t s) {
    using T = typename real_of<P>::type;
    const Coord c = cb_coords(g, p, s);
    bool flip;
    const int64_t nb = hop_neighbour<MU, FWD>(g, s, c, flip);
    const char *src = in + (p ^ 1) * hb;
    char *dst = out + p * hb;
    if constexpr (P == LQCD_F16) {
        // copy the stored binary16 words and carry the sign in the site scale
        const char *ts = src + (nb >> TILE_SHIFT) * spinor_tile_bytes(P);
        char *td = dst + (s >> TILE_SHIFT) * spinor_tile_bytes(P);
        const int ls = (int)(nb & (TILE - 1)), ld = (int)(s & (TILE - 1));
#pragma unroll
        for (int k = 0; k < 3; ++k)
            reinterpret_cast<v4u *>(td)[k * TILE + ld] = reinterpret_cast<const v4u *>(ts)[k * TILE + ls];
        const float sc = reinterpret_cast<const float *>(ts + 3 * TILE * WORD)[ls];
        reinterpret_cast<float *>(td + 3 * TILE * WORD)[ld] = flip ? -sc : sc;
    } else {
        cplx<T> v[12];
        load_spinor<P>(src, nb, v);
        if (flip) {
#pragma unroll
            for (int k = 0; k < 12; ++k) v[k] = {-v[k].re, -v[k].im};
        }
        store_spinor<P>(dst, s, v);
    }
}

template <int P>
__global__ __launch_bounds__(256) void cshift_k(Geom g, char *out, const char *in, int64_t hb,
                                                int mu, int fwd, int64_t bpp) {
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int p = blk >= bpp ? 1 : 0;
    const int64_t s = (blk - p * bpp) * 256 + threadIdx.x;
    if (s >= g.vh) return;
    switch (mu * 2 + fwd) {
        case 0: shift_site<P, 0, false>(g, out, in, hb, p, s); break;
        case 1: shift_site<P, 0, true>(g, out, in, hb, p, s); break;
        case 2: shift_site<P, 1, false>(g, out, in, hb, p, s); break;
        case 3: shift_site<P, 1, true>(g, out, in, hb, p, s); break;
        case 4: shift_site<P, 2, false>(g, out, in, hb, p, s); break;
        case 5: shift_site<P, 2, true>(g, out, in, hb, p, s); break;
        case 6: shift_site<P, 3, false>(g, out, in, hb, p, s); break;
        default: shift_site<P, 3, true>(g, out, in, hb, p, s); break;
    }
}

// One 16-byte word of one site per thread: a wave moves word `word` of the
// 64 sites of one tile (FP64 12 words, FP32 6, binary16 3 and the scale),
// so every load and store is one coalesced 1 KB run (256 B for the scale).
template <int P, int MU, bool FWD>
__device__ __forceinline__ void shift_word(const Geom &g, char *out, const char *in, int64_t hb,
                                           int p, int64_t s, int word) {
    const Coord c = cb_coords(g, p, s);
    bool flip;
    const int64_t nb = hop_neighbour<MU, FWD>(g, s, c, flip);
    const char *ts = in + (p ^ 1) * hb + (nb >> TILE_SHIFT) * spinor_tile_bytes(P);
    char *td = out + p * hb + (s >> TILE_SHIFT) * spinor_tile_bytes(P);
    const int ls = (int)(nb & (TILE - 1)), ld = (int)(s & (TILE - 1));
    if constexpr (P == LQCD_F16) {
        if (word < 3) {
            reinterpret_cast<v4u *>(td)[word * TILE + ld] = reinterpret_cast<const v4u *>(ts)[word * TILE + ls];
        } else {
            const float sc = reinterpret_cast<const float *>(ts + 3 * TILE * WORD)[ls];
            reinterpret_cast<float *>(td + 3 * TILE * WORD)[ld] = flip ? -sc : sc;
        }
    } else if constexpr (P == LQCD_F64) {
        v2d v = reinterpret_cast<const v2d *>(ts)[word * TILE + ls];
        if (flip) v = -v;
        reinterpret_cast<v2d *>(td)[word * TILE + ld] = v;
    } else {
        v4f v = reinterpret_cast<const v4f *>(ts)[word * TILE + ls];
        if (flip) v = -v;
        reinterpret_cast<v4f *>(td)[word * TILE + ld] = v;
    }
}

template <int P>
__global__ __launch_bounds__(256) void cshift_words_k(Geom g, char *out, const char *in, int64_t hb,
                                                      int mu, int fwd, int64_t wpp) {
    constexpr int NW = P == LQCD_F64 ? 12 : P == LQCD_F32 ? 6 : 4;
    const int64_t gw = xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (gw >= 2 * wpp) return;
    const int p = gw >= wpp ? 1 : 0;
    const int64_t lw = gw - p * wpp;
    const int64_t tile = lw / NW;
    const int word = (int)(lw - tile * NW);
    const int64_t s = tile * TILE + (threadIdx.x & 63);
    if (s >= g.vh) return;
    switch (mu * 2 + fwd) {
        case 0: shift_word<P, 0, false>(g, out, in, hb, p, s, word); break;
        case 1: shift_word<P, 0, true>(g, out, in, hb, p, s, word); break;
        case 2: shift_word<P, 1, false>(g, out, in, hb, p, s, word); break;
        case 3: shift_word<P, 1, true>(g, out, in, hb, p, s, word); break;
        case 4: shift_word<P, 2, false>(g, out, in, hb, p, s, word); break;
        case 5: shift_word<P, 2, true>(g, out, in, hb, p, s, word); break;
        case 6: shift_word<P, 3, false>(g, out, in, hb, p, s, word); break;
        default: shift_word<P, 3, true>(g, out, in, hb, p, s, word); break;
    }
}

// split_rotate, vectors that tile the wavefront: VL | 64, permutation in registers.
template <typename E>
__global__ __launch_bounds__(256) void split_rotate_wave_k(E *out, const E *in, int64_t n,
                                                           int vl, int w, int r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    // every lane takes part in the exchange; lanes past n carry a dummy value
    E x = i < n ? in[i] : E{};
    const int e = lane % vl;                       // element index within its vector
    const int src = (lane - e) + (e / w) * w + (e % w + r) % w;
    E y;
    if constexpr (sizeof(E) == 8) {
        y = __shfl(x, src, 64);
    } else {
        y.x = __shfl(x.x, src, 64);
        y.y = __shfl(x.y, src, 64);
    }
    if (i < n) out[i] = y;
}

// split_rotate, any VL: each lane gathers its source element.
template <typename E>
__global__ __launch_bounds__(256) void split_rotate_gather_k(E *out, const E *in, int64_t n,
                                                             int vl, int w, int r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t base = i - i % vl;
    const int e = (int)(i - base);
    out[i] = in[base + (e / w) * w + (e % w + r) % w];
}

}  // namespace lqcd

using namespace lqcd;

extern "C" int lqcd_cshift(const lqcd_geom_t *gg, void *out, const void *in, int mu, int dir,
                           int prec, void *stream) {
    Geom g;
    if (!make_geom(gg, &g) || !valid_prec(prec)) return LQCD_EINVAL;
    if (mu < 0 || mu > 3 || (dir != 1 && dir != -1)) return LQCD_EINVAL;
    if (!out || !in || out == in || (((uintptr_t)out | (uintptr_t)in) & 15)) return LQCD_EINVAL;
    const int64_t hb = (int64_t)half_spinor_bytes(g, prec);
    hipStream_t st = (hipStream_t)stream;
    const int fwd = dir > 0 ? 1 : 0;
    if (LQCD_LAYOUT_AOS) {
        // site-major ablation layout: one site per thread
        const int64_t bpp = (g.vh + 255) / 256;
        dim3 grid((unsigned)(2 * bpp)), block(256);
        if (prec == LQCD_F64) cshift_k<LQCD_F64><<<grid, block, 0, st>>>(g, (char *)out, (const char *)in, hb, mu, fwd, bpp);
        else if (prec == LQCD_F32) cshift_k<LQCD_F32><<<grid, block, 0, st>>>(g, (char *)out, (const char *)in, hb, mu, fwd, bpp);
        else cshift_k<LQCD_F16><<<grid, block, 0, st>>>(g, (char *)out, (const char *)in, hb, mu, fwd, bpp);
        return check_launch();
    }
    // one word per thread: FP64 at 32^4 80 -> 75 us per shift in t (62.8% ->
    // 67.3% of 8 TB/s, HIP events, two runs each), FP32 unchanged
    const int nw = prec == LQCD_F64 ? 12 : prec == LQCD_F32 ? 6 : 4;
    const int64_t wpp = g.ntiles * nw;  // waves per parity
    dim3 grid((unsigned)((2 * wpp + 3) / 4)), block(256);
    if (prec == LQCD_F64) cshift_words_k<LQCD_F64><<<grid, block, 0, st>>>(g, (char *)out, (const char *)in, hb, mu, fwd, wpp);
    else if (prec == LQCD_F32) cshift_words_k<LQCD_F32><<<grid, block, 0, st>>>(g, (char *)out, (const char *)in, hb, mu, fwd, wpp);
    else cshift_words_k<LQCD_F16><<<grid, block, 0, st>>>(g, (char *)out, (const char *)in, hb, mu, fwd, wpp);
    return check_launch();
}

extern "C" int lqcd_split_rotate(void *out, const void *in, int64_t nvec, int vl, int s, int r,
                                 int elem_bytes, void *stream) {
    if (!out || !in || out == in || nvec < 0 || vl < 1 || s < 1 || vl % s) return LQCD_EINVAL;
    if (elem_bytes != 8 && elem_bytes != 16) return LQCD_EINVAL;
    if (((uintptr_t)out | (uintptr_t)in) & (elem_bytes - 1)) return LQCD_EINVAL;
    const int64_t n = nvec * (int64_t)vl;
    if (nvec > 0 && n / nvec != vl) return LQCD_EINVAL;
    if (n == 0) return LQCD_OK;
    if ((n + 255) / 256 > 0x7fffffff) return LQCD_EINVAL;
    const int w = vl / s;
    const int rr = ((r % w) + w) % w;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipStream_t st = (hipStream_t)stream;
    const bool in_wave = 64 % vl == 0;
    if (elem_bytes == 8) {
        if (in_wave) split_rotate_wave_k<double><<<grid, block, 0, st>>>((double *)out, (const double *)in, n, vl, w, rr);
        else split_rotate_gather_k<double><<<grid, block, 0, st>>>((double *)out, (const double *)in, n, vl, w, rr);
    } else {
        if (in_wave) split_rotate_wave_k<double2><<<grid, block, 0, st>>>((double2 *)out, (const double2 *)in, n, vl, w, rr);
        else split_rotate_gather_k<double2><<<grid, block, 0, st>>>((double2 *)out, (const double2 *)in, n, vl, w, rr);
    }
    return check_launch();
}
