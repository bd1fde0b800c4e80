// The per-site hopping term shared by the operator and the solver kernels.
#pragma once

#include "lqcd_internal.h"

namespace lqcd {

constexpr int HOP_BLOCK = 128;

// Ends one hop: the accumulator is pinned in registers (an empty asm that
// reads and writes it) and the scheduler may not move instructions across.
// Without this the compiler sinks all hop arithmetic below the last load, so
// every loaded spinor and link stays live at once, the register demand
// exceeds the file and occupancy collapses to one wave per SIMD.
template <typename T>
__device__ __forceinline__ void hop_fence(cplx<T> acc[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) asm volatile("" : "+v"(acc[k].re), "+v"(acc[k].im));
    __builtin_amdgcn_sched_barrier(0);
}

struct HopArgs {
    Geom g;
    char *out[2];         // output half field for output parity p
    const char *in[2];    // input half field (opposite parity) read by output parity p
    const char *y[2];     // optional beta * y term, parity p
    const char *U;        // gauge field
    double alpha, beta;
    double *partial;      // optional per-block |out|^2
    int64_t bpp;          // blocks per parity
    int par0;             // parity of the first bpp blocks
    int xcd;              // XCD-aware block renumbering
};

int hop_launch(const HopArgs &a, int prec, int link, bool dag, int nparity, hipStream_t st);
int64_t hop_partials(const Geom &g, int nparity);

// Spin projection (1 + S g_mu): with the unit constants of the chiral basis,
//   h0 = psi_0 + S c0 psi_a0,   h1 = psi_1 + S c1 psi_a1,
// and the full four-row result is rebuilt from the two colour vectors
// chi = U h as  row 0 = chi0, row 1 = chi1, row a0 = S conj(c0) chi0,
// row a1 = S conj(c1) chi1  (the projector has rank two).
// Unit codes: 0 -> 1, 1 -> -1, 2 -> i, 3 -> -i.
template <int MU> struct Proj;
template <> struct Proj<0> { static constexpr int a0 = 3, c0 = 2, a1 = 2, c1 = 2; };
template <> struct Proj<1> { static constexpr int a0 = 3, c0 = 1, a1 = 2, c1 = 0; };
template <> struct Proj<2> { static constexpr int a0 = 2, c0 = 2, a1 = 3, c1 = 3; };
template <> struct Proj<3> { static constexpr int a0 = 2, c0 = 0, a1 = 3, c1 = 0; };

__host__ __device__ constexpr int neg_code(int c) { return c ^ 1; }
__host__ __device__ constexpr int conj_code(int c) { return c < 2 ? c : (c ^ 1); }

// Rows 0 and 1 of (1 + S g_mu) psi.
template <int MU, int S, typename T>
__device__ __forceinline__ void project_half(const cplx<T> psi[12], cplx<T> h0[3], cplx<T> h1[3]) {
    using PR = Proj<MU>;
    constexpr int k0 = S > 0 ? PR::c0 : neg_code(PR::c0);
    constexpr int k1 = S > 0 ? PR::c1 : neg_code(PR::c1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h0[c] = psi[c] + mul_unit<k0>(psi[PR::a0 * 3 + c]);
        h1[c] = psi[3 + c] + mul_unit<k1>(psi[PR::a1 * 3 + c]);
    }
}

// Project, multiply by U (or U^dag) and accumulate one hop into acc.
template <int MU, int S, bool UDAG, typename T>
__device__ __forceinline__ void hop_accumulate(const cplx<T> psi[12], const cplx<T> u[9], T sign,
                                               cplx<T> acc[12]) {
    using PR = Proj<MU>;
    constexpr int k0 = S > 0 ? PR::c0 : neg_code(PR::c0);
    constexpr int k1 = S > 0 ? PR::c1 : neg_code(PR::c1);
    constexpr int r0 = S > 0 ? conj_code(PR::c0) : neg_code(conj_code(PR::c0));
    constexpr int r1 = S > 0 ? conj_code(PR::c1) : neg_code(conj_code(PR::c1));
    cplx<T> h0[3], h1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h0[c] = scale(sign, psi[c] + mul_unit<k0>(psi[PR::a0 * 3 + c]));
        h1[c] = scale(sign, psi[3 + c] + mul_unit<k1>(psi[PR::a1 * 3 + c]));
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cplx<T> x0, x1;
        if constexpr (UDAG) {
            x0 = cmul_conj(u[a], h0[0]) + cmul_conj(u[3 + a], h0[1]) + cmul_conj(u[6 + a], h0[2]);
            x1 = cmul_conj(u[a], h1[0]) + cmul_conj(u[3 + a], h1[1]) + cmul_conj(u[6 + a], h1[2]);
        } else {
            x0 = u[3 * a] * h0[0] + u[3 * a + 1] * h0[1] + u[3 * a + 2] * h0[2];
            x1 = u[3 * a] * h1[0] + u[3 * a + 1] * h1[1] + u[3 * a + 2] * h1[2];
        }
        acc[a] = acc[a] + x0;
        acc[3 + a] = acc[3 + a] + x1;
        acc[PR::a0 * 3 + a] = acc[PR::a0 * 3 + a] + mul_unit<r0>(x0);
        acc[PR::a1 * 3 + a] = acc[PR::a1 * 3 + a] + mul_unit<r1>(x1);
    }
}

// Forward and backward hops in direction MU for the site s of parity p.
template <int MU, int P, int LK, bool DAG>
__device__ __forceinline__ void hop_direction(const Geom &g, const char *__restrict__ in,
                                              const char *__restrict__ U, int p, int64_t s,
                                              const Coord &c, cplx<typename real_of<P>::type> acc[12]) {
    using T = typename real_of<P>::type;
    // forward hop uses (1 - g) (S = -1), backward (1 + g); the adjoint swaps them
    constexpr int SF = DAG ? 1 : -1;
    constexpr int SB = -SF;
    int64_t fwd, bwd;
    bool at_last, at_first;
    if constexpr (MU == 0) {
        const int64_t row = s - (c.x >> 1);
        const int xp = c.x + 1 == g.L[0] ? 0 : c.x + 1;
        const int xm = c.x == 0 ? g.L[0] - 1 : c.x - 1;
        fwd = row + (xp >> 1);
        bwd = row + (xm >> 1);
        at_last = c.x == g.L[0] - 1;
        at_first = c.x == 0;
    } else {
        const int xm = MU == 1 ? c.y : MU == 2 ? c.z : c.t;
        const int L = g.L[MU];
        const int64_t st = MU == 1 ? g.sy : MU == 2 ? g.sz : g.st;
        at_last = xm == L - 1;
        at_first = xm == 0;
        fwd = at_last ? s - (int64_t)(L - 1) * st : s + st;
        bwd = at_first ? s + (int64_t)(L - 1) * st : s - st;
    }
    const T sgn_f = (at_last && g.bc[MU] < 0) ? T(-1) : T(1);
    const T sgn_b = (at_first && g.bc[MU] < 0) ? T(-1) : T(1);
    {
        cplx<T> psi[12], u[9];
        load_spinor<P>(in, fwd, psi);
        load_link<P, LK>(U, g.ntiles, p, s, MU, u);
        hop_accumulate<MU, SF, false>(psi, u, sgn_f, acc);
    }
    hop_fence(acc);
    {
        cplx<T> psi[12], u[9];
        load_spinor<P>(in, bwd, psi);
        load_link<P, LK>(U, g.ntiles, p ^ 1, bwd, MU, u);
        hop_accumulate<MU, SB, true>(psi, u, sgn_b, acc);
    }
    hop_fence(acc);
}

// acc = (D_hop in)(x) (or D_hop^dag) for the site s of parity p.
template <int P, int LK, bool DAG>
__device__ __forceinline__ void hop_site(const Geom &g, const char *__restrict__ in,
                                         const char *__restrict__ U, int p, int64_t s,
                                         cplx<typename real_of<P>::type> acc[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {0, 0};
    const Coord c = cb_coords(g, p, s);
    hop_direction<0, P, LK, DAG>(g, in, U, p, s, c, acc);
    hop_direction<1, P, LK, DAG>(g, in, U, p, s, c, acc);
    hop_direction<2, P, LK, DAG>(g, in, U, p, s, c, acc);
    hop_direction<3, P, LK, DAG>(g, in, U, p, s, c, acc);
}

}  // namespace lqcd
