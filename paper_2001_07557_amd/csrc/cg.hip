// Conjugate gradient on the even-odd normal system A = Mhat^dag Mhat with
// reliable updates: the inner iteration runs in the storage precision of the
// sloppy gauge field (FP64, FP32 or binary16 storage with FP32 arithmetic),
// global sums are FP64 and fixed-order, and the true residual b - A x is
// recomputed in FP64 every `reliable_every` iterations, whenever a
// reduced-precision inner residual has fallen by 1/delta since the last
// update (delta below), and whenever the inner residual reaches the
// tolerance.  CG scalars live in device memory, so an iteration is a stream
// of kernels with no host round trip; the host reads the residual every few
// iterations, and every iteration once the decay so far says the tolerance
// is near, so the solve stops at the first iteration that reaches it.
//
// Per iteration: 4 hop kernels (the second also produces |Mhat p|^2 = <p, A p>
// block partials; the fourth does x += a p, r -= a Ap and the |r|^2 partials
// in its epilogue, so Ap is never stored), p = r + b p, and two single-block
// kernels that finish the sums and form alpha, beta.

#include <chrono>
#include <cmath>

#include "lqcd_internal.h"
#include "reduce.h"
#include "hop_common.h"
#include "blas.h"

namespace lqcd {

constexpr int CG_BLOCK = 256;
constexpr int CHECK_EVERY = 10;
// A reduced-precision inner recurrence is trusted only while its residual is
// within a factor delta of the last true residual: past that point the
// computed and true residuals part (rounding of the inner precision), so a
// reliable update is taken.  delta = 0.1 for binary16 storage (unit roundoff
// 2^-11), 1e-3 for FP32 (2^-24: after a 1000-fold drop the rounding carried
// by the recurrence is still ~1e-3 of the residual); FP64 inner iterations
// need it only at the end.
constexpr double DELTA_F16 = 0.1;
constexpr double DELTA_F32 = 1e-3;
// A reduced-precision recurrence residual runs ahead of the true one, so the
// final reliable update is taken when it reaches tol / 2 rather than tol
// (squared: 0.25): an update taken when the recurrence first touches tol
// finds the true residual still just above it and costs a second FP64 update
// a few iterations later.
constexpr double INNER_MARGIN2 = 0.25;

enum { S_RR = 0, S_PAP, S_ALPHA, S_RROLD, S_BETA, S_OUT, S_COUNT = 16 };
enum { OP_ALPHA = 0, OP_RRNEW, OP_RESET, OP_SUM, OP_SETRR };

// Fixed-order sum of the block partials followed by the scalar recurrence.
// One block; thread t adds entries t, t + B, t + 2B, ... in four interleaved
// chains so that four loads are in flight (one chain per thread left the
// 8192 hop partials of a 32^4 solve at 15 us, a third of a hop launch).
constexpr int SCALAR_BLOCK = 512;
template <int OP>
__global__ __launch_bounds__(SCALAR_BLOCK) void cg_scalar_k(const double *partial, int64_t n,
                                                            int stride, double *sc) {
    const int64_t B = blockDim.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t i = threadIdx.x;
    for (; i + 3 * B < n; i += 4 * B) {
        a0 += partial[i * stride];
        a1 += partial[(i + B) * stride];
        a2 += partial[(i + 2 * B) * stride];
        a3 += partial[(i + 3 * B) * stride];
    }
    for (; i < n; i += B) a0 += partial[i * stride];
    double v[1] = {(a0 + a1) + (a2 + a3)};
    block_sum<1>(v);
    if (threadIdx.x == 0) {
        const double s = v[0];
        if constexpr (OP == OP_ALPHA) {
            // <p, A p> = 0 only when p = 0: the iteration has terminated
            // exactly (e.g. a source spanned by few eigenvectors); take no step
            // and let the next residual check confirm convergence.
            sc[S_PAP] = s;
            sc[S_ALPHA] = s > 0.0 ? sc[S_RR] / s : 0.0;
        } else if constexpr (OP == OP_RRNEW || OP == OP_RESET) {
            // RRNEW: rr_old <- rr before the update; RESET keeps rr_old of the
            // iteration and replaces rr by the norm of the recomputed residual
            if constexpr (OP == OP_RRNEW) sc[S_RROLD] = sc[S_RR];
            sc[S_RR] = s;
            sc[S_BETA] = sc[S_RROLD] > 0.0 ? s / sc[S_RROLD] : 0.0;
        } else if constexpr (OP == OP_SETRR) {
            sc[S_RR] = s;
        } else {
            sc[S_OUT] = s;
        }
    }
}

// p = rs + beta p.
template <int P>
__global__ __launch_bounds__(CG_BLOCK) void cg_direction_k(char *p, const char *rs, const double *sc,
                                                           int64_t vh) {
    using T = typename real_of<P>::type;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= vh) return;
    const T beta = (T)sc[S_BETA];
    cplx<T> vr[12], vp[12];
    load_spinor<P>(rs, s, vr);
    load_spinor<P>(p, s, vp);
#pragma unroll
    for (int k = 0; k < 12; ++k) vp[k] = {vr[k].re + beta * vp[k].re, vr[k].im + beta * vp[k].im};
    store_spinor<P>(p, s, vp);
}

// x64 += xs (inner precision), xs = 0.
template <int P>
__global__ __launch_bounds__(CG_BLOCK) void cg_fold_k(char *x64, char *xs, int64_t vh) {
    using T = typename real_of<P>::type;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= vh) return;
    cplx<double> vx[12];
    cplx<T> v[12];
    load_spinor<LQCD_F64>(x64, s, vx);
    load_spinor<P>(xs, s, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        vx[k] = {vx[k].re + (double)v[k].re, vx[k].im + (double)v[k].im};
        v[k] = {0, 0};
    }
    store_spinor<LQCD_F64>(x64, s, vx);
    store_spinor<P>(xs, s, v);
}

// r = b - r (FP64, in place), per-block |r|^2.
__global__ __launch_bounds__(CG_BLOCK) void cg_residual_k(char *r, const char *b, int64_t vh,
                                                          double *partial) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[1] = {0.0};
    if (s < vh) {
        cplx<double> vr[12], vb[12];
        load_spinor<LQCD_F64>(r, s, vr);
        load_spinor<LQCD_F64>(b, s, vb);
        double nr = 0;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            vr[k] = vb[k] - vr[k];
            nr += norm2(vr[k]);
        }
        store_spinor<LQCD_F64>(r, s, vr);
        acc[0] = nr;
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc[0];
}

// ---------------------------------------------------------------------------
// host side of the solver
// ---------------------------------------------------------------------------

struct CGWork {
    char *xs, *rs, *p, *te, *to;      // inner precision
    char *r64, *te64, *to64;          // FP64
    double *partial;
    double *sc;
    size_t bytes;
};

static size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

static int64_t cg_partials(const Geom &g) {
    const int64_t a = hop_partials(g, 1);
    const int64_t b = (g.vh + CG_BLOCK - 1) / CG_BLOCK;
    const int64_t c = reduce_blocks(g, 1) * 2;
    int64_t m = a > b ? a : b;
    return m > c ? m : c;
}

static CGWork cg_layout(const Geom &g, int prec, char *base) {
    CGWork w{};
    const size_t hb = align256(half_spinor_bytes(g, prec));
    const size_t hb64 = align256(half_spinor_bytes(g, LQCD_F64));
    size_t off = 0;
    auto take = [&](size_t n) {
        char *p = base ? base + off : nullptr;
        off += align256(n);
        return p;
    };
    w.xs = take(hb);
    w.rs = take(hb);
    w.p = take(hb);
    w.te = take(hb);
    w.to = take(hb);
    w.r64 = take(hb64);
    w.te64 = take(hb64);
    w.to64 = take(hb64);
    w.partial = (double *)take(sizeof(double) * cg_partials(g));
    w.sc = (double *)take(sizeof(double) * S_COUNT);
    w.bytes = off;
    return w;
}

// Iterations the inner residual rr still needs to reach target when log(rr)
// falls by -rate per iteration (rate < 0; rate = 0: not known yet).
static int iterations_left(double rr, double rate, double target) {
    if (!(rr > target)) return 0;
    if (!(rate < 0.0)) return 1 << 20;
    const double n = std::ceil(std::log(target / rr) / rate);
    return n > (double)(1 << 20) ? 1 << 20 : (int)n;
}

// Iterations until the next host read: CHECK_EVERY while the tolerance is
// far, fewer as it nears, one once it is about an iteration away, so the
// solve stops at the first iteration whose residual reaches it instead of up
// to CHECK_EVERY - 1 later.
static int read_gap(int left) {
    const int n = (int)(0.7 * left);
    return n < 1 ? 1 : n > CHECK_EVERY ? CHECK_EVERY : n;
}

// A drift-triggered reliable update is put off while the tolerance is
// predicted this close (in iterations): the final update follows soon, and
// reading the residual every iteration near the end would otherwise add an
// FP64 update a few iterations before the last one (at 32^4 FP32 inner:
// three updates instead of two).  It is put off only until the inner
// residual has fallen DRIFT_HARD (squared: 1e-4, a further factor 100, about
// the most that reads every ten iterations let it drift) below the drift
// threshold: without that bound an 8^4 FP32-inner solve to 1e-12, whose
// recurrence keeps predicting the end, took 300 iterations instead of
// under 200.  binary16 inner solves, whose drift rule fires at every
// tenfold fall, take every drift update (put off, the 32^4 solve needed 55
// iterations instead of 46).
constexpr int DRIFT_DEFER = CHECK_EVERY;
constexpr double DRIFT_HARD = 1e-4;

struct Solver {
    Geom g;
    hipStream_t st;
    double kappa;
    int prec, link;
    const char *U;
    int link64;
    const char *U64;
    CGWork w;

    int hop(int out_par, char *out, const char *in, const char *y, double alpha, bool dag, int pr,
            int lk, const char *U_, double *partial, char *cg_x = nullptr,
            const char *cg_p = nullptr) {
        HopArgs a{};
        a.cg_x = cg_x;
        a.cg_p = cg_p;
        a.cg_alpha = w.sc + S_ALPHA;
        a.g = g;
        a.U = U_;
        a.alpha = alpha;
        a.beta = 1.0;
        a.par0 = out_par;
        a.out[out_par] = out;
        a.in[out_par] = in;
        a.y[out_par] = y;
        a.partial = partial;
        return hop_launch(a, pr, lk, dag, 1, st);
    }

    // One inner iteration's operator and update: te = Mhat p (with the
    // <p, A p> = |Mhat p|^2 partials, summed into alpha), then
    // Mhat^dag te = A p formed inside the last hop, which updates xs and rs
    // and leaves the |rs|^2 partials.
    int apply_a_update(int pr, int lk, const char *U_) {
        const double k2 = -kappa * kappa;
        int rc = hop(LQCD_ODD, w.to, w.p, nullptr, 1.0, false, pr, lk, U_, nullptr);
        if (!rc) rc = hop(LQCD_EVEN, w.te, w.to, w.p, k2, false, pr, lk, U_, w.partial);
        if (!rc) {
            cg_scalar_k<OP_ALPHA><<<1, SCALAR_BLOCK, 0, st>>>(w.partial, hop_partials(g, 1), 1, w.sc);
            rc = check_launch();
        }
        if (!rc) rc = hop(LQCD_ODD, w.to, w.te, nullptr, 1.0, true, pr, lk, U_, nullptr);
        if (!rc) rc = hop(LQCD_EVEN, w.rs, w.to, w.te, k2, true, pr, lk, U_, w.partial, w.xs, w.p);
        return rc;
    }

    // out = Mhat^dag Mhat x; the block partials of |Mhat x|^2 go to `partial`
    int apply_a(int pr, int lk, const char *U_, const char *x, char *out, char *te, char *to,
                double *partial) {
        const double k2 = -kappa * kappa;
        int rc = hop(LQCD_ODD, to, x, nullptr, 1.0, false, pr, lk, U_, nullptr);
        if (!rc) rc = hop(LQCD_EVEN, te, to, x, k2, false, pr, lk, U_, partial);
        if (!rc) rc = hop(LQCD_ODD, to, te, nullptr, 1.0, true, pr, lk, U_, nullptr);
        if (!rc) rc = hop(LQCD_EVEN, out, to, te, k2, true, pr, lk, U_, nullptr);
        return rc;
    }

    dim3 grid() const { return dim3((unsigned)((g.vh + CG_BLOCK - 1) / CG_BLOCK)); }
    int64_t nblk() const { return (g.vh + CG_BLOCK - 1) / CG_BLOCK; }

    int read(double *host, int slot) {
        hipError_t e = hipMemcpyAsync(host, w.sc + slot, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            set_hip_error(e);
            return LQCD_EHIP;
        }
        return LQCD_OK;
    }

    // |v|^2 of an FP64 or inner-precision half field into scalar slot via OP
    template <int OP>
    int norm_into(const char *v, int pr) {
        launch_reduce(g, 1, v, nullptr, pr, w.partial, st);
        cg_scalar_k<OP><<<1, SCALAR_BLOCK, 0, st>>>(w.partial, reduce_blocks(g, 1), 2, w.sc);
        return check_launch();
    }

    // r64 = b - A64 x64; returns |r64|^2 on the host
    int true_residual(char *x64, const char *b, double *rr) {
        int rc = apply_a(LQCD_F64, link64, U64, x64, w.r64, w.te64, w.to64, nullptr);
        if (rc) return rc;
        cg_residual_k<<<grid(), CG_BLOCK, 0, st>>>(w.r64, b, g.vh, w.partial);
        cg_scalar_k<OP_SUM><<<1, SCALAR_BLOCK, 0, st>>>(w.partial, nblk(), 1, w.sc);
        rc = check_launch();
        if (rc) return rc;
        return read(rr, S_OUT);
    }

    template <int P>
    int run(char *x64, const char *b, double tol, int maxiter, int reliable_every,
            lqcd_cg_stats_t *stats) {
        stats->iterations = 0;
        stats->reliable_updates = 0;
        double bb = 0.0;
        int rc = norm_into<OP_SUM>(b, LQCD_F64);
        if (!rc) rc = read(&bb, S_OUT);
        if (rc) return rc;
        if (!std::isfinite(bb)) return LQCD_ENAN;
        if (bb == 0.0) {
            // the solution of A x = 0 is x = 0
            hipError_t e = hipMemsetAsync(x64, 0, half_spinor_bytes(g, LQCD_F64), st);
            if (e != hipSuccess) {
                set_hip_error(e);
                return LQCD_EHIP;
            }
            stats->true_residual = 0.0;
            stats->iterated_residual = 0.0;
            return LQCD_OK;
        }
        const double target = tol * tol * bb;
        double rr = 0.0;
        // a zero starting guess (the common case) needs no FP64 operator
        // application: r = b
        double xx = 0.0;
        rc = norm_into<OP_SUM>(x64, LQCD_F64);
        if (!rc) rc = read(&xx, S_OUT);
        if (rc) return rc;
        if (xx == 0.0) {
            launch_convert(g, 1, w.r64, LQCD_F64, b, LQCD_F64, st);
            rc = check_launch();
            rr = bb;
        } else {
            rc = true_residual(x64, b, &rr);
        }
        if (rc) return rc;
        if (!std::isfinite(rr)) return LQCD_ENAN;
        stats->true_residual = std::sqrt(rr / bb);
        stats->iterated_residual = stats->true_residual;
        if (rr <= target) return LQCD_OK;

        // inner start: rs = r64, xs = 0, p = rs, rr = |rs|^2
        const size_t hb = half_spinor_bytes(g, P);
        hipError_t e = hipMemsetAsync(w.xs, 0, hb, st);
        if (e != hipSuccess) {
            set_hip_error(e);
            return LQCD_EHIP;
        }
        launch_convert(g, 1, w.rs, P, w.r64, LQCD_F64, st);
        launch_convert(g, 1, w.p, P, w.rs, P, st);
        rc = norm_into<OP_SETRR>(w.rs, P);
        if (rc) return rc;

        int k = 0;
        double rr_it = rr;
        double rr_ref = rr;  // true residual at the last reliable update
        const double delta = P == LQCD_F64 ? 0.0 : P == LQCD_F32 ? DELTA_F32 : DELTA_F16;
        const double drift = delta * delta;
        const double target_inner = P == LQCD_F64 ? target : INNER_MARGIN2 * target;
        const int defer = P == LQCD_F32 ? DRIFT_DEFER : 0;
        // residual at the last host read, the decay of log(rr) per iteration
        // between the last two reads (kept across reliable updates), and the
        // iteration of the next read
        int k_seen = 0;
        double rr_seen = rr;
        double rate = 0.0;
        int next_read = CHECK_EVERY;
        while (true) {
            rc = apply_a_update(P, link, U);
            if (rc) return rc;
            cg_scalar_k<OP_RRNEW><<<1, SCALAR_BLOCK, 0, st>>>(w.partial, hop_partials(g, 1), 1, w.sc);
            rc = check_launch();
            if (rc) return rc;
            ++k;
            bool reliable = reliable_every > 0 && k % reliable_every == 0;
            if (reliable || k >= next_read || k >= maxiter) {
                rc = read(&rr_it, S_RR);
                if (rc) return rc;
                if (!std::isfinite(rr_it)) {
                    stats->iterations = k;
                    return LQCD_ENAN;
                }
                if (k > k_seen && rr_it > 0.0 && rr_it < rr_seen)
                    rate = std::log(rr_it / rr_seen) / (double)(k - k_seen);
                const int left = iterations_left(rr_it, rate, target_inner);
                if (rr_it <= target_inner) reliable = true;
                if (rr_it < drift * rr_ref && (left > defer || rr_it < DRIFT_HARD * drift * rr_ref))
                    reliable = true;
                next_read = k + read_gap(left);
                rr_seen = rr_it;
                k_seen = k;
            }
            if (reliable || k >= maxiter) {
                cg_fold_k<P><<<grid(), CG_BLOCK, 0, st>>>(x64, w.xs, g.vh);
                rc = true_residual(x64, b, &rr);
                if (rc) return rc;
                stats->reliable_updates += 1;
                stats->iterations = k;
                stats->true_residual = std::sqrt(rr / bb);
                stats->iterated_residual = std::sqrt(rr_it / bb);
                if (!std::isfinite(rr)) return LQCD_ENAN;
                if (rr <= target) return LQCD_OK;
                if (k >= maxiter) return LQCD_ENOCONV;
                rr_ref = rr;
                // restart the inner residual from the FP64 one, keep p
                launch_convert(g, 1, w.rs, P, w.r64, LQCD_F64, st);
                rc = norm_into<OP_RESET>(w.rs, P);
                if (rc) return rc;
                rr_seen = rr;
                k_seen = k;
                next_read = k + read_gap(iterations_left(rr, rate, target_inner));
            }
            cg_direction_k<P><<<grid(), CG_BLOCK, 0, st>>>(w.p, w.rs, w.sc, g.vh);
        }
    }
};

}  // namespace lqcd

using namespace lqcd;

extern "C" size_t lqcd_cg_workspace_bytes(const lqcd_geom_t *gg, int inner_prec, int inner_link) {
    Geom g;
    if (!make_geom(gg, &g) || !valid_link(inner_prec, inner_link)) return 0;
    return cg_layout(g, inner_prec, nullptr).bytes;
}

extern "C" int lqcd_cg_solve(const lqcd_geom_t *gg, void *x_e, const void *b_e, const void *U_hi,
                             int link_hi, const void *U_lo, int inner_prec, int inner_link,
                             double kappa, double tol, int maxiter, int reliable_every,
                             void *workspace, size_t workspace_bytes, lqcd_cg_stats_t *stats,
                             void *stream) {
    const auto t0 = std::chrono::steady_clock::now();
    lqcd_cg_stats_t local{};
    lqcd_cg_stats_t *st = stats ? stats : &local;
    *st = lqcd_cg_stats_t{};
    Solver s{};
    auto finish = [&](int rc) {
        st->status = rc;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return rc;
    };
    if (!make_geom(gg, &s.g)) return finish(LQCD_EINVAL);
    if (!valid_link(inner_prec, inner_link) || !valid_link(LQCD_F64, link_hi)) return finish(LQCD_EINVAL);
    if (!x_e || !b_e || !U_hi || !U_lo || !workspace) return finish(LQCD_EINVAL);
    if (((uintptr_t)x_e | (uintptr_t)b_e | (uintptr_t)U_hi | (uintptr_t)U_lo) & 15) return finish(LQCD_EINVAL);
    if ((uintptr_t)workspace & 255) return finish(LQCD_EINVAL);
    if (!(tol > 0.0) || maxiter <= 0 || reliable_every < 0 || !std::isfinite(kappa)) return finish(LQCD_EINVAL);
    if (x_e == b_e) return finish(LQCD_EINVAL);
    s.w = cg_layout(s.g, inner_prec, (char *)workspace);
    if (workspace_bytes < s.w.bytes) return finish(LQCD_ESMALL);
    s.st = (hipStream_t)stream;
    s.kappa = kappa;
    s.prec = inner_prec;
    s.link = inner_link;
    s.U = (const char *)U_lo;
    s.U64 = (const char *)U_hi;
    s.link64 = link_hi;
    int rc;
    if (inner_prec == LQCD_F64) rc = s.run<LQCD_F64>((char *)x_e, (const char *)b_e, tol, maxiter, reliable_every, st);
    else if (inner_prec == LQCD_F32) rc = s.run<LQCD_F32>((char *)x_e, (const char *)b_e, tol, maxiter, reliable_every, st);
    else rc = s.run<LQCD_F16>((char *)x_e, (const char *)b_e, tol, maxiter, reliable_every, st);
    const hipError_t e = hipStreamSynchronize(s.st);
    if (e != hipSuccess && rc == LQCD_OK) {
        set_hip_error(e);
        rc = LQCD_EHIP;
    }
    return finish(rc);
}
