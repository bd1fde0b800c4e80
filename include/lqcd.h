/*
 * lqcd.h - C ABI of the MI355X Wilson-Dirac library (liblqcd.so).
 *
 * The operator is the Wilson hopping term whose generic (not hand-unrolled)
 * kernel the paper times on KNL in Sec. 3.3 (Fig. 4d); the paper does not
 * write it out, so the definitions below are the textbook ones, stated in
 * full:
 *
 *   (D_hop psi)(x) = sum_{mu=0..3} [ s+_mu(x) (1 - g_mu) U_mu(x) psi(x+mu)
 *                                  + s-_mu(x) (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *
 * with mu = 0,1,2,3 = x,y,z,t, gamma matrices in the DeGrand-Rossi chiral
 * basis (gamma5 = diag(1,1,-1,-1)), s+_mu(x) = bc[mu] on the last slice
 * x_mu = L_mu - 1 and s-_mu(x) = bc[mu] on the first slice x_mu = 0 (else 1).
 * D_hop^dag is the same sum with (1 - g_mu) and (1 + g_mu) exchanged; the
 * Wilson matrix is M = 1 - kappa D_hop.  Sites have parity (x+y+z+t) mod 2;
 * D_eo (odd -> even) and D_oe (even -> odd) are the off-diagonal blocks of
 * D_hop, and Mhat = 1 - kappa^2 D_eo D_oe is the Schur operator on even sites.
 * Boundary conditions are applied inside the kernels (one GPU, no halo).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every pointer named as a field (spinor, gauge, force, workspace) is
 *    DEVICE memory owned by the caller.  The library never allocates, frees
 *    or retains device memory and keeps no global state besides the HIP
 *    module, whose one static device array (the scratch of
 *    lqcd_dot_noalloc) comes with it.  Host pointers are named so
 *    explicitly (stats, result).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call is enqueued on it and returns without waiting, except where
 *    a function states that it synchronises the stream.
 *  - Return value: LQCD_OK (0) or a negative status; lqcd_strerror() gives a
 *    text.  No C++ exception crosses this interface.  Arguments are checked
 *    before any work is enqueued, and an invalid call enqueues nothing.
 *  - Canonical (user) layouts, lexicographic sites with x fastest, complex
 *    numbers as (re, im) pairs of doubles (canon_prec = LQCD_F64) or floats
 *    (canon_prec = LQCD_F32):
 *        spinor  complex[Lt][Lz][Ly][Lx][4 spin][3 colour]
 *        links   complex[Lt][Lz][Ly][Lx][4 mu][3 row][3 col]
 *    An even or odd half field in canonical form is a full-size array of
 *    which only the sites of that parity are read or written.
 *  - Internal layouts (opaque; sizes from the *_bytes queries) hold a half
 *    field as tiles of 64 consecutive checkerboard sites, each tile a run of
 *    64-lane "words" of 16 bytes so that a wavefront reads one word of 64
 *    sites in one coalesced 1 KiB access.  A full field is the even half
 *    followed by the odd half.  Field pointers must be 16-byte aligned and
 *    the solver workspace 256-byte aligned (LQCD_EINVAL otherwise).
 *  - Geometry: dims = {Lx, Ly, Lz, Lt}, each even and >= 2; bc[mu] = +1
 *    (periodic) or -1 (antiperiodic).
 */
#ifndef LQCD_H
#define LQCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LQCD_OK        0
#define LQCD_EINVAL   -1   /* bad geometry, NULL or misaligned pointer, unsupported combination */
#define LQCD_EHIP     -2   /* HIP launch or runtime error */
#define LQCD_ENOCONV  -3   /* solver hit maxiter; x holds the last iterate */
#define LQCD_ENAN     -4   /* non-finite residual detected */
#define LQCD_ESMALL   -5   /* workspace smaller than the size query returned, or a
                              field too large for the static scratch of lqcd_dot_noalloc */

/* storage precisions: arithmetic is FP64 for LQCD_F64 and FP32 otherwise;
   the hopping term on binary16 storage forms each projected half-spinor from
   the stored values of the neighbour site in binary16 (one rounding of the
   exact sum), multiplies by the link in FP32 (binary16 products exact) and
   applies the neighbour's scale last (a reading: the paper does not treat
   reduced precision) */
#define LQCD_F64   0
#define LQCD_F32   1
#define LQCD_F16   2       /* binary16 storage; spinors carry one FP32 scale
                              per site (max |real| of the site); hopping-term
                              launches take V/2 <= 44.7M sites (each parity's
                              links below 4 GB), else LQCD_EINVAL */

/* link storage: full 3x3 (18 reals) or rows 0 and 1 only (12 reals), with
   row 2 = conj(row0 x row1) rebuilt in registers (valid for SU(3) only) */
#define LQCD_LINK18 18
#define LQCD_LINK12 12

/* field subsets */
#define LQCD_EVEN 0
#define LQCD_ODD  1
#define LQCD_FULL 2

typedef struct {
    int32_t dims[4];   /* Lx, Ly, Lz, Lt */
    int32_t bc[4];     /* +1 periodic, -1 antiperiodic */
} lqcd_geom_t;

typedef struct {
    int32_t iterations;        /* inner iterations performed */
    int32_t reliable_updates;  /* FP64 true-residual recomputations */
    int32_t status;            /* same value the call returns */
    int32_t reserved;
    double  true_residual;     /* ||b - A x|| / ||b|| in FP64 at exit */
    double  iterated_residual; /* last inner-precision ||r|| / ||b|| */
    double  seconds;           /* wall time from entry to return */
} lqcd_cg_stats_t;

/* ---------------------------------------------------------------------- */
/* library information                                                     */
/* ---------------------------------------------------------------------- */

/* Version as 10000*major + 100*minor + patch. */
int lqcd_version(void);

/* Static text for a status code (never NULL). */
const char *lqcd_strerror(int status);

/* Last HIP error text recorded by a failing call on this thread, or "". */
const char *lqcd_last_hip_error(void);

/* ---------------------------------------------------------------------- */
/* sizes of internal fields (0 on invalid arguments)                       */
/* ---------------------------------------------------------------------- */

/* Bytes of a spinor field in internal layout; subset EVEN/ODD = half field. */
size_t lqcd_spinor_bytes(const lqcd_geom_t *g, int prec, int subset);

/* Bytes of a gauge field (4 links per site) in internal layout.
   Supported: (F64|F32, LINK18|LINK12) and (F16, LINK12). */
size_t lqcd_gauge_bytes(const lqcd_geom_t *g, int prec, int link);

/* ---------------------------------------------------------------------- */
/* layout conversion (untimed set-up work)                                 */
/* ---------------------------------------------------------------------- */

/* Layout conversion has no passage in the paper (the layouts are this
   library's).  Canonical spinor -> internal.  src is a full canonical array; for subset
   EVEN/ODD only that parity is read and dst is a half field.  Values are
   rounded to `prec` (F16: per-site scale, see LQCD_F16). */
int lqcd_pack_spinor(const lqcd_geom_t *g, void *dst, const void *src_canon,
                     int canon_prec, int prec, int subset, void *stream);

/* Internal -> canonical.  For subset EVEN/ODD only sites of that parity are
   written to dst_canon; the others are left untouched. */
int lqcd_unpack_spinor(const lqcd_geom_t *g, void *dst_canon, const void *src,
                       int canon_prec, int prec, int subset, void *stream);

/* Canonical links -> internal (LINK12 keeps rows 0 and 1). */
int lqcd_pack_gauge(const lqcd_geom_t *g, void *dst, const void *src_canon,
                    int canon_prec, int prec, int link, void *stream);

/* Internal links (or a force / link gradient, which is LINK18) -> canonical;
   LINK12 input is expanded with the third-row reconstruction. */
int lqcd_unpack_gauge(const lqcd_geom_t *g, void *dst_canon, const void *src,
                      int canon_prec, int prec, int link, void *stream);

/* ---------------------------------------------------------------------- */
/* the operator                                                            */
/* ---------------------------------------------------------------------- */

/* The operator of Sec. 3.3 (Fig. 4d), as defined at the top of this header.
   Full lattice:  out = alpha * D_hop in + beta * y   (y may be NULL: beta
   ignored).  M = 1 - kappa D_hop is alpha = -kappa, beta = 1, y = in.
   out, in, y: full spinor fields of precision prec; U: gauge field of
   (prec, link).  out must not alias in; it may alias y. */
int lqcd_dslash(const lqcd_geom_t *g, void *out, const void *in, const void *y,
                const void *U, double alpha, double beta, int prec, int link,
                void *stream);

/* Same with D_hop^dag (projectors 1 + g_mu forward, 1 - g_mu backward). */
int lqcd_dslash_dagger(const lqcd_geom_t *g, void *out, const void *in, const void *y,
                       const void *U, double alpha, double beta, int prec, int link,
                       void *stream);

/* Even-odd blocks: out_e = alpha * D_eo in_o + beta * y_e (lqcd_meo) and
   out_o = alpha * D_oe in_e + beta * y_o (lqcd_moe); dagger != 0 applies the
   corresponding block of D_hop^dag, i.e. (D_oe)^dag for meo and (D_eo)^dag
   for moe.  Half fields; out must not alias in. */
int lqcd_meo(const lqcd_geom_t *g, void *out_e, const void *in_o, const void *y_e,
             const void *U, double alpha, double beta, int dagger, int prec, int link,
             void *stream);
int lqcd_moe(const lqcd_geom_t *g, void *out_o, const void *in_e, const void *y_o,
             const void *U, double alpha, double beta, int dagger, int prec, int link,
             void *stream);

/* Decomposition in t, the one-GPU part of the paper's multi-node shift
 * (Sec. 3.1: arrays are split at the domain boundary and the pieces sent to
 * the neighbouring node).  For the even-odd hop of output parity out_par the
 * sites of the t-slices 0 and Lt-1 need input across the t boundary; a
 * sender packs it as two faces, each one value per site of a t-slice:
 *   face_fwd[j] = bc[3] rows 0, 1 of (1 + S g_t) in(j on slice 0),
 *   face_bwd[j] = bc[3] U_t(y)^dag rows 0, 1 of (1 - S g_t) in(y = j on slice Lt-1),
 * S = -1 (S = +1 with dagger != 0), j the checkerboard index within the
 * slice, `in` the input half field (parity 1 - out_par), U the gauge field.
 * The receiver multiplies face_fwd by its own U_t.  Faces are stored in the
 * arithmetic precision as tiles of 64 sites of six complex numbers (FP64
 * 96 bytes per site, FP32 48); for binary16 storage face_fwd holds the
 * binary16 half-spinor in units of the site scale, with that scale times
 * bc[3] kept apart (52 bytes per site), and face_bwd the six FP32 complex
 * numbers of U_t(y)^dag times that half-spinor with the same kind of factor
 * kept apart, in the same 52-byte tiles, so the receiver's arithmetic is the
 * unsplit hop's; lqcd_face_bytes gives the size of one face.  On one
 * GPU the faces of this lattice's own t wrap stand in for the neighbours'.
 * lqcd_hop_region computes the hop (as lqcd_meo / lqcd_moe: out = alpha
 * D in + beta y) on region 0, the interior slices 1 .. Lt-2 (no face
 * needed; faces may be NULL), or region 1, the slices 0 and Lt-1, whose
 * hops across the t boundary read face_fwd / face_bwd instead of `in`.
 * Both regions together give the unsplit launch's result bit for bit.  Every
 * t-slice must be a whole number of 64-site tiles ((Lx/2) Ly Lz divisible by
 * 64), else LQCD_EINVAL (and lqcd_face_bytes returns 0). */
size_t lqcd_face_bytes(const lqcd_geom_t *g, int prec);
int lqcd_face_pack(const lqcd_geom_t *g, void *face_fwd, void *face_bwd, const void *in,
                   const void *U, int out_par, int dagger, int prec, int link, void *stream);
int lqcd_hop_region(const lqcd_geom_t *g, int out_par, int region, void *out, const void *in,
                    const void *y, const void *U, const void *face_fwd, const void *face_bwd,
                    double alpha, double beta, int dagger, int prec, int link, void *stream);

/* Schur operator on even sites: out_e = Mhat in_e (dagger = 0) or
   Mhat^dag in_e (dagger != 0), Mhat^dag = 1 - kappa^2 (D_oe)^dag (D_eo)^dag.
   tmp_o: caller's odd half field of the same precision (scratch). */
int lqcd_mhat(const lqcd_geom_t *g, void *out_e, const void *in_e, void *tmp_o,
              const void *U, double kappa, int dagger, int prec, int link, void *stream);

/* ---------------------------------------------------------------------- */
/* BLAS-1 with deterministic wavefront reductions                          */
/* ---------------------------------------------------------------------- */

/* Inner products and vector updates of the solver (the paper has no solver;
   these are the plain definitions).
   Bytes of device workspace a reduction over `subset` needs. */
size_t lqcd_reduce_workspace_bytes(const lqcd_geom_t *g, int subset);

/* result[0] + i result[1] = <a, b> = sum conj(a) b over every site of the
   subset (host array of 2 doubles).  Per-thread partials in the field's
   arithmetic precision, wave64 and block sums in FP64, final sum over blocks
   in a fixed order: bitwise reproducible.  Synchronises the stream. */
int lqcd_dot(const lqcd_geom_t *g, int subset, const void *a, const void *b, int prec,
             void *workspace, double *result, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lqcd_dot
 * without the workspace argument.  The block partials live in a static
 * device array of the library (1 MiB per GPU, held until the process ends),
 * so the call allocates nothing; arguments, result and synchronisation as for
 * lqcd_dot.  Fields of more than LQCD_DOT_NOALLOC_MAX_SITES sites in the
 * subset (V/2 for EVEN/ODD, V for FULL) return LQCD_ESMALL before any work
 * is enqueued.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (two host threads, or two streams without ordering)
 * race and may return wrong sums.  A call leaves nothing behind that a later
 * call depends on. */
#define LQCD_DOT_NOALLOC_MAX_SITES 16776960
int lqcd_dot_noalloc(const lqcd_geom_t *g, int subset, const void *a, const void *b, int prec,
                     double *result, void *stream);

/* *result = ||a||^2 (host double); same reduction and synchronisation. */
int lqcd_norm2(const lqcd_geom_t *g, int subset, const void *a, int prec,
               void *workspace, double *result, void *stream);

/* y = a * x + b * y for real a, b (fields of one precision and subset). */
int lqcd_axpby(const lqcd_geom_t *g, int subset, double a, const void *x, double b,
               void *y, int prec, void *stream);

/* dst = src with a change of storage precision (same subset).  With equal
 * precisions it is a byte copy of the internal layout (bit-exact, also for
 * binary16 storage). */
int lqcd_convert(const lqcd_geom_t *g, int subset, void *dst, int dst_prec,
                 const void *src, int src_prec, void *stream);

/* ---------------------------------------------------------------------- */
/* solver                                                                  */
/* ---------------------------------------------------------------------- */

/* Bytes of workspace lqcd_cg_solve needs for the given inner precision. */
size_t lqcd_cg_workspace_bytes(const lqcd_geom_t *g, int inner_prec, int inner_link);

/* The paper has no solver: Hestenes-Stiefel CG on the normal system of the
 * Sec. 3.3 operator, with FP64 reliable updates around a reduced-precision
 * inner iteration.
 * Solve A x = b on even sites, A = Mhat^dag Mhat, by CG with reliable updates.
 *   x_e:   FP64 even half field; in: initial guess, out: solution.
 *   b_e:   FP64 even half field (right-hand side).
 *   U_hi:  FP64 gauge field (link_hi reals), used for the reliable updates
 *          (true residual b - A x recomputed in FP64).
 *   U_lo:  gauge field of (inner_prec, inner_link) for the inner iterations;
 *          may equal U_hi when inner_prec = LQCD_F64 and links match.
 *   The inner loop runs CG in inner_prec with FP64 block and grid sums.
 *   A reliable update folds the inner solution into x_e, recomputes the true
 *   residual in FP64 and restarts the inner residual from it, keeping the
 *   search direction; it is taken every `reliable_every` iterations (0 =
 *   never on a schedule), whenever the inner residual has fallen since the
 *   last update by 1000x (FP32 inner) or 10x (F16 inner), beyond which the
 *   inner recurrence is not trusted (for FP32 inner iterations put off, by
 *   at most a further 100x fall, while the decay so far puts the tolerance
 *   within ten iterations, when the final update comes first),
 *   and when the inner residual reaches tol (tol/2 for FP32 and F16 inner
 *   iterations, whose recurrence residual runs ahead of the true one).  The
 *   solve stops when ||b - A x|| / ||b|| <= tol in FP64.  The host reads the
 *   inner residual every 10 iterations while the tolerance is far and every
 *   iteration once the decay so far puts it within reach, so `iterations` is
 *   the first iteration whose inner residual reached that threshold (when the
 *   FP64 check then confirms it).
 *   workspace: device memory of lqcd_cg_workspace_bytes() bytes.
 *   stats: host struct filled on return (may be NULL).
 * Synchronises the stream.  Returns LQCD_ENOCONV after maxiter inner
 * iterations (x_e then holds the best iterate) and LQCD_ENAN on a non-finite
 * residual.  A call with x_e = previous result resumes the solve. */
int lqcd_cg_solve(const lqcd_geom_t *g, void *x_e, const void *b_e,
                  const void *U_hi, int link_hi, const void *U_lo, int inner_prec,
                  int inner_link, double kappa, double tol, int maxiter,
                  int reliable_every, void *workspace, size_t workspace_bytes,
                  lqcd_cg_stats_t *stats, void *stream);

/* ---------------------------------------------------------------------- */
/* differentiation                                                         */
/* ---------------------------------------------------------------------- */

/* The paper has no derivatives: the textbook link derivative of the Sec. 3.3
 * operator.  Link derivative of coeff * Re(Y^dag D_hop X) for every link (owner
 * computes, no atomics).  With
 *   W_mu(x) = coeff * s+_mu(x) [ X(x+mu) (x) ((1-g_mu) Y(x))^dag
 *                              + ((1+g_mu) Y(x+mu)) (x) X(x)^dag ],
 * (a (x) b^dag)_ij = sum_spin a_{s,i} conj(b_{s,j}), the result written is
 *   mode 1: G = W^dag, the raw complex gradient dS/dRe U + i dS/dIm U of
 *           the 3x3 links the operator applies;
 *   mode 2: (link = LINK12 only) the raw gradient with respect to the
 *           stored rows 0 and 1 of 12-real links, whose row 2 the operator
 *           rebuilds as conj(row0 x row1): row0 = G_0 + conj(row1 x G_2),
 *           row1 = G_1 + conj(G_2 x row0), row 2 = 0;
 *   mode 0: F = TA(G U^dag), the su(3) force for U -> exp(eps T) U, where
 *           TA(A) = (A - A^dag)/2 - tr(A - A^dag)/6.
 * X, Y: full spinor fields (prec); U: gauge field (prec, link);
 * F_out: LINK18 field of precision prec (F64 or F32); accumulate != 0 adds
 * to F_out instead of overwriting it. */
int lqcd_fermion_force(const lqcd_geom_t *g, void *F_out, const void *X, const void *Y,
                       const void *U, double coeff, int mode, int accumulate,
                       int prec, int link, void *stream);

/* ---------------------------------------------------------------------- */
/* shifts and lattice SU(3) products (the paper's building blocks)          */
/* ---------------------------------------------------------------------- */

/* Shift of a full spinor field: out(x) = s in(x + dir mu_hat), dir = +1 or
   -1, with s = bc[mu] when the step wraps around the lattice (from the last
   slice for dir = +1, the first for dir = -1) and 1 otherwise.  The shift
   that the stencils of Sec. 3.1 are built from; with one site per lane it
   needs no lane rearrangement.  out must not alias in.  All
   precisions; binary16 fields are copied exactly (the sign rides on the
   site scale). */
int lqcd_cshift(const lqcd_geom_t *g, void *out, const void *in, int mu, int dir, int prec,
                void *stream);

/* The two per-site operations the generic operator below is composed of
 * (the paper's generic Wilson kernel, Sec. 3.3 and Fig. 4d, is built from
 * stencil shifts, Sec. 3.1; these are its other two steps).  Full spinor
 * fields, prec F64 or F32, out / acc must not alias in.
 *   lqcd_colour_mul:   out(x) = U_mu(x) in(x), or U_mu(x)^dag in(x) when
 *                      adjoint != 0, for each of the four spins.
 *   lqcd_spin_project: acc(x) = (1 + sign g_mu) in(x), sign = +1 or -1,
 *                      added to acc when accumulate != 0 (else overwritten). */
int lqcd_colour_mul(const lqcd_geom_t *g, void *out, const void *in, const void *U, int mu,
                    int adjoint, int prec, int link, void *stream);
int lqcd_spin_project(const lqcd_geom_t *g, void *acc, const void *in, int mu, int sign,
                      int accumulate, int prec, void *stream);

/* out = D_hop in (dagger = 0) or D_hop^dag in, composed only of the library's
 * generic kernels: for each mu, cshift(in, mu, +1) -> colour_mul(U_mu) ->
 * spin_project(1 - g_mu) and colour_mul(U_mu^dag) -> cshift(-1) ->
 * spin_project(1 + g_mu) (projectors exchanged for the adjoint), 24 launches
 * each streaming full fields: the generic counterpart of the fused
 * lqcd_dslash, as in the paper's comparison of its generic and hand-unrolled
 * Wilson kernels (Sec. 3.3, Fig. 4d).  tmp1, tmp2: caller's full spinor
 * fields of the same precision (scratch); no two of out, in, tmp1, tmp2 may
 * be the same buffer.  prec F64 or F32. */
int lqcd_dslash_generic(const lqcd_geom_t *g, void *out, const void *in, const void *U,
                        void *tmp1, void *tmp2, int dagger, int prec, int link, void *stream);

/* The lane permutation of Sec. 3.1 on nvec consecutive vectors of vl
   elements of elem_bytes (8: one double or FP32 complex, 16: one FP64
   complex): every vector is split into s blocks of w = vl/s elements and each
   block is rotated left by r,  out[v][i] = in[v][(i + r) mod w + (i div w) w].
   s = 1 is a plain rotation.  (For complex data stored as reals the paper
   rotates by 2r reals; with elem_bytes = 16 r counts complexes.)  Vectors
   with vl dividing 64 are permuted in registers inside a wavefront.
   out must not alias in; EINVAL if s does not divide vl. */
int lqcd_split_rotate(void *out, const void *in, int64_t nvec, int vl, int s, int r,
                      int elem_bytes, void *stream);

/* Lattice SU(3) product W_mu(x) = op(U_mu(x)) op(V_mu(x)) for all 4V links,
   op = hermitian conjugate when adj_u / adj_v != 0: the SU(3) matrix-matrix
   workload of Sec. 3.3 (Fig. 4a-c).  All three fields share (prec, link),
   prec F64 or F32; LINK12 inputs are rebuilt to 3x3 and the product is
   stored by its rows 0 and 1 (SU(3) is closed under products).  W may alias
   U or V. */
int lqcd_su3_mul(const lqcd_geom_t *g, void *W, const void *U, const void *V, int adj_u,
                 int adj_v, int prec, int link, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LQCD_H */
