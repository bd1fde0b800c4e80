"""Python binding of liblqcd.so: the Wilson hopping operator on MI355X.

Every function here marshals torch tensors (device memory) and the current
torch stream into the C ABI of ``include/lqcd.h``; all arithmetic runs in
the library's HIP kernels.  Calls raise :class:`LQCDError` on a non-zero
status and :class:`RuntimeError` when handed host tensors.

The operator is the Wilson hopping term that the paper applies in Sec. 3.3
(Fig. 4d) without writing it out; the conventions (hopping form
M = 1 - kappa D_hop, DeGrand-Rossi gamma basis, forward projector 1 - g_mu,
boundary phases on the hops) are stated in ``include/lqcd.h``.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _lib

F64, F32, F16 = 0, 1, 2
LINK18, LINK12 = 18, 12
EVEN, ODD, FULL = 0, 1, 2
OK, EINVAL, EHIP, ENOCONV, ENAN, ESMALL = 0, -1, -2, -3, -4, -5

PREC_NAMES = {F64: "f64", F32: "f32", F16: "f16"}


class LQCDError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = _lib.load()
        msg = lib.lqcd_strerror(status).decode()
        hip = lib.lqcd_last_hip_error().decode()
        super().__init__(f"{where}: status {status} ({msg}){' HIP: ' + hip if hip else ''}")
        self.status = status


def _check(rc: int, where: str):
    if rc != OK:
        raise LQCDError(rc, where)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise RuntimeError("liblqcd operates on device tensors only (got a host tensor)")
    if not t.is_contiguous():
        raise RuntimeError("liblqcd needs contiguous tensors")
    return t.data_ptr()


# ----------------------------------------------------------------------------
# geometry and fields
# ----------------------------------------------------------------------------

class Lattice:
    """Lattice dims (Lx, Ly, Lz, Lt), each even, and per-direction boundary
    signs (+1 periodic, -1 antiperiodic; default antiperiodic in time)."""

    def __init__(self, dims: Sequence[int], bc: Sequence[int] = (1, 1, 1, -1)):
        self.dims = tuple(int(d) for d in dims)
        self.bc = tuple(int(b) for b in bc)
        self.geom = _lib.GeomT((ctypes.c_int32 * 4)(*self.dims), (ctypes.c_int32 * 4)(*self.bc))
        self.volume = 1
        for d in self.dims:
            self.volume *= d

    @property
    def half_volume(self) -> int:
        return self.volume // 2

    def ref(self):
        return ctypes.byref(self.geom)

    def spinor_bytes(self, prec: int, subset: int) -> int:
        n = _lib.load().lqcd_spinor_bytes(self.ref(), prec, subset)
        if n == 0:
            raise LQCDError(EINVAL, "spinor_bytes")
        return n

    def gauge_bytes(self, prec: int, link: int) -> int:
        n = _lib.load().lqcd_gauge_bytes(self.ref(), prec, link)
        if n == 0:
            raise LQCDError(EINVAL, "gauge_bytes")
        return n

    def spinor_shape(self):
        lx, ly, lz, lt = self.dims
        return (lt, lz, ly, lx, 4, 3)

    def links_shape(self):
        lx, ly, lz, lt = self.dims
        return (lt, lz, ly, lx, 4, 3, 3)


def _device_bytes(n: int, device=None) -> torch.Tensor:
    # 256-byte granules; torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(((n + 255) // 256) * 256, dtype=torch.uint8,
                       device=device if device is not None else "cuda")


@dataclass
class SpinorField:
    """Spinor field (or even/odd half) in the library's internal layout."""
    lattice: Lattice
    prec: int
    subset: int
    buf: torch.Tensor

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()

    def half(self, parity: int) -> "SpinorField":
        """View of the even or odd half of a full field (shares memory)."""
        if self.subset != FULL:
            raise RuntimeError("half() needs a full field")
        hb = self.lattice.spinor_bytes(self.prec, EVEN)
        return SpinorField(self.lattice, self.prec, parity, self.buf[parity * hb:(parity + 1) * hb])


@dataclass
class GaugeField:
    """Links (or a link-shaped force) in the library's internal layout."""
    lattice: Lattice
    prec: int
    link: int
    buf: torch.Tensor

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()


def new_spinor(lat: Lattice, prec: int, subset: int, device=None, zero: bool = True) -> SpinorField:
    """A spinor field in the internal layout; zero=False leaves it
    uninitialised (for outputs that a kernel overwrites entirely)."""
    buf = _device_bytes(lat.spinor_bytes(prec, subset), device)
    if zero:
        buf.zero_()
    return SpinorField(lat, prec, subset, buf)


def new_gauge(lat: Lattice, prec: int, link: int, device=None, zero: bool = True) -> GaugeField:
    """A gauge (or force) field in the internal layout; zero=False leaves it
    uninitialised."""
    buf = _device_bytes(lat.gauge_bytes(prec, link), device)
    if zero:
        buf.zero_()
    return GaugeField(lat, prec, link, buf)


def _canon_prec(t: torch.Tensor) -> int:
    if t.dtype == torch.complex128:
        return F64
    if t.dtype == torch.complex64:
        return F32
    raise RuntimeError(f"canonical fields are complex128 or complex64, got {t.dtype}")


def pack_spinor(lat: Lattice, psi: torch.Tensor, prec: int, subset: int = FULL,
                out: Optional[SpinorField] = None) -> SpinorField:
    """Canonical complex[Lt][Lz][Ly][Lx][4][3] -> internal (only `subset` sites read)."""
    if tuple(psi.shape) != lat.spinor_shape():
        raise RuntimeError(f"spinor shape {tuple(psi.shape)} != {lat.spinor_shape()}")
    # every site of the field (a half field holds one parity) is written
    f = out if out is not None else new_spinor(lat, prec, subset, psi.device, zero=False)
    _check(_lib.load().lqcd_pack_spinor(lat.ref(), f.ptr, _ptr(psi), _canon_prec(psi), prec,
                                        subset, _stream()), "pack_spinor")
    return f


def unpack_spinor(f: SpinorField, dtype=torch.complex128, out: Optional[torch.Tensor] = None):
    """Internal -> canonical; sites outside the field's subset are zero (or
    left as they were in `out`)."""
    lat = f.lattice
    if out is None:
        # a half field leaves the other parity's sites untouched: zero them
        alloc = torch.empty if f.subset == FULL else torch.zeros
        out = alloc(lat.spinor_shape(), dtype=dtype, device=f.buf.device)
    _check(_lib.load().lqcd_unpack_spinor(lat.ref(), _ptr(out), f.ptr, _canon_prec(out), f.prec,
                                          f.subset, _stream()), "unpack_spinor")
    return out


def pack_gauge(lat: Lattice, U: torch.Tensor, prec: int, link: int) -> GaugeField:
    """Canonical complex[Lt][Lz][Ly][Lx][4][3][3] -> internal links."""
    if tuple(U.shape) != lat.links_shape():
        raise RuntimeError(f"links shape {tuple(U.shape)} != {lat.links_shape()}")
    f = new_gauge(lat, prec, link, U.device, zero=False)
    _check(_lib.load().lqcd_pack_gauge(lat.ref(), f.ptr, _ptr(U), _canon_prec(U), prec, link,
                                       _stream()), "pack_gauge")
    return f


def unpack_gauge(f: GaugeField, dtype=torch.complex128) -> torch.Tensor:
    """Internal links or force -> canonical (LINK12 rows are completed)."""
    lat = f.lattice
    out = torch.empty(lat.links_shape(), dtype=dtype, device=f.buf.device)
    _check(_lib.load().lqcd_unpack_gauge(lat.ref(), _ptr(out), f.ptr, _canon_prec(out), f.prec,
                                         f.link, _stream()), "unpack_gauge")
    return out


# ----------------------------------------------------------------------------
# operator
# ----------------------------------------------------------------------------

def _same(*fields):
    p = fields[0].prec
    for f in fields[1:]:
        if f is not None and f.prec != p:
            raise RuntimeError("all fields of one call share a storage precision")


def dslash(out: SpinorField, inp: SpinorField, U: GaugeField, alpha: float = 1.0,
           beta: float = 0.0, y: Optional[SpinorField] = None, dagger: bool = False):
    """out = alpha * D_hop inp + beta * y on the full lattice (D_hop^dag if dagger)."""
    _same(out, inp, y, U)
    for f in (out, inp) + ((y,) if y is not None else ()):
        if f.subset != FULL:
            raise RuntimeError("dslash works on full fields")
    fn = _lib.load().lqcd_dslash_dagger if dagger else _lib.load().lqcd_dslash
    _check(fn(out.lattice.ref(), out.ptr, inp.ptr, y.ptr if y is not None else None, U.ptr,
              alpha, beta, U.prec, U.link, _stream()), "dslash")
    return out


def wilson(out: SpinorField, inp: SpinorField, U: GaugeField, kappa: float, dagger: bool = False):
    """out = M inp = inp - kappa D_hop inp (M^dag if dagger)."""
    return dslash(out, inp, U, -kappa, 1.0, inp, dagger)


def meo(out: SpinorField, inp: SpinorField, U: GaugeField, alpha: float = 1.0, beta: float = 0.0,
        y: Optional[SpinorField] = None, dagger: bool = False):
    """out_e = alpha * D_eo inp_o + beta * y_e (block of D_hop^dag if dagger)."""
    _same(out, inp, y, U)
    if out.subset != EVEN or inp.subset != ODD or (y is not None and y.subset != EVEN):
        raise RuntimeError("meo maps an odd half field to an even one")
    _check(_lib.load().lqcd_meo(out.lattice.ref(), out.ptr, inp.ptr, y.ptr if y is not None else None,
                                U.ptr, alpha, beta, int(dagger), U.prec, U.link, _stream()), "meo")
    return out


def moe(out: SpinorField, inp: SpinorField, U: GaugeField, alpha: float = 1.0, beta: float = 0.0,
        y: Optional[SpinorField] = None, dagger: bool = False):
    """out_o = alpha * D_oe inp_e + beta * y_o (block of D_hop^dag if dagger)."""
    _same(out, inp, y, U)
    if out.subset != ODD or inp.subset != EVEN or (y is not None and y.subset != ODD):
        raise RuntimeError("moe maps an even half field to an odd one")
    _check(_lib.load().lqcd_moe(out.lattice.ref(), out.ptr, inp.ptr, y.ptr if y is not None else None,
                                U.ptr, alpha, beta, int(dagger), U.prec, U.link, _stream()), "moe")
    return out


def face_buffer(lat: Lattice, prec: int, device=None) -> torch.Tensor:
    """Device buffer for one t-face (lqcd_face_bytes bytes)."""
    n = _lib.load().lqcd_face_bytes(lat.ref(), prec)
    if n == 0:
        raise LQCDError(EINVAL, "face_bytes (t-slices must be whole 64-site tiles)")
    return _device_bytes(n, device)


def face_pack(face_fwd: torch.Tensor, face_bwd: torch.Tensor, inp: SpinorField, U: GaugeField,
              out_parity: int, dagger: bool = False):
    """Pack the two t-faces the hop of output parity `out_parity` needs from
    across the t boundary (inp: the input half field, parity 1 - out_parity)."""
    _same(inp, U)
    if inp.subset != 1 - out_parity:
        raise RuntimeError("face_pack reads the half field of the other parity")
    _check(_lib.load().lqcd_face_pack(inp.lattice.ref(), _ptr(face_fwd), _ptr(face_bwd), inp.ptr,
                                      U.ptr, out_parity, int(dagger), U.prec, U.link, _stream()),
           "face_pack")


def hop_region(out: SpinorField, inp: SpinorField, U: GaugeField, region: int,
               face_fwd: Optional[torch.Tensor] = None, face_bwd: Optional[torch.Tensor] = None,
               alpha: float = 1.0, beta: float = 0.0, y: Optional[SpinorField] = None,
               dagger: bool = False):
    """The even-odd hop into `out` (parity out.subset) on region 0 (t-slices
    1 .. Lt-2) or region 1 (slices 0 and Lt-1, t boundary read from the faces)."""
    _same(out, inp, y, U)
    if out.subset not in (EVEN, ODD) or inp.subset != 1 - out.subset or (
            y is not None and y.subset != out.subset):
        raise RuntimeError("hop_region maps a half field to the other parity")
    _check(_lib.load().lqcd_hop_region(out.lattice.ref(), out.subset, region, out.ptr, inp.ptr,
                                       y.ptr if y is not None else None, U.ptr, _ptr(face_fwd),
                                       _ptr(face_bwd), alpha, beta, int(dagger), U.prec, U.link,
                                       _stream()), "hop_region")
    return out


def mhat(out: SpinorField, inp: SpinorField, tmp: SpinorField, U: GaugeField, kappa: float,
         dagger: bool = False):
    """out_e = Mhat inp_e (Mhat^dag if dagger); tmp is an odd scratch field."""
    _same(out, inp, tmp, U)
    _check(_lib.load().lqcd_mhat(out.lattice.ref(), out.ptr, inp.ptr, tmp.ptr, U.ptr, kappa,
                                 int(dagger), U.prec, U.link, _stream()), "mhat")
    return out


# ----------------------------------------------------------------------------
# BLAS-1
# ----------------------------------------------------------------------------

def _reduce_ws(lat: Lattice, subset: int, device) -> torch.Tensor:
    return _device_bytes(_lib.load().lqcd_reduce_workspace_bytes(lat.ref(), subset), device)


def dot(a: SpinorField, b: SpinorField) -> complex:
    """<a, b> = sum conj(a) b (deterministic FP64 grid sum); synchronises."""
    _same(a, b)
    ws = _reduce_ws(a.lattice, a.subset, a.buf.device)
    res = (ctypes.c_double * 2)()
    _check(_lib.load().lqcd_dot(a.lattice.ref(), a.subset, a.ptr, b.ptr, a.prec, ws.data_ptr(),
                                res, _stream()), "dot")
    return complex(res[0], res[1])


def norm2(a: SpinorField) -> float:
    ws = _reduce_ws(a.lattice, a.subset, a.buf.device)
    res = (ctypes.c_double * 1)()
    _check(_lib.load().lqcd_norm2(a.lattice.ref(), a.subset, a.ptr, a.prec, ws.data_ptr(), res,
                                  _stream()), "norm2")
    return float(res[0])


def axpby(a: float, x: SpinorField, b: float, y: SpinorField):
    """y = a x + b y."""
    _same(x, y)
    _check(_lib.load().lqcd_axpby(x.lattice.ref(), x.subset, a, x.ptr, b, y.ptr, x.prec,
                                  _stream()), "axpby")
    return y


def convert(dst: SpinorField, src: SpinorField):
    _check(_lib.load().lqcd_convert(dst.lattice.ref(), dst.subset, dst.ptr, dst.prec, src.ptr,
                                    src.prec, _stream()), "convert")
    return dst


# ----------------------------------------------------------------------------
# solver and force
# ----------------------------------------------------------------------------

@dataclass
class CGStats:
    status: int
    iterations: int
    reliable_updates: int
    true_residual: float
    iterated_residual: float
    seconds: float


def cg_workspace(lat: Lattice, inner_prec: int, inner_link: int, device=None) -> torch.Tensor:
    return _device_bytes(_lib.load().lqcd_cg_workspace_bytes(lat.ref(), inner_prec, inner_link),
                         device)


def cg_solve(x: SpinorField, b: SpinorField, U_hi: GaugeField, U_lo: GaugeField, kappa: float,
             tol: float = 1e-10, maxiter: int = 20000, reliable_every: int = 100,
             workspace: Optional[torch.Tensor] = None, raise_on_error: bool = True) -> CGStats:
    """Solve Mhat^dag Mhat x = b on even sites (x: FP64 initial guess / result)."""
    if x.prec != F64 or b.prec != F64 or x.subset != EVEN or b.subset != EVEN:
        raise RuntimeError("cg_solve takes FP64 even half fields")
    if U_hi.prec != F64:
        raise RuntimeError("U_hi must be an FP64 gauge field")
    lat = x.lattice
    ws = workspace if workspace is not None else cg_workspace(lat, U_lo.prec, U_lo.link, x.buf.device)
    st = _lib.CGStatsT()
    rc = _lib.load().lqcd_cg_solve(lat.ref(), x.ptr, b.ptr, U_hi.ptr, U_hi.link, U_lo.ptr,
                                   U_lo.prec, U_lo.link, kappa, tol, maxiter, reliable_every,
                                   ws.data_ptr(), ws.numel(), ctypes.byref(st), _stream())
    stats = CGStats(rc, st.iterations, st.reliable_updates, st.true_residual,
                    st.iterated_residual, st.seconds)
    if rc != OK and raise_on_error:
        raise LQCDError(rc, "cg_solve")
    return stats


def fermion_force(X: SpinorField, Y: SpinorField, U: GaugeField, coeff: float, mode: int = 0,
                  out: Optional[GaugeField] = None, accumulate: bool = False) -> GaugeField:
    """Link derivative of coeff * Re(Y^dag D_hop X): mode 0 su(3) force
    F = TA(G U^dag), mode 1 raw gradient G, mode 2 (12-real U only) G carried
    onto the stored rows 0 and 1 (all LINK18 fields)."""
    _same(X, Y, U)
    lat = X.lattice
    if out is None:
        out = new_gauge(lat, U.prec, LINK18, X.buf.device, zero=accumulate)
    _check(_lib.load().lqcd_fermion_force(lat.ref(), out.ptr, X.ptr, Y.ptr, U.ptr, coeff, mode,
                                          int(accumulate), U.prec, U.link, _stream()),
           "fermion_force")
    return out


def solve_and_force(phi_e: SpinorField, U_hi: GaugeField, U_lo: GaugeField, kappa: float,
                    tol: float = 1e-10, maxiter: int = 20000, reliable_every: int = 100,
                    U_force: Optional[GaugeField] = None, events: Optional[list] = None,
                    out: Optional[GaugeField] = None):
    """Pseudofermion solve plus force for S = phi_e^dag (Mhat^dag Mhat)^-1 phi_e.

    1. X_e = (Mhat^dag Mhat)^-1 phi_e by mixed-precision CG (FP64 result);
    2. X_o = D_oe X_e, Y_e = Mhat X_e, Y_o = (D_eo)^dag Y_e recomputed by hop
       kernels in the force precision (nothing from the solve is kept but X_e);
    3. F = TA(G U^dag) with G the link derivative of 2 kappa^2 Re(Y^dag dD_hop X).
    U_force (default U_lo; an FP32 field when U_lo is binary16) sets the
    precision of steps 2-3.  Returns (F, cg stats, X_e, X, Y); `out` (a
    LINK18 field of the force precision) receives F if given.  With
    `events` a list, (stage name, torch.cuda.Event) pairs are appended at the
    start and after each stage, on the current stream.
    """

    def mark(name):
        if events is not None:
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            events.append((name, e))

    mark("start")
    lat = phi_e.lattice
    Uf = U_force if U_force is not None else U_lo
    if Uf.prec == F16:
        raise RuntimeError("the force runs in FP64 or FP32: pass an FP32 U_force")
    x = new_spinor(lat, F64, EVEN, phi_e.buf.device)
    stats = cg_solve(x, phi_e, U_hi, U_lo, kappa, tol=tol, maxiter=maxiter,
                     reliable_every=reliable_every)
    mark("solve")
    fp = Uf.prec
    X = new_spinor(lat, fp, FULL, x.buf.device, zero=False)
    Y = new_spinor(lat, fp, FULL, x.buf.device, zero=False)
    Xe, Xo, Ye, Yo = X.half(EVEN), X.half(ODD), Y.half(EVEN), Y.half(ODD)
    convert(Xe, x)  # a copy (FP64) or a rounding to the force precision
    moe(Xo, Xe, Uf)
    tmp = new_spinor(lat, fp, ODD, x.buf.device, zero=False)
    mhat(Ye, Xe, tmp, Uf, kappa)
    moe(Yo, Ye, Uf, dagger=True)
    del tmp
    mark("recompute")
    F = fermion_force(X, Y, Uf, 2.0 * kappa * kappa, mode=0, out=out)
    mark("force")
    return F, stats, x, X, Y


# ----------------------------------------------------------------------------
# shifts and SU(3) products
# ----------------------------------------------------------------------------

def cshift(out: SpinorField, inp: SpinorField, mu: int, direction: int) -> SpinorField:
    """out(x) = bc^[wrap] inp(x + direction mu_hat) on full fields."""
    _same(out, inp)
    if out.subset != FULL or inp.subset != FULL:
        raise RuntimeError("cshift works on full fields")
    _check(_lib.load().lqcd_cshift(out.lattice.ref(), out.ptr, inp.ptr, mu, direction, out.prec,
                                   _stream()), "cshift")
    return out


def colour_mul(out: SpinorField, inp: SpinorField, U: GaugeField, mu: int,
               adjoint: bool = False) -> SpinorField:
    """out(x) = U_mu(x) inp(x) (U_mu(x)^dag with adjoint) on full fields."""
    _same(out, inp, U)
    if out.subset != FULL or inp.subset != FULL:
        raise RuntimeError("colour_mul works on full fields")
    _check(_lib.load().lqcd_colour_mul(out.lattice.ref(), out.ptr, inp.ptr, U.ptr, mu,
                                       int(adjoint), U.prec, U.link, _stream()), "colour_mul")
    return out


def spin_project(acc: SpinorField, inp: SpinorField, mu: int, sign: int,
                 accumulate: bool = True) -> SpinorField:
    """acc(x) (+)= (1 + sign g_mu) inp(x) on full fields."""
    _same(acc, inp)
    if acc.subset != FULL or inp.subset != FULL:
        raise RuntimeError("spin_project works on full fields")
    _check(_lib.load().lqcd_spin_project(acc.lattice.ref(), acc.ptr, inp.ptr, mu, sign,
                                         int(accumulate), acc.prec, _stream()), "spin_project")
    return acc


def dslash_generic(out: SpinorField, inp: SpinorField, U: GaugeField, tmp1: SpinorField,
                   tmp2: SpinorField, dagger: bool = False) -> SpinorField:
    """out = D_hop inp (D_hop^dag with dagger) composed of the generic kernels
    (shift, colour product, projector); tmp1, tmp2 are full scratch fields."""
    _same(out, inp, U, tmp1, tmp2)
    for f in (out, inp, tmp1, tmp2):
        if f.subset != FULL:
            raise RuntimeError("dslash_generic works on full fields")
    _check(_lib.load().lqcd_dslash_generic(out.lattice.ref(), out.ptr, inp.ptr, U.ptr, tmp1.ptr,
                                           tmp2.ptr, int(dagger), U.prec, U.link, _stream()),
           "dslash_generic")
    return out


def split_rotate(out: torch.Tensor, inp: torch.Tensor, s: int, r: int) -> torch.Tensor:
    """Split each row (last axis, length VL) into s blocks and rotate each
    block left by r elements (float64, complex64 or complex128 tensors)."""
    if inp.dtype != out.dtype or inp.shape != out.shape:
        raise RuntimeError("split_rotate needs matching tensors")
    eb = {torch.float64: 8, torch.complex64: 8, torch.complex128: 16}.get(inp.dtype)
    if eb is None:
        raise RuntimeError("split_rotate takes float64, complex64 or complex128")
    vl = inp.shape[-1]
    nvec = inp.numel() // vl if vl else 0
    _check(_lib.load().lqcd_split_rotate(_ptr(out), _ptr(inp), nvec, vl, s, r, eb, _stream()),
           "split_rotate")
    return out


def su3_mul(W: GaugeField, U: GaugeField, V: GaugeField, adj_u: bool = False,
            adj_v: bool = False) -> GaugeField:
    """W = op(U) op(V) on every link."""
    if not (W.prec == U.prec == V.prec and W.link == U.link == V.link):
        raise RuntimeError("su3_mul fields share precision and link format")
    _check(_lib.load().lqcd_su3_mul(W.lattice.ref(), W.ptr, U.ptr, V.ptr, int(adj_u), int(adj_v),
                                    W.prec, W.link, _stream()), "su3_mul")
    return W
