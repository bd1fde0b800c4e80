"""torch.autograd wrapper of the Wilson matrix with hand-written adjoints.

phi = M psi = psi - kappa D_hop[U] psi on canonical device tensors.  The
backward pass runs two library kernels:

* dL/dpsi = M^dag g (the adjoint hopping kernel),
* dL/dU from the fermion-force kernel with X = psi, Y = g, c0 = -kappa: the raw
  complex gradient G = dL/dRe U + i dL/dIm U of the function computed
  (``link_grad="raw"``, what torch optimisers and gradcheck expect; with
  12-real links the operator reads only rows 0 and 1 of U and rebuilds row 2,
  so the kernel carries G through that rebuild and row 2 gets zero) or the
  su(3)-projected force F = TA(G U^dag) for U -> exp(eps T) U
  (``link_grad="su3"``).

Only psi and U are saved for backward; phi is not kept.
"""

from __future__ import annotations

import torch

from . import lqcd as L


class WilsonMatrix(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi, U, kappa, lattice, prec, link, link_grad):
        if link_grad not in ("raw", "su3"):
            raise ValueError("link_grad is 'raw' or 'su3'")
        Uf = L.pack_gauge(lattice, U.contiguous(), prec, link)
        pf = L.pack_spinor(lattice, psi.contiguous(), prec, L.FULL)
        of = L.new_spinor(lattice, prec, L.FULL, psi.device, zero=False)
        L.wilson(of, pf, Uf, kappa)
        ctx.save_for_backward(psi, U)
        ctx.cfg = (kappa, lattice, prec, link, link_grad)
        return L.unpack_spinor(of, dtype=psi.dtype)

    @staticmethod
    def backward(ctx, g):
        psi, U = ctx.saved_tensors
        kappa, lattice, prec, link, link_grad = ctx.cfg
        Uf = L.pack_gauge(lattice, U.contiguous(), prec, link)
        gf = L.pack_spinor(lattice, g.contiguous().to(psi.dtype), prec, L.FULL)
        gpsi = gU = None
        if ctx.needs_input_grad[0]:
            of = L.new_spinor(lattice, prec, L.FULL, psi.device, zero=False)
            L.wilson(of, gf, Uf, kappa, dagger=True)
            gpsi = L.unpack_spinor(of, dtype=psi.dtype)
        if ctx.needs_input_grad[1]:
            pf = L.pack_spinor(lattice, psi.contiguous(), prec, L.FULL)
            if link_grad == "su3":
                mode = 0
            else:
                mode = 2 if link == L.LINK12 else 1
            F = L.fermion_force(pf, gf, Uf, -kappa, mode=mode)
            gU = L.unpack_gauge(F, dtype=U.dtype)
        return gpsi, gU, None, None, None, None, None


def wilson_matrix(psi: torch.Tensor, U: torch.Tensor, kappa: float, lattice: L.Lattice,
                  prec: int = L.F64, link: int = L.LINK18, link_grad: str = "raw") -> torch.Tensor:
    """Differentiable M psi on canonical complex device tensors."""
    return WilsonMatrix.apply(psi, U, kappa, lattice, prec, link, link_grad)


class NormalSolve(torch.autograd.Function):
    """x_e = (Mhat^dag Mhat)^-1 b_e on canonical device tensors (even sites).

    Backward is the adjoint solve with the same solver (A is hermitian):
    lambda = A^-1 g; dL/db = lambda on even sites, and the link gradient is
    kappa^2 [W(X(lambda), Y(Mhat x)) + W(X(x), Y(Mhat lambda))] from two
    force-kernel calls, X(v) = (v, D_oe v), Y(v) = (v, (D_eo)^dag v) recomputed
    by hop kernels.  Only x and U are kept from the forward solve.
    """

    @staticmethod
    def forward(ctx, b, U, kappa, lattice, inner_prec, inner_link, tol):
        U_hi = L.pack_gauge(lattice, U.contiguous(), L.F64, L.LINK18)
        U_lo = U_hi if (inner_prec, inner_link) == (L.F64, L.LINK18) else L.pack_gauge(
            lattice, U.contiguous().to(torch.complex64) if inner_prec == L.F32 else U.contiguous(),
            inner_prec, inner_link)
        bf = L.pack_spinor(lattice, b.contiguous().to(torch.complex128), L.F64, L.EVEN)
        x = L.new_spinor(lattice, L.F64, L.EVEN, b.device)
        L.cg_solve(x, bf, U_hi, U_lo, kappa, tol=tol)
        xe = L.unpack_spinor(x)
        ctx.save_for_backward(xe, U)
        ctx.cfg = (kappa, lattice, inner_prec, inner_link, tol)
        return xe.to(b.dtype)

    @staticmethod
    def backward(ctx, g):
        xe, U = ctx.saved_tensors
        kappa, lat, inner_prec, inner_link, tol = ctx.cfg
        dev = xe.device
        U_hi = L.pack_gauge(lat, U.contiguous().to(torch.complex128), L.F64, L.LINK18)
        U_lo = U_hi if (inner_prec, inner_link) == (L.F64, L.LINK18) else L.pack_gauge(
            lat, U.contiguous().to(torch.complex64) if inner_prec == L.F32 else U.contiguous(),
            inner_prec, inner_link)
        gf = L.pack_spinor(lat, g.contiguous().to(torch.complex128), L.F64, L.EVEN)
        lam = L.new_spinor(lat, L.F64, L.EVEN, dev)
        L.cg_solve(lam, gf, U_hi, U_lo, kappa, tol=tol)
        gb = gU = None
        if ctx.needs_input_grad[0]:
            gb = L.unpack_spinor(lam).to(g.dtype)
        if ctx.needs_input_grad[1]:
            x = L.pack_spinor(lat, xe, L.F64, L.EVEN)
            tmp = L.new_spinor(lat, L.F64, L.ODD, dev, zero=False)

            def x_field(v):  # (v, D_oe v)
                f = L.new_spinor(lat, L.F64, L.FULL, dev, zero=False)
                L.convert(f.half(L.EVEN), v)
                L.moe(f.half(L.ODD), v, U_hi)
                return f

            def y_field(v):  # (Mhat v, (D_eo)^dag Mhat v)
                f = L.new_spinor(lat, L.F64, L.FULL, dev, zero=False)
                L.mhat(f.half(L.EVEN), v, tmp, U_hi, kappa)
                L.moe(f.half(L.ODD), f.half(L.EVEN), U_hi, dagger=True)
                return f

            G = L.fermion_force(x_field(lam), y_field(x), U_hi, kappa * kappa, mode=1)
            L.fermion_force(x_field(x), y_field(lam), U_hi, kappa * kappa, mode=1, out=G,
                            accumulate=True)
            gU = L.unpack_gauge(G, dtype=U.dtype)
        return gb, gU, None, None, None, None, None


def normal_solve(b: torch.Tensor, U: torch.Tensor, kappa: float, lattice: L.Lattice,
                 inner_prec: int = L.F64, inner_link: int = L.LINK18,
                 tol: float = 1e-12) -> torch.Tensor:
    """Differentiable x_e = (Mhat^dag Mhat)^-1 b_e (canonical tensors, even sites)."""
    return NormalSolve.apply(b, U, kappa, lattice, inner_prec, inner_link, tol)
