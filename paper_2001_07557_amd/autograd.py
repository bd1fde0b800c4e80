"""torch.autograd wrapper of the Wilson matrix with hand-written adjoints.

phi = M psi = psi - kappa D_hop[U] psi on canonical device tensors.  The
backward pass runs two library kernels:

* dL/dpsi = M^dag g (the adjoint hopping kernel),
* dL/dU from the fermion-force kernel with X = psi, Y = g, c0 = -kappa: the raw
  complex gradient G = dL/dRe U + i dL/dIm U (``link_grad="raw"``, what torch
  optimisers and gradcheck expect) or the su(3)-projected force
  F = TA(G U^dag) for U -> exp(eps T) U (``link_grad="su3"``).

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
        of = L.new_spinor(lattice, prec, L.FULL, psi.device)
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
            of = L.new_spinor(lattice, prec, L.FULL, psi.device)
            L.wilson(of, gf, Uf, kappa, dagger=True)
            gpsi = L.unpack_spinor(of, dtype=psi.dtype)
        if ctx.needs_input_grad[1]:
            pf = L.pack_spinor(lattice, psi.contiguous(), prec, L.FULL)
            F = L.fermion_force(pf, gf, Uf, -kappa, mode=1 if link_grad == "raw" else 0)
            gU = L.unpack_gauge(F, dtype=U.dtype)
        return gpsi, gU, None, None, None, None, None


def wilson_matrix(psi: torch.Tensor, U: torch.Tensor, kappa: float, lattice: L.Lattice,
                  prec: int = L.F64, link: int = L.LINK18, link_grad: str = "raw") -> torch.Tensor:
    """Differentiable M psi on canonical complex device tensors."""
    return WilsonMatrix.apply(psi, U, kappa, lattice, prec, link, link_grad)
