"""Gradients of Wilson-operator actions and the su(3) force (oracle).

TEST INFRASTRUCTURE.  Conventions:

* complex gradients follow PyTorch: grad = dS/dRe + i dS/dIm (no 1/2);
* for an action whose variation is dS = c0 Re( Y^dag (dD_hop) X ), the
  coefficient of Re tr(dU_mu(x) W_mu(x)) is
      W_mu(x) = c0 s+_mu(x) [ X(x+mu) (x) ((1 - g_mu) Y(x))^dag
                             + ((1 + g_mu) Y(x+mu)) (x) X(x)^dag ],
  where (a (x) b^dag)_ij = sum_spin a_{s,i} conj(b_{s,j}); one boundary sign
  per link because the backward hop from x+mu crosses the same boundary,
  s-_mu(x+mu) = s+_mu(x);
* the raw link gradient is G = W^dag;
* the force for left-multiplied variations U -> exp(eps T) U, T traceless
  anti-hermitian, is F = TA(G U^dag) with
  TA(A) = (A - A^dag)/2 - tr(A - A^dag)/6 * 1, so dS/deps = Re tr(T^dag F).

Uses: |M psi|^2 -> c0 = -2 kappa, X = psi, Y = M psi; an upstream gradient
g on phi = M psi -> c0 = -kappa, X = psi, Y = g; the pseudofermion action
phi_e^dag (Mhat^dag Mhat)^-1 phi_e -> c0 = +2 kappa^2 with
X = (X_e, D_oe X_e) and Y = (Mhat X_e, (D_eo)^dag Mhat X_e), X_e the solution.
"""

from __future__ import annotations

import numpy as np

from . import dirac, solver


def outer_spin_sum(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """sum_s a_{s,i} conj(b_{s,j}) -> [..][3][3].

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    return np.einsum("...si,...sj->...ij", a, np.conj(b))


def link_gradient(X, Y, U, c0, bc=dirac.DEFAULT_BC) -> np.ndarray:
    """Raw gradient G_mu(x) = W_mu(x)^dag of c0 Re(Y^dag D_hop X) w.r.t. U.

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    dims = dirac.dims_of(X)
    G = np.zeros_like(U)
    for mu in range(4):
        x_up = dirac.shift(X, mu, +1)
        y_up = dirac.shift(Y, mu, +1)
        t1 = outer_spin_sum(x_up, dirac.spin_mul(dirac.ONE4 - dirac.GAMMA[mu], Y))
        t2 = outer_spin_sum(dirac.spin_mul(dirac.ONE4 + dirac.GAMMA[mu], y_up), X)
        w = c0 * dirac.sign_fwd(dims, bc, mu)[..., None, None] * (t1 + t2)
        G[..., mu, :, :] = dirac.dagger3(w)
    return G


def rows01_gradient(G, U) -> np.ndarray:
    """Raw gradient with respect to the stored rows 0 and 1 of 12-real links.

    When the operator uses V = (row0, row1, conj(row0 x row1)) built from the
    stored rows, and G is the raw gradient with respect to V, the chain rule
    through d row2 = conj(d row0 x row1 + row0 x d row1) gives
        grad row0 = G_0 + conj(row1 x G_2),   grad row1 = G_1 + conj(G_2 x row0),
    and zero for the stored row 2, which the operator never reads.

    The paper does not treat derivatives or link compression; chain rule of
    the standard 12-real form in the conventions of this module's header.
    """
    out = np.zeros_like(G)
    r0, r1, g2 = U[..., 0, :], U[..., 1, :], G[..., 2, :]
    out[..., 0, :] = G[..., 0, :] + np.conj(np.cross(r1, g2))
    out[..., 1, :] = G[..., 1, :] + np.conj(np.cross(g2, r0))
    return out


def traceless_antihermitian(a: np.ndarray) -> np.ndarray:
    """TA(A) = (A - A^dag)/2 - tr(A - A^dag)/6 * 1.

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    d = 0.5 * (a - dirac.dagger3(a))
    tr = np.trace(d, axis1=-2, axis2=-1)
    return d - (tr / 3.0)[..., None, None] * np.eye(3)


def su3_force(G, U) -> np.ndarray:
    """F_mu(x) = TA(G_mu(x) U_mu(x)^dag).

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    return traceless_antihermitian(G @ dirac.dagger3(U))


def action_norm(psi, U, kappa, bc=dirac.DEFAULT_BC) -> float:
    """S = sum_x |(M psi)(x)|^2.

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    phi = dirac.wilson(psi, U, kappa, bc)
    return float(np.vdot(phi.ravel(), phi.ravel()).real)


def grad_psi_norm(psi, U, kappa, bc=dirac.DEFAULT_BC) -> np.ndarray:
    """dS/dpsi for S = |M psi|^2: 2 M^dag M psi.

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    return 2.0 * dirac.wilson(dirac.wilson(psi, U, kappa, bc), U, kappa, bc, dagger=True)


def grad_links_norm(psi, U, kappa, bc=dirac.DEFAULT_BC) -> np.ndarray:
    """dS/dU for S = |M psi|^2 (raw complex gradient, PyTorch convention).

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    phi = dirac.wilson(psi, U, kappa, bc)
    return link_gradient(psi, phi, U, -2.0 * kappa, bc)


def vjp(psi, U, kappa, g, bc=dirac.DEFAULT_BC):
    """Vector-Jacobian product of phi = M psi for an upstream gradient g.

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    gpsi = dirac.wilson(g, U, kappa, bc, dagger=True)
    gU = link_gradient(psi, g, U, -kappa, bc)
    return gpsi, gU


def pseudofermion_fields(x_e, U, kappa, bc=dirac.DEFAULT_BC):
    """(X, Y) on the full lattice for S = phi_e^dag (Mhat^dag Mhat)^-1 phi_e.

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    x_o = dirac.moe(x_e, U, bc)
    y_e = dirac.mhat(x_e, U, kappa, bc)
    y_o = dirac.moe(y_e, U, bc, dagger=True)
    return dirac.project(x_e, 0) + x_o, y_e + y_o


def pseudofermion_force(x_e, U, kappa, bc=dirac.DEFAULT_BC):
    """su(3) force of the pseudofermion action given its solution X_e.

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    X, Y = pseudofermion_fields(x_e, U, kappa, bc)
    return su3_force(link_gradient(X, Y, U, 2.0 * kappa ** 2, bc), U)


def link_gradient_at(X, Y, U, c0, links, bc=dirac.DEFAULT_BC) -> np.ndarray:
    """G_mu(x) for a list of links given as rows (x, y, z, t, mu); [n][3][3].

    Same definition as :func:`link_gradient`, evaluated link by link from
    the fields at x and x + mu (for fields too large to shift whole).

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    dims = dirac.dims_of(X)
    links = np.asarray(links, dtype=np.int64)
    n = links.shape[0]
    out = np.zeros((n, 3, 3), dtype=np.complex128)

    def at(field, c):
        return field[c[:, 3], c[:, 2], c[:, 1], c[:, 0]]

    sites = links[:, :4]
    for mu in range(4):
        sel = np.nonzero(links[:, 4] == mu)[0]
        if sel.size == 0:
            continue
        here = sites[sel]
        up = here.copy()
        up[:, mu] = (here[:, mu] + 1) % dims[mu]
        sgn = np.where(here[:, mu] == dims[mu] - 1, float(bc[mu]), 1.0)
        x_h, y_h, x_u, y_u = at(X, here), at(Y, here), at(X, up), at(Y, up)
        pm = dirac.ONE4 - dirac.GAMMA[mu]
        pp = dirac.ONE4 + dirac.GAMMA[mu]
        t1 = np.einsum("nsi,nsj->nij", x_u, np.conj(np.einsum("st,ntc->nsc", pm, y_h)))
        t2 = np.einsum("nsi,nsj->nij", np.einsum("st,ntc->nsc", pp, y_u), np.conj(x_h))
        w = c0 * sgn[:, None, None] * (t1 + t2)
        out[sel] = np.conj(np.swapaxes(w, -1, -2))
    return out


def su3_force_at(G, U_links) -> np.ndarray:
    """TA(G U^dag) for gathered links ([n][3][3] each).

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    return traceless_antihermitian(G @ dirac.dagger3(U_links))


def _xy_fields(v_e, U, bc):
    """(v, D_oe v) and (v, (D_eo)^dag v) as full fields."""
    ve = dirac.project(v_e, 0)
    return ve + dirac.moe(ve, U, bc), ve + dirac.moe(ve, U, bc, dagger=True)


def normal_solve_vjp(x_e, g_e, U, kappa, bc=dirac.DEFAULT_BC, tol=1e-13):
    """Vector-Jacobian product of x = A^-1 b, A = Mhat^dag Mhat (even sites).

    For dL = Re(g^dag dx):  dL/db = lambda = A^-1 g (A is hermitian), and
    dx = -A^-1 dA x gives dL = -Re(lambda^dag dA x) with
    dA = dMhat^dag Mhat + Mhat^dag dMhat and
    Re(a^dag dMhat b) = -kappa^2 Re(Y(a)^dag dD_hop X(b)),
    X(b) = (b, D_oe b), Y(a) = (a, (D_eo)^dag a), so
    dL = kappa^2 [Re(Y(Mhat x)^dag dD X(lambda)) + Re(Y(Mhat lambda)^dag dD X(x))].
    Returns (lambda, raw link gradient G).

    The paper does not treat derivatives; textbook definition in the
    conventions of this module's header.
    """
    lam, _, _ = solver.solve_normal(g_e, U, kappa, bc, tol=tol)
    X1, _ = _xy_fields(lam, U, bc)
    _, Y1 = _xy_fields(dirac.mhat(x_e, U, kappa, bc), U, bc)
    X2, _ = _xy_fields(x_e, U, bc)
    _, Y2 = _xy_fields(dirac.mhat(lam, U, kappa, bc), U, bc)
    G = link_gradient(X1, Y1, U, kappa ** 2, bc) + link_gradient(X2, Y2, U, kappa ** 2, bc)
    return lam, G
