"""Wilson hopping operator, plain FP64 definition (oracle; test infrastructure).

Conventions (the paper names the operator in Sec. 3.3 / Fig. 4d without
defining it; these are the readings used throughout):

* directions mu = 0,1,2,3 = x,y,z,t; canonical arrays are indexed
  [t][z][y][x][spin][colour], so direction mu lives on array axis 3 - mu;
* DeGrand-Rossi chiral gamma basis, gamma5 = g_x g_y g_z g_t = diag(1,1,-1,-1);
* hopping term
      (D_hop psi)(x) = sum_mu [ s+_mu(x) (1 - g_mu) U_mu(x) psi(x + mu)
                              + s-_mu(x) (1 + g_mu) U_mu(x - mu)^dag psi(x - mu) ]
  with s+_mu(x) = bc_mu when x_mu = L_mu - 1 (else 1) and s-_mu(x) = bc_mu when
  x_mu = 0 (else 1); bc = (+1,+1,+1,-1) is periodic in space and
  antiperiodic in time;
* the adjoint D_hop^dag is the same sum with (1 - g_mu) and (1 + g_mu)
  exchanged;
* Wilson matrix M = 1 - kappa D_hop;
* parity(x) = (x + y + z + t) mod 2, even = 0; the even-odd blocks are
  D_eo = P_e D_hop P_o and D_oe = P_o D_hop P_e with P_e, P_o the projectors
  on even and odd sites, and the Schur operator on even sites is
  Mhat = 1 - kappa^2 D_eo D_oe, Mhat^dag = 1 - kappa^2 (D_oe)^dag (D_eo)^dag.

Even-odd vectors are represented as full canonical arrays that vanish on the
other parity.
"""

from __future__ import annotations

from typing import Sequence

import numpy as np

DEFAULT_BC = (1, 1, 1, -1)

_i = 1j
GAMMA = np.array([
    # gamma_x
    [[0, 0, 0, _i], [0, 0, _i, 0], [0, -_i, 0, 0], [-_i, 0, 0, 0]],
    # gamma_y
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    # gamma_z
    [[0, 0, _i, 0], [0, 0, 0, -_i], [-_i, 0, 0, 0], [0, _i, 0, 0]],
    # gamma_t
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
], dtype=np.complex128)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ONE4 = np.eye(4, dtype=np.complex128)


def dims_of(field) -> tuple:
    lt, lz, ly, lx = field.shape[:4]
    return (lx, ly, lz, lt)


def shift(field: np.ndarray, mu: int, s: int) -> np.ndarray:
    """field(x + s mu_hat), periodic wrap (boundary signs applied separately).

    Shifts of Sec. 3.1 (the building block of the paper's stencils).
    """
    return np.roll(field, -s, axis=3 - mu)


def cshift(field: np.ndarray, mu: int, s: int, bc=DEFAULT_BC) -> np.ndarray:
    """out(x) = field(x + s mu_hat) times bc_mu when the step crosses the
    boundary (s = +1 from the last slice, s = -1 from the first).

    Shifts of Sec. 3.1 (the building block of the paper's stencils).
    """
    dims = dims_of(field)
    out = shift(field, mu, s)
    edge = dims[mu] - 1 if s > 0 else 0
    sign = np.where(coord(dims, mu) == edge, float(bc[mu]), 1.0)
    return out * sign.reshape(sign.shape + (1,) * (field.ndim - 4))


def coord(dims: Sequence[int], mu: int) -> np.ndarray:
    """Array [t][z][y][x] holding the coordinate x_mu of each site."""
    lx, ly, lz, lt = dims
    grids = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                        indexing="ij")
    return grids[3 - mu]


def sign_fwd(dims, bc, mu) -> np.ndarray:
    """s+_mu(x): bc_mu on the last slice in direction mu, 1 elsewhere.

    Operator timed in Sec. 3.3 (Fig. 4d); the paper gives no formula, so this
    is the textbook definition in the conventions of this module's header.
    """
    return np.where(coord(dims, mu) == dims[mu] - 1, float(bc[mu]), 1.0)


def sign_bwd(dims, bc, mu) -> np.ndarray:
    """s-_mu(x): bc_mu on the first slice in direction mu, 1 elsewhere.

    Operator timed in Sec. 3.3 (Fig. 4d); the paper gives no formula, so this
    is the textbook definition in the conventions of this module's header.
    """
    return np.where(coord(dims, mu) == 0, float(bc[mu]), 1.0)


def spin_mul(p: np.ndarray, chi: np.ndarray) -> np.ndarray:
    """(p chi)_s = sum_t p_st chi_t, for every site and colour."""
    return np.einsum("st,...tc->...sc", p, chi)


def colour_mul(u: np.ndarray, chi: np.ndarray) -> np.ndarray:
    """(u chi)_a = sum_b u_ab chi_b, for every site and spin."""
    return np.einsum("...ab,...sb->...sa", u, chi)


def dagger3(u: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(u, -1, -2))


def dhop(psi: np.ndarray, U: np.ndarray, bc=DEFAULT_BC, dagger: bool = False) -> np.ndarray:
    """D_hop psi (or D_hop^dag psi) on the full lattice.

    Operator timed in Sec. 3.3 (Fig. 4d); the paper gives no formula, so this
    is the textbook definition in the conventions of this module's header.
    """
    dims = dims_of(psi)
    out = np.zeros_like(psi)
    sg = -1.0 if dagger else 1.0
    for mu in range(4):
        p_fwd = ONE4 - sg * GAMMA[mu]
        p_bwd = ONE4 + sg * GAMMA[mu]
        umu = U[..., mu, :, :]
        fwd = colour_mul(umu, shift(psi, mu, +1))
        fwd = fwd * sign_fwd(dims, bc, mu)[..., None, None]
        bwd = shift(colour_mul(dagger3(umu), psi), mu, -1)
        bwd = bwd * sign_bwd(dims, bc, mu)[..., None, None]
        out += spin_mul(p_fwd, fwd) + spin_mul(p_bwd, bwd)
    return out


def dhop_binary16(q: np.ndarray, s: np.ndarray, U: np.ndarray, bc=DEFAULT_BC,
                  dagger: bool = False) -> np.ndarray:
    """D_hop (or D_hop^dag) of a spinor field held in per-site scaled binary16
    storage: stored values q, site scales s (links.f16_spinor_parts).

    Reading for binary16 storage (the paper does not treat reduced
    precision): every hop first forms the projected spinor (1 -+ g_mu) q of
    the neighbour site from its stored values, rounds it to binary16 (one
    rounding of the exact sum, ties to even; rows 2 and 3 of a projected
    spinor are unit multiples of rows 0 and 1, so rounding all four rows is
    rounding the half-spinor), multiplies by that site's scale and by the
    link; everything else is exact.  With no rounding this is dhop(q s).
    """
    from oracle.links import round_half

    dims = dims_of(q)
    out = np.zeros_like(q)
    sg = -1.0 if dagger else 1.0
    sc = s[..., None, None]
    for mu in range(4):
        p_fwd = ONE4 - sg * GAMMA[mu]
        p_bwd = ONE4 + sg * GAMMA[mu]
        umu = U[..., mu, :, :]
        hf = round_half(spin_mul(p_fwd, q)) * sc
        hb = round_half(spin_mul(p_bwd, q)) * sc
        fwd = colour_mul(umu, shift(hf, mu, +1)) * sign_fwd(dims, bc, mu)[..., None, None]
        bwd = shift(colour_mul(dagger3(umu), hb), mu, -1) * sign_bwd(dims, bc, mu)[..., None, None]
        out += fwd + bwd
    return out


def wilson(psi, U, kappa, bc=DEFAULT_BC, dagger=False):
    """M psi = psi - kappa D_hop psi (M^dag with dagger=True).

    Operator timed in Sec. 3.3 (Fig. 4d); the paper gives no formula, so this
    is the textbook definition in the conventions of this module's header.
    """
    return psi - kappa * dhop(psi, U, bc, dagger)


# ----------------------------------------------------------------------------
# even-odd
# ----------------------------------------------------------------------------

def odd_mask(dims) -> np.ndarray:
    lx, ly, lz, lt = dims
    s = sum(coord(dims, mu) for mu in range(4))
    return (s % 2) == 1


def project(psi: np.ndarray, parity: int) -> np.ndarray:
    """P_parity psi: keep the sites of the given parity, zero the others.

    Operator timed in Sec. 3.3 (Fig. 4d); the paper gives no formula, so this
    is the textbook definition in the conventions of this module's header.
    """
    m = odd_mask(dims_of(psi))
    keep = m if parity == 1 else ~m
    return psi * keep[..., None, None]


def meo(psi_o, U, bc=DEFAULT_BC, dagger=False):
    """Even rows, odd columns of D_hop (or of D_hop^dag).

    Operator timed in Sec. 3.3 (Fig. 4d); the paper gives no formula, so this
    is the textbook definition in the conventions of this module's header.
    """
    return project(dhop(project(psi_o, 1), U, bc, dagger), 0)


def moe(psi_e, U, bc=DEFAULT_BC, dagger=False):
    """Odd rows, even columns of D_hop (or of D_hop^dag).

    Operator timed in Sec. 3.3 (Fig. 4d); the paper gives no formula, so this
    is the textbook definition in the conventions of this module's header.
    """
    return project(dhop(project(psi_e, 0), U, bc, dagger), 1)


def meo_binary16(q_o, s_o, U, bc=DEFAULT_BC, dagger=False):
    """D_eo on binary16 storage (dhop_binary16; q_o, s_o of the odd sites).

    Reading for binary16 storage; the paper does not treat reduced precision.
    """
    m = odd_mask(dims_of(q_o))
    return project(dhop_binary16(q_o * m[..., None, None], s_o * m, U, bc, dagger), 0)


def moe_binary16(q_e, s_e, U, bc=DEFAULT_BC, dagger=False):
    """D_oe on binary16 storage (dhop_binary16; q_e, s_e of the even sites).

    Reading for binary16 storage; the paper does not treat reduced precision.
    """
    m = ~odd_mask(dims_of(q_e))
    return project(dhop_binary16(q_e * m[..., None, None], s_e * m, U, bc, dagger), 1)


def mhat(x_e, U, kappa, bc=DEFAULT_BC):
    """Schur operator on even sites: x_e - kappa^2 D_eo D_oe x_e.

    Operator timed in Sec. 3.3 (Fig. 4d); the paper gives no formula, so this
    is the textbook definition in the conventions of this module's header.
    """
    return project(x_e, 0) - kappa ** 2 * meo(moe(x_e, U, bc), U, bc)


def mhat_dag(x_e, U, kappa, bc=DEFAULT_BC):
    """Adjoint Schur operator: x_e - kappa^2 (D_oe)^dag (D_eo)^dag x_e.

    (D_eo)^dag is the odd-even block of D_hop^dag and (D_oe)^dag its even-odd
    block.

    Operator timed in Sec. 3.3 (Fig. 4d); the paper gives no formula, so this
    is the textbook definition in the conventions of this module's header.
    """
    return project(x_e, 0) - kappa ** 2 * meo(moe(x_e, U, bc, True), U, bc, True)


def normal_op(x_e, U, kappa, bc=DEFAULT_BC):
    """A x_e = Mhat^dag Mhat x_e (hermitian positive definite).

    Operator timed in Sec. 3.3 (Fig. 4d); the paper gives no formula, so this
    is the textbook definition in the conventions of this module's header.
    """
    return mhat_dag(mhat(x_e, U, kappa, bc), U, kappa, bc)


# ----------------------------------------------------------------------------
# per-site sampling for lattices too large for the whole-field routines
# ----------------------------------------------------------------------------

def dhop_at(psi, U, sites: np.ndarray, bc=DEFAULT_BC, dagger=False) -> np.ndarray:
    """(D_hop psi)(x) for a list of sites x given as rows (x, y, z, t).

    Returns an array [n][4][3].  Neighbour coordinates wrap modulo L_mu and
    pick up bc_mu when the hop crosses the boundary.

    Operator timed in Sec. 3.3 (Fig. 4d); the paper gives no formula, so this
    is the textbook definition in the conventions of this module's header.
    """
    dims = dims_of(psi)
    sites = np.asarray(sites, dtype=np.int64)
    out = np.zeros((sites.shape[0], 4, 3), dtype=np.complex128)
    sg = -1.0 if dagger else 1.0

    def at(field, c):
        return field[c[:, 3], c[:, 2], c[:, 1], c[:, 0]]

    for mu in range(4):
        L = dims[mu]
        up = sites.copy()
        up[:, mu] = (sites[:, mu] + 1) % L
        dn = sites.copy()
        dn[:, mu] = (sites[:, mu] - 1) % L
        s_up = np.where(sites[:, mu] == L - 1, float(bc[mu]), 1.0)
        s_dn = np.where(sites[:, mu] == 0, float(bc[mu]), 1.0)
        u_here = at(U, sites)[:, mu]
        u_dn = at(U, dn)[:, mu]
        fwd = np.einsum("nab,nsb->nsa", u_here, at(psi, up)) * s_up[:, None, None]
        bwd = np.einsum("nab,nsb->nsa", dagger3(u_dn), at(psi, dn)) * s_dn[:, None, None]
        out += np.einsum("st,ntc->nsc", ONE4 - sg * GAMMA[mu], fwd)
        out += np.einsum("st,ntc->nsc", ONE4 + sg * GAMMA[mu], bwd)
    return out


def dhop_at_binary16(q, s, U, sites: np.ndarray, bc=DEFAULT_BC, dagger=False) -> np.ndarray:
    """dhop_binary16 at a list of sites (rows x, y, z, t); q, s and U are
    indexed like arrays (they may gather from larger fields on demand).

    Reading for binary16 storage; the paper does not treat reduced precision.
    """
    from oracle.links import round_half

    dims = tuple(q.shape[3 - mu] for mu in range(4))
    sites = np.asarray(sites, dtype=np.int64)
    out = np.zeros((sites.shape[0], 4, 3), dtype=np.complex128)
    sg = -1.0 if dagger else 1.0

    def at(field, c):
        return field[c[:, 3], c[:, 2], c[:, 1], c[:, 0]]

    for mu in range(4):
        L = dims[mu]
        up = sites.copy()
        up[:, mu] = (sites[:, mu] + 1) % L
        dn = sites.copy()
        dn[:, mu] = (sites[:, mu] - 1) % L
        s_up = np.where(sites[:, mu] == L - 1, float(bc[mu]), 1.0)
        s_dn = np.where(sites[:, mu] == 0, float(bc[mu]), 1.0)
        hf = round_half(np.einsum("st,ntc->nsc", ONE4 - sg * GAMMA[mu], at(q, up))) \
            * at(s, up)[:, None, None]
        hb = round_half(np.einsum("st,ntc->nsc", ONE4 + sg * GAMMA[mu], at(q, dn))) \
            * at(s, dn)[:, None, None]
        out += np.einsum("nab,nsb->nsa", at(U, sites)[:, mu], hf) * s_up[:, None, None]
        out += np.einsum("nab,nsb->nsa", dagger3(at(U, dn)[:, mu]), hb) * s_dn[:, None, None]
    return out


def site_parity(sites: np.ndarray) -> np.ndarray:
    return np.asarray(sites).sum(axis=1) % 2
