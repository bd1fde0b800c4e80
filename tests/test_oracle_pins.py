"""Pins of the FP64 oracle against facts fixed by the mathematics.

Each test checks the oracle against something other than itself: closed
forms of the free operator in momentum space, the adjoint defined by the
inner product, gauge covariance, an independently assembled dense matrix,
exact solutions, and central finite differences of the action.
"""

import itertools

import numpy as np
import pytest

import lattice_inputs as LI
from oracle import dirac, force, links, solver
from oracle.dirac import GAMMA, GAMMA5, ONE4
from tests.dense_wilson import dense_dhop, parity_vector

KAPPA = 0.124
BC = (1, 1, 1, -1)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def multiset_dist(a, b):
    """Largest distance in a greedy nearest-neighbour matching of a to b."""
    b = list(np.asarray(b).ravel())
    worst = 0.0
    for z in np.asarray(a).ravel():
        d = [abs(z - w) for w in b]
        k = int(np.argmin(d))
        worst = max(worst, d[k])
        b.pop(k)
    return worst


def unit_links(dims):
    U = np.zeros(LI.links_shape(dims), dtype=np.complex128)
    U[...] = np.eye(3)
    return U


def plane_wave(dims, p, u):
    """e^{i p.x} u on every site, u a [4][3] spin-colour vector."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[..., None, None] * u, ph


def momenta(dims, bc=BC):
    """All lattice momenta compatible with the boundary conditions."""
    axes = []
    for mu in range(4):
        L = dims[mu]
        off = 0.5 if bc[mu] == -1 else 0.0
        axes.append([2 * np.pi * (n + off) / L for n in range(L)])
    return list(itertools.product(*axes))


def d_of_p(p, dagger=False):
    """Free hopping term in momentum space: sum_mu 2 cos p - 2 i g sin p."""
    sg = -1.0 if dagger else 1.0
    return sum(2 * np.cos(p[mu]) * ONE4 - sg * 2j * np.sin(p[mu]) * GAMMA[mu]
               for mu in range(4))


# ----------------------------------------------------------------------------
# gamma matrices
# ----------------------------------------------------------------------------

def test_gamma_clifford_hermitian_chiral():
    for mu in range(4):
        assert np.allclose(GAMMA[mu], GAMMA[mu].conj().T)
        for nu in range(4):
            anti = GAMMA[mu] @ GAMMA[nu] + GAMMA[nu] @ GAMMA[mu]
            assert np.allclose(anti, 2.0 * (mu == nu) * ONE4)
    # chiral (DeGrand-Rossi) basis: gamma5 diagonal
    assert np.allclose(GAMMA5, np.diag([1, 1, -1, -1]))
    for mu in range(4):
        assert np.allclose(GAMMA5 @ GAMMA[mu], -GAMMA[mu] @ GAMMA5)


# ----------------------------------------------------------------------------
# free field: plane waves are eigenvectors with closed-form eigenvalues
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10)])
def test_free_field_plane_waves(dims):
    rng = np.random.default_rng(7)
    U = unit_links(dims)
    ps = momenta(dims)
    if len(ps) > 300:
        ps = [ps[i] for i in rng.choice(len(ps), 300, replace=False)]
    for p in ps:
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi, ph = plane_wave(dims, p, u)
        for dag in (False, True):
            got = dirac.dhop(psi, U, BC, dagger=dag)
            want = ph[..., None, None] * (d_of_p(p, dag) @ u)
            assert np.abs(got - want).max() < 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10)])
def test_free_field_spectrum(dims):
    """eig M(p) = 1 - 2k sum cos p +- 2ik sqrt(sum sin^2 p), doubly degenerate.

    Built from the operator by applying it to the four spin basis plane waves
    at each momentum, so it depends only on the Clifford algebra.
    """
    U = unit_links(dims)
    for p in momenta(dims)[::7]:
        cols = []
        for s in range(4):
            u = np.zeros((4, 3), dtype=np.complex128)
            u[s, 0] = 1.0
            psi, ph = plane_wave(dims, p, u)
            m = dirac.wilson(psi, U, KAPPA, BC)
            cols.append((m[0, 0, 0, 0, :, 0] / ph[0, 0, 0, 0]))
        mp = np.array(cols).T
        ev = np.linalg.eigvals(mp)
        c = np.sum(np.cos(p))
        s = np.sqrt(np.sum(np.sin(p) ** 2))
        want = [1 - 2 * KAPPA * c + 2j * KAPPA * s] * 2 + [1 - 2 * KAPPA * c - 2j * KAPPA * s] * 2
        assert multiset_dist(ev, want) < 1e-12


# ----------------------------------------------------------------------------
# adjoint, gamma5-hermiticity, gauge covariance
# ----------------------------------------------------------------------------

def test_dagger_is_adjoint_and_gamma5_hermitian():
    dims = (4, 4, 4, 4)
    U, psi = LI.workload_fields(0, dims)
    rng = np.random.default_rng(11)
    phi = LI.gaussian_spinor(rng, dims)
    lhs = np.vdot(phi, dirac.dhop(psi, U, BC))
    rhs = np.vdot(dirac.dhop(phi, U, BC, dagger=True), psi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-14
    g5 = lambda f: dirac.spin_mul(GAMMA5, f)  # noqa: E731
    assert rel(g5(dirac.dhop(g5(psi), U, BC)), dirac.dhop(psi, U, BC, dagger=True)) < 1e-14


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10)])
def test_gauge_covariance(dims):
    U, psi = LI.workload_fields(1, dims)
    om = LI.random_gauge_transform(1, dims)
    Ug = LI.gauge_transform_links(U, om)
    psig = LI.gauge_transform_spinor(psi, om)
    for dag in (False, True):
        lhs = dirac.dhop(psig, Ug, BC, dagger=dag)
        rhs = LI.gauge_transform_spinor(dirac.dhop(psi, U, BC, dagger=dag), om)
        assert rel(lhs, rhs) < 1e-14


def test_translation_covariance_periodic():
    """With periodic boundaries, shifting fields and links commutes with D_hop."""
    dims = (4, 4, 4, 6)
    U, psi = LI.workload_fields(2, dims)
    pbc = (1, 1, 1, 1)
    for mu in range(4):
        lhs = dirac.dhop(dirac.shift(psi, mu, 1), dirac.shift(U, mu, 1), pbc)
        rhs = dirac.shift(dirac.dhop(psi, U, pbc), mu, 1)
        assert rel(lhs, rhs) < 1e-14


# ----------------------------------------------------------------------------
# dense matrices on tiny lattices
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 2, 4)])
def test_dense_matrix_matches_oracle(dims):
    U, _ = LI.workload_fields(3, dims)
    n = 12 * LI.volume(dims)
    for dag in (False, True):
        D = dense_dhop(U, dims, BC, dagger=dag)
        rng = np.random.default_rng(5)
        for _ in range(6):
            v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
            got = dirac.dhop(v.reshape(LI.spinor_shape(dims)), U, BC, dagger=dag).ravel()
            assert rel(got, D @ v) < 1e-14
    D = dense_dhop(U, dims, BC)
    Dd = dense_dhop(U, dims, BC, dagger=True)
    assert np.abs(Dd - D.conj().T).max() < 1e-14
    # gamma5-hermiticity makes det M real and pairs eigenvalues with conjugates
    M = np.eye(n) - KAPPA * D
    ev = np.linalg.eigvals(M)
    assert multiset_dist(ev, ev.conj()) < 1e-10
    sign, logdet = np.linalg.slogdet(M)
    assert abs(sign.imag) < 1e-10


def test_dense_free_spectrum_2x4():
    """Free 2^4, antiperiodic t: eig M = 1 - 2k sum_i cos p_i +- 2ik."""
    dims = (2, 2, 2, 2)
    D = dense_dhop(unit_links(dims), dims, BC)
    ev = np.linalg.eigvals(np.eye(192) - KAPPA * D)
    want = []
    for px, py, pz in itertools.product([0, np.pi], repeat=3):
        for _pt in (np.pi / 2, 3 * np.pi / 2):
            c = np.cos(px) + np.cos(py) + np.cos(pz)
            want += [1 - 2 * KAPPA * c + 2j * KAPPA] * 6 + [1 - 2 * KAPPA * c - 2j * KAPPA] * 6
    assert multiset_dist(ev, want) < 1e-10


# ----------------------------------------------------------------------------
# even-odd
# ----------------------------------------------------------------------------

def test_even_odd_blocks():
    dims = (4, 4, 4, 4)
    U, psi = LI.workload_fields(4, dims)
    full = dirac.dhop(psi, U, BC)
    split = dirac.meo(psi, U, BC) + dirac.moe(psi, U, BC)
    assert rel(split, full) < 1e-15
    # D_hop only connects opposite parities
    assert np.abs(dirac.project(dirac.dhop(dirac.project(psi, 0), U, BC), 0)).max() == 0.0
    # adjoint blocks: <a_e, D_eo b_o> = <(D_eo)^dag a_e, b_o>, (D_eo)^dag = odd rows of D^dag
    rng = np.random.default_rng(9)
    a = dirac.project(LI.gaussian_spinor(rng, dims), 0)
    b = dirac.project(LI.gaussian_spinor(rng, dims), 1)
    lhs = np.vdot(a, dirac.meo(b, U, BC))
    rhs = np.vdot(dirac.moe(a, U, BC, dagger=True), b)
    assert abs(lhs - rhs) / abs(lhs) < 1e-14


def test_schur_operator_adjoint_and_dense():
    dims = (2, 2, 2, 4)
    U, _ = LI.workload_fields(5, dims)
    D = dense_dhop(U, dims, BC)
    par = parity_vector(dims)
    e = np.where(par == 0)[0]
    o = np.where(par == 1)[0]
    Deo = D[np.ix_(e, o)]
    Doe = D[np.ix_(o, e)]
    Mhat = np.eye(len(e)) - KAPPA ** 2 * Deo @ Doe
    rng = np.random.default_rng(13)
    v = rng.standard_normal(12 * LI.volume(dims)) + 1j * rng.standard_normal(12 * LI.volume(dims))
    v[o] = 0
    field = v.reshape(LI.spinor_shape(dims))
    got = dirac.mhat(field, U, KAPPA, BC).ravel()
    assert rel(got[e], Mhat @ v[e]) < 1e-14 and np.abs(got[o]).max() == 0.0
    gotd = dirac.mhat_dag(field, U, KAPPA, BC).ravel()
    assert rel(gotd[e], Mhat.conj().T @ v[e]) < 1e-14


def test_even_plane_wave_schur_eigenvalues():
    """On even-site plane waves Mhat acts as 1 - k^2 D(p)^2, eig 1 - 4k^2 (C +- iS)^2."""
    dims = (4, 4, 4, 4)
    U = unit_links(dims)
    rng = np.random.default_rng(3)
    for p in momenta(dims)[::5]:
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi, ph = plane_wave(dims, p, u)
        psi_e = dirac.project(psi, 0)
        got = dirac.mhat(psi_e, U, KAPPA, BC)
        dp = d_of_p(p)
        want = dirac.project(ph[..., None, None] * ((ONE4 - KAPPA ** 2 * dp @ dp) @ u), 0)
        assert np.abs(got - want).max() < 1e-12
        ev = np.linalg.eigvals(ONE4 - KAPPA ** 2 * dp @ dp)
        C = np.sum(np.cos(p))
        S = np.sqrt(np.sum(np.sin(p) ** 2))
        w = [1 - 4 * KAPPA ** 2 * (C + 1j * S) ** 2] * 2 + [1 - 4 * KAPPA ** 2 * (C - 1j * S) ** 2] * 2
        assert multiset_dist(ev, w) < 1e-12


# ----------------------------------------------------------------------------
# sampled evaluation
# ----------------------------------------------------------------------------

def test_sampled_sites_match_field():
    dims = (4, 6, 8, 10)
    U, psi = LI.workload_fields(6, dims)
    rng = np.random.default_rng(17)
    sites = np.stack([rng.integers(0, dims[m], 50) for m in range(4)], axis=1)
    sites[0] = [0, 0, 0, 0]
    sites[1] = [dims[0] - 1, dims[1] - 1, dims[2] - 1, dims[3] - 1]
    for dag in (False, True):
        full = dirac.dhop(psi, U, BC, dagger=dag)
        got = dirac.dhop_at(psi, U, sites, BC, dagger=dag)
        want = full[sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]]
        assert np.abs(got - want).max() < 1e-13


# ----------------------------------------------------------------------------
# CG
# ----------------------------------------------------------------------------

def test_cg_free_field_exact_solution():
    dims = (4, 4, 4, 4)
    U = unit_links(dims)
    p = momenta(dims)[37]
    u = np.arange(12).reshape(4, 3) * (0.3 + 0.2j) + 1.0
    b, ph = plane_wave(dims, p, u)
    b = dirac.project(b, 0)
    x, it, res = solver.solve_normal(b, U, KAPPA, BC, tol=1e-12)
    dp = d_of_p(p)
    mp = ONE4 - KAPPA ** 2 * dp @ dp
    xp = np.linalg.solve(mp.conj().T @ mp, u)
    want = dirac.project(ph[..., None, None] * xp, 0)
    assert res <= 1e-12
    assert rel(x, want) < 1e-11


def test_cg_matches_dense_solve():
    dims = (2, 2, 2, 4)
    U, psi = LI.workload_fields(7, dims)
    D = dense_dhop(U, dims, BC)
    par = parity_vector(dims)
    e = np.where(par == 0)[0]
    o = np.where(par == 1)[0]
    Mhat = np.eye(len(e)) - KAPPA ** 2 * D[np.ix_(e, o)] @ D[np.ix_(o, e)]
    b = dirac.project(psi, 0)
    x, it, res = solver.solve_normal(b, U, KAPPA, BC, tol=1e-12)
    xd = np.linalg.solve(Mhat.conj().T @ Mhat, b.ravel()[e])
    assert res <= 1e-12
    assert rel(x.ravel()[e], xd) < 1e-10
    assert solver.true_residual(x, b, U, KAPPA, BC) <= 1e-12


def test_full_solution_via_schur():
    dims = (4, 4, 4, 4)
    U, b = LI.workload_fields(8, dims)
    x, _ = solver.full_solution(b, U, KAPPA, BC, tol=1e-12)
    assert rel(dirac.wilson(x, U, KAPPA, BC), b) < 1e-10


# ----------------------------------------------------------------------------
# gradients and force (central finite differences of the action)
# ----------------------------------------------------------------------------

def gell_mann():
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j; l[1][1, 0] = 1j
    l[2][0, 0] = 1; l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j; l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j; l[6][2, 1] = 1j
    l[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return l


def expm_ah(T, h):
    """exp(h T) for anti-hermitian T through the eigen-decomposition of iT."""
    w, v = np.linalg.eigh(1j * T)
    return v @ np.diag(np.exp(-1j * h * w)) @ v.conj().T


def test_grad_psi_finite_differences():
    dims = (4, 4, 4, 4)
    U, psi = LI.workload_fields(9, dims)
    g = force.grad_psi_norm(psi, U, KAPPA, BC)
    rng = LI.fd_rng(9)
    h = 1e-5
    for _ in range(16):
        idx = tuple(int(rng.integers(0, n)) for n in psi.shape)
        for part in (1.0, 1j):
            pp = psi.copy(); pp[idx] += part * h
            pm = psi.copy(); pm[idx] -= part * h
            fd = (force.action_norm(pp, U, KAPPA, BC) - force.action_norm(pm, U, KAPPA, BC)) / (2 * h)
            an = g[idx].real if part == 1.0 else g[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_raw_link_gradient_finite_differences():
    dims = (4, 4, 4, 4)
    U, psi = LI.workload_fields(10, dims)
    G = force.grad_links_norm(psi, U, KAPPA, BC)
    rng = LI.fd_rng(10)
    h = 1e-5
    picks = [(dims[3] - 1, 0, 0, 0, 3), (0, 0, 0, dims[0] - 1, 0)]
    picks += [tuple(int(rng.integers(0, n)) for n in U.shape[:5]) for _ in range(8)]
    for site_mu in picks:
        i, j = int(rng.integers(0, 3)), int(rng.integers(0, 3))
        idx = site_mu + (i, j)
        for part in (1.0, 1j):
            up = U.copy(); up[idx] += part * h
            um = U.copy(); um[idx] -= part * h
            fd = (force.action_norm(psi, up, KAPPA, BC) - force.action_norm(psi, um, KAPPA, BC)) / (2 * h)
            an = G[idx].real if part == 1.0 else G[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_rows01_gradient_finite_differences():
    """Gradient with respect to the stored rows 0 and 1 of 12-real links
    (the operator applies V = (row0, row1, conj(row0 x row1))) against
    central differences of |M[V] psi|^2 in those entries; the stored row 2 is
    never read, so its gradient is zero.  The rows are generic complex rows,
    not SU(3), so both cross-product terms of the chain rule matter."""
    dims = (4, 4, 4, 4)
    U, psi = LI.workload_fields(17, dims)
    rng = LI.fd_rng(17)
    R = U + 0.3 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))

    def S(rows):
        return force.action_norm(psi, links.reconstruct(rows[..., :2, :]), KAPPA, BC)

    V = links.reconstruct(R[..., :2, :])
    G12 = force.rows01_gradient(force.grad_links_norm(psi, V, KAPPA, BC), R)
    h = 1e-5
    picks = [(dims[3] - 1, 0, 0, 0, 3), (0, 0, 0, dims[0] - 1, 0)]
    picks += [tuple(int(rng.integers(0, n)) for n in R.shape[:5]) for _ in range(8)]
    for site_mu in picks:
        for i in range(3):
            j = int(rng.integers(0, 3))
            idx = site_mu + (i, j)
            for part in (1.0, 1j):
                rp = R.copy(); rp[idx] += part * h
                rm = R.copy(); rm[idx] -= part * h
                fd = (S(rp) - S(rm)) / (2 * h)
                an = G12[idx].real if part == 1.0 else G12[idx].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    assert np.all(G12[..., 2, :] == 0)


def test_su3_force_finite_differences():
    dims = (4, 4, 4, 4)
    U, psi = LI.workload_fields(11, dims)
    F = force.su3_force(force.grad_links_norm(psi, U, KAPPA, BC), U)
    # F is traceless anti-hermitian
    assert np.abs(F + np.conj(np.swapaxes(F, -1, -2))).max() < 1e-13
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-13
    lam = gell_mann()
    rng = LI.fd_rng(11)
    h = 1e-5
    picks = [(dims[3] - 1, 1, 2, 3, 3)] + [tuple(int(rng.integers(0, n)) for n in U.shape[:5])
                                          for _ in range(6)]
    for site_mu in picks:
        a = int(rng.integers(0, 8))
        T = 0.5j * lam[a]
        up = U.copy(); up[site_mu] = expm_ah(T, h) @ U[site_mu]
        um = U.copy(); um[site_mu] = expm_ah(T, -h) @ U[site_mu]
        fd = (force.action_norm(psi, up, KAPPA, BC) - force.action_norm(psi, um, KAPPA, BC)) / (2 * h)
        an = np.trace(T.conj().T @ F[site_mu]).real
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_vjp_with_upstream_gradient():
    dims = (4, 4, 4, 4)
    U, psi = LI.workload_fields(12, dims)
    g = LI.gaussian_spinor(np.random.default_rng(21), dims)
    gpsi, gU = force.vjp(psi, U, KAPPA, g, BC)

    def L(ps, uu):
        return np.vdot(g, dirac.wilson(ps, uu, KAPPA, BC)).real

    rng = LI.fd_rng(12)
    h = 1e-5
    for _ in range(6):
        idx = tuple(int(rng.integers(0, n)) for n in psi.shape)
        pp = psi.copy(); pp[idx] += 1j * h
        pm = psi.copy(); pm[idx] -= 1j * h
        assert abs((L(pp, U) - L(pm, U)) / (2 * h) - gpsi[idx].imag) < 1e-7
        li = tuple(int(rng.integers(0, n)) for n in U.shape)
        up = U.copy(); up[li] += h
        um = U.copy(); um[li] -= h
        assert abs((L(psi, up) - L(psi, um)) / (2 * h) - gU[li].real) < 1e-7


def test_force_gauge_covariance():
    dims = (4, 4, 4, 4)
    U, psi = LI.workload_fields(13, dims)
    om = LI.random_gauge_transform(13, dims)
    F = force.su3_force(force.grad_links_norm(psi, U, KAPPA, BC), U)
    Ug = LI.gauge_transform_links(U, om)
    psig = LI.gauge_transform_spinor(psi, om)
    Fg = force.su3_force(force.grad_links_norm(psig, Ug, KAPPA, BC), Ug)
    want = om[..., None, :, :] @ F @ np.conj(np.swapaxes(om, -1, -2))[..., None, :, :]
    assert rel(Fg, want) < 1e-13


def test_pseudofermion_force_finite_differences():
    dims = (2, 2, 2, 4)
    U, phi = LI.workload_fields(14, dims)
    phi_e = dirac.project(phi, 0)

    def S(uu):
        x, _, _ = solver.solve_normal(phi_e, uu, KAPPA, BC, tol=1e-14, maxiter=5000)
        return np.vdot(phi_e, x).real

    x_e, _, _ = solver.solve_normal(phi_e, U, KAPPA, BC, tol=1e-14, maxiter=5000)
    F = force.pseudofermion_force(x_e, U, KAPPA, BC)
    lam = gell_mann()
    rng = LI.fd_rng(14)
    h = 1e-5
    for _ in range(5):
        site_mu = tuple(int(rng.integers(0, n)) for n in U.shape[:5])
        T = 0.5j * lam[int(rng.integers(0, 8))]
        up = U.copy(); up[site_mu] = expm_ah(T, h) @ U[site_mu]
        um = U.copy(); um[site_mu] = expm_ah(T, -h) @ U[site_mu]
        fd = (S(up) - S(um)) / (2 * h)
        an = np.trace(T.conj().T @ F[site_mu]).real
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


# ----------------------------------------------------------------------------
# link compression and reduced-precision storage
# ----------------------------------------------------------------------------

def test_compression_round_trip_su3_only():
    U, _ = LI.workload_fields(15, (4, 4, 4, 4))
    R = links.reconstruct(links.compress(U))
    assert np.abs(R - U).max() < 1e-15 * 8
    # a U(3) matrix with det != 1 is not reproduced
    q = U[0, 0, 0, 0, 0] * np.exp(0.3j)
    assert np.abs(links.reconstruct(links.compress(q)) - q).max() > 1e-2


def test_fp16_spinor_storage_bounds():
    dims = (4, 4, 4, 4)
    _, psi = LI.workload_fields(16, dims)
    q = links.round_f16_spinor(psi)
    scale = np.maximum(np.abs(psi.real).max(axis=(-1, -2)), np.abs(psi.imag).max(axis=(-1, -2)))
    err = np.maximum(np.abs(q.real - psi.real), np.abs(q.imag - psi.imag)).max(axis=(-1, -2))
    # binary16 has an 11-bit significand: half-ulp of values <= 1 is <= 2^-12
    assert np.all(err <= scale * (2.0 ** -11))


# An FP32 pair (x, s) for which binary16(x * fl32(1/s)) and binary16(x / s)
# differ (found by a seeded search over IEEE arithmetic; the test re-checks it).
F16_X_BITS, F16_S_BITS = 1063116027, 1073232281


def on_site_grid(values, scale):
    """True where value == fl32(h * scale) for the binary16 number h nearest
    value / scale, |h| <= 1: the value lies on the site's scaled binary16 grid."""
    s32 = np.asarray(scale, dtype=np.float32)[..., None, None]
    out = np.ones(values.shape, dtype=bool)
    for part in (values.real, values.imag):
        v32 = part.astype(np.float32)
        h = (v32.astype(np.float64) / s32.astype(np.float64)).astype(np.float16)
        back = (h.astype(np.float32) * s32).astype(np.float32)
        out &= (back == v32) & (np.abs(h.astype(np.float64)) <= 1.0) & (v32.astype(np.float64) == part)
    return out


def test_fp16_spinor_storage_rule():
    """binary16 spinor storage is a reading (the paper has no reduced
    precision): one FP32 scale per site, the largest |real| among all 24 reals
    of the site, and stored = binary16(real x fl32(1/scale)).  Pinned by
    properties that do not reuse the oracle's formula: every stored value lies
    on its site's scaled binary16 grid (a per-spin scale puts the small spins
    elsewhere), the site's largest entry comes back exactly, and for a
    constructed entry the reciprocal multiply and a division round to
    different binary16 numbers."""
    rng = np.random.default_rng(61)
    dims = (2, 2, 2, 4)
    psi = LI.gaussian_spinor(rng, dims)
    psi[..., 0, :] *= 100.0   # spin 0 sets the site scale
    psi[..., 3, :] *= 1e-3    # spin 3 far below it
    q = links.round_f16_spinor(psi)
    re32, im32 = psi.real.astype(np.float32), psi.imag.astype(np.float32)
    scale = np.maximum(np.abs(re32).max(axis=(-1, -2)), np.abs(im32).max(axis=(-1, -2)))
    assert np.all(on_site_grid(q, scale))
    big = np.maximum(np.abs(q.real).max(axis=(-1, -2)), np.abs(q.imag).max(axis=(-1, -2)))
    assert np.array_equal(big, scale.astype(np.float64))
    # multiply by the rounded reciprocal, not divide
    x = np.array([F16_X_BITS], dtype=np.uint32).view(np.float32)[0]
    s = np.array([F16_S_BITS], dtype=np.uint32).view(np.float32)[0]
    mul = np.float16(np.float32(x * np.float32(np.float32(1) / s)))
    div = np.float16(np.float32(x / s))
    assert mul != div
    site = np.zeros((1, 1, 1, 1, 4, 3), dtype=np.complex128)
    site[..., 0, 0] = float(s)
    site[..., 2, 1] = 1j * float(x)
    got = links.round_f16_spinor(site)[0, 0, 0, 0, 2, 1].imag
    assert got == float(np.float32(np.float32(mul) * s))
    assert got != float(np.float32(np.float32(div) * s))


def test_fp16_spinor_parts_agree_with_storage():
    """The (q, s) parts are the stored binary16 values and the site scale of
    the storage rule pinned above: q are binary16 numbers, the site's
    largest |q| is exactly 1, and fl32(q s) is round_f16_spinor."""
    rng = np.random.default_rng(63)
    psi = LI.gaussian_spinor(rng, (2, 2, 2, 4)) * 7.0
    q, sc = links.f16_spinor_parts(psi)
    assert np.array_equal(q.real, q.real.astype(np.float16).astype(np.float64))
    assert np.array_equal(q.imag, q.imag.astype(np.float16).astype(np.float64))
    big = np.maximum(np.abs(q.real).max(axis=(-1, -2)), np.abs(q.imag).max(axis=(-1, -2)))
    assert np.all(big == 1.0)
    back = (q.real * sc[..., None, None]).astype(np.float32) \
        + 1j * (q.imag * sc[..., None, None]).astype(np.float32)
    assert np.array_equal(back, links.round_f16_spinor(psi))


def test_binary16_hop_exact_when_projections_are_representable():
    """With stored values on a coarse grid every projected sum q_a + k q_b is
    a binary16 number, so the rounding of the binary16 hop does nothing and
    it must equal the FP64 hop of q s (a dropped scale, sign or link, or a
    projector applied to the wrong rows, would not)."""
    rng = np.random.default_rng(64)
    dims = (2, 2, 4, 4)
    U, _ = LI.workload_fields(3, dims)
    q = (rng.integers(-8, 9, LI.spinor_shape(dims)) + 1j * rng.integers(-8, 9, LI.spinor_shape(dims))) / 16.0
    sc = rng.uniform(0.5, 4.0, dims[::-1]).astype(np.float32).astype(np.float64)
    for dag in (False, True):
        want = dirac.dhop(q * sc[..., None, None], U, dagger=dag)
        got = dirac.dhop_binary16(q, sc, U, dagger=dag)
        assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))


def test_binary16_hop_rounds_the_projected_half_spinor():
    """Constructed values fix where the binary16 hop rounds: the projected
    sum 1 + 2^-11 is a tie between binary16 neighbours and goes to 1 (ties to
    even); the scale multiplies the rounded value (rounding q s instead gives
    another number at scale 3); the rounding comes before the link (with a
    link phase, rounding the product instead differs); the sum 1 - 2^-11 is a
    binary16 number and stays."""
    dims = (2, 2, 2, 4)
    t0 = 1
    q = np.zeros(LI.spinor_shape(dims), dtype=np.complex128)
    # site y = (0, 0, 0, t0): spin 0 = 1, spin 2 = -2^-11 (colour 0)
    q[t0, 0, 0, 0, 0, 0] = 1.0
    q[t0, 0, 0, 0, 2, 0] = -2.0 ** -11
    sc = np.ones(dims[::-1])
    sc[t0, 0, 0, 0] = 3.0
    U = np.zeros(LI.links_shape(dims), dtype=np.complex128)
    U[...] = np.eye(3)
    theta = 0.3
    phase = np.diag([np.exp(1j * theta), np.exp(-1j * theta), 1.0])
    U[t0 - 1, 0, 0, 0, 3] = phase          # U_t(x), x = y - t
    out = dirac.dhop_binary16(q, sc, U)
    # forward t-hop into x = y - t: (1 - g_t) rows 0 and 2 of y, times U_t(x)
    x0 = out[t0 - 1, 0, 0, 0]
    assert x0[0, 0] == 3.0 * np.exp(1j * theta)     # 3 x binary16(1 + 2^-11) = 3
    assert x0[2, 0] == -3.0 * np.exp(1j * theta)
    exact = dirac.dhop(q * sc[..., None, None], U)[t0 - 1, 0, 0, 0]
    assert exact[0, 0] != x0[0, 0]
    # backward t-hop into y + t: (1 + g_t) row 0 = 1 - 2^-11, representable
    x1 = out[t0 + 1, 0, 0, 0]
    assert x1[0, 0] == 3.0 * (1.0 - 2.0 ** -11)
    # rounding q s (scale first) would give binary16(3 (1 + 2^-11)) = 3 + 2^-9
    assert float(np.float16(3.0 * (1 + 2.0 ** -11))) != 3.0
    # rounding after the link: binary16 of the phase times 1 + 2^-11
    after = complex(np.float16((np.exp(1j * theta) * (1 + 2.0 ** -11)).real),
                    np.float16((np.exp(1j * theta) * (1 + 2.0 ** -11)).imag)) * 3.0
    assert after != x0[0, 0]


def test_binary16_sites_match_field():
    """The site-by-site binary16 hop equals the field version."""
    rng = np.random.default_rng(65)
    dims = (4, 2, 2, 4)
    U, psi = LI.workload_fields(4, dims)
    q, sc = links.f16_spinor_parts(psi)
    Ur = links.reconstruct(links.round_f16_links(links.compress(U)))
    sites = np.stack([rng.integers(0, d, 40) for d in dims], 1)
    for dag in (False, True):
        field = dirac.dhop_binary16(q, sc, Ur, dagger=dag)
        got = dirac.dhop_at_binary16(q, sc, Ur, sites, dagger=dag)
        want = field[sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]]
        assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))


# ----------------------------------------------------------------------------
# generators
# ----------------------------------------------------------------------------

def test_haar_su3_unitary_det_one():
    u = LI.haar_su3(np.random.default_rng(1), 20000)
    assert LI.unitarity_defect(u) < 2e-15
    assert np.abs(LI.det3(u) - 1).max() < 2e-15


def test_haar_su3_moments():
    """Character orthogonality on SU(3): E tr U = 0, E |tr U|^2 = 1, E (tr U)^3 = 1."""
    u = LI.haar_su3(np.random.default_rng(2), 100000)
    tr = np.trace(u, axis1=-2, axis2=-1)
    assert abs(tr.mean()) < 0.01
    assert abs((np.abs(tr) ** 2).mean() - 1.0) < 0.012
    assert abs((tr ** 3).mean() - 1.0) < 0.05


def test_ape_smoothing_raises_plaquette():
    U, _ = LI.workload_fields(17, (4, 4, 4, 4))
    plaq = [LI.average_plaquette(U)]
    for _ in range(4):
        U = LI.ape_smooth(U, steps=1, alpha=0.5)
        plaq.append(LI.average_plaquette(U))
    assert abs(plaq[0]) < 0.05
    assert all(b > a for a, b in zip(plaq, plaq[1:]))
    assert LI.unitarity_defect(U.reshape(-1, 3, 3)) < 1e-14
    assert np.abs(LI.det3(U) - 1).max() < 1e-14


def test_sampled_link_gradient_matches_field():
    dims = (4, 6, 2, 8)
    U, X = LI.workload_fields(18, dims)
    Y = LI.gaussian_spinor(np.random.default_rng(19), dims)
    bc = (1, -1, 1, -1)
    G = force.link_gradient(X, Y, U, 0.7, bc)
    rng = np.random.default_rng(20)
    links = np.stack([rng.integers(0, d, 60) for d in dims] + [rng.integers(0, 4, 60)], 1)
    links[0] = [dims[0] - 1, 0, 0, 0, 0]
    links[1] = [0, dims[1] - 1, 0, dims[3] - 1, 1]
    links[2] = [1, 1, 1, dims[3] - 1, 3]
    got = force.link_gradient_at(X, Y, U, 0.7, links, bc)
    want = G[links[:, 3], links[:, 2], links[:, 1], links[:, 0], links[:, 4]]
    assert np.abs(got - want).max() < 1e-13
    ul = U[links[:, 3], links[:, 2], links[:, 1], links[:, 0], links[:, 4]]
    F = force.su3_force(G, U)[links[:, 3], links[:, 2], links[:, 1], links[:, 0], links[:, 4]]
    assert np.abs(force.su3_force_at(got, ul) - F).max() < 1e-13


# ----------------------------------------------------------------------------
# shifts, the lane permutation of Sec. 3.1, SU(3) products
# ----------------------------------------------------------------------------

def test_cshift_is_the_hop_of_the_free_operator():
    """With unit links, D_hop is the projector-weighted sum of the shifts."""
    dims = (4, 6, 2, 4)
    _, psi = LI.workload_fields(21, dims)
    U = unit_links(dims)
    want = dirac.dhop(psi, U, BC)
    got = sum(dirac.spin_mul(ONE4 - GAMMA[m], dirac.cshift(psi, m, 1, BC)) +
              dirac.spin_mul(ONE4 + GAMMA[m], dirac.cshift(psi, m, -1, BC)) for m in range(4))
    assert np.abs(got - want).max() < 1e-14
    # a shift there and back is the identity (sign squared)
    for m in range(4):
        assert np.array_equal(dirac.cshift(dirac.cshift(psi, m, 1, BC), m, -1, BC), psi)
    # L_mu shifts forward multiply by the boundary sign
    x = psi
    for _ in range(dims[3]):
        x = dirac.cshift(x, 3, 1, BC)
    assert np.array_equal(x, -psi)


def test_split_rotate_pins():
    from oracle.shift import split_rotate
    rng = np.random.default_rng(22)
    v = rng.standard_normal((3, 32))
    # s = 1 is a plain rotation
    for r in range(5):
        assert np.array_equal(split_rotate(v, 1, r), np.roll(v, -r, axis=-1))
    # the definition element by element on one case
    vl, s, r = 32, 4, 3
    w = vl // s
    want = np.array([v[0][(i + r) % w + (i // w) * w] for i in range(vl)])
    assert np.array_equal(split_rotate(v, s, r)[0], want)
    # blocks rotate independently; r = w is the identity; rotations compose
    for s in (1, 2, 4, 8):
        w = 32 // s
        assert np.array_equal(split_rotate(v, s, w), v)
        assert np.array_equal(split_rotate(split_rotate(v, s, 2), s, 3), split_rotate(v, s, 5))
    # complex data stored as (re, im) pairs rotates by 2 r reals
    z = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    reals = z.view(np.float64)
    assert np.array_equal(split_rotate(reals, 4, 2 * 3).view(np.complex128), split_rotate(z, 4, 3))


def _to_lanes(F, n):
    """Full lattice array F (axis k = dimension d-1-k, dimension 0 fastest)
    in the layout of Sec. 3.1: dimension i of length L_i is cut into n_i
    blocks of O_i = L_i / n_i sites; the sites o + b O of one sublattice
    share a vector, lane sum_i b_i stride_i with stride_0 = 1."""
    d = F.ndim
    L = [F.shape[d - 1 - i] for i in range(d)]
    O = [L[i] // n[i] for i in range(d)]
    nl = int(np.prod(n))
    out = np.empty(tuple(O[d - 1 - k] for k in range(d)) + (nl,), dtype=F.dtype)
    for lane in range(nl):
        b, rem = [], lane
        for i in range(d):
            b.append(rem % n[i])
            rem //= n[i]
        idx = tuple(slice(b[d - 1 - k] * O[d - 1 - k], (b[d - 1 - k] + 1) * O[d - 1 - k])
                    for k in range(d))
        out[..., lane] = F[idx]
    return out


@pytest.mark.parametrize("dims,n", [((8, 4), (4, 2)), ((4, 8), (2, 4)), ((8, 8, 8), (4, 4, 4)),
                                    ((4, 8, 8), (2, 4, 4)), ((8, 4, 6), (4, 2, 3))])
def test_split_rotate_is_the_lattice_shift(dims, n):
    """What the lane permutation is for (Sec. 3.1): shifting a lattice stored
    with sublattice vectors.  Shift the full lattice by one site in direction
    mu (np.roll, independent of the oracle), store both fields in the vector
    layout, and compare: away from the sublattice edge a shift copies whole
    vectors; on the edge the vector is the neighbour's vector permuted by
    split_rotate with s = prod_{i>mu} n_i blocks and r = prod_{i<mu} n_i lanes."""
    from oracle.shift import split_rotate
    d = len(dims)
    rng = np.random.default_rng(27)
    F = rng.standard_normal(tuple(dims[d - 1 - k] for k in range(d)))
    Fv = _to_lanes(F, n)
    for mu in range(d):
        axis = d - 1 - mu
        G = np.roll(F, -1, axis=axis)          # G(x) = F(x + mu)
        Gv = _to_lanes(G, n)
        O_mu = dims[mu] // n[mu]
        s = int(np.prod(n[mu + 1:]))
        r = int(np.prod(n[:mu]))
        for o in range(O_mu):
            take = [slice(None)] * d
            take[axis] = o
            got = Gv[tuple(take)]
            if o < O_mu - 1:
                src = [slice(None)] * d
                src[axis] = o + 1
                assert np.array_equal(got, Fv[tuple(src)])
            else:
                src = [slice(None)] * d
                src[axis] = 0
                assert np.array_equal(got, split_rotate(Fv[tuple(src)], s, r))


def test_su3_product_pins():
    U, _ = LI.workload_fields(23, (2, 2, 2, 2))
    V, _ = LI.workload_fields(24, (2, 2, 2, 2))
    W = links.su3_product(U, V)
    # index sum written out on a few links
    for idx in [(0, 0, 0, 0, 0), (1, 1, 0, 1, 3), (0, 1, 1, 0, 2)]:
        u, v = U[idx], V[idx]
        want = np.array([[sum(u[i, k] * v[k, j] for k in range(3)) for j in range(3)] for i in range(3)])
        assert np.abs(W[idx] - want).max() < 1e-15
    # closure in SU(3); U^dag U = 1
    assert LI.unitarity_defect(W.reshape(-1, 3, 3)) < 1e-14
    assert np.abs(LI.det3(W) - 1).max() < 1e-14
    eye = links.su3_product(U, U, adj_u=True)
    assert np.abs(eye - np.eye(3)).max() < 1e-14
    # the second dagger: U U^dag = 1, and U^dag V^dag = (V U)^dag
    assert np.abs(links.su3_product(U, U, adj_v=True) - np.eye(3)).max() < 1e-14
    vu = links.su3_product(V, U)
    both = links.su3_product(U, V, adj_u=True, adj_v=True)
    assert np.abs(both - np.conj(np.swapaxes(vu, -1, -2))).max() < 1e-14


def test_normal_solve_vjp_finite_differences():
    """L = Re(g^dag A(U)^-1 b) differentiated by tight solves on 2^3x4."""
    dims = (2, 2, 2, 4)
    U, b = LI.workload_fields(25, dims)
    b = dirac.project(b, 0)
    g = dirac.project(LI.gaussian_spinor(np.random.default_rng(26), dims), 0)

    def L(uu, bb):
        x, _, _ = solver.solve_normal(bb, uu, KAPPA, BC, tol=1e-14, maxiter=5000)
        return np.vdot(g, x).real

    x, _, _ = solver.solve_normal(b, U, KAPPA, BC, tol=1e-14, maxiter=5000)
    lam, G = force.normal_solve_vjp(x, g, U, KAPPA, BC, tol=1e-14)
    rng = np.random.default_rng(27)
    h = 1e-5
    for _ in range(6):
        idx = tuple(int(rng.integers(0, n)) for n in U.shape)
        for part in (1.0, 1j):
            up = U.copy(); up[idx] += part * h
            um = U.copy(); um[idx] -= part * h
            fd = (L(up, b) - L(um, b)) / (2 * h)
            an = G[idx].real if part == 1.0 else G[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    even = np.argwhere(~LI.parity_mask(dims))
    for k in range(4):
        t, z, y, xx = even[int(rng.integers(0, len(even)))]
        idx = (t, z, y, xx, int(rng.integers(0, 4)), int(rng.integers(0, 3)))
        for part in (1.0, 1j):
            bp = b.copy(); bp[idx] += part * h
            bm = b.copy(); bm[idx] -= part * h
            fd = (L(U, bp) - L(U, bm)) / (2 * h)
            an = lam[idx].real if part == 1.0 else lam[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
