"""GPU parity of the shift, the lane permutation and the SU(3) product."""

import numpy as np
import pytest
import torch

import lattice_inputs as LI
import paper_2001_07557_amd as P
from oracle import dirac, links
from oracle.shift import split_rotate
from tests.gpu_helpers import dev, f32, host, rel, site_rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,bc", [((4, 4, 4, 4), (1, 1, 1, -1)), ((6, 4, 2, 6), (-1, 1, -1, -1)),
                                     ((2, 2, 2, 2), (1, 1, 1, -1))])
@pytest.mark.parametrize("prec", [P.F64, P.F32, P.F16])
def test_cshift_bit_exact(dims, bc, prec):
    lat = P.Lattice(dims, bc)
    _, psi = LI.workload_fields(40, dims)
    src = P.pack_spinor(lat, dev(psi), prec)
    stored = host(P.unpack_spinor(src))  # the values the field holds
    out = P.new_spinor(lat, prec, P.FULL)
    for mu in range(4):
        for d in (1, -1):
            P.cshift(out, src, mu, d)
            assert np.array_equal(host(P.unpack_spinor(out)), dirac.cshift(stored, mu, d, bc))


def test_dslash_composed_from_shifts():
    """The fused hopping kernel equals the sum over directions of projected,
    link-multiplied shifts (shifts on the GPU, products on the host)."""
    dims = (4, 6, 4, 4)
    lat = P.Lattice(dims)
    U, psi = LI.workload_fields(41, dims)
    Uf = P.pack_gauge(lat, dev(U), P.F64, 18)
    src = P.pack_spinor(lat, dev(psi), P.F64)
    fused = P.new_spinor(lat, P.F64, P.FULL)
    P.dslash(fused, src, Uf)
    sh = P.new_spinor(lat, P.F64, P.FULL)
    total = np.zeros_like(psi)
    for mu in range(4):
        P.cshift(sh, src, mu, 1)
        total += dirac.spin_mul(dirac.ONE4 - dirac.GAMMA[mu],
                                dirac.colour_mul(U[..., mu, :, :], host(P.unpack_spinor(sh))))
        # backward: shift U^dag psi by -mu (U^dag psi formed on the host)
        upsi = dirac.colour_mul(dirac.dagger3(U[..., mu, :, :]), psi)
        P.cshift(sh, P.pack_spinor(lat, dev(upsi), P.F64), mu, -1)
        total += dirac.spin_mul(dirac.ONE4 + dirac.GAMMA[mu], host(P.unpack_spinor(sh)))
    assert rel(host(P.unpack_spinor(fused)), total) < 1e-14


@pytest.mark.parametrize("prec", [P.F64, P.F32])
def test_colour_mul_and_spin_project(prec):
    """The two per-site kernels of the generic operator against the
    oracle's colour and spin products."""
    dims = (6, 4, 2, 6)
    lat = P.Lattice(dims, (1, 1, 1, -1))
    U, psi = LI.workload_fields(44, dims)
    tdt = torch.complex64 if prec == P.F32 else torch.complex128
    Ur, pr = (f32(U), f32(psi)) if prec == P.F32 else (U, psi)
    tol = 2e-6 if prec == P.F32 else 1e-15
    Uf = P.pack_gauge(lat, dev(U).to(tdt), prec, 18)
    src = P.pack_spinor(lat, dev(psi).to(tdt), prec)
    out = P.new_spinor(lat, prec, P.FULL)
    for mu in range(4):
        for adj in (False, True):
            P.colour_mul(out, src, Uf, mu, adjoint=adj)
            u = Ur[..., mu, :, :]
            want = dirac.colour_mul(dirac.dagger3(u) if adj else u, pr)
            got = host(P.unpack_spinor(out))
            assert rel(got, want) < tol
            assert site_rel(got, want) < tol
        for sign in (1, -1):
            proj = dirac.ONE4 + sign * dirac.GAMMA[mu]
            # each entry is one addition of two stored values (times units),
            # rounded once to the storage precision
            want = dirac.spin_mul(proj, pr)
            if prec == P.F32:
                want = f32(want)
            P.spin_project(out, src, mu, sign, accumulate=False)
            assert np.array_equal(host(P.unpack_spinor(out)), want)
            P.spin_project(out, src, mu, sign, accumulate=True)
            assert np.array_equal(host(P.unpack_spinor(out)), 2 * want)


@pytest.mark.parametrize("dims,bc", [((4, 4, 4, 4), (1, 1, 1, -1)), ((6, 4, 2, 6), (-1, 1, 1, -1)),
                                     ((2, 2, 2, 2), (1, 1, 1, -1)), ((8, 6, 4, 10), (-1, 1, -1, 1))])
@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F64, 12), (P.F32, 18), (P.F32, 12)])
def test_generic_dslash_vs_oracle(dims, bc, prec, link):
    """D_hop and its adjoint composed on the GPU from shifts, colour
    products and projections (24 launches) against the oracle, and against
    the fused kernel."""
    lat = P.Lattice(dims, bc)
    U, psi = LI.workload_fields(45, dims)
    tdt = torch.complex64 if prec == P.F32 else torch.complex128
    if prec == P.F32:
        Ur, pr, tol = f32(U), f32(psi), 2e-6
        if link == 12:
            Ur = links.reconstruct(links.compress(Ur))
    else:
        Ur, pr, tol = U, psi, 1e-13
    Uf = P.pack_gauge(lat, dev(U).to(tdt), prec, link)
    src = P.pack_spinor(lat, dev(psi).to(tdt), prec)
    out, fused = P.new_spinor(lat, prec, P.FULL), P.new_spinor(lat, prec, P.FULL)
    t1, t2 = P.new_spinor(lat, prec, P.FULL), P.new_spinor(lat, prec, P.FULL)
    for dag in (False, True):
        P.dslash_generic(out, src, Uf, t1, t2, dagger=dag)
        got = host(P.unpack_spinor(out))
        want = dirac.dhop(pr, Ur, bc, dagger=dag)
        assert rel(got, want) < tol
        if prec == P.F32:
            assert site_rel(got, want) < tol
        P.dslash(fused, src, Uf, dagger=dag)
        assert rel(got, host(P.unpack_spinor(fused))) < tol


@pytest.mark.slow
@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F32, 12)])
def test_generic_dslash_32x4_sampled(prec, link):
    """The generic operator at the size the benchmark times it (32^4)
    against the oracle at 256 sampled sites including every corner."""
    from tests.gpu_helpers import DeviceGather
    dims = (32, 32, 32, 32)
    lat = P.Lattice(dims)
    Ud, psid = LI.workload_fields_device(46, dims, "cuda")
    tdt = torch.complex64 if prec == P.F32 else torch.complex128
    tol = 2e-6 if prec == P.F32 else 1e-13
    Uf = P.pack_gauge(lat, Ud.to(tdt), prec, link)
    src = P.pack_spinor(lat, psid.to(tdt), prec)
    out = P.new_spinor(lat, prec, P.FULL)
    t1, t2 = P.new_spinor(lat, prec, P.FULL), P.new_spinor(lat, prec, P.FULL)
    Uc = P.unpack_gauge(Uf)  # the links the kernels apply (row 2 rebuilt)
    pc = P.unpack_spinor(src)
    rng = np.random.default_rng(47)
    corners = np.array([[x, y, z, t] for x in (0, 31) for y in (0, 31) for z in (0, 31)
                        for t in (0, 31)])
    for dag in (False, True):
        P.dslash_generic(out, src, Uf, t1, t2, dagger=dag)
        res = P.unpack_spinor(out)
        sites = np.concatenate([corners, np.stack([rng.integers(0, 32, 240) for _ in dims], 1)])
        want = dirac.dhop_at(DeviceGather(pc), DeviceGather(Uc), sites, dagger=dag)
        got = res[sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]].cpu().numpy()
        assert rel(got, want) < tol
        if prec == P.F32:
            assert site_rel(got, want) < tol


@pytest.mark.parametrize("vl,s,r", [(64, 1, 5), (64, 4, 3), (32, 2, 7), (16, 8, 1), (8, 8, 0),
                                    (256, 4, 9), (48, 3, 5), (2, 1, 1), (1, 1, 3)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.complex128, torch.complex64])
def test_split_rotate(vl, s, r, dtype):
    rng = np.random.default_rng(vl * 100 + s)
    nvec = 37
    x = rng.standard_normal((nvec, vl)) + (1j * rng.standard_normal((nvec, vl)) if dtype.is_complex else 0)
    t = torch.from_numpy(x).to(dtype).cuda()
    out = torch.empty_like(t)
    P.split_rotate(out, t, s, r)
    want = split_rotate(t.cpu().numpy(), s, r)
    assert np.array_equal(out.cpu().numpy(), want)


def test_split_rotate_complex_as_reals():
    """Rotating complex data by r equals rotating its (re, im) reals by 2r."""
    rng = np.random.default_rng(3)
    z = torch.from_numpy(rng.standard_normal((5, 32)) + 1j * rng.standard_normal((5, 32))).cuda()
    oz = torch.empty_like(z)
    P.split_rotate(oz, z, 4, 3)
    re = torch.view_as_real(z).reshape(5, 64).contiguous()
    orr = torch.empty_like(re)
    P.split_rotate(orr, re, 4, 6)
    assert torch.equal(torch.view_as_real(oz).reshape(5, 64), orr)


@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F64, 12), (P.F32, 18), (P.F32, 12)])
@pytest.mark.parametrize("adj", [(False, False), (True, False), (False, True), (True, True)])
def test_su3_product(prec, link, adj):
    dims = (6, 4, 2, 6)
    lat = P.Lattice(dims)
    U, _ = LI.workload_fields(42, dims)
    V, _ = LI.workload_fields(43, dims)
    tdt = torch.complex64 if prec == P.F32 else torch.complex128
    Uf = P.pack_gauge(lat, dev(U).to(tdt), prec, link)
    Vf = P.pack_gauge(lat, dev(V).to(tdt), prec, link)
    Wf = P.new_gauge(lat, prec, link)
    P.su3_mul(Wf, Uf, Vf, *adj)
    Ur = host(P.unpack_gauge(Uf))  # the matrices the kernel multiplies
    Vr = host(P.unpack_gauge(Vf))
    want = links.su3_product(Ur, Vr, *adj)
    got = host(P.unpack_gauge(Wf))
    tol = 1e-14 if prec == P.F64 else 2e-6
    assert rel(got, want) < tol
    if prec == P.F32:
        assert site_rel(got, want, per=9) < tol
    # in place: W may alias U
    P.su3_mul(Uf, Uf, Vf, *adj)
    assert rel(host(P.unpack_gauge(Uf)), want) < tol


@pytest.mark.slow
def test_su3_product_48x3x96_sampled():
    from tests.gpu_helpers import DeviceGather
    dims = (48, 48, 48, 96)
    lat = P.Lattice(dims)
    Ud, _ = LI.workload_fields_device(6, dims, "cuda")
    Vd, _ = LI.workload_fields_device(7, dims, "cuda")
    Uf = P.pack_gauge(lat, Ud.to(torch.complex64), P.F32, 12)
    Vf = P.pack_gauge(lat, Vd.to(torch.complex64), P.F32, 12)
    del Ud, Vd
    Wf = P.new_gauge(lat, P.F32, 12)
    P.su3_mul(Wf, Uf, Vf)
    rng = np.random.default_rng(1)
    idx = tuple(torch.as_tensor(rng.integers(0, n, 512)) for n in (96, 48, 48, 48, 4))
    Ur = P.unpack_gauge(Uf, torch.complex64)[idx].cpu().numpy().astype(np.complex128)
    Vr = P.unpack_gauge(Vf, torch.complex64)[idx].cpu().numpy().astype(np.complex128)
    Wr = P.unpack_gauge(Wf, torch.complex64)[idx].cpu().numpy().astype(np.complex128)
    assert rel(Wr, links.su3_product(Ur, Vr)) < 2e-6
    assert site_rel(Wr, links.su3_product(Ur, Vr), per=9) < 2e-6
