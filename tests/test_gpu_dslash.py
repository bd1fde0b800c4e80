"""GPU parity of the hopping operator against the FP64 oracle.

Bars: FP64 <= 1e-13 and FP32 <= 2e-6 relative (norm-wise over the field);
FP32 is compared with the oracle evaluated on the FP32-rounded inputs and
with the oracle on the FP64 inputs.  binary16 storage is compared with the
oracle's binary16 hop (stored values and site scales of the input, the
projected half-spinor rounded to binary16, rows 0 and 1 of the links rounded
to binary16): the output is itself stored in binary16 with a per-site scale,
so an entry may be off by half a binary16 unit of the site's largest real
part in both its real and imaginary parts, sqrt(2) 2^-12 = 3.5e-4 of the
site's largest entry; bar 5e-4, per site and norm-wise.
"""

import numpy as np
import pytest
import torch

import lattice_inputs as LI
import paper_2001_07557_amd as P
from oracle import dirac, links
from tests.gpu_helpers import dev, f32, host, rel, site_rel

pytestmark = pytest.mark.gpu

KAPPA = 0.124
TOL64 = 1e-13
TOL32 = 2e-6
TOL16 = 5e-4

GEOMS = [
    ((4, 4, 4, 4), (1, 1, 1, -1)),     # the 4^4 single-application workload
    ((2, 2, 2, 2), (1, 1, 1, -1)),     # every neighbour is also the opposite neighbour
    ((6, 4, 2, 6), (1, 1, 1, -1)),     # ragged: 144 sites per parity, 2.25 tiles
    ((8, 6, 4, 10), (-1, 1, -1, 1)),   # anisotropic, other boundary signs
    ((2, 4, 6, 8), (-1, -1, -1, -1)),
]


def fields(k, dims):
    U, psi = LI.workload_fields(k, dims)
    return U, psi


@pytest.mark.parametrize("prec", [P.F64, P.F32, P.F16])
def test_spinor_pack_round_trip(prec):
    dims = (6, 4, 2, 6)
    lat = P.Lattice(dims)
    _, psi = fields(1, dims)
    for subset in (P.EVEN, P.ODD, P.FULL):
        f = P.pack_spinor(lat, dev(psi), prec, subset)
        back = host(P.unpack_spinor(f))
        want = psi if prec == P.F64 else f32(psi) if prec == P.F32 else links.round_f16_spinor(psi)
        if subset != P.FULL:
            want = dirac.project(want, subset)
        assert np.array_equal(back, want)
    if prec == P.F16:
        # the storage rule on a constructed site: scale = the site's largest
        # |real| (spin 0), the entry x stored as binary16(x * fl32(1/scale)),
        # which for this FP32 pair differs from binary16(x / scale)
        x = float(np.array([1063116027], dtype=np.uint32).view(np.float32)[0])
        sc = float(np.array([1073232281], dtype=np.uint32).view(np.float32)[0])
        site = np.zeros(lat.spinor_shape(), dtype=np.complex128)
        site[0, 0, 0, 0, 0, 0] = sc
        site[0, 0, 0, 0, 2, 1] = 1j * x
        back = host(P.unpack_spinor(P.pack_spinor(lat, dev(site), prec, P.FULL)))
        assert np.array_equal(back, links.round_f16_spinor(site))
        mul = np.float32(np.float16(np.float32(np.float32(x) * np.float32(np.float32(1) / np.float32(sc)))))
        assert back[0, 0, 0, 0, 2, 1].imag == float(np.float32(mul * np.float32(sc)))


@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F64, 12), (P.F32, 18), (P.F32, 12), (P.F16, 12)])
def test_gauge_pack_round_trip(prec, link):
    dims = (6, 4, 2, 6)
    lat = P.Lattice(dims)
    U, _ = fields(2, dims)
    back = host(P.unpack_gauge(P.pack_gauge(lat, dev(U), prec, link)))
    if prec == P.F64 and link == 18:
        assert np.array_equal(back, U)
    elif prec == P.F64:
        assert np.abs(back - U).max() < 1e-14
    elif prec == P.F32:
        assert np.abs(back - U).max() < 2e-6
    else:
        assert np.abs(back - U).max() < 3e-3


@pytest.mark.parametrize("dims,bc", GEOMS)
@pytest.mark.parametrize("link", [18, 12])
def test_full_dslash_fp64(dims, bc, link):
    lat = P.Lattice(dims, bc)
    U, psi = fields(3, dims)
    Uf = P.pack_gauge(lat, dev(U), P.F64, link)
    pf = P.pack_spinor(lat, dev(psi), P.F64)
    out = P.new_spinor(lat, P.F64, P.FULL)
    for dag in (False, True):
        P.dslash(out, pf, Uf, 1.0, 0.0, None, dagger=dag)
        assert rel(host(P.unpack_spinor(out)), dirac.dhop(psi, U, bc, dagger=dag)) < TOL64
        P.wilson(out, pf, Uf, KAPPA, dagger=dag)
        assert rel(host(P.unpack_spinor(out)), dirac.wilson(psi, U, KAPPA, bc, dagger=dag)) < TOL64


@pytest.mark.parametrize("dims,bc", GEOMS[:3])
@pytest.mark.parametrize("link", [18, 12])
def test_full_dslash_fp32(dims, bc, link):
    lat = P.Lattice(dims, bc)
    U, psi = fields(4, dims)
    U32, psi32 = f32(U), f32(psi)
    Uf = P.pack_gauge(lat, dev(U).to(torch.complex64), P.F32, link)
    pf = P.pack_spinor(lat, dev(psi).to(torch.complex64), P.F32)
    out = P.new_spinor(lat, P.F32, P.FULL)
    for dag in (False, True):
        P.wilson(out, pf, Uf, KAPPA, dagger=dag)
        got = host(P.unpack_spinor(out))
        want32 = dirac.wilson(psi32, U32, KAPPA, bc, dagger=dag)
        assert rel(got, want32) < TOL32
        assert site_rel(got, want32) < TOL32
        assert rel(got, dirac.wilson(psi, U, KAPPA, bc, dagger=dag)) < TOL32
        # alpha D_hop alone (no y term: on small lattices the spin rows are
        # rebuilt by four waves in parallel)
        P.dslash(out, pf, Uf, alpha=-0.7, dagger=dag)
        want = -0.7 * dirac.dhop(psi32, U32 if link == 18 else links.reconstruct(links.compress(U32)),
                                 bc, dagger=dag)
        got = host(P.unpack_spinor(out))
        assert rel(got, want) < TOL32
        assert site_rel(got, want) < TOL32


class rounded:
    """Sampled reads of a device field with the oracle's storage rounding
    applied to what is gathered (binary16: per-site scale for spinors,
    entries of rows 0 and 1 for links, row 2 rebuilt); other precisions pass
    through.  Both roundings act site by site, so rounding the samples is
    rounding the field."""

    def __init__(self, gather, prec, kind):
        self.g, self.prec, self.kind = gather, prec, kind
        self.shape = gather.shape

    def __getitem__(self, idx):
        v = self.g[idx]
        if self.prec != P.F16:
            return v
        if self.kind == "spinor":
            return links.round_f16_spinor(v)
        return links.reconstruct(links.round_f16_links(links.compress(v)))


class parts16:
    """Sampled reads of a device spinor field as its binary16 storage parts:
    part 0 the stored values, part 1 the site scales (links.f16_spinor_parts,
    which acts site by site)."""

    def __init__(self, gather, part):
        self.g, self.part = gather, part
        self.shape = gather.shape

    def __getitem__(self, idx):
        return links.f16_spinor_parts(self.g[idx])[self.part]


def hop_at(src, Ur, prec, sites, dag):
    """Oracle hop at sampled sites: binary16 storage through the binary16
    hop, the other precisions through the FP64 hop of the rounded fields."""
    from tests.gpu_helpers import DeviceGather
    if prec == P.F16:
        g = DeviceGather(src)
        return dirac.dhop_at_binary16(parts16(g, 0), parts16(g, 1), rounded(DeviceGather(Ur), prec, "links"),
                                      sites, dagger=dag)
    return dirac.dhop_at(DeviceGather(src), DeviceGather(Ur), sites, dagger=dag)


def want_eo(prec, psi, psr, Ur, out_par, dag, bc=dirac.DEFAULT_BC):
    """Oracle D_eo (out_par even) or D_oe of the stored input psi: binary16
    storage through the binary16 hop, the other precisions through the FP64
    hop of the rounded input psr."""
    if prec == P.F16:
        q, sc = links.f16_spinor_parts(psi)
        fn = dirac.meo_binary16 if out_par == P.EVEN else dirac.moe_binary16
        return fn(q, sc, Ur, bc, dagger=dag)
    fn = dirac.meo if out_par == P.EVEN else dirac.moe
    return fn(dirac.project(psr, 1 - out_par), Ur, bc, dagger=dag)


def eo_case(prec, link, dims=(16, 16, 16, 16), k=5):
    """The 16^4 even-odd workload with rounded copies for reduced precision."""
    U, psi = fields(k, dims)
    rng = np.random.default_rng(50 + k)
    y = LI.gaussian_spinor(rng, dims)
    if prec == P.F32:
        Ur, psr, yr = f32(U), f32(psi), f32(y)
        if link == 12:
            Ur = links.reconstruct(links.compress(Ur))
        tdt = torch.complex64
    elif prec == P.F16:
        Ur = links.reconstruct(links.round_f16_links(links.compress(U)))
        psr, yr = links.round_f16_spinor(psi), links.round_f16_spinor(y)
        tdt = torch.complex128
    else:
        Ur, psr, yr = U, psi, y
        tdt = torch.complex128
    return U, psi, y, Ur, psr, yr, tdt


@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F64, 12), (P.F32, 18), (P.F32, 12), (P.F16, 12)])
def test_even_odd_16x4(prec, link):
    dims = (16, 16, 16, 16)
    lat = P.Lattice(dims)
    U, psi, y, Ur, psr, yr, tdt = eo_case(prec, link, dims)
    Uf = P.pack_gauge(lat, dev(U).to(tdt), prec, link)
    tol = {P.F64: TOL64, P.F32: TOL32, P.F16: TOL16}[prec]
    alpha, beta = -KAPPA ** 2, 1.0
    for out_par, fn in ((P.EVEN, P.meo), (P.ODD, P.moe)):
        inp = P.pack_spinor(lat, dev(psi).to(tdt), prec, 1 - out_par)
        yf = P.pack_spinor(lat, dev(y).to(tdt), prec, out_par)
        out = P.new_spinor(lat, prec, out_par)
        for dag in (False, True):
            fn(out, inp, Uf, 1.0, 0.0, None, dagger=dag)
            want = want_eo(prec, psi, psr, Ur, out_par, dag)
            got = host(P.unpack_spinor(out))
            assert rel(got, want) < tol
            if prec != P.F64:
                assert site_rel(got, want) < tol
            fn(out, inp, Uf, alpha, beta, yf, dagger=dag)
            want = alpha * want + beta * dirac.project(yr, out_par)
            got = host(P.unpack_spinor(out))
            assert rel(got, want) < tol
            if prec != P.F64:
                assert site_rel(got, want) < tol


def _split_hop(out, inp, Uf, out_par, alpha, beta, yf, dag, send, recv):
    """The even-odd hop as a t decomposition would run it: pack the faces,
    'exchange' them (a device copy into receive buffers, standing in for the
    transfer to and from the neighbouring domain), interior slices, then the
    boundary slices from the received faces."""
    P.face_pack(send[0], send[1], inp, Uf, out_par, dagger=dag)
    recv[0].copy_(send[0])
    recv[1].copy_(send[1])
    P.hop_region(out, inp, Uf, 0, alpha=alpha, beta=beta, y=yf, dagger=dag)
    P.hop_region(out, inp, Uf, 1, recv[0], recv[1], alpha=alpha, beta=beta, y=yf, dagger=dag)


@pytest.mark.parametrize("dims,bc", [((8, 8, 8, 8), (1, 1, 1, -1)), ((4, 4, 8, 6), (-1, 1, 1, -1)),
                                     ((8, 4, 4, 2), (1, 1, 1, -1)), ((8, 8, 4, 4), (1, -1, 1, 1))])
@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F64, 12), (P.F32, 18), (P.F32, 12), (P.F16, 12)])
def test_t_split_hop_bit_identical(dims, bc, prec, link):
    """Interior plus boundary launches with packed and received t-faces give
    the unsplit even-odd hop bit for bit (both parities, adjoint, with and
    without the alpha D + beta y epilogue) and match the oracle; Lt = 2 has
    no interior."""
    lat = P.Lattice(dims, bc)
    U, psi, y, Ur, psr, yr, tdt = eo_case(prec, link, dims, k=15)
    Uf = P.pack_gauge(lat, dev(U).to(tdt), prec, link)
    tol = {P.F64: TOL64, P.F32: TOL32, P.F16: TOL16}[prec]
    nbytes = lat.spinor_bytes(prec, P.EVEN)
    send = [P.face_buffer(lat, prec), P.face_buffer(lat, prec)]
    recv = [P.face_buffer(lat, prec), P.face_buffer(lat, prec)]
    for out_par, fn in ((P.EVEN, P.meo), (P.ODD, P.moe)):
        inp = P.pack_spinor(lat, dev(psi).to(tdt), prec, 1 - out_par)
        yf = P.pack_spinor(lat, dev(y).to(tdt), prec, out_par)
        ref = P.new_spinor(lat, prec, out_par)
        split = P.new_spinor(lat, prec, out_par)
        for dag in (False, True):
            for alpha, beta, yy in ((1.0, 0.0, None), (-KAPPA ** 2, 1.0, yf)):
                fn(ref, inp, Uf, alpha, beta, yy, dagger=dag)
                split.buf.fill_(0x7f)  # every byte of the result must be written
                _split_hop(split, inp, Uf, out_par, alpha, beta, yy, dag, send, recv)
                torch.cuda.synchronize()
                assert torch.equal(split.buf[:nbytes], ref.buf[:nbytes]), (out_par, dag, alpha)
                want = alpha * want_eo(prec, psi, psr, Ur, out_par, dag, bc)
                if yy is not None:
                    want = want + beta * dirac.project(yr, out_par)
                got = host(P.unpack_spinor(split))
                assert rel(got, want) < tol
                if prec != P.F64:
                    assert site_rel(got, want) < tol


@pytest.mark.slow
@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F32, 12), (P.F16, 12)])
def test_t_split_hop_48x3x12(prec, link):
    """One GPU's share of 48^3x96 split eight ways in t (48^3x12, the size
    the benchmark times the split on): split hop bit-identical to the
    unsplit one, and the oracle at 256 sampled sites of the two boundary
    slices."""
    from tests.gpu_helpers import DeviceGather
    dims = (48, 48, 48, 12)
    lat = P.Lattice(dims)
    Ud, psid = LI.workload_fields_device(16, dims, "cuda")
    tdt = torch.complex64 if prec == P.F32 else torch.complex128
    Uf = P.pack_gauge(lat, Ud.to(tdt), prec, link)
    Uc = P.unpack_gauge(Uf)
    tol = {P.F64: TOL64, P.F32: TOL32, P.F16: TOL16}[prec]
    nbytes = lat.spinor_bytes(prec, P.EVEN)
    send = [P.face_buffer(lat, prec), P.face_buffer(lat, prec)]
    recv = [P.face_buffer(lat, prec), P.face_buffer(lat, prec)]
    rng = np.random.default_rng(17)
    mask = torch.from_numpy(LI.parity_mask(dims)).cuda()
    for out_par, fn in ((P.EVEN, P.meo), (P.ODD, P.moe)):
        inp = P.pack_spinor(lat, psid.to(tdt), prec, 1 - out_par)
        src = P.unpack_spinor(inp)  # the stored input (zero on the other parity)
        ref = P.new_spinor(lat, prec, out_par)
        split = P.new_spinor(lat, prec, out_par)
        for dag in (False, True):
            fn(ref, inp, Uf, dagger=dag)
            split.buf.fill_(0x7f)
            _split_hop(split, inp, Uf, out_par, 1.0, 0.0, None, dag, send, recv)
            torch.cuda.synchronize()
            assert torch.equal(split.buf[:nbytes], ref.buf[:nbytes]), (out_par, dag)
            sites = np.stack([rng.integers(0, d, 1024) for d in dims], 1)
            sites[:, 3] = np.where(rng.integers(0, 2, 1024) == 0, 0, dims[3] - 1)
            sites = sites[sites.sum(1) % 2 == out_par][:256]
            want = hop_at(src, Uc, prec, sites, dag)
            got = P.unpack_spinor(split)[sites[:, 3], sites[:, 2], sites[:, 1],
                                         sites[:, 0]].cpu().numpy()
            assert rel(got, want) < tol
            if prec != P.F64:
                assert site_rel(got, want) < tol
    del mask


@pytest.mark.parametrize("prec,link", [(P.F64, 12), (P.F32, 12)])
def test_schur_operator(prec, link):
    dims = (8, 8, 8, 8)
    lat = P.Lattice(dims)
    U, psi, y, Ur, psr, yr, tdt = eo_case(prec, link, dims, k=6)
    Uf = P.pack_gauge(lat, dev(U).to(tdt), prec, link)
    x = P.pack_spinor(lat, dev(psi).to(tdt), prec, P.EVEN)
    tmp = P.new_spinor(lat, prec, P.ODD)
    out = P.new_spinor(lat, prec, P.EVEN)
    tol = TOL64 if prec == P.F64 else TOL32
    P.mhat(out, x, tmp, Uf, KAPPA)
    want = dirac.mhat(dirac.project(psr, 0), Ur, KAPPA)
    assert rel(host(P.unpack_spinor(out)), want) < tol
    if prec == P.F32:
        assert site_rel(host(P.unpack_spinor(out)), want) < tol
    P.mhat(out, x, tmp, Uf, KAPPA, dagger=True)
    want = dirac.mhat_dag(dirac.project(psr, 0), Ur, KAPPA)
    assert rel(host(P.unpack_spinor(out)), want) < tol
    if prec == P.F32:
        assert site_rel(host(P.unpack_spinor(out)), want) < tol


def test_full_equals_even_odd_blocks():
    dims = (8, 4, 6, 4)
    lat = P.Lattice(dims)
    U, psi = fields(7, dims)
    Uf = P.pack_gauge(lat, dev(U), P.F64, 18)
    full = P.new_spinor(lat, P.F64, P.FULL)
    P.dslash(full, P.pack_spinor(lat, dev(psi), P.F64), Uf)
    e = P.new_spinor(lat, P.F64, P.EVEN)
    o = P.new_spinor(lat, P.F64, P.ODD)
    P.meo(e, P.pack_spinor(lat, dev(psi), P.F64, P.ODD), Uf)
    P.moe(o, P.pack_spinor(lat, dev(psi), P.F64, P.EVEN), Uf)
    t = P.unpack_spinor(e)
    P.unpack_spinor(o, out=t)
    assert np.array_equal(host(t), host(P.unpack_spinor(full)))


def test_adjoint_dot_test_on_gpu():
    dims = (8, 8, 8, 8)
    lat = P.Lattice(dims)
    U, psi = fields(8, dims)
    phi = LI.gaussian_spinor(np.random.default_rng(3), dims)
    Uf = P.pack_gauge(lat, dev(U), P.F64, 12)
    a = P.pack_spinor(lat, dev(psi), P.F64)
    b = P.pack_spinor(lat, dev(phi), P.F64)
    da = P.new_spinor(lat, P.F64, P.FULL)
    db = P.new_spinor(lat, P.F64, P.FULL)
    P.dslash(da, a, Uf)
    P.dslash(db, b, Uf, dagger=True)
    lhs = P.dot(b, da)
    rhs = P.dot(db, a)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_bitwise_deterministic():
    dims = (16, 16, 16, 16)
    lat = P.Lattice(dims)
    U, psi = fields(9, dims)
    Uf = P.pack_gauge(lat, dev(U).to(torch.complex64), P.F32, 12)
    inp = P.pack_spinor(lat, dev(psi).to(torch.complex64), P.F32, P.ODD)
    o1 = P.new_spinor(lat, P.F32, P.EVEN)
    o2 = P.new_spinor(lat, P.F32, P.EVEN)
    P.meo(o1, inp, Uf)
    for _ in range(3):
        P.meo(o2, inp, Uf)
    torch.cuda.synchronize()
    assert torch.equal(o1.buf, o2.buf)


def test_gauge_covariance_on_gpu():
    dims = (4, 6, 4, 8)
    lat = P.Lattice(dims)
    U, psi = fields(10, dims)
    om = LI.random_gauge_transform(10, dims)
    Ug = LI.gauge_transform_links(U, om)
    psig = LI.gauge_transform_spinor(psi, om)
    out = P.new_spinor(lat, P.F64, P.FULL)
    P.dslash(out, P.pack_spinor(lat, dev(psig), P.F64), P.pack_gauge(lat, dev(Ug), P.F64, 12))
    lhs = host(P.unpack_spinor(out))
    P.dslash(out, P.pack_spinor(lat, dev(psi), P.F64), P.pack_gauge(lat, dev(U), P.F64, 12))
    rhs = LI.gauge_transform_spinor(host(P.unpack_spinor(out)), om)
    assert rel(lhs, rhs) < TOL64


def test_hip_graph_replays_match_eager():
    """The even-odd step captured in a HIP graph and replayed several times,
    with eager work and synchronisation in between, gives the eager result
    bit for bit on every replay."""
    dims = (8, 8, 8, 8)
    lat = P.Lattice(dims)
    U, psi = fields(11, dims)
    for prec, link, tdt in ((P.F64, 18, torch.complex128), (P.F32, 12, torch.complex64),
                            (P.F16, 12, torch.complex128)):
        Uf = P.pack_gauge(lat, dev(U).to(tdt), prec, link)
        xo = P.pack_spinor(lat, dev(psi).to(tdt), prec, P.ODD)
        xe = P.pack_spinor(lat, dev(psi).to(tdt), prec, P.EVEN)
        ye = P.new_spinor(lat, prec, P.EVEN)
        yo = P.new_spinor(lat, prec, P.ODD)
        tmp = P.new_spinor(lat, prec, P.ODD)
        me = P.new_spinor(lat, prec, P.EVEN)

        def step():
            P.meo(ye, xo, Uf, -KAPPA, 1.0, xe)
            P.moe(yo, xe, Uf, dagger=True)
            P.mhat(me, xe, tmp, Uf, KAPPA)

        step()
        torch.cuda.synchronize()
        want = [t.buf.clone() for t in (ye, yo, me)]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        for _ in range(3):
            for t in (ye, yo, me):
                t.buf.zero_()
            P.dslash(P.new_spinor(lat, prec, P.FULL), P.pack_spinor(lat, dev(psi).to(tdt), prec),
                     Uf)  # unrelated eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for t, w in zip((ye, yo, me), want):
                assert torch.equal(t.buf, w)


# Large lattices reach the other traversal orders: (32, 32, 36, 16) has whole
# tiles per (z, t) plane but Lz is not a multiple of 8, so four z-slabs are
# shared by the eight XCDs; (24, 24, 24, 24) has 288-site planes, so the
# bricks are made of two-plane groups (nine tiles); (18, 18, 42, 40) has
# 162-site planes and a ragged last tile (V/2 = 272160), so tiles are visited
# in plain order.
@pytest.mark.slow
@pytest.mark.parametrize("dims", [(32, 32, 32, 32), (48, 48, 48, 96), (32, 32, 36, 16),
                                  (18, 18, 42, 40), (24, 24, 24, 24)])
@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F64, 12), (P.F32, 12), (P.F32, 18), (P.F16, 12)])
def test_full_size_sampled(dims, prec, link):
    """Full-size even-odd hops (the launch shapes and traversal orders the
    benchmark times) against the oracle evaluated site by site at 256
    sampled output sites, including every boundary corner of each parity."""
    from tests.gpu_helpers import DeviceGather
    lat = P.Lattice(dims)
    Ud, psid = LI.workload_fields_device(2, dims, "cuda")
    tdt = torch.complex64 if prec == P.F32 else torch.complex128
    if prec == P.F32:
        Ur, pr = Ud.to(tdt).to(torch.complex128), psid.to(tdt).to(torch.complex128)
        tol = TOL32
    elif prec == P.F16:
        Ur, pr, tol = Ud, psid, TOL16
    else:
        Ur, pr, tol = Ud, psid, TOL64
    Uf = P.pack_gauge(lat, Ud.to(tdt), prec, link)
    rng = np.random.default_rng(11)
    for out_par, fn in ((P.EVEN, P.meo), (P.ODD, P.moe)):
        inp = P.pack_spinor(lat, psid.to(tdt), prec, 1 - out_par)
        out = P.new_spinor(lat, prec, out_par)
        mask = torch.from_numpy(LI.parity_mask(dims)).cuda()
        src = pr.clone()
        src[mask if out_par == P.ODD else ~mask] = 0
        for dag in (False, True):
            fn(out, inp, Uf, dagger=dag)
            res = P.unpack_spinor(out)
            sites = np.stack([rng.integers(0, d, 1024) for d in dims], 1)
            corners = np.array([[x, y, z, t] for x in (0, dims[0] - 1) for y in (0, dims[1] - 1)
                                for z in (0, dims[2] - 1) for t in (0, dims[3] - 1)])
            sites = np.concatenate([corners, sites])
            sites = sites[sites.sum(1) % 2 == out_par][:256]
            want = hop_at(src, Ur, prec, sites, dag)
            got = res[sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]].cpu().numpy()
            assert rel(got, want) < tol
            if prec != P.F64:
                assert site_rel(got, want) < tol


@pytest.mark.slow
@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F64, 12), (P.F32, 18), (P.F32, 12), (P.F16, 12)])
def test_every_site_haar_24x4(prec, link):
    """Every output site of the 24^4 even-odd hop (bricks of two-plane
    groups, four z-slabs shared by the eight XCDs) with Haar links against
    the oracle's whole field, per site and norm-wise: D_eo and the adjoint
    D_oe."""
    dims = (24, 24, 24, 24)
    lat = P.Lattice(dims)
    U, psi, y, Ur, psr, yr, tdt = eo_case(prec, link, dims, k=7)
    Uf = P.pack_gauge(lat, dev(U).to(tdt), prec, link)
    tol = {P.F64: TOL64, P.F32: TOL32, P.F16: TOL16}[prec]
    for out_par, fn, dag in ((P.EVEN, P.meo, False), (P.ODD, P.moe, True)):
        inp = P.pack_spinor(lat, dev(psi).to(tdt), prec, 1 - out_par)
        out = P.new_spinor(lat, prec, out_par)
        fn(out, inp, Uf, dagger=dag)
        got = host(P.unpack_spinor(out))
        want = want_eo(prec, psi, psr, Ur, out_par, dag)
        assert rel(got, want) < tol
        assert site_rel(got, want) < max(tol, 1e-12)


@pytest.mark.slow
@pytest.mark.parametrize("dims", [(32, 32, 32, 32), (32, 32, 36, 16), (18, 18, 42, 40),
                                  (24, 24, 24, 24)])
@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F32, 12), (P.F16, 12)])
def test_full_lattice_large_sampled(dims, prec, link):
    """Both-parity D_hop (even and odd tiles paired in one launch, links kept
    cached) and its adjoint on large lattices against the oracle at 256
    sampled sites including every boundary corner."""
    from tests.gpu_helpers import DeviceGather
    lat = P.Lattice(dims)
    Ud, psid = LI.workload_fields_device(6, dims, "cuda")
    tdt = torch.complex64 if prec == P.F32 else torch.complex128
    if prec == P.F32:
        Ur, pr, tol = Ud.to(tdt).to(torch.complex128), psid.to(tdt).to(torch.complex128), TOL32
    elif prec == P.F16:
        Ur, pr, tol = Ud, psid, TOL16
    else:
        Ur, pr, tol = Ud, psid, TOL64
    Uf = P.pack_gauge(lat, Ud.to(tdt), prec, link)
    inp = P.pack_spinor(lat, psid.to(tdt), prec)
    out = P.new_spinor(lat, prec, P.FULL)
    rng = np.random.default_rng(14)
    corners = np.array([[x, y, z, t] for x in (0, dims[0] - 1) for y in (0, dims[1] - 1)
                        for z in (0, dims[2] - 1) for t in (0, dims[3] - 1)])
    for dag in (False, True):
        P.dslash(out, inp, Uf, dagger=dag)
        res = P.unpack_spinor(out)
        sites = np.concatenate([corners, np.stack([rng.integers(0, d, 240) for d in dims], 1)])
        want = hop_at(pr, Ur, prec, sites, dag)
        got = res[sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]].cpu().numpy()
        assert rel(got, want) < tol
        if prec != P.F64:
            assert site_rel(got, want) < tol


@pytest.mark.slow
@pytest.mark.parametrize("dims", [(32, 32, 32, 32), (48, 48, 48, 96), (32, 32, 36, 16)])
@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F64, 12), (P.F32, 18), (P.F32, 12)])
def test_full_lattice_bands_equal_even_odd(dims, prec, link):
    """Both-parity launches whose z-slabs are cut into y-bands (48^3x96: six
    bands in FP64, three in FP32; 32^4: two in FP64; 32x32x36x16, four slabs
    each shared by two XCDs: four in FP64, two in FP32) against the two
    even-odd launches, which walk whole slabs: D_hop, M = 1 - kappa D_hop and
    their adjoints agree bit for bit at every site, so every tile of the
    banded order is visited exactly once."""
    lat = P.Lattice(dims)
    Ud, psid = LI.workload_fields_device(8, dims, "cuda")
    tdt = torch.complex64 if prec == P.F32 else torch.complex128
    Uf = P.pack_gauge(lat, Ud.to(tdt), prec, link)
    del Ud
    full_in = P.pack_spinor(lat, psid.to(tdt), prec)
    ein = P.pack_spinor(lat, psid.to(tdt), prec, P.EVEN)
    oin = P.pack_spinor(lat, psid.to(tdt), prec, P.ODD)
    del psid
    full = P.new_spinor(lat, prec, P.FULL)
    e = P.new_spinor(lat, prec, P.EVEN)
    o = P.new_spinor(lat, prec, P.ODD)
    for dag in (False, True):
        for with_m in (False, True):
            if with_m:
                P.wilson(full, full_in, Uf, KAPPA, dagger=dag)
                P.meo(e, oin, Uf, -KAPPA, 1.0, ein, dagger=dag)
                P.moe(o, ein, Uf, -KAPPA, 1.0, oin, dagger=dag)
            else:
                P.dslash(full, full_in, Uf, dagger=dag)
                P.meo(e, oin, Uf, dagger=dag)
                P.moe(o, ein, Uf, dagger=dag)
            t = P.unpack_spinor(e)
            P.unpack_spinor(o, out=t)
            assert torch.equal(t, P.unpack_spinor(full)), (dag, with_m)
            del t
            torch.cuda.empty_cache()


@pytest.mark.slow
@pytest.mark.parametrize("dims", [(24, 24, 24, 24), (32, 32, 36, 16), (32, 32, 32, 32)])
@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F64, 12), (P.F32, 18), (P.F32, 12)])
def test_plane_wave_every_site(dims, prec, link):
    """Free field (unit links) on a plane wave psi(x) = e^{ip.x} u: D_hop is
    diagonal, D_hop psi = sum_mu [2 cos p_mu - 2i sin p_mu g_mu] psi (+2i for
    the adjoint), with the t momentum shifted by pi/L_t for the antiperiodic
    wrap.  Compared at every output site of the blocked traversals (z-plane
    groups at 24^4, four slabs at 32x32x36x16, eight at 32^4), so a tile
    visited twice or never fails, for the even-odd blocks, their adjoints and
    the both-parity launch."""
    lat = P.Lattice(dims)
    lx, ly, lz, lt = dims
    k = (1, 2, 3, 1)
    p = (2 * np.pi * k[0] / lx, 2 * np.pi * k[1] / ly, 2 * np.pi * k[2] / lz,
         (2 * np.pi * k[3] + np.pi) / lt)
    ct, cz, cy, cx = torch.meshgrid(*[torch.arange(n, device="cuda", dtype=torch.float64)
                                      for n in (lt, lz, ly, lx)], indexing="ij")
    phase = torch.exp(1j * (p[0] * cx + p[1] * cy + p[2] * cz + p[3] * ct))
    rng = np.random.default_rng(21)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = phase[..., None, None] * dev(u)
    tdt = torch.complex64 if prec == P.F32 else torch.complex128
    tol = TOL32 if prec == P.F32 else TOL64
    eye = torch.eye(3, dtype=tdt, device="cuda")
    Uf = P.pack_gauge(lat, eye.expand(lt, lz, ly, lx, 4, 3, 3).contiguous(), prec, link)
    odd = torch.from_numpy(LI.parity_mask(dims)).cuda()
    for dag in (False, True):
        sg = 1.0 if dag else -1.0
        m = sum(2 * np.cos(p[mu]) * np.eye(4) + sg * 2j * np.sin(p[mu]) * dirac.GAMMA[mu]
                for mu in range(4))
        want = phase[..., None, None] * dev(m @ u)
        for out_par, fn in ((P.EVEN, P.meo), (P.ODD, P.moe)):
            inp = P.pack_spinor(lat, psi.to(tdt), prec, 1 - out_par)
            out = P.new_spinor(lat, prec, out_par)
            fn(out, inp, Uf, dagger=dag)
            sel = odd if out_par == P.ODD else ~odd
            got = P.unpack_spinor(out)[sel]
            assert rel(host(got), host(want[sel])) < tol
            if prec == P.F32:
                assert site_rel(host(got), host(want[sel])) < tol
        full_in = P.pack_spinor(lat, psi.to(tdt), prec)
        full_out = P.new_spinor(lat, prec, P.FULL)
        P.dslash(full_out, full_in, Uf, dagger=dag)
        assert rel(host(P.unpack_spinor(full_out)), host(want)) < tol
        if prec == P.F32:
            assert site_rel(host(P.unpack_spinor(full_out)), host(want)) < tol


@pytest.mark.slow
@pytest.mark.parametrize("dims", [(24, 24, 24, 24), (32, 32, 32, 32)])
@pytest.mark.parametrize("prec,link", [(P.F64, 18), (P.F64, 12), (P.F32, 12)])
def test_gamma5_hermiticity_full_size(dims, prec, link):
    """D_hop^dag = g5 D_hop g5 (g5 = diag(1, 1, -1, -1) in the chiral basis)
    and <phi, D psi> = <D^dag phi, psi> at full size, every site, with
    Haar-random links: properties of the operator that hold at any size,
    checked on the blocked traversals of the even-odd and full-lattice
    launches (the adjoint kernel against the forward one)."""
    lat = P.Lattice(dims)
    Ud, psid = LI.workload_fields_device(12, dims, "cuda")
    _, phid = LI.workload_fields_device(13, dims, "cuda")
    tdt = torch.complex64 if prec == P.F32 else torch.complex128
    tol = TOL32 if prec == P.F32 else TOL64
    Uf = P.pack_gauge(lat, Ud.to(tdt), prec, link)
    g5 = torch.tensor([1.0, 1.0, -1.0, -1.0], dtype=tdt, device="cuda")[:, None]
    psi = psid.to(tdt)
    # full lattice
    a = P.pack_spinor(lat, psi, prec)
    a5 = P.pack_spinor(lat, g5 * psi, prec)
    d = P.new_spinor(lat, prec, P.FULL)
    d5 = P.new_spinor(lat, prec, P.FULL)
    P.dslash(d, a, Uf, dagger=True)
    P.dslash(d5, a5, Uf)
    want = g5 * P.unpack_spinor(d5, tdt)
    assert rel(host(P.unpack_spinor(d, tdt)), host(want)) < tol
    b = P.pack_spinor(lat, phid.to(tdt), prec)
    P.dslash(d5, a, Uf)
    P.dslash(d, b, Uf, dagger=True)
    lhs, rhs = P.dot(b, d5), P.dot(d, a)
    assert abs(lhs - rhs) / abs(lhs) < tol
    # even-odd blocks
    for out_par, fn in ((P.EVEN, P.meo), (P.ODD, P.moe)):
        inp = P.pack_spinor(lat, psi, prec, 1 - out_par)
        inp5 = P.pack_spinor(lat, g5 * psi, prec, 1 - out_par)
        o = P.new_spinor(lat, prec, out_par)
        o5 = P.new_spinor(lat, prec, out_par)
        fn(o, inp, Uf, dagger=True)
        fn(o5, inp5, Uf)
        want = g5 * P.unpack_spinor(o5, tdt)
        assert rel(host(P.unpack_spinor(o, tdt)), host(want)) < tol
