"""Host-side checks of the C ABI: the library loads, exports every function
include/lqcd.h declares, and rejects invalid arguments before touching the
GPU.  None of these calls launches a kernel."""

import ctypes
import os
import re

import pytest

from paper_2001_07557_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lqcd.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lqcd_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("liblqcd.so not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_boundary():
    names = header_functions()
    for want in ("lqcd_dslash", "lqcd_dslash_dagger", "lqcd_meo", "lqcd_moe", "lqcd_cg_solve",
                 "lqcd_fermion_force", "lqcd_pack_spinor", "lqcd_pack_gauge"):
        assert want in names


def test_every_declared_symbol_is_exported_and_bound(lib):
    names = header_functions()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding signatures must mirror the header"


def geom(dims, bc=(1, 1, 1, -1)):
    return _lib.GeomT((ctypes.c_int32 * 4)(*dims), (ctypes.c_int32 * 4)(*bc))


def test_version_and_strerror(lib):
    assert lib.lqcd_version() >= 10000
    for code in (0, -1, -2, -3, -4, -5, 7):
        assert isinstance(lib.lqcd_strerror(code), bytes)


def test_sizes(lib):
    g = geom((16, 16, 16, 16))
    vh = 16 ** 4 // 2
    assert lib.lqcd_spinor_bytes(ctypes.byref(g), 0, 0) == vh * 192
    assert lib.lqcd_spinor_bytes(ctypes.byref(g), 1, 2) == 2 * vh * 96
    assert lib.lqcd_spinor_bytes(ctypes.byref(g), 2, 0) == (vh // 64) * (3 * 1024 + 256)
    assert lib.lqcd_gauge_bytes(ctypes.byref(g), 0, 18) == 2 * vh * 4 * 144
    assert lib.lqcd_gauge_bytes(ctypes.byref(g), 1, 12) == 2 * vh * 4 * 48
    assert lib.lqcd_gauge_bytes(ctypes.byref(g), 2, 12) == 2 * vh * 4 * 24
    # ragged last tile rounds up to whole tiles
    g2 = geom((6, 4, 2, 6))
    assert lib.lqcd_spinor_bytes(ctypes.byref(g2), 0, 0) == 3 * 12 * 1024


@pytest.mark.parametrize("dims,bc", [((3, 4, 4, 4), (1, 1, 1, -1)), ((4, 4, 4, 0), (1, 1, 1, -1)),
                                     ((4, 4, 4, 4), (1, 1, 2, -1)), ((1, 4, 4, 4), (1, 1, 1, 1))])
def test_invalid_geometry_rejected(lib, dims, bc):
    g = geom(dims, bc)
    assert lib.lqcd_spinor_bytes(ctypes.byref(g), 0, 2) == 0
    fake = ctypes.c_void_p(4096)
    assert lib.lqcd_dslash(ctypes.byref(g), fake, ctypes.c_void_p(8192), None, ctypes.c_void_p(16384),
                           1.0, 0.0, 0, 18, None) == -1


def test_invalid_arguments_rejected(lib):
    g = geom((4, 4, 4, 4))
    a, b, u = ctypes.c_void_p(4096), ctypes.c_void_p(8192), ctypes.c_void_p(16384)
    # unsupported precision / link combinations
    assert lib.lqcd_gauge_bytes(ctypes.byref(g), 2, 18) == 0
    assert lib.lqcd_meo(ctypes.byref(g), a, b, None, u, 1.0, 0.0, 0, 2, 18, None) == -1
    assert lib.lqcd_meo(ctypes.byref(g), a, b, None, u, 1.0, 0.0, 0, 5, 12, None) == -1
    # NULL, aliasing and misalignment
    assert lib.lqcd_meo(ctypes.byref(g), None, b, None, u, 1.0, 0.0, 0, 0, 18, None) == -1
    assert lib.lqcd_meo(ctypes.byref(g), a, a, None, u, 1.0, 0.0, 0, 0, 18, None) == -1
    assert lib.lqcd_meo(ctypes.byref(g), ctypes.c_void_p(4100), b, None, u, 1.0, 0.0, 0, 0, 18,
                        None) == -1
    # force: F16 not supported, bad mode
    assert lib.lqcd_fermion_force(ctypes.byref(g), a, b, ctypes.c_void_p(12288), u, 1.0, 0, 0, 2,
                                  12, None) == -1
    assert lib.lqcd_fermion_force(ctypes.byref(g), a, b, ctypes.c_void_p(12288), u, 1.0, 3, 0, 0,
                                  18, None) == -1
    # solver: tolerance, maxiter, workspace alignment and size
    st = _lib.CGStatsT()
    ws = ctypes.c_void_p(1 << 20)
    need = lib.lqcd_cg_workspace_bytes(ctypes.byref(g), 1, 12)
    assert need > 0
    assert lib.lqcd_cg_solve(ctypes.byref(g), a, b, u, 18, u, 1, 12, 0.124, 0.0, 100, 100, ws,
                             need, ctypes.byref(st), None) == -1
    assert lib.lqcd_cg_solve(ctypes.byref(g), a, b, u, 18, u, 1, 12, 0.124, 1e-10, 0, 100, ws,
                             need, ctypes.byref(st), None) == -1
    assert lib.lqcd_cg_solve(ctypes.byref(g), a, b, u, 18, u, 1, 12, 0.124, 1e-10, 100, 100,
                             ctypes.c_void_p((1 << 20) + 16), need, ctypes.byref(st), None) == -1
    assert lib.lqcd_cg_solve(ctypes.byref(g), a, b, u, 18, u, 1, 12, 0.124, 1e-10, 100, 100, ws,
                             need - 1, ctypes.byref(st), None) == -5
    assert st.status == -5
    # reductions: NULL result pointer
    assert lib.lqcd_norm2(ctypes.byref(g), 0, a, 0, ws, None, None) == -1
    # allocation-free inner product: NULL operand, and a field larger than its
    # static scratch (64^4 sites, full field) is refused before any HIP call
    res = (ctypes.c_double * 2)()
    assert lib.lqcd_dot_noalloc(ctypes.byref(g), 2, a, None, 0, res, None) == -1
    assert lib.lqcd_dot_noalloc(ctypes.byref(g), 2, a, b, 0, None, None) == -1
    big = geom((64, 64, 64, 64))
    assert lib.lqcd_dot_noalloc(ctypes.byref(big), 2, a, b, 1, res, None) == -5
    # force: mode 2 (rows 0, 1 of 12-real links) needs 12-real links
    assert lib.lqcd_fermion_force(ctypes.byref(g), a, b, ctypes.c_void_p(12288), u, 1.0, 2, 0, 0,
                                  18, None) == -1


def test_product_path_has_no_cpu_fallback():
    """The binding refuses host tensors instead of computing on the CPU."""
    import torch
    import paper_2001_07557_amd as P
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("liblqcd.so not built")
    lat = P.Lattice((4, 4, 4, 4))
    psi = torch.zeros(lat.spinor_shape(), dtype=torch.complex128)
    with pytest.raises(RuntimeError):
        P.pack_spinor(lat, psi, P.F64)


def test_volume_limit_and_empty_vectors(lib):
    # a grid of one thread per site must fit 32 bits: V <= 2^31
    g = geom((1 << 12, 1 << 12, 1 << 8, 2))
    assert lib.lqcd_spinor_bytes(ctypes.byref(g), 0, 2) == 0
    ok = geom((1 << 10, 1 << 10, 1 << 10, 2))  # exactly 2^31 sites
    assert lib.lqcd_spinor_bytes(ctypes.byref(ok), 1, 0) == (1 << 30) * 96
    # split_rotate: s must divide vl; zero vectors is a no-op
    a, b = ctypes.c_void_p(4096), ctypes.c_void_p(8192)
    assert lib.lqcd_split_rotate(a, b, 4, 64, 3, 1, 8, None) == -1
    assert lib.lqcd_split_rotate(a, b, 4, 64, 4, 1, 12, None) == -1
    assert lib.lqcd_split_rotate(a, a, 4, 64, 4, 1, 8, None) == -1
    assert lib.lqcd_split_rotate(a, b, 0, 64, 4, 1, 8, None) == 0
    # cshift: direction and mu ranges
    g4 = geom((4, 4, 4, 4))
    assert lib.lqcd_cshift(ctypes.byref(g4), a, b, 4, 1, 0, None) == -1
    assert lib.lqcd_cshift(ctypes.byref(g4), a, b, 0, 2, 0, None) == -1
    # generic operator and its kernels: FP64 / FP32 only, no aliasing, mu / sign ranges
    t1, t2 = ctypes.c_void_p(12288), ctypes.c_void_p(16384)
    u = ctypes.c_void_p(20480)
    assert lib.lqcd_dslash_generic(ctypes.byref(g4), a, b, u, t1, t2, 0, 2, 12, None) == -1
    assert lib.lqcd_dslash_generic(ctypes.byref(g4), a, b, u, t1, t1, 0, 0, 18, None) == -1
    assert lib.lqcd_dslash_generic(ctypes.byref(g4), a, a, u, t1, t2, 0, 0, 18, None) == -1
    assert lib.lqcd_colour_mul(ctypes.byref(g4), a, b, u, 4, 0, 0, 18, None) == -1
    assert lib.lqcd_spin_project(ctypes.byref(g4), a, b, 0, 2, 0, 0, None) == -1
    assert lib.lqcd_spin_project(ctypes.byref(g4), a, a, 0, 1, 0, 0, None) == -1
    # t decomposition: slices must be whole tiles; region 0 or 1; faces for region 1
    assert lib.lqcd_face_bytes(ctypes.byref(g4), 0) == 0  # 4^4: 32 sites per slice
    g8 = geom((8, 8, 8, 8))
    assert lib.lqcd_face_bytes(ctypes.byref(g8), 0) == 256 * 6 * 16
    assert lib.lqcd_face_bytes(ctypes.byref(g8), 1) == 256 * 6 * 8
    assert lib.lqcd_face_bytes(ctypes.byref(g8), 2) == 256 * 52
    assert lib.lqcd_hop_region(ctypes.byref(g8), 0, 2, a, b, None, u, t1, t2, 1.0, 0.0, 0, 0, 18,
                               None) == -1
    assert lib.lqcd_hop_region(ctypes.byref(g8), 0, 1, a, b, None, u, None, t2, 1.0, 0.0, 0, 0, 18,
                               None) == -1
    assert lib.lqcd_hop_region(ctypes.byref(g4), 0, 0, a, b, None, u, None, None, 1.0, 0.0, 0, 0,
                               18, None) == -1
    assert lib.lqcd_face_pack(ctypes.byref(g8), t1, t1, b, u, 0, 0, 0, 18, None) == -1
    # binary16 hops address a parity's links by 32-bit offsets: V/2 <= 44.7M sites
    g100 = geom((100, 100, 100, 100))
    assert lib.lqcd_meo(ctypes.byref(g100), a, b, None, u, 1.0, 0.0, 0, 2, 12, None) == -1
    assert lib.lqcd_face_pack(ctypes.byref(g100), t1, t2, b, u, 0, 0, 2, 12, None) == -1
    # SU(3) product: binary16 is not a product precision
    assert lib.lqcd_su3_mul(ctypes.byref(g4), a, b, ctypes.c_void_p(12288), 0, 0, 2, 12, None) == -1


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
