"""The allocation-free inner product lqcd_dot_noalloc against lqcd_dot with
caller workspace, both called through the C ABI.  The two run the same
kernels on the same inputs, so their results agree bit for bit; the
allocation-free call keeps its block partials in the library's static device
array, which the second, smaller call must not read stale values from."""

import ctypes

import numpy as np
import pytest
import torch

import lattice_inputs as LI
import paper_2001_07557_amd as P
from paper_2001_07557_amd import _lib

from .gpu_helpers import dev, host

pytestmark = pytest.mark.gpu


def _fields(dims, prec, subset, seed):
    lat = P.Lattice(dims)
    rng = np.random.default_rng(seed)
    a = P.pack_spinor(lat, dev(LI.gaussian_spinor(rng, dims)).to(
        torch.complex64 if prec == P.F32 else torch.complex128), prec, subset)
    b = P.pack_spinor(lat, dev(LI.gaussian_spinor(rng, dims)).to(
        torch.complex64 if prec == P.F32 else torch.complex128), prec, subset)
    return lat, a, b


def _dot_workspace(lib, lat, subset, a, b, prec):
    ws = torch.empty(lib.lqcd_reduce_workspace_bytes(lat.ref(), subset), dtype=torch.uint8,
                     device="cuda")
    res = (ctypes.c_double * 2)()
    rc = lib.lqcd_dot(lat.ref(), subset, a.ptr, b.ptr, prec, ws.data_ptr(), res,
                      torch.cuda.current_stream().cuda_stream)
    assert rc == 0, lib.lqcd_strerror(rc)
    return complex(res[0], res[1])


def _dot_noalloc(lib, lat, subset, a, b, prec):
    res = (ctypes.c_double * 2)()
    rc = lib.lqcd_dot_noalloc(lat.ref(), subset, a.ptr, b.ptr, prec, res,
                              torch.cuda.current_stream().cuda_stream)
    assert rc == 0, lib.lqcd_strerror(rc)
    return complex(res[0], res[1])


def test_dot_noalloc_matches_workspace_entry_on_consecutive_calls():
    lib = _lib.load()
    # a large full field (4096 reduction blocks), then a small ragged even
    # half (one partly filled block), then the large one again
    cases = [((32, 32, 32, 32), P.F32, P.FULL, 11),
             ((6, 4, 2, 6), P.F64, P.EVEN, 12),
             ((32, 32, 32, 32), P.F32, P.FULL, 11)]
    seen = []
    for dims, prec, subset, seed in cases:
        print(f"noalloc dot: dims {dims} prec {prec} subset {subset}", flush=True)
        lat, a, b = _fields(dims, prec, subset, seed)
        want = _dot_workspace(lib, lat, subset, a, b, prec)
        got = _dot_noalloc(lib, lat, subset, a, b, prec)
        assert got == want, (dims, got, want)
        # and the value itself against the stored inputs summed on the host
        ra, rb = host(P.unpack_spinor(a)), host(P.unpack_spinor(b))
        ref = np.vdot(ra, rb)
        tol = 1e-13 if prec == P.F64 else 2e-6
        assert abs(got - ref) <= tol * np.linalg.norm(ra) * np.linalg.norm(rb)
        seen.append(got)
    assert seen[0] == seen[2]


def test_dot_noalloc_rejects_fields_beyond_its_scratch():
    lib = _lib.load()
    # 64^4 sites in a full field exceed the static scratch by one block;
    # the even half fits
    big = P.Lattice((64, 64, 64, 64))
    res = (ctypes.c_double * 2)()
    fake_a, fake_b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21)
    assert lib.lqcd_dot_noalloc(big.ref(), P.FULL, fake_a, fake_b, P.F32, res, None) == -5
    assert big.half_volume <= 16776960 < big.volume
