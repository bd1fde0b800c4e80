"""Seeded synthetic inputs for the Wilson-Dirac operator.

Both the CPU oracle and the GPU path consume the arrays made here; the module
holds none of the operator's arithmetic (no hopping term, no spin projector,
no link compression).  It provides

* lattice geometry helpers and the canonical array shapes,
* Haar-random SU(3) links (Gram-Schmidt QR of a complex Gaussian 3x3 with the
  positive-diagonal phase fix, then det(Q)^(-1/3) on the principal branch),
* Gaussian spinors (i.i.d. N(0,1) real and imaginary parts),
* APE-like smoothing (Jacobi update of all links with the six staples, then
  the unitary polar factor and the det fix to return to SU(3)),
* random local gauge transformations and the average plaquette.

Canonical layouts, lexicographic site order with x fastest:

* spinor  complex[Lt][Lz][Ly][Lx][4 spin][3 colour]
* links   complex[Lt][Lz][Ly][Lx][4 mu][3 row][3 col], mu = 0,1,2,3 = x,y,z,t

Seed recipe for workload k: ``numpy.random.default_rng(1000 + k)`` draws the
link normals (V,4,3,3,2) first and the spinor normals (V,4,3,2) second; a
random gauge transformation uses seed 2000 + k and the selection of
finite-difference entries 3000 + k.  Lattices too large to draw on the host
are drawn on the device with ``torch.Generator`` seeded with the same number.

The matrix helpers accept numpy arrays or torch tensors (CPU or GPU); numpy
inputs give numpy outputs.
"""

from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import torch

__all__ = [
    "volume", "spinor_shape", "links_shape", "parity_mask",
    "haar_su3", "normals_to_haar", "gaussian_spinor", "workload_fields",
    "workload_fields_device", "ape_smooth", "random_gauge_transform",
    "gauge_transform_links", "gauge_transform_spinor", "average_plaquette",
    "det3", "unitarity_defect", "fd_rng",
]


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def volume(dims: Sequence[int]) -> int:
    lx, ly, lz, lt = dims
    return lx * ly * lz * lt


def spinor_shape(dims: Sequence[int]) -> Tuple[int, ...]:
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx, 4, 3)


def links_shape(dims: Sequence[int]) -> Tuple[int, ...]:
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx, 4, 3, 3)


def parity_mask(dims: Sequence[int]) -> np.ndarray:
    """Boolean array [Lt,Lz,Ly,Lx]: True on odd sites ((x+y+z+t) odd)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly),
                             np.arange(lx), indexing="ij")
    return ((x + y + z + t) % 2) == 1


# ----------------------------------------------------------------------------
# small-matrix helpers (elementwise, batched over leading axes)
# ----------------------------------------------------------------------------

def _as_torch(a):
    if isinstance(a, np.ndarray):
        return torch.from_numpy(a), True
    return a, False


def _back(t, was_numpy):
    return t.numpy() if was_numpy else t


def det3(m):
    """Determinant of a batch of 3x3 matrices (explicit cofactor expansion)."""
    m, was_np = _as_torch(m)
    a = m
    d = (a[..., 0, 0] * (a[..., 1, 1] * a[..., 2, 2] - a[..., 1, 2] * a[..., 2, 1])
         - a[..., 0, 1] * (a[..., 1, 0] * a[..., 2, 2] - a[..., 1, 2] * a[..., 2, 0])
         + a[..., 0, 2] * (a[..., 1, 0] * a[..., 2, 1] - a[..., 1, 1] * a[..., 2, 0]))
    return _back(d, was_np)


def _inv3(a):
    """Inverse of a batch of 3x3 matrices via the adjugate."""
    c00 = a[..., 1, 1] * a[..., 2, 2] - a[..., 1, 2] * a[..., 2, 1]
    c01 = a[..., 1, 2] * a[..., 2, 0] - a[..., 1, 0] * a[..., 2, 2]
    c02 = a[..., 1, 0] * a[..., 2, 1] - a[..., 1, 1] * a[..., 2, 0]
    c10 = a[..., 0, 2] * a[..., 2, 1] - a[..., 0, 1] * a[..., 2, 2]
    c11 = a[..., 0, 0] * a[..., 2, 2] - a[..., 0, 2] * a[..., 2, 0]
    c12 = a[..., 0, 1] * a[..., 2, 0] - a[..., 0, 0] * a[..., 2, 1]
    c20 = a[..., 0, 1] * a[..., 1, 2] - a[..., 0, 2] * a[..., 1, 1]
    c21 = a[..., 0, 2] * a[..., 1, 0] - a[..., 0, 0] * a[..., 1, 2]
    c22 = a[..., 0, 0] * a[..., 1, 1] - a[..., 0, 1] * a[..., 1, 0]
    det = a[..., 0, 0] * c00 + a[..., 0, 1] * c01 + a[..., 0, 2] * c02
    # inverse = adjugate / det, adjugate = transpose of the cofactor matrix
    adj = torch.stack([torch.stack([c00, c10, c20], -1),
                       torch.stack([c01, c11, c21], -1),
                       torch.stack([c02, c12, c22], -1)], -2)
    return adj / det[..., None, None]


def _fix_det(q):
    """Multiply a unitary batch by det^(-1/3) (principal branch) -> SU(3)."""
    d = det3(q)
    phase = torch.exp(-1j * torch.angle(d) / 3.0)
    return q * phase[..., None, None]


def _gram_schmidt_columns(z):
    """Orthonormalise the columns of z (modified Gram-Schmidt, two passes).

    The implied R of z = QR has a positive real diagonal, which is the phase
    convention under which Q is Haar-distributed on U(3) when z is a complex
    Gaussian matrix.
    """
    cols = []
    for j in range(3):
        v = z[..., :, j]
        for _ in range(2):
            for q in cols:
                v = v - (q.conj() * v).sum(-1, keepdim=True) * q
        v = v / torch.linalg.vector_norm(v, dim=-1, keepdim=True)
        cols.append(v)
    return torch.stack(cols, dim=-1)


def normals_to_haar(n):
    """Haar SU(3) matrices from real normals of shape (..., 3, 3, 2)."""
    n, was_np = _as_torch(n)
    z = torch.complex(n[..., 0], n[..., 1])
    u = _fix_det(_gram_schmidt_columns(z))
    return _back(u.contiguous(), was_np)


def haar_su3(rng: np.random.Generator, count: int) -> np.ndarray:
    return normals_to_haar(rng.standard_normal((count, 3, 3, 2)))


def unitarity_defect(u) -> float:
    """max |U^dag U - 1| over a batch."""
    u, _ = _as_torch(u)
    eye = torch.eye(3, dtype=u.dtype, device=u.device)
    return float((u.conj().transpose(-1, -2) @ u - eye).abs().max())


def _polar_unitary(v, iters: int = 40):
    """Unitary polar factor of a batch of invertible 3x3 matrices.

    Scaled Newton iteration X <- (zeta X + (zeta X)^(-dagger)) / 2 with the
    Frobenius-norm scaling; it converges quadratically to the unitary factor W
    of V = W P (the same W as A B^dagger from the SVD V = A S B^dagger).
    """
    x = v
    for _ in range(iters):
        xinv = _inv3(x)
        zeta = torch.sqrt(torch.linalg.matrix_norm(xinv) / torch.linalg.matrix_norm(x))
        zeta = zeta[..., None, None]
        xn = 0.5 * (zeta * x + xinv.conj().transpose(-1, -2) / zeta)
        done = float((xn - x).abs().max()) < 1e-15
        x = xn
        if done:
            break
    return x


# ----------------------------------------------------------------------------
# fields
# ----------------------------------------------------------------------------

def gaussian_spinor(rng: np.random.Generator, dims: Sequence[int]) -> np.ndarray:
    n = rng.standard_normal((volume(dims), 4, 3, 2))
    return (n[..., 0] + 1j * n[..., 1]).reshape(spinor_shape(dims))


def workload_fields(k: int, dims: Sequence[int]):
    """Haar links and a Gaussian spinor for workload number k (host, FP64)."""
    rng = np.random.default_rng(1000 + k)
    v = volume(dims)
    u = normals_to_haar(rng.standard_normal((v, 4, 3, 3, 2))).reshape(links_shape(dims))
    n = rng.standard_normal((v, 4, 3, 2))
    psi = (n[..., 0] + 1j * n[..., 1]).reshape(spinor_shape(dims))
    return np.ascontiguousarray(u), np.ascontiguousarray(psi)


def workload_fields_device(k: int, dims: Sequence[int], device, chunk: int = 1 << 22):
    """Device-drawn Haar links and Gaussian spinor (complex128 torch tensors).

    Used for lattices whose host draw would dominate a run; the numbers come
    from ``torch.Generator(device).manual_seed(1000 + k)``, links first.
    """
    g = torch.Generator(device=device)
    g.manual_seed(1000 + k)
    v = volume(dims)
    u = torch.empty((v * 4, 3, 3), dtype=torch.complex128, device=device)
    for s in range(0, v * 4, chunk):
        e = min(v * 4, s + chunk)
        n = torch.randn((e - s, 3, 3, 2), generator=g, dtype=torch.float64, device=device)
        u[s:e] = normals_to_haar(n)
    n = torch.randn((v, 4, 3, 2), generator=g, dtype=torch.float64, device=device)
    psi = torch.complex(n[..., 0], n[..., 1])
    return u.reshape(links_shape(dims)), psi.reshape(spinor_shape(dims))


def fd_rng(k: int) -> np.random.Generator:
    return np.random.default_rng(3000 + k)


# ----------------------------------------------------------------------------
# smoothing, gauge transformations, plaquette
# ----------------------------------------------------------------------------

def _shift(field, mu: int, s: int):
    """field(x + s*mu_hat) on a periodic lattice (mu axis = 3 - mu)."""
    return torch.roll(field, shifts=-s, dims=3 - mu)


def _dag(a):
    return a.conj().transpose(-1, -2)


def ape_smooth(u, steps: int = 10, alpha: float = 0.5):
    """APE-like smoothing with reprojection to SU(3).

    V_mu(x) = (1-alpha) U_mu(x) + alpha/6 * sum_{nu != mu} [
        U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
      + U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) ],
    all links updated at once from the previous field (gauge field periodic in
    every direction), then V -> W det(W)^(-1/3) with W the unitary polar
    factor of V.
    """
    u, was_np = _as_torch(u)
    for _ in range(steps):
        new = torch.empty_like(u)
        for mu in range(4):
            umu = u[..., mu, :, :]
            acc = torch.zeros_like(umu)
            for nu in range(4):
                if nu == mu:
                    continue
                unu = u[..., nu, :, :]
                upper = unu @ _shift(umu, nu, 1) @ _dag(_shift(unu, mu, 1))
                low = _dag(unu) @ umu @ _shift(unu, mu, 1)
                acc = acc + upper + _shift(low, nu, -1)
            v = (1.0 - alpha) * umu + (alpha / 6.0) * acc
            new[..., mu, :, :] = _fix_det(_polar_unitary(v))
        u = new
    return _back(u.contiguous(), was_np)


def random_gauge_transform(k: int, dims: Sequence[int]) -> np.ndarray:
    """Haar SU(3) matrix per site, shape [Lt,Lz,Ly,Lx,3,3] (seed 2000 + k)."""
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(2000 + k)
    return haar_su3(rng, volume(dims)).reshape((lt, lz, ly, lx, 3, 3))


def gauge_transform_links(u, omega):
    """U_mu(x) -> Omega(x) U_mu(x) Omega(x+mu)^dag."""
    u, was_np = _as_torch(u)
    om, _ = _as_torch(omega)
    out = torch.empty_like(u)
    for mu in range(4):
        out[..., mu, :, :] = om @ u[..., mu, :, :] @ _dag(_shift(om, mu, 1))
    return _back(out, was_np)


def gauge_transform_spinor(psi, omega):
    """psi(x) -> Omega(x) psi(x) (colour rotation of every spin component)."""
    p, was_np = _as_torch(psi)
    om, _ = _as_torch(omega)
    out = torch.einsum("...ab,...sb->...sa", om, p)
    return _back(out.contiguous(), was_np)


def average_plaquette(u) -> float:
    """<Re tr(U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag)> / 3, mu < nu."""
    u, _ = _as_torch(u)
    tot = 0.0
    cnt = 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            umu = u[..., mu, :, :]
            unu = u[..., nu, :, :]
            p = umu @ _shift(unu, mu, 1) @ _dag(_shift(umu, nu, 1)) @ _dag(unu)
            tot += float(torch.diagonal(p, dim1=-2, dim2=-1).sum(-1).real.mean()) / 3.0
            cnt += 1
    return tot / cnt

