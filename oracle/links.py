"""12-real link compression and reduced-precision storage (oracle).

TEST INFRASTRUCTURE.  A link U in SU(3) is stored by its rows 0 and 1; the
third row follows from unitarity and det U = 1 as row2 = conj(row0 x row1)
(cross product of the two rows).  The reconstruction is exact only on SU(3):
a U(3) matrix with det != 1 comes back rotated by det^*.

Half-precision spinor storage keeps, per site, one FP32 scale equal to the
largest absolute value among the site's 24 reals and the 24 reals times the
FP32 reciprocal of that scale rounded to IEEE binary16; links in half precision are stored as the
binary16 rounding of their (bounded by one) entries.
"""

from __future__ import annotations

import numpy as np


def compress(U: np.ndarray) -> np.ndarray:
    """Rows 0 and 1 of each link (12 reals).

    The paper does not treat link compression; the standard 12-real form of an
    SU(3) matrix (third row from unitarity and det U = 1).
    """
    return U[..., :2, :].copy()


def reconstruct(rows01: np.ndarray) -> np.ndarray:
    """Full 3x3 links from rows 0 and 1: row 2 = conj(row0 x row1).

    The paper does not treat link compression; the standard 12-real form of an
    SU(3) matrix (third row from unitarity and det U = 1).
    """
    a = rows01[..., 0, :]
    b = rows01[..., 1, :]
    c = np.conj(np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                          a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                          a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1))
    return np.concatenate([rows01, c[..., None, :]], axis=-2)


def round_f32(z: np.ndarray) -> np.ndarray:
    """Round a complex128 array to complex64 and back (FP32 storage).

    Storage rounding of the reduced-precision variants; the paper does not
    treat reduced precision.
    """
    return z.astype(np.complex64).astype(np.complex128)


def round_f16_links(z: np.ndarray) -> np.ndarray:
    """Links rounded to IEEE binary16 entry by entry and back.

    Storage rounding of the reduced-precision variants; the paper does not
    treat reduced precision.
    """
    re = z.real.astype(np.float16).astype(np.float64)
    im = z.imag.astype(np.float16).astype(np.float64)
    return re + 1j * im


def round_f16_spinor(psi: np.ndarray) -> np.ndarray:
    """Per-site scaled binary16 storage of a canonical spinor field.

    scale = max |real| over the site's 24 reals (FP32); stored value =
    binary16(real * r) with r = 1/scale rounded to FP32 and the product in
    FP32; the value seen by the arithmetic is stored * scale (FP32).

    Storage rounding of the reduced-precision variants; the paper does not
    treat reduced precision.
    """
    re = psi.real.astype(np.float32)
    im = psi.imag.astype(np.float32)
    scale = np.maximum(np.abs(re).max(axis=(-1, -2)), np.abs(im).max(axis=(-1, -2)))
    safe = np.where(scale > 0, scale, np.float32(1.0))
    r = (np.float32(1.0) / safe).astype(np.float32)[..., None, None]
    safe = safe[..., None, None]
    qre = (re * r).astype(np.float16).astype(np.float32) * safe
    qim = (im * r).astype(np.float16).astype(np.float32) * safe
    return qre.astype(np.float64) + 1j * qim.astype(np.float64)


def f16_spinor_parts(psi: np.ndarray):
    """The two parts of the per-site scaled binary16 storage of a spinor
    field: the stored binary16 values q (as complex128) and the FP32 site
    scale s (float64 array over the sites), by the rule of round_f16_spinor.
    The arithmetic of a binary16 hop starts from q and applies s last.

    Storage rounding of the reduced-precision variants; the paper does not
    treat reduced precision.
    """
    re = psi.real.astype(np.float32)
    im = psi.imag.astype(np.float32)
    scale = np.maximum(np.abs(re).max(axis=(-1, -2)), np.abs(im).max(axis=(-1, -2)))
    safe = np.where(scale > 0, scale, np.float32(1.0))
    r = (np.float32(1.0) / safe).astype(np.float32)[..., None, None]
    qre = (re * r).astype(np.float16).astype(np.float64)
    qim = (im * r).astype(np.float16).astype(np.float64)
    return qre + 1j * qim, safe.astype(np.float64)


def round_half(z: np.ndarray) -> np.ndarray:
    """Each real and imaginary part rounded to the nearest IEEE binary16
    value (ties to even), as complex128.

    Rounding of the reduced-precision variants; the paper does not treat
    reduced precision.
    """
    return z.real.astype(np.float16).astype(np.float64) + 1j * z.imag.astype(np.float16).astype(np.float64)


def su3_product(U: np.ndarray, V: np.ndarray, adj_u: bool = False, adj_v: bool = False) -> np.ndarray:
    """W = op(U) op(V) link by link (op = identity or hermitian conjugate).

    The per-link SU(3) matrix product of Sec. 3.3 (Fig. 4a-c), written with
    the library matrix product.
    """
    a = np.conj(np.swapaxes(U, -1, -2)) if adj_u else U
    b = np.conj(np.swapaxes(V, -1, -2)) if adj_v else V
    return a @ b
