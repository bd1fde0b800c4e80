"""Lane permutation of Sec. 3.1 (oracle; test infrastructure).

``split_rotate`` splits a vector of VL lanes into s equal blocks of
w = VL / s lanes and rotates every block left by r lanes:
out[i] = in[(i + r) mod w + (i div w) w].  With s = 1 it is a plain rotation
of the whole vector; for complex data stored as (re, im) pairs the rotation
count is given in reals, i.e. twice the number of complex lanes.
"""

from __future__ import annotations

import numpy as np


def split_rotate(v: np.ndarray, s: int, r: int) -> np.ndarray:
    """Rotate each of the s contiguous blocks of the last axis left by r.

    Sec. 3.1, the lane permutation defined there.
    """
    vl = v.shape[-1]
    if s <= 0 or vl % s:
        raise ValueError("split count must divide the vector length")
    blocks = v.reshape(v.shape[:-1] + (s, vl // s))
    return np.roll(blocks, -r, axis=-1).reshape(v.shape)
