"""Plain FP64 CPU oracle for the Wilson-Dirac hot path.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the package's
``smoke()`` entry and the ``cpu_baseline`` leg of ``bench.py`` may import or
call anything in this package.  The GPU path never routes through it, and it
shares no code with the GPU path: it works on the canonical (lexicographic,
x fastest) arrays with explicit 4x4 gamma matrices and full 3x3 links, in
complex128, with numpy primitives (roll, einsum, matmul) as its only helpers.

The paper (Sec. 3.3, Fig. 4d) times the Wilson Dirac operator but never
writes it down; every definition below is the textbook Wilson hopping term in
the conventions listed in each module, and each function is pinned by the
CPU tests against facts fixed by the mathematics (plane-wave eigenvalues of
the free operator, gamma5-hermiticity, gauge covariance, a dense 2^4 matrix
assembled independently, exact solutions of the free even-odd system,
central finite differences of the action).

Modules:

* ``dirac``  - gamma matrices, D_hop and its adjoint, M = 1 - kappa D_hop,
               even-odd blocks, the Schur operator, per-site sampling.
* ``solver`` - conjugate gradient on the normal even-odd system.
* ``force``  - gradients of |M psi|^2 and the su(3) fermion force.
* ``links``  - 12-real link compression and third-row reconstruction.
* ``shift``  - the lane permutation ``split_rotate`` of Sec. 3.1.
"""

from . import dirac, solver, force, links, shift  # noqa: F401
