"""MI355X-native Wilson-Dirac hot path (hopping operator, even-odd Schur
operator, mixed-precision CG, fermion force) behind the C ABI of
``include/lqcd.h``, with a thin torch binding and an autograd wrapper.
"""

from .lqcd import (  # noqa: F401
    F64, F32, F16, LINK18, LINK12, EVEN, ODD, FULL,
    LQCDError, Lattice, SpinorField, GaugeField, CGStats,
    new_spinor, new_gauge, pack_spinor, unpack_spinor, pack_gauge, unpack_gauge,
    dslash, wilson, meo, moe, mhat, dot, norm2, axpby, convert,
    cg_workspace, cg_solve, fermion_force, solve_and_force, cshift, split_rotate, su3_mul,
    colour_mul, spin_project, dslash_generic, face_buffer, face_pack, hop_region,
)
from .autograd import NormalSolve, WilsonMatrix, normal_solve, wilson_matrix  # noqa: F401
