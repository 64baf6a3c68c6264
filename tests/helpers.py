"""Shared helpers of the GPU tests.

The c^2 operator the HIP path steps with comes from the oracle whenever a
result is compared with an oracle stepper: the oracle's TT-SVD of the dense c^2
(Sec. 4.3, the velocity field encoded as a diagonal MPO) is loaded through
mpsw_set_velocity_mpo, and the same cores, contracted by the oracle, give the
dense c^2 the oracle steppers multiply by.  The device's own TT-SVD of c^2
(mpsw_set_velocity_dense) is compared with the oracle's separately.
"""
import sys

import numpy as np

from oracle import mps as M
from oracle import stepper as S

ORDER_NAMES = {0: "sequential", 1: "interleaved"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def order_name(ordering):
    return ORDER_NAMES[ordering] if isinstance(ordering, int) else ordering


def oracle_c2(c2, eps_c, ordering=0):
    """(bonds, cores, dense) of the oracle's c^2 operator for the dense field c2
    (cores in the given site order, dense in field layout)."""
    c2 = np.asarray(c2, dtype=np.float64)
    o = order_name(ordering)
    n = int(c2.shape[0]).bit_length() - 1
    ref = S.c2_mps(c2, n, eps_c, o)
    return M.bonds_of(ref), ref, M.from_sites(M.to_dense(ref), n, o, c2.ndim)


def oracle_velocity(st, c2, eps_c, ordering=0):
    """Load the oracle's c^2 operator into the state; returns its dense c^2."""
    bonds, cores, dense = oracle_c2(c2, eps_c, ordering)
    st.set_velocity_mpo(bonds, cores)
    return dense


def cut_is_flagged(ds, step):
    """Whether the oracle stepper flagged a cut (mps.cut_flags) at or before `step`."""
    f = ds.first_flag()
    return f is not None and f <= step
