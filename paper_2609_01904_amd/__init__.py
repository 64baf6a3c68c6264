"""MI355X quantics-MPS acoustic wave stepper (HIP library + ctypes binding).

The hot path (one time step of eq. 17 of Nemeth & Vattay, with three
compressions) runs in libmpsw.so, built from ``csrc/`` for gfx950; ``mpsw``
is a thin binding of its C ABI (include/mpsw.h).
"""
from . import mpsw  # noqa: F401
