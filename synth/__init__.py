"""Seeded synthetic inputs shared by the tests, the bench and the oracle.

This module only *generates inputs*: velocity models, source wavelets, initial
fields and random tensor-train cores.  It holds none of the solver's arithmetic
(no FDTD update, no MPO, no rounding), so both the HIP path and the oracle can
take their inputs from here without sharing any of the method.

Paper: Nemeth & Vattay, "Quantum Circuit and Tensor Network Implementation of
the 2D Acoustic Wave Equation".  Grid conventions follow Sec. 2 (N = 2^n points
per axis, spacing dh, lambda = dt/dh) and Sec. 5 (dh = 10 m, dt = 1 ms, source
depth / position as described there).
"""
from .velocity import layered_fault_velocity, layered_fault_velocity_3d, constant_velocity
from .wavelet import ricker, impulse
from .fields import (plane_wave_fields, sine_mode_fields, random_fields, random_mps_cores, wavefront_fields,
                     wavefront_fields_3d)
from .configs import CONFIGS, get_config, batch_shots

__all__ = [
    "layered_fault_velocity", "layered_fault_velocity_3d", "constant_velocity", "ricker", "impulse",
    "plane_wave_fields", "sine_mode_fields", "random_fields", "random_mps_cores", "wavefront_fields",
    "wavefront_fields_3d", "CONFIGS", "batch_shots", "get_config",
]
