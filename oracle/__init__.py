"""FP64 CPU oracle for the quantics-MPS acoustic wave step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the solver computes, written from the paper
(Nemeth & Vattay, "Quantum Circuit and Tensor Network Implementation of the 2D
Acoustic Wave Equation").  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import it; the library never calls it, and it shares
no code with the HIP path (it takes its inputs from the separate ``synth``
package, which holds no solver arithmetic).

Modules
-------
fdtd     dense FDTD update (Sec. 2, eq. 2), discrete energy, brute-force operators
circuit  classical simulation of the incrementer / decrementer circuits
         (Sec. 3.1, eq. 5 and Fig. 1)
lcu      statevector simulation of the update of eq. 7 as a linear combination
         of unitaries built from those circuits (Sec. 3.2, eq. 6)
mps      quantics MPS arithmetic: shift MPOs (Sec. 4.2, eqs. 9-15), Laplacian
         MPO sum (eq. 16), diagonal c^2 MPO (Sec. 4.3), sums, Hadamard
         products, TT-SVD and rounding (QR sweep + truncated SVD sweep, Sec. 4.3)
stepper  the MPS time step (eq. 17) with three roundings per step, and a
         dense-detour stepper that computes the same rounded states through
         dense TT-SVDs
mlp, rrf references for the learned truncation rank and the randomized range
         finder (see those modules)

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
closed forms, brute force, invariants or the circuit rule, never against the
HIP path.
"""
