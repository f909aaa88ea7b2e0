"""CPU oracle for the time-reversible adaptive-grid split-operator method
(Choi & Vanicek, arXiv:1909.06412), plain FP64 NumPy/SciPy.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the bench's
cpu_baseline leg may import or run anything here.  It shares no code with the HIP
path: its inputs come from the seeded `workloads` module and nowhere else.

Parity status: every function is pinned by a test in tests/test_oracle_*.py
against closed forms, brute-force sums, invariants or numbers printed in the
paper, except where a module header says "parity unpinned".
"""
from .grid import Grid, f_matrix_bruteforce, fourier_q_to_p_bruteforce  # noqa: F401
from . import closed_forms, gradient, potentials, propagate  # noqa: F401
from .propagate import (Wavepacket, from_physical, gaussian, observables, regrid,  # noqa: F401
                        composition, propagate as run, step, stage, T_substep, V_substep,
                        naive_step, autocorrelation, spectrum, state_distance, inner)
