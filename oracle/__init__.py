"""Plain CPU FP64 oracle for the Chebyshev/KPM linear-scaling Kubo path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP library
(no kernels, headers, helpers, tables or pre/post-processing); the only
thing both sides see is the seeded input data.

Every function follows one passage of Fan, Vierimaa & Harju, "GPUQT: an
efficient linear-scaling quantum transport code fully implemented on graphics
processing units" (Comput. Phys. Commun.; arXiv:1705.01387), written as the
plain definition or as the algorithm's steps in the paper's order, in
complex128 / float64, with scipy sparse products, scipy's Bessel function and
numpy's pairwise sums as the only library steps.

Pins: every function here is checked against results fixed by the paper or
by mathematics, not by itself (tests/test_oracle_pins.py): exact
diagonalisation, matrix exponentials, FFT closed forms of clean lattices,
Jacobi-Anger, Chebyshev-Gauss quadrature, ballistic identities, finite
differences.
"""
from .operators import operators, position_differences, gershgorin_bound
from .kpm import (chebyshev_moments, chebyshev_series, jackson, kpm_reconstruct, chebyshev_T)
from .transport import (evolution_coefficients, evolve, commutator_evolve,
                        dos_moments, vac_moments, msd_moments, auto_terms)
from .adjoint import moments_gradient, vac_gradient, entry_list, tie_hermitian
from .postprocess import sigma_vac, sigma_msd, transport_lengths

__all__ = [
    "operators", "position_differences", "gershgorin_bound",
    "chebyshev_moments", "chebyshev_series", "jackson", "kpm_reconstruct", "chebyshev_T",
    "evolution_coefficients", "evolve", "commutator_evolve",
    "dos_moments", "vac_moments", "msd_moments", "auto_terms",
    "moments_gradient", "vac_gradient", "entry_list", "tie_hermitian", "sigma_vac", "sigma_msd",
    "transport_lengths",
]
