"""CPU oracle for the nonequilibrium-DMFT lattice step (Freericks, "Quenching Bloch
oscillations in a strongly correlated material", arXiv:0711.0999).

THIS PACKAGE IS TEST INFRASTRUCTURE.  It is a plain, slow, obviously correct
complex128 implementation of what the GPU path computes, written from the paper's
Section II (Formalism).  Only the test-suite, the smoke entry point and the CPU
baseline leg of the benchmark may import it.  It shares no code with the HIP
library: no kernels, headers, helpers or constant tables.

Modules (each function cites the passage it follows):
  contour     discrete Kadanoff-Baym-Keldysh contour, leftpoint weights and the
              paper's point-split operator M  (eqs. time_discrete,
              integration_weights, the M matrix and eq. det)
  quadrature  Gauss-Hermite nodes for the joint DOS  (eq. joint_dos, Sec. II
              quadrature paragraph)
  green       noninteracting contour Green's function in the field
              (eq. g_contour_non_final2)
  lattice     lattice Dyson equation and rho-weighted sum -> G_loc, current,
              density, zeroth moment  (eqs. dyson, g_loc, current_def)
  impurity    Falicov-Kimball impurity solution and self-energy update
              (eqs. effective_medium, dynamical_mean_field, g_imp_solve)
  dmft        the self-consistency loop  (Sec. II summary paragraph)
  mlp         numpy reference of the warm-start network and its gradients
  sketch      randomized range finder / SVD used for the Sigma sketch

Readings of the paper (where it is silent, garbled or ambiguous) are stated in
the docstrings of the functions that take them.

Parity status: every function here is pinned by a test in tests/test_oracle_*.py
against closed forms, special cases, library routines or brute force, except
where a docstring says "parity unpinned".
"""

from . import contour, quadrature, green, lattice, impurity, dmft  # noqa: F401
