"""CPU oracle for the BOSP linear-response eigensolver (plain FP64 NumPy/SciPy).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference the GPU library is checked against.  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may
import it.  It shares no code with the library (``paper_2506_08355_amd``)
and imports nothing from it; the only module both sides use is ``gen``,
which builds the seeded inputs and holds none of the method's arithmetic.

Modules
  biorth      MGS-Biorth / CGS-Biorth (Section 3.1)
  small_lrep  Cholesky + SVD solution of the projected problem (Section 3.2)
  bosp        the BOSP iteration with batching/moving (Algorithm "BOSP
              algorithm", Sections 3.2-3.3), dense and Casida operators
  exact       exact spectra of the synthetic workloads (pins)
  generalized the generalized LREP with an SPD metric B (eigenvalues by
              reduction to standard form, residuals, B-biorthogonality)
  nullspace   basis of N(K) from a symmetric eigendecomposition, subspace
              distance (principal angles)

Every function is pinned by a CPU test (``pytest -m "not gpu"``) against
values the paper prints, closed forms, or exact identities.
"""
from .biorth import mgs_biorth, cgs_biorth
from .small_lrep import small_lrep, small_lrep_bruteforce, NotSPDError
from .bosp import (DenseOperator, CasidaOperator, bosp_solve, cg_columns,
                   residual_eps, sign_normalise, nullspace_basis, BospResult,
                   NotConvergedError)
from . import exact, generalized, nullspace

__all__ = [
    "mgs_biorth", "cgs_biorth", "small_lrep", "small_lrep_bruteforce",
    "NotSPDError", "DenseOperator", "CasidaOperator", "bosp_solve",
    "cg_columns", "residual_eps", "sign_normalise", "nullspace_basis",
    "BospResult", "NotConvergedError", "exact", "generalized", "nullspace",
]
