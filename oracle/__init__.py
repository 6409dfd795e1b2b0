"""CPU oracle for polynomial-filter Floquet diagonalisation (test infrastructure).

This package is the plain, slow, obviously-correct reference that the HIP path
is checked against.  It is *test infrastructure*: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the GPU library (``paper_2102_05054_amd``)
and imports nothing from it; both sides take their inputs from the seeded
generators in ``workloads`` only.

Everything is computed in complex128 / float64 with NumPy (LAPACK ``zgeev`` for
the full eigendecomposition, which is the paper's own full-diagonalisation
baseline).  Where the method reaches an exact result with a plain definition
(U, the geometric sum, the eigenpairs closest to the target), the oracle is that
definition written out.  Each function names the passage of the paper it
follows.

Modules
-------
models        dense U from explicit Kronecker products, and an independent
              per-site / per-gate matrix-free U (kicked Ising, brickwork)
filters       the geometric-sum filter by its definition, its closed forms
eig           full diagonalisation, target selection, Rayleigh quotients and
              residuals
gram_schmidt  classical Gram-Schmidt with one re-orthogonalisation
entanglement  entanglement entropy of a cut and Page's random-state value
"""

from . import models, filters, eig, gram_schmidt, entanglement  # noqa: F401
