"""MI355X (gfx950) polynomial-filter Floquet diagonalisation.

The computation lives in ``libfloquet.so`` (HIP kernels + C ABI, see
``include/floquet.h``); this package is a thin binding whose functions take
torch tensors for device memory and streams.
"""

from .api import (FloquetOp, arnoldi_eigs_batched, brickwork, circuit, host_schur, kicked_ising,  # noqa: F401
                  paper_parameters, set_graph_capture)
from ._lib import FloquetError, LIB_PATH  # noqa: F401
