"""CPU FP64 correctness oracle for block Chebyshev-Davidson.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the paper's method: the normalized Laplacian of Eq. 1, the
Chebyshev filter of Alg. 3, DGKS orthonormalization (Sec. 2) and the
inner-outer-restart Davidson loop of Alg. 2.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import it; the product library never
does, and the two share no code.  Its single C routine (the sparse apply of A)
is built with gcc into oracle/_build/.

Pins (tests/test_oracle_*.py): CSR against a brute-force dense adjacency; dinv
against exact rational arithmetic; the filter against the closed form
Q p_m(Lambda) Q^T X and cycle-graph Fourier modes; orthonormalization against
its invariants; the solver against dense eigendecomposition and closed-form
spectra (cycle, path, complete, complete bipartite, hypercube); Philox against
its published known-answer vectors; the tall-skinny QR (tsqr.py, Sec. 3.3) against
a hand-worked factorization, LAPACK's QR and the Cholesky factor of X^T X.  Parity unpinned: the dependence threshold
1e-10 of the orthonormalizer (the paper gives none), and iteration counts
(the paper prints none).
"""

from .csr import CSR, build_csr, dense_laplacian  # noqa: F401
from ._lib import apply_laplacian, build, num_threads  # noqa: F401
from .filter import cheb_filter, sigma_schedule  # noqa: F401
from .orth import dgks  # noqa: F401
from .philox import philox4x32_10, random_block  # noqa: F401
from .solve import Params, Result, bchdav, resolve_params  # noqa: F401
