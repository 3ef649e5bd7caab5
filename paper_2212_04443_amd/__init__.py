"""Block Chebyshev-Davidson for the smallest eigenpairs of the normalized graph
Laplacian (Pang & Yang, arXiv 2212.04443) on AMD Instinct MI355X.

The compute path is libchebdav.so (HIP, gfx950), declared in include/chebdav.h;
`paper_2212_04443_amd.chebdav` is its thin ctypes binding.
"""

import os

PACKAGE_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PACKAGE_DIR, "libchebdav.so")
