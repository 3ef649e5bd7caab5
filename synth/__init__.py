"""Seeded synthetic graph generators.

This module produces edge lists (int64 arrays of shape (E, 2), 0-based, one
row per undirected edge) and nothing else: it holds none of the eigensolver's
arithmetic, so both the CPU oracle and the GPU path may consume its output.

Generators:
  * stochastic block model (SBM) graphs, the synthetic stand-in for the
    Graph Challenge static SBM graphs the paper clusters (Sec. 4.1, Table 2);
  * Chung-Lu power-law graphs (largest connected component), the stand-in for
    the skewed MAWI / Graph500 matrices of Table 2;
  * graphs whose normalized-Laplacian spectrum has a closed form (cycle, path,
    complete, complete bipartite, hypercube, disjoint unions).
"""

from .graphs import (  # noqa: F401
    sbm,
    sbm_block_sizes,
    chung_lu,
    chung_lu_weights,
    cycle_graph,
    path_graph,
    complete_graph,
    complete_bipartite_graph,
    hypercube_graph,
    star_graph,
    disjoint_union,
    relabel,
    CONFIGS,
    make_config_graph,
)
