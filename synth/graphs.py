"""Edge-list generators (see package docstring).

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.  Every
function returns ``edges`` as a C-contiguous int64 array of shape (E, 2) with
``edges[:, 0] < edges[:, 1]`` (no self-loops, no duplicates) unless stated
otherwise.
"""

from __future__ import annotations

import math

import numpy as np

DEFAULT_SEED = 20221208


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Bernoulli sampling of a set of M candidate pairs by geometric skipping
# (Batagelj & Brandes 2005): the gaps between successive successes of i.i.d.
# Bernoulli(p) trials are Geometric(p), so the success positions are the
# partial sums of Geometric(p) draws, minus one.
# ---------------------------------------------------------------------------
def _bernoulli_positions(rng, n_candidates: int, p: float) -> np.ndarray:
    if n_candidates <= 0 or p <= 0.0:
        return np.zeros(0, dtype=np.int64)
    if p >= 1.0:
        return np.arange(n_candidates, dtype=np.int64)
    out = []
    pos = -1
    expected = n_candidates * p
    batch = int(expected + 10.0 * math.sqrt(expected) + 64)
    while True:
        gaps = rng.geometric(p, size=batch).astype(np.int64)
        cs = np.cumsum(gaps) + pos
        keep = cs[cs < n_candidates]
        out.append(keep)
        if keep.size < cs.size:
            break
        pos = int(cs[-1])
        batch = max(64, batch // 4)
    return np.concatenate(out)


def _unrank_upper(idx: np.ndarray, n: int):
    """Map row-major ranks of the strict upper triangle of an n x n matrix to
    (i, j) with i < j.  Row i holds n-1-i entries and starts at
    off(i) = i*(2n-i-1)/2."""
    idx = idx.astype(np.int64)
    b = 2.0 * n - 1.0
    i = np.floor((b - np.sqrt(b * b - 8.0 * idx.astype(np.float64))) / 2.0).astype(np.int64)
    i = np.clip(i, 0, n - 2)

    def off(r):
        return r * (2 * n - r - 1) // 2

    # exact integer fix-up of the floating-point estimate
    for _ in range(3):
        too_big = off(i) > idx
        i = np.where(too_big, i - 1, i)
        too_small = off(i + 1) <= idx
        i = np.where(too_small, i + 1, i)
    j = idx - off(i) + i + 1
    return i, j


# ---------------------------------------------------------------------------
# Stochastic block model
# ---------------------------------------------------------------------------
def sbm_block_sizes(n: int, n_blocks: int, uneven: bool, seed: int) -> np.ndarray:
    """Block sizes summing to n.  Equal: floor(n/B) plus one for the first
    n mod B blocks.  Uneven: weights w_i = 1 + U(0,1), n_i = floor(n w_i / sum w),
    remainder to the largest fractional parts (ties to the lower index)."""
    if not uneven:
        sizes = np.full(n_blocks, n // n_blocks, dtype=np.int64)
        sizes[: n % n_blocks] += 1
        return sizes
    rng = _rng(seed)
    w = 1.0 + rng.random(n_blocks)
    exact = n * w / w.sum()
    sizes = np.floor(exact).astype(np.int64)
    rem = n - int(sizes.sum())
    frac = exact - sizes
    order = np.lexsort((np.arange(n_blocks), -frac))
    sizes[order[:rem]] += 1
    return sizes


def sbm(n: int, n_blocks: int, *, p_in=None, p_out=None, d_in=None, d_out=None,
        uneven: bool = False, seed: int = DEFAULT_SEED):
    """Undirected SBM with block-contiguous node numbering.

    Either give the edge probabilities (p_in, p_out) directly, or the expected
    intra- and inter-block degrees (d_in, d_out), in which case
    p_in,r = d_in/(n_r - 1) and p_out = d_out/(n - n/B).

    Returns (edges, labels)."""
    sizes = sbm_block_sizes(n, n_blocks, uneven, seed)
    starts = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    labels = np.repeat(np.arange(n_blocks, dtype=np.int32), sizes)
    rng = _rng(seed + 1)
    parts = []
    for r in range(n_blocks):
        nr = int(sizes[r])
        if nr < 2:
            continue
        pr = p_in if p_in is not None else min(1.0, d_in / (nr - 1))
        pos = _bernoulli_positions(rng, nr * (nr - 1) // 2, pr)
        i, j = _unrank_upper(pos, nr)
        parts.append(np.stack([i + starts[r], j + starts[r]], axis=1))
    po = p_out if p_out is not None else min(1.0, d_out / (n - n / n_blocks))
    # inter-block edges: sample the whole strict upper triangle with p_out and
    # drop intra-block pairs (those are drawn above with their own probability)
    pos = _bernoulli_positions(rng, n * (n - 1) // 2, po)
    i, j = _unrank_upper(pos, n)
    keep = labels[i] != labels[j]
    parts.append(np.stack([i[keep], j[keep]], axis=1))
    edges = np.ascontiguousarray(np.concatenate(parts).astype(np.int64))
    return edges, labels


# ---------------------------------------------------------------------------
# Chung-Lu power law
# ---------------------------------------------------------------------------
def chung_lu_weights(n: int, gamma: float, mean_degree: float, cap: float) -> np.ndarray:
    """Expected-degree sequence w_i = c (i + 1)^(-1/(gamma-1)), capped at `cap`,
    with c chosen (bisection) so that mean(w) = mean_degree.  Hubs first.  The
    bisection stops once an iteration leaves its bracket unchanged: every later
    iteration would repeat it, so c is the bisection's limit."""
    x = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    lo, hi = 0.0, mean_degree * n
    for _ in range(200):
        c = 0.5 * (lo + hi)
        m = np.minimum(c * x, cap).mean()
        nlo, nhi = (c, hi) if m < mean_degree else (lo, c)
        if nlo == lo and nhi == hi:
            break
        lo, hi = nlo, nhi
    return np.minimum(0.5 * (lo + hi) * x, cap)


def _search_threads(cdf: np.ndarray, r: np.ndarray, threads: int = 16) -> np.ndarray:
    """np.searchsorted(cdf, r, side="right") over chunks of r on a thread pool
    (the search releases the interpreter lock); the result is the same array."""
    from concurrent.futures import ThreadPoolExecutor
    out = np.empty(r.shape, dtype=np.int64)
    step = max(1, -(-len(r) // threads))

    def one(a):
        out[a:a + step] = np.searchsorted(cdf, r[a:a + step], side="right")

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, range(0, len(r), step)))
    return out


def chung_lu(n: int, *, gamma: float = 2.1, mean_degree: float = 16.0, cap=None,
             seed: int = DEFAULT_SEED, lcc: bool = True):
    """Chung-Lu graph on expected degrees w (see chung_lu_weights).

    Sampling: draw Poisson(S/2) endpoint pairs i.i.d. with P(u) = w_u / S
    (S = sum w), drop self-loops and merge duplicates, so that pair {u, v} is an
    edge with probability 1 - exp(-w_u w_v / S), which is w_u w_v / S to first
    order (the cap keeps w_u w_v / S <= cap^2 / S).  Optionally keep only the
    largest connected component, relabelled order-preserving (hubs first).

    Returns (edges, n_nodes)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    if cap is None:
        cap = math.sqrt(n)
    w = chung_lu_weights(n, gamma, mean_degree, cap)
    rng = _rng(seed)
    s = float(w.sum())
    n_pairs = int(rng.poisson(s / 2.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = _search_threads(cdf, rng.random(n_pairs))
    v = _search_threads(cdf, rng.random(n_pairs))
    np.minimum(u, n - 1, out=u)
    np.minimum(v, n - 1, out=v)
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * n + hi)
    edges = np.stack([key // n, key % n], axis=1).astype(np.int64)
    if not lcc:
        return np.ascontiguousarray(edges), n
    # the keys are sorted, so the upper-triangle pattern is already in row order
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(edges[:, 0], minlength=n), out=indptr[1:])
    a = csr_matrix((np.ones(len(edges), dtype=np.int8), edges[:, 1].astype(np.int32), indptr), shape=(n, n))
    _, comp = connected_components(a, directed=False)
    big = np.argmax(np.bincount(comp))
    in_lcc = comp == big
    new_id = np.cumsum(in_lcc) - 1
    ek = in_lcc[edges[:, 0]] & in_lcc[edges[:, 1]]
    edges = new_id[edges[ek]].astype(np.int64)
    return np.ascontiguousarray(edges), int(in_lcc.sum())


# ---------------------------------------------------------------------------
# Graphs with closed-form normalized-Laplacian spectra
# ---------------------------------------------------------------------------
def cycle_graph(n: int) -> np.ndarray:
    i = np.arange(n, dtype=np.int64)
    e = np.stack([i, (i + 1) % n], axis=1)
    return np.ascontiguousarray(np.sort(e, axis=1))


def path_graph(n: int) -> np.ndarray:
    i = np.arange(n - 1, dtype=np.int64)
    return np.ascontiguousarray(np.stack([i, i + 1], axis=1))


def complete_graph(n: int) -> np.ndarray:
    i, j = np.triu_indices(n, 1)
    return np.ascontiguousarray(np.stack([i, j], axis=1).astype(np.int64))


def complete_bipartite_graph(p: int, q: int) -> np.ndarray:
    i, j = np.meshgrid(np.arange(p), np.arange(p, p + q), indexing="ij")
    return np.ascontiguousarray(np.stack([i.ravel(), j.ravel()], axis=1).astype(np.int64))


def hypercube_graph(d: int) -> np.ndarray:
    n = 1 << d
    i = np.arange(n, dtype=np.int64)
    parts = []
    for b in range(d):
        j = i ^ (1 << b)
        m = i < j
        parts.append(np.stack([i[m], j[m]], axis=1))
    return np.ascontiguousarray(np.concatenate(parts))


def star_graph(n: int) -> np.ndarray:
    j = np.arange(1, n, dtype=np.int64)
    return np.ascontiguousarray(np.stack([np.zeros_like(j), j], axis=1))


def disjoint_union(graphs):
    """graphs: list of (edges, n).  Returns (edges, n_total)."""
    parts, off = [], 0
    for e, n in graphs:
        parts.append(np.asarray(e, dtype=np.int64).reshape(-1, 2) + off)
        off += n
    edges = np.concatenate(parts) if parts else np.zeros((0, 2), dtype=np.int64)
    return np.ascontiguousarray(edges), off


def relabel(edges: np.ndarray, n: int, seed: int) -> np.ndarray:
    """Apply a seeded random permutation of node ids."""
    perm = _rng(seed).permutation(n).astype(np.int64)
    e = perm[edges]
    return np.ascontiguousarray(np.sort(e, axis=1))


# ---------------------------------------------------------------------------
# The five benchmark workloads (shapes of the paper's Sec. 4 experiments).
# ---------------------------------------------------------------------------
CONFIGS = {
    # SBM 5k, 4 equal blocks, p_in = 0.016, p_out = 0.0008; k = kb = 4, m = 11
    "sbm5k": dict(kind="sbm", n=5000, blocks=4, p_in=0.016, p_out=0.0008, uneven=False,
                  k=4, kb=4, m=11, seed_offset=0),
    # SBM 200k, 32 uneven blocks, d_in = 20, d_out = 4; k = kb = 32, m = 15
    "sbm200k": dict(kind="sbm", n=200_000, blocks=32, d_in=20.0, d_out=4.0, uneven=True,
                    k=32, kb=32, m=15, seed_offset=1),
    # SBM 2M, 64 uneven blocks, d_in = 26, d_out = 4; k = kb = 64, m = 20
    "sbm2m": dict(kind="sbm", n=2_000_000, blocks=64, d_in=26.0, d_out=4.0, uneven=True,
                  k=64, kb=64, m=20, seed_offset=2),
    # held-out SBM 1M, 32 uneven blocks, d_in = 20, d_out = 4; k = kb = 32, m = 15
    "sbm1m": dict(kind="sbm", n=1_000_000, blocks=32, d_in=20.0, d_out=4.0, uneven=True,
                  k=32, kb=32, m=15, seed_offset=3),
    # Chung-Lu 8M, gamma 2.1, mean degree 16, cap sqrt(N), LCC; k = kb = 64, m = 20
    "chunglu8m": dict(kind="chung_lu", n=8_000_000, gamma=2.1, mean_degree=16.0,
                      k=64, kb=64, m=20, seed_offset=4),
}


def make_config_graph(name: str, seed: int = DEFAULT_SEED, n_override=None):
    """Edge list for a named workload.  Returns (edges, n_nodes, cfg); for SBM
    workloads cfg["labels"] holds the planted block of every node."""
    cfg = dict(CONFIGS[name])
    n = int(n_override or cfg["n"])
    s = seed + cfg["seed_offset"]
    if cfg["kind"] == "sbm":
        edges, labels = sbm(n, cfg["blocks"], p_in=cfg.get("p_in"), p_out=cfg.get("p_out"),
                            d_in=cfg.get("d_in"), d_out=cfg.get("d_out"), uneven=cfg["uneven"], seed=s)
        cfg["labels"] = labels
        return edges, n, cfg
    edges, n2 = chung_lu(n, gamma=cfg["gamma"], mean_degree=cfg["mean_degree"], seed=s)
    return edges, n2, cfg
