"""Oracle: block Chebyshev-Davidson with inner-outer restart (Alg. 2), FP64.

The loop follows Alg. 2 step by step (the step numbers below are the order of
its statements), with Alg. 3 as the filter and DGKS as the orthonormalizer.
Readings of what the paper leaves open or prints inconsistently:

  * ordering: the Ritz values are taken in ascending order everywhere (the
    smallest eigenvalues are wanted, Eq. 2, and the restarts keep the leading
    columns); ties keep their index order;
  * filter interval: cut = low_nwb, upper = upperb = 2, scale point = lowb = 0;
    the first cut is lowb + (upperb - lowb) k_want / N, used as printed;
  * convergence test: ||A v - theta v||_2 <= tol with ||v|| = 1, evaluated from
    the maintained W = A V as W(:, i) - V(:, kc + i) theta_i;
  * any converged pair among the first kb active ones is locked (not only a
    leading run), which is why the locked set is re-sorted;
  * low_nwb = median of the kact retained non-converged Ritz values (mean of the
    two middle ones for an even count); if that median is not strictly inside
    (lowb, upperb) the previous cut is kept;
  * k_ri = max(floor(act_max/2), act_max - 3 kb), k_ro = dim_max - 2 kb - kc,
    act_max = max(5 kb, 30), dim_max = max(act_max + 2 kb, k_want + 30)
    (Sec. 2, Sec. 4);
  * "symmetrize H": the new columns are mirrored into the rows and the new
    kb x kb diagonal block is replaced by (C + C^T)/2;
  * missing vectors (no or too few start vectors, V_init exhausted, fewer than
    kb - e_c active Ritz vectors) are filled with Philox columns numbered in the
    order they are drawn;
  * itmax defaults to 1000; the k_want smallest locked pairs are returned;
  * exit certificate (Table 1 counts an extra SpMM for the residuals): once
    k_want pairs are locked, ||A v - lambda v||_2 of the k_want smallest is
    recomputed from a fresh product with A.  Pairs above certify_tol (default
    tol) are un-locked, the smallest kb first, together with the locked pairs
    above rank k_want - 1 (so that the loop goes on); they lead the next block
    to filter, ahead of V_init columns and Ritz vectors.  After refine_sweeps
    such rounds (default 3) a failing certificate ends the run unconverged;
  * an outer restart keeps dim_max - 2 kb - kc columns, or k_ro if that is
    smaller and positive.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from ._lib import apply_laplacian
from .filter import cheb_filter
from .orth import dgks
from .philox import random_block


@dataclass
class Params:
    k_want: int
    kb: int
    m: int
    tol: float = 1e-8
    itmax: int = 1000
    act_max: int = 0
    dim_max: int = 0
    k_ri: int = 0
    upperb: float = 2.0
    lowb: float = 0.0
    low_nwb0: float | None = None
    seed: int = 0
    k_ro: int = 0
    refine_sweeps: int = 0
    certify_tol: float = 0.0


@dataclass
class Result:
    evals: np.ndarray
    evecs: np.ndarray
    converged: int
    iterations: int
    n_spmm_filter: int
    n_spmm_other: int
    n_random: int
    max_residual: float
    history: list = field(default_factory=list)
    certified: int = 0
    n_unlocked: int = 0
    status: str = "ok"


def resolve_params(p: Params, n: int) -> Params:
    q = Params(**p.__dict__)
    if q.act_max <= 0:
        q.act_max = max(5 * q.kb, 30)
    if q.dim_max <= 0:
        q.dim_max = max(q.act_max + 2 * q.kb, q.k_want + 30)
    if q.k_ri <= 0:
        q.k_ri = max(q.act_max // 2, q.act_max - 3 * q.kb)
    if q.low_nwb0 is None:
        q.low_nwb0 = q.lowb + (q.upperb - q.lowb) * q.k_want / n
    if q.refine_sweeps == 0:
        q.refine_sweeps = 3
    q.refine_sweeps = max(0, q.refine_sweeps)
    if q.certify_tol <= 0:
        q.certify_tol = q.tol
    if not (1 <= q.kb and 1 <= q.k_want <= n and q.m >= 1):
        raise ValueError("need kb >= 1, 1 <= k_want <= n, m >= 1")
    if not (1 <= q.k_ri <= q.act_max - q.kb):
        raise ValueError("need 1 <= k_ri <= act_max - kb")
    if q.dim_max < q.k_want + 2 * q.kb + 1 or q.dim_max < q.act_max:
        raise ValueError("need dim_max >= max(k_want + 2 kb + 1, act_max)")
    if q.dim_max > n:
        raise ValueError("dim_max must not exceed n")
    return q


def _median(x: np.ndarray) -> float:
    s = np.sort(x)
    h = len(s) // 2
    return float(s[h]) if len(s) % 2 else 0.5 * (float(s[h - 1]) + float(s[h]))


def bchdav(csr, params: Params, V_init: np.ndarray | None = None) -> Result:
    n = csr.n
    p = resolve_params(params, n)
    kb, m = p.kb, p.m
    k_init = 0 if V_init is None else V_init.shape[1]
    next_rand = 0
    n_random = 0

    def rand_cols(count):
        nonlocal next_rand, n_random
        blk = random_block(p.seed, n, np.arange(next_rand, next_rand + count))
        next_rand += count
        n_random += count
        return blk

    V = np.zeros((n, p.dim_max), order="F")
    W = np.zeros((n, p.act_max), order="F")
    H = np.zeros((p.act_max, p.act_max))
    # steps 1-3
    upperb, lowb, low_nwb = p.upperb, p.lowb, p.low_nwb0
    take = min(kb, k_init)
    parts = []
    if take:
        parts.append(np.asarray(V_init[:, :take], dtype=np.float64))
    if take < kb:
        parts.append(rand_cols(kb - take))
    V_tmp = np.asfortranarray(np.concatenate(parts, axis=1))
    k_i = kb
    kc = ksub = kact = 0
    evals = np.zeros(0)
    it = 0
    n_filter = n_other = 0
    history = []
    cert_rounds = 0
    n_unlocked = 0
    status = "noconv"
    cert = None  # fresh residuals of the last certificate
    while it < p.itmax:
        it += 1
        # step 5: filter
        V[:, ksub:ksub + kb] = cheb_filter(csr, V_tmp, m, low_nwb, upperb, lowb)
        n_filter += m
        # step 6: orthonormalize against V(:, 1:ksub)
        Q, nrep, next_rand = dgks(V[:, :ksub], V[:, ksub:ksub + kb], p.seed, next_rand)
        n_random += nrep
        V[:, ksub:ksub + kb] = Q
        # step 7
        W[:, kact:kact + kb] = apply_laplacian(csr, np.asfortranarray(V[:, ksub:ksub + kb]))
        n_other += 1
        kact += kb
        ksub += kb
        # step 8: last kb columns of H, symmetrized
        C = V[:, kc:ksub].T @ W[:, kact - kb:kact]
        H[:kact, kact - kb:kact] = C
        H[kact - kb:kact, :kact - kb] = C[:kact - kb, :].T
        blk = C[kact - kb:kact, :]
        H[kact - kb:kact, kact - kb:kact] = 0.5 * (blk + blk.T)
        # step 9: eigen-decomposition, ascending (stable for ties)
        D, Y = np.linalg.eigh(H[:kact, :kact])
        order = np.argsort(D, kind="stable")
        D, Y = D[order], Y[:, order]
        kold = kact
        # step 10: inner restart
        inner = kact + kb > p.act_max
        if inner:
            kact = p.k_ri
            ksub = kc + kact
        # step 11: subspace rotation
        V[:, kc:kc + kact] = V[:, kc:kc + kold] @ Y[:, :kact]
        W[:, :kact] = W[:, :kold] @ Y[:, :kact]
        D = D[:kact].copy()
        # step 12: residuals of the first kb active pairs; lock the converged ones
        nres = min(kb, kact)
        R = W[:, :nres] - V[:, kc:kc + nres] * D[:nres]
        res = np.sqrt(np.sum(R * R, axis=0))
        conv = res <= p.tol
        ec = int(conv.sum())
        history.append(dict(iteration=it, kc=kc, kact=kact, ksub=ksub, low_nwb=low_nwb,
                            res=res.copy(), ritz=D.copy(), ec=ec, inner_restart=inner,
                            outer_restart=False, n_unlocked=0))
        if ec:
            conv_idx = np.nonzero(conv)[0]
            rest = np.array([i for i in range(kact) if not (i < nres and conv[i])], dtype=np.int64)
            perm = np.concatenate([conv_idx, rest]).astype(np.int64)
            V[:, kc:kc + kact] = V[:, kc + perm]
            W[:, :kact] = W[:, perm]
            D = D[perm]
            evals = np.concatenate([evals, D[:ec]])
            srt = np.argsort(evals, kind="stable")
            evals = evals[srt]
            V[:, :kc + ec] = V[:, srt]
            kc += ec
        # step 13, with the exit certificate
        unlocked = np.zeros((n, 0))
        if kc >= p.k_want:
            Vk = np.asfortranarray(V[:, :p.k_want])
            Rk = apply_laplacian(csr, Vk) - Vk * evals[:p.k_want]
            cert = np.sqrt(np.sum(Rk * Rk, axis=0))
            n_other += 1
            bad = [t for t in range(p.k_want) if not cert[t] <= p.certify_tol][:kb]
            if not bad:
                status = "ok"
                break
            if cert_rounds >= p.refine_sweeps:
                status = "certificate"
                break
            cert_rounds += 1
            out = set(bad)
            for t in range(kc - 1, -1, -1):  # the largest locked pairs, until kc < k_want
                if kc - len(out) < p.k_want:
                    break
                out.add(t)
            out = sorted(out)
            keep = [t for t in range(kc) if t not in out]
            nu = len(out)
            unlocked = V[:, out].copy()
            nact = kact - ec  # the retained active columns follow the locked ones
            V[:, :kc - nu + nact] = V[:, keep + list(range(kc, kc + nact))]
            evals = evals[keep]
            kc -= nu
            ksub -= nu
            n_unlocked += nu
            history[-1]["n_unlocked"] = nu
        # step 14
        if ec:
            W[:, :kact - ec] = W[:, ec:kact]
            kact -= ec
        # step 15
        D_act = D[ec:ec + kact]
        H[:, :] = 0.0
        H[np.arange(kact), np.arange(kact)] = D_act
        # step 16: outer restart
        if ksub + kb > p.dim_max:
            kact = p.dim_max - 2 * kb - kc
            if p.k_ro > 0:
                kact = min(kact, p.k_ro)
            ksub = kc + kact
            history[-1]["outer_restart"] = True
        # step 17: next block to filter (progressive filtering), after any
        # pairs the certificate un-locked
        nu = unlocked.shape[1]
        parts = [unlocked] if nu else []
        n_from_init = max(0, min(ec, k_init - k_i, kb - nu))
        if n_from_init:
            parts.append(np.asarray(V_init[:, k_i:k_i + n_from_init], dtype=np.float64))
        n_ritz = min(kb - ec, kact, kb - nu - n_from_init)
        if n_ritz:
            parts.append(V[:, kc:kc + n_ritz])
        pad = kb - nu - n_from_init - n_ritz
        if pad:
            parts.append(rand_cols(pad))
        V_tmp = np.asfortranarray(np.concatenate(parts, axis=1))
        k_i += n_from_init
        # step 18
        if kact:
            med = _median(D_act[:kact])
            if lowb < med < upperb:
                low_nwb = med
    k_out = min(kc, p.k_want)
    evecs = np.array(V[:, :k_out])
    ev = evals[:k_out].copy()
    if status == "noconv" and k_out:
        R = apply_laplacian(csr, np.asfortranarray(evecs)) - evecs * ev
        cert = np.sqrt(np.sum(R * R, axis=0))
        n_other += 1
    if k_out:
        max_res = float(np.max(cert))
        certified = int(np.sum(cert <= p.certify_tol))
    else:
        max_res = float("nan")
        certified = 0
    return Result(evals=ev, evecs=evecs, converged=kc, iterations=it, n_spmm_filter=n_filter,
                  n_spmm_other=n_other, n_random=n_random, max_residual=max_res, history=history,
                  certified=certified, n_unlocked=n_unlocked, status=status)
