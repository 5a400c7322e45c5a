"""Sampling indices and the DEIM pseudo-inverse (oracle, test infrastructure).

Hyper-reduction replaces f by Phi_F (Z^T Phi_F)^+ Z^T f, where Z selects n_s
rows (eq. DEIM_f, eq. sol-ls-hyper); only the indices and the n x n_s matrix
(Z^T Phi_F)^+ are stored.  The rows are chosen greedily (Sec. 3.7): classic
DEIM takes one row per basis vector, the row where the residual of
interpolating the next basis vector from the previous ones at the rows chosen
so far is largest; the oversampled variant (GNAT / Carlberg) allows
n_s >= n and replaces the interpolation by a least-squares fit on the chosen
rows.  The paper uses n_s = min(N, lambda n) with oversampling factor lambda.

Reading of the oversampled greedy (the paper only cites it):

* iteration k = 1..n takes a_k = floor(n_s / n) + [k <= n_s mod n] rows;
* the residual is r = u_1 for k = 1 and r = u_k - U[:, :k-1] c otherwise,
  with c the least-squares fit of U[Z, k] by U[Z, :k-1] on the rows Z chosen
  so far;
* the a_k rows are the unselected rows of largest key
  key(j) = floor(|r_j| / max_i |r_i| * 2^40), ties to the smallest row index.
  The key quantises the residual on a 2^-40 relative grid so that two
  correct FP64 evaluations that differ only in rounding choose the same rows,
  including the exact ties that symmetric meshes produce;
* n_s = N returns all rows in order.

For n_s = n this is classic DEIM, whose indices equal the pivots of
row-pivoted LU of U (Sec. 3.7).
"""
from __future__ import annotations

import numpy as np

KEY_BITS = 40
COND_LIMIT = 1e12


class RankDeficient(RuntimeError):
    pass


def rows_per_iteration(n: int, ns: int):
    return [ns // n + (1 if k < ns % n else 0) for k in range(n)]


def residual_keys(r: np.ndarray) -> np.ndarray:
    m = float(np.max(np.abs(r)))
    if m == 0.0:
        return np.zeros(len(r), dtype=np.int64)
    return np.floor(np.ldexp(np.abs(r) / m, KEY_BITS)).astype(np.int64)


def greedy_deim(U: np.ndarray, ns: int) -> np.ndarray:
    """Selected row indices (in selection order) for the basis U (N x n)."""
    N, n = U.shape
    ns = min(ns, N)
    if ns == N:
        return np.arange(N, dtype=np.int64)
    if ns < n:
        raise ValueError("n_s must be at least n")
    Z: list[int] = []
    chosen = np.zeros(N, dtype=bool)
    for k, a_k in enumerate(rows_per_iteration(n, ns)):
        if k == 0:
            r = U[:, 0].copy()
        else:
            A = U[Z, :k]
            b = U[Z, k]
            Q, R = np.linalg.qr(A)
            c = np.linalg.solve(R, Q.T @ b)
            r = U[:, k] - U[:, :k] @ c
        key = residual_keys(r)
        for _ in range(a_k):
            cand = np.where(chosen, -1, key)
            j = int(np.argmax(cand))  # first maximum = smallest index among ties
            Z.append(j)
            chosen[j] = True
    return np.array(Z, dtype=np.int64)


def qdeim(U: np.ndarray, ns: int) -> np.ndarray:
    """Q-DEIM row indices (Sec. 3.7 names it as the alternative to the greedy choice): the pivots of
    the QR factorisation with column pivoting of U^T.

    Column j of U^T is row j of U.  Step k of the pivoted QR takes the unselected row j of largest
    norm of W[j, k:], where W is U with the reflectors of the previous steps applied to its columns
    k.., then applies the Householder reflector that maps the pivot row's W[p, k:] to a multiple of
    e_1 to every row.  The norm is compared through the same quantised key as the greedy choice
    (2^-40 of the largest norm over all rows, ties to the smallest row index).

    Reading for n_s > n (the paper does not say how Q-DEIM oversamples): the pivoted QR is run in
    rounds, each restarting from U and skipping the rows chosen in earlier rounds, until n_s rows
    are chosen; each round adds up to n rows that span the row space of U well among those left.
    n_s = N returns all rows in order.
    """
    N, n = U.shape
    ns = min(ns, N)
    if ns == N:
        return np.arange(N, dtype=np.int64)
    if ns < n:
        raise ValueError("n_s must be at least n")
    Z: list[int] = []
    chosen = np.zeros(N, dtype=bool)
    while len(Z) < ns:
        W = U.astype(np.float64).copy()
        for k in range(n):
            if len(Z) == ns:
                break
            norms = np.sqrt(np.sum(W[:, k:] ** 2, axis=1))
            key = residual_keys(norms)
            j = int(np.argmax(np.where(chosen, -1, key)))
            Z.append(j)
            chosen[j] = True
            x = W[j, k:].copy()
            alpha, xn2 = x[0], float(np.sum(x[1:] ** 2))
            if xn2 == 0.0:
                continue
            beta = -np.copysign(np.sqrt(alpha * alpha + xn2), alpha)
            v = x / (alpha - beta)
            v[0] = 1.0
            tau = (beta - alpha) / beta
            W[:, k:] -= tau * np.outer(W[:, k:] @ v, v)
    return np.array(Z, dtype=np.int64)


def deim_pinv(U: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """(Z^T U)^+ (n x n_s) through a QR factorisation of Z^T U."""
    ZU = U[Z, :]
    if np.linalg.cond(ZU) > COND_LIMIT:
        raise RankDeficient("Z^T Phi_F is numerically rank deficient")
    Q, R = np.linalg.qr(ZU)
    return np.linalg.solve(R, Q.T)


def closure_elements(mesh, en: np.ndarray, Z1: np.ndarray, Z2: np.ndarray) -> np.ndarray:
    """Sorted ids of the elements whose force the sampled rows need.

    A sampled kinematic row (c, node) receives contributions from every
    element containing the node; a sampled thermodynamic row belongs to one
    element (the thermodynamic space is discontinuous).
    """
    nodes = set(int(z) % mesh.n_nodes for z in Z1)
    nt = 2 ** mesh.dim
    els = set(int(z) // nt for z in Z2)
    for K in range(en.shape[0]):
        if any(int(a) in nodes for a in en[K]):
            els.add(K)
    return np.array(sorted(els), dtype=np.int64)
