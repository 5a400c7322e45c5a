"""Proper orthogonal decomposition (oracle, test infrastructure).

POD takes the thin SVD of the snapshot matrix of deviations from the offset,
S = U Sigma V^T (eq. SVD), and keeps the leading n left singular vectors,
with n the smallest integer whose singular-value sum reaches the fraction
epsilon of the total (eq. energy_criteria; the sum is over sigma_i, not
sigma_i^2, as printed; default epsilon = 0.9999).

Singular vectors are unique only up to sign (and rotation inside repeated
singular values, which the paper notes leaves the POD objective unchanged).
Reading used for comparisons: each column is flipped so that its entry of
largest magnitude is positive, ties going to the smallest row index.
"""
from __future__ import annotations

import numpy as np


def energy_dimension(sigma: np.ndarray, energy_frac: float) -> int:
    """Smallest n with sum_{i<=n} sigma_i / sum_i sigma_i >= energy_frac."""
    total = float(np.sum(sigma))
    if total <= 0.0:
        return 1
    acc = 0.0
    for i, s in enumerate(sigma):
        acc += float(s)
        if acc / total >= energy_frac:
            return i + 1
    return len(sigma)


def canonical_signs(Phi: np.ndarray) -> np.ndarray:
    """Flip columns so the largest-magnitude entry (first such row) is positive."""
    Phi = Phi.copy()
    for k in range(Phi.shape[1]):
        i = int(np.argmax(np.abs(Phi[:, k])))  # argmax returns the first maximum
        if Phi[i, k] < 0:
            Phi[:, k] = -Phi[:, k]
    return Phi


def pod_basis(S: np.ndarray, energy_frac: float = 0.9999, n_fixed: int = 0, n_max: int = 0):
    """Return (Phi, sigma, n) for the snapshot matrix S (N x m)."""
    U, sigma, _ = np.linalg.svd(S, full_matrices=False)
    n = n_fixed if n_fixed > 0 else energy_dimension(sigma, energy_frac)
    if n_max > 0:
        n = min(n, n_max)
    n = min(n, U.shape[1])
    return canonical_signs(U[:, :n]), sigma, n
