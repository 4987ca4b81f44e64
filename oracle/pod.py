"""Oracle: proper orthogonal decomposition (Sec. 3.1, Eq. pod_cutoff, Eq. pod_energy).

POD basis of rank r = the first r left singular vectors of the snapshot
matrix U (thin SVD U = Phi Sigma Psi^T), computed here with the library SVD
directly (no Gram matrix).  Readings:
  * no centring of the snapshots (the paper takes the SVD of U itself);
  * Eq. pod_energy prints "E_r < delta_E"; the intended rule is the smallest r
    with E_r >= delta_E;
  * singular vectors are defined up to sign: each column is flipped so that its
    largest-magnitude entry is positive.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np


def energy_rank(sigma: np.ndarray, delta: float) -> int:
    """Smallest r with E_r = sum_{i<=r} sigma_i^2 / sum_i sigma_i^2 >= delta."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    tot = s2.sum()
    if tot == 0.0:
        return 0
    e = np.cumsum(s2) / tot
    return int(min(np.searchsorted(e, delta, side="left") + 1, s2.size))


def fix_signs(Phi: np.ndarray) -> np.ndarray:
    idx = np.argmax(np.abs(Phi), axis=0)
    sgn = np.sign(Phi[idx, np.arange(Phi.shape[1])])
    sgn[sgn == 0] = 1.0
    return Phi * sgn[None, :]


def pod(U: np.ndarray, r: int | None = None, energy: float | None = None):
    """Return (Phi_r, sigma) for snapshot matrix U (N x T)."""
    Phi, sigma, _ = np.linalg.svd(U, full_matrices=False)
    if r is None:
        r = sigma.size if energy is None else energy_rank(sigma, energy)
    return fix_signs(Phi[:, :r]), sigma


def projection_error(u: np.ndarray, Phi: np.ndarray) -> float:
    """Eq. projerr: ||u - Phi Phi^T u|| / ||u|| (Frobenius norm for a matrix of columns)."""
    d = u - Phi @ (Phi.T @ u)
    return float(np.linalg.norm(d) / np.linalg.norm(u))
