"""Oracle: error metrics of Sec. 5 (Eq. mse).

E(u) = sqrt(sum_k ||u(t_k) - u_ref(t_k)||^2) / sqrt(sum_k ||u_ref(t_k)||^2),
the relative space-time L2 error over the recorded time levels.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np


def rel_l2(u: np.ndarray, u_ref: np.ndarray) -> float:
    """Eq. mse for arrays of snapshots (any shape; all entries summed)."""
    u = np.asarray(u, dtype=np.float64)
    u_ref = np.asarray(u_ref, dtype=np.float64)
    num = np.sqrt(np.sum((u - u_ref) ** 2))
    den = np.sqrt(np.sum(u_ref ** 2))
    return float(num / den) if den > 0 else float(num)
