"""Oracle: Operator Inference least squares and Schwarz-aware lambda selection.

Eq. quadratic_opinf / Eq. opinf_schwarz_inference (Sec. 3.2, 4.2.1): with
reduced snapshots Q = Phi^T U (r x T), reduced accelerations Qdd = Phi^T U''
and reduced Schwarz data S^ = Phi_S^T S (r_S x T), find

    argmin_O  || O D^T - Qdd ||_F^2 + lambda ||O||_F^2,
    D = [ Q^T | (Q (x) Q)^T | (Q (x) Q (x) Q)^T | S^^T | 1 ]   (T x p),
    O = [A | H | C | B | c]  (r x p)   (linear: no H, C; quadratic: no C; cubic: all)

(signs folded into the operators, see oracle/rom.py).  Readings:
  * D_t^2(U) "e.g. by finite differences": the FOM's own Newmark accelerations
    at the snapshot times are used (for the explicit central-difference scheme at
    unit stride they equal the second difference quotient of U);
  * compressed quadratic columns q_i q_j, i <= j (width r(r+1)/2);
  * lambda is one scalar for all blocks (Remark on per-operator lambda: not
    used), applied in units of the training amplitude alpha = the largest
    ||q_j||_2 over all training columns.  The paper fixes no units for its
    absolute grid 10^-10..1, while the eigenvalues of D^T D scale with powers of
    the length unit (about T alpha^2 for the linear and boundary columns, T alpha^4
    for the quadratic ones; alpha ~ 1e-3 m here), so in raw SI data most of the
    grid would shrink the operators and the choice would depend on the unit.
    The fit is posed on the data scaled to unit amplitude (q/alpha, s^/alpha),
    with time in steps (tau = t/dt):
        argmin || dt^2 Qdd/alpha - At Q/alpha - Ht (Q/alpha)^(2) - Bt S^/alpha - ct 1^T ||^2
               + lambda ||[At Ht Bt ct]||^2,
    mapped back with A = At/dt^2, H = Ht/(dt^2 alpha), C = Ct/(dt^2 alpha^2),
    B = Bt/dt^2, c = alpha ct/dt^2 (the cubic block is weighted lambda alpha^6).  In physical units this is the raw ridge problem with
    the penalty lambda (alpha^2 ||A||^2 + alpha^4 ||H||^2 + alpha^2 ||B||^2 + ||c||^2):
    dt cancels from the minimiser (the time scaling only keeps the arithmetic
    of order one) and a change of length unit maps the operators exactly
    (dt = 1, alpha = 1 is the raw fit); no centering;
  * when T < p the objective still has a unique minimiser (lambda > 0).
The ridge problem is solved by its definition as an ordinary least-squares
problem on the stacked system [D; sqrt(lambda) I] X = [Qdd^T; 0] (library SVD
solver), not via normal equations.

Alg. 3 (Sec. 4.2.3): for each lambda in the grid 10^{-10 + 10 (j-1)/(n-1)},
fit, roll the ROM out over the training time grid with the Schwarz data frozen
to the training values, starting from the training (q, q', q'') at j = 0, and
score E(lambda) = ||Q_rom - Q||_F / ||Q||_F (Eq. schwarz_regularization_error).
Readings: "large penalty" = +inf; "unstable" = a non-finite state or
||q|| > 1e6 max_j ||q_j||; ties go to the smallest lambda; several training
trajectories -> mean of their errors; the fit uses all snapshots together.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from .rom import Operators, kron2, kron3, newmark_reduced_step


def lambda_grid(n: int = 11) -> np.ndarray:
    if n == 1:
        return np.array([1e-10])
    delta = 10.0 / (n - 1)
    return np.array([10.0 ** (-10.0 + delta * j) for j in range(n)])


def data_matrix(Q: np.ndarray, Shat: Optional[np.ndarray], form: str = "linear",
                with_c: bool = False) -> np.ndarray:
    cols = [Q.T]
    if form in ("quadratic", "cubic"):
        cols.append(kron2(Q).T)
    if form == "cubic":
        cols.append(kron3(Q).T)
    if Shat is not None and Shat.shape[0] > 0:
        cols.append(Shat.T)
    if with_c:
        cols.append(np.ones((Q.shape[1], 1)))
    return np.hstack(cols)


def ridge(D: np.ndarray, R: np.ndarray, lam: float) -> np.ndarray:
    """argmin_X ||D X - R||_F^2 + lam ||X||_F^2  (X: p x r)."""
    p = D.shape[1]
    Daug = np.vstack([D, np.sqrt(lam) * np.eye(p)])
    Raug = np.vstack([R, np.zeros((p, R.shape[1]))])
    X, *_ = np.linalg.lstsq(Daug, Raug, rcond=None)
    return X


def split_operators(X: np.ndarray, r: int, form: str, rS: int, with_c: bool) -> Operators:
    O = X.T                                   # r x p
    k = 0
    A = O[:, k:k + r]; k += r
    H = None
    if form in ("quadratic", "cubic"):
        w = r * (r + 1) // 2
        H = O[:, k:k + w]; k += w
    C = None
    if form == "cubic":
        w3 = r * (r + 1) * (r + 2) // 6
        C = O[:, k:k + w3]; k += w3
    B = None
    if rS > 0:
        B = O[:, k:k + rS]; k += rS
    c = O[:, k] if with_c else None
    return Operators(A.copy(), None if H is None else H.copy(),
                     None if B is None else B.copy(), None if c is None else c.copy(),
                     None if C is None else C.copy())


def amplitude_scale(Qs: List[np.ndarray]) -> float:
    """alpha: the largest column norm ||q_j||_2 over all training trajectories (1 if zero)."""
    a = max(float(np.max(np.linalg.norm(Q, axis=0))) for Q in Qs)
    return a if a > 0.0 else 1.0


def fit(Qs: List[np.ndarray], Qdds: List[np.ndarray], Shats: List[Optional[np.ndarray]],
        lam: float, form: str = "linear", with_c: bool = False, dt: float = 1.0,
        alpha: float = 1.0) -> Operators:
    """Ridge fit in the normalised variables (tau = t/dt, q/alpha), returned in physical units."""
    Qn = [Q / alpha for Q in Qs]
    Sn = [None if S is None else S / alpha for S in Shats]
    D = np.vstack([data_matrix(Q, S, form, with_c) for Q, S in zip(Qn, Sn)])
    R = np.hstack([dt * dt * Qdd / alpha for Qdd in Qdds]).T
    X = ridge(D, R, lam)
    r = Qs[0].shape[0]
    rS = 0 if Shats[0] is None else Shats[0].shape[0]
    o = split_operators(X, r, form, rS, with_c)
    dt2 = dt * dt
    return Operators(o.A / dt2,
                     None if o.H is None else o.H / (dt2 * alpha),
                     None if o.B is None else o.B / dt2,
                     None if o.c is None else o.c * alpha / dt2,
                     None if o.C is None else o.C / (dt2 * alpha * alpha))


def rollout_frozen(ops: Operators, q0, qd0, qdd0, Shat: Optional[np.ndarray], n_cols: int,
                   dt: float, beta: float = 0.0, gamma: float = 0.5, stride: int = 1) -> np.ndarray:
    """Alg. 3 inner loop: from snapshot column j to j+1, `stride` time steps with the
    training boundary input frozen; returns r x n_cols at the snapshot times.

    Reading (Alg. 3 assumes a snapshot per step): with snapshots every `stride` steps the
    boundary input of the steps in between is interpolated linearly between the two
    snapshots (exactly S^[:, j+1] at the end of the interval; stride 1 is the plain rule)."""
    r = q0.shape[0]
    out = np.zeros((r, n_cols), dtype=np.result_type(q0, ops.A))
    q, qd, qdd = np.array(q0), np.array(qd0), np.array(qdd0)
    out[:, 0] = q
    with np.errstate(all="ignore"):
        for j in range(n_cols - 1):
            for m in range(1, stride + 1):
                if Shat is None:
                    gh = np.zeros(0)
                else:
                    gh = Shat[:, j] + (m / stride) * (Shat[:, j + 1] - Shat[:, j])
                q, qd, qdd = newmark_reduced_step(ops, q, qd, qdd, gh, dt, beta, gamma)
            out[:, j + 1] = q
            if not np.all(np.isfinite(q)):
                out[:, j + 1:] = np.nan
                break
    return out


def trajectory_error(Qrom: np.ndarray, Q: np.ndarray, blowup: float = 1e6) -> float:
    if not np.all(np.isfinite(Qrom)):
        return np.inf
    if np.max(np.linalg.norm(Qrom, axis=0)) > blowup * np.max(np.linalg.norm(Q, axis=0)):
        return np.inf
    return float(np.linalg.norm(Qrom - Q) / np.linalg.norm(Q))


def select_lambda(trajs: List[dict], lambdas, form: str = "linear", with_c: bool = False,
                  dt: float = 1.0, beta: float = 0.0, gamma: float = 0.5, stride: int = 1):
    """Alg. 3.  trajs: dicts with Q (r x T), Qd0 (r), Qdd (r x T), Shat (r_S x T | None);
    snapshots every `stride` time steps of length dt.

    Returns (lambda_star, E (n_lambda,), operators refit at lambda_star).
    """
    Qs = [t["Q"] for t in trajs]
    Qdds = [t["Qdd"] for t in trajs]
    Shats = [t.get("Shat") for t in trajs]
    alpha = amplitude_scale(Qs)
    E = np.zeros(len(lambdas))
    for li, lam in enumerate(lambdas):
        ops = fit(Qs, Qdds, Shats, lam, form, with_c, dt, alpha)
        errs = []
        for t in trajs:
            Qrom = rollout_frozen(ops, t["Q"][:, 0], t["Qd0"], t["Qdd"][:, 0], t.get("Shat"),
                                  t["Q"].shape[1], dt, beta, gamma, stride)
            errs.append(trajectory_error(Qrom, t["Q"]))
        E[li] = np.mean(errs)
    best = int(np.argmin(E))            # first minimiser = smallest lambda on ties
    lam_star = float(lambdas[best])
    return lam_star, E, fit(Qs, Qdds, Shats, lam_star, form, with_c, dt, alpha)
