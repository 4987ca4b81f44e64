"""Oracle: the OpInf subdomain model and compressed Kronecker powers.

Model (Eq. opinf_model_schwarz, Sec. 4.2), written with the signs folded into
the operators:   q'' = A q + H (q (x) q) + B g^ + c
i.e. A = -K_bar, H = -H_bar, B = B_bar; c is an optional constant term (the
paper's form has none).  g^ = Phi_S^T s is the Schwarz data s on the overlap
boundary expressed in the boundary POD basis (Sec. 4.2.1).  The exterior
Dirichlet data chi are identically zero for the clamped bars, so the Phi_D^T chi
block of g^ vanishes and is omitted.

Compressed quadratic power (footnote to Eq. quadratic_model): the symmetric
q (x) q is parameterised by its independent entries q_i q_j, i <= j, listed
row by row of the upper triangle; width r(r+1)/2.  The cubic power of COpInf
likewise: q_i q_j q_k, i <= j <= k, lexicographic; width r(r+1)(r+2)/6.

The time integrator is the textbook Newmark-beta of oracle/newmark.py applied
to the reduced state (the ROM equation in Eq. schwarz_opinf_discrete carries
the same garbled scaling as Eq. schwarz_discrete).  Implicit steps solve
q+ - beta dt^2 f(q+) = q~ by Newton's method.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .newmark import SubdomainGeometry


def kron2(q: np.ndarray) -> np.ndarray:
    """[q_i q_j]_{i<=j}, upper triangle row by row.  q: (r,) or (r, T)."""
    r = q.shape[0]
    i, j = np.triu_indices(r)
    return q[i] * q[j]


def kron2_jacobian(q: np.ndarray) -> np.ndarray:
    """d kron2(q) / dq  ->  (r(r+1)/2, r)."""
    r = q.shape[0]
    i, j = np.triu_indices(r)
    J = np.zeros((i.size, r), dtype=q.dtype)
    J[np.arange(i.size), i] += q[j]
    J[np.arange(i.size), j] += q[i]
    return J


def kron3(q: np.ndarray) -> np.ndarray:
    """[q_i q_j q_k]_{i<=j<=k}, lexicographic in (i, j, k); width r(r+1)(r+2)/6 (the
    compressed cubic power of Sec. 3, footnote to Eq. quadratic_model).  q: (r,) or (r, T)."""
    r = q.shape[0]
    idx = [(i, j, k) for i in range(r) for j in range(i, r) for k in range(j, r)]
    i, j, k = (np.array(t, dtype=np.int64) for t in zip(*idx)) if idx else (np.zeros(0, np.int64),) * 3
    return q[i] * q[j] * q[k]


def kron3_jacobian(q: np.ndarray) -> np.ndarray:
    """d kron3(q) / dq  ->  (r(r+1)(r+2)/6, r)."""
    r = q.shape[0]
    idx = [(i, j, k) for i in range(r) for j in range(i, r) for k in range(j, r)]
    J = np.zeros((len(idx), r), dtype=q.dtype)
    for m, (i, j, k) in enumerate(idx):
        J[m, i] += q[j] * q[k]
        J[m, j] += q[i] * q[k]
        J[m, k] += q[i] * q[j]
    return J


def newmark_reduced_step(ops, q0, qd0, qdd0, gh, dt, beta=0.0, gamma=0.5):
    """One Newmark-beta step of q'' = ops.rhs(q, g^) with boundary input gh at the new time."""
    qt = q0 + dt * qd0 + (0.5 - beta) * dt * dt * qdd0
    if beta == 0.0:
        q = qt
        qdd = ops.rhs(q, gh)
    else:
        q = qt.copy()
        for _ in range(50):
            res = q - beta * dt * dt * ops.rhs(q, gh) - qt
            J = np.eye(q.shape[0]) - beta * dt * dt * ops.rhs_jac(q)
            dq = np.linalg.solve(J, res)
            q = q - dq
            if np.linalg.norm(dq) <= 1e-15 * (1.0 + np.linalg.norm(q)):
                break
        qdd = (q - qt) / (beta * dt * dt)
    qd = qd0 + dt * ((1.0 - gamma) * qdd0 + gamma * qdd)
    return q, qd, qdd


class Operators:
    """Reduced operators (A, H, B, c, C) of q'' = A q + H (q (x) q) + C (q (x) q (x) q) + B g^ + c
    (C: the cubic operator of COpInf, Eq. opinf_rom)."""

    def __init__(self, A, H=None, B=None, c=None, C=None):
        self.A, self.H, self.B, self.c, self.C = A, H, B, c, C
        self.r = A.shape[0]

    def rhs(self, q, gh):
        out = self.A @ q
        if self.H is not None:
            out = out + self.H @ kron2(q)
        if self.C is not None:
            out = out + self.C @ kron3(q)
        if self.B is not None and gh.size:
            out = out + self.B @ gh
        if self.c is not None:
            out = out + (self.c if q.ndim == 1 else self.c[:, None])
        return out

    def rhs_jac(self, q):
        J = self.A.astype(np.result_type(self.A, q))
        if self.H is not None:
            J = J + self.H @ kron2_jacobian(q)
        if self.C is not None:
            J = J + self.C @ kron3_jacobian(q)
        return J


@dataclass
class RomState:
    q: np.ndarray
    qd: np.ndarray
    qdd: np.ndarray
    s: np.ndarray      # Schwarz values last imposed (for the lifted field)

    def copy(self):
        return RomState(self.q.copy(), self.qd.copy(), self.qdd.copy(), self.s.copy())


class OpInfModel:
    kind = "opinf"

    def __init__(self, geom: SubdomainGeometry, Phi, PhiS, A, H=None, B=None, c=None,
                 dt: float = 1.0, beta: float = 0.0, gamma: float = 0.5, C=None):
        self.geom = geom
        self.Phi, self.PhiS = Phi, PhiS
        self.A, self.H, self.B, self.c, self.C = A, H, B, c, C
        self.dt, self.beta, self.gamma = dt, beta, gamma
        self.r = A.shape[0]
        self.ops = Operators(A, H, B, c, C)
        self.sch_dofs = geom.sch_dofs
        self.free_dofs = geom.free_dofs
        self.dir_dofs = geom.dir_dofs
        self.n_dofs = geom.n_dofs
        self.mesh = geom.mesh
        self.z_lo, self.z_hi = geom.z_lo, geom.z_hi

    # q'' = f(q, g^)
    def ghat(self, s: np.ndarray) -> np.ndarray:
        if self.PhiS is None or self.B is None:
            return np.zeros(0)
        return self.PhiS.T @ s

    def rhs(self, q, gh):
        return self.ops.rhs(q, gh)

    def rhs_jac(self, q):
        return self.ops.rhs_jac(q)

    def initial_state(self, u0_global, v0_global) -> RomState:
        """q0 = Phi^T u0, q'0 = Phi^T v0 on free DOFs; q''0 = f(q0, g^0) (consistent start)."""
        u = self.geom.restrict(u0_global)
        v = self.geom.restrict(v0_global)
        f = self.free_dofs
        q = self.Phi.T @ u[f]
        qd = self.Phi.T @ v[f]
        s = u[self.sch_dofs].copy()
        qdd = self.rhs(q, self.ghat(s))
        return RomState(q, qd, qdd, s)

    def state_from_reduced(self, q, qd, qdd, s) -> RomState:
        return RomState(np.array(q), np.array(qd), np.array(qdd), np.array(s))

    def step(self, st: RomState, s_new: np.ndarray) -> RomState:
        q, qd, qdd = newmark_reduced_step(self, st.q, st.qd, st.qdd, self.ghat(s_new),
                                          self.dt, self.beta, self.gamma)
        return RomState(q, qd, qdd, np.array(s_new, copy=True))

    def field(self, st: RomState) -> np.ndarray:
        """Lifted nodal field: Phi q on free DOFs, imposed Schwarz data, zero Dirichlet."""
        u = np.zeros(self.n_dofs, dtype=np.result_type(st.q, self.Phi, st.s))
        u[self.free_dofs] = self.Phi @ st.q
        u[self.sch_dofs] = st.s
        return u

    def predictor(self, st: RomState, t: float) -> np.ndarray:
        p = RomState(st.q + t * st.qd + 0.5 * t * t * st.qdd, st.qd, st.qdd, st.s)
        return self.field(p)

    # Eq. conv_criterion in reduced coordinates (Phi has orthonormal columns,
    # so these equal the norms of the lifted free-DOF vectors).
    def diff_norm2(self, new: RomState, old: RomState) -> float:
        d = (new.q - old.q) + self.dt * (new.qd - old.qd)
        return float(np.sum(d * d).real)

    def norm2(self, st: RomState) -> float:
        d = st.q + self.dt * st.qd
        return float(np.sum(d * d).real)

    def free_u(self, st: RomState) -> np.ndarray:
        return self.Phi @ st.q
