"""Oracle: Saint Venant-Kirchhoff hyperelasticity on hex8 elements and its explicit
Newmark FOM.

App. A.2: free-energy density A(E) = lam/2 (tr E)^2 + mu tr(E^2) with the Green-Lagrange
strain E = (F^T F - I)/2, F = I + grad u (the printed "1/2 F^T F - I" is read as the
derivation right after it states, E = (grad u + grad u^T + grad u^T grad u)/2); second
Piola-Kirchhoff stress S = lam tr(E) I + 2 mu E, first P = F S.  The Galerkin internal
force of node a (Sec. 2, total Lagrangian form of Eq. weak_form) is
    f_a = sum_elements sum_gauss w det(J) P grad N_a,
with the full 2x2x2 Gauss rule of the linear model (oracle/fem.py).  f is a cubic
polynomial of the nodal displacements; its linearisation at u = 0 is the linear elastic
K of the same lam, mu.  The explicit Newmark step is that of oracle/newmark.py with
K u+ replaced by f(u+).
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

from .fem import GAUSS_POINTS, GAUSS_WEIGHTS, lame, shape_grads_ref
from .newmark import FomModel, FomState


def _grads(Xe):
    """Per Gauss point: w det(J) (E,) and dN/dX (E, 8, 3) of elements with corners Xe (E, 8, 3)."""
    out = []
    for g, w in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
        dN = shape_grads_ref(g)
        J = np.einsum('ad,eai->eid', dN, Xe)
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        out.append((w * detJ, np.einsum('ad,edi->eai', dN, Jinv)))
    return out


def element_energy_and_force(Xe, ue, lam, mu):
    """Stored energy (E,) and internal force (E, 8, 3) of elements with corner
    coordinates Xe and displacements ue (E, 8, 3); complex ue gives complex results
    (no conjugation anywhere, so the complex step differentiates them)."""
    nE = Xe.shape[0]
    W = np.zeros(nE, dtype=ue.dtype)
    f = np.zeros((nE, 8, 3), dtype=ue.dtype)
    I = np.eye(3)
    for wdet, dNdX in _grads(Xe):
        Gu = np.einsum('eai,eaj->eij', ue, dNdX)          # (grad u)_ij = sum_a u_a,i dN_a/dX_j
        F = I[None] + Gu
        E = 0.5 * (np.einsum('eki,ekj->eij', F, F) - I[None])
        trE = np.einsum('eii->e', E)
        S = lam * trE[:, None, None] * I[None] + 2.0 * mu * E
        P = np.einsum('eik,ekj->eij', F, S)
        W = W + wdet * (0.5 * lam * trE * trE + mu * np.einsum('eij,eij->e', E, E))
        f = f + wdet[:, None, None] * np.einsum('eij,eaj->eai', P, dNdX)
    return W, f


def internal_force(mesh, u, lam, mu):
    """Assembled f(u) (3n, DOF order 3*node + c) and the stored energy of a SubMesh."""
    ue = u.reshape(-1, 3)[mesh.conn]                       # (E, 8, 3)
    Xe = mesh.X[mesh.conn]
    W, fe = element_energy_and_force(Xe, ue, lam, mu)
    f = np.zeros((mesh.n_nodes, 3), dtype=fe.dtype)
    np.add.at(f, mesh.conn.ravel(), fe.reshape(-1, 3))
    return f.reshape(-1), W.sum()


class SvkFomModel(FomModel):
    """FE subdomain with the Saint Venant-Kirchhoff material, explicit Newmark (beta = 0):
        u+ = u + dt v + dt^2/2 a;  a+ = M^-1 ( -f(u+) ) on free DOFs;  v+ = v + dt (a + a+)/2."""
    kind = "fom"

    def __init__(self, bar, z_lo, z_hi, dt, clamp_ends=True, lateral_fix=()):
        super().__init__(bar, z_lo, z_hi, dt, beta=0.0, gamma=0.5, clamp_ends=clamp_ends, lateral_fix=lateral_fix)
        self.lam, self.mu = lame(bar.E, bar.nu)

    def force(self, u):
        return internal_force(self.mesh, u, self.lam, self.mu)[0]

    def initial_state(self, u0_global, v0_global) -> FomState:
        u = self.restrict(u0_global)
        v = self.restrict(v0_global)
        u[self.dir_dofs] = 0.0
        v[self.dir_dofs] = 0.0
        v[self.sch_dofs] = 0.0
        a = np.zeros_like(u)
        f = self.free_dofs
        a[f] = -self.force(u)[f] / self.m_f
        return FomState(u, v, a)

    def step(self, st: FomState, s_new: np.ndarray) -> FomState:
        dt, g = self.dt, self.gamma
        f = self.free_dofs
        u = np.zeros_like(st.u)
        u[self.sch_dofs] = s_new
        u[f] = st.u[f] + dt * st.v[f] + 0.5 * dt * dt * st.a[f]
        a_f = -self.force(u)[f] / self.m_f
        v = np.zeros_like(st.v)
        a = np.zeros_like(st.a)
        v[f] = st.v[f] + dt * ((1.0 - g) * st.a[f] + g * a_f)
        a[f] = a_f
        return FomState(u, v, a)

    def energy(self, st: FomState) -> float:
        return float(0.5 * st.v @ (self.m * st.v) + internal_force(self.mesh, st.u, self.lam, self.mu)[1])
