"""Oracle: one subdomain's FE model advanced by Newmark-beta.

Sec. 2 (Eq. matrix_vector_form_with_dbcs): unknowns are the free DOFs; the
constrained DOFs carry prescribed values -- zero on clamped (exterior
Dirichlet) faces, and the Schwarz data s on the overlap boundary
(Sec. 4.1, the boundary d_S Omega_i = d Omega_i cap Omega_j).

Time stepping (Sec. 4.1).  Eq. schwarz_discrete is printed with a garbled
scaling (M / (dt beta) where Newmark needs M / (dt^2 beta), and an
acceleration coefficient that cannot express beta = 0), so the oracle takes
the textbook Newmark-beta scheme it denotes:
    u~   = u + dt v + (1/2 - beta) dt^2 a                       (predictor)
    beta = 0 : u+ = u~ ;  a+ = M^-1 ( -K u+ )   on free DOFs     (explicit)
    beta > 0 : (M/(beta dt^2) + K_ff) u+_f = M u~_f/(beta dt^2) - K_fc u+_c
               a+ = (u+ - u~) / (beta dt^2)                      (implicit)
    v+   = v + dt ((1 - gamma) a + gamma a+)
with the lumped (row-sum) mass M for both variants.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from paper_2511_20687_amd.inputs import Bar
from .fem import SubMesh, assemble


@dataclass
class FomState:
    u: np.ndarray   # all DOFs (3n), constrained DOFs hold prescribed values
    v: np.ndarray
    a: np.ndarray

    def copy(self):
        return FomState(self.u.copy(), self.v.copy(), self.a.copy())


class SubdomainGeometry:
    """Mesh of node layers z_lo..z_hi and its DOF partition.

    Exterior z-faces (z_lo == 0, z_hi == nz) are clamped when ``clamp_ends``;
    interior z-faces are Schwarz boundaries.  ``lateral_fix`` lists the
    components held at zero on the lateral faces x, y = 0, L (used by the
    effectively-1D bar of Sec. 5.1; empty = traction-free lateral faces).
    """

    def __init__(self, bar: Bar, z_lo: int, z_hi: int, clamp_ends: bool = True,
                 lateral_fix=()):
        self.bar, self.z_lo, self.z_hi = bar, z_lo, z_hi
        self.mesh = SubMesh(bar, z_lo, z_hi)
        mesh = self.mesh
        n = 3 * mesh.n_nodes
        fixed = np.zeros(n, dtype=bool)
        sch = np.zeros(n, dtype=bool)
        faces = [(0, z_lo == 0), (mesh.nzs, z_hi == bar.nz)]
        for kl, exterior in faces:
            nodes = mesh.layer_nodes(kl)
            dofs = (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()
            if exterior:
                if clamp_ends:
                    fixed[dofs] = True
            else:
                sch[dofs] = True
        for c in lateral_fix:
            fixed[3 * mesh.lateral_nodes() + c] = True
        fixed &= ~sch
        self.n_dofs = n
        self.sch_dofs = np.nonzero(sch)[0]
        self.dir_dofs = np.nonzero(fixed)[0]
        self.free_dofs = np.nonzero(~(sch | fixed))[0]
        self.constrained = np.nonzero(sch | fixed)[0]

    @property
    def n_free(self):
        return self.free_dofs.size

    @property
    def n_sch(self):
        return self.sch_dofs.size

    def restrict(self, field_global: np.ndarray) -> np.ndarray:
        """Global SoA field (3, n_global) -> local DOF vector (3n) in oracle order."""
        loc = field_global[:, self.mesh.global_ids]          # (3, n_local)
        return loc.T.reshape(-1).astype(field_global.dtype)


class FomModel(SubdomainGeometry):
    kind = "fom"

    def __init__(self, bar: Bar, z_lo: int, z_hi: int, dt: float, beta: float = 0.0,
                 gamma: float = 0.5, clamp_ends: bool = True, lateral_fix=()):
        super().__init__(bar, z_lo, z_hi, clamp_ends, lateral_fix)
        self.dt, self.beta, self.gamma = dt, beta, gamma
        self.K, self.m = assemble(self.mesh)
        f = self.free_dofs
        self.K_ff = self.K[f][:, f].tocsc()
        self.K_fc = self.K[f][:, self.constrained].tocsr()
        self.m_f = self.m[f]
        self._lu = None
        if beta > 0.0:
            import scipy.sparse as sp
            Aff = sp.diags(self.m_f / (beta * dt * dt)) + self.K_ff
            self._lu = spla.splu(Aff.tocsc())

    # -- initial state ----------------------------------------------------
    def initial_state(self, u0_global: np.ndarray, v0_global: np.ndarray) -> FomState:
        """Restrict the global IC; zero the exterior-Dirichlet DOFs; a0 = M^-1(-K u0) on free DOFs.

        The Schwarz DOFs keep the global IC values at t0 (same field for all subdomains).
        """
        u = self.restrict(u0_global)
        v = self.restrict(v0_global)
        u[self.dir_dofs] = 0.0
        v[self.dir_dofs] = 0.0
        v[self.sch_dofs] = 0.0
        a = np.zeros_like(u)
        f = self.free_dofs
        a[f] = -(self.K @ u)[f] / self.m_f
        return FomState(u, v, a)

    # -- one Newmark step with Schwarz data s_new at the new time ---------
    def step(self, st: FomState, s_new: np.ndarray) -> FomState:
        dt, b, g = self.dt, self.beta, self.gamma
        f = self.free_dofs
        u = np.zeros_like(st.u)
        u[self.sch_dofs] = s_new
        ut = st.u[f] + dt * st.v[f] + (0.5 - b) * dt * dt * st.a[f]
        if b == 0.0:
            u[f] = ut
            a_f = -(self.K @ u)[f] / self.m_f
        else:
            rhs = self.m_f * ut / (b * dt * dt) - self.K_fc @ u[self.constrained]
            if np.iscomplexobj(rhs):
                u[f] = self._lu.solve(rhs.real) + 1j * self._lu.solve(rhs.imag)
            else:
                u[f] = self._lu.solve(rhs)
            a_f = (u[f] - ut) / (b * dt * dt)
        v = np.zeros_like(st.v)
        a = np.zeros_like(st.a)
        v[f] = st.v[f] + dt * ((1.0 - g) * st.a[f] + g * a_f)
        a[f] = a_f
        return FomState(u, v, a)

    def predictor(self, st: FomState, t: float) -> np.ndarray:
        """Newmark displacement predictor a time t ahead of state st (all DOFs)."""
        return st.u + t * st.v + 0.5 * t * t * st.a

    # -- Schwarz helpers (Eq. conv_criterion, free DOFs) ------------------
    def field(self, st: FomState) -> np.ndarray:
        return st.u

    def diff_norm2(self, new: FomState, old: FomState) -> float:
        f = self.free_dofs
        d = (new.u[f] - old.u[f]) + self.dt * (new.v[f] - old.v[f])
        return float(np.sum(d * d).real)

    def norm2(self, st: FomState) -> float:
        f = self.free_dofs
        d = st.u[f] + self.dt * st.v[f]
        return float(np.sum(d * d).real)

    def free_u(self, st: FomState) -> np.ndarray:
        return st.u[self.free_dofs]

    # -- energy of the discrete scheme ------------------------------------
    def energy(self, st: FomState) -> float:
        """E_h = 1/2 v^T M v + 1/2 u^T K u + (beta - 1/4) dt^2/2 a^T M a (homogeneous BCs)."""
        u, v, a = st.u, st.v, st.a
        return float(0.5 * v @ (self.m * v) + 0.5 * u @ (self.K @ u)
                     + (self.beta - 0.25) * 0.5 * self.dt ** 2 * a @ (self.m * a))


def single_domain(bar: Bar, dt: float, beta: float = 0.0, gamma: float = 0.5,
                  clamp_ends: bool = True, lateral_fix=()) -> FomModel:
    """The whole bar as one FE model (no Schwarz boundary)."""
    return FomModel(bar, 0, bar.nz, dt, beta, gamma, clamp_ends, lateral_fix)


def run_single(model: FomModel, u0_global, v0_global, n_steps: int, record_every: int = 1):
    """Advance a Schwarz-free model n_steps; return the states every record_every steps."""
    st = model.initial_state(u0_global, v0_global)
    empty = np.zeros(0, dtype=st.u.dtype)
    out = [st.copy()]
    for k in range(1, n_steps + 1):
        st = model.step(st, empty)
        if k % record_every == 0:
            out.append(st.copy())
    return out
