"""Oracle: multiplicative overlapping Schwarz alternating method (O-SAM).

Follows Sec. 4.1: the time axis is split into controller steps I_k (one
Newmark step per controller step here); within each, Alg. 1 iterates the
subdomain problems in index order (Gauss-Seidel, Remark additive_sam: the
multiplicative variant), each taking Dirichlet data on its Schwarz boundary
from the newest iterate of the neighbour that contains it, until the
criterion Eq. conv_criterion holds.  The additive variant of the same remark
(additive=True) solves the subdomains of an iteration independently: each takes
its data from the neighbours' iterates of the previous iteration (Jacobi).  Sec. 4.2 (OpInf-FOM, OpInf-OpInf) uses
the same loop with ROM subdomains (transfer = pointwise projection of the
lifted field, then Phi_S^T restriction inside the ROM).

Sub-stepping (Sec. 4.1, Eq. schwarz_discrete and the figure of field transfer within a
controller step): subdomain i advances each controller step of length Dt in n_i = n_sub
Newmark steps of dt_i = Dt / n_i.  Its Schwarz data at t_{k-1} + l dt_i come from the
source's trajectory over the same controller step (its states at t_{k-1} + m dt_j,
m = 0 .. n_j, m = 0 being the accepted state) through the temporal interpolant Xi: linear
interpolation in time between the two trajectory points that bracket the destination time
(the source's own points when the times coincide, so equal n_sub needs no interpolation).
A source not yet advanced in the step supplies its guess at every destination time.

Readings (the paper is silent or ambiguous):
  * initial guess phi^(0) of a neighbour not yet advanced in this controller
    step: HOLD = its state at t_{k-1}; PREDICTOR = its Newmark displacement
    predictor u + tau v + tau^2/2 a from its state at t_{k-1}, at the time tau into
    the step where the destination needs data (t_k for one step per controller step);
  * Xi (garbled as a column vector of length n_j acting on n_j source states): the
    source's trajectory includes its state at t_{k-1}, and interpolation is linear
    in time;
  * the criterion needs iterate n-1, so it is tested from n >= min_iter (2);
    if min_iter = 1, iterate 0 is read as the subdomain's state at t_{k-1};
    "or": either the absolute or the relative test suffices; dt in the
    denominator is each subdomain's own dt; norms run over free DOFs
    (reduced coordinates for ROM subdomains);
  * at most max_iter (32) iterations; not converging within the cap is not an
    error (the run continues with the last iterate);
  * pointwise projection Pi (Sec. 4.1): evaluate the source's trilinear FE field
    at the destination node.  For the structured bars the isoparametric map is
    affine per axis, so the reference coordinates follow from the grid index.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from .fem import HEX8_CORNERS, shape_values


class OutsideError(ValueError):
    pass


def _locate(f: float, n: int):
    """Cell index and reference coordinate in [-1,1] of grid coordinate f in [0, n]."""
    if f < -1e-9 or f > n + 1e-9:
        raise OutsideError(f)
    i = int(np.floor(f))
    i = min(max(i, 0), n - 1)
    t = f - i
    if abs(t) < 1e-9:
        t = 0.0
    if abs(t - 1.0) < 1e-9:
        t = 1.0
    return i, 2.0 * t - 1.0


def pointwise_projection(dst, dst_rows: np.ndarray, src) -> sp.csr_matrix:
    """Pi: rows = dst DOFs ``dst.sch_dofs[dst_rows]``, columns = all DOFs of src."""
    bar = src.mesh.bar
    hx, hy, hz = bar.Lx / bar.nx, bar.Ly / bar.ny, bar.Lz / bar.nz
    z0 = src.z_lo * hz
    rows, cols, vals = [], [], []
    for r, d in enumerate(dst.sch_dofs[dst_rows]):
        node, comp = divmod(int(d), 3)
        x, y, z = dst.mesh.X[node]
        i, xi = _locate(x / hx, bar.nx)
        j, eta = _locate(y / hy, bar.ny)
        k, zeta = _locate((z - z0) / hz, src.mesh.nzs)
        N = shape_values(np.array([xi, eta, zeta]))
        for a in range(8):
            if N[a] == 0.0:
                continue
            di, dj, dk = (int(c > 0) for c in HEX8_CORNERS[a])
            sn = src.mesh.node_id(i + di, j + dj, k + dk)
            rows.append(r)
            cols.append(3 * sn + comp)
            vals.append(N[a])
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(dst_rows), src.n_dofs))


def _z_range(m):
    h = m.mesh.bar.Lz / m.mesh.bar.nz
    return m.z_lo * h, m.z_hi * h


@dataclass
class SchwarzOptions:
    tol_abs: float = 1.0e-8
    tol_rel: float = 1.0e-12
    min_iter: int = 2
    max_iter: int = 32
    guess: str = "hold"          # "hold" | "predictor"
    additive: bool = False       # True: every subdomain reads the previous iteration's iterates


@dataclass
class StepInfo:
    iters: int
    converged: bool
    abs2: float
    den2: float


class Coupled:
    """S overlapping subdomain models (FomModel / OpInfModel) on one bar."""

    def __init__(self, models: list):
        self.models = models
        self.blocks = []
        for i, mi in enumerate(models):
            blocks = []
            if mi.sch_dofs.size:
                nodes = mi.sch_dofs // 3
                zc = mi.mesh.X[nodes, 2]
                owner = np.full(mi.sch_dofs.size, -1)
                for j, mj in enumerate(models):
                    if j == i:
                        continue
                    lo, hi = _z_range(mj)
                    tol = 1e-9 * (hi - lo)
                    inside = (zc > lo + tol) & (zc < hi - tol) & (owner < 0)
                    owner[inside] = j
                if np.any(owner < 0):
                    raise OutsideError(f"subdomain {i}: Schwarz node outside every neighbour")
                for j in np.unique(owner):
                    rows = np.nonzero(owner == j)[0]
                    blocks.append((int(j), rows, pointwise_projection(mi, rows, models[j])))
            self.blocks.append(blocks)

    def initial_states(self, u0_global, v0_global):
        return [m.initial_state(u0_global, v0_global) for m in self.models]

    def n_sub(self, i) -> int:
        return int(getattr(self.models[i], "n_sub", 1))

    def schwarz_data(self, i, latest, start, guess, l: int = None):
        """Schwarz data of subdomain i at its sub-step l (time t_{k-1} + l dt_i; default
        l = n_i, i.e. t_k).  latest[j]: trajectory of source j in this step (list of its
        states at sub-steps 0 .. n_j) or None (not yet advanced: the guess)."""
        mi = self.models[i]
        ni = self.n_sub(i)
        l = ni if l is None else l
        dtype = np.result_type(*[m.field(s).dtype for m, s in zip(self.models, start)])
        s = np.zeros(mi.sch_dofs.size, dtype=dtype)
        for j, rows, Pi in self.blocks[i]:
            mj = self.models[j]
            nj = self.n_sub(j)
            if latest[j] is not None:
                # Xi: destination time l dt_i = (l nj / ni) dt_j on the source's grid
                num = l * nj
                m0, rem = divmod(num, ni)
                if rem == 0:
                    fld = mj.field(latest[j][m0])
                else:
                    w = rem / ni
                    fld = (1.0 - w) * mj.field(latest[j][m0]) + w * mj.field(latest[j][m0 + 1])
            elif guess == "hold":
                fld = mj.field(start[j])
            else:
                fld = mj.predictor(start[j], l * mi.dt)
            s[rows] = Pi @ fld
        return s

    def advance(self, i, start_i, src, start, guess):
        """Subdomain i through the n_i sub-steps of one controller step; its trajectory."""
        traj = [start_i]
        st = start_i
        for l in range(1, self.n_sub(i) + 1):
            st = self.models[i].step(st, self.schwarz_data(i, src, start, guess, l))
            traj.append(st)
        return traj

    def step(self, start: list, opts: SchwarzOptions):
        """One controller step (Alg. 1 inner loop). Returns (new states, StepInfo)."""
        S = len(self.models)
        dts = [m.dt * self.n_sub(i) for i, m in enumerate(self.models)]
        if max(dts) - min(dts) > 1e-12 * max(dts):
            raise ValueError("subdomains must share the controller step dt * n_sub")
        latest: List[Optional[list]] = [None] * S
        # iterate 0 of each subdomain (only compared against when min_iter = 1)
        prev: List[Optional[object]] = list(start)
        info = StepInfo(0, False, float('nan'), float('nan'))
        for n in range(1, opts.max_iter + 1):
            # multiplicative: the newest iterates, updated as the sweep goes; additive: those of
            # the previous iteration for every subdomain
            src = list(latest) if opts.additive else latest
            for i in range(S):
                traj = self.advance(i, start[i], src, start, opts.guess)
                prev[i] = latest[i][-1] if latest[i] is not None else start[i]
                latest[i] = traj
            info.iters = n
            if n >= opts.min_iter:
                abs2 = sum(m.diff_norm2(a[-1], b) for m, a, b in zip(self.models, latest, prev))
                den2 = sum(m.norm2(a[-1]) for m, a in zip(self.models, latest))
                info.abs2, info.den2 = abs2, den2
                if abs2 < opts.tol_abs ** 2 or abs2 < opts.tol_rel ** 2 * den2:
                    info.converged = True
                    break
        return [t[-1] for t in latest], info

    def run(self, u0_global, v0_global, n_steps: int, opts: SchwarzOptions = SchwarzOptions(),
            every: int = 1, record=("u",), states=None):
        """Advance n_steps controller steps; record every ``every`` steps (step 0 included).

        record: any of "u" (free-DOF displacement, lifted for ROMs), "v", "a"
        (FOM free DOFs), "s" (Schwarz values), "q", "qd", "qdd" (ROM reduced).
        Returns dict: rec[name][i] -> (n_rec, len) array per subdomain, "iters" -> (n_steps,).
        """
        if states is None:
            states = self.initial_states(u0_global, v0_global)
        S = len(self.models)
        rec = {name: [[] for _ in range(S)] for name in record}

        def take(sts):
            for i, (m, st) in enumerate(zip(self.models, sts)):
                for name in record:
                    if name == "u":
                        rec[name][i].append(m.free_u(st))
                    elif name == "s":
                        rec[name][i].append(st.s.copy() if m.kind == "opinf" else st.u[m.sch_dofs].copy())
                    elif name in ("v", "a"):
                        if m.kind == "fom":
                            rec[name][i].append(getattr(st, name)[m.free_dofs].copy())
                    elif name in ("q", "qd", "qdd"):
                        if m.kind == "opinf":
                            rec[name][i].append(getattr(st, name).copy())

        take(states)
        iters = np.zeros(n_steps, dtype=np.int64)
        conv = np.zeros(n_steps, dtype=bool)
        for k in range(1, n_steps + 1):
            states, info = self.step(states, opts)
            iters[k - 1] = info.iters
            conv[k - 1] = info.converged
            if k % every == 0:
                take(states)
        out = {name: [np.array(x) if len(x) else None for x in rec[name]] for name in record}
        out["iters"] = iters
        out["converged"] = conv
        out["states"] = states
        return out


def union_field(models, free_u_list, nodes_total: int, bar) -> np.ndarray:
    """Single-domain displacement (3, n_global) from subdomain free-DOF values; at nodes
    shared by several subdomains the lowest-index subdomain's value is taken."""
    out = np.full((3, nodes_total), np.nan)
    for m, fu in reversed(list(zip(models, free_u_list))):
        full = np.zeros(m.n_dofs, dtype=fu.dtype)
        full[m.free_dofs] = fu
        loc = full.reshape(-1, 3).T
        mask = np.zeros(m.n_dofs, dtype=bool)
        mask[m.free_dofs] = True
        mnode = mask.reshape(-1, 3).all(axis=1)
        gid = m.mesh.global_ids[mnode]
        out[:, gid] = loc[:, mnode]
    return out
