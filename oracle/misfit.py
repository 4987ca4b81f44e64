"""Oracle: trajectory misfit of a coupled run and its exact directional derivatives.

J = 1/2 sum_{k = every, 2 every, ... <= n} [ sum_FOM ||u_k - u_obs,k||^2 (free DOFs)
                                            + sum_OpInf ||q_k - q_obs,k||^2 ]

evaluated by running the oracle's multiplicative Schwarz loop (Alg. 1) as it stands.  The
derivative of J along a direction delta of the parameters theta = (OpInf A, H, B, c,
q0, q'0; FOM u0, v0 on free DOFs) is taken by the complex step,

    dJ/dtheta . delta = Im J(theta + i h delta) / h,   h = 1e-30,

which is exact to rounding for the analytic map the run evaluates (every step is
built of sums and products; the convergence test reads real parts only).  Initial
accelerations follow from the perturbed state (a0 = M^-1(-K u0), q''0 = f(q0, g^0)); the
Schwarz data at t_0 are constants of the initial condition.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

from typing import Callable, Dict, List

import numpy as np

from .newmark import FomState
from .rom import RomState
from .schwarz import Coupled, SchwarzOptions


def fom_state(model, u: np.ndarray, v: np.ndarray) -> FomState:
    """State of a FOM subdomain from local DOF vectors (Schwarz/Dirichlet values kept):
    a = M^-1(-K u) on free DOFs."""
    a = np.zeros_like(u + v)
    f = model.free_dofs
    a[f] = -(model.K @ u)[f] / model.m_f
    return FomState(u, v, a)


def rom_state(model, q: np.ndarray, qd: np.ndarray, s: np.ndarray) -> RomState:
    """State of an OpInf subdomain: q''0 = f(q0, g^(s0))."""
    return RomState(q, qd, model.rhs(q, model.ghat(s)), np.array(s))


def misfit(models: list, states: list, n_steps: int, every: int, obs: Dict[int, np.ndarray],
           opts: SchwarzOptions = SchwarzOptions()) -> complex:
    """obs[i]: (n_steps // every, len) with len = free DOFs (FOM, oracle order) or r (OpInf)."""
    out = Coupled(models).run(None, None, n_steps, opts, every=every, record=("u", "q"), states=states)
    J = 0.0
    for i, m in enumerate(models):
        if i not in obs:
            continue
        traj = out["q"][i] if m.kind == "opinf" else out["u"][i]
        d = traj[1:1 + obs[i].shape[0]] - obs[i]
        J = J + 0.5 * np.sum(d * d)
    return J


def directional_derivative(J_of: Callable[[float], complex], h: float = 1e-30) -> float:
    """J_of(eps) evaluates J(theta + eps delta) (complex eps allowed)."""
    return float(np.imag(J_of(1j * h)) / h)
