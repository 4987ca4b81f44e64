"""Helpers for GPU parity tests: run the same coupled problem through the oracle and
through libosam, and bring the library's free-DOF records into the oracle's order."""
import numpy as np

from paper_2511_20687_amd.inputs import Bar
from oracle.newmark import FomModel
from oracle.schwarz import Coupled, SchwarzOptions


def oracle_fom_coupled(bar: Bar, layers, dt, u0, v0, n_steps, opts=None, record=("u",)):
    models = [FomModel(bar, lo, hi, dt) for lo, hi in layers]
    out = Coupled(models).run(u0, v0, n_steps, opts or SchwarzOptions(), record=record)
    return models, out


def lib_free_index(bar: Bar, lo: int, hi: int) -> np.ndarray:
    """For each oracle free DOF (node-major, dof = 3*node + c), its index in the library's
    free-DOF vector [3][free nodes] (free nodes = layers 1..nzs-1)."""
    from paper_2511_20687_amd.osam import free_dof_map
    return free_dof_map(bar.nx, bar.ny, hi - lo)


def lib_sch_index(bar: Bar, lo: int, hi: int) -> np.ndarray:
    """For each oracle Schwarz DOF (node-major), its index in the library's [3][sch nodes]."""
    npl = (bar.nx + 1) * (bar.ny + 1)
    nzs = hi - lo
    faces = []
    if lo > 0:
        faces.append(np.arange(0, npl))
    if hi < bar.nz:
        faces.append(np.arange(nzs * npl, (nzs + 1) * npl))
    nodes = np.concatenate(faces)
    nsch = nodes.size
    out = np.empty((nsch, 3), dtype=np.int64)
    pos = np.arange(nsch)
    for c in range(3):
        out[:, c] = c * nsch + pos
    return out.ravel()


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def torch_dtype(precision):
    import torch
    return torch.float64 if precision == "f64" else torch.float32


def restrict_free_lib(field_global, bar: Bar, lo: int, hi: int) -> np.ndarray:
    """Global SoA field (3, n_global) -> the library's free-DOF vector [3][free nodes]."""
    npl = (bar.nx + 1) * (bar.ny + 1)
    gids = np.arange(npl * (lo + 1), npl * hi)
    return np.asarray(field_global)[:, gids].reshape(-1)


def synthetic_rom(seed, n_free, n_sch, r, rs, dt, quadratic=False, with_c=False, scale_b=1.0):
    """Seeded synthetic OpInf data: orthonormal Phi, Phi_S; A = -V diag(w^2) V^T with
    w dt <= 1 (stable explicit Newmark); small B, H, c."""
    from paper_2511_20687_amd.inputs import random_normal
    Phi, _ = np.linalg.qr(random_normal(seed, (n_free, r)))
    PhiS = np.linalg.qr(random_normal(seed + 1, (n_sch, rs)))[0] if rs else None
    Vm, _ = np.linalg.qr(random_normal(seed + 2, (r, r)))
    w2 = (np.linspace(0.05, 0.9, r) / dt) ** 2
    A = -(Vm * w2) @ Vm.T
    B = scale_b * (1.0 / dt) ** 2 * 0.01 * random_normal(seed + 3, (r, rs)) if rs else None
    H = 1e-3 * (1.0 / dt) ** 2 * random_normal(seed + 4, (r, r * (r + 1) // 2)) if quadratic else None
    c = 1e-6 * (1.0 / dt) ** 2 * random_normal(seed + 5, (r,)) if with_c else None
    return dict(Phi=Phi, PhiS=PhiS, A=A, B=B, H=H, c=c)
