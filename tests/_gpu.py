"""Helpers for GPU parity tests: run the same coupled problem through the oracle and
through libosam, and bring the library's free-DOF records into the oracle's order."""
import numpy as np

from paper_2511_20687_amd.inputs import Bar
from oracle.newmark import FomModel
from oracle.schwarz import Coupled, SchwarzOptions


def oracle_fom_coupled(bar: Bar, layers, dt, u0, v0, n_steps, opts=None, record=("u",), lateral_fix=()):
    models = [FomModel(bar, lo, hi, dt, lateral_fix=lateral_fix) for lo, hi in layers]
    out = Coupled(models).run(u0, v0, n_steps, opts or SchwarzOptions(), record=record)
    return models, out


def lib_free_index(bar: Bar, lo: int, hi: int) -> np.ndarray:
    """For each oracle free DOF (node-major, dof = 3*node + c), its index in the library's
    free-DOF vector [3][free nodes] (free nodes = layers 1..nzs-1)."""
    from paper_2511_20687_amd.osam import free_dof_map
    return free_dof_map(bar.nx, bar.ny, hi - lo)


def lib_index_of(model) -> np.ndarray:
    """Library free-DOF index of each oracle free DOF of ``model`` (any lateral condition)."""
    from paper_2511_20687_amd.osam import lib_dof_index
    bar = model.bar
    return lib_dof_index(bar.nx, bar.ny, model.z_hi - model.z_lo, model.free_dofs)


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


from paper_2511_20687_amd.inputs import synthetic_rom  # noqa: E402,F401
