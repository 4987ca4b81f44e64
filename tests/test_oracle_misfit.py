"""Oracle misfit and its complex-step directional derivatives (the reference for the GPU
adjoint), pinned by central finite differences and by the exact quadratic dependence of J
on the initial velocity (J is a quadratic polynomial in q'0 when the ROM is linear)."""
import numpy as np

from paper_2511_20687_amd.inputs import Bar, gaussian_pulse_u, random_normal, slab_layers, synthetic_rom
from oracle.misfit import directional_derivative, fom_state, misfit, rom_state
from oracle.newmark import FomModel, SubdomainGeometry
from oracle.rom import OpInfModel


def _problem(quadratic):
    bar = Bar(2, 2, 20)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    fom = FomModel(bar, *layers[0], dt)
    g = SubdomainGeometry(bar, *layers[1])
    R = synthetic_rom(21, g.n_free, g.n_sch, 5, 3, dt, quadratic=quadratic, with_c=True)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.4, 0.08)
    v0 = np.zeros_like(u0)
    n, every = 40, 4
    obs = {0: 1e-4 * random_normal(22, (n // every, fom.n_free)), 1: 1e-4 * random_normal(23, (n // every, 5))}
    return bar, dt, fom, g, R, u0, v0, n, every, obs


def _J(quadratic, direction):
    bar, dt, fom, g, R, u0, v0, n, every, obs = _problem(quadratic)
    d = direction

    def J_of(eps):
        A = R["A"] + eps * d["A"]
        H = None if R["H"] is None else R["H"] + eps * d["H"]
        B = R["B"] + eps * d["B"]
        c = R["c"] + eps * d["c"]
        rom = OpInfModel(g, R["Phi"], R["PhiS"], A, H, B, c, dt=dt)
        ul, vl = fom.restrict(u0).astype(complex), fom.restrict(v0).astype(complex)
        ul[fom.free_dofs] += eps * d["u0"]
        vl[fom.free_dofs] += eps * d["v0"]
        s0 = g.restrict(u0)[g.sch_dofs]
        q0 = R["Phi"].T @ g.restrict(u0)[g.free_dofs] + eps * d["q0"]
        qd0 = np.zeros(5) + eps * d["qd0"]
        st = [fom_state(fom, ul, vl), rom_state(rom, q0, qd0, s0)]
        return misfit([fom, rom], st, n, every, obs)
    return J_of


def _direction(seed, quadratic):
    bar, dt, fom, g, R, *_ = _problem(quadratic)
    sc = lambda a: np.abs(a).max() if a is not None and a.size else 1.0
    d = {k: 1e-3 * sc(R[k]) * random_normal(seed + i, R[k].shape) for i, k in enumerate(("A", "B", "c"))}
    d["H"] = None if R["H"] is None else 1e-3 * sc(R["H"]) * random_normal(seed + 7, R["H"].shape)
    d["u0"] = 1e-6 * random_normal(seed + 3, (fom.n_free,))
    d["v0"] = 1e-3 * random_normal(seed + 4, (fom.n_free,))
    d["q0"] = 1e-6 * random_normal(seed + 5, (5,))
    d["qd0"] = 1e-3 * random_normal(seed + 6, (5,))
    return d


def test_complex_step_matches_central_differences():
    d = _direction(30, True)
    J_of = _J(True, d)
    cs = directional_derivative(J_of)
    eps = 1e-4
    fd = (np.real(J_of(eps)) - np.real(J_of(-eps))) / (2 * eps)
    assert abs(cs - fd) <= 1e-6 * abs(cs)


def test_misfit_is_quadratic_in_the_initial_velocity_of_a_linear_rom():
    """Linear ROM and FOM: J(theta + t delta) is a quadratic polynomial in t when delta moves
    only q'0, so J(t) = J0 + t J'(0) + t^2/2 J''  with J'(0) from the complex step."""
    d = _direction(40, False)
    for k in ("A", "B", "c", "u0", "v0", "q0"):
        d[k] = np.zeros_like(d[k])
    J_of = _J(False, d)
    J0, Jp = np.real(J_of(0.0)), directional_derivative(J_of)
    t = 1.0
    J1, Jm = np.real(J_of(t)), np.real(J_of(-t))
    curv = J1 + Jm - 2 * J0
    assert abs((J1 - Jm) / 2 - t * Jp) <= 1e-9 * (abs(J1) + abs(J0))
    assert abs(np.real(J_of(2 * t)) - (J0 + 2 * t * Jp + 2 * curv)) <= 1e-9 * (abs(J1) + abs(J0))
