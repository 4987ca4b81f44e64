"""Pins of the oracle's Newmark-beta stepping against closed forms (Sec. 4.1, Sec. 5.1)."""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, gaussian_pulse_u
from oracle.newmark import FomModel, run_single, single_domain
from tests._bars import bar_1d, sine_mode_u


@pytest.mark.parametrize("beta", [0.0, 0.25])
def test_exact_discrete_mode(beta):
    """A discrete eigenmode u_k = sin(m pi z_k / L) of the 1D chain evolves as u0 cos(n theta):
    explicit  cos theta = 1 - dt^2 w^2 / 2,  implicit (beta=1/4)  cos theta = (1 - dt^2 w^2/4)/(1 + dt^2 w^2/4),
    w^2 = (4 c^2 / h^2) sin^2(k h / 2)."""
    bar = bar_1d(40)
    c = np.sqrt(bar.E / bar.rho)
    h = bar.Lz / bar.nz
    dt = 0.3 * h / c
    m = 3
    kw = m * np.pi / bar.Lz
    w2 = 4 * c * c / (h * h) * np.sin(kw * h / 2) ** 2
    if beta == 0.0:
        cth = 1 - 0.5 * dt * dt * w2
    else:
        cth = (1 - 0.25 * dt * dt * w2) / (1 + 0.25 * dt * dt * w2)
    theta = np.arccos(cth)
    model = single_domain(bar, dt, beta=beta, lateral_fix=(0, 1))
    u0 = sine_mode_u(bar, m)
    traj = run_single(model, u0, np.zeros_like(u0), 300, record_every=50)
    base = model.restrict(u0)
    base[model.dir_dofs] = 0.0
    for idx, st in enumerate(traj):
        n = 50 * idx
        assert np.abs(st.u - base * np.cos(n * theta)).max() <= 2e-12


@pytest.mark.parametrize("beta", [0.0, 0.25])
def test_algorithmic_energy_conserved(beta):
    """gamma = 1/2, undamped, homogeneous BCs: E_h = 1/2 v'Mv + 1/2 u'Ku + (beta - 1/4) dt^2/2 a'Ma
    is exactly conserved by Newmark-beta; the physical energy stays within that offset."""
    bar = Bar(2, 2, 12, Lx=0.1, Ly=0.1, Lz=0.6)
    dt = bar.explicit_dt()
    model = single_domain(bar, dt, beta=beta)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.3, 0.05)
    traj = run_single(model, u0, np.zeros_like(u0), 400, record_every=20)
    E = np.array([model.energy(st) for st in traj])
    assert np.abs(E - E[0]).max() <= 1e-11 * abs(E[0])
    phys = np.array([0.5 * st.v @ (model.m * st.v) + 0.5 * st.u @ (model.K @ st.u) for st in traj])
    offset = np.array([abs(beta - 0.25) * 0.5 * dt * dt * st.a @ (model.m * st.a) for st in traj])
    assert np.all(np.abs(phys - E[0]) <= offset * (1 + 1e-9) + 1e-12 * abs(E[0]))


def _dalembert(z, t, L, c, f):
    """Clamped-clamped 1D wave: odd 2L-periodic extension F of f, u = (F(z-ct) + F(z+ct))/2.
    (Eq. disp_exact is the special case of one full bar traversal.)"""
    def F(x):
        x = np.mod(x, 2 * L)
        return np.where(x <= L, f(x), -f(2 * L - x))
    return 0.5 * (F(z - c * t) + F(z + c * t))


def test_second_order_convergence_to_analytic_solution():
    L, a, b, s = 1.0, 1e-3, 0.35, 0.06
    f = lambda z: a * np.exp(-(z - b) ** 2 / (2 * s * s))
    errs = []
    for nz in (100, 200):
        bar = bar_1d(nz, L)
        c = np.sqrt(bar.E / bar.rho)
        h = L / nz
        dt = 0.25 * h / c
        T = 0.55 * L / c                  # past one reflection at z = 0
        n = int(round(T / dt))
        model = single_domain(bar, dt, lateral_fix=(0, 1))
        u0 = gaussian_pulse_u(bar, a, b, s)
        st = run_single(model, u0, np.zeros_like(u0), n, record_every=n)[-1]
        z = model.mesh.X[:, 2]
        exact = _dalembert(z, n * dt, L, c, f)
        errs.append(np.abs(st.u[2::3] - exact).max())
    rate = np.log2(errs[0] / errs[1])
    assert errs[1] < 5e-3 * a
    assert 1.8 < rate < 2.3
