"""Pins of the oracle's Saint Venant-Kirchhoff FE model (App. A.2) and of cubic OpInf
(COpInf: the cubic operator of Eq. opinf_rom, compressed cubic power)."""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, random_normal
from oracle.fem import SubMesh, assemble, lame
from oracle.opinf import fit
from oracle.rom import kron3, kron3_jacobian
from oracle.svk import SvkFomModel, element_energy_and_force, internal_force
from tests._bars import bar_1d


@pytest.fixture(scope="module")
def small():
    bar = Bar(2, 2, 3, Lx=0.1, Ly=0.12, Lz=0.15)
    mesh = SubMesh(bar, 0, bar.nz)
    K, m = assemble(mesh)
    lam, mu = lame(bar.E, bar.nu)
    return bar, mesh, K, lam, mu


def test_linearisation_is_the_linear_elastic_stiffness(small):
    """f(eps u) = eps K u + O(eps^2): the remainder shrinks fourfold when eps halves, and
    relative to eps K u it vanishes with eps (App. A.1 is the linearisation of A.2)."""
    bar, mesh, K, lam, mu = small
    u = random_normal(3, (mesh.n_nodes * 3,))
    Ku = K @ u
    rem = []
    for eps in (1e-6, 5e-7):
        f = internal_force(mesh, eps * u, lam, mu)[0]
        rem.append(np.linalg.norm(f - eps * Ku))
        assert rem[-1] <= 1e-3 * eps * np.linalg.norm(Ku)
    assert 3.6 <= rem[0] / rem[1] <= 4.4


def test_force_is_the_gradient_of_the_stored_energy(small):
    """Complex-step directional derivative of W equals f(u) . v (P = dA/dF)."""
    bar, mesh, K, lam, mu = small
    u = 0.02 * random_normal(4, (mesh.n_nodes * 3,)) * bar.Lz
    v = random_normal(5, (mesh.n_nodes * 3,))
    h = 1e-30
    Wc = internal_force(mesh, u + 1j * h * v, lam, mu)[1]
    f = internal_force(mesh, u, lam, mu)[0]
    assert np.isclose(Wc.imag / h, f @ v, rtol=1e-12)


def test_finite_rigid_rotation_is_stress_free(small):
    """u = (R - I) X for a finite rotation R: E = 0, zero energy and force.  A linear
    model would give forces of the order of K u."""
    bar, mesh, K, lam, mu = small
    th = 0.7
    ax = np.array([1.0, 2.0, 2.0]) / 3.0
    Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    R = np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * Kx @ Kx
    u = (mesh.X @ R.T - mesh.X).ravel()
    f, W = internal_force(mesh, u, lam, mu)
    scale = np.linalg.norm(K @ u)
    assert np.linalg.norm(f) <= 1e-12 * scale
    assert abs(W) <= 1e-12 * abs(0.5 * u @ (K @ u))


def test_frame_indifference(small):
    """A rotation superposed on a deformation rotates the nodal forces: f(R(X+u) - X) = R f(u)."""
    bar, mesh, K, lam, mu = small
    u = 0.05 * random_normal(6, (mesh.n_nodes, 3)) * bar.Lz
    c, s = np.cos(0.9), np.sin(0.9)
    R = np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    f0 = internal_force(mesh, u.ravel(), lam, mu)[0].reshape(-1, 3)
    ur = (mesh.X + u) @ R.T - mesh.X
    f1 = internal_force(mesh, ur.ravel(), lam, mu)[0].reshape(-1, 3)
    assert np.abs(f1 - f0 @ R.T).max() <= 1e-10 * np.abs(f0).max()


def test_force_is_cubic_along_rays(small):
    """f(t u) is a cubic polynomial of t: its fourth difference vanishes, the third does not."""
    bar, mesh, K, lam, mu = small
    u = 0.1 * random_normal(7, (mesh.n_nodes * 3,)) * bar.Lz
    F = [internal_force(mesh, t * u, lam, mu)[0] for t in range(5)]
    d4 = F[4] - 4 * F[3] + 6 * F[2] - 4 * F[1] + F[0]
    d3 = F[3] - 3 * F[2] + 3 * F[1] - F[0]
    assert np.linalg.norm(d4) <= 1e-10 * np.linalg.norm(F[4])
    assert np.linalg.norm(d3) >= 1e-3 * np.linalg.norm(F[1])


def test_kron3_layout_and_jacobian():
    q = np.array([2.0, 3.0, 5.0])
    k = kron3(q)
    assert k.shape == (10,)
    assert np.allclose(k[:4], [8.0, 12.0, 20.0, 18.0])           # (0,0,0) (0,0,1) (0,0,2) (0,1,1)
    assert np.isclose(k[-1], 125.0)
    q = random_normal(8, (4,))
    dq = random_normal(9, (4,))
    h = 1e-30
    assert np.allclose(kron3(q + 1j * h * dq).imag / h, kron3_jacobian(q) @ dq, rtol=1e-13)


def test_cubic_opinf_recovers_the_projected_svk_model():
    """1D-reduced clamped bar with the SVK material (free DOFs: the 8 axial displacements of
    the inner nodes; Phi = I): the FE acceleration -M^-1 f(q) is exactly cubic in q, so COpInf
    fitted without regularisation on 400 random states recovers it: A = -M^-1 K_ff and the
    learned model reproduces the FE accelerations at fresh states (Eq. quadratic_opinf with
    the cubic term; intrusive recovery)."""
    bar = bar_1d(3, L=0.3)
    m = SvkFomModel(bar, 0, bar.nz, dt=1e-6, lateral_fix=(0, 1))
    f = m.free_dofs
    n = f.size
    assert n == 8
    Q = 0.02 * bar.h * random_normal(11, (n, 400))

    def accel(q):
        u = np.zeros(m.n_dofs)
        u[f] = q
        return -m.force(u)[f] / m.m_f

    R = np.stack([accel(Q[:, t]) for t in range(Q.shape[1])], axis=1)
    ops = fit([Q], [R], [None], 0.0, form="cubic")
    A_int = -(m.K_ff.toarray()) / m.m_f[:, None]
    assert np.abs(ops.A - A_int).max() <= 1e-7 * np.abs(A_int).max()
    Qt = 0.02 * bar.h * random_normal(12, (n, 20))
    for t in range(Qt.shape[1]):
        a = accel(Qt[:, t])
        assert np.linalg.norm(ops.rhs(Qt[:, t], np.zeros(0)) - a) <= 1e-7 * np.linalg.norm(a)
    # a quadratic model cannot: the cubic terms are essential at these strains
    quad = fit([Q], [R], [None], 0.0, form="quadratic")
    a = accel(Qt[:, 0])
    assert np.linalg.norm(quad.rhs(Qt[:, 0], np.zeros(0)) - a) >= 1e-5 * np.linalg.norm(a)
