"""Pins of the oracle's FE discretisation (Sec. 2, App. A.1) against closed forms."""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar
from oracle.fem import SubMesh, assemble, element_matrices, lame
from oracle.newmark import FomModel
from tests._bars import bar_1d


@pytest.fixture(scope="module")
def small():
    bar = Bar(2, 3, 4, Lx=0.1, Ly=0.15, Lz=0.4)
    mesh = SubMesh(bar, 0, bar.nz)
    K, m = assemble(mesh)
    return bar, mesh, K, m


def test_rigid_body_modes_in_null_space(small):
    bar, mesh, K, m = small
    X = mesh.X
    nrm = abs(K).max()
    for c in range(3):
        t = np.zeros((mesh.n_nodes, 3)); t[:, c] = 1.0
        assert np.abs(K @ t.ravel()).max() <= 1e-12 * nrm
    # infinitesimal rotations u = w x X
    for w in np.eye(3):
        u = np.cross(np.broadcast_to(w, X.shape), X)
        assert np.abs(K @ u.ravel()).max() <= 1e-12 * nrm * np.abs(X).max()


def test_symmetry_and_positive_semidefinite(small):
    bar, mesh, K, m = small
    Kd = K.toarray()
    assert np.abs(Kd - Kd.T).max() <= 1e-12 * np.abs(Kd).max()
    ev = np.linalg.eigvalsh(Kd)
    assert ev.min() >= -1e-9 * ev.max()
    # exactly six zero-energy modes (no hourglass modes with full integration)
    assert np.sum(ev < 1e-9 * ev.max()) == 6


def test_patch_test_uniform_strain(small):
    """Linear displacement field -> zero nodal force at interior nodes."""
    bar, mesh, K, m = small
    G = np.array([[1.0, 0.3, -0.2], [0.1, -0.5, 0.4], [0.7, 0.2, 0.9]]) * 1e-3
    u = (mesh.X @ G.T).ravel()
    f = (K @ u).reshape(-1, 3)
    i, j, k = mesh.ijk.T
    interior = (i > 0) & (i < bar.nx) & (j > 0) & (j < bar.ny) & (k > 0) & (k < bar.nz)
    assert interior.sum() > 0
    assert np.abs(f[interior]).max() <= 1e-9 * np.abs(f).max()


def test_boundary_traction_of_uniform_stress(small):
    """The nodal forces of a uniform strain on the face z = L integrate to sigma_zz * area."""
    bar, mesh, K, m = small
    lam, mu = lame(bar.E, bar.nu)
    eps = 1e-4
    u = np.zeros((mesh.n_nodes, 3)); u[:, 2] = eps * mesh.X[:, 2]
    f = (K @ u.ravel()).reshape(-1, 3)
    top = mesh.ijk[:, 2] == bar.nz
    sigma_zz = (lam + 2 * mu) * eps
    assert np.isclose(f[top, 2].sum(), sigma_zz * bar.Lx * bar.Ly, rtol=1e-12)


def test_lumped_mass_totals(small):
    bar, mesh, K, m = small
    V = bar.Lx * bar.Ly * bar.Lz
    for c in range(3):
        assert np.isclose(m[c::3].sum(), bar.rho * V, rtol=1e-13)
    # each node gets rho V_e / 8 from every adjacent element (parallelepipeds)
    Ve = V / (bar.nx * bar.ny * bar.nz)
    count = np.zeros(mesh.n_nodes)
    np.add.at(count, mesh.conn.ravel(), 1.0)
    assert np.allclose(m[0::3], bar.rho * Ve / 8 * count, rtol=1e-13)


def test_element_stiffness_of_unit_cube_trace():
    """tr(K_e) of the unit cube: sum over a,c of int (grad N_a : C : grad N_a) has closed form
    tr = sum_a int |grad N_a|^2 (lam + 3 mu)... checked against the 1-element energy of
    a pure dilatation  u = eps X: energy = 1/2 u^T K u = 1/2 (3 lam + 2 mu) * 3 eps^2 * V."""
    X = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                  [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=float)[None]
    lam, mu = 2.0, 3.0
    Ke, Me = element_matrices(X, lam, mu, 5.0)
    eps = 0.01
    u = (eps * X[0]).ravel()
    energy = 0.5 * u @ Ke[0] @ u
    # sigma = (3 lam + 2 mu) eps I, strain energy density = 1/2 sigma:eps
    assert np.isclose(energy, 0.5 * (3 * lam + 2 * mu) * eps * 3 * eps, rtol=1e-13)
    # consistent mass: total = rho V per component
    assert np.isclose(Me[0][0::3, 0::3].sum(), 5.0, rtol=1e-13)


def test_one_dimensional_reduction():
    """nu = 0 and lateral x, y fixed: a z-field uniform over the cross-section gives the
    1D chain  a_k = (E / (rho h^2)) (u_{k+1} - 2 u_k + u_{k-1})  at every free node."""
    bar = bar_1d(20, L=1.0)
    m = FomModel(bar, 0, bar.nz, dt=1e-7, lateral_fix=(0, 1))
    h = bar.Lz / bar.nz
    z = bar.node_z()
    rng = np.random.default_rng(0)
    layer_vals = rng.standard_normal(bar.nz + 1) * 1e-3
    layer_vals[0] = layer_vals[-1] = 0.0
    ug = np.zeros((3, bar.n_nodes))
    ug[2] = layer_vals[np.round(z / h).astype(int)]
    st = m.initial_state(ug, np.zeros_like(ug))
    a = st.a.reshape(-1, 3)
    k = m.mesh.ijk[:, 2]
    free_nodes = (k > 0) & (k < bar.nz)
    expect = (bar.E / (bar.rho * h * h)) * (layer_vals[k[free_nodes] + 1] - 2 * layer_vals[k[free_nodes]]
                                            + layer_vals[k[free_nodes] - 1])
    assert np.allclose(a[free_nodes, 2], expect, rtol=1e-10, atol=1e-10 * np.abs(expect).max())
    assert np.abs(a[:, :2]).max() == 0.0
