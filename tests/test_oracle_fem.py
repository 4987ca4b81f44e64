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


def test_interior_stencil_x_rows_sum_to_a_diagonal_block_and_resolve_in_x():
    """The x-resolved form of the interior stencil that the FE kernels add in: on a uniform
    box grid (unequal hx, hy, hz) the nine blocks K_(+-1,dy,dz) of an interior node sum to a
    diagonal block (the off-diagonal edge and corner entries cancel in pairs), the same for
    dx = +1 and -1, and for any
    field sum_d K_d (u_{i+d} - u_i) = S_0(i) + S_-1(i-1) + S_+1(i+1)
    + K_x ((u_{i-1} - u_i) + (u_{i+1} - u_i)), with S_dx(j) = sum over the (dy, dz) rows of
    K_(dx,dy,dz) (u_row(j) - u(j)) formed at column j and K_x that row sum."""
    bar = Bar(6, 5, 6, Lx=0.12, Ly=0.2, Lz=0.45)
    mesh = SubMesh(bar, 0, bar.nz)
    K, _ = assemble(mesh)
    K = K.tocsr()

    def block(n, m):
        return K[3 * n:3 * n + 3, 3 * m:3 * m + 3].toarray()

    i, j, k = 3, 2, 3
    node = mesh.node_id(i, j, k)
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    C = {d: block(node, mesh.node_id(i + d[0], j + d[1], k + d[2])) for d in offs if d != (0, 0, 0)}
    scale = np.abs(C[(1, 0, 0)]).max()
    for dx in (-1, 1):
        Kx = sum(C[(dx, dy, dz)] for dz in (-1, 0, 1) for dy in (-1, 0, 1))
        assert np.abs(Kx - np.diag(np.diag(Kx))).max() <= 1e-12 * scale
        assert np.all(np.abs(np.diag(Kx)) > 1e-3 * scale)
    Kx = sum(C[(1, dy, dz)] for dz in (-1, 0, 1) for dy in (-1, 0, 1))
    Kxm = sum(C[(-1, dy, dz)] for dz in (-1, 0, 1) for dy in (-1, 0, 1))
    assert np.abs(Kxm - Kx).max() <= 1e-12 * scale   # one K serves both sides
    rng = np.random.default_rng(5)
    u = rng.standard_normal((mesh.n_nodes, 3))

    def U(a, b, c):
        return u[mesh.node_id(a, b, c)]

    direct = sum(C[d] @ (U(i + d[0], j + d[1], k + d[2]) - U(i, j, k)) for d in C)

    def S(dx, col):   # formed at column col from its own values
        return sum(C[(dx, dy, dz)] @ (U(col, j + dy, k + dz) - U(col, j, k))
                   for dz in (-1, 0, 1) for dy in (-1, 0, 1) if (dy, dz) != (0, 0))

    resolved = S(0, i) + S(-1, i - 1) + S(1, i + 1) + Kx @ ((U(i - 1, j, k) - U(i, j, k)) + (U(i + 1, j, k) - U(i, j, k)))
    assert np.abs(resolved - direct).max() <= 1e-12 * np.abs(direct).max()


@pytest.mark.parametrize("a,b", [(0, 1), (1, 0), (1, 2), (2, 1), (0, 2), (2, 0)])
def test_simple_shear_energy(small, a, b):
    """Simple shear u_a = g x_b (engineering shear strain g, App. A.1): the strain energy
    1/2 u^T K u equals 1/2 mu g^2 V, the energy density of sigma = lam tr(eps) I + 2 mu eps
    for a traceless strain with eps_ab = eps_ba = g/2.  A shear modulus taken as 2 mu on the
    engineering strains (or mu/2 on tensor ones) doubles (halves) the energy."""
    bar, mesh, K, m = small
    lam, mu = lame(bar.E, bar.nu)
    g = 1e-3
    u = np.zeros((mesh.n_nodes, 3))
    u[:, a] = g * mesh.X[:, b]
    W = 0.5 * u.ravel() @ (K @ u.ravel())
    V = bar.Lx * bar.Ly * bar.Lz
    assert np.isclose(W, 0.5 * mu * g * g * V, rtol=1e-12)


def test_shear_traction_on_end_face(small):
    """u_x = g z: the nodal forces on the face z = L sum to the shear traction times the
    area, sigma_xz A = mu g Lx Ly, and vanish in y and z (on z = 0 the opposite force)."""
    bar, mesh, K, m = small
    lam, mu = lame(bar.E, bar.nu)
    g = 2e-4
    u = np.zeros((mesh.n_nodes, 3))
    u[:, 0] = g * mesh.X[:, 2]
    f = (K @ u.ravel()).reshape(-1, 3)
    top = mesh.ijk[:, 2] == bar.nz
    bot = mesh.ijk[:, 2] == 0
    area = bar.Lx * bar.Ly
    assert np.isclose(f[top, 0].sum(), mu * g * area, rtol=1e-12)
    assert np.isclose(f[bot, 0].sum(), -mu * g * area, rtol=1e-12)
    assert abs(f[top, 1].sum()) <= 1e-12 * mu * g * area
    assert abs(f[top, 2].sum()) <= 1e-12 * mu * g * area


def test_general_uniform_strain_energy(small):
    """Any uniform strain eps (symmetric part of a displacement gradient G): energy
    1/2 u^T K u = 1/2 (lam tr(eps)^2 + 2 mu eps:eps) V (App. A.1 energy density)."""
    bar, mesh, K, m = small
    lam, mu = lame(bar.E, bar.nu)
    G = np.array([[0.3, -1.1, 0.4], [0.2, -0.5, 0.9], [-0.7, 0.6, 0.8]]) * 1e-4
    u = mesh.X @ G.T
    eps = 0.5 * (G + G.T)
    W = 0.5 * u.ravel() @ (K @ u.ravel())
    V = bar.Lx * bar.Ly * bar.Lz
    assert np.isclose(W, 0.5 * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps)) * V, rtol=1e-12)
