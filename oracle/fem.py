"""Oracle: isoparametric hex8 Galerkin finite elements for linear elasticity.

Follows Sec. 2 (Eq. weak_form -> Eq. matrix_vector_form, M phi'' + K phi = f)
with the linear elastic energy of App. A.1 (sigma = lambda tr(eps) I + 2 mu eps).
Readings where the paper is silent:
  * quadrature: full 2x2x2 Gauss rule for stiffness and mass;
  * mass: the explicit Newmark variant lumps the mass (Sec. 5 intro); lumping
    is the row sum of the consistent mass matrix;
  * DOF numbering (oracle-internal): dof = 3*node + component.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from paper_2511_20687_amd.inputs import Bar

# Local hex8 node order: reference-cube corners (xi, eta, zeta).
HEX8_CORNERS = np.array([
    [-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
    [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)

_G = 1.0 / np.sqrt(3.0)
GAUSS_POINTS = np.array([[x, y, z] for z in (-_G, _G) for y in (-_G, _G) for x in (-_G, _G)])
GAUSS_WEIGHTS = np.ones(8)


def lame(E: float, nu: float):
    """Lame constants from Young's modulus and Poisson's ratio."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def shape_values(xi: np.ndarray) -> np.ndarray:
    """Trilinear shape functions N_a(xi) = 1/8 prod (1 + xi_a xi)  -> (8,)."""
    return 0.125 * np.prod(1.0 + HEX8_CORNERS * xi[None, :], axis=1)


def shape_grads_ref(xi: np.ndarray) -> np.ndarray:
    """dN_a/dxi_d at reference point xi -> (8, 3)."""
    c = HEX8_CORNERS
    t = 1.0 + c * xi[None, :]
    g = np.empty((8, 3))
    g[:, 0] = 0.125 * c[:, 0] * t[:, 1] * t[:, 2]
    g[:, 1] = 0.125 * c[:, 1] * t[:, 0] * t[:, 2]
    g[:, 2] = 0.125 * c[:, 2] * t[:, 0] * t[:, 1]
    return g


def elasticity_matrix(lam: float, mu: float) -> np.ndarray:
    """Voigt 6x6 matrix of sigma = lam tr(eps) I + 2 mu eps (engineering shear strains)."""
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def element_matrices(X: np.ndarray, lam: float, mu: float, rho: float):
    """Element stiffness (24x24) and consistent mass (24x24) of hex8 elements.

    X: (E, 8, 3) nodal coordinates.  Element DOF order 3*a + c.
    K_e = sum_g w_g det(J_g) B_g^T D B_g,   M_e = sum_g w_g det(J_g) rho N_g N_g^T (x) I_3.
    """
    nE = X.shape[0]
    D = elasticity_matrix(lam, mu)
    Ke = np.zeros((nE, 24, 24), dtype=X.dtype)
    Me = np.zeros((nE, 24, 24), dtype=X.dtype)
    for g, w in zip(GAUSS_POINTS, GAUSS_WEIGHTS):
        dN = shape_grads_ref(g)                       # (8,3)
        J = np.einsum('ad,eai->eid', dN, X)           # J[e,i,d] = dx_i/dxi_d
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)                       # Jinv[e,d,i] = dxi_d/dx_i
        dNdx = np.einsum('ad,edi->eai', dN, Jinv)     # (E,8,3)
        B = np.zeros((nE, 6, 24), dtype=X.dtype)
        for a in range(8):
            bx, by, bz = dNdx[:, a, 0], dNdx[:, a, 1], dNdx[:, a, 2]
            B[:, 0, 3 * a + 0] = bx
            B[:, 1, 3 * a + 1] = by
            B[:, 2, 3 * a + 2] = bz
            B[:, 3, 3 * a + 0] = by   # gamma_xy
            B[:, 3, 3 * a + 1] = bx
            B[:, 4, 3 * a + 1] = bz   # gamma_yz
            B[:, 4, 3 * a + 2] = by
            B[:, 5, 3 * a + 0] = bz   # gamma_xz
            B[:, 5, 3 * a + 2] = bx
        Ke += w * detJ[:, None, None] * np.einsum('eki,kl,elj->eij', B, D, B)
        N = shape_values(g)
        NN = np.outer(N, N)
        Me += w * rho * detJ[:, None, None] * np.kron(NN, np.eye(3))[None, :, :]
    return Ke, Me


class SubMesh:
    """Structured hex8 mesh of the node layers z_lo..z_hi of a global bar grid.

    Local node (i, j, kl) has id i + (nx+1)(j + (ny+1) kl) and global layer z_lo + kl.
    """

    def __init__(self, bar: Bar, z_lo: int, z_hi: int):
        self.bar, self.z_lo, self.z_hi = bar, z_lo, z_hi
        nx, ny = bar.nx, bar.ny
        self.nzs = z_hi - z_lo
        self.npl = (nx + 1) * (ny + 1)
        self.n_nodes = self.npl * (self.nzs + 1)
        kk, jj, ii = np.meshgrid(np.arange(self.nzs + 1), np.arange(ny + 1), np.arange(nx + 1),
                                 indexing='ij')
        self.ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)   # local node order
        self.X = np.stack([self.ijk[:, 0] * (bar.Lx / nx),
                           self.ijk[:, 1] * (bar.Ly / ny),
                           (self.ijk[:, 2] + z_lo) * (bar.Lz / bar.nz)], axis=1)
        self.global_ids = self.ijk[:, 0] + (nx + 1) * (self.ijk[:, 1] + (ny + 1) * (self.ijk[:, 2] + z_lo))
        ek, ej, ei = np.meshgrid(np.arange(self.nzs), np.arange(ny), np.arange(nx), indexing='ij')
        ei, ej, ek = ei.ravel(), ej.ravel(), ek.ravel()
        conn = []
        for cx, cy, cz in HEX8_CORNERS:
            di, dj, dk = int(cx > 0), int(cy > 0), int(cz > 0)
            conn.append((ei + di) + (nx + 1) * ((ej + dj) + (ny + 1) * (ek + dk)))
        self.conn = np.stack(conn, axis=1)            # (E, 8)

    def node_id(self, i, j, kl):
        return i + (self.bar.nx + 1) * (j + (self.bar.ny + 1) * kl)

    def layer_nodes(self, kl: int) -> np.ndarray:
        return np.arange(kl * self.npl, (kl + 1) * self.npl)

    def lateral_nodes(self) -> np.ndarray:
        i, j = self.ijk[:, 0], self.ijk[:, 1]
        return np.nonzero((i == 0) | (i == self.bar.nx) | (j == 0) | (j == self.bar.ny))[0]


def assemble(mesh: SubMesh, chunk: int = 20000):
    """Global stiffness K (CSR, 3n x 3n) and row-sum-lumped mass vector m (3n).

    K = sum_e P_e^T K_e P_e, assembled element by element (duplicates summed).
    """
    bar = mesh.bar
    lam, mu = lame(bar.E, bar.nu)
    n = 3 * mesh.n_nodes
    K = sp.csr_matrix((n, n))
    m = np.zeros(n)
    edofs_all = (3 * mesh.conn[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 24)
    for s in range(0, mesh.conn.shape[0], chunk):
        conn = mesh.conn[s:s + chunk]
        Xe = mesh.X[conn]                              # (E,8,3)
        Ke, Me = element_matrices(Xe, lam, mu, bar.rho)
        ed = edofs_all[s:s + chunk]
        rows = np.repeat(ed, 24, axis=1).ravel()
        cols = np.tile(ed, (1, 24)).ravel()
        K = K + sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(n, n)).tocsr()
        np.add.at(m, ed.ravel(), Me.sum(axis=2).ravel())
    K.sum_duplicates()
    return K, m
