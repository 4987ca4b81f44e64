"""Small bar set-ups shared by the oracle pin tests (geometry only, no method arithmetic)."""
import numpy as np

from paper_2511_20687_amd.inputs import Bar


def bar_1d(nz, L=1.0, E=1.0e9, rho=1000.0, w=None):
    """Effectively-1D bar of Sec. 5.1: nu = 0, 1 x 1 element cross-section (cubic elements
    by default, so the explicit stability limit is set by the axial waves)."""
    w = L / nz if w is None else w
    return Bar(1, 1, nz, Lx=w, Ly=w, Lz=L, E=E, nu=0.0, rho=rho)


def sine_mode_u(bar, m):
    """u_z = sin(m pi z / L) at every node, (3, n) SoA."""
    z = bar.node_z()
    u = np.zeros((3, bar.n_nodes))
    u[2] = np.sin(m * np.pi * z / bar.Lz)
    return u
