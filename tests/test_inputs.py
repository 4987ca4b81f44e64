"""CPU pins of the seeded input generators that carry a closed form."""
import numpy as np

from paper_2511_20687_amd.inputs import modal_snapshots


def test_modal_snapshots_have_the_stated_svd_and_accelerations():
    dt = 1e-6
    M = modal_snapshots(5, 3000, 400, 12, dt, 3.0)
    U, Udd = M.snapshots()
    # thin SVD: the library SVD's singular values and, up to sign, its left vectors
    P, s, _ = np.linalg.svd(U, full_matrices=False)
    assert np.allclose(s[:12], M.sigma, rtol=1e-12)
    assert s[12] <= 1e-12 * s[0]
    assert np.allclose(np.abs(np.sum(P[:, :12] * M.Phi, axis=0)), 1.0, atol=1e-10)
    # orthonormal modes and coefficient rows orthogonal over the samples
    assert np.allclose(M.Phi.T @ M.Phi, np.eye(12), atol=1e-12)
    C = M.coefficients()
    assert np.allclose(C @ C.T, np.diag(M.sigma ** 2), atol=1e-12)
    # the stated accelerations are the central second difference of the samples (to rounding)
    fd = (U[:, 2:] - 2 * U[:, 1:-1] + U[:, :-2]) / dt ** 2
    assert np.abs(fd - Udd[:, 1:-1]).max() <= 1e-6 * np.abs(Udd).max()
    # the explicit Newmark step from the first sample with zero velocity reproduces the samples
    q, v, a = U[:, 0].copy(), np.zeros(U.shape[0]), Udd[:, 0].copy()
    w2 = M.omega2()
    for j in range(1, 60):
        q = q + dt * v + 0.5 * dt * dt * a
        a_new = M.Phi @ (-w2 * (M.Phi.T @ q))
        v = v + 0.5 * dt * (a + a_new)
        a = a_new
        assert np.abs(q - U[:, j]).max() <= 1e-9 * np.abs(U).max()
    assert len(set(M.freq.tolist())) == 12 and M.freq.min() >= 1 and M.freq.max() < M.T // 8
