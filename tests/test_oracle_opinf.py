"""Pins of the oracle's POD (Sec. 3.1) and OpInf learning (Sec. 3.2, 4.2, Alg. 3)."""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, gaussian_pulse_u, random_normal, slab_layers
from oracle.metrics import rel_l2
from oracle.newmark import FomModel
from oracle.opinf import (amplitude_scale, data_matrix, fit, lambda_grid, ridge, rollout_frozen, select_lambda,
                          trajectory_error)
from oracle.pod import energy_rank, pod, projection_error
from oracle.rom import OpInfModel, Operators, kron2, kron2_jacobian
from oracle.schwarz import Coupled, SchwarzOptions


# ---------------------------------------------------------------- POD
def _orth(seed, n, k):
    q, _ = np.linalg.qr(random_normal(seed, (n, k)))
    return q


def test_pod_recovers_prescribed_svd_and_eckart_young():
    N, T = 60, 25
    L, R = _orth(1, N, T), _orth(2, T, T)
    sig = 2.0 ** -np.arange(T)
    U = L @ np.diag(sig) @ R.T
    for r in (1, 5, 12):
        Phi, s = pod(U, r=r)
        assert np.allclose(s, sig, rtol=1e-12, atol=1e-15)
        assert np.abs(Phi.T @ Phi - np.eye(r)).max() <= 1e-13
        # same subspace as the prescribed left singular vectors
        P1, P2 = Phi @ Phi.T, L[:, :r] @ L[:, :r].T
        assert np.abs(P1 - P2).max() <= 1e-12
        err = np.linalg.norm(U - Phi @ (Phi.T @ U)) ** 2
        assert np.isclose(err, np.sum(sig[r:] ** 2), rtol=1e-10)
        # any other orthonormal r-basis does worse
        V = _orth(3 + r, N, r)
        assert np.linalg.norm(U - V @ (V.T @ U)) ** 2 > err
        assert np.isclose(projection_error(U, Phi), np.sqrt(np.sum(sig[r:] ** 2) / np.sum(sig ** 2)))


def test_energy_rank_rule():
    s = np.sqrt(np.array([50.0, 30.0, 15.0, 4.0, 1.0]))   # energies sum to 100
    assert energy_rank(s, 0.5) == 1
    assert energy_rank(s, 0.80) == 2
    assert energy_rank(s, 0.95) == 3
    assert energy_rank(s, 0.9500001) == 4
    assert energy_rank(s, 1.0) == 5


def test_pod_sign_convention():
    U = np.array([[0.0, 0.0], [-3.0, 0.0], [0.0, 2.0]])
    Phi, _ = pod(U, r=2)
    assert np.all(Phi[np.argmax(np.abs(Phi), axis=0), [0, 1]] > 0)


# ---------------------------------------------------------------- kron2
def test_kron2_layout_and_jacobian():
    q = np.array([2.0, 3.0, 5.0])
    assert np.allclose(kron2(q), [4, 6, 10, 9, 15, 25])
    J = kron2_jacobian(q)
    h = 1e-20
    for k in range(3):
        e = np.zeros(3, dtype=complex); e[k] = 1j * h
        assert np.allclose(J[:, k], kron2(q + e).imag / h)


# ---------------------------------------------------------------- ridge
def test_ridge_closed_form_orthonormal_design():
    D = _orth(7, 40, 6)
    R = random_normal(8, (40, 3))
    for lam in (0.0, 1e-3, 0.7):
        X = ridge(D, R, lam)
        assert np.allclose(X, D.T @ R / (1.0 + lam), rtol=1e-12, atol=1e-14)


def test_ridge_exact_data_and_shrinkage():
    D = random_normal(9, (50, 8))
    X0 = random_normal(10, (8, 2))
    assert np.allclose(ridge(D, D @ X0, 0.0), X0, rtol=1e-11)
    n1 = np.linalg.norm(ridge(D, D @ X0, 1e-2))
    n2 = np.linalg.norm(ridge(D, D @ X0, 1e1))
    assert n2 < n1 < np.linalg.norm(X0) * (1 + 1e-12)


# ---------------------------------------------------------------- OpInf on FOM data
@pytest.fixture(scope="module")
def training():
    """FOM-FOM training run on a small bar; snapshots of subdomain 2."""
    bar = Bar(1, 1, 12, Lx=1.0 / 12, Ly=1.0 / 12, Lz=1.0)
    dt = bar.explicit_dt()
    u0 = gaussian_pulse_u(bar, 1e-3, 0.35, 0.08)
    v0 = np.zeros_like(u0)
    models = [FomModel(bar, lo, hi, dt) for lo, hi in slab_layers(bar.nz, 2)]
    cp = Coupled(models)
    T = 400
    out = cp.run(u0, v0, T - 1, SchwarzOptions(), record=("u", "v", "a", "s"))
    return dict(bar=bar, dt=dt, u0=u0, v0=v0, models=models, cp=cp, out=out, T=T)


def _reduce(tr, i=1, tol=1e-10):
    out = tr["out"]
    U, A, S, V = out["u"][i].T, out["a"][i].T, out["s"][i].T, out["v"][i].T
    _, sig = pod(U)
    r = int(np.sum(sig > tol * sig[0]))
    Phi, _ = pod(U, r=r)
    _, sS = pod(S)
    rS = int(np.sum(sS > tol * sS[0]))
    PhiS, _ = pod(S, r=rS)
    return U, A, S, V, Phi, PhiS


def test_intrusive_operator_recovery(training):
    """Linear FOM data, full-rank bases, lambda = 0: OpInf returns the projected FE operators
    A = -Phi^T M^-1 K_ff Phi, B = -Phi^T M^-1 K_fs Phi_S (finite-dt form of the recovery claim
    in Sec. 3.2)."""
    m = training["models"][1]
    U, A, S, V, Phi, PhiS = _reduce(training)
    ops = fit([Phi.T @ U], [Phi.T @ A], [PhiS.T @ S], 0.0)
    Minv = 1.0 / m.m_f
    K_fs = m.K[m.free_dofs][:, m.sch_dofs].toarray()
    A_int = -Phi.T @ (Minv[:, None] * (m.K_ff @ Phi))
    B_int = -Phi.T @ (Minv[:, None] * K_fs) @ PhiS
    assert np.abs(ops.A - A_int).max() <= 1e-8 * np.abs(A_int).max()
    assert np.abs(ops.B - B_int).max() <= 1e-8 * np.abs(B_int).max()


def test_quadratic_fit_of_linear_data_has_no_quadratic_part(training):
    U, A, S, V, Phi, PhiS = _reduce(training)
    Phi = Phi[:, :6]                     # keep p = r + r(r+1)/2 + r_S below T
    Q, Qdd, Sh = Phi.T @ U, Phi.T @ A, PhiS.T @ S
    # rows of Qdd that the linear model explains exactly: use a synthetic linear target
    Ax = random_normal(11, (6, 6)); Bx = random_normal(12, (6, Sh.shape[0]))
    target = Ax @ Q + Bx @ Sh
    ops = fit([Q], [target], [Sh], 0.0, form="quadratic")
    assert np.abs(ops.H).max() <= 1e-6 * np.abs(ops.A).max()
    assert np.allclose(ops.A, Ax, rtol=1e-6, atol=1e-8 * np.abs(Ax).max())


def test_full_rank_rom_reproduces_training_trajectory(training):
    U, A, S, V, Phi, PhiS = _reduce(training)
    Q, Qdd, Sh = Phi.T @ U, Phi.T @ A, PhiS.T @ S
    ops = fit([Q], [Qdd], [Sh], 0.0)
    Qrom = rollout_frozen(ops, Q[:, 0], Phi.T @ V[:, 0], Qdd[:, 0], Sh, Q.shape[1], training["dt"])
    assert trajectory_error(Qrom, Q) <= 1e-9


def test_coupled_fom_opinf_full_rank_reproduces_fom_fom(training):
    tr = training
    U, A, S, V, Phi, PhiS = _reduce(tr)
    ops = fit([Phi.T @ U], [Phi.T @ A], [PhiS.T @ S], 0.0)
    fom1 = tr["models"][0]
    rom = OpInfModel(tr["models"][1], Phi, PhiS, ops.A, None, ops.B, None, dt=tr["dt"])
    hyb = Coupled([fom1, rom]).run(tr["u0"], tr["v0"], tr["T"] - 1, SchwarzOptions())
    assert rel_l2(hyb["u"][0], tr["out"]["u"][0]) <= 1e-9
    assert rel_l2(hyb["u"][1], tr["out"]["u"][1]) <= 1e-9


def test_lambda_selection_prefers_least_regularisation_on_exact_data(training):
    U, A, S, V, Phi, PhiS = _reduce(training)
    Q, Qdd, Sh = Phi.T @ U, Phi.T @ A, PhiS.T @ S
    traj = dict(Q=Q, Qd0=Phi.T @ V[:, 0], Qdd=Qdd, Shat=Sh)
    lams = lambda_grid(11)
    lam, E, ops = select_lambda([traj], lams, dt=training["dt"])
    assert lam == lams[0]
    assert E[0] == E.min() and E[-1] > 10 * E[0]
    # ties resolve to the smallest lambda; non-finite candidates are penalised
    lam2, E2, _ = select_lambda([traj, traj], lams[:2], dt=training["dt"])
    assert lam2 == lams[0] or E2[0] <= E2[1]
    bad = Operators(np.array([[1e8]]))
    Qb = rollout_frozen(bad, np.ones(1), np.zeros(1), np.zeros(1), None, 4000, 1.0)
    assert trajectory_error(Qb, np.ones((1, 4000))) == np.inf


def test_lambda_grid_matches_paper():
    g = lambda_grid(11)
    assert g[0] == 1e-10 and np.isclose(g[-1], 1.0) and np.allclose(np.diff(np.log10(g)), 1.0)


def test_data_matrix_columns():
    Q = np.arange(6.0).reshape(2, 3)
    Sh = np.ones((1, 3))
    D = data_matrix(Q, Sh, "quadratic", True)
    assert D.shape == (3, 2 + 3 + 1 + 1)
    assert np.allclose(D[:, 2:5], kron2(Q).T)
    assert np.allclose(D[:, -1], 1.0)


def test_normalised_fit_recovers_intrusive_operators(training):
    """At lambda = 0 the change of variables (tau = t/dt, q/alpha) does not move the minimiser."""
    m = training["models"][1]
    U, A, S, V, Phi, PhiS = _reduce(training)
    Q = Phi.T @ U
    alpha = amplitude_scale([Q])
    assert alpha == np.linalg.norm(Q, axis=0).max()
    ops = fit([Q], [Phi.T @ A], [PhiS.T @ S], 0.0, dt=training["dt"], alpha=alpha)
    Minv = 1.0 / m.m_f
    K_fs = m.K[m.free_dofs][:, m.sch_dofs].toarray()
    A_int = -Phi.T @ (Minv[:, None] * (m.K_ff @ Phi))
    B_int = -Phi.T @ (Minv[:, None] * K_fs) @ PhiS
    assert np.abs(ops.A - A_int).max() <= 1e-8 * np.abs(A_int).max()
    assert np.abs(ops.B - B_int).max() <= 1e-8 * np.abs(B_int).max()


@pytest.mark.parametrize("with_c", [False, True])
def test_normalised_fit_is_stationary_point_of_scaled_objective(with_c):
    """First-order conditions of the normalised ridge objective written in physical units:
    J = ||(dt^2/alpha) E||^2 + lambda dt^4 (||A||^2 + alpha^2 ||H||^2 + ||B||^2 + ||c||^2/alpha^2),
    E = Qdd - A Q - H Q^(2) - B S^ - c 1^T, so at the minimiser
    E Q^T = lambda alpha^2 A,  E (Q^(2))^T = lambda alpha^4 H,  E S^^T = lambda alpha^2 B,
    E 1 = lambda c.  Checked on random data with magnitudes far from one."""
    r, rs, T = 4, 2, 60
    Q = 3e-4 * random_normal(41, (r, T))
    Sh = 2e-4 * random_normal(42, (rs, T))
    Qdd = 5e6 * random_normal(43, (r, T))
    dt, lam = 2.5e-6, 1e-3
    alpha = amplitude_scale([Q])
    o = fit([Q], [Qdd], [Sh], lam, form="quadratic", with_c=with_c, dt=dt, alpha=alpha)
    K = kron2(Q)
    E = Qdd - o.A @ Q - o.H @ K - o.B @ Sh
    if with_c:
        E = E - o.c[:, None]
    scale = np.abs(E).max() * np.abs(Q).max() * T
    assert np.abs(E @ Q.T - lam * alpha ** 2 * o.A).max() <= 1e-9 * scale
    assert np.abs(E @ K.T - lam * alpha ** 4 * o.H).max() <= 1e-9 * scale * np.abs(Q).max()
    assert np.abs(E @ Sh.T - lam * alpha ** 2 * o.B).max() <= 1e-9 * scale
    if with_c:
        assert np.abs(E.sum(axis=1) - lam * o.c).max() <= 1e-9 * np.abs(E).max() * T
    # the raw fit (dt = alpha = 1) with the same lambda is a different, over-regularised model
    raw = fit([Q], [Qdd], [Sh], lam, form="quadratic", with_c=with_c)
    assert np.abs(raw.A - o.A).max() > 1e-3 * np.abs(o.A).max()


def test_strided_rollout_equals_every_stride_th_step_of_the_full_rollout():
    """Alg. 3 rollout with snapshots every 3 steps: with a boundary input linear in time the
    interpolation between snapshots is exact, so the strided rollout equals every third
    column of the step-by-step rollout (a dropped or doubled step, or an interpolation with
    the wrong weight, breaks the equality)."""
    from oracle.opinf import Operators, rollout_frozen
    rng = np.random.default_rng(5)
    r, rs, dt, stride, ncol = 4, 2, 1e-3, 3, 9
    Vm = np.linalg.qr(rng.standard_normal((r, r)))[0]
    A = -(Vm * (np.linspace(100.0, 900.0, r) ** 2)) @ Vm.T
    B = rng.standard_normal((r, rs))
    ops = Operators(A=A, H=None, B=B, c=None)
    q0, qd0 = rng.standard_normal(r), rng.standard_normal(r)
    a, b = rng.standard_normal(rs), rng.standard_normal(rs)
    full_n = stride * (ncol - 1) + 1
    S_full = a[:, None] + b[:, None] * np.arange(full_n)[None, :] * dt     # linear in time
    qdd0 = A @ q0 + B @ S_full[:, 0]
    full = rollout_frozen(ops, q0, qd0, qdd0, S_full, full_n, dt)
    strided = rollout_frozen(ops, q0, qd0, qdd0, S_full[:, ::stride], ncol, dt, stride=stride)
    assert np.allclose(strided, full[:, ::stride], rtol=1e-12, atol=1e-14)
    # and stride 1 is the plain rule
    assert np.array_equal(rollout_frozen(ops, q0, qd0, qdd0, S_full, full_n, dt, stride=1), full)


@pytest.mark.parametrize("with_c", [False, True])
def test_normalised_fit_is_a_block_weighted_ridge_independent_of_dt(with_c):
    """What the normalised fit is, in physical units: the ridge problem on the raw data with
    the penalty lambda (alpha^2 ||A||^2 + alpha^4 ||H||^2 + alpha^2 ||B||^2 + ||c||^2)
    (Eq. quadratic_opinf with one scalar lambda, posed in units of the training amplitude).
    dt cancels from the minimiser, and a change of the length unit by s maps the operators as
    A -> A, B -> B, H -> H / s, c -> s c (lambda keeps its meaning).  The weighted problem is
    solved here by its own stacked system, not through fit()."""
    r, rs, T = 4, 2, 60
    Q = 3e-4 * random_normal(51, (r, T))
    Sh = 2e-4 * random_normal(52, (rs, T))
    Qdd = 5e6 * random_normal(53, (r, T))
    lam = 1e-3
    alpha = amplitude_scale([Q])
    o1 = fit([Q], [Qdd], [Sh], lam, form="quadratic", with_c=with_c, dt=2.5e-6, alpha=alpha)
    o2 = fit([Q], [Qdd], [Sh], lam, form="quadratic", with_c=with_c, dt=7.0e-3, alpha=alpha)
    for x, y in ((o1.A, o2.A), (o1.H, o2.H), (o1.B, o2.B)) + (((o1.c, o2.c),) if with_c else ()):
        assert np.abs(x - y).max() <= 1e-9 * np.abs(x).max()
    # the block-weighted ridge written out directly
    D = data_matrix(Q, Sh, "quadratic", with_c)
    w = r * (r + 1) // 2
    weights = np.concatenate([np.full(r, alpha), np.full(w, alpha ** 2), np.full(rs, alpha)]
                             + ([np.ones(1)] if with_c else []))
    p = D.shape[1]
    Daug = np.vstack([D, np.sqrt(lam) * np.diag(weights)])
    Raug = np.vstack([Qdd.T, np.zeros((p, r))])
    X, *_ = np.linalg.lstsq(Daug, Raug, rcond=None)
    O = X.T
    assert np.abs(O[:, :r] - o1.A).max() <= 1e-8 * np.abs(o1.A).max()
    assert np.abs(O[:, r:r + w] - o1.H).max() <= 1e-8 * np.abs(o1.H).max()
    assert np.abs(O[:, r + w:r + w + rs] - o1.B).max() <= 1e-8 * np.abs(o1.B).max()
    if with_c:
        assert np.abs(O[:, -1] - o1.c).max() <= 1e-8 * np.abs(o1.c).max()
    # unit change (metres -> millimetres): every datum scales by s, alpha too
    s = 1e3
    o3 = fit([s * Q], [s * Qdd], [s * Sh], lam, form="quadratic", with_c=with_c, dt=2.5e-6,
             alpha=amplitude_scale([s * Q]))
    assert np.abs(o3.A - o1.A).max() <= 1e-8 * np.abs(o1.A).max()
    assert np.abs(o3.B - o1.B).max() <= 1e-8 * np.abs(o1.B).max()
    assert np.abs(s * o3.H - o1.H).max() <= 1e-8 * np.abs(o1.H).max()
    if with_c:
        assert np.abs(o3.c - s * o1.c).max() <= 1e-8 * np.abs(s * o1.c).max()
