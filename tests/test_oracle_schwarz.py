"""Pins of the oracle's O-SAM controller (Sec. 4.1, Alg. 1, Eq. conv_criterion)."""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, gaussian_pulse_u, slab_layers
from oracle.metrics import rel_l2
from oracle.newmark import FomModel, run_single, single_domain
from oracle.schwarz import Coupled, SchwarzOptions, pointwise_projection, union_field
from oracle.newmark import SubdomainGeometry


def _single_ref(bar, dt, u0, n, beta=0.0):
    sd = single_domain(bar, dt, beta=beta)
    return sd, run_single(sd, u0, np.zeros_like(u0), n)


def _free_ref(m, sd, traj):
    node, comp = m.free_dofs // 3, m.free_dofs % 3
    sdofs = 3 * m.mesh.global_ids[node] + comp
    return np.array([st.u[sdofs] for st in traj])


@pytest.mark.parametrize("S,guess,additive", [(2, "hold", False), (2, "predictor", False), (3, "hold", False),
                                              (3, "hold", True), (3, "predictor", True)])
def test_explicit_schwarz_recovers_single_domain(S, guess, additive):
    """Conforming meshes, explicit Newmark: the converged FOM-FOM iterate equals the
    single-domain FE solution (every free row of K is complete in some subdomain), for the
    multiplicative and the additive variant."""
    bar = Bar(3, 3, 30, Lx=0.1, Ly=0.1, Lz=1.0)
    dt = bar.explicit_dt()
    u0 = gaussian_pulse_u(bar, 1e-3, 0.3, 0.05)
    models = [FomModel(bar, lo, hi, dt) for lo, hi in slab_layers(bar.nz, S)]
    n = 150
    out = Coupled(models).run(u0, np.zeros_like(u0), n, SchwarzOptions(guess=guess, additive=additive))
    sd, traj = _single_ref(bar, dt, u0, n)
    for i, m in enumerate(models):
        assert rel_l2(out["u"][i], _free_ref(m, sd, traj)) <= 1e-13
    # finite iteration counts of the explicit scheme with one step per controller step:
    # PREDICTOR data is already final -> 2; HOLD needs one more sweep (2 or 3).
    if guess == "predictor":
        assert np.all(out["iters"] == 2)
    else:
        assert set(np.unique(out["iters"])) <= {2, 3}
        assert np.any(out["iters"] == 3)
    assert np.all(out["converged"])


def test_implicit_schwarz_converges_geometrically_to_single_domain():
    bar = Bar(2, 2, 24, Lx=0.1, Ly=0.1, Lz=1.0)
    dt = 8.0 * bar.explicit_dt()          # implicit: unconditionally stable
    u0 = gaussian_pulse_u(bar, 1e-3, 0.4, 0.08)
    # narrow overlap (2 layers) so that the Schwarz contraction is slow enough to observe
    models = [FomModel(bar, lo, hi, dt, beta=0.25) for lo, hi in ((0, 13), (11, 24))]
    n = 60
    opts = SchwarzOptions(tol_abs=1e-14, tol_rel=1e-14, max_iter=64)
    out = Coupled(models).run(u0, np.zeros_like(u0), n, opts)
    sd, traj = _single_ref(bar, dt, u0, n, beta=0.25)
    assert np.all(out["converged"])
    assert out["iters"].max() > 3            # genuinely iterative
    for i, m in enumerate(models):
        assert rel_l2(out["u"][i], _free_ref(m, sd, traj)) <= 1e-9


def test_additive_schwarz_converges_to_the_same_fixed_point_more_slowly():
    """Additive variant (Remark additive_sam), implicit Newmark with a narrow overlap: the
    iteration still converges to the single-domain solution, the subdomains of an iteration
    see only the previous iteration's data (with two subdomains the second one's additive
    iterate 2n is its multiplicative iterate n), and it needs more iterations than the
    multiplicative variant (Jacobi vs Gauss-Seidel: close to twice as many for two
    subdomains)."""
    bar = Bar(2, 2, 24, Lx=0.1, Ly=0.1, Lz=1.0)
    dt = 8.0 * bar.explicit_dt()
    u0 = gaussian_pulse_u(bar, 1e-3, 0.4, 0.08)
    models = [FomModel(bar, lo, hi, dt, beta=0.25) for lo, hi in ((0, 13), (11, 24))]
    n = 30
    mult = Coupled(models).run(u0, np.zeros_like(u0), n, SchwarzOptions(tol_abs=1e-14, tol_rel=1e-14, max_iter=200))
    add = Coupled(models).run(u0, np.zeros_like(u0), n,
                              SchwarzOptions(tol_abs=1e-14, tol_rel=1e-14, max_iter=200, additive=True))
    sd, traj = _single_ref(bar, dt, u0, n, beta=0.25)
    assert np.all(add["converged"]) and np.all(mult["converged"])
    for i, m in enumerate(models):
        assert rel_l2(add["u"][i], _free_ref(m, sd, traj)) <= 1e-9
    ratio = add["iters"].sum() / mult["iters"].sum()
    assert 1.4 <= ratio <= 2.3, ratio
    # one controller step with a fixed iteration count: additive iterate 2n of subdomain 1
    # pairs with multiplicative iterate n (two subdomains: Jacobi's even iterates of one
    # subdomain follow the Gauss-Seidel sequence)
    c = Coupled(models)
    st = c.initial_states(u0, np.zeros_like(u0))
    fixed = dict(tol_abs=0.0, tol_rel=0.0, min_iter=1)
    a4, _ = c.step(st, SchwarzOptions(max_iter=4, additive=True, **fixed))
    m2, _ = c.step(st, SchwarzOptions(max_iter=2, **fixed))
    assert rel_l2(a4[1].u, m2[1].u) <= 1e-14


def test_cap_and_unreachable_tolerance():
    bar = Bar(2, 2, 20, Lz=1.0)
    dt = bar.explicit_dt()
    u0 = gaussian_pulse_u(bar, 1e-3, 0.5, 0.05)
    models = [FomModel(bar, lo, hi, dt) for lo, hi in slab_layers(bar.nz, 2)]
    cp = Coupled(models)
    out = cp.run(u0, np.zeros_like(u0), 5, SchwarzOptions(tol_abs=0.0, tol_rel=0.0, max_iter=7))
    assert np.all(out["iters"] == 7) and not np.any(out["converged"])
    one = cp.run(u0, np.zeros_like(u0), 5, SchwarzOptions(min_iter=1, max_iter=1))
    assert np.all(one["iters"] == 1)


def test_pointwise_projection_reproduces_trilinear_fields():
    """Pi of a non-matching source grid is exact for fields trilinear in x, y, z."""
    coarse = Bar(3, 2, 10, Lx=0.1, Ly=0.1, Lz=1.0)
    fine = Bar(5, 4, 30, Lx=0.1, Ly=0.1, Lz=1.0)
    src = SubdomainGeometry(coarse, 0, 7)        # z in [0, 0.7]
    dst = SubdomainGeometry(fine, 12, 30)        # Schwarz face at z = 0.4
    rows = np.arange(dst.sch_dofs.size)
    Pi = pointwise_projection(dst, rows, src)
    X = src.mesh.X
    fld = np.stack([1 + 2 * X[:, 0] - X[:, 1] + 3 * X[:, 2] + 5 * X[:, 0] * X[:, 1] * X[:, 2],
                    X[:, 0] * X[:, 2] - 0.5,
                    X[:, 1] * X[:, 2] + X[:, 0] * X[:, 1]], axis=1).ravel()
    Xd = dst.mesh.X[dst.sch_dofs // 3]
    comp = dst.sch_dofs % 3
    exact = np.choose(comp, [1 + 2 * Xd[:, 0] - Xd[:, 1] + 3 * Xd[:, 2] + 5 * Xd[:, 0] * Xd[:, 1] * Xd[:, 2],
                             Xd[:, 0] * Xd[:, 2] - 0.5,
                             Xd[:, 1] * Xd[:, 2] + Xd[:, 0] * Xd[:, 1]])
    assert np.abs(Pi @ fld - exact).max() <= 1e-13
    # conforming grids -> injection (one unit weight per row)
    src2 = SubdomainGeometry(fine, 0, 20)
    P2 = pointwise_projection(dst, rows, src2)
    assert np.all(np.diff(P2.indptr) == 1) and np.all(P2.data == 1.0)


def test_union_field_reassembles_single_domain():
    bar = Bar(2, 2, 20)
    dt = bar.explicit_dt()
    u0 = gaussian_pulse_u(bar, 1e-3, 0.3, 0.05)
    models = [FomModel(bar, lo, hi, dt) for lo, hi in slab_layers(bar.nz, 2)]
    out = Coupled(models).run(u0, np.zeros_like(u0), 40, SchwarzOptions(), every=40)
    uni = union_field(models, [out["u"][i][-1] for i in range(2)], bar.n_nodes, bar)
    sd, traj = _single_ref(bar, dt, u0, 40)
    ref = traj[-1].u.reshape(-1, 3).T
    interior = ~np.isnan(uni[0])
    assert np.abs(uni[:, interior] - ref[:, interior]).max() <= 1e-15


# ---------------------------------------------------------------- sub-stepping (Xi)
def _substepped(bar, layers, Dt, n_sub, beta=0.0, lateral_fix=()):
    ms = []
    for (lo, hi), ns in zip(layers, n_sub):
        m = FomModel(bar, lo, hi, Dt / ns, beta=beta, lateral_fix=lateral_fix)
        m.n_sub = ns
        ms.append(m)
    return ms


@pytest.mark.parametrize("S,guess", [(2, "hold"), (2, "predictor"), (3, "hold")])
def test_equal_substeps_recover_single_domain_with_the_substep(S, guess):
    """Every subdomain takes m = 3 explicit Newmark steps per controller step (Sec. 4.1,
    Eq. schwarz_discrete with n_1 = n_2): the source's trajectory points coincide with the
    destination's times, and the converged iterate equals the single-domain solution with
    step Dt/3.  Unlike one step per controller step with PREDICTOR, the guess is not the final
    data at the inner sub-steps, so every step takes a third sweep."""
    bar = Bar(3, 3, 30, Lx=0.1, Ly=0.1, Lz=1.0)
    dt = bar.explicit_dt()
    u0 = gaussian_pulse_u(bar, 1e-3, 0.3, 0.05)
    models = _substepped(bar, slab_layers(bar.nz, S), 3 * dt, [3] * S)
    n = 50
    opts = SchwarzOptions(guess=guess, tol_abs=1e-30, tol_rel=1e-14)
    out = Coupled(models).run(u0, np.zeros_like(u0), n, opts)
    sd, traj = _single_ref(bar, dt, u0, 3 * n)
    for i, m in enumerate(models):
        assert rel_l2(out["u"][i], _free_ref(m, sd, traj[::3])) <= 1e-12
    assert np.all(out["converged"])
    assert out["iters"].max() >= 3


def test_equal_substeps_implicit_converge_to_single_domain():
    bar = Bar(2, 2, 24, Lx=0.1, Ly=0.1, Lz=1.0)
    dt = 4.0 * bar.explicit_dt()
    u0 = gaussian_pulse_u(bar, 1e-3, 0.4, 0.08)
    models = _substepped(bar, ((0, 13), (11, 24)), 2 * dt, [2, 2], beta=0.25)
    n = 30
    out = Coupled(models).run(u0, np.zeros_like(u0), n, SchwarzOptions(tol_abs=1e-14, tol_rel=1e-14, max_iter=64))
    sd, traj = _single_ref(bar, dt, u0, 2 * n, beta=0.25)
    assert np.all(out["converged"]) and out["iters"].max() > 3
    for i, m in enumerate(models):
        assert rel_l2(out["u"][i], _free_ref(m, sd, traj[::2])) <= 1e-9


def test_temporal_interpolant_is_exact_for_fields_linear_in_time():
    """Xi on trajectories whose every nodal value is linear in time (value m dt_j at source
    sub-step m): the data at destination sub-step l equal l dt_i for every pair of step
    counts, the guess excluded (sources advanced)."""
    bar = Bar(2, 2, 20)
    Dt = 1.0
    for ni, nj in ((1, 2), (2, 1), (3, 2), (2, 3), (4, 4)):
        models = _substepped(bar, slab_layers(bar.nz, 2), Dt, [ni, nj])
        cp = Coupled(models)
        st = cp.initial_states(np.zeros((3, bar.n_nodes)), np.zeros((3, bar.n_nodes)))
        src = models[1]

        def state(val):
            x = st[1].copy()
            x.u[:] = val
            return x

        traj = [state(m * Dt / nj) for m in range(nj + 1)]
        for l in range(1, ni + 1):
            s = cp.schwarz_data(0, [None, traj], st, "hold", l)
            assert np.allclose(s, l * Dt / ni, rtol=1e-15, atol=1e-15), (ni, nj, l)


def test_mixed_substeps_second_order_in_time():
    """Implicit Newmark (beta = 1/4) with 1 and 2 sub-steps per controller step on the two
    subdomains of the 1D-reduced bar: the converged coupled solution approaches the
    single-domain solution of the same mesh at second order in the controller step (a
    temporal interpolant that held the end value instead of interpolating would be first
    order)."""
    from tests._bars import bar_1d
    bar = bar_1d(40, L=1.0)
    lf = (0, 1)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.45, 0.08)
    t_end = 80 * bar.explicit_dt()
    fine = FomModel(bar, 0, bar.nz, t_end / 640, beta=0.25, lateral_fix=lf)
    ref = run_single(fine, u0, np.zeros_like(u0), 640)[-1].u
    errs = []
    for nsteps in (20, 40, 80):
        Dt = t_end / nsteps
        models = _substepped(bar, ((0, 24), (16, 40)), Dt, [1, 2], beta=0.25, lateral_fix=lf)
        out = Coupled(models).run(u0, np.zeros_like(u0), nsteps, SchwarzOptions(tol_abs=1e-16, tol_rel=1e-13,
                                                                                max_iter=100), every=nsteps)
        m = models[0]
        node, comp = m.free_dofs // 3, m.free_dofs % 3
        exact = ref[3 * m.mesh.global_ids[node] + comp]
        errs.append(np.linalg.norm(out["u"][0][-1] - exact) / np.linalg.norm(exact))
        assert np.all(out["converged"])
    rates = [np.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(rates) >= 1.8, (errs, rates)
