"""GPU parity of the window engine against the FP64 oracle: subdomains that take several
Newmark steps per controller step with Schwarz data through the temporal interpolant Xi,
and the implicit Newmark scheme (beta = 1/4) on FOM (conjugate gradients) and OpInf
(Newton) subdomains (Sec. 4.1, Eq. conv_criterion, Alg. 1; Sec. 4.2 couplings).

Bar 3 x 3 x 30 (about 300 nodes per subdomain, several workgroup strides of the node loops),
synthetic OpInf operators (seeded, r = 7).  Tolerances: FP64 1e-10 on the recorded
trajectories (the implicit solves stop at a relative residual of 1e-14) and equal iteration
counts; FP32 1e-4.  The convergence sums of every step are compared with the oracle's
(relative 1e-8: they are differences of nearly equal iterates near convergence).
"""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, gaussian_pulse_u, slab_layers
from oracle.newmark import FomModel, SubdomainGeometry
from oracle.rom import OpInfModel
from oracle.schwarz import Coupled, SchwarzOptions
from tests._gpu import lib_free_index, lib_sch_index, rel_err, synthetic_rom, torch_dtype

pytestmark = pytest.mark.gpu

BAR = Bar(3, 3, 30)


def _models(bar, layers, Dt, kinds, betas, subs, roms):
    models = []
    for i, ((lo, hi), kind, beta, ns) in enumerate(zip(layers, kinds, betas, subs)):
        dt = Dt / ns
        if kind == "fom":
            m = FomModel(bar, lo, hi, dt, beta=beta)
        else:
            R = roms[i]
            g = SubdomainGeometry(bar, lo, hi)
            m = OpInfModel(g, R["Phi"], R["PhiS"], R["A"], R["H"], R["B"], R["c"], dt=dt, beta=beta)
        m.n_sub = ns
        models.append(m)
    return models


def _roms(bar, layers, kinds, subs, Dt, quadratic, seed=41, r=7, rs=4):
    roms = {}
    for i, ((lo, hi), kind) in enumerate(zip(layers, kinds)):
        if kind == "opinf":
            g = SubdomainGeometry(bar, lo, hi)
            roms[i] = synthetic_rom(seed + 10 * i, g.n_free, g.n_sch, r, rs, Dt / subs[i], quadratic, False)
    return roms


def _context(bar, layers, Dt, kinds, betas, subs, roms, precision, batch=1, engine=0):
    from paper_2511_20687_amd import osam
    ctx = osam.Context(0, precision, batch)
    sds = osam.add_bar_subdomains(ctx, bar, layers, Dt, beta=list(betas), n_sub=list(subs))
    for i, (lo, hi) in enumerate(layers):
        if kinds[i] != "opinf":
            continue
        R = roms[i]
        Phi = np.zeros_like(R["Phi"])
        Phi[lib_free_index(bar, lo, hi)] = R["Phi"]
        PhiS = np.zeros_like(R["PhiS"])
        PhiS[lib_sch_index(bar, lo, hi)] = R["PhiS"]
        ctx.set_opinf(sds[i], Phi, PhiS, R["A"], R["H"], R["B"], R["c"])
    if engine:
        ctx.set_engine(engine)
    return ctx, sds


def _records(ctx, kinds, n, precision, batch=1):
    import torch
    recs = []
    for i, kind in enumerate(kinds):
        z = ctx.sizes(i)
        t = torch.zeros((batch, n + 1, z["r"] if kind == "opinf" else z["n_free"]), dtype=torch_dtype(precision),
                        device="cuda:0")
        ctx.set_record(i, 1, n + 1, u=t)
        recs.append(t)
    return recs


def _compare(bar, layers, kinds, recs, ref, tol, inst=0):
    for i, (lo, hi) in enumerate(layers):
        got = recs[i][inst].double().cpu().numpy()
        if kinds[i] == "opinf":
            err = rel_err(got, ref["q"][i])
        else:
            err = rel_err(got[:, lib_free_index(bar, lo, hi)], ref["u"][i])
        print(f"  subdomain {i} ({kinds[i]}): {err:.3e}")
        assert err <= tol, (i, err)


def _run_case(kinds, betas, subs, Dt_factor, guess, additive, precision, quadratic=False, n=60, engine=0,
              opts=None):
    from paper_2511_20687_amd import osam
    bar = BAR
    Dt = Dt_factor * bar.explicit_dt()
    layers = slab_layers(bar.nz, len(kinds))
    roms = _roms(bar, layers, kinds, subs, Dt, quadratic)
    models = _models(bar, layers, Dt, kinds, betas, subs, roms)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.4, 0.06)
    v0 = np.zeros_like(u0)
    o = opts or dict()
    print(f"[window {kinds} beta={betas} n_sub={subs} Dt={Dt_factor}dt {guess} additive={additive} "
          f"{precision}] oracle", flush=True)
    ref = Coupled(models).run(u0, v0, n, SchwarzOptions(guess=guess, additive=additive, **o), record=("u", "q"))
    ctx, sds = _context(bar, layers, Dt, kinds, betas, subs, roms, precision, engine=engine)
    recs = _records(ctx, kinds, n, precision)
    ctx.set_initial(0, u0, v0)
    print("  gpu", flush=True)
    info = ctx.run(n, osam.Options(guess=1 if guess == "predictor" else 0, additive=additive, **o))
    return bar, layers, ref, ctx, recs, info


@pytest.mark.parametrize("kinds,quadratic", [(("fom", "fom"), False), (("fom", "opinf"), True),
                                             (("opinf", "fom", "opinf"), True)])
def test_window_engine_explicit_single_step_matches_oracle(kinds, quadratic):
    """The window engine on a context the single-step path also runs (engine = 1)."""
    bar, layers, ref, ctx, recs, info = _run_case(kinds, [0.0] * len(kinds), [1] * len(kinds), 1.0, "hold", False,
                                                  "f64", quadratic, n=80, engine=1)
    _compare(bar, layers, kinds, recs, ref, 1e-10)
    assert info[0]["total_iters"] == int(ref["iters"].sum())
    assert info[0]["steps"] == 80


@pytest.mark.parametrize("guess,additive", [("hold", False), ("predictor", False), ("hold", True)])
def test_implicit_fom_fom_matches_oracle(guess, additive):
    """Implicit Newmark (beta = 1/4) at 16 times the explicit step with tight tolerances: a
    genuinely geometric Schwarz iteration (6 sweeps per step in the oracle).  The relative
    tolerance 1e-10 stays well above the error of the GPU's iterative solves (relative
    residual 1e-14, condition number about 50), so both sides stop at the same iterate."""
    tight = dict(tol_abs=1e-14, tol_rel=1e-10, max_iter=64)
    bar, layers, ref, ctx, recs, info = _run_case(("fom", "fom"), [0.25, 0.25], [1, 1], 16.0, guess, additive,
                                                  "f64", n=40, opts=tight)
    _compare(bar, layers, ("fom", "fom"), recs, ref, 1e-10)
    assert info[0]["total_iters"] == int(ref["iters"].sum())
    assert ref["iters"].max() >= 5
    print("  CG iterations (most per solve):", ctx.solver_stats(0), ctx.solver_stats(1))


@pytest.mark.parametrize("kinds,betas,subs", [
    (("fom", "fom"), (0.0, 0.0), (2, 3)),
    (("fom", "fom"), (0.25, 0.0), (1, 4)),      # implicit-explicit with mixed steps
    (("fom", "fom", "fom"), (0.0, 0.25, 0.0), (3, 1, 2)),
    (("fom", "opinf"), (0.0, 0.25), (4, 1)),
    (("opinf", "fom"), (0.25, 0.0), (2, 3)),
])
def test_substepped_mixed_schemes_match_oracle(kinds, betas, subs):
    """Different Newmark schemes and step counts per subdomain in one controller step:
    Schwarz data through Xi at every sub-step."""
    bar, layers, ref, ctx, recs, info = _run_case(kinds, list(betas), list(subs), 2.0, "hold", False, "f64",
                                                  quadratic=True, n=40)
    _compare(bar, layers, kinds, recs, ref, 1e-10)
    assert info[0]["total_iters"] == int(ref["iters"].sum())


@pytest.mark.parametrize("kinds,quadratic,guess", [
    (("fom", "opinf"), False, "hold"),
    (("fom", "opinf"), True, "predictor"),
    (("opinf", "opinf"), True, "hold"),
    (("opinf", "fom", "opinf"), True, "hold"),
])
def test_implicit_opinf_couplings_match_oracle(kinds, quadratic, guess):
    """Implicit OpInf subdomains: Newton on q+ - beta dt^2 f(q+) = q~ (linear and quadratic)."""
    k = len(kinds)
    bar, layers, ref, ctx, recs, info = _run_case(kinds, [0.25] * k, [1] * k, 2.0, guess, False, "f64",
                                                  quadratic=quadratic, n=40)
    _compare(bar, layers, kinds, recs, ref, 1e-10)
    assert info[0]["total_iters"] == int(ref["iters"].sum())


def test_implicit_fp32_matches_oracle():
    bar, layers, ref, ctx, recs, info = _run_case(("fom", "opinf"), [0.25, 0.25], [1, 2], 2.0, "hold", False,
                                                  "f32", quadratic=True, n=40)
    _compare(bar, layers, ("fom", "opinf"), recs, ref, 1e-4)


def test_convergence_sums_of_each_step_match_oracle():
    """schwarz_step one controller step at a time: the iteration count, the numerator and the
    denominator of Eq. conv_criterion of every step against the oracle's (implicit FOM-FOM
    with a tight tolerance, so the criterion is tested on small differences)."""
    from paper_2511_20687_amd import osam
    bar = BAR
    Dt = 4.0 * bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    kinds = ("fom", "fom")
    models = _models(bar, layers, Dt, kinds, [0.25, 0.25], [1, 2], {})
    u0 = gaussian_pulse_u(bar, 1e-3, 0.4, 0.06)
    v0 = np.zeros_like(u0)
    opts = SchwarzOptions(tol_abs=1e-10, tol_rel=1e-9)
    cp = Coupled(models)
    states = cp.initial_states(u0, v0)
    ctx, _ = _context(bar, layers, Dt, kinds, [0.25, 0.25], [1, 2], {}, "f64")
    ctx.set_initial(0, u0, v0)
    for k in range(25):
        states, info = cp.step(states, opts)
        got = ctx.schwarz_step(osam.Options(tol_abs=1e-10, tol_rel=1e-9))[0]
        assert got["last_iters"] == info.iters and got["steps"] == k + 1
        assert abs(got["den2"] - info.den2) <= 1e-10 * info.den2
        assert abs(got["abs2"] - info.abs2) <= 1e-8 * info.abs2 + 1e-30, (k, got["abs2"], info.abs2)


def test_batch_instances_match_their_own_runs():
    """Three instances with different pulses in one context: each equals the oracle's run of
    its own initial condition (per-instance convergence: iteration counts differ)."""
    from paper_2511_20687_amd import osam
    bar = BAR
    Dt = 3.0 * bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    kinds, betas, subs = ("fom", "opinf"), [0.25, 0.0], [1, 3]
    roms = _roms(bar, layers, kinds, subs, Dt, True)
    models = _models(bar, layers, Dt, kinds, betas, subs, roms)
    n = 30
    ctx, _ = _context(bar, layers, Dt, kinds, betas, subs, roms, "f64", batch=3)
    recs = _records(ctx, kinds, n, "f64", batch=3)
    pulses = [(1e-3, 0.35, 0.05), (2e-3, 0.5, 0.07), (0.5e-3, 0.6, 0.04)]
    refs = []
    for b, (a, c, s) in enumerate(pulses):
        u0 = gaussian_pulse_u(bar, a, c, s)
        refs.append(Coupled(models).run(u0, np.zeros_like(u0), n, SchwarzOptions(), record=("u", "q")))
        ctx.set_initial(b, u0, np.zeros_like(u0))
    info = ctx.run(n, osam.Options())
    for b in range(3):
        _compare(bar, layers, kinds, recs, refs[b], 1e-10, inst=b)
        assert info[b]["total_iters"] == int(refs[b]["iters"].sum())
