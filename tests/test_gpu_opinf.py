"""GPU parity of the OpInf paths (libosam via the C ABI) against the FP64 oracle.

* online couplings with seeded synthetic operators (FOM-OpInf, OpInf-OpInf,
  OpInf-FOM-OpInf; linear and quadratic, with and without the constant term);
* POD of a snapshot matrix with a prescribed spectrum;
* the whole learning pipeline (FOM-FOM training run -> POD -> least squares ->
  Alg. 3 -> online FOM-OpInf run) on a small bar.
Tolerances: FP64 1e-10 unless stated (learning: see each test), FP32 1e-4.
"""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, gaussian_pulse_u, random_normal, slab_layers
from oracle.newmark import FomModel, SubdomainGeometry
from oracle.opinf import lambda_grid, select_lambda
from oracle.pod import energy_rank, pod
from oracle.rom import OpInfModel
from oracle.schwarz import Coupled, SchwarzOptions
from tests._gpu import (lib_free_index, lib_index_of, lib_sch_index, rel_err, restrict_free_lib, synthetic_rom,
                        torch_dtype)

pytestmark = pytest.mark.gpu


def _build(bar, layers, dt, kinds, roms, precision):
    """Oracle models + a library context with the same subdomains and operators."""
    from paper_2511_20687_amd import osam
    models = []
    ctx = osam.Context(0, precision, 1)
    sds = osam.add_bar_subdomains(ctx, bar, layers, dt)
    for i, ((lo, hi), kind) in enumerate(zip(layers, kinds)):
        if kind == "fom":
            models.append(FomModel(bar, lo, hi, dt))
        else:
            g = SubdomainGeometry(bar, lo, hi)
            R = roms[i]
            models.append(OpInfModel(g, R["Phi"], R["PhiS"], R["A"], R["H"], R["B"], R["c"], dt=dt))
            li = lib_free_index(bar, lo, hi)
            Phi_lib = np.zeros_like(R["Phi"])
            Phi_lib[li] = R["Phi"]
            PhiS_lib = None
            if R["PhiS"] is not None:
                PhiS_lib = np.zeros_like(R["PhiS"])
                PhiS_lib[lib_sch_index(bar, lo, hi)] = R["PhiS"]
            ctx.set_opinf(sds[i], Phi_lib, PhiS_lib, R["A"], R["H"], R["B"], R["c"])
    return models, ctx, sds


def _roms_for(bar, layers, kinds, dt, r, rs, quadratic, with_c, seed):
    roms = {}
    for i, ((lo, hi), kind) in enumerate(zip(layers, kinds)):
        if kind != "opinf":
            continue
        g = SubdomainGeometry(bar, lo, hi)
        roms[i] = synthetic_rom(seed + 10 * i, g.n_free, g.n_sch, r, rs, dt, quadratic, with_c)
    return roms


@pytest.mark.parametrize("kinds,quadratic,with_c,precision,tol,guess", [
    (("fom", "opinf"), False, False, "f64", 1e-10, "hold"),
    (("fom", "opinf"), True, True, "f64", 1e-10, "hold"),
    (("opinf", "fom"), True, False, "f64", 1e-10, "hold"),
    (("opinf", "opinf"), True, False, "f64", 1e-10, "hold"),
    (("opinf", "opinf"), True, False, "f64", 1e-10, "predictor"),
    (("opinf", "fom", "opinf"), True, False, "f64", 1e-10, "hold"),
    (("opinf", "fom", "opinf"), True, True, "f64", 1e-10, "predictor"),
    (("fom", "opinf"), True, False, "f32", 1e-4, "hold"),
    (("opinf", "fom", "opinf"), True, False, "f32", 1e-4, "hold"),
])
def test_synthetic_opinf_couplings_match_oracle(kinds, quadratic, with_c, precision, tol, guess):
    import torch
    bar = Bar(3, 3, 36)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, len(kinds))
    roms = _roms_for(bar, layers, kinds, dt, r=9, rs=5, quadratic=quadratic, with_c=with_c, seed=21)
    models, ctx, sds = _build(bar, layers, dt, kinds, roms, precision)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.45, 0.06)
    v0 = np.zeros_like(u0)
    n = 150
    print(f"[{kinds} quad={quadratic} c={with_c} {precision} {guess}] oracle", flush=True)
    ref = Coupled(models).run(u0, v0, n, SchwarzOptions(guess=guess), record=("u", "q"))
    recs = []
    for i, sd in enumerate(sds):
        z = ctx.sizes(sd)
        length = z["r"] if kinds[i] == "opinf" else z["n_free"]
        t = torch.zeros((1, n + 1, length), dtype=torch_dtype(precision), device="cuda:0")
        ctx.set_record(sd, 1, n + 1, u=t)
        recs.append(t)
    ctx.set_initial(0, u0, v0)
    print("gpu", flush=True)
    from paper_2511_20687_amd import osam
    info = ctx.run(n, osam.Options(guess=1 if guess == "predictor" else 0))
    for i, (lo, hi) in enumerate(layers):
        got = recs[i][0].cpu().numpy()
        if kinds[i] == "opinf":
            err = rel_err(got, ref["q"][i])
        else:
            err = rel_err(got[:, lib_free_index(bar, lo, hi)], ref["u"][i])
        print(f"subdomain {i} ({kinds[i]}): {err:.3e}")
        assert err <= tol
    if precision == "f64":
        assert info[0]["total_iters"] == int(ref["iters"].sum())


def test_pod_of_prescribed_spectrum_matches_oracle():
    """Snapshots X = L diag(s) R^T with known singular values (seeded, both sides)."""
    import torch
    from paper_2511_20687_amd import osam
    bar = Bar(2, 2, 24)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    ctx = osam.Context(0, "f64", 1)
    sds = osam.add_bar_subdomains(ctx, bar, layers, dt)
    z = ctx.sizes(1)
    N, NS, T = z["n_free"], z["n_sch"], 60
    L = np.linalg.qr(random_normal(31, (N, T)))[0]
    R = np.linalg.qr(random_normal(32, (T, T)))[0]
    s = 10.0 ** (-np.arange(T) / 8.0)
    U = L @ np.diag(s) @ R.T
    S = random_normal(33, (NS, T)) * 1e-3
    Udd = random_normal(34, (N, T))
    dev = "cuda:0"
    Ut = torch.tensor(U.T[None].copy(), device=dev)    # [1][T][N]
    Uddt = torch.tensor(Udd.T[None].copy(), device=dev)
    St = torch.tensor(S.T[None].copy(), device=dev)
    V0 = torch.zeros((1, N), dtype=torch.float64, device=dev)
    out = ctx.learn_opinf(1, Ut, Uddt, St, V0, 1, T, r=12, r_s=4, lambdas=[1e-8])
    assert out["r"] == 12 and out["r_s"] == 4
    assert np.allclose(out["sigma"][:12], s[:12], rtol=1e-9)
    Phi = ctx.get_opinf(1)["Phi"]
    Phi_o, _ = pod(U, r=12)
    assert np.abs(Phi.T @ Phi - np.eye(12)).max() <= 1e-12
    assert np.abs(Phi - Phi_o).max() <= 1e-9          # same sign convention
    # energy criterion on the boundary basis
    ctx2 = osam.Context(0, "f64", 1)
    osam.add_bar_subdomains(ctx2, bar, layers, dt)
    out2 = ctx2.learn_opinf(1, Ut, Uddt, St, V0, 1, T, r=0, r_s=0, energy=1 - 1e-6, energy_bnd=0.99,
                            lambdas=[1e-8])
    _, sig = pod(U)
    e = np.cumsum(sig ** 2) / np.sum(sig ** 2)
    assert out2["r"] == int(np.searchsorted(e, 1 - 1e-6) + 1)


@pytest.mark.parametrize("r,energy", [(40, None), (0, 1 - 1e-6)])
def test_pod_leading_modes_by_subspace_iteration(r, energy):
    """Gram larger than the block of the subspace iteration (T = 300 snapshots): a fixed
    r = 40 (block 72), and the energy criterion, met only after the block widens from 16
    to 64 leading modes (r = 60).  The boundary basis sees a flat random (Marchenko-Pastur)
    spectrum, the slow case of the iteration.  sigma, Phi and PhiS against the oracle's SVD."""
    import torch
    from paper_2511_20687_amd import osam
    bar = Bar(4, 4, 40)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    ctx = osam.Context(0, "f64", 1)
    osam.add_bar_subdomains(ctx, bar, layers, dt)
    z = ctx.sizes(1)
    N, NS, T = z["n_free"], z["n_sch"], 300
    L = np.linalg.qr(random_normal(41, (N, T)))[0]
    R = np.linalg.qr(random_normal(42, (T, T)))[0]
    s = 10.0 ** (-np.arange(T) / 20.0)
    U = L @ np.diag(s) @ R.T
    S = random_normal(43, (NS, T)) * 1e-3
    Udd = random_normal(44, (N, T))
    dev = "cuda:0"
    Ut = torch.tensor(U.T[None].copy(), device=dev)
    Uddt = torch.tensor(Udd.T[None].copy(), device=dev)
    St = torch.tensor(S.T[None].copy(), device=dev)
    V0 = torch.zeros((1, N), dtype=torch.float64, device=dev)
    print(f"[pod subspace r={r} energy={energy} N={N} NS={NS} T={T}]", flush=True)
    out = ctx.learn_opinf(1, Ut, Uddt, St, V0, 1, T, r=r, r_s=4, energy=energy or 1 - 1e-6, lambdas=[1e-8])
    r_o = r or energy_rank(s, energy)
    assert out["r"] == r_o and out["r_s"] == 4
    assert np.allclose(out["sigma"][:r_o], s[:r_o], rtol=1e-9)
    ops = ctx.get_opinf(1)
    Phi_o, _ = pod(U, r=r_o)
    assert np.abs(ops["Phi"].T @ ops["Phi"] - np.eye(r_o)).max() <= 1e-12
    assert np.abs(ops["Phi"] - Phi_o).max() <= 1e-9
    PhiS_o, _ = pod(S, r=4)
    err_s = np.abs(ops["PhiS"] - PhiS_o).max()
    print(f"  max |Phi - Phi_o| {np.abs(ops['Phi'] - Phi_o).max():.2e}, max |PhiS - PhiS_o| {err_s:.2e}")
    assert err_s <= 1e-8


def _train_oracle_and_gpu(bar, layers, dt, u0, v0, T, precision, lateral_fix=()):
    """FOM-FOM training run on both sides; snapshots of subdomain 1 (U, U'', S, v0)."""
    import torch
    from paper_2511_20687_amd import osam
    models = [FomModel(bar, lo, hi, dt, lateral_fix=lateral_fix) for lo, hi in layers]
    ref = Coupled(models).run(u0, v0, T - 1, SchwarzOptions(), record=("u", "a", "s", "v"))
    ctx = osam.Context(0, precision, 1)
    sds = osam.add_bar_subdomains(ctx, bar, layers, dt, lateral_fix=lateral_fix)
    z = ctx.sizes(1)
    dev = "cuda:0"
    dt_ = torch_dtype(precision)
    U = torch.zeros((1, T, z["n_free"]), dtype=dt_, device=dev)
    A = torch.zeros((1, T, z["n_free"]), dtype=dt_, device=dev)
    S = torch.zeros((1, T, z["n_sch"]), dtype=dt_, device=dev)
    ctx.set_record(1, 1, T, u=U, a=A, s=S)
    ctx.set_initial(0, u0, v0)
    ctx.run(T - 1)
    lo, hi = layers[1]
    V0 = torch.tensor(restrict_free_lib(v0, bar, lo, hi)[None, :], dtype=dt_, device=dev)
    return models, ref, ctx, (U, A, S, V0)


@pytest.mark.parametrize("lateral_fix", [(), (0, 1)])
@pytest.mark.parametrize("form", ["linear", "quadratic"])
def test_learning_pipeline_matches_oracle(form, lateral_fix):
    """Train on a FOM-FOM run, learn OpInf for subdomain 2 with Alg. 3, run FOM-OpInf online.

    Compared: POD singular values, lambda*, the selected E(lambda), and the online
    coupled trajectories (lifted displacement), FP64 on both sides."""
    bar = Bar(2, 2, 40)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.3, 0.06)
    v0 = np.zeros_like(u0)
    T = 400
    r = 8 if form == "linear" else 6
    print(f"[learn {form} lateral {lateral_fix}]", flush=True)
    models, ref, ctx, (U, A, S, V0) = _train_oracle_and_gpu(bar, layers, dt, u0, v0, T, "f64", lateral_fix)
    lams = lambda_grid(11)
    out = ctx.learn_opinf(1, U, A, S, V0, 1, T, form=form, r=r, r_s=0, energy_bnd=1 - 1e-6,
                          lambdas=list(lams))
    # oracle: same steps
    Uo, Ao, So, Vo = (ref[k][1].T for k in ("u", "a", "s", "v"))
    Phi, sig = pod(Uo, r=r)
    from oracle.pod import energy_rank
    _, sS = pod(So)
    rs = energy_rank(sS, 1 - 1e-6)
    PhiS, _ = pod(So, r=rs)
    traj = dict(Q=Phi.T @ Uo, Qd0=Phi.T @ Vo[:, 0], Qdd=Phi.T @ Ao, Shat=PhiS.T @ So)
    lam, E, ops = select_lambda([traj], lams, form=form, dt=dt)
    print("sigma", out["sigma"][:r], sig[:r])
    print("E gpu", out["E_lambda"], "\nE ora", E)
    assert out["r_s"] == rs
    assert np.allclose(out["sigma"][:r], sig[:r], rtol=1e-8)
    assert out["lambda_star"] == lam
    fin = np.isfinite(E) & (E < 1.0)
    assert np.allclose(out["E_lambda"][fin], E[fin], rtol=1e-5, atol=1e-9)
    # online FOM-OpInf on both sides, same IC
    g = SubdomainGeometry(bar, *layers[1], lateral_fix=lateral_fix)
    rom = OpInfModel(g, Phi, PhiS, ops.A, ops.H, ops.B, ops.c, dt=dt)
    on = Coupled([models[0], rom]).run(u0, v0, 300, SchwarzOptions(), record=("u",))
    import torch
    recs = []
    for sd in range(2):
        z = ctx.sizes(sd)
        length = z["n_free"] if sd == 0 else z["r"]
        t = torch.zeros((1, 301, length), dtype=torch.float64, device="cuda:0")
        ctx.set_record(sd, 1, 301, u=t)
        recs.append(t)
    ctx.set_initial(0, u0, v0)
    ctx.run(300)
    fom_u = recs[0][0].cpu().numpy()[:, lib_index_of(models[0])]
    e0 = rel_err(fom_u, on["u"][0])
    Phi_g = ctx.get_opinf(1)["Phi"]
    rom_u = (Phi_g @ recs[1][0].cpu().numpy().T).T[:, lib_index_of(g)]
    e1 = rel_err(rom_u, on["u"][1])
    print("online errors", e0, e1)
    assert e0 <= 1e-7 and e1 <= 1e-7


@pytest.mark.parametrize("form", ["linear", "quadratic"])
def test_learning_two_trajectories_strided_snapshots_matches_oracle(form):
    """Two training trajectories (different pulses), snapshots every 3 time steps: POD
    singular values, r_s, lambda* and E(lambda) of Alg. 3 against the oracle (its rollout
    takes 3 steps per snapshot interval with the boundary input interpolated linearly)."""
    import torch
    from paper_2511_20687_amd import osam
    from oracle.pod import energy_rank
    bar = Bar(2, 2, 40)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    stride, T = 3, 100
    pulses = [gaussian_pulse_u(bar, 1e-3, 0.3, 0.06), gaussian_pulse_u(bar, 1.5e-3, 0.2, 0.05)]
    r = 8 if form == "linear" else 6
    print(f"[learn 2 trajectories stride {stride} {form}]", flush=True)
    models = [FomModel(bar, lo, hi, dt) for lo, hi in layers]
    refs = [Coupled(models).run(u0, np.zeros_like(u0), stride * (T - 1), SchwarzOptions(), every=stride,
                                record=("u", "a", "s", "v")) for u0 in pulses]
    ctx = osam.Context(0, "f64", 2)
    osam.add_bar_subdomains(ctx, bar, layers, dt)
    z = ctx.sizes(1)
    dev = "cuda:0"
    U = torch.zeros((2, T, z["n_free"]), dtype=torch.float64, device=dev)
    A = torch.zeros((2, T, z["n_free"]), dtype=torch.float64, device=dev)
    S = torch.zeros((2, T, z["n_sch"]), dtype=torch.float64, device=dev)
    ctx.set_record(1, stride, T, u=U, a=A, s=S)
    for b, u0 in enumerate(pulses):
        ctx.set_initial(b, u0, np.zeros_like(u0))
    ctx.run(stride * (T - 1))
    V0 = torch.zeros((2, z["n_free"]), dtype=torch.float64, device=dev)
    lams = lambda_grid(11)
    out = ctx.learn_opinf(1, U, A, S, V0, 2, T, form=form, r=r, r_s=0, energy_bnd=1 - 1e-6,
                          lambdas=list(lams), stride=stride)
    Uo = np.hstack([rf["u"][1].T for rf in refs])
    Ao = np.hstack([rf["a"][1].T for rf in refs])
    So = np.hstack([rf["s"][1].T for rf in refs])
    Phi, sig = pod(Uo, r=r)
    _, sS = pod(So)
    rs = energy_rank(sS, 1 - 1e-6)
    PhiS, _ = pod(So, r=rs)
    trajs = [dict(Q=Phi.T @ rf["u"][1].T, Qd0=Phi.T @ rf["v"][1][0], Qdd=Phi.T @ rf["a"][1].T,
                  Shat=PhiS.T @ rf["s"][1].T) for rf in refs]
    lam, E, _ = select_lambda(trajs, lams, form=form, dt=dt, stride=stride)
    print("E gpu", out["E_lambda"], "\nE ora", E)
    assert out["r_s"] == rs
    assert np.allclose(out["sigma"][:r], sig[:r], rtol=1e-8)
    assert out["lambda_star"] == lam
    fin = np.isfinite(E) & (E < 1.0)
    assert fin.any()
    assert np.allclose(out["E_lambda"][fin], E[fin], rtol=1e-5, atol=1e-9)
