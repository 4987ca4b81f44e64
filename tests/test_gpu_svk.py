"""GPU parity of the Saint Venant-Kirchhoff FOM and cubic OpInf (COpInf) against the FP64
oracle (App. A.2 material; Eq. opinf_rom with the cubic term; Sec. 4.1 Schwarz loop).

The pulse has strains of a few percent, so the nonlinear part of the internal force is
visible at far above the parity tolerance (checked: the SVK run differs from the linear
one).  Tolerances: FP64 1e-10 with equal iteration counts; FP32 1e-4.
"""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, gaussian_pulse_u, random_normal, slab_layers
from oracle.newmark import FomModel, SubdomainGeometry
from oracle.opinf import lambda_grid, select_lambda
from oracle.pod import energy_rank, pod
from oracle.rom import OpInfModel
from oracle.schwarz import Coupled, SchwarzOptions
from oracle.svk import SvkFomModel
from tests._gpu import lib_free_index, lib_index_of, lib_sch_index, rel_err, synthetic_rom, torch_dtype

pytestmark = pytest.mark.gpu

BAR = Bar(3, 3, 30)
AMP = 2e-2       # 2 cm over a 6 cm wide pulse: axial strains of about 0.2


def _records(ctx, kinds, n, precision):
    import torch
    recs = []
    for i, kind in enumerate(kinds):
        z = ctx.sizes(i)
        t = torch.zeros((1, n + 1, z["r"] if kind == "opinf" else z["n_free"]), dtype=torch_dtype(precision),
                        device="cuda:0")
        ctx.set_record(i, 1, n + 1, u=t)
        recs.append(t)
    return recs


@pytest.mark.parametrize("precision,tol,lateral_fix", [("f64", 1e-10, ()), ("f64", 1e-10, (0, 1)),
                                                       ("f32", 1e-4, ())])
def test_svk_fom_fom_matches_oracle(precision, tol, lateral_fix):
    from paper_2511_20687_amd import osam
    bar = BAR
    dt = 0.5 * bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    u0 = gaussian_pulse_u(bar, AMP, 0.4, 0.06)
    v0 = np.zeros_like(u0)
    n = 60
    print(f"[svk fom-fom {precision} lateral_fix={lateral_fix}] oracle", flush=True)
    models = [SvkFomModel(bar, lo, hi, dt, lateral_fix=lateral_fix) for lo, hi in layers]
    ref = Coupled(models).run(u0, v0, n, SchwarzOptions(), record=("u",))
    lin = Coupled([FomModel(bar, lo, hi, dt, lateral_fix=lateral_fix) for lo, hi in layers]).run(
        u0, v0, n, SchwarzOptions(), record=("u",))
    assert rel_err(lin["u"][0], ref["u"][0]) > 1e-4          # the nonlinear force matters
    ctx = osam.Context(0, precision, 1)
    osam.add_bar_subdomains(ctx, bar, layers, dt, lateral_fix=lateral_fix, material="svk")
    recs = _records(ctx, ("fom", "fom"), n, precision)
    ctx.set_initial(0, u0, v0)
    print("  gpu", flush=True)
    info = ctx.run(n)
    for i, m in enumerate(models):
        err = rel_err(recs[i][0].double().cpu().numpy()[:, lib_index_of(m)], ref["u"][i])
        print(f"  subdomain {i}: {err:.3e}")
        assert err <= tol
    if precision == "f64":
        assert info[0]["total_iters"] == int(ref["iters"].sum())


def _cubic_rom(seed, g, r, rs, dt):
    R = synthetic_rom(seed, g.n_free, g.n_sch, r, rs, dt, True, False)
    r3 = r * (r + 1) * (r + 2) // 6
    R["C"] = 1e-1 * (1.0 / dt) ** 2 * random_normal(seed + 7, (r, r3))
    return R


@pytest.mark.parametrize("kinds,beta", [(("fom", "opinf"), 0.0), (("opinf", "fom"), 0.25),
                                        (("opinf", "opinf"), 0.0)])
def test_cubic_opinf_couplings_match_oracle(kinds, beta):
    """SVK FOM next to a cubic OpInf subdomain (synthetic operators), explicit and implicit
    (Newton on the cubic reduced equation)."""
    from paper_2511_20687_amd import osam
    bar = BAR
    dt = 0.5 * bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    u0 = gaussian_pulse_u(bar, AMP, 0.4, 0.06)
    v0 = np.zeros_like(u0)
    n = 60
    models, roms = [], {}
    for i, ((lo, hi), kind) in enumerate(zip(layers, kinds)):
        if kind == "fom":
            models.append(SvkFomModel(bar, lo, hi, dt))
        else:
            g = SubdomainGeometry(bar, lo, hi)
            R = roms[i] = _cubic_rom(71 + 10 * i, g, 6, 3, dt)
            models.append(OpInfModel(g, R["Phi"], R["PhiS"], R["A"], R["H"], R["B"], None, dt=dt, beta=beta,
                                     C=R["C"]))
    print(f"[cubic {kinds} beta={beta}] oracle", flush=True)
    ref = Coupled(models).run(u0, v0, n, SchwarzOptions(), record=("u", "q"))
    ctx = osam.Context(0, "f64", 1)
    sds = osam.add_bar_subdomains(ctx, bar, layers, dt, beta=[beta if k == "opinf" else 0.0 for k in kinds],
                                  material=["svk" if k == "fom" else "linear" for k in kinds])
    for i, (lo, hi) in enumerate(layers):
        if kinds[i] != "opinf":
            continue
        R = roms[i]
        Phi = np.zeros_like(R["Phi"])
        Phi[lib_free_index(bar, lo, hi)] = R["Phi"]
        PhiS = np.zeros_like(R["PhiS"])
        PhiS[lib_sch_index(bar, lo, hi)] = R["PhiS"]
        ctx.set_opinf(sds[i], Phi, PhiS, R["A"], R["H"], R["B"])
        ctx.set_opinf_cubic(sds[i], R["C"])
        assert np.array_equal(ctx.get_opinf_cubic(sds[i]), R["C"])
    recs = _records(ctx, kinds, n, "f64")
    ctx.set_initial(0, u0, v0)
    print("  gpu", flush=True)
    info = ctx.run(n)
    for i, (lo, hi) in enumerate(layers):
        got = recs[i][0].cpu().numpy()
        err = rel_err(got, ref["q"][i]) if kinds[i] == "opinf" else rel_err(got[:, lib_free_index(bar, lo, hi)],
                                                                            ref["u"][i])
        print(f"  subdomain {i} ({kinds[i]}): {err:.3e}")
        assert err <= 1e-10
    assert info[0]["total_iters"] == int(ref["iters"].sum())


def test_cubic_learning_pipeline_matches_oracle():
    """SVK FOM-FOM training run -> POD -> cubic least squares -> Alg. 3 -> online SVK-FOM /
    COpInf run, on the GPU and in the oracle: singular values, r_S, lambda*, E(lambda) and
    the online trajectories."""
    import torch
    from paper_2511_20687_amd import osam
    bar = Bar(2, 2, 30)
    dt = 0.5 * bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    u0 = gaussian_pulse_u(bar, AMP, 0.4, 0.06)
    v0 = np.zeros_like(u0)
    T, r = 300, 5
    print("[cubic learning] oracle training run", flush=True)
    models = [SvkFomModel(bar, lo, hi, dt) for lo, hi in layers]
    ref = Coupled(models).run(u0, v0, T - 1, SchwarzOptions(), record=("u", "a", "s", "v"))
    ctx = osam.Context(0, "f64", 1)
    osam.add_bar_subdomains(ctx, bar, layers, dt, material="svk")
    z = ctx.sizes(1)
    U = torch.zeros((1, T, z["n_free"]), dtype=torch.float64, device="cuda:0")
    A = torch.zeros_like(U)
    S = torch.zeros((1, T, z["n_sch"]), dtype=torch.float64, device="cuda:0")
    ctx.set_record(1, 1, T, u=U, a=A, s=S)
    ctx.set_initial(0, u0, v0)
    ctx.run(T - 1)
    g = SubdomainGeometry(bar, *layers[1])
    li = lib_index_of(models[1])
    Uo, Ao, So, Vo = (ref[k][1].T for k in ("u", "a", "s", "v"))
    assert rel_err(U[0].cpu().numpy()[:, li].T, Uo) <= 1e-10
    lo, hi = layers[1]
    V0 = torch.zeros((1, z["n_free"]), dtype=torch.float64, device="cuda:0")
    lams = lambda_grid(11)
    out = ctx.learn_opinf(1, U, A, S, V0, 1, T, form="cubic", r=r, r_s=0, energy_bnd=1 - 1e-6,
                          lambdas=list(lams))
    Phi, sig = pod(Uo, r=r)
    _, sS = pod(So)
    rs = energy_rank(sS, 1 - 1e-6)
    PhiS, _ = pod(So, r=rs)
    traj = dict(Q=Phi.T @ Uo, Qd0=Phi.T @ Vo[:, 0], Qdd=Phi.T @ Ao, Shat=PhiS.T @ So)
    lam, E, ops = select_lambda([traj], lams, form="cubic", dt=dt)
    print("E gpu", out["E_lambda"], "\nE ora", E, "\nlambda*", out["lambda_star"], lam)
    assert out["r"] == r and out["r_s"] == rs
    assert np.allclose(out["sigma"][:r], sig[:r], rtol=1e-8)
    assert out["lambda_star"] == lam
    fin = np.isfinite(E) & (E < 1.0)
    assert fin.any()
    assert np.allclose(out["E_lambda"][fin], E[fin], rtol=1e-5, atol=1e-9)
    Cg = ctx.get_opinf_cubic(1)
    assert np.abs(Cg).max() > 0.0
    # online: the learned operators on both sides
    rom = OpInfModel(g, Phi, PhiS, ops.A, ops.H, ops.B, None, dt=dt, C=ops.C)
    n = 200
    on = Coupled([models[0], rom]).run(u0, v0, n, SchwarzOptions(), record=("u",))
    r0 = torch.zeros((1, n + 1, ctx.sizes(0)["n_free"]), dtype=torch.float64, device="cuda:0")
    r1 = torch.zeros((1, n + 1, r), dtype=torch.float64, device="cuda:0")
    ctx.set_record(0, 1, n + 1, u=r0)
    ctx.set_record(1, 1, n + 1, u=r1)
    ctx.set_initial(0, u0, v0)
    ctx.run(n)
    e0 = rel_err(r0[0].cpu().numpy()[:, lib_index_of(models[0])], on["u"][0])
    Phi_g = ctx.get_opinf(1)["Phi"]
    e1 = rel_err((Phi_g @ r1[0].cpu().numpy().T).T[:, li], on["u"][1])
    print("online errors", e0, e1)
    assert e0 <= 1e-7 and e1 <= 1e-7
