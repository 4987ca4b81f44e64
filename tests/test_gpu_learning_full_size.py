"""Learning at the benchmark size (24x24x240 bar: N = 268,125 free DOFs of the OpInf
subdomain, T = 2000 snapshots, r = 40, boundary basis by the 1 - 1e-6 energy criterion,
Alg. 3 over the 11-value grid) against the oracle, FP64.

The snapshots have a known thin SVD (inputs.modal_snapshots: orthonormal modes times
cosines orthonormal over the samples, exact accelerations), so the oracle's POD is the
closed form itself (the library SVD of a 268,125 x 2000 matrix would take minutes on the
host); the oracle then projects, fits and selects lambda by its own fit / rollout code.
Compared: sigma (1e-9), r_S, lambda*, E(lambda) and the fitted operators.
"""
import numpy as np
import pytest

from oracle.opinf import lambda_grid, select_lambda
from oracle.pod import energy_rank, fix_signs
from paper_2511_20687_amd.inputs import CFG2, modal_snapshots
from tests._gpu import rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_learning_at_benchmark_size_matches_oracle():
    import torch
    from paper_2511_20687_amd import osam
    w = CFG2
    ctx = osam.Context(0, "f64", 1)
    osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    z = ctx.sizes(1)
    N, NS, T, r = z["n_free"], z["n_sch"], w.train_steps, w.r
    print(f"[learning at full size N={N} NS={NS} T={T} r={r}]", flush=True)
    M = modal_snapshots(91, N, T, 60, w.dt, 4.0)     # 60 modes over 4 decades
    MS = modal_snapshots(92, NS, T, 12, w.dt, 9.0)   # boundary traces
    U, Udd = M.snapshots()
    S, _ = MS.snapshots()
    dev = "cuda:0"
    Ut = torch.tensor(np.ascontiguousarray(U.T)[None], device=dev)
    del U
    Uddt = torch.tensor(np.ascontiguousarray(Udd.T)[None], device=dev)
    del Udd
    St = torch.tensor(np.ascontiguousarray(S.T)[None], device=dev)
    V0 = torch.zeros((1, N), dtype=torch.float64, device=dev)
    lams = lambda_grid(11)
    out = ctx.learn_opinf(1, Ut, Uddt, St, V0, 1, T, form="linear", r=r, r_s=0, energy_bnd=1 - 1e-6,
                          lambdas=list(lams))
    del Ut, Uddt, St
    print("  gpu: r_s", out["r_s"], "lambda*", out["lambda_star"], flush=True)
    # oracle: the closed-form POD (sign convention of the oracle), then its fit and Alg. 3
    d = np.sign(fix_signs(M.Phi[:, :r])[0] / M.Phi[0, :r])
    C = M.coefficients()[:r]
    rs = energy_rank(MS.sigma, 1 - 1e-6)
    dS = np.sign(fix_signs(MS.Phi[:, :rs])[0] / MS.Phi[0, :rs])
    traj = dict(Q=d[:, None] * C, Qd0=np.zeros(r), Qdd=d[:, None] * (-M.omega2()[:r, None] * C),
                Shat=dS[:, None] * MS.coefficients()[:rs])
    lam, E, ops = select_lambda([traj], lams, form="linear", dt=w.dt)
    print("  oracle: r_s", rs, "lambda*", lam, flush=True)
    assert out["r"] == r and out["r_s"] == rs
    assert np.allclose(out["sigma"][:r], M.sigma[:r], rtol=1e-9)
    assert out["lambda_star"] == lam
    fin = np.isfinite(E) & (E < 1.0)
    assert fin.any()
    assert np.allclose(out["E_lambda"][fin], E[fin], rtol=1e-5, atol=1e-9)
    g = ctx.get_opinf(1)
    AB_gpu, AB_ora = np.hstack([g["A"], g["B"]]), np.hstack([ops.A, ops.B])
    print(f"  operators: rel err {rel_err(AB_gpu, AB_ora):.2e}", flush=True)
    assert rel_err(AB_gpu, AB_ora) <= 1e-6
    # the basis: the first columns of the closed form, signs fixed
    Phi = g["Phi"]
    assert np.abs(Phi - M.Phi[:, :r] * d[None, :]).max() <= 1e-9
