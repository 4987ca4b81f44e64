"""GPU checks of boundary calls of the C ABI against the FP64 oracle and against each other:
the device lift of an OpInf subdomain (osam_get_state), schwarz_step against run, the
convergence sums of Eq. conv_criterion per step, and the binding's stream handling."""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, gaussian_pulse_u, slab_layers
from oracle.newmark import FomModel, SubdomainGeometry
from oracle.rom import OpInfModel
from oracle.schwarz import Coupled, SchwarzOptions
from tests._gpu import lib_free_index, lib_sch_index, rel_err, synthetic_rom

pytestmark = pytest.mark.gpu


def _hybrid(precision="f64", batch=1, kinds=("fom", "opinf"), nz=30, r=6, rs=4, seed=31):
    from paper_2511_20687_amd import osam
    bar = Bar(3, 3, nz)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, len(kinds))
    ctx = osam.Context(0, precision, batch)
    sds = osam.add_bar_subdomains(ctx, bar, layers, dt)
    models = []
    for i, ((lo, hi), kind) in enumerate(zip(layers, kinds)):
        if kind == "fom":
            models.append(FomModel(bar, lo, hi, dt))
            continue
        g = SubdomainGeometry(bar, lo, hi)
        R = synthetic_rom(seed + i, g.n_free, g.n_sch, r, rs, dt, quadratic=True)
        models.append(OpInfModel(g, R["Phi"], R["PhiS"], R["A"], R["H"], R["B"], dt=dt))
        Phi = np.zeros_like(R["Phi"])
        Phi[lib_free_index(bar, lo, hi)] = R["Phi"]
        PhiS = np.zeros_like(R["PhiS"])
        PhiS[lib_sch_index(bar, lo, hi)] = R["PhiS"]
        ctx.set_opinf(sds[i], Phi, PhiS, R["A"], R["H"], R["B"])
    u0 = gaussian_pulse_u(bar, 1e-3, 0.45, 0.06)
    return bar, dt, layers, ctx, sds, models, u0, np.zeros_like(u0)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_device_lift_of_opinf_state(precision, tol):
    """osam_get_state of an OpInf subdomain lifts on the device: Phi q on free DOFs (Sec.
    4.2), zero on constrained DOFs, compared with the oracle's lifted field after 60 coupled
    steps and with Phi times the library's own reduced state; the velocity lifts as Phi q'."""
    bar, dt, layers, ctx, sds, models, u0, v0 = _hybrid(precision)
    n = 60
    print(f"[lift {precision}] oracle", flush=True)
    out = Coupled(models).run(u0, v0, n, SchwarzOptions(), record=())
    st = out["states"][1]
    ctx.set_initial(0, u0, v0)
    print("gpu", flush=True)
    ctx.run(n)
    u, v, a = ctx.get_state(1, 0)
    q, qd, qdd = ctx.get_reduced(1, 0)
    m = models[1]
    ref = m.field(st)                                   # oracle order: 3*node + c
    got = u.T.reshape(-1)                               # [3][n_nodes] -> node-major
    f, s = m.free_dofs, m.sch_dofs
    e_free = rel_err(got[f], ref[f])
    e_phiq = rel_err(got[f], m.Phi @ q)
    e_v = rel_err(v.T.reshape(-1)[f], m.Phi @ st.qd)
    print(f"lift: free {e_free:.2e}, vs Phi q(lib) {e_phiq:.2e}, velocity {e_v:.2e}")
    assert e_free <= (1e-10 if precision == "f64" else 1e-4)
    assert e_v <= (1e-10 if precision == "f64" else 1e-4)
    assert e_phiq <= tol
    assert np.abs(got[s]).max() == 0.0 and np.abs(got[m.dir_dofs]).max() == 0.0


@pytest.mark.parametrize("graph", [0, 32])
def test_schwarz_step_repeated_equals_run(graph):
    """n calls of schwarz_step leave the same bits and iteration counts as one run(n), with
    and without graph replay; the per-step convergence sums abs2 / den2 of the last step
    (Eq. conv_criterion) agree with the oracle's."""
    import torch
    from paper_2511_20687_amd import osam
    n = 40
    res = []
    for mode in ("run", "step"):
        bar, dt, layers, ctx, sds, models, u0, v0 = _hybrid("f64", kinds=("fom", "opinf", "fom"), nz=36)
        ctx.set_graph(graph)
        recs = []
        for i, sd in enumerate(sds):
            z = ctx.sizes(sd)
            t = torch.zeros((1, n + 1, z["r"] or z["n_free"]), dtype=torch.float64, device="cuda:0")
            ctx.set_record(sd, 1, n + 1, u=t)
            recs.append(t)
        ctx.set_initial(0, u0, v0)
        print(f"[graph {graph}] {mode}", flush=True)
        if mode == "run":
            info = ctx.run(n)
            steps = None
        else:
            steps = [ctx.schwarz_step()[0] for _ in range(n)]
            info = [steps[-1]]
        res.append(([t.cpu().numpy() for t in recs], info[0], steps))
    (ra, ia, _), (rb, ib, steps) = res
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y)
    assert ia["total_iters"] == ib["total_iters"] and ia["steps"] == ib["steps"] == n
    # per-step sums against the oracle's controller (HOLD, explicit)
    cp = Coupled(models)
    sts = cp.initial_states(u0, v0)
    for k in range(n):
        sts, oi = cp.step(sts, SchwarzOptions())
        g = steps[k]
        assert g["last_iters"] == oi.iters and bool(g["last_converged"]) == oi.converged
        assert abs(g["den2"] - oi.den2) <= 1e-11 * oi.den2
        assert abs(g["abs2"] - oi.abs2) <= 1e-11 * oi.den2


def test_context_follows_torch_current_stream():
    """A context created under torch.cuda.stream(s) runs on s; the records equal those of a
    context on its own stream bit for bit."""
    import torch
    out = []
    s = torch.cuda.Stream()
    for use_side in (False, True):
        if use_side:
            with torch.cuda.stream(s):
                bar, dt, layers, ctx, sds, models, u0, v0 = _hybrid("f64")
                assert ctx.stream.cuda_stream == s.cuda_stream
                t = torch.zeros((1, 31, ctx.sizes(0)["n_free"]), dtype=torch.float64, device="cuda:0")
                ctx.set_record(0, 1, 31, u=t)
                ctx.set_initial(0, u0, v0)
                ctx.run(30)
                got = t.clone()
            torch.cuda.current_stream().wait_stream(s)
        else:
            bar, dt, layers, ctx, sds, models, u0, v0 = _hybrid("f64")
            t = torch.zeros((1, 31, ctx.sizes(0)["n_free"]), dtype=torch.float64, device="cuda:0")
            ctx.set_record(0, 1, 31, u=t)
            ctx.set_initial(0, u0, v0)
            ctx.run(30)
            got = t.clone()
        out.append(got.cpu().numpy())
    assert np.array_equal(out[0], out[1])
