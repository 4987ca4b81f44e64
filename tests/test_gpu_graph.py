"""Graph mode of run (osam_set_graph): captured sweeps replayed, on one stream or with the FOM
and OpInf kernels of a sweep on two streams and the decision in the finisher kernel (Alg. 1,
Eq. conv_criterion).

Every replay is checked against the sequential launches of the same context: identical
records (the kernels compute the same values) and identical iteration counts; between the
replays the context does eager (non-graph) work and host synchronisations.  FP64 FOM-FOM
is also checked against the oracle.
"""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, draw_pulses, gaussian_pulse_u, slab_layers
from oracle.newmark import SubdomainGeometry
from tests._gpu import lib_free_index, lib_index_of, lib_sch_index, oracle_fom_coupled, rel_err, synthetic_rom

pytestmark = pytest.mark.gpu


def _context(kinds, precision, batch, bar, seed=61):
    from paper_2511_20687_amd import osam
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, len(kinds))
    ctx = osam.Context(0, precision, batch)
    sds = osam.add_bar_subdomains(ctx, bar, layers, dt)
    for i, (lo, hi) in enumerate(layers):
        if kinds[i] != "opinf":
            continue
        g = SubdomainGeometry(bar, lo, hi)
        R = synthetic_rom(seed + i, g.n_free, g.n_sch, 8, 4, dt, quadratic=True, with_c=True)
        Phi = np.zeros_like(R["Phi"])
        Phi[lib_free_index(bar, lo, hi)] = R["Phi"]
        PhiS = np.zeros_like(R["PhiS"])
        PhiS[lib_sch_index(bar, lo, hi)] = R["PhiS"]
        ctx.set_opinf(sds[i], Phi, PhiS, R["A"], R["H"], R["B"], R["c"])
    return ctx, sds, layers


def _run(ctx, sds, bar, batch, n, graph, precision, streams=1, opts=None):
    import torch
    dtp = torch.float64 if precision == "f64" else torch.float32
    recs = []
    for sd in sds:
        z = ctx.sizes(sd)
        length = z["r"] if z["r"] > 0 else z["n_free"]
        t = torch.zeros((batch, n + 1, length), dtype=dtp, device="cuda:0")
        ctx.set_record(sd, 1, n + 1, u=t)
        recs.append(t)
    for b, p in enumerate(draw_pulses(71, batch, s=0.06)):
        u0 = p.u0(bar)
        ctx.set_initial(b, u0, np.zeros_like(u0))
    ctx.set_graph(graph, streams)
    info = ctx.run(n) if opts is None else ctx.run(n, opts)
    ctx.sync()
    return [t.cpu().numpy() for t in recs], info


@pytest.mark.parametrize("streams", [1, 2])
@pytest.mark.parametrize("kinds,precision,batch,n,rounds", [
    (("fom", "fom"), "f64", 1, 150, 16),
    (("fom", "opinf"), "f32", 1, 137, 16),
    (("opinf", "fom", "opinf"), "f32", 20, 61, 6),
    (("opinf", "opinf"), "f32", 3, 90, 2),
])
def test_graph_replays_equal_sequential_launches(kinds, precision, batch, n, rounds, streams):
    bar = Bar(3, 3, 36)
    ctx, sds, layers = _context(kinds, precision, batch, bar)
    print(f"[graph {kinds} {precision} B={batch} n={n} rounds={rounds} streams={streams}]", flush=True)
    ref, info_ref = _run(ctx, sds, bar, batch, n, 0, precision)
    for rep in range(3):                          # replays with eager work in between
        got, info = _run(ctx, sds, bar, batch, n, rounds, precision, streams)
        for i in range(len(sds)):
            assert np.array_equal(got[i], ref[i]), (rep, i, float(np.abs(got[i] - ref[i]).max()))
        assert [x["steps"] for x in info] == [n] * batch
        assert [x["total_iters"] for x in info] == [x["total_iters"] for x in info_ref]
        again, _ = _run(ctx, sds, bar, batch, n, 0, precision)
        for i in range(len(sds)):
            assert np.array_equal(again[i], ref[i])
    if kinds == ("fom", "fom"):
        u0 = draw_pulses(71, 1, s=0.06)[0].u0(bar)
        models, oref = oracle_fom_coupled(bar, layers, bar.explicit_dt(), u0, np.zeros_like(u0), n)
        for i, m in enumerate(models):
            assert rel_err(got[i][0][:, lib_index_of(m)], oref["u"][i]) <= 1e-10
        assert info[0]["total_iters"] == int(oref["iters"].sum())


def test_autotune_choice_is_valid_cached_and_result_preserving():
    """osam_autotune picks a launch configuration by trial runs; a second context of the same
    configuration gets it from the cache; runs after tuning agree with the default launch
    configuration (FP32 bar: the batched OpInf path rounds in another order)."""
    bar = Bar(3, 3, 36)
    kinds, batch, n = ("fom", "opinf"), 4, 80
    ref_ctx, sds, _ = _context(kinds, "f32", batch, bar)
    ref, info_ref = _run(ref_ctx, sds, bar, batch, n, 0, "f32")
    ctx, sds, _ = _context(kinds, "f32", batch, bar)
    for b, p in enumerate(draw_pulses(71, batch, s=0.06)):
        u0 = p.u0(bar)
        ctx.set_initial(b, u0, np.zeros_like(u0))
    t = ctx.autotune(trial_steps=10)
    print("tuning", t, flush=True)
    assert not t["from_cache"] and t["ms_per_step"] > 0
    assert t["fe"][0][0] in (64, 128, 256, 1024) and t["rom_path"][1] in (1, 2)
    assert t["graph"] in ((0, 1), (32, 1), (128, 1), (32, 2))
    assert ctx.get_fe_launch(sds[0])[0] == t["fe"][0][0] and ctx.rom_path(sds[1]) == t["rom_path"][1]
    got, info = _run_tuned(ctx, sds, bar, batch, n, t)
    for i in range(len(sds)):
        assert max(rel_err(got[i][b], ref[i][b]) for b in range(batch)) <= 1e-5
    assert [x["total_iters"] for x in info] == [x["total_iters"] for x in info_ref]
    ctx2, sds2, _ = _context(kinds, "f32", batch, bar)
    for b, p in enumerate(draw_pulses(71, batch, s=0.06)):
        u0 = p.u0(bar)
        ctx2.set_initial(b, u0, np.zeros_like(u0))
    t2 = ctx2.autotune(trial_steps=10)
    assert t2["from_cache"] and t2["fe"] == t["fe"] and t2["rom_path"] == t["rom_path"] and t2["graph"] == t["graph"]


def _run_tuned(ctx, sds, bar, batch, n, t):
    """_run without touching the launch mode the tuner chose."""
    import torch
    recs = []
    for sd in sds:
        z = ctx.sizes(sd)
        length = z["r"] if z["r"] > 0 else z["n_free"]
        r = torch.zeros((batch, n + 1, length), dtype=torch.float32, device="cuda:0")
        ctx.set_record(sd, 1, n + 1, u=r)
        recs.append(r)
    for b, p in enumerate(draw_pulses(71, batch, s=0.06)):
        u0 = p.u0(bar)
        ctx.set_initial(b, u0, np.zeros_like(u0))
    info = ctx.run(n)
    ctx.sync()
    return [r.cpu().numpy() for r in recs], info
