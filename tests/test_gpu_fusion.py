"""Fused sweeps (osam_set_fusion): every subdomain's step of a Schwarz sweep (Alg. 1) in one
launch, the decision of Eq. conv_criterion in the finisher kernel.

Checked against the sequential launches of the same context: identical records and
iteration counts, with host launches and with graph replays (eager work between them),
for FOM-FOM, FOM-OpInf, OpInf-FOM-OpInf (batch 20, fused and batched OpInf paths) and
OpInf-OpInf (the OpInf source's predictor formed from its accepted state; batched path with
both f0 contractions in one launch), in FP64 and FP32, with one and three node layers per FE
thread (FP64 too: its sweep kernel with an OpInf body and three layers per FE thread spills
heavily, and these cases guard it).  FP64 FOM-FOM is also checked
against the oracle.
"""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, draw_pulses
from tests._gpu import lib_index_of, oracle_fom_coupled, rel_err
from tests.test_gpu_graph import _context, _run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kc", [1, 3])
@pytest.mark.parametrize("kinds,precision,batch,n,rom_path", [
    (("fom", "fom"), "f64", 1, 120, 0),
    (("fom", "fom"), "f32", 2, 90, 0),
    (("fom", "opinf"), "f32", 1, 137, 0),
    (("opinf", "fom", "opinf"), "f32", 20, 61, 1),
    (("opinf", "fom", "opinf"), "f32", 20, 61, 2),
    (("opinf", "opinf"), "f32", 3, 90, 0),
    (("opinf", "opinf"), "f32", 20, 61, 2),
    (("opinf", "opinf"), "f64", 2, 90, 0),
    (("fom", "opinf", "fom"), "f64", 2, 70, 0),
])
def test_fused_sweeps_equal_sequential_launches(kinds, precision, batch, n, rom_path, kc):
    bar = Bar(3, 3, 36)
    ctx, sds, layers = _context(kinds, precision, batch, bar)
    if rom_path:
        for i, k in enumerate(kinds):
            if k == "opinf":
                ctx.set_rom_path(sds[i], rom_path)
    print(f"[fusion {kinds} {precision} B={batch} n={n} path={rom_path} kc={kc}]", flush=True)
    ref, info_ref = _run(ctx, sds, bar, batch, n, 0, precision)
    for graph in (0, 16, 16):
        ctx.set_fusion(True, kc)
        got, info = _run(ctx, sds, bar, batch, n, graph, precision)
        for i in range(len(sds)):
            assert np.array_equal(got[i], ref[i]), (graph, i, float(np.abs(got[i] - ref[i]).max()))
        assert [x["steps"] for x in info] == [n] * batch
        assert [x["total_iters"] for x in info] == [x["total_iters"] for x in info_ref]
        ctx.set_fusion(False)
        again, _ = _run(ctx, sds, bar, batch, n, 0, precision)   # eager, unfused, in between
        for i in range(len(sds)):
            assert np.array_equal(again[i], ref[i])
    if kinds == ("fom", "fom") and precision == "f64":
        u0 = draw_pulses(71, 1, s=0.06)[0].u0(bar)
        models, oref = oracle_fom_coupled(bar, layers, bar.explicit_dt(), u0, np.zeros_like(u0), n)
        for i, m in enumerate(models):
            assert rel_err(got[i][0][:, lib_index_of(m)], oref["u"][i]) <= 1e-10


@pytest.mark.parametrize("kinds,precision,batch,n,rom_path", [
    (("fom", "fom"), "f64", 1, 120, 0),
    (("fom", "opinf"), "f32", 1, 137, 0),
    (("opinf", "fom", "opinf"), "f32", 20, 61, 2),
    (("opinf", "opinf"), "f64", 2, 90, 0),
])
def test_fused_sweeps_with_predictor_guess(kinds, precision, batch, n, rom_path):
    """PREDICTOR initial guess (the neighbour's Newmark displacement predictor at t_k): fused
    sweeps and graph replays give the bits and iteration counts of the sequential launches;
    the explicit step leaves that displacement unchanged, so every step converges at its
    second iterate and ends where HOLD's iteration ends (same bits).  FP64 FOM-FOM is also
    checked against the oracle with the same guess."""
    from paper_2511_20687_amd import osam
    bar = Bar(3, 3, 36)
    ctx, sds, layers = _context(kinds, precision, batch, bar)
    if rom_path:
        for i, k in enumerate(kinds):
            if k == "opinf":
                ctx.set_rom_path(sds[i], rom_path)
    pred = osam.Options(guess=1)
    print(f"[fusion predictor {kinds} {precision} B={batch} n={n} path={rom_path}]", flush=True)
    ref, info_ref = _run(ctx, sds, bar, batch, n, 0, precision, opts=pred)
    assert [x["total_iters"] for x in info_ref] == [2 * n] * batch
    hold, _ = _run(ctx, sds, bar, batch, n, 0, precision)
    for i in range(len(sds)):
        assert np.array_equal(hold[i], ref[i]), i
    for graph in (0, 16):
        ctx.set_fusion(True, 1)
        got, info = _run(ctx, sds, bar, batch, n, graph, precision, opts=pred)
        ctx.set_fusion(False)
        for i in range(len(sds)):
            assert np.array_equal(got[i], ref[i]), (graph, i)
        assert [x["total_iters"] for x in info] == [x["total_iters"] for x in info_ref]
    if kinds == ("fom", "fom") and precision == "f64":
        from oracle.schwarz import SchwarzOptions
        u0 = draw_pulses(71, 1, s=0.06)[0].u0(bar)
        models, oref = oracle_fom_coupled(bar, layers, bar.explicit_dt(), u0, np.zeros_like(u0), n,
                                          opts=SchwarzOptions(guess="predictor"))
        assert int(oref["iters"].sum()) == 2 * n
        for i, m in enumerate(models):
            assert rel_err(ref[i][0][:, lib_index_of(m)], oref["u"][i]) <= 1e-10


def test_fusion_rejects_too_many_subdomains():
    from paper_2511_20687_amd import osam
    bar = Bar(3, 3, 60)
    ctx, sds, _ = _context(("fom",) * 5, "f64", 1, bar)
    with pytest.raises(osam.OsamError):
        ctx.set_fusion(True, 1)
    ctx.set_fusion(False)
