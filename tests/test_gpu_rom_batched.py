"""GPU parity of the batched OpInf path and of the BF16-H precision.

The batched path evaluates f0 = A q + H (q (x) q) + c once per controller step on the
matrix cores over tiles of 16 instances (Sec. 4.2, Eq. opinf_model_schwarz; the explicit
predictor q(t_k) is fixed within a step) and sums g^ of FOM-fed faces over splits of the
face DOFs.  Checked against the FP64 oracle on sampled instances of a ragged batch
(20 = 16 + 4) and against the fused path on every instance.  The BF16-H precision rounds
the operands of the quadratic contraction only; its error is reported against the oracle
with a quadratic term made strong enough (~1 % of the linear one) that a wrong BF16
fragment layout could not hide.
"""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, draw_pulses, slab_layers
from oracle.newmark import FomModel, SubdomainGeometry
from oracle.rom import OpInfModel
from oracle.schwarz import Coupled, SchwarzOptions
from tests._gpu import lib_free_index, lib_sch_index, rel_err, synthetic_rom

pytestmark = pytest.mark.gpu
B = 20
CHECK = (0, 9, 19)
N_STEPS = 120


def _problem(kinds, quadratic, with_c, h_scale=1.0):
    bar = Bar(3, 3, 36)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, len(kinds))
    roms = {}
    for i, (lo, hi) in enumerate(layers):
        if kinds[i] == "opinf":
            g = SubdomainGeometry(bar, lo, hi)
            R = synthetic_rom(41 + 10 * i, g.n_free, g.n_sch, 9, 5, dt, quadratic, with_c)
            if quadratic:
                R["H"] = R["H"] * h_scale
            roms[i] = R
    return dict(bar=bar, dt=dt, layers=layers, kinds=kinds, roms=roms, pulses=draw_pulses(43, B, s=0.06))


def _gpu_run(P, precision, path, n=N_STEPS, keep=False):
    import torch
    from paper_2511_20687_amd import osam
    bar, layers, kinds = P["bar"], P["layers"], P["kinds"]
    ctx = osam.Context(0, precision, B)
    sds = osam.add_bar_subdomains(ctx, bar, layers, P["dt"])
    for i, (lo, hi) in enumerate(layers):
        if kinds[i] != "opinf":
            continue
        R = P["roms"][i]
        Phi = np.zeros_like(R["Phi"])
        Phi[lib_free_index(bar, lo, hi)] = R["Phi"]
        PhiS = np.zeros_like(R["PhiS"])
        PhiS[lib_sch_index(bar, lo, hi)] = R["PhiS"]
        ctx.set_opinf(sds[i], Phi, PhiS, R["A"], R["H"], R["B"], R["c"])
        ctx.set_rom_path(sds[i], path)
    recs = []
    for i, sd in enumerate(sds):
        z = ctx.sizes(sd)
        length = z["r"] if kinds[i] == "opinf" else z["n_free"]
        t = torch.zeros((B, n + 1, length), dtype=torch.float32, device="cuda:0")
        ctx.set_record(sd, 1, n + 1, u=t)
        recs.append(t)
    for b, p in enumerate(P["pulses"]):
        u0 = p.u0(bar)
        ctx.set_initial(b, u0, np.zeros_like(u0))
    ctx.run(n)
    used = [ctx.rom_path(sd) for sd in sds]
    if keep:
        return ctx, sds, used
    return [t.double().cpu().numpy() for t in recs], used


def _oracle(P, b):
    bar, dt = P["bar"], P["dt"]
    models = []
    for i, (lo, hi) in enumerate(P["layers"]):
        if P["kinds"][i] == "fom":
            models.append(FomModel(bar, lo, hi, dt))
        else:
            R = P["roms"][i]
            models.append(OpInfModel(SubdomainGeometry(bar, lo, hi), R["Phi"], R["PhiS"], R["A"], R["H"], R["B"],
                                     R["c"], dt=dt))
    u0 = P["pulses"][b].u0(bar)
    return Coupled(models).run(u0, np.zeros_like(u0), N_STEPS, SchwarzOptions(), record=("u", "q"))


def _errors(P, recs, b, ref):
    out = []
    for i, (lo, hi) in enumerate(P["layers"]):
        got = recs[i][b]
        if P["kinds"][i] == "opinf":
            out.append(rel_err(got, ref["q"][i]))
        else:
            out.append(rel_err(got[:, lib_free_index(P["bar"], lo, hi)], ref["u"][i]))
    return out


@pytest.mark.parametrize("kinds,quadratic,with_c", [
    (("fom", "opinf"), True, True),
    (("opinf", "opinf"), True, False),
    (("opinf", "fom", "opinf"), True, True),
    (("fom", "opinf"), False, False),
])
def test_batched_path_matches_oracle_and_fused_path_f32(kinds, quadratic, with_c):
    P = _problem(kinds, quadratic, with_c)
    print(f"[batched {kinds} quad={quadratic} c={with_c}] gpu", flush=True)
    rb, used_b = _gpu_run(P, "f32", 2)
    rf, used_f = _gpu_run(P, "f32", 1)
    assert used_b == [2 if k == "opinf" else 0 for k in kinds]
    assert used_f == [1 if k == "opinf" else 0 for k in kinds]
    for b in CHECK:
        errs = _errors(P, rb, b, _oracle(P, b))
        print(f"instance {b}: batched vs oracle {['%.2e' % e for e in errs]}")
        assert max(errs) <= 1e-4
    # two FP32 evaluation orders of the same map: the FP32 bar on every instance
    for i in range(len(kinds)):
        d = max(rel_err(rb[i][b], rf[i][b]) for b in range(B))
        print(f"subdomain {i}: batched vs fused, worst instance {d:.2e}")
        assert d <= 1e-4


@pytest.mark.parametrize("kinds", [("opinf", "opinf"), ("fom", "opinf")])
def test_bf16h_precision_error_against_oracle(kinds):
    P = _problem(kinds, True, True, h_scale=1e3)
    print(f"[bf16h {kinds}] gpu", flush=True)
    # one step: q'' differs from the FP32 path by the operand rounding of the quadratic
    # term (~1 % of q'' here, rounded to ~2^-9), far below a misplaced fragment (~1e-2)
    c32, sds, _ = _gpu_run(P, "f32", 2, n=1, keep=True)
    c16, _, used = _gpu_run(P, "f32_bf16h", 0, n=1, keep=True)
    assert used == [2 if k == "opinf" else 0 for k in kinds]
    worst = 0.0
    for i, k in enumerate(kinds):
        if k != "opinf":
            continue
        for b in range(B):
            a32, a16 = c32.get_reduced(sds[i], b)[2], c16.get_reduced(sds[i], b)[2]
            worst = max(worst, float(np.linalg.norm(a16 - a32) / np.linalg.norm(a32)))
    print(f"one step: BF16-H vs FP32 q'' relative difference, worst instance {worst:.2e}")
    assert 0.0 < worst <= 1e-3
    del c32, c16
    r32, _ = _gpu_run(P, "f32", 2)
    r16, _ = _gpu_run(P, "f32_bf16h", 0)
    for b in CHECK:
        ref = _oracle(P, b)
        e32, e16 = _errors(P, r32, b, ref), _errors(P, r16, b, ref)
        print(f"instance {b}: FP32 {['%.2e' % e for e in e32]}, BF16-H {['%.2e' % e for e in e16]}")
        assert max(e32) <= 1e-4
        # reported error of the BF16-H precision on this deliberately strong quadratic term
        assert max(e16) <= 5e-3
