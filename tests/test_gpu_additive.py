"""The additive Schwarz variant (Remark additive_sam; osam_schwarz_opts.additive): every
subdomain of an iteration takes its neighbours' iterates of the previous iteration, so the
first iteration of a step starts every face from the initial guess.

Checked against the oracle's additive controller (FP64: records and iteration counts),
with FOM and OpInf subdomains on both sides of faces, in sequential launches and fused
sweeps; with the explicit step the accepted iterates are those of the multiplicative
variant (the data of the second iteration is already final), which is checked bit for bit.
"""
import numpy as np
import pytest

from oracle.schwarz import Coupled, SchwarzOptions
from paper_2511_20687_amd.inputs import Bar, gaussian_pulse_u, slab_layers
from tests._gpu import lib_free_index, lib_index_of, oracle_fom_coupled, rel_err
from tests.test_gpu_fom import _lib_run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("S", [2, 3])
def test_additive_fom_matches_oracle_and_multiplicative_bits(S):
    from paper_2511_20687_amd import osam
    bar = Bar(3, 3, 36)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, S)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.45, 0.06)
    v0 = np.zeros_like(u0)
    n = 150
    print(f"[additive FOM S={S}] gpu", flush=True)
    _, rec, info = _lib_run(bar, layers, dt, u0, v0, n, "f64", opts=osam.Options(additive=True))
    _, rec_m, info_m = _lib_run(bar, layers, dt, u0, v0, n, "f64")
    models, ref = oracle_fom_coupled(bar, layers, dt, u0, v0, n, opts=SchwarzOptions(additive=True))
    _, ref_m = oracle_fom_coupled(bar, layers, dt, u0, v0, n)
    assert info[0]["total_iters"] == int(ref["iters"].sum())
    assert info_m[0]["total_iters"] == int(ref_m["iters"].sum())
    for i, m in enumerate(models):
        assert rel_err(rec[i][0][0][:, lib_index_of(m)], ref["u"][i]) <= 1e-10
        assert np.array_equal(rec[i][0], rec_m[i][0]), i
    print(f"iterations: additive {info[0]['total_iters']}, multiplicative {info_m[0]['total_iters']}")


@pytest.mark.parametrize("kinds,fused", [(("fom", "opinf", "fom"), False), (("opinf", "fom", "opinf"), False),
                                         (("opinf", "opinf"), False), (("opinf", "fom", "opinf"), True)])
def test_additive_opinf_couplings_match_oracle(kinds, fused):
    import torch
    from paper_2511_20687_amd import osam
    from tests.test_gpu_opinf import _build, _roms_for
    from tests._gpu import torch_dtype
    bar = Bar(3, 3, 36)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, len(kinds))
    roms = _roms_for(bar, layers, kinds, dt, r=9, rs=5, quadratic=True, with_c=False, seed=23)
    models, ctx, sds = _build(bar, layers, dt, kinds, roms, "f64")
    if fused:
        ctx.set_fusion(True, 1)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.45, 0.06)
    v0 = np.zeros_like(u0)
    n = 120
    print(f"[additive {kinds} fused={fused}] oracle", flush=True)
    ref = Coupled(models).run(u0, v0, n, SchwarzOptions(additive=True), record=("u", "q"))
    recs = []
    for i, sd in enumerate(sds):
        z = ctx.sizes(sd)
        length = z["r"] if kinds[i] == "opinf" else z["n_free"]
        t = torch.zeros((1, n + 1, length), dtype=torch_dtype("f64"), device="cuda:0")
        ctx.set_record(sd, 1, n + 1, u=t)
        recs.append(t)
    ctx.set_initial(0, u0, v0)
    print("gpu", flush=True)
    info = ctx.run(n, osam.Options(additive=True))
    for i, (lo, hi) in enumerate(layers):
        got = recs[i][0].cpu().numpy()
        err = rel_err(got, ref["q"][i]) if kinds[i] == "opinf" else rel_err(got[:, lib_free_index(bar, lo, hi)],
                                                                             ref["u"][i])
        assert err <= 1e-10, (i, err)
    assert info[0]["total_iters"] == int(ref["iters"].sum())


def test_additive_option_is_validated():
    from paper_2511_20687_amd import osam
    bar = Bar(2, 2, 24)
    ctx = osam.Context(0, "f64", 1)
    osam.add_bar_subdomains(ctx, bar, slab_layers(bar.nz, 2), bar.explicit_dt())
    u0 = gaussian_pulse_u(bar, 1e-3, 0.45, 0.06)
    ctx.set_initial(0, u0, np.zeros_like(u0))
    o = osam.Options()
    o.additive = 2
    with pytest.raises(osam.OsamError):
        ctx.run(1, o)
