"""GPU parity of the FOM-FOM Schwarz path (libosam via the C ABI) against the FP64 oracle.

Tolerances (relative space-time L2 of the displacement, Eq. mse): 1e-10 in FP64,
1e-4 in FP32.
"""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import CFG1, Bar, Pulse, gaussian_pulse_u, random_normal, slab_layers
from oracle.schwarz import SchwarzOptions
from tests._gpu import lib_free_index, lib_index_of, lib_sch_index, oracle_fom_coupled, rel_err, torch_dtype

pytestmark = pytest.mark.gpu


def _lib_run(bar, layers, dt, u0, v0, n, precision, opts=None, batch=1, record_s=False, lateral_fix=(),
             fe_launch=None, xshare=False, fusion_kc=0):
    import torch
    from paper_2511_20687_amd import osam
    ctx = osam.Context(0, precision, batch)
    sds = osam.add_bar_subdomains(ctx, bar, layers, dt, lateral_fix=lateral_fix)
    if fe_launch is not None:
        for sd in sds:
            ctx.set_fe_launch(sd, *fe_launch)
            assert ctx.get_fe_launch(sd)[0] == fe_launch[0]
    for sd in sds:
        ctx.set_fe_xshare(sd, xshare)
    if fusion_kc:
        ctx.set_fusion(True, fusion_kc)
    dev = torch.device("cuda:0")
    recs = []
    for sd in sds:
        z = ctx.sizes(sd)
        ru = torch.zeros((batch, n + 1, z["n_free"]), dtype=torch_dtype(precision), device=dev)
        rs = torch.zeros((batch, n + 1, z["n_sch"]), dtype=torch_dtype(precision), device=dev) \
            if record_s else None
        ctx.set_record(sd, 1, n + 1, u=ru, s=rs)
        recs.append((ru, rs))
    for b in range(batch):
        ctx.set_initial(b, u0[b] if isinstance(u0, list) else u0, v0[b] if isinstance(v0, list) else v0)
    info = ctx.run(n, opts or osam.Options())
    torch.cuda.synchronize()
    return ctx, [(ru.cpu().numpy(), None if rs is None else rs.cpu().numpy()) for ru, rs in recs], info


@pytest.mark.parametrize("lateral", ["workload", "traction-free"])
@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_cfg1_fom_fom_matches_oracle(precision, tol, lateral):
    """Bar 4x4x40, two slabs with 20% overlap, 1000 explicit steps, pulse (1e-3, 0.25, 0.05);
    lateral faces as in the workload (x, y held) and traction-free."""
    w = CFG1
    bar, dt, layers = w.bar, w.dt, w.layers
    lf = w.lateral_fix if lateral == "workload" else ()
    u0 = Pulse(1e-3, 0.25, w.pulse_width).u0(bar)
    v0 = np.zeros_like(u0)
    n = w.steps
    print(f"[cfg1 {precision} {lateral}] oracle", flush=True)
    models, ref = oracle_fom_coupled(bar, layers, dt, u0, v0, n, lateral_fix=lf)
    print(f"[cfg1 {precision} {lateral}] gpu", flush=True)
    ctx, recs, info = _lib_run(bar, layers, dt, u0, v0, n, precision, lateral_fix=lf)
    for i, m in enumerate(models):
        got = recs[i][0][0][:, lib_index_of(m)]
        err = rel_err(got, ref["u"][i])
        print(f"subdomain {i}: rel err {err:.3e}")
        assert err <= tol
    assert info[0]["steps"] == n
    # iteration counts: FP64 reproduces the oracle's decisions exactly
    if precision == "f64":
        assert info[0]["total_iters"] == int(ref["iters"].sum())
        assert info[0]["max_iters"] == int(ref["iters"].max())


@pytest.mark.parametrize("lateral_fix", [(0, 1), (2,), (0, 1, 2)])
def test_lateral_dirichlet_matches_oracle_f64(lateral_fix):
    """Lateral faces holding components at zero (Sec. 5.1 holds x and y); a seeded IC with all
    three components nonzero everywhere, so the held DOFs must be zeroed and stay zero."""
    bar = Bar(3, 4, 30)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    u0 = 1e-5 * random_normal(71, (3, bar.n_nodes))
    v0 = 1e-2 * random_normal(72, (3, bar.n_nodes))
    n = 150
    print(f"[lateral {lateral_fix}] oracle", flush=True)
    models, ref = oracle_fom_coupled(bar, layers, dt, u0, v0, n, lateral_fix=lateral_fix)
    print(f"[lateral {lateral_fix}] gpu", flush=True)
    ctx, recs, info = _lib_run(bar, layers, dt, u0, v0, n, "f64", lateral_fix=lateral_fix)
    for i, m in enumerate(models):
        idx = lib_index_of(m)
        got = recs[i][0][0]
        assert rel_err(got[:, idx], ref["u"][i]) <= 1e-10
        held = np.setdiff1d(np.arange(got.shape[1]), idx)
        assert held.size > 0 and np.all(got[:, held] == 0.0)
    assert info[0]["total_iters"] == int(ref["iters"].sum())


def test_three_slabs_and_schwarz_records_f64():
    """Three subdomains (middle one with two Schwarz faces); records of the Schwarz data."""
    bar = Bar(3, 2, 36)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 3)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.4, 0.06)
    v0 = np.zeros_like(u0)
    v0[2] = 3.0 * np.exp(-((bar.node_z() - 0.7) ** 2) / (2 * 0.05 ** 2))
    n = 200
    models, ref = oracle_fom_coupled(bar, layers, dt, u0, v0, n, record=("u", "s"))
    ctx, recs, info = _lib_run(bar, layers, dt, u0, v0, n, "f64", record_s=True)
    for i, (lo, hi) in enumerate(layers):
        assert rel_err(recs[i][0][0][:, lib_free_index(bar, lo, hi)], ref["u"][i]) <= 1e-10
        assert rel_err(recs[i][1][0][:, lib_sch_index(bar, lo, hi)], ref["s"][i]) <= 1e-10
    assert info[0]["total_iters"] == int(ref["iters"].sum())


def test_predictor_guess_and_iteration_cap_f64():
    from paper_2511_20687_amd import osam
    bar = Bar(2, 2, 30)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.5, 0.05)
    v0 = np.zeros_like(u0)
    n = 60
    _, ref = oracle_fom_coupled(bar, layers, dt, u0, v0, n, SchwarzOptions(guess="predictor"))
    ctx, recs, info = _lib_run(bar, layers, dt, u0, v0, n, "f64", osam.Options(guess=1))
    assert info[0]["total_iters"] == 2 * n
    for i, (lo, hi) in enumerate(layers):
        assert rel_err(recs[i][0][0][:, lib_free_index(bar, lo, hi)], ref["u"][i]) <= 1e-10
    # unreachable tolerance: every step runs to the cap and is reported unconverged
    ctx2, _, info2 = _lib_run(bar, layers, dt, u0, v0, 5, "f64",
                              osam.Options(tol_abs=0.0, tol_rel=0.0, max_iter=4))
    assert info2[0]["total_iters"] == 20 and info2[0]["unconverged"] == 5


def test_batched_instances_match_unbatched_f32():
    """Independent instances in one launch give bitwise the single-instance results."""
    bar = Bar(6, 5, 48)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    pulses = [Pulse(1e-3, 0.3, 0.05), Pulse(2e-3, 0.2, 0.04), Pulse(0.7e-3, 0.35, 0.06)]
    u0 = [p.u0(bar) for p in pulses]
    v0 = [np.zeros_like(x) for x in u0]
    n = 120
    _, recs, info = _lib_run(bar, layers, dt, u0, v0, n, "f32", batch=3)
    for b in range(3):
        _, r1, _ = _lib_run(bar, layers, dt, u0[b], v0[b], n, "f32")
        for i in range(2):
            assert np.array_equal(recs[i][0][b], r1[i][0][0])


def test_repeat_runs_are_bitwise_identical_f32():
    bar = Bar(8, 8, 80)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    u0 = Pulse().u0(bar)
    v0 = np.zeros_like(u0)
    _, r1, _ = _lib_run(bar, layers, dt, u0, v0, 50, "f32")
    _, r2, _ = _lib_run(bar, layers, dt, u0, v0, 50, "f32")
    for i in range(2):
        assert np.array_equal(r1[i][0], r2[i][0])


def test_state_readback_and_nonfinite_detection_f64():
    from paper_2511_20687_amd import osam
    bar = Bar(2, 2, 20)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.5, 0.05)
    v0 = np.zeros_like(u0)
    models, ref = oracle_fom_coupled(bar, layers, dt, u0, v0, 10, record=("u",))
    ctx, _, info = _lib_run(bar, layers, dt, u0, v0, 10, "f64")
    st = ref["states"]
    for i, m in enumerate(models):
        u, v, a = ctx.get_state(i, 0)
        assert rel_err(u.T.ravel(), st[i].u) <= 1e-12
        assert rel_err(v.T.ravel()[m.free_dofs], st[i].v[m.free_dofs]) <= 1e-12
        assert rel_err(a.T.ravel()[m.free_dofs], st[i].a[m.free_dofs]) <= 1e-12
    # a NaN in the initial field is reported as OSAM_E_NONFINITE
    bad = u0.copy()
    bad[2, bad.shape[1] // 3] = np.nan
    ctx2 = osam.Context(0, "f64", 1)
    osam.add_bar_subdomains(ctx2, bar, layers, dt)
    ctx2.set_initial(0, bad, v0)
    info2 = ctx2.run(5, osam.Options(), check=False)
    assert info2[0]["status"] == osam.OSAM_E_NONFINITE


@pytest.mark.parametrize("lateral", [(0, 1), ()])
@pytest.mark.parametrize("kc", [1, 5, 64])
def test_layer_staged_fe_variant_f32(kc, lateral):
    """The layer-staged FE variant (whole layers in LDS, 1024-thread workgroups of kc layers,
    boundary columns in a second launch) against the column kernel on every record of a
    batch of 2 (u and the Schwarz face data, three slabs, a 6 x 5 cross-section) and
    against the oracle (FP32 bar)."""
    bar = Bar(6, 5, 48)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 3)
    u0 = [gaussian_pulse_u(bar, 1e-3, 0.3, 0.05), gaussian_pulse_u(bar, 2e-3, 0.6, 0.04)]
    v0 = [np.zeros_like(u0[0]), np.zeros_like(u0[1])]
    v0[1][0] = 2.0 * np.exp(-((bar.node_z() - 0.5) ** 2) / (2 * 0.05 ** 2))
    n = 200
    print(f"[layer-staged kc={kc} lateral={lateral}] gpu", flush=True)
    _, rc, ic = _lib_run(bar, layers, dt, u0, v0, n, "f32", batch=2, record_s=True, lateral_fix=lateral)
    _, rl, il = _lib_run(bar, layers, dt, u0, v0, n, "f32", batch=2, record_s=True, lateral_fix=lateral,
                         fe_launch=(1024, kc))
    for i in range(len(layers)):
        for b in range(2):
            du = rel_err(rl[i][0][b], rc[i][0][b])
            ds = rel_err(rl[i][1][b], rc[i][1][b])
            assert du <= 1e-6 and ds <= 1e-6, (i, b, du, ds)
    assert [x["total_iters"] for x in il] == [x["total_iters"] for x in ic]
    models, ref = oracle_fom_coupled(bar, layers, dt, u0[1], v0[1], n, record=("u", "s"), lateral_fix=lateral)
    for i, m in enumerate(models):
        lo, hi = layers[i]
        e_u = rel_err(rl[i][0][1][:, lib_index_of(m)], ref["u"][i])
        e_s = rel_err(rl[i][1][1][:, lib_sch_index(bar, lo, hi)], ref["s"][i])
        print(f"subdomain {i}: u {e_u:.2e}, s {e_s:.2e}")
        assert e_u <= 1e-4 and e_s <= 1e-4


@pytest.mark.parametrize("fusion_kc", [0, 1, 3])
@pytest.mark.parametrize("kc", [1, 3])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("cross", [(6, 5), (70, 3)])
def test_fe_xshare_layout_is_bitwise_identical(cross, precision, kc, fusion_kc):
    """The interior layout with x-neighbours taken from adjacent lanes (osam_set_fe_xshare)
    against the layout that loads every neighbour: the same bits (every interior path adds
    the stencil in one x-resolved order, whether the x-offset partial sums are formed where
    the values are and moved across lanes, with one layer per thread, or formed from whole
    neighbourhoods): records of u and the Schwarz faces of three slabs, batch of 2, iteration
    counts; with FE launches (one and three layers per thread) and inside fused sweeps.
    Rows of 71 nodes (70 x 3) wrap
    inside waves; FP64 is also checked against the oracle.  Cubic elements of 1/36 m (Bar
    default lengths would make the 70 x 3 elements needle-shaped and the explicit step
    unstable)."""
    nx, ny = cross
    h = 1.0 / 36   # cubic elements (the explicit step size assumes them)
    bar = Bar(nx, ny, 36, Lx=nx * h, Ly=ny * h, Lz=36 * h)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 3)
    lateral = (0, 1)
    u0 = [gaussian_pulse_u(bar, 1e-3, 0.3, 0.05), gaussian_pulse_u(bar, 2e-3, 0.6, 0.04)]
    v0 = [np.zeros_like(u0[0]), np.zeros_like(u0[1])]
    v0[1][0] = 2.0 * np.exp(-((bar.node_z() - 0.5) ** 2) / (2 * 0.05 ** 2))
    n = 80
    print(f"[xshare {cross} {precision} kc={kc} fusion={fusion_kc}] gpu", flush=True)
    _, r0, i0 = _lib_run(bar, layers, dt, u0, v0, n, precision, batch=2, record_s=True, lateral_fix=lateral,
                         fe_launch=(256, kc), fusion_kc=fusion_kc)
    _, r1, i1 = _lib_run(bar, layers, dt, u0, v0, n, precision, batch=2, record_s=True, lateral_fix=lateral,
                         fe_launch=(256, kc), xshare=True, fusion_kc=fusion_kc)
    for i in range(len(layers)):
        assert np.array_equal(r1[i][0], r0[i][0]), (i, float(np.abs(r1[i][0] - r0[i][0]).max()))
        assert np.array_equal(r1[i][1], r0[i][1])
    assert [x["total_iters"] for x in i1] == [x["total_iters"] for x in i0]
    if precision == "f64" and kc == 1 and fusion_kc == 0:
        models, ref = oracle_fom_coupled(bar, layers, dt, u0[1], v0[1], n, record=("u", "s"), lateral_fix=lateral)
        for i, m in enumerate(models):
            lo, hi = layers[i]
            assert rel_err(r1[i][0][1][:, lib_index_of(m)], ref["u"][i]) <= 1e-10
            assert rel_err(r1[i][1][1][:, lib_sch_index(bar, lo, hi)], ref["s"][i]) <= 1e-10
