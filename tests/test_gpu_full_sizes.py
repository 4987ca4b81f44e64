"""Parity at the benchmark sizes, in the launch configuration the tuned runs use.

* 24x24x240 FOM-OpInf (the bench line's bar and slabs; seeded synthetic linear OpInf of the
  learned size r = 40 on Omega_2): fused sweeps with one layer per FE thread and graphs of
  32 sweeps.  FP64 against the oracle over 12 controller steps (1e-10, equal iteration
  counts); FP32 in the same configuration against that FP64 run (1e-4).
* 48x48x480 OpInf-OpInf with 256 instances (quadratic r = 100 on both slabs): the batched path
  (f0 on the matrix cores, both subdomains' f0 in one launch) inside fused sweeps against the
  fused OpInf path with separate launches, every instance (FP32, 1e-4).  The operators are
  seeded and stable; Phi is a block basis (orthonormal columns on disjoint DOF blocks), which
  keeps the set-up cheap at 2 million DOFs per subdomain without changing what the step
  kernels compute.
* 64x64x640 with 16 instances (three FOM slabs): the x-shared FE layout and fused sweeps give
  the bits of the plain FE launches (final states of the first and last instance).
The oracle cannot run the two larger cases; they are checked against the library's
configurations whose small-size parity with the oracle the other test files establish.
"""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, draw_pulses, gaussian_pulse_u, random_normal, slab_layers
from tests._gpu import lib_free_index, lib_index_of, lib_sch_index, rel_err

pytestmark = pytest.mark.gpu


def test_bar24_fom_opinf_tuned_launch_matches_oracle():
    import torch
    from paper_2511_20687_amd import osam
    from oracle.schwarz import Coupled, SchwarzOptions
    from tests.test_gpu_opinf import _build, _roms_for
    bar = Bar(24, 24, 240)
    dt = bar.explicit_dt()
    layers = [(0, 144), (96, 240)]
    kinds = ("fom", "opinf")
    roms = _roms_for(bar, layers, kinds, dt, r=40, rs=4, quadratic=False, with_c=False, seed=31)
    # the pulse starts inside the overlap (z = 0.4 .. 0.6) and crosses both Schwarz faces
    # within the 200 steps (c_p n dt = 0.21 m), so the transfers carry the wave
    u0 = gaussian_pulse_u(bar, 1e-3, 0.5, 0.02)
    v0 = np.zeros_like(u0)
    n = 200
    recs = {}
    print("[bar24 tuned launch] oracle set-up", flush=True)
    models, ctx64, _ = _build(bar, layers, dt, kinds, roms, "f64")
    for precision in ("f64", "f32"):
        if precision == "f64":
            ctx = ctx64
        else:   # the same operators in an FP32 context
            ctx = osam.Context(0, "f32", 1)
            sds = osam.add_bar_subdomains(ctx, bar, layers, dt)
            R = roms[1]
            Phi = np.zeros_like(R["Phi"])
            Phi[lib_free_index(bar, *layers[1])] = R["Phi"]
            PhiS = np.zeros_like(R["PhiS"])
            PhiS[lib_sch_index(bar, *layers[1])] = R["PhiS"]
            ctx.set_opinf(sds[1], Phi, PhiS, R["A"], R["H"], R["B"], R["c"])
        ctx.set_fusion(True, 1)
        ctx.set_graph(32, 1)
        dtp = torch.float64 if precision == "f64" else torch.float32
        ru = torch.zeros((1, n + 1, ctx.sizes(0)["n_free"]), dtype=dtp, device="cuda:0")
        rq = torch.zeros((1, n + 1, 40), dtype=dtp, device="cuda:0")
        ctx.set_record(0, 1, n + 1, u=ru)
        ctx.set_record(1, 1, n + 1, u=rq)
        ctx.set_initial(0, u0, v0)
        print(f"[bar24 tuned launch {precision}] gpu", flush=True)
        info = ctx.run(n)
        ctx.sync()
        recs[precision] = (ru[0].cpu().numpy().astype(np.float64), rq[0].cpu().numpy().astype(np.float64),
                           info[0]["total_iters"])
        del ctx
    del ctx64
    print("[bar24 tuned launch] oracle", flush=True)
    ref = Coupled(models).run(u0, v0, n, SchwarzOptions(), record=("u", "q"))
    u64, q64, it64 = recs["f64"]
    li = lib_index_of(models[0])
    e_u = rel_err(u64[:, li], ref["u"][0])
    e_q = rel_err(q64, ref["q"][1])
    # per-node check: the largest error of any DOF at any step against the field's largest value
    m_u = np.abs(u64[:, li] - ref["u"][0]).max() / np.abs(ref["u"][0]).max()
    print(f"FP64 vs oracle: u {e_u:.2e} (max-abs {m_u:.2e}), q {e_q:.2e}")
    assert e_u <= 1e-10 and e_q <= 1e-10 and m_u <= 1e-10
    assert it64 == int(ref["iters"].sum())
    # the transfers carried the wave: the overlap-face values are far above round-off
    face = np.abs(ref["u"][0][:, -3 * (bar.nx + 1) * (bar.ny + 1):]).max()
    assert face >= 1e-3 * np.abs(ref["u"][0]).max()
    u32, q32, _ = recs["f32"]
    e32 = rel_err(u32[:, li], ref["u"][0])
    m32 = np.abs(u32[:, li] - ref["u"][0]).max() / np.abs(ref["u"][0]).max()
    print(f"FP32 vs oracle: u {e32:.2e} (max-abs {m32:.2e}), q {rel_err(q32, ref['q'][1]):.2e}")
    assert e32 <= 1e-4 and m32 <= 1e-4 and rel_err(q32, ref["q"][1]) <= 1e-4


def _block_rom(seed, n_free, n_sch, r, rs, dt):
    """Stable quadratic operators and block bases (disjoint DOF blocks, orthonormal columns)."""
    Phi = np.zeros((n_free, r))
    for k, blk in enumerate(np.array_split(np.arange(n_free), r)):
        Phi[blk, k] = 1.0 / np.sqrt(len(blk))
    PhiS = np.zeros((n_sch, rs))
    for k, blk in enumerate(np.array_split(np.arange(n_sch), rs)):
        PhiS[blk, k] = 1.0 / np.sqrt(len(blk))
    w = np.linspace(0.1, 0.8, r) / dt
    A = -np.diag(w * w) + 0.01 * np.diag(w) @ random_normal(seed, (r, r)) @ np.diag(w) / r
    H = 1e-3 * random_normal(seed + 1, (r, r * (r + 1) // 2)) / (dt * dt)
    B = 0.05 * random_normal(seed + 2, (r, rs)) / (dt * dt)
    return Phi, PhiS, A, H, B


def test_bar48_opinf_opinf_256_batched_fused_sweeps_match_fused_path():
    import torch
    from paper_2511_20687_amd import osam
    bar = Bar(48, 48, 480)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    batch, n, r, rs = 256, 10, 100, 12
    opts = osam.Options(tol_abs=1e-8, tol_rel=1e-6)
    pulses = draw_pulses(3, batch, s=0.05)
    out = {}
    for mode in ("batched_fused_sweeps", "fused_path"):
        ctx = osam.Context(0, "f32", batch)
        sds = osam.add_bar_subdomains(ctx, bar, layers, dt)
        for i in sds:
            z = ctx.sizes(i)
            Phi, PhiS, A, H, B = _block_rom(40 + 10 * i, z["n_free"], z["n_sch"], r, rs, dt)
            ctx.set_opinf(i, Phi, PhiS, A, H, B)
            del Phi
            ctx.set_rom_path(i, 2 if mode == "batched_fused_sweeps" else 1)
        if mode == "batched_fused_sweeps":
            ctx.set_fusion(True, 1)
            ctx.set_graph(32, 1)
        recs = [torch.zeros((batch, n + 1, r), dtype=torch.float32, device="cuda:0") for _ in sds]
        for i in sds:
            ctx.set_record(i, 1, n + 1, u=recs[i])
        for b, p in enumerate(pulses):
            u0 = p.u0(bar)
            ctx.set_initial(b, u0, np.zeros_like(u0))
        print(f"[bar48 B=256 {mode}] gpu", flush=True)
        ctx.run(n, opts)
        ctx.sync()
        out[mode] = [t.cpu().numpy().astype(np.float64) for t in recs]
        del ctx, recs
        torch.cuda.empty_cache()
    worst = 0.0
    for i in range(2):
        for b in range(batch):
            worst = max(worst, rel_err(out["batched_fused_sweeps"][i][b], out["fused_path"][i][b]))
    print(f"batched path in fused sweeps vs fused path, worst instance: {worst:.2e}")
    assert worst <= 1e-4


def test_bar64_fom_16_instances_layouts_and_fused_sweeps_are_bitwise_equal():
    from paper_2511_20687_amd import osam
    bar = Bar(64, 64, 640)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 3)
    batch, n = 16, 3
    pulses = draw_pulses(5, batch, s=0.05)
    states = {}
    for mode in ("plain", "xshare", "fused"):
        ctx = osam.Context(0, "f32", batch)
        sds = osam.add_bar_subdomains(ctx, bar, layers, dt, lateral_fix=(0, 1))
        for i in sds:
            ctx.set_fe_launch(i, 256, 1)
            ctx.set_fe_xshare(i, mode == "xshare")
        if mode == "fused":
            ctx.set_fusion(True, 1)
        for b, p in enumerate(pulses):
            u0 = p.u0(bar)
            ctx.set_initial(b, u0, np.zeros_like(u0))
        print(f"[bar64 B=16 {mode}] gpu", flush=True)
        info = ctx.run(n)
        states[mode] = ([ctx.get_state(1, b)[0] for b in (0, batch - 1)], [x["total_iters"] for x in info])
        del ctx
    for mode in ("xshare", "fused"):
        for k in range(2):
            assert np.array_equal(states[mode][0][k], states["plain"][0][k]), (mode, k)
        assert states[mode][1] == states["plain"][1]


@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f32_bf16h", 1e-2)])
def test_bar48_opinf_opinf_256_matches_oracle(precision, tol):
    """48x48x480 OpInf-OpInf, quadratic r = 100 on both slabs, 256 instances in the bench's
    launch configuration (batched f0 on the matrix cores inside fused sweeps, graphs of 32):
    4 instances against the FP64 oracle over 50 controller steps.  FP32 to 1e-4; BF16-H
    (BF16 operands of the quadratic contraction) reports its error and is held to 1e-2."""
    import scipy.sparse as sp
    import torch
    from paper_2511_20687_amd import osam
    from oracle.newmark import SubdomainGeometry
    from oracle.rom import OpInfModel
    from oracle.schwarz import Coupled, SchwarzOptions
    bar = Bar(48, 48, 480)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    batch, n, r, rs, n_or = 256, 50, 100, 12, 4
    opts = osam.Options(tol_abs=1e-8, tol_rel=1e-6)
    pulses = draw_pulses(3, batch, s=0.05)
    ctx = osam.Context(0, precision, batch)
    sds = osam.add_bar_subdomains(ctx, bar, layers, dt)
    models = []
    for i in sds:
        z = ctx.sizes(i)
        Phi, PhiS, A, H, B = _block_rom(40 + 10 * i, z["n_free"], z["n_sch"], r, rs, dt)
        ctx.set_opinf(i, Phi, PhiS, A, H, B)
        g = SubdomainGeometry(bar, *layers[i])
        Phi_o = sp.csr_matrix(Phi)[lib_index_of(g)]          # oracle DOF order
        del Phi
        models.append(OpInfModel(g, Phi_o, PhiS[lib_sch_index(bar, *layers[i])], A, H, B, dt=dt))
        ctx.set_rom_path(i, 2)
    ctx.set_fusion(True, 1)
    ctx.set_graph(32, 1)
    recs = [torch.zeros((batch, n + 1, r), dtype=torch.float32, device="cuda:0") for _ in sds]
    for i in sds:
        ctx.set_record(i, 1, n + 1, u=recs[i])
    for b, p in enumerate(pulses):
        u0 = p.u0(bar)
        ctx.set_initial(b, u0, np.zeros_like(u0))
    print(f"[bar48 B=256 {precision} vs oracle] gpu", flush=True)
    ctx.run(n, opts)
    ctx.sync()
    got = [t.cpu().numpy().astype(np.float64) for t in recs]
    del ctx, recs
    print("oracle", flush=True)
    cp = Coupled(models)
    worst = 0.0
    for b in range(n_or):
        u0 = pulses[b].u0(bar)
        ref = cp.run(u0, np.zeros_like(u0), n, SchwarzOptions(tol_abs=1e-8, tol_rel=1e-6), record=("q",))
        for i in range(2):
            e = rel_err(got[i][b], ref["q"][i])
            worst = max(worst, e)
        print(f"instance {b}: worst subdomain error {worst:.2e}", flush=True)
    print(f"{precision} vs FP64 oracle, worst of {n_or} instances: {worst:.2e}")
    assert worst <= tol
