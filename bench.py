"""Benchmark: coupled Schwarz steps/s of the FOM-OpInf hybrid on one MI355X.

Workload (default): bar 24x24x240 hex8 (150,625 nodes), two z-slabs with 20%
overlap; subdomain 1 FOM, subdomain 2 linear OpInf r = 40 learned from 2000
snapshots of a FOM-FOM training run (seeded pulse), boundary basis by the
1 - 1e-6 energy criterion, lambda by Alg. 3 over the 11-point grid; online run
of 5000 controller steps, FP32 state, FP64 convergence sums.

One benchmark step = one complete online coupled run (5000 controller steps of
the multiplicative Schwarz loop).  value = controller steps per second.
Learning and the training run are set-up (timed separately, reported).
Also reported: the FOM-FOM run of the same bar on the same GPU, the accuracy of
the hybrid against it (Eq. mse), FE DOF-updates/s, the FE kernel's achieved
bandwidth vs the HBM peak (of the fused sweep kernel when the autotuner picks fused
sweeps: FE step and OpInf step in one launch), and the FP64 CPU oracle timed on a
bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 algorithmic bytes per FE DOF-iteration-update (the unit of work of the explicit
# step): read u, v, a at t_{k-1} and the previous iterate's u, v; write u, v, a; the lumped
# mass, 4 B per node (8 x 4 B + 4/3 B)
FE_BYTES_PER_DOF = 32.0 + 4.0 / 3.0
# what the step kernel itself moves per DOF: read P, V0, A0, V1(prev), write V1, A1, P2
# (7 x 4 B; the mass is folded into the stencil coefficients, u(t_k) is the predictor P)
FE_KERNEL_BYTES_PER_DOF = 28.0


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_context(w, precision, batch=1):
    from paper_2511_20687_amd import osam
    ctx = osam.Context(0, precision, batch)
    osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    return ctx


def _guarded(name, fn):
    """A secondary leg: its failure is reported in the JSON line instead of ending the bench."""
    try:
        return fn()
    except Exception as e:
        _log(f"{name} failed: {e!r}")
        return {"error": repr(e)}


def opts_for(w):
    from paper_2511_20687_amd import osam
    return osam.Options(tol_abs=w.tol_abs, tol_rel=w.tol_rel, min_iter=w.min_iter, max_iter=w.max_iter,
                        guess=w.guess)


def train_and_learn(w, pulse, precision):
    """FOM-FOM training run recording subdomain 2 snapshots, then learn_opinf on it."""
    import torch
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import Bar
    ctx = build_context(w, precision)
    rom_sd = w.models.index("opinf")
    z = ctx.sizes(rom_sd)
    T = w.train_steps
    dt_ = torch.float32 if precision == "f32" else torch.float64
    dev = "cuda:0"
    U = torch.zeros((1, T, z["n_free"]), dtype=dt_, device=dev)
    A = torch.zeros((1, T, z["n_free"]), dtype=dt_, device=dev)
    S = torch.zeros((1, T, z["n_sch"]), dtype=dt_, device=dev)
    ctx.set_record(rom_sd, 1, T, u=U, a=A, s=S)
    u0 = pulse.u0(w.bar)
    v0 = np.zeros_like(u0)
    ctx.set_initial(0, u0, v0)
    t0 = time.perf_counter()
    ctx.run(T - 1, opts_for(w))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    lo, hi = w.layers[rom_sd]
    npl = (w.bar.nx + 1) * (w.bar.ny + 1)
    V0 = torch.tensor(v0[:, npl * (lo + 1):npl * hi].reshape(1, -1), dtype=dt_, device=dev)
    from paper_2511_20687_amd.inputs import lambda_grid_values
    t0 = time.perf_counter()
    out = ctx.learn_opinf(rom_sd, U, A, S, V0, 1, T, form=w.form, r=w.r, r_s=0,
                          energy_bnd=1 - 1e-6, lambdas=lambda_grid_values(11))
    torch.cuda.synchronize()
    t_learn = time.perf_counter() - t0
    del U, A, S
    return ctx, out, t_train, t_learn


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched OpInf-OpInf comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-large-fe", action="store_true", help="skip the 64x64x640 FE step timing")
    ap.add_argument("--no-survey", action="store_true",
                    help="skip the 24x24x240 hybrid under traction-free lateral faces and s = 0.05")
    ap.add_argument("--fixed-launch", action="store_true",
                    help="skip the hybrid's autotuner and run fused sweeps (one layer per FE thread) in graphs of "
                         "128 sweeps, the choice it makes for this workload on MI355X without a profiler: under "
                         "rocprofv3 the per-launch overhead changes the tuner's timings and so its choice")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the 4x4x40 legs (explicit, implicit, mixed steps, Saint Venant-Kirchhoff)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(every instance and subdomain runs on one device); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import CFG2, draw_pulses
    w = CFG2
    pulse = draw_pulses(w.seed, 1, s=w.pulse_width)[0]
    n = w.steps
    _log(f"workload {w.name}: pulse a={pulse.a:.4e} b={pulse.b:.4f} s={pulse.s}; dt={w.dt:.4e}")

    # ---- set-up: training run + learning (untimed for the metric) ----
    ctx, learned, t_train, t_learn = train_and_learn(w, pulse, w.precision)
    _log(f"training run {w.train_steps - 1} steps: {t_train:.2f} s; learning: {t_learn:.2f} s; "
         f"r={learned['r']} r_s={learned['r_s']} lambda*={learned['lambda_star']:.1e}")
    opts = opts_for(w)
    u0 = pulse.u0(w.bar)
    v0 = np.zeros_like(u0)

    # ---- launch configuration by the library's autotuner (untimed set-up) ----
    ctx.set_initial(0, u0, v0)
    t0 = time.perf_counter()
    if args.fixed_launch:
        ctx.set_fusion(True, 1)
        ctx.set_graph(128, 1)
        tuning = {"fixed": True, "fusion_kc": 1, "graph": (128, 1)}
    else:
        tuning = ctx.autotune(trial_steps=200, opts=opts)
    t_tune = time.perf_counter() - t0
    _log(f"autotune {t_tune:.2f} s: {tuning}")

    # ---- timed region: K complete online FOM-OpInf runs ----
    for i in range(args.warmup):
        ctx.set_initial(0, u0, v0)
        ctx.run(n, opts)
        _log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    times, infos = [], []
    for i in range(args.steps):
        ctx.set_initial(0, u0, v0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.run(n, opts)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        infos.append(info[0])
        _log(f"step {i + 1}/{args.steps}: {times[-1] * 1e3:.1f} ms ({n / times[-1]:.0f} steps/s)")
    total = sum(times)
    value = args.steps * n / total
    iters = infos[-1]["total_iters"]
    z0 = ctx.sizes(0)
    fe_dofs = z0["n_free"]
    dof_updates_per_s = fe_dofs * iters / times[-1]

    # ---- dominant kernel timing with HIP events (same workload and launch configuration,
    # extra pass): the fused sweep kernel when the tuner chose fused sweeps, else the FE kernel
    from paper_2511_20687_amd.profiling import read_traffic, rom_bytes_per_launch
    fused = tuning.get("fusion_kc", 0) > 0
    ctx.set_initial(0, u0, v0)
    ctx.set_timing(True)
    ctx.run(n, opts)
    k_ms, k_launches = ctx.get_timing(0)      # fused: the sweep kernel, reported for every subdomain
    rom_ms, rom_launches = ctx.get_timing(1)
    ctx.set_timing(False)
    k_avg_us = 1e3 * k_ms / max(k_launches, 1)
    face = 3 * (w.bar.nx + 1) * (w.bar.ny + 1)      # DOFs of one Schwarz face (each way)
    rom_alg = rom_bytes_per_launch(learned["r"], learned["r_s"], face, face)
    fe_alg = FE_BYTES_PER_DOF * fe_dofs
    alg_bytes = fe_alg + rom_alg if fused else fe_alg
    k_gbs = alg_bytes / (k_avg_us * 1e-6) / 1e9
    traffic_bytes, traffic_src = read_traffic("bar24_sweep" if fused else "bar24")
    # the FE kernel alone (one launch per subdomain), for reference
    fe_avg_us = None
    if fused:
        ctx.set_fusion(False)
        ctx.set_initial(0, u0, v0)
        ctx.set_timing(True)
        ctx.run(n, opts)
        fe_ms, fe_launches = ctx.get_timing(0)
        rom_ms, rom_launches = ctx.get_timing(1)
        ctx.set_timing(False)
        ctx.set_fusion(True, tuning["fusion_kc"])
        fe_avg_us = 1e3 * fe_ms / max(fe_launches, 1)
    else:
        fe_avg_us = k_avg_us

    # ---- accuracy vs FOM-FOM and FOM-FOM throughput on the same GPU ----
    every = 10
    ncol = n // every + 1
    dev = "cuda:0"
    recs = []
    for sd in range(2):
        z = ctx.sizes(sd)
        length = z["n_free"] if sd == 0 else z["r"]
        t = torch.zeros((1, ncol, length), dtype=torch.float32, device=dev)
        ctx.set_record(sd, every, ncol, u=t)
        recs.append(t)
    ctx.set_initial(0, u0, v0)
    ctx.run(n, opts)
    learned_ops = ctx.get_opinf(1)
    Phi = torch.tensor(learned_ops["Phi"], dtype=torch.float64, device=dev)
    hyb = [recs[0][0].double(), (Phi @ recs[1][0].double().T).T]
    # the first recorded columns, for the comparison with the FP64 oracle
    hyb_head = [recs[0][0, : args.cpu_steps // every + 1].double().cpu().numpy(),
                recs[1][0, : args.cpu_steps // every + 1].double().cpu().numpy()]
    del recs
    ff = build_context(w, w.precision)
    frec = []
    for sd in range(2):
        z = ff.sizes(sd)
        t = torch.zeros((1, ncol, z["n_free"]), dtype=torch.float32, device=dev)
        ff.set_record(sd, every, ncol, u=t)
        frec.append(t)
    ff.set_initial(0, u0, v0)
    ff.run(n, opts)
    errs = []
    for sd in range(2):
        ref = frec[sd][0].double()
        errs.append(float(torch.linalg.norm(hyb[sd] - ref) / torch.linalg.norm(ref)))
    del frec, hyb
    ff2 = build_context(w, w.precision)
    ff2.set_initial(0, u0, v0)
    ff_tuning = ff2.autotune(trial_steps=200, opts=opts)   # the best FOM-FOM launch on this GPU too
    ff2.set_initial(0, u0, v0)
    ff2.run(n, opts)      # warm-up
    ff2.set_initial(0, u0, v0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    finfo = ff2.run(n, opts)
    torch.cuda.synchronize()
    t_ff = time.perf_counter() - t0
    fom_fom_value = n / t_ff
    _log(f"hybrid {value:.0f} steps/s, FOM-FOM {fom_fom_value:.0f} steps/s, errors {errs}")

    # ---- batched OpInf-OpInf (48x48x480, 256 instances) against FOM-FOM on this GPU ----
    batched = None
    if not args.no_batched:
        from paper_2511_20687_amd import batched_case
        del ctx, ff, ff2
        torch.cuda.empty_cache()
        batched = _guarded("batched OpInf-OpInf", lambda: batched_case.run(log=_log))

    # ---- adjoint of the coupled rollout, 24x24x240 FOM + quadratic OpInf r=60 ----
    adjoint = None
    if not args.no_adjoint:
        adjoint = _guarded("adjoint", lambda: adjoint_timing(_log))

    # ---- the FE step at the large bar's size (HBM-bound) ----
    large_fe = None
    if not args.no_large_fe:
        large_fe = large_fe_timing(_log)

    # ---- the same hybrid under traction-free lateral faces and s = 0.05 (errors, energy ranks) ----
    survey = None
    if not args.no_survey:
        from paper_2511_20687_amd import survey_case
        survey = _guarded("hybrid under other input readings", lambda: survey_case.run(_log))

    # ---- latency-bound legs on the 4x4x40 bar (both engines) ----
    latency = None
    if not args.no_latency:
        from paper_2511_20687_amd import window_case
        latency = _guarded("latency legs", lambda: window_case.run(_log))

    # ---- CPU oracle: timed on a bounded sample; every GPU result's error against it ----
    cpu = None
    if not args.no_cpu_baseline:
        cpu = _guarded("CPU baseline",
                       lambda: cpu_baseline(w, pulse, args.cpu_steps, every, learned_ops, hyb_head))
        if latency and "error" not in latency:
            oracle_legs = _guarded("oracle of the latency legs", lambda: oracle_latency_legs(latency))
            for k, v in latency.items():
                if k.startswith("_"):
                    continue
                v[0].update(oracle_legs.get(k, {}) if isinstance(oracle_legs, dict) else {})
    if latency and "error" not in latency:
        latency = {k: v[0] for k, v in latency.items() if not k.startswith("_")}

    line = {
        "metric": "coupled Schwarz steps/s (FOM-OpInf hybrid, <=1e-3 rel err target vs FOM-FOM)",
        "value": value,
        "unit": "controller steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 convergence sums)",
        "data": "synthetic (seeded Gaussian pulse; operators learned on the GPU from a FOM-FOM run)",
        "config": {"workload": w.name, "bar": "24x24x240 hex8, [0,0.1]^2x[0,1] m, E=1e9 nu=0.25 rho=1000",
                   "subdomains": "z node layers 0-144 FOM, 96-240 linear OpInf", "r": learned["r"],
                   "r_s": learned["r_s"], "lambda_star": learned["lambda_star"],
                   "controller_steps_per_run": n, "dt": w.dt, "train_snapshots": w.train_steps,
                   "schwarz_initial_guess": "predictor" if w.guess else "hold",
                   "parallelism": "single GPU"},
        "schwarz_iters_per_step": iters / n,
        "fom_fom_steps_per_s": fom_fom_value,
        "speedup_vs_fom_fom": value / fom_fom_value,
        "rel_err_vs_fom_fom": {"fom_subdomain": errs[0], "opinf_subdomain": errs[1]},
        "rel_err_vs_fp64_oracle": (cpu or {}).get("rel_err_vs_fp64_oracle"),
        "fe_dof_updates_per_s": dof_updates_per_s,
        "fe_kernel_avg_us": fe_avg_us,
        "rom_kernel_avg_us": 1e3 * rom_ms / max(rom_launches, 1),
        "sweep_kernel_avg_us": k_avg_us if fused else None,
        "train_run_s": t_train,
        "learn_s": t_learn,
        "launch": {"hybrid": tuning, "fom_fom": ff_tuning, "autotune_s": t_tune},
        "roofline": {"bound": "hbm", "achieved": k_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": k_gbs / HBM_PEAK_GBS, "traffic": traffic_bytes,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_source": traffic_src,
                     "kernel": ("sweep_kernel<float, 1, 0, true> (FE step + OpInf step in one launch; every "
                                "workgroup first takes the previous sweep's convergence decision)" if fused
                                else "fe_lds_kernel<step> + boundary fe_kernel<float, step>"
                                if tuning["fe"][0][0] == 1024 else "fe_kernel<float, step>"),
                     "kernel_avg_us": k_avg_us,
                     "launch_shape": ([512, tuning["fusion_kc"]] if fused else tuning["fe"][0]),
                     "bytes_per_dof": FE_BYTES_PER_DOF, "kernel_bytes_per_dof": FE_KERNEL_BYTES_PER_DOF,
                     "dofs_per_launch": fe_dofs,
                     "algorithmic_bytes_per_launch": alg_bytes, "fe_bytes_per_launch": fe_alg,
                     "rom_bytes_per_launch": rom_alg if fused else None},
        "cpu_baseline": cpu,
        "batched_opinf_opinf": batched,
        "adjoint": adjoint,
        "large_fe": large_fe,
        "latency_legs_bar_4x4x40": latency,
        "hybrid_bar_24x24x240_other_readings": survey,
    }
    print(json.dumps(line), flush=True)


def large_fe_timing(log):
    """The FE step kernel at the 64x64x640 bar's size: three FOM slabs, 16 instances of seeded
    multi-pulse initial velocities, the middle slab's launches timed with HIP events over a few
    controller steps (the launch shape the library picks by default).  A failure is reported in
    the result instead of ending the bench."""
    import torch
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import CFG5, draw_multi_pulse_v
    from paper_2511_20687_amd.profiling import read_traffic
    w = CFG5
    try:
        ctx = osam.Context(0, "f32", w.batch)
        sds = osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
        mid = sds[1]
        u0 = np.zeros((3, w.bar.n_nodes))
        for b, mp in enumerate(draw_multi_pulse_v(w.seed, w.batch)):
            ctx.set_initial(b, u0, mp.v0(w.bar))
        opts = osam.Options(tol_abs=w.tol_abs, tol_rel=w.tol_rel, guess=w.guess)
        ctx.run(2, opts)
        ctx.set_timing(True)
        ctx.run(6, opts)
        torch.cuda.synchronize()
        ms, launches = ctx.get_timing(mid)
        ctx.set_timing(False)
        us = 1e3 * ms / max(launches, 1)
        dofs = ctx.sizes(mid)["n_free"] * w.batch
        alg = FE_BYTES_PER_DOF * dofs
        gbs = alg / (us * 1e-6) / 1e9
        traffic, src = read_traffic("bar64")
        block, kc = ctx.get_fe_launch(mid)
        del ctx
        torch.cuda.empty_cache()
        log(f"large FE step: {us:.1f} us per launch, {gbs:.0f} GB/s algorithmic")
        return {"workload": "fom_bar_64x64x640_b16 (middle of three FOM slabs, FE step)", "fe_kernel_avg_us": us,
                "launches": launches, "dofs_per_launch": dofs, "algorithmic_bytes_per_launch": alg,
                "achieved_GBs": gbs, "peak_GBs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS,
                "traffic": traffic, "traffic_source": src, "launch_shape": [block, kc]}
    except Exception as e:   # reported, not fatal: the headline line must still print
        log(f"large FE step failed: {e!r}")
        return {"error": repr(e)}


def adjoint_timing(log):
    """run_adjoint on the 24x24x240 bar (FOM 0-144, quadratic OpInf r=60 on 96-240 with seeded
    synthetic operators of the learned sizes), 2000 steps, checkpoints every 100 steps, misfit
    over every step, FP32; against the forward Schwarz run of the same context."""
    import torch
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import CFG4, draw_pulses, synthetic_rom
    w = CFG4
    ctx = osam.Context(0, "f32", 1)
    osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    z = ctx.sizes(1)
    R = synthetic_rom(w.seed, z["n_free"], z["n_sch"], w.r, 10, w.dt, quadratic=True, with_c=True)
    ctx.set_opinf(1, R["Phi"], R["PhiS"], R["A"], R["H"], R["B"], R["c"])
    u0 = draw_pulses(w.seed, 1, s=w.pulse_width)[0].u0(w.bar)
    n, K = w.steps, w.checkpoint
    gen = torch.Generator(device="cuda:0").manual_seed(w.seed)
    obs = {0: 1e-5 * torch.randn((n, ctx.sizes(0)["n_free"]), generator=gen, device="cuda:0"),
           1: 1e-5 * torch.randn((n, w.r), generator=gen, device="cuda:0")}
    ctx.set_initial(0, u0, np.zeros_like(u0))
    ctx.run_adjoint(50, 25, 1, {0: obs[0][:50], 1: obs[1][:50]})      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, _ = ctx.run_adjoint(n, K, 1, obs)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    ctx.set_initial(0, u0, np.zeros_like(u0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run(n)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    log(f"adjoint {n} steps: {t_adj:.3f} s, forward {t_fwd:.3f} s, J={J:.6e}")
    return dict(workload=w.name, steps=n, checkpoint_every=K, precision="f32", adjoint_s=t_adj,
                forward_s=t_fwd, adjoint_over_forward=t_adj / t_fwd, J=J,
                operators="seeded synthetic, learned sizes (r=60 quadratic, r_S=10)")


def _oracle_index(model):
    """Library free-DOF index of each oracle free DOF, and library Schwarz-DOF index of each
    oracle Schwarz DOF, of a bar subdomain (argument marshalling between the two layouts)."""
    from paper_2511_20687_amd.osam import lib_dof_index
    bar = model.bar
    nzs = model.z_hi - model.z_lo
    free = lib_dof_index(bar.nx, bar.ny, nzs, model.free_dofs)
    npl = (bar.nx + 1) * (bar.ny + 1)
    node, comp = model.sch_dofs // 3, model.sch_dofs % 3
    lo_face = model.z_lo > 0
    nsch = npl * (int(lo_face) + int(model.z_hi < bar.nz))
    pos = np.where(node < npl, node, node - nzs * npl + (npl if lo_face else 0))
    return free, comp * nsch + pos


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(w, pulse, n_steps, every, ops, hyb_head):
    """FP64 oracle, one thread, on the first n_steps controller steps of the same hybrid with
    the operators the GPU learned; the error of the GPU's FP32 run against it (Eq. mse over
    the steps recorded every `every` steps, free DOFs / reduced coordinates)."""
    from threadpoolctl import threadpool_limits
    from oracle.newmark import FomModel, SubdomainGeometry
    from oracle.rom import OpInfModel
    from oracle.schwarz import Coupled, SchwarzOptions
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        lo, hi = w.layers[0]
        fom = FomModel(w.bar, lo, hi, w.dt, lateral_fix=w.lateral_fix)
        g = SubdomainGeometry(w.bar, *w.layers[1], lateral_fix=w.lateral_fix)
        free, sch = _oracle_index(g)
        rom = OpInfModel(g, ops["Phi"][free], ops["PhiS"][sch] if ops["PhiS"].shape[1] else None, ops["A"], None,
                         ops["B"] if ops["B"].shape[1] else None, None, dt=w.dt)
        cp = Coupled([fom, rom])
        u0 = pulse.u0(w.bar)
        st = cp.initial_states(u0, np.zeros_like(u0))
        t_setup = time.perf_counter() - t0
        opts = SchwarzOptions(tol_abs=w.tol_abs, tol_rel=w.tol_rel, guess="predictor" if w.guess else "hold")
        rec = [[fom.free_u(st[0])], [st[1].q.copy()]]
        t0 = time.perf_counter()
        its = 0
        for k in range(1, n_steps + 1):
            st, info = cp.step(st, opts)
            its += info.iters
            if k % every == 0:
                rec[0].append(fom.free_u(st[0]))
                rec[1].append(st[1].q.copy())
        t = time.perf_counter() - t0
    ffree, _ = _oracle_index(fom)
    errs = {"fom_subdomain": _rel(hyb_head[0][:, ffree], np.array(rec[0])),
            "opinf_subdomain": _rel(hyb_head[1], np.array(rec[1])),
            "steps_compared": f"0..{n_steps} every {every} (FP32 GPU run vs this FP64 oracle run)"}
    return {"value": n_steps / t, "unit": "controller steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_steps} controller steps of the same FOM-OpInf hybrid with the operators the GPU "
                      f"learned (FP64 numpy/scipy, one thread; setup {t_setup:.1f} s excluded; "
                      f"{its / n_steps:.2f} Schwarz iterations/step)",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(), "rel_err_vs_fp64_oracle": errs}


def oracle_latency_legs(legs):
    """The FP64 oracle on each 4x4x40 leg (full length, one thread): its steps/s and the Eq. mse
    error of the GPU's FP64 records against it."""
    from threadpoolctl import threadpool_limits
    from oracle.newmark import FomModel
    from oracle.schwarz import Coupled, SchwarzOptions
    from oracle.svk import SvkFomModel
    inp = legs["_inputs"]
    bar, layers = inp["bar"], inp["layers"]
    out = {}
    for name, leg in legs.items():
        if name.startswith("_"):
            continue
        res, recs = leg
        models = []
        for (lo, hi), beta, ns in zip(layers, res["beta"], res["n_sub"]):
            cls = SvkFomModel if res["material"] == "svk" else FomModel
            m = cls(bar, lo, hi, res["dt"] / ns, lateral_fix=(0, 1)) if cls is SvkFomModel else \
                cls(bar, lo, hi, res["dt"] / ns, beta=beta, lateral_fix=(0, 1))
            m.n_sub = ns
            models.append(m)
        u0 = inp["u_svk"] if res["material"] == "svk" else inp["u0"]
        n = res["controller_steps"]
        every = n // (recs[0].shape[0] - 1)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            ref = Coupled(models).run(u0, np.zeros_like(u0), n, SchwarzOptions(), every=every, record=("u",))
            t = time.perf_counter() - t0
        errs = [_rel(recs[i][:, _oracle_index(m)[0]], ref["u"][i]) for i, m in enumerate(models)]
        out[name] = {"rel_err_vs_fp64_oracle": errs, "oracle_steps_per_s": n / t,
                     "oracle_iters_per_step": float(ref["iters"].mean()), "gpu_vs_oracle_speed": res["steps_per_s"] * t / n}
    return out


if __name__ == "__main__":
    main()
