"""Latency-bound legs of the benchmark on the 4x4x40 bar (1,025 nodes, two slabs with 20%
overlap, clamped ends, lateral x and y held, FP64): one controller step costs a few launches
and one host read-back per Schwarz iteration, so the figure is microseconds per controller
step, not bandwidth.

  * explicit FOM-FOM with one Newmark step per controller step (the single-step path,
    1000 steps, HOLD guess);
  * implicit FOM-FOM (beta = 1/4, dt = 4 x the explicit step, 250 steps: the same end time);
  * implicit-explicit with mixed steps (Sec. 4.1): subdomain 1 implicit with one step per
    controller step, subdomain 2 explicit with four (250 steps of 4 x the explicit step);
  * Saint Venant-Kirchhoff FOM-FOM (App. A.2; explicit, half the linear explicit step,
    a 2 cm pulse: strains of about 0.1; 200 steps).

Each leg returns its throughput, iteration counts and the recorded displacements of every
subdomain (every `every` steps) for the comparison with the FP64 oracle that bench.py runs
on the host.
"""
from __future__ import annotations

import time

import numpy as np


def _leg(name, bar, layers, dt, n, betas, subs, material, u0, every, log, opts=None, warm=1, tune=False):
    import torch
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import Bar  # noqa: F401
    ctx = osam.Context(0, "f64", 1)
    osam.add_bar_subdomains(ctx, bar, layers, dt, lateral_fix=(0, 1), beta=list(betas), n_sub=list(subs),
                            material=material)
    o = opts or osam.Options()
    v0 = np.zeros_like(u0)
    tuning = None
    if tune:
        # the single-step path's launch configuration for this shape (fused sweeps, graphs)
        ctx.set_initial(0, u0, v0)
        tuning = ctx.autotune(trial_steps=200, opts=o)
    for _ in range(warm):
        ctx.set_initial(0, u0, v0)
        ctx.run(n, o)
    ctx.set_initial(0, u0, v0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = ctx.run(n, o)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    # records of the same run (separate pass, not timed)
    ncol = n // every + 1
    recs = []
    for sd in range(len(layers)):
        z = ctx.sizes(sd)
        r = torch.zeros((1, ncol, z["n_free"]), dtype=torch.float64, device="cuda:0")
        ctx.set_record(sd, every, ncol, u=r)
        recs.append(r)
    ctx.set_initial(0, u0, v0)
    ctx.run(n, o)
    solver = [max(ctx.solver_stats(sd)) for sd in range(len(layers))]
    out = {"controller_steps": n, "steps_per_s": n / t, "us_per_step": 1e6 * t / n,
           "schwarz_iters_per_step": info[0]["total_iters"] / n, "max_iters": info[0]["max_iters"],
           "max_solver_iters": solver, "dt": dt, "beta": list(betas), "n_sub": list(subs),
           "material": material, "launch": tuning,
           "bound": "latency (a few launches per Schwarz iteration, one host read-back per controller step)"}
    log(f"{name}: {out['us_per_step']:.1f} us/step, {out['schwarz_iters_per_step']:.2f} iterations/step")
    return out, [r[0].cpu().numpy() for r in recs]


def run(log):
    """The four legs on the 4x4x40 bar; returns {name: (result, records)}."""
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import CFG1, gaussian_pulse_u
    w = CFG1
    bar, layers = w.bar, w.layers
    dtx = w.dt
    u0 = gaussian_pulse_u(bar, 1e-3, 0.25, 0.05)
    legs = {}
    legs["explicit_fom_fom"] = _leg("explicit FOM-FOM (single-step path)", bar, layers, dtx, 1000, (0.0, 0.0),
                                    (1, 1), "linear", u0, 50, log, tune=True)
    legs["implicit_fom_fom"] = _leg("implicit FOM-FOM", bar, layers, 4 * dtx, 250, (0.25, 0.25), (1, 1), "linear",
                                    u0, 10, log)
    legs["implicit_explicit_mixed_steps"] = _leg("implicit / explicit x4", bar, layers, 4 * dtx, 250, (0.25, 0.0),
                                                 (1, 4), "linear", u0, 10, log)
    u_svk = gaussian_pulse_u(bar, 2e-2, 0.25, 0.05)
    legs["svk_fom_fom"] = _leg("SVK FOM-FOM", bar, layers, 0.5 * dtx, 200, (0.0, 0.0), (1, 1), "svk", u_svk, 10,
                               log)
    legs["_inputs"] = {"u0": u0, "u_svk": u_svk, "dt_explicit": dtx, "bar": bar, "layers": layers,
                       "opts": osam.Options()}
    return legs
