"""Batched OpInf-OpInf coupling on the 48x48x480 bar against FOM-FOM on the same GPU.

Quadratic OpInf (Sec. 3.2, Eq. quadratic_opinf; r = 100, H 100 x 5050) on both overlapping
subdomains, coupled by the multiplicative Schwarz loop (Alg. 1, Sec. 4.2.3), for a batch of 256
seeded Gaussian pulses (amplitude U[0.5, 2] 1e-3, centre U[0.15, 0.35]).

Training set (a reading: the configuration leaves it open): FOM-FOM runs of 2000 steps with the
pulses of draws 257, 258, ... of the same seed stream (w.train_runs of them), snapshots every
w.train_stride steps, so T = 2000 per subdomain over all runs.  Learning per subdomain (Alg. 2):
POD with the energy criterion for the boundary basis, the quadratic fit, Alg. 3 over the
11-value grid.  Online: draws 1-256, 2000 steps, in FP32 and in the BF16-H precision, on the
single-step path and on the persistent OpInf engine.
Reported: batched OpInf-OpInf steps/s (x 256 instances); FOM-FOM steps/s for the same 256
instances on the same GPU, timed over its whole 2000-step run (recording every `every` steps);
and the Eq. mse error of the OpInf-OpInf displacement against that FOM-FOM run for every
instance (mean, max, and the share of instances within the 1e-3 target), with target_met.
"""
from __future__ import annotations

import time

import numpy as np


def _train_and_learn(w, log):
    import torch
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import draw_pulses, lambda_grid_values
    ntr, stride = w.train_runs, w.train_stride
    T = w.train_steps // stride
    ctx = osam.Context(0, "f32", ntr)
    sds = osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    dev = "cuda:0"
    rec = {}
    for sd in sds:
        z = ctx.sizes(sd)
        rec[sd] = (torch.zeros((ntr, T, z["n_free"]), device=dev), torch.zeros((ntr, T, z["n_free"]), device=dev),
                   torch.zeros((ntr, T, z["n_sch"]), device=dev))
        ctx.set_record(sd, stride, T, u=rec[sd][0], a=rec[sd][1], s=rec[sd][2])
    for b, p in enumerate(draw_pulses(w.seed, ntr, skip=256, s=w.pulse_width)):
        u0 = p.u0(w.bar)
        ctx.set_initial(b, u0, np.zeros_like(u0))
    opts = osam.Options(tol_abs=w.tol_abs, tol_rel=w.tol_rel, min_iter=w.min_iter, max_iter=w.max_iter,
                        guess=w.guess)
    t0 = time.perf_counter()
    ctx.run(stride * (T - 1), opts)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"training: {ntr} FOM-FOM runs of {stride * (T - 1)} steps in {t_train:.2f} s")
    # the workload's form, and a linear model of the same size from the same snapshots (the
    # elastodynamics are linear: the comparison shows what the quadratic term costs in accuracy)
    ops, learned, t_learn = {}, {}, {}
    for form in (w.form, "linear"):
        lctx = ctx if form == w.form else osam.Context(0, "f32", ntr)
        if form != w.form:
            osam.add_bar_subdomains(lctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
        ops[form], learned[form] = {}, {}
        t0 = time.perf_counter()
        for sd in sds:
            z = lctx.sizes(sd)
            V0 = torch.zeros((ntr, z["n_free"]), device=dev)
            out = lctx.learn_opinf(sd, rec[sd][0], rec[sd][1], rec[sd][2], V0, ntr, T, form=form, r=w.r, r_s=0,
                                   energy_bnd=1 - 1e-6, lambdas=lambda_grid_values(11), stride=stride)
            learned[form][sd] = dict(r=out["r"], r_s=out["r_s"], lambda_star=out["lambda_star"])
            ops[form][sd] = lctx.get_opinf(sd, quadratic=form != "linear")
            torch.cuda.synchronize()
        t_learn[form] = time.perf_counter() - t0
        log(f"learning ({form}): {learned[form]} in {t_learn[form]:.2f} s")
        del lctx
    del rec, ctx
    return ops, learned, t_train, t_learn


def _initial(ctx, w, n, skip=0):
    from paper_2511_20687_amd.inputs import draw_pulses
    for b, p in enumerate(draw_pulses(w.seed, n, skip=skip, s=w.pulse_width)):
        u0 = p.u0(w.bar)
        ctx.set_initial(b, u0, np.zeros_like(u0))


def run(w=None, every=400, log=print) -> dict:
    import torch
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import CFG3
    w = w or CFG3
    B, n = w.batch, w.steps
    opts = osam.Options(tol_abs=w.tol_abs, tol_rel=w.tol_rel, min_iter=w.min_iter, max_iter=w.max_iter,
                        guess=w.guess)
    ops, learned, t_train, t_learn = _train_and_learn(w, log)
    dev = "cuda:0"
    ncol = n // every + 1
    result = dict(workload=w.name, batch=B, steps=n, schwarz_initial_guess="predictor" if w.guess else "hold",
                  train_runs=w.train_runs, train_stride=w.train_stride, train_s=t_train, learn_s=t_learn,
                  learned={form: {str(k): v for k, v in lf.items()} for form, lf in learned.items()})
    qrec = {}
    # engine 0: the single-step path (batched f0 on the matrix cores, fused sweeps, graphs;
    # autotuned); engine 2: the persistent OpInf engine (all steps in one launch)
    variants = {"f32": (w.form, "f32", 0), "f32_bf16h": (w.form, "f32_bf16h", 0), "linear_f32": ("linear", "f32", 0),
                "f32_persistent": (w.form, "f32", 2), "linear_f32_persistent": ("linear", "f32", 2)}
    for key, (form, prec, engine) in variants.items():
        ctx = osam.Context(0, prec, B)
        sds = osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
        for sd in sds:
            o = ops[form][sd]
            ctx.set_opinf(sd, o["Phi"], o["PhiS"], o["A"], o["H"], o["B"], o["c"])
        _initial(ctx, w, B)
        if engine == 0:
            tune = ctx.autotune(trial_steps=50, opts=opts)
        else:
            ctx.set_engine(engine)
            tune = "persistent OpInf engine (one launch, one workgroup per instance)"
        recs = [torch.zeros((B, ncol, learned[form][sd]["r"]), device=dev) for sd in sds]
        for sd in sds:
            ctx.set_record(sd, every, ncol, u=recs[sd])
        _initial(ctx, w, B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.run(n, opts)
        torch.cuda.synchronize()
        dt_run = time.perf_counter() - t0
        iters = float(np.mean([i["total_iters"] for i in info])) / n
        result[key] = dict(form=form, precision=prec, engine=engine, steps_per_s=n / dt_run,
                           instance_steps_per_s=B * n / dt_run, schwarz_iters_per_step=iters, launch=tune)
        log(f"OpInf-OpInf {key}: {n / dt_run:.0f} steps/s x {B} instances, {iters:.2f} iterations/step")
        qrec[key] = recs
        del ctx
        torch.cuda.synchronize()

    # FOM-FOM for the same 256 instances on the same GPU: timed over the whole run, which also
    # records the reference displacements every `every` steps
    ff = osam.Context(0, "f32", B)
    sds = osam.add_bar_subdomains(ff, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    _initial(ff, w, B)
    ff_tune = ff.autotune(trial_steps=3, opts=opts)
    frec = [torch.zeros((B, ncol, ff.sizes(sd)["n_free"]), device=dev) for sd in sds]
    for sd in sds:
        ff.set_record(sd, every, ncol, u=frec[sd])
    _initial(ff, w, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ff.run(n, opts)
    torch.cuda.synchronize()
    t_ff = time.perf_counter() - t0
    result["fom_fom"] = dict(steps_per_s=n / t_ff, instance_steps_per_s=B * n / t_ff, timed_steps=n,
                             launch=ff_tune, note=f"timed run records every {every} steps")
    log(f"FOM-FOM: {n / t_ff:.1f} steps/s x {B} instances")
    del ff
    # accuracy of every instance (the lift Phi q one instance at a time)
    from paper_2511_20687_amd.inputs import draw_pulses
    pulses = draw_pulses(w.seed, B, s=w.pulse_width)
    for key, (form, prec, _) in variants.items():
        Phis = [torch.tensor(np.ascontiguousarray(ops[form][sd]["Phi"].T), dtype=torch.float32, device=dev)
                for sd in sds]
        errs = []
        for b in range(B):
            num = den = 0.0
            for sd in sds:
                lifted = torch.matmul(qrec[key][sd][b], Phis[sd]).double()    # [ncol][n_free]
                ref = frec[sd][b].double()
                num += float(torch.sum((lifted - ref) ** 2))
                den += float(torch.sum(ref ** 2))
            errs.append((num / den) ** 0.5)
        errs = np.array(errs)
        worst = [dict(instance=int(b), err=float(errs[b]), a=pulses[b].a, b=pulses[b].b)
                 for b in np.argsort(errs)[-3:][::-1]]
        result[key]["rel_err_vs_fom_fom"] = dict(mean=float(errs.mean()), max=float(errs.max()),
                                                 median=float(np.median(errs)),
                                                 within_1e3=float(np.mean(errs <= 1e-3)), instances=B,
                                                 record_every=every, worst=worst)
        result[key]["target_met"] = bool(errs.mean() <= 1e-3)
        result[key]["speedup_vs_fom_fom"] = result[key]["steps_per_s"] / result["fom_fom"]["steps_per_s"]
        log(f"OpInf-OpInf {key} error vs FOM-FOM over {B} instances: mean {errs.mean():.3e}, "
            f"max {errs.max():.3e}, within 1e-3: {np.mean(errs <= 1e-3):.2f}; worst {worst}")
        del Phis
    result["speedup_vs_fom_fom"] = result["f32"]["speedup_vs_fom_fom"]
    result["target_met"] = result["f32"]["target_met"]
    met = [k for k in variants if result[k]["target_met"]]
    result["variants_meeting_target"] = met
    del frec, qrec
    torch.cuda.synchronize()
    return result


if __name__ == "__main__":
    import json
    import sys
    print(json.dumps(run(log=lambda m: print(m, file=sys.stderr, flush=True))))
