"""Batched OpInf-OpInf coupling on the 48x48x480 bar against FOM-FOM on the same GPU.

Quadratic OpInf (Sec. 3.2, Eq. quadratic_opinf; r = 100, H 100 x 5050) on both overlapping
subdomains, coupled by the multiplicative Schwarz loop (Alg. 1, Sec. 4.2.3), for a batch of 256
seeded Gaussian pulses (amplitude U[0.5, 2] 1e-3, centre U[0.15, 0.35]).

Training set (a reading: the configuration leaves it open): 4 FOM-FOM runs of 2000 steps with
the pulses of draws 257-260 of the same seed stream, snapshots every 4 steps, so T = 2000 per
subdomain.  Learning per subdomain (Alg. 2): POD with the energy criterion for the boundary
basis, the quadratic fit, Alg. 3 over the 11-value grid.  Online: draws 1-256, 2000 steps, in
FP32 and in the BF16-H precision.  Reported: batched OpInf-OpInf steps/s (x 256 instances),
FOM-FOM steps/s for the same 256 instances on the same GPU, and the Eq. mse error of the
OpInf-OpInf displacement against FOM-FOM on the first n_acc instances.
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
    ops, learned = {}, {}
    t0 = time.perf_counter()
    for sd in sds:
        z = ctx.sizes(sd)
        V0 = torch.zeros((ntr, z["n_free"]), device=dev)
        out = ctx.learn_opinf(sd, rec[sd][0], rec[sd][1], rec[sd][2], V0, ntr, T, form=w.form, r=w.r, r_s=0,
                              energy_bnd=1 - 1e-6, lambdas=lambda_grid_values(11), stride=stride)
        learned[sd] = dict(r=out["r"], r_s=out["r_s"], lambda_star=out["lambda_star"])
        ops[sd] = ctx.get_opinf(sd, quadratic=True)
        del rec[sd]
        torch.cuda.synchronize()
    t_learn = time.perf_counter() - t0
    log(f"learning: {learned} in {t_learn:.2f} s")
    del ctx
    return ops, learned, t_train, t_learn


def _initial(ctx, w, n, skip=0):
    from paper_2511_20687_amd.inputs import draw_pulses
    for b, p in enumerate(draw_pulses(w.seed, n, skip=skip, s=w.pulse_width)):
        u0 = p.u0(w.bar)
        ctx.set_initial(b, u0, np.zeros_like(u0))


def run(w=None, n_acc=16, fom_steps=100, every=100, log=print) -> dict:
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
                  train_s=t_train, learn_s=t_learn,
                  learned={str(k): v for k, v in learned.items()})
    lifted = {}
    for prec in ("f32", "f32_bf16h"):
        ctx = osam.Context(0, prec, B)
        sds = osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
        for sd in sds:
            o = ops[sd]
            ctx.set_opinf(sd, o["Phi"], o["PhiS"], o["A"], o["H"], o["B"], o["c"])
        _initial(ctx, w, B)
        tune = ctx.autotune(trial_steps=50, opts=opts)
        recs = [torch.zeros((B, ncol, learned[sd]["r"]), device=dev) for sd in sds]
        for sd in sds:
            ctx.set_record(sd, every, ncol, u=recs[sd])
        _initial(ctx, w, B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.run(n, opts)
        torch.cuda.synchronize()
        dt_run = time.perf_counter() - t0
        iters = float(np.mean([i["total_iters"] for i in info])) / n
        result[prec] = dict(steps_per_s=n / dt_run, instance_steps_per_s=B * n / dt_run,
                            schwarz_iters_per_step=iters, launch=tune)
        log(f"OpInf-OpInf {prec}: {n / dt_run:.0f} steps/s x {B} instances, {iters:.2f} iterations/step")
        lifted[prec] = []
        for sd in sds:
            PhiT = torch.tensor(np.ascontiguousarray(ops[sd]["Phi"].T), dtype=torch.float32, device=dev)
            lifted[prec].append(torch.matmul(recs[sd][:n_acc].contiguous(), PhiT))   # [n_acc][ncol][n_free]
            del PhiT
        del ctx, recs
        torch.cuda.synchronize()

    # FOM-FOM throughput for the same 256 instances on the same GPU
    ff = osam.Context(0, "f32", B)
    osam.add_bar_subdomains(ff, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    _initial(ff, w, B)
    ff_tune = ff.autotune(trial_steps=3, opts=opts)
    _initial(ff, w, B)
    ff.run(2, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ff.run(fom_steps, opts)
    torch.cuda.synchronize()
    t_ff = time.perf_counter() - t0
    result["fom_fom"] = dict(steps_per_s=fom_steps / t_ff, instance_steps_per_s=B * fom_steps / t_ff,
                             timed_steps=fom_steps, launch=ff_tune)
    log(f"FOM-FOM: {fom_steps / t_ff:.1f} steps/s x {B} instances")
    del ff
    torch.cuda.synchronize()

    # accuracy: FOM-FOM trajectories of the first n_acc instances
    fa = osam.Context(0, "f32", n_acc)
    sds = osam.add_bar_subdomains(fa, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    frec = [torch.zeros((n_acc, ncol, fa.sizes(sd)["n_free"]), device=dev) for sd in sds]
    for sd in sds:
        fa.set_record(sd, every, ncol, u=frec[sd])
    _initial(fa, w, n_acc)
    fa.run(n, opts)
    torch.cuda.synchronize()
    for prec in ("f32", "f32_bf16h"):
        errs = []
        for b in range(n_acc):
            num = sum(float(torch.sum((lifted[prec][sd][b].double() - frec[sd][b].double()) ** 2)) for sd in sds)
            den = sum(float(torch.sum(frec[sd][b].double() ** 2)) for sd in sds)
            errs.append((num / den) ** 0.5)
        result[prec]["rel_err_vs_fom_fom"] = dict(mean=float(np.mean(errs)), max=float(np.max(errs)),
                                                  instances=n_acc, record_every=every)
        log(f"OpInf-OpInf {prec} error vs FOM-FOM: mean {np.mean(errs):.3e}, max {np.max(errs):.3e}")
    result["speedup_vs_fom_fom"] = result["f32"]["steps_per_s"] / result["fom_fom"]["steps_per_s"]
    del fa, frec, lifted
    torch.cuda.synchronize()
    return result


if __name__ == "__main__":
    import json
    import sys
    print(json.dumps(run(log=lambda m: print(m, file=sys.stderr, flush=True))))
