"""The 24x24x240 FOM-OpInf hybrid under other readings of its inputs.

The headline run holds x and y at zero on the lateral faces and uses a pulse of width
s = 0.02, as the bar of Sec. 5.1 does.  This leg runs the same pipeline (FOM-FOM training
run of 2000 steps, Alg. 2 with Alg. 3 over the 11-value lambda grid, online FOM-OpInf run of
5000 steps, PREDICTOR guess, FP32) with traction-free lateral faces and with s = 0.05, and
reports for each case:
  * the POD energy ranks of the training snapshots (smallest r with E_r >= 1 - 1e-4 and
    1 - 1e-6, Eq. pod_energy; "> 128" past the library's largest basis);
  * for r = 40, 80 and 120: lambda*, the frozen-boundary rollout error Alg. 3 found for it, the
    Eq. mse error of the hybrid against the FOM-FOM run over the whole online run, and how many
    eigenvalues of the learned A lie off the negative real axis (modes that the explicit step
    does not keep bounded);
  * the smallest of those r whose error is within 1e-3, or None.
"""
from __future__ import annotations

import numpy as np

R_VALUES = (40, 80, 120)
CASES = (("traction_free", (), 0.05), ("traction_free", (), 0.02), ("lateral_xy_held", (0, 1), 0.05))


def _energy_rank(ctx, sd, U, A, S, V0, T, energy):
    from paper_2511_20687_amd import osam
    try:
        out = ctx.learn_opinf(sd, U, A, S, V0, 1, T, r=0, r_s=0, energy=energy, energy_bnd=1 - 1e-6,
                              lambdas=[1e-6])
        return int(out["r"])
    except osam.OsamError as e:
        if "larger than 128" in str(e):
            return "> 128"
        raise


def run(log=print, every=10) -> dict:
    import torch
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import CFG2, draw_pulses, lambda_grid_values
    base = CFG2
    opts = osam.Options(tol_abs=base.tol_abs, tol_rel=base.tol_rel, min_iter=base.min_iter,
                        max_iter=base.max_iter, guess=base.guess)
    dev = "cuda:0"
    n, T = base.steps, base.train_steps
    ncol = n // every + 1
    result = dict(workload=base.name, online_steps=n, train_snapshots=T, r_values=list(R_VALUES), cases=[])
    for name, lateral, s in CASES:
        pulse = draw_pulses(base.seed, 1, s=s)[0]
        u0 = pulse.u0(base.bar)
        v0 = np.zeros_like(u0)

        def context():
            c = osam.Context(0, base.precision, 1)
            osam.add_bar_subdomains(c, base.bar, base.layers, base.dt, lateral_fix=lateral)
            return c

        # training run: snapshots of subdomain 2
        tr = context()
        z = tr.sizes(1)
        U = torch.zeros((1, T, z["n_free"]), device=dev)
        A = torch.zeros((1, T, z["n_free"]), device=dev)
        S = torch.zeros((1, T, z["n_sch"]), device=dev)
        tr.set_record(1, 1, T, u=U, a=A, s=S)
        tr.set_initial(0, u0, v0)
        tr.run(T - 1, opts)
        V0 = torch.zeros((1, z["n_free"]), device=dev)
        ranks = {}
        for e in (1 - 1e-4, 1 - 1e-6):
            ranks[f"{e:.6f}"] = _energy_rank(context(), 1, U, A, S, V0, T, e)
        # FOM-FOM reference of the online run
        ff = context()
        frec = [torch.zeros((1, ncol, ff.sizes(sd)["n_free"]), device=dev) for sd in range(2)]
        for sd in range(2):
            ff.set_record(sd, every, ncol, u=frec[sd])
        ff.set_initial(0, u0, v0)
        ff.run(n, opts)
        refs = [f[0].double() for f in frec]
        del frec, ff
        rows = []
        for r in R_VALUES:
            c = context()
            out = c.learn_opinf(1, U, A, S, V0, 1, T, form="linear", r=r, r_s=0, energy_bnd=1 - 1e-6,
                                lambdas=lambda_grid_values(11))
            ops = c.get_opinf(1)
            ev = np.linalg.eigvals(ops["A"])
            off_axis = int(np.sum((np.abs(ev.imag) > 1e-9 * np.abs(ev).max()) | (ev.real > 0)))
            recs = [torch.zeros((1, ncol, c.sizes(0)["n_free"]), device=dev),
                    torch.zeros((1, ncol, r), device=dev)]
            for sd in range(2):
                c.set_record(sd, every, ncol, u=recs[sd])
            c.set_initial(0, u0, v0)
            info = c.run(n, opts, check=False)
            Phi = torch.tensor(ops["Phi"], dtype=torch.float64, device=dev)
            hyb = [recs[0][0].double(), (Phi @ recs[1][0].double().T).T]
            num = sum(float(torch.sum((h - f) ** 2)) for h, f in zip(hyb, refs))
            den = sum(float(torch.sum(f ** 2)) for f in refs)
            finite = info[0]["status"] == 0 and np.isfinite(num)
            err = (num / den) ** 0.5 if finite else None     # None: the hybrid went non-finite
            e_star = float(np.min(out["E_lambda"]))
            rows.append(dict(r=r, r_s=out["r_s"], lambda_star=out["lambda_star"],
                             alg3_rollout_error=e_star if np.isfinite(e_star) else None,
                             rel_err_vs_fom_fom=err, eigenvalues_off_negative_axis=off_axis))
            log(f"survey readings {name} s={s}: r={r} lambda*={out['lambda_star']:.0e} err={err} "
                f"A eigenvalues off the negative axis: {off_axis}")
            del c, recs, hyb, Phi
        met = [row["r"] for row in rows if row["rel_err_vs_fom_fom"] is not None and row["rel_err_vs_fom_fom"] <= 1e-3]
        result["cases"].append(dict(lateral=name, pulse_width=s, energy_rank=ranks, runs=rows,
                                    smallest_r_within_1e3=min(met) if met else None))
        del U, A, S, V0, refs, tr
        torch.cuda.synchronize()
    return result


if __name__ == "__main__":
    import json
    import sys
    print(json.dumps(run(log=lambda m: print(m, file=sys.stderr, flush=True))))
