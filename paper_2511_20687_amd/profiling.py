"""Profiling helpers for the FE step kernel and the fused sweep kernel on the 24x24x240 bar
(FOM-OpInf coupling).

Used under rocprofv3 to produce the summaries in profiles/:

    python -m paper_2511_20687_amd.profiling workload [steps [fused]]  # coupled run, synthetic r=40 OpInf
    python -m paper_2511_20687_amd.profiling large [steps [block kc]]  # 64x64x640, OpInf-FOM-OpInf, B=16
    python -m paper_2511_20687_amd.profiling copy               # plain copy of 256 MiB (calibration)
    python -m paper_2511_20687_amd.profiling rom [steps [bf16]]  # 48x48x480 OpInf-OpInf r=100 quadratic, B=256
    python -m paper_2511_20687_amd.profiling learn [T [r]]      # learning on 268,125 x T seeded snapshots
    python -m paper_2511_20687_amd.profiling summarize OUTDIR [bar24|bar64|bar24_sweep]   # counters -> profiles/*.txt

The workload runs exactly the FE kernel work of the bench (same subdomain, launch shape and
coupling pattern); the OpInf operators are seeded synthetic ones of the learned sizes, so no
training run is needed.  The calibration copy lets the FETCH_SIZE / WRITE_SIZE counters
be scaled to bytes: scale = known bytes / counted bytes of the copy kernel.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 256 << 20
# algorithmic FP32 bytes per FE DOF-iteration-update (read u, v, a and the previous iterate's
# u, v; write u, v, a; the lumped mass, 4 B per node)
FE_ALG_BYTES = 32.0 + 4.0 / 3.0
_CSRC = "paper_2511_20687_amd/csrc/"
SOURCES = {   # the sources each profiled kernel is built from
    "fe": tuple(_CSRC + f for f in ("fe_kernels.hip", "fe_body.hpp", "stencil.hpp", "osam_device.hpp")),
    "sweep": tuple(_CSRC + f for f in ("sweep_kernels.hip", "fe_body.hpp", "rom_body.hpp", "stencil.hpp",
                                       "osam_device.hpp")),
}


def source_hash(kernel: str = "fe") -> str:
    h = hashlib.sha256()
    for rel in SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def rom_bytes_per_launch(r: int, rs: int, n_in: int, n_exp: int) -> float:
    """FP32 algorithmic bytes of one OpInf step launch (fused path, one instance): A, B,
    the Phi_S block and values of the FOM-fed face, the Pi Phi rows and values of the push,
    and the reduced state (3 r read, 3 r written)."""
    return 4.0 * (r * r + r * rs + rs * n_in + n_in + r * n_exp + n_exp + 6 * r)


def workload(steps: int = 200, fused: bool = False) -> None:
    import torch
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import CFG2, draw_pulses, synthetic_rom
    w = CFG2
    ctx = osam.Context(0, w.precision, 1)
    osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    z = ctx.sizes(1)
    R = synthetic_rom(w.seed, z["n_free"], z["n_sch"], w.r, 1, w.dt)
    ctx.set_opinf(1, R["Phi"], R["PhiS"], R["A"], None, R["B"])
    u0 = draw_pulses(w.seed, 1, s=w.pulse_width)[0].u0(w.bar)
    ctx.set_initial(0, u0, np.zeros_like(u0))
    if fused:
        ctx.set_fusion(True, 1)
    info = ctx.run(steps, osam.Options(tol_abs=w.tol_abs, tol_rel=w.tol_rel))
    torch.cuda.synchronize()
    print(f"workload done: {steps} steps{' (fused sweeps)' if fused else ''}, {info[0]['total_iters']} "
          f"Schwarz iterations, {z['n_free']} FE DOFs", flush=True)


def large_context(steps: int = 0):
    """The 64x64x640 three-subdomain hybrid (quadratic OpInf r=120 outer subdomains, FOM middle)
    with 16 instances of the seeded multi-pulse initial velocity; OpInf operators are seeded
    synthetic ones of the sizes this configuration learns (H 120 x 7260)."""
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import CFG5, draw_multi_pulse_v, synthetic_rom
    w = CFG5
    ctx = osam.Context(0, w.precision, w.batch)
    osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    for i, kind in enumerate(w.models):
        if kind != "opinf":
            continue
        z = ctx.sizes(i)
        R = synthetic_rom(w.seed + 10 * i, z["n_free"], z["n_sch"], w.r, 20, w.dt, quadratic=True)
        ctx.set_opinf(i, R["Phi"], R["PhiS"], R["A"], R["H"], R["B"])
        del R
    u0 = np.zeros((3, w.bar.n_nodes))
    for b, mp in enumerate(draw_multi_pulse_v(w.seed, w.batch)):
        ctx.set_initial(b, u0, mp.v0(w.bar))
    return w, ctx


def large(steps: int = 20, block: int = 0, kc: int = 0) -> None:
    import torch
    from paper_2511_20687_amd import osam
    w, ctx = large_context()
    fom = w.models.index("fom")
    if block or kc:
        ctx.set_fe_launch(fom, block, kc)
    nf = ctx.sizes(fom)["n_free"]
    opts = osam.Options(tol_abs=w.tol_abs, tol_rel=w.tol_rel)
    ctx.run(2, opts)                                   # warm-up
    ctx.set_timing(True)
    info = ctx.run(steps, opts)
    torch.cuda.synchronize()
    ms, n = ctx.get_timing(fom)
    us = 1e3 * ms / max(n, 1)
    alg = FE_ALG_BYTES * nf * w.batch
    print(f"large done: {steps} steps, {info[0]['total_iters']} Schwarz iterations (instance 0), "
          f"FE launches {n}, FE avg {us:.1f} us, {nf} FE DOFs x {w.batch} instances, "
          f"algorithmic {alg / 1e6:.1f} MB per launch -> {alg / (us * 1e-6) / 1e9:.0f} GB/s", flush=True)


def rom(steps: int = 50, bf16: bool = False) -> None:
    """Batched OpInf-OpInf on the 48x48x480 bar: quadratic r = 100 on both subdomains (H 100 x
    5050), 256 instances, the batched path (f0 on the matrix cores), PREDICTOR guess; seeded
    synthetic operators of the learned sizes."""
    import torch
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import CFG3, draw_pulses, synthetic_rom
    w = CFG3
    ctx = osam.Context(0, "f32_bf16h" if bf16 else "f32", w.batch)
    osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    for sd in range(2):
        z = ctx.sizes(sd)
        R = synthetic_rom(w.seed + sd, z["n_free"], z["n_sch"], w.r, 1, w.dt, quadratic=True)
        ctx.set_opinf(sd, R["Phi"], R["PhiS"], R["A"], R["H"], R["B"])
        ctx.set_rom_path(sd, 2)
    for b, p in enumerate(draw_pulses(w.seed, w.batch, s=w.pulse_width)):
        u0 = p.u0(w.bar)
        ctx.set_initial(b, u0, np.zeros_like(u0))
    info = ctx.run(steps, osam.Options(tol_abs=w.tol_abs, tol_rel=w.tol_rel, guess=w.guess))
    torch.cuda.synchronize()
    print(f"rom done: {steps} steps x {w.batch} instances, {info[0]['total_iters']} iterations (instance 0)",
          flush=True)


def learn(T: int = 2000, r: int = 40) -> None:
    """OpInf learning (POD by the FP64 Gram on the matrix cores, least squares, Alg. 3) on the
    24x24x240 bar's OpInf subdomain (268,125 free DOFs) from seeded random snapshots (T
    columns, FP32) with a decaying spectrum."""
    import torch
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import CFG2, lambda_grid_values
    w = CFG2
    ctx = osam.Context(0, "f32", 1)
    osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    z = ctx.sizes(1)
    g = torch.Generator(device="cuda:0").manual_seed(2)
    modes = torch.randn((1, 64, z["n_free"]), generator=g, device="cuda:0")
    coef = torch.randn((1, T, 64), generator=g, device="cuda:0") * torch.logspace(0, -6, 64, device="cuda:0")
    U = torch.bmm(coef, modes).contiguous()
    A = torch.bmm(coef.flip(2).contiguous(), modes).contiguous()
    S = torch.randn((1, T, z["n_sch"]), generator=g, device="cuda:0") * 1e-3
    V0 = torch.zeros((1, z["n_free"]), device="cuda:0")
    out = ctx.learn_opinf(1, U, A, S, V0, 1, T, r=r, r_s=1, lambdas=lambda_grid_values(11))
    torch.cuda.synchronize()
    print(f"learn done: N={z['n_free']} T={T} r={out['r']} lambda*={out['lambda_star']}", flush=True)


def copy() -> None:
    import torch
    n = COPY_BYTES // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy done: {COPY_BYTES} bytes x 3", flush=True)


def _counter_rows(d: str):
    rows = []
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            rows += list(csv.DictReader(f))
    return rows


def _mean_counter(rows, name_part, counter):
    vals = [float(r["Counter_Value"]) for r in rows
            if name_part in r["Kernel_Name"] and r["Counter_Name"] == counter]
    return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)


# the fused sweep of the 24x24x240 workload: FE step of Omega_1 plus the OpInf step
# (r = 40, r_S = 1, one FOM-fed face and one push face of 3 x 625 DOFs)
_SWEEP24_BYTES = FE_ALG_BYTES * 268125 + rom_bytes_per_launch(40, 1, 1875, 1875)

CASES = {
    # name: (subdirectory prefix, kernel name filter, algorithmic bytes per launch, summary file,
    #        source set, title)
    "bar24": ("", "fe_kernel<float, 0", FE_ALG_BYTES * 268125, "fe_kernel_bar24x24x240_traffic.txt", "fe",
              "FE step kernel, 24x24x240 bar, Omega_1 268125 FE DOFs, FP32, launch 256 threads x 1 layer"),
    "bar64": ("large_", "fe_kernel<float, 0", FE_ALG_BYTES * 16 * 4322175, "fe_kernel_bar64x64x640_b16_traffic.txt", "fe",
              "FE step kernel, 64x64x640 bar, middle FOM subdomain 4322175 FE DOFs x 16 instances, FP32, "
              "launch 256 threads x 1 layer, x-shared interior rows"),
    "bar24_sweep": ("sweep_", "sweep_kernel<float, 1", _SWEEP24_BYTES, "sweep_kernel_bar24x24x240_traffic.txt",
                    "sweep", "fused sweep kernel (FE step of Omega_1, 268125 FE DOFs, + OpInf step r=40), "
                    "24x24x240 bar, FP32, 512 threads x 1 layer"),
}


def summarize(outdir: str, case: str = "bar24") -> None:
    """outdir holds the rocprofv3 results of the passes fetch_copy, write_copy and
    <prefix>fetch_fe, <prefix>write_fe of the case."""
    prefix, kname, alg_bytes, fname, kernel, title = CASES[case]
    get = lambda sub: _counter_rows(os.path.join(outdir, sub))
    fc, nfc = _mean_counter(get("fetch_copy"), "copy", "FETCH_SIZE")
    wc, nwc = _mean_counter(get("write_copy"), "copy", "WRITE_SIZE")
    ff, nff = _mean_counter(get(prefix + "fetch_fe"), kname, "FETCH_SIZE")
    wf, nwf = _mean_counter(get(prefix + "write_fe"), kname, "WRITE_SIZE")
    kib = COPY_BYTES / 1024.0
    sf = kib / fc if fc else None
    sw = kib / wc if wc else None
    fetch_b = ff * sf * 1024 if (ff and sf) else None
    write_b = wf * sw * 1024 if (wf and sw) else None
    args = {"bar24": "workload 100", "bar24_sweep": "workload 100 fused", "bar64": "large 4 256 1"}[case]
    lines = [
        f"# HBM traffic (rocprofv3 --pmc), {title}",
        "# commands, from the repository root after `cd /tmp && export TMPDIR=/tmp` (OUT: an output folder):",
        "#   timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch_copy -o run -- "
        "python3 -m paper_2511_20687_amd.profiling copy",
        "#   timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write_copy -o run -- "
        "python3 -m paper_2511_20687_amd.profiling copy",
        f"#   timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/{prefix}fetch_fe -o run -- "
        f"python3 -m paper_2511_20687_amd.profiling {args}",
        f"#   timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/{prefix}write_fe -o run -- "
        f"python3 -m paper_2511_20687_amd.profiling {args}",
        f"#   python3 -m paper_2511_20687_amd.profiling summarize OUT {case}",
        "# scale = known bytes of the copy / its counted KiB; traffic = counted KiB x scale, per launch",
        f"kernel_source_sha256_16={source_hash(kernel)}",
        f"copy_bytes={COPY_BYTES}",
        f"copy_fetch_kib_per_dispatch={fc} (n={nfc})",
        f"copy_write_kib_per_dispatch={wc} (n={nwc})",
        f"fetch_scale={sf}",
        f"write_scale={sw}",
        f"kernel_fetch_kib_per_dispatch={ff} (n={nff})",
        f"kernel_write_kib_per_dispatch={wf} (n={nwf})",
        f"kernel_fetch_bytes_per_launch={fetch_b}",
        f"kernel_write_bytes_per_launch={write_b}",
        f"kernel_traffic_bytes_per_launch={None if fetch_b is None or write_b is None else fetch_b + write_b}",
        f"algorithmic_bytes_per_launch={alg_bytes:.0f}",
    ]
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    path = os.path.join(ROOT, "profiles", fname)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_traffic(case: str = "bar24"):
    """(traffic bytes per launch, details) from the committed summary of a case, or (None,
    reason) when it is missing or was taken for another version of the kernel's sources."""
    _, _, _, fname, kernel, _ = CASES[case]
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None, "no PMC summary"
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k] = v.split(" ")[0]
    if kv.get("kernel_source_sha256_16") != source_hash(kernel):
        return None, "kernel sources changed since the counters were taken"
    try:
        return float(kv["kernel_traffic_bytes_per_launch"]), path
    except (KeyError, ValueError):
        return None, "incomplete PMC summary"


if __name__ == "__main__":
    cmd = sys.argv[1] if len(sys.argv) > 1 else "workload"
    if cmd == "workload":
        workload(int(sys.argv[2]) if len(sys.argv) > 2 else 200, len(sys.argv) > 3 and sys.argv[3] == "fused")
    elif cmd == "large":
        a = [int(x) for x in sys.argv[2:5]]
        large(*a)
    elif cmd == "copy":
        copy()
    elif cmd == "rom":
        rom(int(sys.argv[2]) if len(sys.argv) > 2 else 50, len(sys.argv) > 3 and sys.argv[3] == "bf16")
    elif cmd == "learn":
        learn(*[int(x) for x in sys.argv[2:4]])
    elif cmd == "summarize":
        summarize(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "bar24")
    else:
        raise SystemExit(f"unknown command {cmd}")
