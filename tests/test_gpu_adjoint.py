"""GPU adjoint of the coupled rollout (run_adjoint) against the FP64 oracle.

The oracle evaluates J by its own multiplicative Schwarz loop and differentiates it by the
complex step (oracle/misfit.py); the GPU differentiates the converged explicit map by a
checkpointed discrete adjoint.  Checked: J, directional derivatives along seeded random
directions in every parameter block, central differences of the GPU's own J, the
torch.autograd wrapper, and J against a plain Schwarz run of the library.
"""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, gaussian_pulse_u, random_normal, slab_layers, synthetic_rom
from oracle.misfit import directional_derivative, fom_state, misfit, rom_state
from oracle.newmark import FomModel, SubdomainGeometry
from oracle.rom import OpInfModel
from tests._gpu import lib_index_of, torch_dtype

pytestmark = pytest.mark.gpu
R_ = 5


def _setup(lateral_fix=(), quadratic=True):
    bar = Bar(2, 2, 20)
    dt = bar.explicit_dt()
    layers = slab_layers(bar.nz, 2)
    fom = FomModel(bar, *layers[0], dt, lateral_fix=lateral_fix)
    g = SubdomainGeometry(bar, *layers[1], lateral_fix=lateral_fix)
    R = synthetic_rom(21, g.n_free, g.n_sch, R_, 3, dt, quadratic=quadratic, with_c=True)
    u0 = gaussian_pulse_u(bar, 1e-3, 0.4, 0.08)
    v0 = np.zeros_like(u0)
    n, every = 40, 4
    obs_o = {0: 1e-4 * random_normal(22, (n // every, fom.n_free)), 1: 1e-4 * random_normal(23, (n // every, R_))}
    return dict(bar=bar, dt=dt, layers=layers, fom=fom, g=g, R=R, u0=u0, v0=v0, n=n, every=every, obs_o=obs_o,
                lf=lateral_fix)


def _lib_rom(P, A=None, H=None, B=None, c=None):
    """Operators and bases in the library layouts (free DOFs [3][nodes], Schwarz [3][nodes])."""
    from paper_2511_20687_amd import osam
    bar, layers, R, g = P["bar"], P["layers"], P["R"], P["g"]
    nzs = layers[1][1] - layers[1][0]
    li = lib_index_of(g)
    Phi = np.zeros((3 * (bar.nx + 1) * (bar.ny + 1) * (nzs - 1), R_))
    Phi[li] = R["Phi"]
    npl = (bar.nx + 1) * (bar.ny + 1)
    PhiS = np.zeros_like(R["PhiS"])
    PhiS[(np.arange(npl)[:, None] + npl * np.arange(3)[None, :]).ravel()] = R["PhiS"]
    return (Phi, PhiS, R["A"] if A is None else A, R["H"] if H is None else H, R["B"] if B is None else B,
            R["c"] if c is None else c)


def _gpu(P, precision="f64"):
    import torch
    from paper_2511_20687_amd import osam
    ctx = osam.Context(0, precision, 1)
    osam.add_bar_subdomains(ctx, P["bar"], P["layers"], P["dt"], lateral_fix=P["lf"])
    ctx.set_opinf(1, *_lib_rom(P))
    ctx.set_initial(0, P["u0"], P["v0"])
    fom, dev, dtp = P["fom"], "cuda:0", torch_dtype(precision)
    nf_lib = ctx.sizes(0)["n_free"]
    o0 = np.zeros((P["obs_o"][0].shape[0], nf_lib))
    o0[:, lib_index_of(fom)] = P["obs_o"][0]
    obs = {0: torch.tensor(o0, dtype=dtp, device=dev), 1: torch.tensor(P["obs_o"][1], dtype=dtp, device=dev)}
    return ctx, obs


def _oracle_J(P, d, eps):
    R, fom, g, dt = P["R"], P["fom"], P["g"], P["dt"]
    A = R["A"] + eps * d["A"]
    H = None if R["H"] is None else R["H"] + eps * d["H"]
    B, c = R["B"] + eps * d["B"], R["c"] + eps * d["c"]
    rom = OpInfModel(g, R["Phi"], R["PhiS"], A, H, B, c, dt=dt)
    st0 = fom.initial_state(P["u0"], P["v0"])   # clamped-end DOFs zeroed, as the library does
    ul, vl = st0.u.astype(complex), st0.v.astype(complex)
    ul[fom.free_dofs] += eps * d["u0"]
    vl[fom.free_dofs] += eps * d["v0"]
    s0 = g.restrict(P["u0"])[g.sch_dofs]
    q0 = R["Phi"].T @ g.restrict(P["u0"])[g.free_dofs] + eps * d["q0"]
    qd0 = R["Phi"].T @ g.restrict(P["v0"])[g.free_dofs] + eps * d["qd0"]
    st = [fom_state(fom, ul, vl), rom_state(rom, q0, qd0, s0)]
    return misfit([fom, rom], st, P["n"], P["every"], P["obs_o"])


def _direction(P, seed):
    R, fom = P["R"], P["fom"]
    sc = lambda a: np.abs(a).max()
    d = {k: 1e-3 * sc(R[k]) * random_normal(seed + i, R[k].shape) for i, k in enumerate(("A", "B", "c"))}
    d["H"] = None if R["H"] is None else 1e-3 * sc(R["H"]) * random_normal(seed + 7, R["H"].shape)
    d["u0"] = 1e-6 * random_normal(seed + 3, (fom.n_free,))
    d["v0"] = 1e-3 * random_normal(seed + 4, (fom.n_free,))
    d["q0"] = 1e-6 * random_normal(seed + 5, (R_,))
    d["qd0"] = 1e-3 * random_normal(seed + 6, (R_,))
    return d


def _dot(P, grads, d):
    gr, gf = grads[1], grads[0]
    li = lib_index_of(P["fom"])
    s = sum(float(np.sum(gr[k] * d[k])) for k in ("A", "B", "c", "q0", "qd0"))
    if d["H"] is not None:
        s += float(np.sum(gr["H"] * d["H"]))
    s += float(np.dot(gf["u0"].cpu().numpy()[li], d["u0"])) + float(np.dot(gf["v0"].cpu().numpy()[li], d["v0"]))
    return s


@pytest.mark.parametrize("lateral_fix", [(), (0, 1)])
def test_adjoint_matches_oracle_complex_step_f64(lateral_fix):
    P = _setup(lateral_fix)
    print(f"[adjoint f64 lateral {lateral_fix}]", flush=True)
    ctx, obs = _gpu(P)
    J, grads = ctx.run_adjoint(P["n"], 7, P["every"], obs)
    J_o = float(np.real(_oracle_J(P, _direction(P, 50), 0.0)))
    print("J gpu", J, "oracle", J_o)
    assert abs(J - J_o) <= 1e-12 * abs(J_o)
    # components held by the lateral condition start at zero whatever u0, v0 say: zero gradient
    if lateral_fix:
        fom = P["fom"]
        held = np.setdiff1d(np.arange(grads[0]["u0"].numel()), lib_index_of(fom))   # library free, oracle Dirichlet
        assert held.size > 0
        for k in ("u0", "v0"):
            assert float(grads[0][k].abs().cpu().numpy()[held].max()) == 0.0
    for seed in (50, 60, 70):
        d = _direction(P, seed)
        dd_o = directional_derivative(lambda e: _oracle_J(P, d, e))
        dd_g = _dot(P, grads, d)
        print("directional", seed, dd_g, dd_o)
        assert abs(dd_g - dd_o) <= 1e-8 * abs(dd_o)
    # every block on its own (a wrong transpose in one block cannot hide behind the others)
    for blk in ("A", "H", "B", "c", "q0", "qd0", "u0", "v0"):
        d = _direction(P, 80)
        for k in d:
            if k != blk and d[k] is not None:
                d[k] = np.zeros_like(d[k])
        dd_o = directional_derivative(lambda e: _oracle_J(P, d, e))
        dd_g = _dot(P, grads, d)
        assert abs(dd_g - dd_o) <= 1e-8 * abs(dd_o) + 1e-30, (blk, dd_g, dd_o)


def test_adjoint_central_differences_and_autograd_f64():
    import torch
    from paper_2511_20687_amd import osam
    P = _setup()
    ctx, obs = _gpu(P)
    Phi, PhiS, A, H, B, c = _lib_rom(P)
    q0 = P["R"]["Phi"].T @ P["g"].restrict(P["u0"])[P["g"].free_dofs]
    qd0 = np.zeros(R_)
    F = osam.rollout_misfit_function()
    tA, tH, tB, tc = (torch.tensor(x, dtype=torch.float64, requires_grad=True) for x in (A, H, B, c))
    tq, tqd = (torch.tensor(x, dtype=torch.float64, requires_grad=True) for x in (q0, qd0))
    J = F.apply(ctx, 1, P["n"], 9, P["every"], obs, P["u0"], P["v0"], Phi, PhiS, tA, tH, tB, tc, tq, tqd)
    J.backward()
    d = _direction(P, 90)
    gd = sum(float(torch.sum(t.grad * torch.tensor(d[k]))) for t, k in ((tA, "A"), (tH, "H"), (tB, "B"), (tc, "c")))
    gd += float(torch.sum(tqd.grad * torch.tensor(d["qd0"]))) + float(torch.sum(tq.grad * torch.tensor(d["q0"])))
    eps = 1e-3
    Js = []
    for sgn in (1, -1):
        Jx = F.apply(ctx, 1, P["n"], 9, P["every"], obs, P["u0"], P["v0"], Phi, PhiS,
                     *(torch.tensor(x + sgn * eps * d[k]) for x, k in ((A, "A"), (H, "H"), (B, "B"), (c, "c"),
                                                                      (q0, "q0"), (qd0, "qd0"))))
        Js.append(float(Jx))
    fd = (Js[0] - Js[1]) / (2 * eps)
    print("fd", fd, "adjoint", gd)
    assert abs(fd - gd) <= 1e-6 * abs(gd)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_adjoint_misfit_equals_schwarz_run(precision, tol):
    """J of the adjoint's forward pass equals J from the records of an ordinary run."""
    import torch
    P = _setup()
    ctx, obs = _gpu(P, precision)
    J, _ = ctx.run_adjoint(P["n"], 16, P["every"], obs)
    dev, dtp, n, ev = "cuda:0", torch_dtype(precision), P["n"], P["every"]
    ru = torch.zeros((1, n // ev + 1, ctx.sizes(0)["n_free"]), dtype=dtp, device=dev)
    rq = torch.zeros((1, n // ev + 1, R_), dtype=dtp, device=dev)
    ctx.set_record(0, ev, n // ev + 1, u=ru)
    ctx.set_record(1, ev, n // ev + 1, u=rq)
    ctx.set_initial(0, P["u0"], P["v0"])
    ctx.run(n)
    du = (ru[0, 1:].double() - obs[0].double()).cpu().numpy()
    dq = (rq[0, 1:].double() - obs[1].double()).cpu().numpy()
    J_run = 0.5 * (np.sum(du * du) + np.sum(dq * dq))
    print("J adjoint", J, "J run", J_run)
    assert abs(J - J_run) <= tol * J_run


def _cfg4_context(precision, theta, P4):
    """FOM (layers 0-144) + quadratic OpInf r=60 (96-240) on the 24x24x240 bar at parameters theta."""
    from paper_2511_20687_amd import osam
    w = P4["w"]
    ctx = osam.Context(0, precision, 1)
    osam.add_bar_subdomains(ctx, w.bar, w.layers, w.dt, lateral_fix=w.lateral_fix)
    _set_theta(ctx, theta, P4)
    return ctx


def _set_theta(ctx, theta, P4):
    ctx.set_opinf(1, P4["Phi"], P4["PhiS"], theta["A"], theta["H"], theta["B"], theta["c"])
    ctx.set_initial(0, theta["u0g"], theta["v0g"])
    ctx.set_reduced(1, 0, theta["q0"], theta["qd0"])


def _cfg4_problem():
    """Seeded cfg4-sized problem: synthetic stable quadratic operators of the learned sizes plus
    1e-3 relative Gaussian noise (the perturbed start), the training pulse as u0, v0 = 0."""
    from paper_2511_20687_amd import osam
    from paper_2511_20687_amd.inputs import CFG4, draw_pulses
    w = CFG4
    nx, ny = w.bar.nx, w.bar.ny
    npl = (nx + 1) * (ny + 1)
    (lo0, hi0), (lo1, hi1) = w.layers
    nf_rom = 3 * npl * (hi1 - lo1 - 1)
    rs = 10
    R = synthetic_rom(w.seed, nf_rom, 3 * npl, w.r, rs, w.dt, quadratic=True, with_c=True)
    noisy = lambda k, a, i: a * (1.0 + 1e-3 * random_normal(w.seed * 100 + i, a.shape))
    theta = {k: noisy(k, R[k], i) for i, k in enumerate(("A", "H", "B", "c"))}
    u0g = draw_pulses(w.seed, 1, s=w.pulse_width)[0].u0(w.bar)
    u_rom = u0g[:, (lo1 + 1) * npl:hi1 * npl].ravel()
    theta.update(u0g=u0g, v0g=np.zeros_like(u0g), q0=R["Phi"].T @ u_rom, qd0=np.zeros(w.r))
    nfn = npl * (hi0 - lo0 - 1)
    # FOM free DOFs (library order) whose perturbation changes nothing but the FOM start:
    # every free node except the OpInf subdomain's Schwarz layer (its t_0 data are constants)
    fn = np.arange(nfn)
    keep = (fn // npl + 1 + lo0) != lo1
    return dict(w=w, Phi=R["Phi"], PhiS=R["PhiS"], theta=theta, npl=npl, nfn=nfn, keep=keep)


def _cfg4_direction(P4, seed):
    """One direction over every parameter block, each block normalised to the block's size
    (velocities to |u0| / (1000 dt))."""
    th, w = P4["theta"], P4["w"]
    d = {}
    for i, k in enumerate(("A", "H", "B", "c", "q0")):
        x = random_normal(seed * 1000 + i, th[k].shape)
        d[k] = x * (np.linalg.norm(th[k]) / np.linalg.norm(x))
    vs = np.linalg.norm(th["u0g"]) / (1000.0 * w.dt)
    x = random_normal(seed * 1000 + 5, (w.r,))
    d["qd0"] = x * (vs / np.linalg.norm(x)) * (np.linalg.norm(th["q0"]) / np.linalg.norm(th["u0g"]))
    for j, k in ((6, "u0"), (7, "v0")):
        x = random_normal(seed * 1000 + j, (3, P4["nfn"])) * P4["keep"][None, :]
        x *= (np.linalg.norm(th["u0g"]) if k == "u0" else vs) / np.linalg.norm(x)
        d[k] = x
    return d


def _shift(P4, d, eps):
    th = dict(P4["theta"])
    for k in ("A", "H", "B", "c", "q0", "qd0"):
        th[k] = th[k] + eps * d[k]
    npl, nfn = P4["npl"], P4["nfn"]
    for k, g in (("u0", "u0g"), ("v0", "v0g")):
        x = th[g].copy()
        x[:, npl:npl + nfn] += eps * d[k]
        th[g] = x
    return th


def _run_J(ctx, n, obs):
    """J of an ordinary Schwarz run (records of every step), in float64."""
    import torch
    dev = "cuda:0"
    dtp = obs[0].dtype
    ru = torch.zeros((1, n + 1, obs[0].shape[1]), dtype=dtp, device=dev)
    rq = torch.zeros((1, n + 1, obs[1].shape[1]), dtype=dtp, device=dev)
    ctx.set_record(0, 1, n + 1, u=ru)
    ctx.set_record(1, 1, n + 1, u=rq)
    ctx.run(n)
    J = 0.5 * (torch.sum((ru[0, 1:].double() - obs[0].double()) ** 2) +
               torch.sum((rq[0, 1:].double() - obs[1].double()) ** 2))
    ctx.set_record(0, 0, 0)
    ctx.set_record(1, 0, 0)
    return float(J)


def _gdot(P4, g, d):
    s = sum(float(np.sum(g[1][k] * d[k])) for k in ("A", "H", "B", "c", "q0", "qd0"))
    for k in ("u0", "v0"):
        s += float(np.sum(g[0][k].double().cpu().numpy().reshape(3, -1) * d[k]))
    return s


def test_adjoint_cfg4_size_fd_32_directions_f64():
    """24x24x240 bar, FOM + quadratic OpInf r=60, 2000 steps, checkpoints every 100 steps,
    misfit over every step: the adjoint gradient along 32 seeded directions agrees with
    central differences of the Schwarz run (FP64) within 1e-5 relative."""
    import torch
    P4 = _cfg4_problem()
    w, n = P4["w"], P4["w"].steps
    print(f"[adjoint cfg4 FD] n={n} r={w.r} K={w.checkpoint}", flush=True)
    ctx = _cfg4_context("f64", P4["theta"], P4)
    nf = ctx.sizes(0)["n_free"]
    gen = torch.Generator(device="cuda:0").manual_seed(w.seed)
    obs = {0: 1e-5 * torch.randn((n, nf), generator=gen, dtype=torch.float64, device="cuda:0"),
           1: 1e-5 * torch.randn((n, w.r), generator=gen, dtype=torch.float64, device="cuda:0")}
    J, g = ctx.run_adjoint(n, w.checkpoint, 1, obs)
    J_run = _run_J(ctx, n, obs)
    print("J adjoint", J, "J run", J_run, flush=True)
    assert abs(J - J_run) <= 1e-12 * J_run
    held = g[0]["u0"].double().cpu().numpy().reshape(3, -1)

    def fd(d, eps):
        Js = []
        for sgn in (1.0, -1.0):
            _set_theta(ctx, _shift(P4, d, sgn * eps), P4)
            Js.append(_run_J(ctx, n, obs))
        return (Js[0] - Js[1]) / (2.0 * eps)

    # central differences carry an O(eps^2) truncation error; the fastest reduced modes turn
    # ~1800 rad over the run, so eps = 1e-7 (relative, per block) is used; the first
    # directions also show eps = 1e-6 to make the eps^2 behaviour visible
    worst = 0.0
    for k in range(32):
        d = _cfg4_direction(P4, w.seed * 64 + k)
        ad = _gdot(P4, g, d)
        f7 = fd(d, 1e-7)
        rel = abs(f7 - ad) / abs(ad)
        worst = max(worst, rel)
        extra = ""
        if k < 4:
            f6 = fd(d, 1e-6)
            extra = f" | eps=1e-6: rel {abs(f6 - ad) / abs(ad):.2e}"
        print(f"direction {k:2d} adjoint {ad:.12e} fd {f7:.12e} rel {rel:.2e}{extra}", flush=True)
    print("worst relative difference", worst)
    assert worst <= 1e-5
    assert np.isfinite(held).all()


def test_adjoint_cfg4_size_f32_against_f64():
    """The FP32 adjoint at the same size, reported against the FP64 one (errors printed;
    asserted at 1e-2 relative per block, far above the observed values)."""
    import torch
    P4 = _cfg4_problem()
    w, n = P4["w"], P4["w"].steps
    res = {}
    for prec, dtp in (("f64", torch.float64), ("f32", torch.float32)):
        ctx = _cfg4_context(prec, P4["theta"], P4)
        nf = ctx.sizes(0)["n_free"]
        gen = torch.Generator(device="cuda:0").manual_seed(w.seed)
        obs = {0: (1e-5 * torch.randn((n, nf), generator=gen, dtype=torch.float64, device="cuda:0")).to(dtp),
               1: (1e-5 * torch.randn((n, w.r), generator=gen, dtype=torch.float64, device="cuda:0")).to(dtp)}
        res[prec] = ctx.run_adjoint(n, w.checkpoint, 1, obs)
        del ctx
    (J64, g64), (J32, g32) = res["f64"], res["f32"]
    print("J f64", J64, "f32", J32, "rel", abs(J32 - J64) / J64)
    assert abs(J32 - J64) <= 1e-4 * J64
    for k in ("A", "H", "B", "c", "q0", "qd0"):
        e = np.linalg.norm(g32[1][k] - g64[1][k]) / np.linalg.norm(g64[1][k])
        print(f"dJ/d{k}: FP32 vs FP64 relative L2 {e:.3e}")
        assert e <= 1e-2
    for k in ("u0", "v0"):
        a, b = g32[0][k].double(), g64[0][k].double()
        e = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        print(f"dJ/d{k}: FP32 vs FP64 relative L2 {e:.3e}")
        assert e <= 1e-2


def test_autograd_device_parameters_and_no_boundary_operator():
    """The torch.autograd wrapper with parameters on cuda:0 and without a boundary operator
    (r_S = 0, B = None): gradients come back on the parameters' device and dtype, None for
    None inputs, equal to those of the same call with CPU parameters, and match a central
    difference of J along a random direction of A."""
    import torch
    from paper_2511_20687_amd import osam
    P = _setup()
    ctx, obs = _gpu(P)
    Phi, PhiS, A, H, B, c = _lib_rom(P)
    q0 = P["R"]["Phi"].T @ P["g"].restrict(P["u0"])[P["g"].free_dofs]
    qd0 = np.zeros(R_)
    F = osam.rollout_misfit_function()
    args = (ctx, 1, P["n"], 9, P["every"], obs, P["u0"], P["v0"], Phi, None)
    grads = {}
    for dev in ("cuda:0", "cpu"):
        tA, tH, tc, tq, tqd = (torch.tensor(x, dtype=torch.float64, device=dev, requires_grad=True)
                               for x in (A, H, c, q0, qd0))
        J = F.apply(*args, tA, tH, None, tc, tq, tqd)
        J.backward()
        for t in (tA, tH, tc, tq, tqd):
            assert t.grad is not None and t.grad.device == t.device and t.grad.dtype == torch.float64
        grads[dev] = [t.grad.cpu().numpy() for t in (tA, tH, tc, tq, tqd)]
    for a, b in zip(grads["cuda:0"], grads["cpu"]):
        assert np.array_equal(a, b)
    dA = random_normal(95, A.shape)
    # a step of 1e-5 of A's scale keeps the central difference's O(eps^2) term (the rollout is
    # nonlinear in A over its steps) below 1e-7 of the derivative
    eps = 1e-5 * np.abs(A).max() / np.abs(dA).max()
    Js = []
    for sgn in (1, -1):
        Jx = F.apply(*args, *(torch.tensor(x) for x in (A + sgn * eps * dA, H)), None,
                     *(torch.tensor(x) for x in (c, q0, qd0)))
        Js.append(float(Jx))
    fd = (Js[0] - Js[1]) / (2 * eps)
    ad = float(np.sum(grads["cpu"][0] * dA))
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
