"""run_noalloc (the controller loop without device allocation) against run: the same records,
states and iteration counts, on two calls in a row, the second on a smaller problem (the
static scratch array keeps the first call's contents; nothing in it must start at zero)."""
import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar, gaussian_pulse_u, slab_layers
from oracle.newmark import SubdomainGeometry
from tests._gpu import lib_free_index, lib_sch_index, synthetic_rom

pytestmark = pytest.mark.gpu


def _pair(bar, kinds, batch, engine=0, beta=0.0):
    """Two identical contexts (FOM / OpInf subdomains of a bar, FP64) with records."""
    import torch
    from paper_2511_20687_amd import osam
    dt = (4.0 if beta else 1.0) * bar.explicit_dt()
    layers = slab_layers(bar.nz, len(kinds))
    out = []
    for _ in range(2):
        ctx = osam.Context(0, "f64", batch)
        sds = osam.add_bar_subdomains(ctx, bar, layers, dt, beta=beta)
        for i, (lo, hi) in enumerate(layers):
            if kinds[i] != "opinf":
                continue
            g = SubdomainGeometry(bar, lo, hi)
            R = synthetic_rom(61 + i, g.n_free, g.n_sch, 6, 3, dt, True, False)
            Phi = np.zeros_like(R["Phi"])
            Phi[lib_free_index(bar, lo, hi)] = R["Phi"]
            PhiS = np.zeros_like(R["PhiS"])
            PhiS[lib_sch_index(bar, lo, hi)] = R["PhiS"]
            ctx.set_opinf(sds[i], Phi, PhiS, R["A"], R["H"], R["B"], R["c"])
        if engine:
            ctx.set_engine(engine)
        recs = []
        for i, kind in enumerate(kinds):
            z = ctx.sizes(i)
            t = torch.zeros((batch, 41, z["r"] if kind == "opinf" else z["n_free"]), dtype=torch.float64,
                            device="cuda:0")
            ctx.set_record(i, 1, 41, u=t)
            recs.append(t)
        for b in range(batch):
            u0 = gaussian_pulse_u(bar, 1e-3 * (1 + b), 0.3 + 0.1 * b, 0.05)
            ctx.set_initial(b, u0, np.zeros_like(u0))
        out.append((ctx, recs))
    return out


def _check(bar, kinds, batch, engine=0, beta=0.0):
    from paper_2511_20687_amd import osam
    (ca, ra), (cb, rb) = _pair(bar, kinds, batch, engine, beta)
    opts = osam.Options()
    ia = ca.run(40, opts)
    if engine or beta:
        # the window engine sets its buffers up in a first run call
        ib0 = cb.run(0, opts)
        assert all(i["steps"] == 0 for i in ib0)
    ib = cb.run_noalloc(40, opts)
    for i in range(len(kinds)):
        assert np.array_equal(ra[i].cpu().numpy(), rb[i].cpu().numpy()), i
    for b in range(batch):
        assert ia[b]["total_iters"] == ib[b]["total_iters"] and ib[b]["steps"] == 40
        for i in range(len(kinds)):
            ua = ca.get_state(i, b)[0]
            ub = cb.get_state(i, b)[0]
            assert np.array_equal(ua, ub)


def test_run_noalloc_equals_run_twice_with_a_smaller_second_problem():
    print("[run_noalloc: 4 instances, FOM-OpInf-FOM on 4x4x40]", flush=True)
    _check(Bar(4, 4, 40), ("fom", "opinf", "fom"), 4)
    print("[run_noalloc: 1 instance, FOM-FOM on 2x2x20]", flush=True)
    _check(Bar(2, 2, 20), ("fom", "fom"), 1)


def test_run_noalloc_window_engine():
    print("[run_noalloc: window engine, implicit FOM-OpInf, 2 instances]", flush=True)
    _check(Bar(3, 3, 30), ("fom", "opinf"), 2, beta=0.25)
    print("[run_noalloc: window engine on request, explicit FOM-FOM, 1 instance]", flush=True)
    _check(Bar(2, 2, 20), ("fom", "fom"), 1, engine=1)


def test_run_noalloc_needs_a_wired_context():
    from paper_2511_20687_amd import osam
    bar = Bar(2, 2, 20)
    ctx = osam.Context(0, "f64", 1)
    osam.add_bar_subdomains(ctx, bar, slab_layers(bar.nz, 2), bar.explicit_dt())
    with pytest.raises(osam.OsamError) as e:
        ctx.run_noalloc(5)
    assert e.value.code == osam.OSAM_E_ORDER
