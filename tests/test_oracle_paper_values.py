"""Oracle pinned to values the paper prints (fixtures under tests/golden/, each with its citation).

Sec. 5.1: for the effectively-1D bar, 28 POD modes capture 99.9999% of the snapshot energy
for the Symmetric Gaussian initial condition and 56 for the Rounded Square, in either
subdomain.  The count exercises the whole oracle chain: hex8 stiffness and lumped mass,
explicit Newmark, the multiplicative Schwarz coupling of the two slabs, and the POD energy
criterion (a dropped term or a wrong sign anywhere changes the wave and the count).
"""
import json
import os

import numpy as np
import pytest

from paper_2511_20687_amd.inputs import Bar
from oracle.newmark import FomModel
from oracle.pod import energy_rank, pod
from oracle.schwarz import Coupled, SchwarzOptions

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sec5_1_pod_modes.json")


def _ic(bar, kind):
    z = bar.node_z() - 0.5
    if kind == "symmetric_gaussian":
        f = 1e-3 * np.exp(-(z ** 2) / (2 * 0.02 ** 2))
    else:
        a, b, s = 5e-4, 100.0, 0.6
        f = a * np.tanh(-b * (z + 0.5 - s)) + a * np.tanh(b * (z - 0.5 + s))
    u0 = np.zeros((3, bar.n_nodes))
    u0[2] = f
    return u0


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["symmetric_gaussian", "rounded_square"])
def test_pod_mode_count_of_section_5_1(kind):
    ref = json.load(open(GOLDEN))
    bar = Bar(1, 1, 1000, Lx=1e-3, Ly=1e-3, Lz=1.0, E=1e9, nu=0.0, rho=1000.0)
    dt = 1e-7
    models = [FomModel(bar, lo, hi, dt, lateral_fix=(0, 1)) for lo, hi in ((0, 750), (250, 1000))]
    u0 = _ic(bar, kind)
    out = Coupled(models).run(u0, np.zeros_like(u0), 10000, SchwarzOptions(), every=10, record=("u",))
    for i in range(2):
        _, sig = pod(out["u"][i].T)
        assert energy_rank(sig, ref["energy"]) == ref["modes"][kind]
