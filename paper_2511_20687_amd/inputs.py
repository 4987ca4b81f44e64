"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method itself: it only draws random
numbers (SplitMix64, Steele, Lea & Flood 2014), names the synthetic bar
workloads, and evaluates the prescribed initial fields on the global node
grid.  Both the CPU oracle and the HIP path receive what is generated here and
apply boundary conditions, restriction to subdomains, etc. on their own.

Global node numbering of a structured ``nx x ny x nz`` hex8 bar over
``[0,Lx] x [0,Ly] x [0,Lz]``: node ``(i, j, k)`` has id
``i + (nx+1) * (j + (ny+1) * k)`` and position ``(i*Lx/nx, j*Ly/ny, k*Lz/nz)``.
Vector fields are structure-of-arrays, shape ``(3, n_nodes)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

_M64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (published constants); one 64-bit stream per seed."""

    def __init__(self, seed: int):
        self.state = seed & _M64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _M64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def uniform(self, a: float = 0.0, b: float = 1.0) -> float:
        """U[a, b] = a + (b - a) * (x >> 11) * 2^-53."""
        return a + (b - a) * ((self.next_u64() >> 11) * (2.0 ** -53))

    def normal(self) -> float:
        """Standard normal by Box-Muller from two uniforms (first output)."""
        u1 = 1.0 - self.uniform()  # in (0, 1]
        u2 = self.uniform()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)

    def uniform_array(self, n: int, a: float = 0.0, b: float = 1.0) -> np.ndarray:
        return np.array([self.uniform(a, b) for _ in range(n)], dtype=np.float64)

    def normal_array(self, n: int) -> np.ndarray:
        return np.array([self.normal() for _ in range(n)], dtype=np.float64)

    def skip(self, n: int) -> "SplitMix64":
        for _ in range(n):
            self.next_u64()
        return self


# ---------------------------------------------------------------------------
# Bar geometry, material and the decomposition of the bar into z-slabs.
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Bar:
    nx: int
    ny: int
    nz: int
    Lx: float = 0.1
    Ly: float = 0.1
    Lz: float = 1.0
    E: float = 1.0e9
    nu: float = 0.25
    rho: float = 1000.0

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def h(self) -> float:
        return self.Lz / self.nz

    def node_z(self) -> np.ndarray:
        """z coordinate of every node (global numbering)."""
        k = np.arange(self.nz + 1, dtype=np.float64)
        z = k * (self.Lz / self.nz)
        return np.repeat(z, (self.nx + 1) * (self.ny + 1))

    def p_wave_speed(self) -> float:
        """Dilatational wave speed sqrt(E(1-nu)/((1+nu)(1-2nu)rho))."""
        E, nu, rho = self.E, self.nu, self.rho
        return math.sqrt(E * (1.0 - nu) / ((1.0 + nu) * (1.0 - 2.0 * nu) * rho))

    def explicit_dt(self, courant: float = 0.25) -> float:
        """Workload time step: courant * h / c_p (h = element size along z)."""
        return courant * self.h / self.p_wave_speed()


def slab_layers(nz: int, n_sub: int, overlap_frac: float = 0.2) -> List[Tuple[int, int]]:
    """Node-layer ranges [lo, hi] of ``n_sub`` overlapping z-slabs.

    Interior cut c_k = round(k*nz/n_sub) is widened by +-round(overlap_frac/2*nz)
    node layers, so every overlap band spans ``overlap_frac`` of the bar.
    """
    half = int(round(0.5 * overlap_frac * nz))
    cuts = [int(round(k * nz / n_sub)) for k in range(1, n_sub)]
    out = []
    for s in range(n_sub):
        lo = 0 if s == 0 else cuts[s - 1] - half
        hi = nz if s == n_sub - 1 else cuts[s] + half
        out.append((lo, hi))
    return out


# ---------------------------------------------------------------------------
# Initial fields (prescribed data of the workloads).
# ---------------------------------------------------------------------------
def gaussian_pulse_u(bar: Bar, a: float, b: float, s: float) -> np.ndarray:
    """u(x,0) = (0, 0, a exp(-(z-b)^2/(2 s^2))) at every node, shape (3, n_nodes)."""
    z = bar.node_z()
    u = np.zeros((3, bar.n_nodes), dtype=np.float64)
    u[2] = a * np.exp(-((z - b) ** 2) / (2.0 * s * s))
    return u


def multi_pulse_v(bar: Bar, amps: Sequence[float], centers: Sequence[float],
                  widths: Sequence[float]) -> np.ndarray:
    """v_z(z) = sum_m a_m exp(-(z-z_m)^2/(2 s_m^2)) at every node, shape (3, n_nodes)."""
    z = bar.node_z()
    v = np.zeros((3, bar.n_nodes), dtype=np.float64)
    for a, c, s in zip(amps, centers, widths):
        v[2] += a * np.exp(-((z - c) ** 2) / (2.0 * s * s))
    return v


@dataclass(frozen=True)
class Pulse:
    a: float = 1.0e-3
    b: float = 0.25
    s: float = 0.05

    def u0(self, bar: Bar) -> np.ndarray:
        return gaussian_pulse_u(bar, self.a, self.b, self.s)


def draw_pulses(seed: int, n: int, skip: int = 0, s: float = 0.05) -> List[Pulse]:
    """n pulses with a ~ U[0.5,2]*1e-3, b ~ U[0.15,0.35] from the stream of ``seed``.

    ``skip`` draws (pairs) are discarded first, so disjoint index ranges of one
    stream give independent training and test instances.
    """
    g = SplitMix64(seed)
    g.skip(2 * skip)
    out = []
    for _ in range(n):
        a = g.uniform(0.5, 2.0) * 1.0e-3
        b = g.uniform(0.15, 0.35)
        out.append(Pulse(a, b, s))
    return out


@dataclass(frozen=True)
class MultiPulseV:
    amps: Tuple[float, ...]
    centers: Tuple[float, ...]
    widths: Tuple[float, ...]

    def v0(self, bar: Bar) -> np.ndarray:
        return multi_pulse_v(bar, self.amps, self.centers, self.widths)


def draw_multi_pulse_v(seed: int, n: int, skip: int = 0, m: int = 4) -> List[MultiPulseV]:
    """Initial-velocity fields: sum of m Gaussians, a_m ~ +-U[5,20] m/s (random sign),
    z_m ~ U[0.1,0.9], s_m ~ U[0.03,0.08]."""
    g = SplitMix64(seed)
    g.skip(4 * m * skip)
    out = []
    for _ in range(n):
        amps, cs, ws = [], [], []
        for _ in range(m):
            sign = 1.0 if g.uniform() < 0.5 else -1.0
            amps.append(sign * g.uniform(5.0, 20.0))
            cs.append(g.uniform(0.1, 0.9))
            ws.append(g.uniform(0.03, 0.08))
        out.append(MultiPulseV(tuple(amps), tuple(cs), tuple(ws)))
    return out


# ---------------------------------------------------------------------------
# The five synthetic bar workloads.
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    bar: Bar
    n_sub: int
    models: Tuple[str, ...]          # "fom" | "opinf" per subdomain (z order)
    steps: int
    precision: str                   # "f64" | "f32"
    form: str = "linear"             # OpInf form: "linear" | "quadratic"
    r: int = 0
    batch: int = 1
    seed: int = 0
    train_steps: int = 0             # snapshots per training trajectory
    train_runs: int = 1
    train_stride: int = 1
    checkpoint: int = 0
    tol_abs: float = 1.0e-8
    tol_rel: float = 1.0e-12
    min_iter: int = 2
    max_iter: int = 32
    # initial guess of the Schwarz iteration: 0 HOLD (the neighbour's accepted value at
    # t_{k-1}), 1 PREDICTOR (its Newmark displacement predictor at t_k, which the explicit
    # scheme's step does not change: the iteration then converges at its second iterate)
    guess: int = 0
    # displacement components held at zero on the lateral faces: x and y, as for
    # the effectively-1D bar of Sec. 5.1 (empty = traction-free lateral faces)
    lateral_fix: Tuple[int, ...] = (0, 1)
    # width s of the seeded Gaussian pulses (Sec. 5.1's Symmetric Gaussian uses 0.02)
    pulse_width: float = 0.02

    @property
    def layers(self) -> List[Tuple[int, int]]:
        return slab_layers(self.bar.nz, self.n_sub)

    @property
    def dt(self) -> float:
        return self.bar.explicit_dt()

    def scaled(self, nx: int, ny: int, nz: int, **kw) -> "Workload":
        """Same workload on another grid (for parity cases the oracle finishes fast)."""
        return replace(self, bar=replace(self.bar, nx=nx, ny=ny, nz=nz), **kw)


CFG1 = Workload("fom_fom_bar_4x4x40_f64", Bar(4, 4, 40), 2, ("fom", "fom"), 1000, "f64",
                pulse_width=0.05)
CFG2 = Workload("fom_opinf_bar_24x24x240_r40", Bar(24, 24, 240), 2, ("fom", "opinf"), 5000,
                "f32", form="linear", r=40, seed=2, train_steps=2000, tol_rel=1.0e-6, guess=1)
CFG3 = Workload("opinf_opinf_bar_48x48x480_r100_b256", Bar(48, 48, 480), 2, ("opinf", "opinf"),
                2000, "f32", form="quadratic", r=100, batch=256, seed=3, train_steps=2000,
                train_runs=16, train_stride=16, tol_rel=1.0e-6, pulse_width=0.05, guess=1)
CFG4 = Workload("adjoint_fom_qopinf_bar_24x24x240_r60", Bar(24, 24, 240), 2, ("fom", "opinf"),
                2000, "f32", form="quadratic", r=60, seed=4, train_steps=2000, checkpoint=100,
                tol_rel=1.0e-6)
CFG5 = Workload("opinf_fom_opinf_bar_64x64x640_r120_b16", Bar(64, 64, 640), 3,
                ("opinf", "fom", "opinf"), 10000, "f32", form="quadratic", r=120, batch=16,
                seed=5, train_steps=2000, train_runs=2, train_stride=10, tol_rel=1.0e-6)
WORKLOADS = {w.name: w for w in (CFG1, CFG2, CFG3, CFG4, CFG5)}


def nominal_pulse() -> Pulse:
    return Pulse(1.0e-3, 0.25, 0.05)


# ---------------------------------------------------------------------------
# Random dense inputs for component-level parity cases.
# ---------------------------------------------------------------------------
def random_matrix(seed: int, rows: int, cols: int, scale: float = 1.0) -> np.ndarray:
    """rows x cols matrix of U[-scale, scale] entries, filled row-major from one stream.

    Generated with numpy's PCG64 seeded by the first SplitMix64 output, so large
    matrices are cheap to make and still reproducible from one integer seed.
    """
    g = SplitMix64(seed)
    rng = np.random.Generator(np.random.PCG64(g.next_u64()))
    return rng.uniform(-scale, scale, size=(rows, cols))


def random_normal(seed: int, shape, scale: float = 1.0) -> np.ndarray:
    g = SplitMix64(seed)
    rng = np.random.Generator(np.random.PCG64(g.next_u64()))
    return scale * rng.standard_normal(size=shape)


def lambda_grid_values(n: int = 11) -> list:
    """Candidate regularisation parameters of Sec. 5: 10^(-10 + 10 (j-1)/(n-1)), j = 1..n."""
    if n == 1:
        return [1e-10]
    return [10.0 ** (-10.0 + 10.0 * j / (n - 1)) for j in range(n)]


def synthetic_rom(seed, n_free, n_sch, r, rs, dt, quadratic=False, with_c=False, scale_b=1.0):
    """Seeded synthetic OpInf data for parity cases and CPU timing: orthonormal Phi,
    Phi_S; A = -V diag(w^2) V^T with w dt <= 0.9 (a stable explicit step); small B, H, c."""
    Phi, _ = np.linalg.qr(random_normal(seed, (n_free, r)))
    PhiS = np.linalg.qr(random_normal(seed + 1, (n_sch, rs)))[0] if rs else None
    Vm, _ = np.linalg.qr(random_normal(seed + 2, (r, r)))
    w2 = (np.linspace(0.05, 0.9, r) / dt) ** 2
    A = -(Vm * w2) @ Vm.T
    B = scale_b * (1.0 / dt) ** 2 * 0.01 * random_normal(seed + 3, (r, rs)) if rs else None
    H = 1e-3 * (1.0 / dt) ** 2 * random_normal(seed + 4, (r, r * (r + 1) // 2)) if quadratic else None
    c = 1e-6 * (1.0 / dt) ** 2 * random_normal(seed + 5, (r,)) if with_c else None
    return dict(Phi=Phi, PhiS=PhiS, A=A, B=B, H=H, c=c)


@dataclass
class ModalSnapshots:
    """Snapshots with a known singular value decomposition (for learning at full size).

    Column j (time t_j = j dt, j < T) of the displacement snapshots is
    sum_k Phi[:, k] sigma_k v_k(j) with v_k(j) = sqrt(2 / T) cos(2 pi f_k j / T), distinct
    integer frequencies 0 < f_k < T / 2: the v_k are orthonormal over the T samples, so
    Phi diag(sigma) V^T is the thin SVD (Phi orthonormal).  Each mode is a free oscillation of
    the explicit central-difference step: its acceleration is -w_k^2 times it with
    w_k^2 = (4 / dt^2) sin^2(pi f_k / T), the second difference of the samples, so that step
    started from the first sample with zero velocity reproduces every sample exactly."""
    Phi: np.ndarray          # [n][m] orthonormal
    sigma: np.ndarray        # [m] descending
    freq: np.ndarray         # [m] integer frequencies
    T: int
    dt: float

    def coefficients(self) -> np.ndarray:
        """[m][T]: sigma_k v_k(j)."""
        j = np.arange(self.T)
        return (self.sigma[:, None] * math.sqrt(2.0 / self.T)
                * np.cos(2.0 * math.pi * self.freq[:, None] * j[None, :] / self.T))

    def omega2(self) -> np.ndarray:
        return (4.0 / self.dt ** 2) * np.sin(math.pi * self.freq / self.T) ** 2

    def snapshots(self) -> Tuple[np.ndarray, np.ndarray]:
        """(U, Udd), each [n][T]."""
        C = self.coefficients()
        return self.Phi @ C, self.Phi @ (-self.omega2()[:, None] * C)


def modal_snapshots(seed: int, n: int, T: int, m: int, dt: float, decades: float) -> ModalSnapshots:
    """Seeded ModalSnapshots: sigma log-spaced over `decades` decades from 1, frequencies a
    seeded draw of m distinct integers in [1, T/8) (slow modes: resolved by the time step)."""
    Phi = np.linalg.qr(random_normal(seed, (n, m)))[0]
    g = np.random.Generator(np.random.PCG64(SplitMix64(seed + 1).next_u64()))
    freq = np.sort(g.choice(np.arange(1, T // 8), size=m, replace=False)).astype(np.int64)
    g.shuffle(freq)
    sigma = np.logspace(0.0, -decades, m)
    return ModalSnapshots(Phi=Phi, sigma=sigma, freq=freq, T=T, dt=dt)
