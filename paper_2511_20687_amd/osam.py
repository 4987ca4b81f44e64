"""ctypes binding of libosam (include/osam.h).

Argument marshalling only: every computation runs in the HIP kernels of
libosam.so.  Host arrays are numpy float64; device buffers (records,
snapshots) are torch CUDA tensors passed by data pointer.  The library must
have been built (``python -m paper_2511_20687_amd.build``); importing this
module on a machine without it raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libosam.so")

OSAM_OK, OSAM_E_INVALID, OSAM_E_OOM, OSAM_E_HIP = 0, -1, -2, -3
OSAM_E_NONFINITE, OSAM_E_SINGULAR, OSAM_E_OUTSIDE, OSAM_E_ORDER = -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "OOM", -3: "HIP", -4: "NONFINITE", -5: "SINGULAR",
                -6: "OUTSIDE", -7: "ORDER"}
EXPORTED = ["osam_version", "osam_ctx_create", "osam_ctx_destroy", "osam_last_error",
            "create_subdomain", "osam_couple", "osam_set_initial", "osam_get_state",
            "osam_get_reduced", "osam_sizes", "osam_set_record", "learn_opinf", "osam_set_opinf",
            "osam_get_opinf", "schwarz_step", "run", "osam_set_timing", "osam_get_timing",
            "osam_set_fe_launch", "osam_get_fe_launch", "osam_set_reduced", "run_adjoint",
            "osam_set_rom_path", "osam_get_rom_path", "osam_set_graph", "osam_set_fusion", "osam_set_fe_xshare",
            "osam_autotune",
            "osam_sync", "osam_set_engine", "osam_get_solver_stats", "run_noalloc", "osam_set_opinf_cubic",
            "osam_get_opinf_cubic", "osam_set_state", "osam_checkpoint_size", "osam_save_checkpoint",
            "osam_load_checkpoint"]


class OsamError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"osam error {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class SubdomainDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("Lx", C.c_double), ("Ly", C.c_double), ("Lz", C.c_double),
                ("z_lo", C.c_int32), ("z_hi", C.c_int32),
                ("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double),
                ("clamp_ends", C.c_int32), ("lateral_fix", C.c_int32), ("dt", C.c_double),
                ("beta", C.c_double), ("gamma", C.c_double), ("n_sub", C.c_int32), ("material", C.c_int32)]


class Record(C.Structure):
    _fields_ = [("every", C.c_int64), ("n_cols", C.c_int64), ("u", C.c_void_p), ("a", C.c_void_p),
                ("s", C.c_void_p)]


class OpinfDesc(C.Structure):
    _fields_ = [("form", C.c_int32), ("with_c", C.c_int32), ("r", C.c_int32), ("r_s", C.c_int32),
                ("energy", C.c_double), ("energy_bnd", C.c_double), ("n_lambda", C.c_int32),
                ("lambdas", C.POINTER(C.c_double)), ("n_traj", C.c_int32), ("T", C.c_int64),
                ("U", C.c_void_p), ("Udd", C.c_void_p), ("S", C.c_void_p), ("V0", C.c_void_p),
                ("sigma_out", C.POINTER(C.c_double)), ("E_lambda_out", C.POINTER(C.c_double)),
                ("lambda_star_out", C.POINTER(C.c_double)), ("r_out", C.POINTER(C.c_int32)),
                ("rs_out", C.POINTER(C.c_int32)), ("stride", C.c_int32)]


class Misfit(C.Structure):
    _fields_ = [("every", C.c_int64), ("obs", C.c_void_p * 8)]


class Grads(C.Structure):
    _fields_ = [("dA", C.POINTER(C.c_double) * 8), ("dH", C.POINTER(C.c_double) * 8),
                ("dB", C.POINTER(C.c_double) * 8), ("dc", C.POINTER(C.c_double) * 8),
                ("dq0", C.POINTER(C.c_double) * 8), ("dqd0", C.POINTER(C.c_double) * 8),
                ("du0", C.c_void_p * 8), ("dv0", C.c_void_p * 8)]


class Tuning(C.Structure):
    _fields_ = [("fe_block", C.c_int32 * 8), ("fe_kc", C.c_int32 * 8), ("rom_path", C.c_int32 * 8),
                ("graph_rounds", C.c_int32), ("graph_streams", C.c_int32), ("ms_per_step", C.c_double),
                ("from_cache", C.c_int32), ("fusion_kc", C.c_int32), ("fe_xs", C.c_int32 * 8)]


class SchwarzOpts(C.Structure):
    _fields_ = [("tol_abs", C.c_double), ("tol_rel", C.c_double), ("min_iter", C.c_int32),
                ("max_iter", C.c_int32), ("guess", C.c_int32), ("additive", C.c_int32)]


class InstanceInfo(C.Structure):
    _fields_ = [("steps", C.c_int64), ("last_iters", C.c_int32), ("last_converged", C.c_int32),
                ("abs2", C.c_double), ("den2", C.c_double), ("total_iters", C.c_int64),
                ("max_iters", C.c_int32), ("unconverged", C.c_int64), ("status", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libosam.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2511_20687_amd.build`")
    # torch ships its own HIP runtime under the same soname as the system one that
    # libosam links: load torch first so both resolve to the runtime torch was built
    # against (loaded the other way round, torch finds no GPU)
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    lib.osam_version.restype = i32
    lib.osam_ctx_create.argtypes = [C.POINTER(vp), i32, i32, i32, vp]
    lib.osam_ctx_create.restype = i32
    lib.osam_ctx_destroy.argtypes = [vp]
    lib.osam_ctx_destroy.restype = None
    lib.osam_last_error.argtypes = [vp]
    lib.osam_last_error.restype = C.c_char_p
    lib.create_subdomain.argtypes = [vp, C.POINTER(SubdomainDesc), C.POINTER(i32)]
    lib.create_subdomain.restype = i32
    lib.osam_couple.argtypes = [vp]
    lib.osam_couple.restype = i32
    lib.osam_set_initial.argtypes = [vp, i32, dp, dp]
    lib.osam_set_initial.restype = i32
    lib.osam_get_state.argtypes = [vp, i32, i32, dp, dp, dp]
    lib.osam_get_state.restype = i32
    lib.osam_get_reduced.argtypes = [vp, i32, i32, dp, dp, dp]
    lib.osam_get_reduced.restype = i32
    lib.osam_sizes.argtypes = [vp, i32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64),
                               C.POINTER(i32), C.POINTER(i32)]
    lib.osam_sizes.restype = i32
    lib.osam_set_record.argtypes = [vp, i32, C.POINTER(Record)]
    lib.osam_set_record.restype = i32
    if hasattr(lib, "learn_opinf"):
        lib.learn_opinf.argtypes = [vp, i32, C.POINTER(OpinfDesc)]
        lib.learn_opinf.restype = i32
    lib.osam_set_opinf.argtypes = [vp, i32, i32, i32, dp, dp, dp, dp, dp, dp]
    lib.osam_set_opinf.restype = i32
    lib.osam_get_opinf.argtypes = [vp, i32, dp, dp, dp, dp, dp, dp]
    lib.osam_get_opinf.restype = i32
    lib.schwarz_step.argtypes = [vp, C.POINTER(SchwarzOpts), C.POINTER(InstanceInfo)]
    lib.schwarz_step.restype = i32
    lib.run.argtypes = [vp, i64, C.POINTER(SchwarzOpts), C.POINTER(InstanceInfo)]
    lib.osam_set_reduced.argtypes = [vp, i32, i32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.osam_set_reduced.restype = i32
    lib.run_adjoint.argtypes = [vp, i64, i64, C.POINTER(Misfit), C.POINTER(C.c_double), C.POINTER(Grads)]
    lib.run_adjoint.restype = i32
    lib.run.restype = i32
    lib.osam_set_timing.argtypes = [vp, i32]
    lib.osam_set_timing.restype = i32
    lib.osam_get_timing.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(i64)]
    lib.osam_get_timing.restype = i32
    lib.osam_set_fe_launch.argtypes = [vp, i32, i32, i32]
    lib.osam_set_fe_launch.restype = i32
    lib.osam_get_fe_launch.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32)]
    lib.osam_get_fe_launch.restype = i32
    lib.osam_autotune.argtypes = [vp, i64, C.POINTER(SchwarzOpts), C.POINTER(Tuning)]
    lib.osam_autotune.restype = i32
    lib.osam_set_graph.argtypes = [vp, i32, i32]
    lib.osam_set_graph.restype = i32
    lib.osam_set_fe_xshare.argtypes = [vp, i32, i32]
    lib.osam_set_fe_xshare.restype = i32
    lib.osam_set_fusion.argtypes = [vp, i32, i32]
    lib.osam_set_fusion.restype = i32
    lib.osam_set_rom_path.argtypes = [vp, i32, i32]
    lib.osam_set_rom_path.restype = i32
    lib.osam_get_rom_path.argtypes = [vp, i32, C.POINTER(i32)]
    lib.osam_get_rom_path.restype = i32
    lib.osam_sync.argtypes = [vp]
    lib.osam_sync.restype = i32
    lib.osam_set_state.argtypes = [vp, i32, i32, dp, dp, dp]
    lib.osam_set_state.restype = i32
    lib.osam_checkpoint_size.argtypes = [vp, C.POINTER(i64)]
    lib.osam_checkpoint_size.restype = i32
    lib.osam_save_checkpoint.argtypes = [vp, i32, vp]
    lib.osam_save_checkpoint.restype = i32
    lib.osam_load_checkpoint.argtypes = [vp, i32, vp]
    lib.osam_load_checkpoint.restype = i32
    lib.osam_set_opinf_cubic.argtypes = [vp, i32, dp]
    lib.osam_set_opinf_cubic.restype = i32
    lib.osam_get_opinf_cubic.argtypes = [vp, i32, dp]
    lib.osam_get_opinf_cubic.restype = i32
    lib.run_noalloc.argtypes = [vp, i64, C.POINTER(SchwarzOpts), C.POINTER(InstanceInfo)]
    lib.run_noalloc.restype = i32
    lib.osam_set_engine.argtypes = [vp, i32]
    lib.osam_set_engine.restype = i32
    lib.osam_get_solver_stats.argtypes = [vp, i32, C.POINTER(i32)]
    lib.osam_get_solver_stats.restype = i32
    _lib = lib
    return lib


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _devptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


@dataclass
class Options:
    tol_abs: float = 1.0e-8
    tol_rel: float = 1.0e-12
    min_iter: int = 2
    max_iter: int = 32
    guess: int = 0          # 0 HOLD, 1 PREDICTOR
    additive: bool = False  # the additive variant (neighbours' iterates of the previous iteration)

    def c(self) -> SchwarzOpts:
        return SchwarzOpts(self.tol_abs, self.tol_rel, self.min_iter, self.max_iter, self.guess, int(self.additive))


class Context:
    """One libosam context: a batch of coupled-subdomain instances on one GPU."""

    def __init__(self, device: int = 0, precision: str = "f64", batch: int = 1, stream=None):
        """stream: None = torch's current stream on `device` when the context is created
        (if that is torch's default stream, a stream of the context's own, ordered after
        torch's current stream on entry to every call that reads device tensors and before
        it on return); a torch.cuda.Stream or a raw hipStream_t handle (int) otherwise."""
        import torch
        self.lib = load_library()
        self.precision = precision
        self.device = device
        self.batch = batch
        if stream is None:
            cur = torch.cuda.current_stream(device)
            stream = cur if cur.cuda_stream != 0 else torch.cuda.Stream(device)
        elif isinstance(stream, int):
            stream = torch.cuda.ExternalStream(stream, device=device)
        self.stream = stream
        h = C.c_void_p()
        prec = {"f64": 0, "f32": 1, "f32_bf16h": 2}[precision]
        st = self.lib.osam_ctx_create(C.byref(h), device, prec, batch, C.c_void_p(stream.cuda_stream))
        if st != OSAM_OK:
            raise OsamError(st, "osam_ctx_create failed")
        self.h = h
        self.n_sd = 0

    # -- helpers -----------------------------------------------------------
    def _order_in(self):
        """The context's stream waits for what torch has queued on its current stream
        (device inputs written by torch)."""
        import torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _order_out(self):
        """Torch's current stream waits for the context's work (device outputs)."""
        import torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)

    def _check(self, st: int):
        if st != OSAM_OK:
            raise OsamError(st, self.lib.osam_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.osam_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- set-up ------------------------------------------------------------
    def create_subdomain(self, nx, ny, nz, Lx, Ly, Lz, z_lo, z_hi, E, nu, rho, dt,
                         clamp_ends=True, beta=0.0, gamma=0.5, lateral_fix=(), n_sub=1, material="linear") -> int:
        """lateral_fix: components (0 = x, 1 = y, 2 = z) held at zero on the lateral faces;
        dt: the controller step, taken in n_sub Newmark steps of dt / n_sub; material:
        "linear" (linear elasticity) or "svk" (Saint Venant-Kirchhoff)."""
        mask = 0
        for c in lateral_fix:
            mask |= 1 << int(c)
        d = SubdomainDesc(nx, ny, nz, Lx, Ly, Lz, z_lo, z_hi, E, nu, rho, int(clamp_ends), mask, dt,
                          beta, gamma, int(n_sub), {"linear": 0, "svk": 1}[material])
        sid = C.c_int32()
        self._check(self.lib.create_subdomain(self.h, C.byref(d), C.byref(sid)))
        self.n_sd += 1
        return sid.value

    def couple(self):
        self._check(self.lib.osam_couple(self.h))

    def sizes(self, sd: int) -> dict:
        nn, nf, ns = C.c_int64(), C.c_int64(), C.c_int64()
        r, rs = C.c_int32(), C.c_int32()
        self._check(self.lib.osam_sizes(self.h, sd, C.byref(nn), C.byref(nf), C.byref(ns),
                                        C.byref(r), C.byref(rs)))
        return dict(n_nodes=nn.value, n_free=nf.value, n_sch=ns.value, r=r.value, r_s=rs.value)

    def set_initial(self, inst: int, u0: np.ndarray, v0: np.ndarray):
        u0, v0 = _f64(u0), _f64(v0)
        self._check(self.lib.osam_set_initial(self.h, inst, _dptr(u0), _dptr(v0)))

    def get_state(self, sd: int, inst: int = 0):
        n = self.sizes(sd)["n_nodes"]
        u, v, a = (np.zeros((3, n)) for _ in range(3))
        self._check(self.lib.osam_get_state(self.h, sd, inst, _dptr(u), _dptr(v), _dptr(a)))
        return u, v, a

    def set_state(self, sd: int, inst: int, x, xd, xdd):
        """FOM: u, v, a [3][n_nodes] (osam_get_state layout); OpInf: q, q', q'' [r]."""
        x, xd, xdd = _f64(x), _f64(xd), _f64(xdd)
        self._check(self.lib.osam_set_state(self.h, sd, inst, _dptr(x), _dptr(xd), _dptr(xdd)))

    def save_checkpoint(self, inst: int = 0) -> bytes:
        n = C.c_int64()
        self._check(self.lib.osam_checkpoint_size(self.h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self.lib.osam_save_checkpoint(self.h, inst, buf))
        return buf.raw

    def load_checkpoint(self, inst: int, blob: bytes):
        n = C.c_int64()
        self._check(self.lib.osam_checkpoint_size(self.h, C.byref(n)))
        if len(blob) != n.value:
            raise ValueError(f"checkpoint of {len(blob)} bytes, this context's instances take {n.value}")
        buf = C.create_string_buffer(blob, len(blob))
        self._check(self.lib.osam_load_checkpoint(self.h, inst, buf))

    def get_reduced(self, sd: int, inst: int = 0):
        r = self.sizes(sd)["r"]
        q, qd, qdd = (np.zeros(r) for _ in range(3))
        self._check(self.lib.osam_get_reduced(self.h, sd, inst, _dptr(q), _dptr(qd), _dptr(qdd)))
        return q, qd, qdd

    def _torch_dtype(self):
        import torch
        return torch.float64 if self.precision == "f64" else torch.float32

    def _check_buffer(self, name: str, t, shape):
        """A device buffer handed to the library: a contiguous torch tensor on this context's
        GPU, in the context precision, of exactly ``shape`` (the library writes or reads that
        many elements through the raw pointer)."""
        if t is None:
            return
        import torch
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
        if t.dtype != self._torch_dtype():
            raise ValueError(f"{name}: dtype {t.dtype} does not match the context precision {self.precision}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: must be contiguous")
        if tuple(t.shape) != tuple(int(x) for x in shape):
            raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
        if not t.is_cuda or (t.device.index if t.device.index is not None else 0) != self.device:
            raise ValueError(f"{name}: must live on cuda:{self.device}, is on {t.device}")

    def set_record(self, sd: int, every: int, n_cols: int, u=None, a=None, s=None):
        """u, a, s: torch device tensors [batch][n_cols][len] in the context precision:
        u and a of a FOM subdomain len = free DOFs, u of an OpInf subdomain len = r (q),
        s len = Schwarz DOFs."""
        if every > 0:
            z = self.sizes(sd)
            lu = z["r"] if z["r"] > 0 else z["n_free"]
            self._check_buffer("u", u, (self.batch, n_cols, lu))
            self._check_buffer("a", a, (self.batch, n_cols, z["n_free"]))
            self._check_buffer("s", s, (self.batch, n_cols, z["n_sch"]))
        self._keep = getattr(self, "_keep", {})
        self._keep[sd] = (u, a, s)
        rec = Record(every, n_cols, _devptr(u), _devptr(a), _devptr(s))
        self._check(self.lib.osam_set_record(self.h, sd, C.byref(rec)))

    def set_opinf(self, sd: int, Phi, PhiS, A, H=None, B=None, c=None):
        Phi = np.asfortranarray(np.asarray(Phi, dtype=np.float64))
        r = Phi.shape[1]
        rs = 0 if PhiS is None else np.asarray(PhiS).shape[1]
        PhiS_f = None if PhiS is None else np.asfortranarray(np.asarray(PhiS, dtype=np.float64))
        A_f = np.asfortranarray(np.asarray(A, dtype=np.float64))
        H_f = None if H is None else np.asfortranarray(np.asarray(H, dtype=np.float64))
        B_f = None if B is None else np.asfortranarray(np.asarray(B, dtype=np.float64))
        c_f = None if c is None else _f64(c)
        p = lambda a: None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))
        self._check(self.lib.osam_set_opinf(self.h, sd, r, rs, p(Phi), p(PhiS_f), p(A_f), p(H_f),
                                            p(B_f), p(c_f)))

    def set_opinf_cubic(self, sd: int, C3):
        """Cubic operator [r x r(r+1)(r+2)/6] (compressed q_a q_b q_c, a <= b <= c), or None."""
        Cf = None if C3 is None else np.asfortranarray(np.asarray(C3, dtype=np.float64))
        self._check(self.lib.osam_set_opinf_cubic(self.h, sd, None if Cf is None else
                                                  Cf.ctypes.data_as(C.POINTER(C.c_double))))

    def get_opinf_cubic(self, sd: int):
        r = self.sizes(sd)["r"]
        Cf = np.zeros((r, r * (r + 1) * (r + 2) // 6), order="F")
        self._check(self.lib.osam_get_opinf_cubic(self.h, sd, Cf.ctypes.data_as(C.POINTER(C.c_double))))
        return Cf

    def get_opinf(self, sd: int, quadratic: bool = False, with_c: bool = False):
        z = self.sizes(sd)
        r, rs, nf, ns = z["r"], z["r_s"], z["n_free"], z["n_sch"]
        Phi = np.zeros((nf, r), order="F")
        PhiS = np.zeros((ns, rs), order="F")
        A = np.zeros((r, r), order="F")
        H = np.zeros((r, r * (r + 1) // 2), order="F") if quadratic else None
        B = np.zeros((r, rs), order="F")
        c = np.zeros(r) if with_c else None
        p = lambda a: None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))
        self._check(self.lib.osam_get_opinf(self.h, sd, p(Phi), p(PhiS), p(A), p(H), p(B), p(c)))
        return dict(Phi=Phi, PhiS=PhiS, A=A, H=H, B=B, c=c)

    def learn_opinf(self, sd: int, U, Udd, S, V0, n_traj: int, T: int, form: str = "linear",
                    r: int = 0, r_s: int = 0, energy: float = 1 - 1e-6, energy_bnd: float = 1 - 1e-6,
                    lambdas: Sequence[float] = (1e-10,), with_c: bool = False, stride: int = 1):
        lam = _f64(list(lambdas))
        z = self.sizes(sd)
        if n_traj < 1 or T < 1:
            raise ValueError("n_traj and T must be >= 1")
        for name, t, ln in (("U", U, z["n_free"]), ("Udd", Udd, z["n_free"]), ("S", S, z["n_sch"])):
            if t is None:
                raise ValueError(f"{name}: snapshots are required")
            self._check_buffer(name, t, (n_traj, T, ln))
        if V0 is None:
            raise ValueError("V0: initial velocities are required")
        self._check_buffer("V0", V0, (n_traj, z["n_free"]))
        nsig = min(z["n_free"], n_traj * T)
        sig = np.zeros(nsig)
        E = np.zeros(len(lam))
        ls = C.c_double()
        ro, rso = C.c_int32(), C.c_int32()
        d = OpinfDesc({"linear": 0, "quadratic": 1, "cubic": 2}[form], int(with_c), r, r_s, energy, energy_bnd, len(lam),
                      _dptr(lam), n_traj, T, _devptr(U), _devptr(Udd), _devptr(S), _devptr(V0),
                      _dptr(sig), _dptr(E), C.pointer(ls), C.pointer(ro), C.pointer(rso), stride)
        self._order_in()
        self._check(self.lib.learn_opinf(self.h, sd, C.byref(d)))
        self._order_out()
        return dict(sigma=sig, E_lambda=E, lambda_star=ls.value, r=ro.value, r_s=rso.value)

    # -- time loop ---------------------------------------------------------
    def _infos(self):
        return (InstanceInfo * self.batch)()

    @staticmethod
    def _info_list(arr) -> List[dict]:
        return [dict(steps=i.steps, last_iters=i.last_iters, last_converged=i.last_converged,
                     abs2=i.abs2, den2=i.den2, total_iters=i.total_iters, max_iters=i.max_iters,
                     unconverged=i.unconverged, status=i.status) for i in arr]

    def schwarz_step(self, opts: Options = Options()) -> List[dict]:
        info = self._infos()
        o = opts.c()
        self._order_in()
        self._check(self.lib.schwarz_step(self.h, C.byref(o), info))
        self._order_out()
        return self._info_list(info)

    def run_noalloc(self, n_steps: int, opts: Options = Options()) -> List[dict]:
        """run without device allocation (partial sums in the library's static array)."""
        info = self._infos()
        o = opts.c()
        self._order_in()
        st = self.lib.run_noalloc(self.h, n_steps, C.byref(o), info)
        self._order_out()
        self._check(st)
        return self._info_list(info)

    def run(self, n_steps: int, opts: Options = Options(), check: bool = True) -> List[dict]:
        info = self._infos()
        o = opts.c()
        self._order_in()
        st = self.lib.run(self.h, n_steps, C.byref(o), info)
        self._order_out()
        if check:
            self._check(st)
        return self._info_list(info)

    def set_reduced(self, sd: int, inst: int, q0, qd0):
        """Reduced initial state of an OpInf subdomain (after set_initial, before any step)."""
        q0, qd0 = _f64(q0), _f64(qd0)
        self._check(self.lib.osam_set_reduced(self.h, sd, inst, _dptr(q0), _dptr(qd0)))

    def run_adjoint(self, n_steps: int, checkpoint_every: int, every: int, obs: dict):
        """Misfit J and its gradient (see run_adjoint in osam.h).

        obs: {subdomain id: device tensor [n_obs, n_free] (FOM) or [n_obs, r] (OpInf)}.
        Returns (J, grads) with grads[sd] = dict(A, H, B, c, q0, qd0) (numpy float64, the
        layouts of set_opinf) for OpInf subdomains and dict(u0, v0) (device tensors
        [n_free]) for FOM subdomains."""
        import torch
        m = Misfit()
        m.every = every
        keep = []
        for sd, t in obs.items():
            t = t.contiguous()
            keep.append(t)
            m.obs[sd] = t.data_ptr()
        g = Grads()
        out = {}
        for sd in range(self.n_sd):
            z = self.sizes(sd)
            if z["r"] > 0:
                r, rs = z["r"], z["r_s"]
                d = dict(A=np.zeros((r, r), order="F"), B=np.zeros((r, max(rs, 1)), order="F"),
                         H=np.zeros((r, r * (r + 1) // 2), order="F"), c=np.zeros(r),
                         q0=np.zeros(r), qd0=np.zeros(r))
                g.dA[sd] = _dptr(d["A"])
                g.dH[sd] = _dptr(d["H"])
                g.dB[sd] = _dptr(d["B"])
                g.dc[sd] = _dptr(d["c"])
                g.dq0[sd] = _dptr(d["q0"])
                g.dqd0[sd] = _dptr(d["qd0"])
                if rs == 0:
                    d["B"] = np.zeros((r, 0))
            else:
                dtp = torch.float64 if self.precision == "f64" else torch.float32
                d = dict(u0=torch.zeros(z["n_free"], dtype=dtp, device=f"cuda:{self.device}"),
                         v0=torch.zeros(z["n_free"], dtype=dtp, device=f"cuda:{self.device}"))
                g.du0[sd] = d["u0"].data_ptr()
                g.dv0[sd] = d["v0"].data_ptr()
            out[sd] = d
        J = C.c_double()
        self._order_in()
        self._check(self.lib.run_adjoint(self.h, n_steps, checkpoint_every, C.byref(m), C.byref(J), C.byref(g)))
        self._order_out()
        del keep
        return J.value, out

    def set_timing(self, enable: bool):
        self._check(self.lib.osam_set_timing(self.h, int(enable)))

    def get_timing(self, sd: int):
        ms, n = C.c_double(), C.c_int64()
        self._check(self.lib.osam_get_timing(self.h, sd, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def set_fe_launch(self, sd: int, block: int = 0, kc: int = 0):
        self._check(self.lib.osam_set_fe_launch(self.h, sd, block, kc))

    def get_fe_launch(self, sd: int):
        b, k = C.c_int32(), C.c_int32()
        self._check(self.lib.osam_get_fe_launch(self.h, sd, C.byref(b), C.byref(k)))
        return b.value, k.value

    def autotune(self, trial_steps: int = 20, opts: "Options" = None) -> dict:
        """Fastest launch configuration by trial runs (osam_autotune); the trials advance the
        state, so set the initial condition again afterwards."""
        t = Tuning()
        o = (opts or Options()).c()
        self._order_in()
        self._check(self.lib.osam_autotune(self.h, trial_steps, C.byref(o), C.byref(t)))
        self._order_out()
        n = self.n_sd
        return dict(fe=[(t.fe_block[i], t.fe_kc[i]) for i in range(n)], rom_path=list(t.rom_path[:n]),
                    fe_xs=list(t.fe_xs[:n]), graph=(t.graph_rounds, t.graph_streams), fusion_kc=t.fusion_kc,
                    ms_per_step=t.ms_per_step,
                    from_cache=bool(t.from_cache))

    def set_graph(self, rounds: int, streams: int = 1):
        """Replay captured graphs of `rounds` Schwarz sweeps (0: launch every sweep);
        streams = 2 runs the FOM and OpInf kernels of a sweep concurrently."""
        self._check(self.lib.osam_set_graph(self.h, rounds, streams))

    def set_fe_xshare(self, sd: int, enable: bool):
        """Interior layout of the FE kernel (osam_set_fe_xshare): x-neighbours across lanes."""
        self._check(self.lib.osam_set_fe_xshare(self.h, sd, int(bool(enable))))

    def set_fusion(self, enable: bool, kc: int = 1):
        """Run each Schwarz sweep as one launch (osam_set_fusion); kc node layers per FE thread."""
        self._check(self.lib.osam_set_fusion(self.h, int(bool(enable)), kc))

    def set_rom_path(self, sd: int, path: int):
        """0 automatic, 1 fused, 2 batched (see osam_set_rom_path)."""
        self._check(self.lib.osam_set_rom_path(self.h, sd, path))

    def rom_path(self, sd: int) -> int:
        p = C.c_int32()
        self._check(self.lib.osam_get_rom_path(self.h, sd, C.byref(p)))
        return p.value

    def set_engine(self, engine: int):
        """0: automatic (the single-step explicit path where it applies), 1: the window engine,
        2: the persistent OpInf engine (contexts of explicit OpInf subdomains only)."""
        self._check(self.lib.osam_set_engine(self.h, int(engine)))

    def solver_stats(self, sd: int) -> List[int]:
        """Most CG (FOM) or Newton (OpInf) iterations of an implicit sub-step, per instance."""
        out = (C.c_int32 * self.batch)()
        self._check(self.lib.osam_get_solver_stats(self.h, sd, out))
        return list(out)

    def sync(self):
        self._check(self.lib.osam_sync(self.h))


def free_dof_map(nx: int, ny: int, nzs: int) -> np.ndarray:
    """Library free-DOF index [3][free nodes] of every (node, comp) free DOF in node-major
    order (node ids i + (nx+1)(j + (ny+1) k), layers 1..nzs-1)."""
    npl = (nx + 1) * (ny + 1)
    nfn = npl * (nzs - 1)
    nodes = np.arange(npl, npl * nzs)
    out = np.empty((nodes.size, 3), dtype=np.int64)
    for c in range(3):
        out[:, c] = c * nfn + (nodes - npl)
    return out.ravel()


def add_bar_subdomains(ctx: Context, bar, layers, dt: float, lateral_fix=(), beta=0.0, gamma=0.5,
                       n_sub=None, material="linear") -> List[int]:
    """Create one FOM subdomain per node-layer range of a bar (inputs.Bar); beta, gamma: one
    value or one per subdomain; n_sub: Newmark steps per controller step dt, per subdomain."""
    k = len(layers)
    per = lambda x: list(x) if isinstance(x, (list, tuple)) else [x] * k
    betas, gammas, subs, mats = per(beta), per(gamma), per(1 if n_sub is None else n_sub), per(material)
    return [ctx.create_subdomain(bar.nx, bar.ny, bar.nz, bar.Lx, bar.Ly, bar.Lz, lo, hi, bar.E, bar.nu,
                                 bar.rho, dt, lateral_fix=lateral_fix, beta=b, gamma=g, n_sub=s, material=m)
            for (lo, hi), b, g, s, m in zip(layers, betas, gammas, subs, mats)]


def lib_dof_index(nx: int, ny: int, nzs: int, dofs: np.ndarray) -> np.ndarray:
    """Library free-DOF index [3][free nodes] of node-major DOF ids 3*node + c (node in
    layers 1..nzs-1 of the subdomain)."""
    dofs = np.asarray(dofs, dtype=np.int64)
    npl = (nx + 1) * (ny + 1)
    nfn = npl * (nzs - 1)
    node, comp = dofs // 3, dofs % 3
    return comp * nfn + (node - npl)


def rollout_misfit_function():
    """torch.autograd.Function computing the trajectory misfit J of a coupled run and,
    in backward, its gradient through run_adjoint.

    apply(ctx_osam, sd, n_steps, checkpoint_every, every, obs, u0_global, v0_global,
          Phi, PhiS, A, H, B, c, q0, qd0) -> J  (scalar float64 tensor)

    A, H, B, c (float64, the layouts of set_opinf; H/c may be None), q0, qd0 (float64 [r]) are
    differentiable; set_opinf, set_initial and set_reduced are called in forward, so the
    context is left at the initial state of these inputs.  The forward J comes from the
    same adjoint pass that backward uses (computed once, cached)."""
    import torch

    class RolloutMisfit(torch.autograd.Function):
        @staticmethod
        def forward(fctx, octx, sd, n_steps, K, every, obs, u0g, v0g, Phi, PhiS, A, H, B, c, q0, qd0):
            npy = lambda t: None if t is None else t.detach().cpu().numpy().astype(np.float64)
            octx.set_opinf(sd, Phi, PhiS, npy(A), npy(H), npy(B), npy(c))
            octx.set_initial(0, u0g, v0g)
            octx.set_reduced(sd, 0, npy(q0), npy(qd0))
            J, grads = octx.run_adjoint(n_steps, K, every, obs)
            fctx.grads = grads[sd]
            # gradients go back on each input's device and dtype; None inputs get None
            fctx.meta = [None if t is None else (t.device, t.dtype) for t in (A, H, B, c, q0, qd0)]
            return torch.tensor(J, dtype=torch.float64, device=A.device)

        @staticmethod
        def backward(fctx, gJ):
            g = fctx.grads
            s = float(gJ)
            out = []
            for key, meta in zip(("A", "H", "B", "c", "q0", "qd0"), fctx.meta):
                if meta is None:
                    out.append(None)
                else:
                    out.append(torch.as_tensor(np.asarray(g[key]) * s, dtype=meta[1], device=meta[0]))
            return (None,) * 10 + tuple(out)

    return RolloutMisfit
