"""Python binding of libgpe.so (the gfx950 split-step GPE library, ``include/gpe.h``).

Argument marshalling only: every step of the propagation runs in the library's HIP
kernels.  torch supplies device memory and the stream; wave functions are complex64
CUDA tensors of shape (ny, nx), contiguous, updated in place.

The library must have been built (``python -m paper_2404_14401_amd.build_lib`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GPE_LIB_PATH selects another build of the same library (kernel-variant tuning runs).
LIB_PATH = os.environ.get("GPE_LIB_PATH") or os.path.join(_HERE, "libgpe.so")

OK = 0
ERR_INVALID, ERR_NOMEM, ERR_DEVICE, ERR_NONFINITE, ERR_UNSUPPORTED = -1, -2, -3, -4, -5
NOBS = 6
CONTROL = {"x": 0, "pump": 1}
SCHED = {"const": 0, "ramp": 1, "knots": 2, "pulse": 3}
LOSS = {"fidelity": 0, "energy": 1}
ADJ_MODE = {"auto": 0, "reconstruct": 1, "checkpoint": 2, "store": 3}

# Every entry point the header declares (checked by the CPU tests against include/gpe.h).
EXPORTS = (
    "gpe_plan_create", "gpe_plan_destroy", "gpe_set_potential", "gpe_step_real", "gpe_step_real_k",
    "gpe_step_imag", "gpe_step_imag_k", "gpe_momentum_orders",
    "gpe_energy", "gpe_norm", "gpe_get_cavity", "gpe_set_cavity", "gpe_sync", "gpe_last_error",
    "gpe_set_timing", "gpe_get_timing",
    "gpe_batch_create", "gpe_batch_destroy", "gpe_step_batched", "gpe_batch_tune", "gpe_batch_info",
    "gpe_batch_get_cavity", "gpe_batch_sync", "gpe_adjoint", "gpe_step_real_noalloc",
)


class GpeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gpe error {code}: {msg}")
        self.code = code


class PlanDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("lx", C.c_double), ("ly", C.c_double),
        ("dt", C.c_double), ("g", C.c_double), ("stream", C.c_void_p), ("max_bytes", C.c_size_t),
    ]


class Schedule(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("nknots", C.c_int32), ("v0", C.c_double), ("v1", C.c_double),
        ("t0", C.c_double), ("t1", C.c_double), ("knots", C.POINTER(C.c_double)),
    ]


class PotentialDesc(C.Structure):
    _fields_ = [
        ("wx", C.c_double), ("wy", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
        ("kx_lat", C.c_double), ("ky_lat", C.c_double), ("sx", Schedule), ("sy", Schedule),
        ("cavity", C.c_int32), ("vc", C.c_double), ("kc", C.c_double), ("delta_c", C.c_double),
        ("kappa", C.c_double), ("eta", C.c_double), ("alpha0_re", C.c_double), ("alpha0_im", C.c_double),
        ("v_user", C.c_void_p), ("n_atoms", C.c_double), ("probe_omega", C.c_double),
        ("probe_detuning", C.c_double), ("probe_phase", C.c_double),
    ]


_lib = None


def lib():
    """Load libgpe.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2404_14401_amd/build_lib.py")
        L = C.CDLL(LIB_PATH)
        P, D, I64, I = C.c_void_p, C.c_double, C.c_int64, C.c_int
        L.gpe_plan_create.argtypes = [C.POINTER(P), C.POINTER(PlanDesc)]
        L.gpe_plan_destroy.argtypes = [P]
        L.gpe_set_potential.argtypes = [P, C.POINTER(PotentialDesc)]
        L.gpe_step_real.argtypes = [P, P, I64, D, P]
        L.gpe_step_imag.argtypes = [P, P, I64, D, P]
        L.gpe_step_real_k.argtypes = [P, P, I64, D, P]
        L.gpe_step_imag_k.argtypes = [P, P, I64, D, P]
        L.gpe_momentum_orders.argtypes = [P, P, C.c_int, C.c_int, C.c_int, P]
        L.gpe_energy.argtypes = [P, P, D, P]
        L.gpe_norm.argtypes = [P, P, P]
        L.gpe_get_cavity.argtypes = [P, P]
        L.gpe_set_cavity.argtypes = [P, P, I]
        L.gpe_sync.argtypes = [P]
        L.gpe_set_timing.argtypes = [P, I]
        L.gpe_get_timing.argtypes = [P, P]
        L.gpe_last_error.restype = C.c_char_p
        L.gpe_batch_create.argtypes = [C.POINTER(P), I, P, P]
        L.gpe_batch_destroy.argtypes = [P]
        L.gpe_step_batched.argtypes = [P, P, I64, D]
        L.gpe_batch_tune.argtypes = [P, C.c_char_p]
        L.gpe_batch_info.argtypes = [P, I, P]
        L.gpe_batch_get_cavity.argtypes = [P, I, P]
        L.gpe_batch_sync.argtypes = [P, P]
        L.gpe_adjoint.argtypes = [P, P, P, I64, D, P, I, I, I, I, D, P, P, P, P]
        L.gpe_step_real_noalloc.argtypes = [C.POINTER(PlanDesc), C.POINTER(PotentialDesc), P, I64, D, P]
        for name in EXPORTS:
            if name != "gpe_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != OK:
        raise GpeError(rc, lib().gpe_last_error().decode())


def _stream_handle(stream) -> int | None:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream) or None


def _sched(s, keep: list) -> Schedule:
    if s is None:
        return Schedule(0, 0, 0.0, 0.0, 0.0, 1.0, None)
    out = Schedule(SCHED[s.kind], 0, float(s.v0), float(s.v1), float(s.t0), float(s.t1), None)
    if s.kind == "knots":
        k = np.ascontiguousarray(s.knots, dtype=np.float64)
        keep.append(k)
        out.nknots = k.size
        out.knots = k.ctypes.data_as(C.POINTER(C.c_double))
    return out


def potential_desc(setup, v_user=None):
    """PotentialDesc from a workloads.Setup (keeps the knot arrays alive with it)."""
    keep: list = []
    d = PotentialDesc()
    d.wx, d.wy, d.x0, d.y0 = setup.wx, setup.wy, setup.x0, setup.y0
    d.kx_lat, d.ky_lat = setup.kx_lat, setup.ky_lat
    d.sx = _sched(setup.sx, keep)
    d.sy = _sched(setup.sy, keep)
    d.cavity = (2 if setup.cavity_mode == "adiabatic" else 1) if setup.cavity else 0
    d.n_atoms = float(setup.n_atoms)
    d.probe_omega, d.probe_detuning, d.probe_phase = setup.probe_omega, setup.probe_detuning, setup.probe_phase
    d.vc, d.kc, d.delta_c, d.kappa, d.eta = setup.vc, setup.kc, setup.delta_c, setup.kappa, setup.eta
    a0 = complex(setup.alpha0)
    d.alpha0_re, d.alpha0_im = a0.real, a0.imag
    d.v_user = v_user.data_ptr() if v_user is not None else None
    return d, keep


def _ptr(t, dtype_name: str = "complex64"):
    import torch

    want = getattr(torch, dtype_name)
    if not t.is_cuda or t.dtype != want or not t.is_contiguous():
        raise ValueError(f"expected a contiguous CUDA {dtype_name} tensor, got {t.dtype} on {t.device}")
    return t.data_ptr()


class Plan:
    """One condensate: grid (ny, nx) on a box (ly, lx), step dt, interaction g."""

    def __init__(self, nx: int, ny: int, lx: float, ly: float, dt: float, g: float = 0.0, stream=None,
                 max_bytes: int = 0):
        self.nx, self.ny, self.lx, self.ly, self.dt, self.g = nx, ny, lx, ly, dt, g
        self.stream = stream
        d = PlanDesc(nx, ny, lx, ly, dt, g, _stream_handle(stream), max_bytes)
        h = C.c_void_p()
        check(lib().gpe_plan_create(C.byref(h), C.byref(d)))
        self._h = h
        self._keep = None

    @classmethod
    def from_setup(cls, setup, stream=None, v_user=None):
        p = cls(setup.nx, setup.ny, setup.lx, setup.ly, setup.dt, setup.g, stream)
        p.set_potential(setup, v_user)
        return p

    def close(self):
        if getattr(self, "_h", None):
            lib().gpe_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_potential(self, setup, v_user=None):
        d, keep = potential_desc(setup, v_user)
        self._keep = (keep, v_user)
        check(lib().gpe_set_potential(self._h, C.byref(d)))

    def step_real(self, psi, nsteps: int, t0: float = 0.0, obs=None):
        check(lib().gpe_step_real(self._h, _ptr(psi), int(nsteps), float(t0),
                                  _ptr(obs, "float64") if obs is not None else None))

    def step_real_k(self, psik, nsteps: int, t0: float = 0.0, obs=None):
        """Real-time steps in the T/2-V-T/2 ordering on the Fourier-space state FFT2(psi)."""
        check(lib().gpe_step_real_k(self._h, _ptr(psik), int(nsteps), float(t0),
                                    _ptr(obs, "float64") if obs is not None else None))

    def step_imag_k(self, psik, nsteps: int, t: float = 0.0, obs=None):
        """Imaginary-time steps in the T/2-V-T/2 ordering on the Fourier-space state; unit norm after each."""
        check(lib().gpe_step_imag_k(self._h, _ptr(psik), int(nsteps), float(t),
                                    _ptr(obs, "float64") if obs is not None else None))

    def momentum_orders(self, psik, axis: int, order_step: int, nmax: int):
        """Populations of the momentum orders -nmax..nmax (fractions of the total) and
        the norm, from a Fourier-space state."""
        out = np.zeros(2 * nmax + 2)
        check(lib().gpe_momentum_orders(self._h, _ptr(psik), int(axis), int(order_step), int(nmax),
                                        out.ctypes.data))
        return out[:-1], float(out[-1])

    def step_imag(self, psi, nsteps: int, t: float = 0.0, obs=None):
        check(lib().gpe_step_imag(self._h, _ptr(psi), int(nsteps), float(t),
                                  _ptr(obs, "float64") if obs is not None else None))

    def energy(self, psi, t: float = 0.0) -> dict:
        out = (C.c_double * 6)()
        check(lib().gpe_energy(self._h, _ptr(psi), float(t), out))
        return dict(zip(("ekin", "epot", "eint", "e", "mu", "norm"), list(out)))

    def norm(self, psi) -> float:
        out = C.c_double()
        check(lib().gpe_norm(self._h, _ptr(psi), C.byref(out)))
        return out.value

    def cavity(self) -> dict:
        out = (C.c_double * 4)()
        check(lib().gpe_get_cavity(self._h, out))
        return {"alpha": complex(out[0], out[1]), "theta": out[2], "theta_prev": out[3]}

    def set_cavity(self, alpha: complex, theta: float, theta_prev: float, have_history: bool = True):
        s = (C.c_double * 4)(alpha.real, alpha.imag, theta, theta_prev)
        check(lib().gpe_set_cavity(self._h, s, int(have_history)))

    def sync(self):
        check(lib().gpe_sync(self._h))

    def set_timing(self, every: int):
        """Bracket every `every`-th step's passes with HIP events (0: off)."""
        check(lib().gpe_set_timing(self._h, int(every)))

    def timing(self) -> dict:
        out = (C.c_double * 4)()
        check(lib().gpe_get_timing(self._h, out))
        return {"col_ms": out[0], "col_n": int(out[1]), "row_ms": out[2], "row_n": int(out[3])}


class Batch:
    """Many independent condensates (sizes may differ, dt shared) advanced together."""

    def __init__(self, setups, stream=None):
        n = len(setups)
        descs = (PlanDesc * n)()
        pots = (PotentialDesc * n)()
        self._keep = []
        sh = _stream_handle(stream)
        for i, s in enumerate(setups):
            descs[i] = PlanDesc(s.nx, s.ny, s.lx, s.ly, s.dt, s.g, sh, 0)
            d, keep = potential_desc(s)
            pots[i] = d
            self._keep.append(keep)
        h = C.c_void_p()
        check(lib().gpe_batch_create(C.byref(h), n, descs, pots))
        self._h = h
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            lib().gpe_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, psis):
        if len(psis) != self.n:
            raise ValueError(f"expected {self.n} wave functions")
        return (C.c_void_p * self.n)(*[_ptr(p) for p in psis])

    def step(self, psis, nsteps: int, t0: float = 0.0):
        arr = self._ptrs(psis)
        check(lib().gpe_step_batched(self._h, arr, int(nsteps), float(t0)))

    def tune(self, cache_path: str | None = None):
        check(lib().gpe_batch_tune(self._h, cache_path.encode() if cache_path else None))

    def groups(self) -> list[dict]:
        out = (C.c_int * 8)()
        check(lib().gpe_batch_info(self._h, 0, out))
        res = []
        for g in range(out[7]):
            check(lib().gpe_batch_info(self._h, g, out))
            res.append(dict(nx=out[0], ny=out[1], members=out[2], lds=bool(out[3]), radix=out[4],
                            row_threads=out[5], col_blocks=out[6]))
        return res

    def sync(self) -> None:
        """Wait for the batch; raises GpeError (ERR_NONFINITE, .member set) if a member's
        wave function went non-finite."""
        bad = C.c_int(-1)
        rc = lib().gpe_batch_sync(self._h, C.byref(bad))
        if rc != OK:
            err = GpeError(rc, lib().gpe_last_error().decode())
            err.member = bad.value
            raise err

    def cavity(self, member: int) -> complex:
        """Cavity field of one member after the last call."""
        out = np.zeros(4)
        check(lib().gpe_batch_get_cavity(self._h, int(member), out.ctypes.data))
        return complex(out[0], out[1])


def adjoint(batch: Batch, psi0s, targets, nsteps: int, knots, t0: float = 0.0, mode: str = "auto",
            drift_tol: float = 1e-4, psi_finals=None, control: str = "x", loss: str = "fidelity",
            want_grad: bool = True):
    """Loss 1 - |<target|psi(T)>|^2 (loss "fidelity") or E_kin + E_pot + E_int of psi(T)
    (loss "energy", targets None) and its gradient w.r.t. the knot values of the
    x-lattice (control "x") or pump, y-lattice (control "pump"), depth of every batch
    member (discrete adjoint on the GPU).  knots: array (n, M).
    Returns (loss[n], grad[n, M], info dict); with want_grad False only the forward
    sweep runs and grad is None."""
    k = np.ascontiguousarray(knots, dtype=np.float64)
    n, m = k.shape
    if n != batch.n:
        raise ValueError("one row of knots per batch member")
    out = np.zeros(n)
    grad = np.zeros((n, m)) if want_grad else None
    info = np.zeros(4)
    fin = batch._ptrs(psi_finals) if psi_finals is not None else None
    tg = batch._ptrs(targets) if targets is not None else None
    check(lib().gpe_adjoint(batch._h, batch._ptrs(psi0s), tg, int(nsteps), float(t0),
                            k.ctypes.data, m, CONTROL[control], LOSS[loss], ADJ_MODE[mode], float(drift_tol),
                            out.ctypes.data, grad.ctypes.data if want_grad else None, fin, info.ctypes.data))
    return out, grad, {"mode": {0: "loss", 1: "reconstruct", 2: "checkpoint", 3: "store"}[int(info[0])],
                       "drift": info[1],
                        "workspace_bytes": int(info[2]), "forward_steps": int(info[3])}


def step_real_noalloc(setup, psi, nsteps: int, t0: float = 0.0, stream=None, v_user=None, nonfinite=None):
    """gpe_step_real_noalloc: real-time steps of `psi` under the plan and potential that
    `setup` describes, without a plan and without allocating (the library's static
    scratch holds every table).  nonfinite: optional CUDA int32 tensor of one element
    that receives 1 if a kick met a non-finite value, else 0."""
    d = PlanDesc(setup.nx, setup.ny, setup.lx, setup.ly, setup.dt, setup.g, _stream_handle(stream), 0)
    pd, keep = potential_desc(setup, v_user)
    flag = _ptr(nonfinite, "int32") if nonfinite is not None else None
    check(lib().gpe_step_real_noalloc(C.byref(d), C.byref(pd), _ptr(psi), int(nsteps), float(t0), flag))
    del keep
