"""Python face of the FP64 CPU oracle (``gpe_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the product package.
It shares no code with the HIP path.

Every routine marshals numpy arrays into the C oracle and back; the arithmetic
lives in ``gpe_oracle.c`` (split step: paper Sec. 3.1; imaginary time: Sec. 3.3;
cavity potential and field: Sec. 5.3, Eqs. 10-14).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpe_oracle.c")
_LIB = os.path.join(_HERE, "libgpe_oracle.so")

NOBS = 6  # norm, Theta, Re alpha, Im alpha, <x>, <y>


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE arithmetic, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Sched(C.Structure):
    _fields_ = [
        ("kind", C.c_int),
        ("nknots", C.c_int),
        ("v0", C.c_double),
        ("v1", C.c_double),
        ("t0", C.c_double),
        ("t1", C.c_double),
        ("knots", C.POINTER(C.c_double)),
    ]


class _Problem(C.Structure):
    _fields_ = [
        ("nx", C.c_int),
        ("ny", C.c_int),
        ("lx", C.c_double),
        ("ly", C.c_double),
        ("dt", C.c_double),
        ("g", C.c_double),
        ("wx", C.c_double),
        ("wy", C.c_double),
        ("x0", C.c_double),
        ("y0", C.c_double),
        ("kx_lat", C.c_double),
        ("ky_lat", C.c_double),
        ("sx", _Sched),
        ("sy", _Sched),
        ("cavity", C.c_int),
        ("vc", C.c_double),
        ("kc", C.c_double),
        ("delta_c", C.c_double),
        ("kappa", C.c_double),
        ("eta", C.c_double),
        ("vuser", C.POINTER(C.c_double)),
        ("n_atoms", C.c_double),
        ("probe_omega", C.c_double),
        ("probe_detuning", C.c_double),
        ("probe_phase", C.c_double),
    ]


class _State(C.Structure):
    _fields_ = [
        ("t", C.c_double),
        ("alpha_re", C.c_double),
        ("alpha_im", C.c_double),
        ("theta", C.c_double),
        ("theta_prev", C.c_double),
        ("have_theta", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P, D, I64 = C.c_void_p, C.c_double, C.c_int64
        _lib.orc_step_real.argtypes = [P, P, P, I64, P]
        _lib.orc_step_imag.argtypes = [P, P, P, I64, P]
        _lib.orc_energy.argtypes = [P, P, D, D, D, P]
        _lib.orc_norm.argtypes = [P, P]
        _lib.orc_norm.restype = D
        _lib.orc_theta.argtypes = [P, P]
        _lib.orc_theta.restype = D
        _lib.orc_fft1d.argtypes = [P, C.c_int, C.c_int]
        _lib.orc_fft2d.argtypes = [P, C.c_int, C.c_int, C.c_int]
        _lib.orc_dft1d.argtypes = [P, P, C.c_int, C.c_int]
        _lib.orc_dft2d.argtypes = [P, P, C.c_int, C.c_int, C.c_int]
        _lib.orc_potential_grid.argtypes = [P, D, D, D, P]
        _lib.orc_adjoint.argtypes = [P, D, P, P, I64, I64, C.c_int, P, P, P]
        _lib.orc_adjoint_axis.argtypes = [P, C.c_int, D, P, P, I64, I64, C.c_int, P, P, P]
        _lib.orc_set_threads.argtypes = [C.c_int]
        _lib.orc_set_threads.restype = C.c_int
    return _lib


def set_threads(n: int = 0) -> int:
    """Set (n > 0) and return the OpenMP thread count the oracle uses."""
    return lib().orc_set_threads(int(n))


@dataclass
class Sched:
    """Lattice depth vs time: const (v0), ramp (v0 -> v1 on [t0, t1]), knots, or
    pulse (v0 on t0 <= t < t1, v1 outside)."""

    kind: str = "const"
    v0: float = 0.0
    v1: float = 0.0
    t0: float = 0.0
    t1: float = 1.0
    knots: np.ndarray | None = None


@dataclass
class Problem:
    """Grid, step and potential of one condensate (oscillator units, hbar = m = 1)."""

    nx: int
    ny: int
    lx: float
    ly: float
    dt: float
    g: float = 0.0
    wx: float = 1.0
    wy: float = 1.0
    x0: float = 0.0
    y0: float = 0.0
    kx_lat: float = 0.0
    ky_lat: float = 0.0
    sx: Sched = field(default_factory=Sched)
    sy: Sched = field(default_factory=Sched)
    cavity: int = 0          # 0 off, 1 (True) field ODE, 2 adiabatic field (Eqs. 14-15)
    vc: float = 0.0
    kc: float = 0.0
    delta_c: float = 0.0
    kappa: float = 0.0
    eta: float = 0.0
    vuser: np.ndarray | None = None
    n_atoms: float = 0.0
    probe_omega: float = 0.0
    probe_detuning: float = 0.0
    probe_phase: float = 0.0

    def _sched(self, s: Sched, keep: list) -> _Sched:
        kind = {"const": 0, "ramp": 1, "knots": 2, "pulse": 3}[s.kind]
        out = _Sched(kind, 0, s.v0, s.v1, s.t0, s.t1, None)
        if kind == 2:
            k = np.ascontiguousarray(s.knots, dtype=np.float64)
            keep.append(k)
            out.nknots = k.size
            out.knots = k.ctypes.data_as(C.POINTER(C.c_double))
        return out

    def cstruct(self):
        keep: list = []
        p = _Problem()
        p.nx, p.ny, p.lx, p.ly, p.dt, p.g = self.nx, self.ny, self.lx, self.ly, self.dt, self.g
        p.wx, p.wy, p.x0, p.y0 = self.wx, self.wy, self.x0, self.y0
        p.kx_lat, p.ky_lat = self.kx_lat, self.ky_lat
        p.sx = self._sched(self.sx, keep)
        p.sy = self._sched(self.sy, keep)
        p.cavity = int(self.cavity)
        p.vc, p.kc, p.delta_c, p.kappa, p.eta = self.vc, self.kc, self.delta_c, self.kappa, self.eta
        p.n_atoms = self.n_atoms
        p.probe_omega, p.probe_detuning, p.probe_phase = self.probe_omega, self.probe_detuning, self.probe_phase
        if self.vuser is not None:
            v = np.ascontiguousarray(self.vuser, dtype=np.float64)
            assert v.shape == (self.ny, self.nx)
            keep.append(v)
            p.vuser = v.ctypes.data_as(C.POINTER(C.c_double))
        return p, keep

    # grid helpers (Sec. 3.1: FFT grid, periodic)
    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dy(self) -> float:
        return self.ly / self.ny

    def xs(self) -> np.ndarray:
        return -0.5 * self.lx + np.arange(self.nx) * self.dx

    def ys(self) -> np.ndarray:
        return -0.5 * self.ly + np.arange(self.ny) * self.dy


@dataclass
class State:
    t: float = 0.0
    alpha: complex = 0j
    theta: float = 0.0
    theta_prev: float = 0.0
    have_theta: bool = False

    def _to_c(self) -> _State:
        return _State(self.t, self.alpha.real, self.alpha.imag, self.theta, self.theta_prev, int(self.have_theta))

    def _from_c(self, s: _State) -> None:
        self.t, self.alpha = s.t, complex(s.alpha_re, s.alpha_im)
        self.theta, self.theta_prev, self.have_theta = s.theta, s.theta_prev, bool(s.have_theta)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def step_real(prob: Problem, state: State, psi, nsteps: int, want_obs: bool = False):
    """Advance psi (copied, FP64) by nsteps real-time split steps; returns (psi, obs|None)."""
    p, keep = prob.cstruct()
    s = state._to_c()
    out = _c128(psi).copy()
    assert out.shape == (prob.ny, prob.nx)
    obs = np.zeros((nsteps, NOBS)) if want_obs else None
    lib().orc_step_real(C.byref(p), C.byref(s), out.ctypes.data, int(nsteps),
                        obs.ctypes.data if want_obs else None)
    state._from_c(s)
    return out, obs


def step_imag(prob: Problem, state: State, psi, nsteps: int, want_obs: bool = False):
    """Advance psi by nsteps imaginary-time steps (normalised after each)."""
    p, keep = prob.cstruct()
    s = state._to_c()
    out = _c128(psi).copy()
    assert out.shape == (prob.ny, prob.nx)
    obs = np.zeros((nsteps, NOBS)) if want_obs else None
    lib().orc_step_imag(C.byref(p), C.byref(s), out.ctypes.data, int(nsteps),
                        obs.ctypes.data if want_obs else None)
    state._from_c(s)
    return out, obs


def energy(prob: Problem, psi, t: float = 0.0, alpha: complex = 0j) -> dict:
    """Energy functional {ekin, epot, eint, e, mu, norm} (per unit norm)."""
    p, keep = prob.cstruct()
    a = _c128(psi)
    out = np.zeros(6)
    lib().orc_energy(C.byref(p), a.ctypes.data, float(t), float(alpha.real), float(alpha.imag),
                     out.ctypes.data)
    return dict(zip(("ekin", "epot", "eint", "e", "mu", "norm"), out.tolist()))


def norm(prob: Problem, psi) -> float:
    p, keep = prob.cstruct()
    a = _c128(psi)  # keep the (possibly converted) array alive across the call
    return lib().orc_norm(C.byref(p), a.ctypes.data)


def theta(prob: Problem, psi) -> float:
    p, keep = prob.cstruct()
    a = _c128(psi)
    return lib().orc_theta(C.byref(p), a.ctypes.data)


def cos2(prob: Problem, psi) -> float:
    """integral cos^2(kc x) |psi|^2 dx dy (the dispersive-shift overlap)."""
    lib().orc_cos2.restype = C.c_double
    lib().orc_cos2.argtypes = [C.c_void_p, C.c_void_p]
    p, keep = prob.cstruct()
    a = _c128(psi)
    return float(lib().orc_cos2(C.byref(p), a.ctypes.data))


def alpha_adiabatic(prob: Problem, psi, t: float = 0.0) -> complex:
    """The adiabatic cavity field of the density of psi at time t (Eqs. 14-15)."""
    lib().orc_alpha_adiabatic.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
    p, keep = prob.cstruct()
    a = _c128(psi)
    out = np.zeros(2)
    lib().orc_alpha_adiabatic(C.byref(p), a.ctypes.data, float(t), out.ctypes.data)
    return complex(out[0], out[1])


def potential(prob: Problem, t: float = 0.0, alpha: complex = 0j) -> np.ndarray:
    p, keep = prob.cstruct()
    v = np.zeros((prob.ny, prob.nx))
    lib().orc_potential_grid(C.byref(p), float(t), float(alpha.real), float(alpha.imag), v.ctypes.data)
    return v


def fft1d(a, inverse: bool = False) -> np.ndarray:
    out = _c128(a).copy()
    lib().orc_fft1d(out.ctypes.data, out.size, int(inverse))
    return out


def fft2d(a, inverse: bool = False) -> np.ndarray:
    out = _c128(a).copy()
    ny, nx = out.shape
    lib().orc_fft2d(out.ctypes.data, nx, ny, int(inverse))
    return out


def dft1d(a, inverse: bool = False) -> np.ndarray:
    a = _c128(a)
    out = np.zeros_like(a)
    lib().orc_dft1d(a.ctypes.data, out.ctypes.data, a.size, int(inverse))
    return out


def dft2d(a, inverse: bool = False) -> np.ndarray:
    a = _c128(a)
    out = np.zeros_like(a)
    ny, nx = a.shape
    lib().orc_dft2d(a.ctypes.data, out.ctypes.data, nx, ny, int(inverse))
    return out


def adjoint(prob: Problem, t0: float, psi0, target, nsteps: int, ckpt: int = 0, loss: str = "fidelity",
            control: str = "x"):
    """Loss and its gradient w.r.t. the knot values of the x-lattice (control "x") or the
    y-lattice, i.e. pump (control "y"), depth schedule (discrete adjoint); cavity off, or
    the adiabatic field with the fidelity loss.

    Returns (loss, grad[M], psi_final)."""
    p, keep = prob.cstruct()
    a0, tg = _c128(psi0), _c128(target)
    axis = {"x": 0, "y": 1}[control]
    m = (prob.sx if axis == 0 else prob.sy).knots.size
    grad = np.zeros(m)
    lossv = C.c_double(0)
    fin = np.zeros_like(a0)
    if ckpt <= 0:
        ckpt = max(1, int(round(np.sqrt(nsteps))))
    rc = lib().orc_adjoint_axis(C.byref(p), axis, float(t0), a0.ctypes.data, tg.ctypes.data, int(nsteps),
                                int(ckpt), {"fidelity": 0, "energy": 1}[loss], C.byref(lossv), grad.ctypes.data,
                                fin.ctypes.data)
    if rc != 0:
        raise ValueError("oracle adjoint: unsupported problem (cavity on or controls not knots)")
    return lossv.value, grad, fin


def _step_k(fn, prob: Problem, state: State, psik, nsteps: int, want_obs: bool):
    p, keep = prob.cstruct()
    s = state._to_c()
    out = _c128(psik).copy()
    assert out.shape == (prob.ny, prob.nx)
    obs = np.zeros(nsteps) if want_obs else None
    rc = fn(C.byref(p), C.byref(s), out.ctypes.data, int(nsteps), obs.ctypes.data if want_obs else None)
    if rc != 0:
        raise ValueError("the Fourier-space ordering runs without the cavity")
    state._from_c(s)
    return out, obs


def step_real_k(prob: Problem, state: State, psik, nsteps: int, want_obs: bool = False):
    """Real-time steps in the T/2-V-T/2 ordering with psi_k = FFT2(psi) kept in Fourier space."""
    lib().orc_step_real_k.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    return _step_k(lib().orc_step_real_k, prob, state, psik, nsteps, want_obs)


def step_imag_k(prob: Problem, state: State, psik, nsteps: int, want_obs: bool = False):
    """Imaginary-time steps in the T/2-V-T/2 ordering (Fourier-space state)."""
    lib().orc_step_imag_k.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    return _step_k(lib().orc_step_imag_k, prob, state, psik, nsteps, want_obs)


def momentum_orders(prob: Problem, psik, axis: int, order_step: int, nmax: int):
    """Populations of the momentum orders -nmax..nmax (fractions) and the norm of a
    Fourier-space state psik = FFT2(psi)."""
    lib().orc_momentum_orders.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]
    p, keep = prob.cstruct()
    a = _c128(psik)
    assert a.shape == (prob.ny, prob.nx)
    out = np.zeros(2 * nmax + 2)
    if lib().orc_momentum_orders(C.byref(p), a.ctypes.data, int(axis), int(order_step), int(nmax), out.ctypes.data):
        raise ValueError("bad axis, order_step or nmax")
    return out[:-1], float(out[-1])
