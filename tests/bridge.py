"""Test-side helpers: turn a workload Setup into the oracle's Problem and compare
fields.  Imports the oracle, so only tests may use it."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2404_14401_amd.workloads import Setup


def problem(s: Setup) -> O.Problem:
    def sch(x):
        return O.Sched(x.kind, x.v0, x.v1, x.t0, x.t1, x.knots)

    return O.Problem(nx=s.nx, ny=s.ny, lx=s.lx, ly=s.ly, dt=s.dt, g=s.g, wx=s.wx, wy=s.wy, x0=s.x0,
                     y0=s.y0, kx_lat=s.kx_lat, ky_lat=s.ky_lat, sx=sch(s.sx), sy=sch(s.sy),
                     cavity=(2 if s.cavity_mode == "adiabatic" else 1) if s.cavity else 0, vc=s.vc, kc=s.kc,
                     delta_c=s.delta_c, kappa=s.kappa, eta=s.eta, n_atoms=s.n_atoms, probe_omega=s.probe_omega,
                     probe_detuning=s.probe_detuning, probe_phase=s.probe_phase)


def state(s: Setup, t: float = 0.0) -> O.State:
    return O.State(t=t, alpha=complex(s.alpha0))


def rel_l2(a, ref) -> float:
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))
