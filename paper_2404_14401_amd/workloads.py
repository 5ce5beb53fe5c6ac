"""Seeded synthetic workloads: grid/potential parameters and initial wave functions.

This module holds data only -- box sizes, step counts, potential parameters and
seeded initial states -- and none of the split-step arithmetic.  Both the GPU
path's tests/benchmarks and the CPU oracle's tests draw their inputs from here, so
the two sides always start from the same complex64-rounded values.

Units are the dimensionless oscillator units of the paper (Sec. 3.2): hbar = m = 1,
lengths in l = sqrt(hbar/(m w)), times in 1/w.  Grids are x_i = -L/2 + i L/N.

The five workloads follow the method's use in the paper: imaginary-time ground
states (Sec. 3.3, Sec. 5.1), real-time lattice dynamics (Sec. 5.2), the
self-consistent cavity potential (Sec. 5.3), plus a batched parameter sweep and an
optimal-control gradient of the lattice depth.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np


@dataclass
class Schedule:
    """Lattice depth vs time: 'const' (v0), 'ramp' (v0 -> v1 on [t0, t1], clamped),
    'knots' (piecewise-linear through `knots` spread evenly on [t0, t1]) or 'pulse'
    (v0 for t0 <= t < t1, v1 outside: a lattice flashed on)."""

    kind: str = "const"
    v0: float = 0.0
    v1: float = 0.0
    t0: float = 0.0
    t1: float = 1.0
    knots: np.ndarray | None = None


@dataclass
class Setup:
    """One condensate: grid, step, interaction and external potential."""

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
    sx: Schedule = field(default_factory=Schedule)
    sy: Schedule = field(default_factory=Schedule)
    cavity: bool = False
    vc: float = 0.0
    kc: float = 0.0
    delta_c: float = 0.0
    kappa: float = 0.0
    eta: float = 0.0
    alpha0: complex = 0j
    # "ode": the field follows d alpha/dt = (i Delta_c - kappa) alpha - i eta Theta;
    # "adiabatic": alpha = N sqrt(Vp U0) Theta / (Delta_c - N U0 C + i kappa) from the
    # current density (Sec. 5.3), N = n_atoms
    cavity_mode: str = "ode"
    n_atoms: float = 0.0
    # on-axis probe of the adiabatic field (Sec. 5.4): alpha += Omega_c e^{i (Delta_p t + phi)}
    # / (Delta_c - N U0 C + i kappa)
    probe_omega: float = 0.0
    probe_detuning: float = 0.0
    probe_phase: float = 0.0

    def xs(self) -> np.ndarray:
        return -0.5 * self.lx + np.arange(self.nx) * (self.lx / self.nx)

    def ys(self) -> np.ndarray:
        return -0.5 * self.ly + np.arange(self.ny) * (self.ly / self.ny)

    def with_(self, **kw) -> "Setup":
        return replace(self, **kw)


def to_c64(psi: np.ndarray) -> np.ndarray:
    """Round an FP64 state to complex64: both sides start from these exact values."""
    return np.ascontiguousarray(psi, dtype=np.complex64)


def normalise(s: Setup, psi: np.ndarray) -> np.ndarray:
    """Scale to unit norm, sum |psi|^2 dx dy = 1 (normalisation convention)."""
    da = (s.lx / s.nx) * (s.ly / s.ny)
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2) * da)


def gaussian(s: Setup, width: float = 1.0, cx: float = 0.0, cy: float = 0.0) -> np.ndarray:
    x, y = np.meshgrid(s.xs(), s.ys())
    return normalise(s, np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * width**2)).astype(np.complex128))


def noisy_gaussian(s: Setup, seed: int, width: float = 1.5, amp: float = 0.05) -> np.ndarray:
    """Gaussian of the given width times (1 + amp*xi), xi ~ U[-1, 1) i.i.d. in C order
    from PCG64(seed), normalised in FP64 and rounded to complex64."""
    x, y = np.meshgrid(s.xs(), s.ys())
    xi = np.random.Generator(np.random.PCG64(seed)).uniform(-1.0, 1.0, size=(s.ny, s.nx))
    psi = np.exp(-(x**2 + y**2) / (2 * width**2)) * (1.0 + amp * xi)
    return to_c64(normalise(s, psi.astype(np.complex128)))


def thomas_fermi_guess(s: Setup, mu: float) -> np.ndarray:
    """sqrt(max(mu - V_trap, 0)/g) (trap only), smoothed by a small floor, normalised:
    a synthetic start close to a strongly interacting ground state (Sec. 5.1)."""
    x, y = np.meshgrid(s.xs(), s.ys())
    v = 0.5 * (s.wx**2 * (x - s.x0) ** 2 + s.wy**2 * (y - s.y0) ** 2)
    dens = np.maximum(mu - v, 0.0) / max(s.g, 1e-30)
    psi = np.sqrt(dens) + 1e-3 * np.exp(-(x**2 + y**2) / (2 * (0.25 * s.lx) ** 2))
    return normalise(s, psi.astype(np.complex128))


def random_state(s: Setup, seed: int) -> np.ndarray:
    """Smooth random complex field (band-limited noise) for pass-level checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((s.ny, s.nx)) + 1j * rng.standard_normal((s.ny, s.nx))
    return to_c64(normalise(s, z))


# ----------------------------------------------------------------- workloads

def imag_ground_64(g: float) -> Setup:
    """Imaginary-time ground state: 64x64 on [-8, 8)^2, harmonic trap w = 1,
    dtau = 1e-3, 2000 steps, g in {0, 100}."""
    return Setup(nx=64, ny=64, lx=16.0, ly=16.0, dt=1e-3, g=g)


IMAG_64_STEPS = 2000


def dipole_lattice_256() -> Setup:
    """Real-time dynamics on 256x256, [-16, 16)^2, g = 500, trap centre moved to
    (0, 0.5), lattice Vx(t) cos^2(2x) ramped 0 -> 10 over the first 5000 steps
    (t = 2.5), dt = 5e-4, 10000 steps."""
    return Setup(nx=256, ny=256, lx=32.0, ly=32.0, dt=5e-4, g=500.0, y0=0.5, kx_lat=2.0,
                 sx=Schedule("ramp", 0.0, 10.0, 0.0, 2.5))


DIPOLE_256_STEPS = 10000


def cavity_1024(seed: int = 0) -> Setup:
    """Self-consistent cavity run on 1024x1024, [-32, 32)^2, trap w = 0.05, g = 1000,
    red-detuned pump lattice Vp cos^2(y) with Vp = -25 (50 recoil energies, E_r = k^2/2),
    cavity lattice Vc = -25, k = 1, Delta_c = -20, kappa = 10, eta = 5 U[0,1) from
    PCG64(seed), dt = 2e-4, 20000 steps, alpha_0 = 0.  With these depths the eta range
    straddles the self-organisation threshold: the lowest seeds stay in the normal phase,
    the highest organise within the run."""
    eta = 5.0 * np.random.Generator(np.random.PCG64(seed)).uniform()
    return Setup(nx=1024, ny=1024, lx=64.0, ly=64.0, dt=2e-4, g=1000.0, wx=0.05, wy=0.05,
                 ky_lat=1.0, sy=Schedule("const", CAVITY_DEPTH), cavity=True, vc=CAVITY_DEPTH, kc=1.0,
                 delta_c=-20.0, kappa=10.0, eta=float(eta))


CAVITY_DEPTH = -25.0
CAVITY_RELAX_STEPS = 2000
CAVITY_RELAX_DTAU = 0.01


def cavity_start_guess(s: Setup) -> np.ndarray:
    """Start of the cavity run before relaxation: the Thomas-Fermi profile of the trap
    (mu = w sqrt(g / pi)).  The run starts from it after CAVITY_RELAX_STEPS imaginary-time
    steps of dtau = CAVITY_RELAX_DTAU in trap + pump with the cavity off (cavity_relax)."""
    return thomas_fermi_guess(s, float(np.sqrt(s.g / np.pi) * s.wx))


def cavity_relax(s: Setup) -> Setup:
    """The imaginary-time set-up that relaxes cavity_start_guess: trap + pump, no cavity."""
    return s.with_(cavity=False, dt=CAVITY_RELAX_DTAU)


CAVITY_1024_STEPS = 20000


def cavity_1024_adiabatic(seed: int = 0) -> Setup:
    """The cavity run with the adiabatic field of Sec. 5.3 (Eqs. 14-15) in place of the
    field ODE: N = eta / sqrt(Vp Vc), so that N sqrt(Vp Vc) is the ODE's coupling, and
    the dispersive shift N Vc C that the ODE leaves out."""
    s = cavity_1024(seed)
    return s.with_(cavity_mode="adiabatic", n_atoms=s.eta / np.sqrt(s.vc * s.sy.v0))


def cavity_scaled(n: int, seed: int = 0) -> Setup:
    """The cavity workload's physics on an n x n grid with the same spacing
    dx = 1/16 (box n/16), for parity at sizes the oracle finishes in seconds."""
    s = cavity_1024(seed)
    return s.with_(nx=n, ny=n, lx=n / 16.0, ly=n / 16.0)


# Kapitza-Dirac diffraction (Sec. 5.2, Fig. 4), dimensionless (hbar = m = 1, unit trap
# frequency): the paper's 2^9 grid and a box of 30 length units, a y lattice
# commensurate with the box (48 periods of cos^2, so neighbouring momentum orders 2k
# apart sit KD_ORDER_STEP = 48 FFT bins apart, orders up to |n| = 4 below the grid's
# Nyquist bin), depth -10 E_r (a red-detuned light shift), E_r = k^2/2, and
# dt = 1.75e-4 ~ 2.2e-3 hbar/E_r.  The populations are read at the steps of
# KD_SNAPSHOTS, t E_r / hbar = 0.46, 0.87, 1.40, spaced as the paper's 18, 34, 55 us.
# g = 1000 puts the Thomas-Fermi radius at ~6 (about ten lattice periods).
KD_ORDER_STEP = 48
KD_SNAPSHOTS = (210, 396, 640)
KD_G = 1000.0


def kapitza_dirac_512(g: float = 0.0) -> Setup:
    """Isotropic unit trap plus a lattice V0 cos^2(k y) flashed on at t = 0 for the
    whole run; g = 0 (non-interacting) or KD_G (interacting)."""
    lx = 30.0
    k = np.pi * KD_ORDER_STEP / lx
    er = 0.5 * k * k
    dt = 1.75e-4
    return Setup(nx=512, ny=512, lx=lx, ly=lx, dt=dt, g=g, wx=1.0, wy=1.0, ky_lat=k,
                 sy=Schedule("pulse", -10.0 * er, 0.0, 0.0, KD_SNAPSHOTS[-1] * dt))


def kapitza_dirac_start(s: Setup) -> np.ndarray:
    """The condensate before the flash: the trap's Gaussian ground state for g = 0, the
    Thomas-Fermi profile sqrt((mu - V)/g) with mu = sqrt(g / pi) (2D, unit trap) for g > 0;
    rounded to complex64."""
    if s.g == 0.0:
        return to_c64(gaussian(s, 1.0))
    return to_c64(thomas_fermi_guess(s, float(np.sqrt(s.g / np.pi))))


# Self-organisation in a transversely pumped cavity (Sec. 5.3, Fig. 5), dimensionless:
# a 128^2 grid on [-8, 8)^2 (dx = 1/8), unit isotropic trap, g = 200 (Thomas-Fermi
# radius ~4, about five lattice periods), pump lattice Vp cos^2(k y) and cavity mode
# along x with k = 2 (E_r = k^2/2 = 2), both red detuned (Vp, U0 < 0), U0 = -2e-3,
# N = 2000 atoms (N |U0| = 4, so the dispersive shift is ~2), kappa = 5 and a negative
# detuning.  Each member ramps the pump from 0 to its final depth linearly over T = 2
# (a shortened stand-in for the paper's 0 -> 15 E_r ramp), then holds it.  The sweep
# is a grid of final depths (0.5 .. 15 E_r) times detunings, Fig. 5b's axes.
SO_DT = 1e-3
SO_RAMP = 2.0


def self_organisation_128(vp_er: float, delta_c: float, g: float = 200.0) -> Setup:
    k = 2.0
    er = 0.5 * k * k
    return Setup(nx=128, ny=128, lx=16.0, ly=16.0, dt=SO_DT, g=g, wx=1.0, wy=1.0, ky_lat=k,
                 sy=Schedule("ramp", 0.0, -vp_er * er, 0.0, SO_RAMP), cavity=True, cavity_mode="adiabatic",
                 vc=-2e-3, kc=k, delta_c=delta_c, kappa=5.0, n_atoms=2000.0)


def self_organisation_sweep(n_vp: int = 16, detunings=(-5.0, -10.0, -20.0, -40.0, -80.0)) -> list[Setup]:
    """Members in (detuning, depth) order: final depths evenly on [0.5, 15] E_r."""
    return [self_organisation_128(float(v), float(d)) for d in detunings for v in np.linspace(0.5, 15.0, n_vp)]


def bragg_probe_128(vp_er: float, delta_p: float, omega_er: float = 10.0, delta_c: float = -10.0) -> Setup:
    """Cavity Bragg spectroscopy (Sec. 5.4, Fig. 6) on the self-organisation setup: the
    pump held at vp_er E_r (below or near threshold) and the on-axis probe of strength
    omega_er E_r at detuning delta_p from the pump.  The probing run starts from the
    imaginary-time ground state of the same setup with the probe off."""
    er = 2.0
    s = self_organisation_128(vp_er, delta_c)
    return s.with_(sy=Schedule("const", -vp_er * er), probe_omega=omega_er * er, probe_detuning=delta_p)


def self_organisation_start(s: Setup) -> np.ndarray:
    """Thomas-Fermi profile of the trap alone, mu = sqrt(g / pi); complex64.  The finite
    trap gives Theta != 0 from the start, so no symmetry-breaking seed is needed."""
    return to_c64(thomas_fermi_guess(s, float(np.sqrt(s.g / np.pi))))


@dataclass
class BatchMember:
    setup: Setup
    psi0: np.ndarray


def sweep_208(seed: int = 0, counts=(128, 64, 16)) -> list[Setup]:
    """Batched sweep: 128 at 128^2 on [-8,8)^2, 64 at 256^2 on [-16,16)^2, 16 at 512^2
    on [-32,32)^2 (dx = 0.125), trap w = 1 plus the 2D lattice V0 (cos^2 2x + cos^2 2y),
    (V0, g) ~ (U[0,20], U[50,1000]) from PCG64(seed) in instance order, dt = 5e-4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for n, cnt in zip((128, 256, 512), counts):
        for _ in range(cnt):
            v0 = float(rng.uniform(0.0, 20.0))
            g = float(rng.uniform(50.0, 1000.0))
            out.append(Setup(nx=n, ny=n, lx=n * 0.125, ly=n * 0.125, dt=5e-4, g=g,
                             kx_lat=2.0, ky_lat=2.0, sx=Schedule("const", v0), sy=Schedule("const", v0)))
    return out


SWEEP_STEPS = 5000


def control_512(b: int, n: int = 512, nknots: int = 200, nsteps: int = 5000) -> Setup:
    """Optimal-control member b: n x n on [-16, 16)^2, trap w = 1, g = 300, lattice
    V0(t) cos^2(2x) piecewise-linear over `nknots` values ~ U[0, 15] from PCG64(b),
    knots spread over [0, T], T = nsteps * dt, dt = 5e-4."""
    knots = np.random.Generator(np.random.PCG64(b)).uniform(0.0, 15.0, size=nknots)
    dt = 5e-4
    return Setup(nx=n, ny=n, lx=32.0, ly=32.0, dt=dt, g=300.0, kx_lat=2.0,
                 sx=Schedule("knots", t0=0.0, t1=nsteps * dt, knots=knots))


CONTROL_STEPS = 5000
CONTROL_BATCH = 16
