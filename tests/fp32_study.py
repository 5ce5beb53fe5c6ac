"""Precision study behind the choice of FP64 arithmetic (CPU only; test infrastructure).

Emulates, in numpy, the split step of the GPU passes -- radix-4 Stockham transforms whose
inverse is the exact adjoint of the forward transform (reversed passes, conjugated
twiddles), complex64 storage after every pass, the kick and the kinetic factor applied in
FP64 -- with the transform arithmetic and twiddles in one of four precisions, and compares
the dipole + lattice workload (256^2, 1e4 steps) with the FP64 oracle:

  f32-plain     FP32 arithmetic, twiddles rounded to FP32
  f32-unit      FP32 arithmetic, each twiddle the FP32 pair with the smallest |c^2 + s^2 - 1|
                within +-6 ulps of the rounded one
  f64-unit      FP64 arithmetic with those FP32 unit-searched twiddles (the twiddles' share)
  f64           FP64 arithmetic and twiddles (the shipped design)

Usage: python tests/fp32_study.py VARIANT [STEPS]   (prints final rel-L2 and norm drift)
"""
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2404_14401_amd import workloads as W  # noqa: E402
from tests.bridge import problem, state  # noqa: E402


def _unit_pair(c0, s0, win=6):
    """The FP32 (c, s) within +-win ulps of (c0, s0) with the smallest |c^2 + s^2 - 1|."""
    def around(x):
        x = np.float32(x)
        out, up, dn = [x], x, x
        for _ in range(win):
            up, dn = np.nextafter(up, np.float32(2)), np.nextafter(dn, np.float32(-2))
            out += [up, dn]
        return np.array(out, dtype=np.float64)
    c, s = around(c0)[:, None], around(s0)[None, :]
    err = np.abs(c * c + s * s - 1.0)
    i, j = np.unravel_index(np.argmin(err), err.shape)
    return c[i, 0], s[0, j]


def twiddles(n, kind):
    """W_n^m = exp(-2 pi i m / n), m < n, in the precision of `kind`."""
    a = -2.0 * np.pi * np.arange(n) / n
    c, s = np.cos(a), np.sin(a)
    if kind == "f64":
        return c + 1j * s
    if kind in ("f32-plain",):
        return (c.astype(np.float32) + 1j * s.astype(np.float32)).astype(np.complex64)
    out = np.empty(n, np.complex128)
    for m in range(n):
        if np.isclose(abs(c[m]), 1.0) or np.isclose(abs(s[m]), 1.0):
            out[m] = complex(round(c[m]), round(s[m]))
        else:
            out[m] = complex(*_unit_pair(c[m], s[m]))
    return out.astype(np.complex64) if kind == "f32-unit" else out


def _dft4(a, inv):
    t0, t1, t2, d = a[0] + a[2], a[0] - a[2], a[1] + a[3], a[1] - a[3]
    t3 = (d * (1j if inv else -1j)).astype(a[0].dtype)
    return [t0 + t2, t1 + t3, t0 - t2, t1 - t3]


def fwd(x, tw):
    """Unscaled forward transform along the last axis (radix-4 Stockham, DIT)."""
    n = x.shape[-1]
    u = np.arange(n // 4)
    for p in range(int(round(math.log(n, 4)))):
        ns = 4 ** p
        j, base = u % ns, (u // ns) * 4 * ns + u % ns
        a = [x[..., u + r * (n // 4)] for r in range(4)]
        if ns > 1:
            for r in range(1, 4):
                a[r] = a[r] * tw[r * j * (n // (4 * ns))]
        y = np.empty_like(x)
        for r, v in enumerate(_dft4(a, False)):
            y[..., base + r * ns] = v
        x = y
    return x


def adj(y, tw):
    """The exact adjoint of fwd: its passes reversed, each conjugate-transposed."""
    n = y.shape[-1]
    u = np.arange(n // 4)
    for p in reversed(range(int(round(math.log(n, 4))))):
        ns = 4 ** p
        j, base = u % ns, (u // ns) * 4 * ns + u % ns
        a = _dft4([y[..., base + r * ns] for r in range(4)], True)
        if ns > 1:
            for r in range(1, 4):
                a[r] = a[r] * np.conj(tw[r * j * (n // (4 * ns))])
        x = np.empty_like(y)
        for r in range(4):
            x[..., u + r * (n // 4)] = a[r]
        y = x
    return y


def run(kind, s, psi0, nsteps):
    ct = np.complex128 if kind.startswith("f64") else np.complex64
    twx, twy = twiddles(s.nx, kind).astype(ct), twiddles(s.ny, kind).astype(ct)
    prob = problem(s)
    kx = 2 * np.pi * np.fft.fftfreq(s.nx, s.lx / s.nx)
    ky = 2 * np.pi * np.fft.fftfreq(s.ny, s.ly / s.ny)
    kin = (np.exp(-0.5j * (kx[None, :] ** 2 + ky[:, None] ** 2) * s.dt) / (s.nx * s.ny)).T

    def kick(p, t, h):  # FP64 phase from the stored values, result stored in complex64
        p64 = p.astype(np.complex128)
        th = (O.potential(prob, t) + s.g * np.abs(p64) ** 2) * h
        return (p64 * np.exp(-1j * th)).astype(np.complex64)

    x = fwd(kick(psi0, 0.0, 0.5 * s.dt).astype(ct), twx).astype(np.complex64)
    for n in range(nsteps):
        c = fwd(x.T.astype(ct), twy)
        c = (c.astype(np.complex128) * kin).astype(np.complex64).astype(ct)
        x = adj(c, twy).T.astype(np.complex64)
        r = adj(x.astype(ct), twx).astype(np.complex64)
        if n + 1 < nsteps:
            x = fwd(kick(r, (n + 1) * s.dt, s.dt).astype(ct), twx).astype(np.complex64)
        else:
            x = kick(r, (n + 1) * s.dt, 0.5 * s.dt)
    return x


def main(kind, nsteps=W.DIPOLE_256_STEPS):
    s = W.dipole_lattice_256()
    s0 = s.with_(y0=0.0, sx=W.Schedule("const", 0.0), dt=0.005)
    gs, _ = O.step_imag(problem(s0), state(s0), W.thomas_fermi_guess(s0, float(np.sqrt(s.g / np.pi))), 3000)
    psi0 = W.to_c64(gs)
    ref, _ = O.step_real(problem(s), state(s), psi0, nsteps)
    t = time.time()
    out = run(kind, s, psi0, nsteps).astype(np.complex128)
    da = s.lx / s.nx * s.ly / s.ny
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    drift = (np.sum(np.abs(out) ** 2) - np.sum(np.abs(psi0.astype(np.complex128)) ** 2)) * da
    tw = twiddles(s.nx, kind)
    mod = float(np.abs(np.abs(tw.astype(np.complex128)) ** 2 - 1).max())
    print(f"{kind:10s} {nsteps} steps: rel-L2 {err:.2e}, norm drift {drift:+.2e} ({drift / nsteps:+.1e} per step), "
          f"max twiddle |c^2+s^2-1| {mod:.1e}  [{time.time() - t:.0f} s]", flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else W.DIPOLE_256_STEPS)
