"""Write the FP64 oracle's reference for the full cavity workload (1024x1024, 2e4 steps).

Calls only oracle/ (and the seeded workload definitions).  The start state is
workloads.cavity_start_guess relaxed by CAVITY_RELAX_STEPS imaginary-time steps of
CAVITY_RELAX_DTAU in trap + pump with the cavity off (workloads.cavity_relax), rounded
to complex64; it does not depend on the seed (eta enters only the cavity) and is stored
with the references, so that the GPU test starts from the very same values.

Stored per seed: the whole final state (complex64), the final energy functional, and
alpha, Theta and the norm every 100 steps.  With --series-only, the final state is kept
on every 16th point only (a seed whose run is checked through its field and overlap).

Usage: python tests/golden/make_cavity_1024.py [--series-only] SEED [SEED ...]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2404_14401_amd import workloads as W  # noqa: E402
from tests.bridge import problem, state  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
START = os.path.join(HERE, "cavity_1024_start.npz")
SUB = 16


def start_state(s=None, path=START):
    """The run's start (module doc): loaded when stored, else computed on the oracle and stored."""
    if os.path.exists(path):
        g = np.load(path)
        return (g["re"] + 1j * g["im"]).astype(np.complex64)
    s = s or W.cavity_1024(0)
    relax = W.cavity_relax(s)
    psi, _ = O.step_imag(problem(relax), state(relax), W.cavity_start_guess(s), W.CAVITY_RELAX_STEPS)
    psi = W.to_c64(psi)
    np.savez_compressed(path, re=psi.real.astype(np.float32), im=psi.imag.astype(np.float32),
                        relax_steps=W.CAVITY_RELAX_STEPS, relax_dtau=W.CAVITY_RELAX_DTAU)
    return psi


def main(seed: int, series_only: bool = False, nsteps: int = W.CAVITY_1024_STEPS):
    s = W.cavity_1024(seed)
    t = time.time()
    psi0 = start_state(s)
    st = state(s)
    psi, obs = O.step_real(problem(s), st, psi0, nsteps, want_obs=True)
    e = O.energy(problem(s), psi, nsteps * s.dt, st.alpha)
    out = os.path.join(HERE, f"cavity_1024_seed{seed}.npz")
    fields = dict(energy=np.array([e[k] for k in ("ekin", "epot", "eint", "e", "mu", "norm")]),
                  alpha=obs[99::100, 2] + 1j * obs[99::100, 3], theta=obs[99::100, 1], norm=obs[99::100, 0],
                  seed=seed, nsteps=nsteps, eta=s.eta, depth=W.CAVITY_DEPTH)
    if series_only:
        fields.update(psi_sub=psi[::SUB, ::SUB].astype(np.complex64), sub=SUB)
    else:
        fields.update(psi=psi.astype(np.complex64), sub=1)
    np.savez_compressed(out, **fields)
    print(f"wrote {out} in {time.time() - t:.0f} s; eta {s.eta:.4f}, final alpha {st.alpha}, "
          f"max |alpha| {np.abs(fields['alpha']).max():.3e}, E {e['e']}", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    series = "--series-only" in args
    seeds = [int(a) for a in args if not a.startswith("--")] or [4]
    for sd in seeds:
        main(sd, series)
