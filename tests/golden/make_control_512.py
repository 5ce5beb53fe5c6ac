"""Write the FP64 oracle's reference gradient for one member of the optimal-control
workload at full size (512^2, 5000 real-time steps, 200 lattice-depth knots).

Calls only oracle/ (and the seeded workload definitions).  Start and target are the
oracle's imaginary-time ground states (800 steps of dtau = 0.01 from a Gaussian of width
1.5) at lattice depth 0 and 15, rounded to complex64 and stored, so that the GPU test
starts from the very same values.  Stored: the loss 1 - |<target|psi(T)>|^2, its
gradient with respect to the 200 knots (the oracle's discrete adjoint with sqrt(N)
checkpoints), and central differences of the oracle's loss (h = 1e-3) on three knots
drawn from PCG64(100 + member).

Usage: python tests/golden/make_control_512.py [MEMBER]   (default 3)
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
H = 1e-3
RELAX_STEPS, RELAX_DTAU = 800, 0.01


def ground_state(s, depth):
    r = s.with_(dt=RELAX_DTAU, sx=W.Schedule("const", depth))
    psi, _ = O.step_imag(problem(r), state(r), W.to_c64(W.gaussian(r, 1.5)), RELAX_STEPS)
    return W.to_c64(psi)


def fidelity_loss(s, psi0, target, knots):
    """1 - |<target|psi(T)>|^2 with <a|b> = sum conj(a) b dx dy, psi(T) from the oracle."""
    sk = s.with_(sx=W.Schedule("knots", t0=s.sx.t0, t1=s.sx.t1, knots=knots))
    psi, _ = O.step_real(problem(sk), state(sk), psi0, W.CONTROL_STEPS)
    ov = np.vdot(target.astype(np.complex128), psi) * (s.lx / s.nx) * (s.ly / s.ny)
    return 1.0 - abs(ov) ** 2


def main(member: int = 3):
    t = time.time()
    s = W.control_512(member)
    psi0, target = ground_state(s, 0.0), ground_state(s, 15.0)
    loss, grad, _ = O.adjoint(problem(s), 0.0, psi0, target, W.CONTROL_STEPS)
    ms = np.sort(np.random.Generator(np.random.PCG64(100 + member)).choice(s.sx.knots.size, 3, replace=False))
    fd = []
    for m in ms:
        kp, km = s.sx.knots.copy(), s.sx.knots.copy()
        kp[m] += H
        km[m] -= H
        fd.append((fidelity_loss(s, psi0, target, kp) - fidelity_loss(s, psi0, target, km)) / (2 * H))
    out = os.path.join(HERE, f"control_512_member{member}.npz")
    np.savez_compressed(out, member=member, nsteps=W.CONTROL_STEPS, loss=loss, grad=grad, fd_knots=ms,
                        fd=np.array(fd), fd_h=H, psi0_re=psi0.real, psi0_im=psi0.imag, target_re=target.real,
                        target_im=target.imag)
    print(f"wrote {out} in {time.time() - t:.0f} s; loss {loss:.8f}, |grad| {np.linalg.norm(grad):.4e}, "
          f"fd vs adjoint at {list(ms)}: {[(float(f), float(grad[m])) for f, m in zip(fd, ms)]}", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 3)
