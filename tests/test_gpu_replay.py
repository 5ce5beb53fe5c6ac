"""Single plans replay captured chunks of steps as HIP graphs (calls without per-step
observables).  The replayed launches must give exactly the results of launching every
step, across several calls in a row with other GPU work and synchronisation between
them, and with the potential replaced between calls."""
import numpy as np
import pytest

from paper_2404_14401_amd import workloads as W
from tests.gpu_util import to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu

# step counts around the replay threshold: the smallest replayed call (two chunks, no
# middle remainder in real time), a call whose imaginary steps fill the chunks exactly,
# and two chunks with remainders
STEP_COUNTS = (66, 65 + 32, 73)


def setup_for(kind):
    if kind == "cavity":
        return W.cavity_scaled(128, 1)
    if kind == "imag":
        return W.imag_ground_64(100.0).with_(nx=128, ny=256, lx=16.0, ly=32.0, kx_lat=1.0, sx=W.Schedule("const", 4.0))
    # a ramped lattice: every kick sits at its own time
    return W.Setup(nx=256, ny=128, lx=32.0, ly=16.0, dt=2e-3, g=200.0, kx_lat=2.0,
                   sx=W.Schedule("ramp", 0.0, 8.0, 0.0, 0.2))


def run_calls(kind, replay, n0, monkeypatch):
    torch = torch_cuda()
    from paper_2404_14401_amd import gpe

    if replay:
        monkeypatch.delenv("GPE_PLAN_GRAPH", raising=False)
    else:
        monkeypatch.setenv("GPE_PLAN_GRAPH", "0")
    monkeypatch.setenv("GPE_PATH", "multipass")
    s = setup_for(kind)
    plan = gpe.Plan.from_setup(s)
    d = to_dev(W.to_c64(W.gaussian(s, 1.5, 0.3, -0.2)))
    out = []
    t = 0.0
    for call in range(3):
        if call == 2:
            plan.set_potential(s.with_(wx=1.3))
        (plan.step_imag if kind == "imag" else plan.step_real)(d, n0 + call, t)
        t += (n0 + call) * s.dt
        out.append(to_host(d))
        torch.cuda.synchronize()
        _ = (d.abs() ** 2).sum().item()  # other work on the stream between calls
        out.append(plan.cavity()["alpha"] if kind == "cavity" else 0j)
    return out


@pytest.mark.parametrize("n0", STEP_COUNTS)
@pytest.mark.parametrize("kind", ["real", "imag", "cavity"])
def test_replayed_chunks_equal_launching_every_step(kind, n0, monkeypatch):
    a = run_calls(kind, True, n0, monkeypatch)
    b = run_calls(kind, False, n0, monkeypatch)
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y))
