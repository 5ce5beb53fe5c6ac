"""Every path runs twice from the same inputs and must give bitwise-equal outputs.

The reductions are per-work-group partials summed in a fixed order and no kernel uses
floating-point atomics, so a race in LDS (a missing barrier, an exchange read before it
is written) would show up here as a non-repeatable result."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2404_14401_amd import workloads as W
from tests.gpu_util import to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def twice(fn):
    torch = torch_cuda()
    a, b = fn(), fn()
    torch.cuda.synchronize()
    return a, b


def same(a, b):
    torch = torch_cuda()
    if isinstance(a, (list, tuple)):
        return all(same(x, y) for x, y in zip(a, b))
    if isinstance(a, torch.Tensor):
        return bool((a.view(torch.float32) == b.view(torch.float32)).all()) if a.is_complex() else bool((a == b).all())
    return np.array_equal(np.asarray(a), np.asarray(b))


@pytest.mark.parametrize("path", ["lds", "multipass"])
@pytest.mark.parametrize("kind", ["real", "imag", "cavity", "adiabatic"])
def test_plain_paths_are_bitwise_repeatable(path, kind, monkeypatch):
    torch = torch_cuda()
    from paper_2404_14401_amd import gpe

    monkeypatch.setenv("GPE_PATH", path)
    s = {"real": W.Setup(nx=128, ny=64, lx=16.0, ly=10.0, dt=0.01, g=50.0, kx_lat=1.0,
                         sx=W.Schedule("ramp", 0.0, 5.0, 0.0, 0.5)),
         "imag": W.imag_ground_64(100.0),
         "cavity": W.cavity_scaled(128, 0),
         "adiabatic": W.self_organisation_128(14.0, -10.0)}[kind]
    psi0 = W.to_c64(W.gaussian(s, 1.5, 0.2, -0.1))

    def run():
        plan = gpe.Plan.from_setup(s)
        d = to_dev(psi0)
        obs = torch.zeros((200, 6), dtype=torch.float64, device="cuda")
        (plan.step_imag if kind == "imag" else plan.step_real)(d, 200, 0.0, obs)
        return d, obs, plan.cavity()["alpha"]

    a, b = twice(run)
    assert same(a, b)


def test_fourier_space_and_momentum_orders_are_bitwise_repeatable():
    torch = torch_cuda()
    from paper_2404_14401_amd import gpe

    s = W.kapitza_dirac_512(W.KD_G)
    psik0 = W.to_c64(O.fft2d(W.kapitza_dirac_start(s)))

    def run():
        plan = gpe.Plan.from_setup(s)
        d = to_dev(psik0)
        plan.step_real_k(d, 100, 0.0)
        e = to_dev(psik0)
        plan.step_imag_k(e, 20, 0.0)
        return d, e, plan.momentum_orders(d, 1, W.KD_ORDER_STEP, 4)[0]

    a, b = twice(run)
    assert same(a, b)


def test_batched_and_adjoint_are_bitwise_repeatable():
    torch = torch_cuda()
    from paper_2404_14401_amd import gpe

    sweep = W.sweep_208(3, counts=(3, 2, 1))
    setups = sweep + [W.self_organisation_128(12.0, -10.0).with_(nx=256, ny=256, lx=32.0, ly=32.0, dt=sweep[0].dt)]
    psi0 = [W.to_c64(W.gaussian(x, 1.0)) for x in setups]

    def run_batch():
        b = gpe.Batch(setups)
        devs = [to_dev(p) for p in psi0]
        b.step(devs, 120, 0.0)
        return devs, [b.cavity(len(setups) - 1)]

    a, b = twice(run_batch)
    assert same(a, b)

    n = 40
    ctl = [W.control_512(k, nknots=10, nsteps=n).with_(nx=128, ny=128, lx=8.0, ly=8.0) for k in range(2)]
    knots = np.stack([x.sx.knots for x in ctl])
    p0 = [W.to_c64(W.gaussian(x, 1.0, 0.2, 0.0)) for x in ctl]
    tg = [W.to_c64(W.gaussian(x, 0.9, -0.2, 0.1)) for x in ctl]

    def run_adj():
        bb = gpe.Batch(ctl)
        loss, grad, _ = gpe.adjoint(bb, [to_dev(p) for p in p0], [to_dev(t) for t in tg], n, knots,
                                    mode="reconstruct")
        return loss, grad

    a, b = twice(run_adj)
    assert same(a, b)
