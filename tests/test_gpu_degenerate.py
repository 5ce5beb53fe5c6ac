"""Degenerate step counts through the C ABI: zero steps leave the state and the cavity
field bit-for-bit untouched on every entry point, negative counts are rejected without
side effects (later calls match the same calls on a fresh plan or batch bit for bit), and the adjoint
rejects fewer than one step."""
import numpy as np
import pytest

from paper_2404_14401_amd import workloads as W
from tests.gpu_util import to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def start(s, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    psi = W.gaussian(s, 1.0) * (1 + 0.05 * rng.standard_normal((s.ny, s.nx)))
    return W.to_c64(psi / np.sqrt(np.sum(np.abs(psi) ** 2) * s.lx * s.ly / (s.nx * s.ny)))


def setup(n, mode):
    s = W.cavity_scaled(n, 0)
    if mode == "off":
        return s.with_(cavity=False)
    if mode == "adiabatic":
        return s.with_(cavity_mode="adiabatic", n_atoms=s.eta / np.sqrt(s.vc * s.sy.v0))
    return s


@pytest.mark.parametrize("path", ["auto", "multipass"])
@pytest.mark.parametrize("mode", ["off", "ode", "adiabatic"])
def test_plan_zero_and_negative_steps_change_nothing(path, mode, monkeypatch):
    torch = torch_cuda()
    from paper_2404_14401_amd import gpe

    monkeypatch.setenv("GPE_PATH", path)
    s = setup(32 if path == "auto" else 64, mode)  # 32^2 auto: the LDS-resident path
    psi0 = start(s, 3)
    p = gpe.Plan.from_setup(s)
    d = to_dev(psi0)
    p.step_real(d, 7, 0.0)
    before, cav = to_host(d), p.cavity()
    obs = torch.zeros((0, gpe.NOBS), dtype=torch.float64, device="cuda")
    p.step_real(d, 0, 7 * s.dt, obs)
    p.step_imag(d, 0, 7 * s.dt)
    for bad in (lambda: p.step_real(d, -1, 0.0), lambda: p.step_imag(d, -3, 0.0)):
        with pytest.raises(gpe.GpeError) as e:
            bad()
        assert e.value.code == gpe.ERR_INVALID
    assert np.array_equal(to_host(d), before)
    assert p.cavity() == cav
    # the rejected and empty calls left no trace: continuing matches the same two calls
    # on a fresh plan (a call boundary itself is not free: its half kicks are not merged)
    p.step_real(d, 5, 7 * s.dt)
    q = gpe.Plan.from_setup(s)
    e2 = to_dev(psi0)
    q.step_real(e2, 7, 0.0)
    q.step_real(e2, 5, 7 * s.dt)
    assert np.array_equal(to_host(d), to_host(e2))
    assert p.cavity() == q.cavity()


@pytest.mark.parametrize("mode", ["off", "ode", "adiabatic"])
def test_batch_zero_and_negative_steps_change_nothing(mode):
    torch_cuda()
    from paper_2404_14401_amd import gpe

    setups = [setup(64, mode), setup(128, mode), setup(256, mode)]
    psi0 = [start(s, i) for i, s in enumerate(setups)]
    b = gpe.Batch(setups)
    devs = [to_dev(x) for x in psi0]
    b.step(devs, 6, 0.0)
    before = [to_host(x) for x in devs]
    cav = [b.cavity(i) for i in range(len(setups))]
    b.step(devs, 0, 6 * setups[0].dt)
    with pytest.raises(gpe.GpeError) as e:
        b.step(devs, -2, 0.0)
    assert e.value.code == gpe.ERR_INVALID
    for x, y in zip(devs, before):
        assert np.array_equal(to_host(x), y)
    assert [b.cavity(i) for i in range(len(setups))] == cav
    b.step(devs, 4, 6 * setups[0].dt)
    fresh = gpe.Batch(setups)
    other = [to_dev(x) for x in psi0]
    fresh.step(other, 6, 0.0)
    fresh.step(other, 4, 6 * setups[0].dt)
    for x, y in zip(devs, other):
        assert np.array_equal(to_host(x), to_host(y))
    assert [b.cavity(i) for i in range(len(setups))] == [fresh.cavity(i) for i in range(len(setups))]


def test_adjoint_rejects_fewer_than_one_step():
    torch_cuda()
    from paper_2404_14401_amd import gpe

    s = W.control_512(0, n=64, nknots=8, nsteps=40)
    b = gpe.Batch([s])
    psi = to_dev(start(s, 0))
    for n in (0, -1):
        with pytest.raises(gpe.GpeError) as e:
            gpe.adjoint(b, [psi], [psi], n, s.sx.knots[None, :])
        assert e.value.code == gpe.ERR_INVALID
    loss, grad, _ = gpe.adjoint(b, [psi], [psi], 1, s.sx.knots[None, :])
    assert np.isfinite(loss).all() and np.isfinite(grad).all()
