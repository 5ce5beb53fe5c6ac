"""Failure handling on the GPU path: non-finite detection, argument validation of live
plans, memory cap.  Every condition is forced from the host; no kernel faults."""
import ctypes

import numpy as np
import pytest

from paper_2404_14401_amd import workloads as W
from tests.gpu_util import to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def test_nan_in_psi_is_reported_at_the_next_sync():
    torch_cuda()
    from paper_2404_14401_amd import gpe

    s = W.cavity_scaled(256, 0)
    plan = gpe.Plan.from_setup(s)
    psi = W.to_c64(W.gaussian(s, 1.0))
    psi[10, 10] = np.nan
    d = to_dev(psi)
    plan.step_real(d, 5, 0.0)  # cavity on: the overlap reduction sees the NaN
    with pytest.raises(gpe.GpeError) as e:
        plan.sync()
    assert e.value.code == gpe.ERR_NONFINITE


def test_live_plan_validates_arguments():
    torch = torch_cuda()
    from paper_2404_14401_amd import gpe

    s = W.imag_ground_64(0.0)
    plan = gpe.Plan.from_setup(s)
    d = to_dev(W.gaussian(s, 1.0))
    with pytest.raises(gpe.GpeError) as e:
        plan.step_real(d, -1, 0.0)
    assert e.value.code == gpe.ERR_INVALID
    with pytest.raises(gpe.GpeError):
        plan.step_real(d, 1, float("inf"))
    bad = W.Setup(**{**s.__dict__, "sx": W.Schedule("ramp", 0.0, 1.0, 2.0, 1.0)})
    with pytest.raises(gpe.GpeError):
        plan.set_potential(bad)
    with pytest.raises(ValueError):
        plan.step_real(torch.zeros((64, 64), dtype=torch.complex128, device="cuda"), 1, 0.0)


def test_memory_cap_is_enforced():
    torch_cuda()
    from paper_2404_14401_amd import gpe

    with pytest.raises(gpe.GpeError) as e:
        gpe.Plan(1024, 1024, 64.0, 64.0, 1e-3, 1.0, max_bytes=1 << 20)
    assert e.value.code == gpe.ERR_NOMEM


def test_checkpoint_resume_of_cavity_state_is_bitwise():
    """Stopping after n steps, saving (psi, alpha, Theta history) and resuming in a
    fresh plan reproduces the uninterrupted run exactly."""
    torch_cuda()
    from paper_2404_14401_amd import gpe

    s = W.cavity_scaled(256, 1)
    psi0 = W.to_c64(W.gaussian(s, 1.0))
    a = gpe.Plan.from_setup(s)
    da = to_dev(psi0)
    a.step_real(da, 40, 0.0)
    saved_psi = da.clone()
    cav = a.cavity()
    a.step_real(da, 40, 40 * s.dt)
    b = gpe.Plan.from_setup(s)
    b.set_cavity(cav["alpha"], cav["theta"], cav["theta_prev"], True)
    b.step_real(saved_psi, 40, 40 * s.dt)
    assert (da == saved_psi).all()
    assert b.cavity()["alpha"] == a.cavity()["alpha"]


def test_widened_entry_points_validate_arguments():
    """Argument errors of the Fourier-space stepping, the momentum orders, the cavity
    and probe settings and the adjoint control: reported before anything launches."""
    torch = torch_cuda()
    from paper_2404_14401_amd import gpe

    s = W.imag_ground_64(0.0)
    plan = gpe.Plan.from_setup(s)
    d = to_dev(W.gaussian(s, 1.0))
    for call in (lambda: plan.step_real_k(d, -1, 0.0), lambda: plan.step_real_k(d, 1, float("nan")),
                 lambda: plan.momentum_orders(d, 2, 8, 1), lambda: plan.momentum_orders(d, 0, 0, 1),
                 lambda: plan.momentum_orders(d, 1, 8, 4), lambda: plan.momentum_orders(d, 0, 8, -1)):
        with pytest.raises(gpe.GpeError) as e:
            call()
        assert e.value.code == gpe.ERR_INVALID
    pops, nrm = plan.momentum_orders(d, 0, 8, 3)   # (2*3+1)*8 = 56 <= 64 bins: valid
    assert pops.shape == (7,) and nrm > 0
    adia = W.self_organisation_128(5.0, -10.0).with_(nx=64, ny=64, lx=8.0, ly=8.0)
    for bad in (adia.with_(vc=0.01),                                  # pump < 0, U0 > 0
                adia.with_(n_atoms=-1.0),
                adia.with_(cavity_mode="ode", probe_omega=1.0),        # probe needs the adiabatic field
                adia.with_(probe_detuning=float("inf"))):
        with pytest.raises(gpe.GpeError) as e:
            gpe.Plan.from_setup(bad)
        assert e.value.code == gpe.ERR_INVALID
    knots = np.linspace(0.0, 1.0, 4)
    ctl = s.with_(kx_lat=1.0, sx=W.Schedule("knots", t0=0.0, t1=0.1, knots=knots))
    b = gpe.Batch([ctl])
    with pytest.raises(gpe.GpeError) as e:   # the y lattice has no knots
        gpe.adjoint(b, [d], [d], 10, knots[None, :], control="pump")
    assert e.value.code == gpe.ERR_INVALID


def _nan_state(s, at=(10, 10)):
    psi = W.to_c64(W.gaussian(s, 1.0))
    psi[at] = np.nan
    return psi


@pytest.mark.parametrize("path, n, nsteps", [("multipass", 128, 5), ("multipass", 128, 80), ("lds", 32, 5)])
def test_nan_is_reported_on_paths_that_reduce_nothing(path, n, nsteps, monkeypatch):
    """A plain real-time call without cavity or observables runs no reduction; its kicks
    still flag a non-finite input (multi-pass with and without replayed chunks, and the
    grid kept in LDS), and gpe_sync reports it."""
    torch_cuda()
    from paper_2404_14401_amd import gpe

    monkeypatch.setenv("GPE_PATH", path)
    s = W.Setup(nx=n, ny=n, lx=16.0, ly=16.0, dt=1e-3, g=10.0)
    plan = gpe.Plan.from_setup(s)
    clean = to_dev(W.to_c64(W.gaussian(s, 1.0)))
    plan.step_real(clean, nsteps, 0.0)
    plan.sync()  # a finite state is not flagged
    d = to_dev(_nan_state(s))
    plan.step_real(d, nsteps, 0.0)
    with pytest.raises(gpe.GpeError) as e:
        plan.sync()
    assert e.value.code == gpe.ERR_NONFINITE


def test_nan_is_reported_by_the_fourier_space_ordering_without_observables():
    torch_cuda()
    from paper_2404_14401_amd import gpe

    s = W.Setup(nx=128, ny=64, lx=16.0, ly=8.0, dt=1e-3, g=10.0)
    plan = gpe.Plan.from_setup(s)
    d = to_dev(_nan_state(s, (3, 70)))
    plan.step_real_k(d, 4, 0.0)
    with pytest.raises(gpe.GpeError) as e:
        plan.sync()
    assert e.value.code == gpe.ERR_NONFINITE


def test_norm_and_energy_report_a_nonfinite_input():
    torch_cuda()
    from paper_2404_14401_amd import gpe

    s = W.Setup(nx=64, ny=64, lx=16.0, ly=16.0, dt=1e-3, g=10.0)
    plan = gpe.Plan.from_setup(s)
    d = to_dev(_nan_state(s))
    for call in (lambda: plan.norm(d), lambda: plan.energy(d)):
        with pytest.raises(gpe.GpeError) as e:
            call()
        assert e.value.code == gpe.ERR_NONFINITE
    inf = W.to_c64(W.gaussian(s, 1.0))
    inf[5, 7] = np.inf
    with pytest.raises(gpe.GpeError) as e:
        plan.norm(to_dev(inf))
    assert e.value.code == gpe.ERR_NONFINITE


@pytest.mark.parametrize("bad", [1, 2])
def test_nan_in_a_cavity_free_batch_member_is_reported(bad):
    """A cavity-free batch reduces nothing; a member's non-finite state is still flagged,
    by the batched kick passes (256^2, multi-pass) or at the end of the call (64^2, in
    LDS), and gpe_batch_sync names the first bad member."""
    torch_cuda()
    from paper_2404_14401_amd import gpe

    setups = [W.Setup(nx=256, ny=256, lx=32.0, ly=32.0, dt=5e-4, g=100.0),
              W.Setup(nx=256, ny=256, lx=32.0, ly=32.0, dt=5e-4, g=200.0),
              W.Setup(nx=64, ny=64, lx=8.0, ly=8.0, dt=5e-4, g=50.0)]
    b = gpe.Batch(setups)
    lds = {(g["nx"], g["ny"]): g["lds"] for g in b.groups()}
    assert not lds[(256, 256)] and lds[(64, 64)]
    psis = [to_dev(W.to_c64(W.gaussian(s, 1.0))) for s in setups]
    b.step(psis, 60, 0.0)
    b.sync()  # finite members are not flagged
    member = 1 if bad == 1 else 2
    psis[member] = to_dev(_nan_state(setups[member], (7, 9)))
    b.step(psis, 60, 0.0)
    with pytest.raises(gpe.GpeError) as e:
        b.sync()
    assert e.value.code == gpe.ERR_NONFINITE and e.value.member == member
    with pytest.raises(gpe.GpeError):
        b.cavity(member)
    b.cavity(0)  # the other members' state is readable
