"""gpe_step_real_noalloc (no plan, static scratch) against gpe_step_real on a fresh plan
of the same description: several calls in a row on one device, each smaller than the
one before, every one equal to the plan path; a repeated call is unaffected by what the
calls before it left in the scratch; the non-finite flag reports a host-injected NaN."""
import numpy as np
import pytest

from paper_2404_14401_amd import workloads as W
from tests.gpu_util import rel_l2, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def cases():
    # the longest lines a plan takes (8192, the largest tables) with the field ODE, along x
    # and along y (whose column step then runs as three passes); multi-pass with the field ODE; multi-pass, non-square, lattice knots, no cavity;
    # whole grid in LDS (real time at 32^2) with the adiabatic field
    rng = np.random.default_rng(5)
    knots = W.Schedule("knots", t0=0.0, t1=0.05, knots=rng.uniform(0.0, 8.0, 40))
    return [
        ("wide_8192x32", W.cavity_scaled(32, seed=2).with_(nx=8192, lx=512.0), 12),
        ("tall_16x8192", W.cavity_scaled(32, seed=4).with_(nx=16, lx=1.0, ny=8192, ly=512.0), 12),
        ("cavity_256", W.cavity_scaled(256, seed=1), 40),
        ("knots_128x64", W.Setup(nx=128, ny=64, lx=16.0, ly=8.0, dt=1e-3, g=150.0, kx_lat=2.0, sx=knots), 30),
        ("adiabatic_32", W.self_organisation_128(8.0, -20.0).with_(nx=32, ny=32, lx=8.0, ly=8.0), 25),
    ]


def run_plan(s, psi0, n):
    from paper_2404_14401_amd import gpe

    d = to_dev(psi0)
    p = gpe.Plan.from_setup(s)
    p.step_real(d, n, 0.0)
    p.sync()
    return to_host(d)


def run_noalloc(s, psi0, n, flag=None):
    from paper_2404_14401_amd import gpe

    d = to_dev(psi0)
    gpe.step_real_noalloc(s, d, n, 0.0, nonfinite=flag)
    return to_host(d)


def test_noalloc_calls_in_a_row_equal_the_plan_path():
    torch = torch_cuda()
    outs = {}
    flag = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    for name, s, n in cases():
        psi0 = W.to_c64(W.random_state(s, seed=3))
        ref = run_plan(s, psi0, n)
        got = run_noalloc(s, psi0, n, flag)
        print(f"{name}: rel-L2 {rel_l2(got, ref):.2e}", flush=True)
        assert rel_l2(got, ref) <= 1e-6, name
        assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref)), name
        assert int(flag.item()) == 0, name
        outs[name] = (s, psi0, n, got)
    # the second case again, after the others: the scratch they left behind changes nothing
    s, psi0, n, first = outs["knots_128x64"]
    again = run_noalloc(s, psi0, n)
    assert np.array_equal(again, first)


def test_noalloc_flags_a_non_finite_input():
    torch = torch_cuda()
    s = W.cavity_scaled(128, seed=0)
    psi0 = W.to_c64(W.random_state(s, seed=1))
    psi0[17, 33] = np.nan
    flag = torch.zeros((1,), dtype=torch.int32, device="cuda")
    run_noalloc(s, psi0, 3, flag)
    assert int(flag.item()) == 1
    # a finite input afterwards clears it
    run_noalloc(s, W.to_c64(W.random_state(s, seed=1)), 3, flag)
    assert int(flag.item()) == 0


def test_noalloc_refuses_bad_arguments():
    torch_cuda()
    from paper_2404_14401_amd import gpe

    s = W.cavity_scaled(128, seed=0)
    d = to_dev(W.to_c64(W.random_state(s, seed=1)))
    with pytest.raises(gpe.GpeError):
        gpe.step_real_noalloc(s, d, -1)
    many = W.Schedule("knots", t0=0.0, t1=1.0, knots=np.ones(257))
    with pytest.raises(gpe.GpeError):
        gpe.step_real_noalloc(s.with_(sx=many, kx_lat=1.0), d, 2)
    with pytest.raises(gpe.GpeError):
        gpe.step_real_noalloc(s.with_(nx=16384), d, 2)
