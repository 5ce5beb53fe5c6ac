"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar (per workload, after its step count): relative L2 error of psi <= 1e-4 and
relative energy error <= 1e-5; pass-level checks are tighter.  Both the LDS-resident
path (small grids) and the multi-pass path (any grid; forced with GPE_PATH) are run.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2404_14401_amd import workloads as W
from tests.bridge import problem, state
from tests.gpu_util import rel_l2, rel_l2_phase_aligned, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu

TOL_L2 = 1e-4
TOL_E = 1e-5


def make_plan(setup, path, monkeypatch):
    torch_cuda()
    from paper_2404_14401_amd import gpe

    monkeypatch.setenv("GPE_PATH", path)
    return gpe.Plan.from_setup(setup)


def rel_e(a, b):
    return abs(a - b) / abs(b)


# ------------------------------------------------------------ pass level

@pytest.mark.parametrize("path", ["lds", "multipass"])
@pytest.mark.parametrize("shape", [(64, 64), (128, 32), (32, 128), (16, 16)])
def test_free_flow_single_steps_match_spectral_propagation(path, shape, monkeypatch):
    """V = g = 0: a step is exactly the kinetic factor; checks FFT signs, k ordering,
    scaling and the transposed axes on non-square grids."""
    nx, ny = shape
    s = W.Setup(nx=nx, ny=ny, lx=nx * 0.2, ly=ny * 0.15, dt=0.01, g=0.0, wx=0.0, wy=0.0)
    psi0 = W.to_c64(W.gaussian(s, 0.8, 0.3, -0.2) * np.exp(1j * 0.7 * s.xs()[None, :]))
    ref, _ = O.step_real(problem(s), state(s), psi0, 3)
    plan = make_plan(s, path, monkeypatch)
    d = to_dev(psi0)
    plan.step_real(d, 3, 0.0)
    assert rel_l2(to_host(d), ref) < 2e-6


@pytest.mark.parametrize("shape", [(4096, 16), (16, 4096), (2048, 64)])
def test_free_flow_extreme_aspect_ratios(shape, monkeypatch):
    """The largest line lengths the plan takes (4096) in either pass, against the
    oracle's spectral propagation."""
    nx, ny = shape
    s = W.Setup(nx=nx, ny=ny, lx=nx * 0.05, ly=ny * 0.15, dt=0.01, g=0.0, wx=0.0, wy=0.0)
    psi0 = W.to_c64(W.gaussian(s, 0.8, 0.3, -0.2) * np.exp(1j * 0.7 * s.xs()[None, :]))
    ref, _ = O.step_real(problem(s), state(s), psi0, 3)
    plan = make_plan(s, "multipass", monkeypatch)
    d = to_dev(psi0)
    plan.step_real(d, 3, 0.0)
    assert rel_l2(to_host(d), ref) < 2e-6


@pytest.mark.parametrize("fold", ["fold", "tail"])
def test_imag_fold_at_2048_row_work_groups(fold, monkeypatch):
    """Imaginary time on 1024 x 2048 (2048 row work-groups of one line): with the tail between
    steps left out (every entry work-group sums the 2048 exit norm partials itself) and with
    the tail kernel, against the oracle pointwise on white noise in a trap and lattice."""
    monkeypatch.setenv("GPE_FOLD_ROWS", "2048" if fold == "fold" else "1024")
    s = W.Setup(nx=1024, ny=2048, lx=64.0, ly=128.0, dt=0.002, g=300.0, wx=0.08, wy=0.05,
                kx_lat=1.0, sx=W.Schedule("const", 2.0))
    psi0 = W.random_state(s, 31)
    ref, _ = O.step_imag(problem(s), state(s), psi0, 4)
    plan = make_plan(s, "multipass", monkeypatch)
    d = to_dev(psi0)
    plan.step_imag(d, 4, 0.0)
    _assert_pointwise(to_host(d), ref)
    assert abs(plan.norm(d) - 1.0) < 1e-6

def test_largest_grid_steps_with_every_potential_term(monkeypatch):
    """4096^2, the plan's largest grid: two real steps and one imaginary step with the
    trap, both lattices, g and the cavity field ODE, against the oracle."""
    s = W.Setup(nx=4096, ny=4096, lx=64.0, ly=64.0, dt=0.002, g=200.0, wx=0.1, wy=0.12, x0=0.5,
                kx_lat=1.1, ky_lat=0.9, sx=W.Schedule("ramp", 0.0, 4.0, 0.0, 0.01), sy=W.Schedule("const", 1.0),
                cavity=True, vc=1.0, kc=0.9, delta_c=-5.0, kappa=2.0, eta=2.0, alpha0=0.1 + 0.05j)
    psi0 = W.to_c64(W.gaussian(s, 6.0, 0.5, -0.3) * np.exp(1j * 0.2 * s.ys()[:, None]))
    for mode, n in (("real", 2), ("imag", 1)):
        st = state(s)
        fn = O.step_real if mode == "real" else O.step_imag
        ref, _ = fn(problem(s), st, psi0, n)
        plan = make_plan(s, "multipass", monkeypatch)
        d = to_dev(psi0)
        (plan.step_real if mode == "real" else plan.step_imag)(d, n, 0.0)
        assert rel_l2(to_host(d), ref) < 2e-6, mode
        if mode == "real":
            assert abs(plan.cavity()["alpha"] - st.alpha) < 1e-7


@pytest.mark.parametrize("path", ["lds", "multipass"])
def test_one_step_with_every_potential_term(path, monkeypatch):
    """Trap (displaced, anisotropic), both lattices (ramp and const), cavity terms
    with a non-zero field: one real and one imaginary step."""
    s = W.Setup(nx=64, ny=32, lx=12.0, ly=8.0, dt=0.02, g=30.0, wx=1.1, wy=0.8, x0=0.3, y0=-0.2,
                kx_lat=1.3, ky_lat=2.1, sx=W.Schedule("ramp", 1.0, 3.0, 0.0, 0.1),
                sy=W.Schedule("const", 2.0), cavity=True, vc=1.5, kc=1.7, delta_c=-4.0, kappa=2.0,
                eta=3.0, alpha0=0.4 - 0.3j)
    psi0 = W.random_state(s, 11)
    for mode in ("real", "imag"):
        st = state(s, 0.05)
        if mode == "real":
            ref, _ = O.step_real(problem(s), st, psi0, 2)
        else:
            ref, _ = O.step_imag(problem(s), st, psi0, 2)
        plan = make_plan(s, path, monkeypatch)
        d = to_dev(psi0)
        (plan.step_real if mode == "real" else plan.step_imag)(d, 2, 0.05)
        assert rel_l2(to_host(d), ref) < 2e-6, mode
        if mode == "real":
            assert abs(plan.cavity()["alpha"] - st.alpha) < 1e-9


@pytest.mark.parametrize("path", ["lds", "multipass"])
def test_energy_and_norm_functionals(path, monkeypatch):
    s = W.Setup(nx=128, ny=64, lx=16.0, ly=10.0, dt=0.01, g=50.0, kx_lat=1.0, sx=W.Schedule("const", 2.0))
    psi0 = W.random_state(s, 5)
    plan = make_plan(s, path, monkeypatch)
    d = to_dev(psi0)
    e = plan.energy(d, 0.0)
    ref = O.energy(problem(s), psi0)
    for k in ("ekin", "epot", "eint", "e", "mu", "norm"):
        assert rel_e(e[k], ref[k]) < 1e-9, k
    assert rel_e(plan.norm(d), O.norm(problem(s), psi0)) < 1e-12


@pytest.mark.parametrize("path", ["lds", "multipass"])
def test_energy_inside_a_ramp_is_taken_at_the_given_time(path, monkeypatch):
    """Energy with a lattice that is still ramping: V must be evaluated at t itself."""
    s = W.Setup(nx=64, ny=64, lx=12.0, ly=12.0, dt=0.01, g=40.0, kx_lat=1.5, sx=W.Schedule("ramp", 0.0, 30.0, 0.0, 1.0))
    psi0 = W.random_state(s, 9)
    plan = make_plan(s, path, monkeypatch)
    d = to_dev(psi0)
    for t in (0.0, 0.37, 0.8):
        assert rel_e(plan.energy(d, t)["e"], O.energy(problem(s), psi0, t)["e"]) < 1e-9, t


def _assert_pointwise(out, ref, l2=2e-6, amax=1e-5):
    """rel-L2 and the largest pointwise error against the largest value: an indexing
    slip in one tile or row shows in the second even where the first averages it away."""
    assert rel_l2(out, ref) < l2
    err = np.abs(out - ref)
    assert err.max() <= amax * np.abs(ref).max(), (np.unravel_index(err.argmax(), err.shape), err.max())


@pytest.mark.parametrize("shape", [(1024, 1024), (2048, 512), (512, 2048)])
@pytest.mark.parametrize("mode", ["real", "imag"])
def test_full_spectrum_states_on_the_headline_launch_shapes(shape, mode, monkeypatch):
    """White-noise states (every kx, ky mode and every row and column populated,
    box-edge points included) through the headline launch shapes: one line per row
    work-group, narrow column tiles in the XCD-aware order, the merged real-time kick
    of the middle row passes and the field ODE with a non-zero field (1024^2 runs the
    cavity workload's physics at alpha0 = 0.3 - 0.2i).  Three real or two imaginary
    steps against the oracle, pointwise."""
    nx, ny = shape
    if shape == (1024, 1024):
        s = W.cavity_1024(2).with_(alpha0=0.3 - 0.2j)
    else:
        s = W.Setup(nx=nx, ny=ny, lx=nx / 16.0, ly=ny / 16.0, dt=2e-4, g=800.0, wx=0.05, wy=0.07, x0=0.7,
                    kx_lat=1.0, ky_lat=2.0, sx=W.Schedule("ramp", 0.0, 3.0, 0.0, 1e-3), sy=W.Schedule("const", 1.5),
                    cavity=True, vc=1.5, kc=1.0, delta_c=-20.0, kappa=10.0, eta=4.0, alpha0=0.2 + 0.1j)
    psi0 = W.random_state(s, 31)
    n = 3 if mode == "real" else 2
    st = state(s)
    ref, _ = (O.step_real if mode == "real" else O.step_imag)(problem(s), st, psi0, n)
    plan = make_plan(s, "multipass", monkeypatch)
    d = to_dev(psi0)
    (plan.step_real if mode == "real" else plan.step_imag)(d, n, 0.0)
    _assert_pointwise(to_host(d), ref)
    if mode == "real":
        assert abs(plan.cavity()["alpha"] - st.alpha) <= 1e-6 * abs(st.alpha)


@pytest.mark.parametrize("shape", [(8192, 64), (64, 8192), (8192, 512)])
@pytest.mark.parametrize("mode", ["real", "imag"])
def test_8192_point_lines(shape, mode, monkeypatch):
    """Lines of 8192 points, the longest a plan takes: row passes at radix 16 (512 threads
    per line), the column step in three passes (the single pass, one column per tile, in
    test_long_columns_in_three_passes).  White-noise states with
    the field ODE and every potential term, three real or two imaginary steps against the
    oracle, pointwise; the energy functional on the same grid."""
    nx, ny = shape
    s = W.Setup(nx=nx, ny=ny, lx=nx / 16.0, ly=ny / 16.0, dt=2e-4, g=800.0, wx=0.05, wy=0.07, x0=0.7,
                kx_lat=1.0, ky_lat=2.0, sx=W.Schedule("ramp", 0.0, 3.0, 0.0, 1e-3), sy=W.Schedule("const", 1.5),
                cavity=True, vc=1.5, kc=1.0, delta_c=-20.0, kappa=10.0, eta=4.0, alpha0=0.2 + 0.1j)
    psi0 = W.random_state(s, 17)
    n = 3 if mode == "real" else 2
    st = state(s)
    ref, _ = (O.step_real if mode == "real" else O.step_imag)(problem(s), st, psi0, n)
    plan = make_plan(s, "multipass", monkeypatch)
    d = to_dev(psi0)
    (plan.step_real if mode == "real" else plan.step_imag)(d, n, 0.0)
    out = to_host(d)
    _assert_pointwise(out, ref)
    if mode == "real":
        assert abs(plan.cavity()["alpha"] - st.alpha) <= 1e-6 * abs(st.alpha)
    else:
        assert rel_e(plan.energy(d, 0.0)["e"], O.energy(problem(s), ref, 0.0, st.alpha)["e"]) < 1e-7


@pytest.mark.parametrize("shape", [(64, 8192), (16, 4096), (512, 4096)])
@pytest.mark.parametrize("mode", ["real", "imag"])
@pytest.mark.parametrize("split", ["three", "one"])
def test_long_columns_in_three_passes(shape, mode, split, monkeypatch):
    """The column step on 4096- and 8192-point columns as three passes (128-point transforms
    of rows strided by ny/128 with the cross twiddles; (ny/128)-point transforms of contiguous
    rows with the kinetic factor and back; the inverse 128-point transforms) and as the
    single pass, on white noise with the field ODE (its tail rides on the first of the three
    passes), against the oracle pointwise."""
    monkeypatch.setenv("GPE_COL_SPLIT_MIN", "4096" if split == "three" else str(1 << 30))
    nx, ny = shape
    s = W.Setup(nx=nx, ny=ny, lx=nx / 16.0, ly=ny / 16.0, dt=2e-4, g=800.0, wx=0.05, wy=0.07, y0=0.4,
                kx_lat=1.0, ky_lat=2.0, sx=W.Schedule("const", 2.0), sy=W.Schedule("ramp", 0.0, 3.0, 0.0, 1e-3),
                cavity=True, vc=1.5, kc=1.0, delta_c=-20.0, kappa=10.0, eta=4.0, alpha0=0.1 - 0.2j)
    psi0 = W.random_state(s, 23)
    n = 3 if mode == "real" else 2
    st = state(s)
    ref, _ = (O.step_real if mode == "real" else O.step_imag)(problem(s), st, psi0, n)
    plan = make_plan(s, "multipass", monkeypatch)
    d = to_dev(psi0)
    (plan.step_real if mode == "real" else plan.step_imag)(d, n, 0.0)
    _assert_pointwise(to_host(d), ref)
    if mode == "real":
        assert abs(plan.cavity()["alpha"] - st.alpha) <= 1e-6 * abs(st.alpha)

def test_8192_squared_three_pass_columns_match_the_single_pass(monkeypatch):
    """The largest grid, 8192^2, with every potential term and white noise: two real and two
    imaginary steps with the column step in three passes and in one (the one-pass column
    step is checked against the oracle at smaller sizes; the oracle takes minutes here).
    The two agree to their rounding, and real time keeps the norm."""
    import torch

    from paper_2404_14401_amd import gpe

    s = W.Setup(nx=8192, ny=8192, lx=512.0, ly=512.0, dt=2e-4, g=800.0, wx=0.01, wy=0.012, x0=0.7,
                kx_lat=1.0, ky_lat=2.0, sx=W.Schedule("ramp", 0.0, 3.0, 0.0, 1e-3), sy=W.Schedule("const", 1.5))
    rng = np.random.Generator(np.random.PCG64(41))
    z = torch.from_numpy((rng.standard_normal((8192, 8192), dtype=np.float32)
                          + 1j * rng.standard_normal((8192, 8192), dtype=np.float32)).astype(np.complex64))
    torch_cuda()
    psi0 = z.to("cuda")
    psi0 /= torch.sqrt(torch.sum(torch.abs(psi0) ** 2) * (s.lx / s.nx) * (s.ly / s.ny))
    out = {}
    for split in ("three", "one"):
        monkeypatch.setenv("GPE_COL_SPLIT_MIN", "4096" if split == "three" else str(1 << 30))
        monkeypatch.setenv("GPE_PATH", "multipass")
        p = gpe.Plan.from_setup(s)
        r = psi0.clone()
        p.step_real(r, 2, 0.0)
        i = psi0.clone()
        p.step_imag(i, 2, 0.0)
        out[split] = (r, i, p.norm(r))
        p.close()
    for k in (0, 1):
        a, b = out["three"][k], out["one"][k]
        assert float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) < 1e-6, k
    assert abs(out["three"][2] - 1.0) < 1e-5 and abs(out["one"][2] - 1.0) < 1e-5

# ----------------------------------------------- imaginary-time ground state

@pytest.mark.parametrize("path", ["lds", "multipass"])
@pytest.mark.parametrize("g", [0.0, 100.0])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_imag_ground_state_64(path, g, seed, monkeypatch):
    """64x64 on [-8,8)^2, dtau = 1e-3, 2000 steps, seed-perturbed Gaussian (seeds 0-2)."""
    s = W.imag_ground_64(g)
    psi0 = W.noisy_gaussian(s, seed)
    ref, robs = O.step_imag(problem(s), state(s), psi0, W.IMAG_64_STEPS, want_obs=True)
    plan = make_plan(s, path, monkeypatch)
    import torch

    d = to_dev(psi0)
    obs = torch.zeros((W.IMAG_64_STEPS, 6), dtype=torch.float64, device="cuda")
    plan.step_imag(d, W.IMAG_64_STEPS, 0.0, obs)
    out = to_host(d)
    assert rel_l2(out, ref) < TOL_L2
    assert rel_e(plan.energy(d)["e"], O.energy(problem(s), ref)["e"]) < TOL_E
    o = obs.cpu().numpy()
    assert np.abs(o[:, 0] - robs[:, 0]).max() < 3e-7  # pre-normalisation norms (c64 state)
    assert abs(plan.norm(d) - 1.0) < 1e-6


@pytest.mark.parametrize("shape", [(256, 64), (64, 512)])
@pytest.mark.parametrize("cavity", ["off", "adiabatic"])
def test_imag_on_wide_and_tall_grids_with_replayed_chunks(shape, cavity, monkeypatch):
    """Imaginary time on non-square multi-pass grids (dx = 1/8, anisotropic trap, both
    lattices) for 400 steps without per-step records, so that the plan replays captured
    chunks with the pending renormalisation carried between them; with the adiabatic
    field, alpha follows the state."""
    nx, ny = shape
    s = W.Setup(nx=nx, ny=ny, lx=nx / 8.0, ly=ny / 8.0, dt=2e-3, g=200.0, wx=0.15, wy=0.2, x0=0.4,
                kx_lat=1.0, ky_lat=1.5, sx=W.Schedule("const", 1.0), sy=W.Schedule("const", -2.0))
    if cavity == "adiabatic":
        s = s.with_(cavity=True, cavity_mode="adiabatic", vc=-0.2, kc=1.5, delta_c=-6.0, kappa=3.0, n_atoms=50.0)
    psi0 = W.noisy_gaussian(s, 2)
    n = 400
    st = state(s)
    ref, _ = O.step_imag(problem(s), st, psi0, n)
    plan = make_plan(s, "multipass", monkeypatch)
    d = to_dev(psi0)
    plan.step_imag(d, n, 0.0)
    assert rel_l2(to_host(d), ref) < TOL_L2
    assert rel_e(plan.energy(d)["e"], O.energy(problem(s), ref, 0.0, st.alpha)["e"]) < TOL_E
    assert abs(plan.norm(d) - 1.0) < 1e-6
    if cavity == "adiabatic":
        a = plan.cavity()["alpha"]
        assert abs(a - st.alpha) <= 1e-4 * abs(st.alpha) and abs(st.alpha) > 1e-3


# --------------------------------------------------------------- real time

@pytest.mark.parametrize("path", ["lds", "multipass"])
def test_real_time_ramp_and_displaced_trap(path, monkeypatch):
    s0 = W.Setup(nx=64, ny=64, lx=16.0, ly=16.0, dt=0.01, g=100.0)
    gs, _ = O.step_imag(problem(s0), state(s0), W.gaussian(s0, 1.5), 1500)
    psi0 = W.to_c64(gs)
    s = s0.with_(dt=1e-3, y0=0.5, kx_lat=2.0, sx=W.Schedule("ramp", 0.0, 5.0, 0.0, 1.0))
    nsteps = 2000
    ref, robs = O.step_real(problem(s), state(s), psi0, nsteps, want_obs=True)
    plan = make_plan(s, path, monkeypatch)
    import torch

    d = to_dev(psi0)
    obs = torch.zeros((nsteps, 6), dtype=torch.float64, device="cuda")
    plan.step_real(d, nsteps, 0.0, obs)
    out = to_host(d)
    assert rel_l2(out, ref) < TOL_L2
    t = nsteps * s.dt
    assert rel_e(plan.energy(d, t)["e"], O.energy(problem(s), ref, t)["e"]) < TOL_E
    o = obs.cpu().numpy()
    assert np.abs(o[:, 0] - robs[:, 0]).max() < 1e-5       # norm
    assert np.abs(o[:, 5] - robs[:, 5]).max() < 1e-5       # <y> dipole
    assert np.abs(o[:, 4] - robs[:, 4]).max() < 1e-5       # <x>


@pytest.mark.parametrize("path", ["lds", "multipass"])
def test_calls_compose(path, monkeypatch):
    """Two calls of n steps equal one call of 2n steps (time and cavity history carried)."""
    s = W.cavity_scaled(64, 1)
    psi0 = W.to_c64(W.gaussian(s, 1.0))
    plan = make_plan(s, path, monkeypatch)
    a = to_dev(psi0)
    plan.step_real(a, 300, 0.0)
    plan.step_real(a, 300, 300 * s.dt)
    al1 = plan.cavity()["alpha"]
    plan2 = make_plan(s, path, monkeypatch)
    b = to_dev(psi0)
    plan2.step_real(b, 600, 0.0)
    al2 = plan2.cavity()["alpha"]
    # the split call adds one real-space round trip (one more complex64 rounding)
    assert rel_l2(to_host(a), to_host(b)) < 1e-5
    assert abs(al1 - al2) < 1e-6 * max(1.0, abs(al2))


# ----------------------------------------------------------------- cavity

@pytest.mark.parametrize("path", ["lds", "multipass"])
@pytest.mark.parametrize("seed", [0, 3])
def test_cavity_self_consistent_128(path, seed, monkeypatch):
    """Cavity workload physics (dx = 1/16, Vp = Vc = 3, k = 1, Delta_c = -20,
    kappa = 10, eta from the seed) on a 128^2 box: psi and the field alpha."""
    s = W.cavity_scaled(128, seed)
    psi0 = W.to_c64(W.thomas_fermi_guess(s.with_(wx=0.4, wy=0.4), np.sqrt(s.g / np.pi) * 0.4))
    nsteps = 2000
    st = state(s)
    ref, robs = O.step_real(problem(s), st, psi0, nsteps, want_obs=True)
    plan = make_plan(s, path, monkeypatch)
    import torch

    d = to_dev(psi0)
    obs = torch.zeros((nsteps, 6), dtype=torch.float64, device="cuda")
    plan.step_real(d, nsteps, 0.0, obs)
    out = to_host(d)
    assert rel_l2(out, ref) < TOL_L2
    o = obs.cpu().numpy()
    aref = robs[:, 2] + 1j * robs[:, 3]
    agpu = o[:, 2] + 1j * o[:, 3]
    assert np.abs(agpu - aref).max() <= 1e-4 * max(np.abs(aref).max(), 1e-3)
    assert np.abs(o[:, 1] - robs[:, 1]).max() < 1e-6  # Theta
    t = nsteps * s.dt
    assert rel_e(plan.energy(d, t)["e"], O.energy(problem(s), ref, t, st.alpha)["e"]) < TOL_E
