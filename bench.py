#!/usr/bin/env python3
"""Throughput of the split-step GPE hot path on one MI355X.

Workload: the self-consistent cavity run -- 1024x1024 grid on [-32, 32)^2, complex64
state in HBM, harmonic trap w = 0.05, g = 1000, pump lattice Vp cos^2(y) with Vp = 3,
cavity lattice Vc = 3, k = 1, Delta_c = -20, kappa = 10, eta from seed 0, dt = 2e-4.
One step = one full symmetric split step (half kick, FFT2, kinetic factor, IFFT2,
half kick; Sec. 3.1) with the fused overlap reduction Theta and the cavity-field update.
The state is synthetic (a Thomas-Fermi-shaped start), already resident on the GPU.

Prints ONE JSON line: grid-point-steps/s, the roofline of the dominant kernel (HIP
events around sampled launches inside the timed region), and the FP64 oracle timed on
a bounded sample on the host cores (all threads and one).  Further legs, each
skippable: the 208-member batched sweep, the control adjoint (three ways of getting the
forward states back), the widened rows (Fourier-space ordering, Kapitza-Dirac,
adiabatic field, self-organisation sweep), the paper-shaped imaginary-time grid sweep
64^2..4096^2, a 64 x 1024^2 batch whose state does not fit the Infinity Cache, the
device-copy bandwidth, and the same step written with torch.fft (complex64 and
complex128) as a side comparison.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
METRIC = "grid-point-steps/s (1024^2 c64) & %HBM roofline; batched + adjoint vs plain"
HBM_PEAK_GBS = 8000.0
B_PASS = 16  # algorithmic bytes per point per pass: one complex64 read + one write


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("kernels.h", "kernels_plan.hip", "fft_engine.h", "physics.h", "gpe_internal.h"):
        with open(os.path.join(HERE, "paper_2404_14401_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_KERNELS = {"column_pass": "col_pass<1024, 0>", "row_pass_mid": "row_pass<1024, 1, false>"}


def traffic_from(root: str, copy_mib: int = 64) -> dict:
    """HBM bytes per launch of the two cavity-step passes from four rocprofv3 counter runs
    under root (fetch/, write/: FETCH_SIZE and WRITE_SIZE of the bench; copy_fetch/,
    copy_write/: the same counters of --copy-calibration copy_mib), each counter scaled so
    that the copy of known size reads right."""
    import csv
    import glob

    def load(name):
        path = glob.glob(os.path.join(root, name, "**", "*counter_collection.csv"), recursive=True)[0]
        vals = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals

    def mean_kib(vals, pattern):
        v = [x for k, xs in vals.items() if pattern in k for x in xs]
        if not v:
            raise ValueError(f"no launches of {pattern} under {root}")
        return sum(v) / len(v), len(v)

    copy_bytes = copy_mib << 20
    scale_f = copy_bytes / (1024 * mean_kib(load("copy_fetch"), "copyBuffer")[0])
    scale_w = copy_bytes / (1024 * mean_kib(load("copy_write"), "copyBuffer")[0])
    fe, wr = load("fetch"), load("write")
    out = {"source_sha": kernel_source_sha(),
           "calibration": {"fetch_scale": scale_f, "write_scale": scale_w, "copy_bytes": copy_bytes}, "kernels": {}}
    for key, pat in TRAFFIC_KERNELS.items():
        (f, n), (w, _) = mean_kib(fe, pat), mean_kib(wr, pat)
        fb, wb = 1024 * scale_f * f, 1024 * scale_w * w
        out["kernels"][key] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb, "launches": n}
    return out


def load_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they were
    taken on the current kernel sources."""
    path = os.path.join(HERE, "profiles", "traffic_cavity_1024.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha") != kernel_source_sha():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(setup, psi0, budget_s: float, one_core_s: float, sweep_steps: int = 0, sweep_max_n: int = 0,
                 sweep_per_run: int = 1000):
    """The oracle on all the host's threads (budget_s of work), and on one thread
    (one_core_s of work, 0: skip); and its time for the grid sweep's workload at
    2^6 .. 2^sweep_max_n from sweep_steps-step samples scaled to sweep_per_run steps."""
    sys.path.insert(0, HERE)
    from oracle import oracle as O
    from tests.bridge import problem, state

    def timed(threads, budget):
        cores = O.set_threads(threads)
        prob, st = problem(setup), state(setup)
        t = time.perf_counter()
        psi, _ = O.step_real(prob, st, psi0, 1)
        one = time.perf_counter() - t
        n = max(2, int(budget / max(one, 1e-6)))
        t = time.perf_counter()
        O.step_real(prob, st, psi, n)
        return cores, n, setup.nx * setup.ny * n / (time.perf_counter() - t)

    all_threads = O.set_threads(0)
    cores, n, value = timed(all_threads, budget_s)
    out = {
        "value": value,
        "unit": "grid-point-steps/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{n} real-time cavity steps at {setup.nx}x{setup.ny}, FP64 C oracle "
                  f"(own radix-2 FFT, OpenMP over rows/columns), after 1 untimed step",
        "host": {"nproc": os.cpu_count(), "model": _cpu_model()},
    }
    if one_core_s > 0:
        c1, n1, v1 = timed(1, one_core_s)
        out["one_core"] = {"value": v1, "cores": c1, "sample": f"{n1} steps, same workload"}
        O.set_threads(all_threads)
    if sweep_steps > 0:
        from paper_2404_14401_amd import workloads as W

        rows = []
        for n in range(6, sweep_max_n + 1):
            s = sweep_setup(n)
            t0 = time.perf_counter()
            O.step_imag(problem(s), state(s), W.gaussian(s, 1.5), sweep_steps)
            rows.append({"n": n, "ms_per_run": 1e3 * (time.perf_counter() - t0) * sweep_per_run / sweep_steps})
        out["grid_sweep"] = {"sample": f"{sweep_steps} imaginary-time steps per grid scaled to {sweep_per_run}, "
                                       f"all host threads", "rows": rows}
    return out


def bench_batched(steps: int, tune_cache: str | None):
    """The 208-member mixed-size sweep (128 x 128^2, 64 x 256^2, 16 x 512^2, dx = 0.125,
    lattice depth and g from seed 0): one batched call vs looping the plain solver."""
    import numpy as np
    import torch

    from paper_2404_14401_amd import gpe
    from paper_2404_14401_amd import workloads as W

    setups = W.sweep_208(0)
    psis = [torch.from_numpy(W.to_c64(W.gaussian(s, 1.0))).to("cuda") for s in setups]
    pts = sum(s.nx * s.ny for s in setups)
    b = gpe.Batch(setups)
    t = time.perf_counter()
    b.tune(tune_cache)
    tune_s = time.perf_counter() - t
    b.step(psis, 60, 0.0)  # warm-up: kernels loaded, step graph captured
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    b.step(psis, steps, 0.0)
    ev1.record()
    torch.cuda.synchronize()
    t_b = ev0.elapsed_time(ev1) / 1e3
    plans = [gpe.Plan.from_setup(s) for s in setups]
    for p, x in zip(plans, psis):
        p.step_real(x, 2, 0.0)
    torch.cuda.synchronize()
    ev0.record()
    for p, x in zip(plans, psis):
        p.step_real(x, steps, 0.0)
    ev1.record()
    torch.cuda.synchronize()
    t_p = ev0.elapsed_time(ev1) / 1e3
    return {
        "workload": "208 real-time condensates (128 x 128^2, 64 x 256^2, 16 x 512^2), trap + 2D lattice, "
                    "per-member depth U[0,20] and g U[50,1000] from seed 0, dt=5e-4, c64 state",
        "steps": steps,
        "value": pts * steps / t_b,
        "unit": "grid-point-steps/s",
        "plain_loop_value": pts * steps / t_p,
        "speedup_vs_plain_loop": t_p / t_b,
        "groups": b.groups(),
        "tune_s": tune_s,
    }


def bench_adjoint(steps: int, nb: int, tune_cache: str | None = None):
    """Optimal-control gradient: nb members at 512^2, `steps` real-time steps, lattice
    depth over 200 knots from PCG64(member), g = 300; loss = 1 - |<target|psi(T)>|^2 with
    the target the ground state at V0 = 15.  Forward alone vs forward + reverse, in each
    way of getting the forward states back: reconstruction, segment restarts, and the
    stored trajectory (every kick's output kept in HBM; its first call also allocates it,
    later calls reuse it, as an optimiser's repeated gradients would)."""
    import numpy as np
    import torch

    from paper_2404_14401_amd import gpe
    from paper_2404_14401_amd import workloads as W

    setups = [W.control_512(b, nsteps=steps) for b in range(nb)]
    s0 = setups[0]
    # ground states on the GPU (imaginary time): psi(0) at V0 = 0, target at V0 = 15
    gs = s0.with_(dt=0.01, sx=W.Schedule("const", 0.0))
    tg = s0.with_(dt=0.01, sx=W.Schedule("const", 15.0))
    states = []
    for s in (gs, tg):
        p = gpe.Plan.from_setup(s)
        x = torch.from_numpy(W.to_c64(W.gaussian(s, 1.5))).to("cuda")
        p.step_imag(x, 800, 0.0)
        states.append(x)
    psi0 = [states[0].clone() for _ in range(nb)]
    tgts = [states[1] for _ in range(nb)]
    knots = np.stack([s.sx.knots for s in setups])
    b = gpe.Batch(setups)
    b.tune(tune_cache)  # the forward it is compared with runs its tuned shapes
    gpe.adjoint(b, psi0, tgts, 20, knots[:, :], mode="reconstruct")  # warm-up
    work = [x.clone() for x in psi0]
    torch.cuda.synchronize()
    t = time.perf_counter()
    b.step(work, steps, 0.0)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t
    out = {"workload": f"{nb} x 512^2 real-time control problems, {steps} steps, dt=5e-4, 200 knots, g=300",
           "steps": steps, "forward_s": t_fwd}
    def run(bb, mode, fwd, kn, **kw):
        torch.cuda.synchronize()
        t = time.perf_counter()
        loss, grad, info = gpe.adjoint(bb, psi0, tgts, steps, kn, mode=mode, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        return {"forward_plus_reverse_s": dt, "ratio_to_forward": dt / fwd, "drift": info["drift"],
                "workspace_bytes": info["workspace_bytes"], "mean_loss": float(np.mean(loss)),
                "grad_norm": float(np.linalg.norm(grad)), "grad": grad}

    ref = None
    for mode in ("reconstruct", "checkpoint", "store"):
        try:
            # the first call of a mode sizes its workspace (checkpoint slots, the trajectory),
            # which later calls reuse: the figure is the second call, the first reported beside it
            first = run(b, mode, t_fwd, knots)
            out[mode] = run(b, mode, t_fwd, knots) if mode in ("checkpoint", "store") else first
        except gpe.GpeError as e:  # the stored trajectory may not fit the device
            out[mode] = {"error": str(e)}
            continue
        if mode in ("checkpoint", "store"):
            out[mode]["first_call_s"] = first["forward_plus_reverse_s"]
        g = out[mode].pop("grad")
        if ref is None:
            ref = g
        else:
            out[mode]["grad_rel_diff_vs_reconstruct"] = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
    b.close()
    # pump-amplitude control through the adiabatic cavity field (probe passes in both sweeps)
    ca = [W.control_512(b, nsteps=steps).with_(
        kx_lat=0.0, sx=W.Schedule("const", 0.0), ky_lat=2.0, cavity=True, cavity_mode="adiabatic", vc=-0.05, kc=2.0,
        delta_c=-8.0, kappa=4.0, n_atoms=200.0,
        sy=W.Schedule("knots", t0=0.0, t1=steps * setups[0].dt, knots=-3.0 - setups[b].sx.knots)) for b in range(nb)]
    kc = np.stack([s.sy.knots for s in ca])
    bc = gpe.Batch(ca)
    bc.tune(tune_cache)
    gpe.adjoint(bc, psi0, tgts, 20, kc, mode="reconstruct", control="pump")  # warm-up
    work = [x.clone() for x in psi0]
    torch.cuda.synchronize()
    t = time.perf_counter()
    bc.step(work, steps, 0.0)
    torch.cuda.synchronize()
    t_fc = time.perf_counter() - t
    cav = {"workload": f"{nb} x 512^2, adiabatic cavity field, pump depth over 200 knots", "forward_s": t_fc}
    for mode in ("reconstruct", "store"):
        try:
            r = run(bc, mode, t_fc, kc, control="pump")
            if mode == "store":
                r = run(bc, mode, t_fc, kc, control="pump")
        except gpe.GpeError as e:
            cav[mode] = {"error": str(e)}
            continue
        r.pop("grad")
        cav[mode] = r
    bc.close()
    out["adiabatic_cavity_pump"] = cav
    return out


def _timed(fn) -> float:
    import torch

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / 1e3


def bench_library_fft(steps: int, us_per_step: float):
    """Side comparison, not the product path: the cavity workload's split step at 1024^2
    written with torch's FFT (hipFFT on ROCm) and elementwise complex64 ops -- V/2 kick,
    fft2, kinetic factor, ifft2, V/2 kick and the per-step overlap sum Theta, with the
    field held at zero.  Also the fft2 + ifft2 pair alone, the library route's floor."""
    import numpy as np
    import torch

    from paper_2404_14401_amd import workloads as W

    s = W.cavity_1024(0)
    dev = "cuda"
    y, x = np.meshgrid(s.ys(), s.xs(), indexing="ij")
    v = (0.5 * s.wx ** 2 * (x - s.x0) ** 2 + 0.5 * s.wy ** 2 * (y - s.y0) ** 2
         + s.sy.v0 * np.cos(s.ky_lat * y) ** 2)
    V = torch.from_numpy(v.astype(np.float32)).to(dev)
    cxcy = torch.from_numpy((np.cos(s.kc * x) * np.cos(s.kc * y)).astype(np.float32)).to(dev)
    kx = 2 * np.pi * np.fft.fftfreq(s.nx, d=s.lx / s.nx)
    ky = 2 * np.pi * np.fft.fftfreq(s.ny, d=s.ly / s.ny)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    K = torch.from_numpy(np.exp(-0.5j * k2 * s.dt).astype(np.complex64)).to(dev)
    one = torch.ones_like(V)
    psi = torch.from_numpy(W.to_c64(W.thomas_fermi_guess(s, float(np.sqrt(s.g / np.pi) * s.wx)))).to(dev)
    h, g = 0.5 * s.dt, s.g

    def step(p):
        d = p.real * p.real + p.imag * p.imag
        p = p * torch.polar(one, -(V + g * d) * h)
        p = torch.fft.ifft2(torch.fft.fft2(p) * K)
        d = p.real * p.real + p.imag * p.imag
        p = p * torch.polar(one, -(V + g * d) * h)
        return p, (d * cxcy).sum()

    def run(n):
        nonlocal psi
        for _ in range(n):
            psi, _ = step(psi)

    run(20)
    t = _timed(lambda: run(steps))
    q = psi.clone()
    tf = _timed(lambda: [torch.fft.ifft2(torch.fft.fft2(q)) for _ in range(steps)])
    n = s.nx * s.ny
    out = {"what": "torch.fft (hipFFT) + elementwise complex64 split step, cavity workload at 1024^2, "
                   "field held at 0, Theta summed each step",
           "steps": steps, "us_per_step": 1e6 * t / steps, "value": n * steps / t, "unit": "grid-point-steps/s",
           "fft2_ifft2_pair_us": 1e6 * tf / steps,
           "this_library_speedup": (1e6 * t / steps) / us_per_step}
    # the same in complex128 (the paper's double-precision runs)
    V, cxcy, K, one = V.double(), cxcy.double(), K.to(torch.complex128), one.double()
    psi = psi.to(torch.complex128)
    run(5)
    t2 = _timed(lambda: run(steps))
    out["complex128"] = {"us_per_step": 1e6 * t2 / steps, "value": n * steps / t2,
                         "this_library_speedup": (1e6 * t2 / steps) / us_per_step}
    return out


def _torch_imag_steps(s, psi, nsteps: int):
    """The paper's route for comparison: imaginary-time split steps written with torch's
    FFT and elementwise ops in psi's dtype (V/2 decay, fft2, kinetic decay, ifft2, V/2
    decay, renormalisation), on psi's device; returns the elapsed seconds."""
    import numpy as np
    import torch

    real = torch.float64 if psi.dtype == torch.complex128 else torch.float32
    y, x = np.meshgrid(s.ys(), s.xs(), indexing="ij")
    V = torch.from_numpy(0.5 * s.wx ** 2 * x ** 2 + 0.5 * s.wy ** 2 * y ** 2).to(psi.device, real)
    kx = 2 * np.pi * np.fft.fftfreq(s.nx, d=s.lx / s.nx)
    ky = 2 * np.pi * np.fft.fftfreq(s.ny, d=s.ly / s.ny)
    K = torch.from_numpy(np.exp(-0.5 * (ky[:, None] ** 2 + kx[None, :] ** 2) * s.dt)).to(psi.device, real)
    dA, h = (s.lx / s.nx) * (s.ly / s.ny), 0.5 * s.dt

    def run(p, n):
        for _ in range(n):
            p = p * torch.exp(-(V + s.g * (p.real * p.real + p.imag * p.imag)) * h)
            p = torch.fft.ifft2(torch.fft.fft2(p) * K)
            p = p * torch.exp(-(V + s.g * (p.real * p.real + p.imag * p.imag)) * h)
            p = p / torch.sqrt((p.real * p.real + p.imag * p.imag).sum() * dA)
        return p

    run(psi, 2)
    if psi.is_cuda:
        return _timed(lambda: run(psi, nsteps))
    t = time.perf_counter()
    run(psi, nsteps)
    return time.perf_counter() - t


def sweep_setup(n: int):
    """Grid-sweep workload: imaginary time, g = 0, harmonic trap w = 1, 2^n x 2^n on
    [-8, 8)^2, dtau = 1e-3 (the paper's timing experiment, Sec. 4.1)."""
    from paper_2404_14401_amd import workloads as W

    return W.imag_ground_64(0.0).with_(nx=1 << n, ny=1 << n)


def bench_grid_sweep(steps: int, runs: int, side_steps: int):
    """The paper's timing experiment reshaped for this library (Sec. 4.1): imaginary time
    for a non-interacting condensate in a fixed harmonic trap, Nx = Ny = 2^n on
    [-8, 8)^2, dtau = 1e-3, `steps` steps per run, the mean over `runs` runs; n from 6 to
    13 (the paper's range; 8192^2 is the plan's largest grid).  Small grids take the LDS-resident path.  Beside it, on
    bounded samples of `side_steps` steps scaled to `steps`: the paper's route (torch.fft
    and elementwise ops) on the GPU in complex128 and complex64.  (The oracle's times for
    the same sweep are part of the cpu_baseline leg.)"""
    import numpy as np
    import torch

    from paper_2404_14401_amd import gpe
    from paper_2404_14401_amd import workloads as W

    rows = []
    for n in range(6, 14):
        s = sweep_setup(n)
        p = gpe.Plan.from_setup(s)
        psi = torch.from_numpy(W.to_c64(W.gaussian(s, 1.5))).to("cuda")
        p.step_imag(psi, 10, 0.0)
        ts = [_timed(lambda: p.step_imag(psi, steps, 0.0)) for _ in range(runs)]
        t = float(np.mean(ts))
        pts = s.nx * s.ny
        row = {"n": n, "grid": pts, "ms_per_run": 1e3 * t, "ms_runs": [1e3 * x for x in ts],
               "value": pts * steps / t, "hbm_frac": 32 * pts * steps / t / (HBM_PEAK_GBS * 1e9)}
        p.close()
        if side_steps > 0:
            scale = steps / side_steps
            for name, dt in (("torch_c128_ms_per_run", torch.complex128), ("torch_c64_ms_per_run", torch.complex64)):
                row[name] = 1e3 * scale * _torch_imag_steps(s, psi.to(dt), side_steps)
        del psi
        rows.append(row)
    return {"workload": f"imaginary time, g=0, harmonic trap w=1, [-8,8)^2, dtau=1e-3, {steps} steps per run, "
                        f"mean of {runs} runs; torch route from {side_steps}-step samples scaled to {steps} steps",
            "unit": "grid-point-steps/s", "rows": rows}


def bench_eta_sweep(steps: int, seeds: int = 4):
    """The cavity workload's eta sweep (seeds 0 .. seeds-1, each its own eta) as one batch
    of 1024^2 field-ODE runs, against running the seeds one after the other."""
    import numpy as np
    import torch

    from paper_2404_14401_amd import gpe
    from paper_2404_14401_amd import workloads as W

    setups = [W.cavity_1024(k) for k in range(seeds)]
    s0 = setups[0]
    psi0 = torch.from_numpy(W.to_c64(W.thomas_fermi_guess(s0, float(np.sqrt(s0.g / np.pi) * s0.wx)))).to("cuda")
    psis = [psi0.clone() for _ in setups]
    b = gpe.Batch(setups)
    b.step(psis, 4, 0.0)
    t_b = _timed(lambda: b.step(psis, steps, 4 * s0.dt))
    plans = [gpe.Plan.from_setup(s) for s in setups]
    ws = [psi0.clone() for _ in setups]
    for p, w in zip(plans, ws):
        p.step_real(w, 4, 0.0)
    t_p = _timed(lambda: [p.step_real(w, steps, 4 * s0.dt) for p, w in zip(plans, ws)])
    pts = seeds * s0.nx * s0.ny
    out = {"workload": f"cavity run at 1024^2 for eta seeds 0..{seeds - 1} in one batch, field ODE", "steps": steps,
           "value": pts * steps / t_b, "unit": "grid-point-steps/s", "us_per_batch_step": 1e6 * t_b / steps,
           "hbm_frac": 32 * pts * steps / t_b / (HBM_PEAK_GBS * 1e9), "plain_runs_value": pts * steps / t_p,
           "speedup_vs_plain_runs": t_p / t_b, "alpha": [str(b.cavity(i)) for i in range(seeds)]}
    b.close()
    return out


def bench_out_of_cache(steps: int, members: int):
    """A state larger than the 256 MB Infinity Cache: `members` real-time condensates at
    1024^2 (trap + pump lattice of the cavity workload, field off) in one batch, so the
    per-step traffic has to come from HBM."""
    import numpy as np
    import torch

    from paper_2404_14401_amd import gpe
    from paper_2404_14401_amd import workloads as W

    s = W.cavity_1024(0).with_(cavity=False)
    setups = [s] * members
    psi0 = torch.from_numpy(W.to_c64(W.thomas_fermi_guess(s, float(np.sqrt(s.g / np.pi) * s.wx)))).to("cuda")
    psis = [psi0.clone() for _ in range(members)]
    b = gpe.Batch(setups)
    b.step(psis, 4, 0.0)
    t = _timed(lambda: b.step(psis, steps, 4 * s.dt))
    pts = members * s.nx * s.ny
    b.close()
    return {"workload": f"{members} x 1024^2 real-time condensates in one batch (state {8 * pts / 2**20:.0f} MiB), "
                        "trap + pump lattice, field off", "steps": steps, "value": pts * steps / t,
            "unit": "grid-point-steps/s", "us_per_step": 1e6 * t / steps,
            "hbm_frac": 32 * pts * steps / t / (HBM_PEAK_GBS * 1e9)}


def stream_copy_gbs(mib: int = 1024, reps: int = 20) -> float:
    """Device-to-device copy bandwidth (read + write bytes) of a `mib` MiB buffer."""
    import torch

    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    t = _timed(lambda: [b.copy_(a) for _ in range(reps)])
    return 2 * a.numel() * reps / t / 1e9


def bench_widened(steps: int, tune_cache: str | None = None):
    """The paths beyond the main step: the Fourier-space ordering with momentum-order
    populations (Kapitza-Dirac, 512^2, and the 1024^2 grid without the cavity), the
    adiabatic cavity field at 1024^2 (probe pass + two passes per step), and the
    self-organisation sweep in batched form (80 members at 128^2, tuned shapes)."""
    import numpy as np
    import torch

    from paper_2404_14401_amd import gpe
    from paper_2404_14401_amd import workloads as W

    out = {}
    # Fourier-space ordering on the 1024^2 grid (cavity off): two passes per step
    s = W.cavity_1024(0).with_(cavity=False)
    n = s.nx * s.ny
    psik = torch.fft.fft2(torch.from_numpy(W.to_c64(W.thomas_fermi_guess(s, float(np.sqrt(s.g / np.pi) * s.wx))))
                          .to("cuda"))
    p = gpe.Plan.from_setup(s)
    p.step_real_k(psik, 20, 0.0)
    t = _timed(lambda: p.step_real_k(psik, steps, 0.0))
    tm = _timed(lambda: [p.momentum_orders(psik, 1, 64, 7) for _ in range(20)]) / 20
    out["kspace_1024"] = {"value": n * steps / t, "unit": "grid-point-steps/s", "steps": steps,
                          "us_per_step": 1e6 * t / steps, "b_alg_per_point_step": 32,
                          "hbm_frac": 32 * n * steps / t / (HBM_PEAK_GBS * 1e9),
                          "momentum_orders_us": 1e6 * tm}
    # adiabatic field at 1024^2: 8 B (probe read) + 2 x 16 B per point-step
    s = W.cavity_1024_adiabatic(0)
    psi = torch.from_numpy(W.to_c64(W.thomas_fermi_guess(s, float(np.sqrt(s.g / np.pi) * s.wx)))).to("cuda")
    p = gpe.Plan.from_setup(s)
    p.step_real(psi, 20, 0.0)
    t = _timed(lambda: p.step_real(psi, steps, 20 * s.dt))
    out["adiabatic_1024"] = {"value": n * steps / t, "unit": "grid-point-steps/s", "steps": steps,
                             "us_per_step": 1e6 * t / steps, "b_alg_per_point_step": 40,
                             "hbm_frac": 40 * n * steps / t / (HBM_PEAK_GBS * 1e9),
                             "alpha": str(p.cavity()["alpha"])}
    # Kapitza-Dirac at 512^2: the full flash with the three population snapshots
    s = W.kapitza_dirac_512(W.KD_G)
    psik = torch.fft.fft2(torch.from_numpy(W.kapitza_dirac_start(s)).to("cuda"))
    p = gpe.Plan.from_setup(s)

    def kd():
        n0 = 0
        pops = []
        for snap in W.KD_SNAPSHOTS:
            p.step_real_k(psik, snap - n0, n0 * s.dt)
            n0 = snap
            pops.append(p.momentum_orders(psik, 1, W.KD_ORDER_STEP, 2)[0].tolist())
        return pops

    kd()
    psik = torch.fft.fft2(torch.from_numpy(W.kapitza_dirac_start(s)).to("cuda"))
    res = []
    t = _timed(lambda: res.append(kd()))
    m = W.KD_SNAPSHOTS[-1]
    out["kapitza_dirac_512"] = {"value": s.nx * s.ny * m / t, "unit": "grid-point-steps/s", "steps": m,
                                "run_ms": 1e3 * t, "orders_-2..2_at_snapshots": res[0]}
    # self-organisation sweep: 16 depths x 5 detunings at 128^2, batched vs plain loop
    setups = W.self_organisation_sweep()
    psis = [torch.from_numpy(W.self_organisation_start(x)).to("cuda") for x in setups]
    b = gpe.Batch(setups)
    t = time.perf_counter()
    b.tune(tune_cache)
    tune_s = time.perf_counter() - t
    b.step(psis, 20, 0.0)
    t_b = _timed(lambda: b.step(psis, steps, 20 * W.SO_DT))
    plans = [gpe.Plan.from_setup(x) for x in setups]
    t_p = _timed(lambda: [q.step_real(y, steps, 0.0) for q, y in zip(plans, psis)])
    pts = sum(x.nx * x.ny for x in setups)
    out["self_organisation_sweep_128"] = {"members": len(setups), "value": pts * steps / t_b,
                                          "unit": "grid-point-steps/s", "steps": steps,
                                          "plain_loop_value": pts * steps / t_p, "speedup_vs_plain_loop": t_p / t_b,
                                          "tune_s": tune_s,
                                          "photons_max": float(max(abs(b.cavity(i)) ** 2 for i in range(len(setups))))}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--timing-every", type=int, default=16,
                    help="bracket every k-th step's passes with HIP events (roofline)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work (0: skip)")
    ap.add_argument("--batched-steps", type=int, default=200, help="steps of the 208-member sweep (0: skip)")
    ap.add_argument("--adjoint-steps", type=int, default=5000, help="steps of the control gradient (0: skip)")
    ap.add_argument("--adjoint-batch", type=int, default=16)
    ap.add_argument("--widened-steps", type=int, default=2000,
                    help="steps of the Fourier-space, adiabatic-field and sweep legs (0: skip)")
    ap.add_argument("--side-steps", type=int, default=200,
                    help="steps of the torch.fft side comparison (0: skip)")
    ap.add_argument("--sweep-steps", type=int, default=1000,
                    help="steps per run of the 64^2..4096^2 imaginary-time grid sweep (0: skip)")
    ap.add_argument("--sweep-runs", type=int, default=5)
    ap.add_argument("--sweep-side-steps", type=int, default=50,
                    help="steps of the torch-route and oracle samples in the grid sweep (0: skip)")
    ap.add_argument("--sweep-oracle-max-n", type=int, default=9,
                    help="largest 2^n grid of the grid sweep the oracle is timed on (cpu_baseline leg)")
    ap.add_argument("--eta-steps", type=int, default=2000,
                    help="steps of the batched eta sweep of the cavity workload (0: skip)")
    ap.add_argument("--ooc-steps", type=int, default=20,
                    help="steps of the 64 x 1024^2 out-of-cache batch (0: skip)")
    ap.add_argument("--ooc-members", type=int, default=64)
    ap.add_argument("--cpu-one-core", type=float, default=5.0,
                    help="seconds of single-thread oracle work (0: skip)")
    ap.add_argument("--tune-cache", default=os.path.join(HERE, "profiles", "tune_cache.txt"))
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 10 device copies of MIB MiB (scale for rocprofv3 byte counters)")
    ap.add_argument("--traffic-from", metavar="DIR",
                    help="only print the per-launch HBM bytes from rocprofv3 counter runs under DIR "
                         "(fetch/, write/, copy_fetch/, copy_write/; no GPU used)")
    args = ap.parse_args()
    if args.traffic_from:
        print(json.dumps(traffic_from(args.traffic_from), indent=1))
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": 4 * n, "copies": 10}), flush=True)
        return 0

    from paper_2404_14401_amd import gpe
    from paper_2404_14401_amd import workloads as W

    setup = W.cavity_1024(seed=0)
    npts = setup.nx * setup.ny
    # the run's start: the Thomas-Fermi guess relaxed in imaginary time (trap + pump,
    # cavity off), here by the library itself
    psi = torch.from_numpy(W.to_c64(W.cavity_start_guess(setup))).to("cuda")
    relax = gpe.Plan.from_setup(W.cavity_relax(setup))
    relax.step_imag(psi, W.CAVITY_RELAX_STEPS, 0.0)
    relax.sync()
    relax.close()
    psi0 = psi.cpu().numpy()
    plan = gpe.Plan.from_setup(setup)
    # device copies first: their measurement also brings the GPU to its working clock
    copy = stream_copy_gbs()

    plan.step_real(psi, args.warmup, 0.0)
    plan.sync()
    torch.cuda.synchronize()

    # pass timing on the last step of every window (one window in a 20-step run)
    plan.set_timing(max(1, min(args.timing_every, args.steps - 1)))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record()
    plan.step_real(psi, args.steps, args.warmup * setup.dt)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1)
    plan.sync()
    tim = plan.timing()
    plan.set_timing(0)

    value = npts * args.steps / (ms / 1e3)
    passes = {"column_pass": tim["col_ms"], "row_pass_mid": tim["row_ms"]}
    dom = max(passes, key=passes.get)
    dom_ms = passes[dom]
    achieved = B_PASS * npts / (dom_ms / 1e3) / 1e9
    traffic = load_traffic(dom)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "cavity-QED self-consistent real-time split step, 1024x1024 on [-32,32)^2, "
                        "complex64 state, g=1000, trap w=0.05, red-detuned Vp=Vc=-25, k=1, Delta_c=-20, "
                        "kappa=10, eta=5*U(seed 0), dt=2e-4, from the relaxed trap + pump ground state",
            "grid": [setup.ny, setup.nx],
            "storage": "c64",
            "arithmetic": "f64 registers",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": B_PASS * npts,
            "launch_ms": dom_ms,
            "launches_timed": tim["col_n"] if dom == "column_pass" else tim["row_n"],
        },
        "passes_ms": passes,
        "step_roofline": {"b_alg_per_point_step": 2 * B_PASS,
                          "frac": 2 * B_PASS * value / (HBM_PEAK_GBS * 1e9)},
        "wall_s": wall,
    }
    out["stream_copy_gbs"] = copy
    # the side legs run on their own: the headline's plan and state are released first
    plan.close()
    del psi
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    out["step_roofline"]["frac_of_stream_copy"] = 2 * B_PASS * value / (copy * 1e9)
    if args.batched_steps > 0:
        log("batched sweep ...")
        out["batched"] = bench_batched(args.batched_steps, args.tune_cache)
    if args.widened_steps > 0:
        log("widened rows ...")
        out["widened"] = bench_widened(args.widened_steps, args.tune_cache)
    if args.adjoint_steps > 0:
        log("adjoint ...")
        out["adjoint"] = bench_adjoint(args.adjoint_steps, args.adjoint_batch, args.tune_cache)
    if args.sweep_steps > 0:
        log("grid sweep ...")
        out["grid_sweep"] = bench_grid_sweep(args.sweep_steps, args.sweep_runs, args.sweep_side_steps)
    if args.eta_steps > 0:
        log("eta sweep batch ...")
        out["eta_sweep_1024"] = bench_eta_sweep(args.eta_steps)
    if args.ooc_steps > 0:
        log("out-of-cache batch ...")
        out["out_of_cache"] = bench_out_of_cache(args.ooc_steps, args.ooc_members)
    if args.side_steps > 0:
        log("torch.fft side comparison ...")
        out["library_fft_side"] = bench_library_fft(args.side_steps, 1e3 * out["ms_per_step"])
    if args.cpu_budget > 0:
        log(f"timing the oracle for ~{args.cpu_budget:.0f} s ...")
        out["cpu_baseline"] = cpu_baseline(setup, psi0, args.cpu_budget, args.cpu_one_core,
                                           args.sweep_side_steps if args.sweep_steps > 0 else 0,
                                           args.sweep_oracle_max_n, max(args.sweep_steps, 1))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
