"""Helpers shared by the GPU tests: device arrays, plans, comparisons.  Uses the oracle
only through tests.bridge (test infrastructure)."""
from __future__ import annotations

import numpy as np
import pytest


def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def to_dev(a: np.ndarray):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).to("cuda")


def to_host(t) -> np.ndarray:
    import torch

    torch.cuda.synchronize()
    return t.detach().to("cpu").numpy().astype(np.complex128)


def rel_l2(a, ref) -> float:
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def rel_l2_phase_aligned(a, ref) -> float:
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    ov = np.vdot(a, ref)
    ph = ov / abs(ov) if abs(ov) > 0 else 1.0
    return float(np.linalg.norm(a * ph - ref) / np.linalg.norm(ref))


def plain_plan_like(batch, setup):
    """A plain plan on the same kernels as the batch group of `setup`'s grid size
    (LDS-resident or multi-pass), so that member and plan agree to rounding."""
    import os

    from paper_2404_14401_amd import gpe

    lds = {(g["nx"], g["ny"]): g["lds"] for g in batch.groups()}[(setup.nx, setup.ny)]
    old = os.environ.get("GPE_PATH")
    os.environ["GPE_PATH"] = "lds" if lds else "multipass"
    try:
        return gpe.Plan.from_setup(setup)
    finally:
        if old is None:
            del os.environ["GPE_PATH"]
        else:
            os.environ["GPE_PATH"] = old
