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
