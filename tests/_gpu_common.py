"""Shared helpers of the GPU tests: device check and error metrics.  Every
GPU test calls the HIP library through the C-ABI binding."""
import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2502_04217_amd import csipm
    csipm.lib()          # raises if the library is not built: no fallback
    return torch


def rel_inf(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.abs(ref).max())
    return float(np.abs(got - ref).max()) / (den if den > 0 else 1.0)


def rel2(got, ref):
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = float(np.linalg.norm(ref))
    return float(np.linalg.norm(got - ref)) / (den if den > 0 else 1.0)


def say(*a):
    print(*a, flush=True)
