"""The C-ABI library loads and exports every entry point declared in
include/csipm.h (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csipm.h")
LIB = os.path.join(ROOT, "paper_2502_04217_amd", "libcsipm.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(csipm_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for must in ["csipm_create", "csipm_solve", "csipm_apply_K", "csipm_apply_Pinv", "csipm_get_iterate",
                 "csipm_get_residuals", "csipm_mlp_loss_grad", "csipm_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libcsipm.so not built (run python -m paper_2502_04217_amd.build)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_calls():
    """Calls that touch no device: sizes, defaults, status strings."""
    from paper_2502_04217_amd import csipm
    assert csipm.workspace_bytes((256, 256, 256)) > 200 * 256 ** 3
    assert csipm.workspace_bytes((6, 8, 8)) > 0
    assert csipm.workspace_bytes((8, 8, 2)) == 0
    assert csipm.workspace_bytes((1, 8, 8)) > 0
    assert csipm.workspace_bytes((15, 21, 8)) > 0
    assert csipm.workspace_bytes((8, 8, 15)) > 0      # odd N3: the full-spectrum transforms
    assert csipm.workspace_bytes((45, 45, 45)) > 0
    assert csipm.workspace_bytes((8, 8, 11)) == 0
    assert csipm.workspace_bytes((80, 100, 120)) > 0
    assert csipm.workspace_bytes((8, 8, 22)) == 0     # half length 11
    assert csipm.workspace_bytes((8, 2048, 8)) == 0


def _smooth(n):
    for f in (2, 3, 5, 7):
        while n % f == 0:
            n //= f
    return n == 1


def test_supported_extents_are_the_7_smooth_ones():
    """Every extent 2^a 3^b 5^c 7^d up to 1024 has kernels on every axis
    (axis 3: at least 3; on axes 1 and 2 also 1 and 2), and no other does."""
    from paper_2502_04217_amd import csipm
    for N in range(1, 1100):
        want12 = N <= 1024 and _smooth(N)
        assert (csipm.workspace_bytes((N, 4, 4)) > 0) == want12, N
        assert (csipm.workspace_bytes((4, N, 4)) > 0) == want12, N
        assert (csipm.workspace_bytes((4, 4, N)) > 0) == (want12 and N >= 3), N
    o = csipm.default_options()
    assert o.tol == 1e-6 and o.sigma == 0.1 and o.tau == 0.99
    assert o.pc_min_missing == 0.01 and o.pc_min_cg == 2 and o.pc_max_relevant == 0.5
    assert o.refine_trust == 2e-6
    assert csipm.lib().csipm_status_string(-5) == b"unsupported grid"
    assert csipm.lib().csipm_mlp_scratch_bytes(65) == 2 * 1250 * 8
