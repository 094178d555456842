"""CPU-only checks of the C-ABI library: it loads without a GPU, exports every function the
header declares, and validates arguments on the host (no kernel is launched here)."""
import ctypes
import os
import re

import pytest

from paper_1502_07266_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "helm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(helm_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert "helm_setup" in names and "helm_apply" in names and "helm_solve" in names
    L = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding knows all of them
    assert set(names) <= set(binding._SIGS), set(names) - set(binding._SIGS)


def test_error_strings():
    L = binding.lib()
    for code in (0, 1, -1, -2, -3, -4):
        assert L.helm_error_string(code).decode().startswith("HELM_")
    assert b"unknown" in L.helm_error_string(77)


def test_plan_bytes_matches_factor_layout():
    # c3: n = 127, b = p = 5, d = 1: 123 groups per axis, blocks 25/30/36, complex64
    nbytes, nlines, maxb = binding.plan_bytes(127, 5, 150.0, 5, 1, binding.HELM_C64)
    assert nlines == 123 ** 2 and maxb == 36
    F = 127 * (25 ** 2 + 2 * 122 * 30 ** 2 + 122 ** 2 * 36 ** 2)
    assert nbytes >= F * 8 and nbytes < F * 8 + 127 ** 3 * 8 + 10 ** 6
    # c1 in complex128
    nbytes, nlines, maxb = binding.plan_bytes(31, 6, 180.0, 6, 1, binding.HELM_C128)
    assert nlines == 26 ** 2 and maxb == 49
    # ragged groups: n - b = 13 layers in groups of d = 3
    _, nlines, maxb = binding.plan_bytes(16, 3, 90.0, 2, 3, binding.HELM_C64)
    assert nlines == (1 + 5) ** 2 and maxb == 25


@pytest.mark.parametrize("args", [
    (10, 6, 180.0, 6, 1),     # n < 2b+1
    (31, 0, 1.0, 0, 1),       # b < 1
    (31, 6, 180.0, 7, 1),     # p > b
    (31, 6, 180.0, 6, 0),     # d < 1
    (31, 6, -1.0, 6, 1),      # C <= 0
    (31, 6, 180.0, 6, 6),     # block (p+d)^2 = 144 > 128
])
def test_invalid_parameters_rejected(args):
    with pytest.raises(binding.HelmError) as e:
        binding.plan_bytes(*args)
    assert e.value.code == binding.HELM_EINVAL


def test_null_handle_rejected():
    L = binding.lib()
    assert L.helm_apply(None, None, None, 1, None) == binding.HELM_EINVAL
    assert L.helm_solve(None, None, None, 1, 1e-6, 50, 10, 0, None, None, None) == binding.HELM_EINVAL
    assert L.helm_set_launch(None, 8) == binding.HELM_EINVAL
    assert L.helm_update_medium(None, None, None, None, None) == binding.HELM_EINVAL
    L.helm_destroy(None)


def test_wide_windows_are_solved_by_one_chain():
    """A block above 64 unknowns off the middle groups switches every line to one chain:
    blocks up to 128 (complex64) or 96 (complex128) are accepted."""
    _, nlines, maxb = binding.plan_bytes(31, 6, 180.0, 6, 3, binding.HELM_C64)
    assert maxb == 81
    _, _, maxb = binding.plan_bytes(31, 6, 180.0, 6, 3, binding.HELM_C128)
    assert maxb == 81
    with pytest.raises(binding.HelmError):
        binding.plan_bytes(31, 6, 180.0, 6, 5, binding.HELM_C128)     # 11 x 11 = 121 > 96
