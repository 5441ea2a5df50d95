"""CPU checks of the boundary: the library loads and exports every symbol
declared in include/q2sv.h (no device calls)."""
import ctypes
import os
import re

import pytest

from paper_2208_10978_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "q2sv.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(sv_\w+)\(", text, flags=re.M)))


def test_header_and_binding_agree():
    assert set(declared_symbols()) == set(binding.EXPORTED)


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="library not built")
def test_argument_validation_needs_no_device():
    lib = binding.lib()
    h = ctypes.c_void_p()
    assert lib.sv_alloc(0, 0, ctypes.c_void_p(16), 1 << 20, None, ctypes.byref(h)) == binding.SV_EINVAL
    assert "n_qubits" in binding.sv_last_error()
    assert lib.sv_alloc(4, 7, ctypes.c_void_p(16), 1 << 20, None, ctypes.byref(h)) == binding.SV_EINVAL
    assert lib.sv_alloc(4, 0, ctypes.c_void_p(16), 100, None, ctypes.byref(h)) == binding.SV_EINVAL
    assert "smaller" in binding.sv_last_error()
    assert lib.sv_alloc(4, 0, ctypes.c_void_p(8), 1 << 20, None, ctypes.byref(h)) == binding.SV_EINVAL
    assert lib.sv_prepare_hf(None, 0) == binding.SV_EINVAL
    assert lib.sv_hamiltonian_create(0, None, None, 0, ctypes.byref(h)) == binding.SV_EINVAL
