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


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="library not built")
def test_resident_rotation_list_validation_needs_no_device():
    """sv_rotations_create copies and splits the list on the host: bad input is
    refused with a message, a good list gives a handle that frees cleanly."""
    import numpy as np
    x = np.array([0b0011, 0b1100], np.uint64)
    z = np.array([0b0001, 0b0100], np.uint64)
    with pytest.raises(binding.Q2svError, match="param_of_rot"):
        binding.sv_rotations_create(4, x, z, [0, 2], [0.5, -0.5], 2)          # parameter index out of range
    with pytest.raises(binding.Q2svError, match="qubit"):
        binding.sv_rotations_create(3, x, z, [0, 1], [0.5, -0.5], 2)          # acts on qubit 3 of a 3-qubit state
    with pytest.raises(binding.Q2svError, match="dphi"):
        binding.sv_rotations_create(4, x, z, [0, 1], [0.5, float("nan")], 2)
    r = binding.sv_rotations_create(4, x, z, [0, 1], [0.5, -0.5], 2)
    assert r.value
    binding.sv_rotations_free(r)


def _fresh(code: str) -> str:
    """Run code in a new interpreter: a device's failure mark lasts for the
    process, so it must not leak into the other tests."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


_PRELUDE = """
import ctypes
from paper_2208_10978_amd import binding as B
L = B.lib()
h = ctypes.c_void_p()
assert L.sv_alloc(4, B.SV_C128, ctypes.c_void_p(256), 1 << 20, None, ctypes.byref(h)) == B.SV_OK
"""


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="library not built")
def test_injected_device_failure_is_sticky():
    """After a device failure every later call on that device returns
    SV_EDEVICE with the first message and does no device work (the state
    handle here points at no real memory, so any launch would fail anyway);
    argument errors on NULL handles are still SV_EINVAL; sv_free releases."""
    _fresh(_PRELUDE + """
assert L.sv_inject_device_failure(b"planted for the test") == B.SV_OK
for rc in (L.sv_prepare_hf(h, 0), L.sv_apply_pauli_rotations(h, None, None, 0),
           L.sv_normalize(h, None), L.sv_set_real_hint(h, 1)):
    assert rc == B.SV_EDEVICE, rc
    msg = B.sv_last_error()
    assert "unusable after an earlier failure" in msg and "planted for the test" in msg, msg
h2 = ctypes.c_void_p()
assert L.sv_alloc(4, B.SV_C128, ctypes.c_void_p(256), 1 << 20, None, ctypes.byref(h2)) == B.SV_EDEVICE
hh = ctypes.c_void_p()
assert L.sv_hamiltonian_create(4, None, None, 0, ctypes.byref(hh)) == B.SV_EDEVICE
assert L.sv_prepare_hf(None, 0) == B.SV_EINVAL
assert L.sv_free(h) == B.SV_EDEVICE
print("ok")
""")


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="library not built")
def test_a_real_failed_launch_is_sticky_without_a_gpu():
    """With no GPU present the first kernel launch fails for real; that
    failure (not an injected one) must make later calls fail the same way."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present: no launch may be made on a fake buffer")
    _fresh(_PRELUDE + """
rc = L.sv_prepare_hf(h, 0)
assert rc == B.SV_EDEVICE, rc
first = B.sv_last_error()
assert L.sv_prepare_hf(h, 1) == B.SV_EDEVICE
assert first in B.sv_last_error() and "earlier failure" in B.sv_last_error()
print("ok")
""")


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="library not built")
def test_concurrent_calls_on_one_handle_get_ebusy():
    """One thread holds the handle in a long call (argument validation of a
    long rotation list whose last angle is not finite: SV_EINVAL, no device
    work); a second thread's calls on the same handle meanwhile return
    SV_EBUSY, and SV_EINVAL (its own bad argument) once the handle is free."""
    import threading
    import numpy as np
    lib = binding.lib()
    h = ctypes.c_void_p()
    assert lib.sv_alloc(4, binding.SV_C128, ctypes.c_void_p(256), 1 << 20, None, ctypes.byref(h)) == binding.SV_OK
    n = 4_000_000
    p = np.zeros((n, 2), dtype=np.uint64)
    phi = np.zeros(n)
    phi[-1] = np.nan
    seen = {"busy": 0, "inval": 0, "other": []}
    done = threading.Event()

    def other():
        while not done.is_set():
            rc = lib.sv_prepare_hf(h, 1 << 4)  # occ_mask >= 2^n: EINVAL when the handle is free
            if rc == binding.SV_EBUSY:
                seen["busy"] += 1
            elif rc == binding.SV_EINVAL:
                seen["inval"] += 1
            else:
                seen["other"].append(rc)

    t = threading.Thread(target=other)
    t.start()
    try:
        for _ in range(20):
            rc = lib.sv_apply_pauli_rotations(h, p.ctypes.data_as(ctypes.c_void_p),
                                              phi.ctypes.data_as(ctypes.c_void_p), n)
            assert rc == binding.SV_EINVAL
            if seen["busy"]:
                break
    finally:
        done.set()
        t.join()
    assert seen["busy"] > 0 and seen["inval"] > 0 and not seen["other"], seen
    assert lib.sv_prepare_hf(h, 1 << 4) == binding.SV_EINVAL
    assert "occ_mask" in binding.sv_last_error()
