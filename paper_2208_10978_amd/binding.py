"""ctypes binding of libq2sv.so, with the C names (argument marshalling only).

Every computation happens in the HIP library; nothing here falls back to the
CPU.  If the library has not been built, importing a function raises.
Host arrays are NumPy; device buffers (amplitudes, outputs) are torch CUDA
(HIP) tensors passed by pointer, and work is enqueued on the stream given at
``sv_alloc`` (by default torch's current stream).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libq2sv.so")

SV_C128 = 0
SV_C64 = 1
SV_R64 = 2
SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_EBUSY = 0, -1, -2, -3, -4
SV_MAX_QUBITS = 34


class Q2svError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"q2sv error {code}: {msg}")
        self.code = code


class DeviceFailure(Q2svError):
    """SV_EDEVICE: the device failed and stays unusable for this process."""


class Busy(Q2svError):
    """SV_EBUSY: another call on the same state handle is in progress."""


_lib = None
_c = ctypes
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2208_10978_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "sv_alloc": [_c.c_int, _c.c_int, _vp, _c.c_size_t, _vp, _c.POINTER(_vp)],
            "sv_free": [_vp],
            "sv_set_stream": [_vp, _vp],
            "sv_set_real_hint": [_vp, _c.c_int],
            "sv_inject_device_failure": [_c.c_char_p],
            "sv_prepare_hf": [_vp, _c.c_uint64],
            "sv_apply_pauli_rotations": [_vp, _vp, _vp, _i64],
            "sv_expect_pauli_sum": [_vp, _vp, _vp, _i64, _vp],
            "sv_adjoint_grad": [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp],
            "sv_adjoint_grad_params": [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp],
            "sv_hamiltonian_create": [_c.c_int, _vp, _vp, _i64, _c.POINTER(_vp)],
            "sv_hamiltonian_free": [_vp],
            "sv_expect_hamiltonian": [_vp, _vp, _vp],
            "sv_expect_hamiltonian_noalloc": [_vp, _vp, _vp],
            "sv_adjoint_grad_params_h": [_vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp],
            "sv_rotations_create": [_c.c_int, _vp, _i64, _vp, _vp, _i64, _c.POINTER(_vp)],
            "sv_rotations_free": [_vp],
            "sv_apply_rotations_h": [_vp, _vp, _vp],
            "sv_adjoint_grad_params_hr": [_vp, _vp, _vp, _vp, _vp, _vp, _vp],
            "sv_adjoint_grad_params_deflated": [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, _i64, _vp, _vp,
                                                _i64, _vp, _vp, _vp],
            "sv_overlap": [_vp, _vp, _vp],
            "sv_normalize": [_vp, _vp],
            "sv_gather_amplitudes": [_vp, _vp, _i64, _vp],
            "sv_profile_begin": [],
            "sv_profile_end": [ctypes.c_char_p, _c.c_size_t],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _c.c_int
        L.sv_last_error.argtypes = []
        L.sv_last_error.restype = _c.c_char_p
        _lib = L
    return _lib


EXPORTED = (
    "sv_alloc", "sv_free", "sv_set_stream", "sv_set_real_hint", "sv_inject_device_failure",
    "sv_prepare_hf",
    "sv_apply_pauli_rotations",
    "sv_expect_pauli_sum", "sv_adjoint_grad", "sv_adjoint_grad_params", "sv_hamiltonian_create",
    "sv_hamiltonian_free", "sv_expect_hamiltonian", "sv_expect_hamiltonian_noalloc", "sv_adjoint_grad_params_h",
    "sv_rotations_create", "sv_rotations_free", "sv_apply_rotations_h", "sv_adjoint_grad_params_hr",
    "sv_adjoint_grad_params_deflated", "sv_overlap", "sv_normalize",
    "sv_gather_amplitudes", "sv_profile_begin", "sv_profile_end", "sv_last_error",
)


def sv_last_error() -> str:
    return lib().sv_last_error().decode()


def _check(rc):
    if rc != SV_OK:
        cls = DeviceFailure if rc == SV_EDEVICE else Busy if rc == SV_EBUSY else Q2svError
        raise cls(rc, sv_last_error())


def _paulis(x, z) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    if x.shape != z.shape or x.ndim != 1:
        raise ValueError("x and z must be 1-d arrays of equal length")
    return np.ascontiguousarray(np.stack([x, z], axis=1))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_vp) if a is not None and a.size else None


def _dev(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return _vp(t.data_ptr())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


# --------------------------------------------------------------------------
# C functions with the same names
# --------------------------------------------------------------------------
def sv_alloc(n_qubits: int, dtype: int, amps, stream=None):
    """``amps``: contiguous complex128/complex64/float64 device tensor of >= 2^n entries."""
    if not amps.is_contiguous():
        raise ValueError("amps must be contiguous")
    h = _vp()
    _check(lib().sv_alloc(int(n_qubits), int(dtype), _dev(amps), amps.numel() * amps.element_size(),
                          _stream_handle(stream), ctypes.byref(h)))
    return h


def sv_free(s):
    _check(lib().sv_free(s))


def sv_set_stream(s, stream):
    _check(lib().sv_set_stream(s, _stream_handle(stream)))


def sv_set_real_hint(s, psi_is_real: bool):
    _check(lib().sv_set_real_hint(s, int(bool(psi_is_real))))


def sv_inject_device_failure(msg: str = ""):
    _check(lib().sv_inject_device_failure(msg.encode()))


def sv_prepare_hf(s, occ_mask: int):
    _check(lib().sv_prepare_hf(s, ctypes.c_uint64(int(occ_mask))))


def sv_apply_pauli_rotations(s, x, z, phi):
    p = _paulis(x, z)
    ph = _f64(phi)
    _check(lib().sv_apply_pauli_rotations(s, _ptr(p), _ptr(ph), len(ph)))


def sv_expect_pauli_sum(s, x, z, coef, out_dev):
    p = _paulis(x, z)
    c = _f64(coef)
    _check(lib().sv_expect_pauli_sum(s, _ptr(p), _ptr(c), len(c), _dev(out_dev)))


def sv_adjoint_grad(psi, lam, hx, hz, hc, rx, rz, phi, energy_dev, grad_dev):
    hp = _paulis(hx, hz)
    c = _f64(hc)
    rp = _paulis(rx, rz)
    ph = _f64(phi)
    _check(lib().sv_adjoint_grad(psi, lam, _ptr(hp), _ptr(c), len(c), _ptr(rp), _ptr(ph), len(ph),
                                 _dev(energy_dev), _dev(grad_dev)))


def sv_adjoint_grad_params(psi, lam, hx, hz, hc, rx, rz, phi, param_of_rot, dphi_dtheta, n_params,
                           energy_dev, grad_theta_dev):
    hp = _paulis(hx, hz)
    c = _f64(hc)
    rp = _paulis(rx, rz)
    ph = _f64(phi)
    pr = np.ascontiguousarray(param_of_rot, dtype=np.int32)
    d = _f64(dphi_dtheta)
    _check(lib().sv_adjoint_grad_params(psi, lam, _ptr(hp), _ptr(c), len(c), _ptr(rp), _ptr(ph), len(ph),
                                        _ptr(pr), _ptr(d), int(n_params), _dev(energy_dev),
                                        _dev(grad_theta_dev)))


def sv_hamiltonian_create(n_qubits: int, x, z, coef):
    p = _paulis(x, z)
    c = _f64(coef)
    h = _vp()
    _check(lib().sv_hamiltonian_create(int(n_qubits), _ptr(p), _ptr(c), len(c), ctypes.byref(h)))
    return h


def sv_hamiltonian_free(h):
    _check(lib().sv_hamiltonian_free(h))


def sv_expect_hamiltonian(s, h, out_dev):
    _check(lib().sv_expect_hamiltonian(s, h, _dev(out_dev)))


def sv_expect_hamiltonian_noalloc(s, h, out_dev):
    _check(lib().sv_expect_hamiltonian_noalloc(s, h, _dev(out_dev)))


def sv_adjoint_grad_params_h(psi, lam, h, rx, rz, phi, param_of_rot, dphi_dtheta, n_params, energy_dev,
                             grad_theta_dev):
    rp = _paulis(rx, rz)
    ph = _f64(phi)
    pr = np.ascontiguousarray(param_of_rot, dtype=np.int32)
    d = _f64(dphi_dtheta)
    _check(lib().sv_adjoint_grad_params_h(psi, lam, h, _ptr(rp), _ptr(ph), len(ph), _ptr(pr), _ptr(d),
                                          int(n_params), _dev(energy_dev), _dev(grad_theta_dev)))


def sv_rotations_create(n_qubits: int, rx, rz, param_of_rot, dphi_dtheta, n_params: int):
    rp = _paulis(rx, rz)
    pr = np.ascontiguousarray(param_of_rot, dtype=np.int32)
    d = _f64(dphi_dtheta)
    if not (len(pr) == len(d) == len(rp)):
        raise ValueError("rotation arrays differ in length")
    r = _vp()
    _check(lib().sv_rotations_create(int(n_qubits), _ptr(rp), len(rp), _ptr(pr), _ptr(d), int(n_params),
                                     ctypes.byref(r)))
    return r


def sv_rotations_free(r):
    _check(lib().sv_rotations_free(r))


def sv_apply_rotations_h(s, r, theta):
    th = _f64(theta)
    _check(lib().sv_apply_rotations_h(s, r, _ptr(th)))


def sv_adjoint_grad_params_hr(psi, lam, h, r, theta, energy_dev, grad_theta_dev):
    th = _f64(theta)
    _check(lib().sv_adjoint_grad_params_hr(psi, lam, h, r, _ptr(th), _dev(energy_dev), _dev(grad_theta_dev)))


def sv_adjoint_grad_params_deflated(psi, lam, h, proj, alpha, rx, rz, phi, param_of_rot, dphi_dtheta, n_params,
                                    energy_dev, ovl_dev, grad_theta_dev):
    """proj: sequence of state handles; alpha: their weights (Eq. 12)."""
    k = len(proj)
    arr = (_vp * max(k, 1))(*[ctypes.c_void_p(p.value if isinstance(p, ctypes.c_void_p) else p) for p in proj])
    al = _f64(alpha)
    if len(al) != k:
        raise ValueError("alpha and proj differ in length")
    rp = _paulis(rx, rz)
    ph = _f64(phi)
    pr = np.ascontiguousarray(param_of_rot, dtype=np.int32)
    d = _f64(dphi_dtheta)
    _check(lib().sv_adjoint_grad_params_deflated(psi, lam, h, ctypes.cast(arr, _vp), _ptr(al), k, _ptr(rp),
                                                 _ptr(ph), len(ph), _ptr(pr), _ptr(d), int(n_params),
                                                 _dev(energy_dev), _dev(ovl_dev), _dev(grad_theta_dev)))


def sv_overlap(a, b, out_dev):
    _check(lib().sv_overlap(a, b, _dev(out_dev)))


def sv_normalize(s, norm2_dev=None):
    _check(lib().sv_normalize(s, _dev(norm2_dev)))


def sv_gather_amplitudes(s, idx, out_dev):
    ix = np.ascontiguousarray(idx, dtype=np.uint64)
    _check(lib().sv_gather_amplitudes(s, _ptr(ix), len(ix), _dev(out_dev)))


def sv_profile_begin():
    _check(lib().sv_profile_begin())


def sv_profile_end() -> dict:
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().sv_profile_end(buf, len(buf)))
    return json.loads(buf.value.decode())
