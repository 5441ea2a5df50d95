"""GPU parity: HF preparation and Pauli rotations against the oracle."""
import numpy as np
import pytest
import torch

from oracle import statevector as osv
from paper_2208_10978_amd import binding as B
from paper_2208_10978_amd.engine import StateVector
from tests.gpu_common import announce, to_np_state
from workloads import random_rotations

pytestmark = pytest.mark.gpu


def random_general(n, count, seed):
    """Arbitrary strings (any x, z), including diagonal ones and same-x runs."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 1 << n, size=count, dtype=np.uint64)
    z = rng.integers(0, 1 << n, size=count, dtype=np.uint64)
    x[::7] = 0                          # diagonal strings
    for k in range(3, count, 5):        # same-x neighbours
        x[k] = x[k - 1]
    phi = rng.uniform(-2.0, 2.0, size=count)
    return x, z, phi


def random_state_tensor(n, seed, dtype):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    v /= np.linalg.norm(v)
    return v


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_prepare_hf(dtype):
    announce(f"prepare_hf {dtype}")
    s = StateVector(10, dtype)
    s.prepare_hf(0b1011001)
    torch.cuda.synchronize()
    v = to_np_state(s.amps)
    want = np.zeros(1 << 10); want[0b1011001] = 1
    assert np.array_equal(v, want)


@pytest.mark.parametrize("n", [1, 3, 9, 13, 14, 16, 17])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_random_rotation_lists(n, dtype):
    announce(f"random rotations n={n} {dtype}")
    count = 60
    x, z, phi = random_general(n, count, 100 + n)
    v0 = random_state_tensor(n, n, dtype)
    s = StateVector(n, dtype)
    s.amps.copy_(torch.from_numpy(v0).to(s.amps.dtype))
    s.apply_rotations(x, z, phi)
    torch.cuda.synchronize()
    got = to_np_state(s.amps)
    want = osv.apply_rotations(v0.copy(), x, z, phi)
    tol = 1e-12 if dtype == "c128" else 2e-5
    assert np.abs(got - want).max() < tol


@pytest.mark.parametrize("n", [12, 18, 22])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_uccd_type_rotations(n, dtype):
    """4-qubit X/Y strings over random qubits (the raw-sweep workload)."""
    announce(f"4-support rotations n={n} {dtype}")
    x, z, phi = random_rotations(n, 40, 4242 + n, amplitude=0.5)
    psi0 = osv.basis_state(n, (1 << (n // 2)) - 1)
    s = StateVector(n, dtype)
    s.prepare_hf((1 << (n // 2)) - 1)
    s.apply_rotations(x, z, phi)
    torch.cuda.synchronize()
    got = to_np_state(s.amps)
    want = osv.apply_rotations(psi0, x, z, phi)
    tol = 1e-12 if dtype == "c128" else 2e-5
    assert np.abs(got - want).max() < tol


def test_rotation_list_validation():
    announce("validation")
    s = StateVector(6, "c128")
    with pytest.raises(B.Q2svError):
        s.apply_rotations(np.array([1 << 6], dtype=np.uint64), np.array([0], dtype=np.uint64), [0.1])
    with pytest.raises(B.Q2svError):
        s.apply_rotations(np.array([1], dtype=np.uint64), np.array([0], dtype=np.uint64), [np.nan])
    s.apply_rotations(np.array([], dtype=np.uint64), np.array([], dtype=np.uint64), [])


@pytest.mark.parametrize("n", [5, 15])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_degenerate_rotations(n, dtype):
    """The identity string (a global phase), phi = 0 and 2 pi (R = I and -I), a
    rotation followed by its inverse, the same string repeated, and a run of
    more same-x strings than one fused run holds (9 > 8) so the planner splits
    it; against the oracle, one call."""
    announce(f"degenerate rotations n={n} {dtype}")
    rng = np.random.default_rng(900 + n)
    xa, za = int(rng.integers(1, 1 << n)), int(rng.integers(0, 1 << n))
    xs, zs, ph = [0, xa, xa, xa, xa, 0], [0, za, za, za, za, 5 % (1 << n)], [0.7, 0.0, 2 * np.pi, 0.3, -0.3, 1.1]
    xs += [xa] * 3; zs += [za] * 3; ph += [0.2, 0.2, 0.2]
    xb = int(rng.integers(1, 1 << n))
    for k in range(9):
        xs.append(xb); zs.append(int(rng.integers(0, 1 << n))); ph.append(float(rng.uniform(-1, 1)))
    x = np.array(xs, dtype=np.uint64); z = np.array(zs, dtype=np.uint64)
    v0 = random_state_tensor(n, 31 + n, dtype)
    s = StateVector(n, dtype)
    s.amps.copy_(torch.from_numpy(v0).to(s.amps.dtype))
    s.apply_rotations(x, z, ph)
    torch.cuda.synchronize()
    got = to_np_state(s.amps)
    want = osv.apply_rotations(v0.copy(), x, z, ph)
    tol = 1e-12 if dtype == "c128" else 2e-5
    assert np.abs(got - want).max() < tol
    s.free()
