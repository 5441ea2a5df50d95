"""Pins for the rotation step (Eq. 11) and Algorithm 2."""
import json
import os

import numpy as np
import pytest

from oracle import dense, fermion, pauli
from oracle import statevector as sv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("seed", range(6))
def test_rotation_matches_expm(seed):
    n = 5
    rng = np.random.default_rng(100 + seed)
    x, z = int(rng.integers(1 << n)), int(rng.integers(1 << n))
    phi = float(rng.uniform(-3, 3))
    psi = random_state(n, seed)
    assert np.allclose(sv.rotate(psi, x, z, phi), dense.rotation_matrix(x, z, n, phi) @ psi, atol=1e-13)


def test_rotation_on_basis_state_closed_form():
    n = 6
    for x, z, k, phi in [(0b101001, 0b100001, 0b010110, 0.7), (0b11, 0b10, 5, -1.3), (0, 0b1111, 9, 0.4)]:
        out = sv.rotate(sv.basis_state(n, k), x, z, phi)
        want = np.zeros(1 << n, dtype=complex)
        want[k] += np.cos(phi / 2)
        omega = 1j ** (pauli.popcount(x & z) % 4)
        want[k ^ x] += -1j * np.sin(phi / 2) * omega * (-1) ** pauli.popcount(k & z)
        assert np.allclose(out, want, atol=1e-15)


def test_rotation_inverse_period_and_norm():
    n = 4
    psi = random_state(n, 7)
    x, z = pauli.from_label("XYZY")
    back = sv.rotate(sv.rotate(psi, x, z, 0.9), x, z, -0.9)
    assert np.allclose(back, psi, atol=1e-15)
    assert np.allclose(sv.rotate(psi, x, z, 2 * np.pi), -psi, atol=1e-14)
    assert abs(np.linalg.norm(sv.rotate(psi, x, z, 1.1)) - 1) < 1e-14


@pytest.mark.parametrize("label", ["XYZX", "YIIX", "ZZIZ", "IIYI", "IIII", "XXXX", "YZZY"])
def test_algorithm2_circuit_equals_exp_i_theta_p(label):
    n = len(label)
    x, z = pauli.from_label(label)
    theta = 0.37
    psi = random_state(n, 3)
    out = psi
    for g in dense.algorithm2_gates(x, z, n, theta):
        out = dense.apply_gate(out, g)
    want = dense.rotation_matrix(x, z, n, -2 * theta) @ psi   # exp(i theta P)
    assert np.allclose(out, want, atol=1e-13)
    assert np.allclose(out, sv.rotate(psi, x, z, -2 * theta), atol=1e-13)


def test_table1_h2_cnot_count():
    gold = json.load(open(os.path.join(GOLDEN, "table1_h2_uccsd_cnots.json")))
    rots = fermion.uccsd_rotations(gold["n_qubits"], gold["n_electrons"])
    total = sum(dense.count_cnots(dense.algorithm2_gates(x, z, gold["n_qubits"], 0.1)) for x, z, _, _ in rots)
    assert total == gold["uccsd_cnot_gates"]
