"""Pins for oracle.pauli: every operation against dense Kronecker matrices."""
import itertools

import numpy as np

from oracle import pauli


def all_strings(n):
    return [(x, z) for x in range(1 << n) for z in range(1 << n)]


def test_label_roundtrip_and_factors():
    for lab in ["I", "X", "Y", "Z", "XYZI", "ZZXY"]:
        x, z = pauli.from_label(lab)
        assert pauli.to_label(x, z, len(lab)) == lab
    # Y on qubit 0 is i X Z
    x, z = pauli.from_label("Y")
    y = np.array([[0, -1j], [1j, 0]])
    assert np.allclose(pauli.dense(x, z, 1), y)


def test_dense_is_little_endian():
    # X on qubit 0 flips bit 0 of the index
    x, z = pauli.from_label("XI")
    m = pauli.dense(x, z, 2)
    e0 = np.zeros(4); e0[0] = 1
    assert np.allclose(m @ e0, np.eye(4)[1])


def test_apply_matches_dense_all_strings_n3():
    rng = np.random.default_rng(0)
    psi = rng.normal(size=8) + 1j * rng.normal(size=8)
    for x, z in all_strings(3):
        assert np.allclose(pauli.apply(psi, x, z), pauli.dense(x, z, 3) @ psi, atol=1e-14)


def test_product_matches_dense_all_pairs_n2():
    for (x1, z1), (x2, z2) in itertools.product(all_strings(2), repeat=2):
        e, x3, z3 = pauli.product(x1, z1, x2, z2)
        lhs = pauli.dense(x1, z1, 2) @ pauli.dense(x2, z2, 2)
        assert np.allclose(lhs, (1j ** e) * pauli.dense(x3, z3, 2))


def test_commute_matches_dense():
    for (x1, z1), (x2, z2) in itertools.product(all_strings(2), repeat=2):
        a, b = pauli.dense(x1, z1, 2), pauli.dense(x2, z2, 2)
        assert pauli.commute(x1, z1, x2, z2) == np.allclose(a @ b, b @ a)


def test_strings_are_hermitian_involutions():
    for x, z in all_strings(3):
        m = pauli.dense(x, z, 3)
        assert np.allclose(m, m.conj().T)
        assert np.allclose(m @ m, np.eye(8))


def test_random_pauli_sum_refuses_impossible_counts():
    import pytest
    from workloads import random_pauli_sum
    with pytest.raises(ValueError):
        random_pauli_sum(4, 256, 0)
    x, z, c = random_pauli_sum(4, 255, 0)
    assert len(set(zip(x.tolist(), z.tolist()))) == 255
