"""Pins for the oracle pieces of the NEXT rows: generalized excitations
(UCCGSD, Table 1), rotation lists of any excitation sequence (Eq. 11), the
ADAPT pool gradient (Section 5.1) and the variational loop of Eq. 9."""
import itertools

import numpy as np
import pytest

from oracle import fermion
from oracle import statevector as sv
from paper_2208_10978_amd.vqe import vqe
from workloads import synthetic_integrals, uniform_amplitudes


def brute_generalized(n):
    """Every spin-conserving single and double up to the sign of its
    generator, by enumerating ordered index tuples and canonicalising."""
    spin = lambda q: q % 2
    singles, doubles = set(), set()
    for p, q in itertools.permutations(range(n), 2):
        if spin(p) == spin(q):
            singles.add(tuple(sorted((p, q))))
    for p, q, r, s in itertools.permutations(range(n), 4):
        if sorted((spin(p), spin(q))) == sorted((spin(r), spin(s))):
            a, b = tuple(sorted((p, q))), tuple(sorted((r, s)))
            doubles.add(min(a, b) + max(a, b))
    return singles, doubles


@pytest.mark.parametrize("n", [4, 6, 8])
def test_uccgsd_set_is_every_spin_conserving_operator_once(n):
    singles, doubles = fermion.uccgsd_excitations(n)
    bs, bd = brute_generalized(n)
    assert len(singles) == len(set(singles)) and set(singles) == bs
    assert len(doubles) == len(set(doubles)) and set(doubles) == bd
    m = n // 2
    assert len(singles) == 2 * m * (m - 1) // 2


@pytest.mark.parametrize("n,ne", [(4, 2), (6, 3)])
def test_generalized_rotation_list_equals_fermionic_exponentials(n, ne):
    singles, doubles = fermion.uccgsd_excitations(n)
    seq = singles + doubles
    theta = uniform_amplitudes(len(seq), 0.4, 900 + n)
    basis, phi_f = fermion.ucc_state_fermionic(n, ne, theta, excitations=seq)
    rots = fermion.excitation_rotations(seq)
    psi = sv.apply_rotations(sv.basis_state(n, fermion.hf_index(ne)), [r[0] for r in rots], [r[1] for r in rots],
                             [r[3] * theta[r[2]] for r in rots])
    assert np.abs(psi[basis] - phi_f).max() < 1e-12
    assert np.abs(psi).sum() - np.abs(psi[basis]).sum() < 1e-12


def test_pool_gradient_equals_finite_difference_of_an_appended_operator():
    n, ne = 6, 2
    h, eri = synthetic_integrals(n, 606)
    singles, doubles = fermion.uccsd_excitations(n, ne)
    circ = singles + doubles
    theta = uniform_amplitudes(len(circ), 0.2, 707)
    gs, gd = fermion.uccgsd_excitations(n)
    pool = (gs + gd)[::7]
    g = fermion.pool_gradients(h, eri, n, ne, theta, pool, excitations=circ)
    basis = fermion.sector_basis(n, *fermion.electron_counts(ne))
    H = fermion.determinant_hamiltonian(h, eri, basis)

    def energy(extra, t):
        _, psi = fermion.ucc_state_fermionic(n, ne, list(theta) + [t], basis=basis, excitations=circ + [extra])
        return np.real(np.vdot(psi, H @ psi))
    d = 1e-4
    for k, op in enumerate(pool):
        fd = (-energy(op, 2 * d) + 8 * energy(op, d) - 8 * energy(op, -d) + energy(op, -2 * d)) / (12 * d)
        assert abs(fd - g[k]) <= 1e-8 + 1e-7 * abs(g[k]), (op, fd, g[k])
    assert np.abs(g).max() > 1e-3   # the screening is not trivially zero


def test_uccgsd_vqe_reaches_the_exact_ground_state_at_4_qubits():
    """Two electrons in two spatial orbitals: the four-parameter generalized
    product spans the (1 alpha, 1 beta) sector, so Eq. 9's minimum is the
    exact ground-state energy (the three-parameter UCCSD product does not
    reach it for these integrals)."""
    n, ne = 4, 2
    h, eri = synthetic_integrals(n, 77)
    basis = fermion.sector_basis(n, *fermion.electron_counts(ne))
    H = fermion.determinant_hamiltonian(h, eri, basis).toarray()
    e0 = np.linalg.eigvalsh(H)[0]
    gs, gd = fermion.uccgsd_excitations(n)
    seq = gs + gd

    def fg(th):
        def e(t):
            _, p = fermion.ucc_state_fermionic(n, ne, t, basis=basis, excitations=seq)
            return np.real(np.vdot(p, H @ p))
        eye = np.eye(len(th))
        return e(th), np.array([(e(th + 1e-6 * eye[k]) - e(th - 1e-6 * eye[k])) / 2e-6 for k in range(len(th))])
    best = min(vqe(fg, uniform_amplitudes(len(seq), 1.0, s))["energy"] for s in range(3))
    assert abs(best - e0) < 1e-9


def dense_raise(n, j):
    """|1><0| on qubit j of n (qubit q = bit q of the index), by Kronecker
    products; independent of the Pauli algebra."""
    up = np.array([[0.0, 0.0], [1.0, 0.0]])
    m = np.array([[1.0]])
    for q in range(n - 1, -1, -1):
        m = np.kron(m, up if q == j else np.eye(2))
    return m


@pytest.mark.parametrize("n", [4, 5])
def test_qubit_excitation_rotations_equal_the_dense_exponential(n):
    from scipy.linalg import expm
    singles = [(i, a) for i, a in itertools.combinations(range(n), 2)]
    doubles = [(i, j, a, b) for i, j, a, b in itertools.permutations(range(n), 4) if i < j and a < b][:6]
    seq = singles[:5] + doubles
    theta = uniform_amplitudes(len(seq), 0.6, 1500 + n)
    rots = fermion.qubit_excitation_rotations(seq)
    rng = np.random.default_rng(n)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    got = sv.apply_rotations(psi.copy(), [r[0] for r in rots], [r[1] for r in rots],
                             [r[3] * theta[r[2]] for r in rots])
    ref = psi.copy()
    for t, exc in zip(theta, seq):
        if len(exc) == 2:
            i, a = exc
            T = dense_raise(n, a) @ dense_raise(n, i).T
        else:
            i, j, a, b = exc
            T = dense_raise(n, a) @ dense_raise(n, b) @ dense_raise(n, j).T @ dense_raise(n, i).T
        ref = expm(t * (T - T.T)) @ ref
    assert np.abs(got - ref).max() < 1e-12
    # no Jordan-Wigner tails: every string lives on the excitation's qubits
    for (x, z, p, _), exc in zip(rots, [seq[r[2]] for r in rots]):
        sup = sum(1 << q for q in exc)
        assert x == sup and (z & ~sup) == 0


def test_rotation_pool_gradient_equals_finite_difference():
    n, ne = 6, 2
    h, eri = synthetic_integrals(n, 616)
    terms = fermion.jw_hamiltonian(h, eri)
    hx, hz, hc = [k[0] for k in terms], [k[1] for k in terms], list(terms.values())
    s, d = fermion.uccsd_excitations(n, ne)
    rots = fermion.excitation_rotations(s + d)
    theta = uniform_amplitudes(len(s + d), 0.3, 617)
    psi = sv.apply_rotations(sv.basis_state(n, fermion.hf_index(ne)), [r[0] for r in rots], [r[1] for r in rots],
                             [r[3] * theta[r[2]] for r in rots])
    # odd-Y strings on flip masks of the Hamiltonian, and a few others
    px = [k[0] for k in terms if k[0]][:12] + [0b110000, 0b000111]
    pz = [x & -x for x in px]
    g = sv.rotation_pool_gradients(psi, hx, hz, hc, px, pz)
    dd = 1e-4
    for k, (x, z) in enumerate(zip(px, pz)):
        def e(t):
            p = sv.rotate(psi, x, z, t)
            return sv.expectation(p, hx, hz, hc)[0].real
        fd = (-e(2 * dd) + 8 * e(dd) - 8 * e(-dd) + e(-2 * dd)) / (12 * dd)
        assert abs(fd - g[k]) < 1e-9 + 1e-7 * abs(g[k])
    assert np.abs(g).max() > 1e-3


def test_adapt_loop_with_oracle_callables_reaches_the_exact_ground_state_at_4_qubits():
    """The ADAPT loop (Section 5.1) over the generalized pool, every number
    from the oracle: it stops on a vanishing pool gradient at the exact
    ground-state energy."""
    from paper_2208_10978_amd.problem import uccgsd_rotations
    from paper_2208_10978_amd.vqe import adapt_vqe
    from tests.adapt_oracle import oracle_callables
    n, ne = 4, 2
    h, eri = synthetic_integrals(n, 77)
    basis = fermion.sector_basis(n, *fermion.electron_counts(ne))
    e0 = np.linalg.eigvalsh(fermion.determinant_hamiltonian(h, eri, basis).toarray())[0]
    mk, screen = oracle_callables(h, eri, n, ne)
    res = adapt_vqe(mk, screen, uccgsd_rotations(n), n, max_ops=8, grad_tol=1e-6)
    assert abs(res["energies"][-1] - e0) < 1e-8
    assert res["max_gradients"][-1] < 1e-6 or len(res["chosen"]) == 8
    assert all(b <= a + 1e-12 for a, b in zip(res["energies"], res["energies"][1:]))
