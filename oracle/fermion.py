"""Second quantization on occupation bitstrings (oracle).

Conventions (readings of Sections 3.1-3.2 and 5.1, where the paper is silent):

* Spin orbitals are interleaved: qubit ``2p`` is spatial orbital p with spin
  alpha, qubit ``2p + 1`` the same orbital with spin beta.  Occupation of
  qubit q is bit q of the basis index (Eq. 6 maps occupations to qubits).
* The Hartree-Fock determinant fills the lowest ``n_e`` qubits; for odd
  ``n_e`` that gives one more alpha than beta electron.
* Ladder operators carry the Jordan-Wigner sign of the occupied orbitals
  below them: ``a_j |k> = (-1)^{|k & (2^j - 1)|} |k ^ 2^j>`` when bit j is set.
* The Hamiltonian of Eq. 3 with chemist's-notation integrals (pq|rs) over
  spatial orbitals is ``H = sum_{pq,s} h_pq a+_{ps} a_{qs}
  + 1/2 sum_{pqrs,s,t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}``.
* UCCSD (Eq. 10 with the Trotter product of Eq. 11): spin-orbital singles
  ``tau_ia = a+_a a_i`` and doubles ``tau_ijab = a+_a a+_b a_j a_i``
  (i < j occupied, a < b virtual, total spin projection conserved), one
  amplitude each; singles first, then doubles, both in lexicographic order
  of (i, a) and (i, j, a, b).

Two independent routes are given for every object: direct action on
bitstrings (no Pauli algebra) and the Jordan-Wigner Pauli form built by
multiplying ladder operators with the Pauli algebra of ``oracle.pauli``.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse
import scipy.sparse.linalg

from . import pauli


# ----------------------------------------------------------------------------
# orbitals and excitations
# ----------------------------------------------------------------------------

def spin_of(q: int) -> int:
    return q % 2


def occupied_qubits(n_electrons: int):
    return list(range(n_electrons))


def hf_index(n_electrons: int) -> int:
    return (1 << n_electrons) - 1


def uccsd_excitations(n_qubits: int, n_electrons: int):
    occ = occupied_qubits(n_electrons)
    vir = list(range(n_electrons, n_qubits))
    singles = [(i, a) for i in occ for a in vir if spin_of(i) == spin_of(a)]
    doubles = []
    for i, j in itertools.combinations(occ, 2):
        for a, b in itertools.combinations(vir, 2):
            if sorted((spin_of(i), spin_of(j))) == sorted((spin_of(a), spin_of(b))):
                doubles.append((i, j, a, b))
    return singles, doubles


def uccgsd_excitations(n_qubits: int):
    """Generalized singles and doubles (Table 1's UCCGSD: excitation
    operators that do not tell occupied from virtual orbitals): singles
    ``a+_q a_p`` for p < q of one spin, doubles ``a+_r a+_s a_q a_p`` for
    p < q, r < s, {p, q} and {r, s} disjoint, (p, q) < (r, s), spin
    projection conserved.  Each unordered pair of index pairs appears once
    (the generator of (r, s) -> (p, q) is minus that of (p, q) -> (r, s))."""
    singles = [(p, q) for p, q in itertools.combinations(range(n_qubits), 2) if spin_of(p) == spin_of(q)]
    pairs = list(itertools.combinations(range(n_qubits), 2))
    doubles = []
    for a in range(len(pairs)):
        for b in range(a + 1, len(pairs)):
            (p, q), (r, s) = pairs[a], pairs[b]
            if {p, q} & {r, s}:
                continue
            if sorted((spin_of(p), spin_of(q))) == sorted((spin_of(r), spin_of(s))):
                doubles.append((p, q, r, s))
    return singles, doubles


def excitation_ops(exc):
    """Ladder-operator word of tau, rightmost applied first: list of
    ``(qubit, is_creation)`` in left-to-right order."""
    if len(exc) == 2:
        i, a = exc
        return [(a, True), (i, False)]
    i, j, a, b = exc
    return [(a, True), (b, True), (j, False), (i, False)]


# ----------------------------------------------------------------------------
# route 1: operators acting on bitstrings
# ----------------------------------------------------------------------------

def apply_word(word, states: np.ndarray):
    """Apply a word of ladder operators (rightmost first) to an array of
    basis indices.  Returns ``(new_states, signs)``; sign 0 means the
    result vanishes."""
    k = states.astype(np.int64).copy()
    sign = np.ones(k.shape, dtype=np.int64)
    for q, create in reversed(word):
        bit = (k >> q) & 1
        below = np.bitwise_count(k & ((1 << q) - 1)).astype(np.int64)
        ok = (bit == 0) if create else (bit == 1)
        sign = sign * np.where(ok, 1 - 2 * (below & 1), 0)
        k = k ^ (1 << q)
    return k, sign


def _matrix_from_words(words_coefs, basis: np.ndarray):
    pos = {int(s): t for t, s in enumerate(basis)}
    dim = len(basis)
    rows, cols, vals = [], [], []
    for word, coef in words_coefs:
        out, sg = apply_word(word, basis)
        for t in np.nonzero(sg)[0]:
            o = int(out[t])
            if o in pos:
                rows.append(pos[o])
                cols.append(t)
                vals.append(coef * sg[t])
    return scipy.sparse.coo_matrix((vals, (rows, cols)), shape=(dim, dim)).tocsr()


def hamiltonian_words(h: np.ndarray, eri: np.ndarray):
    """The terms of Eq. 3 as (ladder word, coefficient) pairs."""
    M = h.shape[0]
    words = []
    for p in range(M):
        for q in range(M):
            if h[p, q] != 0.0:
                for s in (0, 1):
                    words.append(([(2 * p + s, True), (2 * q + s, False)], float(h[p, q])))
    for p, q, r, s_ in itertools.product(range(M), repeat=4):
        v = eri[p, q, r, s_]
        if v == 0.0:
            continue
        for sg in (0, 1):
            for tg in (0, 1):
                P, Q, R, S = 2 * p + sg, 2 * q + sg, 2 * r + tg, 2 * s_ + tg
                if P == R or Q == S:
                    continue
                words.append(([(P, True), (R, True), (S, False), (Q, False)], 0.5 * float(v)))
    return words


def determinant_hamiltonian(h, eri, basis) -> scipy.sparse.csr_matrix:
    """H of Eq. 3 as a sparse matrix over the given basis indices, built by
    applying ladder operators to bitstrings (no Pauli algebra)."""
    return _matrix_from_words(hamiltonian_words(h, eri), np.asarray(basis, dtype=np.int64))


def sector_basis(n_qubits: int, n_alpha: int, n_beta: int) -> np.ndarray:
    ks = np.arange(1 << n_qubits, dtype=np.int64)
    a_mask = sum(1 << q for q in range(0, n_qubits, 2))
    b_mask = sum(1 << q for q in range(1, n_qubits, 2))
    na = np.bitwise_count(ks & a_mask)
    nb = np.bitwise_count(ks & b_mask)
    return ks[(na == n_alpha) & (nb == n_beta)]


def electron_counts(n_electrons: int):
    return (n_electrons + 1) // 2, n_electrons // 2


def generator_matrix(exc, basis) -> scipy.sparse.csr_matrix:
    """``tau - tau^dagger`` over the basis, from bitstring action."""
    word = excitation_ops(exc)
    dag = [(q, not c) for q, c in reversed(word)]
    return _matrix_from_words([(word, 1.0), (dag, -1.0)], np.asarray(basis, dtype=np.int64))


def checked_order(n_qubits: int, n_electrons: int, order=None):
    """The excitation sequence to apply: lexicographic by default, or a given
    sequence, which must be a permutation of the UCCSD excitation set."""
    singles, doubles = uccsd_excitations(n_qubits, n_electrons)
    if order is None:
        return singles + doubles
    order = [tuple(int(v) for v in e) for e in order]
    if len(order) != len(singles) + len(doubles) or set(order) != set(singles + doubles):
        raise ValueError("the excitation sequence is not a permutation of the UCCSD excitations")
    return order


def ucc_state_fermionic(n_qubits: int, n_electrons: int, theta, basis=None, order=None, excitations=None):
    """``prod_i exp(theta_i (tau_i - tau_i^dag)) |HF>`` in excitation order,
    each factor a sparse matrix exponential.  ``excitations`` (any sequence of
    singles (i, a) and doubles (i, j, a, b)) replaces the UCCSD sequence.
    Returns (basis, coefficients)."""
    if basis is None:
        basis = sector_basis(n_qubits, *electron_counts(n_electrons))
    basis = np.asarray(basis, dtype=np.int64)
    psi = np.zeros(len(basis), dtype=np.complex128)
    psi[int(np.nonzero(basis == hf_index(n_electrons))[0][0])] = 1.0
    seq = checked_order(n_qubits, n_electrons, order) if excitations is None else [tuple(e) for e in excitations]
    for exc, th in zip(seq, theta):
        g = generator_matrix(exc, basis)
        psi = scipy.sparse.linalg.expm_multiply(float(th) * g, psi)
    return basis, psi


def slater_condon_hf_energy(h, eri, n_electrons: int) -> float:
    """Hartree-Fock determinant energy: one-electron diagonal plus Coulomb
    minus same-spin exchange, summed over occupied spin orbitals."""
    occ = occupied_qubits(n_electrons)
    e = 0.0
    for i in occ:
        e += h[i // 2, i // 2]
    for i in occ:
        for j in occ:
            p, r = i // 2, j // 2
            e += 0.5 * eri[p, p, r, r]
            if spin_of(i) == spin_of(j):
                e -= 0.5 * eri[p, r, r, p]
    return float(e)


# ----------------------------------------------------------------------------
# route 2: Jordan-Wigner by Pauli algebra
# ----------------------------------------------------------------------------

def ladder_pauli(j: int, create: bool):
    """``a_j = Z_{<j} (X_j + i Y_j)/2``, ``a+_j = Z_{<j} (X_j - i Y_j)/2``."""
    low = (1 << j) - 1
    return {(1 << j, low): 0.5, (1 << j, low | (1 << j)): (-0.5j if create else 0.5j)}


def poly_mul(a: dict, b: dict) -> dict:
    out: dict = {}
    for (x1, z1), c1 in a.items():
        for (x2, z2), c2 in b.items():
            e, x3, z3 = pauli.product(x1, z1, x2, z2)
            out[(x3, z3)] = out.get((x3, z3), 0) + c1 * c2 * (1j ** e)
    return out


def qubit_ladder_pauli(j: int, create: bool):
    """Qubit ladder without a string: ``Q_j = (X_j + i Y_j)/2`` lowers qubit j
    (|1> -> |0>), ``Q+_j = (X_j - i Y_j)/2`` raises it."""
    return {(1 << j, 0): 0.5, (1 << j, 1 << j): (-0.5j if create else 0.5j)}


def word_pauli(word, ladder=ladder_pauli) -> dict:
    poly = {(0, 0): 1.0 + 0j}
    for q, create in word:
        poly = poly_mul(poly, ladder(q, create))
    return poly


def jw_hamiltonian(h, eri, drop_tol: float = 1e-12):
    """Pauli form of Eq. 3: dict ``{(x, z): real coefficient}``."""
    acc: dict = {}
    for word, coef in hamiltonian_words(h, eri):
        for key, c in word_pauli(word).items():
            acc[key] = acc.get(key, 0) + coef * c
    out = {}
    for key, c in acc.items():
        if abs(c.imag) > 1e-10:
            raise AssertionError("non-Hermitian JW coefficient")
        if abs(c.real) > drop_tol:
            out[key] = float(c.real)
    return out


def truncate(terms: dict, threshold: float) -> dict:
    """Keep terms with |c| strictly above the threshold, and the identity."""
    return {k: c for k, c in terms.items() if abs(c) > threshold or k == (0, 0)}


def uccsd_rotations(n_qubits: int, n_electrons: int, order=None):
    """Rotation list of the Trotterised UCCSD circuit (Eq. 11), excitations in
    the given sequence (lexicographic by default); parameter i is the i-th
    excitation of the sequence.  See ``excitation_rotations``."""
    return excitation_rotations(checked_order(n_qubits, n_electrons, order))


def qubit_excitation_rotations(excitations, first_param: int = 0):
    """Qubit-excitation-based operators (Section 5.1): the rotation list of
    ``prod_i exp(theta_i (T_i - T_i^dag))`` where ``T_i`` is the excitation's
    word with qubit ladders (``qubit_ladder_pauli``) in place of fermionic
    ones, so no Jordan-Wigner strings.  Same output form as
    ``excitation_rotations``."""
    return excitation_rotations(excitations, first_param, ladder=qubit_ladder_pauli)


def excitation_rotations(excitations, first_param: int = 0, ladder=ladder_pauli):
    """Rotation list of ``prod_i exp(theta_i (tau_i - tau_i^dag))`` (Eq. 11)
    for any sequence of excitations; parameter ``first_param + i`` is the
    i-th excitation.

    ``tau - tau^dag = i sum_j c_j P_j`` with real c_j, so
    ``exp(theta (tau - tau^dag)) = prod_j R(P_j, -2 c_j theta)``; the strings
    of one excitation commute and are listed by increasing z mask.
    Returns a list of ``(x, z, param_index, dphi_dtheta)``."""
    out = []
    for pos, exc in enumerate(excitations):
        idx = first_param + pos
        word = excitation_ops(exc)
        dag = [(q, not c) for q, c in reversed(word)]
        poly = word_pauli(word, ladder)
        for k, v in word_pauli(dag, ladder).items():
            poly[k] = poly.get(k, 0) - v
        strings = []
        for (x, z), g in poly.items():
            if abs(g) < 1e-14:
                continue
            if abs(g.real) > 1e-14:
                raise AssertionError("generator term not anti-Hermitian")
            strings.append((x, z, g.imag))
        for x, z, c in sorted(strings, key=lambda t: t[1]):
            out.append((x, z, idx, -2.0 * c))
    return out


def pool_gradients(h, eri, n_qubits: int, n_electrons: int, theta, pool, excitations=None):
    """ADAPT operator-pool screening (Section 5.1): for each pool
    operator A = tau - tau^dag appended after the circuit with amplitude 0,
    dE/dtheta_A = <psi|[H, A]|psi> = 2 Re <psi|H A|psi>, from the
    determinant-space H and A (bitstring action, no Pauli algebra)."""
    basis = sector_basis(n_qubits, *electron_counts(n_electrons))
    _, psi = ucc_state_fermionic(n_qubits, n_electrons, theta, basis=basis, excitations=excitations)
    hpsi = determinant_hamiltonian(h, eri, basis) @ psi
    return np.array([2.0 * np.real(np.vdot(hpsi, generator_matrix(exc, basis) @ psi)) for exc in pool])


def hamiltonian_on_basis_state(h, eri, k: int) -> dict:
    """``H |k>`` as ``{k': <k'|H|k>}``, by bitstring action; works at any
    qubit count because it never forms a 2^n vector."""
    out: dict = {}
    state = np.array([int(k)], dtype=np.int64)
    for word, coef in hamiltonian_words(h, eri):
        kk, sg = apply_word(word, state)
        if sg[0] != 0:
            key = int(kk[0])
            out[key] = out.get(key, 0.0) + coef * int(sg[0])
    return out


def excited_determinant(exc, n_electrons: int):
    """``tau |HF> = sign |k>``; returns ``(k, sign)``."""
    kk, sg = apply_word(excitation_ops(exc), np.array([hf_index(n_electrons)], dtype=np.int64))
    return int(kk[0]), int(sg[0])
