"""Host-side problem builders: the Jordan-Wigner Pauli-sum Hamiltonian and
the Trotterised UCCSD rotation list, as packed ``uint64`` masks.

Conventions (the paper leaves them open; Sections 3.1-3.2, 5.1):

* qubit q is bit q of a basis index; spin orbital ``(p, alpha)`` is qubit
  ``2p`` and ``(p, beta)`` is ``2p + 1``; the Hartree-Fock determinant fills
  the lowest ``n_e`` qubits (Eq. 6), so its index is ``2^n_e - 1``;
* the Hamiltonian of Eq. 3 with chemist's-notation integrals is
  ``sum h_pq a+_ps a_qs + 1/2 sum (pq|rs) a+_ps a+_rt a_st a_qs``;
* JW: ``a_j = Z_{<j} (X_j + i Y_j)/2``;
* UCCSD (Eq. 10-11): singles ``a+_a a_i`` and doubles ``a+_a a+_b a_j a_i``
  (i < j occupied, a < b virtual, spin projection conserved), applied in a
  given excitation sequence (by default the tile-major sequence of
  ``workloads.uccsd_excitation_order``); ``tau - tau^dag = i sum_j c_j P_j``
  and the factor ``exp(theta (tau - tau^dag))`` becomes the commuting
  rotations ``R(P_j, phi_j)``, ``phi_j = -2 c_j theta``, listed by increasing z.

The Pauli algebra here works on whole arrays of strings at once: a ladder
word of length L expands into 2^L strings, multiplied factor by factor with
the symplectic phase rule, then equal strings are merged.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np


def _popc(a: np.ndarray) -> np.ndarray:
    return np.bitwise_count(a).astype(np.int64)


@dataclass
class PauliSum:
    """``H = sum_t c_t P_t`` with ``P = i^{|x&z|} X^x Z^z`` and real c."""
    n_qubits: int
    x: np.ndarray  # uint64
    z: np.ndarray  # uint64
    c: np.ndarray  # float64

    def __len__(self):
        return int(self.x.shape[0])

    def truncated(self, threshold: float) -> "PauliSum":
        keep = (np.abs(self.c) > threshold) | ((self.x == 0) & (self.z == 0))
        return PauliSum(self.n_qubits, self.x[keep], self.z[keep], self.c[keep])

    @property
    def n_groups(self) -> int:
        return int(np.unique(self.x).shape[0])

    def one_norm(self) -> float:
        return float(np.abs(self.c).sum())


@dataclass
class RotationList:
    """Rotations ``R(P_k, phi_k) = exp(-i phi_k P_k / 2)`` applied in order;
    ``phi_k = dphi_dtheta[k] * theta[param[k]]``."""
    n_qubits: int
    x: np.ndarray
    z: np.ndarray
    param: np.ndarray        # int32
    dphi_dtheta: np.ndarray  # float64
    n_params: int

    def __len__(self):
        return int(self.x.shape[0])

    def angles(self, theta) -> np.ndarray:
        theta = np.asarray(theta, dtype=np.float64)
        return self.dphi_dtheta * theta[self.param]


def _expand_words(qubits: np.ndarray, create: np.ndarray, coef: np.ndarray, jw: bool = True):
    """Pauli expansion of ladder words.  ``qubits``/``create`` are (W, L);
    word w is ``op[w,0] op[w,1] ... op[w,L-1]``.  Each factor is
    ``(X_j Z_{<j} -/+ i Y_j Z_{<j}) / 2`` (creation takes the minus sign);
    with ``jw=False`` the qubit ladder ``(X_j -/+ i Y_j) / 2`` (no Z string).

    The running product is kept as ``i^ph X^x Z^z``; ``Y_j = i X_j Z_j`` adds
    one to ph and moving ``Z^z`` past ``X^{x'}`` adds ``2 |z & x'|``.  At the
    end ``X^x Z^z = i^{-|x & z|} P`` gives the canonical string.
    Returns x, z (uint64) and complex coefficients of the W * 2^L strings."""
    W, L = qubits.shape
    one = np.uint64(1)
    x = np.zeros(W, dtype=np.uint64)
    z = np.zeros(W, dtype=np.uint64)
    ph = np.zeros(W, dtype=np.int64)
    amp = coef.astype(np.complex128) * (0.5 ** L)
    for t in range(L):
        q = qubits[:, t].astype(np.uint64)
        bit = one << q
        low = bit - one
        fx = np.concatenate([bit, bit])
        if not jw:
            low = np.zeros_like(bit)
        fz = np.concatenate([low, low | bit])
        fph = np.concatenate([np.zeros(len(q), np.int64), np.ones(len(q), np.int64)])
        famp = np.concatenate([np.ones(len(q)), np.where(create[:, t], -1j, 1j)])
        x, z, ph, amp = (np.concatenate([x, x]), np.concatenate([z, z]),
                         np.concatenate([ph, ph]), np.concatenate([amp, amp]) * famp)
        ph = ph + fph + 2 * _popc(z & fx)
        x, z = x ^ fx, z ^ fz
        qubits = np.concatenate([qubits, qubits])
        create = np.concatenate([create, create])
    ph = ph - _popc(x & z)
    return x, z, amp * (1j ** (ph % 4))


def _merge(x, z, c, n_qubits, drop_tol):
    order = np.lexsort((z, x))
    x, z, c = x[order], z[order], c[order]
    new = np.ones(x.shape[0], dtype=bool)
    new[1:] = (x[1:] != x[:-1]) | (z[1:] != z[:-1])
    idx = np.cumsum(new) - 1
    summed = np.zeros(int(idx[-1]) + 1 if len(idx) else 0, dtype=np.complex128)
    np.add.at(summed, idx, c)
    ux, uz = x[new], z[new]
    return ux, uz, summed


def jordan_wigner(h: np.ndarray, eri: np.ndarray, drop_tol: float = 1e-12) -> PauliSum:
    """JW Pauli sum of Eq. 3 for spatial integrals ``h`` (M, M) and chemist's
    ``eri`` (M, M, M, M) on ``n = 2M`` qubits."""
    M = h.shape[0]
    n = 2 * M
    if n > 64:
        raise ValueError("at most 64 qubits")
    xs, zs, cs = [], [], []
    # one-body words a+_{ps} a_{qs}
    pq = np.array([(p, q, s) for p in range(M) for q in range(M) for s in (0, 1) if h[p, q] != 0.0])
    if len(pq):
        qub = np.stack([2 * pq[:, 0] + pq[:, 2], 2 * pq[:, 1] + pq[:, 2]], axis=1)
        cre = np.tile(np.array([True, False]), (len(pq), 1))
        x, z, c = _expand_words(qub, cre, h[pq[:, 0], pq[:, 1]])
        xs.append(x); zs.append(z); cs.append(c)
    # two-body words a+_{ps} a+_{rt} a_{st} a_{qs}, weight (pq|rs)/2
    p, q, r, s = (a.ravel() for a in np.meshgrid(*(np.arange(M),) * 4, indexing="ij"))
    v = eri[p, q, r, s]
    nz = v != 0.0
    p, q, r, s, v = p[nz], q[nz], r[nz], s[nz], v[nz]
    for sg, tg in itertools.product((0, 1), repeat=2):
        P, Q, R, S = 2 * p + sg, 2 * q + sg, 2 * r + tg, 2 * s + tg
        ok = (P != R) & (Q != S)
        qub = np.stack([P[ok], R[ok], S[ok], Q[ok]], axis=1)
        cre = np.tile(np.array([True, True, False, False]), (int(ok.sum()), 1))
        x, z, c = _expand_words(qub, cre, 0.5 * v[ok])
        xs.append(x); zs.append(z); cs.append(c)
    x, z, c = _merge(np.concatenate(xs), np.concatenate(zs), np.concatenate(cs), n, drop_tol)
    if np.abs(c.imag).max(initial=0.0) > 1e-10:
        raise AssertionError("JW Hamiltonian has a non-real coefficient")
    keep = np.abs(c.real) > drop_tol
    return PauliSum(n, x[keep], z[keep], c.real[keep].copy())


def uccsd_excitations(n_qubits: int, n_electrons: int):
    occ = range(n_electrons)
    vir = range(n_electrons, n_qubits)
    singles = [(i, a) for i in occ for a in vir if i % 2 == a % 2]
    doubles = [(i, j, a, b)
               for i, j in itertools.combinations(occ, 2)
               for a, b in itertools.combinations(vir, 2)
               if sorted((i % 2, j % 2)) == sorted((a % 2, b % 2))]
    return singles, doubles


def uccsd_rotations(n_qubits: int, n_electrons: int, order="tile") -> RotationList:
    """``order``: "tile", "lex" or an explicit excitation sequence."""
    if isinstance(order, str):
        from workloads import uccsd_excitation_order
        seq = uccsd_excitation_order(n_qubits, n_electrons, order)
    else:
        seq = [tuple(int(v) for v in e) for e in order]
    singles, doubles = uccsd_excitations(n_qubits, n_electrons)
    if len(seq) != len(singles) + len(doubles) or set(seq) != set(singles + doubles):
        raise ValueError("the excitation sequence is not a permutation of the UCCSD excitations")
    return excitation_rotations(n_qubits, seq)


def uccgsd_excitations(n_qubits: int):
    """Generalized singles (p -> q, p < q, one spin) and doubles
    ((p, q) -> (r, s), p < q, r < s, disjoint pairs, (p, q) < (r, s), spin
    projection conserved): the UCCGSD operators of Table 1, which do not tell
    occupied from virtual orbitals."""
    singles = [(p, q) for p, q in itertools.combinations(range(n_qubits), 2) if p % 2 == q % 2]
    pairs = list(itertools.combinations(range(n_qubits), 2))
    doubles = [(p, q, r, s)
               for k, (p, q) in enumerate(pairs) for (r, s) in pairs[k + 1:]
               if not ({p, q} & {r, s}) and sorted((p % 2, q % 2)) == sorted((r % 2, s % 2))]
    return singles, doubles


def uccgsd_rotations(n_qubits: int) -> RotationList:
    """Trotterised UCCGSD: generalized singles, then doubles."""
    singles, doubles = uccgsd_excitations(n_qubits)
    return excitation_rotations(n_qubits, singles + doubles)


def excitation_rotations(n_qubits: int, seq) -> RotationList:
    """Rotation list of ``prod_i exp(theta_i (tau_i - tau_i^dag))`` (Eq. 11) for
    a sequence of excitations: singles (i, a) with ``tau = a+_a a_i`` and
    doubles (i, j, a, b) with ``tau = a+_a a+_b a_j a_i``; parameter i is the
    i-th excitation.  ``tau - tau^dag = i sum_j c_j P_j``, so the factor is
    ``prod_j R(P_j, -2 c_j theta)``; the strings of one excitation commute and
    are listed by increasing z."""
    return _generator_rotations(n_qubits, seq, True)


def qeb_rotations(n_qubits: int, seq) -> RotationList:
    """Qubit-excitation-based operators (Section 5.1): as
    ``excitation_rotations`` with the qubit ladder ``Q+_j = (X_j - i Y_j)/2``,
    ``Q_j = (X_j + i Y_j)/2`` in place of the fermionic one, so the strings
    carry no Jordan-Wigner Z tails (2 strings per single, 8 per double, on the
    excitation's own qubits only)."""
    return _generator_rotations(n_qubits, seq, False)


def operator_of(pool: RotationList, k: int, new_param: int) -> RotationList:
    """The rotations of pool operator (parameter) k, renumbered to new_param."""
    sel = pool.param == k
    return RotationList(pool.n_qubits, pool.x[sel].copy(), pool.z[sel].copy(),
                        np.full(int(sel.sum()), new_param, dtype=np.int32), pool.dphi_dtheta[sel].copy(),
                        new_param + 1)


def concat_rotations(a: RotationList, b: RotationList) -> RotationList:
    """a then b; b's parameters follow a's."""
    return RotationList(a.n_qubits, np.concatenate([a.x, b.x]), np.concatenate([a.z, b.z]),
                        np.concatenate([a.param, b.param + a.n_params]).astype(np.int32),
                        np.concatenate([a.dphi_dtheta, b.dphi_dtheta]), a.n_params + b.n_params)


def empty_rotations(n_qubits: int) -> RotationList:
    return RotationList(n_qubits, np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0, np.int32),
                        np.zeros(0, np.float64), 0)


def pauli_entangler_rotations(n_qubits: int, x, z) -> RotationList:
    """One parameter per Pauli string: ``exp(-i theta_k P_k / 2)`` in order
    (the Pauli entanglers of Section 5.1)."""
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    k = len(x)
    return RotationList(n_qubits, x, z, np.arange(k, dtype=np.int32), np.ones(k), k)


def entangler_pool(ham: PauliSum, max_weight: int = 4):
    """A Pauli-entangler pool from the Hamiltonian's flip masks: for every
    distinct nonzero x of its strings with at most ``max_weight`` flipped
    qubits, the string with Y on the lowest flipped qubit and X on the others
    (an odd number of Y, so its rotation keeps real amplitudes real).
    Returns (x, z) arrays, x ascending."""
    xs = np.unique(np.asarray(ham.x, dtype=np.uint64))
    xs = xs[(xs != 0) & (_popc(xs) <= max_weight)]
    return xs, xs & (~xs + np.uint64(1))


def _generator_rotations(n_qubits: int, seq, jw: bool) -> RotationList:
    seq = [tuple(int(v) for v in e) for e in seq]
    xs, zs, ps, ds = [], [], [], []
    for idx, exc in enumerate(seq):
        if len(exc) == 2:
            i, a = exc
            word = [(a, True), (i, False)]
        else:
            i, j, a, b = exc
            word = [(a, True), (b, True), (j, False), (i, False)]
        dag = [(q, not cr) for q, cr in reversed(word)]
        qub = np.array([[q for q, _ in word], [q for q, _ in dag]])
        cre = np.array([[cr for _, cr in word], [cr for _, cr in dag]])
        x, z, c = _expand_words(qub, cre, np.array([1.0, -1.0]), jw)
        x, z, c = _merge(x, z, c, n_qubits, 0.0)
        keep = np.abs(c) > 1e-14
        x, z, c = x[keep], z[keep], c[keep]
        if np.abs(c.real).max(initial=0.0) > 1e-14:
            raise AssertionError("excitation generator is not anti-Hermitian")
        order = np.argsort(z, kind="stable")
        xs.append(x[order]); zs.append(z[order])
        ps.append(np.full(len(order), idx, dtype=np.int32))
        ds.append(-2.0 * c.imag[order])
    if not seq:
        return RotationList(n_qubits, np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0, np.int32),
                            np.zeros(0, np.float64), 0)
    return RotationList(n_qubits, np.concatenate(xs), np.concatenate(zs), np.concatenate(ps),
                        np.concatenate(ds), len(seq))
