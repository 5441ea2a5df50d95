"""Excitation sequences of the Trotterised UCCSD ansatz (input data).

The paper's Trotter product (Section 5.1, Eq. 11) fixes which excitations
appear but not their order, and the order changes the state.  The sequence is
therefore an input that the oracle and the GPU path both consume.  Two
sequences are provided; both list every spin-conserving single (i, a) first,
then every double (i, j, a, b) with i < j occupied and a < b virtual, under
interleaved spin orbitals (qubit 2p alpha, 2p + 1 beta) with the lowest n_e
qubits occupied:

* ``"lex"``   lexicographic order of (i, a) and (i, j, a, b);
* ``"tile"``  tile-major order.  Tiles are (L u O_t, V_t) with L the lowest
  ``low`` qubits, O_t a ``occ_block``-set of the other occupied qubits and V_t
  a ``vir_block``-set of virtual qubits, so a tile spans at most
  low + occ_block + vir_block qubits.  The sets O_t come from a greedy pair
  covering of the occupied qubits above L (every pair and every single qubit
  lies in some O_t), the sets V_t from a greedy pair covering of the virtual
  qubits; tiles run over O_t (outer) and V_t (inner).  Each excitation is
  listed with the first tile that contains all of its qubits, in
  lexicographic order within a tile.  Consecutive excitations then share few
  qubits beyond one tile, which is what lets an LDS-tiled sweep apply many of
  them per pass over the state.

Greedy covering: among all k-subsets in lexicographic order, repeatedly take
the first one that covers the most uncovered pairs and single points.
"""
from __future__ import annotations

import itertools


def _singles_doubles(n_qubits: int, n_electrons: int):
    occ = range(n_electrons)
    vir = range(n_electrons, n_qubits)
    singles = [(i, a) for i in occ for a in vir if i % 2 == a % 2]
    doubles = [(i, j, a, b)
               for i, j in itertools.combinations(occ, 2)
               for a, b in itertools.combinations(vir, 2)
               if sorted((i % 2, j % 2)) == sorted((a % 2, b % 2))]
    return singles, doubles


def greedy_pair_cover(points, k: int):
    pts = list(points)
    if len(pts) <= k:
        return [tuple(pts)]
    need = set(itertools.combinations(pts, 2)) | {(p,) for p in pts}
    cands = list(itertools.combinations(pts, k))
    sets = []
    while need:
        best, best_n = None, -1
        for s in cands:
            ss = set(s)
            cnt = sum(1 for e in need if ss.issuperset(e))
            if cnt > best_n:
                best, best_n = s, cnt
        sets.append(best)
        bs = set(best)
        need = {e for e in need if not bs.issuperset(e)}
    return sets


def uccsd_excitation_order(n_qubits: int, n_electrons: int, order: str = "tile", low: int = 3,
                           occ_block: int = 5, vir_block: int = 4):
    """List of excitations in application order: tuples (i, a) then (i, j, a, b)."""
    singles, doubles = _singles_doubles(n_qubits, n_electrons)
    if order == "lex":
        return singles + doubles
    if order != "tile":
        raise ValueError(order)
    occ = list(range(n_electrons))
    vir = list(range(n_electrons, n_qubits))
    lowq = [q for q in occ if q < low]
    rest = [q for q in occ if q >= low]
    co = greedy_pair_cover(rest, occ_block) if rest else [()]
    cv = greedy_pair_cover(vir, vir_block) if vir else [()]
    tiles = [(set(lowq) | set(a), set(b)) for a in co for b in cv]
    out = []
    for group in (singles, doubles):
        seen = set()
        for ot, vt in tiles:
            for e in group:
                if e in seen:
                    continue
                half = len(e) // 2
                if set(e[:half]) <= ot and set(e[half:]) <= vt:
                    seen.add(e)
                    out.append(e)
        if len(seen) != len(group):
            raise AssertionError("tiles do not cover every excitation")
    return out
