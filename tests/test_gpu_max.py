"""33 qubits, complex64 (64 GiB): amplitude indices past 2^32, where any
32-bit index arithmetic would show.  Exact pins that need no full-state
oracle:

* Starting from a basis state with qubit 32 set, K rotations leave at most
  2^K nonzero amplitudes (the closure of the start index under the flip
  masks), which the host computes in FP64 (tests/sparse_host.py).  Every one
  of them, and a sample of other indices (zero), must match the GPU's up to
  the complex64 rounding of the K rotations.
* The expectation of a Pauli sum on a basis state keeps only its diagonal
  (x = 0) strings: sum_t c_t (-1)^{|k & z_t|} (Eq. 2 on a determinant)."""
import numpy as np
import pytest
import torch

from oracle import pauli
from paper_2208_10978_amd.engine import StateVector
from tests.gpu_common import announce
from tests.sparse_host import closure, rotate_sparse
from workloads import random_pauli_sum

pytestmark = pytest.mark.gpu

N = 33


def rotations_through_the_top_qubits(count, seed):
    """Weight-4 strings on uniform qubits, every other one forced onto qubit
    32 or 31 so that pairs straddle index 2^32; random X/Y/Z per qubit with at
    least one X or Y."""
    rng = np.random.default_rng(seed)
    xs, zs = [], []
    while len(xs) < count:
        qs = set(int(q) for q in rng.choice(N, size=4, replace=False))
        if len(xs) % 2 == 0:
            qs = set(list(qs)[:3]) | {32 if len(xs) % 4 == 0 else 31}
        x = z = 0
        for q in qs:
            kind = int(rng.integers(0, 3))  # 0 = X, 1 = Y, 2 = Z
            if kind in (0, 1):
                x |= 1 << q
            if kind in (1, 2):
                z |= 1 << q
        if x == 0:
            continue
        xs.append(x)
        zs.append(z)
    phi = rng.uniform(-1.0, 1.0, size=count)
    return np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64), phi


def test_rotations_and_expectation_past_index_2_32():
    announce("33-qubit complex64: rotations and expectation past index 2^32")
    k0 = (1 << 32) | (1 << 30) | 0x0F0F_00FF
    s = StateVector(N, "c64")
    try:
        s.prepare_hf(k0)
        hx, hz, hc = random_pauli_sum(N, 300, 3333)
        e = s.expect_terms(hx, hz, hc).cpu().numpy()
        want = sum(float(c) * (-1) ** pauli.popcount(k0 & int(zz)) for xx, zz, c in zip(hx, hz, hc) if int(xx) == 0)
        assert abs(e[1] - 1.0) < 1e-12
        assert abs(e[0] - want) <= 1e-12 * float(np.abs(hc).sum())

        x, z, phi = rotations_through_the_top_qubits(10, 3334)
        s.apply_rotations(x, z, phi)
        amp = {j: (1.0 + 0j if j == k0 else 0j) for j in closure(k0, x)}
        for xx, zz, pp in zip(x, z, phi):
            amp = rotate_sparse(amp, xx, zz, pp)
        support = sorted(amp)
        assert max(support) >= 1 << 32 and min(support) < 1 << 32
        rng = np.random.default_rng(3335)
        others = [int(v) for v in rng.integers(0, 1 << N, size=64, dtype=np.uint64) if int(v) not in amp]
        got = s.amplitudes(support + others).cpu().numpy()
        got = got[0::2] + 1j * got[1::2]
        for j, g in zip(support, got[:len(support)]):
            assert abs(g - amp[j]) <= 4e-6, (hex(j), g, amp[j])
        assert np.all(got[len(support):] == 0)
        norm = sum(abs(v) ** 2 for v in got[:len(support)])
        assert abs(norm - 1.0) < 1e-5
    finally:
        s.free()
        del s
        torch.cuda.empty_cache()
