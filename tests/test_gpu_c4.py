"""The raw-sweep workload at full size (32 qubits, complex64, 32 GiB): exact
pins that need no full-state oracle.

* A rotation changes an amplitude from itself and its partner only, so after
  a batch of K rotations an amplitude depends on at most 2^K amplitudes
  before the batch (its closure under XOR with the batch's flip masks).
  Gathering those pre-values and applying the batch to them on the host in
  FP64 reproduces the GPU's amplitude up to the complex64 rounding of the
  batch, whatever fusion the GPU used.
* The expectation of a Pauli sum on a basis state keeps only its diagonal
  (x = 0) strings: sum_t c_t (-1)^{|k & z_t|}."""
import numpy as np
import pytest
import torch

from oracle import pauli
from oracle import statevector as osv
from paper_2208_10978_amd.engine import Hamiltonian, StateVector
from paper_2208_10978_amd.problem import PauliSum
from tests.gpu_common import announce
from tests.sparse_host import closure, rotate_sparse
from workloads import random_pauli_sum, random_rotations

N = 32


def test_sparse_helper_matches_the_oracle_rotation():
    n = 6
    rng = np.random.default_rng(1)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    x, z, phi = random_rotations(n, 3, 11)
    ref = osv.apply_rotations(psi.copy(), x, z, phi)
    amp = {j: psi[j] for j in range(1 << n)}
    for xx, zz, pp in zip(x, z, phi):
        amp = rotate_sparse(amp, xx, zz, pp)
    assert max(abs(amp[j] - ref[j]) for j in range(1 << n)) < 1e-14


@pytest.fixture(scope="module")
def state32():
    s = StateVector(N, "c64")
    yield s
    s.free()
    torch.cuda.empty_cache()


@pytest.mark.gpu
def test_rotation_batch_against_sampled_host_recomputation(state32):
    announce("32-qubit rotation batch, sampled recomputation")
    s = state32
    x, z, phi = random_rotations(N, 208, 4242)
    hf = (1 << 16) - 1
    s.prepare_hf(hf)
    s.apply_rotations(x[:200], z[:200], phi[:200])
    bx, bz, bp = x[200:], z[200:], phi[200:]
    rng = np.random.default_rng(4242)
    # indices with sizeable amplitudes (HF moved by a few prefix flips) and uniform ones
    samples = []
    for _ in range(48):
        m = hf
        for k in rng.choice(200, size=int(rng.integers(1, 4)), replace=False):
            m ^= int(x[k])
        samples.append(m)
    samples += [int(v) for v in rng.integers(0, 1 << N, size=16, dtype=np.uint64)]
    pre_idx = sorted(set().union(*[closure(m, bx) for m in samples]))
    pre = s.amplitudes(pre_idx).cpu().numpy()
    pre = dict(zip(pre_idx, pre[0::2] + 1j * pre[1::2]))
    s.apply_rotations(bx, bz, bp)
    post = s.amplitudes(samples).cpu().numpy()
    post = post[0::2] + 1j * post[1::2]
    scale = max(abs(v) for v in pre.values())
    assert scale > 1e-3
    for m, got in zip(samples, post):
        amp = {j: pre[j] for j in closure(m, bx)}
        for xx, zz, pp in zip(bx, bz, bp):
            amp = rotate_sparse(amp, xx, zz, pp)
        assert abs(got - amp[m]) <= 1e-6 * scale, (m, got, amp[m])


@pytest.mark.gpu
def test_expectation_on_a_basis_state(state32):
    announce("32-qubit random-sum expectation on a basis state")
    s = state32
    hx, hz, hc = random_pauli_sum(N, 2000, 4343)
    k = 0x5A5A0F0F
    s.prepare_hf(k)
    h = Hamiltonian(PauliSum(N, hx, hz, hc))
    out = s.expect(h).cpu().numpy()
    ref = sum(float(c) * (-1) ** pauli.popcount(k & int(zz)) for xx, zz, c in zip(hx, hz, hc) if int(xx) == 0)
    assert abs(out[1] - 1.0) < 1e-12
    assert abs(out[0] - ref) < 1e-9 * max(1.0, abs(ref))
    h.free()
