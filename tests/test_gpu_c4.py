"""The raw-sweep workload at full size (32 qubits, complex64, 32 GiB): exact
pins that need no full-state oracle.

* A rotation changes an amplitude from itself and its partner only, so after
  a batch of K rotations an amplitude depends on at most 2^K amplitudes
  before the batch (its closure under XOR with the batch's flip masks).
  Gathering those pre-values and applying the batch to them on the host in
  FP64 reproduces the GPU's amplitude up to the complex64 rounding of the
  batch, whatever fusion the GPU used.
* The expectation of a Pauli sum on a basis state keeps only its diagonal
  (x = 0) strings: sum_t c_t (-1)^{|k & z_t|}.
* From a basis state, K rotations leave at most 2^K nonzero amplitudes (the
  closure of the start index), so every nonzero amplitude can be gathered
  and <psi|H|psi> of any sum evaluated on the host over that sparse set."""
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


def _closure_sum(n, rx, extra_seed):
    """A Pauli sum whose flip masks connect the closure of a start index under
    the rotation masks rx: three strings for every mask and every pairwise
    XOR of two, with random z masks (some on the top two qubits) and
    c ~ U[-1, 1]."""
    rng = np.random.default_rng(extra_seed)
    masks = sorted({int(a) for a in rx} | {int(a) ^ int(b) for i, a in enumerate(rx) for b in rx[i + 1:]})
    ex, ez, ec = [], [], []
    for xm in masks:
        for _ in range(3):
            zm = int(rng.integers(0, 1 << n, dtype=np.uint64)) | (int(rng.integers(0, 4)) << (n - 2))
            ex.append(xm)
            ez.append(zm)
            ec.append(float(rng.uniform(-1.0, 1.0)))
    return np.array(ex, dtype=np.uint64), np.array(ez, dtype=np.uint64), np.array(ec)


def _sparse_energy(amp: dict, hx, hz, hc):
    """(sum_t c_t <psi|P_t|psi>, sum of the magnitudes of its products) over
    a dict of the nonzero amplitudes, with P|k> = i^{|x&z|} (-1)^{|k & z|}
    |k ^ x>, in FP64."""
    idx = np.array(sorted(amp), dtype=np.uint64)
    val = np.array([amp[int(i)] for i in idx])
    e, scale = 0j, 0.0
    for x, z, c in zip(hx, hz, hc):
        src = idx ^ np.uint64(x)                  # <m|P|src> psi[src]
        at = np.minimum(np.searchsorted(idx, src), len(idx) - 1)
        hit = idx[at] == src
        if not hit.any():
            continue
        w = 1j ** (pauli.popcount(int(x) & int(z)) % 4)
        sgn = 1.0 - 2.0 * (np.bitwise_count(src[hit] & np.uint64(z)) & 1)
        t = float(c) * w * np.conj(val[hit]) * sgn * val[at[hit]]
        e += t.sum()
        scale += np.abs(t).sum()
    return complex(e), float(scale)


def _evolve_sparse(k0, rx, rz, rphi):
    """R_K ... R_1 |k0> on the host in FP64, over the closure of k0."""
    amp = {j: 0j for j in closure(k0, rx)}
    amp[int(k0)] = 1.0 + 0j
    for x, z, p in zip(rx, rz, rphi):
        amp = rotate_sparse(amp, x, z, p)
    return amp


def test_sparse_energy_helper_matches_the_oracle():
    """The host helpers of the 32-qubit check at 10 qubits, against the
    oracle's dense rotation and term-by-term expectation."""
    n = 10
    rx, rz, rphi = random_rotations(n, 5, 77, amplitude=1.5)
    hx, hz, hc = random_pauli_sum(n, 300, 78)
    ex, ez, ec = _closure_sum(n, rx, 79)
    hx, hz, hc = np.concatenate([hx, ex]), np.concatenate([hz, ez]), np.concatenate([hc, ec])
    k0 = 0b0000011111
    amp = _evolve_sparse(k0, rx, rz, rphi)
    psi = osv.apply_rotations(osv.basis_state(n, k0), rx, rz, rphi)
    assert max(abs(psi[j] - amp.get(j, 0j)) for j in range(1 << n)) < 1e-14
    e, scale = _sparse_energy(amp, hx, hz, hc)
    want, _ = osv.expectation(psi, hx, hz, hc)
    assert abs(e - want) < 1e-13 * scale
    assert scale > 1.0


@pytest.mark.gpu
def test_expectation_off_diagonal_groups_at_full_size(state32):
    """Eq. 2 at 32 qubits with off-diagonal groups contributing: psi is
    R_9 ... R_1 |2^16 - 1> for nine seeded 4-qubit rotations (angles up to
    1.5, at least one on the top two qubits), so at most 512 amplitudes are
    nonzero.  All of them are gathered (a sample of the others must read
    exactly zero) and checked against the host's FP64 evolution from the
    start state; the sum is the 10^4-term random workload sum plus three
    strings for every rotation mask and pairwise XOR of two.  The host
    evaluates <psi|H|psi> / <psi|psi> over the gathered amplitudes in FP64;
    both sides reduce the same complex64 values in FP64, so they agree to
    FP64 rounding."""
    announce("32-qubit expectation with off-diagonal groups, sparse closure")
    s = state32
    seed = 9090
    while True:   # the first seed from 9090 whose rotations reach qubit 30 or 31
        rx, rz, rphi = random_rotations(N, 9, seed, amplitude=1.5)
        if any(int(v) >> (N - 2) for v in rx):
            break
        seed += 1
    k0 = (1 << 16) - 1
    ref = _evolve_sparse(k0, rx, rz, rphi)
    support = sorted(ref)
    ex, ez, ec = _closure_sum(N, rx, seed + 1)
    hx, hz, hc = random_pauli_sum(N, 10_000, 4343)
    hx, hz, hc = np.concatenate([hx, ex]), np.concatenate([hz, ez]), np.concatenate([hc, ec])
    s.prepare_hf(k0)
    s.apply_rotations(rx, rz, rphi)
    got = s.amplitudes(support).cpu().numpy()
    amp = dict(zip(support, got[0::2] + 1j * got[1::2]))
    assert max(abs(amp[j] - ref[j]) for j in support) <= 2e-6
    assert sum(abs(v) > 1e-3 for v in amp.values()) > 64      # the state is spread over the closure
    rng = np.random.default_rng(seed)
    others = [int(v) for v in rng.integers(0, 1 << N, size=256, dtype=np.uint64) if int(v) not in amp]
    zeros = s.amplitudes(others).cpu().numpy()
    assert not np.any(zeros)
    h = Hamiltonian(PauliSum(N, hx, hz, hc))
    try:
        out = s.expect(h).cpu().numpy()
    finally:
        h.free()
    e_host, scale = _sparse_energy(amp, hx, hz, hc)
    norm2 = float(sum(abs(v) ** 2 for v in amp.values()))
    diag = hx == 0
    e_off, _ = _sparse_energy(amp, hx[~diag], hz[~diag], hc[~diag])
    assert abs(e_host.imag) <= 1e-12 * scale
    assert abs(e_off.real) > 1e-2                              # off-diagonal groups carry weight
    assert abs(out[1] - norm2) <= 1e-12
    assert abs(out[0] - e_host.real / norm2) <= 1e-12 * scale, (out[0], e_host.real / norm2)
