"""The allocation-free expectation against the allocating one, through the C
ABI: same Pauli sum handle, same state, bitwise equal outputs (the two share
every kernel and the reduction order).  Two calls in a row on the shared
device array, the second on a smaller state, so the second reads an array
still holding the first call's partial sums.  Complex128 and complex64."""
import pytest
import torch

from paper_2208_10978_amd import binding as B
from paper_2208_10978_amd.engine import Hamiltonian, StateVector
from paper_2208_10978_amd.problem import PauliSum, jordan_wigner, uccsd_rotations
from tests.gpu_common import announce
from workloads import random_pauli_sum, synthetic_integrals, uniform_amplitudes

pytestmark = pytest.mark.gpu


def _ucc_state(n, dtype, seed):
    h, eri = synthetic_integrals(n, seed)
    ham = jordan_wigner(h, eri)
    rot = uccsd_rotations(n, n // 2)
    s = StateVector(n, dtype)
    s.prepare_hf((1 << (n // 2)) - 1)
    s.apply_rotations(rot.x, rot.z, rot.angles(uniform_amplitudes(rot.n_params, 0.1, seed + 1)))
    return s, Hamiltonian(ham)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_expectation_matches_the_allocating_call(dtype):
    announce(f"allocation-free expectation, {dtype}")
    big, h_big = _ucc_state(22, dtype, 1122)
    small, h_small = _ucc_state(10, dtype, 1110)
    try:
        ref_big = big.expect(h_big).clone()        # builds the tables and diagonal
        ref_small = small.expect(h_small).clone()
        out_big = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        out_small = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        B.sv_expect_hamiltonian_noalloc(big.handle, h_big.handle, out_big)
        B.sv_expect_hamiltonian_noalloc(small.handle, h_small.handle, out_small)
        torch.cuda.synchronize()
        assert torch.equal(out_big, ref_big), (out_big, ref_big)
        assert torch.equal(out_small, ref_small), (out_small, ref_small)
        # and once more in the other order
        B.sv_expect_hamiltonian_noalloc(big.handle, h_big.handle, out_big)
        torch.cuda.synchronize()
        assert torch.equal(out_big, ref_big)
    finally:
        for o in (big, small, h_big, h_small):
            o.free()


def test_noalloc_rejects_a_sum_whose_tables_are_not_built():
    announce("allocation-free expectation, tables not built")
    s = StateVector(12, "c128")
    hx, hz, hc = random_pauli_sum(12, 200, 12)
    h = Hamiltonian(PauliSum(12, hx, hz, hc))
    try:
        s.prepare_hf(0b111111)
        out = torch.zeros(2, dtype=torch.float64, device="cuda")
        with pytest.raises(B.Q2svError) as ei:
            B.sv_expect_hamiltonian_noalloc(s.handle, h.handle, out)
        assert ei.value.code == B.SV_EINVAL
        s.expect(h, out)
        ref = out.clone()
        B.sv_expect_hamiltonian_noalloc(s.handle, h.handle, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    finally:
        s.free()
        h.free()
