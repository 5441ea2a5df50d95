"""Real states (SV_R64): the amplitudes of a circuit of real rotations kept as
FP64 real parts only.  Every UCC string has an odd number of Y factors, so
each rotation exp(-i phi P / 2) of Eq. 11 is a real orthogonal matrix and
the state stays real from the Hartree-Fock basis state (Eq. 6); a real
Hamiltonian (Eq. 1) keeps lambda = H psi of Algorithm 1 real.  Checked
element by element and in energy and gradient against the oracle's complex
FP64 simulation, against the complex128 GPU path at larger sizes, and the
rejection of complex rotations and sums."""
import numpy as np
import pytest
import torch

from oracle import fermion
from oracle import pauli
from oracle import statevector as osv
from paper_2208_10978_amd import binding as B
from paper_2208_10978_amd.engine import StateVector, UCCSDEvaluator
from paper_2208_10978_amd.problem import jordan_wigner, uccsd_rotations
from tests.gpu_common import announce
from workloads import random_pauli_sum, synthetic_integrals, uccsd_excitation_order, uniform_amplitudes

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [8, 12, 16, 18])
def test_rotations_against_the_oracle(n):
    """UCCSD rotations (tile-major sequence) on a real state: every amplitude
    against the oracle, whose state stays real.  8 and 12 qubits fit one
    tile; 16 and 18 take tile passes and whole-state runs."""
    announce(f"real state rotations, {n} qubits")
    ne = n // 2
    rot = uccsd_rotations(n, ne)
    phi = rot.angles(uniform_amplitudes(rot.n_params, 0.3, 6000 + n))
    want = osv.apply_rotations(osv.basis_state(n, (1 << ne) - 1), rot.x, rot.z, phi)
    assert np.abs(want.imag).max() < 1e-14
    s = StateVector(n, "r64")
    s.prepare_hf((1 << ne) - 1)
    s.apply_rotations(rot.x, rot.z, phi)
    got = s.amps.cpu().numpy()
    s.free()
    assert np.abs(got - want.real).max() <= 1e-13


@pytest.mark.parametrize("n", [10, 14])
def test_expectation_against_the_oracle(n):
    """Eq. 2 on a real state, with the molecular sum plus random strings of
    both kinds: a string with an odd number of Y factors has <psi|P|psi> = 0
    on a real state, and the expectation must show it."""
    announce(f"real state expectation, {n} qubits")
    ne = n // 2
    h, eri = synthetic_integrals(n, 1000 + n)
    ham = jordan_wigner(h, eri)
    rx, rz, rc = random_pauli_sum(n, 300, 6100 + n)
    hx, hz, hc = np.concatenate([ham.x, rx]), np.concatenate([ham.z, rz]), np.concatenate([ham.c, rc])
    rot = uccsd_rotations(n, ne)
    phi = rot.angles(uniform_amplitudes(rot.n_params, 0.2, 6200 + n))
    psi = osv.apply_rotations(osv.basis_state(n, (1 << ne) - 1), rot.x, rot.z, phi)
    e_ref, nrm = osv.expectation(psi, hx, hz, hc)
    s = StateVector(n, "r64")
    s.prepare_hf((1 << ne) - 1)
    s.apply_rotations(rot.x, rot.z, phi)
    out = s.expect_terms(hx, hz, hc).cpu().numpy()
    s.free()
    scale = float(np.abs(hc).sum())
    assert abs(out[1] - nrm) <= 1e-13
    assert abs(out[0] - e_ref.real / nrm) <= 1e-13 * scale


@pytest.mark.parametrize("n", [8, 14])
def test_energy_and_gradient_against_the_oracle(n):
    """Energy and dE/dtheta (Algorithm 1 and the chain rule) of the UCCSD
    state against the oracle."""
    announce(f"real state energy+gradient, {n} qubits")
    ne = n // 2
    h, eri = synthetic_integrals(n, 1000 + n)
    ham = jordan_wigner(h, eri)
    order = uccsd_excitation_order(n, ne, "tile")
    rot = uccsd_rotations(n, ne, order)
    theta = uniform_amplitudes(rot.n_params, 0.1, 6300 + n)
    ev = UCCSDEvaluator(ham, rot, ne, "r64")
    e, g = ev.energy_and_grad(theta)
    torch.cuda.synchronize()
    e, g = e.cpu().numpy(), g.cpu().numpy()
    ev.free()
    terms = fermion.jw_hamiltonian(h, eri)
    rots = fermion.uccsd_rotations(n, ne, order)
    phis = [d * theta[p] for _, _, p, d in rots]
    e_ref, g_rot = osv.reverse_mode_gradient(osv.basis_state(n, fermion.hf_index(ne)), [k[0] for k in terms],
                                             [k[1] for k in terms], list(terms.values()), [r[0] for r in rots],
                                             [r[1] for r in rots], phis)
    g_ref = osv.chain_to_parameters(g_rot, [r[2] for r in rots], [r[3] for r in rots], len(theta))
    assert abs(e[0] - e_ref) <= 1e-12 * abs(e_ref)
    assert np.abs(g - g_ref).max() <= 1e-12 * max(1.0, np.abs(g_ref).max())


def test_real_and_complex128_paths_agree_at_22_qubits():
    """At 22 qubits (real-part lambda tiles in both) the real state's energy,
    gradient and state equal the complex128 path's to FP64 rounding."""
    announce("real vs complex128, 22 qubits")
    n, ne = 22, 11
    h, eri = synthetic_integrals(n, 1000 + n)
    ham = jordan_wigner(h, eri)
    rot = uccsd_rotations(n, ne)
    theta = uniform_amplitudes(rot.n_params, 0.05, 6400)
    out = {}
    for dt in ("c128", "r64"):
        ev = UCCSDEvaluator(ham, rot, ne, dt)
        psi = ev.state(theta)
        e, g = ev.energy_and_grad(theta)
        torch.cuda.synchronize()
        out[dt] = (e.cpu().numpy(), g.cpu().numpy(), psi.amps.cpu().numpy())
        psi.free()
        ev.free()
    (ec, gc, pc), (er, gr, pr) = out["c128"], out["r64"]
    assert np.abs(pc.imag).max() == 0.0
    assert np.abs(pr - pc.real).max() <= 1e-13
    assert abs(er[0] - ec[0]) <= 1e-12 * abs(ec[0])
    assert np.abs(gr - gc).max() <= 1e-12 * max(1.0, np.abs(gc).max())


def test_complex_rotations_and_sums_are_rejected():
    """A rotation whose string has an even number of Y factors is complex: a
    real state refuses it, and the adjoint refuses a sum whose odd-Y string
    has a real coefficient (it would make lambda complex).  Nothing runs."""
    announce("real state: complex inputs rejected")
    n = 8
    s = StateVector(n, "r64")
    lam = StateVector(n, "r64")
    s.prepare_hf(0b1111)
    before = s.amps.clone()
    x, z = pauli.from_label("XXII" + "I" * (n - 4))         # X X: no Y, complex rotation
    with pytest.raises(B.Q2svError) as ei:
        s.apply_rotations(np.array([x], np.uint64), np.array([z], np.uint64), np.array([0.3]))
    assert ei.value.code == B.SV_EINVAL
    x1, z1 = pauli.from_label("XYII" + "I" * (n - 4))       # one Y: real rotation
    energy = torch.empty(2, dtype=torch.float64, device="cuda")
    grad = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(B.Q2svError) as ei:
        B.sv_adjoint_grad(s.handle, lam.handle, np.array([x1], np.uint64), np.array([z1], np.uint64),
                          np.array([0.5]), np.array([x1], np.uint64), np.array([z1], np.uint64), np.array([0.0]),
                          energy, grad)
    assert ei.value.code == B.SV_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(s.amps, before)
    s.free()
    lam.free()
