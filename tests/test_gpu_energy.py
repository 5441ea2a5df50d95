"""GPU parity: Pauli-sum expectation and the UCCSD energy and gradient."""
import numpy as np
import pytest
import torch

from oracle import fermion
from oracle import statevector as osv
from paper_2208_10978_amd import binding as B
from paper_2208_10978_amd.engine import StateVector, UCCSDEvaluator, UCCEnergy
from paper_2208_10978_amd.problem import jordan_wigner, uccsd_rotations
from tests.gpu_common import announce, to_np_state
from workloads import random_pauli_sum, synthetic_integrals, uniform_amplitudes

pytestmark = pytest.mark.gpu


def oracle_problem(n, ne, h_seed, t_seed, amp):
    h, eri = synthetic_integrals(n, h_seed)
    terms = fermion.jw_hamiltonian(h, eri)
    rots = fermion.uccsd_rotations(n, ne)
    n_par = max(r[2] for r in rots) + 1
    theta = uniform_amplitudes(n_par, amp, t_seed)
    return h, eri, terms, rots, theta


@pytest.mark.parametrize("n", [4, 9, 14, 18])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_random_pauli_sum_expectation(n, dtype):
    announce(f"expectation random sum n={n} {dtype}")
    hx, hz, hc = random_pauli_sum(n, min(300, 200 if n < 6 else 300), 4343 + n)
    rng = np.random.default_rng(n)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    v /= np.linalg.norm(v)
    s = StateVector(n, dtype)
    s.amps.copy_(torch.from_numpy(v).to(s.amps.dtype))
    out = s.expect_terms(hx, hz, hc)
    torch.cuda.synchronize()
    vv = to_np_state(s.amps)
    e, nrm = osv.expectation(vv, hx, hz, hc)
    got = out.cpu().numpy()
    assert abs(got[1] - nrm) < 1e-12
    assert abs(got[0] - e.real / nrm) < 1e-10 * max(1.0, abs(e.real))


@pytest.mark.parametrize("n,ne", [(8, 4), (10, 5), (14, 7)])
def test_uccsd_energy_c128(n, ne):
    announce(f"uccsd energy n={n}")
    h, eri, terms, rots, theta = oracle_problem(n, ne, 1000 + n, 2000 + n, 0.1)
    psi = osv.basis_state(n, fermion.hf_index(ne))
    phis = [d * theta[p] for _, _, p, d in rots]
    psi = osv.apply_rotations(psi, [r[0] for r in rots], [r[1] for r in rots], phis)
    e_ref, _ = osv.expectation(psi, [k[0] for k in terms], [k[1] for k in terms], list(terms.values()))
    ev = UCCSDEvaluator(jordan_wigner(h, eri), uccsd_rotations(n, ne), ne, "c128")
    out = ev.energy(theta).cpu().numpy()
    assert abs(out[0] - e_ref.real) <= 1e-10 * abs(e_ref.real)
    assert abs(out[1] - 1.0) < 1e-12
    got_state = to_np_state(ev.psi.amps)
    assert np.abs(got_state - psi).max() < 1e-12


@pytest.mark.parametrize("n,ne", [(6, 3), (8, 4), (12, 6)])
def test_adjoint_per_rotation_gradient(n, ne):
    announce(f"adjoint per-rotation n={n}")
    h, eri, terms, rots, theta = oracle_problem(n, ne, 3000 + n, 4000 + n, 0.3)
    hx = [k[0] for k in terms]; hz = [k[1] for k in terms]; hc = list(terms.values())
    rx = np.array([r[0] for r in rots], dtype=np.uint64); rz = np.array([r[1] for r in rots], dtype=np.uint64)
    phis = np.array([d * theta[p] for _, _, p, d in rots])
    psi0 = osv.basis_state(n, fermion.hf_index(ne))
    e_ref, g_ref = osv.reverse_mode_gradient(psi0, hx, hz, hc, rx, rz, phis)
    ham = jordan_wigner(h, eri)
    psi = StateVector(n, "c128"); lam = StateVector(n, "c128")
    psi.prepare_hf(fermion.hf_index(ne))
    psi.apply_rotations(rx, rz, phis)
    energy = torch.empty(2, dtype=torch.float64, device="cuda")
    grad = torch.empty(len(phis), dtype=torch.float64, device="cuda")
    B.sv_adjoint_grad(psi.handle, lam.handle, ham.x, ham.z, ham.c, rx, rz, phis, energy, grad)
    torch.cuda.synchronize()
    assert abs(energy[0].item() - e_ref) <= 1e-10 * abs(e_ref)
    g = grad.cpu().numpy()
    assert np.abs(g - g_ref).max() <= 1e-10 * max(1.0, np.abs(g_ref).max())
    # the reverse sweep returns psi to the HF determinant
    back = to_np_state(psi.amps)
    assert np.abs(back - psi0).max() < 1e-12


@pytest.mark.parametrize("n,ne", [(8, 4), (12, 6), (16, 8)])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_parameter_gradient(n, ne, dtype):
    announce(f"adjoint params n={n} {dtype}")
    h, eri, terms, rots, theta = oracle_problem(n, ne, 5000 + n, 6000 + n, 0.1)
    hx = [k[0] for k in terms]; hz = [k[1] for k in terms]; hc = list(terms.values())
    rx = [r[0] for r in rots]; rz = [r[1] for r in rots]
    phis = [d * theta[p] for _, _, p, d in rots]
    psi0 = osv.basis_state(n, fermion.hf_index(ne))
    e_ref, g_rot = osv.reverse_mode_gradient(psi0, hx, hz, hc, rx, rz, phis)
    g_ref = osv.chain_to_parameters(g_rot, [r[2] for r in rots], [r[3] for r in rots], len(theta))
    ev = UCCSDEvaluator(jordan_wigner(h, eri), uccsd_rotations(n, ne), ne, dtype)
    e, g = ev.energy_and_grad(theta)
    torch.cuda.synchronize()
    e = e.cpu().numpy(); g = g.cpu().numpy()
    if dtype == "c128":
        assert abs(e[0] - e_ref) <= 1e-10 * abs(e_ref)
        assert np.abs(g - g_ref).max() <= 1e-10 * max(1.0, np.abs(g_ref).max())
    else:
        assert abs(e[0] - e_ref) <= 1e-5 * abs(e_ref)
        assert np.abs(g - g_ref).max() <= 1e-4 * max(1.0, np.abs(g_ref).max())


def test_autograd_function_matches_evaluator():
    announce("autograd")
    n, ne = 8, 4
    h, eri = synthetic_integrals(n, 1008)
    ev = UCCSDEvaluator(jordan_wigner(h, eri), uccsd_rotations(n, ne), ne, "c128")
    theta = torch.tensor(uniform_amplitudes(26, 0.1, 2008), dtype=torch.float64, requires_grad=True)
    e = UCCEnergy.apply(theta, ev)
    e.backward()
    e2, g2 = ev.energy_and_grad(theta.detach().numpy())
    assert abs(e.item() - e2[0].item()) < 1e-13
    assert np.abs(theta.grad.numpy() - g2.cpu().numpy()).max() < 1e-13
