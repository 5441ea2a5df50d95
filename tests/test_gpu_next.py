"""NEXT rows on the GPU against the oracle: UCCGSD energy and gradient
(Table 1's generalized ansatz through the same rotation kernels), ADAPT pool
gradients (Section 5.1) and the variational loop of Eq. 9."""
import numpy as np
import pytest
import torch

from oracle import fermion
from oracle import statevector as osv
from paper_2208_10978_amd.engine import UCCSDEvaluator
from paper_2208_10978_amd.problem import excitation_rotations, jordan_wigner, uccgsd_rotations
from paper_2208_10978_amd.vqe import evaluator_objective, vqe
from tests.gpu_common import announce
from workloads import synthetic_integrals, uniform_amplitudes

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,ne", [(6, 3), (8, 4)])
def test_uccgsd_energy_and_gradient(n, ne):
    announce(f"uccgsd energy+grad n={n}")
    h, eri = synthetic_integrals(n, 3000 + n)
    rot = uccgsd_rotations(n)
    ev = UCCSDEvaluator(jordan_wigner(h, eri), rot, ne, "c128")
    theta = uniform_amplitudes(rot.n_params, 0.1, 3100 + n)
    e, g = ev.energy_and_grad(theta)
    torch.cuda.synchronize()
    terms = fermion.jw_hamiltonian(h, eri)
    gs, gd = fermion.uccgsd_excitations(n)
    rots = fermion.excitation_rotations(gs + gd)
    e_ref, g_rot = osv.reverse_mode_gradient(
        osv.basis_state(n, fermion.hf_index(ne)), [k[0] for k in terms], [k[1] for k in terms], list(terms.values()),
        [r[0] for r in rots], [r[1] for r in rots], [r[3] * theta[r[2]] for r in rots])
    g_ref = osv.chain_to_parameters(g_rot, [r[2] for r in rots], [r[3] for r in rots], len(theta))
    assert abs(e[0].item() - e_ref) <= 1e-10 * abs(e_ref)
    assert np.abs(g.cpu().numpy() - g_ref).max() <= 1e-10 * max(1.0, np.abs(g_ref).max())
    ev.free()


@pytest.mark.parametrize("n,ne", [(6, 2), (8, 4)])
def test_adapt_pool_gradients(n, ne):
    announce(f"adapt pool gradients n={n}")
    h, eri = synthetic_integrals(n, 3200 + n)
    singles, doubles = fermion.uccsd_excitations(n, ne)
    circ = singles + doubles
    theta = uniform_amplitudes(len(circ), 0.2, 3300 + n)
    gs, gd = fermion.uccgsd_excitations(n)
    pool = gs + gd
    ev = UCCSDEvaluator(jordan_wigner(h, eri), excitation_rotations(n, circ), ne, "c128")
    g = ev.pool_gradients(theta, excitation_rotations(n, pool)).cpu().numpy()
    ref = fermion.pool_gradients(h, eri, n, ne, theta, pool, excitations=circ)
    assert np.abs(g - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
    ev.free()


def test_vqe_reaches_the_exact_ground_state_with_uccgsd_at_4_qubits():
    announce("vqe uccgsd n=4")
    n, ne = 4, 2
    h, eri = synthetic_integrals(n, 77)
    basis = fermion.sector_basis(n, *fermion.electron_counts(ne))
    e0 = np.linalg.eigvalsh(fermion.determinant_hamiltonian(h, eri, basis).toarray())[0]
    ev = UCCSDEvaluator(jordan_wigner(h, eri), uccgsd_rotations(n), ne, "c128")
    best = min(vqe(evaluator_objective(ev), uniform_amplitudes(ev.rot.n_params, 1.0, s))["energy"] for s in range(3))
    assert abs(best - e0) < 1e-9
    ev.free()


def test_vqe_matches_an_oracle_driven_loop_at_8_qubits():
    announce("vqe uccsd n=8 vs oracle-driven loop")
    n, ne = 8, 4
    h, eri = synthetic_integrals(n, 1008)
    singles, doubles = fermion.uccsd_excitations(n, ne)
    circ = singles + doubles
    ev = UCCSDEvaluator(jordan_wigner(h, eri), excitation_rotations(n, circ), ne, "c128")
    terms = fermion.jw_hamiltonian(h, eri)
    hx, hz, hc = [k[0] for k in terms], [k[1] for k in terms], list(terms.values())
    rots = fermion.excitation_rotations(circ)

    def oracle_fg(th):
        e, gr = osv.reverse_mode_gradient(osv.basis_state(n, fermion.hf_index(ne)), hx, hz, hc,
                                          [r[0] for r in rots], [r[1] for r in rots], [r[3] * th[r[2]] for r in rots])
        return e, osv.chain_to_parameters(gr, [r[2] for r in rots], [r[3] for r in rots], len(th))
    start = np.zeros(len(circ))
    gpu = vqe(evaluator_objective(ev), start)
    ref = vqe(oracle_fg, start)
    assert abs(gpu["energy"] - ref["energy"]) < 1e-8
    basis = fermion.sector_basis(n, *fermion.electron_counts(ne))
    e0 = np.linalg.eigvalsh(fermion.determinant_hamiltonian(h, eri, basis).toarray())[0]
    assert gpu["energy"] >= e0 - 1e-10 and gpu["energy"] < fermion.slater_condon_hf_energy(h, eri, ne)
    ev.free()
