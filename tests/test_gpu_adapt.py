"""Pools of Section 5.1 on the GPU against the oracle: qubit-excitation
circuits (no Jordan-Wigner tails) through the same rotation kernels, Pauli-
entangler screening, and the ADAPT loop driven by the GPU against the same
loop driven by the oracle."""
import numpy as np
import pytest
import torch

from oracle import fermion
from oracle import statevector as osv
from paper_2208_10978_amd.engine import UCCSDEvaluator
from paper_2208_10978_amd.problem import (entangler_pool, jordan_wigner, pauli_entangler_rotations, qeb_rotations,
                                          uccsd_rotations)
from paper_2208_10978_amd.vqe import adapt_vqe, gpu_adapt_vqe
from tests.adapt_oracle import oracle_callables
from tests.gpu_common import announce
from workloads import synthetic_integrals, uniform_amplitudes

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,ne", [(8, 4), (14, 7)])
def test_qeb_energy_and_gradient(n, ne):
    announce(f"qeb energy+grad n={n}")
    h, eri = synthetic_integrals(n, 5100 + n)
    s, d = fermion.uccsd_excitations(n, ne)
    seq = s + d
    theta = uniform_amplitudes(len(seq), 0.15, 5200 + n)
    ev = UCCSDEvaluator(jordan_wigner(h, eri), qeb_rotations(n, seq), ne, "c128")
    e, g = ev.energy_and_grad(theta)
    torch.cuda.synchronize()
    terms = fermion.jw_hamiltonian(h, eri)
    rots = fermion.qubit_excitation_rotations(seq)
    e_ref, g_rot = osv.reverse_mode_gradient(osv.basis_state(n, fermion.hf_index(ne)), [k[0] for k in terms],
                                             [k[1] for k in terms], list(terms.values()), [r[0] for r in rots],
                                             [r[1] for r in rots], [r[3] * theta[r[2]] for r in rots])
    g_ref = osv.chain_to_parameters(g_rot, [r[2] for r in rots], [r[3] for r in rots], len(theta))
    assert abs(e[0].item() - e_ref) <= 1e-10 * abs(e_ref)
    assert np.abs(g.cpu().numpy() - g_ref).max() <= 1e-10 * max(1.0, np.abs(g_ref).max())
    ev.free()


def test_entangler_pool_screening():
    announce("entangler pool screening n=8")
    n, ne = 8, 4
    h, eri = synthetic_integrals(n, 5300)
    ham = jordan_wigner(h, eri)
    circ = uccsd_rotations(n, ne, "lex")
    theta = uniform_amplitudes(circ.n_params, 0.2, 5301)
    px, pz = entangler_pool(ham, 4)
    ev = UCCSDEvaluator(ham, circ, ne, "c128")
    g = ev.pool_gradients(theta, pauli_entangler_rotations(n, px, pz)).cpu().numpy()
    terms = fermion.jw_hamiltonian(h, eri)
    rots = fermion.uccsd_rotations(n, ne)
    psi = osv.apply_rotations(osv.basis_state(n, fermion.hf_index(ne)), [r[0] for r in rots], [r[1] for r in rots],
                              [r[3] * theta[r[2]] for r in rots])
    ref = osv.rotation_pool_gradients(psi, [k[0] for k in terms], [k[1] for k in terms], list(terms.values()),
                                      px, pz)
    assert np.abs(g - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
    ev.free()


@pytest.mark.parametrize("kind", ["qeb", "entangler"])
def test_adapt_on_gpu_matches_the_oracle_driven_loop(kind):
    announce(f"adapt {kind} n=6")
    n, ne = 6, 2
    h, eri = synthetic_integrals(n, 5400)
    ham = jordan_wigner(h, eri)
    if kind == "qeb":
        s, d = fermion.uccgsd_excitations(n)
        pool = qeb_rotations(n, s + d)
    else:
        pool = pauli_entangler_rotations(n, *entangler_pool(ham, 4))
    gpu = gpu_adapt_vqe(ham, ne, pool, max_ops=6, grad_tol=1e-7)
    mk, screen = oracle_callables(h, eri, n, ne)
    ref = adapt_vqe(mk, screen, pool, n, max_ops=6, grad_tol=1e-7)
    assert len(gpu["energies"]) == len(ref["energies"]) and len(gpu["energies"]) > 0
    assert np.abs(np.array(gpu["energies"]) - np.array(ref["energies"])).max() < 1e-8
    assert gpu["energies"][-1] < fermion.slater_condon_hf_energy(h, eri, ne) - 1e-4
