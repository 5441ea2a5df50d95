"""Oracle-driven callables for the ADAPT loop (test helpers): every energy,
gradient and pool screening from the oracle's state vector."""
import numpy as np

from oracle import fermion
from oracle import statevector as osv


def oracle_callables(h, eri, n, ne):
    terms = fermion.jw_hamiltonian(h, eri)
    hx, hz, hc = [k[0] for k in terms], [k[1] for k in terms], list(terms.values())
    psi0 = osv.basis_state(n, fermion.hf_index(ne))

    def state(circuit, theta):
        return osv.apply_rotations(psi0.copy(), circuit.x, circuit.z, circuit.dphi_dtheta * np.asarray(theta)[circuit.param]
                                   if len(circuit) else [])

    def make_objective(circuit):
        def fg(theta):
            phis = circuit.dphi_dtheta * np.asarray(theta)[circuit.param]
            e, gr = osv.reverse_mode_gradient(psi0, hx, hz, hc, circuit.x, circuit.z, phis)
            return e, osv.chain_to_parameters(gr, circuit.param, circuit.dphi_dtheta, circuit.n_params)
        return fg

    def screen(circuit, theta, pool):
        psi = state(circuit, theta)
        g = osv.rotation_pool_gradients(psi, hx, hz, hc, pool.x, pool.z)
        return osv.chain_to_parameters(g, pool.param, pool.dphi_dtheta, pool.n_params)

    return make_objective, screen
