"""Write the 20-qubit reference (energy and dE/dtheta) with the FP64 oracle.

Workload: 20 qubits, 10 electrons, synthetic integrals seed 1020 (untruncated
JW sum), UCCSD in the tile-major excitation sequence, theta ~ U[-0.05, 0.05]
seed 2020.  Calls only oracle/ and the seeded input generators; takes about
15 minutes on one core.  Usage: python tests/golden/make_c2_reference.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import fermion  # noqa: E402
from oracle import statevector as osv  # noqa: E402
from workloads import synthetic_integrals, uccsd_excitation_order, uniform_amplitudes  # noqa: E402


def main():
    n, ne = 20, 10
    t0 = time.time()
    h, eri = synthetic_integrals(n, 1020)
    terms = fermion.jw_hamiltonian(h, eri)
    order = uccsd_excitation_order(n, ne, "tile")
    rots = fermion.uccsd_rotations(n, ne, order)
    theta = uniform_amplitudes(len(order), 0.05, 2020)
    phis = [d * theta[p] for _, _, p, d in rots]
    print(f"{len(terms)} terms, {len(rots)} rotations ({time.time() - t0:.0f} s)", flush=True)
    e, g_rot = osv.reverse_mode_gradient(osv.basis_state(n, fermion.hf_index(ne)), [k[0] for k in terms],
                                         [k[1] for k in terms], list(terms.values()), [r[0] for r in rots],
                                         [r[1] for r in rots], phis)
    g = osv.chain_to_parameters(g_rot, [r[2] for r in rots], [r[3] for r in rots], len(theta))
    out = {
        "source": "oracle (FP64, one rotation at a time, term by term, Algorithm 1); "
                  "written by tests/golden/make_c2_reference.py",
        "n_qubits": n, "n_electrons": ne, "integral_seed": 1020, "theta_seed": 2020, "theta_amplitude": 0.05,
        "order": "tile", "n_terms": len(terms), "n_rotations": len(rots),
        "h_one_norm": float(sum(abs(c) for c in terms.values())),
        "energy": e, "grad_theta": [float(v) for v in g],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_20q_reference.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"E = {e:.15f}; wrote {path} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
