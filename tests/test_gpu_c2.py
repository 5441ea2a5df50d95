"""20-qubit workload (10 electrons, untruncated synthetic JW Hamiltonian,
UCCSD with theta ~ U[-0.05, 0.05]): energy and gradient in complex128 and
complex64 against the FP64 oracle.  The oracle values are stored in
tests/golden/c2_20q_reference.json by tests/golden/make_c2_reference.py
(which calls only the oracle)."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2208_10978_amd.engine import UCCSDEvaluator
from paper_2208_10978_amd.problem import jordan_wigner, uccsd_rotations
from tests.gpu_common import announce
from workloads import synthetic_integrals, uniform_amplitudes

pytestmark = pytest.mark.gpu
REF = os.path.join(os.path.dirname(__file__), "golden", "c2_20q_reference.json")

# complex64 a-priori bound: every pass over the state rounds each amplitude it
# changes once in FP32 with a 2x2 update (gamma ~ 4 roundoffs); unitary passes
# do not amplify the error, so after P passes ||dpsi|| <= P gamma u and
# |dE| <= 2 ||H||_1 P gamma u (+ FP64 reductions, negligible).
U32 = 2.0 ** -24
GAMMA = 4.0


@pytest.fixture(scope="module")
def ref():
    if not os.path.exists(REF):
        pytest.skip("reference not generated")
    return json.load(open(REF))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_c2_energy_and_gradient(ref, dtype):
    announce(f"C2 20q {dtype}")
    n, ne = ref["n_qubits"], ref["n_electrons"]
    h, eri = synthetic_integrals(n, ref["integral_seed"])
    ham = jordan_wigner(h, eri)
    rot = uccsd_rotations(n, ne, ref["order"])
    theta = uniform_amplitudes(rot.n_params, ref["theta_amplitude"], ref["theta_seed"])
    ev = UCCSDEvaluator(ham, rot, ne, dtype)
    e_only = ev.energy(theta).cpu().numpy().copy()
    e, g = ev.energy_and_grad(theta)
    torch.cuda.synchronize()
    e = e.cpu().numpy()
    g = g.cpu().numpy()
    e_ref = ref["energy"]
    g_ref = np.array(ref["grad_theta"])
    err_e = abs(e[0] - e_ref)
    err_g = np.abs(g - g_ref).max()
    announce(f"C2 {dtype}: |dE| = {err_e:.3e}, max |dg| = {err_g:.3e}, |E| = {abs(e_ref):.6f}")
    if dtype == "c128":
        assert err_e <= 1e-10 * abs(e_ref)
        assert abs(e_only[0] - e_ref) <= 1e-10 * abs(e_ref)
        assert err_g <= 1e-10 * max(1.0, np.abs(g_ref).max())
    else:
        passes = rot.n_params  # one fused run per excitation
        bound = 2.0 * ref["h_one_norm"] * passes * GAMMA * U32
        announce(f"C2 c64 a-priori energy bound {bound:.3e}")
        assert err_e <= bound
        assert err_e <= 1e-5 * abs(e_ref)          # what the path actually achieves
        assert abs(e_only[0] - e_ref) <= 1e-5 * abs(e_ref)
        assert err_g <= 1e-4 * max(1.0, np.abs(g_ref).max())
    ev.free()
