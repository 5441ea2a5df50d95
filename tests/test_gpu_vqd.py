"""Variational quantum deflation (Eq. 12) on the GPU against the oracle: the
overlap reduction, the deflated energy and adjoint gradient, and the excited
energy the VQD loop reaches."""
import numpy as np
import pytest
import torch

from oracle import fermion
from oracle import statevector as osv
from paper_2208_10978_amd.engine import StateVector, UCCSDEvaluator
from paper_2208_10978_amd.problem import excitation_rotations, jordan_wigner, uccgsd_rotations
from paper_2208_10978_amd.vqe import vqd
from tests.gpu_common import announce, to_np_state
from workloads import synthetic_integrals, uniform_amplitudes

pytestmark = pytest.mark.gpu


def random_unit(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


def device_state(v, dtype):
    s = StateVector(int(np.log2(len(v))), dtype)
    s.amps.copy_(torch.from_numpy(v).to(s.amps.dtype))
    return s


@pytest.mark.parametrize("n", [3, 10, 17])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_overlap(n, dtype):
    announce(f"overlap n={n} {dtype}")
    a, b = device_state(random_unit(n, 5 + n), dtype), device_state(random_unit(n, 6 + n), dtype)
    got = a.overlap(b).cpu().numpy()
    torch.cuda.synchronize()
    ref = np.vdot(to_np_state(a.amps), to_np_state(b.amps))
    assert abs(got[0] - ref.real) < 1e-12 and abs(got[1] - ref.imag) < 1e-12
    a.free()
    b.free()


@pytest.mark.parametrize("n,ne", [(6, 2), (8, 4), (14, 7)])
def test_deflated_energy_and_gradient(n, ne):
    announce(f"deflated adjoint n={n}")
    h, eri = synthetic_integrals(n, 4100 + n)
    singles, doubles = fermion.uccsd_excitations(n, ne)
    circ = singles + doubles
    theta = uniform_amplitudes(len(circ), 0.2, 4200 + n)
    proj_np = [random_unit(n, 4300 + n), random_unit(n, 4400 + n)]
    alphas = [0.7, 1.3]
    ev = UCCSDEvaluator(jordan_wigner(h, eri), excitation_rotations(n, circ), ne, "c128")
    proj = [device_state(v, "c128") for v in proj_np]
    e, g, ovl = ev.energy_and_grad_deflated(theta, proj, alphas)
    torch.cuda.synchronize()
    terms = fermion.jw_hamiltonian(h, eri)
    rots = fermion.excitation_rotations(circ)
    psi0 = osv.basis_state(n, fermion.hf_index(ne))
    phis = [r[3] * theta[r[2]] for r in rots]
    e_ref, g_rot = osv.deflated_reverse_gradient(psi0, [k[0] for k in terms], [k[1] for k in terms],
                                                 list(terms.values()), proj_np, alphas, [r[0] for r in rots],
                                                 [r[1] for r in rots], phis)
    g_ref = osv.chain_to_parameters(g_rot, [r[2] for r in rots], [r[3] for r in rots], len(theta))
    assert abs(e[0].item() - e_ref) <= 1e-10 * max(1.0, abs(e_ref))
    gg = g.cpu().numpy()
    assert np.abs(gg - g_ref).max() <= 1e-10 * max(1.0, np.abs(g_ref).max())
    psi = osv.apply_rotations(psi0.copy(), [r[0] for r in rots], [r[1] for r in rots], phis)
    o = ovl.cpu().numpy()
    for j, p in enumerate(proj_np):
        ref = np.vdot(p, psi)
        assert abs(o[2 * j] - ref.real) < 1e-12 and abs(o[2 * j + 1] - ref.imag) < 1e-12
    for s in proj:
        s.free()
    ev.free()


def test_vqd_reaches_the_two_lowest_energies_at_4_qubits():
    announce("vqd uccgsd n=4")
    n, ne = 4, 2
    h, eri = synthetic_integrals(n, 77)
    basis = fermion.sector_basis(n, *fermion.electron_counts(ne))
    w = np.linalg.eigvalsh(fermion.determinant_hamiltonian(h, eri, basis).toarray())
    ev = UCCSDEvaluator(jordan_wigner(h, eri), uccgsd_rotations(n), ne, "c128")
    starts = [[uniform_amplitudes(ev.rot.n_params, 1.0, 10 * k + s) for s in range(4)] for k in range(2)]
    res = vqd(ev, 2, 2.0 * (w[-1] - w[0]), starts, gtol=1e-10)
    assert abs(res[0]["energy"] - w[0]) < 1e-9
    assert abs(res[1]["energy_eff"] - w[1]) < 1e-7
    assert abs(res[1]["energy"] - w[1]) < 1e-6
    ov = res[0]["state"].overlap(res[1]["state"]).cpu().numpy()
    assert np.hypot(*ov) < 1e-3
    for r in res:
        r["state"].free()
    ev.free()


def test_deflated_call_rejects_bad_deflation_lists():
    """Validation is synchronous: bad lists raise and leave psi untouched."""
    from paper_2208_10978_amd import binding as B
    announce("deflated call error paths")
    n, ne = 6, 2
    h, eri = synthetic_integrals(n, 4500)
    s, d = fermion.uccsd_excitations(n, ne)
    ev = UCCSDEvaluator(jordan_wigner(h, eri), excitation_rotations(n, s + d), ne, "c128")
    theta = uniform_amplitudes(ev.rot.n_params, 0.1, 4501)
    ok = device_state(random_unit(n, 4502), "c128")
    other = device_state(random_unit(n + 1, 4503), "c128")
    ev.forward_state(theta)
    before = ev.psi.amps.clone()
    phi = ev.rot.angles(theta)

    def call(proj, alphas):
        B.sv_adjoint_grad_params_deflated(ev.psi.handle, ev.lam.handle, ev.h.handle, [p.handle for p in proj], alphas,
                                          ev.rot.x, ev.rot.z, phi, ev.rot.param, ev.rot.dphi_dtheta,
                                          ev.rot.n_params, ev.energy_buf, None, ev.grad_buf)
    for proj, alphas in [([ok] * 9, [1.0] * 9), ([ev.psi], [1.0]), ([other], [1.0]), ([ok], [float("nan")])]:
        with pytest.raises(B.Q2svError):
            call(proj, alphas)
    torch.cuda.synchronize()
    assert torch.equal(ev.psi.amps, before)
    for st in (ok, other):
        st.free()
    ev.free()
