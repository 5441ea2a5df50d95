"""GPU parity: Pauli-sum expectation and the UCCSD energy and gradient."""
import numpy as np
import pytest
import torch

from oracle import fermion
from oracle import pauli
from oracle import statevector as osv
from paper_2208_10978_amd import binding as B
from paper_2208_10978_amd.engine import StateVector, UCCSDEvaluator, UCCEnergy
from paper_2208_10978_amd.problem import jordan_wigner, uccsd_rotations
from tests import c64_bounds as cb
from tests.gpu_common import announce, to_np_state
from workloads import (random_pauli_sum, random_rotations, synthetic_integrals, uccsd_excitation_order,
                       uniform_amplitudes)

pytestmark = pytest.mark.gpu


ORDER = "tile"


def oracle_problem(n, ne, h_seed, t_seed, amp):
    h, eri = synthetic_integrals(n, h_seed)
    terms = fermion.jw_hamiltonian(h, eri)
    rots = fermion.uccsd_rotations(n, ne, uccsd_excitation_order(n, ne, ORDER))
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
    ev = UCCSDEvaluator(jordan_wigner(h, eri), uccsd_rotations(n, ne, ORDER), ne, "c128")
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
    ev = UCCSDEvaluator(jordan_wigner(h, eri), uccsd_rotations(n, ne, ORDER), ne, dtype)
    e, g = ev.energy_and_grad(theta)
    torch.cuda.synchronize()
    e = e.cpu().numpy(); g = g.cpu().numpy()
    if dtype == "c128":
        assert abs(e[0] - e_ref) <= 1e-10 * abs(e_ref)
        assert np.abs(g - g_ref).max() <= 1e-10 * max(1.0, np.abs(g_ref).max())
    else:
        # stated errors (tests/c64_bounds.py) with sigma_H and ||H psi|| of
        # the oracle's final state; one run per excitation plus the
        # renormalisation
        rot = uccsd_rotations(n, ne, ORDER)
        psi_n = osv.apply_rotations(psi0, rx, rz, phis)
        h_psi = osv.apply_hamiltonian(psi_n, hx, hz, hc)
        hn = float(np.linalg.norm(h_psi))
        sigma = float(np.sqrt(max(hn * hn - e_ref * e_ref, 0.0)))
        h1 = float(np.abs(hc).sum())
        runs = rot.n_params + 1
        assert abs(e[0] - e_ref) <= min(cb.energy_bound_probabilistic(runs, sigma, h1), cb.energy_bound(runs, sigma, h1))
        assert np.all(np.abs(g - g_ref) <= cb.parameter_gradient_bounds(rot, runs, h1, hn))


def test_autograd_function_matches_evaluator():
    announce("autograd")
    n, ne = 8, 4
    h, eri = synthetic_integrals(n, 1008)
    ev = UCCSDEvaluator(jordan_wigner(h, eri), uccsd_rotations(n, ne, ORDER), ne, "c128")
    theta = torch.tensor(uniform_amplitudes(26, 0.1, 2008), dtype=torch.float64, requires_grad=True)
    e = UCCEnergy.apply(theta, ev)
    e.backward()
    e2, g2 = ev.energy_and_grad(theta.detach().numpy())
    assert abs(e.item() - e2[0].item()) < 1e-13
    assert np.abs(theta.grad.numpy() - g2.cpu().numpy()).max() < 1e-13


def generic_sum(n, seed, with_diag=True, wide=True):
    """Random weight<=4 strings, plus wide strings (support > 6 bits, and
    > 9 bits when n allows) that exercise the non-enumerated and whole-state
    group paths; optionally without any diagonal (Z-only) term."""
    hx, hz, hc = random_pauli_sum(n, 150 if n >= 6 else 60, seed)
    rng = np.random.default_rng(seed + 1)
    xs, zs, cs = list(hx), list(hz), list(hc)
    if wide and n >= 8:
        for w in ([8, 11] if n >= 11 else [8]):
            for _ in range(3):
                q = rng.choice(n, size=w, replace=False)
                x = 0
                z = 0
                for k, qq in enumerate(q):
                    x |= 1 << int(qq)
                    if k % 2:
                        z |= 1 << int(qq)
                xs.append(x); zs.append(z ^ (1 << int(q[0]) if w % 3 == 0 else z)); cs.append(float(rng.uniform(-1, 1)))
    xs = np.array(xs, dtype=np.uint64); zs = np.array(zs, dtype=np.uint64); cs = np.array(cs)
    if not with_diag:
        keep = xs != 0
        xs, zs, cs = xs[keep], zs[keep], cs[keep]
    return xs, zs, cs


@pytest.mark.parametrize("n", [5, 13, 17])
@pytest.mark.parametrize("with_diag", [True, False])
def test_adjoint_generic_pauli_sums(n, with_diag):
    announce(f"adjoint generic sum n={n} diag={with_diag}")
    hx, hz, hc = generic_sum(n, 900 + n, with_diag)
    rx, rz, rphi = random_rotations(n, 24, 700 + n, amplitude=1.0)
    psi0 = osv.basis_state(n, (1 << (n // 2)) - 1)
    e_ref, g_ref = osv.reverse_mode_gradient(psi0, hx, hz, hc, rx, rz, rphi)
    psi = StateVector(n, "c128"); lam = StateVector(n, "c128")
    psi.prepare_hf((1 << (n // 2)) - 1)
    psi.apply_rotations(rx, rz, rphi)
    out = psi.expect_terms(hx, hz, hc)
    energy = torch.empty(2, dtype=torch.float64, device="cuda")
    grad = torch.empty(len(rphi), dtype=torch.float64, device="cuda")
    B.sv_adjoint_grad(psi.handle, lam.handle, hx, hz, hc, rx, rz, rphi, energy, grad)
    torch.cuda.synchronize()
    scale = max(1.0, float(np.abs(hc).sum()))
    assert abs(out[0].item() - e_ref) <= 1e-12 * scale
    assert abs(energy[0].item() - e_ref) <= 1e-12 * scale
    assert np.abs(grad.cpu().numpy() - g_ref).max() <= 1e-12 * scale
    assert np.abs(to_np_state(psi.amps) - psi0).max() < 1e-12


@pytest.mark.parametrize("n", [6, 15])
def test_expectation_is_bitwise_reproducible(n):
    announce(f"reproducible n={n}")
    hx, hz, hc = generic_sum(n, 1200 + n)
    rx, rz, rphi = random_rotations(n, 10, 1300 + n, amplitude=1.0)
    s = StateVector(n, "c128")
    outs = []
    for _ in range(3):
        s.prepare_hf(3)
        s.apply_rotations(rx, rz, rphi)
        outs.append(s.expect_terms(hx, hz, hc).cpu().numpy().copy())
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_one_hamiltonian_shared_by_states_on_two_streams():
    """A resident Hamiltonian used first on one stream and at once on another
    (its diagonal is built on the first): both expectations match the oracle."""
    from paper_2208_10978_amd.engine import Hamiltonian
    from paper_2208_10978_amd.problem import PauliSum
    announce("shared Hamiltonian, two streams")
    n = 14
    hx, hz, hc = random_pauli_sum(n, 400, 4700)
    H = Hamiltonian(PauliSum(n, np.asarray(hx, np.uint64), np.asarray(hz, np.uint64), np.asarray(hc)))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    vs = [np.random.default_rng(k).normal(size=1 << n) + 1j * np.random.default_rng(k + 9).normal(size=1 << n)
          for k in (1, 2)]
    vs = [v / np.linalg.norm(v) for v in vs]
    states = []
    for v, st in zip(vs, (s1, s2)):
        with torch.cuda.stream(st):
            s = StateVector(n, "c128", stream=st)
            s.amps.copy_(torch.from_numpy(v))
        states.append(s)
    torch.cuda.synchronize()
    outs = []
    for s, st in zip(states, (s1, s2)):
        with torch.cuda.stream(st):
            outs.append(s.expect(H))
    torch.cuda.synchronize()
    for v, o in zip(vs, outs):
        e, nrm = osv.expectation(v, hx, hz, hc)
        got = o.cpu().numpy()
        assert abs(got[0] - e.real / nrm) < 1e-10 * max(1.0, abs(e.real))
    for s in states:
        s.free()
    H.free()


def test_cached_sum_follows_changed_coefficients():
    """A state keeps the grouped form of its last Pauli sum; a later call with
    the same strings but one changed coefficient must not reuse it."""
    announce("cached sum, changed coefficient")
    n = 9
    hx, hz, hc = random_pauli_sum(n, 120, 777)
    rng = np.random.default_rng(778)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    v /= np.linalg.norm(v)
    s = StateVector(n, "c128")
    s.amps.copy_(torch.from_numpy(v))
    first = s.expect_terms(hx, hz, hc).cpu().numpy().copy()
    hc2 = hc.copy()
    hc2[len(hc2) // 2] += 0.25
    second = s.expect_terms(hx, hz, hc2).cpu().numpy().copy()
    e1, _ = osv.expectation(v, hx, hz, hc)
    e2, _ = osv.expectation(v, hx, hz, hc2)
    assert abs(first[0] - e1.real) < 1e-10 * max(1.0, abs(e1.real))
    assert abs(second[0] - e2.real) < 1e-10 * max(1.0, abs(e2.real))
    s.free()


@pytest.mark.parametrize("case", ["real_psi_real_h", "complex_psi_real_h", "one_imag_real_h",
                                  "real_psi_complex_h"])
def test_lambda_real_and_complex_paths(case):
    """lambda = H psi element by element against the oracle at 14 qubits, with
    a real psi and a real sum, a complex psi, one nonzero imaginary amplitude,
    and a sum with odd-Y strings.  A 14-qubit state is too small for the
    real-part tiling (it would leave compute units idle), so every case here
    runs the complex build; the 21-qubit test covers the real-part tiling.
    One rotation at phi = 0 leaves psi as it is, so lam returns H psi."""
    announce(f"lambda paths: {case}")
    n = 14
    h, eri = synthetic_integrals(n, 1000 + n)
    ham = jordan_wigner(h, eri)
    hx, hz, hc = np.asarray(ham.x, np.uint64), np.asarray(ham.z, np.uint64), np.asarray(ham.c)
    if case == "real_psi_complex_h":
        rx_, rz_, rc_ = random_pauli_sum(n, 200, 4900)
        odd = np.array([pauli.popcount(int(a) & int(b)) % 2 == 1 for a, b in zip(rx_, rz_)])
        hx = np.concatenate([hx, rx_[odd]]); hz = np.concatenate([hz, rz_[odd]]); hc = np.concatenate([hc, rc_[odd]])
    rng = np.random.default_rng(4901)
    v = rng.normal(size=1 << n) + (1j * rng.normal(size=1 << n) if case == "complex_psi_real_h" else 0.0)
    if case == "one_imag_real_h":
        v = v + 0j
        v[12345] += 1e-3j
    v = v / np.linalg.norm(v)
    psi = StateVector(n, "c128"); lam = StateVector(n, "c128")
    psi.amps.copy_(torch.from_numpy(np.asarray(v, np.complex128)))
    energy = torch.empty(2, dtype=torch.float64, device="cuda")
    grad = torch.empty(1, dtype=torch.float64, device="cuda")
    B.sv_adjoint_grad(psi.handle, lam.handle, hx, hz, hc, np.array([1], np.uint64), np.array([1], np.uint64),
                      np.array([0.0]), energy, grad)
    torch.cuda.synchronize()
    want = osv.apply_hamiltonian(np.asarray(v, np.complex128), hx, hz, hc)
    got = to_np_state(lam.amps)
    scale = max(1.0, float(np.abs(hc).sum()))
    assert np.abs(got - want).max() <= 1e-12 * scale
    e_ref, _ = osv.expectation(np.asarray(v, np.complex128), hx, hz, hc)
    assert abs(energy[0].item() - e_ref.real) <= 1e-12 * scale
    psi.free(); lam.free()


@pytest.mark.parametrize("case", ["complex_start", "complex_sum", "real"])
def test_reverse_sweep_real_and_complex_paths(case):
    """Every UCCSD rotation is real, so the reverse sweep may update real parts
    only, but only while psi and lambda are real: a complex start state, or a
    sum with odd-Y strings (complex lambda), must take the complex updates.
    Energy and per-rotation gradient (Algorithm 1) against the oracle."""
    announce(f"reverse sweep paths: {case}")
    n, ne = 14, 7
    h, eri = synthetic_integrals(n, 1000 + n)
    ham = jordan_wigner(h, eri)
    hx, hz, hc = np.asarray(ham.x, np.uint64), np.asarray(ham.z, np.uint64), np.asarray(ham.c)
    if case == "complex_sum":
        rx_, rz_, rc_ = random_pauli_sum(n, 200, 5100)
        odd = np.array([pauli.popcount(int(a) & int(b)) % 2 == 1 for a, b in zip(rx_, rz_)])
        hx = np.concatenate([hx, rx_[odd]]); hz = np.concatenate([hz, rz_[odd]]); hc = np.concatenate([hc, rc_[odd]])
    rot = uccsd_rotations(n, ne, ORDER)
    phi = rot.angles(uniform_amplitudes(rot.n_params, 0.1, 5101))
    if case == "complex_start":
        rng = np.random.default_rng(5102)
        psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        psi0 /= np.linalg.norm(psi0)
    else:
        psi0 = osv.basis_state(n, (1 << ne) - 1)
    e_ref, g_ref = osv.reverse_mode_gradient(psi0, hx, hz, hc, rot.x, rot.z, phi)
    psi = StateVector(n, "c128"); lam = StateVector(n, "c128")
    psi.amps.copy_(torch.from_numpy(np.asarray(psi0, np.complex128)))
    psi.apply_rotations(rot.x, rot.z, phi)
    energy = torch.empty(2, dtype=torch.float64, device="cuda")
    grad = torch.empty(len(phi), dtype=torch.float64, device="cuda")
    B.sv_adjoint_grad(psi.handle, lam.handle, hx, hz, hc, rot.x, rot.z, phi, energy, grad)
    torch.cuda.synchronize()
    scale = max(1.0, float(np.abs(hc).sum()))
    assert abs(energy[0].item() - e_ref) <= 1e-12 * scale
    assert np.abs(grad.cpu().numpy() - g_ref).max() <= 1e-12 * scale
    assert np.abs(to_np_state(psi.amps) - psi0).max() < 1e-12
    psi.free(); lam.free()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", ["real_psi", "one_imag"])
def test_lambda_real_tiling_at_21_qubits(case, dtype):
    """At 21 qubits the real-coefficient build of lambda = H psi takes 13-qubit
    real-part tiles when psi is real (enough tiles to fill the device), and
    the complex 12-qubit build when one amplitude has an imaginary part.
    Element by element against the oracle, on a seeded sum of even-Y strings
    of weight <= 4 (real coefficients).  complex64: the oracle takes the
    state's own rounded amplitudes; lambda is accumulated in FP64 within a
    pass but kept in complex64 between passes, so each pass rounds it once:
    |error| <= u (passes) ||c||_1 max|psi| with u = 2^-24 and at most one pass
    per x-group plus one."""
    announce(f"lambda 21 qubits: {case} {dtype}")
    n = 21
    rx_, rz_, rc_ = random_pauli_sum(n, 300, 5200)
    even = np.array([pauli.popcount(int(a) & int(b)) % 2 == 0 for a, b in zip(rx_, rz_)])
    hx, hz, hc = rx_[even], rz_[even], rc_[even]
    rng = np.random.default_rng(5201)
    v = rng.normal(size=1 << n).astype(np.complex128)
    if case == "one_imag":
        v[(1 << 20) + 12345] += 1e-3j
    v /= np.linalg.norm(v)
    psi = StateVector(n, dtype); lam = StateVector(n, dtype)
    psi.amps.copy_(torch.from_numpy(v).to(psi.amps.dtype))
    v = to_np_state(psi.amps)  # the amplitudes as stored (rounded for complex64)
    energy = torch.empty(2, dtype=torch.float64, device="cuda")
    grad = torch.empty(1, dtype=torch.float64, device="cuda")
    B.sv_adjoint_grad(psi.handle, lam.handle, hx, hz, hc, np.array([1], np.uint64), np.array([1], np.uint64),
                      np.array([0.0]), energy, grad)
    torch.cuda.synchronize()
    want = osv.apply_hamiltonian(v, hx, hz, hc)
    got = to_np_state(lam.amps)
    scale = max(1.0, float(np.abs(hc).sum()))
    passes = len(set(int(x) for x in hx)) + 1
    tol = 1e-12 * scale if dtype == "c128" else 2.0 ** -24 * passes * float(np.abs(hc).sum()) * float(np.abs(v).max())
    assert np.abs(got - want).max() <= tol
    e_ref = float(np.vdot(v, want).real / np.vdot(v, v).real)  # Rayleigh quotient from the oracle's H psi
    e_tol = 1e-12 * scale if dtype == "c128" else 1e-6 * scale
    assert abs(energy[0].item() - e_ref) <= e_tol
    psi.free(); lam.free()


@pytest.mark.parametrize("case", ["real_psi", "one_imag"])
def test_real_hint_at_21_qubits(case):
    """sv_set_real_hint: with psi declared real the adjoint call builds lambda
    on the real-part tiling without a stream wait.  A real psi gives the
    oracle's H psi; a psi with one imaginary amplitude (a wrong declaration)
    must give NaN in lambda and the energy, never a silently wrong value."""
    announce(f"real hint 21 qubits: {case}")
    n = 21
    rx_, rz_, rc_ = random_pauli_sum(n, 300, 5200)
    even = np.array([pauli.popcount(int(a) & int(b)) % 2 == 0 for a, b in zip(rx_, rz_)])
    hx, hz, hc = rx_[even], rz_[even], rc_[even]
    rng = np.random.default_rng(5201)
    v = rng.normal(size=1 << n).astype(np.complex128)
    if case == "one_imag":
        v[(1 << 20) + 12345] += 1e-3j
    v /= np.linalg.norm(v)
    psi = StateVector(n, "c128"); lam = StateVector(n, "c128")
    psi.amps.copy_(torch.from_numpy(v))
    B.sv_set_real_hint(psi.handle, True)
    energy = torch.empty(2, dtype=torch.float64, device="cuda")
    grad = torch.empty(1, dtype=torch.float64, device="cuda")
    B.sv_adjoint_grad(psi.handle, lam.handle, hx, hz, hc, np.array([1], np.uint64), np.array([1], np.uint64),
                      np.array([0.0]), energy, grad)
    torch.cuda.synchronize()
    got = to_np_state(lam.amps)
    if case == "real_psi":
        want = osv.apply_hamiltonian(v, hx, hz, hc)
        assert np.abs(got - want).max() <= 1e-12 * max(1.0, float(np.abs(hc).sum()))
        assert np.isfinite(energy[0].item())
    else:
        assert np.isnan(energy[0].item()) and np.isnan(grad[0].item())
        assert np.isnan(got.real).all()
    psi.free(); lam.free()


@pytest.mark.parametrize("n,dtype", [(14, "c128"), (22, "c128"), (22, "c64"), (22, "r64")])
def test_lambda_and_gradient_are_bitwise_reproducible(n, dtype):
    """lambda = H psi, the energy and the per-rotation gradient of repeated
    adjoint calls on the same input are bitwise equal, on one pair of states
    and on a second pair: lambda's sums are fixed point (integer atomic
    adds, whose order does not matter) and every reduction has a fixed
    order.  14 qubits takes the complex build, 22 qubits the real-part tiles
    (a UCCSD state is real)."""
    announce(f"lambda thrice, bitwise: {n} qubits {dtype}")
    ne = n // 2
    h, eri = synthetic_integrals(n, 1000 + n)
    ham = jordan_wigner(h, eri)
    rot = uccsd_rotations(n, ne, ORDER)
    phi = rot.angles(uniform_amplitudes(rot.n_params, 0.1, 5300 + n))
    states = [(StateVector(n, dtype), StateVector(n, dtype)), (StateVector(n, dtype), StateVector(n, dtype))]
    out = []
    for psi, lam in (states[0], states[0], states[1]):
        energy = torch.empty(2, dtype=torch.float64, device="cuda")
        grad = torch.empty(len(phi), dtype=torch.float64, device="cuda")
        psi.prepare_hf((1 << ne) - 1)
        psi.apply_rotations(rot.x, rot.z, phi)
        B.sv_adjoint_grad(psi.handle, lam.handle, ham.x, ham.z, ham.c, rot.x, rot.z, phi, energy, grad)
        torch.cuda.synchronize()
        out.append((energy.clone(), grad.clone(), lam.amps.clone()))
    for psi, lam in states:
        psi.free(); lam.free()
    (e1, g1, l1) = out[0]
    assert torch.isfinite(g1).all() and float(g1.abs().max()) > 0.0
    for e2, g2, l2 in out[1:]:
        assert torch.equal(e1, e2)
        assert torch.equal(g1, g2)
        assert torch.equal(l1, l2)


@pytest.mark.parametrize("n,dtype,k", [(14, "c128", 300), (14, "c128", -300), (22, "r64", 300), (22, "r64", -300),
                                       (14, "c64", 20), (14, "c64", -20)])
def test_lambda_fixed_point_follows_the_state_scale(n, dtype, k):
    """The fixed-point sums of lambda take their scale from psi's largest
    amplitude, so scaling psi by 2^k (exact in floating point) scales lambda
    by exactly 2^k and the gradient by 4^k, bit for bit,
    and leaves the energy <psi|H|psi>/<psi|psi> bitwise unchanged, far from
    unit norm in both directions (complex64 lambda, stored in FP32 after the
    reverse sweep: to one FP32 unit where it is a normal number)."""
    announce(f"lambda under psi * 2^{k}: {n} qubits {dtype}")
    ne = n // 2
    h, eri = synthetic_integrals(n, 1000 + n)
    ham = jordan_wigner(h, eri)
    rot = uccsd_rotations(n, ne, ORDER)
    phi = rot.angles(uniform_amplitudes(rot.n_params, 0.1, 5400 + n))
    psi = StateVector(n, dtype); lam = StateVector(n, dtype)
    out = []
    for scale in (1.0, 2.0 ** k):
        energy = torch.empty(2, dtype=torch.float64, device="cuda")
        grad = torch.empty(len(phi), dtype=torch.float64, device="cuda")
        psi.prepare_hf((1 << ne) - 1)
        psi.apply_rotations(rot.x, rot.z, phi)
        psi.amps.mul_(scale)
        B.sv_adjoint_grad(psi.handle, lam.handle, ham.x, ham.z, ham.c, rot.x, rot.z, phi, energy, grad)
        torch.cuda.synchronize()
        out.append((energy.clone(), grad.clone(), lam.amps.clone()))
    psi.free(); lam.free()
    (e1, g1, l1), (e2, g2, l2) = out
    assert float(g1.abs().max()) > 0.0
    assert torch.equal(e2[0], e1[0])
    assert torch.equal(e2[1], e1[1] * 4.0 ** k)
    assert torch.equal(g2, g1 * 4.0 ** k)
    if dtype == "c64":
        # complex64 lambda after the FP32 reverse sweep: subnormal FP32
        # intermediates (tiny amplitudes) round differently at each scale, so
        # to one FP32 unit where the value is well inside the normal range
        a, b = torch.view_as_real(l1).double(), torch.view_as_real(l2).double()
        normal = a.abs() >= 2.0 ** -60  # far above the subnormal range at both scales
        assert int(normal.sum()) >= 1000
        assert torch.all((b[normal] - a[normal] * 2.0 ** k).abs() <= 2.0 ** -23 * (a[normal] * 2.0 ** k).abs())
    else:
        assert torch.equal(l2, l1 * 2.0 ** k)


@pytest.mark.parametrize("dtype", ["c128", "r64"])
def test_lambda_of_a_zero_state_is_zero(dtype):
    """A zero psi gives lambda = H psi = 0 exactly, also with coefficients
    scaled by 2^40: the fixed-point scale of a zero state stays finite (its
    amplitude exponent is floored), so no term becomes inf * 0."""
    announce(f"lambda of a zero state: 22 qubits {dtype}")
    n = 22
    h, eri = synthetic_integrals(n, 1000 + n)
    ham = jordan_wigner(h, eri)
    coef = np.asarray(ham.c, dtype=np.float64) * 2.0 ** 40
    psi = StateVector(n, dtype); lam = StateVector(n, dtype)
    psi.amps.zero_()
    energy = torch.empty(2, dtype=torch.float64, device="cuda")
    grad = torch.empty(1, dtype=torch.float64, device="cuda")
    # one rotation by angle 0 on a real string (a Y on qubit 0)
    B.sv_adjoint_grad(psi.handle, lam.handle, ham.x, ham.z, coef, np.array([1], np.uint64),
                      np.array([1], np.uint64), np.array([0.0]), energy, grad)
    torch.cuda.synchronize()
    values = torch.view_as_real(lam.amps) if lam.amps.is_complex() else lam.amps
    assert int(torch.count_nonzero(values)) == 0
    assert float(grad[0].item()) == 0.0
    psi.free(); lam.free()
