"""Resident rotation lists (sv_rotations_create; Eq. 10-11 and Algorithm 1):
the evaluator's calls through the resident list against the calls that plan
the list themselves, on the same states, in every amplitude type; a handle
shared by states of two types; amplitudes with exact zeros; the errors."""
import numpy as np
import pytest
import torch

from paper_2208_10978_amd import binding as B
from paper_2208_10978_amd.engine import Hamiltonian, StateVector, UCCSDEvaluator
from paper_2208_10978_amd.problem import jordan_wigner, uccsd_rotations
from tests.gpu_common import announce
from workloads import synthetic_integrals, uniform_amplitudes

pytestmark = pytest.mark.gpu


def _planned_each_call(ham, rot, ne, dtype, theta):
    """Energy, gradient and state from the calls that plan the list themselves."""
    n = ham.n_qubits
    H = Hamiltonian(ham)
    psi, lam = StateVector(n, dtype), StateVector(n, dtype)
    phi = rot.angles(theta)
    psi.prepare_hf((1 << ne) - 1)
    psi.apply_rotations(rot.x, rot.z, phi)
    if dtype == "c64":
        psi.normalize()
    state = psi.amps.clone()
    e = torch.empty(2, dtype=torch.float64, device="cuda")
    g = torch.empty(rot.n_params, dtype=torch.float64, device="cuda")
    B.sv_adjoint_grad_params_h(psi.handle, lam.handle, H.handle, rot.x, rot.z, phi, rot.param, rot.dphi_dtheta,
                               rot.n_params, e, g)
    torch.cuda.synchronize()
    out = (e.cpu().numpy(), g.cpu().numpy(), state.cpu().numpy())
    psi.free(); lam.free(); H.free()
    return out


@pytest.mark.parametrize("n", [8, 14])
@pytest.mark.parametrize("dtype", ["c128", "c64", "r64"])
def test_resident_list_matches_planning_each_call(n, dtype):
    """Same plan, same arithmetic: the state, energy and gradient are bitwise
    equal (lambda in fixed point on both sides), call after call on one
    handle: all amplitudes nonzero, then some exactly zero (their runs have no
    forward records, so the kept schedule is made again), then nonzero again,
    then all zero (every run the identity: the state stays the HF basis
    state)."""
    announce(f"resident rotations n={n} {dtype}")
    ne = n // 2
    h, eri = synthetic_integrals(n, 1000 + n)
    ham = jordan_wigner(h, eri)
    rot = uccsd_rotations(n, ne)
    base = np.asarray(uniform_amplitudes(rot.n_params, 0.1, 7000 + n))
    zeros = base.copy()
    zeros[::5] = 0.0
    ev = UCCSDEvaluator(ham, rot, ne, dtype)
    for theta in (base, zeros, 0.5 * base, np.zeros_like(base)):
        psi = ev.state(theta)
        e, g = ev.energy_and_grad(theta)
        torch.cuda.synchronize()
        got = (e.cpu().numpy(), g.cpu().numpy(), psi.amps.cpu().numpy())
        psi.free()
        want = _planned_each_call(ham, rot, ne, dtype, theta)
        if not np.any(theta):
            hf_state = np.zeros_like(got[2])
            hf_state[(1 << ne) - 1] = 1
            assert np.array_equal(got[2], hf_state)
        assert np.array_equal(got[2], want[2])
        assert np.array_equal(got[0], want[0])
        assert np.array_equal(got[1], want[1])
    ev.free()


def test_one_handle_serves_two_amplitude_types():
    """One resident list drives a complex128 and a real state (a schedule per
    amplitude type): the two agree to FP64 rounding, and each equals its own
    evaluator's result."""
    announce("resident rotations shared by two types")
    n, ne = 12, 6
    h, eri = synthetic_integrals(n, 1012)
    ham = jordan_wigner(h, eri)
    rot = uccsd_rotations(n, ne)
    theta = uniform_amplitudes(rot.n_params, 0.1, 7100)
    r = B.sv_rotations_create(n, rot.x, rot.z, rot.param, rot.dphi_dtheta, rot.n_params)
    H = Hamiltonian(ham)
    res = {}
    for dt in ("c128", "r64"):
        psi, lam = StateVector(n, dt), StateVector(n, dt)
        psi.prepare_hf((1 << ne) - 1)
        B.sv_apply_rotations_h(psi.handle, r, theta)
        e = torch.empty(2, dtype=torch.float64, device="cuda")
        g = torch.empty(rot.n_params, dtype=torch.float64, device="cuda")
        B.sv_adjoint_grad_params_hr(psi.handle, lam.handle, H.handle, r, theta, e, g)
        torch.cuda.synchronize()
        res[dt] = (e.cpu().numpy(), g.cpu().numpy())
        psi.free(); lam.free()
        ev = UCCSDEvaluator(ham, rot, ne, dt)
        e2, g2 = ev.energy_and_grad(theta)
        torch.cuda.synchronize()
        assert np.array_equal(res[dt][0], e2.cpu().numpy()) and np.array_equal(res[dt][1], g2.cpu().numpy())
        ev.free()
    B.sv_rotations_free(r)
    H.free()
    assert abs(res["c128"][0][0] - res["r64"][0][0]) <= 1e-13 * abs(res["c128"][0][0])
    assert np.abs(res["c128"][1] - res["r64"][1]).max() <= 1e-12 * max(1.0, np.abs(res["c128"][1]).max())


def test_resident_list_errors():
    """A list for another n, a real state given a complex rotation, and a
    non-finite theta are refused before any device work; the state is
    unchanged."""
    announce("resident rotations: errors")
    n = 8
    s = StateVector(n, "r64")
    s.prepare_hf(0b1111)
    before = s.amps.clone()
    r10 = B.sv_rotations_create(10, np.array([3], np.uint64), np.array([1], np.uint64), [0], [1.0], 1)
    with pytest.raises(B.Q2svError) as ei:
        B.sv_apply_rotations_h(s.handle, r10, [0.3])
    assert ei.value.code == B.SV_EINVAL
    rc = B.sv_rotations_create(n, np.array([3], np.uint64), np.array([0], np.uint64), [0], [1.0], 1)  # X X: complex
    with pytest.raises(B.Q2svError) as ei:
        B.sv_apply_rotations_h(s.handle, rc, [0.3])
    assert ei.value.code == B.SV_EINVAL
    rr = B.sv_rotations_create(n, np.array([3], np.uint64), np.array([1], np.uint64), [0], [1.0], 1)  # Y X: real
    with pytest.raises(B.Q2svError) as ei:
        B.sv_apply_rotations_h(s.handle, rr, [float("inf")])
    assert ei.value.code == B.SV_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(s.amps, before)
    for r in (r10, rc, rr):
        B.sv_rotations_free(r)
    s.free()
