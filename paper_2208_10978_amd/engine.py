"""Device-resident objects over the C ABI and the UCC energy autograd Function.

``StateVector``   a 2^n complex (or, for real circuits, real FP64) torch
                  tensor on the GPU bound to an sv_state
``Hamiltonian``   a Pauli sum grouped and uploaded once (sv_hamiltonian)
``UCCSDEvaluator`` energy and energy+gradient of the Trotterised UCCSD state
                  (Eq. 10-11) for a fixed Hamiltonian and rotation list, both
                  resident in the library: HF preparation, the rotation sweep,
                  the grouped expectation or lambda = H psi with the reverse
                  sweep (Algorithm 1)
``UCCEnergy``     torch.autograd.Function whose backward returns dE/dtheta
                  computed by the reverse sweep
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B
from .problem import PauliSum, RotationList

_DT = {"c128": (B.SV_C128, torch.complex128), "c64": (B.SV_C64, torch.complex64),
       "r64": (B.SV_R64, torch.float64)}


class StateVector:
    def __init__(self, n_qubits: int, dtype: str = "c128", device: str = "cuda", stream=None):
        code, tdt = _DT[dtype]
        self.n = int(n_qubits)
        self.dtype = dtype
        self.amps = torch.empty(1 << self.n, dtype=tdt, device=device)
        self.stream = stream
        self.handle = B.sv_alloc(self.n, code, self.amps, stream)

    def clone(self) -> "StateVector":
        """A new state with a copy of these amplitudes (same n, dtype, stream)."""
        c = StateVector(self.n, self.dtype, device=self.amps.device, stream=self.stream)
        c.amps.copy_(self.amps)
        return c

    def overlap(self, other: "StateVector", out=None) -> torch.Tensor:
        """<self|other> as a device FP64 tensor (re, im)."""
        out = out if out is not None else torch.empty(2, dtype=torch.float64, device=self.amps.device)
        B.sv_overlap(self.handle, other.handle, out)
        return out

    def prepare_hf(self, occ_mask: int):
        B.sv_prepare_hf(self.handle, occ_mask)

    def apply_rotations(self, x, z, phi):
        B.sv_apply_pauli_rotations(self.handle, x, z, phi)

    def expect(self, h: "Hamiltonian", out=None) -> torch.Tensor:
        out = out if out is not None else torch.empty(2, dtype=torch.float64, device=self.amps.device)
        B.sv_expect_hamiltonian(self.handle, h.handle, out)
        return out

    def expect_terms(self, x, z, c, out=None) -> torch.Tensor:
        out = out if out is not None else torch.empty(2, dtype=torch.float64, device=self.amps.device)
        B.sv_expect_pauli_sum(self.handle, x, z, c, out)
        return out

    def normalize(self, out=None):
        B.sv_normalize(self.handle, out)

    def amplitudes(self, idx) -> torch.Tensor:
        out = torch.empty(2 * len(idx), dtype=torch.float64, device=self.amps.device)
        B.sv_gather_amplitudes(self.handle, idx, out)
        return out

    def set_stream(self, stream):
        B.sv_set_stream(self.handle, stream)

    def free(self):
        if self.handle is not None:
            B.sv_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Hamiltonian:
    def __init__(self, ps: PauliSum):
        self.n = ps.n_qubits
        self.terms = ps
        self.handle = B.sv_hamiltonian_create(ps.n_qubits, ps.x, ps.z, ps.c)

    def free(self):
        if self.handle is not None:
            B.sv_hamiltonian_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class UCCSDEvaluator:
    """E(theta) = <HF| U(theta)^dag H U(theta) |HF> and its gradient.

    ``dtype``: "c128", "c64", or "r64" (real FP64 amplitudes, for circuits of
    real rotations such as UCCSD with a real Hamiltonian: the same results as
    "c128" with half the bytes).  ``renormalize`` rescales psi to unit norm
    (FP64 norm) after the forward sweep; it is on by default for complex64
    amplitudes.  Results are bitwise equal from run to run (lambda = H psi
    is summed in fixed point, the reductions in a fixed order)."""

    def __init__(self, ham: PauliSum, rot: RotationList, n_electrons: int, dtype: str = "c128",
                 stream=None, renormalize=None, hamiltonian: "Hamiltonian" = None):
        self.n = ham.n_qubits
        self.rot = rot
        self.hf = (1 << n_electrons) - 1
        # a resident Hamiltonian may be shared (then the caller frees it)
        self.own_h = hamiltonian is None
        self.h = Hamiltonian(ham) if hamiltonian is None else hamiltonian
        self.psi = StateVector(self.n, dtype, stream=stream)
        self.lam = StateVector(self.n, dtype, stream=stream)
        # HF is real and a rotation whose string has an odd number of Y
        # factors is a real orthogonal matrix, so with such a list psi stays
        # real: the library may then build lambda without a stream wait (it
        # still checks on the device, and a wrong declaration gives NaN)
        x = np.asarray(rot.x, dtype=np.uint64)
        z = np.asarray(rot.z, dtype=np.uint64)
        self.real_circuit = bool(np.all(np.bitwise_count(x & z) % 2 == 1))
        B.sv_set_real_hint(self.psi.handle, self.real_circuit)
        # the rotation list resident in the library: split and scheduled once
        self.rh = B.sv_rotations_create(self.n, rot.x, rot.z, rot.param, rot.dphi_dtheta, rot.n_params)
        self.renormalize = (dtype == "c64") if renormalize is None else renormalize
        dev = self.psi.amps.device
        self.energy_buf = torch.empty(2, dtype=torch.float64, device=dev)
        self.grad_buf = torch.empty(rot.n_params, dtype=torch.float64, device=dev)

    def forward_state(self, theta):
        th = np.asarray(theta, dtype=np.float64)
        self.psi.prepare_hf(self.hf)
        B.sv_apply_rotations_h(self.psi.handle, self.rh, th)
        if self.renormalize:
            self.psi.normalize()
        return self.rot.angles(th)

    def energy(self, theta) -> torch.Tensor:
        """Device tensor [E, <psi|psi>] (E is the Rayleigh quotient)."""
        self.forward_state(theta)
        return self.psi.expect(self.h, self.energy_buf)

    def energy_and_grad(self, theta):
        th = np.asarray(theta, dtype=np.float64)
        self.forward_state(th)
        B.sv_adjoint_grad_params_hr(self.psi.handle, self.lam.handle, self.h.handle, self.rh, th, self.energy_buf,
                                    self.grad_buf)
        return self.energy_buf, self.grad_buf

    def pool_gradients(self, theta, pool: RotationList) -> torch.Tensor:
        """ADAPT operator-pool screening (Section 5.1): dE/dtheta_A at
        theta_A = 0 for every pool operator A appended after the circuit.
        The pool's rotations are the identity there, so one reverse sweep over
        the pool alone (Algorithm 1 with lambda = H psi) gives every
        Im <lambda|P|psi> of its strings.  Returns a device float64 tensor of
        pool.n_params entries; psi is left at U(theta)|HF>."""
        self.forward_state(theta)
        out = torch.empty(pool.n_params, dtype=torch.float64, device=self.psi.amps.device)
        B.sv_adjoint_grad_params_h(self.psi.handle, self.lam.handle, self.h.handle, pool.x, pool.z,
                                   np.zeros(len(pool)), pool.param, pool.dphi_dtheta, pool.n_params,
                                   self.energy_buf, out)
        return out

    def energy_and_grad_deflated(self, theta, lower, alphas):
        """Variational quantum deflation (Eq. 12): energy and dE/dtheta of
        <psi|H_eff|psi>, H_eff = H + sum_j alphas[j] |lower_j><lower_j|, with
        the lower states as StateVectors.  Returns device tensors
        (energy[2], grad[n_params], overlaps <lower_j|psi> as (re, im) pairs)."""
        phi = self.forward_state(theta)
        ovl = torch.empty(max(1, 2 * len(lower)), dtype=torch.float64, device=self.psi.amps.device)
        B.sv_adjoint_grad_params_deflated(self.psi.handle, self.lam.handle, self.h.handle,
                                          [s.handle for s in lower], list(alphas), self.rot.x, self.rot.z, phi,
                                          self.rot.param, self.rot.dphi_dtheta, self.rot.n_params,
                                          self.energy_buf, ovl if lower else None, self.grad_buf)
        return self.energy_buf, self.grad_buf, ovl[:2 * len(lower)]

    def state(self, theta) -> StateVector:
        """U(theta)|HF> as a new StateVector."""
        self.forward_state(theta)
        return self.psi.clone()

    def free_states(self):
        """Release the states and the resident rotation list (a shared
        Hamiltonian stays)."""
        self.psi.free()
        self.lam.free()
        if self.rh is not None:
            B.sv_rotations_free(self.rh)
            self.rh = None

    def free(self):
        self.free_states()
        if self.own_h:
            self.h.free()


class UCCEnergy(torch.autograd.Function):
    """``E = UCCEnergy.apply(theta, evaluator)``; theta is a float64 tensor.
    With gradients enabled the forward pass runs the reverse sweep as well and
    keeps dE/dtheta for the backward pass."""

    @staticmethod
    def forward(ctx, theta, evaluator):
        th = theta.detach().to("cpu", torch.float64).numpy()
        if ctx.needs_input_grad[0]:
            e, g = evaluator.energy_and_grad(th)
            ctx.save_for_backward(g.clone())
        else:
            e = evaluator.energy(th)
        return e[0].clone().to(theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return (grad_out.to(g.device) * g).to(grad_out.device), None
