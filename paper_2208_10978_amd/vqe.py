"""The variational outer loop of Eq. 9: minimise E(theta) with a
quasi-Newton optimiser driven by the adjoint gradient (Algorithm 1).

``vqe(fun_and_grad, theta0)`` is generic: ``fun_and_grad(theta)`` returns
``(E, dE/dtheta)`` as host values.  ``evaluator_objective`` wraps a
``UCCSDEvaluator`` (any rotation list: UCCSD, UCCGSD, ADAPT-grown) so every
evaluation runs on the GPU; only the scalar energy and the gradient vector
cross to the host for the optimiser.

``vqd`` runs the deflation sequence of Eq. 12 and ``adapt_vqe`` grows a
circuit from an operator pool (Section 5.1: fermionic UCCGSD, qubit-
excitation or Pauli-entangler pools), screening the pool with one reverse
sweep per iteration.
"""
from __future__ import annotations

import time

import numpy as np
from scipy.optimize import minimize


def evaluator_objective(evaluator):
    def fun_and_grad(theta):
        e, g = evaluator.energy_and_grad(np.asarray(theta, dtype=np.float64))
        return float(e[0].item()), g.detach().to("cpu").numpy().astype(np.float64)
    return fun_and_grad


def vqe(fun_and_grad, theta0, maxiter: int = 200, gtol: float = 1e-9, method: str = "L-BFGS-B"):
    """Returns a dict with the minimum energy, the amplitudes, the numbers
    of iterations and evaluations, the energy after each iteration and the
    wall time per evaluation."""
    history = []
    n_eval = [0]
    last = [None, None]  # the latest evaluated point and energy
    t0 = time.perf_counter()

    def f(th):
        n_eval[0] += 1
        e, g = fun_and_grad(th)
        last[0], last[1] = np.array(th, copy=True), e
        return e, g

    def record(th):
        history.append(last[1] if last[0] is not None and np.array_equal(th, last[0]) else f(th)[0])

    res = minimize(f, np.asarray(theta0, dtype=np.float64), jac=True, method=method,
                   options={"maxiter": maxiter, "gtol": gtol, "ftol": 1e-15}, callback=record)
    wall = time.perf_counter() - t0
    return {"energy": float(res.fun), "theta": np.asarray(res.x), "n_iter": int(res.nit), "n_eval": n_eval[0],
            "history": history, "converged": bool(res.success), "seconds_per_eval": wall / max(1, n_eval[0])}


def deflated_objective(evaluator, lower, alphas):
    """(energy, gradient) of Eq. 12's effective Hamiltonian on the device."""
    def fun_and_grad(theta):
        e, g, _ = evaluator.energy_and_grad_deflated(np.asarray(theta, dtype=np.float64), lower, alphas)
        return float(e[0].item()), g.detach().to("cpu").numpy().astype(np.float64)
    return fun_and_grad


def vqd(evaluator, n_states: int, alpha: float, theta0s, maxiter: int = 200, gtol: float = 1e-9):
    """Variational quantum deflation (Section 5.1, Eq. 12): state k minimizes
    <psi|H_eff^k|psi>, H_eff^k = H_eff^{k-1} + alpha |Psi_{k-1}><Psi_{k-1}|,
    starting from theta0s[k] (one start, or a list of starts whose best
    minimum is kept).  Returns one dict per state: the minimum of the
    effective energy, the plain energy <H> there, the amplitudes, and the
    state itself (a StateVector; the caller frees it)."""
    lower, out = [], []
    for k in range(n_states):
        starts = theta0s[k]
        starts = [starts] if np.ndim(starts[0]) == 0 else starts
        f = deflated_objective(evaluator, lower, [alpha] * len(lower))
        best = min((vqe(f, t0, maxiter=maxiter, gtol=gtol) for t0 in starts), key=lambda r: r["energy"])
        e_h = float(evaluator.energy(best["theta"])[0].item())
        st = evaluator.state(best["theta"])
        lower.append(st)
        out.append({"energy_eff": best["energy"], "energy": e_h, "theta": best["theta"], "state": st,
                    "n_eval": best["n_eval"], "converged": best["converged"]})
    return out


def adapt_vqe(make_objective, screen, pool, n_qubits: int, max_ops: int = 20, grad_tol: float = 1e-6,
              maxiter: int = 200, gtol: float = 1e-9):
    """ADAPT-VQE (Section 5.1).  ``pool`` is a RotationList whose parameters
    are the pool operators.  Each iteration screens the pool at the current
    optimum (``screen(circuit, theta, pool)`` -> dE/dtheta_A of every pool
    operator appended with amplitude 0), appends the operator of largest
    magnitude, and re-optimises every amplitude (Eq. 9) from the previous
    optimum with 0 for the new one; ``make_objective(circuit)`` gives the
    (E, grad) callable.  Stops when the largest magnitude is below grad_tol
    or after max_ops operators.  Returns the circuit, amplitudes, chosen pool
    indices and the energy and largest screening gradient per iteration."""
    from .problem import concat_rotations, empty_rotations, operator_of

    circuit = empty_rotations(n_qubits)
    theta = np.zeros(0)
    chosen, energies, gmax = [], [], []
    for _ in range(max_ops):
        g = np.asarray(screen(circuit, theta, pool), dtype=np.float64)
        k = int(np.argmax(np.abs(g)))
        gmax.append(float(abs(g[k])))
        if gmax[-1] < grad_tol:
            break
        chosen.append(k)
        circuit = concat_rotations(circuit, operator_of(pool, k, 0))
        res = vqe(make_objective(circuit), np.append(theta, 0.0), maxiter=maxiter, gtol=gtol)
        theta = res["theta"]
        energies.append(res["energy"])
    return {"circuit": circuit, "theta": theta, "chosen": chosen, "energies": energies, "max_gradients": gmax}


def gpu_adapt_vqe(ham, n_electrons: int, pool, dtype: str = "c128", **kw):
    """adapt_vqe with every energy, gradient and pool screening on the GPU
    (one evaluator per circuit length, all sharing one resident Hamiltonian)."""
    from .engine import Hamiltonian, UCCSDEvaluator

    h = Hamiltonian(ham)
    cache = {}

    def evaluator(circuit):
        key = len(circuit)
        if key not in cache:
            for ev in cache.values():
                ev.free_states()
            cache.clear()
            cache[key] = UCCSDEvaluator(ham, circuit, n_electrons, dtype, hamiltonian=h)
        return cache[key]

    def make_objective(circuit):
        return evaluator_objective(evaluator(circuit))

    def screen(circuit, theta, pool_):
        return evaluator(circuit).pool_gradients(theta, pool_).cpu().numpy()

    try:
        return adapt_vqe(make_objective, screen, pool, ham.n_qubits, **kw)
    finally:
        for ev in cache.values():
            ev.free_states()
        h.free()
