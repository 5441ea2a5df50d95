"""The variational outer loop of Eq. 9: minimise E(theta) with a
quasi-Newton optimiser driven by the adjoint gradient (Algorithm 1).

``vqe(fun_and_grad, theta0)`` is generic: ``fun_and_grad(theta)`` returns
``(E, dE/dtheta)`` as host values.  ``evaluator_objective`` wraps a
``UCCSDEvaluator`` (any rotation list: UCCSD, UCCGSD, ADAPT-grown) so every
evaluation runs on the GPU; only the scalar energy and the gradient vector
cross to the host for the optimiser.
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
