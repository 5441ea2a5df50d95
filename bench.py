#!/usr/bin/env python3
"""Benchmark of the UCCSD state-vector path on one MI355X.

Workload (default): 28 qubits, 14 electrons, real FP64 amplitudes (the
UCCSD state of a real Hamiltonian is real; the complex128 step is timed
beside it).  Seeded synthetic
integrals (seed 1028) -> JW Pauli sum truncated at |c| > 1e-6; spin-orbital
UCCSD with 3,381 amplitudes theta ~ U[-0.02, 0.02] (seed 2028) -> 26,460
Pauli rotations.  One step is one energy + full adjoint gradient evaluation:
HF preparation, the rotation sweep, lambda = H psi with the energy, and the
reverse sweep with dE/dtheta (Algorithm 1).  The Hamiltonian is resident in
HBM (grouped and uploaded once, outside the timed region), as in a VQE loop
where H is fixed and theta changes.

Prints one JSON line.  ``value`` is energy+gradient evaluations per second.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


AMP_LABEL = {"r64": "real FP64 amplitudes (the UCCSD state of a real Hamiltonian is real; complex128 gives the same "
                    "results with exactly zero imaginary parts)",
             "c128": "complex128", "c64": "complex64 with FP64 reductions"}


def step_c128(ham, rot, ne, theta, steps, energy_r64):
    """The same energy + gradient step on complex128 states, timed after one
    warm-up: its time per step and per kernel class, and its distance from
    the real-state energy."""
    import torch
    from paper_2208_10978_amd import binding as B
    from paper_2208_10978_amd.engine import UCCSDEvaluator
    ev = UCCSDEvaluator(ham, rot, ne, "c128")
    ev.energy_and_grad(theta)
    torch.cuda.synchronize()
    B.sv_profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        e, _ = ev.energy_and_grad(theta)
        torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    prof = B.sv_profile_end()
    out = {"ms_per_step": 1e3 * dt, "evals_per_s": 1.0 / dt, "steps": steps,
           "energy_minus_real_state": float(e[0].item()) - energy_r64,
           "kernels_ms_per_step": {k: round(v["ms"] / steps, 3) for k, v in prof.items()}}
    ev.free()
    log(f"complex128 step: {1e3 * dt:.1f} ms")
    return out


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor()


TRAFFIC_FILES = {d: os.path.join(ROOT, "profiles", f"hbm_traffic_uccsd_28q_{d}.md") for d in ("r64", "c128")}
KERNEL_SOURCES = ["kernels_sweep.hip", "kernels_pauli_sum.hip", "device_common.h", "q2sv_internal.h", "launch.h",
                  "plan.cpp"]


def measured_traffic(kernel_class: str, n: int, dtype: str):
    """HBM bytes per launch of a tile kernel class from the committed counter
    summary (calibrated FETCH_SIZE + WRITE_SIZE), or None when the summary is
    for another workload or the kernel sources changed since it was taken."""
    import hashlib
    if n != 28 or dtype not in TRAFFIC_FILES or not os.path.exists(TRAFFIC_FILES[dtype]):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2208_10978_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    text = open(TRAFFIC_FILES[dtype]).read()
    if f"`{h.hexdigest()[:16]}`" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip("|").split("|")]
        if len(cells) == 5 and cells[0] == kernel_class:
            return int(cells[4])
    return None


def _oracle_terms_worker(args):
    """One process of the all-cores leg: the oracle's expectation (term by
    term, Eq. 2) over its share of the Pauli terms on a 2^n state of its own;
    returns the seconds spent in the oracle call."""
    n, xs, zs, cs = args
    from threadpoolctl import threadpool_limits

    from oracle import statevector as osv
    with threadpool_limits(limits=1):
        psi = osv.basis_state(n, (1 << (n // 2)) - 1)
        t0 = time.perf_counter()
        osv.expectation(psi, xs, zs, cs)
        return time.perf_counter() - t0


def _oracle_unit_times(n, rot, ham, k_rot=1, k_term=1):
    """Seconds per rotation, per Pauli-string application and per inner
    product of the oracle on a 2^n state (one thread), each averaged over a
    few calls."""
    from oracle import pauli as op
    from oracle import statevector as osv
    psi = osv.basis_state(n, (1 << (n // 2)) - 1)
    t0 = time.perf_counter()
    for k in range(k_rot):
        psi = osv.rotate(psi, int(rot.x[k]), int(rot.z[k]), 0.01)
    t_rot = (time.perf_counter() - t0) / k_rot
    t0 = time.perf_counter()
    for k in range(k_term):
        lam = float(ham.c[k]) * op.apply(psi, int(ham.x[k]), int(ham.z[k]))
    t_term = (time.perf_counter() - t0) / k_term
    t0 = time.perf_counter()
    for _ in range(k_term):
        np.vdot(lam, psi)
    t_dot = (time.perf_counter() - t0) / k_term
    return t_rot, t_term, t_dot


def _algorithm1_seconds(R, T, t_rot, t_term, t_dot, term_rate=None):
    """Seconds of one energy + gradient evaluation by Algorithm 1 as the
    oracle performs it: R rotations forward; H psi as T string
    applications (at term_rate strings/s when the terms are shared among
    processes); backward, per rotation, two inverse rotations, one rotation
    and one string application for dU psi, one inner product."""
    h_side = T / term_rate if term_rate else T * t_term
    return R * t_rot + h_side + R * (3 * t_rot + t_term + t_dot)


def cpu_baseline(n, ham, rot, theta):
    """The oracle (NumPy, FP64) timed on this host on bounded samples.

    * One core, at the full size: one rotation, one Pauli-string application
      and one inner product on a 2^n state, scaled to the operation counts
      of one energy + gradient evaluation by Algorithm 1.
    * All cores, at the full size: the paper's own host parallelism
      (Section 5.2) shares the Pauli terms among processes and sums their
      partial results.  P processes each apply the oracle's expectation to
      one term on a state of their own; the H side of the evaluation is
      scaled by the P-process rate, while the rotation chain (forward and
      backward), which the oracle applies one rotation at a time over the
      whole vector, stays on one core.
    * The 8-qubit configuration in full (energy + gradient by the oracle's
      Algorithm 1), and the 20-qubit one from samples of 20 rotations and 50
      string applications, scaled to its counts (labelled extrapolated)."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle import fermion
    from oracle import statevector as osv
    from paper_2208_10978_amd.problem import jordan_wigner, uccsd_rotations
    from workloads import synthetic_integrals, uniform_amplitudes

    R, T = len(rot), len(ham)
    with threadpool_limits(limits=1):  # one thread for BLAS/OpenMP pools too
        t_rot, t_term, t_dot = _oracle_unit_times(n, rot, ham)
    per_eval_1 = _algorithm1_seconds(R, T, t_rot, t_term, t_dot)

    procs = max(1, min(8, os.cpu_count() or 1))
    jobs = [(n, [int(ham.x[k])], [int(ham.z[k])], [float(ham.c[k])]) for k in range(procs)]
    with mp.get_context("spawn").Pool(procs) as pool:
        pool.map(_oracle_terms_worker, [(10, a, b, c) for _, a, b, c in jobs])  # interpreter start-up
        spent = pool.map(_oracle_terms_worker, jobs)
    term_rate = procs / max(spent)
    per_eval_p = _algorithm1_seconds(R, T, t_rot, t_term, t_dot, term_rate)

    small = {}
    with threadpool_limits(limits=1):
        h8, eri8 = synthetic_integrals(8, 1008)
        terms = fermion.jw_hamiltonian(h8, eri8)
        rots = fermion.uccsd_rotations(8, 4)
        th = uniform_amplitudes(len({r[2] for r in rots}), 0.1, 2008)
        t0 = time.perf_counter()
        osv.reverse_mode_gradient(osv.basis_state(8, fermion.hf_index(4)), [k[0] for k in terms],
                                  [k[1] for k in terms], list(terms.values()), [r[0] for r in rots],
                                  [r[1] for r in rots], [d * th[p] for _, _, p, d in rots])
        small["8q_energy_grad_s"] = time.perf_counter() - t0
        h20, eri20 = synthetic_integrals(20, 1020)
        ham20 = jordan_wigner(h20, eri20)
        rot20 = uccsd_rotations(20, 10)
        u = _oracle_unit_times(20, rot20, ham20, k_rot=20, k_term=50)
        small["20q_energy_grad_s_extrapolated"] = _algorithm1_seconds(len(rot20), len(ham20), *u)
        small["20q_sample"] = (f"20 rotations ({u[0] * 1e3:.1f} ms each), 50 string applications "
                               f"({u[1] * 1e3:.1f} ms) and inner products ({u[2] * 1e3:.1f} ms), scaled to "
                               f"{len(rot20)} rotations and {len(ham20)} terms")
    return {
        "value": 1.0 / per_eval_p,
        "unit": "energy+grad evals/s",
        "cores": procs,
        "kind": "oracle",
        "sample": (f"oracle at {n} qubits: {procs} processes applying one Pauli term each "
                   f"({max(spent):.2f} s, {term_rate:.2f} terms/s) for the H side; the rotation chain on one core "
                   f"(1 rotation {t_rot:.2f} s, 1 string application {t_term:.2f} s, 1 inner product "
                   f"{t_dot:.2f} s); extrapolated to {R} rotations and {T} terms of one Algorithm-1 evaluation "
                   f"({per_eval_p / 3600:.1f} h)"),
        "single_core": {"value": 1.0 / per_eval_1, "cores": 1,
                        "sample": (f"the same per-operation times on one core, extrapolated "
                                   f"({per_eval_1 / 3600:.1f} h)")},
        "small_configs_oracle": small,
        "host": cpu_model(),
        "nproc": os.cpu_count(),
    }


def bench_c4(n_rot: int, n_terms: int):
    """32 qubits, complex64 (32 GiB): a prefix of the random 4-qubit-support
    rotation stream and the expectation of a random weight<=4 Pauli sum."""
    import torch
    from paper_2208_10978_amd import binding as B
    from paper_2208_10978_amd.engine import Hamiltonian, StateVector
    from paper_2208_10978_amd.problem import PauliSum
    from workloads import random_pauli_sum, random_rotations

    n = 32
    log(f"C4: allocating a {n}-qubit complex64 state (32 GiB)")
    s = StateVector(n, "c64")
    x, z, phi = random_rotations(n, n_rot, 4242)
    hx, hz, hc = random_pauli_sum(n, n_terms, 4343)
    ham = Hamiltonian(PauliSum(n, hx, hz, hc))
    s.prepare_hf((1 << 16) - 1)
    s.apply_rotations(x[:64], z[:64], phi[:64])       # warm-up (plans, code load)
    out = s.expect(ham)                               # builds the tiling and the diagonal
    torch.cuda.synchronize()
    B.sv_profile_begin()
    t0 = time.perf_counter()
    s.apply_rotations(x, z, phi)
    torch.cuda.synchronize()
    t_rot = time.perf_counter() - t0
    prof_rot = B.sv_profile_end()
    B.sv_profile_begin()
    t0 = time.perf_counter()
    out = s.expect(ham)
    torch.cuda.synchronize()
    t_exp = time.perf_counter() - t0
    prof_exp = B.sv_profile_end()
    norm = float(out[1].item())
    groups = int(np.unique(hx).shape[0])
    rot_bytes = sum(v["bytes"] for v in prof_rot.values())
    rot_ms = sum(v["ms"] for v in prof_rot.values())
    exp_bytes = sum(v["bytes"] for v in prof_exp.values())
    exp_ms = sum(v["ms"] for v in prof_exp.values())
    res = {
        "workload": f"{n_rot}-rotation prefix of the 10^5-rotation stream + {n_terms}-term expectation, "
                    f"{n} qubits complex64",
        "rotations_per_s": n_rot / t_rot,
        "rotation_passes": int(sum(v["launches"] for k, v in prof_rot.items() if k in
                                   ("k_run_full", "k_tile_forward"))),
        "rotation_sweep_GB_s": rot_bytes / (rot_ms / 1e3) / 1e9 if rot_ms else None,
        "rotation_sweep_hbm_frac": (rot_bytes / (rot_ms / 1e3) / 1e9) / HBM_PEAK_GBS if rot_ms else None,
        "expectation_s": t_exp,
        "x_groups_per_s": groups / t_exp,
        "expectation_GB_s": exp_bytes / (exp_ms / 1e3) / 1e9 if exp_ms else None,
        "expectation_hbm_frac": (exp_bytes / (exp_ms / 1e3) / 1e9) / HBM_PEAK_GBS if exp_ms else None,
        "expectation_kernels": {k: {"ms": round(v["ms"], 3), "launches": v["launches"]} for k, v in prof_exp.items()},
        "norm_after": norm,
    }
    s.free()
    ham.free()
    return res


def bench_c4_stream(n_rot: int, chunk: int):
    """The whole random rotation stream at 32 qubits, complex64 (not part of
    the default run): n_rot seeded 4-support rotations with odd Y count
    (real rotations, so the state stays real) applied to the Hartree-Fock
    state in calls of `chunk` rotations, each timed; after each call the
    FP64 norm <psi|psi> shows the accumulated rounding drift (each rotation
    is unitary, so any departure from 1 is rounding)."""
    import torch
    from paper_2208_10978_amd import binding as B
    from paper_2208_10978_amd.engine import StateVector
    from workloads import random_rotations

    n = 32
    x, z, phi = random_rotations(n, n_rot, 4242)
    s = StateVector(n, "c64")
    s.prepare_hf((1 << 16) - 1)
    s.apply_rotations(x[:64], z[:64], np.zeros(64))   # warm-up at angle 0 (the identity): plans, code load
    torch.cuda.synchronize()
    rows, total_s, passes = [], 0.0, 0
    for k0 in range(0, n_rot, chunk):
        k1 = min(n_rot, k0 + chunk)
        B.sv_profile_begin()
        t0 = time.perf_counter()
        s.apply_rotations(x[k0:k1], z[k0:k1], phi[k0:k1])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = B.sv_profile_end()
        total_s += dt
        p = int(sum(v["launches"] for kk, v in prof.items() if kk in ("k_run_full", "k_tile_forward")))
        passes += p
        nrm = float(s.overlap(s)[0].item())
        rows.append({"rotations": k1, "seconds": round(dt, 3), "passes": p, "norm_minus_1": nrm - 1.0})
        log(f"C4 stream: {k1} rotations, {k1 / total_s:.1f} rotations/s, {passes} passes, |psi|^2 - 1 = {nrm - 1.0:.3e}")
    s.free()
    return {"workload": f"{n_rot} random 4-support rotations (seed 4242), {n} qubits complex64, calls of {chunk}",
            "rotations_per_s": n_rot / total_s, "seconds": total_s, "passes": passes,
            "rotations_per_pass": n_rot / passes, "chunks": rows}


def bench_serve(n_req: int, rhos, seed: int):
    """Served stream (continuous batching) against the one-request-at-a-time
    path on the same Poisson trace: energy + gradient requests with qubit
    counts uniform in {12, 16, 20, 24, 26}, electrons = qubits / 2, seeded
    synthetic H and UCCSD amplitudes per request, complex64 amplitudes with FP64
    reductions.  The offered rate is rho times the measured one-at-a-time
    throughput, for each rho in rhos."""
    from paper_2208_10978_amd.serve import Request, Server, latency_stats
    from workloads import poisson_requests

    base = poisson_requests(n_req, 1.0, seed)

    def trace(rate):
        return [Request(rid=d["id"], n_qubits=d["n_qubits"], n_electrons=d["n_electrons"], h_seed=d["h_seed"],
                        theta_seed=d["theta_seed"], t_arrival=d["t_arrival"] / rate, theta_amplitude=0.05,
                        dtype="c64") for d in base]

    Server(fifo=True).run(trace(1e9)[:2], realtime=False)  # code load, allocator warm-up
    t0 = time.perf_counter()
    alone = Server(fifo=True).run(trace(1e9), realtime=False)
    span = time.perf_counter() - t0
    if any(r.error for r in alone):
        raise RuntimeError(f"serving: {[r.error for r in alone if r.error][:3]}")
    fifo_rate = n_req / span
    log(f"serving: {n_req} requests one at a time in {span:.1f} s")
    out = {
        "workload": f"{n_req} Poisson energy+gradient requests, qubits uniform in {{12,16,20,24,26}}, complex64, "
                    f"offered at rho x the one-at-a-time throughput (seed {seed})",
        "one_at_a_time_evals_per_s": fifo_rate,
        "loads": [],
    }
    for rho in rhos:
        rate = rho * fifo_rate
        log(f"serving: one-at-a-time {fifo_rate:.2f} evals/s; offering {rate:.2f} requests/s (rho {rho:g})")
        srv = Server(max_slots=8)
        mixed = srv.run(trace(rate), realtime=True)
        log(f"serving: rho {rho:g} continuous batching done, p50 {latency_stats(mixed).get('p50_s', 0):.3f} s")
        fifo = Server(fifo=True).run(trace(rate), realtime=True)
        log(f"serving: rho {rho:g} one-at-a-time done, p50 {latency_stats(fifo).get('p50_s', 0):.3f} s")
        out["loads"].append({"rho": rho, "offered_requests_per_s": rate,
                             "continuous_batching": latency_stats(mixed), "fifo_same_trace": latency_stats(fifo),
                             "peak_slots": srv.peak_slots, "peak_hbm_bytes": srv.peak_bytes})
    return out


def bench_small(reps: int = 10):
    """The two small UCCSD configurations: 8 qubits (integrals seed 1008,
    amplitudes U[-0.1, 0.1] seed 2008), launch-bound, and 20 qubits (seeds
    1020 / 2020, U[-0.05, 0.05]), whose 16 MiB complex128 state stays in the
    on-package cache (a cache-resident rate, not an HBM fraction), in
    complex128 and in complex64 with FP64 reductions: the complex64 energy's
    distance from the complex128 one beside its stated bounds.  With R fused
    runs (one per excitation, plus the renormalisation), u = 2^-24 and
    eps = 3 sqrt(2) u R the rigorous bound on ||d psi||, the energy is within
    (2 sigma_H eps + 2 ||H||_1 eps^2) / (1 - eps)^2, and with the Hoeffding
    form (probability 1 - 3e-8) within 72 u sigma_H sqrt(R) + the same
    second-order term; sigma_H = ||(H - E) psi|| is taken from the complex128
    state (lambda = H psi from the adjoint call with one rotation at angle 0)."""
    import torch
    from paper_2208_10978_amd.engine import UCCSDEvaluator
    from paper_2208_10978_amd.problem import jordan_wigner, uccsd_rotations
    from workloads import synthetic_integrals, uniform_amplitudes

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    out = {}
    for n, amp in ((8, 0.1), (20, 0.05)):
        ne = n // 2
        h, eri = synthetic_integrals(n, 1000 + n)
        ham = jordan_wigner(h, eri)
        rot = uccsd_rotations(n, ne)
        theta = uniform_amplitudes(rot.n_params, amp, 2000 + n)
        row = {"n_qubits": n, "pauli_strings": len(ham), "parameters": rot.n_params, "rotations": len(rot)}
        energies = {}
        for dt in ("c128", "c64") if n == 20 else ("c128",):
            ev = UCCSDEvaluator(ham, rot, ne, dt)
            row[f"{dt}_energy_ms"] = timed(lambda: ev.energy(theta))
            row[f"{dt}_energy_grad_ms"] = timed(lambda: ev.energy_and_grad(theta))
            energies[dt] = float(ev.energy(theta)[0].item())
            ev.free()
        row["energy_c128"] = energies["c128"]
        if "c64" in energies:
            import math
            from paper_2208_10978_amd import binding as B
            from paper_2208_10978_amd.engine import StateVector
            ev = UCCSDEvaluator(ham, rot, ne, "c128")
            psi = ev.state(theta)
            lam = StateVector(n, "c128")
            eh = torch.empty(2, dtype=torch.float64, device="cuda")
            gh = torch.empty(1, dtype=torch.float64, device="cuda")
            B.sv_adjoint_grad(psi.handle, lam.handle, ham.x, ham.z, ham.c, np.array([1], np.uint64),
                              np.array([1], np.uint64), np.array([0.0]), eh, gh)
            torch.cuda.synchronize()
            hpsi = float(torch.linalg.vector_norm(lam.amps).item())
            sigma = math.sqrt(max(hpsi * hpsi - float(eh[0].item()) ** 2, 0.0))
            psi.free(); lam.free(); ev.free()
            u, runs, h1 = 2.0 ** -24, rot.n_params + 1, ham.one_norm()
            eps = 3.0 * math.sqrt(2.0) * u * runs
            second = 2.0 * h1 * eps * eps / (1.0 - eps) ** 2
            row["c64_minus_c128"] = energies["c64"] - energies["c128"]
            row["sigma_H"] = sigma
            row["c64_energy_bound_rigorous"] = 2.0 * sigma * eps / (1.0 - eps) ** 2 + second
            row["c64_energy_bound_probabilistic"] = 72.0 * u * sigma * math.sqrt(runs) + second
        out[f"{n}q"] = row
        log(f"small configs: {n} qubits done")
    return out


def bench_next(n: int = 20, reps: int = 3):
    """Figures of the rows beyond the UCCSD hot path on the 20-qubit
    configuration (10 electrons, synthetic integrals seed 1020, amplitudes
    seed 2020, complex128): generalized (UCCGSD) and qubit-excitation
    circuits through the same kernels, ADAPT pool screening over the UCCGSD
    and Pauli-entangler pools, the Eq. 9 loop and the deflated (Eq. 12)
    evaluation.  Each time is the mean of `reps` calls after one warm call."""
    import torch
    from paper_2208_10978_amd.engine import Hamiltonian, UCCSDEvaluator
    from paper_2208_10978_amd.problem import (entangler_pool, excitation_rotations, jordan_wigner,
                                              pauli_entangler_rotations, qeb_rotations, uccgsd_excitations,
                                              uccgsd_rotations, uccsd_excitations, uccsd_rotations)
    from paper_2208_10978_amd.vqe import evaluator_objective, vqe
    from workloads import synthetic_integrals, uniform_amplitudes

    ne = n // 2
    h, eri = synthetic_integrals(n, 1000 + n)
    ham = jordan_wigner(h, eri)
    H = Hamiltonian(ham)
    out = {"workload": f"{n} qubits, {ne} electrons, complex128, {len(ham)} Pauli strings"}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def eval_row(rot, label):
        ev = UCCSDEvaluator(ham, rot, ne, "c128", hamiltonian=H)
        th = uniform_amplitudes(rot.n_params, 0.05, 2000 + n)
        dt = timed(lambda: ev.energy_and_grad(th))
        ev.free_states()
        out[label] = {"parameters": rot.n_params, "rotations": len(rot), "energy_grad_ms": 1e3 * dt,
                      "rotations_per_s_fwd_and_rev": 2 * len(rot) / dt}
        log(f"next: {label} {1e3 * dt:.1f} ms per energy+gradient")

    s, d = uccsd_excitations(n, ne)
    uccsd = uccsd_rotations(n, ne)
    eval_row(uccsd, "uccsd")
    eval_row(uccgsd_rotations(n), "uccgsd")
    eval_row(qeb_rotations(n, s + d), "qeb")

    ev = UCCSDEvaluator(ham, uccsd, ne, "c128", hamiltonian=H)
    th = uniform_amplitudes(uccsd.n_params, 0.05, 2000 + n)
    gs, gd = uccgsd_excitations(n)
    pool = excitation_rotations(n, gs + gd)
    dt = timed(lambda: ev.pool_gradients(th, pool))
    out["adapt_screen_uccgsd_pool"] = {"operators": pool.n_params, "rotations": len(pool), "ms": 1e3 * dt,
                                       "operators_per_s": pool.n_params / dt}
    ent = pauli_entangler_rotations(n, *entangler_pool(ham, 4))
    dt = timed(lambda: ev.pool_gradients(th, ent))
    out["adapt_screen_entangler_pool"] = {"operators": ent.n_params, "ms": 1e3 * dt,
                                          "operators_per_s": ent.n_params / dt}
    log(f"next: pool screening {out['adapt_screen_uccgsd_pool']['ms']:.1f} ms for {pool.n_params} operators")

    res = vqe(evaluator_objective(ev), np.zeros(uccsd.n_params), maxiter=10)
    out["vqe_10_iterations"] = {"evaluations": res["n_eval"], "seconds_per_eval": res["seconds_per_eval"],
                                "energy": res["energy"]}

    lower = [ev.state(uniform_amplitudes(uccsd.n_params, 0.05, 3000 + k)) for k in range(2)]
    dt = timed(lambda: ev.energy_and_grad_deflated(th, lower, [0.5, 0.5]))
    out["vqd_deflated_2_states"] = {"energy_grad_ms": 1e3 * dt}
    for st in lower:
        st.free()
    ev.free_states()
    H.free()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--qubits", type=int, default=28)
    ap.add_argument("--dtype", default="r64", choices=["r64", "c128", "c64"],
                    help="amplitude type of the 28-qubit step: r64 real FP64 (a UCCSD state of a real Hamiltonian "
                         "is real), c128, c64")
    ap.add_argument("--no-c128", action="store_true", help="skip the complex128 step timed beside a real-state run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c4", action="store_true", help="skip the 32-qubit complex64 raw-sweep figures")
    ap.add_argument("--c4-rotations", type=int, default=1000)
    ap.add_argument("--no-serve", action="store_true", help="skip the served-stream figures")
    ap.add_argument("--no-next", action="store_true", help="skip the 8- and 20-qubit figures (small configurations, pool/VQD rows)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 4 GiB device copy three times (calibrates HBM byte counters)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests per offered load of the served stream (the loads are rho 0.8 and 1.0)")
    ap.add_argument("--only-c4", action="store_true",
                    help="only the 32-qubit complex64 figures (for counter runs of the expectation)")
    ap.add_argument("--only-serve", action="store_true", help="only the served-stream figures")
    ap.add_argument("--c4-stream", type=int, default=0,
                    help="only apply this many rotations of the 32-qubit random stream, in calls of 10^4 (drift record)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "q2sv runs on one GPU: --gpus must be 1 (the sharded design is described, not built)"}))
        sys.exit(2)

    import torch
    if args.copy_calibration:
        a = torch.zeros(1 << 28, dtype=torch.complex128, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read_per_copy": a.numel() * 16,
                                               "bytes_written_per_copy": a.numel() * 16, "copies": 3}}))
        return
    if args.only_c4:
        print(json.dumps({"c4": bench_c4(args.c4_rotations, 10_000)}), flush=True)
        return
    if args.c4_stream:
        print(json.dumps({"c4_stream": bench_c4_stream(args.c4_stream, 10_000)}), flush=True)
        return
    if args.only_serve:
        print(json.dumps({"serving": bench_serve(args.serve_requests, (0.8, 1.0), 5151)}), flush=True)
        return
    from paper_2208_10978_amd import binding as B
    from paper_2208_10978_amd.engine import UCCSDEvaluator
    from paper_2208_10978_amd.problem import jordan_wigner, uccsd_rotations
    from workloads import synthetic_integrals, uniform_amplitudes

    n = args.qubits
    ne = n // 2
    log(f"building the {n}-qubit problem")
    h, eri = synthetic_integrals(n, 1000 + n)
    ham = jordan_wigner(h, eri).truncated(1e-6)
    rot = uccsd_rotations(n, ne)
    theta = uniform_amplitudes(rot.n_params, 0.02, 2000 + n)
    log(f"{len(ham)} Pauli strings in {ham.n_groups} x-groups, {rot.n_params} amplitudes, {len(rot)} rotations")

    t0 = time.perf_counter()
    ev = UCCSDEvaluator(ham, rot, ne, args.dtype)
    torch.cuda.synchronize()
    log(f"states allocated ({2 * (1 << n) * (16 if args.dtype == 'c128' else 8) / 2**30:.1f} GiB, {args.dtype})")
    for w in range(args.warmup):
        ev.energy_and_grad(theta)
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done ({time.perf_counter() - t0:.1f} s since setup)")

    B.sv_profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        e, g = ev.energy_and_grad(theta)
        torch.cuda.synchronize()
        log(f"step {k + 1}/{args.steps}: {time.perf_counter() - t0:.2f} s")
    t1 = time.perf_counter()
    prof = B.sv_profile_end()
    elapsed = t1 - t0
    energy = float(e[0].item())
    norm = float(e[1].item())
    grad_norm = float(torch.linalg.vector_norm(g).item())

    # forward sweep alone: Pauli rotations per second
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, args.steps)
    start.record()
    for _ in range(reps):
        ev.forward_state(theta)
    stop.record()
    torch.cuda.synchronize()
    fwd_s = start.elapsed_time(stop) / 1e3 / reps

    # a plain device copy of one state (read + write) as the attainable-bandwidth reference
    copy_s = []
    for _ in range(3):
        start.record()
        ev.lam.amps.copy_(ev.psi.amps)
        stop.record()
        torch.cuda.synchronize()
        copy_s.append(start.elapsed_time(stop) / 1e3)
    copy_gbs = 2 * ev.psi.amps.numel() * ev.psi.amps.element_size() / min(copy_s) / 1e9

    # dominant kernel class by time in the timed region
    dom_name, dom = max(((k, v) for k, v in prof.items() if v["bytes"] > 0), key=lambda kv: kv[1]["ms"])
    achieved = dom["bytes"] / (dom["ms"] / 1e3) / 1e9
    traffic = measured_traffic(dom_name, n, args.dtype)
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": dom_name,
        "avg_launch_ms": round(dom["ms"] / dom["launches"], 4),
        "launches_per_step": dom["launches"] / args.steps,
        "copy_GB_s": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4),
    }
    kernels = {k: {"ms_per_step": round(v["ms"] / args.steps, 3),
                   "GB_s": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None,
                   "launches_per_step": v["launches"] / args.steps} for k, v in prof.items()}

    result = {
        "metric": "Pauli rotations/s + energy(+grad) evals/s at 28-32 qubits; % of HBM peak",
        "value": args.steps / elapsed,
        "unit": "energy+grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "c64" else "f64",
        "data": "synthetic",
        "config": {"workload": f"UCCSD energy + adjoint gradient, {n} qubits, {ne} electrons, "
                               f"{AMP_LABEL[args.dtype]}",
                   "n_qubits": n, "n_electrons": ne, "pauli_strings": len(ham), "x_groups": ham.n_groups,
                   "parameters": rot.n_params, "rotations": len(rot)},
        "rotations_per_s": len(rot) / fwd_s,
        "forward_sweep_ms": 1e3 * fwd_s,
        "energy": energy,
        "norm": norm,
        "grad_norm": grad_norm,
        "roofline": roofline,
        "kernels": kernels,
    }
    ev.free()
    del ev
    torch.cuda.empty_cache()
    if args.dtype == "r64" and not args.no_c128:
        result["complex128_step"] = step_c128(ham, rot, ne, theta, max(1, min(args.steps, 3)), energy)
        torch.cuda.empty_cache()
    if not args.no_c4:
        result["c4"] = bench_c4(args.c4_rotations, 10_000)
    if not args.no_serve:
        result["serving"] = bench_serve(args.serve_requests, (0.8, 1.0), 5151)
    if not args.no_next:
        result["small_configs"] = bench_small()
        result["next_rows"] = bench_next()
    if not args.no_cpu_baseline:
        log("timing the oracle sample on the host")
        result["cpu_baseline"] = cpu_baseline(n, ham, rot, theta)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
