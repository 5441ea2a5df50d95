"""Continuous-batching request loop for UCCSD energy + gradient evaluations.

Requests arrive with their own qubit count, Hamiltonian and amplitudes.  The
server keeps every admitted request's state vectors and Hamiltonian resident
in HBM, admits a waiting request as soon as a slot is free and its bytes fit
the HBM budget, and runs each admitted request on its own HIP stream, so the
work of requests in flight together overlaps on the device.  Waiting
requests are admitted smallest state first (arrival order among equals), and
at most ``max_heavy`` requests of ``heavy_qubits`` or more run at once: a
request of 24 or 26 qubits fills the device by itself, so running two
together only stretches both, while small requests fit beside one and need
not queue behind it.  A request's plans depend only on the request and the
library's sums do not depend on the order of concurrent work (lambda in
fixed point, reductions in a fixed order), so its result is bitwise the
same alone and in any mix.

A failed device (the library's sticky SV_EDEVICE, raised as DeviceFailure)
ends admission: every request in flight, waiting or arriving later fails
with the device's message, and ``device_error`` keeps that message.

Host-side preparation (the JW Pauli sum and the rotation list) runs in a
thread pool ahead of admission.  ``fifo=True`` gives the one-request-at-a-
time baseline on the same trace.  ``Server.start`` / ``submit`` /
``stop`` serve requests submitted online, each resolving a Future.  The
device work is behind an executor (``GpuExecutor``); the scheduling logic
itself is plain Python.
"""
from __future__ import annotations

import concurrent.futures as cf
import time
from dataclasses import dataclass

import numpy as np

from .binding import DeviceFailure
from .problem import PauliSum, RotationList, jordan_wigner, uccsd_rotations


@dataclass
class Request:
    rid: int
    n_qubits: int
    n_electrons: int
    h_seed: int
    theta_seed: int
    t_arrival: float = 0.0          # seconds after the start of the trace
    theta_amplitude: float = 0.05
    dtype: str = "c64"
    # filled by the server
    ham: PauliSum | None = None
    rot: RotationList | None = None
    theta: np.ndarray | None = None
    energy: float | None = None
    norm: float | None = None
    grad: np.ndarray | None = None
    error: str | None = None
    t_admit: float | None = None
    t_done: float | None = None

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival

    def device_bytes(self) -> int:
        amp = 16 if self.dtype == "c128" else 8
        n_amp = 1 << self.n_qubits
        # psi + lam + resident FP64 diagonal + tables and reduction partials
        return 2 * n_amp * amp + n_amp * 8 + (64 << 20)


def prepare(req: Request) -> Request:
    """Host-side problem build (no device work)."""
    from workloads import synthetic_integrals, uniform_amplitudes
    if not 0 < req.n_electrons <= req.n_qubits or req.n_qubits % 2:
        raise ValueError(f"bad request: {req.n_qubits} qubits, {req.n_electrons} electrons")
    h, eri = synthetic_integrals(req.n_qubits, req.h_seed)
    req.ham = jordan_wigner(h, eri)
    req.rot = uccsd_rotations(req.n_qubits, req.n_electrons, "tile")
    req.theta = np.asarray(uniform_amplitudes(req.rot.n_params, req.theta_amplitude, req.theta_seed))
    if not np.all(np.isfinite(req.theta)):
        raise ValueError("non-finite amplitudes")
    return req


class GpuExecutor:
    """Launches a request on its own HIP stream; completion via a HIP event.

    A launch (the Hamiltonian's grouping and tiling, the rotation plans, the
    uploads and the kernel enqueues) runs on a small thread pool: the library
    releases the GIL, so host planning of one request overlaps the serving
    loop and the device work of the others."""

    class Job:
        def __init__(self, req):
            import torch
            from .engine import UCCSDEvaluator
            self.stream = torch.cuda.Stream()
            with torch.cuda.stream(self.stream):
                self.ev = UCCSDEvaluator(req.ham, req.rot, req.n_electrons, req.dtype, stream=self.stream)
                e, g = self.ev.energy_and_grad(req.theta)
                self.e_host = torch.empty(2, dtype=torch.float64, pin_memory=True)
                self.g_host = torch.empty(req.rot.n_params, dtype=torch.float64, pin_memory=True)
                self.e_host.copy_(e, non_blocking=True)
                self.g_host.copy_(g, non_blocking=True)
                self.done = torch.cuda.Event()
                self.done.record(self.stream)

        def ready(self) -> bool:
            return self.done.query()

        def result(self):
            out = float(self.e_host[0]), float(self.e_host[1]), self.g_host.numpy().copy()
            self.ev.free()
            return out

    class Pending:
        def __init__(self, fut):
            self.fut = fut

        def ready(self) -> bool:
            return self.fut.done() and self.fut.result().ready()

        def result(self):
            return self.fut.result().result()

    def __init__(self, launch_workers: int = 4):
        self.pool = cf.ThreadPoolExecutor(max_workers=launch_workers)

    def budget(self) -> int:
        import torch
        free, _ = torch.cuda.mem_get_info()
        return int(free * 0.8)

    def launch(self, req):
        return GpuExecutor.Pending(self.pool.submit(GpuExecutor.Job, req))


class Server:
    """``run(trace)`` serves a whole trace and returns it; ``start()`` /
    ``submit(req) -> Future[(energy, norm, grad)]`` / ``stop()`` serve
    requests submitted online from any thread.  Both use the same loop."""

    def __init__(self, executor=None, hbm_budget_bytes: int | None = None, max_slots: int = 8,
                 prep_workers: int = 4, fifo: bool = False, heavy_qubits: int = 24, max_heavy: int = 1):
        self.ex = executor if executor is not None else GpuExecutor()
        self.budget = int(hbm_budget_bytes if hbm_budget_bytes is not None else self.ex.budget())
        self.max_slots = 1 if fifo else int(max_slots)
        self.heavy_qubits = int(heavy_qubits)
        self.max_heavy = int(max_heavy)
        self.pool = cf.ThreadPoolExecutor(max_workers=prep_workers)
        self.fifo = fifo
        self.peak_bytes = 0
        self.peak_slots = 0
        self.loop_error = None  # what ended the online loop, if it failed
        self.device_error = None  # the device's failure message, once it has failed
        self._thread = None

    # -- the loop ---------------------------------------------------------
    def _serve(self, t0, arrivals, no_more, prep, on_done, idle_wait):
        """``arrivals(now)`` returns the requests that became visible (they
        must have an entry in ``prep``, their host preparation future);
        ``no_more()`` is true once nothing else will arrive; ``on_done(r)``
        sees every finished request (result or error); ``idle_wait(now)`` is
        how long to sleep when nothing is waiting or running."""
        waiting: list = []
        active: list = []
        used = 0

        def device_lost(exc):
            # the device is unusable from here on: fail everything in flight
            # and waiting; later arrivals fail as they come
            self.device_error = str(exc)
            msg = f"device failed: {exc}"
            for _, r in active:
                r.error = msg
                r.t_done = time.perf_counter() - t0
                on_done(r)
            for r in waiting:
                r.error = msg
                r.t_done = time.perf_counter() - t0
                on_done(r)
            active.clear()
            waiting.clear()

        while True:
            now = time.perf_counter() - t0
            # once the device has failed, everything still to come is drained at once
            for r in arrivals(float("inf") if self.device_error else now):
                if r.error is None and self.device_error:
                    r.error = f"device failed: {self.device_error}"
                if r.error is not None:
                    r.t_done = now
                    on_done(r)
                else:
                    waiting.append(r)
            for job, r in list(active):  # completions (a launch that failed fails its request alone)
                try:
                    if not job.ready():
                        continue
                    r.energy, r.norm, r.grad = job.result()
                except DeviceFailure as exc:
                    device_lost(exc)
                    break
                except Exception as exc:
                    r.error = f"{type(exc).__name__}: {exc}"
                r.t_done = time.perf_counter() - t0
                used -= r.device_bytes()
                active.remove((job, r))
                on_done(r)
            if self.device_error:
                used = 0
            if not self.fifo:  # smallest state first, arrival order among equals (a stable sort)
                waiting.sort(key=lambda q: q.n_qubits)
            heavy = sum(1 for _, q in active if q.n_qubits >= self.heavy_qubits)
            i = 0  # admissions
            while i < len(waiting) and len(active) < self.max_slots:
                r = waiting[i]
                fut = prep[id(r)]
                is_heavy = not self.fifo and r.n_qubits >= self.heavy_qubits
                if not fut.done() or used + r.device_bytes() > self.budget or (is_heavy and heavy >= self.max_heavy):
                    if self.fifo:
                        break
                    i += 1
                    continue
                waiting.pop(i)
                try:
                    fut.result()
                    r.t_admit = time.perf_counter() - t0
                    active.append((self.ex.launch(r), r))
                    heavy += int(is_heavy)
                    used += r.device_bytes()
                    self.peak_bytes = max(self.peak_bytes, used)
                    self.peak_slots = max(self.peak_slots, len(active))
                except DeviceFailure as exc:
                    waiting.insert(0, r)
                    device_lost(exc)
                    break
                except Exception as exc:  # a malformed request fails alone
                    r.error = f"{type(exc).__name__}: {exc}"
                    r.t_done = time.perf_counter() - t0
                    on_done(r)
            if not active and not waiting:
                if no_more():
                    return
                time.sleep(idle_wait(time.perf_counter() - t0))
            else:
                time.sleep(0.0002)

    def _check_fits(self, r):
        if r.device_bytes() > self.budget:
            r.error = "request can never fit the HBM budget"

    # -- a whole trace ----------------------------------------------------
    def run(self, requests, realtime: bool = True, on_done=None):
        """Serve a trace.  With ``realtime`` a request becomes visible at its
        arrival time (relative to the start); otherwise all are present at
        once.  Host preparation of every request starts at once.  Returns the
        requests with results and timestamps."""
        reqs = sorted(requests, key=lambda r: (r.t_arrival, r.rid))
        prep = {}
        for r in reqs:
            self._check_fits(r)
            if r.error is None:
                prep[id(r)] = self.pool.submit(prepare, r)
        t0 = time.perf_counter()
        nxt = [0]
        done = [0]

        def arrivals(now):
            out = []
            while nxt[0] < len(reqs) and (not realtime or reqs[nxt[0]].t_arrival <= now):
                out.append(reqs[nxt[0]])
                nxt[0] += 1
            return out

        def finish(r):
            done[0] += 1
            if on_done:
                on_done(r)

        def idle_wait(now):
            if realtime and nxt[0] < len(reqs):
                return max(0.0, min(0.01, reqs[nxt[0]].t_arrival - now))
            return 0.0002

        self._serve(t0, arrivals, lambda: nxt[0] >= len(reqs), prep, finish, idle_wait)
        return reqs

    # -- online -------------------------------------------------------------
    def start(self):
        """Start serving submitted requests on a background thread."""
        import queue
        import threading
        if self._thread is not None:
            raise RuntimeError("server already started")
        self._queue = queue.Queue()
        self._stop = threading.Event()
        self._t0 = time.perf_counter()
        prep, futs = {}, {}

        def arrivals(now):
            out = []
            while True:
                try:
                    r, fut = self._queue.get_nowait()
                except queue.Empty:
                    return out
                # from here on the future cannot be cancelled; a request
                # cancelled before the loop took it is dropped
                if not fut.set_running_or_notify_cancel():
                    continue
                r.t_arrival = now
                self._check_fits(r)
                futs[id(r)] = fut
                if r.error is None:
                    prep[id(r)] = self.pool.submit(prepare, r)
                out.append(r)

        def finish(r):
            fut = futs.pop(id(r))
            prep.pop(id(r), None)
            if r.error is None:
                fut.set_result((r.energy, r.norm, r.grad))
            else:
                fut.set_exception(RuntimeError(r.error))

        def fail_queued(msg):
            while True:
                try:
                    _, fut = self._queue.get_nowait()
                except queue.Empty:
                    break
                if fut.set_running_or_notify_cancel():
                    fut.set_exception(RuntimeError(msg))

        def loop():
            try:
                self._serve(self._t0, arrivals, lambda: self._stop.is_set() and self._queue.empty(), prep, finish,
                            lambda now: 0.001)
            except BaseException as exc:  # a failure of the loop itself fails every open request
                self._stop.set()
                msg = f"serving loop failed: {type(exc).__name__}: {exc}"
                for fut in list(futs.values()):
                    if not fut.done():
                        fut.set_exception(RuntimeError(msg))
                futs.clear()
                fail_queued(msg)
                self.loop_error = exc
                return
            fail_queued("server stopped")  # a submit that raced with stop()

        self._thread = threading.Thread(target=loop, name="q2sv-serve", daemon=True)
        self._thread.start()
        return self

    def submit(self, req: Request) -> cf.Future:
        """Queue a request; the future resolves to (energy, norm, grad) or
        raises with the request's error."""
        if self._thread is None:
            raise RuntimeError("call start() first")
        if self._stop.is_set():
            raise RuntimeError("server is stopping")
        fut: cf.Future = cf.Future()
        self._queue.put((req, fut))
        return fut

    def stop(self, wait: bool = True):
        """Finish everything submitted so far, then end the loop."""
        if self._thread is None:
            return
        self._stop.set()
        if wait:
            self._thread.join()
            self._thread = None


def latency_stats(reqs):
    ok = [r for r in reqs if r.error is None and r.t_done is not None]
    if not ok:
        return {}
    lat = np.array([r.latency for r in ok])
    span = max(r.t_done for r in ok) - min(r.t_arrival for r in ok)
    return {"requests": len(ok), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "evals_per_s": float(len(ok) / span) if span > 0 else None}
