"""Scheduling logic of the serving loop on the CPU, with a fake executor (a
test double that evaluates requests with the FP64 oracle and completes them
after a simulated device time).  No product path runs here."""
import time

import numpy as np

from oracle import statevector as osv
from paper_2208_10978_amd.serve import Request, Server, latency_stats


class FakeExecutor:
    def __init__(self, device_time=0.02, budget=10 ** 12):
        self.device_time = device_time
        self._budget = budget
        self.launch_order = []
        self.live = 0
        self.max_live = 0

    def budget(self):
        return self._budget

    class Job:
        def __init__(self, ex, req):
            self.ex, self.req = ex, req
            self.t_ready = time.perf_counter() + ex.device_time
            phi = req.rot.angles(req.theta)
            e, g = osv.reverse_mode_gradient(osv.basis_state(req.n_qubits, (1 << req.n_electrons) - 1),
                                             req.ham.x, req.ham.z, req.ham.c, req.rot.x, req.rot.z, phi)
            self.out = (e, 1.0, osv.chain_to_parameters(g, req.rot.param, req.rot.dphi_dtheta, req.rot.n_params))

        def ready(self):
            return time.perf_counter() >= self.t_ready

        def result(self):
            self.ex.live -= 1
            return self.out

    def launch(self, req):
        self.launch_order.append(req.rid)
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return FakeExecutor.Job(self, req)


def trace(k=8, gap=0.005):
    return [Request(rid=r, n_qubits=(4, 6)[r % 2], n_electrons=(2, 3)[r % 2], h_seed=100 + r, theta_seed=200 + r,
                    t_arrival=r * gap, theta_amplitude=0.3) for r in range(k)]


def test_results_identical_alone_and_in_the_mix():
    mixed = Server(FakeExecutor(), max_slots=4).run(trace(), realtime=True)
    for r in trace():
        alone = Server(FakeExecutor(), max_slots=1).run([r], realtime=False)[0]
        m = next(x for x in mixed if x.rid == r.rid)
        assert m.error is None and alone.error is None
        assert m.energy == alone.energy
        assert np.array_equal(m.grad, alone.grad)


def test_slots_and_budget_are_respected():
    ex = FakeExecutor(device_time=0.05)
    one = Request(0, 6, 3, 1, 1).device_bytes()
    srv = Server(ex, hbm_budget_bytes=3 * one, max_slots=8)
    out = srv.run(trace(10, gap=0.0), realtime=False)
    assert all(r.error is None for r in out)
    assert srv.peak_bytes <= 3 * one and ex.max_live <= 3
    srv2 = Server(FakeExecutor(device_time=0.05), max_slots=2)
    srv2.run(trace(6, gap=0.0), realtime=False)
    assert srv2.peak_slots <= 2


def test_requests_that_cannot_fit_or_are_malformed_fail_alone():
    reqs = trace(4)
    reqs.append(Request(rid=100, n_qubits=30, n_electrons=15, h_seed=1, theta_seed=1, t_arrival=0.0))
    reqs.append(Request(rid=101, n_qubits=6, n_electrons=9, h_seed=1, theta_seed=1, t_arrival=0.001))
    one = Request(0, 6, 3, 1, 1).device_bytes()
    out = Server(FakeExecutor(), hbm_budget_bytes=4 * one, max_slots=4).run(reqs, realtime=True)
    by = {r.rid: r for r in out}
    assert "never fit" in by[100].error
    assert "bad request" in by[101].error
    assert all(by[r].error is None and by[r].energy is not None for r in range(4))


def test_fifo_runs_one_at_a_time_in_arrival_order():
    ex = FakeExecutor(device_time=0.01)
    out = Server(ex, fifo=True).run(trace(6, gap=0.0), realtime=False)
    assert ex.launch_order == list(range(6)) and ex.max_live == 1
    assert all(r.error is None for r in out)


def test_continuous_batching_admits_while_others_run():
    ex = FakeExecutor(device_time=0.2)
    reqs = trace(4, gap=0.05)
    out = Server(ex, max_slots=4).run(reqs, realtime=True)
    first = next(r for r in out if r.rid == 0)
    later = [r for r in out if r.rid > 0]
    assert any(r.t_admit < first.t_done for r in later)     # admitted before the first finished
    assert ex.max_live >= 2
    stats = latency_stats(out)
    assert stats["requests"] == 4 and stats["p99_s"] >= stats["p50_s"] > 0


def test_a_device_failure_after_launch_fails_its_request_alone():
    class FailingExecutor(FakeExecutor):
        class Bad:
            def __init__(self, ex):
                self.ex = ex

            def ready(self):
                self.ex.live -= 1
                raise RuntimeError("device error")

        def launch(self, req):
            if req.rid == 2:
                self.live += 1
                return FailingExecutor.Bad(self)
            return super().launch(req)

    ex = FailingExecutor()
    out = Server(ex, max_slots=3).run(trace(5), realtime=True)
    by = {r.rid: r for r in out}
    assert "device error" in by[2].error and by[2].t_done is not None
    assert all(by[r].error is None and by[r].energy is not None for r in (0, 1, 3, 4))
    assert ex.live == 0


def test_online_submit_from_two_threads_matches_the_trace_results():
    import threading
    reqs = trace(6, gap=0.0)
    srv = Server(FakeExecutor(device_time=0.005), max_slots=3).start()
    futs = {}

    def client(part):
        for r in part:
            futs[r.rid] = srv.submit(r)
    ts = [threading.Thread(target=client, args=(reqs[k::2],)) for k in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    got = {rid: f.result(timeout=30) for rid, f in futs.items()}
    srv.stop()
    for r in trace(6, gap=0.0):
        alone = Server(FakeExecutor(), max_slots=1).run([r], realtime=False)[0]
        e, norm, g = got[r.rid]
        assert e == alone.energy and np.array_equal(g, alone.grad)


def test_online_errors_and_lifecycle():
    import pytest
    srv = Server(FakeExecutor(), hbm_budget_bytes=1 << 20).start()
    big = Request(rid=1, n_qubits=20, n_electrons=10, h_seed=1, theta_seed=2)
    with pytest.raises(RuntimeError, match="never fit"):
        srv.submit(big).result(timeout=30)
    srv.stop()
    with pytest.raises(RuntimeError):
        srv.submit(big)


def test_online_cancelled_request_does_not_stop_the_loop():
    """A future cancelled before the loop takes its request is dropped; one
    already taken cannot be cancelled.  Either way the loop keeps serving."""
    reqs = trace(3, gap=0.0)
    srv = Server(FakeExecutor(device_time=0.005), max_slots=2).start()
    a = srv.submit(reqs[0])
    b = srv.submit(reqs[1])
    b_cancelled = b.cancel()
    c = srv.submit(reqs[2])
    assert a.result(timeout=30)[2] is not None
    assert c.result(timeout=30)[2] is not None
    if not b_cancelled:
        assert b.result(timeout=30)[2] is not None
    srv.stop()


class _BrokenExecutor(FakeExecutor):
    """Its jobs raise from ready() with an error the loop does not expect
    to handle per request (a BaseException outside Exception)."""

    class Job(FakeExecutor.Job):
        def ready(self):
            raise KeyboardInterrupt("simulated")

    def launch(self, req):
        return _BrokenExecutor.Job(self, req)


def test_online_loop_failure_fails_every_open_request():
    import pytest
    reqs = trace(2, gap=0.0)
    srv = Server(_BrokenExecutor(), max_slots=2).start()
    futs = [srv.submit(r) for r in reqs]
    for f in futs:
        with pytest.raises(RuntimeError, match="serving loop failed"):
            f.result(timeout=30)
    srv._thread.join(timeout=30)
    assert isinstance(srv.loop_error, KeyboardInterrupt)
    with pytest.raises(RuntimeError):
        srv.submit(reqs[0])


class FailingExecutor(FakeExecutor):
    """Reports a failed device (the library's sticky SV_EDEVICE) when the
    third request completes, and at every launch after that."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.dead = False
        self.completed = 0

    class Job(FakeExecutor.Job):
        def result(self):
            from paper_2208_10978_amd.binding import DeviceFailure, SV_EDEVICE
            self.ex.completed += 1
            if self.ex.completed == 3:
                self.ex.dead = True
            if self.ex.dead:
                raise DeviceFailure(SV_EDEVICE, "planted device failure")
            return super().result()

    def launch(self, req):
        from paper_2208_10978_amd.binding import DeviceFailure, SV_EDEVICE
        if self.dead:
            raise DeviceFailure(SV_EDEVICE, "planted device failure")
        self.launch_order.append(req.rid)
        return FailingExecutor.Job(self, req)


def test_a_failed_device_drains_and_reports():
    reqs = trace(10, gap=0.004)
    srv = Server(FailingExecutor(device_time=0.02), max_slots=2)
    out = srv.run(reqs, realtime=True)
    assert srv.device_error is not None and "planted" in srv.device_error
    ok = [r for r in out if r.error is None]
    bad = [r for r in out if r.error is not None]
    assert len(ok) == 2 and len(bad) == 8          # two finished before the failure
    assert all("device failed" in r.error and r.t_done is not None for r in bad)
    for r in ok:                                    # results before the failure are intact
        alone = Server(FakeExecutor(), max_slots=1).run([Request(r.rid, r.n_qubits, r.n_electrons, r.h_seed,
                                                                 r.theta_seed, 0.0, r.theta_amplitude)],
                                                        realtime=False)[0]
        assert alone.energy == r.energy


def test_online_server_fails_open_and_later_requests_after_a_device_failure():
    srv = Server(FailingExecutor(device_time=0.01), max_slots=2).start()
    futs = [srv.submit(r) for r in trace(5, gap=0.0)]
    errs = []
    for f in futs:
        try:
            f.result(timeout=30)
        except RuntimeError as exc:
            errs.append(str(exc))
    assert len(errs) == 3 and all("device failed" in e for e in errs)
    late = srv.submit(trace(1)[0])
    try:
        late.result(timeout=30)
        raise AssertionError("a request after the failure must fail")
    except RuntimeError as exc:
        assert "device failed" in str(exc)
    srv.stop()
    assert srv.device_error is not None


def test_smallest_state_first_and_one_heavy_request_at_a_time():
    """Waiting requests are admitted smallest state first (arrival order among
    equals), and at most max_heavy requests of heavy_qubits or more run at
    once while smaller ones are admitted beside them."""
    class Tracking(FakeExecutor):
        def __init__(self, **kw):
            super().__init__(**kw)
            self.running = []
            self.max_heavy_live = 0

        def launch(self, req):
            self.running = [q for q in self.running if not q[1].ready()]
            job = super().launch(req)
            self.running.append((req, job))
            self.max_heavy_live = max(self.max_heavy_live, sum(1 for q, _ in self.running if q.n_qubits >= 6))
            return job

    # (qubits, electrons): request 0 arrives first and holds the one slot
    # while the others arrive and finish their host preparation
    sizes = [(2, 1), (6, 3), (6, 3), (4, 2), (6, 3), (2, 1), (4, 2)]
    reqs = [Request(rid=i, n_qubits=q, n_electrons=e, h_seed=300 + i, theta_seed=400 + i, theta_amplitude=0.3,
                    t_arrival=0.0 if i == 0 else 0.01) for i, (q, e) in enumerate(sizes)]
    ex = Tracking(device_time=0.3)
    out = Server(ex, max_slots=1, heavy_qubits=6, max_heavy=1).run(reqs, realtime=True)
    assert all(r.error is None for r in out)
    assert ex.launch_order == [0, 5, 3, 6, 1, 2, 4]        # then 2, 4, 4 and the 6-qubit ones in arrival order
    ex2 = Tracking(device_time=0.05)
    out2 = Server(ex2, max_slots=4, heavy_qubits=6, max_heavy=1).run(reqs, realtime=False)
    assert all(r.error is None for r in out2)
    assert ex2.max_heavy_live == 1 and ex2.max_live >= 2    # small ones ran beside a heavy one
    for a, b in zip(sorted(out, key=lambda r: r.rid), sorted(out2, key=lambda r: r.rid)):
        assert a.energy == b.energy and np.array_equal(a.grad, b.grad)
