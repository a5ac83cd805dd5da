"""Host-only tests of the serving loop's scheduling: admission order, slot
and memory limits, rejection of oversized requests, failure handling and
latency accounting, with an executor that only simulates durations."""
import pytest

from paper_2604_15017_amd.serve import Request, Result, Server, latency_stats


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Request rid takes durations[rid] seconds and needs sizes[rid] bytes."""

    def __init__(self, clock, durations, sizes, fail=()):
        self.clock, self.dur, self.sizes, self.fail = clock, durations, sizes, set(fail)
        self.launch_order = []
        self.running = set()
        self.max_running = 0

    def bytes_needed(self, req):
        return self.sizes[req.rid]

    def launch(self, req, slot):
        if req.rid in self.fail:
            raise RuntimeError("injected launch failure")
        self.launch_order.append(req.rid)
        self.running.add(req.rid)
        self.max_running = max(self.max_running, len(self.running))
        return (req.rid, self.clock() + self.dur[req.rid])

    def done(self, h):
        return self.clock() >= h[1]

    def finish(self, req, h):
        self.running.discard(req.rid)
        return Result(req.rid, True, segments=100)


def drive(server, clock, n, dt=1e-3, limit=100000):
    for _ in range(limit):
        server.step()
        if len(server.results) >= n:
            return
        clock.t += dt
    raise AssertionError("did not finish")


def test_fifo_admission_and_slot_limit():
    clk = Clock()
    ex = FakeExecutor(clk, durations={i: 0.01 * (1 + i % 3) for i in range(10)}, sizes={i: 10 for i in range(10)})
    srv = Server(ex, n_slots=3, mem_cap_bytes=1000, clock=clk)
    for i in range(10):
        srv.submit(Request(i, None))
    drive(srv, clk, 10)
    assert ex.launch_order == list(range(10))
    assert ex.max_running == 3 and srv.max_concurrent == 3
    assert all(srv.results[i].ok for i in range(10))


def test_memory_cap_limits_concurrency_and_rejects_oversized():
    clk = Clock()
    sizes = {0: 60, 1: 60, 2: 30, 3: 500, 4: 40}
    ex = FakeExecutor(clk, durations={i: 0.005 for i in sizes}, sizes=sizes)
    srv = Server(ex, n_slots=8, mem_cap_bytes=100, clock=clk)
    for i in sizes:
        srv.submit(Request(i, None))
    drive(srv, clk, len(sizes))
    assert not srv.results[3].ok and "cap" in srv.results[3].error
    assert all(srv.results[i].ok for i in (0, 1, 2, 4))
    assert srv.max_reserved <= 100
    assert srv.reserved == 0 and sorted(srv.free_slots) == list(range(8))
    # 0 and 1 cannot run together (60 + 60 > 100); FIFO keeps 2 behind 1
    assert ex.launch_order.index(1) > ex.launch_order.index(0)


def test_continuous_admission_as_slots_free():
    """A long request does not hold back later short ones once a slot frees."""
    clk = Clock()
    dur = {0: 0.5, 1: 0.01, 2: 0.01, 3: 0.01}
    ex = FakeExecutor(clk, durations=dur, sizes={i: 1 for i in dur})
    srv = Server(ex, n_slots=2, mem_cap_bytes=10, clock=clk)
    for i in dur:
        srv.submit(Request(i, None))
    drive(srv, clk, 4)
    assert srv.results[3].t_done < srv.results[0].t_done


def test_launch_failure_is_reported_and_loop_continues():
    clk = Clock()
    ex = FakeExecutor(clk, durations={i: 0.002 for i in range(5)}, sizes={i: 1 for i in range(5)}, fail={2})
    srv = Server(ex, n_slots=2, mem_cap_bytes=10, clock=clk)
    for i in range(5):
        srv.submit(Request(i, None))
    drive(srv, clk, 5)
    assert not srv.results[2].ok and "injected" in srv.results[2].error
    assert all(srv.results[i].ok for i in (0, 1, 3, 4))
    assert sorted(srv.free_slots) == [0, 1] and srv.reserved == 0


def test_latency_accounting():
    clk = Clock()
    ex = FakeExecutor(clk, durations={0: 0.1, 1: 0.1}, sizes={0: 1, 1: 1})
    srv = Server(ex, n_slots=1, mem_cap_bytes=10, clock=clk)
    srv.submit(Request(0, None))
    srv.submit(Request(1, None))
    drive(srv, clk, 2, dt=1e-3)
    r0, r1 = srv.results[0], srv.results[1]
    assert r0.latency == pytest.approx(0.1, abs=2e-3)
    assert r1.latency == pytest.approx(0.2, abs=3e-3)        # queued behind 0
    assert r1.t_admit >= r0.t_done
    st = latency_stats([r0, r1])
    assert st["completed"] == 2 and st["p99_ms"] >= st["p50_ms"] > 0


def test_serving_request_stream_shape():
    from paper_2604_15017_amd import workloads as W
    reqs = W.serving_requests(200, min_log2_rays=14, max_log2_rays=24)
    kinds = [r.workload.name for r in reqs]
    assert 0.3 < kinds.count("two_layer") / 200 < 0.5
    grads = sum(r.want_grad for r in reqs)
    assert 0.2 < grads / 200 < 0.4
    assert all(r.target is not None for r in reqs if r.want_grad)
    assert {(r.workload.grid.n_x, r.workload.grid.n_z) for r in reqs} == {(128, 256), (256, 512), (512, 1024)}
    assert min(r.total_rays for r in reqs) >= 1 << 13 and max(r.total_rays for r in reqs) <= 1 << 24
