"""The serving scheduler on the CPU: a fake executor and a fake clock (no GPU)."""
import pytest

from paper_2401_09283_amd.serve import Request, Server, poisson_requests, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-9)


class FakeExecutor:
    """Each tick costs `tick` seconds; footprints are given per request; can be told to fail."""

    def __init__(self, clock, tick=0.1, fail_admit=(), fail_step_at=None):
        self.clock, self.tick = clock, tick
        self.fail_admit = set(fail_admit)
        self.fail_step_at = fail_step_at
        self.steps = 0
        self.log = []
        self.resident = set()

    def footprint(self, r):
        return r.inputs["bytes"]

    def work(self, r):
        return r.inputs.get("work", 1.0)

    def admit(self, r):
        if r.rid in self.fail_admit:
            raise RuntimeError("bad geometry")
        self.resident.add(r.rid)
        self.log.append(("admit", r.rid, self.clock()))

    def step(self, reqs):
        self.steps += 1
        if self.fail_step_at is not None and self.steps == self.fail_step_at:
            raise RuntimeError("device error")
        self.log.append(("step", tuple(r.rid for r in reqs), self.clock()))
        self.clock.t += self.tick

    def result(self, r):
        return {"rid": r.rid}

    def release(self, r):
        self.resident.discard(r.rid)
        self.log.append(("release", r.rid, self.clock()))


def make(reqspec):
    return [Request(rid, arr, it, {"bytes": b}) for rid, arr, it, b in reqspec]


def test_fifo_admission_by_slots_and_memory_and_continuous_batching():
    clk = FakeClock()
    ex = FakeExecutor(clk, tick=0.1)
    srv = Server(ex, hbm_budget_bytes=100, max_active=2, clock=clk, sleep=clk.sleep)
    reqs = srv.run(make([(0, 0.0, 3, 60), (1, 0.05, 2, 30), (2, 0.06, 2, 50), (3, 1.0, 1, 10)]))
    assert all(r.status == "done" for r in reqs)
    steps = [e[1] for e in ex.log if e[0] == "step"]
    # 0 alone; 1 joins at the next tick (arrived while 0 was on the GPU); 2 waits for memory
    assert steps[0] == (0,)
    assert steps[1] == (0, 1)
    assert (2,) in steps or any(2 in s for s in steps)
    first2 = next(i for i, s in enumerate(steps) if 2 in s)
    # 2 (50 B) only fits after 0 (60 B) retired
    release0 = next(i for i, e in enumerate(ex.log) if e[0] == "release" and e[1] == 0)
    admit2 = next(i for i, e in enumerate(ex.log) if e[0] == "admit" and e[1] == 2)
    assert admit2 > release0
    assert srv.used == 0 and not ex.resident
    assert first2 >= 2
    s = summarize(reqs)
    assert s["done"] == 4 and s["p50_s"] > 0


def test_budget_never_exceeded_and_oversized_request_fails_alone():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    srv = Server(ex, hbm_budget_bytes=100, max_active=8, clock=clk, sleep=clk.sleep)
    seen = []
    orig = ex.step

    def step(reqs):
        seen.append(sum(r.inputs["bytes"] for r in reqs))
        orig(reqs)

    ex.step = step
    reqs = srv.run(make([(0, 0.0, 2, 40), (1, 0.0, 2, 40), (2, 0.0, 2, 40), (3, 0.0, 1, 500)]))
    assert max(seen) <= 100
    st = {r.rid: r.status for r in reqs}
    assert st == {0: "done", 1: "done", 2: "done", 3: "failed"}
    assert "exceeds" in reqs[3].error


def test_failed_admission_and_failed_tick_do_not_block_others():
    clk = FakeClock()
    ex = FakeExecutor(clk, fail_admit={1}, fail_step_at=2)
    srv = Server(ex, hbm_budget_bytes=1000, max_active=4, clock=clk, sleep=clk.sleep)
    reqs = srv.run(make([(0, 0.0, 3, 10), (1, 0.0, 3, 10), (2, 5.0, 2, 10)]))
    st = {r.rid: r.status for r in reqs}
    assert st[1] == "failed" and "admit" in reqs[1].error
    assert st[0] == "failed" and "step" in reqs[0].error   # the second tick failed
    assert st[2] == "done"                                 # a later request still runs
    assert srv.used == 0


def test_idle_server_waits_for_arrivals():
    clk = FakeClock()
    ex = FakeExecutor(clk, tick=0.01)
    srv = Server(ex, 100, 4, clock=clk, sleep=clk.sleep)
    reqs = srv.run(make([(0, 3.0, 1, 1)]))
    assert reqs[0].t_admit >= 3.0 and reqs[0].status == "done"


def test_poisson_stream_is_seeded():
    a = poisson_requests(64, 2.0, 40, 30)
    b = poisson_requests(64, 2.0, 40, 30)
    assert a == b
    arr = [x[1] for x in a]
    assert arr[0] == 0.0 and all(y >= x for x, y in zip(arr, arr[1:]))
    # mean inter-arrival close to 1 / rate
    assert abs((arr[-1] / 63) - 0.5) < 0.2
    assert {x[2] for x in a} == {"serve128", "serve256", "serve384"}


def _srpt_case(policy):
    clk = FakeClock()
    ex = FakeExecutor(clk, tick=0.1)
    srv = Server(ex, hbm_budget_bytes=1000, max_active=8, clock=clk, sleep=clk.sleep, policy=policy, tick_work=2.0)
    reqs = [Request(0, 0.0, 5, {"bytes": 10, "work": 10.0}), Request(1, 0.0, 3, {"bytes": 10, "work": 1.0}),
            Request(2, 0.0, 2, {"bytes": 10, "work": 1.0})]
    return srv.run(reqs), ex, srv


def test_srpt_advances_the_least_remaining_work_first():
    reqs, ex, srv = _srpt_case("srpt")
    steps = [e[1] for e in ex.log if e[0] == "step"]
    # the two small requests share ticks until they are done, then the large one runs alone
    assert steps == [(1, 2), (1, 2), (1,), (0,), (0,), (0,), (0,), (0,)]
    assert all(r.status == "done" and r.iters_done == r.n_iter for r in reqs)
    done = {r.rid: r.t_done for r in reqs}
    assert done[2] < done[1] < done[0]
    assert srv.used == 0 and not ex.resident


def test_processor_sharing_advances_every_active_request():
    reqs, ex, _ = _srpt_case("all")
    steps = [e[1] for e in ex.log if e[0] == "step"]
    assert steps[:2] == [(0, 1, 2), (0, 1, 2)] and steps[2] == (0, 1)
    assert all(r.status == "done" for r in reqs)
    assert [r.result for r in reqs] == [r.result for r in _srpt_case("srpt")[0]]


def test_srpt_lets_a_large_request_through_when_nothing_smaller_waits():
    clk = FakeClock()
    ex = FakeExecutor(clk, tick=0.1)
    srv = Server(ex, hbm_budget_bytes=1000, max_active=8, clock=clk, sleep=clk.sleep, policy="srpt", tick_work=2.0)
    reqs = srv.run([Request(0, 0.0, 2, {"bytes": 10, "work": 10.0}), Request(1, 0.05, 1, {"bytes": 10, "work": 1.0})])
    steps = [e[1] for e in ex.log if e[0] == "step"]
    # 0 starts alone; 1 arrives during the first tick and overtakes at the next one
    assert steps == [(0,), (1,), (0,)]
    assert all(r.status == "done" for r in reqs)


def test_unknown_policy_is_rejected():
    with pytest.raises(ValueError):
        Server(FakeExecutor(FakeClock()), 100, policy="lifo")


def test_srpt_with_a_waiting_cap_serves_old_requests_first():
    clk = FakeClock()
    ex = FakeExecutor(clk, tick=0.1)
    srv = Server(ex, hbm_budget_bytes=1000, max_active=8, clock=clk, sleep=clk.sleep, policy="srpt", tick_work=2.0,
                 max_wait=0.25)
    reqs = srv.run([Request(0, 0.0, 3, {"bytes": 10, "work": 10.0}), Request(1, 0.05, 6, {"bytes": 10, "work": 1.0})])
    steps = [e[1] for e in ex.log if e[0] == "step"]
    # 1 overtakes 0 at the second tick, until 0 has waited more than 0.25 s; then 0 goes first
    assert steps[:3] == [(0,), (1,), (1,)]
    assert steps[3] == (0,)
    assert all(r.status == "done" and r.iters_done == r.n_iter for r in reqs)
    # without the cap, 0 waits until 1 is done
    clk2 = FakeClock()
    ex2 = FakeExecutor(clk2, tick=0.1)
    Server(ex2, 1000, 8, clock=clk2, sleep=clk2.sleep, policy="srpt", tick_work=2.0).run(
        [Request(0, 0.0, 3, {"bytes": 10, "work": 10.0}), Request(1, 0.05, 6, {"bytes": 10, "work": 1.0})])
    assert [e[1] for e in ex2.log if e[0] == "step"] == [(0,)] + [(1,)] * 6 + [(0,), (0,)]


def test_cancellation_frees_the_slot_and_the_memory():
    clk = FakeClock()

    class CancellingExecutor(FakeExecutor):
        server = None

        def step(self, reqs):
            super().step(reqs)
            if self.steps == 2:
                self.server.cancel(0)   # the long request, while it is active
                self.server.cancel(3)   # a request that has not arrived yet

    ex = CancellingExecutor(clk, tick=0.1)
    srv = Server(ex, hbm_budget_bytes=100, max_active=2, clock=clk, sleep=clk.sleep, policy="all")
    ex.server = srv
    reqs = srv.run(make([(0, 0.0, 50, 60), (1, 0.0, 2, 40), (2, 0.05, 2, 60), (3, 5.0, 1, 10)]))
    st = {r.rid: r.status for r in reqs}
    assert st == {0: "cancelled", 1: "done", 2: "done", 3: "cancelled"}
    # 2 (60 B) could only be admitted once 0 (60 B) was cancelled and released
    rel0 = next(i for i, e in enumerate(ex.log) if e[0] == "release" and e[1] == 0)
    adm2 = next(i for i, e in enumerate(ex.log) if e[0] == "admit" and e[1] == 2)
    assert adm2 > rel0
    assert srv.used == 0 and not ex.resident
    assert sum(1 for e in ex.log if e[0] == "step" and 0 in e[1]) == 2


class FakeAsyncExecutor(FakeExecutor):
    """Enqueues iterations on a simulated device that runs them one after another (each takes
    the request's `cost` seconds of device time); completion is seen through the fake clock."""

    depth = 2

    def __init__(self, clock):
        super().__init__(clock)
        self.device_free = 0.0
        self.jobs = {}          # rid -> completion times of enqueued iterations
        self.max_in_flight = 0

    def step(self, reqs):
        self.steps += 1
        self.log.append(("step", tuple(r.rid for r in reqs), self.clock()))
        for r in reqs:
            assert self.in_flight(r) < self.depth
            start = max(self.device_free, self.clock())
            self.device_free = start + r.inputs.get("cost", 0.1)
            self.jobs.setdefault(r.rid, []).append(self.device_free)
            self.max_in_flight = max(self.max_in_flight, self.in_flight(r))
        self.clock.t += 1e-4   # host time to enqueue

    def in_flight(self, r):
        return sum(1 for t in self.jobs.get(r.rid, []) if t > self.clock())

    def finished(self, r):
        return self.in_flight(r) == 0

    def wait(self, reqs):
        pending = [t for r in reqs for t in self.jobs.get(r.rid, []) if t > self.clock()]
        assert pending, "wait() with nothing in flight"
        self.clock.t = min(pending)

    def result(self, r):
        assert self.finished(r)
        return {"rid": r.rid, "t_last": max(self.jobs[r.rid])}


def test_asynchronous_executor_keeps_depth_and_retires_after_the_device():
    clk = FakeClock()
    ex = FakeAsyncExecutor(clk)
    srv = Server(ex, hbm_budget_bytes=100, max_active=3, clock=clk, sleep=clk.sleep, policy="srpt", tick_work=3.0,
                 min_batch=2)
    reqs = [Request(0, 0.0, 4, {"bytes": 40, "work": 10.0, "cost": 0.2}),
            Request(1, 0.0, 3, {"bytes": 40, "work": 1.0, "cost": 0.05}),
            Request(2, 0.01, 2, {"bytes": 40, "work": 1.0, "cost": 0.05}),
            Request(3, 0.5, 2, {"bytes": 10, "work": 1.0, "cost": 0.05})]
    done = srv.run(reqs)
    assert all(r.status == "done" and r.iters_done == r.n_iter for r in done)
    assert ex.max_in_flight <= FakeAsyncExecutor.depth
    for r in done:
        # a request retires only once its last iteration has finished on the device
        assert r.t_done >= r.result["t_last"] - 1e-12
        assert len(ex.jobs[r.rid]) == r.n_iter
    # request 2 (40 B) could only be admitted after one of the first two retired
    adm2 = next(i for i, e in enumerate(ex.log) if e[0] == "admit" and e[1] == 2)
    first_rel = next(i for i, e in enumerate(ex.log) if e[0] == "release")
    assert adm2 > first_rel
    assert srv.used == 0 and not ex.resident
    # min_batch: while two requests were active, ticks took two even beyond the work budget
    steps = [e[1] for e in ex.log if e[0] == "step"]
    assert steps[0] == (0, 1)
