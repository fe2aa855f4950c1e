"""The serving request loop's host logic on the CPU, against a simulated batch core with
the C-ABI's admission contract (slots, one frame in flight per stream, HBM budget over
resident streams) and a simulated device that runs one batched step per millisecond.
Checks first-come first-served admission, per-stream ordering, least-recently-used
eviction under budget pressure, completion of every request and the latency accounting."""

from types import SimpleNamespace

import numpy as np

from paper_2307_03017_amd import hsgd, scenes, serving


class FakeBatch:
    STEP_S = 1e-3

    def __init__(self, clock, slots, budget):
        self.clock, self.slots, self.budget = clock, slots, budget
        self.used = 0
        self.streams = {}           # id -> (bytes, in_flight)
        self.active = {}            # ticket -> [stream_id, steps_left]
        self.done_at = {}           # ticket -> device completion time
        self.device_free = 0.0
        self.next_ticket = 0
        self.t_ref = 0.0
        self.admit_log = []

    def reference(self, stream=None):
        self.t_ref = self.clock()

    def admit(self, st):
        sid = st.stream_id
        if sid in self.streams and self.streams[sid][1]:
            self.last_refusal = hsgd.HSGD_E_CAPACITY
            return None
        if len(self.active) >= self.slots:
            self.last_refusal = hsgd.HSGD_E_CAPACITY
            return None
        if sid not in self.streams:
            if self.used + st.bytes > self.budget:
                self.last_refusal = hsgd.HSGD_E_BUDGET
                return None
            self.used += st.bytes
            self.streams[sid] = [st.bytes, False]
        self.streams[sid][1] = True
        t = self.next_ticket
        self.next_ticket += 1
        self.active[t] = [sid, st.total]
        self.admit_log.append((t, sid))
        return t

    def step(self, stream=None):
        if not self.active:
            return 0, []
        start = max(self.clock(), self.device_free)
        self.device_free = start + self.STEP_S
        fin = []
        for t in list(self.active):
            self.active[t][1] -= 1
            if self.active[t][1] == 0:
                self.streams[self.active[t][0]][1] = False
                self.done_at[t] = self.device_free
                fin.append(t)
                del self.active[t]
        return len(self.active) + len(fin), fin

    def poll(self, t):
        d = self.done_at.get(t)
        if d is None or self.clock() < d:
            return False, -1.0
        return True, (d - self.t_ref) * 1e3

    def release_stream(self, sid):
        if self.streams[sid][1]:
            return False
        self.used -= self.streams.pop(sid)[0]
        return True

    @property
    def budget_used(self):
        return self.used


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-5            # every host call costs a little time
        return self.t

    def sleep(self, dt):
        self.t += dt


def make_inputs():
    out = []
    for cfg, seed in serving.MIX:
        sc = scenes.make_scene(cfg, seed=seed)
        out.append(SimpleNamespace(sc=sc, inits=[None] * 2))
    return out


def fake_stream(i, si):
    lvl = SimpleNamespace(copy_=lambda src: None)
    return SimpleNamespace(stream_id=i, bytes=si.sc.D * si.sc.W * si.sc.H * 8, total=sum(si.sc.iters),
                           levels=[lvl], result=None)


def run_sim(budget_streams, n=300, rate=60.0, slots=4):
    clock = SimClock()
    inputs = make_inputs()
    sizes = sorted(si.sc.D * si.sc.W * si.sc.H * 8 for si in inputs)
    budget = sum(sizes[-budget_streams:])            # room for the largest few streams
    fb = FakeBatch(clock, slots, budget)
    srv = serving.Server(inputs, batch=fb, make_stream=fake_stream)
    reqs = serving.poisson_requests(n, rate, len(inputs), 2, seed=5)
    done = serving.run(srv, reqs, clock=clock, sleep=clock.sleep)
    return srv, fb, reqs, done, inputs


def test_every_request_completes_in_order_per_stream():
    srv, fb, reqs, done, inputs = run_sim(budget_streams=8)
    assert len(done) == len(reqs)
    assert all(r.done > r.arrival and r.admitted >= r.arrival for r in done)
    # frames of one stream complete in arrival order (one frame in flight per stream)
    for s in range(len(inputs)):
        mine = [r for r in reqs if r.scene == s]
        assert [r.arrival for r in sorted(mine, key=lambda r: r.done)] == [r.arrival for r in mine]
    # latency of a lone 3-iteration frame: about 3 steps
    lat = np.array([r.done - r.arrival for r in done])
    assert np.median(lat) < 0.02
    s = serving.summary(done, 20, inputs)
    assert s["requests"] == len(reqs) - 20 and 0 < s["p50_ms"] <= s["p99_ms"]
    assert 40 < s["frames_per_s"] < 80


def test_budget_pressure_evicts_idle_streams():
    srv, fb, reqs, done, inputs = run_sim(budget_streams=2)
    assert len(done) == len(reqs)
    assert fb.used <= fb.budget
    assert len(srv.streams) <= 8 and len(fb.streams) == len(srv.streams)


def test_first_come_first_served_among_admissible():
    clock = SimClock()
    inputs = make_inputs()
    fb = FakeBatch(clock, 2, 1 << 40)
    srv = serving.Server(inputs, batch=fb, make_stream=fake_stream)
    reqs = [serving.Served(s, 0, 0.0) for s in (0, 1, 2, 3)] + [serving.Served(0, 1, 0.0)]
    serving.run(srv, reqs, clock=clock, sleep=clock.sleep)
    order = [sid for _, sid in fb.admit_log]
    assert order[:2] == [0, 1]                   # two slots, queue order
    assert order.index(2) < order.index(3)
    assert order.count(0) == 2
