"""The serving loop's scheduling on the CPU, against a fake executor with a
simulated clock: every gate applied once and in order, admission in arrival
order within slots and budget, retirement one step late, eviction after an
arena overflow and resumption from the checkpoint, latency statistics."""
import math

import pytest

from paper_1811_05140_amd import serve as SV


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class Fake:
    """Applies gates to lists; time advances with each step by the work of
    its largest state; overflows the listed requests on their first run."""

    def __init__(self, clock, budget, overflow_once=()):
        self.clock = clock
        self.budget = budget
        self.applied = {}
        self.reserved = 0
        self.max_reserved = 0
        self.open_order = []
        self.steps = []
        self.overflow = set(overflow_once)
        self.live = 0
        self.max_live = 0

    def reservation(self, r):
        return int((1 << r.n) * r.arena_factor)

    def open(self, r):
        assert r.arrival <= self.clock.t + 1e-12
        self.reserved += self.reservation(r)
        assert self.reserved <= self.budget
        self.max_reserved = max(self.max_reserved, self.reserved)
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        self.open_order.append(r.rid)
        h = {"rid": r.rid, "gates": [], "need": self.reservation(r)}
        return h

    def step(self, items):
        self.steps.append([(h["rid"], len(g)) for h, g in items])
        work = 0.0
        for h, g in items:
            h["gates"].extend(g)
            work = max(work, len(g) * 1e-3)
        self.clock.t += work

    def close(self, h, r):
        self.reserved -= h["need"]
        self.live -= 1
        if r.rid in self.overflow:
            self.overflow.discard(r.rid)
            raise SV.Overflow("arena")
        self.applied[r.rid] = list(h["gates"])
        return {"ready_at": self.clock.t, "ok": True}


def specs(count, seed=0):
    import random
    rnd = random.Random(seed)
    out = []
    t = 0.0
    for i in range(count):
        t += rnd.expovariate(1.0)
        n = rnd.randint(4, 9)
        out.append({"id": i, "t1": t, "kind": "qft", "n": n, "eb": 1e-4,
                    "gates": [(i, k) for k in range(rnd.randint(3, 30))]})
    return out


@pytest.mark.parametrize("slots,gps,rate", [(4, 1, 2.0), (16, 3, 50.0), (1, 10 ** 6, 5.0),
                                            (64, 1, math.inf)])
def test_every_gate_once_in_order_within_slots_and_budget(slots, gps, rate):
    clk = Clock()
    budget = 3 * (1 << 9)
    ex = Fake(clk, budget)
    sp = specs(60)
    reqs, summ = SV.serve(sp, ex, budget, slots, gps, rate, clock=clk, sleep=clk.sleep)
    for s in sp:
        assert ex.applied[s["id"]] == s["gates"]
    assert ex.max_live <= slots + 1  # one more may be retiring
    assert ex.max_reserved <= budget
    # admission in arrival order
    assert ex.open_order == sorted(ex.open_order, key=lambda i: (sp[i]["t1"], i))
    for r in reqs:
        assert r.arrival <= r.admitted <= r.ready <= r.done
    assert summ["requests"] == 60 and summ["p50_latency_s"] <= summ["p99_latency_s"]
    assert summ["peak_reserved_bytes"] <= budget


def test_step_gates_and_one_step_late_retirement():
    clk = Clock()
    ex = Fake(clk, 1 << 20)
    sp = [{"id": 0, "t1": 0.0, "kind": "qft", "n": 4, "eb": 1e-4, "gates": list(range(5))},
          {"id": 1, "t1": 0.0, "kind": "qft", "n": 4, "eb": 1e-4, "gates": list(range(2))}]
    SV.serve(sp, ex, 1 << 20, 8, 2, math.inf, clock=clk, sleep=clk.sleep)
    # step 1: both get 2 gates; step 2: request 0 gets 2, request 1 (done) is
    # retired after it; step 3: request 0 gets its last gate
    assert ex.steps == [[(0, 2), (1, 2)], [(0, 2)], [(0, 1)]]


def test_overflow_restarts_with_a_larger_arena():
    clk = Clock()
    budget = 1 << 12
    ex = Fake(clk, budget, overflow_once=(3,))
    sp = specs(10, seed=3)
    reqs, summ = SV.serve(sp, ex, budget, 4, 1, 10.0, clock=clk, sleep=clk.sleep)
    r3 = [r for r in reqs if r.rid == 3][0]
    assert r3.restarts == 1 and r3.arena_factor == 2.0 and summ["restarts"] == 1
    for s in sp:
        assert ex.applied[s["id"]] == s["gates"]


class Evicting(Fake):
    """Overflows the listed requests once, at their middle gate: the state
    rolls back to that gate's input, is checkpointed (here: the gates applied
    so far) and resumes from it when the request is admitted again."""

    def open(self, r):
        h = super().open(r)
        if r.checkpoint is not None:
            h["gates"] = list(r.checkpoint)
            r.checkpoint = None
        h["opened_at"] = r.resume
        return h

    def close(self, h, r):
        if r.rid in self.overflow:
            self.overflow.discard(r.rid)
            self.reserved -= h["need"]
            self.live -= 1
            k = len(r.gates) // 2
            r.checkpoint = h["gates"][:k]
            r.resume = k
            raise SV.Overflow("arena")
        return super().close(h, r)


def test_overflow_evicts_and_resumes_from_the_checkpoint():
    clk = Clock()
    budget = 1 << 12
    ex = Evicting(clk, budget, overflow_once=(2, 5))
    sp = specs(10, seed=4)
    reqs, summ = SV.serve(sp, ex, budget, 4, 1, 10.0, clock=clk, sleep=clk.sleep)
    assert summ["restarts"] == 2
    for s in sp:
        assert ex.applied[s["id"]] == s["gates"]
    for rid in (2, 5):
        r = [q for q in reqs if q.rid == rid][0]
        k = len(sp[rid]["gates"]) // 2
        assert r.restarts == 1 and r.arena_factor == 2.0 and r.resume == k
        # the first run sent every gate (those from k on were rolled back);
        # after re-admission only gates k.. go out again: the gates before
        # the checkpoint are not computed twice
        assert sum(g for st in ex.steps for q, g in st if q == rid) == \
            len(sp[rid]["gates"]) + (len(sp[rid]["gates"]) - k)


def test_request_larger_than_the_budget_is_refused():
    clk = Clock()
    ex = Fake(clk, 100)
    with pytest.raises(ValueError):
        SV.serve(specs(3), ex, 100, 4, 1, 1.0, clock=clk, sleep=clk.sleep)


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert SV.percentile(v, 50) == 50 and SV.percentile(v, 99) == 99
    assert SV.percentile(v, 100) == 100 and SV.percentile([7], 99) == 7


def test_reservation_formula_covers_double_buffering():
    # two arenas of 1.3 x raw + 1 MiB, plus metadata
    n, b = 20, 14
    res = SV.reservation_bytes(n, b)
    assert res >= 2 * (1.3 * (16 << n))
    assert SV.reservation_bytes(n, b, 2.0) > res


def test_serving_workload_shape():
    from paper_1811_05140_amd import inputs as I
    reqs = I.serving_workload()
    assert len(reqs) == 512
    assert all(10 <= r["n"] <= 30 and r["eb"] in (1e-3, 1e-4, 1e-5) for r in reqs)
    assert {r["kind"] for r in reqs} == {"qft", "grover", "random"}
    assert all(1 <= r["iterations"] <= 6 for r in reqs if r["kind"] == "grover")
    ts = [r["t1"] for r in reqs]
    assert ts == sorted(ts) and ts[0] > 0
    # unit-rate arrivals: mean gap close to 1
    assert 0.8 < ts[-1] / len(ts) < 1.2


def test_large_requests_one_at_a_time_first_come_first_served():
    """max_large=1: no step holds two large states; large requests open in
    arrival order; a small request may pass a large one that waits."""
    clk = Clock()
    budget = 1 << 16
    ex = Fake(clk, budget)
    ex.is_large = lambda r: r.n >= 8
    sp = specs(80, seed=5)
    reqs, summ = SV.serve(sp, ex, budget, 16, 2, 200.0, clock=clk, sleep=clk.sleep,
                          max_large=1)
    for s in sp:
        assert ex.applied[s["id"]] == s["gates"]
    large = {s["id"] for s in sp if s["n"] >= 8}
    assert large and len(large) < len(sp)
    for st in ex.steps:
        assert sum(1 for rid, _ in st if rid in large) <= 1
    order = [rid for rid in ex.open_order if rid in large]
    assert order == sorted(order, key=lambda i: (sp[i]["t1"], i))
    # some small request was opened before a large one that arrived earlier
    pos = {rid: k for k, rid in enumerate(ex.open_order)}
    passed = any(pos[s] < pos[l] and sp[l]["t1"] < sp[s]["t1"]
                 for l in large for s in pos if s not in large)
    assert passed
    assert summ["requests"] == 80


def test_no_large_limit_keeps_arrival_order():
    clk = Clock()
    budget = 1 << 16
    ex = Fake(clk, budget)
    ex.is_large = lambda r: r.n >= 8
    sp = specs(40, seed=6)
    SV.serve(sp, ex, budget, 16, 2, 4.0, clock=clk, sleep=clk.sleep)
    assert ex.open_order == sorted(ex.open_order, key=lambda i: (sp[i]["t1"], i))
