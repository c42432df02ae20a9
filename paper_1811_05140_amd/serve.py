"""Serving loop: circuits arrive over time, their compressed states stay
resident in HBM, and every step advances all admitted states together.

Scheduling (continuous batching):
  * requests are admitted in arrival order while a slot is free and their
    memory reservation fits the budget still unreserved (a request that does
    not fit waits, and so do the ones behind it);
  * optionally (`max_large`), at most that many "large" requests -- states
    that fill the GPU by themselves, as the executor judges -- are active at
    once, taken first come first served; a large request that must wait
    keeps its place but does not hold back smaller requests behind it.
    Batching adds nothing to the throughput of such states, while sharing
    steps between several of them stretches each one's latency;
  * each step applies the next `gates_per_step` gates of every admitted
    request in one batched launch sequence (one kernel set for all states);
  * a request whose last gate went out in step k is retired after step k + 1
    has been queued, so the device keeps working while the host reads its
    result; retiring frees its reservation, and waiting requests are admitted
    before the next step.
The one-circuit-at-a-time baseline is the same loop with one slot and the
whole circuit as one step, run through sim_apply_gate.

A state whose arena overflows (the library reports SIM_ENOMEM and rolls the
state back to the input of the gate that overflowed) is evicted: the
executor copies its block streams to host memory (a checkpoint) and frees
its device memory, and the request goes back to the head of the queue with
twice the arena; when it is admitted again it resumes from that gate (the
executor sets `resume`, the gate index the checkpoint holds), so no gate is
computed twice.

The executor is the only part that touches the GPU; the scheduler is plain
Python and is tested on the CPU against a fake executor.
"""
import collections
import math
import time


class Overflow(Exception):
    """The state outgrew its arena (it resumes later with a larger one)."""


class Request:
    __slots__ = ("rid", "arrival", "kind", "n", "eb", "basis", "gates", "marked",
                 "iterations", "arena_factor", "restarts", "admitted", "ready", "done",
                 "result", "reserved", "handle", "pos", "large", "resume", "checkpoint")

    def __init__(self, spec, rate):
        self.rid = spec["id"]
        self.arrival = spec["t1"] / rate if rate != math.inf else 0.0
        self.kind = spec["kind"]
        self.n = spec["n"]
        self.eb = spec["eb"]
        self.basis = spec.get("basis", 0)
        self.gates = spec["gates"]
        self.marked = spec.get("marked")
        self.iterations = spec.get("iterations")
        self.arena_factor = 1.0
        self.restarts = 0
        self.admitted = self.ready = self.done = None
        self.result = None
        self.reserved = 0
        self.handle = None
        self.pos = 0
        self.large = False
        self.resume = 0          # gate index a re-admitted request starts at
        self.checkpoint = None   # executor-owned host copy of an evicted state


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100]) of a non-empty list."""
    v = sorted(values)
    k = max(0, min(len(v) - 1, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[k]


def serve(specs, executor, budget_bytes, max_slots, gates_per_step=1, rate=math.inf,
          clock=time.perf_counter, sleep=time.sleep, max_large=None):
    """Run the request stream; returns (requests, summary).  max_large: at
    most this many requests for which executor.is_large(r) holds are active
    at once (None: no such limit)."""
    reqs = [Request(s, rate) for s in specs]
    pending = sorted(reqs, key=lambda r: (r.arrival, r.rid))
    active = []
    retiring = []
    reserved = 0
    large_active = 0
    steps = 0
    peak_active = 0
    peak_reserved = 0
    t0 = clock()
    while pending or active or retiring:
        now = clock() - t0
        # admission: arrival order, slots and budget; a large request over
        # the limit is passed over (it keeps its place)
        i = 0
        while i < len(pending) and pending[i].arrival <= now and len(active) < max_slots:
            r = pending[i]
            big = max_large is not None and executor.is_large(r)
            if big and large_active >= max_large:
                i += 1
                continue
            need = executor.reservation(r)
            if need > budget_bytes:
                raise ValueError("request %d needs %d bytes, more than the budget"
                                 % (r.rid, need))
            if reserved + need > budget_bytes:
                break
            del pending[i]
            r.reserved = need
            reserved += need
            r.large = big
            large_active += int(big)
            r.handle = executor.open(r)
            r.pos = r.resume
            if r.admitted is None:
                r.admitted = now
            active.append(r)
        peak_active = max(peak_active, len(active))
        peak_reserved = max(peak_reserved, reserved)
        if active:
            items = []
            for r in active:
                g = r.gates[r.pos:r.pos + gates_per_step]
                r.pos += len(g)
                items.append((r.handle, g))
            executor.step(items)
            steps += 1
        # retire what finished in the previous step
        for r in retiring:
            try:
                r.result = executor.close(r.handle, r)
                r.ready = r.result.pop("ready_at") - t0
                r.done = clock() - t0
            except Overflow:
                r.restarts += 1
                r.arena_factor *= 2.0
                pending.insert(0, r)
            r.handle = None
            reserved -= r.reserved
            r.reserved = 0
            large_active -= int(r.large)
            r.large = False
        retiring = [r for r in active if r.pos >= len(r.gates)]
        active = [r for r in active if r.pos < len(r.gates)]
        if not active and not retiring and pending:
            wait = min(q.arrival for q in pending) - (clock() - t0)
            if wait > 0:
                sleep(wait)
    lat = [r.ready - r.arrival for r in reqs]
    makespan = max(r.ready for r in reqs) - min(r.arrival for r in reqs)
    gates = sum(len(r.gates) for r in reqs)
    summary = {
        "requests": len(reqs),
        "p50_latency_s": percentile(lat, 50),
        "p99_latency_s": percentile(lat, 99),
        "mean_latency_s": sum(lat) / len(lat),
        "makespan_s": makespan,
        "gates_per_s": gates / makespan if makespan > 0 else float("inf"),
        "requests_per_s": len(reqs) / makespan if makespan > 0 else float("inf"),
        "steps": steps,
        "peak_active": peak_active,
        "peak_reserved_bytes": peak_reserved,
        "restarts": sum(r.restarts for r in reqs),
    }
    return reqs, summary


# ------------------------------------------------------------- executor ----

def reservation_bytes(n, b, arena_factor=1.0, levels=5):
    """Device bytes a state of n qubits holds: two arenas of
    ceil(1.3 * factor * 16 * 2^n) + 1 MiB (the pass's speculative encode at
    the previous level can take up to the raw size before a replay, on top of
    the kept streams), plus descriptors, size tables and reduction scratch."""
    s = min(b, 10)
    nseg = 1 << (n - s)
    nblocks = 1 << (n - b)
    arena = arena_bytes(n, arena_factor)
    # per segment, two descriptor sets of two 4-byte record offsets and an
    # 8-byte norm, the size table (4 bytes per plane and level), the mean
    # pre-pass sums; per block, two sets of header, length, level and scale,
    # the replay and escalation lists, norms, sums and checkpoint offsets
    per_seg = 2 * (8 + 8) + 8 * levels + 16
    per_block = 2 * (32 + 4 + 1 + 8) + 4 + 4 + 8 + 16 + 8
    # (the pass kernels' staging is one device-wide buffer, indexed by
    # hardware wave slot, shared by every sim: not part of a request)
    return 2 * arena + per_seg * nseg + per_block * nblocks + 4096


def arena_bytes(n, arena_factor=1.0):
    return int(math.ceil(1.3 * arena_factor * (16 << n))) + (1 << 20)


class GpuExecutor:
    """Opens one compressed sim per request (own stream), steps them with a
    shared batch, and measures results at retirement.  A request is large
    when a pass over its state has at least `large_units` workgroup units
    (8192: eight per resident workgroup of a full MI355X, so the state keeps
    the GPU busy by itself)."""

    def __init__(self, A, max_slots, gates_per_step=1, sequential=False, tune=None,
                 probs_qubits=4, large_units=8192, arena_scale=0.3):
        self.A = A
        # First arena relative to 1.3 x the raw state: 0.3 gives 0.39 x raw
        # per arena, room for the compressed streams of a pass (ratio >= 4 at
        # theta 4 when a level meets it) plus speculation; a state that still
        # outgrows it is evicted and resumed with twice the arena, so the
        # budget admits by compressed size instead of by raw size.
        self.arena_scale = arena_scale
        self.sequential = sequential
        self.batch = None if sequential else A.Batch(max_slots, gates_per_step)
        self.tune = tune or {}
        self.probs_qubits = probs_qubits
        self.large_units = large_units

    def block_log2(self, r):
        from paper_1811_05140_amd import autotune, inputs
        t = autotune.lookup(self.tune, r.n, inputs.default_ladder(r.eb), 4.0)
        if t is not None:
            return t[0]
        return min(r.n, 14)

    def reservation(self, r):
        return reservation_bytes(r.n, self.block_log2(r), self.arena_scale * r.arena_factor)

    def is_large(self, r):
        s = min(self.block_log2(r), 10)
        units = 1 if r.n == s else 1 << (r.n - s - 1)
        return units >= self.large_units

    def open(self, r):
        sim = self.A.Sim(r.n, self.block_log2(r), r.eb,
                         arena_bytes=arena_bytes(r.n, self.arena_scale * r.arena_factor))
        if r.checkpoint is not None:
            sim.import_state(r.checkpoint)  # resume an evicted state at r.resume
            r.checkpoint = None
        else:
            sim.set_basis(r.basis)
        return sim

    def step(self, items):
        if self.sequential:
            for sim, gates in items:
                sim.run(gates)
            return
        sims = [sim for sim, g in items if g]
        rows = [g for _, g in items if g]
        if not sims:
            return
        P = max(len(g) for g in rows)
        passes = [[g[p] if p < len(g) else None for g in rows] for p in range(P)]
        self.batch.apply(sims, passes, use_graph=False)

    def close(self, sim, r):
        A = self.A
        try:
            nq = min(self.probs_qubits, r.n)
            probs = sim.probs(list(range(nq)))
        except A.SimError as e:
            if e.code == A.SIM_ENOMEM:
                # rolled back to the input of the gate that overflowed (the
                # passes counted since the state was set or imported): evict
                # it to host memory (through the entropy stage: fewer bytes
                # over PCIe and in host memory) and resume from that gate later
                done = sim.stats()["passes"]
                r.checkpoint = sim.export_state(entropy=True)
                r.resume += done
                sim.close()
                raise Overflow(str(e))
            sim.close()
            raise
        ready = time.perf_counter()
        st = sim.stats()
        out = {"ready_at": ready, "probs": probs.tolist(), "normsq": st["normsq"],
               "resident_bytes": st["resident_bytes"], "min_ratio": st["min_ratio"],
               "level_hist": st["level_hist"], "signature": signature(sim, r)}
        if r.kind == "qft":
            out["fidelity"] = sim.fourier_fidelity(r.basis)
        elif r.kind == "grover":
            P, Pc, F = grover_closed_form(sim, r.n, r.marked, r.iterations)
            out.update({"fidelity": F, "p_marked": P, "p_marked_closed_form": Pc})
        sim.close()
        return out


def signature(sim, r):
    """Bytes that pin a final state: every block stream (the whole-state
    export, block 0 first), N^2, the scale and the resident bytes (compared
    between a request run in the mix and alone, and across an eviction; the
    level histogram and replay counts are history since the state was set
    or imported, not state)."""
    import hashlib
    h = hashlib.sha256()
    h.update(sim.export_state())
    st = sim.stats()
    h.update(repr((st["normsq"], st["scale"], st["resident_bytes"])).encode())
    return h.hexdigest()


def grover_closed_form(sim, n, m, k):
    """P(m) and the fidelity to the closed-form Grover state after k
    iterations (sin((2k+1)t) on m, cos((2k+1)t)/sqrt(2^n - 1) elsewhere,
    sin t = 2^(-n/2)), from the amplitude sum and a_m."""
    th = math.asin(2.0 ** (-n / 2.0))
    alpha = math.sin((2 * k + 1) * th)
    beta = math.cos((2 * k + 1) * th) / math.sqrt(float((1 << n) - 1))
    am = complex(sim.amplitudes(m, 1)[0])
    S = sim.amplitude_sum()
    st = sim.stats()
    F = abs(beta * S + (alpha - beta) * am) ** 2 / (st["normsq"] * st["scale"] ** 2)
    return abs(am) ** 2, alpha ** 2, F


def random_fidelity(A, spec, b, arena_factor=1.0):
    """Fidelity of a random-circuit request against its uncompressed run
    (the request is run alone again, compressed, to have its final state;
    its signature must equal the one recorded in the mix)."""
    class R:
        pass
    r = R()
    r.n, r.kind = spec["n"], spec["kind"]
    sim = A.Sim(spec["n"], b, spec["eb"], arena_bytes=arena_bytes(spec["n"], arena_factor))
    sim.set_basis(spec.get("basis", 0))
    sim.run(spec["gates"])
    sig = signature(sim, r)
    ref = A.Sim(spec["n"], b, -1.0)
    ref.set_basis(spec.get("basis", 0))
    ref.run(spec["gates"])
    F = sim.fidelity(ref)
    ref.close()
    sim.close()
    return F, sig
