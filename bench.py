#!/usr/bin/env python3
"""Benchmark of the compressed per-gate loop on one MI355X.

Default workload (qft24): the 24-qubit QFT (312 native gates: H, controlled
phase, SWAP) on a seeded basis state, complex128 state of 2^24 amplitudes
held as 256 compressed blocks of 2^16, default AALC ladder (0, eb/1000,
eb/100, eb/10, eb) with eb = 1e-4 and ratio threshold 4.  One step = encode
the basis state + apply the 312 gates (every gate is one decompress-
normalise-gate-compress pass over all blocks).

--workload batch64: 64 seeded random brick circuits (n in [16, 28], depth
20, eb = 1e-4) advanced together, one captured HIP graph launch per layer,
block size and grid from the autotuner's table; also reports the same
circuits run one at a time and checks that both give the same states.

--workload serve512: 512 requests (QFT, Grover, random; 10..30 qubits;
three error bounds) with Poisson arrivals and a 200 GB compressed-memory
budget, served with continuous batching and one circuit at a time.

--workload qft12: the 12-qubit QFT (64 KiB state, launch-bound): gates/s and
microseconds per gate, beside the whole oracle run.

--workload qft24sweep: QFT-24 at error bounds 1e-3, 1e-4, 1e-5, each with
the default ladder at ratio thresholds 4, 8, 16, 32 and with the fixed bound
alone; throughput, ratios and fidelity per point.

--workload checkpoint: export the whole compressed state to pinned host
memory and import it into a second sim (QFT-24 final state, or --state
grover36); GB/s of checkpoint bytes, the import kernels' roofline entry.

--workload grover36: Grover search on 36 qubits (2^36 amplitudes, 1 TiB as
complex128, more than the 288 GB of HBM), 65536 blocks of 2^20, eb = 1e-5:
H on every qubit, then 8 x (phase flip of a seeded index, diffusion).  One
step = encode |0> + the 52 gates (each diffusion adds a read-only mean pass).

The state is resident in HBM before timing starts.  Prints one JSON line:
gates/s (value), amplitude-GB/s and its fraction of the 8 TB/s HBM peak, the
dominant kernel's roofline entry (HIP events on the sim stream over the timed
region), the fidelity (against the uncompressed FP64 run of the same circuit
for qft24, against the closed-form Grover state for grover36), and the CPU
oracle timed on a block sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("gates/s and amplitude-GB/s (% of HBM peak) at fidelity ≥0.999; "
          "serving p50/p99")
HBM_PEAK_GBS = 8000.0
LOGICAL_BYTES_PER_AMP = 32  # one read + one write of a complex128 per pass


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "gates.h", "device.h"):
        with open(os.path.join(ROOT, "paper_1811_05140_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(workload, kernel):
    """The committed PMC summary of this workload's kernel, if it was taken
    on the current kernel source (else {})."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return {}
    try:
        d = json.load(open(path))
    except ValueError:
        return {}
    if d.get("kernel_source_sha") != kernel_source_hash():
        return {}
    return d.get("kernels", {}).get(kernel) or {}


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed PMC summary (or None)."""
    return measured_counters(workload, kernel).get("hbm_bytes_per_launch")


def cpu_baseline(A, orc, inputs, w, eb, budget_s, name):
    """The CPU oracle on a block sample of the same workload: at every gate
    random block groups are exported from the GPU state and recomputed by the
    oracle until that gate's share of the budget is spent (at least one
    group); the mean time per group, times the number of groups of the gate,
    estimates the oracle's time for the whole gate."""
    import numpy as np
    n, b = w["n"], w["b"]
    s = min(b, 10)
    lad = inputs.default_ladder(eb)
    nb = 1 << (n - b)
    sim = A.Sim(n, b, eb)
    sim.set_basis(w["basis"])
    rng = np.random.default_rng(5)
    n_diffuse = 0
    per_gate = budget_s / len(w["gates"])
    spent = 0.0
    est = 0.0
    groups = 0
    for gate in w["gates"]:
        kind = gate[0]
        mask = 0
        if kind in (inputs.G_U, inputs.G_X):
            mask = 1 << gate[1]
        elif kind == inputs.G_CU:
            mask = 1 << gate[2]
        elif kind == inputs.G_SWAP:
            mask = (1 << gate[1]) | (1 << gate[2])
        mb = mask >> b
        ngroups = nb // 2 if mb else nb
        sc = sim.stats()["scale"]
        tdiff = None
        if kind == inputs.G_DIFFUSE:
            S = sim.amplitude_sum()
            tdiff = (S.real * 2.0 ** (1 - n), S.imag * 2.0 ** (1 - n))
            n_diffuse += 1
        g_spent = 0.0
        g_count = 0
        while g_count == 0 or g_spent < per_gate:
            j = int(rng.integers(0, nb))
            j = min(j, j ^ mb) if mb else j
            in0 = sim.export_block(j)
            in1 = sim.export_block(j ^ mb) if mb else None
            t0 = time.perf_counter()
            orc.process_group(n, b, s, lad, 4.0, sc, tdiff, gate, j, in0, in1)
            g_spent += time.perf_counter() - t0
            g_count += 1
        spent += g_spent
        est += g_spent / g_count * ngroups
        groups += g_count
        sim.apply(gate)
    sim.close()
    return {
        "value": len(w["gates"]) / est,
        "unit": "gates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("all %d %s gates, %d random block groups in total "
                   "(oracle time %.1f s, single thread), each gate's mean group "
                   "time scaled by its groups%s" %
                   (len(w["gates"]), name, groups, spent,
                    "; the oracle's whole-state mean pass of each of the %d "
                    "diffusions is not included" % n_diffuse if n_diffuse else "")),
        "host_cpus": os.cpu_count(),
    }


def cpu_baseline_gates(A, orc, inputs, w, eb, stride, shortcut, name):
    """The CPU oracle on whole gates of the same workload, on all host
    cores: every `stride`-th gate (from the middle of each run of `stride`)
    is applied by the oracle to the whole state -- imported from the GPU run
    just before that gate, which equals the oracle's own state bit for bit --
    with its block groups spread over the host's threads by OpenMP; each
    timed gate stands for the `stride` gates around it.  The oracle's output
    streams are checked against the GPU's after the gate."""
    import hashlib as hl
    n, b = w["n"], w["b"]
    lad = inputs.default_ladder(eb)
    threads = orc.set_threads(min(os.cpu_count() or 1, 16))
    sim = A.Sim(n, b, eb)
    sim.set_shortcut(shortcut)
    sim.set_basis(w["basis"])
    osim = orc.OracleSim(n, b, lad, 4.0)
    osim.set_shortcut(shortcut)
    gates = w["gates"]
    times = []
    same = True
    for k, gate in enumerate(gates):
        if k % stride == stride // 2:
            osim.import_state(sim.export_state())
            t0 = time.perf_counter()
            osim.apply(gate)
            times.append(time.perf_counter() - t0)
            sim.apply(gate)
            same = same and (hl.sha256(osim.export_state()).digest() ==
                             hl.sha256(sim.export_state()).digest())
        else:
            sim.apply(gate)
    sim.close()
    est = sum(times) * stride * len(gates) / (stride * len(times))
    return {
        "value": len(gates) / est,
        "unit": "gates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": ("%d of the %d %s gates (every %dth), each applied by the oracle to the "
                   "whole state on %d threads (OpenMP over block groups), the state "
                   "imported from the GPU run before the gate; timed %.1f s, scaled by %d; "
                   "oracle streams %s the GPU's after every timed gate" %
                   (len(times), len(gates), name, stride, threads, sum(times), stride,
                    "equal to" if same else "DIFFERENT FROM")),
        "host_cpus": os.cpu_count(),
        "host_cpu_model": cpu_model(),
    }


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def calibrate_copy(torch, nbytes, reps):
    """A plain device copy of known size, for scaling HBM counters."""
    x = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": nbytes, "reps": reps}), flush=True)


def coupled_block_mask(inputs, gate, b):
    kind = gate[0]
    if kind in (inputs.G_U, inputs.G_X):
        mask = 1 << gate[1]
    elif kind == inputs.G_CU:
        mask = 1 << gate[2]
    elif kind == inputs.G_SWAP:
        mask = (1 << gate[1]) | (1 << gate[2])
    else:
        mask = 0
    return mask >> b


def cpu_baseline_batch(A, orc, inputs, insts, conf, eb, budget_s):
    """The CPU oracle's cost per amplitude-pass on a block sample of the
    batched workload (instances in a seeded order, every gate, one random
    group per gate, until the budget is spent), times the workload's
    amplitude-passes."""
    import numpy as np
    lad = inputs.default_ladder(eb)
    rng = np.random.default_rng(6)
    order = [int(v) for v in rng.permutation(len(insts))]
    spent = 0.0
    amps = 0
    groups = 0
    used = []
    for k in order:
        if spent >= budget_s:
            break
        n = insts[k]["n"]
        b, _ = conf[k]
        s = min(b, 10)
        nb = 1 << (n - b)
        sim = A.Sim(n, b, eb)
        sim.set_basis(0)
        used.append(n)
        for layer in insts[k]["layers"]:
            for gate in layer:
                mb = coupled_block_mask(inputs, gate, b)
                j = int(rng.integers(0, nb))
                j = min(j, j ^ mb) if mb else j
                in0 = sim.export_block(j)
                in1 = sim.export_block(j ^ mb) if mb else None
                sc = sim.stats()["scale"]
                t0 = time.perf_counter()
                orc.process_group(n, b, s, lad, 4.0, sc, None, gate, j, in0, in1)
                spent += time.perf_counter() - t0
                amps += (2 if mb else 1) << b
                groups += 1
                sim.apply(gate)
        sim.close()
    per_amp = spent / amps
    total_gates = sum(len(g) for i in insts for g in i["layers"])
    total_amps = sum(len(g) << i["n"] for i in insts for g in i["layers"])
    return {
        "value": total_gates / (per_amp * total_amps),
        "unit": "gates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("%d block groups over every gate of %d instances (n = %s; oracle "
                   "time %.1f s, single thread); oracle seconds per amplitude-pass "
                   "times the workload's %.3e amplitude-passes"
                   % (groups, len(used), used, spent, total_amps)),
        "host_cpus": os.cpu_count(),
    }


def bench_batch64(args, A, inputs, stream):
    """64 random brick circuits advanced together: one graph launch per
    layer (each pass of a layer applies one gate to every instance that has
    one)."""
    from paper_1811_05140_amd import autotune
    eb = args.error_bound if args.error_bound is not None else 1e-4
    lad = inputs.default_ladder(eb)
    insts = inputs.random_batch_workload()
    table = autotune.load_table()
    conf = []
    for inst in insts:
        t = autotune.lookup(table, inst["n"], lad, 4.0)
        conf.append(t if t is not None else (min(16, inst["n"]), 2048))
    tuned = all(autotune.lookup(table, i["n"], lad, 4.0) is not None for i in insts)
    sims = []
    for inst, (b, grid) in zip(insts, conf):
        # default arenas (2.1 x raw): a pass's speculative encode at the
        # previous level can take up to the raw size before a replay
        sm = A.Sim(inst["n"], b, eb, stream=stream)
        sm.set_grid(grid)
        sm.set_shortcut(args.shortcut)
        sims.append(sm)
    depth = len(insts[0]["layers"])
    layer_passes = []
    for l in range(depth):
        gl = [i["layers"][l] for i in insts]
        P = max(len(g) for g in gl)
        layer_passes.append([[g[p] if p < len(g) else None for g in gl] for p in range(P)])
    batch = A.Batch(len(insts), max(len(lp) for lp in layer_passes), stream=stream)

    def step(use_graph=True):
        for sm in sims:
            sm.set_basis(0)
        for lp in layer_passes:
            batch.apply(sims, lp, use_graph=use_graph)

    for _ in range(args.warmup):
        step()
    batch.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    batch.sync()
    for sm in sims:
        sm.sync()
    elapsed = time.perf_counter() - t0
    gates_per_inst = [sum(len(g) for g in i["layers"]) for i in insts]
    total_gates = sum(gates_per_inst)
    amp_bytes = sum(g * 32 * (1 << i["n"]) for g, i in zip(gates_per_inst, insts))

    def signature(k):
        # every block stream of the final state, with N^2 and the statistics
        sm = sims[k]
        st = sm.stats()
        return (st["normsq"], st["resident_bytes"], tuple(st["level_hist"]),
                hashlib.sha256(sm.export_state()).hexdigest())

    sig_batch = [signature(k) for k in range(len(insts))]
    stats = [sm.stats() for sm in sims]
    info = batch.info()
    # the same circuits one at a time through sim_apply_gate
    t0 = time.perf_counter()
    for k, inst in enumerate(insts):
        sims[k].set_basis(0)
        for layer in inst["layers"]:
            sims[k].run(layer)
    for sm in sims:
        sm.sync()
    alone_s = time.perf_counter() - t0
    same = all(signature(k) == sig_batch[k] for k in range(len(insts)))
    # per-kernel times of one batched step launched directly (events)
    batch.profile(True)
    batch.profile_read()
    step(use_graph=False)
    prof = batch.profile_read()
    batch.profile(False)
    roofline = None
    if "pass" in prof:
        cnt, tot, mn, mx = prof["pass"]
        # algorithmic bytes of every batched pass of the step (each state's
        # compressed streams in and out plus its per-plane metadata, from an
        # untimed replay of every instance alone, which gives the same
        # streams) over the k_bpass time
        alg = 0
        for k, inst in enumerate(insts):
            flat = [g for layer in inst["layers"] for g in layer]
            alg += pass_stream_bytes(sims[k], 0, flat, inst["n"], conf[k][0],
                                     count_basis=False)
        achieved = alg / (tot / 1000.0) / 1e9
        logical = amp_bytes / (tot / 1000.0) / 1e9
        roofline = {
            "bound": "hbm", "kernel": "pass (batched)", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("batch64", "bpass"),
            "avg_launch_ms": round(tot / cnt, 4), "launches": cnt,
            "algorithmic_bytes_per_launch": alg // cnt,
            "algorithmic_bytes": "compressed streams in + out and per-plane metadata of "
                                 "every state in the pass, averaged over the step's launches",
            "logical_gbs": round(logical, 1),
            "logical_frac": round(logical / HBM_PEAK_GBS, 4),
            "kernels_ms_one_step": {k: round(v[1], 3) for k, v in sorted(prof.items())},
        }
    # fidelity of every instance against its uncompressed run (the runs,
    # one instance at a time, also give the uncompressed path's rate)
    Fs = []
    sv_s = 0.0
    for k, inst in enumerate(insts):
        ref = A.Sim(inst["n"], conf[k][0], -1.0, stream=stream)
        ref.sync()
        t0 = time.perf_counter()
        ref.set_basis(0)
        for layer in inst["layers"]:
            ref.run(layer)
        ref.sync()
        sv_s += time.perf_counter() - t0
        Fs.append(sims[k].fidelity(ref))
        ref.close()
    Fs_sorted = sorted(Fs)
    cpu = None
    if args.cpu_budget > 0 and not args.shortcut:
        from oracle import oracle as orc
        cpu = cpu_baseline_batch(A, orc, inputs, insts, conf, eb, args.cpu_budget)
    for sm in sims:
        sm.close()
    batch.close()
    gps = total_gates * args.steps / elapsed
    amp_gbs = amp_bytes * args.steps / elapsed / 1e9
    b_by_n = {}
    for inst, (b, grid) in zip(insts, conf):
        b_by_n[str(inst["n"])] = [b, grid]
    return {
        "metric": METRIC, "value": round(gps, 2), "unit": "gates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded random brick circuits)",
        "config": {"workload": "batch64", "instances": len(insts),
                   "n_qubits": [i["n"] for i in insts], "depth": depth,
                   "error_bound": eb, "ladder": lad, "theta": 4.0,
                   "gates_per_step": total_gates, "block_log2_and_grid_by_n": b_by_n,
                   "autotuned": tuned, "graph_launch_per_layer": True,
                   "shortcut": args.shortcut},
        # the metric's logical amplitude traffic (32 B per amplitude per gate,
        # what an uncompressed simulator moves) and its fraction of the HBM
        # peak; the HBM fraction of the bytes the pass really moves is
        # hbm_frac (the roofline's algorithmic bytes)
        "amplitude_gbs": round(amp_gbs, 1),
        "logical_frac": round(amp_gbs / HBM_PEAK_GBS, 4),
        "hbm_frac": roofline["frac"] if roofline else None,
        "one_at_a_time_gates_per_s": round(total_gates / alone_s, 2),
        "batch_speedup": round((total_gates * args.steps / elapsed) / (total_gates / alone_s), 3),
        "uncompressed_gates_per_s": round(total_gates / sv_s, 2),
        "compressed_over_uncompressed": round((total_gates * args.steps / elapsed) /
                                              (total_gates / sv_s), 3),
        "alone_equals_batch": same,
        "fidelity": Fs_sorted[0], "fidelity_median": Fs_sorted[len(Fs) // 2],
        "fidelity_ok_count": sum(1 for f in Fs if f >= 0.999),
        "fidelity_ok": bool(Fs_sorted[0] >= 0.999),
        "fidelity_reference": "uncompressed FP64 GPU run of each instance",
        "min_ratio": min(st["min_ratio"] for st in stats),
        "peak_resident_bytes": sum(st["peak_resident"] for st in stats),
        "logical_state_bytes": sum(16 << i["n"] for i in insts),
        "graph": info,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


SERVE_RATE = None  # requests/s; fixed from a saturated run (see --rate)


def bench_serve(args, A, inputs, stream):
    """512 requests (QFT / Grover / random, n in [10, 30], eb in {1e-3, 1e-4,
    1e-5}) with Poisson arrivals at `rate`, 200 GB compressed budget, served
    with continuous batching (at most one large request active: one whose
    pass has 8192 or more units) and, on the same arrivals, one circuit at a
    time; p50/p99 latency, gates/s and per-request fidelity."""
    from paper_1811_05140_amd import autotune, serve as SV
    specs = inputs.serving_workload(count=args.requests)
    table = autotune.load_table()
    budget = int(200e9)
    slots, G = 64, 4
    last = [time.perf_counter()]

    class Progress:
        def __init__(self, ex):
            self.ex = ex
            self.done = 0

        def __getattr__(self, k):
            return getattr(self.ex, k)

        def close(self, h, r):
            out = self.ex.close(h, r)
            self.done += 1
            if time.perf_counter() - last[0] > 10:
                last[0] = time.perf_counter()
                print("serve: %d requests done" % self.done, file=sys.stderr, flush=True)
            return out

    def run(rate, sequential):
        ex = SV.GpuExecutor(A, slots, G, sequential=sequential, tune=table)
        if sequential:
            return SV.serve(specs, Progress(ex), budget, 1, 10 ** 9, rate)
        return SV.serve(specs, Progress(ex), budget, slots, G, rate, max_large=1)

    out = {"metric": METRIC, "unit": "gates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic (seeded request stream)"}
    rate = args.rate
    if rate is None:
        # saturated batched throughput (all requests at t = 0) fixes the rate
        _, sat = run(math.inf, False)
        rate = 0.7 * sat["requests_per_s"]
        out["saturated"] = sat
    reqs, summ = run(rate, False)
    reqs1, summ1 = run(rate, True)
    by1 = {r.rid: r for r in reqs1}
    same = sum(1 for r in reqs if r.result["signature"] == by1[r.rid].result["signature"])
    # random circuits: fidelity against uncompressed runs (n <= 24 all, larger sampled)
    import numpy as np
    rng = np.random.default_rng(7)
    big = [r for r in reqs if r.kind == "random" and r.n > 24]
    pick = {r.rid for r in big if rng.random() < 6.0 / max(1, len(big))}
    checked_random = 0
    for r in reqs:
        if r.kind != "random" or (r.n > 24 and r.rid not in pick):
            continue
        ex = SV.GpuExecutor(A, 1, 1, sequential=True, tune=table)
        F, sig = SV.random_fidelity(A, specs[r.rid], ex.block_log2(r), r.arena_factor)
        assert sig == r.result["signature"]
        r.result["fidelity"] = F
        checked_random += 1
    Fs = [r.result["fidelity"] for r in reqs if "fidelity" in r.result]
    per_kind = {}
    for kind in ("qft", "grover", "random"):
        f = [r.result["fidelity"] for r in reqs if r.kind == kind and "fidelity" in r.result]
        if f:
            per_kind[kind] = {"count": len(f), "min": min(f), "median": sorted(f)[len(f) // 2],
                              "ok": sum(1 for v in f if v >= 0.999)}
    out.update({
        "value": round(summ["gates_per_s"], 2),
        "ms_per_step": round(1000.0 * summ["makespan_s"], 3),
        "config": {"workload": "serve512", "requests": len(specs), "rate_per_s": rate,
                   "n_range": [10, 30], "error_bounds": [1e-3, 1e-4, 1e-5],
                   "budget_bytes": budget, "slots": slots, "gates_per_step": G,
                   "max_large": 1, "large_units": 8192,
                   "gates": sum(len(s["gates"]) for s in specs)},
        "batched": summ, "one_at_a_time": summ1,
        "p50_latency_s": summ["p50_latency_s"], "p99_latency_s": summ["p99_latency_s"],
        "one_at_a_time_p50_s": summ1["p50_latency_s"],
        "one_at_a_time_p99_s": summ1["p99_latency_s"],
        "mix_equals_alone": "%d of %d" % (same, len(reqs)),
        "fidelity": min(Fs) if Fs else None,
        "fidelity_by_kind": per_kind,
        "fidelity_note": ("QFT: closed form (Fourier overlap); Grover: closed form; random: "
                          "uncompressed run, %d of %d random requests (all n <= 24, a "
                          "seeded sample above)" % (checked_random,
                                                    sum(1 for r in reqs if r.kind == "random"))),
        "roofline": None, "cpu_baseline": None,
    })
    return out


def bench_checkpoint(args, A, inputs, stream):
    """Checkpoint and resume of a resident compressed state: the QFT-24 state
    after all 312 gates (default) or the Grover-36 state after its 8
    iterations (--state grover36).  One step = export the whole state
    (kernels stage the block streams in the idle arena, one copy to pinned
    host memory) + import it into a second sim (one copy to the device, the
    record checks, the decode that re-forms the segment norms, N^2).  The
    resumed state is checked to re-export the same bytes and, for QFT-24,
    to finish its circuit identically to the uninterrupted run."""
    import numpy as np
    import torch
    grover = args.state == "grover36"
    w = inputs.grover36_workload() if grover else inputs.qft24_workload()
    eb = 1e-5 if grover else 1e-4
    n, b = w["n"], w["b"]
    src = A.Sim(n, b, eb, stream=stream)
    src.set_basis(w["basis"])
    src.run(w["gates"])
    src.sync()
    nbytes = src.stats()["resident_bytes"]
    host = torch.empty(nbytes + 4096, dtype=torch.uint8, pin_memory=True)
    hv = host.numpy()
    dst = A.Sim(n, b, eb, stream=stream)
    print("checkpoint: %s state, %d bytes" % (args.state, nbytes), file=sys.stderr, flush=True)

    def step(timed_kernels=False):
        assert src.export_state(out=hv) == nbytes
        dst.import_state(hv, nbytes)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    # separate legs and pageable host memory, for the record
    te0 = time.perf_counter()
    for _ in range(args.steps):
        src.export_state(out=hv)
    te1 = time.perf_counter()
    for _ in range(args.steps):
        dst.import_state(hv, nbytes)
    te2 = time.perf_counter()
    pageable = src.export_state()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        dst.import_state(pageable)
    tp1 = time.perf_counter()
    # device kernels, all timed with events on the sim streams
    src.profile(True)
    dst.profile(True)
    src.profile_read()
    dst.profile_read()
    for _ in range(args.steps):
        step()
    prof = dict(src.profile_read())
    prof.update(dst.profile_read())
    src.profile(False)
    dst.profile(False)
    same = dst.export_state() == bytes(hv[:nbytes])
    st = dst.stats()
    ss = src.stats()
    same = same and st["normsq"] == ss["normsq"] and st["scale"] == ss["scale"]
    if not grover:
        # resume: finish a second copy of the circuit's last 60 gates from a
        # checkpoint taken before them, compare with the uninterrupted run
        cut = len(w["gates"]) - 60
        a = A.Sim(n, b, eb, stream=stream)
        a.set_basis(w["basis"])
        a.run(w["gates"][:cut])
        r = A.Sim(n, b, eb, stream=stream)
        r.import_state(a.export_state())
        a.run(w["gates"][cut:])
        r.run(w["gates"][cut:])
        same = same and a.export_state() == r.export_state()
        a.close()
        r.close()
    # the entropy stage (block entropy streams) on this state and, for
    # QFT-24, on the state after 200 gates, where most chunks still hold a
    # few nonzero residuals: sizes, both legs through pinned memory, and the
    # resumed state's v1 streams
    def entropy_leg(sim, label):
        v1 = sim.export_state()
        e = sim.export_state(entropy=True)
        ebuf = torch.empty(len(e) + 4096, dtype=torch.uint8, pin_memory=True)
        ev = ebuf.numpy()
        r = A.Sim(n, b, eb, stream=stream)
        r.import_state(ev, sim.export_state(out=ev, entropy=True))
        c0 = time.perf_counter()
        for _ in range(args.steps):
            ne = sim.export_state(out=ev, entropy=True)
        c1 = time.perf_counter()
        for _ in range(args.steps):
            r.import_state(ev, ne)
        c2 = time.perf_counter()
        ok = r.export_state() == v1 and bytes(ev[:ne]) == e
        r.close()
        return {"state": label, "v1_bytes": len(v1), "entropy_bytes": len(e),
                "v1_over_entropy": round(len(v1) / len(e), 3),
                "logical_ratio": round((16 << n) / len(e), 1),
                "export_ms": round(1000.0 * (c1 - c0) / args.steps, 3),
                "import_ms": round(1000.0 * (c2 - c1) / args.steps, 3),
                "resume_identical": bool(ok)}

    entropy = [entropy_leg(src, "final")]
    if not grover:
        m = A.Sim(n, b, eb, stream=stream)
        m.set_basis(w["basis"])
        m.run(w["gates"][:200])
        entropy.append(entropy_leg(m, "after 200 gates"))
        m.close()
    spb = 1 << (b - min(b, 10))
    nblocks = 1 << (n - b)
    nseg = nblocks * spb
    planes = 2 * nseg
    # algorithmic bytes per launch of each kernel
    alg = {
        "export": 2 * nbytes,                       # read the records, write the streams
        "import_scan": 24 * planes + 64 * nblocks,  # plane headers in, offsets + headers out
        "import_check": 32 * planes,                # headers, widths, first word, offsets
        "import_norm": nbytes + 8 * planes + 8 * nseg,  # every record decoded, norms out
        "import_blocks": 8 * nseg + 8 * nblocks,
    }
    kern = {}
    for name, (cnt, tot, mn, mx) in prof.items():
        kern[name] = {"launches": cnt, "avg_ms": round(tot / cnt, 4)}
        if name in alg:
            kern[name]["gbs"] = round(alg[name] / (tot / cnt / 1000.0) / 1e9, 1)
    name = max((k for k in prof if k in alg), key=lambda k: prof[k][1])
    cnt, tot = prof[name][0], prof[name][1]
    achieved = alg[name] / (tot / cnt / 1000.0) / 1e9
    roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "avg_launch_ms": round(tot / cnt, 4), "launches": cnt,
                "algorithmic_bytes_per_launch": alg[name], "kernels": kern}
    cpu = None
    if args.cpu_budget > 0:
        # the oracle's import is, per block, or_decode_block (records checked
        # as they are read) plus the block normsq: timed on random blocks of
        # this checkpoint until the budget is spent, scaled by bytes
        from oracle import oracle as orc
        starts = [0]
        for _ in range(nblocks):
            starts.append(starts[-1] + int.from_bytes(pageable[starts[-1] + 12:starts[-1] + 16],
                                                      "little"))
        rng = np.random.default_rng(11)
        done_bytes, tcpu, k = 0, 0.0, 0
        budget = min(args.cpu_budget, 20.0)
        while tcpu < budget and k < 4 * nblocks:
            j = int(rng.integers(0, nblocks))
            blk = pageable[starts[j]:starts[j + 1]]
            c0 = time.perf_counter()
            xh = orc.decode_block(blk)
            v = np.ascontiguousarray(xh).view(np.float64)
            orc.pairwise((v[0::2] * v[0::2]) + (v[1::2] * v[1::2]))
            tcpu += time.perf_counter() - c0
            done_bytes += len(blk)
            k += 1
        t_full = tcpu * nbytes / done_bytes
        cpu = {"value": round(nbytes / t_full / 1e9, 4), "unit": "GB/s of checkpoint imported",
               "cores": 1, "kind": "oracle",
               "sample": "%d random blocks of the checkpoint decoded by the oracle's block "
                         "decoder with the block normsq (%.1f s), scaled by bytes to all %d "
                         "blocks" % (k, tcpu, nblocks)}
    gbs = 2 * nbytes * args.steps / elapsed / 1e9
    return {
        "metric": "checkpoint export + import of the compressed state (GB/s of streams, "
                  "both directions, pinned host memory)",
        "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1000.0 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded basis state, generated circuit)",
        "config": {"workload": "checkpoint", "state": args.state, "n_qubits": n,
                   "block_log2": b, "error_bound": eb, "checkpoint_bytes": nbytes,
                   "logical_state_bytes": 16 << n},
        "export_ms": round(1000.0 * (te1 - te0) / args.steps, 3),
        "import_ms": round(1000.0 * (te2 - te1) / args.steps, 3),
        "import_pageable_ms": round(1000.0 * (tp1 - tp0) / args.steps, 3),
        "resume_identical": bool(same),
        "entropy_stage": entropy,
        "roofline": roofline, "cpu_baseline": cpu,
    }


def bench_qft12(args, A, inputs, stream):
    """The 12-qubit QFT (84 gates, 16 blocks of 2^8, eb = 1e-4, default
    ladder): a state of 64 KiB, so a pass is bound by launch latency, and the
    figure is microseconds per gate.  The oracle runs the whole circuit (no
    sampling) on one core, repeated for about 10 s."""
    import torch
    w = inputs.qft12_workload()
    n, b, x, gates = w["n"], w["b"], w["basis"], w["gates"]
    sim = A.Sim(n, b, 1e-4, stream=stream)

    def step():
        sim.set_basis(x)
        sim.run(gates)
    for _ in range(args.warmup):
        step()
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    sim.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gps = len(gates) * args.steps / el
    ref = A.Sim(n, b, -1.0, stream=stream)
    ref.set_basis(x)
    ref.run(gates)
    F = sim.fidelity(ref)
    ref.close()
    st = sim.stats()
    # the same circuit as one captured HIP graph of 84 passes (a batch of one
    # state), replayed each step after the basis encode
    sim2 = A.Sim(n, b, 1e-4, stream=stream)
    batch = A.Batch(1, len(gates), stream=stream)
    passes = [[g] for g in gates]

    def gstep():
        sim2.set_basis(x)
        batch.apply([sim2], passes, use_graph=True)
    for _ in range(max(args.warmup, 1)):
        gstep()
    batch.sync()
    sim2.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gstep()
    batch.sync()
    sim2.sync()
    torch.cuda.synchronize()
    gel = time.perf_counter() - t0
    ggps = len(gates) * args.steps / gel
    graph_same = sim2.export_state() == sim.export_state()
    batch.close()
    sim2.close()
    cpu = None
    if args.cpu_budget > 0:
        from oracle import oracle as orc

        def oracle_rate(threads, budget):
            # the oracle's passes spread block groups over OpenMP threads
            used = orc.set_threads(threads)
            runs, tcpu = 0, 0.0
            while tcpu < budget:
                o = orc.OracleSim(n, b, inputs.default_ladder(1e-4), 4.0)
                c0 = time.perf_counter()
                o.set_basis(x)
                o.run(gates)
                tcpu += time.perf_counter() - c0
                runs += 1
                o.close()
            return len(gates) * runs / tcpu, runs, tcpu, used

        budget = min(args.cpu_budget, 10.0) / 2
        v1, r1, t1, _ = oracle_rate(1, budget)
        va, ra, ta, used = oracle_rate(min(os.cpu_count() or 1, 16), budget)
        cpu = {"value": round(v1, 2), "unit": "gates/s", "cores": 1,
               "kind": "oracle",
               "sample": "the whole QFT-12 circuit (basis encode + 84 gates), %d runs in "
                         "%.1f s, single thread" % (r1, t1),
               "all_cores": {"value": round(va, 2), "cores": used,
                             "sample": "%d runs in %.1f s, OpenMP over block groups"
                                       % (ra, ta)}}
    sim.close()
    return {
        "metric": METRIC, "value": round(gps, 1), "unit": "gates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000.0 * el / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded basis state, generated circuit)",
        "config": {"workload": "qft12", "n_qubits": n, "block_log2": b, "error_bound": 1e-4,
                   "basis": x, "gates_per_step": len(gates)},
        "us_per_gate": round(1e6 / gps, 2),
        "graph_gates_per_s": round(ggps, 1),
        "graph_us_per_gate": round(1e6 / ggps, 2),
        "graph_state_identical": bool(graph_same),
        "amplitude_gbs": round(gps * LOGICAL_BYTES_PER_AMP * (1 << n) / 1e9, 2),
        "fidelity": F, "fidelity_reference": "uncompressed FP64 GPU run",
        "min_ratio": st["min_ratio"], "roofline": None, "cpu_baseline": cpu,
        "note": "64 KiB state: every pass is four kernel launches of a few microseconds; "
                "launch latency, not bandwidth, bounds it",
    }


def bench_qft24_sweep(args, A, inputs, stream):
    """QFT-24 over the error bounds {1e-3, 1e-4, 1e-5}: the default ladder at
    ratio thresholds 4, 8, 16 and 32 (the paper's AALC runs vary the
    threshold), and the fixed bound alone (one lossy level, the paper's
    fixed-bound SZ runs); for 1e-3 and 1e-4 also the pointwise-relative
    ladder at thresholds 4, 16, 32 and the fixed relative bound.  Per point: gates/s, amplitude-GB/s and its HBM
    fraction, minimum / last compression ratio, peak resident bytes, level
    histogram, replays, and the fidelity against one uncompressed FP64 run."""
    import torch
    w = inputs.qft24_workload()
    n, b, x, gates = w["n"], w["b"], w["basis"], w["gates"]
    ref = A.Sim(n, b, -1.0, stream=stream)
    ref.set_basis(x)
    ref.run(gates)
    points = []
    for eb in (1e-3, 1e-4, 1e-5):
        confs = [("aalc", inputs.default_ladder(eb), th) for th in (4.0, 8.0, 16.0, 32.0)]
        confs.append(("fixed", [eb], 4.0))
        if eb >= 1e-4:
            # the pointwise-relative bound of the same size (entries -eps)
            confs += [("relative", inputs.relative_ladder(eb), th) for th in (4.0, 16.0, 32.0)]
            confs.append(("fixed-relative", [-eb], 4.0))
        for mode, lad, th in confs:
            sim = A.Sim(n, b, eb, stream=stream, ladder=lad, theta=th)

            def step():
                sim.set_basis(x)
                sim.run(gates)
            for _ in range(args.warmup):
                step()
            sim.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                step()
            sim.sync()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            gps = len(gates) * args.steps / el
            gbs = gps * LOGICAL_BYTES_PER_AMP * (1 << n) / 1e9
            st = sim.stats()
            F = sim.fidelity(ref)
            pt = {"error_bound": eb, "mode": mode, "ladder": lad,
                  "theta": th if mode in ("aalc", "relative") else None,
                  "gates_per_s": round(gps, 1), "amplitude_gbs": round(gbs, 1),
                  "logical_frac": round(gbs / HBM_PEAK_GBS, 4),
                  "min_ratio": round(st["min_ratio"], 3), "last_ratio": round(st["last_ratio"], 3),
                  "peak_resident_bytes": st["peak_resident"], "fidelity": F,
                  "fidelity_ok": bool(F >= 0.999), "collapsed": st["collapsed"],
                  "level_hist_per_step": [v // (args.warmup + args.steps) for v in st["level_hist"]],
                  "replays_per_step": st["replays"] // (args.warmup + args.steps)}
            print("sweep: %s" % json.dumps(pt), file=sys.stderr, flush=True)
            points.append(pt)
            sim.close()
    ref.close()
    head = [p for p in points if p["error_bound"] == 1e-4 and p["theta"] == 4.0][0]
    return {
        "metric": METRIC, "value": head["gates_per_s"], "unit": "gates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000.0 * len(gates) / head["gates_per_s"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded basis state, generated circuit)",
        "config": {"workload": "qft24sweep", "n_qubits": n, "block_log2": b, "basis": x,
                   "gates_per_step": len(gates), "error_bounds": [1e-3, 1e-4, 1e-5],
                   "thetas": [4, 8, 16, 32], "value_point": "eb 1e-4, theta 4"},
        "fidelity_reference": "uncompressed FP64 GPU run",
        "points": points, "roofline": None, "cpu_baseline": None,
    }


def pass_stream_bytes(sim, x, gates, n, b, count_basis=True):
    """Algorithmic HBM bytes of one step's pass launches (the roofline's
    per-launch figure is this over the launches): each pass reads its input
    state's compressed streams and writes its output's, and per plane reads
    and writes a record offset (4 B each) and writes a size word (4 B), per
    segment a normsq (8 B).  Measured by replaying the step untimed with the
    resident bytes read after every gate; the basis encode reads nothing."""
    s = min(b, 10)
    planes = 2 << (n - s)
    meta = 12 * planes + 8 * (planes // 2)
    sim.set_basis(x)
    prev = sim.stats()["resident_bytes"]
    total = prev + meta if count_basis else 0
    for g in gates:
        sim.apply(g)
        cur = sim.stats()["resident_bytes"]
        total += prev + cur + meta
        prev = cur
    return total


def grover_fidelity(sim, n, m, k):
    """P(m) and F against the closed-form Grover state after k iterations:
    sin((2k+1)t) on m and cos((2k+1)t)/sqrt(2^n - 1) elsewhere, sin t =
    2^(-n/2).  The overlap needs only the amplitude sum and a_m."""
    th = math.asin(2.0 ** (-n / 2.0))
    alpha = math.sin((2 * k + 1) * th)
    beta = math.cos((2 * k + 1) * th) / math.sqrt(float((1 << n) - 1))
    am = complex(sim.amplitudes(m, 1)[0])
    S = sim.amplitude_sum()
    st = sim.stats()
    F = abs(beta * S + (alpha - beta) * am) ** 2 / (st["normsq"] * st["scale"] ** 2)
    return abs(am) ** 2, alpha ** 2, F


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("qft24", "grover36", "batch64", "serve512",
                                           "checkpoint", "qft24sweep", "qft12"),
                    default="qft24")
    ap.add_argument("--state", choices=("qft24", "grover36"), default="qft24",
                    help="checkpoint workload: the state exported and imported")
    ap.add_argument("--rate", type=float, default=SERVE_RATE,
                    help="serve512 arrival rate (requests/s); default: 0.7 x the "
                         "saturated batched throughput, measured first")
    ap.add_argument("--requests", type=int, default=512, help="serve512 request count")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 5 for qft24, 1 for grover36)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default 1 for qft24, 0 for grover36)")
    ap.add_argument("--error-bound", type=float, default=None,
                    help="default 1e-4 for qft24, 1e-5 for grover36")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of oracle time for the CPU baseline (0: skip)")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without per-kernel events (no roofline entry)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only run a device copy of this many bytes (counters)")
    ap.add_argument("--grid", type=int, default=0,
                    help="qft24 / grover36: workgroups of the per-gate unit kernels (0: the "
                         "fastest of 1024, 2048, 3072 and 4096 on one untimed step each, "
                         "before the warmup; -1: the library's default)")
    ap.add_argument("--shortcut", type=int, default=0, choices=(0, 1, 2, 3),
                    help="Sec. V shortcuts for qft24 / grover36: 1 permutation "
                         "levels, 2 skip unchanged blocks, 3 both (default 0: Alg. 2)")
    ap.add_argument("--cpu-stride", type=int, default=16,
                    help="qft24 CPU baseline: time every n-th gate on the whole state")
    args = ap.parse_args()
    grover = args.workload == "grover36"
    if args.steps is None:
        args.steps = {"qft24": 5, "qft24sweep": 3, "qft12": 200}.get(args.workload, 1)
    if args.warmup is None:
        args.warmup = 1 if args.workload != "grover36" else 0
    eb = args.error_bound if args.error_bound is not None else (1e-5 if grover else 1e-4)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this simulator runs on one GPU; --gpus %d is not "
              "supported (multi-GPU sharding is a design note only)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        calibrate_copy(torch, args.calibrate_copy, 10)
        return
    from paper_1811_05140_amd import aalcsim as A
    from paper_1811_05140_amd import inputs

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.workload == "batch64":
        print(json.dumps(bench_batch64(args, A, inputs, stream)), flush=True)
        return
    if args.workload == "serve512":
        # The 512-request serving run took a GPU memory fault (an address
        # outside every allocation, reported at the first retirement's
        # probability query, so raised by an earlier batched pass or basis
        # encode) with the current kernels, arenas of 0.39 x the raw state and
        # the extended tune table.  Until its cause is found the workload does
        # not run.
        sys.exit("bench.py: the serve512 workload is disabled until the cause of its GPU "
                 "memory fault is found")
    if args.workload == "qft12":
        print(json.dumps(bench_qft12(args, A, inputs, stream)), flush=True)
        return
    if args.workload == "qft24sweep":
        print(json.dumps(bench_qft24_sweep(args, A, inputs, stream)), flush=True)
        return
    if args.workload == "checkpoint":
        print(json.dumps(bench_checkpoint(args, A, inputs, stream)), flush=True)
        return
    w = inputs.grover36_workload() if grover else inputs.qft24_workload()
    n, b, x, gates = w["n"], w["b"], w["basis"], w["gates"]
    sim = A.Sim(n, b, eb, stream=stream)
    sim.set_shortcut(args.shortcut)

    def step():
        sim.set_basis(x)
        sim.run(gates)

    # the unit kernels' grid (a launch parameter: results are the same at
    # every grid): by default the fastest candidate on one untimed step of
    # this circuit each, after one untimed step at it, with the pass timers
    # of the timed region on
    grid_trials = None
    if args.grid == 0:
        grid_trials = {}
        if not args.no_profile:
            sim.profile(True, pass_only=True)
        for g in (1024, 2048, 3072, 4096):
            sim.set_grid(g)
            step()
            sim.sync()
            t0 = time.perf_counter()
            step()
            sim.sync()
            grid_trials[g] = round(1000.0 * (time.perf_counter() - t0), 3)
        sim.profile(False)
        sim.set_grid(min(grid_trials, key=grid_trials.get))
    elif args.grid > 0:
        sim.set_grid(args.grid)
    grid_used = (min(grid_trials, key=grid_trials.get) if grid_trials
                 else (args.grid if args.grid > 0 else "library default"))

    for _ in range(args.warmup):
        step()
    sim.sync()
    torch.cuda.synchronize()
    if not args.no_profile:
        sim.profile(True, pass_only=True)
        sim.profile_read()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {} if args.no_profile else sim.profile_read()
    sim.profile(False)
    elapsed = t1 - t0
    # per-kernel split of one more step (all kernels timed), for the record
    split = {}
    if not args.no_profile and not grover:
        sim.profile(True)
        sim.profile_read()
        step()
        split = {k: round(v[1], 3) for k, v in sorted(sim.profile_read().items())}
        sim.profile(False)
    ms_per_step = 1000.0 * elapsed / args.steps
    gates_per_s = len(gates) * args.steps / elapsed
    amp_gbs = gates_per_s * LOGICAL_BYTES_PER_AMP * (1 << n) / 1e9
    st = sim.stats()

    extra = {}
    if grover:
        k = sum(1 for g in gates if g[0] == inputs.G_DIFFUSE)
        P, P_closed, F = grover_fidelity(sim, n, w["marked"], k)
        extra = {"p_marked": P, "p_marked_closed_form": P_closed,
                 "fidelity_reference": "closed-form Grover state"}
    else:
        # fidelity against the uncompressed FP64 run of the same circuit,
        # whose second run (untimed for the metric) gives the uncompressed
        # path's own rate on this circuit
        ref = A.Sim(n, b, -1.0, stream=stream)
        ref.set_basis(x)
        ref.run(gates)
        ref.sync()
        t0 = time.perf_counter()
        ref.set_basis(x)
        ref.run(gates)
        ref.sync()
        sv_gps = len(gates) / (time.perf_counter() - t0)
        F = sim.fidelity(ref)
        ref.close()
        extra = {"fidelity_reference": "uncompressed FP64 GPU run",
                 "uncompressed_gates_per_s": round(sv_gps, 1),
                 "compressed_over_uncompressed": round(gates_per_s / sv_gps, 3)}

    roofline = None
    if prof:
        name, (cnt, tot, mn, mx) = max(prof.items(), key=lambda kv: kv[1][1])
        avg_s = tot / cnt / 1000.0
        # algorithmic bytes of the pass launches of one step (untimed replay)
        alg_step = pass_stream_bytes(sim, x, gates, n, b)
        launches_per_step = len(gates) + 1  # the basis encode is a pass too
        alg_bytes = alg_step / launches_per_step
        achieved = alg_bytes / avg_s / 1e9
        logical = LOGICAL_BYTES_PER_AMP * (1 << n) / avg_s / 1e9
        roofline = {
            "bound": "hbm", "kernel": name,
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.workload, name),
            # share of the VALU issue capacity the pass used, from the
            # committed SQ counters (SQ_INSTS_VALU x 4 cycles over 1024
            # SIMDs x 2.4 GHz x the traced launch time), or None
            "valu_busy": measured_counters(args.workload, name).get("valu_busy"),
            "avg_launch_ms": round(tot / cnt, 4), "launches": cnt,
            "algorithmic_bytes_per_launch": int(alg_bytes),
            "algorithmic_bytes": "compressed streams in + out and per-plane metadata, "
                                 "averaged over the step's pass launches",
            "logical_gbs": round(logical, 1),
            "logical_frac": round(logical / HBM_PEAK_GBS, 4),
            "kernels_ms_one_step": split,
        }
        if not grover:
            roofline["binding"] = ("VALU issue and memory latency, not HBM bandwidth: see the "
                                   "SQ counters in profiles/pass_qft24.md")

    cpu = None
    if args.cpu_budget > 0:
        from oracle import oracle as orc
        if grover:
            cpu = cpu_baseline(A, orc, inputs, w, eb, args.cpu_budget, "Grover-36")
        else:
            cpu = cpu_baseline_gates(A, orc, inputs, w, eb, args.cpu_stride, args.shortcut,
                                     "QFT-24")

    config = {
        "workload": args.workload, "n_qubits": n, "block_log2": b,
        "segment_log2": min(b, 10), "error_bound": eb,
        "ladder": inputs.default_ladder(eb), "theta": 4.0,
        "gates_per_step": len(gates), "shortcut": args.shortcut,
        "grid": grid_used, "grid_trial_ms": grid_trials,
    }
    if grover:
        config.update({"marked": w["marked"], "iterations": k})
    else:
        config["basis"] = x
    out = {
        "metric": METRIC,
        "value": round(gates_per_s, 2),
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded basis state, generated circuit)",
        "config": config,
        # the metric's logical amplitude traffic (32 B per amplitude per gate,
        # what an uncompressed simulator moves) and its fraction of the HBM
        # peak; the HBM fraction of the bytes the pass really moves is
        # hbm_frac (the roofline's algorithmic bytes)
        "amplitude_gbs": round(amp_gbs, 1),
        "logical_frac": round(amp_gbs / HBM_PEAK_GBS, 4),
        "hbm_frac": roofline["frac"] if roofline else None,
        "fidelity": F,
        "fidelity_ok": bool(F >= 0.999),
        "min_ratio": st["min_ratio"],
        "last_ratio": st["last_ratio"],
        "peak_resident_bytes": st["peak_resident"],
        "logical_state_bytes": 16 << n,
        "level_hist": st["level_hist"],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
