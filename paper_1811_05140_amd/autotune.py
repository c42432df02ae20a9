"""Autotuner for the block size and launch shape of the per-gate pass.

For each (n, ladder, theta) it times a calibration circuit -- seeded random
brick layers at that n applied to a seeded basis state -- for every
block_log2 in [12, min(20, n)] and every grid cap in GRIDS, and keeps the
fastest configuration (gates/s; ties go to the smaller resident state).  The
table is written to JSON before a run and only read during it ("frozen").
The block size is the AALC decision unit (Alg. 2 decides per stride), so it
changes the compressed result: the chosen b is recorded with every result
and is what the oracle must be given to reproduce it.  The grid cap changes
only the launch shape, never a result.

    python -m paper_1811_05140_amd.autotune --n 16-28 --error-bound 1e-4 \\
        --out paper_1811_05140_amd/tune_table.json
"""
import argparse
import json
import os
import sys
import time

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_1811_05140_amd import inputs

B_RANGE = (12, 20)
GRIDS = (1024, 2048, 3072, 4096, 8192)
TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json")


def key(n, ladder, theta):
    return "n=%d ladder=%s theta=%r" % (n, ",".join(repr(float(d)) for d in ladder),
                                         float(theta))


def candidates(n, b_range=B_RANGE, grids=GRIDS):
    """(b, grid) pairs searched at n: b in [lo, min(hi, n)], at least one b."""
    lo, hi = b_range
    hi = min(hi, n)
    lo = min(lo, hi)
    return [(b, g) for b in range(lo, hi + 1) for g in grids]


def pick(results):
    """Fastest result; equal speed goes to the smaller resident state, then to
    the smaller b and grid (deterministic)."""
    if not results:
        raise ValueError("no calibration results")
    return max(results, key=lambda r: (r["gates_per_s"], -r["resident_bytes"], -r["b"],
                                       -r["grid"]))


def calibration_circuit(n, layers=2):
    """Seeded brick layers and basis state used to time a configuration."""
    rng = inputs.rng_for(100 + n)
    gates = [g for layer in inputs.random_brick_layers(n, layers, rng) for g in layer]
    x = rng.next() & ((1 << n) - 1)
    return x, gates


def gpu_measure(A, n, ladder, theta, layers=2, reps=2):
    """Return measure(b, grid) -> (gates/s, resident bytes) timing the
    calibration circuit on the GPU (best of `reps`)."""
    x, gates = calibration_circuit(n, layers)
    cache = {}

    def measure(b, grid):
        sim = cache.get(b)
        if sim is None:
            for old in cache.values():
                old.close()
            cache.clear()
            # arenas of 1.3 x the raw state (the default caps at 8 GiB, which
            # a dense state of 29 or more qubits can outgrow)
            sim = A.Sim(n, b, ladder[-1], ladder=list(ladder), theta=theta,
                        arena_bytes=int(1.3 * (16 << n)) + (1 << 20))
            cache[b] = sim
        sim.set_grid(grid)
        best = None
        for _ in range(reps):
            sim.set_basis(x)
            sim.sync()
            t0 = time.perf_counter()
            sim.run(gates)
            sim.sync()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return len(gates) / best, sim.stats()["resident_bytes"]

    def close():
        for s in cache.values():
            s.close()
        cache.clear()

    measure.close = close
    return measure


def tune(n, ladder, theta, measure, b_range=B_RANGE, grids=GRIDS, progress=None):
    results = []
    for b, g in candidates(n, b_range, grids):
        gps, res = measure(b, g)
        results.append({"b": b, "grid": g, "gates_per_s": gps, "resident_bytes": res})
        if progress:
            progress("n=%d b=%d grid=%d: %.1f gates/s" % (n, b, g, gps))
    best = pick(results)
    return {"b": best["b"], "grid": best["grid"], "gates_per_s": best["gates_per_s"],
            "candidates": results}


def save_table(entries, path, meta=None):
    doc = {"format": "aalcsim tune table v1", "meta": meta or {}, "entries": entries}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load_table(path=TABLE_PATH):
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        doc = json.load(f)
    if doc.get("format") != "aalcsim tune table v1":
        raise ValueError("%s is not a tune table" % path)
    return doc["entries"]


def lookup(entries, n, ladder, theta):
    """(b, grid) for this configuration, or None when it was not tuned."""
    e = entries.get(key(n, ladder, theta))
    return None if e is None else (int(e["b"]), int(e["grid"]))


def main():
    ap = argparse.ArgumentParser(description="tune block_log2 and grid per n")
    ap.add_argument("--n", default="16-28", help="qubit counts, e.g. 16-28 or 18,20")
    ap.add_argument("--error-bound", type=float, default=1e-4)
    ap.add_argument("--theta", type=float, default=4.0)
    ap.add_argument("--layers", type=int, default=2)
    ap.add_argument("--out", default=TABLE_PATH)
    args = ap.parse_args()
    if "-" in args.n:
        lo, hi = (int(v) for v in args.n.split("-"))
        ns = list(range(lo, hi + 1))
    else:
        ns = [int(v) for v in args.n.split(",")]
    from paper_1811_05140_amd import aalcsim as A
    ladder = inputs.default_ladder(args.error_bound)
    entries = load_table(args.out)
    for n in ns:
        m = gpu_measure(A, n, ladder, args.theta, layers=args.layers)
        e = tune(n, ladder, args.theta, m,
                 progress=lambda t: print(t, file=sys.stderr, flush=True))
        m.close()
        entries[key(n, ladder, args.theta)] = e
        print("n=%d: b=%d grid=%d %.1f gates/s" % (n, e["b"], e["grid"], e["gates_per_s"]),
              flush=True)
    save_table(entries, args.out, {"calibration": "%d random brick layers per n, seeded"
                                   % args.layers, "grids": list(GRIDS),
                                   "b_range": list(B_RANGE)})


if __name__ == "__main__":
    main()
