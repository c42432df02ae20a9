"""Sec. V shortcuts on the GPU against the oracle with the same shortcuts
(through the C ABI): permutation gates keep each block's previous level;
blocks that a gate leaves unchanged keep their records, with the pass's
normalisation deferred into a per-block scale.  Streams (including the
scale words of kept blocks) equal the oracle's after every gate, alone and
in batched passes, through the one-unit, bulk-round and one-value kernels,
with units of one block and units spanning two blocks; queries, whole-state
export and import of scaled states agree with the oracle.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1811_05140_amd import inputs as I

pytestmark = pytest.mark.gpu

CNOT = (0.0, 0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0)


@pytest.fixture(scope="module")
def A():
    from paper_1811_05140_amd import aalcsim
    return aalcsim


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def rot(th):
    c, s_ = math.cos(th), math.sin(th)
    return (c, 0.0, -s_, 0.0, s_, 0.0, c, 0.0)


def circuit(n, b, rng, count):
    """Gates with qubits at or above b (whole blocks left unchanged),
    permutations (X, SWAP, CNOT) and mixing gates below b."""
    gates = [I.h(q) for q in range(n)]
    for _ in range(count):
        k = int(rng.integers(0, 9))
        hi = int(rng.integers(b, n)) if n > b else int(rng.integers(0, n))
        lo = int(rng.integers(0, b))
        lo = (lo + 1) % b if lo == hi else lo
        other = int(rng.integers(0, n))
        if k == 0:
            gates.append(I.cphase(hi, lo, rng.uniform(0, 2 * math.pi)))
        elif k == 1 and other != hi:
            gates.append(I.cz(hi, other))
        elif k == 2:
            phi = rng.uniform(0, 2 * math.pi)
            gates.append(I.diag1(hi, math.cos(phi), math.sin(phi)))
        elif k == 3:
            gates.append(I.cu(hi, lo, rot(rng.uniform(0, math.pi))))
        elif k == 4:
            gates.append(I.phase_flip(int(rng.integers(0, 1 << n))))
        elif k == 5:
            gates.append(I.u_gate(lo, rot(rng.uniform(0, math.pi))))
        elif k == 6:
            gates.append(I.x(int(rng.integers(0, n))))
        elif k == 7:
            a, c = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(I.swap(a, c))
        else:
            a, c = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(I.cu(a, c, CNOT))
    return gates


CASES = [
    # n, b, ladder, theta, flags, gates, seed
    (12, 8, "default", 4.0, 3, 50, 1),       # units inside one block
    (12, 10, "default", 8.0, 2, 50, 2),      # one segment per block: units over two blocks
    (11, 7, [0.0], 4.0, 2, 40, 3),
    (13, 10, "default", 16.0, 1, 50, 4),     # permutation shortcut alone
    (14, 12, "default", 4.0, 3, 40, 5),
    (10, 10, [1e-5], 1.0, 3, 30, 6),         # a single block
]


@pytest.mark.parametrize("n,b,lad,theta,flags,ng,seed", CASES)
def test_shortcuts_streams_every_gate(A, n, b, lad, theta, flags, ng, seed):
    lad = I.default_ladder(1e-4) if lad == "default" else lad
    gates = circuit(n, b, np.random.default_rng(seed), ng)
    say("shortcuts", n, b, lad, theta, flags, len(gates))
    g = A.Sim(n, b, lad[-1], ladder=lad, theta=theta)
    g.set_shortcut(flags)
    o = orc.OracleSim(n, b, lad, theta)
    o.set_shortcut(flags)
    scaled = 0
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        st = o.export_state()
        assert g.export_state() == st, "gate %d %s" % (k, gate[:3])
        scaled += sum(o.export_block(j)[5] for j in range(1 << (n - b)))
    sg, so = g.stats(), o.stats()
    assert sg["level_hist"] == so["level_hist"]
    assert sg["normsq"] == so["normsq"] and sg["scale"] == so["scale"]
    assert sg["resident_bytes"] == so["resident_bytes"]
    full = o.amplitudes()
    assert np.array_equal(g.amplitudes().view(np.uint64), full.view(np.uint64))
    qs = [n - 1, 0, n // 2]
    assert np.max(np.abs(g.probs(qs) - o.measure_probs(qs))) < 1e-12
    if flags & 2 and n > b:
        assert scaled > 0  # blocks with a deferred scale occurred
    g.close()


def test_shortcuts_batched_with_graphs(A):
    specs = [(12, 8, I.default_ladder(1e-4), 3, 11), (12, 10, I.default_ladder(1e-3), 2, 12),
             (11, 7, [0.0], 3, 13), (13, 9, I.default_ladder(1e-5), 0, 14)]
    circs = [circuit(n, b, np.random.default_rng(seed), 30) for n, b, _, _, seed in specs]
    say("batched shortcuts", [(n, b, f) for n, b, _, f, _ in specs])
    sims, orcs = [], []
    for n, b, lad, flags, _ in specs:
        g = A.Sim(n, b, lad[-1], ladder=lad, theta=4.0)
        g.set_shortcut(flags)
        o = orc.OracleSim(n, b, lad, 4.0)
        o.set_shortcut(flags)
        sims.append(g)
        orcs.append(o)
    batch = A.Batch(len(specs), 4)
    P = max(len(c) for c in circs)
    for start in range(0, P, 4):
        passes = []
        for p in range(start, min(start + 4, P)):
            row = [c[p] if p < len(c) else None for c in circs]
            for k, gate in enumerate(row):
                if gate is not None:
                    orcs[k].apply(gate)
            passes.append(row)
        batch.apply(sims, passes, use_graph=(start // 4) % 2 == 1)
        for k in range(len(specs)):
            assert sims[k].export_state() == orcs[k].export_state(), (start, k)
    batch.close()


def test_grover_phase_flip_skips_and_bulk_rounds(A):
    """Grover with the skip shortcut: PHASE_FLIP keeps every block but one
    (the one-value pass kernel; at grid 64 the same kernel looping over 128
    units, and the bulk-round kernel over 1024 units)."""
    for n, b, grid in ((14, 8, 0), (18, 12, 64), (21, 13, 64)):
        m = (0x2D5B7 * 7) & ((1 << n) - 1)
        gates = I.grover(n, m, 3)
        say("grover skip", n, b, grid)
        g = A.Sim(n, b, 1e-5)
        if grid:
            g.set_grid(grid)
        g.set_shortcut(3)
        o = orc.OracleSim(n, b, I.default_ladder(1e-5), 4.0)
        o.set_shortcut(3)
        for k, gate in enumerate(gates):
            g.apply(gate)
            o.apply(gate)
            if k >= n - 1:
                assert g.export_state() == o.export_state(), (n, k, gate[0])
        assert g.amplitude_sum() == complex(*orc_sum(o))
        g.close()


def orc_sum(o):
    s = o.amplitude_sum()
    return s.real, s.imag


def test_scaled_checkpoints_round_trip(A):
    n, b = 12, 8
    gates = circuit(n, b, np.random.default_rng(21), 40)
    lad = I.default_ladder(1e-4)
    o = orc.OracleSim(n, b, lad, 4.0)
    o.set_shortcut(3)
    g = A.Sim(n, b, 1e-4)
    g.set_shortcut(3)
    cut = None
    for k, gate in enumerate(gates):
        o.apply(gate)
        g.apply(gate)
        if cut is None and k > n and any(o.export_block(j)[5] for j in range(16)):
            cut = k
            break
    assert cut is not None
    ck = o.export_state()
    ck_blocks = [o.export_block(j) for j in range(16)]
    assert g.export_state() == ck
    r = A.Sim(n, b, 1e-4)
    r.set_shortcut(3)
    r.import_state(ck)  # the oracle's checkpoint, with scale words
    assert r.export_state() == ck
    assert r.stats()["normsq"] == o.stats()["normsq"]
    for gate in gates[cut + 1:]:
        o.apply(gate)
        r.apply(gate)
        assert r.export_state() == o.export_state()
    # a malformed scale word is rejected with the state unchanged
    import struct
    j = next(j for j in range(16) if ck_blocks[j][5])
    off = sum(len(ck_blocks[i]) for i in range(j))
    for c in (1.0, -0.5, float("nan")):
        bad = bytearray(ck)
        struct.pack_into("<d", bad, off + 32, c)
        before = r.export_state()
        with pytest.raises(A.SimError):
            r.import_state(bytes(bad))
        assert r.export_state() == before
