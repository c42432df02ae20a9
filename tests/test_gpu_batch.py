"""Batched passes on the GPU: several states of different sizes, block sizes
and ladders advanced by shared kernel launches, directly or as replays of a
captured HIP graph.  Every state's block streams must equal those of the same
state run alone through sim_apply_gate, byte for byte, after every call (so
every graph replay is checked against the eager result, with synchronising
queries between replays), and the oracle's for the smaller states.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1811_05140_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    from paper_1811_05140_amd import aalcsim
    return aalcsim


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def unitary(rng):
    a = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    q, r = np.linalg.qr(a)
    q = q * (np.diag(r) / np.abs(np.diag(r)))
    return tuple(float(v) for z in q.reshape(-1) for v in (z.real, z.imag))


def circuit(n, count, rng):
    gates = []
    for _ in range(count):
        k = int(rng.integers(1, 10))
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        if k == I.G_U:
            gates.append(I.u_gate(a, unitary(rng)))
        elif k == I.G_DIAG1:
            phi = rng.uniform(0, 2 * math.pi)
            gates.append(I.diag1(a, math.cos(phi), math.sin(phi)))
        elif k == I.G_CU:
            gates.append(I.cu(a, b, unitary(rng)))
        elif k == I.G_CPHASE:
            gates.append(I.cphase(a, b, rng.uniform(0, 2 * math.pi)))
        elif k == I.G_CZ:
            gates.append(I.cz(a, b))
        elif k == I.G_SWAP:
            gates.append(I.swap(a, b))
        elif k == I.G_X:
            gates.append(I.x(a))
        elif k == I.G_PHASE_FLIP:
            gates.append(I.phase_flip(int(rng.integers(0, 1 << n))))
        else:
            gates.append(I.diffuse())
    return gates


# (n, block_log2, ladder, basis)
SPECS = [
    (10, 8, I.default_ladder(1e-4), 0x2F1),
    (12, 6, I.default_ladder(1e-3), 0x9A7),
    (13, 10, [1e-4], 0x1234),
    (11, 11, [0.0], 0x3),
    (14, 12, I.default_ladder(1e-5), 0x2ACE),
    (16, 12, I.default_ladder(1e-4), 0xBEEF),
    (9, 6, [1e-6, 1e-3], 0x1FF),
]


def make(A, spec):
    n, b, lad, x = spec
    s = A.Sim(n, b, lad[-1], ladder=lad, theta=4.0)
    s.set_basis(x)
    return s


def streams(sim, n, b):
    return [sim.export_block(j) for j in range(1 << (n - b))]


def test_batch_matches_alone_and_oracle(A):
    rng = np.random.default_rng(11)
    circs = [circuit(n, int(rng.integers(20, 41)), rng) for n, _, _, _ in SPECS]
    say("batch of %d states, %s gates" % (len(SPECS), [len(c) for c in circs]))
    batched = [make(A, sp) for sp in SPECS]
    alone = [make(A, sp) for sp in SPECS]
    orcs = {k: orc.OracleSim(SPECS[k][0], SPECS[k][1], SPECS[k][2], 4.0) for k in (0, 2, 6)}
    for k, o in orcs.items():
        o.set_basis(SPECS[k][3])
    batch = A.Batch(len(SPECS), 8)
    pos = [0] * len(SPECS)
    call = 0
    while any(pos[k] < len(circs[k]) for k in range(len(SPECS))):
        # each call: 8 passes; some states sit out some passes
        passes = []
        for p in range(8):
            row = []
            for k in range(len(SPECS)):
                idle = (k + p + call) % 5 == 0
                if pos[k] < len(circs[k]) and not idle:
                    g = circs[k][pos[k]]
                    pos[k] += 1
                    alone[k].apply(g)
                    if k in orcs:
                        orcs[k].apply(g)
                    row.append(g)
                else:
                    row.append(None)
            passes.append(row)
        use_graph = call % 3 != 0
        say("call %d graph %d" % (call, use_graph))
        batch.apply(batched, passes, use_graph=use_graph)
        for k, (n, b, _, _) in enumerate(SPECS):
            assert streams(batched[k], n, b) == streams(alone[k], n, b), (call, k)
            sb, sa = batched[k].stats(), alone[k].stats()
            for key in ("normsq", "scale", "level_hist", "passes", "resident_bytes",
                        "min_ratio", "replays", "escalations"):
                assert sb[key] == sa[key], (call, k, key)
        call += 1
    for k, o in orcs.items():
        n, b = SPECS[k][0], SPECS[k][1]
        assert streams(batched[k], n, b) == [o.export_block(j) for j in range(1 << (n - b))]
    info = batch.info()
    say("graph info", info)
    # passes holding a diffusion are part of the graph's shape, so these random
    # circuits capture a graph per graph call; reuse is checked with layers below
    assert info["graph_launches"] == sum(1 for c in range(call) if c % 3 != 0)
    assert 1 <= info["graph_builds"] <= info["graph_launches"]
    batch.close()


def test_batch_rejects_bad_calls_and_queues_nothing(A):
    say("batch validation")
    a = make(A, SPECS[0])
    b = make(A, SPECS[1])
    u = A.Sim(10, 8, -1.0)
    ref = streams(a, 10, 8)
    batch = A.Batch(4, 4)
    with pytest.raises(A.SimError) as e:
        batch.apply([a, a], [[I.h(0), I.h(1)]])
    assert e.value.code == A.SIM_EINVAL
    with pytest.raises(A.SimError) as e:
        batch.apply([a, u], [[I.h(0), I.h(1)]])
    assert e.value.code == A.SIM_EUNSUPPORTED
    with pytest.raises(A.SimError) as e:
        # valid first pass, invalid gate (qubit 12 of a 12-qubit state) later
        batch.apply([a, b], [[I.h(0), I.h(1)], [I.h(2), I.h(12)]])
    assert e.value.code == A.SIM_EINVAL
    with pytest.raises(A.SimError):
        batch.apply([a, b], [[I.h(0), I.h(1)]] * 5)  # more passes than the batch holds
    assert streams(a, 10, 8) == ref and a.stats()["passes"] == 0
    batch.close()


def test_random_brick_layers_batched_with_graphs(A):
    # small instances of the batched random-circuit workload, one graph
    # launch per layer, against the same circuits run alone
    rng = I.rng_for(40)
    insts = []
    for i in range(6):
        n = 12 + rng.next() % 5
        insts.append((n, I.random_brick_layers(n, 6, rng)))
    say("brick layers", [n for n, _ in insts])
    sims = [A.Sim(n, min(n, 10), 1e-4) for n, _ in insts]
    solo = [A.Sim(n, min(n, 10), 1e-4) for n, _ in insts]
    batch = A.Batch(len(insts), 32)
    for layer in range(6):
        gl = [layers[layer] for _, layers in insts]
        P = max(len(g) for g in gl)
        passes = [[g[p] if p < len(g) else None for g in gl] for p in range(P)]
        batch.apply(sims, passes, use_graph=True)
        for k, g in enumerate(gl):
            solo[k].run(g)
        for k, (n, _) in enumerate(insts):
            b = min(n, 10)
            assert streams(sims[k], n, b) == streams(solo[k], n, b), (layer, k)
    info = batch.info()
    say("graph info", info)
    # even and odd layers differ only in their CZ pairs: two shapes at most
    assert info["graph_launches"] == 6 and info["graph_builds"] <= 2
    batch.close()
