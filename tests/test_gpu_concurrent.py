"""Sims on their own streams run their passes at the same time (the pass
kernels of every sim on a GPU share one staging buffer, indexed by the
hardware slot of each wave): every state equals the oracle's, stream for
stream, whatever the other sims run beside it."""
import sys

import pytest

from oracle import oracle as orc
from paper_1811_05140_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def test_sims_on_separate_streams_overlap():
    from paper_1811_05140_amd import aalcsim as A
    rng = I.rng_for(41)
    specs = [(15, 10), (16, 12), (14, 7), (17, 13)]
    sims, oracles, circuits = [], [], []
    for k, (n, b) in enumerate(specs):
        layers = I.random_brick_layers(n, 4, rng)
        gates = [g for layer in layers for g in layer]
        if k == 1:
            gates = I.qft(n)[:60]
        circuits.append(gates)
        sims.append(A.Sim(n, b, 1e-4))           # each creates and owns its stream
        oracles.append(orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0))
    basis = [0, 0x5A5A, 0, 0]
    for sm, o, x in zip(sims, oracles, basis):
        sm.set_basis(x)
        o.set_basis(x)
    say("concurrent sims", specs, [len(g) for g in circuits])
    # enqueue gate by gate across the sims without synchronising: their
    # passes run side by side on the GPU
    for i in range(max(len(g) for g in circuits)):
        for sm, gates in zip(sims, circuits):
            if i < len(gates):
                sm.apply(gates[i])
    for o, gates in zip(oracles, circuits):
        o.run(gates)
    for k, (sm, o) in enumerate(zip(sims, oracles)):
        assert sm.export_state() == o.export_state(), k
        assert sm.stats()["normsq"] == o.stats()["normsq"], k
        sm.close()


def test_batch_beside_single_sims():
    """A batch on its own stream and single sims on theirs, enqueued in
    turn: every state equals the oracle's."""
    from paper_1811_05140_amd import aalcsim as A
    rng = I.rng_for(42)
    bspecs = [(13, 9), (14, 10), (12, 12)]
    sspecs = [(15, 11), (16, 10)]
    blayers = [I.random_brick_layers(n, 5, rng) for n, _ in bspecs]
    slayers = [I.random_brick_layers(n, 5, rng) for n, _ in sspecs]
    bsims = [A.Sim(n, b, 1e-4) for n, b in bspecs]
    ssims = [A.Sim(n, b, 1e-4) for n, b in sspecs]
    for sm in bsims + ssims:
        sm.set_basis(0)
    batch = A.Batch(len(bsims), 1)
    say("batch beside single sims", bspecs, sspecs)
    for layer in range(5):
        # the batch takes one gate per state per call (a pass each)
        for i in range(max(len(L[layer]) for L in blayers)):
            batch.apply(bsims, [[L[layer][i] if i < len(L[layer]) else None for L in blayers]])
            for sm, L in zip(ssims, slayers):
                if i < len(L[layer]):
                    sm.apply(L[layer][i])
        for sm, L in zip(ssims, slayers):
            for g in L[layer][max(len(L2[layer]) for L2 in blayers):]:
                sm.apply(g)
    batch.sync()
    for (n, b), L, sm in list(zip(bspecs, blayers, bsims)) + list(zip(sspecs, slayers, ssims)):
        o = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
        o.set_basis(0)
        for layer in L:
            o.run(layer)
        assert sm.export_state() == o.export_state(), (n, b)
        sm.close()
    batch.close()
