"""Pointwise-relative ladder levels on the GPU against the oracle (through
the C ABI): streams after every gate for random gates of every kind, the
QFT that an absolute bound of the same size collapses, Grover's one-value
planes, batched passes, wide magnitudes from a non-unitary gate without
normalisation, and checkpoints in both directions."""
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


def random_gates(n, count, rng):
    gates = []
    for _ in range(count):
        k = int(rng.integers(1, 10))
        a, c = (int(v) for v in rng.choice(n, 2, replace=False))
        if k == I.G_U:
            gates.append(I.u_gate(a, unitary(rng)))
        elif k == I.G_DIAG1:
            phi = rng.uniform(0, 2 * math.pi)
            gates.append(I.diag1(a, math.cos(phi), math.sin(phi)))
        elif k == I.G_CU:
            gates.append(I.cu(a, c, unitary(rng)))
        elif k == I.G_CPHASE:
            gates.append(I.cphase(a, c, rng.uniform(0, 2 * math.pi)))
        elif k == I.G_CZ:
            gates.append(I.cz(a, c))
        elif k == I.G_SWAP:
            gates.append(I.swap(a, c))
        elif k == I.G_X:
            gates.append(I.x(a))
        elif k == I.G_PHASE_FLIP:
            gates.append(I.phase_flip(int(rng.integers(0, 1 << n))))
        else:
            gates.append(I.diffuse())
    return gates


CASES = [
    # n, b, ladder, theta, gates, seed
    (12, 9, [0.0, -1e-5, -1e-4, -1e-3], 4.0, 60, 1),
    (11, 8, [-1e-3], 4.0, 50, 2),
    (13, 10, [-0.01, -0.05], 16.0, 50, 3),
    (10, 10, [0.0, -2.0 ** -19], 2.0, 40, 4),
]


@pytest.mark.parametrize("n,b,lad,theta,ng,seed", CASES)
def test_relative_levels_random_gates(A, n, b, lad, theta, ng, seed):
    rng = np.random.default_rng(seed)
    gates = [I.h(q) for q in range(n)] + random_gates(n, ng, rng)
    say("relative", n, b, lad, theta, len(gates))
    g = A.Sim(n, b, 1e-4, ladder=lad, theta=theta)
    o = orc.OracleSim(n, b, lad, theta)
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        assert g.export_state() == o.export_state(), "gate %d %s" % (k, gate[:3])
    assert g.stats()["level_hist"] == o.stats()["level_hist"]
    assert np.array_equal(g.amplitudes().view(np.uint64), o.amplitudes().view(np.uint64))
    g.close()


def test_relative_qft_does_not_collapse(A):
    n, b, x = 14, 10, 0x2B7D
    gates = I.qft(n)
    say("relative qft", n, b)
    a = A.Sim(n, b, 0.01, ladder=[0.01], theta=4.0)
    a.set_basis(x)
    a.run(gates)
    assert a.stats()["collapsed"]
    g = A.Sim(n, b, 0.01, ladder=[-0.01], theta=4.0)
    o = orc.OracleSim(n, b, [-0.01], 4.0)
    g.set_basis(x)
    o.set_basis(x)
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        assert g.export_state() == o.export_state(), k
    assert not g.stats()["collapsed"]
    assert g.fourier_fidelity(x) > 0.99
    a.close()
    g.close()


def test_relative_grover_and_batched(A):
    n, b = 14, 8
    m = 0x1A2B & ((1 << n) - 1)
    lad = I.relative_ladder(1e-3)
    gates = I.grover(n, m, 3)
    say("relative grover", n, b, lad)
    g = A.Sim(n, b, 1e-3, ladder=lad, theta=4.0)
    o = orc.OracleSim(n, b, lad, 4.0)
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        if k >= n - 1:
            assert g.export_state() == o.export_state(), k
    # batched: two relative states and one absolute one share the passes
    specs = [(12, 8, I.relative_ladder(1e-3), 5), (11, 7, [-1e-4], 6),
             (12, 9, I.default_ladder(1e-4), 7)]
    circs = [[I.h(q) for q in range(n_)] + random_gates(n_, 24, np.random.default_rng(sd))
             for n_, _, _, sd in specs]
    sims = [A.Sim(n_, b_, 1e-4, ladder=l_, theta=4.0) for n_, b_, l_, _ in specs]
    orcs = [orc.OracleSim(n_, b_, l_, 4.0) for n_, b_, l_, _ in specs]
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


def test_relative_wide_magnitudes_and_checkpoints(A):
    """Without normalisation, diagonal gates with huge and tiny factors spread
    the magnitudes over hundreds of binades (log codes far from 0); then a
    checkpoint goes GPU -> oracle and oracle -> GPU and both continue."""
    n, b = 11, 8
    lad = [0.0, -1e-5, -1e-3]
    gates = [I.h(q) for q in range(n)]
    gates += [I.diag1(3, 1e150, 0.0), I.diag1(5, 1e-200, 0.0), I.u_gate(2, unitary(np.random.default_rng(9))),
              I.diag1(9, 0.0, 1e-120), I.cz(1, 7), I.x(8)]
    say("relative wide magnitudes", n, b)
    g = A.Sim(n, b, 1e-3, ladder=lad, theta=4.0, normalize=False)
    o = orc.OracleSim(n, b, lad, 4.0, normalize=False)
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        assert g.export_state() == o.export_state(), k
    ck = g.export_state()
    r = orc.OracleSim(n, b, lad, 4.0, normalize=False)
    r.import_state(ck)
    g2 = A.Sim(n, b, 1e-3, ladder=lad, theta=4.0, normalize=False)
    g2.import_state(o.export_state())
    more = random_gates(n, 20, np.random.default_rng(10))
    for gate in more:
        g.apply(gate)
        r.apply(gate)
        g2.apply(gate)
        st = r.export_state()
        assert g.export_state() == st and g2.export_state() == st
