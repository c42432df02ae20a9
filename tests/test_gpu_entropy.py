"""The entropy stage on the GPU (needs an MI355X), through the C ABI, against
the oracle's entropy stage applied to the oracle's own states:
sim_export_state_entropy equals the oracle's block entropy streams byte for
byte (QFT at every gate, random gates of every kind, Grover with long plane
runs, scaled blocks, segments of 2^7 .. 2^10, blocks of up to 2048 planes);
imports of oracle entropy checkpoints (alone and mixed with v1 streams)
continue bit for bit; malformed entropy streams are rejected with the state
unchanged.
"""
import struct
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


def pair(A, n, b, lad, theta=4.0, shortcut=0):
    # (a negative error bound would select the uncompressed path; the
    # ladder given replaces the default one)
    g = A.Sim(n, b, abs(lad[-1]) or 1e-4, ladder=lad, theta=theta)
    g.set_shortcut(shortcut)
    o = orc.OracleSim(n, b, lad, theta)
    o.set_shortcut(shortcut)
    return g, o


def test_qft_every_gate(A):
    n, b = 14, 12
    lad = I.default_ladder(1e-4)
    g, o = pair(A, n, b, lad)
    g.set_basis(0x2B7D)
    o.set_basis(0x2B7D)
    say("qft14 entropy every gate")
    assert g.export_state(entropy=True) == o.export_state(entropy=True)
    for k, gate in enumerate(I.qft(n)):
        g.apply(gate)
        o.apply(gate)
        assert g.export_state(entropy=True) == o.export_state(entropy=True), k
    g.close()


@pytest.mark.parametrize("n,b,lad,seed", [
    (12, 7, "default", 1),        # s = 7: two chunks per plane
    (12, 8, [0.0], 2),            # lossless: 64-bit residuals
    (13, 11, "default", 3),
    (14, 13, [1e-3], 4),          # a fixed bound: outliers
    (12, 10, "relative", 5),
])
def test_random_gates(A, n, b, lad, seed):
    lad = (I.default_ladder(1e-4) if lad == "default" else
           I.relative_ladder(1e-3) if lad == "relative" else lad)
    rng = np.random.default_rng(seed)
    gates = [I.h(q) for q in range(0, n, 2)]
    for _ in range(40):
        k = int(rng.integers(0, 5))
        a, c = (int(v) for v in rng.choice(n, 2, replace=False))
        if k == 0:
            gates.append(I.h(a))
        elif k == 1:
            gates.append(I.cphase(a, c, rng.uniform(0, 6.3)))
        elif k == 2:
            gates.append(I.u_gate(a, (0.6, 0.0, -0.8, 0.0, 0.8, 0.0, 0.6, 0.0)))
        elif k == 3:
            gates.append(I.swap(a, c))
        else:
            gates.append(I.t_gate(a))
    g, o = pair(A, n, b, lad)
    say("random gates entropy", n, b, lad, seed)
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        if k % 4 == 3 or k == len(gates) - 1:
            assert g.export_state(entropy=True) == o.export_state(entropy=True), k
    g.close()


@pytest.mark.parametrize("n,b", [(18, 16), (21, 20)])
def test_grover_plane_runs(A, n, b):
    m = (0x2D5B7 * 13) & ((1 << n) - 1)
    g, o = pair(A, n, b, I.default_ladder(1e-5))
    gates = I.grover(n, m, 2)
    say("grover entropy", n, b)
    g.run(gates)
    o.run(gates)
    e = g.export_state(entropy=True)
    assert e == o.export_state(entropy=True)
    v1 = g.export_state()
    assert len(e) * 10 < len(v1)
    g.close()


def test_scaled_blocks(A):
    n, b = 13, 11
    lad = I.default_ladder(1e-4)
    g, o = pair(A, n, b, lad, shortcut=3)
    gates = [I.h(q) for q in range(n)] + [I.cphase(12, 3, 0.7), I.diag1(12, 0.6, 0.8),
                                          I.cz(11, 2), I.phase_flip(77)]
    say("scaled entropy")
    for gate in gates:
        g.apply(gate)
        o.apply(gate)
        assert g.export_state(entropy=True) == o.export_state(entropy=True)
    assert any(x[5] & 1 for x in orc.split_streams(o.export_state()))
    g.close()


def test_import_entropy_checkpoints(A):
    n, b = 14, 12
    lad = I.default_ladder(1e-4)
    gates = I.qft(n)
    o = orc.OracleSim(n, b, lad, 4.0)
    o.set_basis(0x1357)
    o.run(gates[:70])
    e = o.export_state(entropy=True)
    v1 = o.export_state()
    # every other block as v1: a mixed checkpoint
    eb, vb = orc.split_streams(e), orc.split_streams(v1)
    mixed = b"".join(vb[j] if j % 2 else eb[j] for j in range(len(eb)))
    say("import entropy checkpoints")
    for data in (e, mixed):
        g = A.Sim(n, b, 1e-4)
        g.import_state(data)
        assert g.export_state() == v1
        assert g.stats()["normsq"] == o.stats()["normsq"]
        r = orc.OracleSim(n, b, lad, 4.0)
        r.import_state(v1)
        for gate in gates[70:]:
            g.apply(gate)
            r.apply(gate)
        assert g.export_state() == r.export_state()
        g.close()


def test_malformed_entropy_streams_rejected(A):
    n, b = 14, 12
    o = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    o.set_basis(0x1357)
    o.run(I.qft(n)[:70])
    blocks = orc.split_streams(o.export_state(entropy=True))
    j = max(range(len(blocks)), key=lambda i: len(blocks[i]))
    e = blocks[j]
    ni = struct.unpack_from("<I", e, 36)[0]
    tags = list(struct.unpack_from("<%dI" % ni, e, 40))
    lit = next(i for i, t in enumerate(tags) if not t & 0xC0000000)
    body = 40 + (4 * ni + 7) // 8 * 8 + sum(t & 0x3FFFFFFF for t in tags[:lit]
                                            if not t & 0x80000000)
    pw = struct.unpack_from("<I", e, body + 8)[0]
    cases = []

    def mut(name, f):
        x = bytearray(e)
        f(x)
        cases.append((name, bytes(x)))

    mut("run at plane 0", lambda x: struct.pack_into("<I", x, 40, 0x80000001))
    mut("body length", lambda x: struct.pack_into("<I", x, 40 + 4 * lit, tags[lit] + 8))
    mut("payload words", lambda x: struct.pack_into("<I", x, body + 8, pw + 1))
    mut("reserved word", lambda x: struct.pack_into("<I", x, body + 20, 1))
    mut("mode byte", lambda x: x.__setitem__(body + 24, 200))
    mut("item count", lambda x: struct.pack_into("<I", x, 36, ni + 1))
    mut("v1 length", lambda x: struct.pack_into("<I", x, 32,
                                                struct.unpack_from("<I", e, 32)[0] + 8))
    nlen = sum(1 for m in e[body + 24:body + 40] if m < 128)
    code_at = body + 40 + (2 * nlen + 7) // 8 * 8
    mut("code bit", lambda x: x.__setitem__(code_at, x[code_at] ^ 1))
    g = A.Sim(n, b, 1e-4)
    g.set_basis(5)
    before = g.export_state()
    for name, bad in cases:
        say("malformed:", name)
        data = b"".join(bad if i == j else blocks[i] for i in range(len(blocks)))
        r = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
        with pytest.raises(ValueError):
            r.import_state(data)
        with pytest.raises(A.SimError):
            g.import_state(data)
        assert g.export_state() == before, name
    g.close()
