"""Pins of the oracle's Sec. V shortcuts (permutation gates keep each
block's previous level; blocks a gate leaves unchanged keep their streams,
normalisation deferred into a per-block scale).  Each is checked against
something other than itself: the literal Alg. 2 run where the shortcut must
change nothing, streams rebuilt step by step from the separately pinned
block encoder, closed forms, and the exported format."""
import math
import struct

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1811_05140_amd import inputs as I

SKIP, PERM = orc.OracleSim.SC_SKIP, orc.OracleSim.SC_PERMUTE
CNOT = (0.0, 0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0)


def hdr_fields(st):
    return struct.unpack_from("<IBBBBIIdd", st, 0)


def high_gate_circuit(n, b, rng, count):
    """Random gates that include diagonal / controlled gates on qubits at or
    above b (which leave whole blocks unchanged) and mixing gates below."""
    gates = [I.h(q) for q in range(n)]
    for _ in range(count):
        k = int(rng.integers(0, 6))
        hi = int(rng.integers(b, n))
        lo = int(rng.integers(0, b))
        if k == 0:
            gates.append(I.cphase(hi, lo, rng.uniform(0, 2 * math.pi)))
        elif k == 1:
            gates.append(I.cz(hi, int(rng.integers(0, n))) if hi else I.cz(0, 1))
        elif k == 2:
            phi = rng.uniform(0, 2 * math.pi)
            gates.append(I.diag1(hi, math.cos(phi), math.sin(phi)))
        elif k == 3:
            th = rng.uniform(0, math.pi)
            c, s_ = math.cos(th), math.sin(th)
            gates.append(I.cu(hi, lo, (c, 0.0, -s_, 0.0, s_, 0.0, c, 0.0)))
        elif k == 4:
            gates.append(I.phase_flip(int(rng.integers(0, 1 << n))))
        else:
            th = rng.uniform(0, math.pi)
            c, s_ = math.cos(th), math.sin(th)
            gates.append(I.u_gate(lo, (c, 0.0, -s_, 0.0, s_, 0.0, c, 0.0)))
    return [g for g in gates if not (g[0] == I.G_CZ and g[1] == g[2])]


def test_skip_changes_nothing_when_exact():
    """Lossless ladder, normalisation off: re-encoding a block the gate left
    unchanged reproduces its stream, so skipping it must give the literal
    Alg. 2 streams bit for bit after every gate."""
    n, b = 9, 6
    gates = high_gate_circuit(n, b, np.random.default_rng(3), 40)
    a = orc.OracleSim(n, b, [0.0], 4.0, normalize=False)
    c = orc.OracleSim(n, b, [0.0], 4.0, normalize=False)
    c.set_shortcut(SKIP)
    for g in gates:
        a.apply(g)
        c.apply(g)
        assert a.export_state() == c.export_state(), g


def test_skip_hand_derived_two_blocks():
    """n = 7, b = 6, lossless, normalised.  After H(0) H(6) every amplitude of
    indices 0, 1, 64, 65 is h h.  CZ(0, 6) leaves block 0 unchanged: it keeps
    its stream and takes c_0 = fl(1 s) = s; block 1 is decoded with s, index
    65 negated, encoded.  N^2 = pairwise(fl(ns_0 fl(s s)), ns_1).  Then H(0)
    touches both blocks: block 0 decoded with fl(c_0 s'), block 1 with s'."""
    n, b = 7, 6
    sim = orc.OracleSim(n, b, [0.0], 4.0)
    sim.set_shortcut(SKIP)
    sim.run([I.h(0), I.h(6)])
    st0 = sim.stats()
    s1 = st0["scale"]
    blk0, blk1 = sim.export_block(0), sim.export_block(1)
    assert hdr_fields(blk0)[2] == 0  # no scale yet
    sim.apply(I.cz(0, 6))
    # block 0: same records, scale flag and c_0 = s1 after the header
    got0 = sim.export_block(0)
    x0 = orc.decode_block(blk0)
    x1 = orc.decode_block(blk1)
    if s1 != 1.0:
        f = hdr_fields(got0)
        assert f[2] == 1 and f[6] == len(blk0) + 8
        assert struct.unpack_from("<d", got0, 32)[0] == s1
        assert got0[32 + 8:] == blk0[32:] and got0[:5] == blk0[:5]
    else:
        assert got0 == blk0
    # block 1: decode * s1, CZ negates every index with bits 0 and 6 set
    # (the odd local indices), lossless encode
    y1 = np.array([complex(v.real * s1, v.imag * s1) for v in x1])
    y1[1::2] = -y1[1::2]
    assert sim.export_block(1) == orc.encode_block(y1, 6, 6, 0.0, 0)
    # N^2 from the weighted block norms
    ns0 = struct.unpack_from("<d", blk0, 24)[0]
    ns1 = struct.unpack_from("<d", sim.export_block(1), 24)[0]
    c2 = s1 * s1
    want_N2 = (ns0 * c2) + ns1 if s1 != 1.0 else ns0 + ns1
    st1 = sim.stats()
    assert st1["normsq"] == want_N2
    s2 = st1["scale"]
    # amplitudes read out with fl(c_0 s2) on block 0
    a = sim.amplitudes()
    fac0 = s1 * s2
    assert np.array_equal(a[:64].real, x0.real * fac0) and np.array_equal(a[:64].imag, x0.imag * fac0)
    # H(0) touches both blocks: block 0 decoded with fl(c_0 s2), c_0 back to 1
    sim.apply(I.h(0))
    h = math.sqrt(0.5)
    z = np.array([complex(v.real * fac0, v.imag * fac0) for v in x0])
    out = z.copy()
    for i in range(0, 64, 2):
        p, q = z[i], z[i + 1]
        # pair update with u = h [[1, 1], [1, -1]], one rounding per operation
        out[i] = complex((h * p.real - 0.0 * p.imag) + (h * q.real - 0.0 * q.imag),
                         (h * p.imag + 0.0 * p.real) + (h * q.imag + 0.0 * q.real))
        out[i + 1] = complex((h * p.real - 0.0 * p.imag) + (-h * q.real - 0.0 * q.imag),
                             (h * p.imag + 0.0 * p.real) + (-h * q.imag + 0.0 * q.real))
    assert sim.export_block(0) == orc.encode_block(out, 6, 6, 0.0, 0)


def test_permutation_gates_keep_previous_levels():
    """Default ladder at theta 4 on a state whose blocks sit at different
    levels (blocks with qubit 7 clear hold a uniform superposition, lossless
    and cheap; blocks with it set hold rotated, non-uniform values that need
    a lossy level): under X, SWAP and CNOT every block is compressed at the
    level its previous stream had, i.e. its stream is the encoding of the
    gated, normalised values at that level (the encoder is pinned on its
    own).  Gates that move amplitudes between the two kinds of block make
    the literal Alg. 2 choose other levels, so the rule has teeth."""
    n, b = 10, 7
    rng = np.random.default_rng(5)
    gates = [I.h(q) for q in range(8)]
    for q in range(7):
        th = rng.uniform(0.2, 1.3)
        c, s_ = math.cos(th), math.sin(th)
        gates.append(I.cu(7, q, (c, 0.0, -s_, 0.0, s_, 0.0, c, 0.0)))
        gates.append(I.cphase(7, q, rng.uniform(0, 6)))
    lad = I.default_ladder(1e-4)
    differs = 0
    for g in (I.x(7), I.x(2), I.swap(1, 7), I.cu(8, 7, CNOT), I.cu(7, 0, CNOT)):
        sim = orc.OracleSim(n, b, lad, 4.0)
        sim.set_shortcut(PERM)
        sim.run(gates)
        before = [sim.export_block(j) for j in range(1 << (n - b))]
        sc = sim.stats()["scale"]
        amps = np.concatenate([orc.decode_block(st) for st in before])
        amps = np.array([complex(v.real * sc, v.imag * sc) for v in amps]) if sc != 1.0 else amps
        gated = orc.sv_run_from(amps, n, g)
        sim.apply(g)
        for j, st in enumerate(before):
            lev = st[4]
            want = orc.encode_block(gated[j << b:(j + 1) << b], b, min(b, 10), lad[lev], lev)
            assert sim.export_block(j) == want, (g, j)
        lit = orc.OracleSim(n, b, lad, 4.0)
        lit.run(gates + [g])
        differs += sum(lit.export_block(j)[4] != before[j][4] for j in range(len(before)))
    assert len({st[4] for st in before}) > 1
    assert differs > 0


def test_near_cnot_is_not_a_permutation():
    """CU whose matrix differs from [[0, 1], [1, 0]] in one bit runs the
    ladder: with PERMUTE on it gives the same streams as with it off."""
    n, b = 10, 7
    near = list(CNOT)
    near[2] = math.nextafter(1.0, 0.0)
    gates = [I.h(q) for q in range(n)] + [I.t_gate(q) for q in range(n)]
    a = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    c = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    c.set_shortcut(PERM)
    for g in gates + [I.cu(3, 9, tuple(near))]:
        a.apply(g)
        c.apply(g)
    assert a.export_state() == c.export_state()


def test_skip_export_import_continues_identically():
    n, b = 9, 6
    gates = high_gate_circuit(n, b, np.random.default_rng(8), 30)
    gates = gates[:20] + [I.cz(6, 0)] + gates[20:]  # leaves blocks 0, 2, 4, 6 unchanged
    lad = I.default_ladder(1e-4)
    a = orc.OracleSim(n, b, lad, 4.0)
    a.set_shortcut(SKIP | PERM)
    a.run(gates[:21])
    assert a.stats()["scale"] != 1.0
    ck = a.export_state()
    flags = [ck_blk[5] for ck_blk in [a.export_block(j) for j in range(1 << (n - b))]]
    assert any(f == 1 for f in flags)  # some blocks carry a deferred scale
    r = orc.OracleSim(n, b, lad, 4.0)
    r.set_shortcut(SKIP | PERM)
    r.import_state(ck)
    assert r.export_state() == ck and r.stats()["normsq"] == a.stats()["normsq"]
    for g in gates[21:]:
        a.apply(g)
        r.apply(g)
        assert a.export_state() == r.export_state()


def test_scaled_stream_malformed_rejected():
    n, b = 7, 6
    sim = orc.OracleSim(n, b, [0.0], 4.0)
    sim.set_shortcut(SKIP)
    sim.run([I.h(0), I.h(6), I.cz(0, 6)])
    st = sim.export_block(0)
    assert st[5] == 1
    good = sim.export_state()
    fresh = orc.OracleSim(n, b, [0.0], 4.0)
    fresh.import_state(good)
    for c in (1.0, float("nan"), -0.5, 0.0, float("inf")):
        bad = bytearray(good)
        struct.pack_into("<d", bad, 32, c)
        with pytest.raises(ValueError):
            fresh.import_state(bytes(bad))
    bad = bytearray(good)
    bad[5] = 3
    with pytest.raises(ValueError):
        fresh.import_state(bytes(bad))


def test_shortcuts_keep_qft_and_grover_closed_forms():
    """With both shortcuts the QFT still meets its closed form and Grover its
    success probability (lossless ladder: only rounding separates them)."""
    n, b, x = 12, 8, 0x9C3
    sim = orc.OracleSim(n, b, [0.0], 4.0)
    sim.set_shortcut(SKIP | PERM)
    sim.set_basis(x)
    sim.run(I.qft(n))
    k = np.arange(1 << n)
    want = np.exp(2j * np.pi * x * k / (1 << n)) / math.sqrt(1 << n)
    assert np.max(np.abs(sim.amplitudes() - want)) < 1e-13
    g = orc.OracleSim(n, b, [0.0], 4.0)
    g.set_shortcut(SKIP | PERM)
    m, it = 0x5A5, 5
    g.run(I.grover(n, m, it))
    p = g.measure_probs(list(range(n)))[m]
    assert abs(p - I.grover_success(n, it)) < 1e-12
