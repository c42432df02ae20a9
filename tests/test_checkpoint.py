"""Checkpoint and resume on the oracle (CPU): whole-state export of the block
streams and import of them into another simulator.

Pins (none re-uses the import code under test as its own reference):
  * the streams written by a pass are the whole state: importing them and
    running the rest of a circuit gives exactly the streams of the
    uninterrupted run, at every remaining gate;
  * an imported state built from independently encoded blocks (the golden
    pinned encoder) has N^2 equal to the pairwise sum of their normsq fields
    and amplitudes fl(xhat * s), s = 1/sqrt(N^2), checked against numpy;
  * every malformed or mismatched stream is rejected and leaves the state
    unchanged.
"""
import math
import struct

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1811_05140_amd import inputs as I


def qft12_half(cut=40):
    w = I.qft12_workload()
    o = orc.OracleSim(w["n"], w["b"], I.default_ladder(1e-4), 4.0)
    o.set_basis(w["basis"])
    o.run(w["gates"][:cut])
    return w, o


def records(stream):
    """(offset, anchor, payload words, outliers) of each plane record."""
    s, b = stream[6], stream[7]
    C = 1 << (s - 6)
    padC = (C + 7) // 8 * 8
    pos, out = 32, []
    for _ in range(2 << (b - s)):
        anc, pw, no = struct.unpack_from("<qII", stream, pos)
        out.append((pos, anc, pw, no))
        pos += 16 + (padC if pw else 0) + 8 * pw + 16 * no
    assert pos == len(stream)
    return out


def test_resume_equals_uninterrupted_run():
    w, o = qft12_half(40)
    ck = o.export_state()
    assert len(ck) == o.stats()["resident_bytes"]
    r = orc.OracleSim(w["n"], w["b"], I.default_ladder(1e-4), 4.0)
    assert r.import_state(ck) == 0
    assert r.export_state() == ck
    so, sr = o.stats(), r.stats()
    assert so["normsq"] == sr["normsq"] and so["scale"] == sr["scale"]
    assert sr["passes"] == 0 and sr["min_ratio"] == sr["last_ratio"]
    for k, g in enumerate(w["gates"][40:]):
        o.apply(g)
        r.apply(g)
        assert o.export_state() == r.export_state(), "gate %d after resume" % (40 + k)
    assert np.array_equal(o.amplitudes().view(np.uint64), r.amplitudes().view(np.uint64))


def test_resume_at_every_cut_matches_closed_form_qft():
    """Resuming at any gate leaves the QFT result within its error budget
    (fidelity to the closed form 2^-n/2 e^(2 pi i x k / 2^n) above 0.999)."""
    w = I.qft12_workload()
    n = w["n"]
    k = np.arange(1 << n)
    want = np.exp(2j * math.pi * w["basis"] * k / (1 << n)) / math.sqrt(1 << n)
    for cut in (0, 1, 17, 60, len(w["gates"])):
        _, o = qft12_half(cut)
        r = orc.OracleSim(n, w["b"], I.default_ladder(1e-4), 4.0)
        r.import_state(o.export_state())
        r.run(w["gates"][cut:])
        a = r.amplitudes()
        F = abs(np.vdot(want, a)) ** 2 / np.vdot(a, a).real
        assert F > 0.999, (cut, F)


def test_import_of_independently_encoded_blocks():
    """Blocks encoded one by one (or_encode_block, pinned by the golden
    streams) and concatenated form a state whose N^2 is the pairwise sum of
    their normsq fields and whose amplitudes are fl(xhat * s)."""
    n, b = 8, 6
    rng = np.random.default_rng(7)
    ladder = [0.0, 1e-3]
    x = rng.normal(size=2 << n) * 0.05
    streams, xh = [], []
    for j in range(1 << (n - b)):
        blk = x[2 * (j << b): 2 * ((j + 1) << b)]
        lev = j % 2
        st = orc.encode_block(blk, b, b, ladder[lev], lev)
        streams.append(st)
        xh.append(orc.decode_block(st))
    r = orc.OracleSim(n, b, ladder, 4.0)
    r.import_state(b"".join(streams))
    norms = np.array([struct.unpack_from("<d", st, 24)[0] for st in streams])
    N2 = orc.pairwise(norms)
    s = 1.0 / math.sqrt(N2)
    st = r.stats()
    assert st["normsq"] == N2 and st["scale"] == s
    want = np.concatenate(xh) * s
    got = r.amplitudes()
    assert np.array_equal(got.view(np.uint64), want.astype(np.complex128).view(np.uint64))


def test_import_all_zero_state_is_collapsed():
    n, b = 7, 6
    z = np.zeros(2 << b)
    st = orc.encode_block(z, b, b, 0.0, 0)
    r = orc.OracleSim(n, b, [0.0], 4.0)
    assert r.import_state(st + st) == -5
    s = r.stats()
    assert s["collapsed"] == 1 and s["scale"] == 1.0 and s["normsq"] == 0.0


def corruptions(ck, nblocks):
    """(name, bytes) pairs, each one defect in an otherwise valid checkpoint."""
    first_len = struct.unpack_from("<I", ck, 12)[0]
    s0 = ck[:first_len]
    recs = records(s0)
    out = []

    def put(name, off, fmt, val):
        b = bytearray(ck)
        struct.pack_into(fmt, b, off, val)
        out.append((name, bytes(b)))

    put("magic", 0, "<I", 0x12345678)
    put("level beyond the ladder", 4, "<B", 7)
    put("delta not the level's bound", 16, "<d", 3e-4)
    put("segment size", 6, "<B", s0[6] - 1)
    put("length too long", 12, "<I", first_len + 8)
    put("length not a multiple of 8", 12, "<I", first_len - 4)
    put("normsq", 24, "<d", struct.unpack_from("<d", ck, 24)[0] * (1 + 2 ** -50))
    put("outlier count in header", 8, "<I", struct.unpack_from("<I", ck, 8)[0] + 1)
    out.append(("truncated", ck[:-8]))
    out.append(("trailing bytes", ck + bytes(8)))
    withpay = [r for r in recs if r[2] > 0]
    if withpay:
        pos, anc, pw, no = withpay[0]
        w0 = s0[pos + 16]
        put("width byte", pos + 16, "<B", w0 + 1)
        put("payload words", pos + 8, "<I", pw + 1)
        lossy = struct.unpack_from("<d", ck, 16)[0] != 0.0
        if lossy:
            put("lossy anchor beyond 2^30 - 1", pos, "<q", 1 << 30)
    return out


def test_corrupted_checkpoints_rejected_state_unchanged():
    w, o = qft12_half(70)
    ck = o.export_state()
    nb = 1 << (w["n"] - w["b"])
    cases = corruptions(ck, nb)
    assert len(cases) >= 11
    _, r = qft12_half(10)
    before = r.export_state()
    for name, bad in cases:
        with pytest.raises(ValueError):
            r.import_state(bad)
        assert r.export_state() == before, name
    # a different ladder: the streams' bounds are not its levels
    r2 = orc.OracleSim(w["n"], w["b"], I.default_ladder(1e-3), 4.0)
    with pytest.raises(ValueError):
        r2.import_state(ck)
    # a different block size
    r3 = orc.OracleSim(w["n"], w["b"] + 1, I.default_ladder(1e-4), 4.0)
    with pytest.raises(ValueError):
        r3.import_state(ck)


def test_record_level_defects_rejected():
    """Defects inside plane records that only a record check finds: a first
    residual that is not 0, an outlier index outside the plane or out of
    order, an outlier in a lossless plane, a lossy chunk wider than 32."""
    b = 6
    # lossy plane with two outliers and a nonzero payload
    x = np.zeros(2 << b)
    x[0::2][:10] = [0.0, 0.2, 0.5, 0.7, 1.0, -0.2, -0.6, 3.0, 0.75, 1e12]
    st = orc.encode_block(x, b, b, 0.25, 0)
    (pos, anc, pw, no), _ = records(st)
    assert pw == 4 and no == 2
    pay = pos + 16 + 8
    outl = pay + 8 * pw

    def bad(off, fmt, val):
        s = bytearray(st)
        struct.pack_into(fmt, s, off, val)
        return bytes(s)

    r = orc.OracleSim(b, b, [0.25], 4.0)
    r.import_state(st)  # the valid stream is accepted
    cases = [
        bad(pay, "<Q", struct.unpack_from("<Q", st, pay)[0] | 1),   # c_0 != 0
        bad(outl, "<I", 64),                                         # index outside
        bad(outl + 16, "<I", 0),                                     # not ascending
    ]
    # chunk 0 widened to 33 bits (29 zero words appended to its payload, so
    # every size still adds up)
    wide = bytearray(st[:outl] + bytes(8 * 29) + st[outl:])
    struct.pack_into("<B", wide, pos + 16, 33)
    struct.pack_into("<I", wide, pos + 8, 33)
    struct.pack_into("<I", wide, 12, len(wide))
    assert [rc[2] for rc in records(bytes(wide))] == [33, 0]
    cases.append(bytes(wide))
    for c in cases:
        with pytest.raises(ValueError):
            r.import_state(c)
    # a lossless plane carrying an outlier
    y = np.zeros(2 << b)
    y[2] = 1.5
    ls = orc.encode_block(y, b, b, 0.0, 0)
    rl = orc.OracleSim(b, b, [0.0], 4.0)
    rl.import_state(ls)
    (p0, a0, pw0, no0), (p1, _, _, _) = records(ls)
    assert no0 == 0
    # the re record gains one outlier (index 3) right after its payload
    s = bytearray(ls[:p1] + struct.pack("<IId", 3, 0, 2.0) + ls[p1:])
    struct.pack_into("<I", s, p0 + 12, 1)
    struct.pack_into("<I", s, 12, len(s))
    struct.pack_into("<I", s, 8, 1)
    assert [r[3] for r in records(bytes(s))] == [1, 0]
    with pytest.raises(ValueError):
        rl.import_state(bytes(s))
