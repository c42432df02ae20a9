"""Pins of the oracle's entropy stage (block entropy stream v1: plane runs,
and per chunk the shortest of fixed-width, Golomb-Rice and sparse codes),
each against something other than the oracle itself: a stream derived by
hand, the chunk-code choice recomputed from its definition by brute force,
exact inversion to the v1 stream over many states, closed-form sizes, and
malformed streams.
"""
import struct

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1811_05140_amd import inputs as I


def bits_to_words(bits):
    """LSB-first bit list -> little-endian u64 words, zero-padded."""
    words = [0] * ((len(bits) + 63) // 64)
    for i, v in enumerate(bits):
        if v:
            words[i >> 6] |= 1 << (i & 63)
    return b"".join(struct.pack("<Q", w) for w in words)


def lsb(v, n):
    return [(v >> i) & 1 for i in range(n)]


def test_hand_derived_entropy_stream():
    """b = 8, s = 6 (one chunk per plane, eight planes), bound 0.5 (e = 1,
    codes = the integer values).  Segments 0 and 1 are equal, so planes 2, 3
    repeat planes 0, 1 (one run of 2); segments 2 and 3 are zero, planes 4, 5
    are verbatim 16-byte records and planes 6, 7 repeat them (run of 2).
    Plane 0: codes 0, -1, ..., -32, then -64 to the end: zigzags 0, 32 ones,
    63, zeros; width 6: fixed 384 bits, sparse 64 + 33 * 6 = 262, Rice k = 0
    64 + 32 + 63 = 159 (k = 1 also 159: the smaller k) -> Rice k = 0, 3
    words, a 64-byte body against the 72-byte v1 record.  Plane 1: a single
    1000 at index 5: residuals 1000, -1000, zigzags 2000, 1999; width 11:
    fixed 704, sparse 64 + 2 * 11 = 86, Rice at best 508 (k = 5) -> sparse,
    2 words, 56 bytes against 112."""
    b, s = 8, 6
    re = np.zeros(64)
    re[1:33] = -np.arange(1, 33)
    re[33:] = -64.0
    im = np.zeros(64)
    im[5] = 1000.0
    x = np.zeros(2 << b)
    for g in (0, 1):
        x[2 * 64 * g:2 * 64 * (g + 1):2] = re
        x[2 * 64 * g + 1:2 * 64 * (g + 1):2] = im
    v1 = orc.encode_block(x, b, s, 0.5, level=3)
    # plane 0: Rice k = 0 -- "0", 32 x "10", 63 ones and "0", 30 x "0"
    rbits = [0] + [1, 0] * 32 + [1] * 63 + [0] + [0] * 30
    assert len(rbits) == 159
    body_a = struct.pack("<qIIII", 0, 6, 0, 3, 0) + bytes([0]) + b"\0" * 7 + \
        struct.pack("<H", 159) + b"\0" * 6 + bits_to_words(rbits)
    # plane 1: sparse width 11 (mode 63 + 11) -- mask bits 5, 6; 2000, 1999
    sbits = lsb((1 << 5) | (1 << 6), 64) + lsb(2000, 11) + lsb(1999, 11)
    body_b = struct.pack("<qIIII", 0, 11, 0, 2, 0) + bytes([74]) + b"\0" * 7 + \
        struct.pack("<H", 86) + b"\0" * 6 + bits_to_words(sbits)
    zero = struct.pack("<qII", 0, 0, 0)
    assert (len(body_a), len(body_b)) == (64, 56)
    tags = struct.pack("<6I", 64, 56, 0x80000002, 0x40000010, 0x40000010, 0x80000002)
    body = body_a + body_b + zero + zero
    total = 32 + 8 + len(tags) + len(body)
    hdr = struct.pack("<I", 0x31454141) + v1[4:12] + struct.pack("<I", total) + v1[16:32]
    want = hdr + struct.pack("<II", len(v1), 6) + tags + body
    assert len(v1) == 32 + 72 + 112 + 72 + 112 + 4 * 16
    assert orc.entropy_encode(v1) == want
    assert orc.entropy_decode(want) == v1


def parse_chunks(e):
    """(mode, z list, width) of every coded chunk of an entropy stream,
    decoded here from the layout (independently of the oracle)."""
    s, b = e[6], e[7]
    C = 1 << (s - 6)
    sc = 8 if e[5] & 1 else 0
    ni = struct.unpack_from("<I", e, 36)[0]
    tags = struct.unpack_from("<%dI" % ni, e, 40 + sc)
    pos = 40 + sc + (4 * ni + 7) // 8 * 8
    out = []
    for t in tags:
        if t & 0x80000000:
            continue
        n = t & 0x3FFFFFFF
        if not t & 0x40000000:
            pw, nout = struct.unpack_from("<II", e, pos + 8)
            if pw:
                cw = struct.unpack_from("<I", e, pos + 16)[0]
                modes = e[pos + 24:pos + 24 + C]
                nl = sum(1 for m in modes if m < 128)
                lens = struct.unpack_from("<%dH" % nl, e, pos + 24 + (C + 7) // 8 * 8)
                cpos = pos + 24 + (C + 7) // 8 * 8 + (2 * nl + 7) // 8 * 8
                big = int.from_bytes(e[cpos:cpos + 8 * cw], "little")
                bp = li = 0
                for m in modes:
                    if m >= 128:
                        w = m - 128
                        z = [(big >> (bp + l * w)) & ((1 << w) - 1) for l in range(64)]
                        bp += 64 * w
                    elif m >= 64:
                        w = m - 63
                        mask = (big >> bp) & ((1 << 64) - 1)
                        q = bp + 64
                        z = []
                        for l in range(64):
                            if mask >> l & 1:
                                z.append((big >> q) & ((1 << w) - 1))
                                q += w
                            else:
                                z.append(0)
                        assert q - bp == lens[li]
                        bp = q
                        li += 1
                    else:
                        k = m
                        q = bp
                        z = []
                        for l in range(64):
                            u = 0
                            while big >> q & 1:
                                u += 1
                                q += 1
                            q += 1
                            z.append((u << k) | ((big >> q) & ((1 << k) - 1)))
                            q += k
                        assert q - bp == lens[li]
                        bp = q
                        li += 1
                        w = max(z).bit_length()
                    out.append((m, z, w))
        pos += n
    return out


def brute_mode(z, w):
    if w == 0:
        return 128
    fixed = 64 * w
    costs = [64 * (k + 1) + sum(v >> k for v in z) for k in range(w)]
    rice = min(costs)
    sparse = 64 + sum(1 for v in z if v) * w
    if fixed <= rice and fixed <= sparse:
        return 128 + w
    if rice <= sparse:
        return costs.index(rice)
    return 63 + w


def chunk_sources(rng):
    """Blocks (b = 10, s = 10) whose planes hit every chunk code: geometric
    residuals, sparse spikes, uniform noise, lossless bit patterns."""
    out = []
    for kind in range(6):
        x = np.zeros(2 << 10)
        if kind == 0:  # smooth walk: small residuals with a few large
            x[:] = np.cumsum(rng.geometric(0.4, 2048) * rng.choice([-1, 1], 2048))
            x[::97] += 5000.0
        elif kind == 1:  # sparse spikes
            idx = rng.choice(2048, 40, replace=False)
            x[idx] = rng.integers(-1000, 1000, 40)
        elif kind == 2:  # uniform noise
            x[:] = rng.integers(-2 ** 20, 2 ** 20, 2048)
        elif kind == 3:  # geometric residuals of widely varying scale
            x[:] = np.cumsum(rng.geometric(0.05, 2048))
        elif kind == 4:
            x[:] = rng.normal(size=2048)
        else:
            x[:] = rng.normal(size=2048) * 1e-3
            x[::5] = 0.0
        for delta, level in ((0.5, 2), (0.0, 0), (1e-4, 1)):
            out.append(orc.encode_block(x / (1.0 if delta != 1e-4 else 3000.0), 10, 10,
                                        delta, level))
    return out


def test_chunk_code_choice_is_the_cheapest():
    rng = np.random.default_rng(5)
    seen = set()
    for v1 in chunk_sources(rng):
        e = orc.entropy_encode(v1)
        for m, z, w in parse_chunks(e):
            assert m == brute_mode(z, w), (m, w)
            seen.add("fixed" if m >= 128 else "sparse" if m >= 64 else "rice")
        assert orc.entropy_decode(e) == v1
    assert seen == {"fixed", "sparse", "rice"}


def states():
    """v1 checkpoints of many states: QFT at several depths, random brick
    circuits, Grover, lossless, fixed-bound (outliers), relative levels,
    scaled blocks, several segment sizes."""
    out = []
    for n, b, lad, gates, basis, sc in [
            (12, 8, I.default_ladder(1e-4), I.qft(12)[:30], 0x5A5, 0),
            (12, 8, I.default_ladder(1e-4), I.qft(12), 0x5A5, 0),
            (13, 11, I.default_ladder(1e-3), I.qft(13)[:60], 0x123, 0),
            (13, 7, [0.0], I.qft(13)[:40], 0x777, 0),
            (14, 12, [1e-3], I.qft(14), 0x2B7D, 0),      # fixed bound: outliers
            (12, 9, I.relative_ladder(1e-3), I.qft(12), 0x3, 0),
            (14, 12, I.default_ladder(1e-5), I.grover(14, 0x1F2E, 3), 0, 3),
            (14, 13, I.default_ladder(1e-4), I.random_brick(14, 6, I.rng_for(9)), 0, 0),
            (12, 8, I.default_ladder(1e-4), I.random_brick(12, 8, I.rng_for(8)), 0, 3)]:
        o = orc.OracleSim(n, b, lad, 4.0)
        o.set_shortcut(sc)
        o.set_basis(basis)
        o.run(gates)
        out.append(o.export_state())
    return out


def test_entropy_stage_inverts_exactly():
    scaled = 0
    for data in states():
        blocks = orc.split_streams(data)
        e = orc.entropy_state(data)
        assert orc.plain_state(e) == data
        for v1, eb in zip(blocks, orc.split_streams(e)):
            s, b = v1[6], v1[7]
            P = 2 << (b - s)
            assert eb[4:12] == v1[4:12] and eb[16:32] == v1[16:32]
            assert struct.unpack_from("<I", eb, 32)[0] == len(v1)
            # never more than the tags and the 8-byte count fields over v1
            assert len(eb) <= len(v1) + 8 + 4 * P + 4
            scaled += bool(v1[5] & 1)
    assert scaled > 0


def test_oracle_resumes_from_entropy_checkpoints():
    n, b = 12, 8
    gates = I.qft(n)
    a = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    a.set_basis(0x5A5)
    a.run(gates[:40])
    e = a.export_state(entropy=True)
    r = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    r.import_state(e)
    assert r.export_state() == a.export_state()
    for g in gates[40:]:
        a.apply(g)
        r.apply(g)
    assert r.export_state() == a.export_state()


@pytest.mark.parametrize("b,s", [(20, 10), (16, 10), (12, 6), (14, 12)])
def test_one_value_block_size_closed_form(b, s):
    """A block whose re planes all hold one value and im planes are zero:
    two verbatim 16-byte records and one run of the other 2^(b-s+1) - 2
    planes: 32 + 8 + 16 (three tags) + 32 bytes; the v1 stream holds
    16 bytes per plane."""
    v = 2.0 ** -10
    hdr = struct.pack("<IBBBBII", 0x31424141, 0, 0, s, b, 0, 0)
    P = 2 << (b - s)
    rec = struct.pack("<qII", struct.unpack("<q", struct.pack("<d", v))[0], 0, 0)
    zero = struct.pack("<qII", 0, 0, 0)
    normsq = v * v * (1 << b)
    v1 = bytearray(hdr + struct.pack("<dd", 0.0, normsq) + (rec + zero) * (P // 2))
    struct.pack_into("<I", v1, 12, len(v1))
    v1 = bytes(v1)
    e = orc.entropy_encode(v1)
    assert len(e) == 88
    assert orc.entropy_decode(e) == v1
    assert len(v1) == 32 + 16 * P
    # the raw block over the entropy stream: 2^(b+4) / 88
    assert (16 << b) / len(e) == pytest.approx(2.0 ** (b + 4) / 88)


def test_malformed_entropy_streams_are_rejected():
    data = states()[0]
    blocks = orc.split_streams(data)
    v1 = max(blocks, key=len)
    e = bytearray(orc.entropy_encode(v1))
    ni = struct.unpack_from("<I", e, 36)[0]
    tags = list(struct.unpack_from("<%dI" % ni, e, 40))
    lit = next(i for i, t in enumerate(tags) if not t & 0xC0000000)
    body = 40 + (4 * ni + 7) // 8 * 8 + sum(t & 0x3FFFFFFF for t in tags[:lit]
                                            if not t & 0x80000000)
    bad = []

    def mut(f):
        x = bytearray(e)
        f(x)
        bad.append(bytes(x))

    mut(lambda x: struct.pack_into("<I", x, 0, 0x31424141))           # v1 magic
    mut(lambda x: struct.pack_into("<I", x, 12, len(e) - 8))          # total
    mut(lambda x: struct.pack_into("<I", x, 32, len(v1) + 8))         # v1 length
    mut(lambda x: struct.pack_into("<I", x, 36, ni + 1))              # item count
    mut(lambda x: struct.pack_into("<I", x, 40, 0x80000001))          # run at plane 0
    mut(lambda x: struct.pack_into("<I", x, 40 + 4 * lit, tags[lit] + 8))   # body length
    mut(lambda x: struct.pack_into("<I", x, body + 8,
                                   struct.unpack_from("<I", e, body + 8)[0] + 1))  # pw
    mut(lambda x: struct.pack_into("<I", x, body + 20, 1))            # reserved word
    mut(lambda x: x.__setitem__(body + 24, 200))                      # mode byte
    bad.append(bytes(e[:-8]))                                         # truncated
    for x in bad:
        with pytest.raises(ValueError):
            orc.entropy_decode(x)
    # a code whose length field disagrees with what it decodes to
    spike = np.zeros(2048)
    spike[100] = 1e6
    blk = orc.encode_block(spike, 10, 10, 0.5, 1)
    e2 = bytearray(orc.entropy_encode(blk))
    modes_at = 40 + 8 + 24
    assert 64 <= e2[modes_at] < 128  # the spike's chunk is sparse
    lens_at = modes_at + 16
    struct.pack_into("<H", e2, lens_at, struct.unpack_from("<H", e2, lens_at)[0] + 1)
    with pytest.raises(ValueError):
        orc.entropy_decode(bytes(e2))


def test_entropy_is_smaller_where_the_fixed_width_packer_wastes():
    """Sparse-phase QFT states (a few nonzero residuals per chunk) and
    one-value Grover blocks shrink several times; a dense final QFT state
    stays within the tags' overhead of v1."""
    o = orc.OracleSim(16, 12, I.default_ladder(1e-4), 4.0)
    o.set_basis(0x1234)
    g = I.qft(16)
    o.run(g[:80])
    v1, e = o.export_state(), o.export_state(entropy=True)
    assert len(e) * 4 < len(v1)
    o.run(g[80:])
    v1, e = o.export_state(), o.export_state(entropy=True)
    assert len(v1) * 0.99 < len(e) <= len(v1) * 1.005
    gr = orc.OracleSim(18, 16, I.default_ladder(1e-5), 4.0)
    gr.run(I.grover(18, 12345, 3))
    v1, e = gr.export_state(), gr.export_state(entropy=True)
    assert len(e) * 15 < len(v1)
