"""Pins of the oracle's pointwise-relative levels (a ladder entry -eps: the
log transform of the relative-bound reference the paper builds on with SZ),
each against something other than the oracle itself: the bound checked in
exact rational arithmetic, the codec's log and power of two against the
math library and at exact points, a stream derived by hand for powers of
two, zeros and non-finite values, ladder validation, and whole circuits
against closed forms where the absolute bound collapses.
"""
import math
import struct
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1811_05140_amd import inputs as I


def bits(x):
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def test_codec_log2_and_exp2_against_math():
    rng = np.random.default_rng(7)
    a = np.exp(rng.uniform(-744.0, 709.0, 20000))
    a = np.concatenate([a, [5e-324, 2.2250738585072014e-308, 1.7976931348623157e308,
                            0.7071067811865476, 1.4142135623730951, 1.0 + 2 ** -52]])
    for v in a:
        got, want = orc.codec_log2(v), math.log2(v)
        assert abs(got - want) <= 2e-14 * max(1.0, abs(want)), v
    for y in rng.uniform(-1022.0, 1023.0, 20000):
        got, want = orc.codec_exp2(y), 2.0 ** y
        assert abs(got - want) <= 1e-15 * want, y
    # exact at the powers of two, both ways, subnormals included
    for j in range(-1074, 1024):
        assert orc.codec_log2(math.ldexp(1.0, j)) == float(j)
        assert orc.codec_exp2(float(j)) == math.ldexp(1.0, j)


def probe_values(rng):
    vals = [0.0, -0.0, 1.0, -1.0, 5e-324, -5e-324, 2.2250738585072014e-308, 1e-300,
            1e300, 1.7976931348623157e308, 0.1, -0.3, math.inf, -math.inf, math.nan]
    vals += list(rng.normal(size=1500) * 10.0 ** rng.integers(-200, 200, 1500))
    vals += list(rng.uniform(-1, 1, 1500) * 2.0 ** -12)
    return vals


@pytest.mark.parametrize("eps", [0.05, 1e-3, 1e-5, 2.0 ** -19])
def test_relative_bound_is_exact(eps):
    """Every decoded value x-hat of a finite x satisfies |x - x-hat| < eps
    |x| in exact rational arithmetic (zeros decode to +0, error 0);
    non-finite values and the rare misses come back bit for bit."""
    rng = np.random.default_rng(int(-math.log2(eps) * 3))
    vals = probe_values(rng)
    b = s = 12
    n = 1 << b
    x = np.zeros(2 * n)
    x[:len(vals)] = vals
    x[n:n + len(vals)] = vals[::-1]
    stream = orc.encode_block(x, b, s, -eps, level=1)
    xh = orc.decode_block_interleaved(stream)
    E = Fraction(eps)
    exact = 0
    for a, ah in zip(x, xh):
        if not math.isfinite(a):
            assert bits(a) == bits(ah)
        elif a == 0.0:
            assert bits(ah) == 0  # +0
        else:
            assert abs(Fraction(a) - Fraction(ah)) < E * abs(Fraction(a)), (a, ah)
            exact += bits(a) == bits(ah)
    nout = struct.unpack_from("<I", stream, 8)[0]
    # inf, -inf and nan in both planes; the rest of the plane (magnitudes
    # from 5e-324 to 1.8e308) fits the log codes with at most a few misses
    assert 6 <= nout <= 6 + 0.002 * 2 * len(vals)


def test_relative_hand_derived_stream():
    """eps with fl(1.4 eps) = 2^-11 gives the log step eL = 2^-10: the value
    +-2^j has log code 1024 j exactly, code c = 2 (1024 j + 2^28) + sign, and
    decodes to +-2^j exactly (no outliers).  re plane: 1, -1, 2, 0.5 then
    zeros; im plane: zeros."""
    eps = 2.0 ** -11 / 1.4
    assert 1.4 * eps == 2.0 ** -11
    Q = 1 << 28
    codes = [2 * (0 + Q), 2 * (0 + Q) + 1, 2 * (1024 + Q), 2 * (-1024 + Q)] + [0] * 60
    # Lorenzo residuals and zigzags of the codes (c_0 = 0; anchor = codes[0])
    c = [0] + [codes[i] - codes[i - 1] for i in range(1, 64)]
    z = [(v << 1) ^ (v >> 63) if v >= 0 else ((v << 1) ^ -1) & 0xFFFFFFFFFFFFFFFF
         for v in c]
    # residuals 1, 2047, -4096, -2 (2^28 - 1024), 0: zigzags by hand
    assert z[:6] == [0, 2, 4094, 8191, 4 * (Q - 1024) - 1, 0]
    w = max(z).bit_length()
    words = [0] * w
    for l, v in enumerate(z):
        for bit in range(w):
            if (v >> bit) & 1:
                pos = l * w + bit
                words[pos >> 6] |= 1 << (pos & 63)
    re = struct.pack("<qII", codes[0], w, 0) + bytes([w]) + b"\0" * 7
    re += b"".join(struct.pack("<Q", v) for v in words)
    im = struct.pack("<qII", 0, 0, 0)
    normsq = 1.0 + 1.0 + 4.0 + 0.25
    total = 32 + len(re) + len(im)
    hdr = struct.pack("<IBBBBIIdd", 0x31424141, 1, 0, 6, 6, 0, total, -eps, normsq)
    x = np.zeros(128)
    x[0:8:2] = [1.0, -1.0, 2.0, 0.5]
    assert orc.encode_block(x, 6, 6, -eps, 1) == hdr + re + im
    back = orc.decode_block_interleaved(hdr + re + im)
    assert np.array_equal(back.view(np.uint64), x.view(np.uint64))


def test_relative_level_ladders():
    lad_ok = [[0.0, -1e-5, -1e-4, -1e-3], [-1e-3], [-0.05], [0.0, -2.0 ** -19]]
    lad_bad = [[0.0, 1e-6, -1e-5], [-1e-4, -1e-5], [-0.06], [-1e-6], [0.0, -0.0],
               [-1e-3, 1e-3]]
    x = np.zeros(128)
    x[0] = 1.0
    for lad in lad_ok:
        buf = orc.aalc_encode(x, 6, 6, lad, 4.0)
        assert buf is not None
    for lad in lad_bad:
        with pytest.raises(Exception):
            orc.aalc_encode(x, 6, 6, lad, 4.0)


def test_relative_level_keeps_small_amplitudes():
    """A fixed absolute bound of 0.01 zeroes every amplitude of a 14-qubit
    QFT (each of magnitude 2^-7 < 0.01 in the end): the state collapses
    (N^2 = 0).  A relative bound of 0.01 cannot zero a nonzero value, and
    the final state meets the closed form closely."""
    n, b, x0 = 14, 10, 0x2B7D
    gates = I.qft(n)
    a = orc.OracleSim(n, b, [0.01], 4.0)
    a.set_basis(x0)
    for g in gates:
        a.apply(g)
    assert a.stats()["collapsed"]
    r = orc.OracleSim(n, b, [-0.01], 4.0)
    r.set_basis(x0)
    for g in gates:
        r.apply(g)
    st = r.stats()
    assert not st["collapsed"]
    k = np.arange(1 << n)
    want = np.exp(2j * np.pi * ((x0 * k) % (1 << n)) / (1 << n)) / 2 ** (n / 2)
    F = orc.fidelity(want, r.amplitudes(), n)
    assert F > 0.99
    # a relative ladder with a lossless first level and theta = 4
    lad = [0.0, -1e-5, -1e-4, -1e-3]
    q = orc.OracleSim(n, b, lad, 4.0)
    q.set_basis(x0)
    for g in gates:
        q.apply(g)
    assert orc.fidelity(want, q.amplitudes(), n) > 0.9999
    assert q.stats()["min_ratio"] >= 1.0
