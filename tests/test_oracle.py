"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: a dense
Kronecker-product simulation, a closed form (QFT, Grover), an exact rational
check of the error bound, streams derived by hand from the format definition,
an exact sum (math.fsum), or numbers the paper prints.
"""
import json
import math
import os
import struct
from fractions import Fraction
from functools import reduce

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1811_05140_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def bits(x):
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def same_bits(a, b):
    a = np.ascontiguousarray(a, dtype=np.complex128).view(np.uint64)
    b = np.ascontiguousarray(b, dtype=np.complex128).view(np.uint64)
    return a.shape == b.shape and bool(np.all(a == b))


# ---------------------------------------------------------------- sums ----

def test_pairwise_tree_shape():
    # Left-to-right gives ((1e16 + 1) - 1e16) + 1 = 1; the tree gives
    # (1e16 + 1) + (-1e16 + 1) = 1e16 + (-1e16) = 0.  Pins the tree order.
    v = np.array([1e16, 1.0, -1e16, 1.0])
    assert orc.pairwise(v) == 0.0
    v8 = np.array([1e16, 1.0, 1.0, 1.0, -1e16, 1.0, 1.0, 1.0])
    # (1e16+1)+(1+1) = 1e16+2 ; (-1e16+1)+(1+1) = -1e16+2 ; sum = 4
    assert orc.pairwise(v8) == 4.0


def test_pairwise_close_to_exact_sum():
    rng = np.random.default_rng(7)
    for m in (1, 2, 64, 4096, 1 << 16):
        v = rng.random(m)
        exact = math.fsum(v)
        assert abs(orc.pairwise(v) - exact) <= 1e-15 * exact * max(1, math.log2(m))


# ------------------------------------------------------------- gates ------

def dense_gate(g, n):
    """Full 2^n x 2^n matrix of a gate from Kronecker products (qubit q is
    bit q, so it is factor n-1-q of the product)."""
    kind, q0, q1, index, u = g
    N = 1 << n
    I2 = np.eye(2, dtype=complex)
    U = np.array([[u[0] + 1j * u[1], u[2] + 1j * u[3]],
                  [u[4] + 1j * u[5], u[6] + 1j * u[7]]])

    def on(ops):
        f = [I2] * n
        for q, m in ops.items():
            f[n - 1 - q] = m
        return reduce(np.kron, f)

    P0 = np.diag([1, 0]).astype(complex)
    P1 = np.diag([0, 1]).astype(complex)
    if kind == I.G_U:
        return on({q0: U})
    if kind == I.G_X:
        return on({q0: np.array([[0, 1], [1, 0]], dtype=complex)})
    if kind == I.G_DIAG1:
        return on({q0: np.diag([1, u[6] + 1j * u[7]])})
    if kind == I.G_CU:
        return on({q0: P0}) + on({q0: P1, q1: U})
    if kind == I.G_CPHASE:
        ph = u[6] + 1j * u[7]
        return np.eye(N) + (ph - 1) * on({q0: P1, q1: P1})
    if kind == I.G_CZ:
        return np.eye(N) - 2 * on({q0: P1, q1: P1})
    if kind == I.G_SWAP:
        M = np.zeros((N, N), dtype=complex)
        for i in range(N):
            b0, b1 = (i >> q0) & 1, (i >> q1) & 1
            j = i & ~((1 << q0) | (1 << q1)) | (b1 << q0) | (b0 << q1)
            M[j, i] = 1
        return M
    if kind == I.G_PHASE_FLIP:
        d = np.ones(N, dtype=complex)
        d[index] = -1
        return np.diag(d)
    if kind == I.G_DIFFUSE:
        return 2.0 / N * np.ones((N, N)) - np.eye(N)
    raise ValueError(kind)


def random_unitary(rng):
    a = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    q, r = np.linalg.qr(a)
    q = q * (np.diag(r) / np.abs(np.diag(r)))
    return tuple(float(v) for z in q.reshape(-1) for v in (z.real, z.imag))


def random_gates(n, count, rng):
    gates = []
    for _ in range(count):
        k = int(rng.integers(1, 10))
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        if k == I.G_U:
            gates.append(I.u_gate(a, random_unitary(rng)))
        elif k == I.G_DIAG1:
            phi = rng.uniform(0, 2 * math.pi)
            gates.append(I.diag1(a, math.cos(phi), math.sin(phi)))
        elif k == I.G_CU:
            gates.append(I.cu(a, b, random_unitary(rng)))
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


@pytest.mark.parametrize("n", [6, 7, 8])
def test_plain_gates_match_dense_matrices(n):
    rng = np.random.default_rng(100 + n)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    amp = np.empty(2 << n)
    amp[0::2], amp[1::2] = psi.real, psi.imag
    ref = psi.copy()
    for g in random_gates(n, 60, rng):
        orc.sv_apply(amp, n, g)
        ref = dense_gate(g, n) @ ref
        got = amp[0::2] + 1j * amp[1::2]
        assert np.max(np.abs(got - ref)) < 1e-13, g


def test_every_gate_kind_against_dense_n10():
    n = 10
    rng = np.random.default_rng(5)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    for g in [I.u_gate(9, random_unitary(rng)), I.diag1(3, 0.6, 0.8),
              I.cu(9, 2, random_unitary(rng)), I.cphase(1, 8, 0.3),
              I.cz(0, 9), I.swap(2, 9), I.x(7), I.phase_flip(777),
              I.diffuse()]:
        amp = np.empty(2 << n)
        amp[0::2], amp[1::2] = psi.real, psi.imag
        orc.sv_apply(amp, n, g)
        ref = dense_gate(g, n) @ psi
        assert np.max(np.abs(amp[0::2] + 1j * amp[1::2] - ref)) < 1e-13, g[0]


def test_diffuse_is_two_mean_minus_psi():
    # DIFFUSE equals the dense 2|s><s| - I; on a uniform state it is identity.
    n = 8
    N = 1 << n
    amp = np.zeros(2 * N)
    amp[0::2] = 1.0 / 16.0
    orc.sv_apply(amp, n, I.diffuse())
    assert np.all(amp[0::2] == 1.0 / 16.0) and np.all(amp[1::2] == 0.0)


# --------------------------------------------------------- closed forms ----

def qft_closed_form(n, x):
    k = np.arange(1 << n)
    return np.exp(2j * np.pi * ((x * k) % (1 << n)) / (1 << n)) / 2 ** (n / 2)


@pytest.mark.parametrize("n,x", [(2, 1), (6, 37), (8, 200), (10, 0x2A5),
                                 (12, 0xBEE), (14, 0x1234)])
def test_qft_uncompressed_closed_form(n, x):
    got = orc.sv_run(n, I.qft(n), basis=x)
    assert np.max(np.abs(got - qft_closed_form(n, x))) < 1e-13


@pytest.mark.parametrize("n,k", [(10, 25), (12, 3), (8, 6)])
def test_grover_uncompressed_closed_form(n, k):
    m = (0x5A5A5A5 * (n + k)) % (1 << n)
    psi = orc.sv_run(n, I.grover(n, m, k))
    p = abs(psi[m]) ** 2
    assert abs(p - I.grover_success(n, k)) < 1e-12
    # the textbook value quoted for n = 10, k = 25
    if (n, k) == (10, 25):
        assert abs(p - 0.99946124474) < 1e-10


def test_qft_gate_count():
    assert len(I.qft(12)) == 84 and len(I.qft(24)) == 312


# ------------------------------------------------ codec: exact invariants ----

def quantiser_probe_values(rng, delta):
    e = 2 * delta
    vals = [0.0, -0.0, delta, -delta, e, 0.5 * e, 1.5 * e, 2.5 * e,
            delta * (1 - 2 ** -52), delta * (1 + 2 ** -52), 1.0, -1.0,
            2 ** 30 * e, 2 ** 30 * e * (1 - 2 ** -40), 5e-324, 1e300,
            math.inf, -math.inf]
    vals += list((rng.integers(-2000, 2000, 200) + 0.5) * e)   # exact ties
    vals += list(rng.normal(scale=100 * delta, size=1500))
    vals += list(rng.uniform(-1, 1, size=1500) * 2.0 ** rng.integers(-40, 1, 1500))
    return vals


@pytest.mark.parametrize("delta", [1e-4, 1e-7, 0.25, 2.0 ** -30])
def test_pointwise_bound_is_exact(delta):
    """Every decoded scalar lies in [x - delta, x + delta], checked in exact
    rational arithmetic; outliers come back bit-exact."""
    rng = np.random.default_rng(int(-math.log2(delta) * 10))
    vals = quantiser_probe_values(rng, delta)
    b = s = 12
    n = 1 << b
    x = np.zeros(2 * n)
    x[:len(vals)] = vals
    x[n:n + len(vals)] = vals[::-1]
    stream = orc.encode_block(x, b, s, delta, level=1)
    xh = orc.decode_block_interleaved(stream)
    D = Fraction(delta)
    for a, ah in zip(x, xh):
        if math.isfinite(a):
            assert abs(Fraction(a) - Fraction(ah)) <= D
        else:
            assert bits(a) == bits(ah)
    # With a power-of-two delta, 2.5 e is an exact tie: q = 2 (even),
    # xhat = 2 e, an error of exactly delta, which the strict rule stores as
    # an outlier; 1.5 e ties to q = 2 as well and is stored the same way.
    if math.frexp(delta)[0] == 0.5:
        for v in (2.5 * 2 * delta, 1.5 * 2 * delta):
            i = vals.index(v)
            assert bits(xh[i]) == bits(x[i])


def test_lossless_round_trip_bit_exact():
    rng = np.random.default_rng(3)
    b, s = 10, 8
    raw = rng.integers(0, 2 ** 63, size=2 << b, dtype=np.uint64) * np.uint64(2) \
        + rng.integers(0, 2, size=2 << b, dtype=np.uint64)
    raw[:8] = [0, 1 << 63, 0x7FF0000000000000, 0xFFF0000000000000,
               0x7FF8000000000000, 1, 0x000FFFFFFFFFFFFF, 0x3FF0000000000000]
    x = raw.view(np.float64)
    stream = orc.encode_block(x, b, s, 0.0, level=0)
    back = orc.decode_block_interleaved(stream)
    assert np.all(back.view(np.uint64) == raw)


def test_decoder_rejects_malformed_streams():
    x = np.zeros(2 << 6)
    x[6] = 1.0
    st = bytearray(orc.encode_block(x, 6, 6, 0.0))
    orc.decode_block(bytes(st))
    for k in (0, 12):           # magic, total length
        bad = bytearray(st)
        bad[k] ^= 1
        with pytest.raises(ValueError):
            orc.decode_block(bytes(bad))
    with pytest.raises(ValueError):
        orc.decode_block(bytes(st[:-8]))


# ----------------------------------- hand-derived streams (format pins) ----

def hdr(level, s, b, nout, total, delta, normsq):
    return struct.pack("<IBBBBIIdd", 0x31424141, level, 0, s, b, nout, total,
                       delta, normsq)


def plane(anchor, pw, nout, widths=b"", payload=(), outliers=()):
    out = struct.pack("<qII", anchor, pw, nout)
    if pw:
        out += widths + b"\0" * ((-len(widths)) % 8)
    out += b"".join(struct.pack("<Q", w) for w in payload)
    out += b"".join(struct.pack("<IId", i, 0, v) for i, v in outliers)
    return out


def test_golden_zero_block_lossless():
    # 64 zero amplitudes, one segment: both planes constant -> no payload.
    want = hdr(0, 6, 6, 0, 64, 0.0, 0.0) + plane(0, 0, 0) + plane(0, 0, 0)
    assert orc.encode_block(np.zeros(128), 6, 6, 0.0, 0) == want


def test_golden_basis_state_lossless():
    # |3> in a block of 64: re plane q = bits = [0,0,0,0x3FF0..0,0,...].
    # c_3 = 0x3FF0000000000000 -> zigzag 0x7FE0000000000000 (63 bits);
    # c_4 = -0x3FF0000000000000 -> zigzag 0x7FDFFFFFFFFFFFFF (63 bits); w = 63.
    # Field l sits at bits [63 l, 63 l + 63): field 3 at 189..251 (its low
    # three bits, all zero, end word 2), field 4 at 252..314.
    # word 3 = (0x7FE0..0 >> 3) | (0xF << 60) = 0xFFFC000000000000
    # word 4 = 0x7FDFFFFFFFFFFFFF >> 4       = 0x07FDFFFFFFFFFFFF
    payload = [0] * 63
    payload[3] = 0xFFFC000000000000
    payload[4] = 0x07FDFFFFFFFFFFFF
    re = plane(0, 63, 0, bytes([63]), payload)
    want = hdr(0, 6, 6, 0, 32 + len(re) + 16, 0.0, 1.0) + re + plane(0, 0, 0)
    assert len(want) == 576
    x = np.zeros(128)
    x[6] = 1.0
    assert orc.encode_block(x, 6, 6, 0.0, 0) == want


LOSSY_RE = [0.0, 0.2, 0.5, 0.7, 1.0, -0.2, -0.6, 3.0, 0.75, 1e12] + [0.0] * 54


def test_golden_lossy_block():
    # delta = 0.25: e = 0.5, r = 2, y = 2x = [0, .4, 1, 1.4, 2, -.4, -1.2, 6,
    # 1.5, 2e12, 0...].  q = [0,0,1,1,2,0,-1,6,2,0,...] (1.5 ties to 2;
    # 2e12 >= 2^30 -> q = 0, outlier).  xhat(8) = 1.0 misses 0.75 by exactly
    # delta -> outlier.  c = [0,0,1,0,1,-2,-1,7,-4,-2,0..],
    # z = [0,0,2,0,2,3,1,14,7,3,0..], w = 4, nibble l of word 0 is z_l:
    # word 0 = 0x00000037E1320200.  normsq: the first eight squares sum to
    # 10.75, which vanishes next to 1e12^2 = 1e24.
    re = plane(0, 4, 2, bytes([4]), [0x00000037E1320200, 0, 0, 0],
               [(8, 0.75), (9, 1e12)])
    want = hdr(1, 6, 6, 2, 32 + len(re) + 16, 0.25, 1e24) + re + plane(0, 0, 0)
    x = np.zeros(128)
    x[0::2] = LOSSY_RE
    assert orc.encode_block(x, 6, 6, 0.25, 1) == want


def test_golden_aalc_choice():
    # Ladder (0, 0.25), theta 4, raw = 16 * 64 = 1024 bytes.  Lossless needs
    # w >= 63 for the re chunk (zigzag(bits(0.2)) = 0x7F93333333333334), so
    # its stream is > 504 bytes and 1024 < 4 * size: rejected.  Level 1 is
    # 136 bytes and 1024 >= 544: chosen.
    x = np.zeros(128)
    x[0::2] = LOSSY_RE
    k, st, sizes = orc.aalc_encode(x, 6, 6, [0.0, 0.25], 4.0)
    assert k == 1 and len(st) == 136 and sizes[0] > 504
    assert st == orc.encode_block(x, 6, 6, 0.25, 1)


def test_aalc_rule_on_many_blocks():
    """Chosen level: first with raw >= theta * size, else the last; every
    tried size equals the length of that level's stream."""
    rng = np.random.default_rng(11)
    ladder = I.default_ladder(1e-3)
    b, s = 10, 8
    raw = 16 << b
    seen = set()
    for t in range(30):
        scale = 10.0 ** rng.uniform(-6, 0)
        x = rng.normal(scale=scale, size=2 << b)
        if t % 3 == 0:
            x[rng.random(2 << b) < 0.9] = 0.0
        for theta in (1.0, 4.0, 16.0, 64.0):
            k, st, sizes = orc.aalc_encode(x, b, s, ladder, theta)
            seen.add(k)
            for j in range(k + 1):
                assert sizes[j] == len(orc.encode_block(x, b, s, ladder[j], j))
            for j in range(k):
                assert raw < theta * sizes[j]
            assert raw >= theta * sizes[k] or k == len(ladder) - 1
            assert len(st) == sizes[k] and st[4] == k
    assert len(seen) >= 3


# ------------------------------------------------ compressed driver -------

def test_lossless_unnormalised_equals_plain_bit_exact():
    """Lossless-only ladder without normalisation reproduces the plain
    state-vector run bit for bit (in-segment, segment-pair and block-pair
    gates of every kind)."""
    rng = np.random.default_rng(21)
    n, b = 9, 7
    gates = I.qft(n) + random_gates(n, 80, rng)
    sim = orc.OracleSim(n, b, [0.0], theta=4.0, normalize=False, s=6)
    sim.set_basis(300)
    sim.run(gates)
    ref = orc.sv_run(n, gates, basis=300)
    assert same_bits(sim.amplitudes(), ref)


def test_qft12_compressed_fidelity_and_threshold():
    w = I.qft12_workload()
    n, b = w["n"], w["b"]
    ref = qft_closed_form(n, w["basis"])
    sim = orc.OracleSim(n, b, I.default_ladder(1e-4), theta=4.0)
    sim.set_basis(w["basis"])
    sim.run(w["gates"])
    F = orc.fidelity(ref, sim.amplitudes(), n)
    assert F > 0.999
    st = sim.stats()
    assert st["passes"] == 84 and st["collapsed"] == 0
    # N^2 s^2 = 1 to rounding
    assert abs(st["normsq"] * st["scale"] ** 2 - 1.0) < 1e-14


def test_grover_compressed_matches_closed_form():
    n, k = 10, 6
    m = 0x2B7
    # Lossless only: the state is exact up to rounding.
    sim = orc.OracleSim(n, 8, [0.0], theta=4.0)
    sim.run(I.grover(n, m, k))
    p = abs(sim.amplitudes(m, 1)[0]) ** 2
    assert abs(p - I.grover_success(n, k)) < 1e-12
    # Default ladder at delta = 1e-5.  The phase flip writes -0.0 into the
    # imaginary part of the marked amplitude, which costs a 64-bit chunk in
    # the lossless im plane, so the marked block drops to delta_1 = 1e-8;
    # the other blocks are constant and stay lossless.
    sim = orc.OracleSim(n, 8, I.default_ladder(1e-5), theta=4.0)
    sim.run(I.grover(n, m, k))
    p = abs(sim.amplitudes(m, 1)[0]) ** 2
    assert abs(p - I.grover_success(n, k)) < 1e-7
    hist = sim.stats()["level_hist"]
    assert hist[0] > 0 and hist[1] > 0 and sum(hist[2:]) == 0


def test_fidelity_properties():
    rng = np.random.default_rng(2)
    n = 8
    a = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    b = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    assert abs(orc.fidelity(a, a, n) - 1.0) < 1e-14
    assert abs(orc.fidelity(a, a * np.exp(0.7j) * 3.0, n) - 1.0) < 1e-14
    F = orc.fidelity(a, b, n)
    assert 0.0 <= F <= 1.0
    e0 = np.zeros(1 << n, dtype=complex)
    e1 = np.zeros(1 << n, dtype=complex)
    e0[0] = e1[1] = 1.0
    assert orc.fidelity(e0, e1, n) == 0.0
    # matches |<a|b>|^2 / (<a|a><b|b>) from numpy
    ref = abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)
    assert abs(F - ref) < 1e-13


def test_process_group_reproduces_driver_pass():
    n, b = 10, 7
    lad = I.default_ladder(1e-4)
    sim = orc.OracleSim(n, b, lad, theta=4.0, s=6)
    gates = I.qft(n)[:30]
    sim.run(gates)
    for g in (I.h(9), I.h(2), I.swap(1, 8), I.cphase(0, 9, 0.4)):
        before = [sim.export_block(j) for j in range(1 << (n - b))]
        sc = sim.stats()["scale"]
        sim.apply(g)
        mb = ((1 << g[1]) | ((1 << g[2]) if g[0] == I.G_SWAP else 0)) >> b \
            if g[0] in (I.G_U, I.G_SWAP) else 0
        for j in range(1 << (n - b)):
            if mb and (j ^ mb) < j:
                continue
            o0, o1 = orc.process_group(n, b, 6, lad, 4.0, sc, None, g, j,
                                       before[j],
                                       before[j ^ mb] if mb else None)
            assert o0 == sim.export_block(j)
            if mb:
                assert o1 == sim.export_block(j ^ mb)


def test_amplitude_sum_pins():
    # basis state: one amplitude 1, the rest 0
    sim = orc.OracleSim(10, 7, I.default_ladder(1e-4), theta=4.0)
    sim.set_basis(0x155)
    assert sim.amplitude_sum() == 1.0 + 0.0j
    # uniform superposition: 2^n equal leaves v sum to 2^n v exactly, so a
    # dropped or doubled leaf anywhere in the tree shows
    sim.set_basis(0)
    sim.run([I.h(q) for q in range(10)])
    a = sim.amplitudes()
    assert np.all(a == a[0])
    assert sim.amplitude_sum() == complex(1024 * a[0].real, 0.0)
    # QFT of a basis state x: sum_k w^(xk) / 2^(n/2) is 2^(n/2) for x = 0 and
    # 0 otherwise (geometric series)
    for x, want in ((0, 32.0), (0x2A5, 0.0)):
        sim = orc.OracleSim(10, 7, [0.0], theta=4.0)
        sim.set_basis(x)
        sim.run(I.qft(10))
        assert abs(sim.amplitude_sum() - want) < 1e-12
    # against an exactly rounded sum of the amplitudes (math.fsum), within
    # the pairwise bound log2(N) * eps * sum |a|
    sim = orc.OracleSim(11, 8, I.default_ladder(1e-4), theta=4.0)
    sim.set_basis(0x3C1)
    sim.run(I.qft(11)[:40])
    a = sim.amplitudes()
    S = sim.amplitude_sum()
    tol = 11 * 2.0 ** -52 * np.abs(a).sum()
    assert abs(S.real - math.fsum(a.real)) <= tol
    assert abs(S.imag - math.fsum(a.imag)) <= tol
    # Grover: before a diffusion the sum is -sin((2i-1)t) + sqrt(N-1) cos((2i-1)t)
    n, m = 10, 0x2B7
    sim = orc.OracleSim(n, 8, [0.0], theta=4.0)
    sim.run([I.h(q) for q in range(n)])
    th = math.asin(2.0 ** (-n / 2))
    for i in range(1, 4):
        sim.apply(I.phase_flip(m))
        want = -math.sin((2 * i - 1) * th) + math.sqrt((1 << n) - 1) * math.cos((2 * i - 1) * th)
        assert abs(sim.amplitude_sum() - want) < 1e-12
        sim.apply(I.diffuse())


def test_measure_probs_uniform_after_qft():
    n = 10
    sim = orc.OracleSim(n, 8, [0.0], theta=4.0)
    sim.set_basis(123)
    sim.run(I.qft(n))
    p = sim.measure_probs([0, 3, 9])
    assert np.allclose(p, 1.0 / 8.0, atol=1e-14)
    assert abs(p.sum() - 1.0) < 1e-14


def test_basis_state_invariants():
    sim = orc.OracleSim(12, 8, I.default_ladder(1e-4), theta=4.0)
    sim.set_basis(0xABC)
    a = sim.amplitudes()
    assert a[0xABC] == 1.0 and np.count_nonzero(a) == 1
    st = sim.stats()
    assert st["normsq"] == 1.0 and st["scale"] == 1.0


# ---------------------------------------------- numbers the paper prints ----

def test_paper_capacity_numbers():
    g = json.load(open(os.path.join(GOLDEN, "paper_capacity.json")))
    PB = g["pb_bytes"]
    for n, pb in g["state_bytes"]:
        assert orc.state_bytes(n) == pb * PB
    for _, mem, q in g["table1"]:
        assert orc.max_qubits(mem * PB) == q
    for ratio, extra in g["extra_qubits"]:
        assert orc.max_qubits(16 << 40, ratio) - orc.max_qubits(16 << 40) == extra
    for mem, ratio, q in g["theta_with_aalc"]:
        assert orc.max_qubits(mem * PB, ratio) == q


def test_splitmix64_published_vector():
    r = I.SplitMix64(0)
    assert [r.next() for _ in range(3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_quantiser_code_range_edge():
    """Codes stay within +-(2^30 - 1) (the quantiser accepts |y| < 2^30 - 1),
    so a lossy residual always fits 32 signed bits.  delta = 0.25 (e = 0.5,
    r = 2, y = 2x): x = +-(2^30 - 0.5)/2 gives |y| = 2^30 - 0.5, out of range:
    outliers with code 0 (under a 2^30 bound they would take codes +-2^30 and
    the residual +2^31 would need 33 bits).  x = +-(2^30 - 1.75)/2 gives
    y = +-(2^30 - 1.75), code +-(2^30 - 2), xhat = +-(2^29 - 1) within 0.125.
    Codes [0, 0, 2^30-2, -(2^30-2), 0, ...] give residuals c_2 = 2^30-2,
    c_3 = -(2^31-4), c_4 = 2^30-2 and zigzags 2^31-4, 2^32-9, 2^31-4: one
    32-bit chunk (fields 2, 3, 4 in words 1 and 2)."""
    xa = (2.0 ** 30 - 0.5) / 2
    xb = (2.0 ** 30 - 1.75) / 2
    x = np.zeros(128)
    x[0:8:2] = [-xa, xa, xb, -xb]
    st = orc.encode_block(x, 6, 6, 0.25, 0)
    anc, pw, no = struct.unpack_from("<qII", st, 32)
    assert (anc, pw, no) == (0, 32, 2)
    assert st[48] == 32
    words = struct.unpack_from("<32Q", st, 56)
    assert words[0] == 0
    assert words[1] == (2 ** 31 - 4) | ((2 ** 32 - 9) << 32)
    assert words[2] == 2 ** 31 - 4
    assert all(w == 0 for w in words[3:])
    o = 56 + 8 * 32
    assert struct.unpack_from("<IIdIId", st, o) == (0, 0, -xa, 1, 0, xa)
    xh = orc.decode_block(st)
    assert list(xh.real[:4]) == [-xa, xa, 2.0 ** 29 - 1, -(2.0 ** 29 - 1)]


# ------------------------------------------- outcome probabilities (Sec. II) --

def test_measure_probs_basis_state_nonmonotone_qubits():
    """|x> has all probability on one outcome: bit k of o is bit qubits[k] of
    x.  Qubits listed out of order (5, 0, 3, 7) with bits 0, 5 and 6 of x set
    give o = 0b0011 = 3; the sorted list (0, 3, 5, 7) would spell 5 and the
    reversed list (7, 3, 0, 5) 12, so only the stated mapping passes."""
    n = 8
    x = (1 << 0) | (1 << 5) | (1 << 6)
    qubits = [5, 0, 3, 7]
    o_want = sum(((x >> q) & 1) << k for k, q in enumerate(qubits))
    assert o_want == 0b0011
    assert sum(((x >> q) & 1) << k for k, q in enumerate(sorted(qubits))) == 5
    assert sum(((x >> q) & 1) << k for k, q in enumerate(qubits[::-1])) == 12
    sim = orc.OracleSim(n, 6, I.default_ladder(1e-4), theta=4.0)
    sim.set_basis(x)
    p = sim.measure_probs(qubits)
    want = np.zeros(16)
    want[o_want] = 1.0
    assert np.array_equal(p, want)


def test_measure_probs_hand_computed_product_state():
    """Real rotations R(a) = [[cos a, -sin a], [sin a, cos a]] on qubits 1, 4
    and 2 of |0>: a product state, so P(o) is the product over listed qubits
    of cos^2 (bit 0) or sin^2 (bit 1) of that qubit's angle; qubit 6 is
    untouched (always 0).  Listed as (4, 6, 1, 2)."""
    n = 7
    ang = {1: 0.3, 4: 1.1, 2: 2.0}
    gates = []
    for q, a in ang.items():
        c, s_ = math.cos(a), math.sin(a)
        gates.append(I.u_gate(q, (c, 0.0, -s_, 0.0, s_, 0.0, c, 0.0)))
    qubits = [4, 6, 1, 2]
    sim = orc.OracleSim(n, 6, [0.0], theta=4.0)
    sim.run(gates)
    p = sim.measure_probs(qubits)
    want = np.zeros(16)
    for o in range(16):
        v = 1.0
        for k, q in enumerate(qubits):
            bit = (o >> k) & 1
            if q not in ang:
                v *= 0.0 if bit else 1.0
            else:
                v *= math.sin(ang[q]) ** 2 if bit else math.cos(ang[q]) ** 2
        want[o] = v
    assert np.max(np.abs(p - want)) < 1e-14
    # the mapping has teeth: P is far from uniform and not symmetric under
    # reversing the qubit list
    assert np.max(np.abs(p - want.reshape(2, 2, 2, 2).transpose().reshape(-1))) > 0.05


def test_measure_probs_two_qubit_entangled_by_hand():
    """R(a) on qubit 3, then CNOT (controlled X) from 3 to 0: amplitudes
    cos a at |0> and sin a at |1001>.  Listing (0, 5, 3): outcomes 0b000 with
    cos^2 a and 0b101 with sin^2 a, nothing else."""
    a = 0.4
    c, s_ = math.cos(a), math.sin(a)
    sim = orc.OracleSim(6, 6, [0.0], theta=4.0)
    sim.run([I.u_gate(3, (c, 0.0, -s_, 0.0, s_, 0.0, c, 0.0)),
             I.cu(3, 0, (0.0, 0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0))])
    p = sim.measure_probs([0, 5, 3])
    want = np.zeros(8)
    want[0b000] = c * c
    want[0b101] = s_ * s_
    assert np.max(np.abs(p - want)) < 1e-15


# ------------------------ normalisation before the gate (Sec. III, Alg. 2) --

def lossless_one_value_plane(vals):
    """Hand encoding (block stream v1) of one lossless 64-scalar plane whose
    nonzero entries are `vals` = {index: value}: q_i = bits(x_i), c_0 = 0,
    c_i = q_i - q_{i-1} mod 2^64, z = zigzag(c), one chunk of width
    max bitlen(z), field l at bits [l w, l w + w)."""
    q = [bits(vals.get(i, 0.0)) for i in range(64)]
    z = [0] + [(((q[i] - q[i - 1]) & (2 ** 64 - 1)) << 1 ^
                (2 ** 64 - 1 if (q[i] - q[i - 1]) & (2 ** 64 - 1) >= 2 ** 63 else 0))
               & (2 ** 64 - 1) for i in range(1, 64)]
    w = max(v.bit_length() for v in z)
    stream = 0
    for l, v in enumerate(z):
        stream |= v << (l * w)
    words = [(stream >> (64 * k)) & (2 ** 64 - 1) for k in range(w)]
    anchor = struct.unpack("<q", struct.pack("<Q", q[0]))[0]
    return plane(anchor, w, 0, bytes([w]) if w else b"", words if w else ())


def test_normalise_before_gate_hand_derived_stream():
    """A stored, unnormalised state with one amplitude 7.0 (n = b = s = 6,
    lossless ladder): N^2 = 49, s = fl(1/fl(sqrt 49)) = fl(1/7).  Alg. 2
    normalises before the gate: x = fl(7 s) = 1.0 exactly, then H on qubit 0
    gives y = fl(h * 1.0) = h at indices 0 and 1 (h = fl(sqrt(1/2))).  Gating
    first and scaling after would give fl(fl(7 h) s) = h - 1 ulp, and skipping
    the normalisation fl(7 h): the stream pins the order."""
    h = math.sqrt(0.5)
    s = 1.0 / math.sqrt(49.0)
    y = h * (7.0 * s)
    assert y == h and (h * 7.0) * s != y
    zero = plane(0, 0, 0)
    re_in = lossless_one_value_plane({0: 7.0})
    inp = hdr(0, 6, 6, 0, 32 + len(re_in) + len(zero), 0.0, 49.0) + re_in + zero
    re_out = lossless_one_value_plane({0: y, 1: y})
    ns = (y * y) + (y * y)  # pairwise over [y^2, y^2, 0, ...]
    want = hdr(0, 6, 6, 0, 32 + len(re_out) + len(zero), 0.0, ns) + re_out + zero
    wrong = lossless_one_value_plane({0: (h * 7.0) * s, 1: (h * 7.0) * s})
    assert wrong != re_out
    sim = orc.OracleSim(6, 6, [0.0], theta=4.0)
    assert sim.import_state(inp) == 0
    st = sim.stats()
    assert st["normsq"] == 49.0 and st["scale"] == s
    sim.apply(I.h(0))
    assert sim.export_block(0) == want
