"""GPU <-> oracle parity through the C ABI (needs an MI355X).

Bar: compressed streams byte-identical to the oracle's, decoded amplitudes
bit-identical (hence within 1e-12), probabilities / fidelities within 1e-12.
Every case prints what it runs before touching the GPU.
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


def random_unitary(rng):
    a = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    q, r = np.linalg.qr(a)
    q = q * (np.diag(r) / np.abs(np.diag(r)))
    return tuple(float(v) for z in q.reshape(-1) for v in (z.real, z.imag))


def random_gates(n, count, rng, kinds=range(1, 10)):
    kinds = list(kinds)
    gates = []
    for _ in range(count):
        k = kinds[int(rng.integers(0, len(kinds)))]
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


def same_bits(a, b):
    a = np.ascontiguousarray(a, dtype=np.complex128).view(np.uint64)
    b = np.ascontiguousarray(b, dtype=np.complex128).view(np.uint64)
    return a.shape == b.shape and bool(np.all(a == b))


def assert_streams_equal(gsim, osim, nblocks, where):
    for j in range(nblocks):
        g = gsim.export_block(j)
        o = osim.export_block(j)
        if g != o:
            k = next((i for i in range(min(len(g), len(o))) if g[i] != o[i]),
                     min(len(g), len(o)))
            raise AssertionError("%s: block %d differs (len gpu %d oracle %d, first "
                                 "byte %d)" % (where, j, len(g), len(o), k))


def test_rsqrt_is_correctly_rounded(A):
    say("rsqrt self-test, 2e6 inputs")
    rng = np.random.default_rng(1)
    x = np.concatenate([
        1.0 + rng.normal(scale=1e-12, size=500000),
        1.0 + rng.normal(scale=1e-6, size=500000),
        np.exp(rng.uniform(-700, 700, size=500000)),
        rng.uniform(0, 4, size=500000)])
    want = 1.0 / np.sqrt(x)
    got = A.debug_rsqrt(x)
    bad = np.nonzero(got.view(np.uint64) != want.view(np.uint64))[0]
    assert bad.size == 0, (x[bad[:5]], got[bad[:5]], want[bad[:5]])


@pytest.mark.parametrize("n,b,x", [(12, 8, 0xABC), (10, 10, 0x3FF), (9, 6, 5)])
def test_basis_state_streams(A, n, b, x):
    say("basis", n, b, x)
    lad = I.default_ladder(1e-4)
    g = A.Sim(n, b, 1e-4)
    g.set_basis(x)
    o = orc.OracleSim(n, b, lad, 4.0)
    o.set_basis(x)
    assert_streams_equal(g, o, 1 << (n - b), "basis")
    assert same_bits(g.amplitudes(), o.amplitudes())


def test_qft12_streams_after_every_gate(A):
    """The 12-qubit QFT workload (16 blocks of 2^8, delta 1e-4, default
    ladder): all 16 block streams byte-identical after each of 84 gates."""
    w = I.qft12_workload()
    n, b = w["n"], w["b"]
    say("qft12 basis", w["basis"])
    g = A.Sim(n, b, 1e-4)
    g.set_basis(w["basis"])
    o = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    o.set_basis(w["basis"])
    for k, gate in enumerate(w["gates"]):
        g.apply(gate)
        o.apply(gate)
        assert_streams_equal(g, o, 1 << (n - b), "gate %d %s" % (k, gate[:3]))
    assert same_bits(g.amplitudes(), o.amplitudes())
    sg, so = g.stats(), o.stats()
    assert sg["normsq"] == so["normsq"] and sg["scale"] == so["scale"]
    assert sg["resident_bytes"] == so["resident_bytes"]
    assert sg["min_ratio"] == so["min_ratio"]
    assert sg["level_hist"] == so["level_hist"]


def test_qft12_fixed_bound(A):
    w = I.qft12_workload()
    n, b = w["n"], w["b"]
    say("qft12 fixed bound 1e-4")
    g = A.Sim(n, b, 1e-4, ladder=[1e-4], theta=4.0)
    g.set_basis(w["basis"])
    o = orc.OracleSim(n, b, [1e-4], 4.0)
    o.set_basis(w["basis"])
    g.run(w["gates"])
    o.run(w["gates"])
    assert_streams_equal(g, o, 1 << (n - b), "end")


@pytest.mark.parametrize("eb,theta,fixed", [(1e-3, 4.0, False), (1e-3, 32.0, False),
                                             (1e-4, 8.0, False), (1e-4, 16.0, False),
                                             (1e-5, 32.0, False), (1e-3, 4.0, True),
                                             (1e-5, 4.0, True)])
def test_qft12_error_bounds_and_thresholds(A, eb, theta, fixed):
    """The error-bound / threshold grid of the QFT runs at 12 qubits: streams
    after every gate, the level histogram and the ratios equal the oracle's
    (the grid reaches every ladder level: thresholds of 32 push most blocks
    to the last one)."""
    w = I.qft12_workload()
    n, b = w["n"], w["b"]
    lad = [eb] if fixed else I.default_ladder(eb)
    say("qft12", "fixed" if fixed else "aalc", eb, theta)
    g = A.Sim(n, b, eb, ladder=lad, theta=theta)
    g.set_basis(w["basis"])
    o = orc.OracleSim(n, b, lad, theta)
    o.set_basis(w["basis"])
    for k, gate in enumerate(w["gates"]):
        g.apply(gate)
        o.apply(gate)
        assert_streams_equal(g, o, 1 << (n - b), "gate %d" % k)
    sg, so = g.stats(), o.stats()
    assert sg["level_hist"] == so["level_hist"] and sg["min_ratio"] == so["min_ratio"]
    assert sg["collapsed"] == so["collapsed"] and sg["normsq"] == so["normsq"]


def test_bulk_rounds_grover21_small_grid(A):
    """A grid of 64 workgroups over 1024 units: the pass, the one-value pass
    and the mean pre-pass take their units in bulk rounds of 4 (zero units
    and one-value units settled one per thread).  Streams after every gate
    equal the oracle's."""
    n, b, m, it = 21, 14, 0x15A3C, 2
    gates = I.grover(n, m, it)
    say("bulk rounds: grover", n, "grid 64")
    g = A.Sim(n, b, 1e-5)
    g.set_grid(64)
    g.set_basis(0)
    o = orc.OracleSim(n, b, I.default_ladder(1e-5), 4.0)
    assert g.export_state() == o.export_state()
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        assert g.export_state() == o.export_state(), "gate %d" % k
    sg, so = g.stats(), o.stats()
    assert sg["normsq"] == so["normsq"] and sg["level_hist"] == so["level_hist"]


@pytest.mark.parametrize("n", [20, 21])
def test_bulk_rounds_sparse_random_n20(A, n):
    """A sparse state on a grid of 64 workgroups: a basis state opened on a
    few high qubits, then gates of every kind.  n = 20 (512 units) runs the
    one-unit kernel looping over them on 63 workgroups; n = 21 (1024 units)
    runs bulk rounds of 8 units, where the basis encode and the zero units go
    through the per-thread path."""
    b = 12
    rng = np.random.default_rng(20)
    gates = [I.h(q) for q in (n - 1, 16, 12, 3)] + random_gates(n, 30, rng)
    x = int(rng.integers(0, 1 << n))
    say("sparse random n=%d grid 64 basis" % n, x)
    g = A.Sim(n, b, 1e-4)
    g.set_grid(64)
    g.set_basis(x)
    o = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    o.set_basis(x)
    assert g.export_state() == o.export_state()
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        assert g.export_state() == o.export_state(), "gate %d %s" % (k, gate[:3])


@pytest.mark.parametrize("ladder", [None, [1e-4]])
def test_bulk_rounds_one_value_planes_every_gate_kind(A, ladder):
    """Bulk rounds (n = 21, grid 64: 1024 units, 8 per round) over planes of
    one value: the uniform superposition, then gates of every kind whose
    qubits are all at or above s = 10 (one-value planes stay one-value
    planes and are settled per thread), mixed with gates on low qubits (full
    path).  Streams after every gate equal the oracle's."""
    n, b = 21, 12
    rng = np.random.default_rng(33)
    hi = lambda: int(rng.integers(10, n))
    gates = [I.h(q) for q in range(n)]
    for rep in range(2):
        a, c = hi(), hi()
        while c == a:
            c = hi()
        gates += [I.u_gate(hi(), random_unitary(rng)), I.x(hi()), I.cu(a, c, random_unitary(rng)),
                  I.swap(a, c), I.diag1(hi(), math.cos(0.3), math.sin(0.3)),
                  I.cphase(a, c, 1.1), I.cz(a, c), I.phase_flip(int(rng.integers(0, 1 << n))),
                  I.diffuse()]
        if rep == 0:
            gates += [I.u_gate(3, random_unitary(rng)), I.cz(2, 15)]
    lad = I.default_ladder(1e-4) if ladder is None else ladder
    say("bulk rounds: one-value planes, ladder", lad)
    g = A.Sim(n, b, 1e-4, ladder=ladder, theta=4.0)
    g.set_grid(64)
    g.set_basis(0)
    o = orc.OracleSim(n, b, lad, 4.0)
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        assert g.export_state() == o.export_state(), "gate %d %s" % (k, gate[:3])


CASES = [
    # n, b, ladder, theta, ngates, seed
    (9, 7, [0.0], 4.0, 60, 1),
    (10, 8, [0.0, 1e-6, 1e-4], 8.0, 60, 2),
    (11, 11, [1e-5], 1.0, 40, 3),
    (12, 9, [0.0, 1e-9, 1e-7, 1e-5, 1e-3], 4.0, 60, 4),
    (8, 6, [0.0, 1e-3, 1e-2], 32.0, 60, 5),
    (13, 12, [0.0, 1e-8, 1e-6], 2.0, 30, 6),
    # one segment per state (units of a single segment)
    (8, 8, [0.0, 1e-6, 1e-4], 4.0, 40, 7),
    (6, 6, [0.0, 1e-3], 8.0, 30, 8),
]


@pytest.mark.parametrize("n,b,lad,theta,ng,seed", CASES)
def test_random_gates_every_kind(A, n, b, lad, theta, ng, seed):
    """Random gates of every kind (in-segment, segment-pair and block-pair
    couplings, diagonal, swap, Grover operators) on a superposition."""
    say("random", n, b, lad, theta, ng, seed)
    rng = np.random.default_rng(seed)
    prep = [I.h(q) for q in range(n)] + random_gates(n, 8, rng, [I.G_U])
    gates = prep + random_gates(n, ng, rng)
    g = A.Sim(n, b, 1e-4, ladder=lad, theta=theta)
    o = orc.OracleSim(n, b, lad, theta)
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        if k % 7 == 6 or k == len(gates) - 1:
            assert_streams_equal(g, o, 1 << (n - b), "gate %d kind %d" % (k, gate[0]))
    assert same_bits(g.amplitudes(), o.amplitudes())
    assert g.stats()["level_hist"] == o.stats()["level_hist"]


def test_lossless_unnormalised_equals_uncompressed(A):
    n, b = 11, 8
    say("lossless vs uncompressed", n, b)
    rng = np.random.default_rng(9)
    gates = I.qft(n) + random_gates(n, 80, rng)
    c = A.Sim(n, b, 0.0, normalize=False)
    u = A.Sim(n, b, -1.0)
    c.set_basis(77)
    u.set_basis(77)
    c.run(gates)
    u.run(gates)
    ref = orc.sv_run(n, gates, basis=77)
    assert same_bits(u.amplitudes(), ref)
    assert same_bits(c.amplitudes(), ref)


def test_uncompressed_path_matches_plain_reference(A):
    n = 14
    say("uncompressed", n)
    rng = np.random.default_rng(10)
    gates = [I.h(q) for q in range(n)] + random_gates(n, 120, rng)
    u = A.Sim(n, 12, -1.0)
    u.run(gates)
    assert same_bits(u.amplitudes(), orc.sv_run(n, gates))


def test_amplitude_ranges_probs_and_fidelity(A):
    n, b = 12, 8
    say("ranges/probs/fidelity", n, b)
    w = I.qft12_workload()
    g = A.Sim(n, b, 1e-3)
    o = orc.OracleSim(n, b, I.default_ladder(1e-3), 4.0)
    g.set_basis(w["basis"])
    o.set_basis(w["basis"])
    g.run(w["gates"])
    o.run(w["gates"])
    full = o.amplitudes()
    for first, count in [(0, 1), (5, 300), (255, 2), (1000, 3096), (4095, 1)]:
        assert same_bits(g.amplitudes(first, count), full[first:first + count])
    for qs in ([0], [3, 11], [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11], [7, 2, 9]):
        pg = g.probs(qs)
        po = o.measure_probs(qs)
        assert np.max(np.abs(pg - po)) < 1e-12
    ref = orc.sv_run(n, w["gates"], basis=w["basis"])
    u = A.Sim(n, b, -1.0)
    u.set_basis(w["basis"])
    u.run(w["gates"])
    Fo = orc.fidelity(ref, full, n)
    assert abs(g.fidelity(u) - Fo) < 1e-12
    assert abs(u.fidelity(g) - Fo) < 1e-12
    assert abs(g.fidelity(g) - 1.0) < 1e-12


def test_grover_n16_full_parity(A):
    n, k, b = 16, 5, 12
    m = 0xBEEF
    say("grover", n, k, b)
    gates = I.grover(n, m, k)
    g = A.Sim(n, b, 1e-5)
    o = orc.OracleSim(n, b, I.default_ladder(1e-5), 4.0)
    g.run(gates)
    o.run(gates)
    assert_streams_equal(g, o, 1 << (n - b), "grover")
    p = g.probs(list(range(n)))[m]
    assert abs(p - I.grover_success(n, k)) < 1e-6


@pytest.mark.parametrize("lad,theta", [
    ([1e-3], 4.0),                       # one lossy level
    ([1e-9, 1e-3], 4.0),                 # the finest lossy level suffices
    ([0.0, 1e-9, 1e-6, 1e-3], 1000.0),   # theta above every ratio: the last level,
                                         # lossless and lossy levels sized below it
])
def test_grover_constant_planes_every_level_kind(A, lad, theta):
    """Grover states are made of planes that hold one value; their DIFFUSE
    and PHASE_FLIP passes encode such units from the value alone.  Streams
    after every gate equal the oracle's for lossless, lossy and last-level
    choices (levels below the chosen one sized)."""
    n, k, b = 12, 3, 10
    m = 0x5A5
    say("grover constant planes", lad, theta)
    gates = I.grover(n, m, k)
    g = A.Sim(n, b, lad[-1], ladder=lad, theta=theta)
    o = orc.OracleSim(n, b, lad, theta)
    for q, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        assert_streams_equal(g, o, 1 << (n - b), "gate %d kind %d" % (q, gate[0]))
    assert g.stats()["level_hist"] == o.stats()["level_hist"]
    assert same_bits(g.amplitudes(), o.amplitudes())


def test_amplitude_sum_and_headers_match_oracle(A):
    for name, n, b, lad, x, gates in (
            ("grover", 16, 12, I.default_ladder(1e-5), 0, I.grover(16, 0xBEEF, 3)),
            ("qft12", 12, 8, I.default_ladder(1e-4), 0x5A3, I.qft(12)[:50])):
        say("amplitude sum and headers", name)
        g = A.Sim(n, b, lad[-1])
        o = orc.OracleSim(n, b, lad, 4.0)
        g.set_basis(x)
        o.set_basis(x)
        for k, gate in enumerate(gates):
            g.apply(gate)
            o.apply(gate)
            if k % 7 == 0 or k == len(gates) - 1:
                assert g.amplitude_sum() == o.amplitude_sum(), (name, k)
                hg = g.export_headers()
                ho = b"".join(o.export_block(j)[:32] for j in range(1 << (n - b)))
                assert hg == ho, (name, k)
                # a sub-range of headers
                assert g.export_headers(1, 2) == hg[32:96]
        g.close()
    say("amplitude sum, uncompressed path")
    u = A.Sim(12, 8, -1.0)
    u.set_basis(0x5A3)
    u.run(I.qft(12)[:50])
    a = u.amplitudes()
    S = u.amplitude_sum()
    assert abs(S.real - math.fsum(a.real)) < 1e-12
    assert abs(S.imag - math.fsum(a.imag)) < 1e-12


def test_many_outliers_per_plane(A):
    # Uniform superposition on 8 qubits: every amplitude is 2^-4 exactly.
    # With the single bound delta = 2^-4 each real part sits on a rounding tie
    # (y = 0.5 -> q = 0, error exactly delta), so all 256 scalars of a real
    # plane are outliers: more than the encoder stages, which exercises its
    # re-encode path; with delta = 2^-3 they are quantised exactly (no
    # outliers).  Streams must equal the oracle's.
    n, b = 8, 8
    for lad in ([2.0 ** -4], [2.0 ** -3], [2.0 ** -5, 2.0 ** -4]):
        say("many outliers", lad)
        g = A.Sim(n, b, lad[-1], ladder=lad, theta=4.0)
        o = orc.OracleSim(n, b, lad, 4.0)
        gates = [I.h(q) for q in range(n)] + [I.t_gate(3), I.h(5), I.cz(1, 6)]
        for gate in gates:
            g.apply(gate)
            o.apply(gate)
            assert_streams_equal(g, o, 1, "outliers %s" % lad)
        g.close()


def test_invalid_gates_rejected(A):
    say("invalid gates")
    g = A.Sim(8, 6, 1e-4)
    for bad in [(I.G_U, 8, 0, 0, I.H), (I.G_CZ, 3, 3, 0, I.ZERO8),
                (I.G_PHASE_FLIP, 0, 0, 256, I.ZERO8), (42, 0, 0, 0, I.ZERO8),
                (I.G_SWAP, -1, 2, 0, I.ZERO8)]:
        with pytest.raises(A.SimError) as e:
            g.apply(bad)
        assert e.value.code == A.SIM_EINVAL
    assert g.stats()["passes"] == 0


def test_arena_overflow_rolls_back(A):
    n, b = 12, 8
    say("arena overflow")
    w = I.qft12_workload()
    # lossless QFT grows to ~16 * 4096 bytes; give each arena 24 KiB
    g = A.Sim(n, b, 0.0, arena_bytes=24 << 10)
    o = orc.OracleSim(n, b, [0.0], 4.0)
    g.set_basis(w["basis"])
    o.set_basis(w["basis"])
    done = 0
    with pytest.raises(A.SimError) as e:
        for gate in w["gates"]:
            g.apply(gate)
            g.sync()
            o.apply(gate)
            done += 1
    assert e.value.code == A.SIM_ENOMEM
    # state is the input of the failing gate
    assert g.stats()["passes"] == done
    assert_streams_equal(g, o, 1 << (n - b), "after rollback")


def test_arena_too_small_for_the_basis_state(A):
    say("arena too small for the basis state")
    # 16 blocks of 2^8: the zero planes alone need 16 * 2 * 16 bytes
    with pytest.raises(A.SimError) as e:
        A.Sim(12, 8, 1e-4, arena_bytes=256)
    assert "arena" in str(e.value)
    g = A.Sim(12, 8, 1e-4)
    g.set_basis(7)
    assert abs(g.amplitudes(7, 1)[0] - 1.0) == 0.0


def test_qft24_sampled_parity_and_fidelity(A):
    """The 24-qubit QFT workload (256 blocks of 2^16): every 24th gate the
    inputs of sampled groups are exported and the oracle recomputes those
    groups; final fidelity against the closed form is reported."""
    w = I.qft24_workload()
    n, b = w["n"], w["b"]
    delta = 1e-4
    lad = I.default_ladder(delta)
    say("qft24 basis", w["basis"])
    g = A.Sim(n, b, delta)
    g.set_basis(w["basis"])
    rng = np.random.default_rng(24)
    nb = 1 << (n - b)
    for k, gate in enumerate(w["gates"]):
        if k % 24 == 5:
            sc = g.stats()["scale"]
            mask = 0
            if gate[0] in (I.G_U, I.G_X):
                mask = 1 << gate[1]
            elif gate[0] == I.G_SWAP:
                mask = (1 << gate[1]) | (1 << gate[2])
            mb = mask >> b
            js = sorted(set(int(v) for v in rng.integers(0, nb, 3)) | {0, w["basis"] >> b})
            groups = sorted({min(j, j ^ mb) for j in js})
            before = {j: g.export_block(j) for grp in groups
                      for j in ((grp, grp ^ mb) if mb else (grp,))}
            g.apply(gate)
            for grp in groups:
                o0, o1 = orc.process_group(n, b, 10, lad, 4.0, sc, None, gate, grp,
                                           before[grp], before[grp ^ mb] if mb else None)
                assert o0 == g.export_block(grp), (k, grp)
                if mb:
                    assert o1 == g.export_block(grp ^ mb), (k, grp ^ mb)
        else:
            g.apply(gate)
    kk = np.arange(1 << n)
    x = w["basis"]
    ref = np.exp(2j * np.pi * ((x * kk) % (1 << n)) / (1 << n)) / 2 ** (n / 2)
    got = g.amplitudes()
    F = orc.fidelity(ref, got, n)
    st = g.stats()
    say("qft24 fidelity", F, "min ratio", st["min_ratio"], "levels", st["level_hist"])
    assert F > 0.99


def test_wide_reduction_many_blocks(A):
    """A state of more than 4096 blocks (n = 19, b = 6: 8192 blocks) takes
    the reduction over several workgroups (runs of 1024 blocks combined by
    the last one): N^2, s, resident bytes, ratios, the level histogram and
    every stream equal the oracle's after each gate, through replays, a
    DIFFUSE (whose pre-pass uses the same scratch) and a PHASE_FLIP."""
    n, b = 19, 6
    rng = np.random.default_rng(19)
    gates = [I.h(q) for q in range(0, n, 3)]
    for _ in range(10):
        a_, c_ = (int(v) for v in rng.choice(n, 2, replace=False))
        gates += [I.cphase(a_, c_, float(rng.uniform(0, 6.3))), I.h(int(rng.integers(0, n)))]
    gates += [I.phase_flip(0x2B5A3), I.diffuse(), I.swap(2, 17), I.t_gate(18)]
    say("wide reduction n=19 b=6", len(gates), "gates")
    g = A.Sim(n, b, 1e-4)
    g.set_basis(0x1D2F3)
    o = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    o.set_basis(0x1D2F3)
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        sg, so = g.stats(), o.stats()
        for key in ("normsq", "scale", "resident_bytes", "min_ratio", "level_hist"):
            assert sg[key] == so[key], (k, key, sg[key], so[key])
        if k % 5 == 4 or k == len(gates) - 1:
            assert g.export_state() == o.export_state(), k
    assert g.stats()["replays"] > 0
    g.close()
