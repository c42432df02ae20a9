"""Checkpoint and resume on the GPU, through the C ABI (needs an MI355X).

Bar: a whole-state export is byte-identical to the oracle's streams; a state
imported from the oracle's or the GPU's own checkpoint continues with block
streams byte-identical to the uninterrupted run after every gate; malformed
checkpoints are rejected with SIM_EINVAL and leave the state unchanged (the
same cases the oracle rejects); an evicted serving request resumes to the
same final state as when it runs alone.  Also the quantiser's code-range
edge (codes +-(2^30 - 0.5) and +-(2^30 - 1.75) of a non-unitary gate)
against the oracle.  Every case prints what it runs before touching the GPU.
"""
import struct
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1811_05140_amd import inputs as I

pytestmark = pytest.mark.gpu

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_checkpoint import corruptions, records  # noqa: E402
from test_gpu_parity import random_gates  # noqa: E402


@pytest.fixture(scope="module")
def A():
    from paper_1811_05140_amd import aalcsim
    return aalcsim


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def test_export_state_equals_oracle_streams(A):
    w = I.qft12_workload()
    n, b = w["n"], w["b"]
    say("export_state qft12 at gates 0, 30, 84")
    g = A.Sim(n, b, 1e-4)
    g.set_basis(w["basis"])
    o = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    o.set_basis(w["basis"])
    cuts = [0, 30, len(w["gates"])]
    done = 0
    for c in cuts:
        g.run(w["gates"][done:c])
        o.run(w["gates"][done:c])
        done = c
        ck = g.export_state()
        assert ck == o.export_state(), c
        assert len(ck) == g.stats()["resident_bytes"]
        buf = np.zeros(len(ck) + 64, dtype=np.uint8)
        assert g.export_state(out=buf) == len(ck) and bytes(buf[:len(ck)]) == ck


@pytest.mark.parametrize("source", ["gpu", "oracle"])
def test_resume_qft12_every_gate_equal_to_uninterrupted(A, source):
    w = I.qft12_workload()
    n, b, cut = w["n"], w["b"], 37
    say("resume qft12 from", source, "at gate", cut)
    o = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    o.set_basis(w["basis"])
    o.run(w["gates"][:cut])
    if source == "gpu":
        g0 = A.Sim(n, b, 1e-4)
        g0.set_basis(w["basis"])
        g0.run(w["gates"][:cut])
        ck = g0.export_state()
        g0.close()
    else:
        ck = o.export_state()
    g = A.Sim(n, b, 1e-4)
    g.apply(I.h(3))  # a state to be replaced
    assert g.import_state(ck) == 0
    assert g.export_state() == ck
    sg, so = g.stats(), o.stats()
    assert sg["normsq"] == so["normsq"] and sg["scale"] == so["scale"]
    assert sg["passes"] == 0 and sg["resident_bytes"] == so["resident_bytes"]
    for k, gate in enumerate(w["gates"][cut:]):
        g.apply(gate)
        o.apply(gate)
        assert g.export_state() == o.export_state(), "gate %d" % (cut + k)
    a, b_ = g.amplitudes(), o.amplitudes()
    assert np.array_equal(a.view(np.uint64), b_.view(np.uint64))


@pytest.mark.parametrize("n,b,eb,seed", [(16, 12, 1e-4, 1), (14, 10, 0.0, 2),
                                         (13, 7, 1e-3, 3)])
def test_resume_random_circuits_all_gate_kinds(A, n, b, eb, seed):
    """Several segments per block (b = 12), lossless-only, and small
    segments (b = 7); gates of every kind, cut in the middle; the oracle's
    checkpoint imported on the GPU continues bit for bit."""
    rng = np.random.default_rng(seed)
    gates = [I.h(q) for q in range(n)] + random_gates(n, 40, rng)
    cut = 25
    say("resume random", n, b, eb, seed, "cut", cut)
    lad = I.default_ladder(eb) if eb > 0 else [0.0]
    o = orc.OracleSim(n, b, lad, 4.0)
    o.set_basis(int(rng.integers(0, 1 << n)))
    o.run(gates[:cut])
    g = A.Sim(n, b, eb)
    assert g.import_state(o.export_state()) == 0
    for k, gate in enumerate(gates[cut:]):
        g.apply(gate)
        o.apply(gate)
    assert g.export_state() == o.export_state()
    assert np.array_equal(g.amplitudes().view(np.uint64), o.amplitudes().view(np.uint64))


def test_resume_grover16_constant_planes(A):
    """Grover states (planes of one value, zero records) through a
    checkpoint: the DIFFUSE mean pre-pass and the one-value-plane pass run
    on imported records."""
    n, m, it = 16, 0x9C3F, 3
    gates = I.grover(n, m, it)
    cut = n + 3
    say("resume grover16 at", cut)
    o = orc.OracleSim(n, 12, I.default_ladder(1e-5), 4.0)
    o.run(gates[:cut])
    g = A.Sim(n, 12, 1e-5)
    assert g.import_state(o.export_state()) == 0
    g.run(gates[cut:])
    o.run(gates[cut:])
    assert g.export_state() == o.export_state()
    sg, so = g.amplitude_sum(), o.amplitude_sum()
    assert np.array_equal(np.array([sg.real, sg.imag]).view(np.uint64),
                          np.array([so.real, so.imag]).view(np.uint64))


def test_corrupted_checkpoints_rejected_state_unchanged(A):
    w = I.qft12_workload()
    n, b = w["n"], w["b"]
    o = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    o.set_basis(w["basis"])
    o.run(w["gates"][:70])
    ck = o.export_state()
    g = A.Sim(n, b, 1e-4)
    g.set_basis(w["basis"])
    g.run(w["gates"][:10])
    before = g.export_state()
    for name, bad in corruptions(ck, 1 << (n - b)):
        say("corrupted checkpoint:", name)
        with pytest.raises(A.SimError) as e:
            g.import_state(bad)
        assert e.value.code == A.SIM_EINVAL, name
        assert g.export_state() == before, name
    # the sim still works: finish the circuit from gate 10 like the oracle
    say("continue after rejections")
    o2 = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    o2.set_basis(w["basis"])
    o2.run(w["gates"])
    g.run(w["gates"][10:])
    assert g.export_state() == o2.export_state()
    # another ladder: the bounds of the streams are not its levels
    g2 = A.Sim(n, b, 1e-3)
    with pytest.raises(A.SimError):
        g2.import_state(ck)


def test_record_level_defects_rejected(A):
    """The record checks of the import kernels: a first residual that is not
    0, an outlier index outside the plane or out of order, a lossy chunk
    wider than 32 bits, an outlier in a lossless plane; each also rejected by
    the oracle."""
    b = 6
    x = np.zeros(2 << b)
    x[0::2][:10] = [0.0, 0.2, 0.5, 0.7, 1.0, -0.2, -0.6, 3.0, 0.75, 1e12]
    st = orc.encode_block(x, b, b, 0.25, 0)
    (pos, anc, pw, no), _ = records(st)
    pay = pos + 16 + 8
    outl = pay + 8 * pw

    def bad(off, fmt, val, src=st):
        s = bytearray(src)
        struct.pack_into(fmt, s, off, val)
        return bytes(s)

    wide = bytearray(st[:outl] + bytes(8 * 29) + st[outl:])
    struct.pack_into("<B", wide, pos + 16, 33)
    struct.pack_into("<I", wide, pos + 8, 33)
    struct.pack_into("<I", wide, 12, len(wide))
    cases = [("c_0 != 0", bad(pay, "<Q", struct.unpack_from("<Q", st, pay)[0] | 1)),
             ("outlier index outside", bad(outl, "<I", 64)),
             ("outliers not ascending", bad(outl + 16, "<I", 0)),
             ("lossy chunk of 33 bits", bytes(wide))]
    say("record defects: valid stream first")
    g = A.Sim(b, b, 0.25, ladder=[0.25], theta=4.0)
    o = orc.OracleSim(b, b, [0.25], 4.0)
    assert g.import_state(st) == 0 and o.import_state(st) == 0
    assert g.export_state() == st
    for name, c in cases:
        say("record defect:", name)
        with pytest.raises(ValueError):
            o.import_state(c)
        with pytest.raises(A.SimError) as e:
            g.import_state(c)
        assert e.value.code == A.SIM_EINVAL, name
        assert g.export_state() == st, name
    y = np.zeros(2 << b)
    y[2] = 1.5
    ls = orc.encode_block(y, b, b, 0.0, 0)
    (p0, _, _, _), (p1, _, _, _) = records(ls)
    s = bytearray(ls[:p1] + struct.pack("<IId", 3, 0, 2.0) + ls[p1:])
    struct.pack_into("<I", s, p0 + 12, 1)
    struct.pack_into("<I", s, 12, len(s))
    struct.pack_into("<I", s, 8, 1)
    say("record defect: outlier in a lossless plane")
    gl = A.Sim(b, b, 0.0)
    with pytest.raises(A.SimError):
        gl.import_state(bytes(s))
    assert gl.import_state(ls) == 0 and gl.export_state() == ls


def test_import_all_zero_state_reports_collapsed(A):
    n, b = 7, 6
    st = orc.encode_block(np.zeros(2 << b), b, b, 0.0, 0)
    say("import all-zero state")
    g = A.Sim(n, b, 0.0)
    assert g.import_state(st + st) == A.SIM_ECOLLAPSED
    s = g.stats()
    assert s["collapsed"] == 1 and s["normsq"] == 0.0 and s["scale"] == 1.0


def test_checkpoint_qft24_full_size_resume(A):
    """QFT-24 (256 blocks of 2^16, eb 1e-4): checkpoint after 150 gates,
    resume in a second sim, finish both: identical whole-state streams and
    the same fidelity to the closed-form QFT."""
    w = I.qft24_workload()
    n, b, cut = w["n"], w["b"], 150
    say("qft24 checkpoint at", cut)
    g = A.Sim(n, b, 1e-4)
    g.set_basis(w["basis"])
    g.run(w["gates"][:cut])
    ck = g.export_state()
    assert len(ck) == g.stats()["resident_bytes"]
    # sampled blocks decode (oracle) to the GPU's unnormalised amplitudes
    s = g.stats()["scale"]
    starts = [0]
    for _ in range(1 << (n - b)):
        starts.append(starts[-1] + struct.unpack_from("<I", ck, starts[-1] + 12)[0])
    assert starts[-1] == len(ck)
    for j in (0, 77, 255):
        blk = ck[starts[j]:starts[j + 1]]
        assert blk == g.export_block(j)
        xh = np.ascontiguousarray(orc.decode_block(blk)).view(np.float64)
        amp = np.zeros(2 << b)  # interleaved (re, im) as the library writes them
        A.check(A.lib.sim_get_amplitudes(g.h, j << b, 1 << b, A._dp(amp)), True)
        want = xh * s
        assert np.array_equal(amp.view(np.uint64), want.view(np.uint64)), j
    r = A.Sim(n, b, 1e-4)
    assert r.import_state(ck) == 0
    say("qft24 finish both")
    g.run(w["gates"][cut:])
    r.run(w["gates"][cut:])
    assert g.export_state() == r.export_state()
    assert g.fourier_fidelity(w["basis"]) == r.fourier_fidelity(w["basis"])
    assert r.fourier_fidelity(w["basis"]) > 0.999


def test_serving_eviction_resumes_to_the_same_state(A):
    """Requests whose first arena is far too small overflow mid-circuit; the
    executor checkpoints them to host memory and resumes them with a larger
    arena; each final state equals the one of a run alone with the default
    arena."""
    from paper_1811_05140_amd import serve as SV
    specs = [
        {"id": 0, "t1": 0.0, "kind": "qft", "n": 21, "eb": 1e-4, "basis": 0x1ABCD,
         "gates": I.qft(21)},
        {"id": 1, "t1": 0.0, "kind": "qft", "n": 12, "eb": 1e-3, "basis": 0x5A5,
         "gates": I.qft(12)},
        {"id": 2, "t1": 0.1, "kind": "qft", "n": 20, "eb": 1e-5, "basis": 0x777,
         "gates": I.qft(20)},
    ]
    say("serving with eviction: 3 requests, first arena x0.03")
    ex = SV.GpuExecutor(A, max_slots=3, gates_per_step=8, arena_scale=0.03)
    budget = 3 * SV.reservation_bytes(21, 14)
    reqs, summ = SV.serve(specs, ex, budget, 3, 8, rate=100.0)
    say(summ)
    assert summ["restarts"] >= 1
    assert any(r.resume > 0 for r in reqs)
    for r in reqs:
        b = ex.block_log2(r)
        sim = A.Sim(r.n, b, r.eb, arena_bytes=SV.arena_bytes(r.n))
        sim.set_basis(r.basis)
        sim.run(specs[r.rid]["gates"])
        assert SV.signature(sim, r) == r.result["signature"], r.rid
        assert r.result["fidelity"] > 0.99
        sim.close()


def test_quantiser_code_range_edge_matches_oracle(A):
    """A non-unitary gate writes values whose codes sit at the edge of the
    quantiser's range: y = +-(2^30 - 0.5) (out of range: outliers, code 0)
    next to each other with opposite signs, and y = +-(2^30 - 1.75) (codes
    +-(2^30 - 2), residual -(2^31 - 4)).  Streams equal the oracle's."""
    b = 6
    xa = (2.0 ** 30 - 0.5) / 2
    xb = (2.0 ** 30 - 1.75) / 2
    for name, u01, u11 in (("xa", -xa, xa), ("xb", xb, -xb), ("mixed", -xa, xb)):
        say("quantiser edge", name)
        u = (0.0, 0.0, u01, 0.0, 0.0, 0.0, u11, 0.0)
        g = A.Sim(b, b, 0.25, ladder=[0.25], theta=4.0, normalize=False)
        g.set_basis(1)
        o = orc.OracleSim(b, b, [0.25], 4.0, normalize=False)
        o.set_basis(1)
        gate = I.u_gate(0, u)
        g.apply(gate)
        o.apply(gate)
        assert g.export_block(0) == o.export_block(0), name
        # the next gate decodes those records and re-encodes
        g.apply(I.x(0))
        o.apply(I.x(0))
        assert g.export_block(0) == o.export_block(0), name
