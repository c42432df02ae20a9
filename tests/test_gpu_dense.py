"""Full-size and dense-block parity on the GPU (needs an MI355X).

* The 24-qubit QFT workload, every gate: the SHA-256 of the whole state
  (every block stream) after the basis encode and after each of the 312 gates
  equals the oracle's, stored in tests/golden/qft24_digests.json by
  tests/golden/make_qft24_digests.py (oracle only), together with N^2 and the
  level histogram, for the default ladder at (1e-4, theta 4), (1e-3, 16) and
  (1e-5, 16), and at (1e-4, 4) with both Sec. V shortcuts.
* Blocks of 2^17 and 2^18 amplitudes (128 and 256 segments per block, the
  block-wide decision instance for large blocks) in dense random states,
  every gate kind, theta 4 and 16 so that replays and escalations occur:
  whole-state streams equal to the oracle's after every gate, through
  sim_apply_gate and through sim_batch_apply.
* Marginal probabilities of a dense random state (not uniform) under a
  non-monotone qubit list, against the oracle.
* Planes with whole steps of +0, -0 and values below some ladder bounds
  (what the codec skips), every gate.
"""
import hashlib
import json
import math
import os
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1811_05140_amd import inputs as I

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def A():
    from paper_1811_05140_amd import aalcsim
    return aalcsim


@pytest.fixture(scope="module", autouse=True)
def oracle_threads():
    orc.set_threads(min(os.cpu_count() or 1, 16))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def _digests():
    with open(os.path.join(HERE, "golden", "qft24_digests.json")) as f:
        return json.load(f)["configs"]


def _cfg_id(c):
    return "eb%g-theta%g-sc%d" % (c["delta"], c["theta"], c.get("shortcut", 0))


@pytest.mark.parametrize("cfg", _digests(), ids=_cfg_id)
def test_qft24_every_gate_digests(A, cfg):
    w = I.qft24_workload()
    n, b = w["n"], w["b"]
    assert (n, b, w["basis"], len(w["gates"])) == (cfg["n"], cfg["b"], cfg["basis"],
                                                  cfg["gates"])
    lad = cfg["ladder"]
    assert lad == I.default_ladder(cfg["delta"])
    L = len(lad)
    say("qft24 every gate, delta", cfg["delta"], "theta", cfg["theta"])
    g = A.Sim(n, b, cfg["delta"], ladder=lad, theta=cfg["theta"])
    g.set_shortcut(cfg.get("shortcut", 0))
    g.set_basis(w["basis"])

    def check(k, where):
        got = hashlib.sha256(g.export_state()).hexdigest()
        st = g.stats()
        assert got == cfg["sha256_after_gate"][k], where
        assert st["normsq"] == float.fromhex(cfg["normsq_after_gate"][k]), where
        assert st["level_hist"][:L] == cfg["level_hist_after_gate"][k], where

    check(0, "basis encode")
    for k, gate in enumerate(w["gates"]):
        g.apply(gate)
        check(k + 1, "gate %d %s" % (k, gate[:3]))
    g.close()


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


def dense_circuit(n, ng, seed):
    """A dense state (H on every qubit, then random single-qubit unitaries),
    then random gates of every kind; some gates touch the top qubits so
    that block pairs couple."""
    rng = np.random.default_rng(seed)
    prep = [I.h(q) for q in range(n)]
    prep += [I.u_gate(int(q), unitary(rng)) for q in rng.choice(n, 6, replace=False)]
    body = random_gates(n, ng, rng)
    body += [I.u_gate(n - 1, unitary(rng)), I.swap(0, n - 1), I.cu(n - 2, 3, unitary(rng))]
    return prep + body


DENSE = [
    # n, b, delta, theta, gates, seed
    (18, 17, 1e-4, 4.0, 24, 181),
    (18, 17, 1e-4, 16.0, 24, 182),
    (19, 18, 1e-5, 4.0, 18, 191),
    (19, 17, 1e-3, 16.0, 18, 192),
]


@pytest.mark.parametrize("n,b,delta,theta,ng,seed", DENSE)
def test_dense_large_blocks_every_gate(A, n, b, delta, theta, ng, seed):
    gates = dense_circuit(n, ng, seed)
    lad = I.default_ladder(delta)
    say("dense large blocks", n, b, delta, theta, len(gates), seed)
    g = A.Sim(n, b, delta, ladder=lad, theta=theta)
    o = orc.OracleSim(n, b, lad, theta)
    esc = rep = 0
    for k, gate in enumerate(gates):
        g.apply(gate)
        o.apply(gate)
        assert g.export_state() == o.export_state(), "gate %d %s" % (k, gate[:3])
    sg, so = g.stats(), o.stats()
    assert sg["level_hist"] == so["level_hist"]
    assert sg["normsq"] == so["normsq"] and sg["scale"] == so["scale"]
    esc, rep = sg["escalations"], sg["replays"]
    say("levels", sg["level_hist"], "replays", rep, "escalations", esc)
    # the cases are chosen so that mispredicted and escalated blocks occur
    assert rep + esc > 0
    g.close()


def test_dense_large_blocks_batched(A):
    """The same kind of states advanced together by sim_batch_apply, one
    gate per pass, against the oracle after every call."""
    specs = [(18, 17, 1e-4, 4.0, 183), (19, 18, 1e-5, 16.0, 193), (19, 17, 1e-3, 4.0, 194)]
    circs = [dense_circuit(n, 14, seed) for n, _, _, _, seed in specs]
    say("batched dense large blocks", [(n, b) for n, b, _, _, _ in specs])
    sims, orcs = [], []
    for n, b, delta, theta, _ in specs:
        lad = I.default_ladder(delta)
        sims.append(A.Sim(n, b, delta, ladder=lad, theta=theta))
        orcs.append(orc.OracleSim(n, b, lad, theta))
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
        say("passes", start, start + len(passes))
        batch.apply(sims, passes, use_graph=(start // 4) % 2 == 1)
        for k in range(len(specs)):
            assert sims[k].export_state() == orcs[k].export_state(), (start, k)
    for k in range(len(specs)):
        assert sims[k].stats()["level_hist"] == orcs[k].stats()["level_hist"]
    batch.close()


def test_probs_of_a_dense_random_state(A):
    n, b = 13, 9
    rng = np.random.default_rng(131)
    gates = [I.h(q) for q in range(n)] + random_gates(n, 60, rng)
    gates = [gt for gt in gates if gt[0] != I.G_DIFFUSE]
    say("probs of a random state", n, b, len(gates))
    g = A.Sim(n, b, 1e-5)
    o = orc.OracleSim(n, b, I.default_ladder(1e-5), 4.0)
    g.run(gates)
    o.run(gates)
    assert g.export_state() == o.export_state()
    for qs in ([5, 0, 11], [12, 3], [2, 9, 4, 7], [8]):
        pg = g.probs(qs)
        po = o.measure_probs(qs)
        assert np.max(np.abs(po - np.full_like(po, po.mean()))) > 1e-4  # not uniform
        assert np.max(np.abs(pg - po)) < 1e-12, qs


@pytest.mark.parametrize("theta", [4.0, 32.0])
def test_steps_of_zeros_and_small_values(A, theta):
    """Planes whose 256-scalar steps are all +0, all -0 or hold values below
    some ladder bounds but not others (the codec's step skips): a superposition
    over qubits 0..7 only, then small rotations that move a little amplitude
    (1e-9 .. 1e-3 of it) into the empty steps, diagonal gates that turn +0
    into -0, and the reverse; streams after every gate equal the oracle's."""
    n, b = 12, 10
    gates = [I.h(q) for q in range(8)]
    for k, eps in enumerate([1e-9, 3e-7, 2e-6, 5e-5, 1e-3]):
        c, s_ = math.cos(eps), math.sin(eps)
        gates.append(I.u_gate(8 + (k % 2), (c, 0.0, -s_, 0.0, s_, 0.0, c, 0.0)))
        gates.append(I.diag1(10 + (k % 2), -1.0, 0.0))       # +0 -> -0 where the bit is 1
        gates.append(I.cphase(k % 8, 9, math.pi * (k + 1) / 7))
        gates.append(I.u_gate(11, (0.0, 0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0)))
    gates.append(I.h(9))
    say("step skips", n, b, theta, len(gates))
    for lad in (I.default_ladder(1e-4), I.default_ladder(1e-3), [0.0]):
        g = A.Sim(n, b, lad[-1], ladder=lad, theta=theta)
        o = orc.OracleSim(n, b, lad, theta)
        for k, gate in enumerate(gates):
            g.apply(gate)
            o.apply(gate)
            assert g.export_state() == o.export_state(), (lad, k, gate[:3])
        assert g.stats()["level_hist"] == o.stats()["level_hist"]
        g.close()
