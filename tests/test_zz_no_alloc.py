"""The allocation-free marginals entry point (sim_measure_probs_noalloc)
against sim_measure_probs, through the C ABI, on two calls in a row, the
second with a smaller state and fewer qubits (so bins left over from the
first call must not leak into the second)."""
import math
import sys

import numpy as np
import pytest

from paper_1811_05140_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    from paper_1811_05140_amd import aalcsim
    return aalcsim


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def state(A, n, b, eb, seed):
    rng = np.random.default_rng(seed)
    sim = A.Sim(n, b, eb)
    gates = [I.h(q) for q in range(n)]
    for _ in range(3 * n):
        q = int(rng.integers(0, n))
        phi = rng.uniform(0, 2 * math.pi)
        gates.append(I.diag1(q, math.cos(phi), math.sin(phi)))
        c, t = (int(v) for v in rng.choice(n, 2, replace=False))
        gates.append(I.cphase(c, t, rng.uniform(0, 2 * math.pi)))
        gates.append(I.u_gate(int(rng.integers(0, n)), (0.6, 0.0, 0.8, 0.0, 0.8, 0.0, -0.6, 0.0)))
    sim.run(gates)
    return sim


def test_noalloc_probs_match_the_allocating_entry_point(A):
    cases = [(14, 10, 1e-5, [0, 13, 5, 7, 2, 9, 11, 1, 3, 12, 4, 6], 1),
             (10, 8, 1e-4, [9, 2, 4], 2),
             (12, 12, -1.0, [3, 0, 11, 7, 5], 3)]
    for n, b, eb, qs, seed in cases:
        say("noalloc probs", n, b, eb, len(qs))
        sim = state(A, n, b, eb, seed)
        want = sim.probs(qs)
        got = sim.probs_noalloc(qs)
        assert got.shape == want.shape
        assert np.max(np.abs(got - want)) < 1e-12, (n, qs)
        assert abs(got.sum() - 1.0) < 1e-9
        again = sim.probs_noalloc(qs)
        assert np.max(np.abs(again - want)) < 1e-12
        sim.close()


def test_noalloc_probs_rejects_more_than_16_qubits(A):
    sim = A.Sim(18, 12, 1e-4)
    with pytest.raises(A.SimError) as e:
        sim.probs_noalloc(list(range(17)))
    assert e.value.code == A.SIM_EINVAL
    p = sim.probs_noalloc(list(range(16)))
    assert p[0] == 1.0 and p[1:].sum() == 0.0
    sim.close()
