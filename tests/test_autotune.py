"""Autotuner logic on the CPU (a synthetic timing function stands in for the
GPU), and on the GPU: a real tuning run, and the grid knob leaving results
unchanged."""
import os

import pytest

from paper_1811_05140_amd import autotune as T
from paper_1811_05140_amd import inputs as I


def test_candidates_respect_n():
    assert {b for b, _ in T.candidates(28)} == set(range(12, 21))
    assert {b for b, _ in T.candidates(14)} == {12, 13, 14}
    assert {b for b, _ in T.candidates(10)} == {10}  # below the range: b = n
    assert len(T.candidates(16)) == 5 * len(T.GRIDS)


def test_pick_and_tie_break():
    r = [{"b": 12, "grid": 2048, "gates_per_s": 10.0, "resident_bytes": 500},
         {"b": 14, "grid": 1024, "gates_per_s": 12.0, "resident_bytes": 900},
         {"b": 16, "grid": 1024, "gates_per_s": 12.0, "resident_bytes": 700}]
    assert T.pick(r)["b"] == 16
    with pytest.raises(ValueError):
        T.pick([])


def test_tune_table_round_trip(tmp_path):
    lad = I.default_ladder(1e-4)
    calls = []

    def fake(b, grid):
        calls.append((b, grid))
        # fastest at b = 15 with the middle grid
        return 1000.0 - 10 * abs(b - 15) - abs(grid - 2048) / 1024.0, 1 << b

    e = T.tune(18, lad, 4.0, fake)
    assert (e["b"], e["grid"]) == (15, 2048)
    assert calls == T.candidates(18)
    path = os.path.join(str(tmp_path), "t.json")
    T.save_table({T.key(18, lad, 4.0): e}, path, {"note": "test"})
    entries = T.load_table(path)
    assert T.lookup(entries, 18, lad, 4.0) == (15, 2048)
    assert T.lookup(entries, 19, lad, 4.0) is None
    assert T.lookup(entries, 18, I.default_ladder(1e-5), 4.0) is None
    assert T.load_table(os.path.join(str(tmp_path), "missing.json")) == {}


def test_committed_table_is_well_formed():
    entries = T.load_table()
    for k, e in entries.items():
        n = int(k.split()[0][2:])
        assert 6 <= e["b"] <= min(20, n) and e["grid"] in T.GRIDS
        assert T.pick(e["candidates"])["b"] == e["b"]


@pytest.mark.gpu
def test_gpu_tuning_run_and_grid_leaves_results_unchanged():
    from paper_1811_05140_amd import aalcsim as A
    lad = I.default_ladder(1e-4)
    print("autotune n=14", flush=True)
    m = T.gpu_measure(A, 14, lad, 4.0, layers=1, reps=1)
    e = T.tune(14, lad, 4.0, m)
    m.close()
    assert 12 <= e["b"] <= 14 and e["gates_per_s"] > 0
    x, gates = T.calibration_circuit(16, 2)
    out = []
    for grid in (64, 4096):
        s = A.Sim(16, 12, 1e-4)
        s.set_grid(grid)
        s.set_basis(x)
        s.run(gates)
        out.append([s.export_block(j) for j in range(16)])
        s.close()
    assert out[0] == out[1]
