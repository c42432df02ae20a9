"""Sims whose device memory is a caller-owned torch buffer (memory contexts,
through the C ABI): results identical to the oracle and to a sim with its
own memory, every buffer inside the context, SIM_EBUDGET when it is
exhausted (state unchanged), memory returned on destroy and reused."""
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


def test_context_sims_match_oracle_and_own_memory(A):
    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    buf = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")
    ctx = A.Context(buf, stream=stream)
    info0 = ctx.info()
    say("context", info0)
    assert info0["used"] == 0 and info0["capacity"] >= (64 << 20) - 256
    w = I.qft12_workload()
    n, b = w["n"], w["b"]
    g = A.Sim(n, b, 1e-4, context=ctx)
    used_g = ctx.info()["used"]
    u = A.Sim(n, b, -1.0, context=ctx)
    own = A.Sim(n, b, 1e-4)
    used = ctx.info()["used"]
    st = g.stats()
    assert used >= st["device_bytes"] + u.stats()["device_bytes"]
    assert used <= info0["capacity"]
    assert int(buf.count_nonzero()) > 0  # the arenas live in the torch buffer
    for sm in (g, u, own):
        sm.set_basis(w["basis"])
        sm.run(w["gates"])
    o = orc.OracleSim(n, b, I.default_ladder(1e-4), 4.0)
    o.set_basis(w["basis"])
    o.run(w["gates"])
    assert g.export_state() == o.export_state() == own.export_state()
    # the first whole-state export keeps an offset table for the sim's life
    used = ctx.info()["used"]
    full = o.amplitudes()
    assert np.array_equal(g.amplitudes().view(np.uint64), full.view(np.uint64))
    qs = [3, 0, 9]
    assert np.max(np.abs(g.probs(qs) - o.measure_probs(qs))) < 1e-12
    assert abs(g.fidelity(u) - own.fidelity(u)) < 1e-15
    assert ctx.info()["used"] == used  # queries gave their temporaries back
    with pytest.raises(A.SimError) as e:
        ctx.close()
    assert e.value.code == A.SIM_EINVAL
    g.close()
    u.close()
    assert ctx.info()["used"] == 0
    # the freed ranges are reused
    g2 = A.Sim(n, b, 1e-4, context=ctx)
    assert ctx.info()["used"] == used_g
    g2.close()
    own.close()
    ctx.close()


def test_context_budget_exhausted(A):
    import torch
    torch.cuda.set_device(0)
    buf = torch.zeros(8 << 20, dtype=torch.uint8, device="cuda")
    ctx = A.Context(buf)
    with pytest.raises(A.SimError) as e:
        A.Sim(20, 12, 1e-4, context=ctx)  # arenas of ~2.1 x 16 MiB do not fit
    assert e.value.code == A.SIM_EBUDGET
    assert ctx.info()["used"] == 0
    # a sim that fits, then a query whose temporary does not
    g = A.Sim(12, 8, 1e-4, context=ctx)
    need = ctx.info()["used"]
    g.close()
    ctx.close()
    tight = torch.zeros(need + 16384, dtype=torch.uint8, device="cuda")
    ctx2 = A.Context(tight)
    g = A.Sim(12, 8, 1e-4, context=ctx2)
    w = I.qft12_workload()
    g.set_basis(w["basis"])
    g.run(w["gates"][:20])
    before = g.export_block(3)
    with pytest.raises(A.SimError) as e:
        g.amplitudes()  # 64 KiB of decoded amplitudes exceed what is left
    assert e.value.code == A.SIM_EBUDGET
    assert g.export_block(3) == before
    assert ctx2.info()["used"] == need
    g.run(w["gates"][20:])
    o = orc.OracleSim(12, 8, I.default_ladder(1e-4), 4.0)
    o.set_basis(w["basis"])
    o.run(w["gates"])
    assert g.export_state() == o.export_state()
    g.close()
    ctx2.close()
