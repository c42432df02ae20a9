"""The C-ABI library loads and exports every function include/aalcsim.h
declares (no GPU needed: nothing here computes)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aalcsim.h")
LIB = os.path.join(ROOT, "paper_1811_05140_amd", "libaalcsim.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sim_create", "sim_apply_gate", "sim_measure_probs",
                     "sim_fidelity", "sim_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_1811_05140_amd import aalcsim
    assert sorted(aalcsim.EXPORTS) == declared_functions()


def test_binding_struct_layouts():
    from paper_1811_05140_amd import aalcsim
    # sim_gate_t: u32 kind, i32 q0, i32 q1, u32 pad, u64 index, f64 u[8]
    assert ctypes.sizeof(aalcsim.Gate) == 88
    assert aalcsim.Gate.index.offset == 16 and aalcsim.Gate.u.offset == 24
    # sim_stats_t ends with arena_bytes, device_bytes
    assert ctypes.sizeof(aalcsim.Stats) == 8 * 8 + 64 + 16 + 24
