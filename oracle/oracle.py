"""ctypes binding of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product package never imports it.

Gates are passed as plain tuples (kind, q0, q1, index, u) where u is a
sequence of 8 floats (2x2 complex matrix, row-major, (re, im) pairs); the
circuit generators produce exactly these tuples.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-shared", "-fPIC"]


def build(force=False):
    """Compile liboracle.so with the host C compiler (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + CFLAGS + [_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("q0", ctypes.c_int32),
                ("q1", ctypes.c_int32), ("pad", ctypes.c_uint32),
                ("index", ctypes.c_uint64), ("u", ctypes.c_double * 8)]


class Stats(ctypes.Structure):
    _fields_ = [("normsq", ctypes.c_double), ("scale", ctypes.c_double),
                ("collapsed", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("resident_bytes", ctypes.c_uint64),
                ("min_ratio", ctypes.c_double), ("last_ratio", ctypes.c_double),
                ("passes", ctypes.c_uint64),
                ("level_hist", ctypes.c_uint64 * 8)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        L = _lib
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        u8p = P(ctypes.c_uint8)
        szp = P(ctypes.c_size_t)
        L.or_pairwise.restype = ctypes.c_double
        L.or_pairwise.argtypes = [dp, ctypes.c_size_t]
        L.or_encode_block.argtypes = [dp, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_int, u8p,
                                      ctypes.c_size_t, szp]
        L.or_decode_block.argtypes = [u8p, ctypes.c_size_t, dp]
        L.or_aalc_encode.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp,
                                     ctypes.c_int, ctypes.c_double, u8p,
                                     ctypes.c_size_t, szp,
                                     P(ctypes.c_uint64)]
        L.or_sv_apply_gate.argtypes = [dp, ctypes.c_int, P(Gate)]
        L.or_create.restype = ctypes.c_void_p
        L.or_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                                ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.or_destroy.argtypes = [ctypes.c_void_p]
        L.or_set_basis.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.or_apply_gate.argtypes = [ctypes.c_void_p, P(Gate)]
        L.or_get_amplitudes.argtypes = [ctypes.c_void_p, ctypes.c_uint64,
                                        ctypes.c_uint64, dp]
        L.or_export_block.argtypes = [ctypes.c_void_p, ctypes.c_uint64, u8p,
                                      ctypes.c_size_t, szp]
        L.or_get_stats.argtypes = [ctypes.c_void_p, P(Stats)]
        L.or_measure_probs.argtypes = [ctypes.c_void_p, P(ctypes.c_int),
                                       ctypes.c_int, dp]
        L.or_process_group.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
            ctypes.c_double, ctypes.c_double, dp, P(Gate), ctypes.c_uint64,
            u8p, ctypes.c_size_t, u8p, ctypes.c_size_t,
            u8p, ctypes.c_size_t, szp, u8p, ctypes.c_size_t, szp]
        L.or_fidelity.restype = ctypes.c_double
        L.or_fidelity.argtypes = [dp, dp, ctypes.c_int]
        L.or_amplitude_sum.argtypes = [ctypes.c_void_p, dp]
        L.or_import_state.argtypes = [ctypes.c_void_p, u8p, ctypes.c_size_t]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_codec_log2.argtypes = [ctypes.c_double]
        L.or_codec_log2.restype = ctypes.c_double
        L.or_codec_exp2.argtypes = [ctypes.c_double]
        L.or_codec_exp2.restype = ctypes.c_double
        L.or_set_shortcut.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.or_entropy_encode.argtypes = [u8p, ctypes.c_size_t, u8p, ctypes.c_size_t, szp]
        L.or_entropy_decode.argtypes = [u8p, ctypes.c_size_t, u8p, ctypes.c_size_t, szp]
    return _lib


def codec_log2(a):
    """The relative levels' log2 of a finite a > 0."""
    return lib().or_codec_log2(float(a))


def codec_exp2(y):
    """The relative levels' power of two."""
    return lib().or_codec_exp2(float(y))


def set_threads(nthreads):
    """Threads for the block groups of each pass; returns the number in
    effect.  Every result is the same for any thread count."""
    return lib().or_set_threads(int(nthreads))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def make_gate(g):
    kind, q0, q1, index, u = g
    out = Gate()
    out.kind, out.q0, out.q1, out.pad, out.index = kind, q0, q1, 0, index
    for k in range(8):
        out.u[k] = float(u[k])
    return out


def _as_complex_interleaved(x):
    x = np.asarray(x)
    if np.iscomplexobj(x):
        out = np.empty(2 * x.size, dtype=np.float64)
        out[0::2] = x.real
        out[1::2] = x.imag
        return out
    return np.ascontiguousarray(x, dtype=np.float64)


def pairwise(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().or_pairwise(_dp(v), v.size)


def encode_block(x, b, s, delta, level=0):
    """Encode 2^b complex values at one error bound; returns bytes."""
    xi = _as_complex_interleaved(x)
    assert xi.size == 2 << b
    cap = 64 + (48 << b) * 2
    out = np.zeros(cap, dtype=np.uint8)
    n = ctypes.c_size_t(0)
    rc = lib().or_encode_block(_dp(xi), b, s, delta, level, _u8p(out), cap,
                               ctypes.byref(n))
    if rc:
        raise RuntimeError("or_encode_block rc=%d" % rc)
    return bytes(out[:n.value])


def decode_block(stream):
    """Decode a block stream; returns complex128 array of 2^b values."""
    buf = np.frombuffer(bytes(stream), dtype=np.uint8).copy()
    b = int(buf[7])
    x = np.zeros(2 << b, dtype=np.float64)
    rc = lib().or_decode_block(_u8p(buf), buf.size, _dp(x))
    if rc:
        raise ValueError("or_decode_block rc=%d" % rc)
    return x[0::2] + 1j * x[1::2]


def decode_block_interleaved(stream):
    buf = np.frombuffer(bytes(stream), dtype=np.uint8).copy()
    b = int(buf[7])
    x = np.zeros(2 << b, dtype=np.float64)
    rc = lib().or_decode_block(_u8p(buf), buf.size, _dp(x))
    if rc:
        raise ValueError("or_decode_block rc=%d" % rc)
    return x


def _coder(fn, data):
    src = np.frombuffer(bytes(data), dtype=np.uint8).copy()
    n = ctypes.c_size_t(0)
    rc = fn(_u8p(src), src.size, None, 0, ctypes.byref(n))
    if rc not in (0, -2):
        raise ValueError("entropy coder rc=%d" % rc)
    out = np.zeros(max(n.value, 1), dtype=np.uint8)
    rc = fn(_u8p(src), src.size, _u8p(out), out.size, ctypes.byref(n))
    if rc:
        raise ValueError("entropy coder rc=%d" % rc)
    return bytes(out[:n.value])


def entropy_encode(stream):
    """Block entropy stream of one block stream v1 (oracle.c defines it)."""
    return _coder(lib().or_entropy_encode, stream)


def entropy_decode(estream):
    """The block stream v1 that a block entropy stream encodes."""
    return _coder(lib().or_entropy_decode, estream)


E_MAGIC = 0x31454141


def split_streams(data):
    """The block streams (v1 or entropy) of a concatenation, in order."""
    data = bytes(data)
    out, pos = [], 0
    while pos < len(data):
        total = int.from_bytes(data[pos + 12:pos + 16], "little")
        if total < 32 or pos + total > len(data):
            raise ValueError("truncated stream at byte %d" % pos)
        out.append(data[pos:pos + total])
        pos += total
    return out


def entropy_state(data):
    """Every v1 block stream of a checkpoint through the entropy stage."""
    return b"".join(entropy_encode(x) for x in split_streams(data))


def plain_state(data):
    """A checkpoint with every entropy-coded block stream decoded to v1."""
    return b"".join(entropy_decode(x) if int.from_bytes(x[:4], "little") == E_MAGIC else x
                    for x in split_streams(data))


def aalc_encode(x, b, s, ladder, theta):
    """Alg. 2 on one block: returns (level, stream bytes, sizes tried)."""
    xi = _as_complex_interleaved(x)
    lad = np.asarray(ladder, dtype=np.float64)
    cap = 64 + (48 << b) * 2
    out = np.zeros(cap, dtype=np.uint8)
    n = ctypes.c_size_t(0)
    sizes = (ctypes.c_uint64 * 8)()
    k = lib().or_aalc_encode(_dp(xi), b, s, _dp(lad), lad.size, theta,
                             _u8p(out), cap, ctypes.byref(n), sizes)
    if k < 0:
        raise RuntimeError("or_aalc_encode rc=%d" % k)
    return k, bytes(out[:n.value]), [int(sizes[i]) for i in range(lad.size)]


def sv_apply(amp, n, gate):
    """Plain uncompressed gate on an interleaved float64 array, in place."""
    g = make_gate(gate)
    rc = lib().or_sv_apply_gate(_dp(amp), n, ctypes.byref(g))
    if rc:
        raise ValueError("or_sv_apply_gate rc=%d" % rc)


def sv_run(n, gates, basis=0):
    """Uncompressed FP64 reference run from |basis>; complex128 result."""
    amp = np.zeros(2 << n, dtype=np.float64)
    amp[2 * basis] = 1.0
    for g in gates:
        sv_apply(amp, n, g)
    return amp[0::2] + 1j * amp[1::2]


def sv_run_from(psi, n, gate):
    """One plain uncompressed gate applied to a copy of complex vector psi."""
    amp = _as_complex_interleaved(np.asarray(psi, dtype=np.complex128)).copy()
    sv_apply(amp, n, gate)
    return amp[0::2] + 1j * amp[1::2]


def fidelity(a, b, n):
    ai = _as_complex_interleaved(a)
    bi = _as_complex_interleaved(b)
    if ai.size != 2 << n or bi.size != 2 << n:
        raise ValueError("fidelity needs two arrays of 2^n complex values")
    return lib().or_fidelity(_dp(ai), _dp(bi), n)


def default_ladder(delta):
    """(0, delta/1000, delta/100, delta/10, delta), each fl(delta / 10^j)."""
    return [0.0, delta / 1000.0, delta / 100.0, delta / 10.0, delta]


class OracleSim:
    """Alg. 2 driver over block streams held in host memory."""

    def __init__(self, n, b, ladder, theta=4.0, normalize=True, s=None):
        self.n, self.b = n, b
        self.s = min(b, 10) if s is None else s
        self.ladder = np.asarray(ladder, dtype=np.float64)
        self.theta = float(theta)
        self.h = lib().or_create(n, b, self.s, _dp(self.ladder),
                                 self.ladder.size, self.theta,
                                 1 if normalize else 0)
        if not self.h:
            raise ValueError("or_create rejected the parameters")

    def close(self):
        if self.h:
            lib().or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    SC_PERMUTE, SC_SKIP = 1, 2

    def set_shortcut(self, flags):
        """Sec. V shortcuts: SC_PERMUTE (permutation gates keep each block's
        previous level), SC_SKIP (blocks a gate leaves unchanged keep their
        streams, normalisation deferred into a per-block scale)."""
        rc = lib().or_set_shortcut(self.h, int(flags))
        if rc:
            raise ValueError("or_set_shortcut rc=%d" % rc)

    def set_basis(self, x):
        rc = lib().or_set_basis(self.h, x)
        if rc:
            raise ValueError("or_set_basis rc=%d" % rc)

    def apply(self, gate):
        g = make_gate(gate)
        return lib().or_apply_gate(self.h, ctypes.byref(g))

    def run(self, gates):
        rc = 0
        for g in gates:
            rc = self.apply(g)
            if rc not in (0, -5):
                raise RuntimeError("or_apply_gate rc=%d" % rc)
        return rc

    def amplitudes(self, first=0, count=None):
        if count is None:
            count = (1 << self.n) - first
        out = np.zeros(2 * count, dtype=np.float64)
        rc = lib().or_get_amplitudes(self.h, first, count, _dp(out))
        if rc:
            raise ValueError("or_get_amplitudes rc=%d" % rc)
        return out[0::2] + 1j * out[1::2]

    def export_block(self, j):
        cap = 72 + (48 << self.b) * 2
        out = np.zeros(cap, dtype=np.uint8)
        n = ctypes.c_size_t(0)
        rc = lib().or_export_block(self.h, j, _u8p(out), cap, ctypes.byref(n))
        if rc:
            raise ValueError("or_export_block rc=%d" % rc)
        return bytes(out[:n.value])

    def export_state(self, entropy=False):
        """Every block's stream, block 0 first (the checkpoint of the state);
        with entropy, each through the entropy stage."""
        data = b"".join(self.export_block(j)
                        for j in range(1 << (self.n - self.b)))
        return entropy_state(data) if entropy else data

    def import_state(self, data):
        """Replace the state by concatenated block streams; returns the code
        (0, or -5 when N^2 of the imported state is 0 or not finite) and
        raises ValueError when a stream is rejected."""
        data = bytes(data)
        try:
            data = plain_state(data)
        except ValueError:
            pass  # or_import_state rejects what cannot be split or decoded
        buf = np.frombuffer(data, dtype=np.uint8).copy()
        rc = lib().or_import_state(self.h, _u8p(buf), buf.size)
        if rc not in (0, -5):
            raise ValueError("or_import_state rc=%d" % rc)
        return rc

    def stats(self):
        st = Stats()
        lib().or_get_stats(self.h, ctypes.byref(st))
        return {"normsq": st.normsq, "scale": st.scale,
                "collapsed": st.collapsed,
                "resident_bytes": st.resident_bytes,
                "min_ratio": st.min_ratio, "last_ratio": st.last_ratio,
                "passes": st.passes,
                "level_hist": [int(st.level_hist[k]) for k in range(8)]}

    def amplitude_sum(self):
        """Pairwise sums (re, im) of the normalised amplitudes."""
        out = np.zeros(2)
        rc = lib().or_amplitude_sum(self.h, _dp(out))
        if rc:
            raise RuntimeError("or_amplitude_sum failed (%d)" % rc)
        return complex(out[0], out[1])

    def measure_probs(self, qubits):
        q = (ctypes.c_int * len(qubits))(*qubits)
        out = np.zeros(1 << len(qubits), dtype=np.float64)
        rc = lib().or_measure_probs(self.h, q, len(qubits), _dp(out))
        if rc:
            raise ValueError("or_measure_probs rc=%d" % rc)
        return out


def process_group(n, b, s, ladder, theta, scale, tdiff, gate, j0, in0,
                  in1=None):
    """One Alg. 2 group from exported input streams; returns output streams."""
    lad = np.asarray(ladder, dtype=np.float64)
    t = np.asarray(tdiff if tdiff is not None else (0.0, 0.0),
                   dtype=np.float64)
    g = make_gate(gate)
    a0 = np.frombuffer(bytes(in0), dtype=np.uint8).copy()
    a1 = np.frombuffer(bytes(in1), dtype=np.uint8).copy() if in1 else \
        np.zeros(1, dtype=np.uint8)
    cap = 64 + (48 << b) * 2
    o0 = np.zeros(cap, dtype=np.uint8)
    o1 = np.zeros(cap, dtype=np.uint8)
    l0 = ctypes.c_size_t(0)
    l1 = ctypes.c_size_t(0)
    rc = lib().or_process_group(n, b, s, _dp(lad), lad.size, theta, scale,
                                _dp(t), ctypes.byref(g), j0, _u8p(a0),
                                a0.size if in0 else 0, _u8p(a1),
                                a1.size if in1 else 0, _u8p(o0), cap,
                                ctypes.byref(l0), _u8p(o1), cap,
                                ctypes.byref(l1))
    if rc:
        raise RuntimeError("or_process_group rc=%d" % rc)
    out0 = bytes(o0[:l0.value])
    out1 = bytes(o1[:l1.value]) if in1 else None
    return out0, out1


def state_bytes(n):
    """Uncompressed complex-double state of n qubits: 2^(n+4) bytes."""
    return 1 << (n + 4)


def max_qubits(memory_bytes, ratio=1.0):
    """Largest qubit count whose state fits in `memory_bytes`, plus the
    floor(log2 ratio) qubits a minimum compression ratio buys."""
    uncompressed = (int(memory_bytes) // 16).bit_length() - 1
    extra = int(ratio).bit_length() - 1 if ratio >= 1 else 0
    return uncompressed + extra
