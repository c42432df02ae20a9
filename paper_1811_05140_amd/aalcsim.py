"""ctypes binding of libaalcsim.so (include/aalcsim.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of the library.  The library must have been built (see build.py);
importing this module on a machine without it raises ImportError instead of
falling back to anything else.

Gates are tuples (kind, q0, q1, index, u) as produced by `inputs`.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaalcsim.so")

SIM_OK, SIM_EINVAL, SIM_ENOMEM, SIM_EBUDGET, SIM_EDEVICE, SIM_ECOLLAPSED, \
    SIM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6

EXPORTS = [
    "sim_create", "sim_create_ex", "sim_destroy", "sim_apply_gate",
    "sim_apply_gates", "sim_measure_probs", "sim_fidelity", "sim_set_basis",
    "sim_set_aalc", "sim_set_normalize", "sim_get_amplitudes",
    "sim_export_block", "sim_stats", "sim_sync", "sim_set_stream",
    "sim_debug_rsqrt", "sim_last_error", "sim_profile", "sim_profile_read",
    "sim_export_headers", "sim_amplitude_sum",
    "sim_batch_create", "sim_batch_destroy", "sim_batch_apply", "sim_batch_sync",
    "sim_batch_info", "sim_set_grid", "sim_batch_profile", "sim_batch_profile_read",
    "sim_fourier_overlap", "sim_export_state", "sim_import_state",
    "sim_export_state_entropy",
    "sim_measure_probs_noalloc",
    "sim_context_create", "sim_context_destroy", "sim_context_info", "sim_create_in",
    "sim_set_shortcut",
]


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


class CollapsedError(SimError):
    pass


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("q0", ctypes.c_int32),
                ("q1", ctypes.c_int32), ("pad", ctypes.c_uint32),
                ("index", ctypes.c_uint64), ("u", ctypes.c_double * 8)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double), ("min_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("normsq", ctypes.c_double), ("scale", ctypes.c_double),
                ("collapsed", ctypes.c_int32), ("compressed", ctypes.c_int32),
                ("resident_bytes", ctypes.c_uint64),
                ("peak_resident", ctypes.c_uint64),
                ("min_ratio", ctypes.c_double), ("last_ratio", ctypes.c_double),
                ("passes", ctypes.c_uint64),
                ("level_hist", ctypes.c_uint64 * 8),
                ("arena_bytes", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64),
                ("replays", ctypes.c_uint64),
                ("escalations", ctypes.c_uint64),
                ("arena_peak", ctypes.c_uint64)]


def _load():
    # PyTorch bundles its own HIP runtime under the same soname as the one the
    # library links; loading torch first makes both use that one runtime, so
    # torch streams and device buffers are valid handles for the library
    # (the other order leaves torch unable to initialise the GPU).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libaalcsim.so is not built (run `python -c 'import __graft_entry__ as g; "
            "g.build()'` or python paper_1811_05140_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    dp = P(ctypes.c_double)
    L.sim_create.restype = vp
    L.sim_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double]
    L.sim_create_ex.restype = vp
    L.sim_create_ex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.c_uint64, vp]
    L.sim_destroy.argtypes = [vp]
    L.sim_destroy.restype = None
    L.sim_apply_gate.argtypes = [vp, P(Gate)]
    L.sim_apply_gates.argtypes = [vp, P(Gate), ctypes.c_size_t]
    L.sim_measure_probs.argtypes = [vp, P(ctypes.c_int), ctypes.c_int, dp]
    L.sim_measure_probs_noalloc.argtypes = [vp, P(ctypes.c_int), ctypes.c_int, dp]
    L.sim_fidelity.argtypes = [vp, vp, dp]
    L.sim_set_basis.argtypes = [vp, ctypes.c_uint64]
    L.sim_set_aalc.argtypes = [vp, dp, ctypes.c_int, ctypes.c_double]
    L.sim_set_normalize.argtypes = [vp, ctypes.c_int]
    L.sim_set_shortcut.argtypes = [vp, ctypes.c_int]
    L.sim_get_amplitudes.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint64, dp]
    L.sim_export_block.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_size_t,
                                   P(ctypes.c_size_t)]
    L.sim_export_headers.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint64, vp,
                                     ctypes.c_size_t]
    L.sim_amplitude_sum.argtypes = [vp, dp]
    L.sim_export_state.argtypes = [vp, vp, ctypes.c_size_t, P(ctypes.c_size_t)]
    L.sim_import_state.argtypes = [vp, vp, ctypes.c_size_t]
    L.sim_export_state_entropy.argtypes = [vp, vp, ctypes.c_size_t, P(ctypes.c_size_t)]
    L.sim_set_grid.argtypes = [vp, ctypes.c_int]
    L.sim_fourier_overlap.argtypes = [vp, ctypes.c_uint64, dp]
    L.sim_stats.argtypes = [vp, P(Stats)]
    L.sim_sync.argtypes = [vp]
    L.sim_set_stream.argtypes = [vp, vp]
    L.sim_debug_rsqrt.argtypes = [dp, dp, ctypes.c_size_t]
    L.sim_profile.argtypes = [vp, ctypes.c_int]
    L.sim_profile_read.argtypes = [vp, P(KernelTime), ctypes.c_int,
                                   P(ctypes.c_int)]
    L.sim_batch_create.restype = vp
    L.sim_batch_create.argtypes = [ctypes.c_int, ctypes.c_int, vp]
    L.sim_batch_destroy.restype = None
    L.sim_batch_destroy.argtypes = [vp]
    L.sim_batch_apply.argtypes = [vp, P(vp), ctypes.c_int, P(Gate), ctypes.c_int,
                                  ctypes.c_int]
    L.sim_batch_sync.argtypes = [vp]
    L.sim_batch_info.argtypes = [vp, P(ctypes.c_uint64), P(ctypes.c_uint64)]
    L.sim_batch_profile.argtypes = [vp, ctypes.c_int]
    L.sim_batch_profile_read.argtypes = [vp, P(KernelTime), ctypes.c_int, P(ctypes.c_int)]
    L.sim_context_create.argtypes = [vp, ctypes.c_size_t, vp, P(vp)]
    L.sim_context_destroy.argtypes = [vp]
    L.sim_context_info.argtypes = [vp] + [P(ctypes.c_uint64)] * 4
    L.sim_create_in.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.c_uint64, P(vp)]
    L.sim_last_error.restype = ctypes.c_char_p
    L.sim_last_error.argtypes = []
    return L


lib = _load()


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def last_error():
    return lib.sim_last_error().decode(errors="replace")


def check(rc, allow_collapsed=False):
    if rc == SIM_OK:
        return rc
    if rc == SIM_ECOLLAPSED:
        if allow_collapsed:
            return rc
        raise CollapsedError(rc, last_error())
    raise SimError(rc, last_error())


def make_gate(g):
    kind, q0, q1, index, u = g
    out = Gate()
    out.kind, out.q0, out.q1, out.pad, out.index = kind, q0, q1, 0, index
    for k in range(8):
        out.u[k] = float(u[k])
    return out


def gate_array(gates):
    arr = (Gate * len(gates))()
    for k, g in enumerate(gates):
        arr[k] = make_gate(g)
    return arr


def _stream_handle(stream):
    """Accept None, an int handle or a torch.cuda.Stream."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Sim:
    """One simulated state on the GPU.

    error_bound > 0: default AALC ladder (0, eb/1000, eb/100, eb/10, eb), theta 4;
    error_bound == 0: lossless only; error_bound < 0: uncompressed FP64.
    """

    def __init__(self, n, block_log2, error_bound, arena_bytes=0, stream=None,
                 ladder=None, theta=None, normalize=True, context=None):
        self._stream_obj = stream  # keep a torch stream alive
        self._context = context    # keep the context (and its buffer) alive
        if context is not None:
            h = ctypes.c_void_p()
            check(lib.sim_create_in(context.h, n, block_log2, float(error_bound),
                                    int(arena_bytes), ctypes.byref(h)))
            self.h = h.value
        else:
            self.h = lib.sim_create_ex(n, block_log2, float(error_bound),
                                       int(arena_bytes), _stream_handle(stream))
        if not self.h:
            raise SimError(SIM_EINVAL, last_error())
        self.n = n
        self.b = min(block_log2, n)
        self.compressed = not error_bound < 0
        if ladder is not None:
            self.set_aalc(ladder, 4.0 if theta is None else theta)
        if not normalize:
            self.set_normalize(False)
        if ladder is not None or not normalize:
            self.set_basis(0)  # encode the initial state under these settings

    def close(self):
        if getattr(self, "h", None):
            lib.sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- state --------------------------------------------------------------
    def set_basis(self, x):
        check(lib.sim_set_basis(self.h, int(x)))

    def set_aalc(self, ladder, theta):
        lad = np.ascontiguousarray(ladder, dtype=np.float64)
        check(lib.sim_set_aalc(self.h, _dp(lad), lad.size, float(theta)))

    SC_PERMUTE, SC_SKIP = 1, 2

    def set_shortcut(self, flags):
        """Sec. V shortcuts: SC_PERMUTE (permutation gates keep each block's
        previous level), SC_SKIP (blocks a gate leaves unchanged keep their
        streams, normalisation deferred into a per-block scale)."""
        check(lib.sim_set_shortcut(self.h, int(flags)))

    def set_normalize(self, on):
        check(lib.sim_set_normalize(self.h, 1 if on else 0))

    def fourier_fidelity(self, x):
        """Fidelity to the closed-form QFT|x> (2^-n/2 e^(2 pi i x k / 2^n))."""
        out = np.zeros(3)
        check(lib.sim_fourier_overlap(self.h, int(x), _dp(out)), True)
        return (out[0] ** 2 + out[1] ** 2) / (float(1 << self.n) * out[2])

    def set_grid(self, max_workgroups):
        check(lib.sim_set_grid(self.h, int(max_workgroups)))

    def set_stream(self, stream):
        self._stream_obj = stream
        check(lib.sim_set_stream(self.h, _stream_handle(stream)))

    def apply(self, gate):
        g = make_gate(gate)
        check(lib.sim_apply_gate(self.h, ctypes.byref(g)))

    def run(self, gates):
        arr = gate_array(gates)
        check(lib.sim_apply_gates(self.h, arr, len(gates)))

    def sync(self, allow_collapsed=True):
        return check(lib.sim_sync(self.h), allow_collapsed)

    # -- queries ------------------------------------------------------------
    def amplitudes(self, first=0, count=None):
        if count is None:
            count = (1 << self.n) - first
        out = np.zeros(2 * count, dtype=np.float64)
        check(lib.sim_get_amplitudes(self.h, first, count, _dp(out)), True)
        return out[0::2] + 1j * out[1::2]

    def probs(self, qubits):
        q = (ctypes.c_int * len(qubits))(*qubits)
        out = np.zeros(1 << len(qubits), dtype=np.float64)
        check(lib.sim_measure_probs(self.h, q, len(qubits), _dp(out)), True)
        return out

    def probs_noalloc(self, qubits):
        """As probs, through the entry point that allocates no device memory
        (bins in a library-held array per GPU; at most 16 qubits)."""
        q = (ctypes.c_int * len(qubits))(*qubits)
        out = np.zeros(1 << len(qubits), dtype=np.float64)
        check(lib.sim_measure_probs_noalloc(self.h, q, len(qubits), _dp(out)), True)
        return out

    def fidelity(self, other):
        F = ctypes.c_double(0.0)
        check(lib.sim_fidelity(self.h, other.h, ctypes.byref(F)), True)
        return F.value

    def export_block(self, j):
        ln = ctypes.c_size_t(0)
        rc = lib.sim_export_block(self.h, j, None, 0, ctypes.byref(ln))
        if rc not in (SIM_OK, SIM_ENOMEM, SIM_ECOLLAPSED):
            check(rc)
        buf = ctypes.create_string_buffer(max(ln.value, 1))
        check(lib.sim_export_block(self.h, j, buf, ln.value, ctypes.byref(ln)), True)
        return buf.raw[:ln.value]

    def export_state(self, out=None, entropy=False):
        """Checkpoint: every block's stream, block 0 first, as bytes (or into
        `out`, a writable buffer such as a pinned uint8 tensor's numpy view,
        when given; then the byte count is returned).  entropy: each stream
        through the entropy stage (sim_export_state_entropy)."""
        fn = lib.sim_export_state_entropy if entropy else lib.sim_export_state
        ln = ctypes.c_size_t(0)
        if out is not None:
            # one call: the library reports the length needed (SIM_ENOMEM)
            # when the buffer is too small
            arr = np.frombuffer(out, dtype=np.uint8)
            check(fn(self.h, arr.ctypes.data, arr.size, ctypes.byref(ln)), True)
            return ln.value
        rc = fn(self.h, None, 0, ctypes.byref(ln))
        if rc not in (SIM_OK, SIM_ENOMEM, SIM_ECOLLAPSED):
            check(rc)
        buf = ctypes.create_string_buffer(max(ln.value, 1))
        check(fn(self.h, buf, ln.value, ctypes.byref(ln)), True)
        return buf.raw[:ln.value]

    def import_state(self, data, nbytes=None):
        """Resume from a checkpoint (bytes, or any buffer with `nbytes`)."""
        arr = np.frombuffer(data, dtype=np.uint8)
        if nbytes is not None:
            arr = arr[:nbytes]
        return check(lib.sim_import_state(self.h, arr.ctypes.data, arr.size), True)

    def export_headers(self, first=0, count=None):
        """32-byte stream headers of blocks [first, first+count), normsq filled."""
        if count is None:
            count = (1 << (self.n - self.b)) - first
        buf = ctypes.create_string_buffer(max(32 * count, 1))
        check(lib.sim_export_headers(self.h, first, count, buf, 32 * count), True)
        return buf.raw[:32 * count]

    def amplitude_sum(self):
        """Pairwise sums (re, im) of the normalised amplitudes over the state."""
        out = np.zeros(2)
        check(lib.sim_amplitude_sum(self.h, _dp(out)), True)
        return complex(out[0], out[1])

    def profile(self, on=True, pass_only=False):
        check(lib.sim_profile(self.h, (2 if pass_only else 1) if on else 0))

    def profile_read(self):
        """{kernel: (launches, total_ms, min_ms, max_ms)} since the last read."""
        arr = (KernelTime * 32)()
        cnt = ctypes.c_int(0)
        check(lib.sim_profile_read(self.h, arr, 32, ctypes.byref(cnt)))
        return {arr[k].name.decode(): (int(arr[k].launches), arr[k].total_ms,
                                       arr[k].min_ms, arr[k].max_ms)
                for k in range(min(cnt.value, 32))}

    def stats(self):
        st = Stats()
        check(lib.sim_stats(self.h, ctypes.byref(st)), True)
        return {"normsq": st.normsq, "scale": st.scale,
                "collapsed": st.collapsed, "compressed": st.compressed,
                "resident_bytes": st.resident_bytes,
                "peak_resident": st.peak_resident,
                "min_ratio": st.min_ratio, "last_ratio": st.last_ratio,
                "passes": st.passes,
                "level_hist": [int(st.level_hist[k]) for k in range(8)],
                "arena_bytes": st.arena_bytes,
                "device_bytes": st.device_bytes,
                "replays": st.replays, "escalations": st.escalations,
                "arena_peak": st.arena_peak}


class Context:
    """Caller-owned device memory for sims (sim_context_create): `buffer` is
    a device tensor (any dtype; its storage is used as raw bytes) that every
    sim created with context=this takes all of its device memory from."""

    def __init__(self, buffer, stream=None):
        self._buffer = buffer  # the storage must outlive the context
        self._stream_obj = stream
        h = ctypes.c_void_p()
        nbytes = buffer.numel() * buffer.element_size()
        check(lib.sim_context_create(ctypes.c_void_p(buffer.data_ptr()), nbytes,
                                     _stream_handle(stream), ctypes.byref(h)))
        self.h = h.value

    def info(self):
        v = [ctypes.c_uint64(0) for _ in range(4)]
        check(lib.sim_context_info(self.h, *[ctypes.byref(x) for x in v]))
        return {"capacity": v[0].value, "used": v[1].value, "peak": v[2].value,
                "largest_free": v[3].value}

    def close(self):
        if getattr(self, "h", None):
            check(lib.sim_context_destroy(self.h))
            self.h = None


class Batch:
    """Many sims advanced by shared kernel launches (optionally one HIP graph
    launch per call)."""

    def __init__(self, max_states, max_passes, stream=None):
        self._stream_obj = stream
        self.h = lib.sim_batch_create(max_states, max_passes, _stream_handle(stream))
        if not self.h:
            raise SimError(SIM_EINVAL, last_error())
        self.max_states, self.max_passes = max_states, max_passes

    def close(self):
        if getattr(self, "h", None):
            lib.sim_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, sims, passes, use_graph=False):
        """passes: list of passes, each a list with one gate tuple (or None)
        per sim."""
        count = len(sims)
        arr = (Gate * (count * len(passes)))()
        for p, row in enumerate(passes):
            if len(row) != count:
                raise ValueError("pass %d has %d gates for %d sims" % (p, len(row), count))
            for k, g in enumerate(row):
                if g is not None:
                    arr[p * count + k] = make_gate(g)
        hs = (ctypes.c_void_p * count)(*[sm.h for sm in sims])
        check(lib.sim_batch_apply(self.h, hs, count, arr, len(passes), 1 if use_graph else 0))

    def sync(self):
        check(lib.sim_batch_sync(self.h))

    def profile(self, on=True, pass_only=False):
        check(lib.sim_batch_profile(self.h, (2 if pass_only else 1) if on else 0))

    def profile_read(self):
        arr = (KernelTime * 32)()
        cnt = ctypes.c_int(0)
        check(lib.sim_batch_profile_read(self.h, arr, 32, ctypes.byref(cnt)))
        return {arr[k].name.decode(): (int(arr[k].launches), arr[k].total_ms,
                                       arr[k].min_ms, arr[k].max_ms)
                for k in range(min(cnt.value, 32))}

    def info(self):
        b = ctypes.c_uint64(0)
        n = ctypes.c_uint64(0)
        check(lib.sim_batch_info(self.h, ctypes.byref(b), ctypes.byref(n)))
        return {"graph_builds": b.value, "graph_launches": n.value}


def debug_rsqrt(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    check(lib.sim_debug_rsqrt(_dp(x), _dp(out), x.size))
    return out


def state_bytes(n):
    """Uncompressed complex-double state of n qubits: 2^(n+4) bytes."""
    return 1 << (n + 4)
