"""Seeded synthetic inputs: circuits as gate lists.

This module generates the workloads only (which gates, on which qubits, with
which 2x2 matrices); it holds none of the compressed-simulation arithmetic.
Both the GPU library and the CPU oracle consume its gate tuples

    (kind, q0, q1, index, u)     u = 8 floats, 2x2 complex row-major

Qubit q is bit q of the amplitude index.  Matrices and phases are computed
once here on the host (math.cos / math.sin / math.sqrt); neither simulator
recomputes them.

Random draws use SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) from the base
seed 1811051400; workload i draws from seed 1811051400 + i.
"""
import math

G_U, G_DIAG1, G_CU, G_CPHASE, G_CZ, G_SWAP, G_X, G_PHASE_FLIP, G_DIFFUSE = \
    range(1, 10)

BASE_SEED = 1811051400
MASK64 = (1 << 64) - 1

_R = math.sqrt(0.5)
ZERO8 = (0.0,) * 8
H = (_R, 0.0, _R, 0.0, _R, 0.0, -_R, 0.0)
X_M = (0.0, 0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0)
SQRT_X = (0.5, 0.5, 0.5, -0.5, 0.5, -0.5, 0.5, 0.5)
SQRT_Y = (0.5, 0.5, -0.5, -0.5, 0.5, 0.5, 0.5, 0.5)
T_PHASE = (math.cos(math.pi / 4), math.sin(math.pi / 4))


class SplitMix64:
    """SplitMix64 generator: 64-bit state advanced by the golden gamma."""

    def __init__(self, seed):
        self.state = seed & MASK64

    def next(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self):
        """Float in [0, 1) from the top 53 bits."""
        return (self.next() >> 11) * (1.0 / (1 << 53))


def rng_for(workload_index):
    return SplitMix64(BASE_SEED + workload_index)


# ---- single gates -------------------------------------------------------

def u_gate(q, u):
    return (G_U, q, 0, 0, tuple(float(v) for v in u))


def h(q):
    return (G_U, q, 0, 0, H)


def x(q):
    return (G_X, q, 0, 0, ZERO8)


def diag1(q, phase_re, phase_im):
    return (G_DIAG1, q, 0, 0, (1.0, 0.0, 0.0, 0.0, 0.0, 0.0,
                               float(phase_re), float(phase_im)))


def t_gate(q):
    return diag1(q, *T_PHASE)


def cu(c, t, u):
    return (G_CU, c, t, 0, tuple(float(v) for v in u))


def cphase(a, b, phi):
    return (G_CPHASE, a, b, 0, (1.0, 0.0, 0.0, 0.0, 0.0, 0.0,
                                math.cos(phi), math.sin(phi)))


def cz(a, b):
    return (G_CZ, a, b, 0, ZERO8)


def swap(a, b):
    return (G_SWAP, a, b, 0, ZERO8)


def phase_flip(m):
    return (G_PHASE_FLIP, 0, 0, int(m), ZERO8)


def diffuse():
    return (G_DIFFUSE, 0, 0, 0, ZERO8)


# ---- circuits -----------------------------------------------------------

def qft(n):
    """Quantum Fourier transform with native H, controlled phase and SWAP.

    For j = n-1 .. 0: H(j), then CP(pi / 2^(j-m)) on (m, j) for m = j-1 .. 0;
    then SWAP(j, n-1-j) for j < n/2.  On |x> it yields
    2^(-n/2) sum_k exp(+2 pi i x k / 2^n) |k>.
    Gate count n + n(n-1)/2 + floor(n/2) (84 at n=12, 312 at n=24).
    """
    gates = []
    for j in range(n - 1, -1, -1):
        gates.append(h(j))
        for m in range(j - 1, -1, -1):
            gates.append(cphase(m, j, math.pi / (1 << (j - m))))
    for j in range(n // 2):
        gates.append(swap(j, n - 1 - j))
    return gates


def grover(n, marked, iterations):
    """H on qubits 0..n-1 in that order, then iterations x (oracle, diffusion).

    The oracle is a phase flip of the marked index and the diffusion is
    2|s><s| - I, both as native n-qubit operations."""
    gates = [h(q) for q in range(n)]
    for _ in range(iterations):
        gates.append(phase_flip(marked))
        gates.append(diffuse())
    return gates


def grover_success(n, k):
    """Closed form P(marked) after k iterations: sin^2((2k+1) asin(2^-n/2))."""
    th = math.asin(2.0 ** (-n / 2.0))
    return math.sin((2 * k + 1) * th) ** 2


def random_brick(n, depth, rng):
    """Depth-`depth` brick circuit: per layer, per qubit one of
    {sqrt X, sqrt Y, T} (draw mod 3), then CZ on (2j, 2j+1) for even layers
    and (2j+1, 2j+2) for odd layers."""
    gates = []
    for layer in range(depth):
        for q in range(n):
            k = rng.next() % 3
            if k == 0:
                gates.append(u_gate(q, SQRT_X))
            elif k == 1:
                gates.append(u_gate(q, SQRT_Y))
            else:
                gates.append(t_gate(q))
        start = 0 if layer % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            gates.append(cz(a, a + 1))
    return gates


def random_brick_layers(n, depth, rng):
    """Same circuit as random_brick, split into its layers."""
    layers = []
    for layer in range(depth):
        gl = []
        for q in range(n):
            k = rng.next() % 3
            gl.append(u_gate(q, SQRT_X) if k == 0 else
                      u_gate(q, SQRT_Y) if k == 1 else t_gate(q))
        start = 0 if layer % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            gl.append(cz(a, a + 1))
        layers.append(gl)
    return layers


def default_ladder(delta):
    """AALC ladder (0, delta/1000, delta/100, delta/10, delta): lossless first,
    then four lossy levels, each fl(delta / 10^j)."""
    return [0.0, delta / 1000.0, delta / 100.0, delta / 10.0, delta]


def relative_ladder(eps):
    """Pointwise-relative AALC ladder: lossless first, then the relative
    bounds eps/100, eps/10, eps (entries -bound), leaving out those below the
    smallest relative bound 2^-19."""
    lad = [0.0]
    for j in (100.0, 10.0, 1.0):
        v = eps / j
        if v >= 2.0 ** -19:
            lad.append(-v)
    return lad


# ---- the workloads -------------------------------------------------------

def qft12_workload():
    """12-qubit QFT on a seeded basis state, blocks of 2^8 (16 blocks)."""
    rng = rng_for(1)
    xb = rng.next() & 0xFFF
    return {"n": 12, "b": 8, "basis": xb, "gates": qft(12)}


def qft24_workload():
    """24-qubit QFT on a seeded basis state, blocks of 2^16 (256 blocks)."""
    rng = rng_for(2)
    xb = rng.next() & 0xFFFFFF
    return {"n": 24, "b": 16, "basis": xb, "gates": qft(24)}


def grover36_workload(n=36, iterations=8, b=20):
    """Grover search, one seeded marked index, 8 iterations, blocks of 2^20."""
    rng = rng_for(3)
    m = rng.next() & ((1 << n) - 1)
    return {"n": n, "b": b, "basis": 0, "marked": m,
            "gates": grover(n, m, iterations)}


def random_batch_workload(count=64, depth=20):
    """Instances with n uniform in [16, 28], depth-20 brick layers."""
    rng = rng_for(4)
    inst = []
    for i in range(count):
        n = 16 + rng.next() % 13
        inst.append({"n": n, "layers": random_brick_layers(n, depth, rng)})
    return inst



def serving_workload(count=512, n_lo=10, n_hi=30, depth=20):
    """Request stream for the serving loop, in arrival order.  Each request:
    unit-rate arrival time `t1` (cumulative Exp(1) gaps; divide by the rate
    lambda for arrivals at that rate), kind uniform over {qft, grover,
    random}, n = n_lo + draw mod (n_hi - n_lo + 1), error bound uniform over
    {1e-3, 1e-4, 1e-5}, then the kind's own draws (QFT: basis x; Grover:
    marked index, iterations 1 + draw mod 6; random: depth-`depth` brick
    circuit)."""
    rng = rng_for(5)
    reqs = []
    t = 0.0
    for i in range(count):
        u = 1.0 - rng.uniform()  # (0, 1]
        t += -math.log(u)
        kind = ("qft", "grover", "random")[rng.next() % 3]
        n = n_lo + rng.next() % (n_hi - n_lo + 1)
        eb = (1e-3, 1e-4, 1e-5)[rng.next() % 3]
        mask = (1 << n) - 1
        r = {"id": i, "t1": t, "kind": kind, "n": n, "eb": eb, "basis": 0}
        if kind == "qft":
            r["basis"] = rng.next() & mask
            r["gates"] = qft(n)
        elif kind == "grover":
            r["marked"] = rng.next() & mask
            r["iterations"] = 1 + rng.next() % 6
            r["gates"] = grover(n, r["marked"], r["iterations"])
        else:
            r["gates"] = random_brick(n, depth, rng)
        reqs.append(r)
    return reqs
