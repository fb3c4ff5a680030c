"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module only *describes* circuits, observables and initial states: it holds
no gate matrix and none of the simulator's arithmetic.  Both sides (the CPU
oracle and the HIP library) read the same op lists and build their own matrices
from the gate names and angles.

Conventions (the paper leaves them open; see the design notes):

* qubit q is bit q of the amplitude index (little-endian);
* for a gate on ``targets = (t0, t1, ...)``, ``t0`` is the least significant
  bit of the gate matrix's row/column index;
* controlled gates list their controls first: ``cx`` is ``(control, target)``,
  ``ccx`` is ``(c1, c2, target)``;
* parametric ops carry ``param >= 0`` and take their angle from a parameter
  vector at that index (``u3`` takes three consecutive entries); ops with
  ``param < 0`` carry fixed ``angles``;
* ``matrix`` ops carry a dense ``2^k x 2^k`` complex matrix in ``matrix``
  (row-major, complex128).

The workloads follow the shapes of the paper's benchmark families (random
supremacy-style circuits and ripple-carry multipliers, Sec. III) plus the
variational ansatz that motivates fast simulation (Sec. I).  They are
stand-ins generated from seeds; none of the original netlists is reproduced.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * np.pi

# Gate names understood by both sides, with their qubit counts and the number
# of angles they take (parametric gates only).
GATE_ARITY = {
    "h": 1, "x": 1, "y": 1, "z": 1, "s": 1, "sdg": 1, "t": 1, "tdg": 1,
    "rx": 1, "ry": 1, "rz": 1, "u3": 1,
    "cx": 2, "cz": 2, "cp": 2, "swap": 2,
    "ccx": 3, "ccz": 3,
}
GATE_NANGLES = {"rx": 1, "ry": 1, "rz": 1, "u3": 3, "cp": 1}


@dataclass(frozen=True)
class Op:
    kind: str
    targets: Tuple[int, ...]
    angles: Tuple[float, ...] = ()
    param: int = -1
    matrix: Optional[np.ndarray] = field(default=None, compare=False, hash=False)

    @property
    def k(self) -> int:
        return len(self.targets)


@dataclass
class Circuit:
    n: int
    ops: List[Op]
    nparams: int = 0
    name: str = ""

    def __len__(self) -> int:
        return len(self.ops)

    def count(self, kind: str) -> int:
        return sum(1 for o in self.ops if o.kind == kind)


@dataclass
class PauliSum:
    """H = sum_t coeff_t * P_t with P_t = i^{|x&z|} X^x Z^z (so a set bit in both
    masks is a Y on that qubit)."""
    n: int
    coeffs: List[float]
    xmasks: List[int]
    zmasks: List[int]

    def __len__(self) -> int:
        return len(self.coeffs)


# ---------------------------------------------------------------- builders

def op(kind: str, *targets: int, angles: Sequence[float] = (), param: int = -1) -> Op:
    if kind not in GATE_ARITY:
        raise ValueError(f"unknown gate {kind!r}")
    if GATE_ARITY[kind] != len(targets):
        raise ValueError(f"{kind} takes {GATE_ARITY[kind]} qubits, got {len(targets)}")
    return Op(kind, tuple(int(t) for t in targets), tuple(float(a) for a in angles), int(param))


def matrix_op(targets: Sequence[int], mat: np.ndarray) -> Op:
    k = len(targets)
    mat = np.ascontiguousarray(np.asarray(mat, dtype=np.complex128))
    if mat.shape != (1 << k, 1 << k):
        raise ValueError("matrix shape does not match the number of targets")
    return Op("matrix", tuple(int(t) for t in targets), (), -1, mat)


def random_unitary(k: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed 2^k x 2^k unitary (QR of a complex Gaussian matrix with
    the phases of R's diagonal folded back)."""
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diagonal(r) / np.abs(np.diagonal(r))
    return q * ph[None, :]


def random_matrix(k: int, rng: np.random.Generator) -> np.ndarray:
    """Dense complex Gaussian 2^k x 2^k matrix (not unitary)."""
    d = 1 << k
    return rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))


# ------------------------------------------------- random supremacy-style

def _u3_layer_angles(rng: np.random.Generator, depth: int, n: int) -> np.ndarray:
    return rng.uniform(0.0, TWO_PI, size=(depth, n, 3))


def random_line_circuit(n: int = 12, depth: int = 20, seed: int = 1) -> Circuit:
    """Layers of U3 on every qubit followed by CZ on nearest neighbours of a
    line: pairs (2i, 2i+1) on even layers, (2i+1, 2i+2) on odd layers."""
    rng = np.random.default_rng(seed)
    ang = _u3_layer_angles(rng, depth, n)
    ops: List[Op] = []
    for layer in range(depth):
        for q in range(n):
            ops.append(op("u3", q, angles=ang[layer, q]))
        start = layer % 2
        for a in range(start, n - 1, 2):
            ops.append(op("cz", a, a + 1))
    return Circuit(n, ops, 0, f"line{n}_d{depth}_s{seed}")


def grid_cz_pairs(rows: int, cols: int, layer: int) -> List[Tuple[int, int]]:
    """CZ pattern of a layer on a rows x cols grid (qubit = cols*r + c).  The
    pattern cycles through horizontal-even, vertical-even, horizontal-odd and
    vertical-odd neighbour pairs; the pairs of one layer are disjoint."""
    phase = layer % 4
    pairs = []
    if phase in (0, 2):
        c0 = 0 if phase == 0 else 1
        for r in range(rows):
            for c in range(c0, cols - 1, 2):
                pairs.append((cols * r + c, cols * r + c + 1))
    else:
        r0 = 0 if phase == 1 else 1
        for r in range(r0, rows - 1, 2):
            for c in range(cols):
                pairs.append((cols * r + c, cols * (r + 1) + c))
    return pairs


def random_grid_circuit(rows: int = 5, cols: int = 6, depth: int = 20, seed: int = 2) -> Circuit:
    """Supremacy-style random circuit on a grid: per layer U3 on every qubit
    (angles uniform in [0, 2pi)) then one of the four CZ patterns."""
    n = rows * cols
    rng = np.random.default_rng(seed)
    ang = _u3_layer_angles(rng, depth, n)
    ops: List[Op] = []
    for layer in range(depth):
        for q in range(n):
            ops.append(op("u3", q, angles=ang[layer, q]))
        for a, b in grid_cz_pairs(rows, cols, layer):
            ops.append(op("cz", a, b))
    return Circuit(n, ops, 0, f"grid{rows}x{cols}_d{depth}_s{seed}")


# ------------------------------------------------------------- multiplier

@dataclass(frozen=True)
class MultiplierLayout:
    """Register layout of the shift-and-add multiplier: a, b, product p and one
    ancilla c, packed from qubit 0 upwards."""
    bits: int = 7

    @property
    def a(self) -> List[int]:
        return list(range(0, self.bits))

    @property
    def b(self) -> List[int]:
        return list(range(self.bits, 2 * self.bits))

    @property
    def p(self) -> List[int]:
        return list(range(2 * self.bits, 4 * self.bits))

    @property
    def anc(self) -> int:
        return 4 * self.bits

    @property
    def n(self) -> int:
        return 4 * self.bits + 1

    def basis_index(self, a: int, b: int, p: int = 0, anc: int = 0) -> int:
        w = self.bits
        return a | (b << w) | (p << (2 * w)) | (anc << (4 * w))


def multiplier_core(bits: int = 7) -> Circuit:
    """Width-(4w+1) multiplier p += a*b built from X/CNOT/Toffoli gates.

    Shift-and-add: for every bit b_i of the multiplier, add a into the product
    window p[i .. i+w] with a ripple-carry adder in the majority / un-majority
    style (one ancilla carries the incoming carry 0), each step controlled on
    b_i.  Only the carry-out and the final sum-restoring Toffolis need the
    control; the rest of the adder runs unconditionally and is undone by the
    un-majority chain when b_i = 0.
    """
    L = MultiplierLayout(bits)
    a, b, p, c = L.a, L.b, L.p, L.anc
    ops: List[Op] = []

    def maj(x, y, w):
        ops.append(op("cx", w, y))
        ops.append(op("cx", w, x))
        ops.append(op("ccx", x, y, w))

    def uma_ctrl(x, y, w, ctrl):
        # restores w and x; y ends as p ^ ctrl*(a ^ carry_in)
        ops.append(op("ccx", x, y, w))
        ops.append(op("cx", w, y))
        ops.append(op("ccx", ctrl, x, y))
        ops.append(op("cx", w, x))

    for i in range(bits):
        win = p[i:i + bits]
        carry_out = p[i + bits]
        # majority chain: carry ripples from the ancilla through a[0..w-1]
        prev = c
        for j in range(bits):
            maj(prev, win[j], a[j])
            prev = a[j]
        ops.append(op("ccx", b[i], a[bits - 1], carry_out))
        for j in reversed(range(bits)):
            prev = c if j == 0 else a[j - 1]
            uma_ctrl(prev, win[j], a[j], b[i])
    return Circuit(L.n, ops, 0, f"mult{bits}")


def multiplier_circuit(a_val: int, b_val: int, bits: int = 7, superpose_a: bool = False) -> Circuit:
    """Input preparation (X on the set bits of a and b, or H on every a qubit)
    followed by the multiplier core."""
    L = MultiplierLayout(bits)
    prep: List[Op] = []
    for j in range(bits):
        if superpose_a:
            prep.append(op("h", L.a[j]))
        elif (a_val >> j) & 1:
            prep.append(op("x", L.a[j]))
    for j in range(bits):
        if (b_val >> j) & 1:
            prep.append(op("x", L.b[j]))
    core = multiplier_core(bits)
    tag = "superpos" if superpose_a else f"a{a_val}"
    return Circuit(L.n, prep + core.ops, 0, f"mult{bits}_{tag}_b{b_val}")


def multiplier_inputs(count: int = 64, bits: int = 7, seed: int = 3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << bits, size=(count, 2))


# -------------------------------------------------------- width sweep

# grid shapes of the standard supremacy-style circuits the sweep cuts down
SWEEP_GRIDS = [(3, 4), (4, 4), (4, 5), (5, 5), (5, 6)]


def remove_qubits(circ: Circuit, width: int, seed: int) -> Circuit:
    """Drops circ.n - width qubits drawn at random (seeded) together with
    every op that touches one of them, and relabels the remaining qubits in
    increasing order: the way the paper reaches widths between the sizes its
    circuit generators produce (§II; the multipliers of §III.A the same way)."""
    if not 1 <= width <= circ.n:
        raise ValueError("width must be between 1 and the circuit's width")
    rng = np.random.default_rng(seed)
    drop = set(int(x) for x in rng.choice(circ.n, circ.n - width, replace=False))
    keep = [q for q in range(circ.n) if q not in drop]
    label = {q: i for i, q in enumerate(keep)}
    ops = [Op(o.kind, tuple(label[t] for t in o.targets), o.angles, o.param, o.matrix)
           for o in circ.ops if all(t in label for t in o.targets)]
    return Circuit(width, ops, circ.nparams, f"{circ.name}_keep{width}_s{seed}")


def width_circuit(family: str, width: int, seed: int = 6) -> Circuit:
    """A `width`-qubit circuit of the sweep, on an equal-superposition input
    (H on every qubit first, as the paper feeds both families).

    "supremacy": the smallest grid circuit of SWEEP_GRIDS (depth 20, seed 2)
    with at least `width` qubits; "multiplier": the smallest (4w+1)-qubit
    multiplier core with at least `width` qubits; either cut down to `width`
    by remove_qubits."""
    if family == "supremacy":
        rows, cols = next(rc for rc in SWEEP_GRIDS if rc[0] * rc[1] >= width)
        full = random_grid_circuit(rows, cols, depth=20, seed=2)
    elif family == "multiplier":
        bits = max(2, (width - 1 + 3) // 4)
        full = multiplier_core(bits)
    else:
        raise ValueError(f"unknown family {family!r}")
    cut = remove_qubits(full, width, seed) if full.n > width else full
    prep = [op("h", q) for q in range(width)]
    return Circuit(width, prep + cut.ops, 0, f"{family}{width}")


# -------------------------------------------------------- variational

def ansatz_circuit(n: int, layers: int) -> Circuit:
    """Per layer: RY then RZ on every qubit (parametric), then a CNOT ladder
    q -> q+1.  Parameter index p = (layer*n + q)*2 + r, r = 0 for RY, 1 for RZ."""
    ops: List[Op] = []
    for layer in range(layers):
        for q in range(n):
            base = (layer * n + q) * 2
            ops.append(op("ry", q, param=base))
            ops.append(op("rz", q, param=base + 1))
        for q in range(n - 1):
            ops.append(op("cx", q, q + 1))
    return Circuit(n, ops, 2 * n * layers, f"ansatz{n}_L{layers}")


def ansatz_params(n: int, layers: int, seed: int = 4) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, TWO_PI, size=2 * n * layers)


def chain_observable(n: int, x_coeff: float = 0.5) -> PauliSum:
    """Open-chain sum_i Z_i Z_{i+1} + x_coeff * sum_i X_i."""
    coeffs, xm, zm = [], [], []
    for i in range(n - 1):
        coeffs.append(1.0)
        xm.append(0)
        zm.append((1 << i) | (1 << (i + 1)))
    for i in range(n):
        coeffs.append(x_coeff)
        xm.append(1 << i)
        zm.append(0)
    return PauliSum(n, coeffs, xm, zm)


def random_pauli_sum(n: int, nterms: int, rng: np.random.Generator) -> PauliSum:
    coeffs = list(rng.standard_normal(nterms))
    xm = [int(v) for v in rng.integers(0, 1 << n, size=nterms)]
    zm = [int(v) for v in rng.integers(0, 1 << n, size=nterms)]
    return PauliSum(n, coeffs, xm, zm)


@dataclass
class BatchSpec:
    ns: np.ndarray        # qubit count per circuit
    layers: np.ndarray    # ansatz layers per circuit
    params: List[np.ndarray]


def batch_spec(count: int = 4096, nmin: int = 10, nmax: int = 20, lmin: int = 4,
               lmax: int = 12, seed: int = 5) -> BatchSpec:
    """Uneven batch of ansatz circuits: qubit counts uniform in [nmin, nmax],
    layers uniform in [lmin, lmax], per-circuit angles uniform in [0, 2pi)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    ls = rng.integers(lmin, lmax + 1, size=count)
    params = [rng.uniform(0.0, TWO_PI, size=2 * int(n) * int(L)) for n, L in zip(ns, ls)]
    return BatchSpec(ns, ls, params)


# ---------------------------------------------------------- closed-form circuits

def ghz_circuit(n: int) -> Circuit:
    ops = [op("h", 0)] + [op("cx", q, q + 1) for q in range(n - 1)]
    return Circuit(n, ops, 0, f"ghz{n}")


def qft_circuit(n: int) -> Circuit:
    """Textbook QFT on little-endian qubits: for the most significant qubit
    downwards, H then controlled phases pi/2^d from each lower qubit, and a
    final bit-reversal by swaps."""
    ops: List[Op] = []
    for j in reversed(range(n)):
        ops.append(op("h", j))
        for m in reversed(range(j)):
            ops.append(op("cp", m, j, angles=(np.pi / (1 << (j - m)),)))
    for q in range(n // 2):
        ops.append(op("swap", q, n - 1 - q))
    return Circuit(n, ops, 0, f"qft{n}")


def random_circuit(n: int, nops: int, rng: np.random.Generator, kinds: Optional[Sequence[str]] = None,
                   max_matrix_k: int = 3) -> Circuit:
    """Random mix of named gates and dense matrices on random (unsorted,
    non-adjacent) targets."""
    named = list(kinds) if kinds is not None else sorted(GATE_ARITY)
    ops: List[Op] = []
    for _ in range(nops):
        choice = rng.integers(0, len(named) + 1)
        if choice == len(named):
            k = int(rng.integers(1, min(max_matrix_k, n) + 1))
            tg = rng.choice(n, size=k, replace=False)
            ops.append(matrix_op(tg, random_unitary(k, rng)))
            continue
        kind = named[choice]
        ar = GATE_ARITY[kind]
        if ar > n:
            continue
        tg = rng.choice(n, size=ar, replace=False)
        angles = rng.uniform(0.0, TWO_PI, size=GATE_NANGLES.get(kind, 0))
        ops.append(op(kind, *tg, angles=angles))
    return Circuit(n, ops, 0, "random")


def random_state(n: int, rng: np.random.Generator, normalise: bool = True) -> np.ndarray:
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    if normalise:
        v /= np.sqrt(np.vdot(v, v).real)
    return v


def sample_indices(n: int, count: int, seed: int) -> np.ndarray:
    """Sorted distinct amplitude indices drawn uniformly from [0, 2^n)
    (numpy PCG64 seeded by `seed`); used to compare states too large to
    copy whole."""
    rng = np.random.default_rng(seed)
    idx = np.unique(rng.integers(0, 1 << n, size=count, dtype=np.uint64))
    return idx


def circuit_digest(circ: Circuit) -> str:
    """SHA-256 over the op list (kinds, qubits, angles, parameter slots,
    matrices): identifies a generated workload in stored reference files."""
    import hashlib
    h = hashlib.sha256()
    h.update(f"{circ.n}:{circ.nparams}".encode())
    for o in circ.ops:
        h.update(o.kind.encode())
        h.update(np.asarray(o.targets, dtype=np.int64).tobytes())
        h.update(np.asarray(o.angles, dtype=np.float64).tobytes())
        h.update(np.int64(o.param).tobytes())
        if o.matrix is not None:
            h.update(np.ascontiguousarray(o.matrix, dtype=np.complex128).tobytes())
    return h.hexdigest()
