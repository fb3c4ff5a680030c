"""Big-endian qubit order at the Python boundary.

The paper's simulator sits inside Cirq (§II) and keeps Cirq's conventions:
qubit 0 is the most significant bit of a state-vector index, and a gate's
matrix on qubits (q_0, ..., q_{k-1}) is indexed with q_0 as its most
significant bit.  The library numbers qubits the other way (qubit q is bit q
of the index, and bit b of a matrix index belongs to the op's b-th target).
Naming the user's qubit q as the library's qubit n-1-q gives every qubit the
index weight it has in Cirq's order, so after the circuit (and any Pauli sum)
is relabelled the state vector needs no permutation: what goes in and comes
out of a State is already in Cirq's order.  Only host-side relabelling
happens here; every gate still runs in the library's kernels.

    state.apply_circuit(from_big_endian(circ))   # circ written in Cirq's order
    psi = state.to_numpy()                        # indexed in Cirq's order
    e = state.expectation(pauli_from_big_endian(H))
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class FrontOp:
    kind: str
    targets: Tuple[int, ...]
    angles: Tuple[float, ...] = ()
    param: int = -1
    matrix: Optional[np.ndarray] = field(default=None, compare=False, hash=False)

    @property
    def k(self) -> int:
        return len(self.targets)


@dataclass
class FrontCircuit:
    n: int
    ops: List[FrontOp]
    nparams: int = 0
    name: str = ""


@dataclass
class FrontPauliSum:
    n: int
    coeffs: List[float]
    xmasks: List[int]
    zmasks: List[int]


def _flip(q: int, n: int) -> int:
    if not 0 <= q < n:
        raise ValueError(f"qubit {q} outside 0..{n - 1}")
    return n - 1 - q


def from_big_endian(circ) -> FrontCircuit:
    """The same circuit in the library's order: qubit q becomes n-1-q, and a
    matrix op's target list is reversed (its first qubit is the matrix
    index's most significant bit, which the library takes from the last
    target).  Named gates keep their argument order (control first)."""
    n = circ.n
    ops = []
    for o in circ.ops:
        t = tuple(_flip(int(q), n) for q in o.targets)
        if o.kind == "matrix":
            t = t[::-1]
        ops.append(FrontOp(o.kind, t, tuple(o.angles), int(o.param), getattr(o, "matrix", None)))
    return FrontCircuit(n, ops, getattr(circ, "nparams", 0), getattr(circ, "name", ""))


def reverse_mask(mask: int, n: int) -> int:
    """Bit q of `mask` moved to bit n-1-q."""
    if mask >> n:
        raise ValueError("mask has a bit at or above n")
    out = 0
    for q in range(n):
        if (mask >> q) & 1:
            out |= 1 << (n - 1 - q)
    return out


def pauli_from_big_endian(H) -> FrontPauliSum:
    """A Pauli sum whose X and Z masks use bit q for Cirq's qubit q, in the
    library's order."""
    return FrontPauliSum(H.n, list(H.coeffs), [reverse_mask(int(x), H.n) for x in H.xmasks],
                         [reverse_mask(int(z), H.n) for z in H.zmasks])
