"""Big-endian (Cirq-order) front end against an independent big-endian
construction: textbook matrices with the op's first qubit as the most
significant bit, applied by tensor contraction on the axis of each qubit of a
state vector whose axis 0 is qubit 0; Pauli operators as Kronecker products
with qubit 0 leftmost."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2106_13995_amd import frontend as F

SQ2 = 1 / np.sqrt(2)
X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]])
Z = np.diag([1.0 + 0j, -1.0])


def textbook(kind, angles):
    if kind == "h":
        return np.array([[SQ2, SQ2], [SQ2, -SQ2]], dtype=complex)
    if kind == "x":
        return X
    if kind == "u3":
        th, ph, la = angles
        c, s = np.cos(th / 2), np.sin(th / 2)
        return np.array([[c, -np.exp(1j * la) * s], [np.exp(1j * ph) * s, np.exp(1j * (ph + la)) * c]])
    if kind == "cx":          # (control, target), control the high bit
        M = np.eye(4, dtype=complex); M[2:, 2:] = X
        return M
    if kind == "ccx":
        M = np.eye(8, dtype=complex); M[6:, 6:] = X
        return M
    if kind == "cz":
        return np.diag([1, 1, 1, -1.0 + 0j])
    raise KeyError(kind)


def big_endian_run(circ):
    n = circ.n
    psi = np.zeros((2,) * n, dtype=complex)
    psi[(0,) * n] = 1.0
    for o in circ.ops:
        M = o.matrix if o.kind == "matrix" else textbook(o.kind, o.angles)
        k = len(o.targets)
        T = M.reshape((2,) * (2 * k))
        psi = np.tensordot(T, psi, axes=(list(range(k, 2 * k)), list(o.targets)))
        # tensordot puts the op's axes first, in target order: move them back
        psi = np.moveaxis(psi, list(range(k)), list(o.targets))
    return psi.reshape(-1)


def random_big_endian_circuit(n, nops, rng):
    ops = []
    for _ in range(nops):
        r = rng.integers(6)
        if r == 0:
            ops.append(W.op("h", int(rng.integers(n))))
        elif r == 1:
            ops.append(W.op("u3", int(rng.integers(n)), angles=rng.uniform(0, 2 * np.pi, 3)))
        elif r == 2:
            a, b = rng.choice(n, 2, replace=False)
            ops.append(W.op("cx", int(a), int(b)))
        elif r == 3:
            a, b, c = rng.choice(n, 3, replace=False)
            ops.append(W.op("ccx", int(a), int(b), int(c)))
        elif r == 4:
            a, b = rng.choice(n, 2, replace=False)
            ops.append(W.op("cz", int(a), int(b)))
        else:
            qs = [int(q) for q in rng.choice(n, 2, replace=False)]
            ops.append(W.matrix_op(qs, W.random_unitary(2, rng)))
    return W.Circuit(n, ops)


def big_endian_pauli(n, x, z):
    """Dense P for masks whose bit q is qubit q, qubit 0 leftmost."""
    P = np.eye(1, dtype=complex)
    for q in range(n):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        f = Y if (xb and zb) else X if xb else Z if zb else np.eye(2)
        P = np.kron(P, f)
    return P


def test_reverse_mask():
    assert F.reverse_mask(0b00011, 5) == 0b11000
    assert F.reverse_mask(0, 5) == 0
    with pytest.raises(ValueError):
        F.reverse_mask(1 << 5, 5)


def test_from_big_endian_matches_big_endian_construction():
    n = 6
    rng = np.random.default_rng(301)
    circ = random_big_endian_circuit(n, 60, rng)
    ref = big_endian_run(circ)
    lib = O.apply_circuit(F.from_big_endian(circ))
    # the relabelled circuit's state vector is already indexed in big-endian order
    np.testing.assert_allclose(lib, ref, atol=1e-12)


def test_pauli_from_big_endian():
    n = 5
    rng = np.random.default_rng(302)
    circ = random_big_endian_circuit(n, 30, rng)
    ref = big_endian_run(circ)
    lib = O.apply_circuit(F.from_big_endian(circ))
    H = W.random_pauli_sum(n, 12, rng)
    dense = sum(c * big_endian_pauli(n, x, z) for c, x, z in zip(H.coeffs, H.xmasks, H.zmasks))
    want = np.vdot(ref, dense @ ref).real
    assert abs(O.expectation(lib, F.pauli_from_big_endian(H)) - want) < 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_big_endian_on_gpu(dtype):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_13995_amd as q
    n = 14
    rng = np.random.default_rng(303)
    circ = random_big_endian_circuit(n, 120, rng)
    ref = big_endian_run(circ)
    s = q.State(n, dtype)
    s.apply_circuit(F.from_big_endian(circ))
    tol = 2e-5 if dtype == "c64" else 1e-12
    assert O.rel_l2(s.to_numpy(), ref) <= tol
    s.close()
    # Pauli sums, on a width where the dense operator is small
    m = 8
    circ = random_big_endian_circuit(m, 40, rng)
    s = q.State(m, dtype)
    s.apply_circuit(F.from_big_endian(circ))
    H = W.random_pauli_sum(m, 10, rng)
    dense = sum(c * big_endian_pauli(m, x, z) for c, x, z in zip(H.coeffs, H.xmasks, H.zmasks))
    psi = s.to_numpy().astype(complex)
    want = np.vdot(psi, dense @ psi).real
    assert abs(s.expectation(F.pauli_from_big_endian(H)) - want) <= 1e-10 * sum(abs(c) for c in H.coeffs)
    s.close()
