"""Pins of the CPU oracle against what the definitions and the mathematics fix.

Every check here uses a route independent of the oracle's group-by-group
loops: Kronecker products, tensor contractions over a reshaped state, library
FFTs, closed forms, classical bit arithmetic, and brute-force dense matrices.
The simulated object is the paper's (Sec. I.A): a 2^n amplitude vector, each
gate a 2^n x 2^n matrix, the circuit their product (Sec. II).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

RNG_SEED = 20210629


# ------------------------------------------------------------- independent routes

PAULI = {
    "I": np.eye(2, dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def tensor_apply(psi, targets, U):
    """Apply U by contracting a reshaped (2,)*n tensor: axis n-1-q is qubit q,
    and U reshaped to (2,)*2k has row axis k-1-b for local bit b."""
    n = int(psi.size).bit_length() - 1
    k = len(targets)
    T = psi.reshape((2,) * n)
    Ut = U.reshape((2,) * (2 * k))
    col_axes = [k + (k - 1 - b) for b in range(k)]
    st_axes = [n - 1 - targets[b] for b in range(k)]
    R = np.tensordot(Ut, T, axes=(col_axes, st_axes))
    # R axes: U row axes (k of them, local bits k-1..0), then the remaining state axes in order
    rest = [a for a in range(n) if a not in st_axes]
    dest = [n - 1 - targets[k - 1 - i] for i in range(k)] + rest
    out = np.empty_like(T)
    out = np.moveaxis(R, list(range(n)), dest)
    return np.ascontiguousarray(out).reshape(-1)


def full_matrix(n, targets, U):
    """Dense 2^n x 2^n matrix of a gate, column by column through tensor_apply."""
    N = 1 << n
    M = np.zeros((N, N), dtype=np.complex128)
    for c in range(N):
        e = np.zeros(N, dtype=np.complex128)
        e[c] = 1
        M[:, c] = tensor_apply(e, list(targets), U)
    return M


def kron_chain(mats_high_to_low):
    out = np.array([[1.0 + 0j]])
    for m in mats_high_to_low:
        out = np.kron(out, m)
    return out


def pauli_dense(n, xmask, zmask):
    """Dense Pauli string from per-qubit 2x2 factors (Kronecker product, qubit 0
    rightmost); a qubit with both bits set carries Y."""
    facs = []
    for q in reversed(range(n)):
        xb, zb = (xmask >> q) & 1, (zmask >> q) & 1
        facs.append(PAULI["Y" if xb and zb else "X" if xb else "Z" if zb else "I"])
    return kron_chain(facs)


def op_matrix(o, params=None):
    if o.kind == "matrix":
        return o.matrix
    return O.gate_matrix(o.kind, O._op_angles(o, params))


def brute_force_circuit(circ, psi0, params=None):
    M = np.eye(1 << circ.n, dtype=np.complex128)
    for o in circ.ops:
        M = full_matrix(circ.n, o.targets, op_matrix(o, params)) @ M
    return M @ psi0


# ------------------------------------------------------------- gate matrices

def test_named_gate_matrices_textbook():
    r2 = 1 / np.sqrt(2)
    np.testing.assert_allclose(O.gate_matrix("h"), r2 * np.array([[1, 1], [1, -1]]), atol=1e-15)
    np.testing.assert_array_equal(O.gate_matrix("x"), PAULI["X"])
    np.testing.assert_array_equal(O.gate_matrix("y"), PAULI["Y"])
    np.testing.assert_array_equal(O.gate_matrix("z"), PAULI["Z"])
    np.testing.assert_allclose(O.gate_matrix("s") @ O.gate_matrix("s"), PAULI["Z"], atol=1e-15)
    np.testing.assert_allclose(np.linalg.matrix_power(O.gate_matrix("t"), 4), PAULI["Z"], atol=1e-15)
    np.testing.assert_allclose(O.gate_matrix("s") @ O.gate_matrix("sdg"), np.eye(2), atol=1e-15)
    np.testing.assert_allclose(O.gate_matrix("t") @ O.gate_matrix("tdg"), np.eye(2), atol=1e-15)


@pytest.mark.parametrize("th", [0.0, 0.3, 1.7, 4.0])
def test_rotations_are_exponentials_of_paulis(th):
    from scipy.linalg import expm
    for kind, P in (("rx", "X"), ("ry", "Y"), ("rz", "Z")):
        np.testing.assert_allclose(O.gate_matrix(kind, [th]), expm(-0.5j * th * PAULI[P]), atol=1e-14)
    # CP(p) = exp(i p |11><11|)
    P11 = np.diag([0, 0, 0, 1]).astype(np.complex128)
    np.testing.assert_allclose(O.gate_matrix("cp", [th]), expm(1j * th * P11), atol=1e-14)


def test_u3_special_cases():
    # U3(theta, -pi/2, pi/2) = RX(theta); U3(theta, 0, 0) = RY(theta);
    # U3(0, 0, lam) = diag(1, e^{i lam}); U3(pi/2, 0, pi) = H
    th = 0.77
    np.testing.assert_allclose(O.gate_matrix("u3", [th, -np.pi / 2, np.pi / 2]), O.gate_matrix("rx", [th]), atol=1e-14)
    np.testing.assert_allclose(O.gate_matrix("u3", [th, 0, 0]), O.gate_matrix("ry", [th]), atol=1e-15)
    np.testing.assert_allclose(O.gate_matrix("u3", [0, 0, 0.4]), np.diag([1, np.exp(0.4j)]), atol=1e-15)
    np.testing.assert_allclose(O.gate_matrix("u3", [np.pi / 2, 0, np.pi]), O.gate_matrix("h"), atol=1e-15)


def test_controlled_gates_as_projector_sums():
    # control = targets[0] is local bit 0: CX = |0><0|_c (x) I + |1><1|_c (x) X with the
    # target as the high local bit: kron(target_factor, control_factor)
    P0 = np.diag([1, 0]).astype(np.complex128)
    P1 = np.diag([0, 1]).astype(np.complex128)
    I2, X, Z = PAULI["I"], PAULI["X"], PAULI["Z"]
    np.testing.assert_array_equal(O.gate_matrix("cx"), np.kron(I2, P0) + np.kron(X, P1))
    np.testing.assert_array_equal(O.gate_matrix("cz"), np.kron(I2, P0) + np.kron(Z, P1))
    ccx = np.kron(I2, np.kron(I2, I2)) - np.kron(I2, np.kron(P1, P1)) + np.kron(X, np.kron(P1, P1))
    np.testing.assert_array_equal(O.gate_matrix("ccx"), ccx)
    ccz = np.eye(8) - 2 * np.kron(P1, np.kron(P1, P1))
    np.testing.assert_array_equal(O.gate_matrix("ccz"), ccz)
    sw = O.gate_matrix("swap")
    for a in range(2):
        for b in range(2):
            e = np.zeros(4)
            e[a + 2 * b] = 1
            assert np.argmax(sw @ e) == b + 2 * a


# ------------------------------------------------------------- gate application

@pytest.mark.parametrize("n", [1, 3, 5, 6])
def test_single_qubit_layer_is_kronecker_product(n):
    rng = np.random.default_rng(RNG_SEED + n)
    Us = [W.random_unitary(1, rng) for _ in range(n)]
    psi0 = W.random_state(n, rng)
    psi = psi0.copy()
    for q in range(n):
        O.apply_matrix(psi, [q], Us[q])
    ref = kron_chain(list(reversed(Us))) @ psi0
    assert O.rel_l2(psi, ref) < 1e-14


@pytest.mark.parametrize("n,q", [(4, 0), (4, 2), (6, 3)])
def test_adjacent_two_qubit_gate_is_kronecker_embedding(n, q):
    rng = np.random.default_rng(RNG_SEED + 10 * n + q)
    U = W.random_matrix(2, rng)
    psi0 = W.random_state(n, rng)
    psi = O.apply_matrix(psi0.copy(), [q, q + 1], U)
    full = kron_chain([np.eye(1 << (n - q - 2)), U, np.eye(1 << q)])
    assert O.rel_l2(psi, full @ psi0) < 1e-14


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_dense_gate_matches_tensor_contraction(k):
    n = 7
    rng = np.random.default_rng(RNG_SEED + k)
    for _ in range(4):
        tg = [int(t) for t in rng.choice(n, size=k, replace=False)]
        U = W.random_matrix(k, rng)
        psi0 = W.random_state(n, rng)
        psi = O.apply_matrix(psi0.copy(), tg, U)
        assert O.rel_l2(psi, tensor_apply(psi0, tg, U)) < 1e-13


def test_tensor_route_agrees_with_kronecker_route():
    # pins the helper itself on a case the Kronecker route covers
    rng = np.random.default_rng(RNG_SEED)
    U = W.random_matrix(2, rng)
    psi0 = W.random_state(5, rng)
    full = kron_chain([np.eye(2), U, np.eye(4)])
    assert O.rel_l2(tensor_apply(psi0, [2, 3], U), full @ psi0) < 1e-14


@pytest.mark.parametrize("n", [3, 5, 6])
def test_random_circuit_matches_dense_product(n):
    rng = np.random.default_rng(RNG_SEED + 100 + n)
    circ = W.random_circuit(n, 40, rng, max_matrix_k=min(n, 4))
    psi0 = W.random_state(n, rng)
    got = O.apply_circuit(circ, psi0)
    ref = brute_force_circuit(circ, psi0)
    assert O.rel_l2(got, ref) < 1e-13


def test_circuit_on_line_matches_dense_product():
    circ = W.random_line_circuit(n=6, depth=6, seed=7)
    ref = brute_force_circuit(circ, O.basis_state(6))
    assert O.rel_l2(O.apply_circuit(circ), ref) < 1e-13


def test_permutation_gates_two_forms_agree_exactly():
    rng = np.random.default_rng(RNG_SEED + 3)
    n = 6
    for kind in O.PERMUTATION_GATES:
        ar = W.GATE_ARITY[kind]
        for _ in range(5):
            tg = [int(t) for t in rng.choice(n, size=ar, replace=False)]
            psi0 = W.random_state(n, rng)
            a = O.apply_matrix(psi0.copy(), tg, O.gate_matrix(kind))
            b = O.apply_permutation(psi0.copy(), kind, tg)
            np.testing.assert_array_equal(a, b)


def test_norm_preserved_and_dagger_inverts():
    rng = np.random.default_rng(RNG_SEED + 4)
    n = 10
    circ = W.random_circuit(n, 200, rng, max_matrix_k=5)
    psi0 = W.random_state(n, rng)
    psi = O.apply_circuit(circ, psi0)
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-13
    back = O.apply_circuit(O.circuit_dagger(circ), psi)
    assert O.rel_l2(back, psi0) < 1e-13


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [2, 5, 12])
def test_ghz_closed_form(n):
    psi = O.apply_circuit(W.ghz_circuit(n))
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = ref[-1] = 1 / np.sqrt(2)
    assert np.max(np.abs(psi - ref)) < 1e-15


@pytest.mark.parametrize("n", [1, 3, 6, 10])
def test_qft_of_basis_state_matches_library_fft(n):
    N = 1 << n
    circ = W.qft_circuit(n)
    for x in sorted({0, 1, N // 3, N - 1}):
        psi = O.apply_circuit(circ, O.basis_state(n, x))
        e = np.zeros(N)
        e[x] = 1
        ref = np.sqrt(N) * np.fft.ifft(e)
        assert np.max(np.abs(psi - ref)) < 1e-13


def test_product_layer_closed_form_matches_full_run():
    circ = W.random_line_circuit(n=10, depth=1, seed=11)
    full = O.apply_circuit(circ)
    u3s = [o for o in circ.ops if o.kind == "u3"]
    pairs = [o.targets for o in circ.ops if o.kind == "cz"]
    idx = np.arange(1 << 10, dtype=np.uint64)
    amp = O.product_cz_amplitudes(10, u3s, pairs, idx)
    assert np.max(np.abs(amp - full)) < 1e-15


def test_grid_layer_closed_form_matches_full_run():
    # a 3x4 grid keeps the oracle run tiny; layer 0 is U3 everywhere + horizontal-even CZs
    circ = W.random_grid_circuit(rows=3, cols=4, depth=1, seed=12)
    full = O.apply_circuit(circ)
    u3s = [o for o in circ.ops if o.kind == "u3"]
    pairs = W.grid_cz_pairs(3, 4, 0)
    amp = O.product_cz_amplitudes(12, u3s, pairs, np.arange(1 << 12, dtype=np.uint64))
    assert np.max(np.abs(amp - full)) < 1e-15


# ------------------------------------------------------------- multiplier

def test_multiplier_classical_exhaustive():
    """Every (a, b) pair of the 7-bit multiplier: output index a + 2^7 b + 2^14 ab."""
    L = W.MultiplierLayout(7)
    core = W.multiplier_core(7)
    assert core.count("cx") == 196 and core.count("ccx") == 154
    a = np.repeat(np.arange(128, dtype=np.uint64), 128)
    b = np.tile(np.arange(128, dtype=np.uint64), 128)
    xs = a | (b << np.uint64(7))
    out = O.classical_run(core, xs)
    np.testing.assert_array_equal(out, a | (b << np.uint64(7)) | ((a * b) << np.uint64(14)))


@pytest.mark.parametrize("bits", [2, 3])
def test_multiplier_state_vector_basis_inputs_exact(bits):
    L = W.MultiplierLayout(bits)
    rng = np.random.default_rng(RNG_SEED + bits)
    for a, b in rng.integers(0, 1 << bits, size=(6, 2)):
        psi = O.apply_circuit(W.multiplier_circuit(int(a), int(b), bits))
        ref = np.zeros(1 << L.n, dtype=np.complex128)
        ref[L.basis_index(int(a), int(b), int(a * b))] = 1.0
        np.testing.assert_array_equal(psi, ref)


def test_multiplier_superposition_closed_form():
    bits = 3
    L = W.MultiplierLayout(bits)
    b = 5
    psi = O.apply_circuit(W.multiplier_circuit(0, b, bits, superpose_a=True))
    ref = np.zeros(1 << L.n, dtype=np.complex128)
    for a in range(1 << bits):
        ref[L.basis_index(a, b, a * b)] = 2.0 ** (-bits / 2)
    assert np.max(np.abs(psi - ref)) < 1e-15


# ------------------------------------------------------------- expectation

@pytest.mark.parametrize("n", [1, 3, 5])
def test_expectation_matches_dense_pauli_sum(n):
    rng = np.random.default_rng(RNG_SEED + 50 + n)
    H = W.random_pauli_sum(n, 12, rng)
    psi = W.random_state(n, rng)
    Hd = sum(c * pauli_dense(n, x, z) for c, x, z in zip(H.coeffs, H.xmasks, H.zmasks))
    ref = np.vdot(psi, Hd @ psi).real
    assert abs(O.expectation(psi, H) - ref) < 1e-13
    for x, z in zip(H.xmasks, H.zmasks):
        assert O.rel_l2(O.pauli_apply(psi, x, z), pauli_dense(n, x, z) @ psi) < 1e-14


def test_expectation_product_state_factorises():
    n = 8
    circ = W.random_line_circuit(n=n, depth=1, seed=3)
    u3s = W.Circuit(n, [o for o in circ.ops if o.kind == "u3"])
    psi = O.apply_circuit(u3s)
    H = W.chain_observable(n)
    # single-qubit Bloch components from each qubit's own 2-vector
    bz, bx = [], []
    for o in u3s.ops:
        v = O.gate_matrix("u3", o.angles)[:, 0]
        bz.append(abs(v[0]) ** 2 - abs(v[1]) ** 2)
        bx.append(2 * (np.conj(v[0]) * v[1]).real)
    ref = sum(bz[i] * bz[i + 1] for i in range(n - 1)) + 0.5 * sum(bx)
    assert abs(O.expectation(psi, H) - ref) < 1e-13


def test_expectation_ghz():
    n = 6
    psi = O.apply_circuit(W.ghz_circuit(n))
    H = W.chain_observable(n)
    assert abs(O.expectation(psi, H) - (n - 1)) < 1e-14


# ------------------------------------------------------------- gradients

@pytest.mark.parametrize("th", [0.1, 1.3, 2.9, 5.0])
def test_single_rotation_gradient_closed_form(th):
    circ = W.Circuit(1, [W.op("ry", 0, param=0)], 1)
    H = W.PauliSum(1, [1.0], [0], [1])
    p = np.array([th])
    assert abs(O.energy(circ, p, H) - np.cos(th)) < 1e-15
    assert abs(O.param_shift_grad(circ, p, H)[0] + np.sin(th)) < 1e-14
    assert abs(O.finite_diff_grad(circ, p, H)[0] + np.sin(th)) < 1e-8


def test_param_shift_matches_finite_differences():
    n, L = 4, 3
    circ = W.ansatz_circuit(n, L)
    p = W.ansatz_params(n, L, seed=9)
    H = W.chain_observable(n)
    ps = O.param_shift_grad(circ, p, H)
    fd = O.finite_diff_grad(circ, p, H, h=1e-4)
    assert np.max(np.abs(ps - fd)) < 1e-7


def test_param_shift_matches_analytic_dense_derivative():
    """d/dtheta exp(-i theta P/2) = -(i/2) P exp(-i theta P/2), inserted into the dense
    product of full 2^n x 2^n matrices."""
    n, L = 3, 2
    circ = W.ansatz_circuit(n, L)
    p = W.ansatz_params(n, L, seed=10)
    H = W.chain_observable(n)
    Hd = sum(c * pauli_dense(n, x, z) for c, x, z in zip(H.coeffs, H.xmasks, H.zmasks))
    mats = [full_matrix(n, o.targets, op_matrix(o, p)) for o in circ.ops]
    gen = {"ry": "Y", "rz": "Z", "rx": "X"}
    psi0 = O.basis_state(n)
    grad = np.zeros(p.size)
    for i, o in enumerate(circ.ops):
        if o.param < 0:
            continue
        M = np.eye(1 << n, dtype=np.complex128)
        dM = np.eye(1 << n, dtype=np.complex128)
        for j, Mj in enumerate(mats):
            M = Mj @ M
            if j == i:
                G = full_matrix(n, o.targets, PAULI[gen[o.kind]])
                dM = (-0.5j * G @ Mj) @ dM
            else:
                dM = Mj @ dM
        psi, dpsi = M @ psi0, dM @ psi0
        grad[o.param] += 2 * np.vdot(psi, Hd @ dpsi).real
    assert np.max(np.abs(O.param_shift_grad(circ, p, H) - grad)) < 1e-12


def test_cp_shift_rule_matches_finite_differences():
    n = 3
    ops = [W.op("h", 0), W.op("h", 1), W.op("ry", 2, angles=(0.4,)),
           W.op("cp", 0, 1, param=0), W.op("cp", 1, 2, param=1), W.op("h", 1)]
    circ = W.Circuit(n, ops, 2)
    H = W.chain_observable(n)
    p = np.array([0.7, 2.1])
    assert np.max(np.abs(O.param_shift_grad(circ, p, H) - O.finite_diff_grad(circ, p, H))) < 1e-8
