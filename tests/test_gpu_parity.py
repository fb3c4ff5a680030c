"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle.

Bars (amplitudes, relative L2 against the complex128 oracle):
complex128 <= 1e-12, complex64 <= 2e-5.  Permutation-only circuits on basis
inputs are compared bit for bit.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c64": 2e-5, "c128": 1e-12}
MODES = {
    "sweep": dict(fuse_k=1, tile_m=-1),
    "tile": dict(fuse_k=1, tile_m=0),
    "tile9": dict(fuse_k=1, tile_m=9),
    "fuse2": dict(fuse_k=2, tile_m=-1),
    "fuse3": dict(fuse_k=3, tile_m=-1),
    "fuse4": dict(fuse_k=4, tile_m=-1),
    "fuse5": dict(fuse_k=5, tile_m=-1),
    "fuse6": dict(fuse_k=6, tile_m=-1),
    "fuse5_lds": dict(fuse_k=5, tile_m=-1, use_mfma=-1),
    "fuse3_tile": dict(fuse_k=3, tile_m=0),
    "fuse5_tile": dict(fuse_k=5, tile_m=0),
    "tile_complex": dict(fuse_k=1, tile_m=0, split_1q=-1),
    "tile12_split": dict(fuse_k=1, tile_m=12, split_1q=1),
    "fuse2_tile": dict(fuse_k=2, tile_m=0),
    "tile13": dict(fuse_k=1, tile_m=13),
    # tiles narrower than the low qubits plus the widest gate: widened by the
    # planner (gates outside the low 5 / 4 qubits need more positions)
    "tile7": dict(fuse_k=1, tile_m=7),
    "fuse5_tile9": dict(fuse_k=5, tile_m=9),
    "fuse6_tile10": dict(fuse_k=6, tile_m=10),
}


@pytest.fixture(scope="module")
def qs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_13995_amd as q
    return q


def _state(q, n, dtype, psi0=None):
    s = q.State(n, dtype)
    if psi0 is not None:
        s.from_numpy(psi0)
    return s


def _rounded(psi, dtype):
    """The input as the device holds it, back in complex128."""
    return psi.astype(np.complex64).astype(np.complex128) if dtype == "c64" else psi.copy()


# ------------------------------------------------------------ single gates

@pytest.mark.parametrize("n", [7, 14])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_one_qubit_gate_every_target(qs, dtype, n):
    # (complex64 targets 1..6 take the lane-exchange sweep; at n = 7 its
    # grid is one partly filled workgroup)
    rng = np.random.default_rng(101)
    psi0 = _rounded(W.random_state(n, rng), dtype)
    s = _state(qs, n, dtype, psi0)
    ref = psi0.copy()
    for t in range(n):
        U = W.random_unitary(1, rng)
        s.apply_gate([t], U)
        O.apply_matrix(ref, [t], U)
    assert O.rel_l2(s.to_numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_two_qubit_gate_all_ordered_pairs(qs, dtype):
    n = 10
    rng = np.random.default_rng(102)
    psi0 = _rounded(W.random_state(n, rng), dtype)
    s = _state(qs, n, dtype, psi0)
    ref = psi0.copy()
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            U = W.random_unitary(2, rng)
            s.apply_gate([a, b], U)
            O.apply_matrix(ref, [a, b], U)
    assert O.rel_l2(s.to_numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("n", [7, 13])
def test_gates_lane_exchange(qs, n):
    """Complex64 dense gates without controls run as lane-exchange sweeps:
    targets among qubits 0..6 keep their lane bits, higher ones take the top
    lane bits (qubit 0 with or without others, any order, one to three
    targets); at n = 7 the grid is one partly filled workgroup."""
    rng = np.random.default_rng(107 + n)
    psi0 = _rounded(W.random_state(n, rng), "c64")
    s = _state(qs, n, "c64", psi0)
    ref = psi0.copy()
    cases = [[0, 1], [1, 0], [0, 6], [5, 2], [6, 3], [0, 1, 2], [2, 0, 1], [1, 4, 6], [6, 5, 0], [3, 1, 5], [0], [3]]
    if n > 7:
        cases += [[n - 1], [n - 2, n - 1], [0, n - 1], [3, n - 1], [2, 7, n - 1], [n - 1, 0, 6], [7, 8, 9]]
    cases += [[int(t) for t in rng.choice(n, size=int(k), replace=False)] for k in rng.integers(1, 4, size=16)]
    for tg in cases:
        U = W.random_unitary(len(tg), rng)
        s.apply_gate(tg, U)
        O.apply_matrix(ref, tg, U)
    assert O.rel_l2(s.to_numpy(), ref) <= TOL["c64"]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_dense_k_qubit_gates_sampled_targets(qs, dtype, k):
    n = 15
    rng = np.random.default_rng(103 + k)
    psi0 = _rounded(W.random_state(n, rng), dtype)
    s = _state(qs, n, dtype, psi0)
    ref = psi0.copy()
    target_sets = [list(range(k)), list(range(n - k, n))[::-1]]
    target_sets += [[int(t) for t in rng.choice(n, size=k, replace=False)] for _ in range(6)]
    for tg in target_sets:
        U = W.random_unitary(k, rng)
        s.apply_gate(tg, U)
        O.apply_matrix(ref, tg, U)
    assert O.rel_l2(s.to_numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_non_unitary_matrix(qs, dtype):
    # the ABI applies any matrix (a projector-like random matrix here)
    n = 12
    rng = np.random.default_rng(104)
    psi0 = _rounded(W.random_state(n, rng), dtype)
    s = _state(qs, n, dtype, psi0)
    ref = psi0.copy()
    for tg in ([0], [11, 3], [5, 9, 1]):
        M = W.random_matrix(len(tg), rng) * 0.5
        s.apply_gate(tg, M)
        O.apply_matrix(ref, tg, M)
    assert O.rel_l2(s.to_numpy(), ref) <= TOL[dtype]


# ------------------------------------------------------------ circuits

@pytest.mark.parametrize("mode", sorted(MODES))
def test_line12_c128_depth20(qs, mode):
    """12-qubit random circuit, complex128, depth 20 from |0...0>."""
    circ = W.random_line_circuit(12, 20, seed=1)
    ref = O.apply_circuit(circ)
    s = _state(qs, 12, "c128")
    s.apply_circuit(circ, **MODES[mode])
    assert O.rel_l2(s.to_numpy(), ref) <= TOL["c128"]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("mode", sorted(MODES))
def test_random_mixed_circuit(qs, dtype, mode):
    n = 14
    rng = np.random.default_rng(105)
    circ = W.random_circuit(n, 120, rng, max_matrix_k=4)
    psi0 = _rounded(W.random_state(n, rng), dtype)
    ref = O.apply_circuit(circ, psi0)
    s = _state(qs, n, dtype, psi0)
    s.apply_circuit(circ, **MODES[mode])
    assert O.rel_l2(s.to_numpy(), ref) <= TOL[dtype]


def controlled_circuit(n, nops, rng):
    """U3 gates, CX / CCX, and dense matrices that are a random 2 x 2 block
    under one or two controls (identity elsewhere), on random qubits: in a
    12-qubit tile of a 14-qubit state the controls land on register, thread
    and out-of-tile bits."""
    ops = []
    for _ in range(nops):
        kind = rng.integers(4)
        if kind == 0:
            ops.append(W.op("u3", int(rng.integers(n)), angles=rng.uniform(0, 2 * np.pi, 3)))
        elif kind == 1:
            a, b = rng.choice(n, 2, replace=False)
            ops.append(W.op("cx", int(a), int(b)))
        elif kind == 2:
            a, b, c = rng.choice(n, 3, replace=False)
            ops.append(W.op("ccx", int(a), int(b), int(c)))
        else:
            nc = int(rng.integers(1, 3))
            qs_ = [int(x) for x in rng.choice(n, nc + 1, replace=False)]
            d = 1 << (nc + 1)
            M = np.eye(d, dtype=np.complex128)
            M[d - 2:, d - 2:] = W.random_unitary(1, rng)
            # target = qs_[0] is matrix bit 0; every control bit is 1 on the last two rows
            ops.append(W.matrix_op(qs_, M))
    return W.Circuit(n, ops)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("mode", ["sweep", "tile", "tile12_split", "fuse2_tile", "fuse5_tile"])
def test_controlled_blocks(qs, dtype, mode):
    n = 14
    rng = np.random.default_rng(111)
    circ = controlled_circuit(n, 160, rng)
    psi0 = _rounded(W.random_state(n, rng), dtype)
    ref = O.apply_circuit(circ, psi0)
    s = _state(qs, n, dtype, psi0)
    s.apply_circuit(circ, **MODES[mode])
    assert O.rel_l2(s.to_numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("family", ["supremacy", "multiplier"])
@pytest.mark.parametrize("n", [13, 14])
def test_width_sweep_circuits(qs, dtype, family, n):
    """The width sweep's cut-down circuits on their superposition input,
    with the library's automatic options (the sweep runs those)."""
    circ = W.width_circuit(family, n)
    s = _state(qs, n, dtype)
    s.apply_circuit(circ)
    assert O.rel_l2(s.to_numpy(), O.apply_circuit(circ)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("mode", ["sweep", "tile", "fuse4", "fuse5_tile"])
def test_grid_circuit_16q(qs, dtype, mode):
    circ = W.random_grid_circuit(4, 4, depth=12, seed=2)
    ref = O.apply_circuit(circ)
    s = _state(qs, 16, dtype)
    s.apply_circuit(circ, **MODES[mode])
    assert O.rel_l2(s.to_numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("mode", ["sweep", "tile", "fuse3", "fuse3_tile", "fuse6"])
def test_small_registers(qs, n, mode):
    rng = np.random.default_rng(106 + n)
    circ = W.random_circuit(n, 30, rng, max_matrix_k=min(n, 3))
    psi0 = W.random_state(n, rng)
    ref = O.apply_circuit(circ, psi0)
    s = _state(qs, n, "c128", psi0)
    s.apply_circuit(circ, **MODES[mode])
    assert O.rel_l2(s.to_numpy(), ref) <= TOL["c128"]


def test_repeated_calls_use_cached_plan(qs):
    circ = W.random_line_circuit(13, 6, seed=8)
    s = _state(qs, 13, "c128")
    for _ in range(3):
        s.apply_circuit(circ, fuse_k=3, tile_m=0)
    ref = O.basis_state(13)
    for _ in range(3):
        ref = O.apply_circuit(circ, ref)
    assert O.rel_l2(s.to_numpy(), ref) <= TOL["c128"]


@pytest.mark.parametrize("mode", ["sweep", "tile", "fuse3"])
def test_parametric_circuit(qs, mode):
    n, L = 10, 3
    circ = W.ansatz_circuit(n, L)
    p = W.ansatz_params(n, L, seed=4)
    ref = O.apply_circuit(circ, params=p)
    s = _state(qs, n, "c128")
    s.apply_circuit(circ, params=p, **MODES[mode])
    assert O.rel_l2(s.to_numpy(), ref) <= TOL["c128"]
    # a second parameter vector on a fresh state
    p2 = p + 0.37
    s.set_basis(0)
    s.apply_circuit(circ, params=p2, **MODES[mode])
    assert O.rel_l2(s.to_numpy(), O.apply_circuit(circ, params=p2)) <= TOL["c128"]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("k", [4, 5, 6])
def test_mfma_block_every_placement(qs, dtype, k):
    """Fused dense blocks on the matrix cores: low, high, mixed and scattered
    targets, including registers smaller than one 64-row workgroup tile."""
    rng = np.random.default_rng(120 + k)
    for n in (k, k + 3, 16):
        psi0 = _rounded(W.random_state(n, rng), dtype)
        s = _state(qs, n, dtype, psi0)
        ref = psi0.copy()
        sets = [list(range(k)), list(range(n - k, n)), [int(t) for t in rng.choice(n, size=k, replace=False)]]
        for tg in sets:
            U = W.random_unitary(k, rng)
            s.apply_gate(tg, U)
            O.apply_matrix(ref, tg, U)
        assert O.rel_l2(s.to_numpy(), ref) <= TOL[dtype], n
        s.close()


# ------------------------------------------------------------ closed forms through the oracle

@pytest.mark.parametrize("mode", ["sweep", "tile", "fuse4"])
def test_ghz_and_qft(qs, mode):
    n = 16
    s = _state(qs, n, "c128")
    s.apply_circuit(W.ghz_circuit(n), **MODES[mode])
    assert O.rel_l2(s.to_numpy(), O.apply_circuit(W.ghz_circuit(n))) <= TOL["c128"]
    x = 12345
    s.set_basis(x)
    s.apply_circuit(W.qft_circuit(n), **MODES[mode])
    ref = O.apply_circuit(W.qft_circuit(n), O.basis_state(n, x))
    assert O.rel_l2(s.to_numpy(), ref) <= TOL["c128"]


@pytest.mark.parametrize("mode", ["sweep", "tile", "fuse3", "fuse6"])
def test_multiplier_basis_inputs_bit_exact(qs, mode):
    bits = 3
    L = W.MultiplierLayout(bits)
    rng = np.random.default_rng(107)
    for a, b in rng.integers(0, 1 << bits, size=(4, 2)):
        circ = W.multiplier_circuit(int(a), int(b), bits)
        s = _state(qs, L.n, "c64")
        s.apply_circuit(circ, **MODES[mode])
        got = s.to_numpy()
        expect_index = int(O.classical_run(circ, [0])[0])
        assert expect_index == L.basis_index(int(a), int(b), int(a * b))
        ref = np.zeros(1 << L.n, dtype=np.complex64)
        ref[expect_index] = 1.0
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_multiplier_superposition(qs, dtype):
    bits = 3
    circ = W.multiplier_circuit(0, 5, bits, superpose_a=True)
    ref = O.apply_circuit(circ)
    s = _state(qs, W.MultiplierLayout(bits).n, dtype)
    s.apply_circuit(circ, fuse_k=1, tile_m=-1)
    assert O.rel_l2(s.to_numpy(), ref) <= TOL[dtype]


# ------------------------------------------------------------ expectation

@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n", [1, 4, 11, 17])
def test_expectation_random_pauli_sums(qs, dtype, n):
    rng = np.random.default_rng(108 + n)
    H = W.random_pauli_sum(n, 25, rng)
    psi = _rounded(W.random_state(n, rng), dtype)
    s = _state(qs, n, dtype, psi)
    got = s.expectation(H)
    ref = O.expectation(psi, H)
    scale = sum(abs(c) for c in H.coeffs)
    assert abs(got - ref) <= 1e-12 * scale
    # deterministic reduction: bitwise identical on repeat
    assert s.expectation(H) == got


def test_expectation_chain_observable_after_circuit(qs):
    n = 14
    circ = W.random_line_circuit(n, 8, seed=9)
    s = _state(qs, n, "c128")
    s.apply_circuit(circ, tile_m=0)
    H = W.chain_observable(n)
    ref = O.expectation(O.apply_circuit(circ), H)
    assert abs(s.expectation(H) - ref) < 1e-11


def test_expectation_empty_sum(qs):
    s = _state(qs, 5, "c64")
    assert s.expectation(W.PauliSum(5, [], [], [])) == 0.0


# ------------------------------------------------------------ error handling on a live state

def test_invalid_gate_leaves_state_unchanged(qs):
    n = 9
    rng = np.random.default_rng(110)
    psi0 = W.random_state(n, rng)
    s = _state(qs, n, "c128", psi0)
    with pytest.raises(qs.QsimError):
        s.apply_gate([3, 3], np.eye(4))
    with pytest.raises(qs.QsimError):
        s.apply_circuit(W.Circuit(n, [W.op("h", 1), W.Op("cx", (2, 9))]))
    np.testing.assert_array_equal(s.to_numpy(), psi0)


def test_autotune_choice_is_used_and_correct(qs, tmp_path, monkeypatch):
    circ = W.random_grid_circuit(4, 4, depth=12, seed=3)
    s = _state(qs, 16, "c64")
    best, ms = s.autotune(circ, reps=1)
    assert ms > 0
    assert best["fuse_k"] in range(1, 7) and best["tile_m"] in (-1, 11, 12, 13)
    # automatic options now take the tuned choice; results stay within the bar
    s.set_basis(0)
    s.apply_circuit(circ)
    assert O.rel_l2(s.to_numpy(), O.apply_circuit(circ)) <= TOL["c64"]
    s.close()


def _simple_sum(n, rng, diag=True, xs_on=True, ys_on=True, low_only=False):
    """Diagonal terms with random Z masks (register, lane and block qubits
    alike) and X_h / Y_h terms: the sums the register passes take."""
    coeffs, xs, zs = [], [], []
    if diag:
        for _ in range(12):
            coeffs.append(float(rng.normal())); xs.append(0); zs.append(int(rng.integers(0, 1 << n)))
        for i in range(n - 1):
            coeffs.append(float(rng.normal())); xs.append(0); zs.append((1 << i) | (1 << (i + 1)))
    qubits = range(min(n, 4)) if low_only else range(n)
    for h in qubits:
        if xs_on:
            coeffs.append(float(rng.normal())); xs.append(1 << h); zs.append(0)
        if ys_on and rng.random() < 0.6:
            coeffs.append(float(rng.normal())); xs.append(1 << h); zs.append(1 << h)
    return W.PauliSum(n, coeffs, xs, zs)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n", [10, 11, 13, 17])
def test_expectation_register_passes(qs, dtype, n):
    """Sums of diagonal terms and single-qubit X / Y terms (the register
    passes, one or more per sum, from the smallest width they take): against
    the oracle on the device's rounded amplitudes, with parts left out."""
    rng = np.random.default_rng(1200 + n)
    psi = _rounded(W.random_state(n, rng), dtype)
    s = _state(qs, n, dtype, psi)
    cases = [_simple_sum(n, rng), _simple_sum(n, rng, diag=False), _simple_sum(n, rng, xs_on=False),
             _simple_sum(n, rng, xs_on=False, ys_on=False), _simple_sum(n, rng, diag=False, low_only=True)]
    for H in cases:
        got = s.expectation(H)
        ref = O.expectation(psi, H)
        scale = sum(abs(c) for c in H.coeffs)
        assert abs(got - ref) <= 1e-12 * scale, (len(H.coeffs), got, ref)
        assert s.expectation(H) == got
    s.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_expectation_tiled_and_wide_groups(qs, dtype):
    """Several X-mask groups per pass over the state (single X and Y terms,
    diagonal ZZ terms with bits inside and outside a tile) next to groups whose
    X mask is too wide for one tile (evaluated alone), at 20 qubits."""
    n = 20
    rng = np.random.default_rng(109)
    psi = _rounded(W.random_state(n, rng), dtype)
    coeffs, xs, zs = [], [], []
    for i in range(n):
        coeffs.append(0.5 + 0.1 * i); xs.append(1 << i); zs.append(0)              # X_i
        coeffs.append(-0.3); xs.append(1 << i); zs.append(1 << i)                   # Y_i
        coeffs.append(1.0); xs.append(0); zs.append((1 << i) | (1 << ((i + 7) % n)))  # Z_i Z_{i+7}
    for _ in range(6):                                                              # wide X masks
        xm = int(rng.integers(1, 1 << n)) | (0xFF << 10)
        coeffs.append(float(rng.normal())); xs.append(xm); zs.append(int(rng.integers(0, 1 << n)))
    H = W.PauliSum(n, coeffs, xs, zs)
    s = _state(qs, n, dtype, psi)
    got = s.expectation(H)
    # the device reads the same (rounded) amplitudes the oracle is given and
    # accumulates in double: only summation order separates the two
    ref = O.expectation(psi, H)
    scale = sum(abs(c) for c in H.coeffs)
    assert abs(got - ref) <= 1e-10 * scale, (got, ref)
    s.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_expectation_product_state_terms_of_order_one(qs, dtype):
    """A product state where every term of the chain observable and of single
    Y terms is O(1), so a dropped, doubled or sign-flipped term moves the sum
    by O(1): against the oracle on the rounded input and the product closed
    form (<Z_i Z_j> = <Z_i><Z_j>, <X_i>, <Y_i> from each qubit's Bloch vector)."""
    n = 20
    rng = np.random.default_rng(113)
    ops = [W.op("u3", qb, angles=(0.3 + 0.1 * (qb % 7), 0.2 * qb, 0.0)) for qb in range(n)]
    circ = W.Circuit(n, ops)
    s = _state(qs, n, dtype)
    s.apply_circuit(circ, fuse_k=1, tile_m=-1)
    psi = s.to_numpy().astype(np.complex128)
    coeffs, xs, zs = [], [], []
    for i in range(n - 1):
        coeffs.append(1.0 + 0.05 * i); xs.append(0); zs.append((1 << i) | (1 << (i + 1)))
    for i in range(n):
        coeffs.append(0.5); xs.append(1 << i); zs.append(0)
        coeffs.append(-0.25); xs.append(1 << i); zs.append(1 << i)
    H = W.PauliSum(n, coeffs, xs, zs)
    got = s.expectation(H)
    assert abs(got - O.expectation(psi, H)) <= 1e-10 * sum(abs(c) for c in coeffs)
    # closed form from the single-qubit states u3|0>
    bloch = []
    for o in ops:
        v = O.gate_matrix("u3", o.angles)[:, 0]
        bloch.append((2 * (np.conj(v[0]) * v[1]).real, 2 * (np.conj(v[0]) * v[1]).imag,
                      abs(v[0]) ** 2 - abs(v[1]) ** 2))
    closed = sum(c * bloch[i][2] * bloch[i + 1][2] for i, c in zip(range(n - 1), coeffs))
    closed += sum(0.5 * bloch[i][0] - 0.25 * bloch[i][1] for i in range(n))
    assert abs(got - closed) <= (1e-5 if dtype == "c64" else 1e-12) * sum(abs(c) for c in coeffs)
    assert min(abs(b[2]) for b in bloch) > 0.2        # every ZZ term is O(1)
    s.close()


def test_plan_cache_eviction_and_stream_switch(qs):
    """A parameter sweep over 40 settings on one state: more plans than the
    state keeps, so evicted plans release their device buffers in stream
    order while later plans are uploaded; half way the state moves to another
    stream (plans then release on that one).  Results are checked along the
    way against the oracle."""
    import torch
    n, layers = 12, 2
    circ = W.ansatz_circuit(n, layers)
    rng = np.random.default_rng(112)
    s = _state(qs, n, "c128")
    side = torch.cuda.Stream()
    for i in range(40):
        if i == 20:
            torch.cuda.synchronize()
            qs.qsim_set_stream(s.handle, side.cuda_stream)
        p = rng.uniform(0, 2 * np.pi, circ.nparams)
        s.set_basis(0)
        s.apply_circuit(circ, params=p)
        if i % 7 == 0 or i >= 36:
            assert O.rel_l2(s.to_numpy(), O.apply_circuit(circ, params=p)) <= TOL["c128"]
    s.close()
    torch.cuda.synchronize()


def test_injected_launch_fault_on_a_live_state(qs, monkeypatch):
    """QSIM_FAULT=launch:2: the first launch point (set_basis) runs, the second
    (the circuit) fails before launching anything; the state then reports
    QSIM_ERR_STATE, and a fresh state on the same device works."""
    n = 10
    s = _state(qs, n, "c64", None)
    monkeypatch.setenv("QSIM_FAULT", "launch:2")
    s.set_basis(0)
    with pytest.raises(qs.QsimError) as e:
        s.apply_circuit(W.ghz_circuit(n))
    assert e.value.status == qs.QSIM_ERR_DEVICE
    monkeypatch.delenv("QSIM_FAULT")
    with pytest.raises(qs.QsimError) as e:
        s.expectation(W.chain_observable(n))
    assert e.value.status == qs.QSIM_ERR_STATE
    s.close()
    s2 = _state(qs, n, "c64")
    s2.apply_circuit(W.ghz_circuit(n))
    assert O.rel_l2(s2.to_numpy(), O.apply_circuit(W.ghz_circuit(n))) <= TOL["c64"]
    s2.close()
