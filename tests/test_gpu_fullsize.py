"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (default options: register-staged tile passes).

The oracle cannot run a 30-qubit depth-20 circuit in a test's time, so these
checks use outputs it computes one index at a time (product-state closed
forms, multiplier arithmetic) and properties that hold at any size (norm,
inverse circuit, complex64 against complex128 and against plain sweeps).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_13995_amd as q
    return q, torch


def amplitudes(state, idx):
    """Selected amplitudes of a device state, read through torch indexing."""
    torch = pytest.importorskip("torch")
    t = state.tensor.view(-1, 2)
    sel = t[torch.as_tensor(np.asarray(idx, dtype=np.int64), device=t.device)].double().cpu().numpy()
    return sel[:, 0] + 1j * sel[:, 1]


def norm2(state):
    return state.expectation(W.PauliSum(state.n, [1.0], [0], [0]))


def sample_indices(n, count, seed):
    rng = np.random.default_rng(seed)
    return np.unique(rng.integers(0, 1 << n, size=count, dtype=np.int64))


@pytest.mark.parametrize("dtype,tol", [("c64", 2e-5), ("c128", 1e-12)])
def test_grid30_first_layer_closed_form(env, dtype, tol):
    """Layer 0 of the 30-qubit grid circuit (U3 everywhere + horizontal-even CZ)
    against the product-state closed form at 2^20 sampled indices."""
    q, torch = env
    circ = W.random_grid_circuit(5, 6, depth=1, seed=2)
    s = q.State(30, dtype)
    s.apply_circuit(circ)
    idx = sample_indices(30, 1 << 20, seed=30)
    got = amplitudes(s, idx)
    u3s = [o for o in circ.ops if o.kind == "u3"]
    ref = O.product_cz_amplitudes(30, u3s, W.grid_cz_pairs(5, 6, 0), idx.astype(np.uint64))
    assert O.rel_l2(got, ref) <= tol
    assert abs(norm2(s) - 1.0) < 10 * tol
    s.close()


def test_grid30_c64_full_circuit_properties(env):
    """The 845-gate benchmark circuit at 30 qubits, complex64, bench options:
    norm preserved; the inverse circuit (same options) returns |0...0>;
    agreement with the complex128 run and with plain gate-by-gate sweeps on
    sampled amplitudes."""
    q, torch = env
    circ = W.random_grid_circuit(5, 6, depth=20, seed=2)
    idx = sample_indices(30, 1 << 18, seed=31)
    s = q.State(30, "c64")
    s.apply_circuit(circ)
    a64 = amplitudes(s, idx)
    assert abs(norm2(s) - 1.0) < 1e-4
    dag = O.circuit_dagger(circ)
    s.apply_circuit(dag)
    back = amplitudes(s, [0, 1, 12345, (1 << 30) - 1])
    assert abs(back[0] - 1.0) < 1e-4 and np.max(np.abs(back[1:])) < 1e-4
    # plain sweeps, same precision
    s.set_basis(0)
    s.apply_circuit(circ, fuse_k=1, tile_m=-1)
    sweep = amplitudes(s, idx)
    s.close()
    del s
    torch.cuda.empty_cache()
    s2 = q.State(30, "c128")
    s2.apply_circuit(circ)
    a128 = amplitudes(s2, idx)
    assert abs(norm2(s2) - 1.0) < 1e-12
    s2.close()
    # complex64 error against complex128 on the sampled amplitudes (the
    # complex128 path is itself held to 1e-12 against the oracle elsewhere)
    assert O.rel_l2(a64, a128) <= 2e-5
    assert O.rel_l2(sweep, a128) <= 2e-5


@pytest.mark.parametrize("mode", [dict(), dict(fuse_k=1, tile_m=-1), dict(fuse_k=1, tile_m=12),
                                  dict(fuse_k=1, tile_m=13)], ids=["auto", "sweeps", "tile12", "tile13"])
def test_multiplier29_basis_inputs_bit_exact(env, mode):
    """The 29-qubit multiplier (7-bit a, b; 14-bit product; ancilla), complex64,
    on the 64 seed-drawn basis inputs: amplitude exactly 1 at a + 2^7 b + 2^14 ab
    and norm exactly 1 (so every other amplitude is exactly 0)."""
    q, torch = env
    L = W.MultiplierLayout(7)
    core = W.multiplier_core(7)
    s = q.State(L.n, "c64")
    pairs = W.multiplier_inputs(64, 7, seed=3)
    # the oracle's classical evaluation of the same netlist gives the target indices
    starts = [L.basis_index(int(a), int(b)) for a, b in pairs]
    outs = O.classical_run(core, starts)
    for (a, b), out in zip(pairs, outs):
        assert int(out) == L.basis_index(int(a), int(b), int(a) * int(b))
        s.set_basis(L.basis_index(int(a), int(b)))
        s.apply_circuit(core, **mode)
        amp = amplitudes(s, [int(out)])[0]
        assert amp == 1.0 + 0.0j, (a, b, amp)
        assert norm2(s) == 1.0
    s.close()


def test_multiplier29_superposition(env):
    """H on all seven a qubits: psi = 2^{-7/2} sum_a |a, b, a*b, 0>."""
    q, torch = env
    L = W.MultiplierLayout(7)
    b = int(W.multiplier_inputs(1, 7, seed=3)[0, 1])
    circ = W.multiplier_circuit(0, b, 7, superpose_a=True)
    s = q.State(L.n, "c64")
    s.apply_circuit(circ)
    idx = [L.basis_index(a, b, a * b) for a in range(128)]
    got = amplitudes(s, idx)
    assert np.max(np.abs(got - 2.0 ** -3.5)) < 1e-6
    assert abs(norm2(s) - 1.0) < 1e-5
    s.close()


def _after_dense(n, u3s, pairs, targets, U, idx):
    """Amplitudes at `idx` of (layer 0 state) followed by the dense gate U on
    `targets` (local bit b = targets[b]), from the closed form of layer 0 at
    the 2^k indices each output needs."""
    k = len(targets)
    tmask = 0
    for t in targets:
        tmask |= 1 << t
    offs = np.zeros(1 << k, dtype=np.uint64)
    for j in range(1 << k):
        o = 0
        for b in range(k):
            if (j >> b) & 1:
                o |= 1 << targets[b]
        offs[j] = o
    base = idx.astype(np.uint64) & np.uint64(~tmask & ((1 << n) - 1))
    rows = np.zeros(idx.size, dtype=np.int64)
    for b, t in enumerate(targets):
        rows |= ((idx >> t) & 1).astype(np.int64) << b
    need = (base[:, None] | offs[None, :]).reshape(-1)
    before = O.product_cz_amplitudes(n, u3s, pairs, need).reshape(idx.size, 1 << k)
    return np.einsum("sj,sj->s", U[rows], before)


@pytest.mark.parametrize("dtype,n,targets,tol", [
    ("c64", 34, [29, 30, 31, 32, 33], 2e-5),   # 128 GiB; k = 5 on scattered (high) targets
    ("c128", 33, [0, 1, 2, 3], 1e-12),        # 128 GiB; k = 4 on the lowest qubits
])
def test_max_width_state(env, dtype, n, targets, tol):
    """Beyond 2^32 amplitudes (64-bit indexing everywhere): layer 0 of a
    2 x n/2 grid circuit (compiled tile passes), then a dense block on the
    matrix cores, against the closed form at 4096 sampled indices."""
    q, torch = env
    rows = 2
    cols = n // rows
    if rows * cols != n:
        cols, rows = n, 1
    circ = W.random_grid_circuit(rows, cols, depth=1, seed=5)
    rng = np.random.default_rng(40 + n)
    U = W.random_unitary(len(targets), rng)
    s = q.State(n, dtype)
    s.apply_circuit(circ)
    s.apply_gate(targets, U)
    idx = sample_indices(n, 4096, seed=41)
    idx[:2] = [0, (1 << n) - 1]
    got = amplitudes(s, idx)
    u3s = [o for o in circ.ops if o.kind == "u3"]
    ref = _after_dense(n, u3s, W.grid_cz_pairs(rows, cols, 0), targets, U, idx.astype(np.int64))
    assert O.rel_l2(got, ref) <= tol
    assert abs(norm2(s) - 1.0) < 10 * tol
    s.close()
    del s
    torch.cuda.empty_cache()


def test_out_of_memory_is_reported(env):
    """Two 34-qubit complex128 states (256 GiB each) do not fit in one
    MI355X's 288 GB: the second qsim_alloc returns QSIM_ERR_OOM, and the
    first state stays usable."""
    q, torch = env
    torch.cuda.empty_cache()
    h1 = q.qsim_alloc(34, q.QSIM_C128)
    try:
        with pytest.raises(q.QsimError) as e:
            q.qsim_alloc(34, q.QSIM_C128)
        assert e.value.status == q.QSIM_ERR_OOM
        q.qsim_set_basis(h1, (1 << 34) - 1)
        H = q.PackedPauliSum(W.PauliSum(34, [1.0, 1.0], [0, 0], [0, 1 << 33]))   # 1 + Z_33
        assert q.qsim_expectation(h1, H) == 0.0
    finally:
        q.qsim_free(h1)
