"""The expectation entry point that allocates no device memory, through the C
ABI, against qsim_expectation (same kernels, same order: bitwise equal) and
the complex128 oracle, on two calls in a row with the second on a smaller
state and a smaller sum, then on a sum too large for the fixed array."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_13995_amd as q
    return q


def _prepared(q, n, dtype, seed):
    circ = W.random_line_circuit(n, 8, seed=seed)
    s = q.State(n, dtype)
    s.apply_circuit(circ)
    psi = s.to_numpy().astype(np.complex128)   # the state as the device holds it
    return s, psi


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_matches_expectation_on_two_calls(q, dtype):
    # first call: 14 qubits, chain observable plus random Pauli terms (several
    # X-mask groups, tile passes and single-group passes); second: 10 qubits,
    # the chain observable only
    chain, rnd = W.chain_observable(14), W.random_pauli_sum(14, 40, np.random.default_rng(21))
    mixed = W.PauliSum(14, chain.coeffs + rnd.coeffs, chain.xmasks + rnd.xmasks, chain.zmasks + rnd.zmasks)
    cases = [(14, mixed, 1), (10, W.chain_observable(10), 2)]
    for n, H, seed in cases:
        print(f"noalloc {dtype} n={n} terms={len(H.coeffs)}", flush=True)
        s, psi = _prepared(q, n, dtype, seed)
        P = q.PackedPauliSum(H)
        ref_dev = q.qsim_expectation(s.handle, P)
        got = q.qsim_expectation_noalloc(s.handle, P)
        assert got == ref_dev, (got, ref_dev)
        # the oracle on the device's (rounded) amplitudes: only the order of
        # the double-precision sums differs
        ref = O.expectation(psi, H)
        scale = float(np.sum(np.abs(H.coeffs)))
        assert abs(got - ref) <= 1e-12 * max(1.0, scale), (got, ref)
        # repeated call: same value again (the array keeps the last call's
        # contents, every partial is rewritten)
        assert q.qsim_expectation_noalloc(s.handle, P) == got
        s.close()


def test_noalloc_rejects_a_sum_beyond_the_array(q):
    n = 24
    s, _ = _prepared(q, n, "c64", 3)
    # one term per distinct X mask, each mask too wide for a tile: at 24
    # qubits a group evaluated alone writes 2048 partials (16 KiB), so 300
    # groups exceed the 4 MiB array
    rng = np.random.default_rng(9)
    xs = rng.choice(np.arange(1, 1 << n), size=300, replace=False) | (0xFF << 12)
    xs = np.unique(xs)
    assert len(xs) > 260
    H = W.PauliSum(n, [1.0] * len(xs), [int(x) for x in xs], [0] * len(xs))
    P = q.PackedPauliSum(H)
    out = ctypes.c_double()
    st = q._lib.qsim_expectation_noalloc(ctypes.c_void_p(s.handle), ctypes.byref(P.h), ctypes.byref(out))
    assert st == q.QSIM_ERR_ARG
    assert "fixed buffer" in q._lib.qsim_last_error().decode()
    # the state is untouched and still usable
    H2 = W.chain_observable(n)
    assert q.qsim_expectation_noalloc(s.handle, q.PackedPauliSum(H2)) == q.qsim_expectation(
        s.handle, q.PackedPauliSum(H2))
    s.close()
