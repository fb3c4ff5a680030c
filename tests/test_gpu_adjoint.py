"""Adjoint gradients on the GPU against the oracle's parameter-shift and
finite-difference gradients, and against GPU finite differences at the
20-qubit, 400-parameter ansatz size.

Bars: complex128 energy <= 1e-12 absolute, gradient <= 1e-10 relative L2
against parameter shift and <= 1e-6 absolute against central differences
(h = 1e-4); complex64 gradient <= 1e-4 relative L2 against complex128.
"""
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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n,layers", [(1, 1), (3, 2), (6, 3), (11, 2)])
def test_ansatz_gradient_matches_parameter_shift(q, n, layers):
    circ = W.ansatz_circuit(n, layers)
    p = W.ansatz_params(n, layers, seed=40 + n)
    H = W.chain_observable(n) if n > 1 else W.PauliSum(1, [1.0, 0.5], [0, 1], [1, 0])
    s = q.State(n, "c128")
    e, g = s.adjoint_grad(circ, p, H)
    assert abs(e - O.energy(circ, p, H)) < 1e-12
    ps = O.param_shift_grad(circ, p, H)
    assert rel(g, ps) < 1e-10
    s.close()


def test_mixed_circuit_with_shared_parameters(q):
    """Fixed gates interleaved with RX/RY/RZ, one parameter used by two ops,
    a parameter no op uses, and an observable with Y terms."""
    n = 8
    rng = np.random.default_rng(41)
    ops = []
    for layer in range(3):
        for qb in range(n):
            ops.append(W.op("h", qb) if (qb + layer) % 3 == 0 else W.op("u3", qb, angles=rng.uniform(0, 6, 3)))
        ops.append(W.op("rx", 0, param=0))
        ops.append(W.op("ry", 5, param=1 + layer))
        ops.append(W.op("rz", 3, param=4))
        ops.append(W.op("rx", 6, param=4))     # shared with the RZ above
        for a in range(layer % 2, n - 1, 2):
            ops.append(W.op("cz", a, a + 1))
        ops.append(W.op("ccx", 1, 2, 7))
        ops.append(W.op("cx", 7, 4))
    circ = W.Circuit(n, ops, 7)
    p = rng.uniform(0, 2 * np.pi, 7)          # index 5, 6 unused
    H = W.random_pauli_sum(n, 10, rng)
    s = q.State(n, "c128")
    e, g = s.adjoint_grad(circ, p, H)
    assert abs(e - O.energy(circ, p, H)) < 1e-12
    ps = O.param_shift_grad(circ, p, H)
    assert rel(g, ps) < 1e-10
    assert g[5] == 0.0 and g[6] == 0.0
    s.close()
    # the batch path (probes of a shared parameter in one pass, and not)
    b = q.Batch([circ, circ], [H, H], "c128")
    eb, gb = b.run(np.concatenate([p, p]))
    assert np.max(np.abs(eb - e)) < 1e-11
    assert rel(gb[:7], ps) < 1e-10 and rel(gb[7:], ps) < 1e-10
    b.close()


def test_state_restored_and_nonzero_input(q):
    n, layers = 9, 2
    circ = W.ansatz_circuit(n, layers)
    p = W.ansatz_params(n, layers, seed=42)
    H = W.chain_observable(n)
    psi0 = W.random_state(n, np.random.default_rng(43))
    s = q.State(n, "c128")
    s.from_numpy(psi0)
    e, g = s.adjoint_grad(circ, p, H)
    assert O.rel_l2(s.to_numpy(), psi0) < 1e-12
    psi = O.apply_circuit(circ, psi0, params=p)
    assert abs(e - O.expectation(psi, H)) < 1e-12
    # the shift rule applied by hand from the same input state
    j = 7
    vals = []
    for sh in (0.5 * np.pi, -0.5 * np.pi):
        pp = p.copy()
        pp[j] += sh
        vals.append(O.expectation(O.apply_circuit(circ, psi0, params=pp), H))
    assert abs(g[j] - 0.5 * (vals[0] - vals[1])) < 1e-11
    s.close()


def test_unsupported_parametric_kind(q):
    circ = W.Circuit(3, [W.op("h", 0), W.op("u3", 1, param=0)], 3)
    s = q.State(3, "c128")
    before = s.to_numpy()
    with pytest.raises(q.QsimError) as err:
        s.adjoint_grad(circ, np.zeros(3), W.chain_observable(3))
    assert err.value.status == q.QSIM_ERR_UNSUPPORTED
    np.testing.assert_array_equal(s.to_numpy(), before)
    s.close()


def test_c64_against_c128(q):
    n, layers = 12, 4
    circ = W.ansatz_circuit(n, layers)
    p = W.ansatz_params(n, layers, seed=44)
    H = W.chain_observable(n)
    s1, s2 = q.State(n, "c64"), q.State(n, "c128")
    e1, g1 = s1.adjoint_grad(circ, p, H)
    e2, g2 = s2.adjoint_grad(circ, p, H)
    assert abs(e1 - e2) < 1e-4
    assert rel(g1, g2) < 1e-4
    s1.close()
    s2.close()


def test_ansatz20_full_size(q):
    """The 20-qubit, 10-layer ansatz (400 parameters) with sum Z_iZ_{i+1} +
    0.5 sum X_i: energy against the oracle; sampled gradient entries against
    GPU central differences (h = 1e-4) and the GPU shift rule, complex128;
    the complex64 gradient against the complex128 one."""
    n, layers = 20, 10
    circ = W.ansatz_circuit(n, layers)
    p = W.ansatz_params(n, layers, seed=4)
    H = W.chain_observable(n)
    s = q.State(n, "c128")
    e, g = s.adjoint_grad(circ, p, H)
    assert abs(e - O.energy(circ, p, H)) < 1e-11
    rng = np.random.default_rng(45)
    sample = sorted(set(rng.choice(p.size, size=8, replace=False).tolist()) | {0, p.size - 1})

    def gpu_energy(pp):
        s.set_basis(0)
        s.apply_circuit(circ, params=pp)
        return s.expectation(H)

    for j in sample:
        vals = {}
        for sh in (1e-4, -1e-4, 0.5 * np.pi, -0.5 * np.pi):
            pp = p.copy()
            pp[j] += sh
            vals[sh] = gpu_energy(pp)
        fd = (vals[1e-4] - vals[-1e-4]) / 2e-4
        shift = 0.5 * (vals[0.5 * np.pi] - vals[-0.5 * np.pi])
        assert abs(g[j] - fd) < 1e-6, (j, g[j], fd)
        assert abs(g[j] - shift) < 1e-10 * max(1.0, abs(shift)), (j, g[j], shift)
    s.close()
    s64 = q.State(n, "c64")
    e64, g64 = s64.adjoint_grad(circ, p, H)
    assert abs(e64 - e) < 1e-4
    assert rel(g64, g) < 1e-4
    s64.close()


@pytest.mark.parametrize("dtype,bar", [("c128", 1e-10), ("c64", 1e-4)])
def test_ansatz20_sampled_gradient_against_oracle_shift(q, dtype, bar):
    """Eight seeded entries of the 400-parameter gradient at 20 qubits against
    the oracle's parameter-shift rule (16 complex128 CPU forward runs), and
    the energy against the oracle's."""
    n, layers = 20, 10
    circ = W.ansatz_circuit(n, layers)
    p = W.ansatz_params(n, layers, seed=4)
    H = W.chain_observable(n)
    s = q.State(n, dtype)
    e, g = s.adjoint_grad(circ, p, H)
    s.close()
    sample = np.random.default_rng(47).choice(p.size, size=8, replace=False)
    ps = O.param_shift_grad(circ, p, H, indices=sample, threaded=True)
    assert rel(g[sample], ps[sample]) < bar, (g[sample], ps[sample])
    assert abs(e - O.energy(circ, p, H, threaded=True)) < (1e-11 if dtype == "c128" else 1e-4)


@pytest.mark.parametrize("dtype,bar", [("c128", 1e-10), ("c64", 1e-4)])
def test_six_qubit_matrix_outside_the_low_qubits(q, dtype, bar):
    """A dense 6-qubit block on qubits 8..13 of a 14-qubit circuit: the
    reverse sweep's 2^10 tiles hold only 5 (c64) / 6 (c128) positions beyond
    the low qubits, so the planner widens them; the gradient must still
    match the oracle's parameter shift."""
    n = 14
    rng = np.random.default_rng(48)
    ops, npar = [], 0
    for qb in range(n):
        ops.append(W.op("ry", qb, param=npar)); npar += 1
    ops.append(W.matrix_op(list(range(8, 14)), W.random_unitary(6, rng)))
    for qb in range(0, n, 3):
        ops.append(W.op("rz", qb, param=npar)); npar += 1
    ops.append(W.op("cx", 2, 11))
    circ = W.Circuit(n, ops, npar)
    p = rng.uniform(0, 2 * np.pi, npar)
    H = W.chain_observable(n)
    s = q.State(n, dtype)
    e, g = s.adjoint_grad(circ, p, H)
    s.close()
    assert rel(g, O.param_shift_grad(circ, p, H)) < bar
    assert abs(e - O.energy(circ, p, H)) < (1e-12 if dtype == "c128" else 1e-5)


def test_autograd_function(q):
    torch = pytest.importorskip("torch")
    n, layers = 5, 2
    circ = W.ansatz_circuit(n, layers)
    p = W.ansatz_params(n, layers, seed=46)
    H = W.chain_observable(n)
    s = q.State(n, "c128")
    theta = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    E = q.expectation(theta, s, circ, H)
    (2.0 * E).backward()
    assert abs(E.item() - O.energy(circ, p, H)) < 1e-12
    assert rel(theta.grad.numpy(), 2.0 * O.param_shift_grad(circ, p, H)) < 1e-10
    s.close()


def _controlled_circuit(n, rng):
    """RY/RZ layers with one-qubit blocks under one or two controls: CX and
    CCX, and controlled random unitaries given as matrices, with the control
    listed before and after the target (so it sits above and below it)."""
    ops, npar = [], 0
    for layer in range(2):
        for qb in range(n):
            ops.append(W.op("ry", qb, param=npar)); npar += 1
            ops.append(W.op("rz", qb, param=npar)); npar += 1
        for a in range(layer % 2, n - 1, 2):
            u = W.random_unitary(1, rng)
            cu = np.eye(4, dtype=np.complex128)
            if a % 4 == 0:      # control = targets[0] (bit 0 of the matrix index)
                cu[np.ix_([1, 3], [1, 3])] = u
                ops.append(W.matrix_op([a, a + 1], cu))
            else:               # control = targets[1]
                cu[2:, 2:] = u
                ops.append(W.matrix_op([a, a + 1], cu))
        ops.append(W.op("cx", n - 1, 0))
        ops.append(W.op("cx", 1, n - 2))
        ops.append(W.op("ccx", 0, n - 1, n // 2))
        ccu = np.eye(8, dtype=np.complex128)
        ccu[np.ix_([5, 7], [5, 7])] = W.random_unitary(1, rng)   # controls on bits 0, 2
        ops.append(W.matrix_op([2, n // 2 + 1, n - 2], ccu))
    return W.Circuit(n, ops, npar)


@pytest.mark.parametrize("n", [7, 13])
def test_controlled_blocks_in_tiles(q, n):
    """Controlled one-qubit blocks as masked pair ops in the adjoint's and the
    batch's LDS tiles: complex128 against the oracle's energy and parameter
    shift, complex64 against complex128, the batch against the per-circuit
    path."""
    rng = np.random.default_rng(60 + n)
    circ = _controlled_circuit(n, rng)
    p = rng.uniform(0, 2 * np.pi, circ.nparams)
    H = W.random_pauli_sum(n, 8, rng)
    s = q.State(n, "c128")
    e, g = s.adjoint_grad(circ, p, H)
    assert abs(e - O.energy(circ, p, H)) < 1e-12
    assert rel(g, O.param_shift_grad(circ, p, H)) < 1e-10
    s.close()
    s = q.State(n, "c64")
    e32, g32 = s.adjoint_grad(circ, p, H)
    assert abs(e32 - e) < 1e-5 and rel(g32, g) < 1e-4
    s.close()
    for dt, tol in (("c128", 1e-10), ("c64", 1e-4)):
        b = q.Batch([circ, circ], [H, H], dt)
        eb, gb = b.run(np.concatenate([p, p]))
        assert np.max(np.abs(eb - e)) < (1e-11 if dt == "c128" else 1e-5)
        assert rel(gb[:circ.nparams], g) < tol and rel(gb[circ.nparams:], g) < tol
        b.close()


def test_device_pointer_calls_are_stream_ordered(q):
    """qsim_adjoint_grad through the C ABI with torch device tensors for the
    parameters, the energy and the gradient: three calls with different
    parameters queued back to back without a host wait, each checked
    afterwards against the oracle's energy and parameter shift (complex128).
    The plan is built once (structure only) and reused by all three."""
    import torch
    n, layers = 7, 2
    circ = q.PackedCircuit(W.ansatz_circuit(n, layers))
    base = W.ansatz_params(n, layers, seed=49)
    H = W.chain_observable(n)
    s = q.State(n, "c128")
    outs, ps = [], []
    for r in range(3):
        p = base + 0.37 * r
        ps.append(p)
        s.set_basis(0)
        e, g = s.adjoint_grad_device(circ, torch.as_tensor(p, device=s.tensor.device), H)
        outs.append((e, g))
    torch.cuda.synchronize()
    wc = W.ansatz_circuit(n, layers)
    for (e, g), p in zip(outs, ps):
        assert abs(float(e.cpu()[0]) - O.energy(wc, p, H)) < 1e-12
        assert rel(g.cpu().numpy(), O.param_shift_grad(wc, p, H)) < 1e-10
    s.close()


def test_host_pointers_rejected_before_device_work(q):
    """The library checks that params, energy and grad are device memory."""
    import ctypes
    n = 4
    circ = q.PackedCircuit(W.ansatz_circuit(n, 1))
    H = q.PackedPauliSum(W.chain_observable(n))
    s = q.State(n, "c128")
    before = s.to_numpy()
    p = np.zeros(circ.c.nops and W.ansatz_circuit(n, 1).nparams)
    g = np.zeros_like(p)
    e = np.zeros(1)
    st = q._lib.qsim_adjoint_grad(ctypes.c_void_p(s.handle), ctypes.byref(circ.c), p.ctypes.data_as(ctypes.c_void_p),
                                  p.size, ctypes.byref(H.h), None, e.ctypes.data_as(ctypes.c_void_p),
                                  g.ctypes.data_as(ctypes.c_void_p))
    assert st == q.QSIM_ERR_ARG
    np.testing.assert_array_equal(s.to_numpy(), before)
    s.close()


def test_checkpoints_match_the_oracle_and_bound_the_drift(q):
    """Forward-state checkpoints (the circuit cut into runs whose first
    states are kept and restored in the reverse sweep): with 1, 3 and 7 cuts
    the complex128 energy and gradient still match the oracle's parameter
    shift; on a deep complex64 circuit the gradient stays within the
    complex64 bar and the state the call hands back (its input, recovered by
    the inverse gates) is closer to the input, since the inverse gates'
    rounding now builds up over one run instead of the whole circuit."""
    circ = W.ansatz_circuit(12, 4)
    circ.ops.insert(5, W.op("h", 3))
    circ.ops.insert(40, W.op("cz", 2, 9))
    p = W.ansatz_params(12, 4, seed=71)
    H = W.chain_observable(12)
    e_ref = O.energy(circ, p, H)
    ps = O.param_shift_grad(circ, p, H, threaded=True)
    s = q.State(12, "c128")
    for ck in (0, 1, 3, 7):
        s.set_basis(0)
        e, g = s.adjoint_grad(circ, p, H, checkpoints=ck)
        assert abs(e - e_ref) < 1e-12, ck
        assert rel(g, ps) < 1e-10, ck
    s.close()

    deep = W.ansatz_circuit(14, 40)
    pd = W.ansatz_params(14, 40, seed=72)
    Hd = W.chain_observable(14)
    s128 = q.State(14, "c128")
    e128, g128 = s128.adjoint_grad(deep, pd, Hd)
    s128.close()
    s64 = q.State(14, "c64")
    drift = {}
    for ck in (0, 15):
        s64.set_basis(0)
        e, g = s64.adjoint_grad(deep, pd, Hd, checkpoints=ck)
        assert abs(e - e128) < 1e-4, ck
        assert rel(g, g128) < 1e-4, ck
        back = s64.to_numpy().astype(np.complex128)
        back[0] -= 1.0
        drift[ck] = float(np.linalg.norm(back))
    s64.close()
    assert drift[15] < 0.5 * drift[0], drift
