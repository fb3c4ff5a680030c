"""Host checks of the synthetic input generators used by the width sweep:
qubit removal keeps exactly the ops on surviving qubits, relabelled in order."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def test_remove_qubits_keeps_ops_on_surviving_qubits():
    full = W.random_grid_circuit(4, 5, depth=6, seed=2)
    cut = W.remove_qubits(full, 17, seed=9)
    assert cut.n == 17
    rng = np.random.default_rng(9)
    drop = set(int(x) for x in rng.choice(full.n, 3, replace=False))
    keep = [q for q in range(full.n) if q not in drop]
    expect = [o for o in full.ops if not (set(o.targets) & drop)]
    assert len(cut.ops) == len(expect)
    for a, b in zip(cut.ops, expect):
        assert a.kind == b.kind and a.angles == b.angles
        assert tuple(keep[t] for t in a.targets) == b.targets


def test_remove_qubits_untouched_qubits_factor_out():
    """Dropping qubits no op touches leaves the state of the others: the cut
    circuit's output equals the full output with those qubits traced at |0>."""
    n = 8
    rng = np.random.default_rng(3)
    ops = [W.op("u3", q, angles=rng.uniform(0, 2 * np.pi, 3)) for q in (0, 2, 3, 5, 6)]
    ops += [W.op("cz", 0, 2), W.op("cx", 3, 6), W.op("ccx", 0, 5, 6)]
    full = W.Circuit(n, ops)
    psi = O.apply_circuit(full).reshape([2] * n)   # axis 0 is qubit n-1
    # remove qubits 1, 4, 7 (untouched): pick a seed whose draw is exactly those
    for seed in range(10000):
        d = set(int(x) for x in np.random.default_rng(seed).choice(n, 3, replace=False))
        if d == {1, 4, 7}:
            break
    cut = W.remove_qubits(full, 5, seed)
    sub = psi[0, :, :, 0, :, :, 0, :]   # qubits 7, 4, 1 at |0>
    np.testing.assert_allclose(O.apply_circuit(cut), sub.reshape(-1), atol=1e-14)


@pytest.mark.parametrize("family", ["supremacy", "multiplier"])
def test_width_circuits(family):
    for n in range(13, 31):
        c = W.width_circuit(family, n)
        assert c.n == n
        assert [o.kind for o in c.ops[:n]] == ["h"] * n
        assert max(max(o.targets) for o in c.ops) == n - 1
        assert all(len(set(o.targets)) == len(o.targets) for o in c.ops)
