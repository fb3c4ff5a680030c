"""Layered batch runs (circuits that fill whole tiles: one launch per pass
index over every tile of every such circuit, register-staged passes) against
the oracle: energies <psi|H|psi> and the parameter-shift gradient (paper
Sec. I.A and II for the state; the gradient is the shift rule on the same
product of gate matrices).

Bars: complex128 energies <= 1e-11 absolute and gradients <= 1e-10 relative
L2; complex64 <= 2e-5 relative (energies) and <= 1e-4 relative (gradients)
against the complex128 oracle.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TWO_PI = 2 * np.pi


@pytest.fixture(scope="module")
def q():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_13995_amd as q
    return q


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def param_circuit(n, nops, nparams, seed):
    """RX / RY / RZ on parameters (some used by several gates, the last one
    by none), among H, U3, CX, CZ, CCX, CCZ, SWAP, CP and dense one-, two-
    and three-qubit unitaries on random qubits."""
    rng = np.random.default_rng(seed)
    fixed = ["h", "u3", "cx", "cz", "ccx", "ccz", "swap", "cp"]
    ops = []
    for i in range(nops):
        r = rng.random()
        if r < 0.45:
            kind = ("rx", "ry", "rz")[int(rng.integers(3))]
            ops.append(W.op(kind, int(rng.integers(n)), param=int(rng.integers(nparams - 1))))
        elif r < 0.85:
            kind = fixed[int(rng.integers(len(fixed)))]
            ar = W.GATE_ARITY[kind]
            tg = [int(t) for t in rng.choice(n, size=ar, replace=False)]
            ops.append(W.op(kind, *tg, angles=rng.uniform(0, TWO_PI, size=W.GATE_NANGLES.get(kind, 0))))
        else:
            k = int(rng.integers(1, 4))
            tg = [int(t) for t in rng.choice(n, size=k, replace=False)]
            ops.append(W.matrix_op(tg, W.random_unitary(k, rng)))
    return W.Circuit(n, ops, nparams, f"param{n}_{seed}")


def observable(n, seed):
    rng = np.random.default_rng(seed)
    H = W.random_pauli_sum(n, 6, rng)
    ch = W.chain_observable(n, x_coeff=0.3)
    return W.PauliSum(n, list(H.coeffs) + list(ch.coeffs), list(H.xmasks) + list(ch.xmasks),
                      list(H.zmasks) + list(ch.zmasks))


def run_checks(q, dtype, ns, nops, seed0, tol_e, tol_g, expect_layered, options=None):
    circs = [param_circuit(n, nops, 9, seed0 + i) for i, n in enumerate(ns)]
    obs = [observable(n, seed0 + 100 + i) for i, n in enumerate(ns)]
    rng = np.random.default_rng(seed0 + 7)
    params = rng.uniform(0, TWO_PI, size=sum(c.nparams for c in circs))
    b = q.Batch(circs, obs, dtype, options=options)
    lay, per = b.layout()
    assert (lay, per) == expect_layered, (lay, per)
    e, g = b.run(params)
    off = 0
    for i, (c, H) in enumerate(zip(circs, obs)):
        p = params[off:off + c.nparams]
        ref_e = O.energy(c, p, H, threaded=True)
        ref_g = O.param_shift_grad(c, p, H, threaded=True)
        assert abs(e[i] - ref_e) < tol_e * max(1.0, abs(ref_e)), (i, c.n, e[i], ref_e)
        assert rel(g[off:off + c.nparams], ref_g) < tol_g, (i, c.n, rel(g[off:off + c.nparams], ref_g))
        assert g[off + c.nparams - 1] == 0.0   # the unused parameter
        off += c.nparams
    b.close()


def test_layered_c128_one_and_several_tiles(q):
    # complex128 tiles hold 11 qubits: n = 11 is one tile, 12..14 are 2..8;
    # n = 7 and 9 run in the persistent kernel next to them
    run_checks(q, "c128", [11, 12, 13, 14, 7, 9, 12], 70, 300, 1e-11, 1e-10, (5, 2))


def test_layered_c64_one_and_several_tiles(q):
    # complex64 tiles hold 11 qubits by default: n = 11 is one tile
    run_checks(q, "c64", [12, 11, 13, 14, 10], 60, 400, 2e-5, 1e-4, (4, 1))


def test_layered_groups_and_replay(q, monkeypatch):
    """A slot budget of one 2^13-amplitude circuit at a time splits the
    layered circuits into groups (each with its own layers, energies and
    reverse layers); replays with new parameters and an energy-only batch
    agree with the oracle too."""
    monkeypatch.setenv("QSIM_BATCH_SLOT_BUDGET", str(2 * 16 * (1 << 13)))
    ns = [13, 12, 11, 13, 12]
    circs = [param_circuit(n, 40, 6, 500 + i) for i, n in enumerate(ns)]
    obs = [observable(n, 600 + i) for i, n in enumerate(ns)]
    rng = np.random.default_rng(77)
    b = q.Batch(circs, obs, "c128")
    assert b.layout() == (5, 0)
    for rep in range(2):
        params = rng.uniform(0, TWO_PI, size=sum(c.nparams for c in circs))
        e, g = b.run(params)
        off = 0
        for i, (c, H) in enumerate(zip(circs, obs)):
            p = params[off:off + c.nparams]
            assert abs(e[i] - O.energy(c, p, H, threaded=True)) < 1e-11
            assert rel(g[off:off + c.nparams], O.param_shift_grad(c, p, H, threaded=True)) < 1e-10
            off += c.nparams
    b.close()
    b2 = q.Batch(circs, obs, "c128", want_grad=False)
    e2, g2 = b2.run(params)
    assert g2 is None
    off = 0
    for i, (c, H) in enumerate(zip(circs, obs)):
        assert abs(e2[i] - O.energy(c, params[off:off + c.nparams], H, threaded=True)) < 1e-11
        off += c.nparams
    b2.close()


def test_layered_edge_circuits(q):
    """A circuit without ops, one whose only gates are fixed, and one whose
    parameters all drive the same qubit, at one and several tiles."""
    H12 = observable(12, 1)
    H13 = observable(13, 2)
    empty = W.Circuit(12, [], 2, "empty")
    fixed = W.Circuit(13, [W.op("h", q) for q in range(13)] + [W.op("cz", 0, 12), W.op("ccx", 3, 7, 11)], 1,
                      "fixed")
    same = W.Circuit(13, [W.op(k, 12, param=j % 3) for j, k in enumerate(["rx", "ry", "rz"] * 4)] +
                     [W.op("cx", 12, 0)], 3, "same")
    circs = [empty, fixed, same]
    obs = [H12, H13, H13]
    params = np.random.default_rng(5).uniform(0, TWO_PI, size=sum(c.nparams for c in circs))
    for dtype, tol_e, tol_g in (("c128", 1e-11, 1e-10), ("c64", 2e-5, 1e-4)):
        b = q.Batch(circs, obs, dtype)
        assert b.layout() == (3, 0)
        e, g = b.run(params)
        off = 0
        for i, (c, H) in enumerate(zip(circs, obs)):
            p = params[off:off + c.nparams]
            ref_e = O.energy(c, p, H)
            assert abs(e[i] - ref_e) < tol_e * max(1.0, abs(ref_e)), (dtype, i)
            ref_g = O.param_shift_grad(c, p, H)
            if np.linalg.norm(ref_g) == 0.0:
                assert np.all(g[off:off + c.nparams] == 0.0)
            else:
                assert rel(g[off:off + c.nparams], ref_g) < tol_g, (dtype, i)
            off += c.nparams
        b.close()


@pytest.mark.parametrize("dtype,options,layout,tol", [
    # 2^11-amplitude tiles in complex64 (eight amplitudes a thread): n = 11
    # is one tile and runs layered too
    ("c64", {"fuse_k": 1, "tile_m": 11}, (4, 1), (2e-5, 1e-4)),
    # fixed-gate runs fused into dense blocks of up to three qubits
    ("c64", {"fuse_k": 3, "tile_m": 12}, (3, 2), (2e-5, 1e-4)),
    ("c128", {"fuse_k": 2, "tile_m": 11}, (4, 1), (1e-11, 1e-10)),
], ids=["c64_tile11", "c64_fuse3", "c128_fuse2"])
def test_layered_options_against_oracle(q, dtype, options, layout, tol):
    run_checks(q, dtype, [11, 12, 13, 14, 9], 60, 700, tol[0], tol[1], layout, options=options)


def test_batch_autotune_choice_is_a_candidate_and_correct(q):
    ns = [12, 13, 11, 14, 10, 12]
    circs = [param_circuit(n, 50, 7, 800 + i) for i, n in enumerate(ns)]
    obs = [observable(n, 900 + i) for i, n in enumerate(ns)]
    params = np.random.default_rng(81).uniform(0, TWO_PI, size=sum(c.nparams for c in circs))
    best, ms = q.Batch.autotune(circs, obs, params, "c64", reps=2)
    assert best["fuse_k"] in (1, 2, 3) and best["tile_m"] in (11, 12) and ms > 0.0
    b = q.Batch(circs, obs, "c64", options=best)
    e, g = b.run(params)
    b.close()
    off = 0
    for i, (c, H) in enumerate(zip(circs, obs)):
        p = params[off:off + c.nparams]
        ref_e = O.energy(c, p, H, threaded=True)
        assert abs(e[i] - ref_e) < 2e-5 * max(1.0, abs(ref_e))
        assert rel(g[off:off + c.nparams], O.param_shift_grad(c, p, H, threaded=True)) < 1e-4
        off += c.nparams
