"""Batched forward + adjoint runs (one persistent kernel per replayed graph)
against per-circuit runs on the same GPU and against the oracle.

Bars: complex128 energies <= 1e-11 absolute and gradients <= 1e-10 relative
L2 against the per-circuit adjoint path and the oracle's parameter shift;
complex64 <= 2e-5 relative against complex128 per-circuit results.
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


def make_batch(spec):
    circs = [W.ansatz_circuit(int(n), int(L)) for n, L in zip(spec.ns, spec.layers)]
    obs = [W.chain_observable(int(n)) for n in spec.ns]
    params = np.concatenate(spec.params)
    return circs, obs, params


def per_circuit(q, circs, obs, params, dtype):
    es, gs = [], []
    states = {}
    off = 0
    for c, H in zip(circs, obs):
        s = states.get(c.n)
        if s is None:
            s = states[c.n] = q.State(c.n, dtype)
        s.set_basis(0)
        e, g = s.adjoint_grad(c, params[off:off + c.nparams], H)
        es.append(e)
        gs.append(g)
        off += c.nparams
    for s in states.values():
        s.close()
    return np.array(es), np.concatenate(gs)


def test_mixed_sizes_c128_against_per_circuit_and_oracle(q):
    # one-tile circuits (n <= 10 in complex128) and multi-tile ones
    spec = W.batch_spec(count=24, nmin=2, nmax=13, lmin=1, lmax=4, seed=50)
    circs, obs, params = make_batch(spec)
    b = q.Batch(circs, obs, "c128")
    e, g = b.run(params)
    e_ref, g_ref = per_circuit(q, circs, obs, params, "c128")
    assert np.max(np.abs(e - e_ref)) < 1e-11
    assert rel(g, g_ref) < 1e-10
    off = 0
    for i, (c, H) in enumerate(zip(circs, obs)):
        p = params[off:off + c.nparams]
        if c.n <= 8:
            assert abs(e[i] - O.energy(c, p, H)) < 1e-11
            assert rel(g[off:off + c.nparams], O.param_shift_grad(c, p, H)) < 1e-10
        off += c.nparams
    b.close()


def test_replay_with_new_parameters_and_energy_only(q):
    spec = W.batch_spec(count=12, nmin=5, nmax=12, lmin=2, lmax=3, seed=51)
    circs, obs, params = make_batch(spec)
    b = q.Batch(circs, obs, "c128")
    for shift in (0.0, 0.3, -1.1):
        p = params + shift
        e, g = b.run(p)
        e_ref, g_ref = per_circuit(q, circs, obs, p, "c128")
        assert np.max(np.abs(e - e_ref)) < 1e-11
        assert rel(g, g_ref) < 1e-10
    b.close()
    b2 = q.Batch(circs, obs, "c128", want_grad=False)
    e2, g2 = b2.run(params)
    assert g2 is None
    assert np.max(np.abs(e2 - per_circuit(q, circs, obs, params, "c128")[0])) < 1e-11
    b2.close()


def test_c64_batch_against_c128(q):
    spec = W.batch_spec(count=16, nmin=8, nmax=14, lmin=2, lmax=5, seed=52)
    circs, obs, params = make_batch(spec)
    b = q.Batch(circs, obs, "c64")
    e, g = b.run(params)
    e_ref, g_ref = per_circuit(q, circs, obs, params, "c128")
    assert np.max(np.abs(e - e_ref)) < 2e-5 * max(1.0, np.max(np.abs(e_ref)))
    assert rel(g, g_ref) < 2e-5
    b.close()


def test_batch_4096_full_size(q):
    """4096 ansatz circuits, qubits 10..20, layers 4..12, complex64: every
    energy and gradient against complex64 per-circuit runs on a stratified
    sample of 128 circuits, energies of sampled n <= 14 circuits against the
    oracle, and finite checks on all outputs."""
    spec = W.batch_spec(count=4096, seed=5)
    circs, obs, params = make_batch(spec)
    b = q.Batch(circs, obs, "c64")
    grid, programs, max_n = b.info()
    assert programs == len({(c.n, len(c.ops)) for c in circs}) and max_n == 20
    e, g = b.run(params)
    assert np.all(np.isfinite(e)) and np.all(np.isfinite(g))
    offs = np.concatenate([[0], np.cumsum([c.nparams for c in circs])])
    sample = list(range(0, 4096, 32))
    se, sg = per_circuit(q, [circs[i] for i in sample], [obs[i] for i in sample],
                         np.concatenate([params[offs[i]:offs[i + 1]] for i in sample]), "c64")
    assert np.max(np.abs(e[sample] - se)) < 2e-5 * max(1.0, np.max(np.abs(se)))
    assert rel(np.concatenate([g[offs[i]:offs[i + 1]] for i in sample]), sg) < 2e-5
    small = [i for i in range(4096) if circs[i].n <= 14][:16]
    for i in small:
        ref = O.energy(circs[i], params[offs[i]:offs[i + 1]], obs[i])
        assert abs(e[i] - ref) < 2e-5 * max(1.0, abs(ref))
    # whole gradients of four n <= 12 circuits against the oracle's parameter
    # shift (complex64 adjoint against complex128 shift: the 1e-4 bar)
    for i in [i for i in range(4096) if circs[i].n <= 12][:4]:
        p = params[offs[i]:offs[i + 1]]
        ps = O.param_shift_grad(circs[i], p, obs[i], threaded=True)
        assert rel(g[offs[i]:offs[i + 1]], ps) < 1e-4, i
    b.close()
