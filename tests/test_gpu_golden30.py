"""The 30-qubit, depth-20 grid circuit (the throughput workload) against the
CPU oracle's stored output.

`tests/golden/grid30_d20_s2.npz` is written by `make_grid30_golden.py`,
which calls only the oracle and the input generators: the complex128 product
of the 845 gate matrices applied to |0...0> (paper, Sec. I.A and Sec. II).
Each launch configuration the benchmark can run (compiled register tiles of
2^12 and 2^13 amplitudes, plain gate-by-gate sweeps, interpreted tiles,
automatic options; complex64 and complex128) is compared on:

  * 65 536 seeded amplitudes and two 4096-amplitude blocks (all values of the
    lowest / highest 12 qubits): relative L2 <= 2e-5 (c64), 1e-12 (c128);
  * the marginal distributions of the lowest and highest 10 qubits, which sum
    over every amplitude of the state: relative L2 <= 2 x the amplitude bar
    (|psi|^2 doubles a relative error to first order);
  * <psi|H|psi> for H = sum Z_i Z_{i+1} + 0.5 sum X_i: for unit vectors,
    |<a|H|a> - <b|H|b>| <= 2 ||H|| ||a - b|| + ||H|| ||a - b||^2 with
    ||H|| <= sum |c_t| = 44, so 2 * 44 * bar (plus the square) bounds it.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grid30_d20_s2.npz")
TOL = {"c64": 2e-5, "c128": 1e-12}
H_NORM_BOUND = 29 * 1.0 + 30 * 0.5

CONFIGS = [
    ("c64", "auto", dict()),
    ("c64", "jit_tile12", dict(fuse_k=1, tile_m=12)),
    ("c64", "jit_tile13", dict(fuse_k=1, tile_m=13)),
    ("c64", "interp_tile13", dict(fuse_k=1, tile_m=13, jit=False)),
    ("c64", "sweeps", dict(fuse_k=1, tile_m=-1)),
    ("c64", "mfma_fuse4", dict(fuse_k=4, tile_m=-1, use_mfma=1)),
    ("c128", "auto", dict()),
    ("c128", "jit_tile12", dict(fuse_k=1, tile_m=12)),
    ("c128", "jit_tile11", dict(fuse_k=1, tile_m=11)),
]


@pytest.fixture(scope="module")
def golden():
    z = np.load(GOLDEN, allow_pickle=False)
    circ = W.random_grid_circuit(5, 6, depth=20, seed=2)
    assert str(z["digest"]) == W.circuit_digest(circ), "the stored output belongs to another circuit"
    idx = W.sample_indices(30, int(z["sample_count"]), int(z["sample_seed"]))
    assert idx.size == z["amps"].size
    return z, circ, idx.astype(np.int64)


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_13995_amd as q
    return q, torch


def _amplitudes(torch, state, idx):
    t = state.tensor.view(-1, 2)
    sel = t[torch.as_tensor(idx, device=t.device)].double().cpu().numpy()
    return sel[:, 0] + 1j * sel[:, 1]


def _marginals(torch, state, bits=10):
    t = state.tensor.view(-1, 2)
    p = (t[:, 0].double() ** 2 + t[:, 1].double() ** 2)
    lo = p.view(-1, 1 << bits).sum(0).cpu().numpy()
    hi = p.view(1 << bits, -1).sum(1).cpu().numpy()
    del p
    return lo, hi


def compare(q, torch, state, golden, dtype):
    """Relative L2 errors of a 30-qubit device state against the stored
    oracle output; returns a dict of them (and the energy difference)."""
    z, circ, idx = golden
    out = {}
    out["samples"] = O.rel_l2(_amplitudes(torch, state, idx), z["amps"])
    out["lo_block"] = O.rel_l2(_amplitudes(torch, state, np.arange(4096)), z["lo_block"])
    out["hi_block"] = O.rel_l2(_amplitudes(torch, state, np.arange(4096) << 18), z["hi_block"])
    lo, hi = _marginals(torch, state)
    out["marg_lo"] = O.rel_l2(lo, z["marg_lo"])
    out["marg_hi"] = O.rel_l2(hi, z["marg_hi"])
    out["energy"] = abs(state.expectation(W.chain_observable(30)) - float(z["energy"]))
    return out


@pytest.mark.parametrize("dtype,name,opts", CONFIGS, ids=[f"{d}-{n}" for d, n, _ in CONFIGS])
def test_grid30_depth20_against_oracle(env, golden, dtype, name, opts, monkeypatch):
    q, torch = env
    z, circ, idx = golden
    opts = dict(opts)
    if not opts.pop("jit", True):
        monkeypatch.setenv("QSIM_JIT", "0")
    bar = TOL[dtype]
    s = q.State(30, dtype)
    s.apply_circuit(q.PackedCircuit(circ), **opts)
    err = compare(q, torch, s, golden, dtype)
    s.close()
    del s
    torch.cuda.empty_cache()
    print(f"grid30 {dtype} {name}: " + " ".join(f"{k}={v:.3e}" for k, v in err.items()), flush=True)
    for key in ("samples", "lo_block", "hi_block"):
        assert err[key] <= bar, (key, err)
    for key in ("marg_lo", "marg_hi"):
        assert err[key] <= 2 * bar, (key, err)
    assert err["energy"] <= H_NORM_BOUND * (2 * bar + bar * bar) + 1e-13, err
