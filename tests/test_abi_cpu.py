"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and rejects invalid arguments before any device work.

No kernel runs here: states are wrapped around a placeholder address that is
never dereferenced, and every call below fails validation first.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qsim.h")

q = pytest.importorskip("paper_2106_13995_amd")

FAKE_PTR = 1 << 40   # 256-byte aligned placeholder, never dereferenced


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qsim_[a-z_]+)\s*\(", text)))


def test_header_declarations_all_exported():
    decl = declared_functions()
    assert set(decl) == set(q.EXPORTS)
    lib = ctypes.CDLL(q.LIB_PATH)
    for name in decl:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header_sizes(tmp_path):
    # the binding's ctypes structs against what a C compiler makes of the header
    import subprocess
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "qsim.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(qsim_op), sizeof(qsim_circuit), '
                   'sizeof(qsim_pauli_term), sizeof(qsim_pauli_sum), sizeof(qsim_options), '
                   'offsetof(qsim_options, checkpoints)); return 0; }\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [ctypes.sizeof(q.QsimOp), ctypes.sizeof(q.QsimCircuit), ctypes.sizeof(q.QsimPauliTerm),
                   ctypes.sizeof(q.QsimPauliSum), ctypes.sizeof(q.QsimOptions), q.QsimOptions.checkpoints.offset]


def test_wrap_validation():
    with pytest.raises(q.QsimError) as e:
        q.qsim_wrap(FAKE_PTR, 0, q.QSIM_C64)
    assert e.value.status == q.QSIM_ERR_ARG
    with pytest.raises(q.QsimError):
        q.qsim_wrap(FAKE_PTR, 36, q.QSIM_C64)
    with pytest.raises(q.QsimError):
        q.qsim_wrap(FAKE_PTR, 35, q.QSIM_C128)
    with pytest.raises(q.QsimError):
        q.qsim_wrap(FAKE_PTR + 8, 10, q.QSIM_C64)
    with pytest.raises(q.QsimError):
        q.qsim_wrap(FAKE_PTR, 10, 7)
    with pytest.raises(q.QsimError):
        q.qsim_wrap(0, 10, q.QSIM_C64)


@pytest.fixture
def fake_state():
    h = q.qsim_wrap(FAKE_PTR, 8, q.QSIM_C64)
    yield h
    q.qsim_free(h)


def test_state_info(fake_state):
    assert q.qsim_state_info(fake_state) == (8, q.QSIM_C64, FAKE_PTR)


@pytest.mark.parametrize("targets,k", [([8], 1), ([-1], 1), ([1, 1], 2), ([0, 1, 2, 3, 4, 5, 6], 7)])
def test_apply_gate_rejects_bad_targets(fake_state, targets, k):
    U = np.eye(1 << min(k, 6), dtype=np.complex128)
    t = (ctypes.c_int * len(targets))(*targets)
    st = q._lib.qsim_apply_gate(ctypes.c_void_p(fake_state), t, k, U.view(np.float64).ctypes.data_as(
        ctypes.POINTER(ctypes.c_double)))
    assert st == q.QSIM_ERR_ARG
    assert q._lib.qsim_last_error().decode()


def _circuit_status(h, circ, params=None, opts=None):
    pc = q.PackedCircuit(circ)
    p = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
    return q._lib.qsim_apply_circuit(ctypes.c_void_p(h), ctypes.byref(pc.c), q._dptr(p),
                                     0 if p is None else p.size,
                                     ctypes.byref(opts) if opts is not None else None)


def test_apply_circuit_validation(fake_state):
    # width mismatch
    assert _circuit_status(fake_state, W.ghz_circuit(5)) == q.QSIM_ERR_ARG
    # duplicate / out-of-range targets are caught in op validation
    bad = W.Circuit(8, [W.Op("cx", (3, 3))])
    assert _circuit_status(fake_state, bad) == q.QSIM_ERR_ARG
    bad = W.Circuit(8, [W.Op("h", (9,))])
    assert _circuit_status(fake_state, bad) == q.QSIM_ERR_ARG
    # parametric op without parameters
    par = W.Circuit(8, [W.op("ry", 0, param=0)], 1)
    assert _circuit_status(fake_state, par) == q.QSIM_ERR_ARG
    assert _circuit_status(fake_state, par, params=np.zeros(0)) == q.QSIM_ERR_ARG
    # parametric index past the end
    par2 = W.Circuit(8, [W.op("u3", 0, param=1)], 3)
    assert _circuit_status(fake_state, par2, params=np.zeros(3)) == q.QSIM_ERR_ARG
    # arity mismatch
    bad = W.Circuit(8, [W.Op("ccx", (0, 1))])
    assert _circuit_status(fake_state, bad) == q.QSIM_ERR_ARG
    # bad options
    assert _circuit_status(fake_state, W.ghz_circuit(8), opts=q.make_options(fuse_k=7)) == q.QSIM_ERR_ARG
    assert _circuit_status(fake_state, W.ghz_circuit(8), opts=q.make_options(tile_m=3)) == q.QSIM_ERR_ARG


def test_matrix_pool_bounds(fake_state):
    op = q.QsimOp()
    op.kind = 0
    op.k = 2
    op.targets[0], op.targets[1] = 0, 1
    op.param = -1
    op.mat_off = 4          # 16 entries needed from offset 4: pool of 16 is too short
    mats = np.zeros(16, dtype=np.complex128)
    c = q.QsimCircuit(8, 1, ctypes.pointer(op), mats.view(np.float64).ctypes.data_as(
        ctypes.POINTER(ctypes.c_double)), 16)
    st = q._lib.qsim_apply_circuit(ctypes.c_void_p(fake_state), ctypes.byref(c), None, 0, None)
    assert st == q.QSIM_ERR_ARG
    assert "pool" in q._lib.qsim_last_error().decode()


def test_expectation_mask_validation(fake_state):
    H = W.PauliSum(9, [1.0], [0], [1 << 8])
    out = ctypes.c_double()
    st = q._lib.qsim_expectation(ctypes.c_void_p(fake_state), ctypes.byref(q.PackedPauliSum(H).h),
                                 ctypes.byref(out))
    assert st == q.QSIM_ERR_ARG


def test_set_basis_validation(fake_state):
    with pytest.raises(q.QsimError):
        q.qsim_set_basis(fake_state, 256)


def test_null_handles():
    assert q._lib.qsim_set_basis(None, 0) == q.QSIM_ERR_ARG
    assert q._lib.qsim_free(None) == q.QSIM_OK


# ------------------------------------------------------------ host planner (no device work)

def _summary(circ, n=None, dtype=1, **opts):
    return q.qsim_plan_summary(n or circ.n, dtype, circ, opts=q.make_options(**opts) if opts else None)


def test_plan_summary_sweeps_count_every_gate():
    circ = W.random_grid_circuit(5, 6, depth=20, seed=2)
    counts, by, fl = _summary(circ, fuse_k=1, tile_m=-1)
    assert counts["sweep_dense"] == circ.count("u3") and counts["sweep_diag"] == circ.count("cz")
    N, s = 2 ** 30, 8
    # a U3 sweep moves 2 N s bytes, a CZ only the quarter with both bits set
    assert by == 600 * 2 * N * s + 245 * 2 * (N // 4) * s
    assert fl == 600 * 16 * N + 245 * 6 * (N // 4)


def test_plan_summary_controls_and_diagonals():
    ops = [W.op("cx", 3, 17), W.op("ccx", 1, 2, 20), W.op("ccz", 4, 5, 6), W.op("cp", 7, 8, angles=(0.3,))]
    circ = W.Circuit(24, ops)
    counts, by, fl = _summary(circ, fuse_k=1, tile_m=-1)
    N, s = 2 ** 24, 8
    assert counts["sweep_dense"] == 2 and counts["sweep_diag"] == 2
    assert by == 2 * (N // 2) * s + 2 * (N // 4) * s + 2 * (N // 8) * s + 2 * (N // 4) * s


def test_plan_summary_tiles_fewer_passes_and_same_flops():
    circ = W.random_grid_circuit(5, 6, depth=20, seed=2)
    c_sw, b_sw, f_sw = _summary(circ, fuse_k=1, tile_m=-1)
    c_t, b_t, f_t = _summary(circ, fuse_k=1, tile_m=12, split_1q=-1)
    assert 10 <= c_t["tile"] <= 40
    assert b_t == c_t["tile"] * 2 * 2 ** 30 * 8
    assert f_t == f_sw                       # same gate arithmetic, grouped differently
    c_f, b_f, f_f = _summary(circ, fuse_k=5, tile_m=-1)
    assert c_f["mfma"] > 0 and sum(c_f.values()) < sum(c_sw.values())


def test_plan_summary_split_rotations():
    # every U3 becomes a real rotation (6 flop per amplitude by lifting) plus
    # an input phase on half the amplitudes (3); CZ arithmetic is unchanged
    circ = W.random_grid_circuit(5, 6, depth=20, seed=2)
    c_p, b_p, f_p = _summary(circ, fuse_k=1, tile_m=12, split_1q=-1)
    c_s, b_s, f_s = _summary(circ, fuse_k=1, tile_m=12)
    N = 2 ** 30
    assert b_s == c_s["tile"] * 2 * N * 8
    u3 = circ.count("u3")
    other = f_p - u3 * 16 * N                 # CZ arithmetic, the same in both plans
    # U3s at 9 flop per amplitude, plus at most one phase per qubit left over
    # at the end (6 flop on half the amplitudes, the global factor on all)
    assert u3 * 9 * N + other <= f_s <= u3 * 9 * N + other + (30 * 3 + 6) * N
    assert f_s < 0.6 * f_p
    # exact gates keep exact phases: X and H split with phase -1, S merges
    ops = [W.op("x", 0), W.op("h", 1), W.op("s", 1), W.op("h", 1), W.op("cx", 0, 1)]
    c1, b1, f1 = _summary(W.Circuit(10, ops), fuse_k=1, tile_m=10)
    assert c1["tile"] == 1 and f1 > 0


def test_split_option_validation(fake_state):
    assert _circuit_status(fake_state, W.ghz_circuit(8), opts=q.make_options(split_1q=2)) == q.QSIM_ERR_ARG


def test_plan_summary_rejects_bad_ops_without_device():
    bad = W.Circuit(8, [W.Op("cz", (2, 2))])
    with pytest.raises(q.QsimError):
        _summary(bad)


@pytest.mark.parametrize("fuse_k,tile_m", [(1, 7), (1, 8), (1, 9), (5, 9), (3, 7), (6, 10)])
def test_small_tiles_place_every_gate(fuse_k, tile_m):
    # A tile of 2^m amplitudes keeps its low 5 (c64) / 4 (c128) qubits for
    # contiguous HBM runs; a gate on qubits outside them needs more positions
    # than a small m leaves.  The planner must widen the tile rather than
    # drop the gate: the arithmetic of the tile plan equals that of one sweep
    # per (fused) gate.
    for circ in (W.random_grid_circuit(4, 4, depth=20, seed=2),
                 W.Circuit(14, [W.op("h", 0), W.op("ccx", 10, 11, 12), W.op("h", 13)])):
        for dtype in (1, 2):
            _, _, f_sweep = _summary(circ, dtype=dtype, fuse_k=fuse_k, tile_m=-1, use_mfma=1)
            c_t, b_t, f_t = _summary(circ, dtype=dtype, fuse_k=fuse_k, tile_m=tile_m, split_1q=-1)
            assert c_t["tile"] >= 1
            assert f_t == pytest.approx(f_sweep, rel=1e-12), (dtype, f_t, f_sweep)


def test_six_qubit_block_outside_low_qubits_in_small_tiles():
    rng = np.random.default_rng(11)
    circ = W.Circuit(14, [W.matrix_op(list(range(8, 14)), W.random_unitary(6, rng))])
    N = 2 ** 14
    for dtype in (1, 2):
        for tile_m in (7, 10):
            c, b, f = _summary(circ, dtype=dtype, fuse_k=1, tile_m=tile_m)
            assert c["tile"] == 1 and f == 8 * 64 * N



# ------------------------------------------------------------ failure paths

def test_injected_launch_fault_invalidates_the_state(monkeypatch):
    """QSIM_FAULT=launch fails the next launch point as a failed kernel launch
    would (nothing is launched): the call returns QSIM_ERR_DEVICE, and every
    later call on that state QSIM_ERR_STATE until it is freed."""
    h = q.qsim_wrap(FAKE_PTR, 8, q.QSIM_C64)
    monkeypatch.setenv("QSIM_FAULT", "launch")
    assert q._lib.qsim_set_basis(ctypes.c_void_p(h), 0) == q.QSIM_ERR_DEVICE
    assert "QSIM_FAULT" in q._lib.qsim_last_error().decode()
    monkeypatch.delenv("QSIM_FAULT")
    assert q._lib.qsim_set_basis(ctypes.c_void_p(h), 0) == q.QSIM_ERR_STATE
    assert _circuit_status(h, W.ghz_circuit(8)) == q.QSIM_ERR_STATE
    out = ctypes.c_double()
    H = q.PackedPauliSum(W.chain_observable(8))
    assert q._lib.qsim_expectation(ctypes.c_void_p(h), ctypes.byref(H.h), ctypes.byref(out)) == q.QSIM_ERR_STATE
    assert q._lib.qsim_free(ctypes.c_void_p(h)) == q.QSIM_OK


def test_injected_fault_at_the_nth_launch_point(monkeypatch):
    """launch:N fails only the N-th launch point: validation errors before it
    still return QSIM_ERR_ARG and leave the state valid."""
    h = q.qsim_wrap(FAKE_PTR, 6, q.QSIM_C64)
    monkeypatch.setenv("QSIM_FAULT", "launch:1")
    assert q._lib.qsim_set_basis(ctypes.c_void_p(h), 1 << 6) == q.QSIM_ERR_ARG   # rejected before any launch
    assert q._lib.qsim_set_basis(ctypes.c_void_p(h), 3) == q.QSIM_ERR_DEVICE
    assert "QSIM_FAULT" in q._lib.qsim_last_error().decode()
    assert q._lib.qsim_set_basis(ctypes.c_void_p(h), 3) == q.QSIM_ERR_STATE
    q.qsim_free(h)
