"""The run-time compiled register tile passes, run on the CPU, against the
oracle (the ordered product of the gate matrices, paper Sec. I.A and II).

`host_emulation/jit_emit.cpp` plans a circuit with the library's host code
and writes the straight-line source the library would hand to the run-time
compiler; `host_emulation/jit_emu.cpp` builds that source for the host
(clang, the same source text) and runs every pass over every tile, with each
workgroup's 256 threads as POSIX threads meeting at a barrier.  The result is
compared with the complex128 oracle at the GPU tolerances.  This checks what
the generator writes (register layouts, LDS exchanges, the sign changes and
scale factors it leaves owed from pass to pass) without a GPU; the GPU tests
run the same passes compiled for gfx950.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
import workloads as W

from circuit_io import write_circuit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2106_13995_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "host_emulation")
HOST_SOURCES = ["abi.cpp", "plan.cpp", "stages.cpp", "gates.cpp", "jit.cpp", "autotune.cpp", "batch.cpp"]
CLANG = "/opt/rocm/llvm/bin/clang++"
TOL = {"c64": 2e-5, "c128": 1e-12}

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(CLANG),
                                reason="needs g++ and ROCm's clang")


@pytest.fixture(scope="module")
def emitter(tmp_path_factory):
    pytest.importorskip("torch")
    d = tmp_path_factory.mktemp("jit_emit")
    exe = str(d / "jit_emit")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                        "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                        *[os.path.join(CSRC, f) for f in HOST_SOURCES], os.path.join(EMU, "jit_emit.cpp"),
                        "-o", exe, "-L/opt/rocm/lib", "-lamdhip64", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def run_emulated(emitter, tmp, circ, tile_m, dtype, map_shift=None, psi0=None):
    d = str(tmp)
    cf = os.path.join(d, "c.bin")
    write_circuit(cf, circ)
    dt = 1 if dtype == "c64" else 2
    env = dict(os.environ)
    if map_shift is not None:
        env["QSIM_MAP_SHIFT"] = str(map_shift)
    r = subprocess.run([emitter, cf, str(tile_m), str(dt), d], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr
    exe = os.path.join(d, "emu")
    flags = ["-O1", "-std=c++17", "-I", d, "-pthread"] + (["-DEMU_DOUBLE"] if dt == 2 else [])
    r = subprocess.run([CLANG, *flags, os.path.join(EMU, "jit_emu.cpp"), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    npdt = np.complex64 if dt == 1 else np.complex128
    if psi0 is None:
        psi = np.zeros(1 << circ.n, dtype=npdt)
        psi[0] = 1
    else:
        psi = np.asarray(psi0, dtype=npdt)
    psi.tofile(os.path.join(d, "in.bin"))
    r = subprocess.run([exe, d, os.path.join(d, "in.bin"), os.path.join(d, "out.bin")], capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    return np.fromfile(os.path.join(d, "out.bin"), dtype=npdt).astype(np.complex128)


def mixed_circuit(n, nops, seed):
    """U3, RY, H, CZ, CCZ, CX, CCX, controlled one-qubit blocks and dense
    two-qubit blocks in random order on random qubits."""
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(nops):
        r = int(rng.integers(9))
        q = [int(x) for x in rng.choice(n, 3, replace=False)]
        if r == 0:
            ops.append(W.op("u3", q[0], angles=rng.uniform(0, 2 * np.pi, 3)))
        elif r == 1:
            ops.append(W.op("cz", q[0], q[1]))
        elif r == 2:
            ops.append(W.op("cx", q[0], q[1]))
        elif r == 3:
            ops.append(W.op("ccx", q[0], q[1], q[2]))
        elif r == 4:
            ops.append(W.op("h", q[0]))
        elif r == 5:
            ops.append(W.op("ccz", q[0], q[1], q[2]))
        elif r == 6:
            M = np.eye(4, dtype=complex)
            M[2:, 2:] = W.random_unitary(1, rng)
            ops.append(W.matrix_op([q[1], q[0]], M))
        elif r == 7:
            ops.append(W.matrix_op([q[0], q[1]], W.random_unitary(2, rng)))
        else:
            ops.append(W.op("ry", q[0], angles=[rng.uniform(0, 2 * np.pi)]))
    return W.Circuit(n, ops)


CASES = [
    # grid circuits: CZ signs owed across every pass, settled in the last
    ("grid3x5", lambda: W.random_grid_circuit(3, 5, depth=12, seed=5), [("c64", 12), ("c64", 13), ("c128", 12)]),
    # exchanges, controlled blocks and dense blocks next to owed signs
    ("mixed14", lambda: mixed_circuit(14, 300, 7), [("c64", 12), ("c128", 12)]),
    # permutation gates only (multiplier on a superposed input)
    ("mult13", lambda: W.multiplier_circuit(5, 6, 3, superpose_a=True), [("c64", 13)]),
]


@pytest.mark.parametrize("name,make,runs", CASES, ids=[c[0] for c in CASES])
def test_compiled_passes_on_the_host_match_the_oracle(emitter, tmp_path, name, make, runs):
    circ = make()
    ref = O.apply_circuit(circ)
    for dtype, tile_m in runs:
        sub = tmp_path / f"{dtype}_{tile_m}"
        sub.mkdir()
        out = run_emulated(emitter, sub, circ, tile_m, dtype)
        err = O.rel_l2(out, ref)
        assert err <= TOL[dtype], (name, dtype, tile_m, err)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_occupancy_maps_on_sparse_states(emitter, tmp_path, dtype):
    """Multiplier circuits (few spreading gates: the passes keep occupancy
    maps, here with 2^6-amplitude chunks so that small states have many) on
    a basis input, a superposed input and a dense random input: the maps may
    only skip tiles that are zero."""
    bits = 4
    L = W.MultiplierLayout(bits)
    core = W.multiplier_core(bits)
    rng = np.random.default_rng(31)
    for k, kind in enumerate(("basis", "superposed", "dense")):
        if kind == "basis":
            psi0 = np.zeros(1 << L.n, dtype=np.complex128)
            psi0[L.basis_index(11, 13)] = 1
        elif kind == "superposed":
            psi0 = np.zeros(1 << L.n, dtype=np.complex128)
            for a in range(16):
                psi0[L.basis_index(a, 9)] = 0.25
        else:
            psi0 = W.random_state(L.n, rng)
        ref = O.apply_circuit(core, psi0)
        sub = tmp_path / kind
        sub.mkdir()
        out = run_emulated(emitter, sub, core, 12, dtype, map_shift=6, psi0=psi0)
        assert O.rel_l2(out, ref) <= TOL[dtype], (kind, O.rel_l2(out, ref))
        if kind == "basis":
            assert np.count_nonzero(out) == 1
