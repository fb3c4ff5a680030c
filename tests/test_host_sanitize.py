"""The host planner under AddressSanitizer and UndefinedBehaviorSanitizer.

`host_sanitize/planner_check.cpp` links the library's host sources (ABI,
planning, fusion, register programs, compiled-pass source, autotuner, batch
set-up) with stub device launchers, and plans the circuits written here at
both precisions under many options.  Any out-of-bounds access, use after
free or undefined operation aborts it.  CPU only (g++); the build takes
about a minute.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import workloads as W
from circuit_io import write_circuit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2106_13995_amd", "csrc")
HOST_SOURCES = ["abi.cpp", "plan.cpp", "stages.cpp", "gates.cpp", "jit.cpp", "autotune.cpp", "batch.cpp"]


def controlled_blocks(n, nops, rng):
    ops = []
    for _ in range(nops):
        r = rng.integers(5)
        if r == 0:
            ops.append(W.op("u3", int(rng.integers(n)), angles=rng.uniform(0, 2 * np.pi, 3)))
        elif r == 1:
            a, b = rng.choice(n, 2, replace=False)
            ops.append(W.op("cx", int(a), int(b)))
        elif r == 2:
            a, b, c = rng.choice(n, 3, replace=False)
            ops.append(W.op("ccx", int(a), int(b), int(c)))
        else:
            k = int(rng.integers(1, 4))
            qs = [int(x) for x in rng.choice(n, k + 1, replace=False)]
            d = 1 << (k + 1)
            M = np.eye(d, dtype=complex)
            M[d - 2:, d - 2:] = W.random_unitary(1, rng)
            ops.append(W.matrix_op(qs, M))
    return W.Circuit(n, ops)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_under_sanitizers(tmp_path):
    pytest.importorskip("torch")
    rng = np.random.default_rng(401)
    circuits = [
        (W.random_grid_circuit(5, 6, depth=20, seed=2), None),
        (W.multiplier_circuit(0, 10, 7, superpose_a=True), None),
        (W.width_circuit("supremacy", 13), None),
        (W.width_circuit("multiplier", 21), None),
        (W.random_circuit(16, 200, rng, max_matrix_k=6), None),
        (controlled_blocks(14, 200, rng), None),
        (W.ansatz_circuit(20, 10), W.ansatz_params(20, 10, seed=4)),
        (W.random_line_circuit(5, 8, seed=1), None),
        # gates wider than a small tile's free positions (the tile is widened)
        (W.Circuit(14, [W.op("h", 0), W.op("ccx", 10, 11, 12)]), None),
        (W.Circuit(14, [W.matrix_op(list(range(8, 14)), W.random_unitary(6, rng)), W.op("h", 3)]), None),
    ]
    files = []
    for i, (c, p) in enumerate(circuits):
        path = str(tmp_path / f"c{i}.bin")
        write_circuit(path, c, p)
        files.append(path)
    exe = str(tmp_path / "planner_check")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    srcs = [os.path.join(CSRC, f) for f in HOST_SOURCES] + [os.path.join(ROOT, "tests", "host_sanitize",
                                                                          "planner_check.cpp")]
    build = subprocess.run(["g++", *flags, *srcs, "-o", exe, "-L/opt/rocm/lib", "-lamdhip64", "-lhiprtc",
                            "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-3000:]
    # a tuning cache with lines outside the accepted option ranges and junk
    cache = tmp_path / "tune.txt"
    cache.write_text("deadbeef 12 1 9 7 0\nabc 12 1 1 99 0\n1 14 2 2 3 0\n12 oops\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", QSIM_JIT="0", QSIM_TUNE_CACHE=str(cache))
    run = subprocess.run([exe, *files], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "planner check:" in run.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    """The CPU oracle built with AddressSanitizer and UBSan, driven through
    every entry point (all gate codes, a dense 6-qubit matrix, rejected
    arguments)."""
    exe = str(tmp_path / "oracle_check")
    build = subprocess.run(["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-fcx-limited-range",
                            "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                            os.path.join(ROOT, "oracle", "qsim_oracle.c"),
                            os.path.join(ROOT, "tests", "host_sanitize", "oracle_check.c"), "-lm", "-o", exe],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-3000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                                  UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1"))
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "oracle check:" in run.stdout
