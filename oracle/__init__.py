"""CPU oracle for the state-vector simulator -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library: the arithmetic
lives in ``qsim_oracle.c`` (plain complex128 C, built with gcc) and this
module only marshals the workload descriptions into it, plus two methods of
differentiating an expectation value built on top of it:

* parameter shift: for a rotation exp(-i theta G / 2) with G^2 = 1 (and for
  the controlled phase, whose generator has eigenvalues 0 and 1) the
  derivative of an expectation is half the difference of the expectations at
  theta +- pi/2;
* central finite differences with step h.

The simulated quantity itself follows the paper (Sec. I.A, Sec. II): a vector
of 2^n complex amplitudes advanced gate by gate, each gate a matrix-vector
product.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsim_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_LIB_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")

# The oracle's own gate numbering (must match the enum in qsim_oracle.c).
CODES: Dict[str, int] = {
    "matrix": 0, "h": 1, "x": 2, "y": 3, "z": 4, "s": 5, "sdg": 6, "t": 7, "tdg": 8,
    "rx": 9, "ry": 10, "rz": 11, "u3": 12, "cx": 13, "cz": 14, "cp": 15, "swap": 16,
    "ccx": 17, "ccz": 18,
}
PERMUTATION_GATES = ("x", "cx", "ccx", "swap")
SHIFTABLE = ("rx", "ry", "rz", "cp")

_lib = None
_lib_omp = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU headers): the single-thread library
    and a second one built with OpenMP, whose gate loop runs over all host
    threads with the same per-amplitude arithmetic (bit-identical results)."""
    for path, extra in ((_LIB_PATH, []), (_LIB_OMP_PATH, ["-fopenmp"])):
        if not force and os.path.exists(path):
            continue
        tmp = path + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fcx-limited-range", "-Wall",
               *extra, "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return _LIB_PATH


def _bind(lib):
    P = ctypes.c_void_p
    i32, i64, u64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.oracle_gate_matrix.argtypes = [i32, P, P]
    lib.oracle_gate_matrix.restype = i32
    lib.oracle_apply_matrix.argtypes = [P, i32, P, i32, P]
    lib.oracle_apply_matrix.restype = i32
    lib.oracle_apply_permutation.argtypes = [P, P, i32, i32, P]
    lib.oracle_apply_permutation.restype = i32
    lib.oracle_apply_circuit.argtypes = [P, i32, i32, P, P, P, P, P, P]
    lib.oracle_apply_circuit.restype = i32
    lib.oracle_pauli_apply.argtypes = [P, P, i32, u64, u64]
    lib.oracle_pauli_apply.restype = None
    lib.oracle_expectation.argtypes = [P, i32, i32, P, P, P]
    lib.oracle_expectation.restype = f64
    lib.oracle_classical_run.argtypes = [i32, P, P, P, i64]
    lib.oracle_classical_run.restype = i32
    lib.oracle_product_cz_amplitudes.argtypes = [i32, P, i32, P, i64, P, P]
    lib.oracle_product_cz_amplitudes.restype = None
    return lib


def _load(threaded: bool = False):
    """The single-thread library, or (threaded=True) the OpenMP build."""
    global _lib, _lib_omp
    if threaded:
        if _lib_omp is None:
            if not os.path.exists(_LIB_OMP_PATH):
                build()
            _lib_omp = _bind(ctypes.CDLL(_LIB_OMP_PATH))
        return _lib_omp
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


# ------------------------------------------------------------ gates

def gate_matrix(kind: str, angles: Sequence[float] = ()) -> np.ndarray:
    lib = _load()
    ang = np.zeros(3)
    ang[:len(angles)] = angles
    U = np.zeros(64, dtype=np.complex128)
    k = lib.oracle_gate_matrix(CODES[kind], _ptr(ang), _ptr(U))
    if k < 0:
        raise ValueError(f"no matrix for {kind}")
    d = 1 << k
    return U[:d * d].reshape(d, d).copy()


def apply_matrix(psi: np.ndarray, targets: Sequence[int], U: np.ndarray) -> np.ndarray:
    """In place on a complex128 vector; returns it."""
    lib = _load()
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous
    n = int(psi.size).bit_length() - 1
    t = np.ascontiguousarray(targets, dtype=np.int32)
    U = _c128(U)
    rc = lib.oracle_apply_matrix(_ptr(psi), n, _ptr(t), len(t), _ptr(U))
    if rc != 0:
        raise ValueError("oracle_apply_matrix rejected its arguments")
    return psi


def apply_permutation(psi: np.ndarray, kind: str, targets: Sequence[int]) -> np.ndarray:
    lib = _load()
    n = int(psi.size).bit_length() - 1
    scratch = np.empty_like(psi)
    t = np.zeros(6, dtype=np.int32)
    t[:len(targets)] = targets
    rc = lib.oracle_apply_permutation(_ptr(psi), _ptr(scratch), n, CODES[kind], _ptr(t))
    if rc != 0:
        raise ValueError(f"{kind} is not a permutation gate")
    return psi


def _op_angles(o: W.Op, params: Optional[np.ndarray]) -> np.ndarray:
    ang = np.zeros(3)
    if o.param >= 0:
        if params is None:
            raise ValueError("parametric op without a parameter vector")
        m = W.GATE_NANGLES.get(o.kind, 0)
        ang[:m] = params[o.param:o.param + m]
    else:
        ang[:len(o.angles)] = o.angles
    return ang


def _pack(circ: W.Circuit, params: Optional[np.ndarray]):
    nops = len(circ.ops)
    codes = np.zeros(nops, dtype=np.int32)
    ks = np.zeros(nops, dtype=np.int32)
    targets = np.full((nops, 6), -1, dtype=np.int32)
    angles = np.zeros((nops, 3))
    offs = np.zeros(nops, dtype=np.int64)
    mats = []
    pos = 0
    for i, o in enumerate(circ.ops):
        codes[i] = CODES[o.kind]
        ks[i] = o.k
        targets[i, :o.k] = o.targets
        if o.kind == "matrix":
            offs[i] = pos
            mats.append(o.matrix.reshape(-1))
            pos += o.matrix.size
        else:
            angles[i] = _op_angles(o, params)
    mats_a = _c128(np.concatenate(mats)) if mats else np.zeros(1, dtype=np.complex128)
    return codes, ks, targets, angles, mats_a, offs


def basis_state(n: int, index: int = 0) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[index] = 1.0
    return psi


def apply_circuit(circ: W.Circuit, psi: Optional[np.ndarray] = None,
                  params: Optional[np.ndarray] = None, threaded: bool = False) -> np.ndarray:
    """Returns the state after the circuit (|0...0> when psi is None); the
    input array is not modified.  threaded=True runs the gate loop of the
    OpenMP build (same results, bit for bit)."""
    out = basis_state(circ.n) if psi is None else _c128(psi).copy()
    if out.size != (1 << circ.n):
        raise ValueError("state size does not match the circuit width")
    return apply_circuit_inplace(out, circ, params, threaded)


def apply_circuit_inplace(psi: np.ndarray, circ: W.Circuit, params: Optional[np.ndarray] = None,
                          threaded: bool = False) -> np.ndarray:
    """The circuit applied to a complex128 vector in place (no copy); returns it."""
    lib = _load(threaded)
    if psi.dtype != np.complex128 or not psi.flags.c_contiguous or psi.size != (1 << circ.n):
        raise ValueError("need a contiguous complex128 vector of 2^n amplitudes")
    codes, ks, targets, angles, mats, offs = _pack(circ, params)
    rc = lib.oracle_apply_circuit(_ptr(psi), circ.n, len(codes), _ptr(codes), _ptr(ks),
                                  _ptr(targets), _ptr(angles), _ptr(mats), _ptr(offs))
    if rc != 0:
        raise ValueError(f"oracle rejected op {-rc - 1}")
    return psi


def circuit_dagger(circ: W.Circuit, params: Optional[np.ndarray] = None) -> W.Circuit:
    """Inverse circuit as dense-matrix ops (conjugate transposes in reverse order)."""
    ops = []
    for o in reversed(circ.ops):
        M = o.matrix if o.kind == "matrix" else gate_matrix(o.kind, _op_angles(o, params))
        ops.append(W.matrix_op(o.targets, M.conj().T))
    return W.Circuit(circ.n, ops, 0, circ.name + "_dag")


# ------------------------------------------------------------ observables

def _pauli_arrays(H: W.PauliSum):
    c = np.ascontiguousarray(H.coeffs, dtype=np.float64)
    x = np.ascontiguousarray(H.xmasks, dtype=np.uint64)
    z = np.ascontiguousarray(H.zmasks, dtype=np.uint64)
    return c, x, z


def pauli_apply(psi: np.ndarray, xmask: int, zmask: int) -> np.ndarray:
    lib = _load()
    psi = _c128(psi)
    n = int(psi.size).bit_length() - 1
    out = np.empty_like(psi)
    lib.oracle_pauli_apply(_ptr(psi), _ptr(out), n, int(xmask), int(zmask))
    return out


def expectation(psi: np.ndarray, H: W.PauliSum) -> float:
    lib = _load()
    psi = _c128(psi)
    n = int(psi.size).bit_length() - 1
    c, x, z = _pauli_arrays(H)
    return float(lib.oracle_expectation(_ptr(psi), n, len(c), _ptr(c), _ptr(x), _ptr(z)))


def energy(circ: W.Circuit, params: np.ndarray, H: W.PauliSum, threaded: bool = False) -> float:
    return expectation(apply_circuit(circ, params=params, threaded=threaded), H)


# ------------------------------------------------------------ gradients

def param_shift_grad(circ: W.Circuit, params: np.ndarray, H: W.PauliSum,
                     indices: Optional[Sequence[int]] = None, threaded: bool = False) -> np.ndarray:
    """dE/dtheta_j by the shift rule, shifting each occurrence of a parameter
    separately and summing (product rule).  With `indices`, only those
    parameters are differentiated (the other entries stay 0)."""
    params = np.asarray(params, dtype=np.float64)
    grad = np.zeros_like(params)
    wanted = None if indices is None else set(int(j) for j in indices)
    for i, o in enumerate(circ.ops):
        if o.param < 0 or (wanted is not None and o.param not in wanted):
            continue
        if o.kind not in SHIFTABLE:
            raise ValueError(f"no shift rule for {o.kind}")
        base = _op_angles(o, params)[0]
        vals = []
        for s in (+0.5 * np.pi, -0.5 * np.pi):
            ops = list(circ.ops)
            ops[i] = W.Op(o.kind, o.targets, (base + s,), -1)
            vals.append(energy(W.Circuit(circ.n, ops, circ.nparams), params, H, threaded))
        grad[o.param] += 0.5 * (vals[0] - vals[1])
    return grad


def finite_diff_grad(circ: W.Circuit, params: np.ndarray, H: W.PauliSum, h: float = 1e-4,
                     indices: Optional[Sequence[int]] = None) -> np.ndarray:
    params = np.asarray(params, dtype=np.float64)
    idx = range(params.size) if indices is None else indices
    grad = np.zeros(params.size)
    for j in idx:
        p = params.copy()
        p[j] += h
        ep = energy(circ, p, H)
        p[j] -= 2 * h
        em = energy(circ, p, H)
        grad[j] = (ep - em) / (2 * h)
    return grad


# ------------------------------------------------------------ classical / closed forms

def classical_run(circ: W.Circuit, inputs: Sequence[int]) -> np.ndarray:
    """Outputs of a permutation-only circuit on basis inputs."""
    lib = _load()
    codes, ks, targets, angles, mats, offs = _pack(circ, None)
    xs = np.ascontiguousarray(inputs, dtype=np.uint64).copy()
    rc = lib.oracle_classical_run(len(codes), _ptr(codes), _ptr(targets), _ptr(xs), xs.size)
    if rc != 0:
        raise ValueError(f"op {-rc - 1} is not a permutation gate")
    return xs


def product_cz_amplitudes(n: int, one_qubit_ops: Sequence[W.Op], cz_pairs, indices) -> np.ndarray:
    """Closed-form amplitudes of (one 1-qubit gate per qubit on |0...0>) then a
    layer of disjoint CZ pairs, evaluated one index at a time."""
    lib = _load()
    col0 = np.zeros((n, 2), dtype=np.complex128)
    for o in one_qubit_ops:
        col0[o.targets[0]] = gate_matrix(o.kind, o.angles)[:, 0]
    pairs = np.ascontiguousarray(np.asarray(cz_pairs, dtype=np.int32).reshape(-1, 2))
    idx = np.ascontiguousarray(indices, dtype=np.uint64)
    out = np.empty(idx.size, dtype=np.complex128)
    lib.oracle_product_cz_amplitudes(n, _ptr(col0), pairs.shape[0], _ptr(pairs), idx.size,
                                     _ptr(idx), _ptr(out))
    return out


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_2 / ||b||_2 in double precision."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))
