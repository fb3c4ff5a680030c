"""Python binding of the qsim HIP library (gfx950).

A thin ctypes layer over ``libqsim.so``: it marshals arguments into the C ABI
declared in ``include/qsim.h`` and nothing else -- every step of gate
application, fusion planning and reduction runs in the library.  PyTorch
supplies device memory (state tensors) and streams.

The functions named ``qsim_*`` mirror the C entry points one to one;
:class:`State` wraps them around a torch-owned state tensor.

The library must be built (``python -m paper_2106_13995_amd.build`` or
``__graft_entry__.build()``); importing this module raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqsim.so")

QSIM_OK = 0
QSIM_ERR_ARG = -1
QSIM_ERR_OOM = -2
QSIM_ERR_DEVICE = -3
QSIM_ERR_UNSUPPORTED = -4
QSIM_ERR_STATE = -5

QSIM_C64 = 1
QSIM_C128 = 2
DTYPES = {"c64": QSIM_C64, "c128": QSIM_C128, "complex64": QSIM_C64, "complex128": QSIM_C128}

GATE_CODES: Dict[str, int] = {
    "matrix": 0, "h": 1, "x": 2, "y": 3, "z": 4, "s": 5, "sdg": 6, "t": 7, "tdg": 8,
    "rx": 9, "ry": 10, "rz": 11, "u3": 12, "cx": 13, "cz": 14, "cp": 15, "swap": 16,
    "ccx": 17, "ccz": 18,
}

KCLASS = {"sweep_dense": 0, "sweep_diag": 1, "tile": 2, "mfma": 3, "expect": 4, "adjoint": 5, "tile_jit": 6}

MAX_K = 6

# Every symbol include/qsim.h declares.
EXPORTS = (
    "qsim_alloc", "qsim_wrap", "qsim_free", "qsim_set_stream", "qsim_state_info",
    "qsim_set_basis", "qsim_copy_to_host", "qsim_copy_from_host", "qsim_apply_gate",
    "qsim_apply_circuit", "qsim_expectation", "qsim_last_error", "qsim_profile_enable",
    "qsim_profile_read", "qsim_plan_summary", "qsim_adjoint_grad", "qsim_batch_create", "qsim_batch_run",
    "qsim_batch_info", "qsim_batch_layout", "qsim_batch_autotune", "qsim_batch_free", "qsim_autotune",
    "qsim_expectation_noalloc",
)


class QsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qsim status {status}: {msg}")
        self.status = status


class QsimOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32), ("targets", ctypes.c_int32 * MAX_K),
                ("param", ctypes.c_int32), ("reserved_", ctypes.c_int32), ("angles", ctypes.c_double * 3),
                ("mat_off", ctypes.c_int64)]


class QsimCircuit(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nops", ctypes.c_int32), ("ops", ctypes.POINTER(QsimOp)),
                ("mats", ctypes.POINTER(ctypes.c_double)), ("nmats", ctypes.c_int64)]


class QsimPauliTerm(ctypes.Structure):
    _fields_ = [("coeff", ctypes.c_double), ("xmask", ctypes.c_uint64), ("zmask", ctypes.c_uint64)]


class QsimPauliSum(ctypes.Structure):
    _fields_ = [("nterms", ctypes.c_int32), ("terms", ctypes.POINTER(QsimPauliTerm))]


class QsimOptions(ctypes.Structure):
    _fields_ = [("fuse_k", ctypes.c_int32), ("tile_m", ctypes.c_int32), ("use_mfma", ctypes.c_int32),
                ("split_1q", ctypes.c_int32), ("deterministic", ctypes.c_int32), ("checkpoints", ctypes.c_int32)]


def _hip_runtimes() -> set:
    try:
        with open("/proc/self/maps") as f:
            return {ln.split()[-1] for ln in f if "libamdhip64" in ln}
    except OSError:
        return set()


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    # torch provides device memory and streams, so the library must bind to
    # the HIP runtime torch already loaded (same soname) rather than a second
    # copy: import torch first, then check that only one runtime is mapped.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise ImportError(f"more than one HIP runtime is loaded: {sorted(rts)}")
    P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
    S = ctypes.c_int
    sig = {
        "qsim_alloc": ([i32, i32, ctypes.POINTER(P)], S),
        "qsim_wrap": ([P, i32, i32, P, ctypes.POINTER(P)], S),
        "qsim_free": ([P], S),
        "qsim_set_stream": ([P, P], S),
        "qsim_state_info": ([P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(P)], S),
        "qsim_set_basis": ([P, u64], S),
        "qsim_copy_to_host": ([P, P, ctypes.c_size_t], S),
        "qsim_copy_from_host": ([P, P, ctypes.c_size_t], S),
        "qsim_apply_gate": ([P, ctypes.POINTER(i32), i32, ctypes.POINTER(ctypes.c_double)], S),
        "qsim_apply_circuit": ([P, ctypes.POINTER(QsimCircuit), ctypes.POINTER(ctypes.c_double), i64,
                                ctypes.POINTER(QsimOptions)], S),
        "qsim_expectation": ([P, ctypes.POINTER(QsimPauliSum), ctypes.POINTER(ctypes.c_double)], S),
        "qsim_expectation_noalloc": ([P, ctypes.POINTER(QsimPauliSum), ctypes.POINTER(ctypes.c_double)], S),
        "qsim_adjoint_grad": ([P, ctypes.POINTER(QsimCircuit), P, i64, ctypes.POINTER(QsimPauliSum),
                               ctypes.POINTER(QsimOptions), P, P], S),
        "qsim_last_error": ([], ctypes.c_char_p),
        "qsim_plan_summary": ([i32, i32, ctypes.POINTER(QsimCircuit), ctypes.POINTER(ctypes.c_double), i64,
                               ctypes.POINTER(QsimOptions), ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double)], S),
        "qsim_profile_enable": ([P, i32], S),
        "qsim_batch_create": ([i32, ctypes.POINTER(QsimCircuit), ctypes.POINTER(i64), ctypes.POINTER(QsimPauliSum),
                               i32, i32, ctypes.POINTER(QsimOptions), ctypes.POINTER(P)], S),
        "qsim_batch_run": ([P, P, P, P, P], S),
        "qsim_batch_info": ([P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)], S),
        "qsim_batch_layout": ([P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)], S),
        "qsim_batch_autotune": ([i32, ctypes.POINTER(QsimCircuit), ctypes.POINTER(i64), ctypes.POINTER(QsimPauliSum),
                                 i32, i32, P, i32, ctypes.POINTER(QsimOptions), ctypes.POINTER(ctypes.c_double)], S),
        "qsim_batch_free": ([P], S),
        "qsim_autotune": ([P, ctypes.POINTER(QsimCircuit), ctypes.POINTER(ctypes.c_double), i64, i32,
                           ctypes.POINTER(QsimOptions), ctypes.POINTER(ctypes.c_double)], S),
        "qsim_profile_read": ([P, i32, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], S),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def _check(status: int) -> None:
    if status != QSIM_OK:
        raise QsimError(status, _lib.qsim_last_error().decode())


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ------------------------------------------------------------ raw entry points

def qsim_alloc(n: int, dtype: int) -> int:
    h = ctypes.c_void_p()
    _check(_lib.qsim_alloc(n, dtype, ctypes.byref(h)))
    return h.value


def qsim_wrap(dev_ptr: int, n: int, dtype: int, stream: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(_lib.qsim_wrap(ctypes.c_void_p(dev_ptr), n, dtype, ctypes.c_void_p(stream or None), ctypes.byref(h)))
    return h.value


def qsim_free(h: int) -> None:
    _check(_lib.qsim_free(ctypes.c_void_p(h)))


def qsim_set_stream(h: int, stream: int) -> None:
    _check(_lib.qsim_set_stream(ctypes.c_void_p(h), ctypes.c_void_p(stream or None)))


def qsim_state_info(h: int) -> Tuple[int, int, int]:
    n, dt, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_void_p()
    _check(_lib.qsim_state_info(ctypes.c_void_p(h), ctypes.byref(n), ctypes.byref(dt), ctypes.byref(p)))
    return n.value, dt.value, p.value or 0


def qsim_set_basis(h: int, index: int) -> None:
    _check(_lib.qsim_set_basis(ctypes.c_void_p(h), index))


def qsim_copy_to_host(h: int, out: np.ndarray) -> None:
    _check(_lib.qsim_copy_to_host(ctypes.c_void_p(h), out.ctypes.data_as(ctypes.c_void_p), out.nbytes))


def qsim_copy_from_host(h: int, src: np.ndarray) -> None:
    src = np.ascontiguousarray(src)
    _check(_lib.qsim_copy_from_host(ctypes.c_void_p(h), src.ctypes.data_as(ctypes.c_void_p), src.nbytes))


def qsim_apply_gate(h: int, targets: Sequence[int], U: np.ndarray) -> None:
    t = (ctypes.c_int * len(targets))(*[int(x) for x in targets])
    U = np.ascontiguousarray(U, dtype=np.complex128)
    _check(_lib.qsim_apply_gate(ctypes.c_void_p(h), t, len(targets), _dptr(U.view(np.float64))))


class PackedCircuit:
    """A circuit marshalled into the C structs (kept alive with its arrays)."""

    def __init__(self, circ):
        ops = (QsimOp * max(1, len(circ.ops)))()
        mats = []
        pos = 0
        for i, o in enumerate(circ.ops):
            op = ops[i]
            op.kind = GATE_CODES[o.kind]
            op.k = len(o.targets)
            for b, t in enumerate(o.targets):
                op.targets[b] = int(t)
            op.param = int(o.param)
            for a, v in enumerate(o.angles):
                op.angles[a] = float(v)
            if o.kind == "matrix":
                op.mat_off = pos
                mats.append(np.ascontiguousarray(o.matrix, dtype=np.complex128).reshape(-1))
                pos += o.matrix.size
        self.ops = ops
        self.mats = np.ascontiguousarray(np.concatenate(mats)) if mats else np.zeros(1, dtype=np.complex128)
        self.c = QsimCircuit(circ.n, len(circ.ops), ops,
                             self.mats.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             pos)
        self.n = circ.n
        self.nops = len(circ.ops)


def make_options(fuse_k: int = 0, tile_m: int = 0, use_mfma: int = 0, split_1q: int = 0,
                 deterministic: int = 0, checkpoints: int = 0) -> QsimOptions:
    return QsimOptions(fuse_k, tile_m, use_mfma, split_1q, deterministic, checkpoints)


def qsim_apply_circuit(h: int, packed: PackedCircuit, params: Optional[np.ndarray] = None,
                       opts: Optional[QsimOptions] = None) -> None:
    p = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
    _check(_lib.qsim_apply_circuit(ctypes.c_void_p(h), ctypes.byref(packed.c), _dptr(p),
                                   0 if p is None else p.size, ctypes.byref(opts) if opts is not None else None))


class PackedPauliSum:
    def __init__(self, H):
        terms = (QsimPauliTerm * max(1, len(H.coeffs)))()
        for i, (c, x, z) in enumerate(zip(H.coeffs, H.xmasks, H.zmasks)):
            terms[i] = QsimPauliTerm(float(c), int(x), int(z))
        self.terms = terms
        self.h = QsimPauliSum(len(H.coeffs), terms)


def qsim_expectation(h: int, packedH: PackedPauliSum) -> float:
    out = ctypes.c_double()
    _check(_lib.qsim_expectation(ctypes.c_void_p(h), ctypes.byref(packedH.h), ctypes.byref(out)))
    return out.value


def qsim_expectation_noalloc(h: int, packedH: PackedPauliSum) -> float:
    """qsim_expectation with its scratch in the library's fixed per-GPU array
    (no device allocation)."""
    out = ctypes.c_double()
    _check(_lib.qsim_expectation_noalloc(ctypes.c_void_p(h), ctypes.byref(packedH.h), ctypes.byref(out)))
    return out.value


def qsim_plan_summary(n: int, dtype: int, circ, params: Optional[np.ndarray] = None,
                      opts: Optional[QsimOptions] = None) -> Tuple[Dict[str, int], float, float]:
    """Host-only planning: passes per kernel class, algorithmic bytes and flops."""
    pc = circ if isinstance(circ, PackedCircuit) else PackedCircuit(circ)
    p = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
    counts = (ctypes.c_int64 * len(KCLASS))()
    by, fl = ctypes.c_double(), ctypes.c_double()
    _check(_lib.qsim_plan_summary(n, dtype, ctypes.byref(pc.c), _dptr(p), 0 if p is None else p.size,
                                  ctypes.byref(opts) if opts is not None else None, counts, ctypes.byref(by),
                                  ctypes.byref(fl)))
    return {name: counts[i] for name, i in KCLASS.items()}, by.value, fl.value


def _device_f64(t, name: str):
    """A contiguous float64 torch tensor on a GPU (device memory for the ABI)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 torch tensor on a GPU")
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


def qsim_adjoint_grad(h: int, packed: PackedCircuit, params_dev, packedH: PackedPauliSum,
                      opts: Optional[QsimOptions], energy_dev, grad_dev) -> None:
    """Queues the adjoint gradient on the state's stream: params_dev (nparams),
    energy_dev (1) and grad_dev (nparams) are float64 device tensors."""
    _check(_lib.qsim_adjoint_grad(ctypes.c_void_p(h), ctypes.byref(packed.c), _device_f64(params_dev, "params"),
                                  params_dev.numel(), ctypes.byref(packedH.h),
                                  ctypes.byref(opts) if opts is not None else None,
                                  _device_f64(energy_dev, "energy"), _device_f64(grad_dev, "grad")))


def qsim_profile_enable(h: int, on: bool) -> None:
    _check(_lib.qsim_profile_enable(ctypes.c_void_p(h), 1 if on else 0))


def qsim_profile_read(h: int, cls: int) -> Tuple[int, float, float, float]:
    """(launches, total ms, algorithmic bytes, algorithmic flops) of one kernel class."""
    n, ms, by, fl = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.qsim_profile_read(ctypes.c_void_p(h), cls, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                  ctypes.byref(fl)))
    return n.value, ms.value, by.value, fl.value


# ------------------------------------------------------------ torch-backed state

class State:
    """A state vector in a torch CUDA tensor, driven through the C ABI on
    torch's current stream."""

    def __init__(self, n: int, dtype: str = "c64", device: str = "cuda:0", init: bool = True):
        import torch
        self.n = n
        self.dtype = DTYPES[dtype]
        real = torch.float32 if self.dtype == QSIM_C64 else torch.float64
        self.tensor = torch.empty(2 << n, dtype=real, device=device)
        self.stream = torch.cuda.current_stream(self.tensor.device).cuda_stream
        self.handle = qsim_wrap(self.tensor.data_ptr(), n, self.dtype, self.stream)
        if init:
            self.set_basis(0)

    def close(self) -> None:
        if getattr(self, "handle", None):
            qsim_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nbytes(self) -> int:
        return self.tensor.numel() * self.tensor.element_size()

    def set_basis(self, index: int = 0) -> None:
        qsim_set_basis(self.handle, index)

    def apply_gate(self, targets: Sequence[int], U: np.ndarray) -> None:
        qsim_apply_gate(self.handle, targets, U)

    @staticmethod
    def packed(circ) -> PackedCircuit:
        """The circuit in the C structs: a PackedCircuit is used as given,
        anything else is marshalled afresh (callers that apply one circuit
        many times pack it once with PackedCircuit(circ))."""
        return circ if isinstance(circ, PackedCircuit) else PackedCircuit(circ)

    def apply_circuit(self, circ, params: Optional[np.ndarray] = None, fuse_k: int = 0, tile_m: int = 0,
                      use_mfma: int = 0, split_1q: int = 0) -> None:
        qsim_apply_circuit(self.handle, self.packed(circ), params, make_options(fuse_k, tile_m, use_mfma, split_1q))

    def expectation(self, H) -> float:
        return qsim_expectation(self.handle, PackedPauliSum(H))

    def adjoint_grad_device(self, circ, params, H, tile_m: int = 0, checkpoints: int = 0):
        """Energy (a one-element tensor) and gradient of <psi|C^dag H C|psi>
        for the state's current content psi, as float64 tensors on the
        state's device, queued on its stream without waiting; `params` is a
        float64 device tensor.  The state is returned to psi (up to
        rounding); `checkpoints` forward states are kept for the reverse
        sweep."""
        import torch
        dev = self.tensor.device
        energy = torch.empty(1, dtype=torch.float64, device=dev)
        grad = torch.empty(params.numel(), dtype=torch.float64, device=dev)
        qsim_adjoint_grad(self.handle, self.packed(circ), params, PackedPauliSum(H),
                          make_options(tile_m=tile_m, checkpoints=checkpoints), energy, grad)
        return energy, grad

    def adjoint_grad(self, circ, params, H, tile_m: int = 0, checkpoints: int = 0):
        """(energy, gradient) as a float and a numpy array: the parameters
        are copied to the device, the gradient back after the call."""
        import torch
        p = torch.as_tensor(np.ascontiguousarray(params, dtype=np.float64)).to(self.tensor.device)
        e, g = self.adjoint_grad_device(circ, p, H, tile_m=tile_m, checkpoints=checkpoints)
        return float(e.cpu()[0]), g.cpu().numpy()

    def autotune(self, circ, params: Optional[np.ndarray] = None, reps: int = 2):
        """Times the candidate options for `circ` on this state (overwriting it)
        and returns (options dict, ms per application) of the fastest."""
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        best = QsimOptions()
        ms = ctypes.c_double()
        _check(_lib.qsim_autotune(ctypes.c_void_p(self.handle), ctypes.byref(self.packed(circ).c), _dptr(p),
                                  0 if p is None else p.size, reps, ctypes.byref(best), ctypes.byref(ms)))
        return {"fuse_k": best.fuse_k, "tile_m": best.tile_m, "use_mfma": best.use_mfma,
                "split_1q": best.split_1q}, ms.value

    def to_numpy(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.complex64 if self.dtype == QSIM_C64 else np.complex128)
        qsim_copy_to_host(self.handle, out)
        return out

    def from_numpy(self, v: np.ndarray) -> None:
        v = np.ascontiguousarray(v, dtype=np.complex64 if self.dtype == QSIM_C64 else np.complex128)
        qsim_copy_from_host(self.handle, v)

    def profile(self, on: bool) -> None:
        qsim_profile_enable(self.handle, on)

    def profile_read(self, cls: str) -> Tuple[int, float, float, float]:
        return qsim_profile_read(self.handle, KCLASS[cls])


# ------------------------------------------------------------ batches

def _pack_batch(circuits, observables):
    """ctypes arrays of a batch's circuits and Pauli sums, its parameter
    offsets, and the objects that must stay alive while they are used."""
    packed = [PackedCircuit(c) for c in circuits]
    Hp = [PackedPauliSum(H) for H in observables]
    offs = [0]
    for c in circuits:
        offs.append(offs[-1] + int(c.nparams))
    n = len(circuits)
    carr = (QsimCircuit * n)(*[p.c for p in packed])
    harr = (QsimPauliSum * n)(*[h.h for h in Hp])
    return n, carr, harr, np.asarray(offs, dtype=np.int64), (packed, Hp, carr, harr)


class Batch:
    """Many independent circuits (each on |0...0>, each with its own parameter
    block and observable) run forward (+ adjoint) in one replayed graph."""

    def __init__(self, circuits, observables, dtype: str = "c64", want_grad: bool = True,
                 options: Optional[dict] = None):
        """`options`: {"fuse_k": 1..3, "tile_m": 11 or 12} (see
        qsim_batch_create), e.g. what Batch.autotune returns."""
        self.ncirc, carr, harr, self.offsets, keep = _pack_batch(circuits, observables)
        self.nparams = int(self.offsets[-1])
        self._keep = keep
        opts = make_options(**options) if options else None
        h = ctypes.c_void_p()
        _check(_lib.qsim_batch_create(self.ncirc, carr, self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      harr, DTYPES[dtype], 1 if want_grad else 0,
                                      ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)))
        self.handle = h.value
        self.want_grad = want_grad

    @staticmethod
    def autotune(circuits, observables, params, dtype: str = "c64", want_grad: bool = True, reps: int = 2):
        """Times the batch under each candidate option set (qsim_batch_autotune)
        and returns (options dict, ms per run) of the fastest; `params` as
        for run()."""
        import torch
        n, carr, harr, offsets, keep = _pack_batch(circuits, observables)
        p = torch.as_tensor(np.ascontiguousarray(params, dtype=np.float64)).to("cuda")
        best = QsimOptions()
        ms = ctypes.c_double()
        _check(_lib.qsim_batch_autotune(n, carr, offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), harr,
                                        DTYPES[dtype], 1 if want_grad else 0, _device_f64(p, "params"), reps,
                                        ctypes.byref(best), ctypes.byref(ms)))
        del keep
        return {"fuse_k": best.fuse_k, "tile_m": best.tile_m}, ms.value

    def info(self) -> Tuple[int, int, int]:
        g, p, m = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.qsim_batch_info(ctypes.c_void_p(self.handle), ctypes.byref(g), ctypes.byref(p), ctypes.byref(m)))
        return g.value, p.value, m.value

    def layout(self) -> Tuple[int, int]:
        """(circuits run layered, circuits run in the persistent kernel)."""
        lay, per = ctypes.c_int(), ctypes.c_int()
        _check(_lib.qsim_batch_layout(ctypes.c_void_p(self.handle), ctypes.byref(lay), ctypes.byref(per), None))
        return lay.value, per.value

    def pass_bytes(self) -> float:
        """Device-memory bytes one run's layered passes read and write."""
        v = ctypes.c_double()
        _check(_lib.qsim_batch_layout(ctypes.c_void_p(self.handle), None, None, ctypes.byref(v)))
        return v.value

    def run_device(self, params, energies=None, grads=None):
        """Queues one batch run on torch's current stream: `params` is a
        float64 device tensor of all parameter blocks; returns the energies
        and (with gradients) the gradient tensors, without waiting."""
        import torch
        if params.numel() != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {params.numel()}")
        dev = params.device
        if energies is None:
            energies = torch.empty(self.ncirc, dtype=torch.float64, device=dev)
        if grads is None and self.want_grad:
            grads = torch.empty(max(1, self.nparams), dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream(dev).cuda_stream
        _check(_lib.qsim_batch_run(ctypes.c_void_p(self.handle), _device_f64(params, "params"),
                                   _device_f64(energies, "energies"),
                                   _device_f64(grads, "grads") if grads is not None else None,
                                   ctypes.c_void_p(stream)))
        return energies, grads

    def run(self, params):
        """Host convenience: numpy (or tensor) parameters in, numpy energies
        and gradients out (copies to and from the device, then a wait)."""
        import torch
        p = torch.as_tensor(np.ascontiguousarray(params, dtype=np.float64)).to("cuda")
        e, g = self.run_device(p)
        return e.cpu().numpy(), (g[:self.nparams].cpu().numpy() if self.want_grad else None)

    def close(self) -> None:
        if getattr(self, "handle", None):
            _check(_lib.qsim_batch_free(ctypes.c_void_p(self.handle)))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ autograd

def _expectation_function():
    import torch

    class Expectation(torch.autograd.Function):
        """E(theta) = <0|C(theta)^dag H C(theta)|0> as a differentiable torch
        function; forward and the adjoint gradient run in one library call and
        backward scales the stored gradient by the incoming grad."""

        @staticmethod
        def forward(ctx, params, state, circ, H):
            # everything stays on the device and in stream order: the
            # parameters are read there, energy and gradient written there
            p = params.detach().to(state.tensor.device, torch.float64).contiguous()
            state.set_basis(0)
            e, g = state.adjoint_grad_device(circ, p, H)
            ctx.save_for_backward(g.to(params.dtype).to(params.device))
            return e[0].to(params.dtype).to(params.device)

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return grad_out * g, None, None, None

    return Expectation


def expectation(params, state: "State", circ, H):
    """Differentiable energy of `circ` applied to |0...0> in `state`."""
    return _expectation_function().apply(params, state, circ, H)
