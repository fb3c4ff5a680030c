"""Circuit files for the host-side test programs (planner check, compiled-pass
emulation): a header (n, nops, nparams, nmats), the qsim_op records as the C
ABI lays them out, the complex128 matrix pool and the parameters."""
import ctypes
import struct

import numpy as np


def write_circuit(path, circ, params=None):
    import paper_2106_13995_amd as q
    pc = q.PackedCircuit(circ)
    raw = ctypes.string_at(ctypes.addressof(pc.ops), ctypes.sizeof(q.QsimOp) * len(circ.ops))
    mats = pc.mats.view(np.float64) if pc.c.nmats else np.zeros(0)
    p = np.zeros(0) if params is None else np.ascontiguousarray(params, dtype=np.float64)
    with open(path, "wb") as f:
        f.write(struct.pack("<iiiq", circ.n, len(circ.ops), p.size, int(pc.c.nmats)))
        f.write(raw)
        f.write(np.ascontiguousarray(mats[:2 * int(pc.c.nmats)]).tobytes())
        f.write(p.tobytes())
