// Device-side description of a batch of independent circuits (shared between
// the host builder and the persistent batch kernel).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "qsim_internal.h"

namespace qsim {

// Tile qubits of batch passes: psi and lambda tiles share LDS (2 x 32 KiB;
// measured on the 4096-circuit mix: 2^12 complex64 amplitudes per tile beat
// 2^11, which has twice the tiles and barriers, and 2^13, which leaves one
// workgroup per compute unit).
inline int batch_tile_max(int dtype) { return dtype == QSIM_C128 ? 11 : 12; }

struct BatchCircuit {
    int32_t prog;        // program (shared structure)
    int32_t nparams;     // this circuit's parameter count
    int64_t param_off;   // offset of its parameters / gradient entries
};

struct BatchProgram {
    int32_t n, m;        // qubits, tile qubits (m = n when the state is one tile)
    int32_t fwd_begin, fwd_end, rev_begin, rev_end;   // pass ranges
    int32_t hg_begin, hg_end;                         // observable term groups
};

struct BatchPass {
    int32_t L, H;
    int32_t hpos[16];
    int32_t op_begin, op_end;
};

struct BatchHGroup {
    uint64_t x;
    int32_t first, count;
};

struct BatchHTerm {
    double wr, wi;
    uint64_t z, pad_;
};

struct BatchDevice {
    const BatchCircuit *circs;
    const int32_t *order;
    const BatchProgram *progs;
    const BatchPass *passes;
    const TileOp *ops;
    const void *pool;
    const BatchHGroup *hgroups;
    const BatchHTerm *hterms;
    const double *params;
    double *energies;
    double *grads;
    void *arena;
    uint64_t slot_amps;
    int *counter;
    int ncirc;
    int want_grad;
    int mmax;            // tile qubits the LDS is sized for
};

hipError_t launch_batch(hipStream_t stream, int dtype, const BatchDevice &d, int grid);

}  // namespace qsim
