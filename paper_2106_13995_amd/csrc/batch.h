// Device-side description of a batch of independent circuits (shared between
// the host builder and the persistent batch kernel).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

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
    // layered programs (all passes register-staged): probes of the reverse
    // sweep, and for each parameter j < nparams the probes that feed it,
    // probe_idx[probe_row[row_off + j] .. probe_row[row_off + j + 1])
    int32_t layered, nprobes, nparams, row_off;
};

// Tile widths layered circuits may run with (256 threads, 2^(m - 8)
// amplitudes per thread in registers), and the default: 2^11 amplitudes in
// both precisions (measured on the 4096-circuit mix in complex64: 356 ms
// against 391 ms with 2^12 tiles, whose reverse kernel holds two waves per
// SIMD instead of four).
inline bool batch_layer_width_ok(int dtype, int m) { return m == 11 || (m == 12 && dtype == QSIM_C64); }
inline int batch_layer_default(int) { return 11; }

struct BatchPass {
    int32_t L, H;
    int32_t hpos[16];
    int32_t op_begin, op_end;   // LDS form: TileOps
    // register-staged form (reg_r > 0): stages [stage_begin, stage_end) of
    // the batch's stage table, whose op ranges index its RegOp table; global
    // qubit of each thread / register bit at the load and at the store
    int32_t reg_r, stage_begin, stage_end;
    int32_t ld_t[8], ld_r[kRegBitsMax], st_t[8], st_r[kRegBitsMax];
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
    const RegStage *stages;
    const RegOp *rops;
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

// ------------------------------------------------------------ layered circuits
//
// Circuits whose programs are register-staged throughout run as layers: one
// launch applies pass s of every such circuit to all of its tiles at once
// (one workgroup per tile), so a large circuit spreads over the whole device
// and small and large ones share each launch.  Each circuit keeps psi and
// lambda in a slot of its own.  Probes leave one partial per (probe, tile)
// and the energy one per chunk of amplitudes; fixed-order reductions turn
// them into the gradient and the energies.

struct BatchLCirc {
    int32_t circ;            // index in the batch (its energy)
    int32_t prog;
    int32_t ntiles;          // tiles of a pass (2^(n - m))
    int32_t nchunks;         // energy chunks (2^n / kBatchChunk, at least 1)
    int64_t param_off;       // its parameters and gradient entries
    int32_t nparams;         // the circuit's parameter count
    int32_t pad_;
    int64_t gfirst;          // first gradient wave (prefix of nparams)
    uint64_t psi_off, lam_off;   // slots in the arena (amplitudes)
    uint64_t pp_off;         // probe partials, [probe][tile]
    uint64_t ep_off;         // energy partials, [chunk]
};

// One circuit's share of a launch: workgroups [first, first + count) take
// its tiles (or chunks) in order.
struct BatchWork {
    int32_t lc;              // layered circuit
    int32_t pass;            // global pass index (-1: energy)
    uint32_t first, count;
};

constexpr int kBatchChunk = 4096;   // amplitudes per energy workgroup

struct BatchStep {
    // 0 forward layer (init: the first), 1 reverse layer, 2 energies,
    // 3 gradient reduction; each over the layered circuits [lc_begin, lc_end)
    int kind;
    int init;
    int wbegin, wend;        // works
    uint32_t wgs;            // workgroups of the launch
    int lc_begin, lc_end;
    int64_t gw_begin, gw_end;   // gradient waves (kind 3)
};

struct BatchLayerDevice {
    void *lam_arena;         // base of lambda slots (null: the arena)
    const BatchLCirc *lc;
    int nlc;
    const BatchWork *works;
    const BatchProgram *progs;
    const BatchPass *passes;
    const RegStage *stages;
    const RegOp *rops;
    const void *pool;
    const BatchHGroup *hgroups;
    const BatchHTerm *hterms;
    const int32_t *probe_row, *probe_idx;
    const double *params;
    double *trig;            // lifting form (P, s, c, 0) of each parameter's rotation
    int64_t nparams;
    double *energies, *grads;
    void *arena;
    double *ppart, *epart;
    int want_grad;
    int R;                   // register bits per thread (tile width - 8)
    std::vector<BatchStep> steps;
};

// Host tables of batch programs (appended to by add_batch_program).
struct BatchTables {
    std::vector<BatchProgram> progs;
    std::vector<BatchPass> passes;
    std::vector<TileOp> ops;
    std::vector<RegStage> stages;
    std::vector<RegOp> rops;
    std::vector<cd> pool;
    std::vector<BatchHGroup> hgroups;
    std::vector<BatchHTerm> hterms;
    std::vector<int32_t> probe_row, probe_idx;
    int nonsingle_max_n = 0;
};

// Plans circuit c with observable H as one batch program and appends it to
// t: layered (register-staged passes, tiles of mL qubits) when c fills whole
// tiles and every pass can be staged, else for the persistent kernel, unless
// layered_only (then *is_layered is false and nothing is appended).
qsim_status add_batch_program(BatchTables &t, const qsim_circuit &c, const qsim_pauli_sum &H, int dtype, int mL,
                              int fuse_k, bool layered_only, bool *is_layered);

// One circuit's adjoint gradient run layered (qsim_adjoint_grad on states of
// 2^11 amplitudes and more): its tables packed for one upload, the launch
// description, and the per-call scratch it needs (rotation table, probe and
// energy partials).
struct LayeredAdjoint {
    std::vector<char> host;
    size_t o_progs = 0, o_passes = 0, o_stages = 0, o_rops = 0, o_pool = 0, o_hg = 0, o_ht = 0, o_lc = 0,
           o_works = 0, o_prow = 0, o_pidx = 0;
    size_t o_trig = 0, o_ppart = 0, o_epart = 0, scratch_bytes = 0;   // offsets in the call's scratch
    double pass_bytes = 0;
    BatchLayerDevice ld{};
};

// Plans the layered adjoint of c (nparams parameters, observable H) on an
// n-qubit state; *ok is false when some pass cannot be register-staged (the
// caller then takes the LDS path).
qsim_status plan_layered_adjoint(const qsim_circuit *c, int64_t nparams, const qsim_pauli_sum *H, int dtype,
                                 LayeredAdjoint &out, bool *ok);
// Points la.ld at the uploaded tables (dev), the state (psi), the second
// state (lam), the call's scratch and the caller's parameters and outputs.
void bind_layered_adjoint(LayeredAdjoint &la, void *dev, void *psi, void *lam, void *scratch,
                          const double *params_dev, double *energy_dev, double *grad_dev);

struct LayeredAdjointPlan {
    std::string key;
    bool ok = false;              // false: some pass cannot be staged (the LDS path runs it)
    LayeredAdjoint la;
    void *dev = nullptr;          // the uploaded tables
    hipStream_t dev_stream = nullptr;
    uint64_t last_use = 0;
    ~LayeredAdjointPlan() {
        if (dev) (void)hipFreeAsync(dev, dev_stream);
    }
};

// Raises the layered kernels' LDS limits (before any capture).
hipError_t batch_layer_setup(int dtype, int R);
hipError_t launch_batch_layered(hipStream_t stream, int dtype, const BatchLayerDevice &d);

}  // namespace qsim
