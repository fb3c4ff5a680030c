// Internal declarations of the qsim HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/qsim.h"

namespace qsim {

using cd = std::complex<double>;

// ------------------------------------------------------------ errors

struct Error {
    qsim_status status;
    std::string msg;
};

qsim_status set_error(qsim_status st, const std::string &msg);
void clear_error();

// ------------------------------------------------------------ host gate model

// A gate in normalised form: a 2^k x 2^k row-major matrix on `targets`
// (targets[b] is bit b of the matrix index).
struct HostGate {
    int k = 0;
    int targets[QSIM_MAX_K] = {0, 0, 0, 0, 0, 0};
    std::vector<cd> M;
    int src_op = -1;   // index of the circuit op it came from (-1 for fused blocks)
    // adjoint probes: Im <lambda|G|psi> with G = X (1), Y (2), Z (3) on
    // targets[0]; no matrix, does not change either state
    int probe_gen = 0;
    int probe_slot = -1;
    // batch programs: a rotation exp(-i theta G / 2) on targets[0] whose
    // matrix is formed on the device from parameter rot_param (G = X, Y, Z for
    // rot_gen 1, 2, 3; rot_inv applies the inverse)
    int rot_gen = 0;
    int rot_param = -1;
    int rot_inv = 0;
    // split single-qubit unitary (forward tile plans): the gate is
    // O diag(1, phase_in) with O = [[c, -s], [s, c]], c, s >= 0; M holds that
    // product for paths that apply it as a plain matrix.  rot_real 1: O by
    // lifting steps, 2: c == 0 (O exchanges the pair with one sign change)
    int rot_real = 0;
    double rot_c = 1.0, rot_s = 0.0;
    cd phase_in = 1.0;
};

// Validates op i of a circuit and returns its normalised gate (matrix built
// from the op's angles or parameters).
qsim_status make_gate(const qsim_circuit *c, int i, const double *params, int64_t nparams, HostGate &g);

// Rewrites a gate list for tile passes: every single-qubit unitary U
// becomes g diag(1, b) O diag(1, a) (O real); diag(1, b) is carried forward
// over gates that commute with it and merged into the next split gate's
// input phase, or emitted as a diagonal gate before the first gate that
// does not commute with it; the global factor is folded into a final
// diagonal gate.  Non-unitary or diagonal gates pass through unchanged.
std::vector<HostGate> split_single_qubit(const std::vector<HostGate> &gates, int n);

// Builds the matrix of a named gate; returns its arity, or -1 for an unknown kind.
int named_gate_matrix(int kind, const double *angles, cd *U);
int named_gate_arity(int kind);

// True when every off-diagonal entry of M is exactly zero.
bool is_diagonal(const HostGate &g);

// Splits a gate into exact controls (bits on which it acts as the identity
// unless the bit is 1) and the reduced gate on the remaining targets.
// Returns the number of controls written to `controls` (global qubit ids).
int extract_controls(const HostGate &g, HostGate &reduced, int *controls);

// Re-expresses a gate with its targets sorted ascending (matrix permuted).
HostGate sorted_targets(const HostGate &g);

// Product B * A of two gates as one gate on the union of their qubits
// (A applied first), formed in double precision.
HostGate fuse_pair(const HostGate &first, const HostGate &second);

// ------------------------------------------------------------ plan

enum PassKind : int { PASS_DENSE = 0, PASS_DIAG = 1, PASS_TILE = 2, PASS_MFMA = 3 };

// Device-side op of a tile pass.
//   dense (type 0): 2^k x 2^k matrix on tile-local positions pos[0..k-1]
//     (ascending; matrix index bit b <-> pos[b]);
//   diagonal (type 1): 2^k entries; kin targets lie inside the tile at local
//     positions pos[0..kin-1] (ascending) and give bit jbit[i] of the
//     diagonal index; the other k - kin lie outside, at global positions
//     gpos[i], giving bit gbit[i] (constant across a tile).
struct TileOp {
    // 0 dense on pos[0..k-1], 1 diagonal (in-tile pos / out-of-tile gpos
    // bits), 3 adjoint probe, 4 device-formed rotation (batch), 5 one-qubit
    // block on pos[0] where the in-tile control positions of mask kin are 1
    int32_t type;
    int32_t k;
    int32_t kin;
    int32_t moff;      // offset of the matrix / diagonal in the pass pool (complex entries)
    int32_t pos[QSIM_MAX_K];
    int32_t jbit[QSIM_MAX_K];
    int32_t gpos[QSIM_MAX_K];
    int32_t gbit[QSIM_MAX_K];
};

// Register-staged tile passes.  A thread holds 2^r amplitudes of a 2^m tile
// in registers (r = m - 8, 256 threads).  A stage fixes which r tile-local
// positions are register bits (R) and which 8 are thread bits (T); dense ops
// of the stage act on register bits only, diagonal ops anywhere.  Between
// stages the tile is exchanged through LDS with an XOR-swizzled address map.
constexpr int kRegBitsMax = 5;

struct RegOp {
    // 0 dense in registers, 1 diagonal (table), 2 diagonal with one non-unit
    // entry, 3 real rotation on one register bit by lifting (pool entry
    // (p, u)), 4 phase table over the register bits (2^r pool entries),
    // 5 signed exchange on one register bit (x0, x1) <- (-x1, x0), 6 one
    // factor (pool entry moff) on the amplitudes whose target bits are all
    // 1: register bits rmask, thread bits tb[0] (a mask of thread-id bits),
    // out-of-tile qubits gp[0] | gp[1] << 32 (a mask of global qubits),
    // 7 one-qubit block on register bit rb[0] under controls (masks as in 6),
    // 8 batched rotation exp(-i theta G / 2), theta the circuit's parameter
    // moff, G = X, Y, Z for rj[0] = 1, 2, 3, inverse when jmatch is 1,
    // 9 batched probe Im <lambda|G|psi> into gradient slot moff (G as in 8),
    // 10 that probe followed by the inverse rotation of parameter moff,
    // 11 two rotations on register bit rb[0]: G = rj[0] (X or Y) of
    // parameter moff, then G = rj[1] of parameter gj[0]; 12 two ops of
    // type 10 on register bit rb[0] (G = rj[0], parameter moff, then
    // G = rj[1], parameter gj[0]; probes jmatch and jmatch + 1);
    // X and Y act on register bit rb[0], Z on the bit that rmask, tb[0] or
    // gp[0..1] names
    int32_t type;
    int32_t code;     // kernel dispatch code (set from the fields below by op_code)
    int32_t k;
    int32_t rmask;    // dense: register bits of the targets (ascending = matrix bit order)
    int32_t moff;     // pool offset of the matrix / diagonal (complex entries)
    int32_t nreg, nthr, nout;
    int32_t jmatch;   // type 2: index of the non-unit diagonal entry; type 7: 1 when the block is X
    // (32-bit fields throughout: the kernel reads them with scalar loads)
    int32_t rb[QSIM_MAX_K], rj[QSIM_MAX_K];   // targets in register bits: bit, diagonal-index bit
    int32_t tb[QSIM_MAX_K], tj[QSIM_MAX_K];   // targets in thread bits
    int32_t gp[QSIM_MAX_K], gj[QSIM_MAX_K];   // targets outside the tile: global qubit
};

struct RegStage {
    int32_t op_begin, op_end;   // RegOps of this stage, relative to the pass's first
    // exchange into this stage (stage 0 is loaded from HBM instead): LDS
    // address, in amplitudes, contributed by each thread / register bit of
    // the previous layout (write) and of this stage's layout (read)
    uint32_t wr_t[8], wr_r[kRegBitsMax], rd_t[8], rd_r[kRegBitsMax];
    // global qubit on each thread / register bit of this stage's layout
    int8_t q_t[8], q_r[kRegBitsMax];
    int8_t pad_[3];
};

struct Pass {
    PassKind kind;
    // sweep passes
    int k = 0;                        // targets of the (reduced) gate
    int targets[QSIM_MAX_K] = {};     // ascending
    int nctrl = 0;
    int ctrls[QSIM_MAX_K] = {};
    std::vector<cd> M;                // dense: 2^k x 2^k on sorted targets; diag: 2^k entries
    // tile passes
    int m = 0;                        // tile qubits
    int L = 0;                        // low qubits always in the tile
    std::vector<int> hpos;            // global positions of the other m - L tile qubits, ascending
    int op_begin = 0, op_end = 0;     // range in Plan::tile_ops
    int pool_begin = 0, pool_end = 0; // range in Plan::tile_pool
    // register-staged form (used when reg_r > 0)
    int reg_r = 0;
    int rop_begin = 0, rop_end = 0;   // range in Plan::reg_ops
    int stage_begin = 0, stage_end = 0;
    int8_t ld_t[8] = {}, ld_r[kRegBitsMax] = {};   // global qubit of each thread / register bit (load)
    int8_t st_t[8] = {}, st_r[kRegBitsMax] = {};   // (store)
    // accounting
    int logical_gates = 0;
    double bytes = 0;                 // algorithmic HBM bytes
    double flops = 0;                 // algorithmic floating-point operations
};

struct Plan {
    int n = 0;
    int dtype = 0;
    std::vector<Pass> passes;
    int items = 0;                    // gates handed to the pass grouping
    std::vector<TileOp> tile_ops;
    std::vector<cd> tile_pool;        // matrices / diagonals of tile ops
    std::vector<RegOp> reg_ops;
    std::vector<RegStage> reg_stages;
    size_t reg_ops_dev_off = 0, reg_stages_dev_off = 0;
    std::vector<double> real_pool;    // real-embedded block matrices of MFMA passes
    size_t real_pool_dev_off = 0;
    // device copies (tile ops + pool rounded to the state precision)
    // `dev` comes from the stream-ordered allocator on `dev_stream` (the
    // owning state's stream; the state updates it when its stream changes) and
    // is released on that stream, behind every kernel queued there that reads
    // it, so dropping a plan never waits for the device
    void *dev = nullptr;
    hipStream_t dev_stream = nullptr;
    size_t dev_bytes = 0;
    size_t pool_dev_off = 0;          // byte offset of the pool inside dev
    bool uploaded = false;
    // run-time compiled kernels of register-staged passes (null: interpreted)
    std::vector<hipFunction_t> jit_fn;
    int jit_map_shift = 0;            // occupancy-map chunk width of the compiled passes (0: none)
    ~Plan();
};

// Run-time compiled register tiles, for circuits without parametric ops.
// QSIM_JIT=0 turns them off, =1 makes a failed compilation an error
// (default: used from QSIM_JIT_MIN_QUBITS = 18 qubits on, and a failed
// compilation leaves the passes interpreted).
int jit_mode();
bool jit_wanted(int n);
// HIP source of the compiled passes; `flops` receives each one's arithmetic
std::string jit_source(const Plan &plan, std::vector<int> &which, std::vector<double> *flops = nullptr);
qsim_status jit_prepare(qsim_state s, Plan &plan, std::string &err);
// Occupancy maps of compiled passes on sparse states: the chunk width (one
// byte per 2^shift amplitudes, three maps in rotation), or 0 for none.
int jit_map_shift(const Plan &plan);
// `maps`: 3 x 2^(n - shift) bytes of device memory when the plan keeps maps.
hipError_t launch_jit_pass(qsim_state s, const Plan &plan, const Pass &p, hipFunction_t fn, void *maps);
hipError_t launch_fill_zero(qsim_state s, void *dst, size_t bytes);

struct PlanOptions {
    int fuse_k = 1;
    int tile_m = -1;
    int use_mfma = -1;
    bool reg_tiles = true;   // register-staged tile passes where eligible
    bool split_1q = true;    // split single-qubit unitaries in tile passes
};

PlanOptions resolve_options(const qsim_options *o, int n, int dtype);

// Options the autotuner chose for this circuit structure (ops and matrices,
// not parameter values) on n qubits of `dtype`, if it has run for it.
bool tuned_options(const qsim_circuit *c, int n, int dtype, qsim_options *out);
void remember_tuning(const qsim_circuit *c, int n, int dtype, const qsim_options &o);

// Builds passes from normalised gates.  Tile passes are widened when a gate
// would not fit next to the low qubits of a 2^tile_m tile.  Returns false if
// a gate could not be placed (nothing of the plan may then be run).
bool build_plan(Plan &plan, const std::vector<HostGate> &gates, const PlanOptions &po);

// Reverse-sweep plan of the adjoint method: tile passes over (psi, lambda)
// holding, for each op from last to first, its probe (if parametric) and its
// inverse.  Returns the tile width used (tile_m, or more when a gate needs
// it), or -1 if a gate could not be placed.
int build_adjoint_plan(Plan &plan, const std::vector<HostGate> &items, int tile_m);

// LDS-resident tile passes (no register staging) over the given ops; returns
// the tile width used, or -1 as build_adjoint_plan.
// `tiles`: state tiles each pass keeps in LDS next to its ops and matrices.
int build_tile_plan(Plan &plan, const std::vector<HostGate> &items, int tile_m, int tiles = 1, bool reg = false);

// Fusion: greedy merge into blocks of at most fuse_k qubits.
std::vector<HostGate> fuse_gates(const std::vector<HostGate> &gates, int fuse_k);

// ------------------------------------------------------------ state

struct Profile {
    bool on = false;
    struct Rec {
        int cls;
        hipEvent_t a, b;
        double bytes, flops;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

struct CachedPlan {
    std::string key;
    std::unique_ptr<Plan> plan;
    uint64_t last_use = 0;
};

// Plans of the adjoint method for one circuit structure: forward and reverse
// tile passes whose parametric rotations take (cos, sin) of their half angle
// from a device table, and the probes of each parameter (device, CSR:
// int32 row[nparams + 1] at offset 0, int32 idx[nprobes] at idx_off).
struct AdjointPlan {
    std::string key;
    Plan fwd, rev;
    int mtile = 0;        // reverse tile width
    int nprobes = 0;
    // forward-state checkpoints: the forward copies the state after pass
    // fwd_cut[j] - 1 into checkpoint j; the reverse restores checkpoint j
    // after pass rev_cut[j] - 1 (reverse runs end there, last run first)
    int nck = 0;
    std::vector<int> fwd_cut, rev_cut, rev_ck;
    int64_t nparams = 0;
    void *dev = nullptr;
    size_t idx_off = 0;
    hipStream_t dev_stream = nullptr;
    uint64_t last_use = 0;
    ~AdjointPlan() {
        if (dev) (void)hipFreeAsync(dev, dev_stream);
    }
};

// The adjoint of one circuit structure and observable run layered
// (register-staged passes; defined with the batch tables).
struct LayeredAdjointPlan;

}  // namespace qsim

struct qsim_state_s {
    int n = 0;
    int dtype = 0;
    void *data = nullptr;
    bool owned = false;
    bool valid = true;
    int device = 0;
    hipStream_t stream = nullptr;
    // scratch for reductions and per-call uploads
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t pinned_ev = nullptr;   // last upload from `pinned`
    bool pinned_ev_pending = false;
    qsim::Profile prof;
    std::vector<qsim::CachedPlan> plans;
    std::unique_ptr<qsim::Plan> transient;   // last uncached plan (single gates)
    void *adj_lam = nullptr;                 // second state of the adjoint method
    void *adj_ck = nullptr;                  // forward-state checkpoints of the adjoint method
    int adj_ck_count = 0;
    std::vector<std::unique_ptr<qsim::AdjointPlan>> adj_plans;
    std::vector<std::unique_ptr<qsim::LayeredAdjointPlan>> adj_lplans;
    void *adj_h = nullptr;                   // the adjoint's Pauli sum on the device
    size_t adj_h_bytes = 0;
    std::string adj_h_key;                   // ... and the terms it was written from
    uint64_t use_clock = 0;
};

namespace qsim {

size_t amp_bytes(int dtype);

// Launchers (kernels_*.hip).  All return hipSuccess or the launch error.
// Whether a sweep pass runs as a lane-exchange kernel (complex64, one to
// three targets, no controls).
bool lane_sweep_ok(int dtype, int n, const Pass &p);
hipError_t launch_dense_sweep(qsim_state s, const Pass &p);
hipError_t launch_diag_sweep(qsim_state s, const Pass &p);
// trig: (cos, sin) of each parameter's half angle, for passes with
// device-parameter rotations (TileOp type 4); may be NULL otherwise.
hipError_t launch_tile_pass(qsim_state s, const Plan &plan, const Pass &p, const double *trig = nullptr);
hipError_t launch_tile_reg_pass(qsim_state s, const Plan &plan, const Pass &p);
hipError_t launch_mfma_pass(qsim_state s, const Plan &plan, const Pass &p);
hipError_t launch_set_basis(qsim_state s, uint64_t index);

// Expectation: writes partial sums to `partials` (double) and returns the
// number written; the final reduction runs in launch_reduce.
hipError_t launch_expect_group(qsim_state s, uint64_t xmask, const void *dev_terms, int nterms,
                               double *partials, int *nwritten);
hipError_t launch_reduce(qsim_state s, const double *partials, int count, double *out);

// <psi|H|psi> with the state's scratch (fixed_dev NULL) or a caller's fixed
// device buffer of fixed_bytes (no allocation).
qsim_status expectation_with(qsim_state s, const qsim_pauli_sum *H, double *out_host, void *fixed_dev,
                             size_t fixed_bytes);

// Several term groups in one pass over the state: tiles of 2^m amplitudes
// (the low L qubits and the H qubits hpos[]) in LDS, every group whose X mask
// lies inside the tile evaluated from there.  Terms carry, in their pad
// field, the local image of their Z mask.  Writes ngroups * grid partials
// (group-major) and returns the count.
constexpr int kExpTileGroups = 64;
// A group is "simple" when its X mask is one qubit h and every term's Z mask
// is 0 (X_h, weight A = sum of their coefficients) or h itself (Y_h, weight
// B); the pair (y, y ^ x) then contributes 2 (A Re + B Im)(conj(psi_y)
// psi_{y^x}) from the member with y_h = 0.
constexpr uint32_t kExpGroupSimple = 1;
struct ExpTileGroup {
    uint32_t xl;          // X mask in tile-local bits
    int32_t first, count; // term range
    uint32_t flags;       // kExpGroupSimple
    double A, B;          // weights of a simple group
};
// The group with X mask 0 (at most one per sum) keeps its terms ordered by
// the register part of their local Z mask (local bits 8 and up for the
// register-staged kernel); dmu[mu] .. dmu[mu + 1] is the range with part mu.
struct ExpTilePass {
    int32_t m, L, H, ngroups;
    int32_t hpos[16];
    int32_t dmu[33];
    ExpTileGroup groups[kExpTileGroups];
};
hipError_t launch_expect_tiles(qsim_state s, const ExpTilePass &p, const void *dev_terms, double *partials,
                               int *nwritten);

// Sums whose X masks are all 0 or one qubit (the diagonal group and X_h / Y_h
// groups): passes of 64-lane wavefronts with 2^R amplitudes per lane in
// registers (R = kExpSimpleR) and no LDS.  Lane bit b is qubit
// lane_q[b] (the low 5 / 4 qubits first), register bit b qubit reg_q[b];
// tile_q lists the 6 + R tile qubits ascending.  Groups on register qubits
// pair registers (reg_bit, weights A of the X_h terms, B of the Y_h terms);
// groups on lane qubits exchange across lanes (lane_bit).  With diag set the
// pass also evaluates the diagonal group: terms diag_first .. diag_end - 1,
// ordered by the register part mu of their Z mask and then its lane part zl
// (each term's pad field holds mu | zl << 8); the terms with register part
// mu are diag_mu[mu] .. diag_mu[mu + 1] - 1.  Each launch writes one partial
// per workgroup.
constexpr int kExpSimpleMaxR = 6;
constexpr int kExpSimpleR = 4;
struct ExpSimplePass {
    int32_t R, ntile_q, nreg_g, nlane_g, diag;
    int32_t lane_q[6];
    int32_t reg_q[kExpSimpleMaxR];
    int32_t tile_q[6 + kExpSimpleMaxR];
    int32_t reg_bit[kExpSimpleMaxR], lane_bit[6];
    double reg_A[kExpSimpleMaxR], reg_B[kExpSimpleMaxR], lane_A[6], lane_B[6];
    int32_t diag_first, diag_end;
    int32_t diag_mu[(1 << kExpSimpleR) + 1];
};
int expect_simple_grid(uint64_t ntiles);
hipError_t launch_expect_simple(qsim_state s, const ExpSimplePass &p, const void *dev_terms, double *partials,
                                int *nwritten);
int expect_group_grid(uint64_t N);

// Adjoint differentiation.
int pauli_apply_grid(uint64_t N);
hipError_t launch_pauli_apply(qsim_state s, void *lam, const void *groups, int ngroups, const void *terms,
                              double *partials);
hipError_t launch_adjoint_pass(qsim_state s, const Plan &plan, const Pass &p, void *lam, double *probe_partials,
                               const double *trig);
hipError_t launch_half_angle_trig(qsim_state s, const double *params, int64_t n, double *trig);
hipError_t launch_gather_gradient(qsim_state s, const double *sums, const int32_t *row, const int32_t *idx,
                                  int64_t nparams, int nprobes, double *grad, double *energy);
hipError_t launch_reduce_rows(qsim_state s, const double *in, int rows, int cols, double *out);

// Profiling hooks around launches.
void prof_begin(qsim_state s, int cls, double bytes, double flops = 0.0);
void prof_end(qsim_state s);

}  // namespace qsim
