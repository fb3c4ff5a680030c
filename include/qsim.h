/*
 * qsim -- state-vector (Schroedinger-type) quantum circuit simulation on one
 * AMD Instinct MI355X (gfx950).  Plain C ABI: plain pointers and sizes, no
 * C++ or PyTorch types.
 *
 * The problem (paper, Sec. I.A "Background"; Sec. II "Methods"): the state of
 * n qubits is a vector of 2^n complex amplitudes held all at once; every gate
 * of a circuit acts on it as a 2^n x 2^n matrix, so simulation is a chain of
 * matrix-vector products whose cost grows linearly with the number of gates.
 * A k-qubit gate is its 2^k x 2^k matrix applied to every group of 2^k
 * amplitudes whose indices agree outside the target bits.
 *
 * Conventions (the paper leaves them open):
 *   - amplitude index x = sum_q bit_q * 2^q: qubit q is bit q (little-endian);
 *   - for a gate on targets[0..k-1], targets[b] is bit b of the gate matrix's
 *     row/column index;
 *   - matrices are row-major, complex128 as interleaved (re, im) doubles;
 *   - state memory is 2^n interleaved complex numbers, complex64 (2 x float)
 *     or complex128 (2 x double), contiguous, at least 256-byte aligned.
 *
 * Errors: every call returns a qsim_status.  Arguments are validated before
 * any device work; on a validation error the state is left unchanged and
 * qsim_last_error() describes the problem.  A failed HIP call returns
 * QSIM_ERR_DEVICE and marks the state invalid; every later call on that state
 * except qsim_free returns QSIM_ERR_STATE.
 *
 * Streams and synchronisation: each state carries a HIP stream (the null
 * stream by default).  Gate, circuit and gradient calls (qsim_apply_gate,
 * qsim_apply_circuit, qsim_adjoint_grad) and qsim_batch_run are
 * stream-ordered and return without waiting for the device; calls that
 * deliver a value to host memory (qsim_copy_to_host, qsim_expectation)
 * synchronise the state's stream.
 *
 * Threads: calls on different states may run concurrently from different host
 * threads; calls on one state must be serialised by the caller.
 */
#ifndef QSIM_H
#define QSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QSIM_OK = 0,
    QSIM_ERR_ARG = -1,          /* invalid argument; nothing was done */
    QSIM_ERR_OOM = -2,          /* device memory could not be allocated */
    QSIM_ERR_DEVICE = -3,       /* a HIP call failed; the state is now invalid */
    QSIM_ERR_UNSUPPORTED = -4,  /* valid request the library does not support */
    QSIM_ERR_STATE = -5         /* the state handle is invalid */
} qsim_status;

typedef enum {
    QSIM_C64 = 1,   /* complex64: 8 bytes per amplitude */
    QSIM_C128 = 2   /* complex128: 16 bytes per amplitude */
} qsim_dtype;

/* Gate kinds.  Named gates follow the textbook / OpenQASM 2 definitions:
 *   H = [[1,1],[1,-1]]/sqrt2; X, Y, Z Pauli; S = diag(1,i); T = diag(1,e^{i pi/4});
 *   SDG, TDG their inverses; RX/RY/RZ(t) = exp(-i t P/2) for P = X/Y/Z;
 *   U3(t,p,l) = [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]];
 *   CX(control, target); CZ; CP(p) = diag(1,1,1,e^{ip}); SWAP;
 *   CCX(c1, c2, target); CCZ = diag(1,...,1,-1).
 * QSIM_GATE_MATRIX applies a dense 2^k x 2^k matrix from the circuit's pool;
 * it is not required to be unitary. */
typedef enum {
    QSIM_GATE_MATRIX = 0,
    QSIM_GATE_H, QSIM_GATE_X, QSIM_GATE_Y, QSIM_GATE_Z,
    QSIM_GATE_S, QSIM_GATE_SDG, QSIM_GATE_T, QSIM_GATE_TDG,
    QSIM_GATE_RX, QSIM_GATE_RY, QSIM_GATE_RZ, QSIM_GATE_U3,
    QSIM_GATE_CX, QSIM_GATE_CZ, QSIM_GATE_CP, QSIM_GATE_SWAP,
    QSIM_GATE_CCX, QSIM_GATE_CCZ,
    QSIM_GATE_COUNT_
} qsim_gate_kind;

#define QSIM_MAX_K 6           /* largest gate / fused block, in qubits */
#define QSIM_MAX_QUBITS_C64 35 /* 256 GiB of complex64 */
#define QSIM_MAX_QUBITS_C128 34

/* One circuit operation.  `k` must equal the gate's arity for named gates
 * and lie in [1, QSIM_MAX_K] for QSIM_GATE_MATRIX.  Parametric gates (RX, RY,
 * RZ, CP: one angle; U3: three) read their angles from params[param ...] when
 * param >= 0, otherwise from `angles`.  For QSIM_GATE_MATRIX, `mat_off` is the
 * offset, in complex entries, of the row-major 2^k x 2^k matrix in the
 * circuit's pool. */
typedef struct {
    int32_t kind;
    int32_t k;
    int32_t targets[QSIM_MAX_K];
    int32_t param;
    int32_t reserved_;
    double angles[3];
    int64_t mat_off;
} qsim_op;

typedef struct {
    int32_t n;             /* circuit width in qubits */
    int32_t nops;
    const qsim_op *ops;    /* host array of nops ops */
    const double *mats;    /* host complex128 pool (interleaved), may be NULL */
    int64_t nmats;         /* complex entries in mats */
} qsim_circuit;

/* H = sum_t coeff_t * P_t with P_t = i^{|x & z|} X^x Z^z: bit q of xmask
 * (zmask) puts an X (Z) on qubit q, both bits a Y. */
typedef struct {
    double coeff;
    uint64_t xmask;
    uint64_t zmask;
} qsim_pauli_term;

typedef struct {
    int32_t nterms;
    const qsim_pauli_term *terms;   /* host array */
} qsim_pauli_sum;

/* Execution options.  Zero-initialised options select automatic choices.
 *   fuse_k:  1 = no gate fusion; 2..6 = merge runs of gates into dense blocks
 *            on at most fuse_k qubits (products formed in double precision and
 *            rounded once); 0 = automatic.
 *   tile_m:  -1 = every gate / block is its own sweep over the state;
 *            m in [7, 13] (c64) / [7, 12] (c128) = group gates into passes
 *            that hold 2^m-amplitude tiles in LDS (larger m is clamped; a
 *            tile is widened when a gate needs more positions next to the
 *            low qubits every tile keeps: 5 or 6 (c64), 4 or 5 (c128), the
 *            planner takes whichever gives fewer passes); 0 = automatic.
 *   use_mfma: -1 never, 1 whenever a fused block has k >= 4, 0 automatic.
 *   split_1q: single-qubit unitaries in tile passes.  1 (and 0, automatic):
 *            each is written as g diag(1, b) O diag(1, a) with O a real
 *            rotation; O runs as three in-place multiply-adds per amplitude
 *            component and the phases travel, merged, to the next gate that
 *            does not commute with them.  -1: every gate is applied as its
 *            complex 2 x 2 matrix.  Both are exact up to rounding.
 *   deterministic: 1 = automatic choices never consult the autotuner's table
 *            (whose entries come from timing), so the passes, and with them
 *            the rounding of every result, depend on the inputs alone; every
 *            reduction already runs in a fixed order, so repeated calls give
 *            bitwise identical results.  0 = the table is used when present.
 *   checkpoints: qsim_adjoint_grad only.  0 = none: the reverse sweep
 *            recovers each earlier state by applying the inverse gates to
 *            the later one.  c in [1, 64] = the circuit is cut into c + 1
 *            runs of about equal gate counts; the forward sweep keeps a copy
 *            of the state at each cut (c extra state-sized device buffers,
 *            allocated on first use and kept with the state), and the
 *            reverse sweep restores the state from that copy when it gets
 *            there, so the rounding of the inverse gates accumulates over
 *            one run instead of the whole circuit.  Other calls ignore it. */
typedef struct {
    int32_t fuse_k;
    int32_t tile_m;
    int32_t use_mfma;
    int32_t split_1q;
    int32_t deterministic;
    int32_t checkpoints;
} qsim_options;

typedef struct qsim_state_s *qsim_state;

/* Allocates a state of n qubits on the current HIP device, owned by the
 * library, initialised to |0...0>.  1 <= n <= 35 (c64) or 34 (c128).
 * QSIM_ERR_OOM if the device memory cannot be allocated.
 * (paper, Sec. I.A: a Schroedinger-type simulator holds all 2^n amplitudes
 * at once; its memory doubles with every qubit.) */
qsim_status qsim_alloc(int n, qsim_dtype dtype, qsim_state *out);

/* Wraps caller-owned device memory (e.g. a PyTorch tensor) holding 2^n
 * amplitudes of `dtype`, 256-byte aligned, without copying or initialising
 * it.  `hip_stream` (a hipStream_t, may be NULL) becomes the state's stream.
 * The caller keeps ownership and must keep the memory alive until qsim_free.
 * (paper, Sec. I.A, Sec. II: the state vector the gates act on, here kept in
 * device memory between gates rather than moved per operation.) */
qsim_status qsim_wrap(void *dev_ptr, int n, qsim_dtype dtype, void *hip_stream, qsim_state *out);

/* Releases the handle and, for qsim_alloc'd states, the device memory (after
 * synchronising the state's stream).  NULL is accepted.  (Sec. I.A: the
 * state vector's lifetime.) */
qsim_status qsim_free(qsim_state s);

/* Makes `hip_stream` (a hipStream_t, may be NULL) the state's stream after
 * waiting for the work queued on the previous one.  (Sec. II: the chain of
 * matrix-vector products runs in order; the stream carries that order.) */
qsim_status qsim_set_stream(qsim_state s, void *hip_stream);

/* Reports the width, dtype and device address of a state (any out pointer
 * may be NULL).  (Sec. I.A: n qubits, 2^n amplitudes.) */
qsim_status qsim_state_info(qsim_state s, int *n, int *dtype, void **dev_ptr);

/* Sets the state to the basis state |index> (index < 2^n). Stream-ordered.
 * (Sec. III: circuits start from basis inputs, e.g. the multiplier's.) */
qsim_status qsim_set_basis(qsim_state s, uint64_t index);

/* Copies the whole state to / from host memory; `bytes` must equal
 * 2^n * bytes-per-amplitude.  Synchronous with respect to the host.
 * (Sec. III: host-device transfers, which the paper finds dominate small
 * circuits, happen only here.) */
qsim_status qsim_copy_to_host(qsim_state s, void *host, size_t bytes);
qsim_status qsim_copy_from_host(qsim_state s, const void *host, size_t bytes);

/* Applies the 2^k x 2^k complex128 row-major host matrix U on `targets`
 * (k in [1, QSIM_MAX_K], distinct qubits < n, any order).  The matrix is
 * copied before returning and rounded once to the state's precision.
 * (paper, Sec. I.A and Sec. II: one gate = one matrix-vector product.) */
qsim_status qsim_apply_gate(qsim_state s, const int *targets, int k, const double *U);

/* Applies a circuit's ops in order (paper, Sec. I.A: the state advanced by
 * each moment's matrix).  `params` (host array of `nparams` doubles; may be
 * NULL with nparams = 0 when no op is parametric) supplies parametric angles;
 * `opts` may be NULL (automatic).
 * The circuit width must equal the state's.  Every op is validated before any
 * device work.  Plans (fusion, pass grouping, uploaded matrices) are cached
 * per state for circuits with no parametric op. */
qsim_status qsim_apply_circuit(qsim_state s, const qsim_circuit *c, const double *params,
                               int64_t nparams, const qsim_options *opts);

/* Writes <psi|H|psi> (no renormalisation) to *out_host, accumulated in double
 * precision with a fixed-order reduction (bitwise reproducible run to run).
 * Synchronises the state's stream.  Qubit masks must lie below 2^n.
 * (Sec. I: expectation values of simulated circuits are what a variational
 * model is trained on; Sec. III evaluates circuits through the simulator's
 * Python interface for that use.) */
qsim_status qsim_expectation(qsim_state s, const qsim_pauli_sum *H, double *out_host);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * value as qsim_expectation, from the same kernels in the same order (so
 * bitwise equal to it), with the partial sums, the uploaded term table and the
 * result in a fixed device array of QSIM_NOALLOC_SCRATCH_BYTES that the
 * library defines once per GPU (held from the library's load until the
 * process ends) instead of memory allocated per state.  The call allocates no
 * device memory and no pinned host memory; the terms are copied from host
 * memory in stream order.  A Pauli sum whose partial sums and terms need more
 * than the array (up to 16 KiB per pass over the state, 32 bytes per term)
 * returns QSIM_ERR_ARG before any device work.  Synchronises the state's
 * stream.  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (other streams or other host threads) race and must be
 * serialised by the caller. */
#define QSIM_NOALLOC_SCRATCH_BYTES (4u << 20)
qsim_status qsim_expectation_noalloc(qsim_state s, const qsim_pauli_sum *H, double *out_host);

/* Energy and gradient of a variational circuit by the adjoint method.
 *
 * E(theta) = <psi_L|H|psi_L> with psi_L = C(theta) psi_0, where psi_0 is the
 * state's content on entry.  Runs the circuit forward, forms
 * lambda = H psi_L, then sweeps the ops from last to first: for an op
 * exp(-i theta_j G / 2) (RX, RY or RZ with param >= 0) it adds
 * Im <lambda|G|psi> to dE/dtheta_j (the product rule over repeated use of
 * theta_j), and applies the op's inverse to both psi and lambda.  This
 * differentiation is not in the paper, whose motivating use is training
 * variational models with simulated expectation values (Sec. I).
 *
 * params_dev: device memory, nparams doubles; energy_dev: device memory, one
 * double; grad_dev: device memory, nparams doubles (overwritten; entries no op
 * uses are 0).  All on the state's device.  Stream-ordered: the call queues
 * its work on the state's stream and returns without waiting (the caller
 * orders reads of energy_dev / grad_dev after it on that stream).  Plans
 * depend on the circuit's structure only (the rotations read their angles
 * from params_dev on the device), so repeated calls with new parameters do
 * no planning.  opts: tile_m > 0 sets the forward tile width; other fields
 * are ignored.  Parametric ops of other kinds return QSIM_ERR_UNSUPPORTED and
 * pointers that are not device memory QSIM_ERR_ARG, before any device work.
 * On return the state holds psi_0 again, up to rounding.  Uses one extra
 * state-sized device buffer per state (allocated on first use, kept until
 * qsim_free). */
qsim_status qsim_adjoint_grad(qsim_state s, const qsim_circuit *c, const double *params_dev, int64_t nparams,
                              const qsim_pauli_sum *H, const qsim_options *opts, double *energy_dev,
                              double *grad_dev);

/* Batched forward + adjoint runs of many independent circuits, for callers
 * that evaluate thousands of small variational circuits (paper, Sec. I: the
 * parameters of a model are adapted from simulated outputs; Sec. III: small
 * circuits lose to host-device overhead).
 *
 * qsim_batch_create validates every circuit (1 <= n <= 26; parametric ops
 * must be RX, RY or RZ), builds one device program per distinct structure
 * (circuit ops, fixed angles and matrices, observable), allocates device
 * memory and captures the whole run in a HIP graph.  Circuits that fill
 * whole tiles (n >= 11 by default) and whose ops all fit
 * register-staged passes run layered: one launch per pass index applies
 * that pass of every such circuit to all of its tiles at once, each circuit
 * with psi/lambda slots of its own (2 x 2^n amplitudes, in groups that fit
 * half the free device memory).  The others run in a persistent kernel, one
 * workgroup per circuit from LDS (a psi/lambda slot per workgroup for
 * circuits wider than one tile).  Circuit i reads its parameters from params[param_offsets[i]
 * .. param_offsets[i+1]) (param indices in its ops are relative to that
 * block), is applied to |0...0>, and yields energies[i] = <psi|Hs[i]|psi>
 * and, when want_grad, grads over the same block.  `opts` (may be NULL):
 * fuse_k 0 or 1 = no fusion, 2 or 3 = runs of fixed (non-parametric) gates
 * merged into dense blocks of at most that many qubits; tile_m 0 =
 * automatic, 11 or 12 (complex64) / 11 (complex128) = tile width of the
 * layered circuits; the other fields are ignored.
 *
 * qsim_batch_run: params_dev (device, nparams doubles), energies_dev (device,
 * ncirc doubles) and grads_dev (device, nparams doubles; may be NULL when the
 * batch was created without gradients).  Stream-ordered on `hip_stream`: a
 * device-to-device copy of the parameters in, the graph, copies of the
 * results out; returns without waiting.  Calls on one batch must be
 * serialised on one stream.  qsim_batch_info reports the persistent grid
 * size, the number of distinct programs and the widest circuit;
 * qsim_batch_layout how many circuits run layered and how many in the
 * persistent kernel, and the device-memory bytes one run's layered passes
 * read and write (every tile in and out once per pass: psi in forward
 * passes, psi and lambda in reverse passes, plus psi read and lambda written
 * for the energies; any pointer may be NULL); qsim_batch_free waits for the
 * batch's work and releases it. */
typedef struct qsim_batch_s *qsim_batch;

qsim_status qsim_batch_create(int ncirc, const qsim_circuit *circs, const int64_t *param_offsets,
                              const qsim_pauli_sum *Hs, qsim_dtype dtype, int want_grad, const qsim_options *opts,
                              qsim_batch *out);
qsim_status qsim_batch_run(qsim_batch b, const double *params_dev, double *energies_dev, double *grads_dev,
                           void *hip_stream);
qsim_status qsim_batch_info(qsim_batch b, int *grid, int *programs, int *max_n);
qsim_status qsim_batch_layout(qsim_batch b, int *layered, int *persistent, double *pass_bytes);

/* Batch autotuner (Sec. IV leaves tuning to future work): creates the batch
 * with each candidate option set (layered tile width 11 and 12 for
 * complex64, 11 for complex128; fixed-gate fusion 1, 2 and 3), replays it
 * once to warm up and `reps` times timed with HIP events on a stream of its
 * own, releases it, and writes the fastest set to *best and its mean time
 * per run in milliseconds to *best_ms (may be NULL).  Arguments as for
 * qsim_batch_create; params_dev as for qsim_batch_run.  Allocates and frees
 * each candidate's device memory in turn; synchronises. */
qsim_status qsim_batch_autotune(int ncirc, const qsim_circuit *circs, const int64_t *param_offsets,
                                const qsim_pauli_sum *Hs, qsim_dtype dtype, int want_grad, const double *params_dev,
                                int reps, qsim_options *best, double *best_ms);
qsim_status qsim_batch_free(qsim_batch b);

/* Autotuner (Sec. IV: the paper leaves kernel-level tuning to future work):
 * applies the circuit with each candidate option set (plain
 * sweeps; LDS tile passes of three tile sizes with fusion widths 1..3;
 * matrix-core blocks of 4..6 qubits), once to warm up and `reps` times timed
 * with HIP events, and writes the fastest set to *best and its mean time per
 * application to *best_ms (may be NULL).  The state's content is overwritten
 * (the circuit runs (reps + 1) times per candidate).  The choice is stored
 * per circuit structure (ops and matrices; parameter values excluded), width
 * and dtype in a process-wide table, appended to the file named by the
 * environment variable QSIM_TUNE_CACHE when set (and read from it on first
 * use); qsim_apply_circuit and qsim_adjoint_grad use it whenever their
 * options are NULL or all zero. */
qsim_status qsim_autotune(qsim_state s, const qsim_circuit *c, const double *params, int64_t nparams, int reps,
                          qsim_options *best, double *best_ms);

/* Plans a circuit for an n-qubit state of `dtype` without touching any
 * device (host-only; Sec. II: the cost of a circuit is its chain of
 * matrix-vector products, reported here pass by pass): validates the ops as
 * qsim_apply_circuit does and
 * reports how many passes of each kind (QSIM_KCLASS_*, `counts` has
 * QSIM_KCLASS_COUNT_ entries) the circuit would take, the algorithmic HBM
 * bytes they move and the floating-point operations their gate arithmetic
 * takes (8 * 2^k per amplitude a dense k-qubit gate changes, 6 per amplitude
 * a diagonal entry other than 1 multiplies).  Any out pointer may be NULL. */
qsim_status qsim_plan_summary(int n, qsim_dtype dtype, const qsim_circuit *c, const double *params,
                              int64_t nparams, const qsim_options *opts, int64_t *counts, double *bytes,
                              double *flops);

/* Thread-local description of the last error on this thread ("" if none).
 * (Not a step of the method: error reporting of this interface.) */
const char *qsim_last_error(void);

/* Per-kernel-class timing of this library's launches on a state (Sec. III:
 * the paper measures wall-clock time per circuit; these events break it down
 * by kernel), measured
 * with HIP events recorded on the state's stream around every launch while
 * enabled.  qsim_profile_enable(s, 1) clears and starts; 0 stops.
 * qsim_profile_read synchronises the stream and reports, for class `cls`
 * (QSIM_KCLASS_*), the number of launches, their summed duration in
 * milliseconds, the summed algorithmic bytes they move and the summed
 * floating-point operations of their gate arithmetic (as qsim_plan_summary). */
typedef enum {
    QSIM_KCLASS_SWEEP_DENSE = 0,  /* dense / controlled gate sweeps over HBM */
    QSIM_KCLASS_SWEEP_DIAG = 1,   /* diagonal-gate sweeps */
    QSIM_KCLASS_TILE = 2,         /* LDS tile passes */
    QSIM_KCLASS_MFMA = 3,         /* MFMA fused-block passes */
    QSIM_KCLASS_EXPECT = 4,       /* expectation passes (and lambda = H psi) */
    QSIM_KCLASS_ADJOINT = 5,      /* reverse tile passes of the adjoint method */
    QSIM_KCLASS_TILE_JIT = 6,     /* register tile passes compiled at run time */
    QSIM_KCLASS_COUNT_ = 7
} qsim_kernel_class;

qsim_status qsim_profile_enable(qsim_state s, int on);
qsim_status qsim_profile_read(qsim_state s, int cls, int64_t *launches, double *ms, double *bytes,
                              double *flops);

#ifdef __cplusplus
}
#endif

#endif /* QSIM_H */
