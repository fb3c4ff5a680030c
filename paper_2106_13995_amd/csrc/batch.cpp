// Host side of batched runs: validation, one program per distinct circuit
// structure (forward passes, reverse passes with probes, observable terms),
// largest-first work order, device buffers and the captured HIP graph that
// runs a whole batch as one replay.
#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>

#include "batch.h"
#include "qsim_internal.h"

namespace qsim {
qsim_status set_error(qsim_status st, const std::string &msg);
}

using namespace qsim;

struct qsim_batch_s {
    int dtype = 0;
    int ncirc = 0;
    int want_grad = 0;
    int64_t nparams = 0;
    int grid = 0;
    void *dev = nullptr;          // programs, circuits, params, outputs, counter
    size_t dev_bytes = 0;
    void *arena = nullptr;        // per-workgroup psi / lambda slots
    double *d_params = nullptr, *d_energy = nullptr, *d_grads = nullptr;   // inside dev
    hipStream_t last_stream = nullptr;   // stream of the last run
    bool ran = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int max_n = 0;
    int programs = 0;
};

namespace {

qsim_status fail(qsim_status st, const std::string &m) { return set_error(st, m); }

void destroy(qsim_batch b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->dev) (void)hipFree(b->dev);
    if (b->arena) (void)hipFree(b->arena);
    delete b;
}

int rotation_generator(int kind) {
    return kind == QSIM_GATE_RX ? 1 : kind == QSIM_GATE_RY ? 2 : kind == QSIM_GATE_RZ ? 3 : 0;
}

std::string structure_key(const qsim_circuit &c, const qsim_pauli_sum &H) {
    std::string k;
    auto put = [&k](const void *p, size_t n) { k.append(static_cast<const char *>(p), n); };
    put(&c.n, sizeof c.n);
    put(c.ops, sizeof(qsim_op) * size_t(c.nops));
    if (c.mats && c.nmats > 0) put(c.mats, sizeof(double) * 2 * size_t(c.nmats));
    put(H.terms, sizeof(qsim_pauli_term) * size_t(H.nterms));
    return k;
}

template <typename T>
void pack_pool(const std::vector<cd> &pool, char *dst) {
    T *p = reinterpret_cast<T *>(dst);
    for (size_t i = 0; i < pool.size(); ++i) {
        p[2 * i] = T(pool[i].real());
        p[2 * i + 1] = T(pool[i].imag());
    }
}

}  // namespace

extern "C" {

qsim_status qsim_batch_create(int ncirc, const qsim_circuit *circs, const int64_t *param_offsets,
                              const qsim_pauli_sum *Hs, qsim_dtype dtype, int want_grad, const qsim_options *opts,
                              qsim_batch *out) {
    (void)opts;
    if (!out) return fail(QSIM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (ncirc < 1 || !circs || !param_offsets || !Hs) return fail(QSIM_ERR_ARG, "empty batch or NULL array");
    if (dtype != QSIM_C64 && dtype != QSIM_C128) return fail(QSIM_ERR_ARG, "dtype must be QSIM_C64 or QSIM_C128");
    if (param_offsets[0] != 0) return fail(QSIM_ERR_ARG, "param_offsets[0] must be 0");
    const int nmax_batch = 26;
    std::map<std::string, int> prog_of;
    std::vector<const qsim_circuit *> prog_circ;
    std::vector<const qsim_pauli_sum *> prog_H;
    std::vector<int> circ_prog(static_cast<size_t>(ncirc));
    for (int i = 0; i < ncirc; ++i) {
        const qsim_circuit &c = circs[i];
        const int64_t np = param_offsets[i + 1] - param_offsets[i];
        const std::string where = "circuit " + std::to_string(i) + ": ";
        if (np < 0) return fail(QSIM_ERR_ARG, where + "param_offsets must not decrease");
        if (c.n < 1 || c.n > nmax_batch) return fail(QSIM_ERR_ARG, where + "n outside [1, 26]");
        if (c.nops < 0 || (c.nops > 0 && !c.ops)) return fail(QSIM_ERR_ARG, where + "bad op array");
        const qsim_pauli_sum &H = Hs[i];
        if (H.nterms < 0 || (H.nterms > 0 && !H.terms)) return fail(QSIM_ERR_ARG, where + "bad Pauli sum");
        const uint64_t lim = (1ull << c.n) - 1;
        for (int t = 0; t < H.nterms; ++t)
            if ((H.terms[t].xmask & ~lim) || (H.terms[t].zmask & ~lim))
                return fail(QSIM_ERR_ARG, where + "Pauli mask has a bit at or above n");
        std::vector<double> zeros(size_t(std::max<int64_t>(np, 1)), 0.0);
        for (int o = 0; o < c.nops; ++o) {
            HostGate g;
            qsim_status st = make_gate(&c, o, zeros.data(), np, g);
            if (st != QSIM_OK) return fail(st, where + qsim_last_error());
            if (c.ops[o].param >= 0 && !rotation_generator(c.ops[o].kind))
                return fail(QSIM_ERR_UNSUPPORTED, where + "parametric ops must be RX, RY or RZ");
        }
        const std::string key = structure_key(c, H);
        auto it = prog_of.find(key);
        if (it == prog_of.end()) {
            const int id = int(prog_circ.size());
            prog_of.emplace(key, id);
            prog_circ.push_back(&c);
            prog_H.push_back(&H);
            circ_prog[size_t(i)] = id;
        } else {
            circ_prog[size_t(i)] = it->second;
        }
    }
    qsim_batch b = new (std::nothrow) qsim_batch_s();
    if (!b) return fail(QSIM_ERR_OOM, "host allocation failed");
    b->dtype = dtype;
    b->ncirc = ncirc;
    b->want_grad = want_grad ? 1 : 0;
    b->nparams = param_offsets[ncirc];
    b->programs = int(prog_circ.size());

    // programs
    std::vector<BatchProgram> progs;
    std::vector<BatchPass> passes;
    std::vector<TileOp> ops;
    std::vector<cd> pool;
    std::vector<BatchHGroup> hgroups;
    std::vector<BatchHTerm> hterms;
    int nonsingle_max_n = 0;
    for (size_t pi = 0; pi < prog_circ.size(); ++pi) {
        const qsim_circuit &c = *prog_circ[pi];
        const qsim_pauli_sum &H = *prog_H[pi];
        std::vector<HostGate> fwd(size_t(c.nops)), rev;
        int64_t np = 0;
        for (int o = 0; o < c.nops; ++o)
            if (c.ops[o].param >= 0) np = std::max<int64_t>(np, c.ops[o].param + 1);
        std::vector<double> zeros(size_t(std::max<int64_t>(np, 1)), 0.0);
        for (int o = 0; o < c.nops; ++o) {
            make_gate(&c, o, zeros.data(), np, fwd[size_t(o)]);
            if (c.ops[o].param >= 0) {
                fwd[size_t(o)].rot_gen = rotation_generator(c.ops[o].kind);
                fwd[size_t(o)].rot_param = c.ops[o].param;
            }
        }
        for (int o = c.nops - 1; o >= 0; --o) {
            const HostGate &g = fwd[size_t(o)];
            if (g.rot_gen) {
                HostGate pr;
                pr.k = 1;
                pr.targets[0] = g.targets[0];
                pr.probe_gen = g.rot_gen;
                pr.probe_slot = g.rot_param;
                rev.push_back(pr);
                HostGate inv = g;
                inv.rot_inv = 1;
                rev.push_back(inv);
            } else {
                HostGate inv = g;
                const int d = 1 << g.k;
                for (int r = 0; r < d; ++r)
                    for (int cc = 0; cc < d; ++cc) inv.M[size_t(r) * d + cc] = std::conj(g.M[size_t(cc) * d + r]);
                rev.push_back(std::move(inv));
            }
        }
        BatchProgram bp{};
        bp.n = c.n;
        bp.m = std::min(c.n, batch_tile_max(dtype));
        if (bp.m < c.n) nonsingle_max_n = std::max(nonsingle_max_n, c.n);
        b->max_n = std::max(b->max_n, c.n);
        for (int dir = 0; dir < 2; ++dir) {
            Plan plan;
            plan.n = c.n;
            plan.dtype = dtype;
            // batch tiles hold L + 6 qubits, so the planner never widens them
            if (build_tile_plan(plan, dir == 0 ? fwd : rev, bp.m) != bp.m) {
                delete b;
                return fail(QSIM_ERR_UNSUPPORTED, "a batch program: the planner could not place every op");
            }
            if (dir == 0 && plan.passes.empty()) {
                // one empty forward pass initialises psi
                Pass p;
                p.kind = PASS_TILE;
                p.m = bp.m;
                p.L = std::min(bp.m, dtype == QSIM_C128 ? 4 : 5);
                for (int q = p.L; q < c.n && int(p.hpos.size()) < bp.m - p.L; ++q) p.hpos.push_back(q);
                plan.passes.push_back(p);
            }
            const int first = int(passes.size());
            const int op_base = int(ops.size());
            const int pool_base = int(pool.size());
            for (const Pass &p : plan.passes) {
                BatchPass bps{};
                bps.L = p.L;
                bps.H = int(p.hpos.size());
                for (int i = 0; i < bps.H; ++i) bps.hpos[i] = p.hpos[size_t(i)];
                bps.op_begin = op_base + p.op_begin;
                bps.op_end = op_base + p.op_end;
                for (int o = p.op_begin; o < p.op_end; ++o) {
                    TileOp t = plan.tile_ops[size_t(o)];
                    if (t.type == 0 || t.type == 1 || t.type == 5) t.moff += pool_base + p.pool_begin;
                    ops.push_back(t);
                }
                passes.push_back(bps);
            }
            pool.insert(pool.end(), plan.tile_pool.begin(), plan.tile_pool.end());
            if (dir == 0) {
                bp.fwd_begin = first;
                bp.fwd_end = int(passes.size());
            } else {
                bp.rev_begin = first;
                bp.rev_end = int(passes.size());
            }
        }
        std::map<uint64_t, std::vector<int>> byx;
        for (int t = 0; t < H.nterms; ++t) byx[H.terms[t].xmask].push_back(t);
        bp.hg_begin = int(hgroups.size());
        for (auto &kv : byx) {
            BatchHGroup g{};
            g.x = kv.first;
            g.first = int(hterms.size());
            g.count = int(kv.second.size());
            hgroups.push_back(g);
            for (int t : kv.second) {
                const qsim_pauli_term &pt = H.terms[t];
                const int ny = __builtin_popcountll(pt.xmask & pt.zmask) & 3;
                const double re[4] = {1, 0, -1, 0}, im[4] = {0, 1, 0, -1};
                BatchHTerm ht{};
                ht.wr = pt.coeff * re[ny];
                ht.wi = pt.coeff * im[ny];
                ht.z = pt.zmask;
                hterms.push_back(ht);
            }
        }
        bp.hg_end = int(hgroups.size());
        progs.push_back(bp);
    }
    // circuits, largest (2^n x ops) first
    std::vector<BatchCircuit> bc(static_cast<size_t>(ncirc));
    std::vector<double> cost(static_cast<size_t>(ncirc));
    for (int i = 0; i < ncirc; ++i) {
        bc[size_t(i)].prog = circ_prog[size_t(i)];
        bc[size_t(i)].nparams = int(param_offsets[i + 1] - param_offsets[i]);
        bc[size_t(i)].param_off = param_offsets[i];
        cost[size_t(i)] = std::ldexp(1.0, circs[i].n) * double(circs[i].nops + 1);
    }
    std::vector<int32_t> order(static_cast<size_t>(ncirc));
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[size_t(a)] > cost[size_t(c)]; });

    // device layout
    const size_t s = amp_bytes(dtype);
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    size_t off = 0;
    auto place = [&](size_t bytes) {
        const size_t o = off;
        off = al(off + std::max<size_t>(bytes, 8));
        return o;
    };
    const size_t o_circs = place(sizeof(BatchCircuit) * bc.size());
    const size_t o_order = place(sizeof(int32_t) * order.size());
    const size_t o_progs = place(sizeof(BatchProgram) * progs.size());
    const size_t o_passes = place(sizeof(BatchPass) * passes.size());
    const size_t o_ops = place(sizeof(TileOp) * ops.size());
    const size_t o_pool = place(s * pool.size());
    const size_t o_hg = place(sizeof(BatchHGroup) * hgroups.size());
    const size_t o_ht = place(sizeof(BatchHTerm) * hterms.size());
    const size_t o_params = place(sizeof(double) * size_t(b->nparams));
    const size_t o_energy = place(sizeof(double) * size_t(ncirc));
    const size_t o_grads = place(sizeof(double) * size_t(b->nparams));
    const size_t o_counter = place(sizeof(int));
    b->dev_bytes = off;
    hipDeviceProp_t prop;
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        destroy(b);
        return fail(QSIM_ERR_DEVICE, "hipGetDeviceProperties failed");
    }
    const int per_cu = 4;
    b->grid = std::max(1, std::min(ncirc, prop.multiProcessorCount * per_cu));
    const uint64_t slot_amps = nonsingle_max_n ? (1ull << nonsingle_max_n) : 0ull;
    if (hipMalloc(&b->dev, b->dev_bytes) != hipSuccess ||
        (slot_amps && hipMalloc(&b->arena, size_t(b->grid) * 2 * slot_amps * s) != hipSuccess)) {
        (void)hipGetLastError();
        destroy(b);
        return fail(QSIM_ERR_OOM, "cannot allocate batch device memory");
    }
    // static part uploaded once, synchronously
    std::vector<char> host(o_params, 0);
    std::memcpy(host.data() + o_circs, bc.data(), sizeof(BatchCircuit) * bc.size());
    std::memcpy(host.data() + o_order, order.data(), sizeof(int32_t) * order.size());
    std::memcpy(host.data() + o_progs, progs.data(), sizeof(BatchProgram) * progs.size());
    if (!passes.empty()) std::memcpy(host.data() + o_passes, passes.data(), sizeof(BatchPass) * passes.size());
    if (!ops.empty()) std::memcpy(host.data() + o_ops, ops.data(), sizeof(TileOp) * ops.size());
    if (dtype == QSIM_C64)
        pack_pool<float>(pool, host.data() + o_pool);
    else
        pack_pool<double>(pool, host.data() + o_pool);
    if (!hgroups.empty()) std::memcpy(host.data() + o_hg, hgroups.data(), sizeof(BatchHGroup) * hgroups.size());
    if (!hterms.empty()) std::memcpy(host.data() + o_ht, hterms.data(), sizeof(BatchHTerm) * hterms.size());
    if (hipMemcpy(b->dev, host.data(), o_params, hipMemcpyHostToDevice) != hipSuccess) {
        destroy(b);
        return fail(QSIM_ERR_DEVICE, "uploading the batch programs failed");
    }
    // capture: counter reset + persistent kernel (parameters and results
    // move device to device around the graph, in stream order)
    char *d = static_cast<char *>(b->dev);
    b->d_params = reinterpret_cast<double *>(d + o_params);
    b->d_energy = reinterpret_cast<double *>(d + o_energy);
    b->d_grads = reinterpret_cast<double *>(d + o_grads);
    BatchDevice bd{};
    bd.circs = reinterpret_cast<const BatchCircuit *>(d + o_circs);
    bd.order = reinterpret_cast<const int32_t *>(d + o_order);
    bd.progs = reinterpret_cast<const BatchProgram *>(d + o_progs);
    bd.passes = reinterpret_cast<const BatchPass *>(d + o_passes);
    bd.ops = reinterpret_cast<const TileOp *>(d + o_ops);
    bd.pool = d + o_pool;
    bd.hgroups = reinterpret_cast<const BatchHGroup *>(d + o_hg);
    bd.hterms = reinterpret_cast<const BatchHTerm *>(d + o_ht);
    bd.params = reinterpret_cast<const double *>(d + o_params);
    bd.energies = reinterpret_cast<double *>(d + o_energy);
    bd.grads = reinterpret_cast<double *>(d + o_grads);
    bd.arena = b->arena;
    bd.slot_amps = slot_amps;
    bd.counter = reinterpret_cast<int *>(d + o_counter);
    bd.ncirc = ncirc;
    bd.want_grad = b->want_grad;
    bd.mmax = batch_tile_max(dtype);
    hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = launch_batch(b->cap_stream, dtype, bd, b->grid);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->cap_stream, &g);
    if (e == hipSuccess) e = ec;
    b->graph = g;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        const std::string msg = std::string("capturing the batch graph failed: ") + hipGetErrorString(e);
        destroy(b);
        return fail(QSIM_ERR_DEVICE, msg);
    }
    *out = b;
    return QSIM_OK;
}

static bool device_memory(const void *p) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

qsim_status qsim_batch_run(qsim_batch b, const double *params_dev, double *energies_dev, double *grads_dev,
                           void *hip_stream) {
    if (!b) return fail(QSIM_ERR_ARG, "batch handle is NULL");
    clear_error();
    if (!energies_dev || (b->nparams > 0 && !params_dev) || (b->want_grad && b->nparams > 0 && !grads_dev))
        return fail(QSIM_ERR_ARG, "NULL argument");
    if (!device_memory(energies_dev) || (b->nparams > 0 && !device_memory(params_dev)) ||
        (b->want_grad && b->nparams > 0 && !device_memory(grads_dev)))
        return fail(QSIM_ERR_ARG, "params, energies and grads must be device memory");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const size_t pbytes = sizeof(double) * size_t(b->nparams);
    hipError_t e = hipSuccess;
    if (b->nparams > 0) e = hipMemcpyAsync(b->d_params, params_dev, pbytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(energies_dev, b->d_energy, sizeof(double) * size_t(b->ncirc), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && b->want_grad && b->nparams > 0)
        e = hipMemcpyAsync(grads_dev, b->d_grads, pbytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail(QSIM_ERR_DEVICE, std::string("batch run failed: ") + hipGetErrorString(e));
    b->last_stream = st;
    b->ran = true;
    return QSIM_OK;
}

qsim_status qsim_batch_info(qsim_batch b, int *grid, int *programs, int *max_n) {
    if (!b) return fail(QSIM_ERR_ARG, "batch handle is NULL");
    if (grid) *grid = b->grid;
    if (programs) *programs = b->programs;
    if (max_n) *max_n = b->max_n;
    return QSIM_OK;
}

qsim_status qsim_batch_free(qsim_batch b) {
    if (b && b->ran) (void)hipStreamSynchronize(b->last_stream);
    if (b && b->cap_stream) (void)hipStreamSynchronize(b->cap_stream);
    destroy(b);
    return QSIM_OK;
}

}  // extern "C"
