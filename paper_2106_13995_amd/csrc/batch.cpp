// Host side of batched runs: validation, one program per distinct circuit
// structure (forward passes, reverse passes with probes, observable terms),
// largest-first work order, device buffers and the captured HIP graph that
// runs a whole batch as one replay.
#include <algorithm>
#include <cstdlib>
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
    void *arena = nullptr;        // per-workgroup psi / lambda slots (persistent kernel)
    void *larena = nullptr;       // per-circuit psi / lambda slots (layered circuits)
    int nlayered = 0;
    double pass_bytes = 0;        // device-memory bytes of one run's layered passes
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
    if (b->larena) (void)hipFree(b->larena);
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

namespace qsim {

// Plans circuit c with observable H as one batch program and appends it to
// t: layered (register-staged passes, tiles of mL qubits) when c fills whole
// tiles and every pass can be staged, else for the persistent kernel, unless
// layered_only (then *is_layered is false and nothing is appended).
qsim_status add_batch_program(BatchTables &t, const qsim_circuit &c, const qsim_pauli_sum &H, int dtype, int mL,
                              int fuse_k, bool layered_only, bool *is_layered) {
    std::vector<BatchProgram> &progs = t.progs;
    std::vector<BatchPass> &passes = t.passes;
    std::vector<TileOp> &ops = t.ops;
    std::vector<RegStage> &stages = t.stages;
    std::vector<RegOp> &rops = t.rops;
    std::vector<cd> &pool = t.pool;
    std::vector<BatchHGroup> &hgroups = t.hgroups;
    std::vector<BatchHTerm> &hterms = t.hterms;
    std::vector<int32_t> &probe_row = t.probe_row, &probe_idx = t.probe_idx;
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
    if (fuse_k > 1) {
        // runs of fixed gates merged into blocks of at most fuse_k qubits
        // (the parametric rotations between them stay as they are)
        std::vector<HostGate> merged, run;
        for (HostGate &g : fwd) {
            if (g.rot_gen) {
                for (HostGate &f : fuse_gates(run, fuse_k)) merged.push_back(std::move(f));
                run.clear();
                merged.push_back(std::move(g));
            } else {
                run.push_back(std::move(g));
            }
        }
        for (HostGate &f : fuse_gates(run, fuse_k)) merged.push_back(std::move(f));
        fwd.swap(merged);
    }
    for (int o = int(fwd.size()) - 1; o >= 0; --o) {
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
    if (c.n >= mL) bp.m = mL;
    // Circuits that fill whole tiles run layered, register-staged
    // throughout; a program with a pass that cannot be staged (a dense
    // block on more than three qubits) and smaller circuits run in the
    // persistent kernel, from LDS.
    bool layered = bp.m == mL;
    Plan plans[2];
    for (int attempt = 0; attempt < 2; ++attempt) {
        bool ok = true;
        for (int dir = 0; dir < 2; ++dir) {
            plans[dir] = Plan();
            plans[dir].n = c.n;
            plans[dir].dtype = dtype;
            std::vector<HostGate> items = dir == 0 ? fwd : rev;
            if (dir == 0 && items.empty() && layered) {
                // an identity on qubit 0 gives the forward sweep the pass
                // that starts psi at |0...0>
                HostGate id;
                id.k = 1;
                id.M = {cd(1.0), cd(0.0), cd(0.0), cd(1.0)};
                items.push_back(id);
            }
            // batch tiles hold L + 6 qubits, so the planner never widens them
            if (build_tile_plan(plans[dir], items, bp.m, 1, layered) != bp.m)
                return fail(QSIM_ERR_UNSUPPORTED, "a batch program: the planner could not place every op");
            if (layered)
                for (const Pass &p : plans[dir].passes) ok = ok && p.reg_r == mL - 8;
        }
        if (ok) break;
        if (layered_only) {
            *is_layered = false;
            return QSIM_OK;
        }
        layered = false;
    }
    if (!layered && bp.m < c.n) t.nonsingle_max_n = std::max(t.nonsingle_max_n, c.n);
    bp.layered = layered ? 1 : 0;
    for (int dir = 0; dir < 2; ++dir) {
        Plan &plan = plans[dir];
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
            if (layered) {
                bps.reg_r = p.reg_r;
                const int rop0 = int(rops.size());
                for (int o = p.rop_begin; o < p.rop_end; ++o) {
                    RegOp r = plan.reg_ops[size_t(o)];
                    // rotations and probes name a parameter, not a pool
                    // entry; a probe's jmatch becomes its index in the
                    // sweep (a fused probe's rotation is the inverse)
                    if (r.type == 9 || r.type == 10) {
                        r.jmatch = bp.nprobes++;
                    } else if (r.type == 12) {
                        r.jmatch = bp.nprobes;
                        bp.nprobes += 2;
                    } else if (r.type != 8 && r.type != 11) {
                        r.moff += pool_base + p.pool_begin;
                    }
                    rops.push_back(r);
                }
                bps.stage_begin = int(stages.size());
                for (int si = p.stage_begin; si < p.stage_end; ++si) {
                    RegStage st = plan.reg_stages[size_t(si)];
                    st.op_begin += rop0;
                    st.op_end += rop0;
                    stages.push_back(st);
                }
                bps.stage_end = int(stages.size());
                for (int i = 0; i < 8; ++i) {
                    bps.ld_t[i] = p.ld_t[i];
                    bps.st_t[i] = p.st_t[i];
                }
                for (int i = 0; i < kRegBitsMax; ++i) {
                    bps.ld_r[i] = p.ld_r[i];
                    bps.st_r[i] = p.st_r[i];
                }
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
    if (layered) {
        // parameter -> its probes (CSR), in sweep order
        bp.nparams = int(np);
        bp.row_off = int(probe_row.size());
        std::vector<std::vector<int32_t>> of(static_cast<size_t>(np));
        for (int pi2 = bp.rev_begin; pi2 < bp.rev_end; ++pi2)
            for (int si = passes[size_t(pi2)].stage_begin; si < passes[size_t(pi2)].stage_end; ++si)
                for (int o = stages[size_t(si)].op_begin; o < stages[size_t(si)].op_end; ++o)
                    if (rops[size_t(o)].type == 9 || rops[size_t(o)].type == 10) {
                        of[size_t(rops[size_t(o)].moff)].push_back(rops[size_t(o)].jmatch);
                    } else if (rops[size_t(o)].type == 12) {
                        of[size_t(rops[size_t(o)].moff)].push_back(rops[size_t(o)].jmatch);
                        of[size_t(rops[size_t(o)].gj[0])].push_back(rops[size_t(o)].jmatch + 1);
                    }
        int32_t at = int32_t(probe_idx.size());
        for (int64_t j = 0; j < np; ++j) {
            probe_row.push_back(at);
            for (int32_t k : of[size_t(j)]) probe_idx.push_back(k);
            at = int32_t(probe_idx.size());
        }
        probe_row.push_back(at);
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
    *is_layered = layered;
    return QSIM_OK;
}

qsim_status plan_layered_adjoint(const qsim_circuit *c, int64_t nparams, const qsim_pauli_sum *H, int dtype,
                                 LayeredAdjoint &out, bool *ok) {
    *ok = false;
    const int mL = batch_layer_default(dtype);
    if (c->n < mL || c->nops < 1) return QSIM_OK;
    // parameters in range and on RX, RY, RZ only (the LDS path reports the
    // error otherwise)
    for (int o = 0; o < c->nops; ++o)
        if (c->ops[o].param >= nparams || (c->ops[o].param >= 0 && !rotation_generator(c->ops[o].kind)))
            return QSIM_OK;
    BatchTables t;
    bool lay = false;
    qsim_status st = add_batch_program(t, *c, *H, dtype, mL, 1, true, &lay);
    if (st != QSIM_OK || !lay) return st;
    const BatchProgram &pg = t.progs[0];
    BatchLCirc l{};
    l.circ = 0;
    l.prog = 0;
    l.ntiles = 1 << (pg.n - pg.m);
    l.nchunks = int(std::max<int64_t>(1, (int64_t(1) << pg.n) / kBatchChunk));
    l.param_off = 0;
    l.nparams = int(nparams);
    l.gfirst = 0;
    l.psi_off = l.lam_off = 0;   // the state and the second state, each its own base
    l.pp_off = l.ep_off = 0;
    std::vector<BatchWork> works;
    std::vector<BatchStep> steps;
    auto layer = [&](int kind, int pass) {
        BatchStep s{};
        s.kind = kind;
        s.init = 0;   // the forward sweep starts from the state's content
        s.wbegin = int(works.size());
        BatchWork w{};
        w.lc = 0;
        w.pass = pass;
        w.first = 0;
        w.count = uint32_t(kind == 2 ? l.nchunks : l.ntiles);
        works.push_back(w);
        s.wend = int(works.size());
        s.wgs = w.count;
        s.lc_begin = 0;
        s.lc_end = 1;
        steps.push_back(s);
    };
    for (int p = pg.fwd_begin; p < pg.fwd_end; ++p) layer(0, p);
    layer(2, -1);
    for (int p = pg.rev_begin; p < pg.rev_end; ++p) layer(1, p);
    BatchStep gr{};
    gr.kind = 3;
    gr.lc_begin = 0;
    gr.lc_end = 1;
    gr.gw_begin = 0;
    gr.gw_end = nparams;
    steps.push_back(gr);
    const double tile = double(amp_bytes(dtype)) * std::ldexp(1.0, mL);
    out.pass_bytes = (2.0 * double(pg.fwd_end - pg.fwd_begin) + 4.0 * double(pg.rev_end - pg.rev_begin)) * tile *
                         double(l.ntiles) +
                     2.0 * double(amp_bytes(dtype)) * std::ldexp(1.0, pg.n);
    // packed tables
    const size_t s = amp_bytes(dtype);
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    size_t off = 0;
    auto place = [&](size_t bytes) {
        const size_t o = off;
        off = al(off + std::max<size_t>(bytes, 8));
        return o;
    };
    out.o_progs = place(sizeof(BatchProgram) * t.progs.size());
    out.o_passes = place(sizeof(BatchPass) * t.passes.size());
    out.o_stages = place(sizeof(RegStage) * t.stages.size());
    out.o_rops = place(sizeof(RegOp) * t.rops.size());
    out.o_pool = place(s * t.pool.size());
    out.o_hg = place(sizeof(BatchHGroup) * t.hgroups.size());
    out.o_ht = place(sizeof(BatchHTerm) * t.hterms.size());
    out.o_lc = place(sizeof(BatchLCirc));
    out.o_works = place(sizeof(BatchWork) * works.size());
    out.o_prow = place(sizeof(int32_t) * t.probe_row.size());
    out.o_pidx = place(sizeof(int32_t) * t.probe_idx.size());
    out.host.assign(off, 0);
    char *h = out.host.data();
    std::memcpy(h + out.o_progs, t.progs.data(), sizeof(BatchProgram) * t.progs.size());
    std::memcpy(h + out.o_passes, t.passes.data(), sizeof(BatchPass) * t.passes.size());
    if (!t.stages.empty()) std::memcpy(h + out.o_stages, t.stages.data(), sizeof(RegStage) * t.stages.size());
    if (!t.rops.empty()) std::memcpy(h + out.o_rops, t.rops.data(), sizeof(RegOp) * t.rops.size());
    if (dtype == QSIM_C64)
        pack_pool<float>(t.pool, h + out.o_pool);
    else
        pack_pool<double>(t.pool, h + out.o_pool);
    if (!t.hgroups.empty()) std::memcpy(h + out.o_hg, t.hgroups.data(), sizeof(BatchHGroup) * t.hgroups.size());
    if (!t.hterms.empty()) std::memcpy(h + out.o_ht, t.hterms.data(), sizeof(BatchHTerm) * t.hterms.size());
    std::memcpy(h + out.o_lc, &l, sizeof(BatchLCirc));
    std::memcpy(h + out.o_works, works.data(), sizeof(BatchWork) * works.size());
    if (!t.probe_row.empty()) std::memcpy(h + out.o_prow, t.probe_row.data(), sizeof(int32_t) * t.probe_row.size());
    if (!t.probe_idx.empty()) std::memcpy(h + out.o_pidx, t.probe_idx.data(), sizeof(int32_t) * t.probe_idx.size());
    // the call's scratch: rotation table, probe partials, energy partials
    size_t so = 0;
    auto splace = [&](size_t bytes) {
        const size_t o = so;
        so = al(so + std::max<size_t>(bytes, 8));
        return o;
    };
    out.o_trig = splace(4 * sizeof(double) * size_t(std::max<int64_t>(nparams, 1)));
    out.o_ppart = splace(sizeof(double) * size_t(pg.nprobes) * size_t(l.ntiles));
    out.o_epart = splace(sizeof(double) * size_t(l.nchunks));
    out.scratch_bytes = so;
    BatchLayerDevice &ld = out.ld;
    ld = BatchLayerDevice{};
    ld.nlc = 1;
    ld.nparams = nparams;
    ld.want_grad = 1;
    ld.R = mL - 8;
    ld.steps = std::move(steps);
    *ok = true;
    return QSIM_OK;
}

void bind_layered_adjoint(LayeredAdjoint &la, void *dev, void *psi, void *lam, void *scratch,
                          const double *params_dev, double *energy_dev, double *grad_dev) {
    char *d = static_cast<char *>(dev);
    char *sc = static_cast<char *>(scratch);
    BatchLayerDevice &ld = la.ld;
    ld.lc = reinterpret_cast<const BatchLCirc *>(d + la.o_lc);
    ld.works = reinterpret_cast<const BatchWork *>(d + la.o_works);
    ld.progs = reinterpret_cast<const BatchProgram *>(d + la.o_progs);
    ld.passes = reinterpret_cast<const BatchPass *>(d + la.o_passes);
    ld.stages = reinterpret_cast<const RegStage *>(d + la.o_stages);
    ld.rops = reinterpret_cast<const RegOp *>(d + la.o_rops);
    ld.pool = d + la.o_pool;
    ld.hgroups = reinterpret_cast<const BatchHGroup *>(d + la.o_hg);
    ld.hterms = reinterpret_cast<const BatchHTerm *>(d + la.o_ht);
    ld.probe_row = reinterpret_cast<const int32_t *>(d + la.o_prow);
    ld.probe_idx = reinterpret_cast<const int32_t *>(d + la.o_pidx);
    ld.params = params_dev;
    ld.trig = reinterpret_cast<double *>(sc + la.o_trig);
    ld.ppart = reinterpret_cast<double *>(sc + la.o_ppart);
    ld.epart = reinterpret_cast<double *>(sc + la.o_epart);
    ld.energies = energy_dev;
    ld.grads = grad_dev;
    ld.arena = psi;
    ld.lam_arena = lam;
}

}  // namespace qsim

extern "C" {

qsim_status qsim_batch_create(int ncirc, const qsim_circuit *circs, const int64_t *param_offsets,
                              const qsim_pauli_sum *Hs, qsim_dtype dtype, int want_grad, const qsim_options *opts,
                              qsim_batch *out) {
    if (!out) return fail(QSIM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (ncirc < 1 || !circs || !param_offsets || !Hs) return fail(QSIM_ERR_ARG, "empty batch or NULL array");
    if (dtype != QSIM_C64 && dtype != QSIM_C128) return fail(QSIM_ERR_ARG, "dtype must be QSIM_C64 or QSIM_C128");
    if (param_offsets[0] != 0) return fail(QSIM_ERR_ARG, "param_offsets[0] must be 0");
    // options: fusion of the fixed gates between parametric ones, and the
    // tile width of layered circuits
    const int fuse_k = opts && opts->fuse_k > 0 ? opts->fuse_k : 1;
    if (opts && (opts->fuse_k < 0 || opts->fuse_k > 3)) return fail(QSIM_ERR_ARG, "batch fuse_k must be 0..3");
    const int mL = opts && opts->tile_m > 0 ? opts->tile_m : batch_layer_default(dtype);
    if (opts && opts->tile_m != 0 && !batch_layer_width_ok(dtype, opts->tile_m))
        return fail(QSIM_ERR_ARG, "batch tile_m must be 0, 11 or 12 (complex64) or 0 or 11 (complex128)");
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
    BatchTables tabs;
    for (size_t pi = 0; pi < prog_circ.size(); ++pi) {
        b->max_n = std::max(b->max_n, prog_circ[pi]->n);
        bool lay = false;
        const qsim_status st = add_batch_program(tabs, *prog_circ[pi], *prog_H[pi], dtype, mL, fuse_k, false, &lay);
        if (st != QSIM_OK) {
            delete b;
            return st;
        }
    }
    std::vector<BatchProgram> &progs = tabs.progs;
    std::vector<BatchPass> &passes = tabs.passes;
    std::vector<TileOp> &ops = tabs.ops;
    std::vector<RegStage> &stages = tabs.stages;
    std::vector<RegOp> &rops = tabs.rops;
    std::vector<cd> &pool = tabs.pool;
    std::vector<BatchHGroup> &hgroups = tabs.hgroups;
    std::vector<BatchHTerm> &hterms = tabs.hterms;
    std::vector<int32_t> &probe_row = tabs.probe_row, &probe_idx = tabs.probe_idx;
    const int nonsingle_max_n = tabs.nonsingle_max_n;
    // circuits, largest (2^n x ops) first; persistent ones in `order`, the
    // layered ones in `lcircs`
    std::vector<BatchCircuit> bc(static_cast<size_t>(ncirc));
    std::vector<double> cost(static_cast<size_t>(ncirc));
    for (int i = 0; i < ncirc; ++i) {
        bc[size_t(i)].prog = circ_prog[size_t(i)];
        bc[size_t(i)].nparams = int(param_offsets[i + 1] - param_offsets[i]);
        bc[size_t(i)].param_off = param_offsets[i];
        cost[size_t(i)] = std::ldexp(1.0, circs[i].n) * double(circs[i].nops + 1);
    }
    std::vector<int32_t> all(static_cast<size_t>(ncirc));
    std::iota(all.begin(), all.end(), 0);
    std::stable_sort(all.begin(), all.end(), [&](int a, int c) { return cost[size_t(a)] > cost[size_t(c)]; });
    std::vector<int32_t> order;
    std::vector<BatchLCirc> lcircs;
    const size_t s = amp_bytes(dtype);
    for (int32_t i : all) {
        const BatchProgram &pg = progs[size_t(bc[size_t(i)].prog)];
        if (!pg.layered) {
            order.push_back(i);
            continue;
        }
        BatchLCirc l{};
        l.circ = i;
        l.prog = bc[size_t(i)].prog;
        l.ntiles = 1 << (pg.n - pg.m);
        l.nchunks = int(std::max<int64_t>(1, (int64_t(1) << pg.n) / kBatchChunk));
        l.param_off = bc[size_t(i)].param_off;
        l.nparams = bc[size_t(i)].nparams;
        lcircs.push_back(l);
    }
    b->nlayered = int(lcircs.size());
    // Layered circuits go in groups whose slots fit the budget; each group
    // runs its forward layers, energies and reverse layers before the next,
    // in slots at the start of the arena.
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = 0;
    }
    size_t budget = std::max<size_t>(size_t(1) << 30, free_b / 2);
    if (const char *ev = std::getenv("QSIM_BATCH_SLOT_BUDGET")) {
        // bytes of layered slots per group (tests: several groups on small batches)
        const long long v = std::atoll(ev);
        if (v > 0) budget = size_t(v);
    }
    std::vector<BatchWork> works;
    std::vector<BatchStep> steps;
    size_t larena_amps = 0;
    uint64_t pp_total = 0, ep_total = 0;
    int64_t gw_total = 0;
    for (size_t g0 = 0; g0 < lcircs.size();) {
        size_t g1 = g0;
        uint64_t amps = 0;
        const uint64_t per = b->want_grad ? 2 : 1;
        while (g1 < lcircs.size()) {
            const uint64_t need = per * (uint64_t(1) << progs[size_t(lcircs[g1].prog)].n);
            if (g1 > g0 && (amps + need) * s > budget) break;
            amps += need;
            ++g1;
        }
        uint64_t at = 0;
        int max_fwd = 0, max_rev = 0;
        const int64_t gw0 = gw_total;
        for (size_t k = g0; k < g1; ++k) {
            BatchLCirc &l = lcircs[k];
            const BatchProgram &pg = progs[size_t(l.prog)];
            const uint64_t N = uint64_t(1) << pg.n;
            l.psi_off = at;
            at += N;
            l.lam_off = b->want_grad ? at : l.psi_off;
            if (b->want_grad) at += N;
            l.pp_off = pp_total;
            if (b->want_grad) pp_total += uint64_t(pg.nprobes) * uint64_t(l.ntiles);
            l.ep_off = ep_total;
            ep_total += uint64_t(l.nchunks);
            l.gfirst = gw_total;
            gw_total += l.nparams;
            max_fwd = std::max(max_fwd, pg.fwd_end - pg.fwd_begin);
            max_rev = std::max(max_rev, pg.rev_end - pg.rev_begin);
        }
        larena_amps = std::max<size_t>(larena_amps, size_t(at));
        auto layer = [&](int kind, int sidx) {
            BatchStep st{};
            st.kind = kind;
            st.init = kind == 0 && sidx == 0;
            st.wbegin = int(works.size());
            uint32_t wgs = 0;
            for (size_t k = g0; k < g1; ++k) {
                const BatchLCirc &l = lcircs[k];
                const BatchProgram &pg = progs[size_t(l.prog)];
                BatchWork w{};
                w.lc = int(k);
                if (kind == 2) {
                    w.pass = -1;
                    w.count = uint32_t(l.nchunks);
                } else {
                    const int b0 = kind == 0 ? pg.fwd_begin : pg.rev_begin, b1 = kind == 0 ? pg.fwd_end : pg.rev_end;
                    if (b0 + sidx >= b1) continue;
                    w.pass = b0 + sidx;
                    w.count = uint32_t(l.ntiles);
                }
                w.first = wgs;
                wgs += w.count;
                works.push_back(w);
            }
            st.wend = int(works.size());
            st.wgs = wgs;
            st.lc_begin = int(g0);
            st.lc_end = int(g1);
            steps.push_back(st);
        };
        for (int k = 0; k < max_fwd; ++k) layer(0, k);
        layer(2, 0);
        if (b->want_grad) {
            for (int k = 0; k < max_rev; ++k) layer(1, k);
            BatchStep gr{};
            gr.kind = 3;
            gr.lc_begin = int(g0);
            gr.lc_end = int(g1);
            gr.gw_begin = gw0;
            gr.gw_end = gw_total;
            steps.push_back(gr);
        }
        g0 = g1;
    }

    // bytes the layered passes move per run: tiles in and out per pass
    // (twice in reverse passes: psi and lambda); the energies read psi and
    // write lambda
    for (const BatchStep &st : steps) {
        const double tile = double(s) * std::ldexp(1.0, mL);
        if (st.kind == 0) b->pass_bytes += 2.0 * tile * st.wgs;
        if (st.kind == 1) b->pass_bytes += 4.0 * tile * st.wgs;
        if (st.kind == 2)
            for (int w = st.wbegin; w < st.wend; ++w) {
                const BatchLCirc &l = lcircs[size_t(works[size_t(w)].lc)];
                b->pass_bytes += (b->want_grad ? 2.0 : 1.0) * double(s) *
                                 std::ldexp(1.0, progs[size_t(l.prog)].n);
            }
    }

    // device layout
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
    const size_t o_stages = place(sizeof(RegStage) * stages.size());
    const size_t o_rops = place(sizeof(RegOp) * rops.size());
    const size_t o_pool = place(s * pool.size());
    const size_t o_hg = place(sizeof(BatchHGroup) * hgroups.size());
    const size_t o_ht = place(sizeof(BatchHTerm) * hterms.size());
    const size_t o_lc = place(sizeof(BatchLCirc) * lcircs.size());
    const size_t o_works = place(sizeof(BatchWork) * works.size());
    const size_t o_prow = place(sizeof(int32_t) * probe_row.size());
    const size_t o_pidx = place(sizeof(int32_t) * probe_idx.size());
    const size_t o_params = place(sizeof(double) * size_t(b->nparams));
    const size_t o_energy = place(sizeof(double) * size_t(ncirc));
    const size_t o_grads = place(sizeof(double) * size_t(b->nparams));
    const size_t o_counter = place(sizeof(int));
    const size_t o_trig = place(4 * sizeof(double) * size_t(b->nparams));
    const size_t o_ppart = place(sizeof(double) * size_t(pp_total));
    const size_t o_epart = place(sizeof(double) * size_t(ep_total));
    b->dev_bytes = off;
    hipDeviceProp_t prop;
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        destroy(b);
        return fail(QSIM_ERR_DEVICE, "hipGetDeviceProperties failed");
    }
    const int per_cu = 4;
    b->grid = std::max(1, std::min(int(order.size()), prop.multiProcessorCount * per_cu));
    const uint64_t slot_amps = nonsingle_max_n ? (1ull << nonsingle_max_n) : 0ull;
    if (hipMalloc(&b->dev, b->dev_bytes) != hipSuccess ||
        (slot_amps && !order.empty() && hipMalloc(&b->arena, size_t(b->grid) * 2 * slot_amps * s) != hipSuccess) ||
        (larena_amps && hipMalloc(&b->larena, larena_amps * s) != hipSuccess)) {
        (void)hipGetLastError();
        destroy(b);
        return fail(QSIM_ERR_OOM, "cannot allocate batch device memory");
    }
    // static part uploaded once, synchronously
    std::vector<char> host(o_params, 0);
    std::memcpy(host.data() + o_circs, bc.data(), sizeof(BatchCircuit) * bc.size());
    if (!order.empty()) std::memcpy(host.data() + o_order, order.data(), sizeof(int32_t) * order.size());
    std::memcpy(host.data() + o_progs, progs.data(), sizeof(BatchProgram) * progs.size());
    if (!passes.empty()) std::memcpy(host.data() + o_passes, passes.data(), sizeof(BatchPass) * passes.size());
    if (!ops.empty()) std::memcpy(host.data() + o_ops, ops.data(), sizeof(TileOp) * ops.size());
    if (!stages.empty()) std::memcpy(host.data() + o_stages, stages.data(), sizeof(RegStage) * stages.size());
    if (!rops.empty()) std::memcpy(host.data() + o_rops, rops.data(), sizeof(RegOp) * rops.size());
    if (dtype == QSIM_C64)
        pack_pool<float>(pool, host.data() + o_pool);
    else
        pack_pool<double>(pool, host.data() + o_pool);
    if (!hgroups.empty()) std::memcpy(host.data() + o_hg, hgroups.data(), sizeof(BatchHGroup) * hgroups.size());
    if (!hterms.empty()) std::memcpy(host.data() + o_ht, hterms.data(), sizeof(BatchHTerm) * hterms.size());
    if (!lcircs.empty()) std::memcpy(host.data() + o_lc, lcircs.data(), sizeof(BatchLCirc) * lcircs.size());
    if (!works.empty()) std::memcpy(host.data() + o_works, works.data(), sizeof(BatchWork) * works.size());
    if (!probe_row.empty()) std::memcpy(host.data() + o_prow, probe_row.data(), sizeof(int32_t) * probe_row.size());
    if (!probe_idx.empty()) std::memcpy(host.data() + o_pidx, probe_idx.data(), sizeof(int32_t) * probe_idx.size());
    if (hipMemcpy(b->dev, host.data(), o_params, hipMemcpyHostToDevice) != hipSuccess) {
        destroy(b);
        return fail(QSIM_ERR_DEVICE, "uploading the batch programs failed");
    }
    // capture: the layered launches, then the counter reset and the
    // persistent kernel (parameters and results move device to device around
    // the graph, in stream order)
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
    bd.stages = reinterpret_cast<const RegStage *>(d + o_stages);
    bd.rops = reinterpret_cast<const RegOp *>(d + o_rops);
    bd.pool = d + o_pool;
    bd.hgroups = reinterpret_cast<const BatchHGroup *>(d + o_hg);
    bd.hterms = reinterpret_cast<const BatchHTerm *>(d + o_ht);
    bd.params = reinterpret_cast<const double *>(d + o_params);
    bd.energies = reinterpret_cast<double *>(d + o_energy);
    bd.grads = reinterpret_cast<double *>(d + o_grads);
    bd.arena = b->arena;
    bd.slot_amps = slot_amps;
    bd.counter = reinterpret_cast<int *>(d + o_counter);
    bd.ncirc = int(order.size());
    bd.want_grad = b->want_grad;
    bd.mmax = batch_tile_max(dtype);
    BatchLayerDevice ld{};
    ld.lc = reinterpret_cast<const BatchLCirc *>(d + o_lc);
    ld.nlc = int(lcircs.size());
    ld.works = reinterpret_cast<const BatchWork *>(d + o_works);
    ld.progs = bd.progs;
    ld.passes = bd.passes;
    ld.stages = bd.stages;
    ld.rops = bd.rops;
    ld.pool = bd.pool;
    ld.hgroups = bd.hgroups;
    ld.hterms = bd.hterms;
    ld.probe_row = reinterpret_cast<const int32_t *>(d + o_prow);
    ld.probe_idx = reinterpret_cast<const int32_t *>(d + o_pidx);
    ld.params = bd.params;
    ld.trig = reinterpret_cast<double *>(d + o_trig);
    ld.nparams = b->nparams;
    ld.energies = bd.energies;
    ld.grads = bd.grads;
    ld.arena = b->larena;
    ld.ppart = reinterpret_cast<double *>(d + o_ppart);
    ld.epart = reinterpret_cast<double *>(d + o_epart);
    ld.want_grad = b->want_grad;
    ld.steps = steps;
    ld.R = mL - 8;
    ld.lam_arena = nullptr;
    hipError_t e = lcircs.empty() ? hipSuccess : batch_layer_setup(dtype, ld.R);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess && !lcircs.empty()) e = launch_batch_layered(b->cap_stream, dtype, ld);
    if (e == hipSuccess && !order.empty()) e = launch_batch(b->cap_stream, dtype, bd, b->grid);
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

qsim_status qsim_batch_layout(qsim_batch b, int *layered, int *persistent, double *pass_bytes) {
    if (!b) return fail(QSIM_ERR_ARG, "batch handle is NULL");
    if (layered) *layered = b->nlayered;
    if (persistent) *persistent = b->ncirc - b->nlayered;
    if (pass_bytes) *pass_bytes = b->pass_bytes;
    return QSIM_OK;
}

qsim_status qsim_batch_autotune(int ncirc, const qsim_circuit *circs, const int64_t *param_offsets,
                                const qsim_pauli_sum *Hs, qsim_dtype dtype, int want_grad, const double *params_dev,
                                int reps, qsim_options *best, double *best_ms) {
    if (!best) return fail(QSIM_ERR_ARG, "best is NULL");
    if (reps < 1) return fail(QSIM_ERR_ARG, "reps must be at least 1");
    if (ncirc < 1 || !param_offsets) return fail(QSIM_ERR_ARG, "empty batch or NULL array");
    const int64_t np = param_offsets[ncirc];
    if (np > 0 && (!params_dev || !device_memory(params_dev)))
        return fail(QSIM_ERR_ARG, "params must be device memory");
    std::vector<qsim_options> cands;
    for (int m : {12, 11})
        if (batch_layer_width_ok(dtype, m))
            for (int f = 1; f <= 3; ++f) {
                qsim_options o{};
                o.fuse_k = f;
                o.tile_m = m;
                cands.push_back(o);
            }
    double *energies = nullptr, *grads = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        if (energies) (void)hipFree(energies);
        if (grads) (void)hipFree(grads);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
    };
    if (hipMalloc(&energies, sizeof(double) * size_t(ncirc)) != hipSuccess ||
        (want_grad && np > 0 && hipMalloc(&grads, sizeof(double) * size_t(np)) != hipSuccess)) {
        (void)hipGetLastError();
        release();
        return fail(QSIM_ERR_OOM, "cannot allocate the autotuner's outputs");
    }
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return fail(QSIM_ERR_DEVICE, "cannot create the autotuner's stream and events");
    }
    double best_t = -1.0;
    for (const qsim_options &o : cands) {
        qsim_batch b = nullptr;
        qsim_status s = qsim_batch_create(ncirc, circs, param_offsets, Hs, dtype, want_grad, &o, &b);
        if (s != QSIM_OK) {
            release();
            return s;
        }
        s = qsim_batch_run(b, params_dev, energies, grads, st);
        if (s == QSIM_OK && hipEventRecord(e0, st) != hipSuccess) s = fail(QSIM_ERR_DEVICE, "event record failed");
        for (int r = 0; r < reps && s == QSIM_OK; ++r) s = qsim_batch_run(b, params_dev, energies, grads, st);
        float ms = 0.0f;
        if (s == QSIM_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            s = fail(QSIM_ERR_DEVICE, "timing the batch failed");
        (void)qsim_batch_free(b);
        if (s != QSIM_OK) {
            release();
            return s;
        }
        const double t = double(ms) / reps;
        if (best_t < 0.0 || t < best_t) {
            best_t = t;
            *best = o;
        }
    }
    release();
    if (best_ms) *best_ms = best_t;
    return QSIM_OK;
}

qsim_status qsim_batch_free(qsim_batch b) {
    if (b && b->ran) (void)hipStreamSynchronize(b->last_stream);
    if (b && b->cap_stream) (void)hipStreamSynchronize(b->cap_stream);
    destroy(b);
    return QSIM_OK;
}

}  // extern "C"
