// Host planner: gate fusion and grouping of gates into device passes.
//
// A pass is one sweep over the state in HBM:
//   PASS_DENSE  one gate on <= 3 targets (plus exact control bits, which
//               restrict the sweep to the amplitudes whose controls are 1);
//   PASS_DIAG   one diagonal gate, touching only amplitudes whose diagonal
//               entry differs from 1;
//   PASS_TILE   a run of gates applied to 2^m-amplitude tiles held in LDS:
//               every dense gate of the run acts inside the tile's qubit set,
//               diagonal gates may act anywhere (bits outside the tile are
//               constant across a tile).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <set>

#include "qsim_internal.h"

namespace qsim {

size_t amp_bytes(int dtype) { return dtype == QSIM_C128 ? 16 : 8; }

static int max_tile_m(int dtype) { return dtype == QSIM_C128 ? 12 : 13; }
static int default_tile_m(int dtype) { return dtype == QSIM_C128 ? 11 : 12; }
static int low_tile_qubits(int dtype) { return dtype == QSIM_C128 ? 4 : 5; }

PlanOptions resolve_options(const qsim_options *o, int n, int dtype) {
    PlanOptions po;
    qsim_options z{};
    if (!o) o = &z;
    po.fuse_k = o->fuse_k == 0 ? 1 : o->fuse_k;
    if (o->tile_m == 0)
        po.tile_m = std::min(n, default_tile_m(dtype));
    else if (o->tile_m < 0)
        po.tile_m = -1;
    else
        po.tile_m = std::min(n, std::min(o->tile_m, max_tile_m(dtype)));
    po.use_mfma = o->use_mfma;
    po.split_1q = o->split_1q >= 0;
    return po;
}

Plan::~Plan() {
    if (dev) (void)hipFreeAsync(dev, dev_stream);
}

// ------------------------------------------------------------ fusion

static uint64_t qmask(const HostGate &g) {
    uint64_t m = 0;
    for (int b = 0; b < g.k; ++b) m |= 1ull << g.targets[b];
    return m;
}

std::vector<HostGate> fuse_gates(const std::vector<HostGate> &gates, int fuse_k) {
    if (fuse_k <= 1) return gates;
    // Blocks in execution order.  A gate joins the last block that shares a
    // qubit with it when the union stays within fuse_k qubits; otherwise it
    // may join any later block (it commutes with those, as they share no
    // qubit with it); otherwise it opens a new block.
    std::vector<HostGate> blocks;
    std::vector<uint64_t> masks;
    for (const HostGate &g : gates) {
        const uint64_t gm = qmask(g);
        int last = -1;
        for (int i = int(blocks.size()) - 1; i >= 0; --i)
            if (masks[i] & gm) { last = i; break; }
        int best = -1, best_size = 1 << 30;
        for (int i = std::max(last, 0); i < int(blocks.size()); ++i) {
            if (i < last) continue;
            const int u = __builtin_popcountll(masks[i] | gm);
            if (u > fuse_k) continue;
            // prefer the dependency block, then the smallest union
            const int score = (i == last ? -100 : 0) + u;
            if (score < best_size) { best_size = score; best = i; }
        }
        if (best < 0) {
            blocks.push_back(g);
            blocks.back().src_op = -1;
            masks.push_back(gm);
        } else {
            blocks[best] = fuse_pair(blocks[best], g);
            blocks[best].src_op = -1;
            masks[best] |= gm;
        }
    }
    return blocks;
}

// ------------------------------------------------------------ passes

static double diag_bytes(const HostGate &g, int n, int dtype) {
    int nonunit = 0;
    const int d = 1 << g.k;
    for (int j = 0; j < d; ++j)
        if (g.M[j * d + j] != cd(1.0)) ++nonunit;
    return 2.0 * double(nonunit) * std::ldexp(1.0, n - g.k) * double(amp_bytes(dtype));
}

// Whether a sweep pass runs as a lane-exchange kernel: complex64, no
// controls, at least 7 qubits, one or two targets anywhere or three with at
// most one above qubit 6 (measured on 30 qubits: three high targets split a
// wave's accesses into eight 128-byte runs and take 0.65 of HBM, against
// 0.70 for the two-stream sweep).
bool lane_sweep_ok(int dtype, int n, const Pass &p) {
    if (dtype != QSIM_C64 || n < 7 || p.kind != PASS_DENSE || p.nctrl != 0 || p.k < 1 || p.k > 3) return false;
    int high = 0;
    for (int b = 0; b < p.k; ++b) high += p.targets[b] > 6;
    return p.k < 3 || high <= 1;
}

static Pass sweep_pass(const HostGate &g, int n, int dtype) {
    Pass p;
    if (is_diagonal(g)) {
        HostGate s = sorted_targets(g);
        p.kind = PASS_DIAG;
        p.k = s.k;
        for (int b = 0; b < s.k; ++b) p.targets[b] = s.targets[b];
        const int d = 1 << s.k;
        p.M.resize(d);
        for (int j = 0; j < d; ++j) p.M[j] = s.M[j * d + j];
        p.bytes = diag_bytes(s, n, dtype);
        p.flops = 6.0 * p.bytes / (2.0 * double(amp_bytes(dtype)));
        return p;
    }
    HostGate red;
    int ctrls[QSIM_MAX_K];
    const int nc = extract_controls(g, red, ctrls);
    HostGate s = sorted_targets(red);
    p.kind = PASS_DENSE;
    p.k = s.k;
    for (int b = 0; b < s.k; ++b) p.targets[b] = s.targets[b];
    p.nctrl = nc;
    std::sort(ctrls, ctrls + nc);
    for (int i = 0; i < nc; ++i) p.ctrls[i] = ctrls[i];
    p.M = s.M;
    p.bytes = 2.0 * std::ldexp(1.0, n - nc) * double(amp_bytes(dtype));
    p.flops = 8.0 * double(1 << s.k) * std::ldexp(1.0, n - nc);
    return p;
}

bool build_reg_program(Plan &plan, Pass &p, uint64_t q, const int *local_of,
                       const std::vector<const HostGate *> &gates);

// Dense block on k >= 4 qubits as a real-embedded matrix product:
// B = [[Re U^T, Im U^T], [-Im U^T, Re U^T]] (2D x 2D, row-major).
static Pass mfma_pass(Plan &plan, const HostGate &g) {
    const HostGate s = sorted_targets(g);
    Pass p;
    p.kind = PASS_MFMA;
    p.k = s.k;
    for (int b = 0; b < s.k; ++b) p.targets[b] = s.targets[b];
    const int D = 1 << s.k, W = 2 * D;
    p.pool_begin = int(plan.real_pool.size());
    plan.real_pool.resize(plan.real_pool.size() + size_t(W) * W);
    double *B = plan.real_pool.data() + p.pool_begin;
    for (int c = 0; c < D; ++c)
        for (int j = 0; j < D; ++j) {
            const cd u = s.M[size_t(c) * D + j];
            B[size_t(j) * W + c] = u.real();
            B[size_t(D + j) * W + c] = -u.imag();
            B[size_t(j) * W + D + c] = u.imag();
            B[size_t(D + j) * W + D + c] = u.real();
        }
    p.pool_end = int(plan.real_pool.size());
    p.bytes = 2.0 * std::ldexp(1.0, plan.n) * double(amp_bytes(plan.dtype));
    p.flops = 8.0 * double(D) * std::ldexp(1.0, plan.n);
    return p;
}

struct TileBuilder {
    int n, dtype, m, L;
    bool reg;
    int tiles = 1;   // state tiles a pass keeps in LDS (2 in adjoint passes)
    Plan &plan;
    // `low`: qubits 0 .. low - 1 are in every tile (0: the precision's default)
    TileBuilder(Plan &p, int n_, int dt, int m_, bool reg_, int low = 0)
        : n(n_), dtype(dt), m(m_), L(0), reg(reg_), plan(p) {
        L = std::min(m, low > 0 ? low : low_tile_qubits(dt));
    }

    // Adds a tile pass over qubit set `q` (must contain the low L qubits)
    // holding the given gates, in order.  With `need_reg` the pass must run
    // as a register program (it holds controlled gates whose controls lie
    // outside the tile); if it cannot, nothing is added and false returned.
    bool emit(uint64_t q, const std::vector<const HostGate *> &gs, bool need_reg = false) {
        Pass p;
        p.kind = PASS_TILE;
        p.m = m;
        p.L = L;
        // pad the tile with the lowest unused qubits (longer contiguous runs)
        for (int b = 0; b < n && __builtin_popcountll(q) < m; ++b) q |= 1ull << b;
        int local_of[64];
        int nl = 0;
        for (int b = 0; b < L; ++b) local_of[b] = nl++;
        for (int b = L; b < n; ++b)
            if ((q >> b) & 1) {
                p.hpos.push_back(b);
                local_of[b] = nl++;
            }
        p.op_begin = int(plan.tile_ops.size());
        p.pool_begin = int(plan.tile_pool.size());
        p.bytes = 2.0 * std::ldexp(1.0, n) * double(amp_bytes(dtype));
        p.logical_gates = int(gs.size());
        // arithmetic of the gates as the pass applies them
        auto pass_flops = [&](bool regform) {
            double f = 0.0;
            const double N = std::ldexp(1.0, n);
            for (const HostGate *g : gs) {
                if (g->probe_gen) continue;
                if (g->rot_gen) {
                    f += 16.0 * N;
                    continue;
                }
                const int d = 1 << g->k;
                if (!is_diagonal(*g) && g->k > 1) {
                    HostGate red;
                    int ctl[QSIM_MAX_K];
                    const int nc = extract_controls(*g, red, ctl);
                    if (red.k == 1) {
                        // a controlled one-qubit block: a complex 2 x 2 product
                        // where the controls are 1 (register programs move the
                        // values of a permutation without arithmetic)
                        const bool perm = red.M[0] == cd(0.0) && red.M[3] == cd(0.0) &&
                                          red.M[1] == cd(1.0) && red.M[2] == cd(1.0);
                        if (!perm || !regform) f += 16.0 * std::ldexp(1.0, n - nc);
                        continue;
                    }
                }
                if (g->rot_real && regform) {
                    // three multiply-adds per component and pair; the input
                    // phase multiplies half the amplitudes
                    if (g->rot_real == 1) f += 6.0 * N;
                    if (g->phase_in != cd(1.0)) f += 3.0 * N;
                } else if (is_diagonal(*g)) {
                    int nonunit = 0;
                    for (int j = 0; j < d; ++j)
                        if (g->M[size_t(j) * d + j] != cd(1.0)) ++nonunit;
                    f += 6.0 * double(nonunit) * std::ldexp(1.0, n - g->k);
                } else {
                    f += 8.0 * double(d) * N;
                }
            }
            return f;
        };
        if (reg) {
            const size_t nrop = plan.reg_ops.size(), nst = plan.reg_stages.size(), npool = plan.tile_pool.size();
            if (build_reg_program(plan, p, q, local_of, gs)) {
                p.op_end = p.op_begin;
                p.flops = pass_flops(true);
                plan.passes.push_back(std::move(p));
                return true;
            }
            plan.reg_ops.resize(nrop);
            plan.reg_stages.resize(nst);
            plan.tile_pool.resize(npool);
            p.reg_r = 0;
        }
        if (need_reg) return false;
        p.flops = pass_flops(false);
        for (const HostGate *g : gs) {
            TileOp op{};
            if (g->probe_gen) {
                op.type = 3;
                op.k = 1;
                op.kin = g->probe_gen;
                op.pos[0] = local_of[g->targets[0]];
                op.moff = g->probe_slot;
                plan.tile_ops.push_back(op);
                continue;
            }
            if (g->rot_gen) {
                op.type = 4;
                op.k = 1;
                op.kin = g->rot_gen;
                op.pos[0] = local_of[g->targets[0]];
                op.moff = g->rot_param;
                op.jbit[0] = g->rot_inv;
                plan.tile_ops.push_back(op);
                continue;
            }
            HostGate s = sorted_targets(*g);
            op.k = s.k;
            op.moff = int(plan.tile_pool.size()) - p.pool_begin;
            const int d = 1 << s.k;
            if (is_diagonal(s)) {
                op.type = 1;
                int nin = 0, nout = 0;
                // targets are ascending globally, hence ascending locally too
                for (int b = 0; b < s.k; ++b) {
                    const int t = s.targets[b];
                    if ((q >> t) & 1) {
                        op.pos[nin] = local_of[t];
                        op.jbit[nin] = b;
                        ++nin;
                    } else {
                        op.gpos[nout] = t;
                        op.gbit[nout] = b;
                        ++nout;
                    }
                }
                op.kin = nin;
                for (int j = 0; j < d; ++j) plan.tile_pool.push_back(s.M[j * d + j]);
            } else {
                // a one-qubit block under controls (all inside the tile here)
                // touches only the pairs where the controls are 1
                HostGate red;
                int ctl[QSIM_MAX_K];
                const int nc = s.k > 1 ? extract_controls(s, red, ctl) : 0;
                bool controlled = nc > 0 && red.k == 1 && ((q >> red.targets[0]) & 1);
                for (int c = 0; c < nc && controlled; ++c) controlled = (q >> ctl[c]) & 1;
                if (controlled) {
                    op.type = 5;
                    op.k = 1;
                    op.pos[0] = local_of[red.targets[0]];
                    for (int c = 0; c < nc; ++c) op.kin |= 1 << local_of[ctl[c]];
                    plan.tile_pool.insert(plan.tile_pool.end(), red.M.begin(), red.M.end());
                } else {
                    op.type = 0;
                    op.kin = s.k;
                    for (int b = 0; b < s.k; ++b) op.pos[b] = local_of[s.targets[b]];
                    plan.tile_pool.insert(plan.tile_pool.end(), s.M.begin(), s.M.end());
                }
            }
            plan.tile_ops.push_back(op);
        }
        p.op_end = int(plan.tile_ops.size());
        p.pool_end = int(plan.tile_pool.size());
        plan.passes.push_back(std::move(p));
        return true;
    }
};

// Greedy grouping of ops into tile passes in dependency order: an op joins
// the pass if the qubits it needs in the tile fit (diagonal ops always fit);
// an op that does not fit blocks its qubits for the rest of the pass.  When
// the pass runs as a register program, a one-qubit block under exact
// controls needs only its target in the tile (its controls become lane and
// block masks); a pass that then fails to become a register program is
// grouped again with every qubit of such ops in the tile.
// At most this many ops per pass, so that a pass's op list and matrices stay
// well inside the LDS next to its tile(s).
static const size_t kMaxOpsPerPass = 128;

// Smallest tile that holds every gate next to the low L qubits: a gate whose
// qubits lie outside the low L needs L + (those qubits) tile positions.
static int tile_m_for(const std::vector<HostGate> &gates, int m, int n, int dtype, int nlow = 0) {
    const int L = std::min(m, nlow > 0 ? nlow : low_tile_qubits(dtype));
    const uint64_t low = (1ull << L) - 1;
    int need = m;
    for (const HostGate &g : gates)
        if (!is_diagonal(g)) need = std::max(need, L + __builtin_popcountll(qmask(g) & ~low));
    return std::min(n, need);
}

// Returns false if some gate could not be placed in any pass (the caller
// reports an error rather than applying part of the circuit).
static bool group_tiles(TileBuilder &tb, const std::vector<HostGate> &gates) {
    const uint64_t low = (1ull << tb.L) - 1;
    const int r = tb.m - 8;
    const bool reg_ctl = tb.reg && r >= 3 && r <= kRegBitsMax;
    const size_t ng = gates.size();
    std::vector<uint64_t> full(ng), target(ng);
    std::vector<char> diag(ng), wide(ng);
    // matrix entries a gate adds to the pass pool when the pass runs from
    // LDS (diagonal: 2^k; one-qubit block under controls: 4; dense: 4^k)
    std::vector<size_t> pool(ng);
    for (size_t i = 0; i < ng; ++i) {
        const HostGate &g = gates[i];
        full[i] = target[i] = qmask(g);
        diag[i] = is_diagonal(g);
        const size_t d = size_t(1) << g.k;
        pool[i] = diag[i] ? d : d * d;
        if (!diag[i] && g.k > 1) {
            HostGate red;
            int ctl[QSIM_MAX_K];
            extract_controls(g, red, ctl);
            if (red.k == 1) {
                pool[i] = 4;
                if (reg_ctl) target[i] = 1ull << red.targets[0];
            }
        }
        if (g.probe_gen || g.rot_gen) pool[i] = 0;
        // dense on more than three qubits: no register program holds it
        wide[i] = !diag[i] && target[i] == full[i] && g.k > 3;
    }
    // An LDS pass holds its tile(s), op list and pool in one workgroup's LDS
    // (160 KiB on gfx950): the ops and matrices a pass takes are bounded by
    // what is left next to the tile(s).
    const size_t lds_cap = size_t(160) * 1024;
    const size_t tile_lds = size_t(tb.tiles) * (amp_bytes(tb.dtype) << tb.m);
    const size_t pool_cap = lds_cap > tile_lds + kMaxOpsPerPass * sizeof(TileOp)
                                ? (lds_cap - tile_lds - kMaxOpsPerPass * sizeof(TileOp)) / amp_bytes(tb.dtype)
                                : 0;
    std::vector<char> done(ng, 0);
    size_t remaining = ng;
    size_t first = 0;
    while (remaining) {
        while (done[first]) ++first;
        bool placed = false;
        for (int attempt = 0; attempt < 2 && !placed; ++attempt) {
            const bool relax = reg_ctl && attempt == 0;
            uint64_t q = low;
            uint64_t blocked = 0;
            bool any_relaxed = false, any_wide = false;
            std::vector<size_t> idx;
            size_t pooled = 0;
            for (size_t i = first; i < ng && idx.size() < kMaxOpsPerPass; ++i) {
                if (done[i]) continue;
                // the pass's matrices would outgrow the LDS next to its tile:
                // the gates from here on go to later passes (the first gate
                // of a pass is always taken; its launch checks the limit)
                if (!idx.empty() && pooled + pool[i] > pool_cap) break;
                const uint64_t gm = full[i];
                if ((gm & blocked) || (wide[i] && any_relaxed)) {
                    blocked |= gm;
                    continue;
                }
                const uint64_t need = diag[i] ? 0 : (relax && !any_wide ? target[i] : gm);
                if (diag[i] || __builtin_popcountll(q | need) <= tb.m) {
                    q |= need;
                    idx.push_back(i);
                    pooled += pool[i];
                    any_relaxed |= !diag[i] && need != gm;
                    any_wide |= bool(wide[i]);
                } else {
                    blocked |= gm;
                }
            }
            if (idx.empty()) return false;   // the tile cannot hold the gate at `first`
            std::vector<const HostGate *> chosen;
            for (size_t i : idx) chosen.push_back(&gates[i]);
            if (!tb.emit(q, chosen, any_relaxed)) continue;
            for (size_t i : idx) done[i] = 1;
            remaining -= idx.size();
            placed = true;
        }
        if (!placed) return false;
    }
    return true;
}

int build_tile_plan(Plan &plan, const std::vector<HostGate> &items, int tile_m, int tiles, bool reg) {
    const int m = tile_m_for(items, std::min(plan.n, tile_m), plan.n, plan.dtype);
    TileBuilder tb(plan, plan.n, plan.dtype, m, reg);
    tb.tiles = tiles;
    plan.items = int(items.size());
    return group_tiles(tb, items) ? m : -1;
}

int build_adjoint_plan(Plan &plan, const std::vector<HostGate> &items, int tile_m) {
    const int m = build_tile_plan(plan, items, tile_m, 2);
    for (Pass &p : plan.passes) p.bytes *= 2.0;   // two states per pass
    return m;
}

bool build_plan(Plan &plan, const std::vector<HostGate> &gates_in, const PlanOptions &po) {
    const int n = plan.n, dtype = plan.dtype;
    std::vector<HostGate> gates = fuse_gates(gates_in, po.fuse_k);
    const int per_block = int(gates_in.size());
    (void)per_block;

    if (po.tile_m < 0) {
        for (const HostGate &g : gates) {
            HostGate red;
            int ctrls[QSIM_MAX_K];
            const bool diag = is_diagonal(g);
            const int nc = diag ? 0 : extract_controls(g, red, ctrls);
            int tlow = 64;
            for (int b = 0; b < red.k && !diag; ++b) tlow = std::min(tlow, red.targets[b]);
            // up to three targets and no controls (complex64): a sweep whose
            // waves exchange partner amplitudes between lanes
            Pass lane;
            if (!diag) lane = sweep_pass(g, n, dtype);
            if (!diag && lane_sweep_ok(dtype, n, lane)) {
                plan.passes.push_back(std::move(lane));
            } else if (!diag && po.reg_tiles && g.k <= 3 && g.k - nc >= 2 && tlow <= 2 && n >= default_tile_m(dtype)) {
                // two or more targets among the lowest qubits: a sweep's
                // threads would each gather a few adjacent amplitudes with
                // strided accesses; a one-gate register tile reads whole
                // lines and applies the gate on register bits
                TileBuilder tb(plan, n, dtype, default_tile_m(dtype), true);
                tb.emit(((1ull << tb.L) - 1) | qmask(g), {&g});
            } else if (diag || g.k - nc <= 3) {
                plan.passes.push_back(sweep_pass(g, n, dtype));
            } else if (po.use_mfma >= 0) {
                plan.passes.push_back(mfma_pass(plan, g));
            } else {
                // wide dense block: a one-gate tile pass over its qubits
                TileBuilder tb(plan, n, dtype, std::min(n, default_tile_m(dtype)), false);
                uint64_t q = (1ull << tb.L) - 1;
                q |= qmask(g);
                tb.emit(q, {&g});
            }
        }
    } else {
        if (po.reg_tiles && po.split_1q) gates = split_single_qubit(gates, n);
        // Every tile holds the low qubits, so every HBM access runs over
        // 2^low consecutive amplitudes.  The default width (256 bytes) and
        // one more qubit (512 bytes) are both planned; the plan with fewer
        // passes is kept (the wider one on a tie).  Which is fewer depends
        // on the circuit: on the 5 x 6 grid the wider block is the grid's
        // first row, and 2^12 tiles take 17 passes instead of 21.
        // (plans are copied here before any upload: no device buffer yet)
        if (plan.dev) return false;
        const Plan shell = plan;
        bool have = false;
        for (int low : {low_tile_qubits(dtype) + 1, low_tile_qubits(dtype)}) {
            Plan trial = shell;
            TileBuilder tb(trial, n, dtype, tile_m_for(gates, po.tile_m, n, dtype, low), po.reg_tiles, low);
            trial.items = int(gates.size());
            if (!group_tiles(tb, gates)) continue;
            if (!have || trial.passes.size() < plan.passes.size()) {
                plan = std::move(trial);
                have = true;
            }
        }
        return have;
    }
    // logical gate counts for sweep passes
    plan.items = int(gates.size());
    for (Pass &p : plan.passes)
        if (p.kind != PASS_TILE) p.logical_gates = 1;
    return true;
}

}  // namespace qsim
