// Host side of register-staged tile passes: splits a tile pass's gates into
// stages whose dense gates act on the stage's register bits, and builds the
// XOR-swizzled LDS address maps of the exchanges between stages.
#include <algorithm>
#include <tuple>
#include <mutex>
#include <map>
#include <array>
#include <cstring>

#include "qsim_internal.h"

namespace qsim {

namespace {

struct LocalGate {
    const HostGate *g;      // targets ascending (sorted_targets form)
    bool diag;
    uint32_t lmask;         // tile-local positions the stage must hold in registers
    uint64_t qmask;         // global qubits
    // a one-qubit gate under exact controls (CX, CCX, ...): `red` is the 2 x 2
    // block it applies where every control is 1; only its target needs a
    // register bit, the controls may sit anywhere
    const HostGate *red = nullptr;
    int nctl = 0;
    int ctl[QSIM_MAX_K] = {};
};

int popc(uint64_t v) { return __builtin_popcountll(v); }

// Rank over GF(2) of a set of bit vectors.
int gf2_rank(uint32_t *v, int n) {
    int rank = 0;
    for (int bit = 31; bit >= 0 && rank < n; --bit) {
        int piv = -1;
        for (int i = rank; i < n; ++i)
            if ((v[i] >> bit) & 1u) { piv = i; break; }
        if (piv < 0) continue;
        std::swap(v[rank], v[piv]);
        for (int i = 0; i < n; ++i)
            if (i != rank && ((v[i] >> bit) & 1u)) v[i] ^= v[rank];
        ++rank;
    }
    return rank;
}

// Number of bank constraints a thread layout satisfies under address map
// `addr` (amplitude units): the lanes of each group of 2^g consecutive lanes
// (g = wb - 1 and g = wb) must fall in distinct bank slots, i.e. the low g
// bits of their address vectors must be independent.
int bank_score(const int *T, const uint32_t *addr, int wb) {
    int score = 0;
    for (int g = wb - 1; g <= wb; ++g) {
        uint32_t v[8];
        for (int b = 0; b < g; ++b) v[b] = addr[T[b]] & ((1u << g) - 1u);
        if (gf2_rank(v, g) == g) ++score;
    }
    return score;
}

void split_layout(uint32_t R, int m, int *Rpos, int *Tpos) {
    int nr = 0, nt = 0;
    for (int p = 0; p < m; ++p) {
        if ((R >> p) & 1u)
            Rpos[nr++] = p;
        else
            Tpos[nt++] = p;
    }
}

// Random search over swizzles of the positions that are low lane bits of
// either layout, keeping the one that satisfies the most bank constraints.
// On 12-qubit tiles with four register bits the best score over 16384
// attempts is already reached within the first 64 for every pair of
// register sets sampled, so the search stops there.
std::array<uint32_t, 16> search_swizzle(int m, int wb, const int *Twp, const int *Trp, uint64_t seed) {
    // Only positions that are among the low lane bits of either layout
    // decide bank conflicts.  Every other position keeps its plain bit, so
    // the register parts of the addresses mostly stay clear of the bits the
    // thread part can set and the kernel adds them as constant offsets.
    uint32_t lanes = 0;
    for (int b = 0; b < wb; ++b) lanes |= (1u << Twp[b]) | (1u << Trp[b]);
    uint32_t best[16] = {};
    int best_score = -1;
    uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
    for (int attempt = 0; attempt < 64 && best_score < 4; ++attempt) {
        uint32_t addr[16];
        for (int p = 0; p < m; ++p) {
            uint32_t sw = 0;
            if (p >= wb && attempt > 0 && ((lanes >> p) & 1u)) {
                x ^= x << 13; x ^= x >> 7; x ^= x << 17;
                sw = uint32_t(x) & ((1u << wb) - 1u);
            }
            addr[p] = (1u << p) ^ sw;
        }
        const int sc = bank_score(Twp, addr, wb) + bank_score(Trp, addr, wb);
        if (sc > best_score) {
            best_score = sc;
            std::memcpy(best, addr, sizeof(uint32_t) * m);
        }
    }
    std::array<uint32_t, 16> out{};
    std::memcpy(out.data(), best, sizeof(uint32_t) * 16);
    return out;
}

// Swizzles found so far, by (tile qubits, bank-slot bits, writing register
// set, reading register set): the search costs far more than the rest
// of planning, and the same pairs of register sets recur across passes and
// plans (a parameter sweep re-plans the same circuit structure every call).
std::mutex g_swizzle_mu;
std::map<std::tuple<int, int, uint32_t, uint32_t>, std::array<uint32_t, 16>> g_swizzles;

// Picks the XOR swizzle of one exchange so that both the writing and the
// reading layout access LDS without bank conflicts where possible.  The
// search is seeded from its key, so a plan's layout does not depend on what
// was planned before it.
void make_exchange(int m, int wb, uint32_t Rw, uint32_t Rr, RegStage &st) {
    int Rwp[kRegBitsMax], Twp[16], Rrp[kRegBitsMax], Trp[16];
    split_layout(Rw, m, Rwp, Twp);
    split_layout(Rr, m, Rrp, Trp);
    const int r = popc(Rw);
    const auto key = std::make_tuple(m, wb, Rw, Rr);
    std::array<uint32_t, 16> found{};
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_swizzle_mu);
        auto it = g_swizzles.find(key);
        if (it != g_swizzles.end()) {
            found = it->second;
            have = true;
        }
    }
    if (!have) {
        found = search_swizzle(m, wb, Twp, Trp, (uint64_t(Rw) << 32) ^ (uint64_t(Rr) << 8) ^ uint64_t(m));
        std::lock_guard<std::mutex> lk(g_swizzle_mu);
        g_swizzles.emplace(key, found);
    }
    const uint32_t *best = found.data();
    for (int b = 0; b < 8; ++b) {
        st.wr_t[b] = best[Twp[b]];
        st.rd_t[b] = best[Trp[b]];
    }
    for (int b = 0; b < kRegBitsMax; ++b) {
        st.wr_r[b] = b < r ? best[Rwp[b]] : 0u;
        st.rd_r[b] = b < r ? best[Rrp[b]] : 0u;
    }
}

int index_in(const int *arr, int n, int v) {
    for (int i = 0; i < n; ++i)
        if (arr[i] == v) return i;
    return -1;
}

// Next register set: the positions of the first dense gates (in dependency
// order) that fit r bits together.
uint32_t next_register_set(const std::vector<LocalGate> &gs, const std::vector<char> &done, int r) {
    uint32_t R = 0;
    uint64_t blocked = 0;
    for (size_t i = 0; i < gs.size(); ++i) {
        if (done[i]) continue;
        const LocalGate &lg = gs[i];
        if (lg.qmask & blocked) {
            blocked |= lg.qmask;
            continue;
        }
        if (lg.diag) continue;
        if (popc(R | lg.lmask) <= r)
            R |= lg.lmask;
        else
            blocked |= lg.qmask;
    }
    return R;
}

// Pads R to r positions with the highest unused positions (keeping the low
// positions on thread bits, where consecutive lanes read consecutive
// addresses).
uint32_t pad_high(uint32_t R, int r, int m) {
    for (int p = m - 1; p >= 0 && popc(R) < r; --p) R |= 1u << p;
    return R;
}

}  // namespace

bool build_reg_program(Plan &plan, Pass &p, uint64_t q, const int *local_of,
                       const std::vector<const HostGate *> &gates) {
    const int m = p.m;
    const int r = m - 8;
    if (r < 3 || r > kRegBitsMax) return false;
    const int wb = plan.dtype == QSIM_C128 ? 4 : 5;
    const int nlow = std::min(6, m - r);   // lane positions that should stay on thread bits for HBM access

    std::vector<HostGate> sorted, reduced;
    sorted.reserve(gates.size());
    reduced.reserve(gates.size());
    std::vector<LocalGate> gs;
    // (rotations formed on the device and gradient probes act on one qubit
    // and carry no matrix: kept as they are)
    for (const HostGate *g : gates) sorted.push_back(g->rot_gen || g->probe_gen ? *g : sorted_targets(*g));
    for (const HostGate &s : sorted) {
        LocalGate lg{&s, is_diagonal(s), 0u, 0ull};
        // Z rotations and Z probes are diagonal: any position will do
        if (s.rot_gen == 3 || s.probe_gen == 3) lg.diag = true;
        for (int b = 0; b < s.k; ++b) {
            lg.qmask |= 1ull << s.targets[b];
            if ((q >> s.targets[b]) & 1) lg.lmask |= 1u << local_of[s.targets[b]];
        }
        if (!lg.diag && s.k > 1) {
            HostGate red;
            const int nc = extract_controls(s, red, lg.ctl);
            if (red.k == 1) {
                if (!((q >> red.targets[0]) & 1)) return false;
                reduced.push_back(std::move(red));
                lg.red = &reduced.back();
                lg.nctl = nc;
                lg.lmask = 1u << local_of[lg.red->targets[0]];
            }
        }
        if (!lg.diag && !lg.red && s.k > 3) return false;
        if (!lg.diag && !lg.red && (lg.qmask & ~q)) return false;   // every target must be in the tile
        gs.push_back(lg);
    }
    const uint32_t lowmask = (1u << nlow) - 1u;
    const uint32_t top = pad_high(0, r, m);

    std::vector<char> done(gs.size(), 0);
    std::vector<std::pair<uint32_t, std::vector<int>>> stages;
    uint32_t R = pad_high(next_register_set(gs, done, r), r, m);
    if (R & lowmask) R = top;   // load with lanes on the low positions, exchange after
    size_t remaining = gs.size();
    for (int guard = 0; guard < 4 * int(gs.size()) + 4; ++guard) {
        std::vector<int> chosen;
        uint64_t blocked = 0;
        for (size_t i = 0; i < gs.size(); ++i) {
            if (done[i]) continue;
            const LocalGate &lg = gs[i];
            if (lg.qmask & blocked) {
                blocked |= lg.qmask;
                continue;
            }
            if (lg.diag || (lg.lmask & ~R) == 0) {
                chosen.push_back(int(i));
                done[i] = 1;
                --remaining;
            } else {
                blocked |= lg.qmask;
            }
        }
        stages.push_back({R, chosen});
        if (!remaining) break;
        R = pad_high(next_register_set(gs, done, r), r, m);
    }
    if (remaining) return false;
    if (stages.back().first & lowmask) stages.push_back({top, {}});

    // emit
    p.reg_r = r;
    p.rop_begin = int(plan.reg_ops.size());
    p.stage_begin = int(plan.reg_stages.size());
    // local position -> global qubit
    int gpos_of_local[16];
    for (int b = 0; b < 64; ++b)
        if ((q >> b) & 1) gpos_of_local[local_of[b]] = b;
    auto set_layout_globals = [&](uint32_t Rm, int8_t *gt, int8_t *gr) {
        int Rp[kRegBitsMax], Tp[16];
        split_layout(Rm, m, Rp, Tp);
        for (int b = 0; b < 8; ++b) gt[b] = int8_t(gpos_of_local[Tp[b]]);
        for (int b = 0; b < r; ++b) gr[b] = int8_t(gpos_of_local[Rp[b]]);
    };
    set_layout_globals(stages.front().first, p.ld_t, p.ld_r);
    set_layout_globals(stages.back().first, p.st_t, p.st_r);

    uint32_t prevR = 0;
    for (size_t si = 0; si < stages.size(); ++si) {
        const uint32_t Rm = stages[si].first;
        RegStage st{};
        if (si > 0) make_exchange(m, wb, prevR, Rm, st);
        int Rp[kRegBitsMax], Tp[16];
        split_layout(Rm, m, Rp, Tp);
        for (int b = 0; b < 8; ++b) st.q_t[b] = int8_t(gpos_of_local[Tp[b]]);
        for (int b = 0; b < kRegBitsMax; ++b) st.q_r[b] = int8_t(b < r ? gpos_of_local[Rp[b]] : -1);
        st.op_begin = int(plan.reg_ops.size()) - p.rop_begin;
        // input phases of split rotations whose register bit no earlier op of
        // the stage changes commute to the stage's start, where they merge
        // into one table over the register bits
        std::vector<cd> table(size_t(1) << r, cd(1.0));
        bool use_table = false;
        uint32_t touched = 0;
        std::vector<RegOp> sops;
        auto pool_off = [&]() { return int(plan.tile_pool.size()) - p.pool_begin; };
        const std::vector<int> &sg = stages[si].second;
        // register bit a gate acts on non-diagonally (-1: none / several)
        auto rot_bit = [&](int gi) {
            const LocalGate &lg = gs[size_t(gi)];
            return (!lg.diag && lg.g->rot_real) ? index_in(Rp, r, local_of[lg.g->targets[0]]) : -1;
        };
        auto nondiag_mask = [&](int gi) {
            const LocalGate &lg = gs[size_t(gi)];
            uint32_t mk = 0;
            if (lg.diag) return mk;
            if (lg.red) return 1u << index_in(Rp, r, local_of[lg.red->targets[0]]);
            for (int b = 0; b < lg.g->k; ++b) mk |= 1u << index_in(Rp, r, local_of[lg.g->targets[b]]);
            return mk;
        };
        std::vector<char> phase_done(sg.size(), 0);
        for (size_t pos = 0; pos < sg.size(); ++pos) {
            const int gi = sg[pos];
            const LocalGate &lg = gs[size_t(gi)];
            const HostGate &s = *lg.g;
            if (s.rot_gen || s.probe_gen) {
                // batched circuits: rotation exp(-i theta G / 2) with theta
                // the circuit's parameter moff (type 8), or the probe
                // Im <lambda|G|psi> into gradient slot moff (type 9); G = X,
                // Y, Z for rj[0] = 1, 2, 3; jmatch 1 inverts the rotation.
                // X and Y act on a register bit, Z on a register, thread or
                // out-of-tile bit.
                RegOp op{};
                op.type = s.rot_gen ? 8 : 9;
                op.k = 1;
                op.moff = s.rot_gen ? s.rot_param : s.probe_slot;
                op.rj[0] = s.rot_gen ? s.rot_gen : s.probe_gen;
                op.jmatch = s.rot_inv;
                const int t = s.targets[0];
                if ((q >> t) & 1) {
                    const int lp = local_of[t];
                    const int ri = index_in(Rp, r, lp);
                    if (ri >= 0) {
                        op.rb[0] = ri;
                        op.rmask = 1 << ri;
                        op.nreg = 1;
                    } else {
                        op.tb[0] = int32_t(1u << index_in(Tp, 8, lp));
                        op.nthr = 1;
                    }
                } else {
                    op.gp[0] = int32_t(uint32_t(1ull << t));
                    op.gp[1] = int32_t(uint32_t((1ull << t) >> 32));
                    op.nout = 1;
                }
                if (op.rj[0] != 3 && op.nreg != 1) return false;
                if (op.nreg) touched |= uint32_t(op.rmask);
                sops.push_back(op);
                continue;
            }
            if (!lg.diag && s.rot_real) {
                const int ri = index_in(Rp, r, local_of[s.targets[0]]);
                if (s.phase_in != cd(1.0) && !phase_done[pos]) {
                    if (!((touched >> ri) & 1u)) {
                        for (size_t i = 0; i < table.size(); ++i)
                            if ((i >> ri) & 1u) table[i] *= s.phase_in;
                        use_table = true;
                    } else {
                        // later rotations whose phases may move up to here:
                        // their bit is already changed in this stage and no
                        // op in between acts on it non-diagonally
                        std::vector<size_t> group{pos};
                        uint32_t blocked = 1u << ri;
                        for (size_t q2 = pos + 1; q2 < sg.size(); ++q2) {
                            const int c = rot_bit(sg[q2]);
                            const HostGate &h = *gs[size_t(sg[q2])].g;
                            if (c >= 0 && h.phase_in != cd(1.0) && !phase_done[q2] && ((touched >> c) & 1u) &&
                                !((blocked >> c) & 1u))
                                group.push_back(q2);
                            blocked |= nondiag_mask(sg[q2]);
                        }
                        if (group.size() >= 2) {
                            // one table over the register bits for all of them
                            std::vector<cd> mid(size_t(1) << r, cd(1.0));
                            for (size_t gq : group) {
                                const int c = rot_bit(sg[gq]);
                                const cd ph = gs[size_t(sg[gq])].g->phase_in;
                                for (size_t i = 0; i < mid.size(); ++i)
                                    if ((i >> c) & 1u) mid[i] *= ph;
                                phase_done[gq] = 1;
                            }
                            RegOp t{};
                            t.type = 4;
                            t.k = r;
                            t.moff = pool_off();
                            plan.tile_pool.insert(plan.tile_pool.end(), mid.begin(), mid.end());
                            sops.push_back(t);
                        } else {
                            RegOp ph{};
                            ph.type = 6;
                            ph.k = 1;
                            ph.moff = pool_off();
                            plan.tile_pool.push_back(s.phase_in);
                            ph.rmask = 1 << ri;
                            sops.push_back(ph);
                        }
                    }
                }
                RegOp op{};
                op.k = 1;
                op.rmask = 1 << ri;
                op.rb[0] = ri;
                op.moff = pool_off();
                if (s.rot_real == 1) {
                    // lifting: x0 += p x1; x1 += u x0; x0 += p x1 gives
                    // [[c, -s], [s, c]] for p = -s / (1 + c), u = s
                    op.type = 3;
                    plan.tile_pool.push_back(cd(-s.rot_s / (1.0 + s.rot_c), s.rot_s));
                } else {
                    op.type = 5;
                    plan.tile_pool.push_back(cd(0.0));
                }
                sops.push_back(op);
                touched |= 1u << ri;
                continue;
            }
            (void)pos;
            if (lg.red) {
                // controlled one-qubit block: target on a register bit,
                // controls as register, thread and out-of-tile masks
                RegOp op{};
                op.type = 7;
                op.k = 1;
                op.rb[0] = index_in(Rp, r, local_of[lg.red->targets[0]]);
                // jmatch 1: the block is X, an exchange without arithmetic
                const std::vector<cd> &B = lg.red->M;
                op.jmatch = B[0] == cd(0.0) && B[1] == cd(1.0) && B[2] == cd(1.0) && B[3] == cd(0.0);
                op.moff = pool_off();
                plan.tile_pool.insert(plan.tile_pool.end(), lg.red->M.begin(), lg.red->M.end());
                uint32_t tmask = 0;
                uint64_t gmask = 0;
                for (int c = 0; c < lg.nctl; ++c) {
                    const int qc = lg.ctl[c];
                    if ((q >> qc) & 1) {
                        const int lp = local_of[qc];
                        const int ri = index_in(Rp, r, lp);
                        if (ri >= 0)
                            op.rmask |= 1 << ri;
                        else
                            tmask |= 1u << index_in(Tp, 8, lp);
                    } else {
                        gmask |= 1ull << qc;
                    }
                }
                op.tb[0] = int32_t(tmask);
                op.gp[0] = int32_t(uint32_t(gmask));
                op.gp[1] = int32_t(uint32_t(gmask >> 32));
                touched |= 1u << op.rb[0];
                sops.push_back(op);
                continue;
            }
            RegOp op{};
            op.k = s.k;
            op.moff = int(plan.tile_pool.size()) - p.pool_begin;
            const int d = 1 << s.k;
            if (!lg.diag) {
                op.type = 0;
                for (int b = 0; b < s.k; ++b) op.rmask |= 1 << index_in(Rp, r, local_of[s.targets[b]]);
                touched |= uint32_t(op.rmask);
                plan.tile_pool.insert(plan.tile_pool.end(), s.M.begin(), s.M.end());
            } else {
                int nonunit = 0, last = -1;
                for (int j = 0; j < d; ++j) {
                    const cd v = s.M[size_t(j) * d + j];
                    plan.tile_pool.push_back(v);
                    if (v != cd(1.0)) { ++nonunit; last = j; }
                }
                op.type = nonunit == 1 ? 2 : 1;
                op.jmatch = last;
                for (int b = 0; b < s.k; ++b) {
                    const int t = s.targets[b];
                    if ((q >> t) & 1) {
                        const int lp = local_of[t];
                        const int ri = index_in(Rp, r, lp);
                        if (ri >= 0) {
                            op.rb[op.nreg] = ri;
                            op.rj[op.nreg] = b;
                            op.rmask |= 1 << ri;
                            ++op.nreg;
                        } else {
                            op.tb[op.nthr] = index_in(Tp, 8, lp);
                            op.tj[op.nthr] = b;
                            ++op.nthr;
                        }
                    } else {
                        op.gp[op.nout] = t;
                        op.gj[op.nout] = b;
                        ++op.nout;
                    }
                }
                if (nonunit == 1 && last == d - 1) {
                    // the all-ones entry (CZ, CP, CCZ, phase gates): masks
                    // instead of index arithmetic
                    RegOp f{};
                    f.type = 6;
                    f.k = s.k;
                    f.moff = op.moff + last;
                    uint32_t tmask = 0;
                    uint64_t gmask = 0;
                    for (int b = 0; b < op.nreg; ++b) f.rmask |= 1 << op.rb[b];
                    for (int b = 0; b < op.nthr; ++b) tmask |= 1u << op.tb[b];
                    for (int b = 0; b < op.nout; ++b) gmask |= 1ull << op.gp[b];
                    f.tb[0] = int32_t(tmask);
                    f.gp[0] = int32_t(uint32_t(gmask));
                    f.gp[1] = int32_t(uint32_t(gmask >> 32));
                    op = f;
                }
            }
            sops.push_back(op);
        }
        if (use_table) {
            RegOp t{};
            t.type = 4;
            t.k = r;
            t.moff = pool_off();
            plan.tile_pool.insert(plan.tile_pool.end(), table.begin(), table.end());
            plan.reg_ops.push_back(t);
        }
        // a probe followed by the inverse rotation it belongs to (same
        // generator, parameter and bit) becomes one op: one pass over the
        // registers, one dispatch
        {
            std::vector<RegOp> fused;
            for (size_t i = 0; i < sops.size(); ++i) {
                const RegOp &a = sops[i];
                if (a.type == 9 && i + 1 < sops.size()) {
                    const RegOp &b = sops[i + 1];
                    if (b.type == 8 && b.jmatch == 1 && b.moff == a.moff && b.rj[0] == a.rj[0] &&
                        b.rmask == a.rmask && b.rb[0] == a.rb[0] && b.tb[0] == a.tb[0] && b.gp[0] == a.gp[0] &&
                        b.gp[1] == a.gp[1]) {
                        RegOp f = a;
                        f.type = 10;
                        fused.push_back(f);
                        ++i;
                        continue;
                    }
                }
                fused.push_back(a);
            }
            sops.swap(fused);
        }
        // two such probe-and-inverse-rotation ops on one register bit become
        // one (the second's parameter in gj[0], generator in rj[1])
        {
            std::vector<RegOp> fused;
            for (size_t i = 0; i < sops.size(); ++i) {
                const RegOp &a = sops[i];
                if (a.type == 10 && a.nreg == 1 && i + 1 < sops.size()) {
                    const RegOp &b = sops[i + 1];
                    if (b.type == 10 && b.nreg == 1 && b.rb[0] == a.rb[0]) {
                        RegOp f = a;
                        f.type = 12;
                        f.rj[1] = b.rj[0];
                        f.gj[0] = b.moff;
                        fused.push_back(f);
                        ++i;
                        continue;
                    }
                }
                fused.push_back(a);
            }
            sops.swap(fused);
        }
        // two forward rotations on one register bit, the first about X or Y,
        // become one op (the second's parameter in gj[0], generator in rj[1])
        {
            std::vector<RegOp> fused;
            for (size_t i = 0; i < sops.size(); ++i) {
                const RegOp &a = sops[i];
                if (a.type == 8 && a.jmatch == 0 && a.nreg == 1 && a.rj[0] != 3 && i + 1 < sops.size()) {
                    const RegOp &b = sops[i + 1];
                    if (b.type == 8 && b.jmatch == 0 && b.nreg == 1 && b.rb[0] == a.rb[0]) {
                        RegOp f = a;
                        f.type = 11;
                        f.rj[1] = b.rj[0];
                        f.gj[0] = b.moff;
                        fused.push_back(f);
                        ++i;
                        continue;
                    }
                }
                fused.push_back(a);
            }
            sops.swap(fused);
        }
        plan.reg_ops.insert(plan.reg_ops.end(), sops.begin(), sops.end());
        st.op_end = int(plan.reg_ops.size()) - p.rop_begin;
        plan.reg_stages.push_back(st);
        prevR = Rm;
    }
    p.rop_end = int(plan.reg_ops.size());
    for (int o = p.rop_begin; o < p.rop_end; ++o) {
        RegOp &op = plan.reg_ops[size_t(o)];
        switch (op.type) {
            case 0: op.code = op.rmask; break;
            case 3: op.code = 64 + op.rb[0]; break;
            case 5: op.code = 72 + op.rb[0]; break;
            case 6: op.code = 128 + op.rmask; break;
            case 4: op.code = 200; break;
            case 7: op.code = (op.jmatch ? 160 : 210) + op.rb[0]; break;
            case 8: op.code = op.rj[0] == 3 ? 236 : (op.rj[0] == 1 ? 220 : 228) + op.rb[0]; break;
            case 9: op.code = op.rj[0] == 3 ? 256 : (op.rj[0] == 1 ? 240 : 248) + op.rb[0]; break;
            case 10: op.code = op.rj[0] == 3 ? 280 : (op.rj[0] == 1 ? 264 : 272) + op.rb[0]; break;
            case 11: op.code = 288 + 8 * ((op.rj[0] - 1) * 3 + op.rj[1] - 1) + op.rb[0]; break;
            case 12: op.code = 344 + 8 * ((op.rj[0] - 1) * 3 + op.rj[1] - 1) + op.rb[0]; break;
            default: op.code = 201; break;
        }
    }
    p.stage_end = int(plan.reg_stages.size());
    p.pool_end = int(plan.tile_pool.size());
    return true;
}

}  // namespace qsim
