// Run-time compiled register-staged tile passes.
//
// The register tile kernel interprets each pass's op list, and a data-
// dependent branch per op over 2^r register amplitudes costs the compiler a
// full copy of the amplitude registers at every join.  For large states the
// planner's register program is instead written out as straight-line HIP
// source, one kernel per pass (amplitudes as named scalars, register and
// layout indices as constants, matrices and parameters still read from the
// uploaded pool), compiled once with hipRTC for gfx950 and kept for the life
// of the process, keyed by what the source is written from.
#include <hip/hiprtc.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "qsim_internal.h"

namespace qsim {

namespace {

struct Src {
    std::string s;
    void operator()(const char *fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        const int n = vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        if (n >= int(sizeof buf)) {
            // a long line: format again into a buffer of its size
            std::vector<char> big(size_t(n) + 1);
            va_start(ap, fmt);
            vsnprintf(big.data(), big.size(), fmt, ap);
            va_end(ap);
            s.append(big.data(), size_t(n));
        } else if (n > 0) {
            s.append(buf, size_t(n));
        }
        s.push_back('\n');
    }
};

int popc32(uint32_t v) { return __builtin_popcount(v); }

int deposit_bits(int j, int mask) {
    int out = 0, b = 0;
    for (int p = 0; p < 31; ++p)
        if ((mask >> p) & 1) {
            if ((j >> b) & 1) out |= 1 << p;
            ++b;
        }
    return out;
}

// x with its sign flipped where the unsigned 0/1 expression `e` is 1, as a
// C expression: the sign bit is XORed into x's bit pattern, so a condition
// that is uniform across the block stays on the scalar unit.
std::string signed_by(double x, const std::string &e, bool f) {
    char buf[96];
    if (f) {
        const float v = float(x);
        uint32_t u;
        std::memcpy(&u, &v, 4);
        snprintf(buf, sizeof buf, "__builtin_bit_cast(float, 0x%08xu ^ ((", u);
        return buf + e + ") << 31))";
    }
    uint64_t u;
    std::memcpy(&u, &x, 8);
    snprintf(buf, sizeof buf, "__builtin_bit_cast(double, 0x%016llxull ^ ((unsigned long long)(",
             (unsigned long long)u);
    return buf + e + ") << 63))";
}

// Exact literal of x in the kernel's precision.
std::string lit(double x, bool f) {
    char buf[64];
    if (f)
        snprintf(buf, sizeof buf, "%af", double(float(x)));
    else
        snprintf(buf, sizeof buf, "%a", x);
    return buf;
}

// Multiplies register amplitude i by the factor v, whose value is known
// here; `on` is a lane predicate (nullptr: every lane).  Exact factors
// (-1, +-i) are sign changes and exchanges; other unit factors on every lane
// are a rotation of (re, im) by three in-place lifting steps (a sign change
// first when Re v < 0 keeps the steps bounded); the rest is a complex
// product with the pool entry P[e], P[e + 1].
double emit_factor(Src &o, bool f, int i, std::complex<double> v, const char *on, int e) {
    const char *T = f ? "float" : "double";
    const char *FMA = f ? "__builtin_fmaf" : "__builtin_fma";
    if (v == std::complex<double>(1.0)) return 0.0;
    if (v == std::complex<double>(-1.0)) {
        if (on)
            o("    ar%d = %s ? -ar%d : ar%d; ai%d = %s ? -ai%d : ai%d;", i, on, i, i, i, on, i, i);
        else
            o("    ar%d = -ar%d; ai%d = -ai%d;", i, i, i, i);
        return 0.0;
    }
    if (v == std::complex<double>(0.0, 1.0) || v == std::complex<double>(0.0, -1.0)) {
        const bool plus = v.imag() > 0;   // i (x + iy) = -y + ix; -i (x + iy) = y - ix
        if (on)
            o("    { const %s xr = ar%d; ar%d = %s ? %sai%d : ar%d; ai%d = %s ? %sxr : ai%d; }", T, i, i, on,
              plus ? "-" : "", i, i, i, on, plus ? "" : "-", i);
        else
            o("    { const %s xr = ar%d; ar%d = %sai%d; ai%d = %sxr; }", T, i, i, plus ? "-" : "", i, i,
              plus ? "" : "-");
        return 0.0;
    }
    if (!on && std::abs(std::abs(v) - 1.0) < 1e-12) {
        double c = v.real(), s = v.imag();
        if (c < 0) {
            o("    ar%d = -ar%d; ai%d = -ai%d;", i, i, i, i);
            c = -c;
            s = -s;
        }
        const std::string P = lit(-s / (1.0 + c), f), U = lit(s, f);
        o("    ar%d = %s(%s, ai%d, ar%d); ai%d = %s(%s, ar%d, ai%d); ar%d = %s(%s, ai%d, ar%d);", i, FMA, P.c_str(), i,
          i, i, FMA, U.c_str(), i, i, i, FMA, P.c_str(), i, i);
        return 6.0;
    }
    o("    { %s dx = P[%d], dy = P[%d];", T, e, e + 1);
    if (on) o("      dx = %s ? dx : %s(1); dy = %s ? dy : %s(0);", on, T, on, T);
    o("      const %s xr = ar%d; ar%d = %s(dx, xr, -dy * ai%d); ai%d = %s(dx, ai%d, dy * xr); }", T, i, i, FMA, i, i,
      FMA, i);
    return 6.0;
}

// A diagonal that the compiled passes owe the amplitudes they store: the
// stored value times (-1)^F(y) times `scale` is the amplitude of index y.
// F is the XOR of the monomials in `mono`, each a product of qubit bits kept
// as the mask of its qubits (mask 0: the constant 1).  Sign changes of
// diagonal gates (CZ, CCZ, Z under controls) join F instead of being applied:
// F commutes with every diagonal op, a real rotation on qubit b takes it
// through by flipping the sign of its off-diagonal constant where dF/dy_b is
// 1, and an exchange on b (a signed swap, a controlled X) reflects F in b.
// The factors the scaled rotations leave out accumulate in `scale`.  Both are
// applied at a store: F when the next pass is not compiled in the same chain,
// the scale then or once it leaves [2^-40, 1].
struct Owed {
    std::set<uint64_t> mono;
    double scale = 1.0;
    void toggle(uint64_t m) {
        if (!mono.erase(m)) mono.insert(m);
    }
    bool depends_on(uint64_t qmask) const {
        for (uint64_t m : mono)
            if (m & qmask) return true;
        return false;
    }
    // F(y with bit q flipped where the monomial c is 1) = F + c dF/dy_q
    void reflect(int q, uint64_t c) {
        const uint64_t qb = 1ull << q;
        std::vector<uint64_t> add;
        for (uint64_t m : mono)
            if (m & qb) add.push_back((m & ~qb) | c);
        for (uint64_t m : add) toggle(m);
    }
};

// Qubit on each register / thread bit of a register stage; qubits outside the
// tile are the block's (bits of `base`).
struct Layout {
    int R = 0;
    int qr[kRegBitsMax] = {};
    int qt[8] = {};
};

// Sign of register i under F in layout ly: a constant part and the XOR of
// monomials over thread and block qubits (evaluated at run time).
struct RegSign {
    bool c = false;
    std::set<uint64_t> rt;
    void add(const RegSign &o) {
        c ^= o.c;
        for (uint64_t m : o.rt)
            if (!rt.erase(m)) rt.insert(m);
    }
};

RegSign sign_of(const Owed &ow, const Layout &ly, int i) {
    RegSign s;
    for (uint64_t m : ow.mono) {
        uint64_t rest = m;
        bool hit = true;
        for (int b = 0; b < ly.R && hit; ++b) {
            const uint64_t qb = 1ull << ly.qr[b];
            if (rest & qb) {
                hit = (i >> b) & 1;
                rest &= ~qb;
            }
        }
        if (!hit) continue;
        if (!rest)
            s.c = !s.c;
        else if (!s.rt.erase(rest))
            s.rt.insert(rest);
    }
    return s;
}

// Run-time parity of a set of monomials over thread and block qubits, as a
// C expression (thread bits from t, block bits from base): single-bit terms
// by one population count over thread bits and one over block bits (uniform
// across the block), products term by term.
std::string rt_expr(const std::set<uint64_t> &rt, const Layout &ly) {
    std::string e;
    uint32_t lin_t = 0;
    uint64_t lin_g = 0;
    char buf[160];
    auto add = [&e](const char *term) {
        if (!e.empty()) e += " ^ ";
        e += term;
    };
    for (uint64_t m : rt) {
        uint32_t tm = 0;
        uint64_t gm = m;
        for (int b = 0; b < 8; ++b)
            if ((m >> ly.qt[b]) & 1) {
                tm |= 1u << b;
                gm &= ~(1ull << ly.qt[b]);
            }
        if (__builtin_popcountll(m) == 1) {
            if (tm)
                lin_t ^= tm;
            else
                lin_g ^= gm;
            continue;
        }
        if (tm && gm)
            snprintf(buf, sizeof buf, "(unsigned)(((t & %uu) == %uu) && ((base & 0x%llxull) == 0x%llxull))", tm, tm,
                     (unsigned long long)gm, (unsigned long long)gm);
        else if (tm)
            snprintf(buf, sizeof buf, "(unsigned)((t & %uu) == %uu)", tm, tm);
        else
            snprintf(buf, sizeof buf, "(unsigned)((base & 0x%llxull) == 0x%llxull)", (unsigned long long)gm,
                     (unsigned long long)gm);
        add(buf);
    }
    if (lin_t) {
        snprintf(buf, sizeof buf, "(__builtin_popcount(t & %uu) & 1u)", lin_t);
        add(buf);
    }
    if (lin_g) {
        snprintf(buf, sizeof buf, "(unsigned)(__builtin_popcountll(base & 0x%llxull) & 1)", (unsigned long long)lin_g);
        add(buf);
    }
    return e.empty() ? std::string("0u") : e;
}

// Sign of every register under F, as C expressions: F splits by the
// register qubits of its monomials, F = XOR over register subsets S of
// [S all 1] * R_S (R_S over thread and block qubits); each R_S is computed
// once and register i XORs those with S inside its bits.  Returns, per
// register, a constant part and the names to XOR (none: constant sign).
struct SignTable {
    std::vector<bool> c;
    std::vector<std::string> e;
};
SignTable emit_sign_table(Src &o, const Owed &ow, const Layout &ly, int NA, const char *pre) {
    std::map<uint32_t, std::set<uint64_t>> parts;   // register subset -> runtime monomials
    std::map<uint32_t, bool> cparts;                 // register subset -> constant term
    for (uint64_t m : ow.mono) {
        uint32_t S = 0;
        uint64_t rest = m;
        for (int b = 0; b < ly.R; ++b)
            if ((rest >> ly.qr[b]) & 1) {
                S |= 1u << b;
                rest &= ~(1ull << ly.qr[b]);
            }
        if (!rest)
            cparts[S] = !cparts[S];
        else if (!parts[S].erase(rest))
            parts[S].insert(rest);
    }
    std::map<uint32_t, std::string> name;
    for (auto &kv : parts) {
        if (kv.second.empty()) continue;
        const std::string nm = std::string(pre) + std::to_string(name.size());
        o("    const unsigned %s = %s;", nm.c_str(), rt_expr(kv.second, ly).c_str());
        name[kv.first] = nm;
    }
    SignTable tb;
    tb.c.assign(size_t(NA), false);
    tb.e.assign(size_t(NA), std::string());
    for (int i = 0; i < NA; ++i) {
        bool c = false;
        for (auto &kv : cparts)
            if (kv.second && (kv.first & ~uint32_t(i)) == 0) c = !c;
        std::string e;
        for (auto &kv : name)
            if ((kv.first & ~uint32_t(i)) == 0) e += (e.empty() ? "" : " ^ ") + kv.second;
        tb.c[size_t(i)] = c;
        tb.e[size_t(i)] = e;
    }
    return tb;
}

// Applies F to every register of the layout (values change sign where F is
// 1) and clears it.
void settle_signs(Src &o, Owed &ow, const Layout &ly, int NA) {
    if (ow.mono.empty()) return;
    o("  {");
    const SignTable tb = emit_sign_table(o, ow, ly, NA, "sgn");
    for (int i = 0; i < NA; ++i) {
        if (tb.e[size_t(i)].empty()) {
            if (tb.c[size_t(i)]) o("    ar%d = -ar%d; ai%d = -ai%d;", i, i, i, i);
            continue;
        }
        o("    { const unsigned e = %s%s;", tb.e[size_t(i)].c_str(), tb.c[size_t(i)] ? " ^ 1u" : "");
        o("      ar%d = e ? -ar%d : ar%d; ai%d = e ? -ai%d : ai%d; }", i, i, i, i, i, i);
    }
    o("  }");
    ow.mono.clear();
}

bool perm_block(const Plan &plan, const Pass &p, const RegOp &op) {
    const cd *u = plan.tile_pool.data() + p.pool_begin + op.moff;
    return u[0] == cd(0.0) && u[3] == cd(0.0) && u[1] == cd(1.0) && u[2] == cd(1.0);
}

}  // namespace

// Occupancy maps for compiled passes on sparse states.  Ops that can spread
// a basis state over several (rotations, dense blocks, controlled blocks that
// are not exchanges) are counted over the compiled passes; with few of them
// a state that starts sparse (a basis state, a few superposed values) stays
// sparse, and the passes keep one byte per chunk of 2^shift amplitudes
// saying whether the chunk may hold a nonzero value.  Returns shift, or 0
// for no maps.
int jit_map_shift(const Plan &plan) {
    // QSIM_MAP_SHIFT (4..13) sets another chunk width (tests use narrow
    // chunks to reach the maps on small states)
    int shift = plan.dtype == QSIM_C128 ? 11 : 12;
    if (const char *e = std::getenv("QSIM_MAP_SHIFT")) {
        const int v = std::atoi(e);
        if (v >= 4 && v <= 13) shift = v;
    }
    int spreading = 0;
    bool any = false;
    for (const Pass &p : plan.passes) {
        if (p.kind != PASS_TILE || p.reg_r <= 0) continue;
        any = true;
        if (p.m < shift) return 0;
        for (int oi = p.rop_begin; oi < p.rop_end; ++oi) {
            const RegOp &op = plan.reg_ops[size_t(oi)];
            if (op.type == 0 || op.type == 3 || (op.type == 7 && !perm_block(plan, p, op))) ++spreading;
        }
    }
    if (!any || spreading > 24 || plan.n < shift + 6) return 0;
    return shift;
}

namespace {

// Emits one pass as kernel `name`; returns the arithmetic it performs per
// thread (flops; a multiply-add counts 2).  `ow` is what earlier passes of
// the chain left owed; with `settle` the pass stores true amplitudes.
double gen_pass(Src &o, const Plan &plan, const Pass &p, const char *name, Owed &ow, bool settle, int map_shift,
                int chain_pos) {
    double fl = 0.0;
    const bool f = plan.dtype == QSIM_C64;
    const char *T = f ? "float" : "double";
    const char *V = f ? "f2" : "d2";
    const char *FMA = f ? "__builtin_fmaf" : "__builtin_fma";
    const int R = p.reg_r, NA = 1 << R;
    auto pool_at = [&](int rel) { return plan.tile_pool[size_t(p.pool_begin + rel)]; };
    o("extern \"C\" __global__ void __launch_bounds__(256) %s(%s *psi, const %s *Pg, unsigned char *maps) {", name,
      V, T);
    o("  const QC %s *P = (const QC %s *)Pg;", T, T);
    // A static tile: its address is a link-time constant that folds into
    // the LDS instructions' offsets (a dynamic array costs an add per access).
    o("  __shared__ %s lds[%d];", V, 1 << p.m);
    o("  const unsigned t = threadIdx.x;");
    o("  unsigned long long base = (unsigned long long)blockIdx.x << %d;", p.L);
    for (int h : p.hpos) o("  base = ((base >> %d) << %d) | (base & 0x%llxull);", h, h + 1, (1ull << h) - 1ull);
    // Occupancy maps (three in rotation, one byte per chunk of 2^shift
    // amplitudes): this pass reads the previous pass's map (not the first
    // pass of a chain), marks the chunks of the tiles it processes in the
    // next one, and clears its share of the third.  A tile's chunks are
    // fixed by its qubits at or above shift.
    std::vector<int> hq;
    if (map_shift > 0) {
        for (int h : p.hpos)
            if (h >= map_shift) hq.push_back(h);
        const unsigned long long C = 1ull << (plan.n - map_shift);
        const unsigned long long share = 1ull << (p.m - map_shift);   // C / number of tiles
        const int R_ = chain_pos % 3, W_ = (chain_pos + 1) % 3, X_ = (chain_pos + 2) % 3;
        o("  unsigned char *const mw = maps + %lluull, *const mx = maps + %lluull;", W_ * C, X_ * C);
        o("  for (unsigned j = t; j < %lluu; j += 256u) mx[(unsigned long long)blockIdx.x * %lluull + j] = 0;", share,
          share);
        o("  unsigned long long ck = base >> %d;", map_shift);
        for (size_t j = 0; j < hq.size(); ++j)
            o("  ck |= (unsigned long long)((t >> %zu) & 1u) << %d;", j, hq[j] - map_shift);
        if (chain_pos > 0)
            o("  if (!__syncthreads_or(t < %uu ? int(maps[%lluull + ck]) : 0)) return;", 1u << hq.size(), R_ * C);
    }
    for (int i = 0; i < NA; ++i) o("  %s ar%d, ai%d;", T, i, i);
    // load
    o("  {");
    o("    unsigned long long gt = base;");
    for (int b = 0; b < 8; ++b) o("    gt |= (unsigned long long)((t >> %d) & 1u) << %d;", b, int(p.ld_t[b]));
    for (int i = 0; i < NA; ++i) {
        unsigned long long off = 0;
        for (int b = 0; b < R; ++b)
            if ((i >> b) & 1) off |= 1ull << p.ld_r[b];
        o("    { const %s w = __builtin_nontemporal_load(psi + (gt | 0x%llxull)); ar%d = w.x; ai%d = w.y; }", V, off,
          i, i);
    }
    o("  }");
    // A tile that is zero everywhere stays zero (every op is linear; owed
    // signs and factors multiply zeros): the block skips its ops and store.
    // Sparse states (basis inputs, few superposed values) then cost the
    // reads and little else.
    {
        std::string nz;
        for (int i = 0; i < NA; ++i) {
            char b[64];
            snprintf(b, sizeof b, "%s(ar%d != %s(0)) | (ai%d != %s(0))", i ? " | " : "", i, T, i, T);
            nz += b;
        }
        o("  if (!__syncthreads_or(int(%s))) return;", nz.c_str());
    }
    Layout ly;
    ly.R = R;
    for (int si = p.stage_begin; si < p.stage_end; ++si) {
        const RegStage &st = plan.reg_stages[size_t(si)];
        // the owed signs are a function of the qubits: they cross the
        // exchange unchanged and are read in the new layout from here on
        for (int b = 0; b < R; ++b) ly.qr[b] = st.q_r[b];
        for (int b = 0; b < 8; ++b) ly.qt[b] = st.q_t[b];
        if (si > p.stage_begin) {
            // The swizzled slot of register i is (thread part) ^ c_i.  Bits of
            // c_i where the thread part is always zero add instead of mixing,
            // so they go to the instruction's constant offset; only the
            // distinct remainders (c_i restricted to the thread part's bits)
            // cost an address computation each.
            o("  {");
            o("    unsigned aw = 0u, ar_ = 0u;");
            uint32_t tw = 0, tr = 0;
            for (int b = 0; b < 8; ++b) {
                tw |= st.wr_t[b];
                tr |= st.rd_t[b];
                if (st.wr_t[b]) o("    aw ^= (0u - ((t >> %d) & 1u)) & %uu;", b, st.wr_t[b]);
                if (st.rd_t[b]) o("    ar_ ^= (0u - ((t >> %d) & 1u)) & %uu;", b, st.rd_t[b]);
            }
            o("    char *const lb = (char *)lds;");
            auto slots = [&](const uint32_t *rbits, uint32_t tmask, const char *tv, const char *pre) {
                std::map<uint32_t, int> mixed;
                std::vector<std::pair<uint32_t, uint32_t>> at;
                at.resize(size_t(NA));
                for (int i = 0; i < NA; ++i) {
                    uint32_t c = 0;
                    for (int b = 0; b < R; ++b)
                        if ((i >> b) & 1) c ^= rbits[b];
                    at[size_t(i)] = {c & tmask, c & ~tmask};
                    if (!mixed.count(c & tmask)) {
                        const int id = int(mixed.size());
                        mixed[c & tmask] = id;
                        o("    const unsigned %s%d = (%s ^ %uu) * %du;", pre, id, tv, c & tmask, f ? 8 : 16);
                    }
                }
                return std::make_pair(mixed, at);
            };
            {
                auto [mixed, at] = slots(st.wr_r, tw, "aw", "w");
                for (int i = 0; i < NA; ++i)
                    o("    *(%s *)(lb + w%d + %uu) = %s{ar%d, ai%d};", V, mixed[at[size_t(i)].first],
                      at[size_t(i)].second * (f ? 8u : 16u), V, i, i);
            }
            o("    __syncthreads();");
            {
                auto [mixed, at] = slots(st.rd_r, tr, "ar_", "r");
                for (int i = 0; i < NA; ++i)
                    o("    { const %s w = *(const %s *)(lb + r%d + %uu); ar%d = w.x; ai%d = w.y; }", V, V,
                      mixed[at[size_t(i)].first], at[size_t(i)].second * (f ? 8u : 16u), i, i);
            }
            o("    __syncthreads();");
            o("  }");
        }
        for (int oi = p.rop_begin + st.op_begin; oi < p.rop_begin + st.op_end; ++oi) {
            const RegOp &op = plan.reg_ops[size_t(oi)];
            const int m2 = 2 * op.moff;
            switch (op.type) {
                case 0: {   // dense on register mask, complex matrix
                    uint64_t qm = 0;
                    for (int b = 0; b < R; ++b)
                        if ((op.rmask >> b) & 1) qm |= 1ull << ly.qr[b];
                    if (ow.depends_on(qm)) settle_signs(o, ow, ly, NA);
                    const int K = popc32(uint32_t(op.rmask)), D = 1 << K;
                    fl += 8.0 * D * NA;   // a complex multiply-add per matrix entry and amplitude
                    o("  {");
                    for (int g = 0; g < NA; ++g) {
                        if (g & op.rmask) continue;
                        o("    {");
                        for (int c = 0; c < D; ++c) {
                            const int ix = g | deposit_bits(c, op.rmask);
                            o("      const %s x%dr = ar%d, x%di = ai%d;", T, c, ix, c, ix);
                        }
                        for (int rr = 0; rr < D; ++rr) {
                            const int ix = g | deposit_bits(rr, op.rmask);
                            const int e0 = m2 + 2 * rr * D;
                            o("      { %s yr = P[%d] * x0r, yi = P[%d] * x0i;", T, e0, e0);
                            o("        yr = %s(-P[%d], x0i, yr); yi = %s(P[%d], x0r, yi);", FMA, e0 + 1, FMA, e0 + 1);
                            for (int c = 1; c < D; ++c) {
                                const int e = e0 + 2 * c;
                                o("        yr = %s(P[%d], x%dr, yr); yr = %s(-P[%d], x%di, yr);", FMA, e, c, FMA,
                                  e + 1, c);
                                o("        yi = %s(P[%d], x%di, yi); yi = %s(P[%d], x%dr, yi);", FMA, e, c, FMA,
                                  e + 1, c);
                            }
                            o("        ar%d = yr; ai%d = yi; }", ix, ix);
                        }
                        o("    }");
                    }
                    o("  }");
                    break;
                }
                case 3: {   // real rotation [[c, -s], [s, c]] on one register bit
                    // As c [[1, -t], [t, 1]] (t = s / c, when c >= s) or
                    // s [[v, -1], [1, v]] (v = c / s): two multiply-adds per
                    // component and pair.  The factor c or s is the same for
                    // every amplitude and joins the owed scale.  Owed signs
                    // that differ between the members of a pair flip the
                    // sign of t or v (a constant here, or chosen per lane or
                    // block at run time); the first form keeps each member's
                    // sign, the second swaps them (F reflected in the bit).
                    // (The pool entry holds the lifting form p = -s / (1 + c),
                    // u = s, used by the interpreted kernel.)
                    const int B = op.rb[0];
                    const cd pu = pool_at(op.moff);
                    const double sv = pu.imag(), cv = -sv / pu.real() - 1.0;
                    const bool tform = cv >= sv;
                    const double kv = tform ? sv / cv : cv / sv;
                    ow.scale *= tform ? cv : sv;
                    fl += 4.0 * NA;
                    o("  {");
                    std::map<std::set<uint64_t>, std::string> kvar;
                    for (int g = 0; g < NA; ++g) {
                        if (g & (1 << B)) continue;
                        const int h = g | (1 << B);
                        RegSign sig = sign_of(ow, ly, g);
                        sig.add(sign_of(ow, ly, h));
                        std::string K, NK;   // the constant and its negation
                        if (sig.rt.empty()) {
                            K = lit(sig.c ? -kv : kv, f);
                            NK = lit(sig.c ? kv : -kv, f);
                        } else {
                            auto it = kvar.find(sig.rt);
                            if (it == kvar.end()) {
                                const std::string nm = "k" + std::to_string(kvar.size());
                                o("    const %s %s = %s;", T, nm.c_str(), signed_by(kv, rt_expr(sig.rt, ly), f).c_str());
                                it = kvar.emplace(sig.rt, nm).first;
                            }
                            K = (sig.c ? "-" : "") + it->second;
                            NK = (sig.c ? "" : "-") + it->second;
                        }
                        for (const char *c : {"ar", "ai"}) {
                            if (tform)
                                o("    { const %s y = %s(%s, %s%d, %s%d); %s%d = %s(%s, %s%d, %s%d); %s%d = y; }", T, FMA,
                                  NK.c_str(), c, h, c, g, c, h, FMA, K.c_str(), c, g, c, h, c, g);
                            else
                                o("    { const %s y = %s(%s, %s%d, -%s%d); %s%d = %s(%s, %s%d, %s%d); %s%d = y; }", T, FMA,
                                  K.c_str(), c, g, c, h, c, h, FMA, K.c_str(), c, h, c, g, c, g);
                        }
                    }
                    o("  }");
                    if (!tform) ow.reflect(ly.qr[B], 0);
                    break;
                }
                case 5: {   // (x0, x1) <- (-x1, x0)
                    const int B = op.rb[0];
                    o("  {");
                    for (int g = 0; g < NA; ++g) {
                        if (g & (1 << B)) continue;
                        const int h = g | (1 << B);
                        o("    { const %s tr = ar%d, ti = ai%d; ar%d = -ar%d; ai%d = -ai%d; ar%d = tr; ai%d = ti; }", T, g,
                          g, g, h, g, h, h, h);
                    }
                    o("  }");
                    ow.reflect(ly.qr[B], 0);   // the members trade their owed signs
                    break;
                }
                case 4: {   // phase table over the register bits (entry 0 is 1)
                    o("  {");
                    for (int i = 1; i < NA; ++i)
                        fl += emit_factor(o, f, i, pool_at(op.moff + i), nullptr, m2 + 2 * i);
                    o("  }");
                    break;
                }
                case 6: {   // factor on the all-ones amplitudes of the op's bits
                    const uint64_t gmask = uint64_t(uint32_t(op.gp[0])) | (uint64_t(uint32_t(op.gp[1])) << 32);
                    const uint32_t tmask = uint32_t(op.tb[0]);
                    if (pool_at(op.moff) == cd(-1.0)) {
                        // a sign change (CZ, CCZ, ...): owed, not applied
                        uint64_t mono = gmask;
                        for (int b = 0; b < R; ++b)
                            if ((op.rmask >> b) & 1) mono |= 1ull << ly.qr[b];
                        for (int b = 0; b < 8; ++b)
                            if ((tmask >> b) & 1u) mono |= 1ull << ly.qt[b];
                        ow.toggle(mono);
                        break;
                    }
                    // A condition on out-of-tile bits only holds for whole
                    // blocks: a uniform branch, taken by the blocks it holds
                    // in, in place of a select on every lane of every block.
                    const bool lane_cond = tmask != 0, block_cond = gmask && !tmask;
                    o("  {");
                    if (lane_cond)
                        o("    const bool on = ((base & 0x%llxull) == 0x%llxull) && ((t & %uu) == %uu);",
                          (unsigned long long)gmask, (unsigned long long)gmask, tmask, tmask);
                    if (block_cond)
                        o("    if ((base & 0x%llxull) == 0x%llxull) {", (unsigned long long)gmask,
                          (unsigned long long)gmask);
                    for (int i = 0; i < NA; ++i) {
                        if ((i & op.rmask) != op.rmask) continue;
                        fl += emit_factor(o, f, i, pool_at(op.moff), lane_cond ? "on" : nullptr, m2);
                    }
                    if (block_cond) o("    }");
                    o("  }");
                    break;
                }
                case 7: {   // 2 x 2 block on bit rb[0] where every control is 1
                    const int B = op.rb[0], rc = op.rmask;
                    const uint64_t gmask = uint64_t(uint32_t(op.gp[0])) | (uint64_t(uint32_t(op.gp[1])) << 32);
                    const uint32_t tmask = uint32_t(op.tb[0]);
                    // lane conditions select; block conditions branch (as for type 6)
                    const bool cond = tmask != 0, block_cond = gmask && !tmask;
                    const cd u[4] = {pool_at(op.moff), pool_at(op.moff + 1), pool_at(op.moff + 2),
                                     pool_at(op.moff + 3)};
                    // an exchange (X under controls: CX, CCX) moves values only
                    const bool perm = u[0] == cd(0.0) && u[3] == cd(0.0) && u[1] == cd(1.0) && u[2] == cd(1.0);
                    uint64_t cmono = gmask;   // product of the controls
                    for (int b = 0; b < R; ++b)
                        if ((rc >> b) & 1) cmono |= 1ull << ly.qr[b];
                    for (int b = 0; b < 8; ++b)
                        if ((tmask >> b) & 1u) cmono |= 1ull << ly.qt[b];
                    if (!perm && ow.depends_on(1ull << ly.qr[B])) settle_signs(o, ow, ly, NA);
                    o("  {");
                    if (cond)
                        o("    const bool on = ((base & 0x%llxull) == 0x%llxull) && ((t & %uu) == %uu);",
                          (unsigned long long)gmask, (unsigned long long)gmask, tmask, tmask);
                    if (block_cond)
                        o("    if ((base & 0x%llxull) == 0x%llxull) {", (unsigned long long)gmask,
                          (unsigned long long)gmask);
                    for (int g = 0; g < NA; ++g) {
                        if ((g & (1 << B)) || (g & rc) != rc) continue;
                        const int h = g | (1 << B);
                        o("    { const %s x0r = ar%d, x0i = ai%d, x1r = ar%d, x1i = ai%d;", T, g, g, h, h);
                        if (perm) {
                            o("      const %s y0r = x1r, y0i = x1i, y1r = x0r, y1i = x0i;", T);
                        } else {
                            fl += 32.0;
                            for (int rr = 0; rr < 2; ++rr) {
                                const int e0 = m2 + 4 * rr, e1 = e0 + 2;
                                o("      const %s y%dr = %s(P[%d], x0r, %s(-P[%d], x0i, %s(P[%d], x1r, -P[%d] * x1i)));", T,
                                  rr, FMA, e0, FMA, e0 + 1, FMA, e1, e1 + 1);
                                o("      const %s y%di = %s(P[%d], x0i, %s(P[%d], x0r, %s(P[%d], x1i, P[%d] * x1r)));", T,
                                  rr, FMA, e0, FMA, e0 + 1, FMA, e1, e1 + 1);
                            }
                        }
                        if (cond)
                            o("      ar%d = on ? y0r : x0r; ai%d = on ? y0i : x0i; ar%d = on ? y1r : x1r; ai%d = on ? y1i : "
                              "x1i; }", g, g, h, h);
                        else
                            o("      ar%d = y0r; ai%d = y0i; ar%d = y1r; ai%d = y1i; }", g, g, h, h);
                    }
                    if (block_cond) o("    }");
                    o("  }");
                    if (perm) ow.reflect(ly.qr[B], cmono);   // values moved where the controls are 1
                    break;
                }
                default: {   // any other diagonal: index from out-of-tile, thread and register bits
                    o("  { int jt = 0;");
                    for (int b = 0; b < op.nout; ++b)
                        o("    jt |= int((base >> %d) & 1ull) << %d;", int(op.gp[b]), int(op.gj[b]));
                    for (int b = 0; b < op.nthr; ++b)
                        o("    jt |= int((t >> %d) & 1u) << %d;", int(op.tb[b]), int(op.tj[b]));
                    for (int i = 0; i < NA; ++i) {
                        int jr = 0;
                        for (int b = 0; b < op.nreg; ++b) jr |= ((i >> op.rb[b]) & 1) << op.rj[b];
                        o("    { const int j = %d + 2 * (jt | %d); const %s dx = Pg[j], dy = Pg[j + 1], xr = ar%d;", m2,
                          jr, T, i);
                        o("      ar%d = %s(dx, xr, -dy * ai%d); ai%d = %s(dx, ai%d, dy * xr); }", i, FMA, i, i, FMA,
                          i);
                    }
                    fl += 6.0 * NA;
                    o("  }");
                    break;
                }
            }
        }
    }
    if (map_shift > 0) o("  if (t < %uu) mw[ck] = 1;", 1u << hq.size());
    // store: owed signs (end of a chain) and the owed scale (end of a chain,
    // or once it leaves [2^-40, 1]) are applied here, one multiply per
    // component
    o("  {");
    if (!settle && ow.scale < std::ldexp(1.0, -40)) {
        const std::string sc = lit(ow.scale, f);
        for (int i = 0; i < NA; ++i) o("    ar%d *= %s; ai%d *= %s;", i, sc.c_str(), i, sc.c_str());
        fl += 2.0 * NA;
        ow.scale = 1.0;
    } else if (settle && (ow.scale != 1.0 || !ow.mono.empty())) {
        const double scv = ow.scale;
        const SignTable tb = emit_sign_table(o, ow, ly, NA, "sgn");
        const std::string P = lit(scv, f), N = lit(-scv, f);
        for (int i = 0; i < NA; ++i) {
            const bool c = tb.c[size_t(i)];
            if (tb.e[size_t(i)].empty()) {
                if (scv == 1.0) {
                    if (c) o("    ar%d = -ar%d; ai%d = -ai%d;", i, i, i, i);
                    continue;
                }
                o("    ar%d *= %s; ai%d *= %s;", i, (c ? N : P).c_str(), i, (c ? N : P).c_str());
                continue;
            }
            o("    { const %s g = %s; ar%d *= g; ai%d *= g; }", T, signed_by(c ? -scv : scv, tb.e[size_t(i)], f).c_str(),
              i, i);
        }
        fl += 2.0 * NA;
        ow.mono.clear();
        ow.scale = 1.0;
    }
    o("    unsigned long long gt = base;");
    for (int b = 0; b < 8; ++b) o("    gt |= (unsigned long long)((t >> %d) & 1u) << %d;", b, int(p.st_t[b]));
    for (int i = 0; i < NA; ++i) {
        unsigned long long off = 0;
        for (int b = 0; b < R; ++b)
            if ((i >> b) & 1) off |= 1ull << p.st_r[b];
        o("    __builtin_nontemporal_store(%s{ar%d, ai%d}, psi + (gt | 0x%llxull));", V, i, i, off);
    }
    o("  }");
    o("}");
    return fl;
}

struct JitModule {
    hipModule_t mod = nullptr;
    std::vector<hipFunction_t> fns;
    std::vector<double> flops_per_thread;   // per compiled pass
};

std::mutex g_mu;
// (device, source key) -> loaded module; modules stay loaded until exit
std::map<std::pair<int, std::string>, std::shared_ptr<JitModule>> g_modules;

// Exact description of everything the generated source depends on: the
// precision and, for each compiled pass in order, its layout fields and the
// register stages, register ops and pool entries it reads (all pass-relative).
// Equal keys give equal source, so a plan whose passes were compiled before
// finds its module without writing the source out again.
std::string source_key(const Plan &plan) {
    std::string k;
    auto put = [&k](const void *p, size_t n) { k.append(static_cast<const char *>(p), n); };
    put(&plan.dtype, sizeof plan.dtype);
    put(&plan.n, sizeof plan.n);
    const int map_shift = jit_map_shift(plan);
    put(&map_shift, sizeof map_shift);
    for (const Pass &p : plan.passes) {
        if (p.kind != PASS_TILE || p.reg_r <= 0) continue;
        const int head[4] = {p.m, p.L, p.reg_r, int(p.hpos.size())};
        put(head, sizeof head);
        put(p.hpos.data(), sizeof(int) * p.hpos.size());
        put(p.ld_t, sizeof p.ld_t);
        put(p.ld_r, sizeof p.ld_r);
        put(p.st_t, sizeof p.st_t);
        put(p.st_r, sizeof p.st_r);
        const int sizes[3] = {p.stage_end - p.stage_begin, p.rop_end - p.rop_begin, p.pool_end - p.pool_begin};
        put(sizes, sizeof sizes);
        put(plan.reg_stages.data() + p.stage_begin, sizeof(RegStage) * size_t(sizes[0]));
        put(plan.reg_ops.data() + p.rop_begin, sizeof(RegOp) * size_t(sizes[1]));
        put(plan.tile_pool.data() + p.pool_begin, sizeof(cd) * size_t(sizes[2]));
    }
    return k;
}
std::string g_last_log;

int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

}  // namespace

int jit_mode() { return env_int("QSIM_JIT", -1); }

bool jit_wanted(int n) {
    const int mode = jit_mode();
    if (mode == 0) return false;
    return n >= env_int("QSIM_JIT_MIN_QUBITS", 18);
}

std::string jit_source(const Plan &plan, std::vector<int> &which, std::vector<double> *flops) {
    Src o;
    o("typedef float f2 __attribute__((ext_vector_type(2)));");
    o("typedef double d2 __attribute__((ext_vector_type(2)));");
    o("#define QC __attribute__((address_space(4)))");
    which.clear();
    auto compiled = [&](size_t i) { return plan.passes[i].kind == PASS_TILE && plan.passes[i].reg_r > 0; };
    Owed ow;   // carried from pass to pass while the next one is compiled too
    const int map_shift = jit_map_shift(plan);
    int chain_pos = 0;
    for (size_t i = 0; i < plan.passes.size(); ++i) {
        const Pass &p = plan.passes[i];
        if (!compiled(i)) continue;
        chain_pos = (i > 0 && compiled(i - 1)) ? chain_pos + 1 : 0;
        char name[48];
        snprintf(name, sizeof name, "qsim_tile_jit_%zu", which.size());
        const bool settle = i + 1 == plan.passes.size() || !compiled(i + 1);
        const double fpt = gen_pass(o, plan, p, name, ow, settle, map_shift, chain_pos);
        if (flops) flops->push_back(fpt * 256.0 * std::ldexp(1.0, plan.n - p.m));
        which.push_back(int(i));
    }
    return o.s;
}

qsim_status jit_prepare(qsim_state s, Plan &plan, std::string &err) {
    plan.jit_fn.assign(plan.passes.size(), nullptr);
    std::vector<int> which;
    for (size_t i = 0; i < plan.passes.size(); ++i)
        if (plan.passes[i].kind == PASS_TILE && plan.passes[i].reg_r > 0) which.push_back(int(i));
    if (which.empty()) return QSIM_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    const auto key = std::make_pair(s->device, source_key(plan));
    auto it = g_modules.find(key);
    std::shared_ptr<JitModule> jm;
    if (it != g_modules.end()) {
        jm = it->second;
    } else {
        std::vector<double> flops;
        const std::string text = jit_source(plan, which, &flops);
        hiprtcProgram prog;
        if (hiprtcCreateProgram(&prog, text.c_str(), "qsim_tiles.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
            err = "hiprtcCreateProgram failed";
            return QSIM_ERR_DEVICE;
        }
        // packed FP32 instructions stay off, as for the prebuilt kernels;
        // CodeGenPrepare and the SLP vectoriser change nothing in this
        // straight-line code and take a quarter of the compile time
        const char *opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
                              "-packed-fp32-ops", "-mllvm", "-disable-cgp", "-fno-slp-vectorize"};
        const hiprtcResult rc = hiprtcCompileProgram(prog, 9, opts);
        if (rc != HIPRTC_SUCCESS) {
            size_t ls = 0;
            hiprtcGetProgramLogSize(prog, &ls);
            std::string log(ls, '\0');
            if (ls) hiprtcGetProgramLog(prog, &log[0]);
            hiprtcDestroyProgram(&prog);
            err = "run-time compilation of tile passes failed: " + log.substr(0, 400);
            return QSIM_ERR_DEVICE;
        }
        size_t cs = 0;
        hiprtcGetCodeSize(prog, &cs);
        std::vector<char> code(cs);
        hiprtcGetCode(prog, code.data());
        hiprtcDestroyProgram(&prog);
        jm = std::make_shared<JitModule>();
        if (hipModuleLoadData(&jm->mod, code.data()) != hipSuccess) {
            err = "loading the compiled tile passes failed";
            return QSIM_ERR_DEVICE;
        }
        for (size_t k = 0; k < which.size(); ++k) {
            char name[48];
            snprintf(name, sizeof name, "qsim_tile_jit_%zu", k);
            hipFunction_t fn = nullptr;
            if (hipModuleGetFunction(&fn, jm->mod, name) != hipSuccess) {
                err = "compiled tile pass missing from its module";
                return QSIM_ERR_DEVICE;
            }
            jm->fns.push_back(fn);
            const Pass &p = plan.passes[size_t(which[k])];
            jm->flops_per_thread.push_back(flops[k] / (256.0 * std::ldexp(1.0, plan.n - p.m)));
        }
        g_modules[key] = jm;
    }
    for (size_t k = 0; k < which.size(); ++k) {
        Pass &p = plan.passes[size_t(which[k])];
        plan.jit_fn[size_t(which[k])] = jm->fns[k];
        p.flops = jm->flops_per_thread[k] * 256.0 * std::ldexp(1.0, plan.n - p.m);
    }
    plan.jit_map_shift = jit_map_shift(plan);
    return QSIM_OK;
}

hipError_t launch_jit_pass(qsim_state s, const Plan &plan, const Pass &p, hipFunction_t fn, void *maps) {
    const bool f = s->dtype == QSIM_C64;
    const size_t amp = f ? 8 : 16;
    void *psi = s->data;
    const char *pool = static_cast<const char *>(plan.dev) + plan.pool_dev_off + size_t(p.pool_begin) * amp;
    const void *pool_arg = pool;
    void *args[] = {&psi, &pool_arg, &maps};
    const uint64_t ntiles = 1ull << (s->n - p.m);
    // the tile is a static LDS array of the kernel (at most 64 KiB)
    return hipModuleLaunchKernel(fn, unsigned(ntiles), 1, 1, 256, 1, 1, 0u, s->stream, args, nullptr);
}

}  // namespace qsim
