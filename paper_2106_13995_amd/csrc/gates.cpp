// Host-side gate model: named gate matrices, structure detection (diagonal,
// control bits), target reordering and double-precision fusion of gates.
#include <algorithm>
#include <cmath>

#include "qsim_internal.h"

namespace qsim {

namespace {
const cd kI(0.0, 1.0);

void identity(cd *U, int d) {
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) U[r * d + c] = (r == c) ? cd(1.0) : cd(0.0);
}

// Index of a full-register basis state in a gate's local basis: bit b of the
// result is bit positions[b] of x.
inline int local_index(uint32_t x, const int *positions, int k) {
    int j = 0;
    for (int b = 0; b < k; ++b) j |= int((x >> positions[b]) & 1u) << b;
    return j;
}
}  // namespace

int named_gate_arity(int kind) {
    switch (kind) {
        case QSIM_GATE_H: case QSIM_GATE_X: case QSIM_GATE_Y: case QSIM_GATE_Z:
        case QSIM_GATE_S: case QSIM_GATE_SDG: case QSIM_GATE_T: case QSIM_GATE_TDG:
        case QSIM_GATE_RX: case QSIM_GATE_RY: case QSIM_GATE_RZ: case QSIM_GATE_U3:
            return 1;
        case QSIM_GATE_CX: case QSIM_GATE_CZ: case QSIM_GATE_CP: case QSIM_GATE_SWAP:
            return 2;
        case QSIM_GATE_CCX: case QSIM_GATE_CCZ:
            return 3;
        default:
            return -1;
    }
}

int named_gate_matrix(int kind, const double *a, cd *U) {
    const int k = named_gate_arity(kind);
    if (k < 0) return -1;
    const int d = 1 << k;
    identity(U, d);
    switch (kind) {
        case QSIM_GATE_H: {
            const double h = 1.0 / std::sqrt(2.0);
            U[0] = h; U[1] = h; U[2] = h; U[3] = -h;
            break;
        }
        case QSIM_GATE_X: U[0] = 0.0; U[1] = 1.0; U[2] = 1.0; U[3] = 0.0; break;
        case QSIM_GATE_Y: U[0] = 0.0; U[1] = -kI; U[2] = kI; U[3] = 0.0; break;
        case QSIM_GATE_Z: U[3] = -1.0; break;
        case QSIM_GATE_S: U[3] = kI; break;
        case QSIM_GATE_SDG: U[3] = -kI; break;
        case QSIM_GATE_T: U[3] = std::polar(1.0, M_PI / 4.0); break;
        case QSIM_GATE_TDG: U[3] = std::polar(1.0, -M_PI / 4.0); break;
        case QSIM_GATE_RX: {
            const double c = std::cos(0.5 * a[0]), s = std::sin(0.5 * a[0]);
            U[0] = c; U[1] = cd(0.0, -s); U[2] = cd(0.0, -s); U[3] = c;
            break;
        }
        case QSIM_GATE_RY: {
            const double c = std::cos(0.5 * a[0]), s = std::sin(0.5 * a[0]);
            U[0] = c; U[1] = -s; U[2] = s; U[3] = c;
            break;
        }
        case QSIM_GATE_RZ:
            U[0] = std::polar(1.0, -0.5 * a[0]);
            U[3] = std::polar(1.0, 0.5 * a[0]);
            break;
        case QSIM_GATE_U3: {
            const double c = std::cos(0.5 * a[0]), s = std::sin(0.5 * a[0]);
            U[0] = c;
            U[1] = -std::polar(s, a[2]);
            U[2] = std::polar(s, a[1]);
            U[3] = std::polar(c, a[1] + a[2]);
            break;
        }
        case QSIM_GATE_CX:    // control = local bit 0, target = local bit 1
            U[1 * 4 + 1] = 0.0; U[3 * 4 + 3] = 0.0; U[1 * 4 + 3] = 1.0; U[3 * 4 + 1] = 1.0;
            break;
        case QSIM_GATE_CZ: U[15] = -1.0; break;
        case QSIM_GATE_CP: U[15] = std::polar(1.0, a[0]); break;
        case QSIM_GATE_SWAP:
            U[1 * 4 + 1] = 0.0; U[2 * 4 + 2] = 0.0; U[1 * 4 + 2] = 1.0; U[2 * 4 + 1] = 1.0;
            break;
        case QSIM_GATE_CCX:   // controls = local bits 0, 1; target = local bit 2
            U[3 * 8 + 3] = 0.0; U[7 * 8 + 7] = 0.0; U[3 * 8 + 7] = 1.0; U[7 * 8 + 3] = 1.0;
            break;
        case QSIM_GATE_CCZ: U[63] = -1.0; break;
        default: return -1;
    }
    return k;
}

bool is_diagonal(const HostGate &g) {
    if (g.probe_gen || g.rot_gen) return false;
    const int d = 1 << g.k;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && g.M[r * d + c] != cd(0.0)) return false;
    return true;
}

// Local bit b is a control when the matrix never changes bit b and is the
// identity on the half where bit b is 0.
static bool bit_is_control(const HostGate &g, int b) {
    const int d = 1 << g.k;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            const cd v = g.M[r * d + c];
            const int rb = (r >> b) & 1, cb = (c >> b) & 1;
            if (rb != cb) {
                if (v != cd(0.0)) return false;
            } else if (rb == 0) {
                if (v != (r == c ? cd(1.0) : cd(0.0))) return false;
            }
        }
    return true;
}

int extract_controls(const HostGate &g, HostGate &reduced, int *controls) {
    reduced = g;
    int nc = 0;
    // never strip the last remaining target
    bool changed = true;
    while (changed && reduced.k > 1) {
        changed = false;
        for (int b = 0; b < reduced.k; ++b) {
            if (!bit_is_control(reduced, b)) continue;
            // drop local bit b, keeping the bit-b = 1 block
            HostGate r;
            r.k = reduced.k - 1;
            r.src_op = reduced.src_op;
            for (int i = 0, j = 0; i < reduced.k; ++i)
                if (i != b) r.targets[j++] = reduced.targets[i];
            const int dn = 1 << r.k, dold = 1 << reduced.k;
            r.M.assign(size_t(dn) * dn, cd(0.0));
            auto expand = [b](int x) {
                const int lo = x & ((1 << b) - 1);
                return ((x >> b) << (b + 1)) | (1 << b) | lo;
            };
            for (int rr = 0; rr < dn; ++rr)
                for (int cc = 0; cc < dn; ++cc) r.M[rr * dn + cc] = reduced.M[expand(rr) * dold + expand(cc)];
            controls[nc++] = reduced.targets[b];
            reduced = std::move(r);
            changed = true;
            break;
        }
    }
    return nc;
}

HostGate sorted_targets(const HostGate &g) {
    HostGate s;
    s.k = g.k;
    s.src_op = g.src_op;
    s.rot_real = g.rot_real;
    s.rot_c = g.rot_c;
    s.rot_s = g.rot_s;
    s.phase_in = g.phase_in;
    int perm[QSIM_MAX_K];  // perm[i] = original local bit of sorted bit i
    for (int i = 0; i < g.k; ++i) perm[i] = i;
    std::sort(perm, perm + g.k, [&](int a, int b) { return g.targets[a] < g.targets[b]; });
    for (int i = 0; i < g.k; ++i) s.targets[i] = g.targets[perm[i]];
    const int d = 1 << g.k;
    auto orig = [&](int j) {
        int o = 0;
        for (int i = 0; i < g.k; ++i) o |= ((j >> i) & 1) << perm[i];
        return o;
    };
    s.M.resize(size_t(d) * d);
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) s.M[r * d + c] = g.M[orig(r) * d + orig(c)];
    return s;
}

// Matrix of gate g embedded in the register spanned by `qubits` (u of them).
static std::vector<cd> embed(const HostGate &g, const int *qubits, int u) {
    const int D = 1 << u, d = 1 << g.k;
    int pos[QSIM_MAX_K];  // position of each gate target inside `qubits`
    uint32_t gmask = 0;
    for (int b = 0; b < g.k; ++b) {
        pos[b] = int(std::find(qubits, qubits + u, g.targets[b]) - qubits);
        gmask |= 1u << pos[b];
    }
    std::vector<cd> E(size_t(D) * D, cd(0.0));
    for (uint32_t r = 0; r < uint32_t(D); ++r)
        for (uint32_t c = 0; c < uint32_t(D); ++c) {
            if ((r & ~gmask) != (c & ~gmask)) continue;
            E[r * D + c] = g.M[local_index(r, pos, g.k) * d + local_index(c, pos, g.k)];
        }
    return E;
}

HostGate fuse_pair(const HostGate &first, const HostGate &second) {
    HostGate out;
    int qs[2 * QSIM_MAX_K];
    int u = 0;
    for (int b = 0; b < first.k; ++b) qs[u++] = first.targets[b];
    for (int b = 0; b < second.k; ++b)
        if (std::find(qs, qs + u, second.targets[b]) == qs + u) qs[u++] = second.targets[b];
    std::sort(qs, qs + u);
    out.k = u;
    for (int i = 0; i < u; ++i) out.targets[i] = qs[i];
    const std::vector<cd> A = embed(first, qs, u), B = embed(second, qs, u);
    const int D = 1 << u;
    out.M.assign(size_t(D) * D, cd(0.0));
    for (int r = 0; r < D; ++r)
        for (int j = 0; j < D; ++j) {
            const cd b = B[r * D + j];
            if (b == cd(0.0)) continue;
            for (int c = 0; c < D; ++c) out.M[r * D + c] += b * A[j * D + c];
        }
    return out;
}

// ------------------------------------------------------------ single-qubit split

namespace {

// U = g diag(1, b) [[c, -s], [s, c]] diag(1, a) with c = |U00|, s = |U10|
// and unit g, a, b, for a 2 x 2 unitary U that is not diagonal.  The phases
// come from normalised matrix entries, not from angles, so that exact
// entries (0, +-1, +-i) give exact phases.  Returns false when U is not
// unitary to 1e-12 or the factors do not reproduce it to 1e-12.
bool euler_split(const std::vector<cd> &U, double &c, double &s, cd &g, cd &a, cd &b) {
    const cd u00 = U[0], u01 = U[1], u10 = U[2], u11 = U[3];
    const double n0 = std::norm(u00) + std::norm(u10), n1 = std::norm(u01) + std::norm(u11);
    const cd ip = std::conj(u00) * u01 + std::conj(u10) * u11;
    if (std::abs(n0 - 1.0) > 1e-12 || std::abs(n1 - 1.0) > 1e-12 || std::abs(ip) > 1e-12) return false;
    c = std::abs(u00);
    s = std::abs(u10);
    if (s == 0.0) return false;
    g = c > 0.0 ? u00 / c : u10 / s;
    b = (u10 / g) / s;
    a = (-u01 / g) / s;
    const cd r[4] = {g * c, -g * s * a, g * b * s, g * b * c * a};
    for (int i = 0; i < 4; ++i)
        if (std::abs(r[i] - U[size_t(i)]) > 1e-12) return false;
    return true;
}

HostGate phase_gate(int q, cd lo, cd hi) {
    HostGate d;
    d.k = 1;
    d.targets[0] = q;
    d.M = {lo, cd(0.0), cd(0.0), hi};
    return d;
}

}  // namespace

std::vector<HostGate> split_single_qubit(const std::vector<HostGate> &gates, int n) {
    // pending[q]: diag(1, pending[q]) still owed on qubit q
    std::vector<cd> pending(size_t(n), cd(1.0));
    cd global(1.0);
    std::vector<HostGate> out;
    out.reserve(gates.size() + size_t(n) + 1);
    auto flush = [&](int q) {
        if (pending[size_t(q)] == cd(1.0)) return;
        out.push_back(phase_gate(q, cd(1.0), pending[size_t(q)]));
        pending[size_t(q)] = cd(1.0);
    };
    for (const HostGate &g : gates) {
        const bool special = g.probe_gen || g.rot_gen || g.rot_real;
        const bool diag = !special && is_diagonal(g);
        if (g.k == 1 && !special) {
            const int q = g.targets[0];
            if (diag && g.M[0] != cd(0.0)) {
                // diag(u0, u1) = u0 diag(1, u1 / u0): merges into the owed phase
                pending[size_t(q)] *= g.M[3] / g.M[0];
                global *= g.M[0];
                continue;
            }
            double c, s;
            cd gg, a, b;
            if (!diag && euler_split(g.M, c, s, gg, a, b)) {
                HostGate r;
                r.k = 1;
                r.targets[0] = q;
                r.src_op = g.src_op;
                r.rot_real = c == 0.0 ? 2 : 1;
                r.rot_c = c;
                r.rot_s = r.rot_real == 2 ? 1.0 : s;
                r.phase_in = a * pending[size_t(q)];
                r.M = {cd(r.rot_c), -r.rot_s * r.phase_in, cd(r.rot_s), r.rot_c * r.phase_in};
                out.push_back(std::move(r));
                pending[size_t(q)] = b;
                global *= gg;
                continue;
            }
        }
        // diagonal gates commute with the owed phases; anything else settles
        // them on its qubits first
        if (!diag)
            for (int i = 0; i < g.k; ++i) flush(g.targets[i]);
        out.push_back(g);
    }
    int last = -1;
    for (int q = 0; q < n; ++q)
        if (pending[size_t(q)] != cd(1.0)) {
            flush(q);
            last = int(out.size()) - 1;
        }
    if (global != cd(1.0)) {
        if (last >= 0) {
            out[size_t(last)].M[0] *= global;
            out[size_t(last)].M[3] *= global;
        } else {
            out.push_back(phase_gate(0, global, global));
        }
    }
    return out;
}

}  // namespace qsim
