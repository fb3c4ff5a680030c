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

}  // namespace qsim
