/*
 * CPU oracle for the state-vector (Schroedinger-type) circuit simulator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header
 * or table with the HIP library: it is a plain, slow, complex128 statement of
 * what the simulator computes, written so that it can be checked by eye.
 *
 * What it computes (paper, Sec. I.A "Background" and Sec. II "Methods"): the
 * state of n qubits is a vector of 2^n complex amplitudes and every gate acts
 * on it as a 2^n x 2^n matrix; the simulator is a chain of matrix-vector
 * products, one per gate, so its cost is linear in the number of gates.  A
 * k-qubit gate's 2^n x 2^n matrix is the gate's 2^k x 2^k matrix on the target
 * bits times the identity on all others, so the product is evaluated group by
 * group: every set of 2^k amplitudes whose indices agree off the target bits
 * is multiplied by the small matrix.
 *
 * Conventions the paper leaves open (each is a stated reading):
 *   - qubit q is bit q of the amplitude index (little-endian);
 *   - targets[b] is bit b of the small matrix's row/column index;
 *   - gate matrices are the textbook / OpenQASM 2 ones (see gate_matrix);
 *   - a Pauli string with masks (x, z) is i^{|x&z|} X^x Z^z.
 *
 * Built with plain gcc (-O2, textbook complex products).  A second build
 * with -fopenmp splits the gate loop over host threads (for timing and for
 * computing large stored references); the per-amplitude arithmetic is the
 * same, so its results are bit-identical to the single-thread build.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Gate codes of the oracle (its own numbering; the Python wrapper maps the
 * gate names of the workload descriptions onto them). */
enum {
    OG_MATRIX = 0,
    OG_H, OG_X, OG_Y, OG_Z, OG_S, OG_SDG, OG_T, OG_TDG,
    OG_RX, OG_RY, OG_RZ, OG_U3,
    OG_CX, OG_CZ, OG_CP, OG_SWAP,
    OG_CCX, OG_CCZ,
    OG_COUNT
};

#define ORACLE_MAX_K 6

static void set_identity(cplx *U, int d)
{
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            U[r * d + c] = (r == c) ? 1.0 : 0.0;
}

/* Number of qubits a gate code acts on (MATRIX: taken from the op). */
int oracle_gate_arity(int code)
{
    switch (code) {
    case OG_H: case OG_X: case OG_Y: case OG_Z: case OG_S: case OG_SDG:
    case OG_T: case OG_TDG: case OG_RX: case OG_RY: case OG_RZ: case OG_U3:
        return 1;
    case OG_CX: case OG_CZ: case OG_CP: case OG_SWAP:
        return 2;
    case OG_CCX: case OG_CCZ:
        return 3;
    default:
        return -1;
    }
}

/*
 * Builds the 2^k x 2^k row-major matrix of a named gate from its definition
 * and returns k (-1 for an unknown code).  Angles: RX/RY/RZ/CP use ang[0];
 * U3 uses (theta, phi, lambda) = ang[0..2].
 *   H  = [[1,1],[1,-1]]/sqrt2          X, Y, Z: Pauli matrices
 *   S  = diag(1, i)    T = diag(1, e^{i pi/4})   (SDG, TDG: conjugates)
 *   RX(t) = exp(-i t X/2), RY(t) = exp(-i t Y/2), RZ(t) = exp(-i t Z/2)
 *   U3(t,p,l) = [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]]
 *   CX (control = targets[0]): flips the target bit when the control is 1
 *   CZ = diag(1,1,1,-1), CP(p) = diag(1,1,1,e^{ip}), SWAP exchanges the bits
 *   CCX flips targets[2] when targets[0] and targets[1] are 1; CCZ = -1 on |111>
 */
int oracle_gate_matrix(int code, const double *ang, cplx *U)
{
    const double r2 = 1.0 / sqrt(2.0);
    double c, s;
    switch (code) {
    case OG_H:
        U[0] = r2; U[1] = r2; U[2] = r2; U[3] = -r2;
        return 1;
    case OG_X:
        U[0] = 0; U[1] = 1; U[2] = 1; U[3] = 0;
        return 1;
    case OG_Y:
        U[0] = 0; U[1] = -I; U[2] = I; U[3] = 0;
        return 1;
    case OG_Z:
        U[0] = 1; U[1] = 0; U[2] = 0; U[3] = -1;
        return 1;
    case OG_S:
        U[0] = 1; U[1] = 0; U[2] = 0; U[3] = I;
        return 1;
    case OG_SDG:
        U[0] = 1; U[1] = 0; U[2] = 0; U[3] = -I;
        return 1;
    case OG_T:
        U[0] = 1; U[1] = 0; U[2] = 0; U[3] = cexp(I * M_PI / 4.0);
        return 1;
    case OG_TDG:
        U[0] = 1; U[1] = 0; U[2] = 0; U[3] = cexp(-I * M_PI / 4.0);
        return 1;
    case OG_RX:
        c = cos(ang[0] / 2.0); s = sin(ang[0] / 2.0);
        U[0] = c; U[1] = -I * s; U[2] = -I * s; U[3] = c;
        return 1;
    case OG_RY:
        c = cos(ang[0] / 2.0); s = sin(ang[0] / 2.0);
        U[0] = c; U[1] = -s; U[2] = s; U[3] = c;
        return 1;
    case OG_RZ:
        U[0] = cexp(-I * ang[0] / 2.0); U[1] = 0; U[2] = 0; U[3] = cexp(I * ang[0] / 2.0);
        return 1;
    case OG_U3:
        c = cos(ang[0] / 2.0); s = sin(ang[0] / 2.0);
        U[0] = c;
        U[1] = -cexp(I * ang[2]) * s;
        U[2] = cexp(I * ang[1]) * s;
        U[3] = cexp(I * (ang[1] + ang[2])) * c;
        return 1;
    case OG_CX:
        /* local index j = control + 2*target: |c=1,t=0> (j=1) <-> |c=1,t=1> (j=3) */
        set_identity(U, 4);
        U[1 * 4 + 1] = 0; U[3 * 4 + 3] = 0;
        U[1 * 4 + 3] = 1; U[3 * 4 + 1] = 1;
        return 2;
    case OG_CZ:
        set_identity(U, 4);
        U[3 * 4 + 3] = -1;
        return 2;
    case OG_CP:
        set_identity(U, 4);
        U[3 * 4 + 3] = cexp(I * ang[0]);
        return 2;
    case OG_SWAP:
        /* |a=1,b=0> (j=1) <-> |a=0,b=1> (j=2) */
        set_identity(U, 4);
        U[1 * 4 + 1] = 0; U[2 * 4 + 2] = 0;
        U[1 * 4 + 2] = 1; U[2 * 4 + 1] = 1;
        return 2;
    case OG_CCX:
        /* j = c1 + 2*c2 + 4*t: j=3 <-> j=7 */
        set_identity(U, 8);
        U[3 * 8 + 3] = 0; U[7 * 8 + 7] = 0;
        U[3 * 8 + 7] = 1; U[7 * 8 + 3] = 1;
        return 3;
    case OG_CCZ:
        set_identity(U, 8);
        U[7 * 8 + 7] = -1;
        return 3;
    default:
        return -1;
    }
}

/*
 * psi <- (U on targets) psi, straight from the definition: for every base
 * index with all target bits clear, gather the 2^k amplitudes of its group
 * (local index j sets target bit targets[b] from bit b of j), multiply by U
 * and scatter back.  Returns 0, or -1 on bad arguments.
 */
int oracle_apply_matrix(cplx *psi, int n, const int *targets, int k, const cplx *U)
{
    if (k < 1 || k > ORACLE_MAX_K || k > n)
        return -1;
    uint64_t tmask = 0;
    for (int b = 0; b < k; ++b) {
        if (targets[b] < 0 || targets[b] >= n)
            return -1;
        if (tmask & (1ull << targets[b]))
            return -1;
        tmask |= 1ull << targets[b];
    }
    const uint64_t N = 1ull << n;
    const int d = 1 << k;
    /* Groups are independent: the threaded build splits the base loop over
     * threads; every amplitude still gets the same operations in the same
     * order, so both builds give bit-identical results. */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t ibase = 0; ibase < (int64_t)N; ++ibase) {
        const uint64_t base = (uint64_t)ibase;
        uint64_t idx[1 << ORACLE_MAX_K];
        cplx v[1 << ORACLE_MAX_K];
        if (base & tmask)
            continue;
        for (int j = 0; j < d; ++j) {
            uint64_t x = base;
            for (int b = 0; b < k; ++b)
                if ((j >> b) & 1)
                    x |= 1ull << targets[b];
            idx[j] = x;
            v[j] = psi[x];
        }
        for (int r = 0; r < d; ++r) {
            cplx acc = 0;
            for (int c = 0; c < d; ++c)
                acc += U[r * d + c] * v[c];
            psi[idx[r]] = acc;
        }
    }
    return 0;
}

/* The classical action of a permutation gate on one basis index. */
static uint64_t permute_index(int code, const int *t, uint64_t x)
{
    switch (code) {
    case OG_X:
        return x ^ (1ull << t[0]);
    case OG_CX:
        return ((x >> t[0]) & 1) ? x ^ (1ull << t[1]) : x;
    case OG_CCX:
        return (((x >> t[0]) & 1) && ((x >> t[1]) & 1)) ? x ^ (1ull << t[2]) : x;
    case OG_SWAP: {
        uint64_t a = (x >> t[0]) & 1, b = (x >> t[1]) & 1;
        if (a != b)
            x ^= (1ull << t[0]) | (1ull << t[1]);
        return x;
    }
    default:
        return x;
    }
}

/*
 * Permutation gates (X, CX, CCX, SWAP) as index maps: the amplitude of basis
 * state x moves to pi(x).  A second, independent statement of these gates;
 * the tests require it to agree exactly with oracle_apply_matrix.
 * `scratch` must hold 2^n amplitudes.  Returns 0, or -1 for a code that is
 * not a permutation gate.
 */
int oracle_apply_permutation(cplx *psi, cplx *scratch, int n, int code, const int *targets)
{
    if (code != OG_X && code != OG_CX && code != OG_CCX && code != OG_SWAP)
        return -1;
    const uint64_t N = 1ull << n;
    for (uint64_t x = 0; x < N; ++x)
        scratch[permute_index(code, targets, x)] = psi[x];
    memcpy(psi, scratch, N * sizeof(cplx));
    return 0;
}

/*
 * A circuit is the ordered chain of its gates' matrix-vector products.
 * Op i: codes[i], its qubits targets[6*i .. 6*i+ks[i]-1], angles
 * angles[3*i .. 3*i+2] for named gates, and for OG_MATRIX a dense matrix at
 * mats + mat_off[i] (complex entries).  Returns 0, or -(i+1) if op i is bad.
 */
int oracle_apply_circuit(cplx *psi, int n, int nops, const int *codes, const int *ks,
                         const int *targets, const double *angles, const cplx *mats,
                         const int64_t *mat_off)
{
    cplx U[(1 << ORACLE_MAX_K) * (1 << ORACLE_MAX_K)];
    for (int i = 0; i < nops; ++i) {
        const cplx *M = U;
        int k;
        if (codes[i] == OG_MATRIX) {
            k = ks[i];
            M = mats + mat_off[i];
        } else {
            k = oracle_gate_matrix(codes[i], angles + 3 * i, U);
            if (k != ks[i])
                return -(i + 1);
        }
        if (oracle_apply_matrix(psi, n, targets + 6 * i, k, M) != 0)
            return -(i + 1);
    }
    return 0;
}

static int popcount64(uint64_t v)
{
    int c = 0;
    while (v) {
        c += (int)(v & 1);
        v >>= 1;
    }
    return c;
}

/*
 * (P psi) for one Pauli string P = i^{|x&z|} X^x Z^z, by definition:
 *   (Z^z phi)_y = (-1)^{|y&z|} phi_y,   (X^x phi)_y = phi_{y^x},
 * so (P psi)_y = i^{|x&z|} (-1)^{|(y^x)&z|} psi_{y^x}.
 */
void oracle_pauli_apply(const cplx *psi, cplx *out, int n, uint64_t x, uint64_t z)
{
    static const cplx ipow[4] = {1.0, I, -1.0, -I};
    const cplx ph = ipow[popcount64(x & z) & 3];
    const uint64_t N = 1ull << n;
    for (uint64_t y = 0; y < N; ++y) {
        uint64_t src = y ^ x;
        double sign = (popcount64(src & z) & 1) ? -1.0 : 1.0;
        out[y] = ph * sign * psi[src];
    }
}

/*
 * <psi|H|psi> for H = sum_t coeff[t] P_t: the real part of
 * sum_t coeff[t] sum_y conj(psi_y) (P_t psi)_y, accumulated in double.
 * No renormalisation.
 */
double oracle_expectation(const cplx *psi, int n, int nterms, const double *coeff,
                          const uint64_t *xmask, const uint64_t *zmask)
{
    static const cplx ipow[4] = {1.0, I, -1.0, -I};
    const uint64_t N = 1ull << n;
    double total = 0.0;
    for (int t = 0; t < nterms; ++t) {
        const cplx ph = ipow[popcount64(xmask[t] & zmask[t]) & 3];
        cplx acc = 0;
        for (uint64_t y = 0; y < N; ++y) {
            uint64_t src = y ^ xmask[t];
            double sign = (popcount64(src & zmask[t]) & 1) ? -1.0 : 1.0;
            acc += conj(psi[y]) * (ph * sign * psi[src]);
        }
        total += coeff[t] * creal(acc);
    }
    return total;
}

/*
 * Classical evaluation of a circuit made only of X, CX, CCX and SWAP on
 * basis inputs: each op's index map applied to an integer.  xs[0..count-1]
 * are updated in place.  Returns 0, or -(i+1) if op i is not a permutation.
 */
int oracle_classical_run(int nops, const int *codes, const int *targets, uint64_t *xs, int64_t count)
{
    for (int i = 0; i < nops; ++i)
        if (codes[i] != OG_X && codes[i] != OG_CX && codes[i] != OG_CCX && codes[i] != OG_SWAP)
            return -(i + 1);
    for (int64_t s = 0; s < count; ++s) {
        uint64_t x = xs[s];
        for (int i = 0; i < nops; ++i)
            x = permute_index(codes[i], targets + 6 * i, x);
        xs[s] = x;
    }
    return 0;
}

/*
 * Amplitudes of a product state followed by one layer of disjoint CZ gates,
 * one index at a time (closed form).  The product state is
 * (u_{n-1} (x) ... (x) u_0)|0...0>, with u_q given by its first column
 * col0[2q], col0[2q+1]; then the CZ on pair (a, b) multiplies by -1 when both
 * bits are set.  out[s] = prod_q col0[2q + y_q] * (-1)^{sum_pairs y_a y_b}.
 */
void oracle_product_cz_amplitudes(int n, const cplx *col0, int npairs, const int *pairs,
                                  int64_t count, const uint64_t *idx, cplx *out)
{
    for (int64_t s = 0; s < count; ++s) {
        uint64_t y = idx[s];
        cplx amp = 1.0;
        for (int q = 0; q < n; ++q)
            amp *= col0[2 * q + ((y >> q) & 1)];
        int parity = 0;
        for (int p = 0; p < npairs; ++p)
            parity ^= (int)(((y >> pairs[2 * p]) & 1) & ((y >> pairs[2 * p + 1]) & 1));
        out[s] = parity ? -amp : amp;
    }
}
