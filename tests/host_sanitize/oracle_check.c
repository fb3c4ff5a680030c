/* The CPU oracle under AddressSanitizer and UBSan (built by
 * tests/test_host_sanitize.py with gcc): every entry point on small inputs,
 * every gate code, a dense 6-qubit matrix, and the rejected arguments. */
#include <complex.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;
int oracle_gate_matrix(int code, const double *ang, cplx *U);
int oracle_apply_matrix(cplx *psi, int n, const int *targets, int k, const cplx *U);
int oracle_apply_permutation(cplx *psi, cplx *scratch, int n, int code, const int *targets);
int oracle_apply_circuit(cplx *psi, int n, int nops, const int *codes, const int *ks, const int *targets,
                         const double *angles, const cplx *mats, const int64_t *mat_off);
void oracle_pauli_apply(const cplx *psi, cplx *out, int n, uint64_t x, uint64_t z);
double oracle_expectation(const cplx *psi, int n, int nterms, const double *coeff, const uint64_t *xmask,
                          const uint64_t *zmask);
int oracle_classical_run(int nops, const int *codes, const int *targets, uint64_t *xs, int64_t count);
void oracle_product_cz_amplitudes(int n, const cplx *col0, int npairs, const int *pairs, int64_t count,
                                  const uint64_t *idx, cplx *out);

int main(void) {
    enum { N = 10, NOPS = 19 };
    const int n = N;
    cplx *psi = calloc((size_t)1 << n, sizeof(cplx));
    cplx *tmp = calloc((size_t)1 << n, sizeof(cplx));
    if (!psi || !tmp) return 2;
    psi[0] = 1.0;
    /* every gate code once (code 0: a dense 6-qubit matrix) */
    int codes[NOPS], ks[NOPS], targets[6 * NOPS];
    double angles[3 * NOPS];
    int64_t offs[NOPS];
    cplx *mats = calloc(64 * 64, sizeof(cplx));
    for (int r = 0; r < 64; ++r) mats[r * 64 + (r * 37 + 5) % 64] = 1.0;   /* a permutation matrix */
    for (int i = 0; i < NOPS; ++i) {
        codes[i] = i;
        offs[i] = 0;
        for (int a = 0; a < 3; ++a) angles[3 * i + a] = 0.3 + 0.1 * i + a;
        cplx U[64 * 64];
        ks[i] = i == 0 ? 6 : oracle_gate_matrix(i, angles + 3 * i, U);
        if (ks[i] < 1) return 3;
        for (int b = 0; b < 6; ++b) targets[6 * i + b] = (3 * i + b) % n;   /* distinct */
    }
    if (oracle_apply_circuit(psi, n, NOPS, codes, ks, targets, angles, mats, offs) != 0) return 4;
    const int pt[3] = {1, 4, 7};
    if (oracle_apply_permutation(psi, tmp, n, 17, pt) != 0) return 5;
    if (oracle_apply_permutation(psi, tmp, n, 1, pt) != -1) return 6;   /* H is not a permutation */
    oracle_pauli_apply(psi, tmp, n, 0x5, 0x9);
    const double coeff[3] = {1.0, 0.5, -0.25};
    const uint64_t xm[3] = {0, 1, 6}, zm[3] = {3, 0, 2};
    const double e = oracle_expectation(psi, n, 3, coeff, xm, zm);
    /* rejected arguments */
    const int bad[2] = {3, 3};
    cplx U4[16] = {0};
    if (oracle_apply_matrix(psi, n, bad, 2, U4) != -1) return 7;
    const int out_of_range[1] = {n};
    if (oracle_apply_matrix(psi, n, out_of_range, 1, U4) != -1) return 8;
    uint64_t xs[4] = {0, 1, 2, 1023};
    const int ccodes[2] = {13, 17}, ctg[12] = {0, 1, 0, 0, 0, 0, 0, 1, 2, 0, 0, 0};
    if (oracle_classical_run(2, ccodes, ctg, xs, 4) != 0) return 9;
    cplx col0[2 * N];
    for (int q = 0; q < n; ++q) {
        col0[2 * q] = 0.6;
        col0[2 * q + 1] = 0.8 * I;
    }
    const int pairs[4] = {0, 1, 2, 3};
    const uint64_t idx[3] = {0, 5, 1023};
    cplx amps[3];
    oracle_product_cz_amplitudes(n, col0, 2, pairs, 3, idx, amps);
    printf("oracle check: energy %.6f\n", e);
    free(psi);
    free(tmp);
    free(mats);
    return 0;
}
