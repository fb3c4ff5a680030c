// Expectation values of Pauli sums whose X masks are 0 or one qubit: the
// diagonal group (products of Z) and groups of X_h / Y_h terms, which is the
// form of the Ising-type observables of variational training (paper, Sec. I:
// models are trained on expectation values of simulated circuits).
//
// <psi|H|psi> = sum_y conj(psi_y) (H psi)_y, read once per pass from HBM.  A
// pass holds, per 64-lane wavefront, tiles of 2^(6+R) amplitudes (R = 4): lane bit b
// is qubit lane_q[b] (the low 5 (complex64) / 4 (complex128) qubits first, so
// 32 / 16 consecutive lanes read 256 contiguous bytes), register bit b of a
// lane's 2^R amplitudes is qubit reg_q[b].  No LDS: a group X_h / Y_h on a
// register qubit pairs registers of one lane; on a lane qubit each lane takes
// its partner's amplitude by a cross-lane exchange.  The diagonal group sums
// w_t (-1)^{|y & z_t|} |psi_y|^2: the sign splits into the lane/block part of
// z_t (one parity per term and tile) and its register part mu_t, and
// sum_k (-1)^{|mu & k|} |a_k|^2 over a lane's registers is the Walsh-Hadamard
// transform of |a|^2, computed in place; terms sharing mu share one
// multiply by its entry.  Everything after the amplitudes'
// conversion is double precision; each lane accumulates its tiles in order,
// and a fixed-order wave sum gives one partial per workgroup.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "qsim_internal.h"

namespace qsim {

// amplitudes as clang vectors (the nontemporal load builtin takes them)
template <typename T> struct EV;
template <> struct EV<float> { using type = f32x2; };
template <> struct EV<double> { using type = f64x2; };
template <typename T> using ev_t = typename EV<T>::type;

struct SimpleTerm {   // as the host's device term record
    double wr, wi;
    uint64_t z;
    uint64_t pad_;
};

// sum over pairs (k, k ^ X) with bit X of k clear of conj(a_k) a_{k^X}:
// real part into sr, imaginary part into si (when WITH_B).
template <int NA, int X, bool WITH_B>
__device__ __forceinline__ void register_pairs(const f64x2 (&a)[NA], double &sr, double &si) {
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        if (k & X) continue;
        const double ar = a[k].x, ai = a[k].y;
        const double br = a[k ^ X].x, bi = a[k ^ X].y;
        sr = fma(ar, br, sr);
        sr = fma(ai, bi, sr);
        if (WITH_B) {
            si = fma(ar, bi, si);
            si = fma(-ai, br, si);
        }
    }
}

template <int NA, bool WITH_B>
__device__ __forceinline__ void register_group(const f64x2 (&a)[NA], int b, double &sr, double &si) {
    switch (b) {
        case 0: register_pairs<NA, 1, WITH_B>(a, sr, si); break;
        case 1: register_pairs<NA, 2, WITH_B>(a, sr, si); break;
        case 2: register_pairs<NA, 4, WITH_B>(a, sr, si); break;
        case 3: register_pairs<NA, 8, WITH_B>(a, sr, si); break;
        default:
            if constexpr (NA == 32) register_pairs<NA, 16, WITH_B>(a, sr, si);
            break;
    }
}

// One 32-bit word of lane (lane ^ 2^B): a quad permutation (DPP, a vector
// ALU move) for B = 0, 1, a swizzle within 32 lanes for B = 2..4, a
// permutation through the LDS crossbar for B = 5.
template <int B>
__device__ __forceinline__ int xor_lane(int v) {
    if constexpr (B == 0)
        return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad lanes 1,0,3,2
    else if constexpr (B == 1)
        return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad lanes 2,3,0,1
    else if constexpr (B < 5)
        return __builtin_amdgcn_ds_swizzle(v, 0x1F | ((1 << B) << 10));   // and 31, xor 2^B
    else
        return __builtin_amdgcn_ds_bpermute(int((threadIdx.x ^ 32u) << 2), v);
}

// The partner's double across lane bit B.  With FROM_FLOAT the value is a
// converted float (complex64 amplitudes): off the quad permutations it
// travels as that float (one word instead of two; both conversions exact).
template <int B, bool FROM_FLOAT>
__device__ __forceinline__ double xor_lane_d(double v) {
    if constexpr (FROM_FLOAT && B >= 2) {
        return double(__builtin_bit_cast(float, xor_lane<B>(__builtin_bit_cast(int, float(v)))));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = uint32_t(xor_lane<B>(int(uint32_t(u)))), hi = uint32_t(xor_lane<B>(int(uint32_t(u >> 32))));
        return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
    }
}

// Every lane adds Re / (+-)Im of conj(a_k) times its partner's a_k across lane
// bit B: summed over all lanes this is twice the sum over pairs (the Y part
// with the sign of the lower member).
template <int NA, bool WITH_B, int B, bool FROM_FLOAT>
__device__ __forceinline__ void lane_pairs(const f64x2 (&a)[NA], double &sr, double &si) {
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        // chunks of eight: the scheduler would otherwise hoist every
        // exchange ahead of the products, holding 2 x 2^R doubles at once
        if (k % 8 == 0) __builtin_amdgcn_sched_barrier(0);
        const double pr = xor_lane_d<B, FROM_FLOAT>(a[k].x);
        const double pi = xor_lane_d<B, FROM_FLOAT>(a[k].y);
        sr = fma(a[k].x, pr, sr);
        sr = fma(a[k].y, pi, sr);
        if (WITH_B) {
            si = fma(a[k].x, pi, si);
            si = fma(-a[k].y, pr, si);
        }
    }
}

template <int NA, bool WITH_B, bool FROM_FLOAT>
__device__ __forceinline__ void lane_group(const f64x2 (&a)[NA], int b, double &sr, double &si) {
    switch (b) {
        case 0: lane_pairs<NA, WITH_B, 0, FROM_FLOAT>(a, sr, si); break;
        case 1: lane_pairs<NA, WITH_B, 1, FROM_FLOAT>(a, sr, si); break;
        case 2: lane_pairs<NA, WITH_B, 2, FROM_FLOAT>(a, sr, si); break;
        case 3: lane_pairs<NA, WITH_B, 3, FROM_FLOAT>(a, sr, si); break;
        case 4: lane_pairs<NA, WITH_B, 4, FROM_FLOAT>(a, sr, si); break;
        default: lane_pairs<NA, WITH_B, 5, FROM_FLOAT>(a, sr, si); break;
    }
}

template <typename T, int R>
__global__ void __launch_bounds__(64)
k_expect_simple(const c2_t<T> *__restrict__ psi, const ExpSimplePass p, const SimpleTerm *__restrict__ terms,
                uint64_t ntiles, double *__restrict__ partials) {
    constexpr int NA = 1 << R;
    static_assert(R == kExpSimpleR, "diag_mu holds 2^kExpSimpleR + 1 offsets");
    const unsigned lane = threadIdx.x;
    uint64_t toff = 0;
    for (int b = 0; b < 6; ++b) toff |= uint64_t((lane >> b) & 1u) << p.lane_q[b];
    uint64_t roff[R];
#pragma unroll
    for (int b = 0; b < R; ++b) roff[b] = 1ull << p.reg_q[b];
    double acc = 0.0;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // the tile's out-of-tile bits: zeros inserted at the tile qubits
        uint64_t base = tile;
        for (int i = 0; i < p.ntile_q; ++i) {
            const uint64_t lo = base & ((1ull << p.tile_q[i]) - 1ull);
            base = ((base - lo) << 1) | lo;
        }
        const uint64_t bt = base | toff;
        // amplitudes in double from here on (converted once: the sums need
        // double products, and one converted copy is all a lane holds)
        f64x2 a[NA];
        const ev_t<T> *ps = reinterpret_cast<const ev_t<T> *>(psi);
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            uint64_t off = bt;
#pragma unroll
            for (int b = 0; b < R; ++b)
                if ((k >> b) & 1) off |= roff[b];
            const ev_t<T> v = __builtin_nontemporal_load(ps + off);
            a[k] = f64x2{double(v.x), double(v.y)};
        }
        for (int g = 0; g < p.nreg_g; ++g) {
            double sr = 0.0, si = 0.0;
            if (p.reg_B[g] != 0.0)
                register_group<NA, true>(a, p.reg_bit[g], sr, si);
            else
                register_group<NA, false>(a, p.reg_bit[g], sr, si);
            acc += 2.0 * (p.reg_A[g] * sr + p.reg_B[g] * si);
        }
        for (int g = 0; g < p.nlane_g; ++g) {
            const unsigned mask = 1u << p.lane_bit[g];
            double sr = 0.0, si = 0.0;
            constexpr bool FF = sizeof(T) == 4;
            if (p.lane_B[g] != 0.0)
                lane_group<NA, true, FF>(a, p.lane_bit[g], sr, si);
            else
                lane_group<NA, false, FF>(a, p.lane_bit[g], sr, si);
            // Im part: the lower member of each pair carries it with +, the
            // upper with - (its product is the conjugate)
            acc += p.lane_A[g] * sr + ((lane & mask) ? -p.lane_B[g] : p.lane_B[g]) * si;
        }
        if (p.diag) {
            double w[NA];
#pragma unroll
            for (int k = 0; k < NA; ++k) w[k] = fma(a[k].x, a[k].x, a[k].y * a[k].y);
#pragma unroll
            for (int bit = 1; bit < NA; bit <<= 1) {
#pragma unroll
                for (int k = 0; k < NA; ++k) {
                    if (k & bit) continue;
                    const double u = w[k], v = w[k | bit];
                    w[k] = u + v;
                    w[k | bit] = u - v;
                }
            }
            // Each term's sign is the parity of its Z mask over the block bits
            // (the same on every lane: a scalar choice), its lane part zl
            // (pad_ holds mu | zl << 8) and its register part mu, which
            // selects the transform entry.  The terms come grouped by mu:
            // each group's signed weights are summed, then one product with
            // its entry, so no entry is chosen at run time.
#pragma unroll
            for (int mu = 0; mu < NA; ++mu) {
                const int t0 = p.diag_mu[mu], t1 = p.diag_mu[mu + 1];
                if (t0 == t1) continue;
                double c = 0.0;
                for (int t = t0; t < t1; ++t) {
                    const SimpleTerm e = terms[t];
                    const uint32_t zl = uint32_t(e.pad_ >> 8);
                    const bool neg = ((__popcll(e.z & base) + __popc(zl & lane)) & 1) != 0;
                    c += neg ? -e.wr : e.wr;
                }
                acc = fma(c, w[mu], acc);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) partials[blockIdx.x] = acc;
}

int expect_simple_grid(uint64_t ntiles) {
    // as many 64-lane workgroups as are resident at once: three per SIMD
    // (about 135 VGPRs per lane)
    return int(std::max<uint64_t>(1, std::min<uint64_t>(ntiles, 256ull * 4 * 3)));
}

hipError_t launch_expect_simple(qsim_state s, const ExpSimplePass &p, const void *dev_terms, double *partials,
                                int *nwritten) {
    const int R = kExpSimpleR;
    if (p.R != R || s->n < 6 + R) return hipErrorInvalidValue;
    const uint64_t ntiles = 1ull << (s->n - 6 - R);
    const int grid = expect_simple_grid(ntiles);
    const SimpleTerm *terms = static_cast<const SimpleTerm *>(dev_terms);
    if (s->dtype == QSIM_C64)
        hipLaunchKernelGGL((k_expect_simple<float, 4>), dim3(grid), dim3(64), 0, s->stream,
                           static_cast<const float2 *>(s->data), p, terms, ntiles, partials);
    else
        hipLaunchKernelGGL((k_expect_simple<double, 4>), dim3(grid), dim3(64), 0, s->stream,
                           static_cast<const double2 *>(s->data), p, terms, ntiles, partials);
    *nwritten = grid;
    return hipGetLastError();
}

}  // namespace qsim
