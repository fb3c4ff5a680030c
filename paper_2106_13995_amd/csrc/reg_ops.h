// Register-op device functions of register-staged tile passes (gfx950),
// shared by the single-state tile passes and the batched kernel.
//
// A thread holds 2^RA amplitudes in registers (vr, vi).  Ops name register
// bits below R; when RA > R the bits from R up select independent copies
// (the batched reverse sweep keeps psi and lambda side by side) and every op
// acts on each copy alike.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "qsim_internal.h"

namespace qsim {

// Op descriptors, stage descriptors and gate matrices are read through the
// constant address space: uniform loads become scalar loads into SGPRs, which
// the vector FMAs take as operands directly.
#define QSIM_CONST __attribute__((address_space(4)))
typedef const QSIM_CONST RegOp CRegOp;
typedef const QSIM_CONST RegStage CRegStage;
template <typename T> using CT = const QSIM_CONST T;   // interleaved (re, im) matrix entries


// Deposits the bits of j into the set bits of mask (compile-time).
__host__ __device__ constexpr int deposit(int j, int mask) {
    int out = 0, b = 0;
    for (int p = 0; p < 31; ++p)
        if ((mask >> p) & 1) {
            if ((j >> b) & 1) out |= 1 << p;
            ++b;
        }
    return out;
}

__host__ __device__ constexpr int popcount_c(int v) {
    int c = 0;
    while (v) {
        c += v & 1;
        v >>= 1;
    }
    return c;
}

// Dense gate on the register bits of MASK: for every group of register
// indices that agree outside MASK, multiply by the 2^k x 2^k matrix.
template <typename T, int R, int MASK>
__device__ __forceinline__ void apply_mask(T *vr, T *vi, CT<T> *U) {
    constexpr int K = popcount_c(MASK);
    constexpr int D = 1 << K;
    constexpr int NA = 1 << R;
    if constexpr (K >= 3) {
        // row by row: one matrix row in registers at a time, outputs kept
        // aside until every row has read the inputs
        T outr[NA], outi[NA];
#pragma unroll
        for (int rr = 0; rr < D; ++rr) {
            T ur[D], ui[D];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                ur[c] = U[2 * (rr * D + c)];
                ui[c] = U[2 * (rr * D + c) + 1];
            }
#pragma unroll
            for (int g = 0; g < NA; ++g) {
                if (g & MASK) continue;
                T orr = T(0), oi = T(0);
#pragma unroll
                for (int c = 0; c < D; ++c)
                    cfma(orr, oi, ur[c], ui[c], vr[g | deposit(c, MASK)], vi[g | deposit(c, MASK)]);
                outr[g | deposit(rr, MASK)] = orr;
                outi[g | deposit(rr, MASK)] = oi;
            }
        }
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            vr[i] = outr[i];
            vi[i] = outi[i];
        }
        return;
    }
    T ur[D * D], ui[D * D];
    {
#pragma unroll
        for (int e = 0; e < D * D; ++e) {
            ur[e] = U[2 * e];
            ui[e] = U[2 * e + 1];
        }
    }
#pragma unroll
    for (int g = 0; g < NA; ++g) {
        if (g & MASK) continue;
        T xr[D], xi[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            xr[j] = vr[g | deposit(j, MASK)];
            xi[j] = vi[g | deposit(j, MASK)];
        }
#pragma unroll
        for (int rr = 0; rr < D; ++rr) {
            T orr = T(0), oi = T(0);
#pragma unroll
            for (int c = 0; c < D; ++c) cfma(orr, oi, ur[rr * D + c], ui[rr * D + c], xr[c], xi[c]);
            vr[g | deposit(rr, MASK)] = orr;
            vi[g | deposit(rr, MASK)] = oi;
        }
    }
}

template <typename T, int R, int MASK>
__device__ __forceinline__ void dispatch_dense(int rmask, T *vr, T *vi, CT<T> *U) {
    if constexpr (MASK < (1 << R)) {
        if constexpr (popcount_c(MASK) <= 3) {
            if (rmask == MASK) {
                apply_mask<T, R, MASK>(vr, vi, U);
                return;
            }
        }
        dispatch_dense<T, R, MASK + 1>(rmask, vr, vi, U);
    }
}

// Real rotation [[c, -s], [s, c]] on register bit B as three lifting steps,
// in place: x0 += p x1, x1 += u x0, x0 += p x1 (p = -s / (1 + c), u = s).
template <typename T, int R, int B>
__device__ __forceinline__ void lift_bit(T *vr, T *vi, T p, T u) {
#pragma unroll
    for (int g = 0; g < (1 << R); ++g) {
        if (g & (1 << B)) continue;
        const int h = g | (1 << B);
        vr[g] = fma(p, vr[h], vr[g]);
        vi[g] = fma(p, vi[h], vi[g]);
        vr[h] = fma(u, vr[g], vr[h]);
        vi[h] = fma(u, vi[g], vi[h]);
        vr[g] = fma(p, vr[h], vr[g]);
        vi[g] = fma(p, vi[h], vi[g]);
    }
}

// [[0, -1], [1, 0]] on register bit B: (x0, x1) <- (-x1, x0).
template <typename T, int R, int B>
__device__ __forceinline__ void swap_bit(T *vr, T *vi) {
#pragma unroll
    for (int g = 0; g < (1 << R); ++g) {
        if (g & (1 << B)) continue;
        const int h = g | (1 << B);
        const T xr = vr[g], xi = vi[g];
        vr[g] = -vr[h];
        vi[g] = -vi[h];
        vr[h] = xr;
        vi[h] = xi;
    }
}

template <typename T, int R, int B>
__device__ __forceinline__ void dispatch_bit(int bit, int type, T *vr, T *vi, CT<T> *P) {
    if constexpr (B < R) {
        if (bit == B) {
            if (type == 3)
                lift_bit<T, R, B>(vr, vi, P[0], P[1]);
            else
                swap_bit<T, R, B>(vr, vi);
            return;
        }
        dispatch_bit<T, R, B + 1>(bit, type, vr, vi, P);
    }
}

// Phase table over the register bits: amplitude i times entry i (entry 0 is
// 1 by construction: every merged phase sits on a bit's 1 half).
template <typename T, int R, int RA = R>
__device__ __forceinline__ void apply_table(T *vr, T *vi, CT<T> *P) {
#pragma unroll
    for (int i = 1; i < (1 << RA); ++i) {
        const int e = i & ((1 << R) - 1);
        if (e == 0) continue;
        const T dx = P[2 * e], dy = P[2 * e + 1];
        const T xr = vr[i], xi = vi[i];
        vr[i] = dx * xr - dy * xi;
        vi[i] = dx * xi + dy * xr;
    }
}

// Factor (dx, dy) on the register amplitudes whose bits in MASK are all 1.
template <typename T, int R, int MASK>
__device__ __forceinline__ void dispatch_ones(int rmask, T *vr, T *vi, T dx, T dy) {
    if constexpr (MASK < (1 << R)) {
        if (rmask == MASK) {
#pragma unroll
            for (int i = 0; i < (1 << R); ++i) {
                if ((i & MASK) != MASK) continue;
                const T xr = vr[i], xi = vi[i];
                vr[i] = dx * xr - dy * xi;
                vi[i] = dx * xi + dy * xr;
            }
            return;
        }
        dispatch_ones<T, R, MASK + 1>(rmask, vr, vi, dx, dy);
    }
}

// Diagonal gate: the diagonal index of register amplitude i collects bits
// from the tile's fixed (out-of-tile) qubits, the thread id and i itself.
template <typename T, int R>
__device__ __forceinline__ void apply_diag(T *vr, T *vi, CRegOp &op, CT<T> *Dg, uint64_t base, uint32_t t) {
    constexpr int NA = 1 << R;
    int jt = 0;
    for (int b = 0; b < op.nout; ++b) jt |= int((base >> op.gp[b]) & 1ull) << op.gj[b];
    for (int b = 0; b < op.nthr; ++b) jt |= int((t >> op.tb[b]) & 1u) << op.tj[b];
    if (op.type == 2) {
        // one non-unit entry: amplitude i changes only where its index bits match
        int regj = 0, rval = 0;
        for (int b = 0; b < op.nreg; ++b) {
            regj |= 1 << op.rj[b];
            rval |= ((op.jmatch >> op.rj[b]) & 1) << op.rb[b];
        }
        if (((jt ^ op.jmatch) & ~regj) != 0) return;
        const T dx = Dg[2 * op.jmatch], dy = Dg[2 * op.jmatch + 1];
        const int rmask = op.rmask;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            if ((i & rmask) != rval) continue;
            const T xr = vr[i], xi = vi[i];
            vr[i] = dx * xr - dy * xi;
            vi[i] = dx * xi + dy * xr;
        }
    } else {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            int j = jt;
            for (int b = 0; b < op.nreg; ++b) j |= ((i >> op.rb[b]) & 1) << op.rj[b];
            const T dx = Dg[2 * j], dy = Dg[2 * j + 1];
            const T xr = vr[i], xi = vi[i];
            vr[i] = dx * xr - dy * xi;
            vi[i] = dx * xi + dy * xr;
        }
    }
}

// Op codes (host side: op_code): dense on register mask m < 32 -> m; lifting
// rotation on bit b -> 64 + b; signed exchange on bit b -> 72 + b; factor on
// the all-ones amplitudes of register mask m -> 128 + m; X on bit b under
// controls (an exchange of the pair) -> 160 + b; phase table -> 200; any
// other diagonal -> 201; 2 x 2 block on bit b under controls -> 210 + b.
// One flat compare chain on the uniform code, one join: the amplitude
// registers keep a single home across ops.
template <int C, int R>
__host__ __device__ constexpr bool code_valid() {
    if (C < 32) return C > 0 && C < (1 << R) && popcount_c(C) <= 3;
    if (C >= 64 && C < 72) return C - 64 < R;
    if (C >= 72 && C < 80) return C - 72 < R;
    if (C >= 128 && C < 160) return C - 128 < (1 << R);
    if (C >= 160 && C < 168) return C - 160 < R;
    if (C >= 210 && C < 218) return C - 210 < R;
    return C == 200 || C == 201;
}

// 2 x 2 block U on register bit B, applied to the pairs whose register
// control bits (rmask) are 1, in lanes and blocks whose thread and
// out-of-tile control bits are 1; elsewhere the pair is kept as it is
// (a select, so the amplitudes stay in place).
template <typename T, int R, int B>
__device__ __forceinline__ void controlled_bit(T *vr, T *vi, CRegOp &op, CT<T> *U, uint64_t base, uint32_t t) {
    const uint64_t gmask = uint64_t(uint32_t(op.gp[0])) | (uint64_t(uint32_t(op.gp[1])) << 32);
    const uint32_t tm = uint32_t(op.tb[0]);
    const bool on = ((base & gmask) == gmask) && ((t & tm) == tm);
    const int rc = op.rmask;
    const T u0r = U[0], u0i = U[1], u1r = U[2], u1i = U[3], u2r = U[4], u2i = U[5], u3r = U[6], u3i = U[7];
#pragma unroll
    for (int g = 0; g < (1 << R); ++g) {
        if (g & (1 << B)) continue;
        const int h = g | (1 << B);
        const bool act = on && ((g & rc) == rc);
        const T x0r = vr[g], x0i = vi[g], x1r = vr[h], x1i = vi[h];
        const T y0r = u0r * x0r - u0i * x0i + u1r * x1r - u1i * x1i;
        const T y0i = u0r * x0i + u0i * x0r + u1r * x1i + u1i * x1r;
        const T y1r = u2r * x0r - u2i * x0i + u3r * x1r - u3i * x1i;
        const T y1i = u2r * x0i + u2i * x0r + u3r * x1i + u3i * x1r;
        vr[g] = act ? y0r : x0r;
        vi[g] = act ? y0i : x0i;
        vr[h] = act ? y1r : x1r;
        vi[h] = act ? y1i : x1i;
    }
}

// X on register bit B under controls (masks as controlled_bit): the pair
// is exchanged where every control is 1 (selects only).
template <typename T, int R, int B>
__device__ __forceinline__ void controlled_x_bit(T *vr, T *vi, CRegOp &op, uint64_t base, uint32_t t) {
    const uint64_t gmask = uint64_t(uint32_t(op.gp[0])) | (uint64_t(uint32_t(op.gp[1])) << 32);
    const uint32_t tm = uint32_t(op.tb[0]);
    const bool on = ((base & gmask) == gmask) && ((t & tm) == tm);
    const int rc = op.rmask;
#pragma unroll
    for (int g = 0; g < (1 << R); ++g) {
        if (g & (1 << B)) continue;
        const int h = g | (1 << B);
        const bool act = on && ((g & rc) == rc);
        const T x0r = vr[g], x0i = vi[g], x1r = vr[h], x1i = vi[h];
        vr[g] = act ? x1r : x0r;
        vi[g] = act ? x1i : x0i;
        vr[h] = act ? x0r : x1r;
        vi[h] = act ? x0i : x1i;
    }
}

// Plane rotation [[c, -s], [s, c]] of (a, b) as three lifting steps, each
// one multiply-add in place: for c >= 0, with P = -s / (1 + c),
//   a += P b;  b += s a;  a += P b;
// for c < 0 it is minus the rotation by (-c, -s), with P = s / (1 - c),
//   a += P b;  b = s a - b;  a = P b - a
// (|P| <= 1 either way).  `neg` selects the second form.
template <typename T>
__device__ __forceinline__ void lift3(T &a, T &b, T P, T s, bool neg) {
    if (!neg) {
        a = fma(P, b, a);
        b = fma(s, a, b);
        a = fma(P, b, a);
    } else {
        a = fma(P, b, a);
        b = fma(s, a, -b);
        a = fma(P, b, -a);
    }
}

// Rotation exp(-i theta G / 2) on register bit B (G = X for GEN 1, Y for
// GEN 2) given c = cos(theta / 2), s = sin(theta / 2):
//   Y: [[c, -s], [s, c]] on the real parts and on the imaginary parts;
//   X: [[c, -is], [-is, c]] is [[c, s], [-s, c]] on (re x0, im x1) and
//      [[c, -s], [s, c]] on (im x0, re x1).
template <typename T, int RA, int B, int GEN, bool NEG>
__device__ __forceinline__ void brot_bit_lift(T *vr, T *vi, T Pp, T sp, T Pm, T sm) {
#pragma unroll
    for (int g = 0; g < (1 << RA); ++g) {
        if (g & (1 << B)) continue;
        const int h = g | (1 << B);
        if constexpr (GEN == 2) {
            lift3(vr[g], vr[h], Pp, sp, NEG);
            lift3(vi[g], vi[h], Pp, sp, NEG);
        } else {
            lift3(vr[g], vi[h], Pm, sm, NEG);
            lift3(vi[g], vr[h], Pp, sp, NEG);
        }
    }
}

// The rotation's lifting multiplier P (as lift3: -s / (1 + c), or
// s / (1 - c) with `neg` when c < 0) and its sine, in double.
template <typename T, int RA, int B, int GEN>
__device__ __forceinline__ void brot_bit(T *vr, T *vi, double P, double s, bool neg) {
    const T Pp = T(P), sp = T(s), Pm = -Pp, sm = -sp;
    if (neg)
        brot_bit_lift<T, RA, B, GEN, true>(vr, vi, Pp, sp, Pm, sm);
    else
        brot_bit_lift<T, RA, B, GEN, false>(vr, vi, Pp, sp, Pm, sm);
}

// Whether the one bit an op names outside the registers (a thread bit in
// tb[0] or an out-of-tile qubit in gp) is 1 for this thread and tile.
__device__ __forceinline__ bool outer_bit(CRegOp &op, uint64_t base, uint32_t t) {
    const uint64_t gmask = uint64_t(uint32_t(op.gp[0])) | (uint64_t(uint32_t(op.gp[1])) << 32);
    return ((base & gmask) != 0) || ((t & uint32_t(op.tb[0])) != 0u);
}

// exp(-i theta Z / 2) = diag(c - is, c + is) on the bit the op names: a
// register bit (rmask), a thread bit or an out-of-tile bit.  Amplitude
// (re, im) turns by [[c, -s'], [s', c]] with s' = s where the bit is 1 and
// -s where it is 0.
template <typename T, int RA, bool NEG>
__device__ __forceinline__ void brot_z_lift(T *vr, T *vi, CRegOp &op, T Pp, T sp, uint64_t base, uint32_t t) {
    const int rm = op.rmask;
    if (rm) {
#pragma unroll
        for (int i = 0; i < (1 << RA); ++i) {
            const bool one = (i & rm) != 0;
            lift3(vr[i], vi[i], one ? Pp : -Pp, one ? sp : -sp, NEG);
        }
    } else {
        const bool up = outer_bit(op, base, t);
        const T P = up ? Pp : -Pp, s = up ? sp : -sp;
#pragma unroll
        for (int i = 0; i < (1 << RA); ++i) lift3(vr[i], vi[i], P, s, NEG);
    }
}

template <typename T, int RA>
__device__ __forceinline__ void brot_z(T *vr, T *vi, CRegOp &op, double P, double s, bool neg, uint64_t base,
                                       uint32_t t) {
    if (neg)
        brot_z_lift<T, RA, true>(vr, vi, op, T(P), T(s), base, t);
    else
        brot_z_lift<T, RA, false>(vr, vi, op, T(P), T(s), base, t);
}

// exp(-i theta Z / 2) on register bit B (lift3 multipliers as brot_bit).
template <typename T, int RA, int B>
__device__ __forceinline__ void brot_z_bit(T *vr, T *vi, double P, double s, bool neg) {
    const T Pp = T(P), sp = T(s);
#pragma unroll
    for (int i = 0; i < (1 << RA); ++i) {
        const bool one = (i >> B) & 1;
        if (neg)
            lift3(vr[i], vi[i], one ? Pp : -Pp, one ? sp : -sp, true);
        else
            lift3(vr[i], vi[i], one ? Pp : -Pp, one ? sp : -sp, false);
    }
}

// Batched-circuit codes: rotation exp(-i theta G / 2) of parameter moff,
// whose lifting form (P, s, cos) of the half angle is at trig[4 * moff]
// (inverse when jmatch is 1: P and s negated): X on bit b -> 220 + b, Y on
// bit b -> 228 + b, Z anywhere -> 236.
// Two rotations on one register bit b, the first (G1 = X or Y, parameter
// moff) then the second (G2 = X, Y or Z, parameter gj[0]), both forward:
// 288 + 8 ((G1 - 1) 3 + G2 - 1) + b.
template <int C, int R>
__host__ __device__ constexpr bool ext_code_valid() {
    if (C >= 220 && C < 228) return C - 220 < R;
    if (C >= 228 && C < 236) return C - 228 < R;
    if (C >= 288 && C < 336) return (C - 288) % 8 < R;
    return C == 236;
}

// Op `code` (valid for R register bits) on an amplitude array of RA >= R
// register bits; with EXT, the batched-circuit codes too (trig: the
// circuit's rotation table).  One flat compare chain on the uniform code.
template <typename T, int R, int C, int RA = R, bool EXT = false>
__device__ __forceinline__ void run_op(int code, T *vr, T *vi, CRegOp &op, CT<T> *U, uint64_t base, uint32_t t,
                                       const QSIM_CONST double *trig = nullptr) {
    if constexpr (C <= (EXT ? 335 : 217)) {
        if constexpr (code_valid<C, R>() || (EXT && ext_code_valid<C, R>())) {
            if (code == C) {
                if constexpr (C >= 288) {
                    constexpr int B = (C - 288) % 8, G1 = (C - 288) / 24 + 1, G2 = ((C - 288) / 8) % 3 + 1;
                    const int m2 = op.gj[0];
                    brot_bit<T, RA, B, G1>(vr, vi, trig[4 * op.moff], trig[4 * op.moff + 1], trig[4 * op.moff + 2] < 0.0);
                    if constexpr (G2 == 3)
                        brot_z_bit<T, RA, B>(vr, vi, trig[4 * m2], trig[4 * m2 + 1], trig[4 * m2 + 2] < 0.0);
                    else
                        brot_bit<T, RA, B, G2>(vr, vi, trig[4 * m2], trig[4 * m2 + 1], trig[4 * m2 + 2] < 0.0);
                } else if constexpr (C >= 220) {
                    const double P = op.jmatch ? -trig[4 * op.moff] : trig[4 * op.moff];
                    const double sn = op.jmatch ? -trig[4 * op.moff + 1] : trig[4 * op.moff + 1];
                    const bool neg = trig[4 * op.moff + 2] < 0.0;
                    if constexpr (C < 228)
                        brot_bit<T, RA, C - 220, 1>(vr, vi, P, sn, neg);
                    else if constexpr (C < 236)
                        brot_bit<T, RA, C - 228, 2>(vr, vi, P, sn, neg);
                    else
                        brot_z<T, RA>(vr, vi, op, P, sn, neg, base, t);
                } else if constexpr (C < 32) {
                    if constexpr (RA > R && popcount_c(C) >= 3) {
                        // row by row keeps all outputs aside: one copy at a time
#pragma unroll
                        for (int h = 0; h < (1 << (RA - R)); ++h) apply_mask<T, R, C>(vr + (h << R), vi + (h << R), U);
                    } else {
                        apply_mask<T, RA, C>(vr, vi, U);
                    }
                } else if constexpr (C < 72) {
                    lift_bit<T, RA, C - 64>(vr, vi, U[0], U[1]);
                } else if constexpr (C < 80) {
                    swap_bit<T, RA, C - 72>(vr, vi);
                } else if constexpr (C >= 160 && C < 168) {
                    controlled_x_bit<T, RA, C - 160>(vr, vi, op, base, t);
                } else if constexpr (C < 160) {
                    const uint64_t gmask = uint64_t(uint32_t(op.gp[0])) | (uint64_t(uint32_t(op.gp[1])) << 32);
                    const uint32_t tm = uint32_t(op.tb[0]);
                    // amplitudes whose out-of-tile or thread bits do not match
                    // multiply by 1 (exact)
                    const bool on = ((base & gmask) == gmask) && ((t & tm) == tm);
                    const T dx = on ? U[0] : T(1), dy = on ? U[1] : T(0);
#pragma unroll
                    for (int i = 0; i < (1 << RA); ++i) {
                        if ((i & (C - 128)) != (C - 128)) continue;
                        const T xr = vr[i], xi = vi[i];
                        vr[i] = dx * xr - dy * xi;
                        vi[i] = dx * xi + dy * xr;
                    }
                } else if constexpr (C == 200) {
                    apply_table<T, R, RA>(vr, vi, U);
                } else if constexpr (C == 201) {
                    apply_diag<T, RA>(vr, vi, op, U, base, t);
                } else {
                    controlled_bit<T, RA, C - 210>(vr, vi, op, U, base, t);
                }
                return;
            }
        }
        run_op<T, R, C + 1, RA, EXT>(code, vr, vi, op, U, base, t, trig);
    } else {
        // the host emits valid codes only; telling the compiler so keeps the
        // amplitudes from being carried through a no-op path
        __builtin_unreachable();
    }
}

// LDS address part of thread t: the XOR of vec[b] over its set bits (the
// eight entries read first, then combined without branches).
template <typename T>
__device__ __forceinline__ uint32_t thread_part(uint32_t t, const QSIM_CONST uint32_t *vec) {
    uint32_t v[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) v[b] = vec[b];
    uint32_t a = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) a ^= (0u - ((t >> b) & 1u)) & v[b];
    return a;
}

}  // namespace qsim
