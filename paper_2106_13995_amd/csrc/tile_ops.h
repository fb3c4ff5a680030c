// Device functions of LDS-resident tile passes (one tile of 2^m amplitudes
// per 256-thread workgroup, ops applied one after another in LDS).
#pragma once

#include "device_common.h"
#include "qsim_internal.h"

namespace qsim {

constexpr int kTileThreads = 256;
constexpr int kMaxTileHigh = 16;
constexpr int kPairBatch = 4;   // pairs a thread reads ahead in pair ops

template <typename T>
struct TileArgs {
    c2_t<T> *psi;
    const TileOp *ops;          // this pass's ops (global memory)
    const c2_t<T> *pool;        // this pass's matrices / diagonals (global memory)
    const double *trig;         // (cos, sin) of every parameter's half angle, for type-4 ops
    int nops;
    int npool;                  // complex entries in the pool
    int m, L, H;
    int hpos[kMaxTileHigh];
};

// Global index offset of tile-local index l: the low L bits stay, bit L+i of
// l moves to hpos[i].
template <typename T>
__device__ __forceinline__ uint64_t tile_scatter(const TileArgs<T> &a, uint32_t l) {
    uint64_t g = l & ((1u << a.L) - 1u);
    const uint32_t h = l >> a.L;
    for (int i = 0; i < a.H; ++i) g |= uint64_t((h >> i) & 1u) << a.hpos[i];
    return g;
}

__device__ __forceinline__ uint32_t insert_zeros32(uint32_t x, const int *pos, int np) {
    for (int i = 0; i < np; ++i) {
        const uint32_t lo = x & ((1u << pos[i]) - 1u);
        x = ((x - lo) << 1) | lo;
    }
    return x;
}

// Dense op on k <= 3 local positions: one thread per group of 2^k amplitudes.
// The matrix is read from LDS (the same address in every lane).
// 2 x 2 block U on tile position op.pos[0] for the pairs whose control
// positions (mask op.kin, all inside the tile) are 1: CX, CCX and other
// one-qubit blocks under controls touch only that part of the tile.
template <typename T>
__device__ __forceinline__ void tile_controlled(c2_t<T> *lds, const TileOp &op, const c2_t<T> *U, uint32_t M) {
    const uint32_t tb = 1u << op.pos[0], cm = uint32_t(op.kin), fixed = tb | cm;
    const uint32_t npairs = M >> __popc(fixed);
    const T u0r = U[0].x, u0i = U[0].y, u1r = U[1].x, u1i = U[1].y;
    const T u2r = U[2].x, u2i = U[2].y, u3r = U[3].x, u3i = U[3].y;
    // kPairBatch pairs per thread are read before any is written (distinct
    // pairs never share an address), so their LDS reads overlap
    for (uint32_t g0 = threadIdx.x; g0 < npairs; g0 += kPairBatch * kTileThreads) {
        uint32_t xs[kPairBatch];
        c2_t<T> a[kPairBatch], b[kPairBatch];
#pragma unroll
        for (int c = 0; c < kPairBatch; ++c) {
            // spread g over the free positions (zeros at the fixed ones, lowest first)
            const uint32_t g = g0 + uint32_t(c) * kTileThreads;
            uint32_t x = g, rest = fixed;
            while (rest) {
                const uint32_t bit = rest & (0u - rest);
                rest ^= bit;
                const uint32_t low = x & (bit - 1u);
                x = ((x - low) << 1) | low;
            }
            xs[c] = x | cm;
            if (g < npairs) {
                a[c] = lds[xs[c]];
                b[c] = lds[xs[c] | tb];
            }
        }
#pragma unroll
        for (int c = 0; c < kPairBatch; ++c) {
            if (g0 + uint32_t(c) * kTileThreads >= npairs) break;
            c2_t<T> y0, y1;
            y0.x = u0r * a[c].x - u0i * a[c].y + u1r * b[c].x - u1i * b[c].y;
            y0.y = u0r * a[c].y + u0i * a[c].x + u1r * b[c].y + u1i * b[c].x;
            y1.x = u2r * a[c].x - u2i * a[c].y + u3r * b[c].x - u3i * b[c].y;
            y1.y = u2r * a[c].y + u2i * a[c].x + u3r * b[c].y + u3i * b[c].x;
            lds[xs[c]] = y0;
            lds[xs[c] | tb] = y1;
        }
    }
}

template <typename T, int K>
__device__ __forceinline__ void tile_dense_small(c2_t<T> *lds, const TileOp &op, const c2_t<T> *U, uint32_t M) {
    constexpr int D = 1 << K;
    const uint32_t ngroups = M >> K;
    int pos[K];
#pragma unroll
    for (int b = 0; b < K; ++b) pos[b] = op.pos[b];
    uint32_t off[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < K; ++b)
            if ((j >> b) & 1) o |= 1u << pos[b];
        off[j] = o;
    }
    // small matrices live in registers for the whole op
    T ur[K <= 2 ? D * D : 1], ui[K <= 2 ? D * D : 1];
    if constexpr (K <= 2) {
#pragma unroll
        for (int e = 0; e < D * D; ++e) { ur[e] = U[e].x; ui[e] = U[e].y; }
    }
    for (uint32_t g = threadIdx.x; g < ngroups; g += kTileThreads) {
        uint32_t x = g;
#pragma unroll
        for (int b = 0; b < K; ++b) {
            const uint32_t lo = x & ((1u << pos[b]) - 1u);
            x = ((x - lo) << 1) | lo;
        }
        T vr[D], vi[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const c2_t<T> w = lds[x + off[j]];
            vr[j] = w.x; vi[j] = w.y;
        }
#pragma unroll
        for (int r = 0; r < D; ++r) {
            T orr = T(0), oi = T(0);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                if constexpr (K <= 2) {
                    cfma(orr, oi, ur[r * D + c], ui[r * D + c], vr[c], vi[c]);
                } else {
                    const c2_t<T> u = U[r * D + c];
                    cfma(orr, oi, u.x, u.y, vr[c], vi[c]);
                }
            }
            c2_t<T> w;
            w.x = orr; w.y = oi;
            lds[x + off[r]] = w;
        }
    }
}

// Dense op on k = 4..6 local positions: every output (group, row) is
// computed into registers from LDS, then written after a barrier.
template <typename T, int K>
__device__ __forceinline__ void tile_dense_wide(c2_t<T> *lds, const TileOp &op, const c2_t<T> *U, uint32_t M) {
    constexpr int D = 1 << K;
    int pos[K];
#pragma unroll
    for (int b = 0; b < K; ++b) pos[b] = op.pos[b];
    auto offset = [&pos](uint32_t j) {
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < K; ++b) o |= ((j >> b) & 1u) << pos[b];
        return o;
    };
    constexpr int kMaxPer = (1 << 13) / kTileThreads;   // M <= 2^13
    T orr[kMaxPer], oi[kMaxPer];
    const uint32_t per = (M + kTileThreads - 1) / kTileThreads;
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
        const uint32_t e = threadIdx.x + uint32_t(i) * kTileThreads;
        T ar = T(0), ai = T(0);
        if (uint32_t(i) < per && e < M) {
            const uint32_t r = e % D, g = e / D;
            uint32_t x = g;
#pragma unroll
            for (int b = 0; b < K; ++b) {
                const uint32_t lo = x & ((1u << pos[b]) - 1u);
                x = ((x - lo) << 1) | lo;
            }
            for (int c = 0; c < D; ++c) {
                const c2_t<T> v = lds[x + offset(uint32_t(c))];
                const c2_t<T> u = U[r * D + c];
                cfma(ar, ai, u.x, u.y, v.x, v.y);
            }
        }
        orr[i] = ar;
        oi[i] = ai;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
        const uint32_t e = threadIdx.x + uint32_t(i) * kTileThreads;
        if (uint32_t(i) >= per || e >= M) continue;
        const uint32_t r = e % D, g = e / D;
        uint32_t x = g;
#pragma unroll
        for (int b = 0; b < K; ++b) {
            const uint32_t lo = x & ((1u << pos[b]) - 1u);
            x = ((x - lo) << 1) | lo;
        }
        c2_t<T> w;
        w.x = orr[i]; w.y = oi[i];
        lds[x + offset(r)] = w;
    }
}

// Diagonal op: the bits of targets outside the tile are fixed for the whole
// tile (taken from its base index); the loop runs over the groups of the
// in-tile targets and skips diagonal entries equal to 1 (a branch that is
// uniform across the workgroup).
template <typename T>
__device__ __forceinline__ void tile_diag(c2_t<T> *lds, const TileOp &op, const c2_t<T> *Dg, uint64_t base,
                                          uint32_t M) {
    int jfix = 0;
    for (int i = 0; i < op.k - op.kin; ++i) jfix |= int((base >> op.gpos[i]) & 1ull) << op.gbit[i];
    const int kin = op.kin;
    const uint32_t ngroups = M >> kin;
    for (int c = 0; c < (1 << kin); ++c) {
        int j = jfix;
        uint32_t off = 0;
        for (int i = 0; i < kin; ++i)
            if ((c >> i) & 1) {
                j |= 1 << op.jbit[i];
                off |= 1u << op.pos[i];
            }
        const c2_t<T> d = Dg[j];
        if (d.x == T(1) && d.y == T(0)) continue;
        for (uint32_t g = threadIdx.x; g < ngroups; g += kTileThreads) {
            const uint32_t x = insert_zeros32(g, op.pos, kin) + off;
            const c2_t<T> w = lds[x];
            c2_t<T> o;
            o.x = d.x * w.x - d.y * w.y;
            o.y = d.x * w.y + d.y * w.x;
            lds[x] = o;
        }
    }
}

// Rotation exp(-i theta G / 2) (or its inverse) on local position p, given
// cs = cos(theta / 2) and sn = sin(theta / 2).
template <typename T>
__device__ __forceinline__ void tile_rotation(c2_t<T> *lds, int p, int gen, double cs, double sn, uint32_t M) {
    // [[a, b], [c, d]] as (re, im)
    T ar, ai, br, bi, cr, ci, dr, di;
    if (gen == 1) {        // X: [[c, -is], [-is, c]]
        ar = T(cs); ai = T(0); br = T(0); bi = T(-sn); cr = T(0); ci = T(-sn); dr = T(cs); di = T(0);
    } else if (gen == 2) { // Y: [[c, -s], [s, c]]
        ar = T(cs); ai = T(0); br = T(-sn); bi = T(0); cr = T(sn); ci = T(0); dr = T(cs); di = T(0);
    } else {               // Z: diag(e^{-i t/2}, e^{i t/2})
        ar = T(cs); ai = T(-sn); br = T(0); bi = T(0); cr = T(0); ci = T(0); dr = T(cs); di = T(sn);
    }
    const uint32_t bit = 1u << p, npairs = M >> 1;
    // kPairBatch pairs per thread are read before any is written (distinct
    // pairs never share an address), so their LDS reads overlap
    for (uint32_t g0 = threadIdx.x; g0 < npairs; g0 += kPairBatch * kTileThreads) {
        uint32_t xs[kPairBatch];
        c2_t<T> u[kPairBatch], v[kPairBatch];
#pragma unroll
        for (int c = 0; c < kPairBatch; ++c) {
            const uint32_t g = g0 + uint32_t(c) * kTileThreads;
            const uint32_t lo = g & (bit - 1u);
            xs[c] = ((g - lo) << 1) | lo;
            if (g < npairs) {
                u[c] = lds[xs[c]];
                v[c] = lds[xs[c] | bit];
            }
        }
#pragma unroll
        for (int c = 0; c < kPairBatch; ++c) {
            if (g0 + uint32_t(c) * kTileThreads >= npairs) break;
            T o0r = T(0), o0i = T(0), o1r = T(0), o1i = T(0);
            cfma(o0r, o0i, ar, ai, u[c].x, u[c].y);
            cfma(o0r, o0i, br, bi, v[c].x, v[c].y);
            cfma(o1r, o1i, cr, ci, u[c].x, u[c].y);
            cfma(o1r, o1i, dr, di, v[c].x, v[c].y);
            c2_t<T> w0, w1;
            w0.x = o0r; w0.y = o0i;
            w1.x = o1r; w1.y = o1i;
            lds[xs[c]] = w0;
            lds[xs[c] | bit] = w1;
        }
    }
}

}  // namespace qsim
