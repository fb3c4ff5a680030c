// HIP kernels for gfx950 (CDNA4, 64-wide wavefronts): gate sweeps over HBM,
// LDS tile passes, basis-state initialisation and expectation values.
//
// Amplitudes are interleaved complex (float2 for complex64, double2 for
// complex128).  Index arithmetic is 64-bit: a state holds up to 2^35
// amplitudes.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "qsim_internal.h"
#include "tile_ops.h"

namespace qsim {

// ------------------------------------------------------------ dense sweep

constexpr int kSweepThreads = 256;

template <typename T, int K>
struct DenseArgs {
    T re[1 << (2 * K)];
    T im[1 << (2 * K)];
    uint64_t cmask;           // control bits (all must be 1)
    uint64_t toff[1 << K];    // offset of local index j
    int npos;                 // targets + controls, ascending
    int pos[QSIM_MAX_K];
};

// One thread applies the gate to V consecutive groups (V = 2 moves two
// complex64 amplitudes per 16-byte access; needs the lowest inserted
// position >= 1 so that the two groups are adjacent in memory).
// NT: nontemporal accesses, used when the lowest inserted position is >= 4
// (the 2^k streams of a group then lie in different cache lines).
template <typename T, int K, int V, bool NT>
__global__ void __launch_bounds__(kSweepThreads)
k_dense_sweep(c2_t<T> *__restrict__ psi, const DenseArgs<T, K> a, uint64_t nthreads) {
    const uint64_t tid = uint64_t(blockIdx.x) * kSweepThreads + threadIdx.x;
    if (tid >= nthreads) return;
    constexpr int D = 1 << K;
    const uint64_t x = insert_zeros(tid * V, a.pos, a.npos) | a.cmask;
    T vr[D][V], vi[D][V];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if constexpr (V == 2) {
            const f32x4 w = ld<NT, f32x4>(psi + x + a.toff[j]);
            vr[j][0] = w.x; vi[j][0] = w.y; vr[j][1] = w.z; vi[j][1] = w.w;
        } else if constexpr (sizeof(T) == 8) {
            const f64x2 w = ld<NT, f64x2>(psi + x + a.toff[j]);
            vr[j][0] = w.x; vi[j][0] = w.y;
        } else {
            const f32x2 w = ld<NT, f32x2>(psi + x + a.toff[j]);
            vr[j][0] = w.x; vi[j][0] = w.y;
        }
    }
#pragma unroll
    for (int r = 0; r < D; ++r) {
        T orr[V], oi[V];
#pragma unroll
        for (int v = 0; v < V; ++v) { orr[v] = T(0); oi[v] = T(0); }
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const T ur = a.re[r * D + c], ui = a.im[r * D + c];
#pragma unroll
            for (int v = 0; v < V; ++v) cfma(orr[v], oi[v], ur, ui, vr[c][v], vi[c][v]);
        }
        if constexpr (V == 2) {
            st<NT, f32x4>(psi + x + a.toff[r], f32x4{orr[0], oi[0], orr[1], oi[1]});
        } else if constexpr (sizeof(T) == 8) {
            st<NT, f64x2>(psi + x + a.toff[r], f64x2{orr[0], oi[0]});
        } else {
            st<NT, f32x2>(psi + x + a.toff[r], f32x2{orr[0], oi[0]});
        }
    }
}

// Dense K-qubit gate (K = 1..3, complex64, no controls) as a lane-exchange
// sweep.  Each lane holds two adjacent amplitudes (one 16-byte access);
// lane bit b stands for amplitude bit lmap[b] and the wave index fills the
// other bits.  Targets are amplitude bit 0 (Z0: both of a lane's amplitudes
// are then in one group) or lane bits: targets below qubit 7 keep their
// natural lane bit, higher ones take the top free lane bits, and the other
// lane bits take the lowest free amplitude bits, so an access instruction
// covers runs of at least 128 contiguous bytes (1 KiB when every target is
// below qubit 7).  A lane takes the rest of its group from the lanes that
// differ in the target lane bits (l ^ dl[e]) and forms
// out(j) = sum over d of M[j][j ^ d] amp(j ^ d), the coefficients read by
// local index from a table in LDS; it writes back its own two amplitudes.
struct LaneArgs {
    float re[64], im[64];   // M, row-major, on the targets in ascending order
    uint32_t dl[8];         // lane offset of partner e: e's bits on the target lane bits
    int32_t lbit[3];        // lane bits of the targets other than qubit 0, in target order
    int32_t lmap[6];        // amplitude bit of each lane bit
    int32_t ins[7];         // amplitude bit 0 and the lane bits' bits, ascending
};

template <int K, bool Z0>
__global__ void __launch_bounds__(kSweepThreads)
k_lane_sweep(float2 *__restrict__ psi, const LaneArgs a, uint64_t nthreads) {
    constexpr int KL = Z0 ? K - 1 : K;
    constexpr int D = 1 << K;
    __shared__ float2 coef[D * D];      // coef[j D + d] = M[j][j ^ d]
    __shared__ uint64_t lane_off[64];   // amplitude offset of each lane
    if (threadIdx.x < D * D) {
        const int j = int(threadIdx.x) / D, d = int(threadIdx.x) % D;
        coef[threadIdx.x] = float2{a.re[j * D + (j ^ d)], a.im[j * D + (j ^ d)]};
    }
    if (threadIdx.x < 64) {
        uint64_t o = 0;
        for (int b = 0; b < 6; ++b) o |= uint64_t((threadIdx.x >> b) & 1u) << a.lmap[b];
        lane_off[threadIdx.x] = o;
    }
    __syncthreads();
    const uint64_t tid = uint64_t(blockIdx.x) * kSweepThreads + threadIdx.x;
    if (tid >= nthreads) return;
    const uint32_t lane = threadIdx.x & 63u;
    // the wave's first amplitude: its index spread over the bits no lane
    // stands for (uniform across the wave, in scalar registers)
    const uint64_t wave = uint64_t(blockIdx.x) * (kSweepThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t x = insert_zeros(wave, a.ins, 7) | lane_off[lane];
    const f32x4 w = ld<true, f32x4>(psi + x);
    float P[1 << KL][4];
    P[0][0] = w.x; P[0][1] = w.y; P[0][2] = w.z; P[0][3] = w.w;
#pragma unroll
    for (int e = 1; e < (1 << KL); ++e) {
        const int d = int(a.dl[e]);
        P[e][0] = __shfl_xor(w.x, d, 64);
        P[e][1] = __shfl_xor(w.y, d, 64);
        P[e][2] = __shfl_xor(w.z, d, 64);
        P[e][3] = __shfl_xor(w.w, d, 64);
    }
    uint32_t jl = 0;
#pragma unroll
    for (int b = 0; b < KL; ++b) jl |= ((lane >> a.lbit[b]) & 1u) << b;
    float out[4];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const uint32_t jA = Z0 ? (uint32_t(s) | (jl << 1)) : jl;
        float ar = 0.0f, ai = 0.0f;
#pragma unroll
        for (int dd = 0; dd < D; ++dd) {
            const int e = Z0 ? (dd >> 1) : dd;
            const int sub = Z0 ? (s ^ (dd & 1)) : s;
            const float2 c = coef[jA * D + dd];
            const float xr = P[e][2 * sub], xi = P[e][2 * sub + 1];
            ar = fma(c.x, xr, fma(-c.y, xi, ar));
            ai = fma(c.x, xi, fma(c.y, xr, ai));
        }
        out[2 * s] = ar;
        out[2 * s + 1] = ai;
    }
    st<true, f32x4>(psi + x, f32x4{out[0], out[1], out[2], out[3]});
}

template <int K>
static hipError_t lane_sweep(qsim_state s, const Pass &p) {
    LaneArgs a{};
    constexpr int D = 1 << K;
    for (int i = 0; i < D * D; ++i) {
        a.re[i] = float(p.M[i].real());
        a.im[i] = float(p.M[i].imag());
    }
    // targets are ascending (sweep passes hold the sorted form)
    const bool z0 = p.targets[0] == 0;
    int lane_of[QSIM_MAX_K];
    uint32_t used_lane = 0;
    uint64_t used_amp = 1;   // bit 0: the two amplitudes of a lane
    for (int b = 0; b < K; ++b) used_amp |= 1ull << p.targets[b];
    for (int b = z0 ? 1 : 0; b < K; ++b)
        if (p.targets[b] <= 6) {
            lane_of[b] = p.targets[b] - 1;
            used_lane |= 1u << lane_of[b];
        }
    for (int b = K - 1; b >= (z0 ? 1 : 0); --b)
        if (p.targets[b] > 6) {
            int l = 5;
            while ((used_lane >> l) & 1u) --l;
            lane_of[b] = l;
            used_lane |= 1u << l;
        }
    int nl = 0;
    for (int b = z0 ? 1 : 0; b < K; ++b) {
        a.lbit[nl++] = lane_of[b];
        a.lmap[lane_of[b]] = p.targets[b];
    }
    int next = 1;
    for (int l = 0; l < 6; ++l) {
        if ((used_lane >> l) & 1u) continue;
        while ((used_amp >> next) & 1ull) ++next;
        a.lmap[l] = next;
        used_amp |= 1ull << next;
    }
    int pos[7];
    pos[0] = 0;
    for (int l = 0; l < 6; ++l) pos[l + 1] = a.lmap[l];
    std::sort(pos, pos + 7);
    for (int i = 0; i < 7; ++i) a.ins[i] = pos[i];
    for (int e = 0; e < (1 << nl); ++e) {
        uint32_t d = 0;
        for (int b = 0; b < nl; ++b)
            if ((e >> b) & 1) d |= 1u << a.lbit[b];
        a.dl[e] = d;
    }
    auto *psi = static_cast<float2 *>(s->data);
    const uint64_t nthr = 1ull << (s->n - 1);   // a multiple of 64 (n >= 7): whole waves leave together
    const dim3 grid(unsigned((nthr + kSweepThreads - 1) / kSweepThreads));
    if (z0)
        hipLaunchKernelGGL((k_lane_sweep<K, true>), grid, dim3(kSweepThreads), 0, s->stream, psi, a, nthr);
    else
        hipLaunchKernelGGL((k_lane_sweep<K, false>), grid, dim3(kSweepThreads), 0, s->stream, psi, a, nthr);
    return hipGetLastError();
}

template <typename T, int K>
static hipError_t dense_sweep_t(qsim_state s, const Pass &p) {
    DenseArgs<T, K> a{};
    constexpr int D = 1 << K;
    for (int i = 0; i < D * D; ++i) {
        a.re[i] = T(p.M[i].real());
        a.im[i] = T(p.M[i].imag());
    }
    int all[QSIM_MAX_K];
    int np = 0;
    a.cmask = 0;
    for (int b = 0; b < p.k; ++b) all[np++] = p.targets[b];
    for (int c = 0; c < p.nctrl; ++c) {
        all[np++] = p.ctrls[c];
        a.cmask |= 1ull << p.ctrls[c];
    }
    std::sort(all, all + np);
    a.npos = np;
    for (int i = 0; i < np; ++i) a.pos[i] = all[i];
    for (int j = 0; j < D; ++j) {
        uint64_t o = 0;
        for (int b = 0; b < K; ++b)
            if ((j >> b) & 1) o |= 1ull << p.targets[b];
        a.toff[j] = o;
    }
    const uint64_t groups = 1ull << (s->n - np);
    auto *psi = static_cast<c2_t<T> *>(s->data);
    const bool nt = all[0] >= 4;
    if constexpr (std::is_same<T, float>::value) {
        // low targets: whole-wave contiguous accesses and lane exchanges
        if (lane_sweep_ok(s->dtype, s->n, p)) return lane_sweep<K>(s, p);
    }
    if constexpr (std::is_same<T, float>::value) {
        if (all[0] >= 1 && groups >= 2) {
            const uint64_t nthr = groups / 2;
            const dim3 grid(unsigned((nthr + kSweepThreads - 1) / kSweepThreads));
            if (nt)
                hipLaunchKernelGGL((k_dense_sweep<T, K, 2, true>), grid, dim3(kSweepThreads), 0, s->stream, psi, a,
                                   nthr);
            else
                hipLaunchKernelGGL((k_dense_sweep<T, K, 2, false>), grid, dim3(kSweepThreads), 0, s->stream, psi, a,
                                   nthr);
            return hipGetLastError();
        }
    }
    {
        const dim3 grid(unsigned((groups + kSweepThreads - 1) / kSweepThreads));
        if (nt)
            hipLaunchKernelGGL((k_dense_sweep<T, K, 1, true>), grid, dim3(kSweepThreads), 0, s->stream, psi, a, groups);
        else
            hipLaunchKernelGGL((k_dense_sweep<T, K, 1, false>), grid, dim3(kSweepThreads), 0, s->stream, psi, a,
                               groups);
    }
    return hipGetLastError();
}

hipError_t launch_dense_sweep(qsim_state s, const Pass &p) {
    const bool f = s->dtype == QSIM_C64;
    switch (p.k) {
        case 1: return f ? dense_sweep_t<float, 1>(s, p) : dense_sweep_t<double, 1>(s, p);
        case 2: return f ? dense_sweep_t<float, 2>(s, p) : dense_sweep_t<double, 2>(s, p);
        case 3: return f ? dense_sweep_t<float, 3>(s, p) : dense_sweep_t<double, 3>(s, p);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------ diagonal sweep

template <typename T>
struct DiagArgs {
    T dre[64];
    T dim[64];
    uint64_t joff[64];
    int nj;                   // non-unit diagonal entries
    int npos;
    int pos[QSIM_MAX_K];
};

template <typename T, int V>
__global__ void __launch_bounds__(kSweepThreads)
k_diag_sweep(c2_t<T> *__restrict__ psi, const DiagArgs<T> a, uint64_t nthreads) {
    const uint64_t tid = uint64_t(blockIdx.x) * kSweepThreads + threadIdx.x;
    if (tid >= nthreads) return;
    const uint64_t x = insert_zeros(tid * V, a.pos, a.npos);
    for (int i = 0; i < a.nj; ++i) {
        const T dr = a.dre[i], di = a.dim[i];
        c2_t<T> *p = psi + x + a.joff[i];
        if constexpr (V == 2) {
            float4 w = *reinterpret_cast<const float4 *>(p);
            float4 o;
            o.x = dr * w.x - di * w.y; o.y = dr * w.y + di * w.x;
            o.z = dr * w.z - di * w.w; o.w = dr * w.w + di * w.z;
            *reinterpret_cast<float4 *>(p) = o;
        } else {
            const c2_t<T> w = *p;
            c2_t<T> o;
            o.x = dr * w.x - di * w.y;
            o.y = dr * w.y + di * w.x;
            *p = o;
        }
    }
}

template <typename T>
static hipError_t diag_sweep_t(qsim_state s, const Pass &p) {
    DiagArgs<T> a{};
    const int D = 1 << p.k;
    a.nj = 0;
    for (int j = 0; j < D; ++j) {
        if (p.M[j] == cd(1.0)) continue;
        uint64_t o = 0;
        for (int b = 0; b < p.k; ++b)
            if ((j >> b) & 1) o |= 1ull << p.targets[b];
        a.dre[a.nj] = T(p.M[j].real());
        a.dim[a.nj] = T(p.M[j].imag());
        a.joff[a.nj] = o;
        ++a.nj;
    }
    if (a.nj == 0) return hipSuccess;
    a.npos = p.k;
    for (int b = 0; b < p.k; ++b) a.pos[b] = p.targets[b];
    const uint64_t groups = 1ull << (s->n - p.k);
    auto *psi = static_cast<c2_t<T> *>(s->data);
    if (std::is_same<T, float>::value && p.targets[0] >= 1 && groups >= 2) {
        const uint64_t nt = groups / 2;
        hipLaunchKernelGGL((k_diag_sweep<T, 2>), dim3(unsigned((nt + kSweepThreads - 1) / kSweepThreads)),
                           dim3(kSweepThreads), 0, s->stream, psi, a, nt);
    } else {
        hipLaunchKernelGGL((k_diag_sweep<T, 1>), dim3(unsigned((groups + kSweepThreads - 1) / kSweepThreads)),
                           dim3(kSweepThreads), 0, s->stream, psi, a, groups);
    }
    return hipGetLastError();
}

hipError_t launch_diag_sweep(qsim_state s, const Pass &p) {
    return s->dtype == QSIM_C64 ? diag_sweep_t<float>(s, p) : diag_sweep_t<double>(s, p);
}

// ------------------------------------------------------------ LDS tile pass

// LDS layout: [tile: 2^m amplitudes][ops][pool].
template <typename T, int KMAX>
__global__ void __launch_bounds__(kTileThreads) k_tile_pass(const TileArgs<T> a) {
    extern __shared__ char lds_raw[];
    c2_t<T> *lds = reinterpret_cast<c2_t<T> *>(lds_raw);
    const uint32_t M = 1u << a.m;
    TileOp *sops = reinterpret_cast<TileOp *>(lds + M);
    c2_t<T> *spool = reinterpret_cast<c2_t<T> *>(sops + a.nops);
    // stage the op list and the matrices in LDS
    {
        const int *src = reinterpret_cast<const int *>(a.ops);
        int *dst = reinterpret_cast<int *>(sops);
        const int nwords = a.nops * int(sizeof(TileOp) / sizeof(int));
        for (int w = threadIdx.x; w < nwords; w += kTileThreads) dst[w] = src[w];
        for (int e = threadIdx.x; e < a.npool; e += kTileThreads) spool[e] = a.pool[e];
    }
    // tile base: the block index with zeros inserted at every tile position
    uint64_t base = uint64_t(blockIdx.x) << a.L;
    for (int i = 0; i < a.H; ++i) {
        const uint64_t lo = base & ((1ull << a.hpos[i]) - 1ull);
        base = ((base - lo) << 1) | lo;
    }
    for (uint32_t l = threadIdx.x; l < M; l += kTileThreads) lds[l] = a.psi[base | tile_scatter(a, l)];
    __syncthreads();
    for (int o = 0; o < a.nops; ++o) {
        const TileOp &op = sops[o];
        const c2_t<T> *U = spool + op.moff;
        if (op.type == 1) {
            tile_diag<T>(lds, op, U, base, M);
        } else if (op.type == 4) {
            // rotation by a parameter held on the device: (cos, sin) of its half angle
            const double cs = a.trig[2 * op.moff];
            const double sn = op.jbit[0] ? -a.trig[2 * op.moff + 1] : a.trig[2 * op.moff + 1];
            tile_rotation<T>(lds, op.pos[0], op.kin, cs, sn, M);
        } else if (op.type == 5) {
            tile_controlled<T>(lds, op, U, M);
        } else {
            switch (op.k) {
                case 1: tile_dense_small<T, 1>(lds, op, U, M); break;
                case 2: tile_dense_small<T, 2>(lds, op, U, M); break;
                case 3: tile_dense_small<T, 3>(lds, op, U, M); break;
                default:
                    if constexpr (KMAX > 3) {
                        switch (op.k) {
                            case 4: tile_dense_wide<T, 4>(lds, op, U, M); break;
                            case 5: tile_dense_wide<T, 5>(lds, op, U, M); break;
                            case 6: tile_dense_wide<T, 6>(lds, op, U, M); break;
                            default: break;
                        }
                    }
                    break;
            }
        }
        __syncthreads();
    }
    for (uint32_t l = threadIdx.x; l < M; l += kTileThreads) a.psi[base | tile_scatter(a, l)] = lds[l];
}

template <typename T>
static hipError_t tile_pass_t(qsim_state s, const Plan &plan, const Pass &p, const double *trig) {
    TileArgs<T> a{};
    a.psi = static_cast<c2_t<T> *>(s->data);
    a.trig = trig;
    a.ops = reinterpret_cast<const TileOp *>(plan.dev) + p.op_begin;
    a.pool = reinterpret_cast<const c2_t<T> *>(static_cast<const char *>(plan.dev) + plan.pool_dev_off) +
             p.pool_begin;
    a.nops = p.op_end - p.op_begin;
    a.npool = p.pool_end - p.pool_begin;
    a.m = p.m;
    a.L = p.L;
    a.H = int(p.hpos.size());
    if (a.H > kMaxTileHigh || a.L + a.H != a.m) return hipErrorInvalidValue;
    for (int i = 0; i < a.H; ++i) a.hpos[i] = p.hpos[i];
    const uint64_t ntiles = 1ull << (s->n - p.m);
    const size_t lds = (sizeof(c2_t<T>) << p.m) + sizeof(TileOp) * size_t(a.nops) + sizeof(c2_t<T>) * size_t(a.npool);
    int kmax = 1;
    for (int o = p.op_begin; o < p.op_end; ++o)
        if (plan.tile_ops[size_t(o)].type == 0) kmax = std::max(kmax, int(plan.tile_ops[size_t(o)].k));
    const void *fn = kmax <= 3 ? reinterpret_cast<const void *>(&k_tile_pass<T, 3>)
                               : reinterpret_cast<const void *>(&k_tile_pass<T, 6>);
    if (lds > 65536) {
        // beyond the default limit: raise it (gfx950 has 160 KiB of LDS per CU)
        if (lds > 160 * 1024) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    if (kmax <= 3)
        hipLaunchKernelGGL((k_tile_pass<T, 3>), dim3(unsigned(ntiles)), dim3(kTileThreads), lds, s->stream, a);
    else
        hipLaunchKernelGGL((k_tile_pass<T, 6>), dim3(unsigned(ntiles)), dim3(kTileThreads), lds, s->stream, a);
    return hipGetLastError();
}

hipError_t launch_tile_pass(qsim_state s, const Plan &plan, const Pass &p, const double *trig) {
    return s->dtype == QSIM_C64 ? tile_pass_t<float>(s, plan, p, trig) : tile_pass_t<double>(s, plan, p, trig);
}

// ------------------------------------------------------------ basis state

template <typename T>
__global__ void __launch_bounds__(256) k_set_basis(c2_t<T> *psi, uint64_t N, uint64_t index) {
    for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < N; i += uint64_t(gridDim.x) * 256) {
        c2_t<T> w;
        w.x = (i == index) ? T(1) : T(0);
        w.y = T(0);
        psi[i] = w;
    }
}

hipError_t launch_set_basis(qsim_state s, uint64_t index) {
    const uint64_t N = 1ull << s->n;
    const unsigned grid = unsigned(std::min<uint64_t>((N + 255) / 256, 65536));
    if (s->dtype == QSIM_C64)
        hipLaunchKernelGGL((k_set_basis<float>), dim3(grid), dim3(256), 0, s->stream,
                           static_cast<float2 *>(s->data), N, index);
    else
        hipLaunchKernelGGL((k_set_basis<double>), dim3(grid), dim3(256), 0, s->stream,
                           static_cast<double2 *>(s->data), N, index);
    return hipGetLastError();
}

// ------------------------------------------------------------ fill

__global__ void __launch_bounds__(256) k_fill_zero(uint32_t *dst, uint64_t words) {
    for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < words; i += uint64_t(gridDim.x) * 256) dst[i] = 0u;
}

// Zeroes `bytes` (a multiple of 4) at dst, stream-ordered.  A kernel rather
// than a memset node, so that a caller may capture it in a graph.
hipError_t launch_fill_zero(qsim_state s, void *dst, size_t bytes) {
    const uint64_t words = bytes / 4;
    const unsigned grid = unsigned(std::max<uint64_t>(1, std::min<uint64_t>((words + 255) / 256, 4096)));
    hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, s->stream, static_cast<uint32_t *>(dst), words);
    return hipGetLastError();
}

// ------------------------------------------------------------ expectation

// Device form of one Pauli term inside a group sharing the X mask:
// weight w = coeff * i^{|x & z|} (complex), sign mask z.
struct ExpTerm {
    double wr, wi;
    uint64_t z;
    uint64_t pad_;
};

constexpr int kExpThreads = 256;

// Sum over y of Re[w_t (-1)^{|(y^x) & z_t|} conj(psi_y) psi_{y^x}] for every
// term of the group, accumulated in double.
template <typename T>
__global__ void __launch_bounds__(kExpThreads)
k_expect(const c2_t<T> *__restrict__ psi, uint64_t N, uint64_t x, const ExpTerm *__restrict__ terms, int nterms,
         double *__restrict__ partials) {
    double acc = 0.0;
    for (uint64_t y = uint64_t(blockIdx.x) * kExpThreads + threadIdx.x; y < N;
         y += uint64_t(gridDim.x) * kExpThreads) {
        const c2_t<T> a = psi[y];
        const c2_t<T> b = x ? psi[y ^ x] : a;
        // conj(a) * b
        const double pr = double(a.x) * double(b.x) + double(a.y) * double(b.y);
        const double pi = double(a.x) * double(b.y) - double(a.y) * double(b.x);
        const uint64_t src = y ^ x;
        double s = 0.0;
        for (int t = 0; t < nterms; ++t) {
            const ExpTerm e = terms[t];
            const double v = e.wr * pr - e.wi * pi;
            s += (__popcll(src & e.z) & 1) ? -v : v;
        }
        acc += s;
    }
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

int expect_group_grid(uint64_t N) {
    const uint64_t want = (N + kExpThreads * 8 - 1) / (kExpThreads * 8);
    return int(std::max<uint64_t>(1, std::min<uint64_t>(want, 2048)));
}

hipError_t launch_expect_group(qsim_state s, uint64_t xmask, const void *dev_terms, int nterms,
                               double *partials, int *nwritten) {
    const uint64_t N = 1ull << s->n;
    const int grid = expect_group_grid(N);
    const ExpTerm *terms = static_cast<const ExpTerm *>(dev_terms);
    if (s->dtype == QSIM_C64)
        hipLaunchKernelGGL((k_expect<float>), dim3(grid), dim3(kExpThreads), 0, s->stream,
                           static_cast<const float2 *>(s->data), N, xmask, terms, nterms, partials);
    else
        hipLaunchKernelGGL((k_expect<double>), dim3(grid), dim3(kExpThreads), 0, s->stream,
                           static_cast<const double2 *>(s->data), N, xmask, terms, nterms, partials);
    *nwritten = grid;
    return hipGetLastError();
}

// Tiled groups: each workgroup takes tiles blockIdx.x, + gridDim.x, ...; per
// tile it loads the 2^m amplitudes into LDS (consecutive lanes on the low
// qubits), then for every group sums Re[w (-1)^{|(y^x) & z|} conj(psi_y)
// psi_{y^x}] over the tile: the parity splits into the tile's fixed
// out-of-tile bits (uniform: scalar unit) and the local bits.  Wave sums
// accumulate per group in LDS in tile order; the workgroup writes one
// partial per group.
template <typename T>
__global__ void __launch_bounds__(kExpThreads)
k_expect_tile(const c2_t<T> *__restrict__ psi, const ExpTilePass p, const ExpTerm *__restrict__ terms,
              uint64_t ntiles, double *__restrict__ partials) {
    extern __shared__ char lds_raw[];
    c2_t<T> *lds = reinterpret_cast<c2_t<T> *>(lds_raw);
    __shared__ double wsum[kExpTileGroups][kExpThreads / 64];
    const uint32_t M = 1u << p.m;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int g = threadIdx.x; g < kExpTileGroups * (kExpThreads / 64); g += kExpThreads)
        wsum[g / (kExpThreads / 64)][g % (kExpThreads / 64)] = 0.0;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        uint64_t base = t << p.L;
        for (int i = 0; i < p.H; ++i) {
            const uint64_t lo = base & ((1ull << p.hpos[i]) - 1ull);
            base = ((base - lo) << 1) | lo;
        }
        __syncthreads();   // the previous tile's readers are done
        for (uint32_t l = threadIdx.x; l < M; l += kExpThreads) {
            uint64_t gi = base | (l & ((1u << p.L) - 1u));
            const uint32_t h = l >> p.L;
            for (int i = 0; i < p.H; ++i) gi |= uint64_t((h >> i) & 1u) << p.hpos[i];
            lds[l] = psi[gi];
        }
        __syncthreads();
        for (int g = 0; g < p.ngroups; ++g) {
            const ExpTileGroup gr = p.groups[g];
            double acc = 0.0;
            for (uint32_t l = threadIdx.x; l < M; l += kExpThreads) {
                const c2_t<T> a = lds[l], b = lds[l ^ gr.xl];
                const double pr = double(a.x) * double(b.x) + double(a.y) * double(b.y);
                const double pi = double(a.x) * double(b.y) - double(a.y) * double(b.x);
                double sm = 0.0;
                for (int tt = gr.first; tt < gr.first + gr.count; ++tt) {
                    const ExpTerm e = terms[tt];
                    const uint32_t zo = uint32_t(__popcll(base & e.z));
                    const double v = e.wr * pr - e.wi * pi;
                    sm += ((uint32_t(__popc((l ^ gr.xl) & uint32_t(e.pad_))) ^ zo) & 1u) ? -v : v;
                }
                acc += sm;
            }
            for (int sft = 32; sft > 0; sft >>= 1) acc += __shfl_xor(acc, sft, 64);
            if (lane == 0) wsum[g][wave] += acc;
        }
    }
    __syncthreads();
    if (threadIdx.x < p.ngroups) {
        double tot = 0.0;
        for (int w = 0; w < kExpThreads / 64; ++w) tot += wsum[threadIdx.x][w];
        partials[size_t(threadIdx.x) * gridDim.x + blockIdx.x] = tot;
    }
}

// The same sums for tiles of exactly KPT * 256 amplitudes, with each
// thread's amplitudes in registers and the terms as the outer loop.
// Amplitude l = t + 256 k of the tile is thread t's k-th, so the local bits
// 0..7 of l are the thread's and bits 8.. the register index k.
//  * X mask 0: for amplitude y = (thread part) + (register part k),
//    (-1)^{|y & z|} = (-1)^{|y_t & z|} (-1)^{|k & mu(z)|} with mu(z) the
//    register part of z.  The thread sums C_mu = sum of w (-1)^{|y_t & z|}
//    over the terms with register part mu (terms arrive ordered by mu), and
//    the weights of all its amplitudes, D_k = sum_mu C_mu (-1)^{|k & mu|},
//    follow by a Walsh-Hadamard transform over the register bits; then
//    D_k |psi_k|^2 is added.  Cost per amplitude: about one term-sign per
//    KPT amplitudes per term, instead of one per amplitude per term.
//  * simple groups (X_h / Y_h terms only): the pair (y, y ^ x) is visited
//    once, from the member with y_h = 0, and adds 2 (A Re + B Im) of
//    conj(psi_y) psi_{y^x}; when h is a register bit both members are in
//    the thread's registers.
//  * other X masks: the pair is visited once and counted twice: for a
//    Hermitian term the two members' summands are complex conjugates, so
//    their sum is twice the real part of either.
template <typename T, int KPT, int KX>
__device__ __forceinline__ void pairs_in_registers(const c2_t<T> (&a)[KPT], double A, double B, bool use_b,
                                                   double &acc) {
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int k = 0; k < KPT; ++k) {
        if (k & KX) continue;
        const double ar = double(a[k].x), ai = double(a[k].y);
        const double br = double(a[k ^ KX].x), bi = double(a[k ^ KX].y);
        sr += ar * br + ai * bi;
        if (use_b) si += ar * bi - ai * br;
    }
    acc += 2.0 * (A * sr + B * si);
}

template <typename T, int KPT>
__global__ void __launch_bounds__(kExpThreads)
k_expect_tile_reg(const c2_t<T> *__restrict__ psi, const ExpTilePass p, const ExpTerm *__restrict__ terms,
                  uint64_t ntiles, double *__restrict__ partials) {
    static_assert(KPT == 8 || KPT == 16, "register tiles of 8 or 16 amplitudes per thread");
    extern __shared__ char lds_raw[];
    c2_t<T> *lds = reinterpret_cast<c2_t<T> *>(lds_raw);
    __shared__ double wsum[kExpTileGroups][kExpThreads / 64];
    const uint32_t t = threadIdx.x;
    const int wave = t / 64, lane = t % 64;
    for (int g = t; g < kExpTileGroups * (kExpThreads / 64); g += kExpThreads)
        wsum[g / (kExpThreads / 64)][g % (kExpThreads / 64)] = 0.0;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        uint64_t base = tile << p.L;
        for (int i = 0; i < p.H; ++i) {
            const uint64_t lo = base & ((1ull << p.hpos[i]) - 1ull);
            base = ((base - lo) << 1) | lo;
        }
        __syncthreads();   // the previous tile's readers are done
#pragma unroll
        for (int k = 0; k < KPT; ++k) {
            const uint32_t l = t + uint32_t(k) * kExpThreads;
            uint64_t gi = base | (l & ((1u << p.L) - 1u));
            const uint32_t h = l >> p.L;
            for (int i = 0; i < p.H; ++i) gi |= uint64_t((h >> i) & 1u) << p.hpos[i];
            lds[l] = psi[gi];
        }
        __syncthreads();
        c2_t<T> a[KPT];
#pragma unroll
        for (int k = 0; k < KPT; ++k) a[k] = lds[t + uint32_t(k) * kExpThreads];
        for (int g = 0; g < p.ngroups; ++g) {
            const ExpTileGroup gr = p.groups[g];
            double acc = 0.0;
            if (gr.xl == 0) {
                double C[KPT];
#pragma unroll
                for (int k = 0; k < KPT; ++k) C[k] = 0.0;
#pragma unroll
                for (int mu = 0; mu < KPT; ++mu) {
                    for (int tt = p.dmu[mu]; tt < p.dmu[mu + 1]; ++tt) {
                        const ExpTerm e = terms[tt];
                        const uint32_t par =
                            (uint32_t(__popcll(base & e.z)) ^ uint32_t(__popc(t & uint32_t(e.pad_) & 0xffu))) & 1u;
                        C[mu] += par ? -e.wr : e.wr;
                    }
                }
#pragma unroll
                for (int bit = 1; bit < KPT; bit <<= 1) {
#pragma unroll
                    for (int k = 0; k < KPT; ++k) {
                        if (k & bit) continue;
                        const double u = C[k], v = C[k | bit];
                        C[k] = u + v;
                        C[k | bit] = u - v;
                    }
                }
#pragma unroll
                for (int k = 0; k < KPT; ++k) {
                    const double ar = double(a[k].x), ai = double(a[k].y);
                    acc += C[k] * (ar * ar + ai * ai);
                }
            } else if ((gr.flags & kExpGroupSimple) && (gr.xl & 0xffu) == 0) {
                // one register bit: both members of every pair are in registers
                const bool use_b = gr.B != 0.0;
                switch (gr.xl >> 8) {
                case 1: pairs_in_registers<T, KPT, 1>(a, gr.A, gr.B, use_b, acc); break;
                case 2: pairs_in_registers<T, KPT, 2>(a, gr.A, gr.B, use_b, acc); break;
                case 4: pairs_in_registers<T, KPT, 4>(a, gr.A, gr.B, use_b, acc); break;
                default:
                    if constexpr (KPT == 16) pairs_in_registers<T, KPT, 8>(a, gr.A, gr.B, use_b, acc);
                    break;
                }
            } else if (gr.flags & kExpGroupSimple) {
                // one thread bit: the member with bit 0 reads its partner from LDS
                const uint32_t xb = gr.xl;
                if ((t & xb) == 0) {
                    const bool use_b = gr.B != 0.0;
                    double sr = 0.0, si = 0.0;
#pragma unroll
                    for (int k = 0; k < KPT; ++k) {
                        const c2_t<T> b = lds[(t ^ xb) + uint32_t(k) * kExpThreads];
                        const double ar = double(a[k].x), ai = double(a[k].y), br = double(b.x), bi = double(b.y);
                        sr += ar * br + ai * bi;
                        if (use_b) si += ar * bi - ai * br;
                    }
                    acc += 2.0 * (gr.A * sr + gr.B * si);
                }
            } else {
                const uint32_t lb = gr.xl & (0u - gr.xl);   // lowest bit of x
                double pr[KPT / 2], pi[KPT / 2];
                uint32_t ly[KPT / 2];   // y ^ x of each pair (its sign bits)
#pragma unroll
                for (int k = 0; k < KPT / 2; ++k) {
                    const uint32_t j = t + uint32_t(k) * kExpThreads;
                    const uint32_t l = ((j & ~(lb - 1u)) << 1) | (j & (lb - 1u));
                    const c2_t<T> av = lds[l], bv = lds[l ^ gr.xl];
                    pr[k] = double(av.x) * double(bv.x) + double(av.y) * double(bv.y);
                    pi[k] = double(av.x) * double(bv.y) - double(av.y) * double(bv.x);
                    ly[k] = l ^ gr.xl;
                }
                for (int tt = gr.first; tt < gr.first + gr.count; ++tt) {
                    const ExpTerm e = terms[tt];
                    const uint32_t zo = uint32_t(__popcll(base & e.z));
                    const uint32_t zl = uint32_t(e.pad_);
#pragma unroll
                    for (int k = 0; k < KPT / 2; ++k) {
                        const double v = e.wr * pr[k] - e.wi * pi[k];
                        acc += ((uint32_t(__popc(ly[k] & zl)) ^ zo) & 1u) ? -2.0 * v : 2.0 * v;
                    }
                }
            }
            for (int sft = 32; sft > 0; sft >>= 1) acc += __shfl_xor(acc, sft, 64);
            if (lane == 0) wsum[g][wave] += acc;
        }
    }
    __syncthreads();
    if (t < uint32_t(p.ngroups)) {
        double tot = 0.0;
        for (int w = 0; w < kExpThreads / 64; ++w) tot += wsum[t][w];
        partials[size_t(t) * gridDim.x + blockIdx.x] = tot;
    }
}

hipError_t launch_expect_tiles(qsim_state s, const ExpTilePass &p, const void *dev_terms, double *partials,
                               int *nwritten) {
    const uint64_t ntiles = 1ull << (s->n - p.m);
    const int grid = int(std::min<uint64_t>(ntiles, 2048));
    const ExpTerm *terms = static_cast<const ExpTerm *>(dev_terms);
    const size_t lds = (s->dtype == QSIM_C64 ? 8u : 16u) << p.m;
    if (s->dtype == QSIM_C64) {
        const c2_t<float> *psi = static_cast<const c2_t<float> *>(s->data);
        if (p.m == 12)
            hipLaunchKernelGGL((k_expect_tile_reg<float, 16>), dim3(grid), dim3(kExpThreads), lds, s->stream, psi,
                               p, terms, ntiles, partials);
        else
            hipLaunchKernelGGL((k_expect_tile<float>), dim3(grid), dim3(kExpThreads), lds, s->stream, psi, p, terms,
                               ntiles, partials);
    } else {
        const c2_t<double> *psi = static_cast<const c2_t<double> *>(s->data);
        if (p.m == 11)
            hipLaunchKernelGGL((k_expect_tile_reg<double, 8>), dim3(grid), dim3(kExpThreads), lds, s->stream, psi,
                               p, terms, ntiles, partials);
        else
            hipLaunchKernelGGL((k_expect_tile<double>), dim3(grid), dim3(kExpThreads), lds, s->stream, psi, p, terms,
                               ntiles, partials);
    }
    *nwritten = grid * p.ngroups;
    return hipGetLastError();
}

__global__ void __launch_bounds__(kExpThreads) k_reduce(const double *__restrict__ partials, int count, double *out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += kExpThreads) acc += partials[i];
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) out[0] = tot;
}

hipError_t launch_reduce(qsim_state s, const double *partials, int count, double *out) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kExpThreads), 0, s->stream, partials, count, out);
    return hipGetLastError();
}

int expect_partials_max() { return 2048; }

}  // namespace qsim
