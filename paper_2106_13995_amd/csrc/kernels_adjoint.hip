// Adjoint differentiation of an expectation value on gfx950.
//
// E(theta) = <psi_L|H|psi_L>, psi_L = U_L ... U_1 psi_0.  With
// lambda_l = U_{l+1}^dag ... U_L^dag H psi_L and psi_l = U_l ... U_1 psi_0, a
// rotation U_l = exp(-i theta G / 2) (G = X, Y or Z on one qubit) gives
// dE/dtheta = Im <lambda_l| G |psi_l>.  The reverse sweep applies U_l^dag to
// both psi and lambda, and takes each such inner product just before.
//
// Kernels: lambda = H psi with the energy's partial sums; LDS tile passes
// that carry both states and evaluate the inner products ("probes") per tile;
// a fixed-order row reduction of the per-tile partial sums.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "qsim_internal.h"
#include "tile_ops.h"

namespace qsim {

// ------------------------------------------------------------ lambda = H psi

// Term of a Pauli sum inside a group that shares one X mask:
// weight w = coeff * i^{|x & z|}, sign mask z.
struct HTerm {
    double wr, wi;
    uint64_t z;
    uint64_t pad_;
};

struct HGroup {
    uint64_t x;
    int32_t first, count;
};

// lambda_y = sum_t w_t (-1)^{|(y^x_t) & z_t|} psi_{y^x_t}; the block also
// accumulates Re(conj(psi_y) lambda_y) for the energy.
template <typename T>
__global__ void __launch_bounds__(kBlockThreads)
k_pauli_apply(const c2_t<T> *__restrict__ psi, c2_t<T> *__restrict__ lam, uint64_t N,
              const HGroup *__restrict__ groups, int ngroups, const HTerm *__restrict__ terms,
              double *__restrict__ partials) {
    double e = 0.0;
    for (uint64_t y = uint64_t(blockIdx.x) * kBlockThreads + threadIdx.x; y < N;
         y += uint64_t(gridDim.x) * kBlockThreads) {
        double ar = 0.0, ai = 0.0;
        for (int g = 0; g < ngroups; ++g) {
            const HGroup gr = groups[g];
            const uint64_t src = y ^ gr.x;
            const c2_t<T> b = psi[src];
            double sr = 0.0, si = 0.0;
            for (int t = gr.first; t < gr.first + gr.count; ++t) {
                const HTerm h = terms[t];
                const double sg = (__popcll(src & h.z) & 1) ? -1.0 : 1.0;
                sr += sg * h.wr;
                si += sg * h.wi;
            }
            ar += sr * double(b.x) - si * double(b.y);
            ai += sr * double(b.y) + si * double(b.x);
        }
        c2_t<T> o;
        o.x = T(ar);
        o.y = T(ai);
        lam[y] = o;
        const c2_t<T> p = psi[y];
        e += double(p.x) * ar + double(p.y) * ai;
    }
    const double tot = block_sum(e);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

int pauli_apply_grid(uint64_t N) {
    const uint64_t want = (N + kBlockThreads * 8 - 1) / (kBlockThreads * 8);
    return int(std::max<uint64_t>(1, std::min<uint64_t>(want, 2048)));
}

hipError_t launch_pauli_apply(qsim_state s, void *lam, const void *groups, int ngroups, const void *terms,
                              double *partials) {
    const uint64_t N = 1ull << s->n;
    const int grid = pauli_apply_grid(N);
    if (s->dtype == QSIM_C64)
        hipLaunchKernelGGL((k_pauli_apply<float>), dim3(grid), dim3(kBlockThreads), 0, s->stream,
                           static_cast<const float2 *>(s->data), static_cast<float2 *>(lam), N,
                           static_cast<const HGroup *>(groups), ngroups, static_cast<const HTerm *>(terms), partials);
    else
        hipLaunchKernelGGL((k_pauli_apply<double>), dim3(grid), dim3(kBlockThreads), 0, s->stream,
                           static_cast<const double2 *>(s->data), static_cast<double2 *>(lam), N,
                           static_cast<const HGroup *>(groups), ngroups, static_cast<const HTerm *>(terms), partials);
    return hipGetLastError();
}

// ------------------------------------------------------------ reverse tile passes

// Im <lambda|G|psi> over one tile for G = X (gen 1), Y (2) or Z (3) on
// tile-local position p, accumulated in double.
template <typename T>
__device__ __forceinline__ double tile_probe(const c2_t<T> *lp, const c2_t<T> *ll, int p, int gen, uint32_t M) {
    double acc = 0.0;
    const uint32_t bit = 1u << p;
    for (uint32_t l = threadIdx.x; l < M; l += kTileThreads) {
        const c2_t<T> lam = ll[l];
        const bool one = (l & bit) != 0;
        double gr, gi;   // (G psi)_l
        if (gen == 3) {
            const c2_t<T> v = lp[l];
            gr = one ? -double(v.x) : double(v.x);
            gi = one ? -double(v.y) : double(v.y);
        } else {
            const c2_t<T> v = lp[l ^ bit];
            if (gen == 1) {
                gr = double(v.x);
                gi = double(v.y);
            } else {   // Y: row 0 takes -i psi_1, row 1 takes +i psi_0
                gr = one ? -double(v.y) : double(v.y);
                gi = one ? double(v.x) : -double(v.x);
            }
        }
        // Im(conj(lam) * g)
        acc += double(lam.x) * gi - double(lam.y) * gr;
    }
    return acc;
}

template <typename T, int KMAX>
__global__ void __launch_bounds__(kTileThreads)
k_adjoint_tile(const TileArgs<T> a, c2_t<T> *__restrict__ lam, double *__restrict__ probe_partials,
               uint32_t ntiles) {
    extern __shared__ char lds_raw[];
    const uint32_t M = 1u << a.m;
    c2_t<T> *lp = reinterpret_cast<c2_t<T> *>(lds_raw);
    c2_t<T> *ll = lp + M;
    TileOp *sops = reinterpret_cast<TileOp *>(ll + M);
    c2_t<T> *spool = reinterpret_cast<c2_t<T> *>(sops + a.nops);
    {
        const int *src = reinterpret_cast<const int *>(a.ops);
        int *dst = reinterpret_cast<int *>(sops);
        const int nwords = a.nops * int(sizeof(TileOp) / sizeof(int));
        for (int w = threadIdx.x; w < nwords; w += kTileThreads) dst[w] = src[w];
        for (int e = threadIdx.x; e < a.npool; e += kTileThreads) spool[e] = a.pool[e];
    }
    uint64_t base = uint64_t(blockIdx.x) << a.L;
    for (int i = 0; i < a.H; ++i) {
        const uint64_t lo = base & ((1ull << a.hpos[i]) - 1ull);
        base = ((base - lo) << 1) | lo;
    }
    for (uint32_t l = threadIdx.x; l < M; l += kTileThreads) {
        const uint64_t g = base | tile_scatter(a, l);
        lp[l] = a.psi[g];
        ll[l] = lam[g];
    }
    __syncthreads();
    // probes: summed within each wave at the op, across the four waves (in
    // the fixed order of a block-wide sum) when the tile is done or the
    // slots are full, so a probe costs no barrier of its own
    constexpr int kSlots = 64;
    __shared__ double wpart[kSlots][kTileThreads / 64];
    __shared__ int wslot[kSlots];
    int np = 0;
    auto flush = [&]() {
        if (threadIdx.x < np) {
            double t = 0.0;
            for (int w = 0; w < kTileThreads / 64; ++w) t += wpart[threadIdx.x][w];
            probe_partials[size_t(wslot[threadIdx.x]) * ntiles + blockIdx.x] = t;
        }
    };
    for (int o = 0; o < a.nops; ++o) {
        const TileOp &op = sops[o];
        const c2_t<T> *U = spool + op.moff;
        if (op.type == 3) {
            double v = tile_probe<T>(lp, ll, op.pos[0], op.kin, M);
            for (int sft = 32; sft > 0; sft >>= 1) v += __shfl_xor(v, sft, 64);
            if (threadIdx.x % 64 == 0) wpart[np][threadIdx.x / 64] = v;
            if (threadIdx.x == 0) wslot[np] = op.moff;
            if (++np == kSlots) {
                __syncthreads();
                flush();
                np = 0;
            }
        } else if (op.type == 1) {
            tile_diag<T>(lp, op, U, base, M);
            tile_diag<T>(ll, op, U, base, M);
        } else if (op.type == 4) {
            const double cs = a.trig[2 * op.moff];
            const double sn = op.jbit[0] ? -a.trig[2 * op.moff + 1] : a.trig[2 * op.moff + 1];
            tile_rotation<T>(lp, op.pos[0], op.kin, cs, sn, M);
            tile_rotation<T>(ll, op.pos[0], op.kin, cs, sn, M);
        } else if (op.type == 5) {
            tile_controlled<T>(lp, op, U, M);
            tile_controlled<T>(ll, op, U, M);
        } else {
            switch (op.k) {
                case 1: tile_dense_small<T, 1>(lp, op, U, M); tile_dense_small<T, 1>(ll, op, U, M); break;
                case 2: tile_dense_small<T, 2>(lp, op, U, M); tile_dense_small<T, 2>(ll, op, U, M); break;
                case 3: tile_dense_small<T, 3>(lp, op, U, M); tile_dense_small<T, 3>(ll, op, U, M); break;
                default:
                    if constexpr (KMAX > 3) {
                        switch (op.k) {
                            case 4: tile_dense_wide<T, 4>(lp, op, U, M); __syncthreads(); tile_dense_wide<T, 4>(ll, op, U, M); break;
                            case 5: tile_dense_wide<T, 5>(lp, op, U, M); __syncthreads(); tile_dense_wide<T, 5>(ll, op, U, M); break;
                            case 6: tile_dense_wide<T, 6>(lp, op, U, M); __syncthreads(); tile_dense_wide<T, 6>(ll, op, U, M); break;
                            default: break;
                        }
                    }
                    break;
            }
        }
        __syncthreads();
    }
    flush();
    for (uint32_t l = threadIdx.x; l < M; l += kTileThreads) {
        const uint64_t g = base | tile_scatter(a, l);
        a.psi[g] = lp[l];
        lam[g] = ll[l];
    }
}

template <typename T>
static hipError_t adjoint_pass_t(qsim_state s, const Plan &plan, const Pass &p, void *lam, double *probe_partials,
                                 const double *trig) {
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
    const uint32_t ntiles = uint32_t(1ull << (s->n - p.m));
    const size_t lds = (2 * sizeof(c2_t<T>) << p.m) + sizeof(TileOp) * size_t(a.nops) +
                       sizeof(c2_t<T>) * size_t(a.npool);
    int kmax = 1;
    for (int o = p.op_begin; o < p.op_end; ++o)
        if (plan.tile_ops[size_t(o)].type == 0) kmax = std::max(kmax, int(plan.tile_ops[size_t(o)].k));
    const void *fn = kmax <= 3 ? reinterpret_cast<const void *>(&k_adjoint_tile<T, 3>)
                               : reinterpret_cast<const void *>(&k_adjoint_tile<T, 6>);
    if (lds > 65536) {
        if (lds > 160 * 1024) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    auto *l = static_cast<c2_t<T> *>(lam);
    if (kmax <= 3)
        hipLaunchKernelGGL((k_adjoint_tile<T, 3>), dim3(ntiles), dim3(kTileThreads), lds, s->stream, a, l,
                           probe_partials, ntiles);
    else
        hipLaunchKernelGGL((k_adjoint_tile<T, 6>), dim3(ntiles), dim3(kTileThreads), lds, s->stream, a, l,
                           probe_partials, ntiles);
    return hipGetLastError();
}

hipError_t launch_adjoint_pass(qsim_state s, const Plan &plan, const Pass &p, void *lam, double *probe_partials,
                               const double *trig) {
    return s->dtype == QSIM_C64 ? adjoint_pass_t<float>(s, plan, p, lam, probe_partials, trig)
                                : adjoint_pass_t<double>(s, plan, p, lam, probe_partials, trig);
}

// (cos, sin) of theta_j / 2 for every parameter, read from device memory.
__global__ void __launch_bounds__(kBlockThreads) k_half_angle_trig(const double *__restrict__ params, int64_t n,
                                                                   double *__restrict__ trig) {
    for (int64_t j = int64_t(blockIdx.x) * kBlockThreads + threadIdx.x; j < n; j += int64_t(gridDim.x) * kBlockThreads) {
        double sn, cs;
        sincos(0.5 * params[j], &sn, &cs);
        trig[2 * j] = cs;
        trig[2 * j + 1] = sn;
    }
}

hipError_t launch_half_angle_trig(qsim_state s, const double *params, int64_t n, double *trig) {
    if (n <= 0) return hipSuccess;
    const int grid = int(std::min<int64_t>((n + kBlockThreads - 1) / kBlockThreads, 1024));
    hipLaunchKernelGGL(k_half_angle_trig, dim3(grid), dim3(kBlockThreads), 0, s->stream, params, n, trig);
    return hipGetLastError();
}

// grad[j] = sum of probe sums sums[idx[k]] for k in [row[j], row[j + 1]) in
// that order (the ops that use parameter j, last op first); energy = sums[nprobes].
__global__ void __launch_bounds__(kBlockThreads)
k_gather_gradient(const double *__restrict__ sums, const int32_t *__restrict__ row, const int32_t *__restrict__ idx,
                  int64_t nparams, int nprobes, double *__restrict__ grad, double *__restrict__ energy) {
    for (int64_t j = int64_t(blockIdx.x) * kBlockThreads + threadIdx.x; j < nparams;
         j += int64_t(gridDim.x) * kBlockThreads) {
        double g = 0.0;
        for (int k = row[j]; k < row[j + 1]; ++k) g += sums[idx[k]];
        grad[j] = g;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) energy[0] = sums[nprobes];
}

hipError_t launch_gather_gradient(qsim_state s, const double *sums, const int32_t *row, const int32_t *idx,
                                  int64_t nparams, int nprobes, double *grad, double *energy) {
    const int grid = int(std::max<int64_t>(1, std::min<int64_t>((nparams + kBlockThreads - 1) / kBlockThreads, 1024)));
    hipLaunchKernelGGL(k_gather_gradient, dim3(grid), dim3(kBlockThreads), 0, s->stream, sums, row, idx, nparams,
                       nprobes, grad, energy);
    return hipGetLastError();
}

// out[r] = sum of row r (`cols` doubles), one block per row, fixed order.
__global__ void __launch_bounds__(kBlockThreads)
k_reduce_rows(const double *__restrict__ in, int cols, double *__restrict__ out) {
    const double *row = in + size_t(blockIdx.x) * cols;
    double acc = 0.0;
    for (int i = threadIdx.x; i < cols; i += kBlockThreads) acc += row[i];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

hipError_t launch_reduce_rows(qsim_state s, const double *in, int rows, int cols, double *out) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_rows, dim3(rows), dim3(kBlockThreads), 0, s->stream, in, cols, out);
    return hipGetLastError();
}

}  // namespace qsim
