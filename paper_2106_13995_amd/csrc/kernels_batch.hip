// Batched forward + adjoint runs of many independent circuits in one
// persistent launch (gfx950).
//
// Each workgroup repeatedly takes the next circuit from an atomic counter
// (circuits are queued largest first) and runs it alone: the forward tile
// passes on psi, lambda = H psi with the energy, then the reverse tile passes
// on (psi, lambda) with the per-parameter probes Im <lambda|G|psi>.  A
// circuit whose state fits one tile keeps psi and lambda in LDS for the
// whole run; larger ones keep them in a per-workgroup slot of device memory
// and stream tiles through LDS.  Circuits of the same structure share one
// program; rotation matrices are formed on the device from each circuit's
// own parameters.  Every workgroup leaves the loop once the counter passes
// the number of circuits, so the grid always drains.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "device_common.h"
#include "qsim_internal.h"
#include "tile_ops.h"

namespace qsim {

template <typename T>
struct BatchArgs {
    const BatchCircuit *circs;
    const int32_t *order;
    const BatchProgram *progs;
    const BatchPass *passes;
    const TileOp *ops;
    const c2_t<T> *pool;
    const BatchHGroup *hgroups;
    const BatchHTerm *hterms;
    const double *params;
    double *energies;
    double *grads;
    c2_t<T> *arena;
    uint64_t slot_amps;     // amplitudes per state in a workgroup's slot
    int *counter;
    int ncirc;
    int want_grad;
    int mmax;
};

// Per-circuit tables in LDS: cos and sin of half of each rotation angle
// (formed once per circuit instead of once per op and tile), and the
// per-wave partial sums of a tile's probes, added to the gradient in a fixed
// order when the tile is done.
constexpr int kBatchTrig = 512;
constexpr int kLoadBatch = 8;   // tile loads a thread keeps in flight
constexpr int kProbeSlots = 64;
struct BatchShared {
    double cs[kBatchTrig], sn[kBatchTrig];
    double probe[kProbeSlots][kTileThreads / 64];
    int probe_param[kProbeSlots];
};


template <typename T>
__device__ __forceinline__ double batch_probe(const c2_t<T> *lp, const c2_t<T> *ll, int p, int gen, uint32_t M) {
    double acc = 0.0;
    const uint32_t bit = 1u << p;
    for (uint32_t l = threadIdx.x; l < M; l += kTileThreads) {
        const c2_t<T> lam = ll[l];
        const bool one = (l & bit) != 0;
        double gr, gi;
        if (gen == 3) {
            const c2_t<T> v = lp[l];
            gr = one ? -double(v.x) : double(v.x);
            gi = one ? -double(v.y) : double(v.y);
        } else {
            const c2_t<T> v = lp[l ^ bit];
            if (gen == 1) {
                gr = double(v.x);
                gi = double(v.y);
            } else {
                gr = one ? -double(v.y) : double(v.y);
                gi = one ? double(v.x) : -double(v.x);
            }
        }
        acc += double(lam.x) * gi - double(lam.y) * gr;
    }
    return acc;
}

// Sums the tile's pending probe partials into the gradient (thread 0, in
// probe order, waves in order: the same order a block-wide sum uses).
__device__ __forceinline__ void flush_probes(BatchShared &sh, int np, double *grd) {
    if (threadIdx.x == 0)
        for (int k = 0; k < np; ++k) {
            double t = 0.0;
            for (int w = 0; w < kTileThreads / 64; ++w) t += sh.probe[k][w];
            grd[sh.probe_param[k]] += t;
        }
}

// Ops of one pass on one tile (psi only, or psi and lambda).
template <typename T>
__device__ void batch_tile_ops(const BatchArgs<T> &a, const BatchPass &ps, c2_t<T> *lp, c2_t<T> *ll, bool both,
                               uint64_t base, uint32_t M, const double *prm, double *grd, BatchShared &sh,
                               bool trig) {
    int np = 0;
    for (int o = ps.op_begin; o < ps.op_end; ++o) {
        const TileOp &op = a.ops[o];
        if (op.type == 3) {
            // per-wave sum now, across waves when the tile is done
            double v = batch_probe<T>(lp, ll, op.pos[0], op.kin, M);
            for (int sft = 32; sft > 0; sft >>= 1) v += __shfl_xor(v, sft, 64);
            if (threadIdx.x % 64 == 0) sh.probe[np][threadIdx.x / 64] = v;
            if (threadIdx.x == 0) sh.probe_param[np] = op.moff;
            if (++np == kProbeSlots) {
                __syncthreads();
                flush_probes(sh, np, grd);
                np = 0;
            }
        } else if (op.type == 4) {
            double cs, sn;
            if (trig) {
                cs = sh.cs[op.moff];
                sn = sh.sn[op.moff];
            } else {
                sincos(0.5 * prm[op.moff], &sn, &cs);
            }
            if (op.jbit[0]) sn = -sn;
            tile_rotation<T>(lp, op.pos[0], op.kin, cs, sn, M);
            if (both) tile_rotation<T>(ll, op.pos[0], op.kin, cs, sn, M);
        } else if (op.type == 1) {
            const c2_t<T> *U = a.pool + op.moff;
            tile_diag<T>(lp, op, U, base, M);
            if (both) tile_diag<T>(ll, op, U, base, M);
        } else if (op.type == 5) {
            const c2_t<T> *U = a.pool + op.moff;
            tile_controlled<T>(lp, op, U, M);
            if (both) tile_controlled<T>(ll, op, U, M);
        } else {
            const c2_t<T> *U = a.pool + op.moff;
            switch (op.k) {
                case 1:
                    tile_dense_small<T, 1>(lp, op, U, M);
                    if (both) tile_dense_small<T, 1>(ll, op, U, M);
                    break;
                case 2:
                    tile_dense_small<T, 2>(lp, op, U, M);
                    if (both) tile_dense_small<T, 2>(ll, op, U, M);
                    break;
                default:
                    tile_dense_small<T, 3>(lp, op, U, M);
                    if (both) tile_dense_small<T, 3>(ll, op, U, M);
                    break;
            }
        }
        __syncthreads();
    }
    flush_probes(sh, np, grd);
}

template <typename T>
__device__ __forceinline__ uint64_t batch_scatter(const BatchPass &ps, uint32_t l) {
    uint64_t g = l & ((1u << ps.L) - 1u);
    const uint32_t h = l >> ps.L;
    for (int i = 0; i < ps.H; ++i) g |= uint64_t((h >> i) & 1u) << ps.hpos[i];
    return g;
}

template <typename T>
__global__ void __launch_bounds__(kTileThreads) k_batch(const BatchArgs<T> a) {
    extern __shared__ char lds_raw[];
    __shared__ int s_next;
    __shared__ BatchShared sh;
    c2_t<T> *lp = reinterpret_cast<c2_t<T> *>(lds_raw);
    c2_t<T> *ll = lp + (1u << a.mmax);
    c2_t<T> *gpsi = a.arena + uint64_t(blockIdx.x) * 2ull * a.slot_amps;
    c2_t<T> *glam = gpsi + a.slot_amps;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_next = atomicAdd(a.counter, 1);
        __syncthreads();
        const int qi = s_next;
        if (qi >= a.ncirc) break;
        const BatchCircuit &cc = a.circs[a.order[qi]];
        const BatchProgram &pg = a.progs[cc.prog];
        const double *prm = a.params + cc.param_off;
        double *grd = a.grads + cc.param_off;
        const int n = pg.n;
        const uint32_t M = 1u << pg.m;
        const uint32_t ntiles = 1u << (n - pg.m);
        const bool single = ntiles == 1;
        const uint64_t N = 1ull << n;
        if (a.want_grad)
            for (int j = threadIdx.x; j < cc.nparams; j += kTileThreads) grd[j] = 0.0;
        const bool trig = cc.nparams <= kBatchTrig;
        if (trig)
            for (int j = threadIdx.x; j < cc.nparams; j += kTileThreads) sincos(0.5 * prm[j], &sh.sn[j], &sh.cs[j]);
        // psi = |0...0>
        if (single) {
            for (uint32_t l = threadIdx.x; l < M; l += kTileThreads) {
                c2_t<T> w;
                w.x = (l == 0) ? T(1) : T(0);
                w.y = T(0);
                lp[l] = w;
            }
        }
        __syncthreads();
        // forward
        for (int pi = pg.fwd_begin; pi < pg.fwd_end; ++pi) {
            const BatchPass &ps = a.passes[pi];
            for (uint32_t t = 0; t < ntiles; ++t) {
                uint64_t base = uint64_t(t) << ps.L;
                for (int i = 0; i < ps.H; ++i) {
                    const uint64_t lo = base & ((1ull << ps.hpos[i]) - 1ull);
                    base = ((base - lo) << 1) | lo;
                }
                if (!single) {
                    // kLoadBatch loads per thread in flight before the LDS writes
                    for (uint32_t l0 = threadIdx.x; l0 < M; l0 += kLoadBatch * kTileThreads) {
                        c2_t<T> w[kLoadBatch];
#pragma unroll
                        for (int c = 0; c < kLoadBatch; ++c) {
                            const uint32_t l = l0 + uint32_t(c) * kTileThreads;
                            if (l >= M) break;
                            const uint64_t gi = base | batch_scatter<T>(ps, l);
                            if (pi == pg.fwd_begin) {
                                w[c].x = (gi == 0) ? T(1) : T(0);
                                w[c].y = T(0);
                            } else {
                                w[c] = gpsi[gi];
                            }
                        }
#pragma unroll
                        for (int c = 0; c < kLoadBatch; ++c) {
                            const uint32_t l = l0 + uint32_t(c) * kTileThreads;
                            if (l >= M) break;
                            lp[l] = w[c];
                        }
                    }
                    __syncthreads();
                }
                batch_tile_ops<T>(a, ps, lp, ll, false, base, M, prm, grd, sh, trig);
                if (!single) {
                    for (uint32_t l = threadIdx.x; l < M; l += kTileThreads) gpsi[base | batch_scatter<T>(ps, l)] = lp[l];
                    __syncthreads();
                }
            }
            __threadfence();
            __syncthreads();
        }
        // lambda = H psi and the energy
        {
            const c2_t<T> *src = single ? lp : gpsi;
            c2_t<T> *dst = single ? ll : glam;
            double e = 0.0;
            for (uint64_t y = threadIdx.x; y < N; y += kTileThreads) {
                double ar = 0.0, ai = 0.0;
                for (int g = pg.hg_begin; g < pg.hg_end; ++g) {
                    const BatchHGroup gr = a.hgroups[g];
                    const uint64_t sy = y ^ gr.x;
                    const c2_t<T> b = src[sy];
                    double sr = 0.0, si = 0.0;
                    for (int t = gr.first; t < gr.first + gr.count; ++t) {
                        const BatchHTerm h = a.hterms[t];
                        const double sg = (__popcll(sy & h.z) & 1) ? -1.0 : 1.0;
                        sr += sg * h.wr;
                        si += sg * h.wi;
                    }
                    ar += sr * double(b.x) - si * double(b.y);
                    ai += sr * double(b.y) + si * double(b.x);
                }
                const c2_t<T> p = src[y];
                e += double(p.x) * ar + double(p.y) * ai;
                c2_t<T> o;
                o.x = T(ar);
                o.y = T(ai);
                dst[y] = o;
            }
            const double tot = block_sum(e);
            if (threadIdx.x == 0) a.energies[a.order[qi]] = tot;
            __threadfence();
            __syncthreads();
        }
        if (!a.want_grad) continue;
        // reverse sweep on (psi, lambda)
        for (int pi = pg.rev_begin; pi < pg.rev_end; ++pi) {
            const BatchPass &ps = a.passes[pi];
            for (uint32_t t = 0; t < ntiles; ++t) {
                uint64_t base = uint64_t(t) << ps.L;
                for (int i = 0; i < ps.H; ++i) {
                    const uint64_t lo = base & ((1ull << ps.hpos[i]) - 1ull);
                    base = ((base - lo) << 1) | lo;
                }
                if (!single) {
                    for (uint32_t l0 = threadIdx.x; l0 < M; l0 += kLoadBatch * kTileThreads) {
                        c2_t<T> wp[kLoadBatch], wl[kLoadBatch];
#pragma unroll
                        for (int c = 0; c < kLoadBatch; ++c) {
                            const uint32_t l = l0 + uint32_t(c) * kTileThreads;
                            if (l >= M) break;
                            const uint64_t gi = base | batch_scatter<T>(ps, l);
                            wp[c] = gpsi[gi];
                            wl[c] = glam[gi];
                        }
#pragma unroll
                        for (int c = 0; c < kLoadBatch; ++c) {
                            const uint32_t l = l0 + uint32_t(c) * kTileThreads;
                            if (l >= M) break;
                            lp[l] = wp[c];
                            ll[l] = wl[c];
                        }
                    }
                    __syncthreads();
                }
                batch_tile_ops<T>(a, ps, lp, ll, true, base, M, prm, grd, sh, trig);
                if (!single) {
                    for (uint32_t l = threadIdx.x; l < M; l += kTileThreads) {
                        const uint64_t gi = base | batch_scatter<T>(ps, l);
                        gpsi[gi] = lp[l];
                        glam[gi] = ll[l];
                    }
                    __syncthreads();
                }
            }
            __threadfence();
            __syncthreads();
        }
    }
}

__global__ void k_zero_counter(int *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0;
}

template <typename T>
static hipError_t launch_batch_t(hipStream_t stream, const BatchDevice &d, int grid) {
    BatchArgs<T> a{};
    a.circs = d.circs;
    a.order = d.order;
    a.progs = d.progs;
    a.passes = d.passes;
    a.ops = d.ops;
    a.pool = static_cast<const c2_t<T> *>(d.pool);
    a.hgroups = d.hgroups;
    a.hterms = d.hterms;
    a.params = d.params;
    a.energies = d.energies;
    a.grads = d.grads;
    a.arena = static_cast<c2_t<T> *>(d.arena);
    a.slot_amps = d.slot_amps;
    a.counter = d.counter;
    a.ncirc = d.ncirc;
    a.want_grad = d.want_grad;
    a.mmax = d.mmax;
    const size_t lds = 2 * (sizeof(c2_t<T>) << d.mmax);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch<T>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, stream, d.counter);
    hipLaunchKernelGGL((k_batch<T>), dim3(grid), dim3(kTileThreads), lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_batch(hipStream_t stream, int dtype, const BatchDevice &d, int grid) {
    return dtype == QSIM_C64 ? launch_batch_t<float>(stream, d, grid) : launch_batch_t<double>(stream, d, grid);
}

}  // namespace qsim
