// Layered batch execution (gfx950): circuits that fill whole tiles run one
// launch per pass index, each launch applying that pass of every such
// circuit to all of its tiles at once (one workgroup per tile).
//
// A workgroup of 256 threads holds its tile in registers, 2^R amplitudes a
// thread, as the single-state register passes do: a stage's dense ops act on
// its register bits and the tile is re-laid out through LDS between stages.
// In the reverse sweep a thread holds psi and lambda side by side (register
// bit R selects lambda), so every op applies to both alike and the probes
// Im <lambda|G|psi> read the two halves.  Rotations read their lifting
// multiplier and sine from a table formed once per run; probes leave one
// partial per (probe, tile), the energy one per chunk, and fixed-order
// reductions give the gradient and the energies (bitwise reproducible).
#include <hip/hip_runtime.h>

#include "batch.h"
#include "device_common.h"
#include "qsim_internal.h"
#include "reg_ops.h"

namespace qsim {

constexpr int kLayerThreads = 256;
constexpr int kLayerProbeSlots = 64;

typedef const QSIM_CONST BatchPass CBatchPass;
typedef const QSIM_CONST BatchWork CBatchWork;
typedef const QSIM_CONST BatchLCirc CBatchLCirc;
typedef const QSIM_CONST BatchProgram CBatchProgram;

template <typename T>
struct LayerArgs {
    const BatchLCirc *lc;
    const BatchWork *works;
    const BatchPass *passes;
    const RegStage *stages;
    const RegOp *rops;
    const c2_t<T> *pool;
    const double *trig;
    c2_t<T> *arena;
    c2_t<T> *lam_arena;
    double *ppart;
    int wbegin, wend;
    int init;
};

// The work item of workgroup `bid`: the last of works[lo, hi) whose first
// workgroup is at most bid (uniform: scalar loads).
__device__ __forceinline__ int find_work(CBatchWork *w, int lo, int hi, uint32_t bid) {
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (w[mid].first <= bid)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// First global index of tile t of a pass: t's bits spread over the
// positions outside the tile.
__device__ __forceinline__ uint64_t layer_tile_base(CBatchPass &ps, uint32_t t) {
    uint64_t base = uint64_t(t) << ps.L;
    for (int i = 0; i < ps.H; ++i) {
        const uint64_t lo = base & ((1ull << ps.hpos[i]) - 1ull);
        base = ((base - lo) << 1) | lo;
    }
    return base;
}

// X / Y rotation on the register bit of code 220 + b / 228 + b.
template <typename T, int R, int RA, int B>
__device__ __forceinline__ void brot_dispatch(int code, T *vr, T *vi, double P, double s, bool neg) {
    if constexpr (B < R) {
        if (code == 220 + B) {
            brot_bit<T, RA, B, 1>(vr, vi, P, s, neg);
            return;
        }
        if (code == 228 + B) {
            brot_bit<T, RA, B, 2>(vr, vi, P, s, neg);
            return;
        }
        brot_dispatch<T, R, RA, B + 1>(code, vr, vi, P, s, neg);
    }
}

// Probe Im <lambda|G|psi> over the thread's amplitudes (psi at [0, 2^R),
// lambda at [2^R, 2^(R+1))), G = X (GEN 1) or Y (GEN 2) on register bit B:
// each pair's terms in the state precision, the pairs summed in double.
template <typename T, int R, int B, int GEN>
__device__ __forceinline__ double bprobe_bit(const T *vr, const T *vi) {
    constexpr int NA = 1 << R;
    double acc = 0.0;
#pragma unroll
    for (int g = 0; g < NA; ++g) {
        if (g & (1 << B)) continue;
        const int h = g | (1 << B);
        const T pgr = vr[g], pgi = vi[g], phr = vr[h], phi = vi[h];
        const T lgr = vr[NA + g], lgi = vi[NA + g], lhr = vr[NA + h], lhi = vi[NA + h];
        T v;
        if constexpr (GEN == 1)   // (X psi)_g = psi_h, (X psi)_h = psi_g
            v = (lgr * phi - lgi * phr) + (lhr * pgi - lhi * pgr);
        else                      // (Y psi)_g = -i psi_h, (Y psi)_h = i psi_g
            v = (lhr * pgr + lhi * pgi) - (lgr * phr + lgi * phi);
        acc += double(v);
    }
    return acc;
}

// Z probe on the bit the op names (as brot_z): amplitudes whose bit is 1
// count negatively.
template <typename T, int R>
__device__ __forceinline__ double bprobe_z(const T *vr, const T *vi, CRegOp &op, uint64_t base, uint32_t t) {
    constexpr int NA = 1 << R;
    const bool up = outer_bit(op, base, t);
    const int rm = op.rmask;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const T v = vr[NA + i] * vi[i] - vi[NA + i] * vr[i];
        const bool one = up || ((i & rm) != 0);
        acc += one ? -double(v) : double(v);
    }
    return acc;
}

template <typename T, int R, int B>
__device__ __forceinline__ double bprobe_dispatch(int code, const T *vr, const T *vi) {
    if constexpr (B < R) {
        if (code == 240 + B) return bprobe_bit<T, R, B, 1>(vr, vi);
        if (code == 248 + B) return bprobe_bit<T, R, B, 2>(vr, vi);
        return bprobe_dispatch<T, R, B + 1>(code, vr, vi);
    }
    return 0.0;
}

// Z probe on register bit B.
template <typename T, int R, int B>
__device__ __forceinline__ double bprobe_z_bit(const T *vr, const T *vi) {
    constexpr int NA = 1 << R;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const T v = vr[NA + i] * vi[i] - vi[NA + i] * vr[i];
        acc += ((i >> B) & 1) ? -double(v) : double(v);
    }
    return acc;
}

// Probe and inverse rotation of generator G on register bit B, parameter m.
template <typename T, int R, int RA, int B, int G>
__device__ __forceinline__ double probe_rotate(T *vr, T *vi, const QSIM_CONST double *trig, int m) {
    const double v = G == 3 ? bprobe_z_bit<T, R, B>(vr, vi) : bprobe_bit<T, R, B, (G == 3 ? 1 : G)>(vr, vi);
    const double P = -trig[4 * m], sn = -trig[4 * m + 1];
    const bool neg = trig[4 * m + 2] < 0.0;
    if constexpr (G == 3)
        brot_z_bit<T, RA, B>(vr, vi, P, sn, neg);
    else
        brot_bit<T, RA, B, G>(vr, vi, P, sn, neg);
    return v;
}

// Two probe-and-inverse-rotation ops on one register bit (codes 344 + ..).
template <typename T, int R, int RA, int C>
__device__ __forceinline__ void probe_pair(int code, T *vr, T *vi, CRegOp &op, const QSIM_CONST double *trig,
                                           double &v1, double &v2) {
    if constexpr (C < 344 + 72) {
        constexpr int B = (C - 344) % 8, G1 = (C - 344) / 24 + 1, G2 = ((C - 344) / 8) % 3 + 1;
        if constexpr (B < R) {
            if (code == C) {
                v1 = probe_rotate<T, R, RA, B, G1>(vr, vi, trig, op.moff);
                v2 = probe_rotate<T, R, RA, B, G2>(vr, vi, trig, op.gj[0]);
                return;
            }
        }
        probe_pair<T, R, RA, C + 1>(code, vr, vi, op, trig, v1, v2);
    }
}

// Sums the pending probes of this tile over the waves (wave order) and
// writes them to their (probe, tile) partials.
__device__ __forceinline__ void layer_flush(const double (*probe)[kLayerThreads / 64], const int *probe_k, int np,
                                            double *pp, uint32_t ntiles, uint32_t tile) {
    const int k = int(threadIdx.x);
    if (k < np) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kLayerThreads / 64; ++w) v += probe[k][w];
        pp[uint64_t(probe_k[k]) * ntiles + tile] = v;
    }
}

// One pass of one circuit on one tile per workgroup.  Forward (BOTH false):
// psi only; reverse: psi and lambda, with probes.  `init` starts psi at
// |0...0> instead of loading it.
template <typename T, int R, bool BOTH>
__global__ void __launch_bounds__(kLayerThreads) k_batch_layer(const LayerArgs<T> a) {
    constexpr int NA = 1 << R;
    constexpr int RA = BOTH ? R + 1 : R;
    constexpr int NV = 1 << RA;
    extern __shared__ char lds_raw[];
    __shared__ double probe[kLayerProbeSlots][kLayerThreads / 64];
    __shared__ int probe_k[kLayerProbeSlots];
    c2_t<T> *lp = reinterpret_cast<c2_t<T> *>(lds_raw);
    c2_t<T> *ll = lp + NA * kLayerThreads;
    CBatchWork *works = (CBatchWork *)(a.works);
    const uint32_t bid = blockIdx.x;
    const int w = find_work(works, a.wbegin, a.wend, bid);
    const uint32_t tile = bid - works[w].first;
    CBatchLCirc &c = ((CBatchLCirc *)(a.lc))[works[w].lc];
    CBatchPass &ps = ((CBatchPass *)(a.passes))[works[w].pass];
    CRegStage *sst = (CRegStage *)(a.stages);
    CRegOp *sop = (CRegOp *)(a.rops);
    CT<T> *spool = (CT<T> *)(a.pool);
    const QSIM_CONST double *trig = (const QSIM_CONST double *)(a.trig) + 4 * c.param_off;
    c2_t<T> *psi = a.arena + c.psi_off;
    c2_t<T> *lam = a.lam_arena + c.lam_off;
    const uint64_t base = layer_tile_base(ps, tile);
    const uint32_t t = threadIdx.x;
    T vr[NV], vi[NV];
    {
        uint64_t gt = base;
#pragma unroll
        for (int b = 0; b < 8; ++b) gt |= uint64_t((t >> b) & 1u) << ps.ld_t[b];
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            uint64_t gi = gt;
#pragma unroll
            for (int b = 0; b < R; ++b)
                if ((i >> b) & 1) gi |= 1ull << ps.ld_r[b];
            if (!BOTH && a.init) {
                vr[i] = gi == 0 ? T(1) : T(0);
                vi[i] = T(0);
            } else {
                const c2_t<T> u = psi[gi];
                vr[i] = u.x;
                vi[i] = u.y;
            }
            if constexpr (BOTH) {
                const c2_t<T> u = lam[gi];
                vr[NA + i] = u.x;
                vi[NA + i] = u.y;
            }
        }
    }
    int np = 0;
    for (int s = ps.stage_begin; s < ps.stage_end; ++s) {
        CRegStage &st = sst[s];
        if (s > ps.stage_begin) {
            const uint32_t aw = thread_part<T>(t, st.wr_t);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                uint32_t ai = aw;
#pragma unroll
                for (int b = 0; b < R; ++b)
                    if ((i >> b) & 1) ai ^= st.wr_r[b];
                c2_t<T> u;
                u.x = vr[i];
                u.y = vi[i];
                (i < NA ? lp : ll)[ai] = u;
            }
            __syncthreads();
            const uint32_t ar = thread_part<T>(t, st.rd_t);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                uint32_t ai = ar;
#pragma unroll
                for (int b = 0; b < R; ++b)
                    if ((i >> b) & 1) ai ^= st.rd_r[b];
                const c2_t<T> u = (i < NA ? lp : ll)[ai];
                vr[i] = u.x;
                vi[i] = u.y;
            }
            __syncthreads();
        }
        for (int o = st.op_begin; o < st.op_end; ++o) {
            CRegOp &op = sop[o];
            const int code = op.code;
            if (code < 240 || (code >= 288 && code < 344)) {
                run_op<T, R, 0, RA, true>(code, vr, vi, op, spool + 2 * op.moff, base, t, trig);
            } else if constexpr (!BOTH) {
                __builtin_unreachable();   // forward passes hold no probes
            } else if (code >= 344) {
                // two probes with their inverse rotations
                if (np + 2 > kLayerProbeSlots) {
                    __syncthreads();
                    layer_flush(probe, probe_k, np, a.ppart + c.pp_off, uint32_t(c.ntiles), tile);
                    __syncthreads();
                    np = 0;
                }
                double v1 = 0.0, v2 = 0.0;
                probe_pair<T, R, RA, 344>(code, vr, vi, op, trig, v1, v2);
                for (int sft = 32; sft > 0; sft >>= 1) {
                    v1 += __shfl_xor(v1, sft, 64);
                    v2 += __shfl_xor(v2, sft, 64);
                }
                if (t % 64 == 0) {
                    probe[np][t / 64] = v1;
                    probe[np + 1][t / 64] = v2;
                }
                if (t == 0) {
                    probe_k[np] = op.jmatch;
                    probe_k[np + 1] = op.jmatch + 1;
                }
                np += 2;
                if (np == kLayerProbeSlots) {
                    __syncthreads();
                    layer_flush(probe, probe_k, np, a.ppart + c.pp_off, uint32_t(c.ntiles), tile);
                    __syncthreads();
                    np = 0;
                }
            } else {
                // probe (240 + ..), or probe and inverse rotation (264 + ..)
                const int pc = code >= 264 ? code - 24 : code;
                double v = pc == 256 ? bprobe_z<T, R>(vr, vi, op, base, t) : bprobe_dispatch<T, R, 0>(pc, vr, vi);
                if (code >= 264) {
                    // the inverse rotation: P and s negated
                    const double P = -trig[4 * op.moff], sn = -trig[4 * op.moff + 1];
                    const bool neg = trig[4 * op.moff + 2] < 0.0;
                    if (pc == 256)
                        brot_z<T, RA>(vr, vi, op, P, sn, neg, base, t);
                    else
                        brot_dispatch<T, R, RA, 0>(pc - 20, vr, vi, P, sn, neg);
                }
                for (int sft = 32; sft > 0; sft >>= 1) v += __shfl_xor(v, sft, 64);
                if (t % 64 == 0) probe[np][t / 64] = v;
                if (t == 0) probe_k[np] = op.jmatch;
                if (++np == kLayerProbeSlots) {
                    __syncthreads();
                    layer_flush(probe, probe_k, np, a.ppart + c.pp_off, uint32_t(c.ntiles), tile);
                    __syncthreads();
                    np = 0;
                }
            }
        }
    }
    {
        uint64_t gt = base;
#pragma unroll
        for (int b = 0; b < 8; ++b) gt |= uint64_t((t >> b) & 1u) << ps.st_t[b];
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            uint64_t gi = gt;
#pragma unroll
            for (int b = 0; b < R; ++b)
                if ((i >> b) & 1) gi |= 1ull << ps.st_r[b];
            c2_t<T> u;
            u.x = vr[i];
            u.y = vi[i];
            psi[gi] = u;
            if constexpr (BOTH) {
                c2_t<T> l;
                l.x = vr[NA + i];
                l.y = vi[NA + i];
                lam[gi] = l;
            }
        }
    }
    if constexpr (BOTH) {
        if (np > 0) {
            __syncthreads();
            layer_flush(probe, probe_k, np, a.ppart + c.pp_off, uint32_t(c.ntiles), tile);
        }
    }
}

// Lifting form of every parameter's rotation: with c, s the cosine and
// sine of half its angle, (P, s, c, 0) where P = -s / (1 + c) for c >= 0 and
// s / (1 - c) otherwise (the forms lift3 takes).
__global__ void k_batch_trig(const double *params, double *trig, int64_t n) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j < n) {
        double s, c;
        sincos(0.5 * params[j], &s, &c);
        trig[4 * j] = c >= 0.0 ? -s / (1.0 + c) : s / (1.0 - c);
        trig[4 * j + 1] = s;
        trig[4 * j + 2] = c;
        trig[4 * j + 3] = 0.0;
    }
}

template <typename T>
struct EnergyArgs {
    const BatchLCirc *lc;
    const BatchWork *works;
    const BatchProgram *progs;
    const BatchHGroup *hgroups;
    const BatchHTerm *hterms;
    c2_t<T> *arena;
    c2_t<T> *lam_arena;
    double *epart;
    int wbegin, wend;
    int want_grad;
};

// lambda = H psi on one chunk of one circuit, and the chunk's part of
// <psi|H|psi>.  H is a sum of Pauli strings grouped by X mask: for each
// group, the amplitude at y ^ x times the signed sum of the group's weights.
// A thread takes kEnergySub amplitudes y = chunk start + thread + 256 k at a
// time, so each term (read once, uniform) serves all of them; whether y is
// inside the state is uniform (states of 2^11 and more amplitudes).
constexpr int kEnergySub = 8;

template <typename T>
__global__ void __launch_bounds__(kLayerThreads) k_batch_energy(const EnergyArgs<T> a) {
    CBatchWork *works = (CBatchWork *)(a.works);
    const uint32_t bid = blockIdx.x;
    const int w = find_work(works, a.wbegin, a.wend, bid);
    const uint32_t chunk = bid - works[w].first;
    CBatchLCirc &c = ((CBatchLCirc *)(a.lc))[works[w].lc];
    CBatchProgram &pg = ((CBatchProgram *)(a.progs))[c.prog];
    const QSIM_CONST BatchHGroup *hg = (const QSIM_CONST BatchHGroup *)(a.hgroups);
    const QSIM_CONST BatchHTerm *ht = (const QSIM_CONST BatchHTerm *)(a.hterms);
    const c2_t<T> *src = a.arena + c.psi_off;
    c2_t<T> *dst = a.lam_arena + c.lam_off;
    const uint64_t N = 1ull << pg.n;
    const uint64_t cbase = uint64_t(chunk) * kBatchChunk;
    double e = 0.0;
    for (int h0 = 0; h0 < kBatchChunk / kLayerThreads; h0 += kEnergySub) {
        if (cbase + uint64_t(h0) * kLayerThreads >= N) break;
        uint64_t y[kEnergySub];
        bool in[kEnergySub];
#pragma unroll
        for (int k = 0; k < kEnergySub; ++k) {
            y[k] = cbase + uint64_t(h0 + k) * kLayerThreads + threadIdx.x;
            in[k] = cbase + uint64_t(h0 + k) * kLayerThreads < N;
        }
        double ar[kEnergySub], ai[kEnergySub];
#pragma unroll
        for (int k = 0; k < kEnergySub; ++k) ar[k] = ai[k] = 0.0;
        for (int g = pg.hg_begin; g < pg.hg_end; ++g) {
            const uint64_t x = hg[g].x;
            const int t0 = hg[g].first, t1 = t0 + hg[g].count;
            T bx[kEnergySub], by[kEnergySub];
#pragma unroll
            for (int k = 0; k < kEnergySub; ++k) {
                if (!in[k]) continue;
                const c2_t<T> b = src[y[k] ^ x];
                bx[k] = b.x;
                by[k] = b.y;
            }
            double sr[kEnergySub], si[kEnergySub];
#pragma unroll
            for (int k = 0; k < kEnergySub; ++k) sr[k] = si[k] = 0.0;
            for (int tt = t0; tt < t1; ++tt) {
                const uint64_t z = ht[tt].z;
                const double wr = ht[tt].wr, wi = ht[tt].wi;
#pragma unroll
                for (int k = 0; k < kEnergySub; ++k) {
                    const bool neg = __popcll((y[k] ^ x) & z) & 1;
                    sr[k] += neg ? -wr : wr;
                    si[k] += neg ? -wi : wi;
                }
            }
#pragma unroll
            for (int k = 0; k < kEnergySub; ++k) {
                if (!in[k]) continue;
                ar[k] += sr[k] * double(bx[k]) - si[k] * double(by[k]);
                ai[k] += sr[k] * double(by[k]) + si[k] * double(bx[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < kEnergySub; ++k) {
            if (!in[k]) continue;
            const c2_t<T> p = src[y[k]];
            e += double(p.x) * ar[k] + double(p.y) * ai[k];
            if (a.want_grad) {
                c2_t<T> o;
                o.x = T(ar[k]);
                o.y = T(ai[k]);
                dst[y[k]] = o;
            }
        }
    }
    const double tot = block_sum(e);
    if (threadIdx.x == 0) a.epart[c.ep_off + chunk] = tot;
}

// energies[circ] = sum of the circuit's chunk partials, in chunk order.
__global__ void k_batch_energy_reduce(const BatchLCirc *lc, int nlc, const double *epart, double *energies) {
    const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nlc) return;
    const BatchLCirc c = lc[i];
    double s = 0.0;
    for (int k = 0; k < c.nchunks; ++k) s += epart[c.ep_off + uint64_t(k)];
    energies[c.circ] = s;
}

// One wave per gradient entry of a layered circuit: the sum over the
// parameter's probes and the circuit's tiles of the probe partials (each
// lane a fixed stride of tiles, then a fixed butterfly).
__global__ void __launch_bounds__(256) k_batch_grad_reduce(const BatchLCirc *lc, int nlc, const BatchProgram *progs,
                                                           const int32_t *probe_row, const int32_t *probe_idx,
                                                           const double *ppart, double *grads, int64_t gw_begin,
                                                           int64_t gw_end) {
    const int64_t gw = gw_begin + int64_t(blockIdx.x) * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (gw >= gw_end) return;
    int lo = 0, hi = nlc;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (lc[mid].gfirst <= gw)
            lo = mid;
        else
            hi = mid;
    }
    const BatchLCirc c = lc[lo];
    const int j = int(gw - c.gfirst);
    const BatchProgram pg = progs[c.prog];
    double acc = 0.0;
    if (j < pg.nparams) {
        const int r0 = probe_row[pg.row_off + j], r1 = probe_row[pg.row_off + j + 1];
        for (int r = r0; r < r1; ++r) {
            const double *pp = ppart + c.pp_off + uint64_t(probe_idx[r]) * uint64_t(c.ntiles);
            for (int tl = lane; tl < c.ntiles; tl += 64) acc += pp[tl];
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) grads[c.param_off + j] = acc;
}

template <typename T, int R>
static hipError_t layer_lds(size_t &fwd, size_t &rev) {
    fwd = sizeof(c2_t<T>) * size_t(kLayerThreads) << R;
    rev = 2 * fwd;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_layer<T, R, false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(fwd));
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_layer<T, R, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(rev));
    return e;
}

hipError_t batch_layer_setup(int dtype, int R) {
    size_t f, r;
    if (dtype == QSIM_C64) return R == 4 ? layer_lds<float, 4>(f, r) : layer_lds<float, 3>(f, r);
    return layer_lds<double, 3>(f, r);
}

template <typename T, int R>
static hipError_t launch_layered_t(hipStream_t stream, const BatchLayerDevice &d) {
    size_t lds_f = sizeof(c2_t<T>) * size_t(kLayerThreads) << R, lds_r = 2 * lds_f;
    LayerArgs<T> la{};
    la.lc = d.lc;
    la.works = d.works;
    la.passes = d.passes;
    la.stages = d.stages;
    la.rops = d.rops;
    la.pool = static_cast<const c2_t<T> *>(d.pool);
    la.trig = d.trig;
    la.arena = static_cast<c2_t<T> *>(d.arena);
    la.lam_arena = static_cast<c2_t<T> *>(d.lam_arena ? d.lam_arena : d.arena);
    la.ppart = d.ppart;
    EnergyArgs<T> ea{};
    ea.lc = d.lc;
    ea.works = d.works;
    ea.progs = d.progs;
    ea.hgroups = d.hgroups;
    ea.hterms = d.hterms;
    ea.arena = static_cast<c2_t<T> *>(d.arena);
    ea.lam_arena = la.lam_arena;
    ea.epart = d.epart;
    ea.want_grad = d.want_grad;
    if (d.nparams > 0)
        hipLaunchKernelGGL(k_batch_trig, dim3(unsigned((d.nparams + 255) / 256)), dim3(256), 0, stream, d.params,
                           d.trig, d.nparams);
    for (const BatchStep &s : d.steps) {
        if (s.kind == 0 || s.kind == 1) {
            if (s.wgs == 0) continue;
            la.wbegin = s.wbegin;
            la.wend = s.wend;
            la.init = s.init;
            if (s.kind == 0)
                hipLaunchKernelGGL((k_batch_layer<T, R, false>), dim3(s.wgs), dim3(kLayerThreads), lds_f, stream, la);
            else
                hipLaunchKernelGGL((k_batch_layer<T, R, true>), dim3(s.wgs), dim3(kLayerThreads), lds_r, stream, la);
        } else if (s.kind == 2) {
            if (s.wgs == 0) continue;
            ea.wbegin = s.wbegin;
            ea.wend = s.wend;
            hipLaunchKernelGGL((k_batch_energy<T>), dim3(s.wgs), dim3(kLayerThreads), 0, stream, ea);
            const int nl = s.lc_end - s.lc_begin;
            hipLaunchKernelGGL(k_batch_energy_reduce, dim3(unsigned((nl + 255) / 256)), dim3(256), 0, stream,
                               d.lc + s.lc_begin, nl, d.epart, d.energies);
        } else if (s.gw_end > s.gw_begin) {
            hipLaunchKernelGGL(k_batch_grad_reduce, dim3(unsigned((s.gw_end - s.gw_begin + 3) / 4)), dim3(256), 0,
                               stream, d.lc + s.lc_begin, s.lc_end - s.lc_begin, d.progs, d.probe_row, d.probe_idx,
                               d.ppart, d.grads, s.gw_begin, s.gw_end);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_batch_layered(hipStream_t stream, int dtype, const BatchLayerDevice &d) {
    if (dtype == QSIM_C64) return d.R == 4 ? launch_layered_t<float, 4>(stream, d) : launch_layered_t<float, 3>(stream, d);
    if (d.R != 3) return hipErrorInvalidValue;
    return launch_layered_t<double, 3>(stream, d);
}

}  // namespace qsim
