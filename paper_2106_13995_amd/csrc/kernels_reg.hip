// Register-staged tile passes for gfx950.
//
// One workgroup of 256 threads (four 64-wide waves) owns a tile of 2^m
// amplitudes; each thread keeps 2^r of them (r = m - 8) in registers.  A
// stage assigns r tile-local positions to register bits and the other 8 to
// thread bits; the stage's dense gates act on register bits only, so they run
// without touching LDS, and its diagonal gates act anywhere (every thread
// knows the full index of each amplitude it holds).  Between stages the tile
// is written to LDS under one layout and read back under the next, through an
// XOR-swizzled address map chosen on the host to keep lanes in distinct
// banks.  The tile is read from and written back to HBM once per pass.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "qsim_internal.h"
#include "reg_ops.h"

namespace qsim {

constexpr int kRegThreads = 256;

template <typename T>
struct RegArgs {
    c2_t<T> *psi;
    const RegStage *stages;
    const RegOp *ops;
    const c2_t<T> *pool;
    int nstages, nops, npool;
    int m, L, H;
    int hpos[16];
    int32_t ld_t[8], ld_r[kRegBitsMax], st_t[8], st_r[kRegBitsMax];
};

template <typename T, int R>
__global__ void __launch_bounds__(kRegThreads) k_tile_reg(const RegArgs<T> a) {
    constexpr int NA = 1 << R;
    extern __shared__ char lds_raw[];
    c2_t<T> *lds = reinterpret_cast<c2_t<T> *>(lds_raw);
    CRegStage *sst = (CRegStage *)(a.stages);
    CRegOp *sop = (CRegOp *)(a.ops);
    CT<T> *spool = (CT<T> *)(a.pool);
    const uint32_t t = threadIdx.x;
    uint64_t base = uint64_t(blockIdx.x) << a.L;
    for (int i = 0; i < a.H; ++i) {
        const uint64_t lo = base & ((1ull << a.hpos[i]) - 1ull);
        base = ((base - lo) << 1) | lo;
    }
    T vr[NA], vi[NA];
    {
        uint64_t gt = base;
#pragma unroll
        for (int b = 0; b < 8; ++b) gt |= uint64_t((t >> b) & 1u) << a.ld_t[b];
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            uint64_t gi = 0;
#pragma unroll
            for (int b = 0; b < R; ++b)
                if ((i >> b) & 1) gi |= 1ull << a.ld_r[b];
            // every amplitude is read once per pass: nontemporal
            if constexpr (sizeof(T) == 4) {
                const f32x2 w = ld<true, f32x2>(a.psi + (gt | gi));
                vr[i] = w.x;
                vi[i] = w.y;
            } else {
                const f64x2 w = ld<true, f64x2>(a.psi + (gt | gi));
                vr[i] = w.x;
                vi[i] = w.y;
            }
        }
    }
    for (int s = 0; s < a.nstages; ++s) {
        CRegStage &st = sst[s];
        if (s > 0) {
            const uint32_t aw = thread_part<T>(t, st.wr_t);
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                uint32_t ai = aw;
#pragma unroll
                for (int b = 0; b < R; ++b)
                    if ((i >> b) & 1) ai ^= st.wr_r[b];
                c2_t<T> w;
                w.x = vr[i];
                w.y = vi[i];
                lds[ai] = w;
            }
            __syncthreads();
            const uint32_t ar = thread_part<T>(t, st.rd_t);
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                uint32_t ai = ar;
#pragma unroll
                for (int b = 0; b < R; ++b)
                    if ((i >> b) & 1) ai ^= st.rd_r[b];
                const c2_t<T> w = lds[ai];
                vr[i] = w.x;
                vi[i] = w.y;
            }
            __syncthreads();
        }
        for (int o = st.op_begin; o < st.op_end; ++o) {
            CRegOp &op = sop[o];
            run_op<T, R, 0>(op.code, vr, vi, op, spool + 2 * op.moff, base, t);
        }
    }
    {
        uint64_t gt = base;
#pragma unroll
        for (int b = 0; b < 8; ++b) gt |= uint64_t((t >> b) & 1u) << a.st_t[b];
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            uint64_t gi = 0;
#pragma unroll
            for (int b = 0; b < R; ++b)
                if ((i >> b) & 1) gi |= 1ull << a.st_r[b];
            if constexpr (sizeof(T) == 4)
                st<true, f32x2>(a.psi + (gt | gi), f32x2{vr[i], vi[i]});
            else
                st<true, f64x2>(a.psi + (gt | gi), f64x2{vr[i], vi[i]});
        }
    }
}

template <typename T, int R>
static hipError_t launch_reg_t(qsim_state s, const Plan &plan, const Pass &p) {
    RegArgs<T> a{};
    a.psi = static_cast<c2_t<T> *>(s->data);
    const char *dev = static_cast<const char *>(plan.dev);
    a.stages = reinterpret_cast<const RegStage *>(dev + plan.reg_stages_dev_off) + p.stage_begin;
    a.ops = reinterpret_cast<const RegOp *>(dev + plan.reg_ops_dev_off) + p.rop_begin;
    a.pool = reinterpret_cast<const c2_t<T> *>(dev + plan.pool_dev_off) + p.pool_begin;
    a.nstages = p.stage_end - p.stage_begin;
    a.nops = p.rop_end - p.rop_begin;
    a.npool = p.pool_end - p.pool_begin;
    a.m = p.m;
    a.L = p.L;
    a.H = int(p.hpos.size());
    if (a.H > 16 || a.L + a.H != a.m || a.m != R + 8) return hipErrorInvalidValue;
    for (int i = 0; i < a.H; ++i) a.hpos[i] = p.hpos[i];
    for (int b = 0; b < 8; ++b) {
        a.ld_t[b] = p.ld_t[b];
        a.st_t[b] = p.st_t[b];
    }
    for (int b = 0; b < kRegBitsMax; ++b) {
        a.ld_r[b] = p.ld_r[b];
        a.st_r[b] = p.st_r[b];
    }
    const size_t lds = sizeof(c2_t<T>) << p.m;
    const uint64_t ntiles = 1ull << (s->n - p.m);
    hipLaunchKernelGGL((k_tile_reg<T, R>), dim3(unsigned(ntiles)), dim3(kRegThreads), lds, s->stream, a);
    return hipGetLastError();
}

hipError_t launch_tile_reg_pass(qsim_state s, const Plan &plan, const Pass &p) {
    const bool f = s->dtype == QSIM_C64;
    switch (p.reg_r) {
        case 3: return f ? launch_reg_t<float, 3>(s, plan, p) : launch_reg_t<double, 3>(s, plan, p);
        case 4: return f ? launch_reg_t<float, 4>(s, plan, p) : launch_reg_t<double, 4>(s, plan, p);
        case 5: return f ? launch_reg_t<float, 5>(s, plan, p) : launch_reg_t<double, 5>(s, plan, p);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace qsim
