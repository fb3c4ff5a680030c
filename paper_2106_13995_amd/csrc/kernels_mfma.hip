// Fused k-qubit blocks (k = 4..6) as a matrix product on the CDNA4 matrix
// cores.
//
// A block's action on the state is Psi' = Psi U^T, where row g of Psi holds
// the 2^k amplitudes of group g (indices agreeing outside the k target bits).
// Complex arithmetic goes through the real embedding
//   [Re Psi', Im Psi'] = [Re Psi, Im Psi] [[Re U^T, Im U^T], [-Im U^T, Re U^T]],
// a real (rows x 2D) x (2D x 2D) product, D = 2^k.  A persistent workgroup
// of four 64-wide waves loads B once (into registers, or LDS for the largest
// blocks) and then loops over blocks of 64 rows: it gathers a block from HBM
// into LDS, starts the loads of its next block, each wave multiplies its 16
// rows by B with v_mfma_f32_16x16x4f32 (complex64) or v_mfma_f64_16x16x4f64
// (complex128), accumulating every 16-column block in registers, writes the
// result back over its own rows, and the workgroup scatters the rows to HBM.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "qsim_internal.h"

namespace qsim {

constexpr int kMfmaRows = 64;
constexpr int kMfmaThreads = 256;
constexpr int kMfmaMaxBlocks = 2048;   // persistent workgroups; each loops over row blocks

template <typename T>
struct MfmaArgs {
    c2_t<T> *psi;
    const T *B;          // 2D x 2D real embedding, row-major [kk][col]
    uint64_t ngroups;
    uint64_t nblocks;    // ceil(ngroups / kMfmaRows)
    int pos[QSIM_MAX_K]; // target positions, ascending
    uint64_t toff[64];   // offset of local index j
};

template <typename T> struct MfmaOp;
// Operands of both instructions: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16].  Result register r of lane l holds D[row][l % 16] with
// row = 4 (l / 16) + r for the f32 instruction and row = 4 r + l / 16 for the
// f64 one.
template <> struct MfmaOp<float> {
    using acc = __attribute__((ext_vector_type(4))) float;
    static __device__ __forceinline__ acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int lane, int r) { return 4 * (lane / 16) + r; }
};
template <> struct MfmaOp<double> {
    using acc = __attribute__((ext_vector_type(4))) double;
    static __device__ __forceinline__ acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int lane, int r) { return 4 * r + lane / 16; }
};

// Where each lane finds B: 0 registers (loaded once per workgroup), 1 LDS
// (staged once per workgroup), 2 global memory (caches).
template <typename T, int K>
constexpr int b_mode() {
    return sizeof(T) == 4 ? (K <= 5 ? 0 : 1) : (K == 4 ? 0 : K == 5 ? 1 : 2);
}

// Row block of 64 groups in LDS: element (r, c) (c < D: Re of local index c,
// c >= D: Im of local index c - D) at r * W + (c ^ (r & 31)); the XOR keeps
// the 32 lanes of a half-wave that walk down a column in distinct banks.
template <int W>
__device__ __forceinline__ int sidx(int r, int c) {
    return r * W + (c ^ (r & 31));
}

// LOWT: the targets are qubits 0 .. K-1, so a group's 2^K amplitudes are
// contiguous and consecutive threads take consecutive amplitudes; otherwise
// consecutive threads take the same local index of consecutive groups.  (The
// launcher runs the persistent kernel for LOWT blocks only; for scattered
// targets it keeps more blocks in flight with k_fused_mfma_rows.)
template <int D, bool LOWT>
__device__ __forceinline__ void elem_rc(int e, int &r, int &j) {
    if constexpr (LOWT) {
        r = e / D;
        j = e % D;
    } else {
        r = e % kMfmaRows;
        j = e / kMfmaRows;
    }
}

template <typename T, int K, bool LOWT>
__global__ void __launch_bounds__(kMfmaThreads) k_fused_mfma(const MfmaArgs<T> a) {
    constexpr int D = 1 << K;
    constexpr int W = 2 * D;          // real row width
    constexpr int NB = W / 16, KS = W / 4;
    constexpr int PER = kMfmaRows * D / kMfmaThreads;
    constexpr int BM = b_mode<T, K>();
    using Op = MfmaOp<T>;
    using acc_t = typename Op::acc;
    extern __shared__ char lds_raw[];
    T *sA = reinterpret_cast<T *>(lds_raw);
    T *sB = sA + kMfmaRows * W;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int kq = lane / 16, lc = lane % 16;

    T breg[BM == 0 ? KS * NB : 1];
    if constexpr (BM == 0) {
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) breg[s * NB + nb] = a.B[(4 * s + kq) * W + nb * 16 + lc];
    } else if constexpr (BM == 1) {
        for (int e = tid; e < W * W; e += kMfmaThreads) sB[e] = a.B[e];
    }

    c2_t<T> pre[PER];
    auto gather = [&](uint64_t blk) {
        const uint64_t g0 = blk * kMfmaRows;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            int r, j;
            elem_rc<D, LOWT>(tid + i * kMfmaThreads, r, j);
            const uint64_t g = g0 + r;
            c2_t<T> v;
            v.x = T(0);
            v.y = T(0);
            if (g < a.ngroups) v = a.psi[LOWT ? (g << K) | uint64_t(j) : insert_zeros(g, a.pos, K) + a.toff[j]];
            pre[i] = v;
        }
    };

    uint64_t blk = blockIdx.x;
    if (blk < a.nblocks) gather(blk);
    for (; blk < a.nblocks; blk += gridDim.x) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            int r, j;
            elem_rc<D, LOWT>(tid + i * kMfmaThreads, r, j);
            sA[sidx<W>(r, j)] = pre[i].x;
            sA[sidx<W>(r, D + j)] = pre[i].y;
        }
        __syncthreads();
        // the next block's amplitudes are in flight during the products
        if (blk + gridDim.x < a.nblocks) gather(blk + gridDim.x);
        const int arow = wave * 16 + lc;
        acc_t c[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) c[nb] = acc_t{};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const T av = sA[sidx<W>(arow, 4 * s + kq)];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                T bv;
                if constexpr (BM == 0)
                    bv = breg[s * NB + nb];
                else if constexpr (BM == 1)
                    bv = sB[(4 * s + kq) * W + nb * 16 + lc];
                else
                    bv = a.B[(4 * s + kq) * W + nb * 16 + lc];
                c[nb] = Op::mma(av, bv, c[nb]);
            }
        }
        // each wave overwrites only its own 16 rows, after reading all of them
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int i = 0; i < 4; ++i) sA[sidx<W>(wave * 16 + Op::out_row(lane, i), nb * 16 + lc)] = c[nb][i];
        __syncthreads();
        const uint64_t g0 = blk * kMfmaRows;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            int r, j;
            elem_rc<D, LOWT>(tid + i * kMfmaThreads, r, j);
            const uint64_t g = g0 + r;
            if (g >= a.ngroups) continue;
            c2_t<T> v;
            v.x = sA[sidx<W>(r, j)];
            v.y = sA[sidx<W>(r, D + j)];
            a.psi[LOWT ? (g << K) | uint64_t(j) : insert_zeros(g, a.pos, K) + a.toff[j]] = v;
        }
        __syncthreads();   // before the next block overwrites the rows
    }
}

// Targets other than the lowest qubits: a group's amplitudes lie far apart,
// and each local index j is a separate run of consecutive groups in memory.
// One workgroup per block of ROWS groups (many blocks in flight per compute
// unit); ROWS up to 256 makes each run 1-2 KiB long, and each wave takes
// ROWS / 64 sixteen-row blocks, so every B element it loads through the
// caches serves that many products.
template <typename T, int K, int ROWS>
__global__ void __launch_bounds__(kMfmaThreads) k_fused_mfma_rows(const MfmaArgs<T> a) {
    constexpr int D = 1 << K;
    constexpr int W = 2 * D;          // real row width
    constexpr int NB = W / 16, KS = W / 4, RB = ROWS / 64;
    using Op = MfmaOp<T>;
    using acc_t = typename Op::acc;
    extern __shared__ char lds_raw[];
    T *sA = reinterpret_cast<T *>(lds_raw);
    const uint64_t g0 = uint64_t(blockIdx.x) * ROWS;
    // consecutive threads take consecutive groups of one local index; every
    // load of the thread is issued before the first LDS store waits on one
    constexpr int PER = ROWS * D / kMfmaThreads;
    c2_t<T> v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + i * kMfmaThreads;
        const int r = e % ROWS, j = e / ROWS;
        const uint64_t g = g0 + r;
        v[i].x = T(0);
        v[i].y = T(0);
        if (g < a.ngroups) v[i] = a.psi[insert_zeros(g, a.pos, K) + a.toff[j]];
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + i * kMfmaThreads;
        const int r = e % ROWS, j = e / ROWS;
        sA[sidx<W>(r, j)] = v[i].x;
        sA[sidx<W>(r, D + j)] = v[i].y;
    }
    __syncthreads();
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int kq = lane / 16, lc = lane % 16;
    const int row0 = wave * 16 * RB;   // this wave's rows: row0 .. row0 + 16 RB - 1
    acc_t c[RB][NB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) c[rb][nb] = acc_t{};
#pragma unroll 2
    for (int s = 0; s < KS; ++s) {
        T bv[NB];
        const T *brow = a.B + size_t(4 * s + kq) * W + lc;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) bv[nb] = brow[nb * 16];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const T av = sA[sidx<W>(row0 + rb * 16 + lc, 4 * s + kq)];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) c[rb][nb] = Op::mma(av, bv[nb], c[rb][nb]);
        }
    }
    // each wave overwrites only its own rows, after reading all of them
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                sA[sidx<W>(row0 + rb * 16 + Op::out_row(lane, i), nb * 16 + lc)] = c[rb][nb][i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + i * kMfmaThreads;
        const int r = e % ROWS, j = e / ROWS;
        const uint64_t g = g0 + r;
        if (g >= a.ngroups) continue;
        c2_t<T> w;
        w.x = sA[sidx<W>(r, j)];
        w.y = sA[sidx<W>(r, D + j)];
        a.psi[insert_zeros(g, a.pos, K) + a.toff[j]] = w;
    }
}

// Rows per workgroup of the scattered-target kernel, measured on a 30-qubit
// complex64 / 29-qubit complex128 state: 256 except complex128 at k = 4, 6
// (64), where the smaller block keeps more workgroups per compute unit.
template <typename T, int K>
constexpr int rows_per_block() {
    return (sizeof(T) == 8 && K != 5) ? 64 : 256;
}

template <typename T, int K>
static hipError_t mfma_t(qsim_state s, const Plan &plan, const Pass &p) {
    MfmaArgs<T> a{};
    a.psi = static_cast<c2_t<T> *>(s->data);
    a.B = reinterpret_cast<const T *>(static_cast<const char *>(plan.dev) + plan.real_pool_dev_off) + p.pool_begin;
    a.ngroups = 1ull << (s->n - K);
    a.nblocks = (a.ngroups + kMfmaRows - 1) / kMfmaRows;
    bool lowt = true;
    for (int b = 0; b < K; ++b) {
        a.pos[b] = p.targets[b];
        lowt = lowt && p.targets[b] == b;
    }
    for (int j = 0; j < (1 << K); ++j) {
        uint64_t o = 0;
        for (int b = 0; b < K; ++b)
            if ((j >> b) & 1) o |= 1ull << p.targets[b];
        a.toff[j] = o;
    }
    constexpr int W = 2 * (1 << K);
    const size_t lds = sizeof(T) * (size_t(kMfmaRows) * W + (b_mode<T, K>() == 1 ? size_t(W) * W : 0));
    if (!lowt) {
        constexpr int ROWS = rows_per_block<T, K>();
        const size_t lds_rows = sizeof(T) * size_t(ROWS) * W;
        if (lds_rows > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fused_mfma_rows<T, K, ROWS>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_rows));
            if (e != hipSuccess) return e;
        }
        const uint64_t blocks = (a.ngroups + ROWS - 1) / ROWS;
        hipLaunchKernelGGL((k_fused_mfma_rows<T, K, ROWS>), dim3(unsigned(blocks)), dim3(kMfmaThreads), lds_rows,
                           s->stream, a);
        return hipGetLastError();
    }
    const void *fn = reinterpret_cast<const void *>(&k_fused_mfma<T, K, true>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    const unsigned blocks = unsigned(std::min<uint64_t>(a.nblocks, kMfmaMaxBlocks));
    hipLaunchKernelGGL((k_fused_mfma<T, K, true>), dim3(blocks), dim3(kMfmaThreads), lds, s->stream, a);
    return hipGetLastError();
}

hipError_t launch_mfma_pass(qsim_state s, const Plan &plan, const Pass &p) {
    const bool f = s->dtype == QSIM_C64;
    switch (p.k) {
        case 4: return f ? mfma_t<float, 4>(s, plan, p) : mfma_t<double, 4>(s, plan, p);
        case 5: return f ? mfma_t<float, 5>(s, plan, p) : mfma_t<double, 5>(s, plan, p);
        case 6: return f ? mfma_t<float, 6>(s, plan, p) : mfma_t<double, 6>(s, plan, p);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace qsim
