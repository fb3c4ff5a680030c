// Fused k-qubit blocks (k = 4..6) as a matrix product on the CDNA4 matrix
// cores.
//
// A block's action on the state is Psi' = Psi U^T, where row g of Psi holds
// the 2^k amplitudes of group g (indices agreeing outside the k target bits).
// Complex arithmetic goes through the real embedding
//   [Re Psi', Im Psi'] = [Re Psi, Im Psi] [[Re U^T, Im U^T], [-Im U^T, Re U^T]],
// a real (rows x 2D) x (2D x 2D) product, D = 2^k.  A workgroup of four
// 64-wide waves takes 64 rows: it gathers them from HBM into LDS (rows
// consecutive in memory when the targets are high bits), each wave multiplies
// its 16 rows by B with v_mfma_f32_16x16x4f32 (complex64) or
// v_mfma_f64_16x16x4f64 (complex128), accumulating every 16-column block in
// registers, writes the result back over its own rows, and the workgroup
// scatters the rows to HBM.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "qsim_internal.h"

namespace qsim {

constexpr int kMfmaRows = 64;
constexpr int kMfmaThreads = 256;

template <typename T>
struct MfmaArgs {
    c2_t<T> *psi;
    const T *B;          // 2D x 2D real embedding, row-major [kk][col]
    uint64_t ngroups;
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

template <typename T, int K>
__global__ void __launch_bounds__(kMfmaThreads) k_fused_mfma(const MfmaArgs<T> a) {
    constexpr int D = 1 << K;
    constexpr int W = 2 * D;          // real row width
    constexpr int S = W + 4;          // LDS row stride (keeps 16 rows x 4 columns in distinct banks)
    using Op = MfmaOp<T>;
    using acc_t = typename Op::acc;
    extern __shared__ char lds_raw[];
    T *sA = reinterpret_cast<T *>(lds_raw);
    const uint64_t g0 = uint64_t(blockIdx.x) * kMfmaRows;
    // gather 64 rows; consecutive threads take consecutive rows of one column
    for (int e = threadIdx.x; e < kMfmaRows * D; e += kMfmaThreads) {
        const int r = e % kMfmaRows, j = e / kMfmaRows;
        const uint64_t g = g0 + r;
        T re = T(0), im = T(0);
        if (g < a.ngroups) {
            const c2_t<T> v = a.psi[insert_zeros(g, a.pos, K) + a.toff[j]];
            re = v.x;
            im = v.y;
        }
        sA[r * S + j] = re;
        sA[r * S + D + j] = im;
    }
    __syncthreads();
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int arow = wave * 16 + (lane % 16);   // A operand: row lane%16, column lane/16 of the k-step
    const int kq = lane / 16;
    acc_t c[W / 16];
#pragma unroll
    for (int nb = 0; nb < W / 16; ++nb) c[nb] = acc_t{};
#pragma unroll 4
    for (int s = 0; s < W / 4; ++s) {
        const T av = sA[arow * S + 4 * s + kq];
        const T *brow = a.B + size_t(4 * s + kq) * W + (lane % 16);
#pragma unroll
        for (int nb = 0; nb < W / 16; ++nb) c[nb] = Op::mma(av, brow[nb * 16], c[nb]);
    }
    // each wave overwrites only its own 16 rows, after reading all of them
#pragma unroll
    for (int nb = 0; nb < W / 16; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i) sA[(wave * 16 + Op::out_row(lane, i)) * S + nb * 16 + (lane % 16)] = c[nb][i];
    __syncthreads();
    for (int e = threadIdx.x; e < kMfmaRows * D; e += kMfmaThreads) {
        const int r = e % kMfmaRows, j = e / kMfmaRows;
        const uint64_t g = g0 + r;
        if (g >= a.ngroups) continue;
        c2_t<T> v;
        v.x = sA[r * S + j];
        v.y = sA[r * S + D + j];
        a.psi[insert_zeros(g, a.pos, K) + a.toff[j]] = v;
    }
}

template <typename T, int K>
static hipError_t mfma_t(qsim_state s, const Plan &plan, const Pass &p) {
    MfmaArgs<T> a{};
    a.psi = static_cast<c2_t<T> *>(s->data);
    a.B = reinterpret_cast<const T *>(static_cast<const char *>(plan.dev) + plan.real_pool_dev_off) + p.pool_begin;
    a.ngroups = 1ull << (s->n - K);
    for (int b = 0; b < K; ++b) a.pos[b] = p.targets[b];
    for (int j = 0; j < (1 << K); ++j) {
        uint64_t o = 0;
        for (int b = 0; b < K; ++b)
            if ((j >> b) & 1) o |= 1ull << p.targets[b];
        a.toff[j] = o;
    }
    constexpr int S = 2 * (1 << K) + 4;
    const size_t lds = sizeof(T) * size_t(kMfmaRows) * S;
    const void *fn = reinterpret_cast<const void *>(&k_fused_mfma<T, K>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    const uint64_t blocks = (a.ngroups + kMfmaRows - 1) / kMfmaRows;
    hipLaunchKernelGGL((k_fused_mfma<T, K>), dim3(unsigned(blocks)), dim3(kMfmaThreads), lds, s->stream, a);
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
