// Expectation values without device allocation: the same passes as
// qsim_expectation, with their partial sums, term table and result in a
// fixed device array this file defines, so the call never allocates device
// memory (for callers under graph capture, in serving loops, or in harnesses
// that forbid allocation).
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds its own copy from module load until the process ends.  Host code
// never uses the variable's name as an address (on the host it is only a
// stand-in for the symbol); the device address of each GPU's copy is looked
// up once per device with hipGetSymbolAddress and kept in g_scratch_ptr.
//
// Calls on one GPU share its array and it keeps the last call's contents:
// the kernels write every partial they later read, so nothing has to start
// at zero, but two calls that overlap on one GPU (different streams, or
// different host threads) race on it.  Callers must serialise them.
#include <hip/hip_runtime.h>

#include <mutex>

#include "qsim_internal.h"

namespace {

constexpr size_t kScratchBytes = QSIM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, resolved once per device with that
// device current (the caller's current device is restored).
qsim_status scratch_on(int device, void **out) {
    if (device < 0 || device >= kMaxDevices)
        return qsim::set_error(QSIM_ERR_UNSUPPORTED, "device index outside the fixed-scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return qsim::set_error(QSIM_ERR_DEVICE, "hipGetDevice failed");
        if (cur != device && hipSetDevice(device) != hipSuccess)
            return qsim::set_error(QSIM_ERR_DEVICE, "hipSetDevice failed");
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return qsim::set_error(QSIM_ERR_DEVICE,
                                   std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return QSIM_OK;
}

}  // namespace

extern "C" qsim_status qsim_expectation_noalloc(qsim_state s, const qsim_pauli_sum *H, double *out_host) {
    if (!s) return qsim::set_error(QSIM_ERR_ARG, "state handle is NULL");
    if (!s->valid) return qsim::set_error(QSIM_ERR_STATE, "state is invalid after an earlier device error");
    void *ptr = nullptr;
    const qsim_status st = scratch_on(s->device, &ptr);
    if (st != QSIM_OK) return st;
    return qsim::expectation_with(s, H, out_host, ptr, kScratchBytes);
}
