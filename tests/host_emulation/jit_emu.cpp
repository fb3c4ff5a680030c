// Runs the run-time compiled tile passes on the host, in order, over every
// tile: each workgroup's 256 threads are POSIX threads meeting at a barrier
// for __syncthreads(), and the tile array is one static array (workgroups run
// one at a time).  Arguments: the directory jit_emit wrote, the input state
// file, the output state file.
#include <pthread.h>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
struct EmuDim { unsigned x; };
static thread_local EmuDim threadIdx;
static EmuDim blockIdx;
static pthread_barrier_t g_bar;
static inline void __syncthreads() { pthread_barrier_wait(&g_bar); }
// block-wide OR of one predicate per thread (barrier, sum, barrier)
static int g_or_acc;
static pthread_mutex_t g_or_mu = PTHREAD_MUTEX_INITIALIZER;
static inline int __syncthreads_or(int v) {
    if (threadIdx.x == 0) g_or_acc = 0;
    pthread_barrier_wait(&g_bar);
    if (v) {
        pthread_mutex_lock(&g_or_mu);
        g_or_acc = 1;
        pthread_mutex_unlock(&g_or_mu);
    }
    pthread_barrier_wait(&g_bar);
    const int r = g_or_acc;
    pthread_barrier_wait(&g_bar);
    return r;
}
#define __global__
#define __launch_bounds__(x)
#define __shared__ static
#include "passes.inc"
#ifndef EMU_DOUBLE
typedef f2 VT; typedef float ST;
#else
typedef d2 VT; typedef double ST;
#endif
typedef void (*Kern)(VT *, const ST *, unsigned char *);
static Kern kernels[] = {
#include "table.inc"
};
struct Arg { Kern k; VT *psi; const ST *pool; unsigned char *maps; unsigned t; };
static void *run(void *a_) {
    Arg *a = static_cast<Arg *>(a_);
    threadIdx.x = a->t;
    a->k(a->psi, a->pool, a->maps);
    return nullptr;
}
int main(int argc, char **argv) {
    const char *dir = argv[1];
    char path[512];
    snprintf(path, sizeof path, "%s/plan.txt", dir);
    FILE *f = fopen(path, "r");
    int n, dt, shift; size_t np;
    if (fscanf(f, "%d %d %zu %d", &n, &dt, &np, &shift) != 4) return 2;
    std::vector<unsigned long long> ntiles(np); std::vector<int> pb(np);
    for (size_t i = 0; i < np; ++i) if (fscanf(f, "%llu %d", &ntiles[i], &pb[i]) != 2) return 2;
    fclose(f);
    snprintf(path, sizeof path, "%s/pool.bin", dir);
    f = fopen(path, "rb"); fseek(f, 0, SEEK_END); long sz = ftell(f); fseek(f, 0, SEEK_SET);
    std::vector<ST> pool(size_t(sz) / sizeof(ST) + 2);
    if (fread(pool.data(), 1, size_t(sz), f) != size_t(sz)) return 2;
    fclose(f);
    std::vector<VT> psi(size_t(1) << n);
    f = fopen(argv[2], "rb");
    if (fread(psi.data(), sizeof(VT), psi.size(), f) != psi.size()) return 3;
    fclose(f);
    // occupancy maps, zeroed before the chain of passes as the library does
    std::vector<unsigned char> maps(shift > 0 ? size_t(3) << (n - shift) : 1, 0);
    pthread_barrier_init(&g_bar, nullptr, 256);
    std::vector<pthread_t> th(256); std::vector<Arg> args(256);
    for (size_t k = 0; k < np; ++k) {
        for (unsigned long long b = 0; b < ntiles[k]; ++b) {
            blockIdx.x = unsigned(b);
            for (unsigned t = 0; t < 256; ++t) {
                args[t] = Arg{kernels[k], psi.data(), pool.data() + 2 * size_t(pb[k]), maps.data(), t};
                pthread_create(&th[t], nullptr, run, &args[t]);
            }
            for (unsigned t = 0; t < 256; ++t) pthread_join(th[t], nullptr);
        }
    }
    f = fopen(argv[3], "wb");
    fwrite(psi.data(), sizeof(VT), psi.size(), f);
    fclose(f);
    return 0;
}
