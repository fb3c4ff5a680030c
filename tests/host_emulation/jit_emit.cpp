// Writes the run-time compiled source of a circuit's register tile passes for
// a host build (tests/test_jit_emulated.py): the passes' source, their grid
// and matrix-pool offsets, the pool in the state precision.  Device launchers
// are stubs that abort: planning must never reach them.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <cmath>
#include <string>

#include "batch.h"
#include "qsim_internal.h"

namespace qsim {
[[noreturn]] static void no_device(const char *what) {
    std::fprintf(stderr, "planner reached a device launch: %s\n", what);
    std::abort();
}
hipError_t launch_adjoint_pass(qsim_state, const Plan &, const Pass &, void *, double *, const double *) {
    no_device("adjoint");
}
hipError_t launch_half_angle_trig(qsim_state, const double *, int64_t, double *) { no_device("trig"); }
hipError_t launch_gather_gradient(qsim_state, const double *, const int32_t *, const int32_t *, int64_t, int, double *,
                                  double *) {
    no_device("gather");
}
hipError_t launch_batch(hipStream_t, int, const BatchDevice &, int) { no_device("batch"); }
hipError_t launch_batch_layered(hipStream_t, int, const BatchLayerDevice &) { no_device("batch"); }
hipError_t batch_layer_setup(int, int) { no_device("batch"); }
hipError_t launch_dense_sweep(qsim_state, const Pass &) { no_device("dense"); }
hipError_t launch_diag_sweep(qsim_state, const Pass &) { no_device("diag"); }
hipError_t launch_expect_group(qsim_state, uint64_t, const void *, int, double *, int *) { no_device("expect"); }
hipError_t launch_expect_tiles(qsim_state, const ExpTilePass &, const void *, double *, int *) { no_device("expect"); }
hipError_t launch_expect_simple(qsim_state, const ExpSimplePass &, const void *, double *, int *) { no_device("expect"); }
int expect_simple_grid(uint64_t) { no_device("expect"); }
int expect_group_grid(uint64_t) { no_device("expect"); }
hipError_t launch_mfma_pass(qsim_state, const Plan &, const Pass &) { no_device("mfma"); }
hipError_t launch_pauli_apply(qsim_state, void *, const void *, int, const void *, double *) { no_device("pauli"); }
hipError_t launch_reduce(qsim_state, const double *, int, double *) { no_device("reduce"); }
hipError_t launch_reduce_rows(qsim_state, const double *, int, int, double *) { no_device("reduce"); }
hipError_t launch_set_basis(qsim_state, uint64_t) { no_device("basis"); }
hipError_t launch_fill_zero(qsim_state, void *, size_t) { no_device("fill"); }
hipError_t launch_tile_pass(qsim_state, const Plan &, const Pass &, const double *) { no_device("tile"); }
hipError_t launch_tile_reg_pass(qsim_state, const Plan &, const Pass &) { no_device("tile"); }
int pauli_apply_grid(uint64_t) { no_device("pauli"); }
}  // namespace qsim

using namespace qsim;

int main(int argc, char **argv) {
    FILE *in = std::fopen(argv[1], "rb");
    int32_t hdr[3];
    if (std::fread(hdr, 4, 3, in) != 3) return 2;
    const int n = hdr[0], nops = hdr[1];
    int64_t nmats = 0;
    if (std::fread(&nmats, 8, 1, in) != 1) return 2;
    std::vector<qsim_op> ops(static_cast<size_t>(nops));
    if (std::fread(ops.data(), sizeof(qsim_op), size_t(nops), in) != size_t(nops)) return 2;
    std::vector<double> mats(static_cast<size_t>(2 * nmats + 2));
    if (nmats && std::fread(mats.data(), 16, size_t(nmats), in) != size_t(nmats)) return 2;
    std::fclose(in);
    qsim_circuit c{};
    c.n = n; c.nops = nops; c.ops = ops.data(); c.mats = mats.data(); c.nmats = nmats;
    const int tile_m = std::atoi(argv[2]);
    const int dt = std::atoi(argv[3]);
    const std::string dir = argv[4];
    const int fuse_k = argc > 5 ? std::atoi(argv[5]) : 1;
    qsim_options o{fuse_k, tile_m, 0, 0, 0};
    std::vector<HostGate> gates(static_cast<size_t>(nops));
    for (int i = 0; i < nops; ++i) if (make_gate(&c, i, nullptr, 0, gates[size_t(i)]) != QSIM_OK) return 4;
    Plan plan; plan.n = n; plan.dtype = dt;
    if (!build_plan(plan, gates, resolve_options(&o, n, dt))) return 6;
    for (const Pass &p : plan.passes)
        if (p.kind != PASS_TILE || p.reg_r <= 0) { std::fprintf(stderr, "plan has a pass that is not compiled\n"); return 7; }
    std::vector<int> which; std::vector<double> flops;
    std::string s = jit_source(plan, which, &flops);
    // host build: no address-space qualifier
    const std::string qc = "#define QC __attribute__((address_space(4)))";
    s.replace(s.find(qc), qc.size(), "#define QC");
    FILE *out = std::fopen((dir + "/passes.inc").c_str(), "w"); std::fputs(s.c_str(), out); std::fclose(out);
    out = std::fopen((dir + "/table.inc").c_str(), "w");
    for (size_t k = 0; k < which.size(); ++k) std::fprintf(out, "qsim_tile_jit_%zu,\n", k);
    std::fclose(out);
    out = std::fopen((dir + "/plan.txt").c_str(), "w");
    std::fprintf(out, "%d %d %zu %d\n", n, dt, which.size(), jit_map_shift(plan));
    for (int i : which) {
        const Pass &p = plan.passes[size_t(i)];
        std::fprintf(out, "%llu %d\n", 1ull << (n - p.m), p.pool_begin);
    }
    std::fclose(out);
    out = std::fopen((dir + "/pool.bin").c_str(), "wb");
    for (const cd &v : plan.tile_pool) {
        if (dt == QSIM_C64) { const float w[2] = {float(v.real()), float(v.imag())}; std::fwrite(w, 4, 2, out); }
        else { const double w[2] = {v.real(), v.imag()}; std::fwrite(w, 8, 2, out); }
    }
    std::fclose(out);
    std::printf("%zu passes\n", which.size());
    return 0;
}
