// Host-side planner check, built with AddressSanitizer and UBSan by
// tests/test_host_sanitize.py: every planning path (sweeps, fusion, tiles,
// register programs, split form, compiled-pass source, adjoint tiles) runs on
// the circuits given as files, at both precisions and many options.  Device
// launchers are stubs that abort: planning must never reach them.
#include <cstdio>
#include <cstdlib>
#include <vector>

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

// LDS a tile pass takes when it runs from LDS (not as a register program):
// `tiles` state tiles, its op list and its matrix pool.
static bool lds_fits(const Pass &p, int dtype, int tiles) {
    if (p.kind != PASS_TILE || p.reg_r > 0) return true;
    const size_t amp = amp_bytes(dtype);
    const size_t lds = size_t(tiles) * (amp << p.m) + sizeof(TileOp) * size_t(p.op_end - p.op_begin) +
                       amp * size_t(p.pool_end - p.pool_begin);
    return lds <= size_t(160) * 1024;
}

int main(int argc, char **argv) {
    long plans = 0, passes = 0;
    for (int f = 1; f < argc; ++f) {
        FILE *in = std::fopen(argv[f], "rb");
        if (!in) return 2;
        int32_t hdr[3];
        if (std::fread(hdr, 4, 3, in) != 3) return 2;
        const int n = hdr[0], nops = hdr[1], nparams = hdr[2];
        int64_t nmats = 0;
        if (std::fread(&nmats, 8, 1, in) != 1) return 2;
        std::vector<qsim_op> ops(static_cast<size_t>(nops));
        std::vector<double> mats(size_t(2 * nmats + 2)), params(size_t(nparams + 1));
        if (std::fread(ops.data(), sizeof(qsim_op), ops.size(), in) != ops.size()) return 2;
        if (std::fread(mats.data(), sizeof(double), size_t(2 * nmats), in) != size_t(2 * nmats)) return 2;
        if (std::fread(params.data(), sizeof(double), size_t(nparams), in) != size_t(nparams)) return 2;
        std::fclose(in);
        qsim_circuit c{};
        c.n = n;
        c.nops = nops;
        c.ops = ops.data();
        c.mats = mats.data();
        c.nmats = nmats;
        // the tuning table (read from QSIM_TUNE_CACHE on first use); a loaded
        // entry must be an option set the ABI accepts
        {
            qsim_options tuned{};
            for (int dt : {QSIM_C64, QSIM_C128})
                if (tuned_options(&c, n, dt, &tuned) &&
                    (tuned.fuse_k < 0 || tuned.fuse_k > QSIM_MAX_K || (tuned.tile_m > 0 && tuned.tile_m < 7)))
                    return 10;
        }
        // (fuse_k, tile_m, use_mfma, split_1q): automatic; sweeps; matrix-core
        // blocks; tiles of several sizes, fused or not; complex 2x2 form; LDS tiles
        const qsim_options opts[] = {{0, 0, 0, 0},  {1, -1, 0, 0}, {2, -1, 0, 0}, {3, -1, 0, 0},  {4, -1, 1, 0},
                                     {5, -1, 0, 0}, {6, -1, 1, 0}, {1, 12, 0, 0}, {1, 13, 0, 0},  {2, 12, 0, 0},
                                     {3, 11, 0, 0}, {5, 12, 0, 0}, {2, 0, 0, 0},  {1, 12, 0, -1}, {1, 9, 0, 0},
                                     {5, 9, 0, 0},  {1, 7, 0, 0},  {6, 10, 0, 0}, {6, 7, -1, 0}};
        for (int dt : {QSIM_C64, QSIM_C128}) {
            if (n > (dt == QSIM_C64 ? 35 : 34)) continue;
            for (const qsim_options &o : opts) {
                int64_t counts[QSIM_KCLASS_COUNT_] = {};
                double by = 0, fl = 0;
                const qsim_status st = qsim_plan_summary(n, qsim_dtype(dt), &c, nparams ? params.data() : nullptr,
                                                         nparams, &o, counts, &by, &fl);
                if (st != QSIM_OK) {
                    std::fprintf(stderr, "%s: plan_summary status %d: %s\n", argv[f], int(st), qsim_last_error());
                    return 3;
                }
                ++plans;
                for (int64_t v : counts) passes += v;
                // the register programs written out as kernel source
                std::vector<HostGate> gates(static_cast<size_t>(nops));
                for (int i = 0; i < nops; ++i)
                    if (make_gate(&c, i, nparams ? params.data() : nullptr, nparams, gates[size_t(i)]) != QSIM_OK)
                        return 4;
                Plan plan;
                plan.n = n;
                plan.dtype = dt;
                if (!build_plan(plan, gates, resolve_options(&o, n, dt))) {
                    std::fprintf(stderr, "%s: build_plan failed\n", argv[f]);
                    return 6;
                }
                // every gate handed to the grouping lands in exactly one pass
                long placed = 0;
                for (const Pass &p : plan.passes) placed += p.logical_gates;
                if (placed != plan.items) {
                    std::fprintf(stderr, "%s: options (%d,%d,%d,%d): %ld of %d gates placed\n", argv[f], o.fuse_k,
                                 o.tile_m, o.use_mfma, o.split_1q, placed, plan.items);
                    return 7;
                }
                // an LDS pass's tile, op list and matrices fit the 160 KiB a
                // workgroup may hold
                for (const Pass &p : plan.passes)
                    if (!lds_fits(p, dt, 1)) {
                        std::fprintf(stderr, "%s: options (%d,%d,%d,%d): an LDS pass needs more than 160 KiB\n",
                                     argv[f], o.fuse_k, o.tile_m, o.use_mfma, o.split_1q);
                        return 11;
                    }
                std::vector<int> which;
                std::vector<double> flops;
                const std::string src = jit_source(plan, which, &flops);
                if (!which.empty() && src.empty()) return 5;
            }
            std::vector<HostGate> gates(static_cast<size_t>(nops));
            for (int i = 0; i < nops; ++i)
                if (make_gate(&c, i, nparams ? params.data() : nullptr, nparams, gates[size_t(i)]) != QSIM_OK) return 4;
            Plan adj;
            adj.n = n;
            adj.dtype = dt;
            if (build_adjoint_plan(adj, gates, std::min(n, 10)) < 0) return 8;
            long placed = 0;
            for (const Pass &p : adj.passes) placed += p.logical_gates;
            if (placed != adj.items) {
                std::fprintf(stderr, "%s: adjoint plan placed %ld of %d gates\n", argv[f], placed, adj.items);
                return 9;
            }
            for (const Pass &p : adj.passes)
                if (!lds_fits(p, dt, 2)) {
                    std::fprintf(stderr, "%s: an adjoint pass needs more than 160 KiB of LDS\n", argv[f]);
                    return 12;
                }
            passes += long(adj.passes.size());
        }
    }
    std::printf("planner check: %ld plans, %ld passes\n", plans, passes);
    return 0;
}
