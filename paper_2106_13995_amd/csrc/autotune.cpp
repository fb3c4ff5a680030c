// Autotuner: times candidate execution options for a circuit on a state and
// remembers the fastest per circuit structure.  The table is process-wide; it
// is also appended to the text file named by QSIM_TUNE_CACHE (one line per
// choice: structure hash, n, dtype, fuse_k, tile_m, use_mfma) and read from it
// on first use, so a later process starts from earlier choices.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "qsim_internal.h"

namespace qsim {

namespace {

std::mutex g_mu;
std::map<std::string, qsim_options> g_table;
bool g_loaded = false;

uint64_t fnv1a(const std::string &s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char ch : s) {
        h ^= ch;
        h *= 1099511628211ull;
    }
    return h;
}

// Structure key: width, dtype, ops with their parameter indices (angles of
// parametric ops are not part of the structure) and matrices.
std::string structure_key(const qsim_circuit *c, int n, int dtype) {
    std::string k;
    auto put = [&k](const void *p, size_t m) { k.append(static_cast<const char *>(p), m); };
    put(&n, sizeof n);
    put(&dtype, sizeof dtype);
    for (int i = 0; i < c->nops; ++i) {
        qsim_op op = c->ops[i];
        if (op.param >= 0) op.angles[0] = op.angles[1] = op.angles[2] = 0.0;
        put(&op, sizeof op);
    }
    if (c->mats && c->nmats > 0) put(c->mats, sizeof(double) * 2 * size_t(c->nmats));
    return k;
}

std::string file_key(uint64_t h) { return "#" + std::to_string(h); }

void load_file_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const char *path = std::getenv("QSIM_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    unsigned long long h;
    int n, dt, fk, tm, mf;
    while (std::fscanf(f, "%llx %d %d %d %d %d", &h, &n, &dt, &fk, &tm, &mf) == 6) {
        // the file is outside the library's control: keep only option sets
        // the ABI would accept from a caller
        const bool ok = (dt == QSIM_C64 || dt == QSIM_C128) && n >= 1 && n <= 35 && fk >= 0 && fk <= QSIM_MAX_K &&
                        (tm == -1 || tm == 0 || (tm >= 7 && tm <= 13)) && mf >= -1 && mf <= 1;
        if (!ok) continue;
        qsim_options o{};
        o.fuse_k = fk;
        o.tile_m = tm;
        o.use_mfma = mf;
        g_table[file_key(h)] = o;
    }
    std::fclose(f);
}

}  // namespace

bool tuned_options(const qsim_circuit *c, int n, int dtype, qsim_options *out) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_file_locked();
    if (g_table.empty()) return false;
    const std::string key = structure_key(c, n, dtype);
    auto it = g_table.find(key);
    if (it == g_table.end()) it = g_table.find(file_key(fnv1a(key)));
    if (it == g_table.end()) return false;
    *out = it->second;
    return true;
}

void remember_tuning(const qsim_circuit *c, int n, int dtype, const qsim_options &o) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_file_locked();
    const std::string key = structure_key(c, n, dtype);
    g_table[key] = o;
    if (const char *path = std::getenv("QSIM_TUNE_CACHE")) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "%llx %d %d %d %d %d\n", (unsigned long long)fnv1a(key), n, dtype, o.fuse_k, o.tile_m,
                         o.use_mfma);
            std::fclose(f);
        }
    }
}

}  // namespace qsim
