// C ABI of the qsim library: argument validation, state lifetime, plan cache
// and dispatch of passes to the HIP kernels.
#include <algorithm>
#include <mutex>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>

#include "batch.h"
#include "qsim_internal.h"

namespace qsim {

static thread_local std::string g_last_error;

qsim_status set_error(qsim_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

void clear_error() { g_last_error.clear(); }

static qsim_status device_error(qsim_state s, hipError_t e, const char *what) {
    if (s) s->valid = false;
    return set_error(QSIM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define QSIM_HIP(s, call, what)                                   \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return device_error((s), e_, what); \
    } while (0)

// Failure injection for tests of the error paths: with QSIM_FAULT=launch
// every launch point fails as a failed kernel launch would (the call returns
// QSIM_ERR_DEVICE and the state becomes invalid); with QSIM_FAULT=launch:N
// only the N-th launch point reached since the variable took its value.
// Nothing is launched at an injected failure.
static std::mutex g_fault_mu;
static std::string g_fault_spec;
static long g_launch_points = 0;

static hipError_t injected_fault() {
    const char *v = std::getenv("QSIM_FAULT");
    if (!v || std::strncmp(v, "launch", 6) != 0) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_fault_mu);
    if (g_fault_spec != v) {
        g_fault_spec = v;
        g_launch_points = 0;
    }
    const long k = ++g_launch_points;
    if (v[6] == ':') return std::atol(v + 7) == k ? hipErrorLaunchFailure : hipSuccess;
    return v[6] == 0 ? hipErrorLaunchFailure : hipSuccess;
}

static qsim_status check_state(qsim_state s) {
    if (!s) return set_error(QSIM_ERR_ARG, "state handle is NULL");
    if (!s->valid) return set_error(QSIM_ERR_STATE, "state is invalid after an earlier device error");
    clear_error();
    return QSIM_OK;
}

static int max_qubits(int dtype) { return dtype == QSIM_C128 ? QSIM_MAX_QUBITS_C128 : QSIM_MAX_QUBITS_C64; }

static bool valid_dtype(int dtype) { return dtype == QSIM_C64 || dtype == QSIM_C128; }

// ------------------------------------------------------------ profiling

void prof_begin(qsim_state s, int cls, double bytes, double flops) {
    if (!s->prof.on) return;
    Profile::Rec r;
    r.cls = cls;
    r.bytes = bytes;
    r.flops = flops;
    for (hipEvent_t *e : {&r.a, &r.b}) {
        if (!s->prof.pool.empty()) {
            *e = s->prof.pool.back();
            s->prof.pool.pop_back();
        } else if (hipEventCreate(e) != hipSuccess) {
            *e = nullptr;
        }
    }
    if (r.a) (void)hipEventRecord(r.a, s->stream);
    s->prof.recs.push_back(r);
}

void prof_end(qsim_state s) {
    if (!s->prof.on || s->prof.recs.empty()) return;
    Profile::Rec &r = s->prof.recs.back();
    if (r.b) (void)hipEventRecord(r.b, s->stream);
}

static void prof_clear(qsim_state s) {
    for (auto &r : s->prof.recs) {
        if (r.a) s->prof.pool.push_back(r.a);
        if (r.b) s->prof.pool.push_back(r.b);
    }
    s->prof.recs.clear();
}

// ------------------------------------------------------------ device buffers

static qsim_status ensure_scratch(qsim_state s, size_t bytes) {
    if (s->scratch_bytes >= bytes) return QSIM_OK;
    QSIM_HIP(s, hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    if (s->scratch) (void)hipFree(s->scratch);
    s->scratch = nullptr;
    s->scratch_bytes = 0;
    const size_t cap = std::max<size_t>(bytes, 1 << 20);
    if (hipMalloc(&s->scratch, cap) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(QSIM_ERR_OOM, "cannot allocate scratch memory");
    }
    s->scratch_bytes = cap;
    return QSIM_OK;
}

// Host staging buffer (pinned) for stream-ordered uploads.  Waits for the
// previous upload from it to finish before handing it out again.
static qsim_status ensure_pinned(qsim_state s, size_t bytes) {
    if (s->pinned_ev_pending) {
        QSIM_HIP(s, hipEventSynchronize(s->pinned_ev), "hipEventSynchronize");
        s->pinned_ev_pending = false;
    }
    if (s->pinned_bytes >= bytes) return QSIM_OK;
    if (s->pinned) (void)hipHostFree(s->pinned);
    s->pinned = nullptr;
    s->pinned_bytes = 0;
    const size_t cap = std::max<size_t>(bytes, 1 << 16);
    if (hipHostMalloc(&s->pinned, cap, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(QSIM_ERR_OOM, "cannot allocate pinned host memory");
    }
    s->pinned_bytes = cap;
    return QSIM_OK;
}

static qsim_status upload_staged(qsim_state s, void *dst, size_t bytes) {
    QSIM_HIP(s, hipMemcpyAsync(dst, s->pinned, bytes, hipMemcpyHostToDevice, s->stream), "hipMemcpyAsync");
    if (!s->pinned_ev) QSIM_HIP(s, hipEventCreateWithFlags(&s->pinned_ev, hipEventDisableTiming), "hipEventCreate");
    QSIM_HIP(s, hipEventRecord(s->pinned_ev, s->stream), "hipEventRecord");
    s->pinned_ev_pending = true;
    return QSIM_OK;
}

// ------------------------------------------------------------ plans

template <typename T>
static void pack_pool(const std::vector<cd> &pool, void *dst) {
    T *p = static_cast<T *>(dst);
    for (size_t i = 0; i < pool.size(); ++i) {
        p[2 * i] = T(pool[i].real());
        p[2 * i + 1] = T(pool[i].imag());
    }
}

static qsim_status upload_plan(qsim_state s, Plan &plan) {
    if (plan.uploaded) return QSIM_OK;
    auto align = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t ops_bytes = plan.tile_ops.size() * sizeof(TileOp);
    plan.reg_stages_dev_off = align(ops_bytes);
    const size_t st_bytes = plan.reg_stages.size() * sizeof(RegStage);
    plan.reg_ops_dev_off = align(plan.reg_stages_dev_off + st_bytes);
    const size_t rop_bytes = plan.reg_ops.size() * sizeof(RegOp);
    plan.pool_dev_off = align(plan.reg_ops_dev_off + rop_bytes);
    plan.real_pool_dev_off = align(plan.pool_dev_off + plan.tile_pool.size() * amp_bytes(plan.dtype));
    const size_t real_bytes = plan.real_pool.size() * amp_bytes(plan.dtype) / 2;
    const size_t total = plan.real_pool_dev_off + real_bytes;
    if (ops_bytes == 0 && st_bytes == 0 && rop_bytes == 0 && plan.tile_pool.empty() && plan.real_pool.empty()) {
        plan.uploaded = true;
        return QSIM_OK;
    }
    if (hipMallocAsync(&plan.dev, total, s->stream) != hipSuccess) {
        (void)hipGetLastError();
        plan.dev = nullptr;
        return set_error(QSIM_ERR_OOM, "cannot allocate device memory for the plan");
    }
    plan.dev_stream = s->stream;
    // staged through the state's pinned buffer, copied in stream order
    qsim_status st = ensure_pinned(s, total);
    if (st != QSIM_OK) return st;
    char *h = static_cast<char *>(s->pinned);
    if (ops_bytes) std::memcpy(h, plan.tile_ops.data(), ops_bytes);
    if (st_bytes) std::memcpy(h + plan.reg_stages_dev_off, plan.reg_stages.data(), st_bytes);
    if (rop_bytes) std::memcpy(h + plan.reg_ops_dev_off, plan.reg_ops.data(), rop_bytes);
    if (plan.dtype == QSIM_C64) {
        pack_pool<float>(plan.tile_pool, h + plan.pool_dev_off);
        float *r = reinterpret_cast<float *>(h + plan.real_pool_dev_off);
        for (size_t i = 0; i < plan.real_pool.size(); ++i) r[i] = float(plan.real_pool[i]);
    } else {
        pack_pool<double>(plan.tile_pool, h + plan.pool_dev_off);
        if (!plan.real_pool.empty())
            std::memcpy(h + plan.real_pool_dev_off, plan.real_pool.data(), sizeof(double) * plan.real_pool.size());
    }
    st = upload_staged(s, plan.dev, total);
    if (st != QSIM_OK) return st;
    plan.dev_bytes = total;
    plan.uploaded = true;
    return QSIM_OK;
}

static qsim_status run_plan(qsim_state s, Plan &plan) {
    QSIM_HIP(s, injected_fault(), "injected fault (QSIM_FAULT)");
    qsim_status st = upload_plan(s, plan);
    if (st != QSIM_OK) return st;
    // occupancy maps of the compiled passes (sparse states), in the state's
    // scratch; zeroed before each chain of compiled passes
    void *maps = nullptr;
    size_t map_bytes = 0;
    if (plan.jit_map_shift > 0 && !plan.jit_fn.empty()) {
        map_bytes = size_t(3) << (s->n - plan.jit_map_shift);
        st = ensure_scratch(s, map_bytes);
        if (st != QSIM_OK) return st;
        maps = s->scratch;
    }
    for (size_t i = 0; i < plan.passes.size(); ++i) {
        const Pass &p = plan.passes[i];
        hipError_t e = hipSuccess;
        const bool jit = p.kind == PASS_TILE && p.reg_r > 0 && i < plan.jit_fn.size() && plan.jit_fn[i];
        if (jit && maps && (i == 0 || !plan.jit_fn[i - 1]))
            QSIM_HIP(s, launch_fill_zero(s, maps, map_bytes), "map clear launch");
        switch (p.kind) {
            case PASS_DENSE:
                prof_begin(s, QSIM_KCLASS_SWEEP_DENSE, p.bytes, p.flops);
                e = launch_dense_sweep(s, p);
                break;
            case PASS_DIAG:
                prof_begin(s, QSIM_KCLASS_SWEEP_DIAG, p.bytes, p.flops);
                e = launch_diag_sweep(s, p);
                break;
            case PASS_TILE:
                if (jit) {
                    prof_begin(s, QSIM_KCLASS_TILE_JIT, p.bytes, p.flops);
                    e = launch_jit_pass(s, plan, p, plan.jit_fn[i], maps);
                } else {
                    prof_begin(s, QSIM_KCLASS_TILE, p.bytes, p.flops);
                    e = p.reg_r > 0 ? launch_tile_reg_pass(s, plan, p) : launch_tile_pass(s, plan, p);
                }
                break;
            case PASS_MFMA:
                prof_begin(s, QSIM_KCLASS_MFMA, p.bytes, p.flops);
                e = launch_mfma_pass(s, plan, p);
                break;
            default:
                return set_error(QSIM_ERR_UNSUPPORTED, "pass kind not supported");
        }
        prof_end(s);
        if (e != hipSuccess) return device_error(s, e, "kernel launch");
    }
    return QSIM_OK;
}

// Validates one op and returns its normalised gate.
qsim_status make_gate(const qsim_circuit *c, int i, const double *params, int64_t nparams, HostGate &g) {
    const qsim_op &op = c->ops[i];
    const int n = c->n;
    char buf[160];
    int k = op.k;
    if (op.kind == QSIM_GATE_MATRIX) {
        if (k < 1 || k > QSIM_MAX_K) {
            snprintf(buf, sizeof buf, "op %d: matrix gate with k=%d outside [1, %d]", i, k, QSIM_MAX_K);
            return set_error(QSIM_ERR_ARG, buf);
        }
    } else {
        const int ar = named_gate_arity(op.kind);
        if (ar < 0) {
            snprintf(buf, sizeof buf, "op %d: unknown gate kind %d", i, op.kind);
            return set_error(QSIM_ERR_ARG, buf);
        }
        if (k != ar) {
            snprintf(buf, sizeof buf, "op %d: gate kind %d acts on %d qubits, op says k=%d", i, op.kind, ar, k);
            return set_error(QSIM_ERR_ARG, buf);
        }
    }
    if (k > n) {
        snprintf(buf, sizeof buf, "op %d: k=%d exceeds the %d-qubit register", i, k, n);
        return set_error(QSIM_ERR_ARG, buf);
    }
    uint64_t seen = 0;
    for (int b = 0; b < k; ++b) {
        const int t = op.targets[b];
        if (t < 0 || t >= n) {
            snprintf(buf, sizeof buf, "op %d: target %d outside [0, %d)", i, t, n);
            return set_error(QSIM_ERR_ARG, buf);
        }
        if (seen & (1ull << t)) {
            snprintf(buf, sizeof buf, "op %d: target %d repeated", i, t);
            return set_error(QSIM_ERR_ARG, buf);
        }
        seen |= 1ull << t;
        g.targets[b] = t;
    }
    g.k = k;
    g.src_op = i;
    const int d = 1 << k;
    g.M.resize(size_t(d) * d);
    if (op.kind == QSIM_GATE_MATRIX) {
        if (!c->mats || op.mat_off < 0 || op.mat_off + int64_t(d) * d > c->nmats) {
            snprintf(buf, sizeof buf, "op %d: matrix at offset %lld does not fit the %lld-entry pool", i,
                     (long long)op.mat_off, (long long)c->nmats);
            return set_error(QSIM_ERR_ARG, buf);
        }
        const double *m = c->mats + 2 * op.mat_off;
        for (int e = 0; e < d * d; ++e) g.M[e] = cd(m[2 * e], m[2 * e + 1]);
        return QSIM_OK;
    }
    double ang[3] = {op.angles[0], op.angles[1], op.angles[2]};
    if (op.param >= 0) {
        const int na = op.kind == QSIM_GATE_U3 ? 3
                       : (op.kind == QSIM_GATE_RX || op.kind == QSIM_GATE_RY || op.kind == QSIM_GATE_RZ ||
                          op.kind == QSIM_GATE_CP)
                           ? 1
                           : 0;
        if (na == 0) {
            snprintf(buf, sizeof buf, "op %d: gate kind %d takes no parameter", i, op.kind);
            return set_error(QSIM_ERR_ARG, buf);
        }
        if (!params || int64_t(op.param) + na > nparams) {
            snprintf(buf, sizeof buf, "op %d: parameter index %d outside the %lld supplied", i, op.param,
                     (long long)nparams);
            return set_error(QSIM_ERR_ARG, buf);
        }
        for (int a = 0; a < na; ++a) ang[a] = params[op.param + a];
    }
    named_gate_matrix(op.kind, ang, g.M.data());
    return QSIM_OK;
}

// Exact cache key: options, width, dtype, ops, referenced matrices and parameters.
static std::string plan_key(qsim_state s, const qsim_circuit *c, const double *params, int64_t nparams,
                            const PlanOptions &po) {
    std::string key;
    auto put = [&key](const void *p, size_t n) { key.append(static_cast<const char *>(p), n); };
    put(&po, sizeof po);
    put(&s->n, sizeof s->n);
    put(&s->dtype, sizeof s->dtype);
    put(c->ops, sizeof(qsim_op) * size_t(c->nops));
    if (c->mats && c->nmats > 0) put(c->mats, sizeof(double) * 2 * size_t(c->nmats));
    if (params && nparams > 0) put(params, sizeof(double) * size_t(nparams));
    return key;
}

static const size_t kMaxCachedPlans = 16;

static qsim_status get_plan(qsim_state s, const qsim_circuit *c, const double *params, int64_t nparams,
                            const qsim_options *opts, Plan **out, bool cache = true) {
    qsim_options tuned{};
    const bool automatic =
        !opts || (opts->fuse_k == 0 && opts->tile_m == 0 && opts->use_mfma == 0 && opts->split_1q == 0);
    const bool deterministic = opts && opts->deterministic;
    if (automatic && !deterministic && tuned_options(c, s->n, s->dtype, &tuned)) opts = &tuned;
    const PlanOptions po = resolve_options(opts, s->n, s->dtype);
    std::string key;
    if (cache) {
        key = plan_key(s, c, params, nparams, po);
        for (auto &cp : s->plans)
            if (cp.key == key) {
                cp.last_use = ++s->use_clock;
                *out = cp.plan.get();
                return QSIM_OK;
            }
    }
    std::vector<HostGate> gates(size_t(c->nops));
    for (int i = 0; i < c->nops; ++i) {
        qsim_status st = make_gate(c, i, params, nparams, gates[size_t(i)]);
        if (st != QSIM_OK) return st;
    }
    std::unique_ptr<Plan> plan(new (std::nothrow) Plan());
    if (!plan) return set_error(QSIM_ERR_OOM, "host allocation failed");
    plan->n = s->n;
    plan->dtype = s->dtype;
    if (!build_plan(*plan, gates, po)) return set_error(QSIM_ERR_UNSUPPORTED, "the planner could not place every op");
    // compiled tiles for fixed circuits only: the split form's structure
    // depends on the gate values, so a parameter sweep would recompile
    bool parametric = false;
    for (int i = 0; i < c->nops; ++i) parametric = parametric || c->ops[i].param >= 0;
    if (cache && !parametric && jit_wanted(s->n)) {
        std::string err;
        if (jit_prepare(s, *plan, err) != QSIM_OK) {
            plan->jit_fn.clear();
            if (jit_mode() == 1) return set_error(QSIM_ERR_DEVICE, err);
        }
    }
    if (!cache) {
        // one transient plan per state; the one it replaces releases its
        // device buffer in stream order, after the kernels that read it
        s->transient = std::move(plan);
        *out = s->transient.get();
        return QSIM_OK;
    }
    if (s->plans.size() >= kMaxCachedPlans) {
        auto lru = std::min_element(s->plans.begin(), s->plans.end(),
                                    [](const CachedPlan &a, const CachedPlan &b) { return a.last_use < b.last_use; });
        s->plans.erase(lru);   // released in stream order
    }
    CachedPlan cp;
    cp.key = std::move(key);
    cp.plan = std::move(plan);
    cp.last_use = ++s->use_clock;
    s->plans.push_back(std::move(cp));
    *out = s->plans.back().plan.get();
    return QSIM_OK;
}

}  // namespace qsim

using namespace qsim;

extern "C" {

const char *qsim_last_error(void) { return g_last_error.c_str(); }

qsim_status qsim_wrap(void *dev_ptr, int n, qsim_dtype dtype, void *hip_stream, qsim_state *out) {
    clear_error();
    if (!out) return set_error(QSIM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!valid_dtype(dtype)) return set_error(QSIM_ERR_ARG, "dtype must be QSIM_C64 or QSIM_C128");
    if (n < 1 || n > max_qubits(dtype)) return set_error(QSIM_ERR_ARG, "n outside the supported range");
    if (!dev_ptr) return set_error(QSIM_ERR_ARG, "device pointer is NULL");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0)
        return set_error(QSIM_ERR_ARG, "device pointer must be 256-byte aligned");
    qsim_state s = new (std::nothrow) qsim_state_s();
    if (!s) return set_error(QSIM_ERR_OOM, "host allocation failed");
    s->n = n;
    s->dtype = dtype;
    s->data = dev_ptr;
    s->owned = false;
    s->stream = static_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&s->device);
    *out = s;
    return QSIM_OK;
}

qsim_status qsim_alloc(int n, qsim_dtype dtype, qsim_state *out) {
    clear_error();
    if (!out) return set_error(QSIM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!valid_dtype(dtype)) return set_error(QSIM_ERR_ARG, "dtype must be QSIM_C64 or QSIM_C128");
    if (n < 1 || n > max_qubits(dtype)) return set_error(QSIM_ERR_ARG, "n outside the supported range");
    void *p = nullptr;
    const size_t bytes = amp_bytes(dtype) << n;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(QSIM_ERR_OOM, "cannot allocate " + std::to_string(bytes) + " bytes of device memory");
    }
    qsim_state s = new (std::nothrow) qsim_state_s();
    if (!s) {
        (void)hipFree(p);
        return set_error(QSIM_ERR_OOM, "host allocation failed");
    }
    s->n = n;
    s->dtype = dtype;
    s->data = p;
    s->owned = true;
    (void)hipGetDevice(&s->device);
    hipError_t e = launch_set_basis(s, 0);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        (void)hipFree(p);
        delete s;
        return set_error(QSIM_ERR_DEVICE, std::string("initialising the state: ") + hipGetErrorString(e));
    }
    *out = s;
    return QSIM_OK;
}

qsim_status qsim_free(qsim_state s) {
    clear_error();
    if (!s) return QSIM_OK;
    (void)hipStreamSynchronize(s->stream);
    s->plans.clear();
    s->adj_plans.clear();
    s->adj_lplans.clear();
    s->transient.reset();
    if (s->adj_h) (void)hipFree(s->adj_h);
    if (s->adj_lam) (void)hipFree(s->adj_lam);
    if (s->adj_ck) (void)hipFree(s->adj_ck);
    prof_clear(s);
    for (hipEvent_t e : s->prof.pool) (void)hipEventDestroy(e);
    if (s->pinned_ev) (void)hipEventDestroy(s->pinned_ev);
    if (s->scratch) (void)hipFree(s->scratch);
    if (s->pinned) (void)hipHostFree(s->pinned);
    if (s->owned && s->data) (void)hipFree(s->data);
    delete s;
    return QSIM_OK;
}

qsim_status qsim_set_stream(qsim_state s, void *hip_stream) {
    qsim_status st = check_state(s);
    if (st != QSIM_OK) return st;
    // order the new stream after everything queued so far on the old one;
    // plans now release their buffers on the new stream
    QSIM_HIP(s, hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    s->stream = static_cast<hipStream_t>(hip_stream);
    for (auto &cp : s->plans) cp.plan->dev_stream = s->stream;
    for (auto &ap : s->adj_plans) {
        ap->fwd.dev_stream = ap->rev.dev_stream = s->stream;
        ap->dev_stream = s->stream;
    }
    for (auto &lp : s->adj_lplans) lp->dev_stream = s->stream;
    if (s->transient) s->transient->dev_stream = s->stream;
    return QSIM_OK;
}

qsim_status qsim_state_info(qsim_state s, int *n, int *dtype, void **dev_ptr) {
    if (!s) return set_error(QSIM_ERR_ARG, "state handle is NULL");
    clear_error();
    if (n) *n = s->n;
    if (dtype) *dtype = s->dtype;
    if (dev_ptr) *dev_ptr = s->data;
    return QSIM_OK;
}

qsim_status qsim_set_basis(qsim_state s, uint64_t index) {
    qsim_status st = check_state(s);
    if (st != QSIM_OK) return st;
    if (index >= (1ull << s->n)) return set_error(QSIM_ERR_ARG, "basis index outside [0, 2^n)");
    QSIM_HIP(s, injected_fault(), "injected fault (QSIM_FAULT)");
    QSIM_HIP(s, launch_set_basis(s, index), "set_basis launch");
    return QSIM_OK;
}

qsim_status qsim_copy_to_host(qsim_state s, void *host, size_t bytes) {
    qsim_status st = check_state(s);
    if (st != QSIM_OK) return st;
    if (!host) return set_error(QSIM_ERR_ARG, "host pointer is NULL");
    if (bytes != (amp_bytes(s->dtype) << s->n)) return set_error(QSIM_ERR_ARG, "byte count does not match the state");
    QSIM_HIP(s, hipMemcpyAsync(host, s->data, bytes, hipMemcpyDeviceToHost, s->stream), "hipMemcpyAsync");
    QSIM_HIP(s, hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    return QSIM_OK;
}

qsim_status qsim_copy_from_host(qsim_state s, const void *host, size_t bytes) {
    qsim_status st = check_state(s);
    if (st != QSIM_OK) return st;
    if (!host) return set_error(QSIM_ERR_ARG, "host pointer is NULL");
    if (bytes != (amp_bytes(s->dtype) << s->n)) return set_error(QSIM_ERR_ARG, "byte count does not match the state");
    QSIM_HIP(s, hipMemcpyAsync(s->data, host, bytes, hipMemcpyHostToDevice, s->stream), "hipMemcpyAsync");
    QSIM_HIP(s, hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    return QSIM_OK;
}

qsim_status qsim_apply_gate(qsim_state s, const int *targets, int k, const double *U) {
    qsim_status st = check_state(s);
    if (st != QSIM_OK) return st;
    if (!targets || !U) return set_error(QSIM_ERR_ARG, "targets or U is NULL");
    if (k < 1 || k > QSIM_MAX_K) return set_error(QSIM_ERR_ARG, "k outside [1, 6]");
    qsim_op op{};
    op.kind = QSIM_GATE_MATRIX;
    op.k = k;
    for (int b = 0; b < k; ++b) op.targets[b] = targets[b];
    op.param = -1;
    op.mat_off = 0;
    qsim_circuit c{};
    c.n = s->n;
    c.nops = 1;
    c.ops = &op;
    c.mats = U;
    c.nmats = int64_t(1) << (2 * k);
    HostGate g;
    st = make_gate(&c, 0, nullptr, 0, g);
    if (st != QSIM_OK) return st;
    qsim_options o{};
    o.fuse_k = 1;
    o.tile_m = -1;
    Plan *plan = nullptr;
    st = get_plan(s, &c, nullptr, 0, &o, &plan, /*cache=*/false);
    if (st != QSIM_OK) return st;
    return run_plan(s, *plan);
}

static qsim_status check_options(const qsim_options *opts) {
    if (!opts) return QSIM_OK;
    if (opts->fuse_k < 0 || opts->fuse_k > QSIM_MAX_K) return set_error(QSIM_ERR_ARG, "fuse_k outside [0, 6]");
    if (opts->tile_m > 0 && opts->tile_m < 7) return set_error(QSIM_ERR_ARG, "tile_m must be -1, 0 or at least 7");
    if (opts->split_1q < -1 || opts->split_1q > 1) return set_error(QSIM_ERR_ARG, "split_1q outside [-1, 1]");
    if (opts->use_mfma < -1 || opts->use_mfma > 1) return set_error(QSIM_ERR_ARG, "use_mfma outside [-1, 1]");
    if (opts->deterministic < 0 || opts->deterministic > 1)
        return set_error(QSIM_ERR_ARG, "deterministic must be 0 or 1");
    if (opts->checkpoints < 0 || opts->checkpoints > 64) return set_error(QSIM_ERR_ARG, "checkpoints outside [0, 64]");
    return QSIM_OK;
}

qsim_status qsim_apply_circuit(qsim_state s, const qsim_circuit *c, const double *params, int64_t nparams,
                               const qsim_options *opts) {
    qsim_status st = check_state(s);
    if (st != QSIM_OK) return st;
    if (!c) return set_error(QSIM_ERR_ARG, "circuit is NULL");
    if (c->n != s->n) return set_error(QSIM_ERR_ARG, "circuit width does not match the state");
    if (c->nops < 0 || (c->nops > 0 && !c->ops)) return set_error(QSIM_ERR_ARG, "bad op array");
    if (nparams < 0) return set_error(QSIM_ERR_ARG, "nparams is negative");
    st = check_options(opts);
    if (st != QSIM_OK) return st;
    if (c->nops == 0) return QSIM_OK;
    Plan *plan = nullptr;
    st = get_plan(s, c, params, nparams, opts, &plan);
    if (st != QSIM_OK) return st;
    return run_plan(s, *plan);
}

}  // extern "C"

namespace qsim {

// <psi|H|psi> into *out_host.  Device scratch: the state's own (grown on
// demand, host staging pinned) when fixed_dev is NULL, else the caller's
// fixed_bytes at fixed_dev (nothing allocated; terms copied from host
// memory; sums that need more than fixed_bytes are rejected).
//
// Terms are grouped by X mask.  When every group is the diagonal one or a
// single-qubit X_h / Y_h group, the sum runs as register passes without LDS
// (launch_expect_simple); otherwise groups whose X mask fits a tile share LDS
// tile passes and the rest take one pass each.
qsim_status expectation_with(qsim_state s, const qsim_pauli_sum *H, double *out_host, void *fixed_dev,
                             size_t fixed_bytes) {
    qsim_status st = check_state(s);
    if (st != QSIM_OK) return st;
    if (!H || !out_host || (H->nterms > 0 && !H->terms)) return set_error(QSIM_ERR_ARG, "NULL argument");
    if (H->nterms < 0) return set_error(QSIM_ERR_ARG, "negative term count");
    const uint64_t lim = (s->n >= 64) ? ~0ull : ((1ull << s->n) - 1);
    for (int t = 0; t < H->nterms; ++t)
        if ((H->terms[t].xmask & ~lim) || (H->terms[t].zmask & ~lim))
            return set_error(QSIM_ERR_ARG, "Pauli mask has a bit at or above n");
    // group terms by X mask
    std::map<uint64_t, std::vector<int>> groups;
    for (int t = 0; t < H->nterms; ++t) groups[H->terms[t].xmask].push_back(t);
    struct DevTerm {
        double wr, wi;
        uint64_t z, pad;
    };
    std::vector<DevTerm> ht(size_t(std::max(H->nterms, 1)));
    std::vector<std::pair<uint64_t, int>> spans;   // (x, first term slot)
    int slot = 0;
    for (auto &kv : groups) {
        spans.push_back({kv.first, slot});
        for (int t : kv.second) {
            const qsim_pauli_term &pt = H->terms[t];
            const int ny = __builtin_popcountll(pt.xmask & pt.zmask) & 3;
            // coeff * i^ny
            const double re[4] = {1, 0, -1, 0}, im[4] = {0, 1, 0, -1};
            ht[size_t(slot)].wr = pt.coeff * re[ny];
            ht[size_t(slot)].wi = pt.coeff * im[ny];
            ht[size_t(slot)].z = pt.zmask;
            ht[size_t(slot)].pad = 0;
            ++slot;
        }
    }
    auto group_terms = [&](size_t gi) {
        return (gi + 1 < spans.size() ? spans[gi + 1].second : slot) - spans[gi].second;
    };
    const uint64_t N = 1ull << s->n;
    const bool c64 = s->dtype == QSIM_C64;

    // ---- register passes for diagonal + single-qubit X / Y groups
    std::vector<ExpSimplePass> spasses;
    {
        const int R = kExpSimpleR, L = c64 ? 5 : 4, F = 6 - L;
        bool ok = s->n >= 6 + R && !spans.empty();
        int diag_gi = -1;
        std::vector<size_t> hi, lo;   // single-qubit groups above / within the low L qubits
        std::vector<double> A(spans.size(), 0.0), B(spans.size(), 0.0);
        for (size_t gi = 0; gi < spans.size() && ok; ++gi) {
            const uint64_t x = spans[gi].first;
            if (x == 0) {
                diag_gi = int(gi);
                continue;
            }
            if (__builtin_popcountll(x) != 1) {
                ok = false;
                break;
            }
            for (int t = spans[gi].second; t < spans[gi].second + group_terms(gi); ++t) {
                if (ht[size_t(t)].z == 0)
                    A[gi] += ht[size_t(t)].wr;
                else if (ht[size_t(t)].z == x)
                    B[gi] += ht[size_t(t)].wi;
                else
                    ok = false;
            }
            (x >> L ? hi : lo).push_back(gi);
        }
        if (ok) {
            const size_t per = size_t(F + R);
            const size_t np = std::max<size_t>(1, (hi.size() + per - 1) / per);
            for (size_t pi = 0; pi < np; ++pi) {
                ExpSimplePass sp{};
                sp.R = R;
                uint64_t used = (1ull << L) - 1;
                for (int b = 0; b < L; ++b) sp.lane_q[b] = b;
                std::vector<size_t> mine;
                for (size_t j = pi * per; j < std::min(hi.size(), (pi + 1) * per); ++j) mine.push_back(hi[j]);
                // the first F on free lane bits, the rest on register bits
                int nl = L, nr = 0;
                for (size_t j = 0; j < mine.size(); ++j) {
                    const size_t gi = mine[j];
                    const int h = __builtin_ctzll(spans[gi].first);
                    used |= 1ull << h;
                    if (nl < 6) {
                        sp.lane_bit[sp.nlane_g] = nl;
                        sp.lane_A[sp.nlane_g] = A[gi];
                        sp.lane_B[sp.nlane_g] = B[gi];
                        ++sp.nlane_g;
                        sp.lane_q[nl++] = h;
                    } else {
                        sp.reg_bit[sp.nreg_g] = nr;
                        sp.reg_A[sp.nreg_g] = A[gi];
                        sp.reg_B[sp.nreg_g] = B[gi];
                        ++sp.nreg_g;
                        sp.reg_q[nr++] = h;
                    }
                }
                // remaining slots: the lowest qubits not used yet
                for (int q = L; q < s->n && (nl < 6 || nr < R); ++q) {
                    if ((used >> q) & 1) continue;
                    used |= 1ull << q;
                    if (nl < 6)
                        sp.lane_q[nl++] = q;
                    else
                        sp.reg_q[nr++] = q;
                }
                sp.ntile_q = 0;
                for (int q = 0; q < s->n; ++q)
                    if ((used >> q) & 1) sp.tile_q[sp.ntile_q++] = q;
                spasses.push_back(sp);
            }
            // groups on the low qubits: spread over the passes, on their lane bit
            for (size_t j = 0; j < lo.size(); ++j) {
                ExpSimplePass &sp = spasses[j % spasses.size()];
                const size_t gi = lo[j];
                sp.lane_bit[sp.nlane_g] = __builtin_ctzll(spans[gi].first);
                sp.lane_A[sp.nlane_g] = A[gi];
                sp.lane_B[sp.nlane_g] = B[gi];
                ++sp.nlane_g;
            }
            if (diag_gi >= 0) {
                // the last pass (the fewest groups): terms ordered by the
                // register part of their Z mask
                ExpSimplePass &sp = spasses.back();
                sp.diag = 1;
                const int first = spans[size_t(diag_gi)].second, cnt = group_terms(size_t(diag_gi));
                // pad = mu | zl << 8: the register part of the Z mask (bit b:
                // register bit b) and its lane part (bit b: lane bit b)
                for (int t = first; t < first + cnt; ++t) {
                    uint32_t mu = 0, zl = 0;
                    for (int b = 0; b < R; ++b)
                        if ((ht[size_t(t)].z >> sp.reg_q[b]) & 1) mu |= 1u << b;
                    for (int b = 0; b < 6; ++b)
                        if ((ht[size_t(t)].z >> sp.lane_q[b]) & 1) zl |= 1u << b;
                    ht[size_t(t)].pad = uint64_t(mu) | (uint64_t(zl) << 8);
                }
                auto key = [](const DevTerm &d) { return ((d.pad & 0xffu) << 8) | (d.pad >> 8); };
                std::stable_sort(ht.begin() + first, ht.begin() + first + cnt,
                                 [&](const DevTerm &a, const DevTerm &b) { return key(a) < key(b); });
                sp.diag_first = first;
                sp.diag_end = first + cnt;
                int t = first;
                for (int mu = 0; mu <= (1 << R); ++mu) {
                    while (t < first + cnt && int(ht[size_t(t)].pad & 0xffu) < mu) ++t;
                    sp.diag_mu[mu] = t;
                }
            }
        }
    }

    // ---- otherwise LDS tile passes (groups whose X mask fits a tile: the low
    // L qubits and m - L others) and one pass per remaining group
    const int mt = std::min(s->n, c64 ? 12 : 11);
    const int Lt = std::min(mt, c64 ? 5 : 4);
    const int kpt_bits = c64 ? 4 : 3;
    std::vector<ExpTilePass> tpasses;
    std::vector<size_t> single;            // groups evaluated alone
    if (spasses.empty()) {
        // passes from the groups with X bits above the low L qubits (greedy,
        // in X-mask order); the groups inside the low L qubits (the diagonal
        // group among them) then go to the passes with the least work
        std::vector<uint64_t> tmask;
        std::vector<std::vector<size_t>> members;
        std::vector<size_t> low_only;
        uint64_t hm = 0;
        for (size_t gi = 0; gi < spans.size(); ++gi) {
            const uint64_t hx = spans[gi].first >> Lt << Lt;
            if (__builtin_popcountll(hx) > mt - Lt) {
                single.push_back(gi);
                continue;
            }
            if (hx == 0) {
                low_only.push_back(gi);
                continue;
            }
            if (members.empty() || __builtin_popcountll(hm | hx) > mt - Lt ||
                members.back().size() == size_t(kExpTileGroups)) {
                members.emplace_back();
                tmask.push_back(0);
                hm = 0;
            }
            hm |= hx;
            members.back().push_back(gi);
            tmask.back() = hm;
        }
        for (size_t gi : low_only) {
            // work of a pass: its groups' terms, the diagonal group's counted
            // once per KPT amplitudes plus its transform
            size_t best = members.size();
            double best_w = 1e300;
            for (size_t pi = 0; pi < members.size(); ++pi) {
                if (members[pi].size() == size_t(kExpTileGroups)) continue;
                double w = 0.0;
                for (size_t g2 : members[pi]) w += spans[g2].first ? 1.0 : 2.0;
                if (w < best_w) { best_w = w; best = pi; }
            }
            if (best == members.size()) {
                members.emplace_back();
                tmask.push_back(0);
            }
            members[best].push_back(gi);
        }
        for (size_t pi = 0; pi < members.size(); ++pi) {
            ExpTilePass tp{};
            tp.m = mt;
            tp.L = Lt;
            uint64_t hq = tmask[pi];
            for (int q = Lt; q < s->n && __builtin_popcountll(hq) < mt - Lt; ++q) hq |= 1ull << q;
            tmask[pi] = hq | ((1ull << Lt) - 1);
            int local_of[64];
            for (int q = 0; q < Lt; ++q) local_of[q] = q;
            for (int q = Lt; q < s->n; ++q)
                if ((hq >> q) & 1) {
                    local_of[q] = Lt + tp.H;
                    tp.hpos[tp.H++] = q;
                }
            auto to_local = [&](uint64_t v) {
                uint32_t o = 0;
                for (int q = 0; q < s->n; ++q)
                    if (((v & tmask[pi]) >> q) & 1) o |= 1u << local_of[q];
                return o;
            };
            for (int mu = 0; mu <= 32; ++mu) tp.dmu[mu] = 0;
            for (size_t gi : members[pi]) {
                const uint64_t x = spans[gi].first;
                const int first = spans[gi].second;
                const int cnt = group_terms(gi);
                ExpTileGroup &g = tp.groups[tp.ngroups++];
                g.xl = to_local(x);
                g.first = first;
                g.count = cnt;
                g.flags = 0;
                g.A = g.B = 0.0;
                for (int t = first; t < first + cnt; ++t) ht[size_t(t)].pad = to_local(ht[size_t(t)].z);
                if (__builtin_popcountll(x) == 1) {
                    bool simple = true;
                    for (int t = first; t < first + cnt; ++t) {
                        if (ht[size_t(t)].z == 0) g.A += ht[size_t(t)].wr;
                        else if (ht[size_t(t)].z == x) g.B += ht[size_t(t)].wi;
                        else simple = false;
                    }
                    if (simple) g.flags = kExpGroupSimple;
                }
                if (x == 0) {
                    // order the diagonal terms by the register part of their
                    // local Z mask (local bits 8 and up) for the register kernel
                    std::stable_sort(ht.begin() + first, ht.begin() + first + cnt,
                                     [&](const DevTerm &a, const DevTerm &b) { return (a.pad >> 8) < (b.pad >> 8); });
                    const int kpt = 1 << kpt_bits;
                    int t = first;
                    for (int mu = 0; mu <= kpt; ++mu) {
                        while (t < first + cnt && mu < kpt && int(ht[size_t(t)].pad >> 8) < mu) ++t;
                        tp.dmu[mu] = mu == kpt ? first + cnt : t;
                    }
                }
            }
            tpasses.push_back(tp);
        }
    }

    // ---- scratch: [partials][terms][result]
    // partials: one per workgroup of each register pass, groups x workgroups
    // of each tile pass, workgroups of each single-group pass
    size_t npart = 0;
    for (const ExpSimplePass &sp : spasses) npart += size_t(expect_simple_grid(N >> (6 + sp.R)));
    for (const ExpTilePass &tp : tpasses) npart += size_t(tp.ngroups) * size_t(std::min<uint64_t>(N >> tp.m, 2048));
    npart += single.size() * size_t(expect_group_grid(N));
    const size_t terms_off = (npart * sizeof(double) + 255) & ~size_t(255);
    const size_t terms_bytes = sizeof(DevTerm) * ht.size();
    const size_t out_off = (terms_off + terms_bytes + 255) & ~size_t(255);
    char *scr = nullptr;
    if (fixed_dev) {
        if (out_off + 256 > fixed_bytes)
            return set_error(QSIM_ERR_ARG, "the Pauli sum needs " + std::to_string(out_off + 256) +
                                               " bytes of scratch; the fixed buffer holds " +
                                               std::to_string(fixed_bytes));
        scr = static_cast<char *>(fixed_dev);
    } else {
        st = ensure_scratch(s, out_off + 256);
        if (st != QSIM_OK) return st;
        scr = static_cast<char *>(s->scratch);
    }
    double *partials = reinterpret_cast<double *>(scr);
    DevTerm *dterms = reinterpret_cast<DevTerm *>(scr + terms_off);
    double *dout = reinterpret_cast<double *>(scr + out_off);
    if (H->nterms > 0) {
        if (fixed_dev) {
            // from pageable host memory: the copy has read it when the call
            // returns, and the stream is synchronised below in any case
            QSIM_HIP(s, hipMemcpyAsync(dterms, ht.data(), terms_bytes, hipMemcpyHostToDevice, s->stream),
                     "hipMemcpyAsync");
        } else {
            st = ensure_pinned(s, terms_bytes);
            if (st != QSIM_OK) return st;
            std::memcpy(s->pinned, ht.data(), terms_bytes);
            st = upload_staged(s, dterms, terms_bytes);
            if (st != QSIM_OK) return st;
        }
    }
    QSIM_HIP(s, injected_fault(), "injected fault (QSIM_FAULT)");
    size_t total = 0;
    for (const ExpSimplePass &sp : spasses) {
        int wrote = 0;
        prof_begin(s, QSIM_KCLASS_EXPECT, double(amp_bytes(s->dtype) << s->n));
        hipError_t e = launch_expect_simple(s, sp, dterms, partials + total, &wrote);
        prof_end(s);
        if (e != hipSuccess) return device_error(s, e, "expectation launch");
        total += size_t(wrote);
    }
    for (const ExpTilePass &tp : tpasses) {
        int wrote = 0;
        prof_begin(s, QSIM_KCLASS_EXPECT, double(amp_bytes(s->dtype) << s->n));
        hipError_t e = launch_expect_tiles(s, tp, dterms, partials + total, &wrote);
        prof_end(s);
        if (e != hipSuccess) return device_error(s, e, "expectation launch");
        total += size_t(wrote);
    }
    for (size_t gi : single) {
        const int first = spans[gi].second;
        const int cnt = group_terms(gi);
        int wrote = 0;
        const double bytes = double(amp_bytes(s->dtype) << s->n) * (spans[gi].first ? 2.0 : 1.0);
        prof_begin(s, QSIM_KCLASS_EXPECT, bytes);
        hipError_t e = launch_expect_group(s, spans[gi].first, dterms + first, cnt, partials + total, &wrote);
        prof_end(s);
        if (e != hipSuccess) return device_error(s, e, "expectation launch");
        total += size_t(wrote);
    }
    if (total == 0) {
        *out_host = 0.0;
        return QSIM_OK;
    }
    QSIM_HIP(s, launch_reduce(s, partials, int(total), dout), "reduce launch");
    QSIM_HIP(s, hipMemcpyAsync(out_host, dout, sizeof(double), hipMemcpyDeviceToHost, s->stream), "hipMemcpyAsync");
    QSIM_HIP(s, hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    s->pinned_ev_pending = false;
    return QSIM_OK;
}

}  // namespace qsim

extern "C" {

qsim_status qsim_expectation(qsim_state s, const qsim_pauli_sum *H, double *out_host) {
    return expectation_with(s, H, out_host, nullptr, 0);
}

qsim_status qsim_plan_summary(int n, qsim_dtype dtype, const qsim_circuit *c, const double *params,
                              int64_t nparams, const qsim_options *opts, int64_t *counts, double *bytes,
                              double *flops) {
    clear_error();
    if (!valid_dtype(dtype)) return set_error(QSIM_ERR_ARG, "dtype must be QSIM_C64 or QSIM_C128");
    if (n < 1 || n > max_qubits(dtype)) return set_error(QSIM_ERR_ARG, "n outside the supported range");
    if (!c || c->n != n) return set_error(QSIM_ERR_ARG, "circuit is NULL or its width is not n");
    if (c->nops < 0 || (c->nops > 0 && !c->ops)) return set_error(QSIM_ERR_ARG, "bad op array");
    if (check_options(opts) != QSIM_OK) return QSIM_ERR_ARG;
    std::vector<HostGate> gates(size_t(c->nops));
    for (int i = 0; i < c->nops; ++i) {
        qsim_status st = make_gate(c, i, params, nparams, gates[size_t(i)]);
        if (st != QSIM_OK) return st;
    }
    Plan plan;
    plan.n = n;
    plan.dtype = dtype;
    if (!build_plan(plan, gates, resolve_options(opts, n, dtype)))
        return set_error(QSIM_ERR_UNSUPPORTED, "the planner could not place every op");
    int64_t cnt[QSIM_KCLASS_COUNT_] = {0};
    double by = 0.0, fl = 0.0;
    for (const Pass &p : plan.passes) {
        const int cls = p.kind == PASS_DENSE ? QSIM_KCLASS_SWEEP_DENSE
                        : p.kind == PASS_DIAG ? QSIM_KCLASS_SWEEP_DIAG
                        : p.kind == PASS_TILE ? QSIM_KCLASS_TILE
                                              : QSIM_KCLASS_MFMA;
        ++cnt[cls];
        by += p.bytes;
        fl += p.flops;
    }
    if (counts)
        for (int i = 0; i < QSIM_KCLASS_COUNT_; ++i) counts[i] = cnt[i];
    if (bytes) *bytes = by;
    if (flops) *flops = fl;
    return QSIM_OK;
}

// Adjoint plans depend on the circuit's structure only: parametric
// rotations read (cos, sin) of their half angle from a table the call fills
// on the device from the caller's parameters, so a training loop plans once.
static const size_t kMaxAdjointPlans = 8;

static int rotation_kind_generator(int kind) {
    return kind == QSIM_GATE_RX ? 1 : kind == QSIM_GATE_RY ? 2 : kind == QSIM_GATE_RZ ? 3 : 0;
}

static qsim_status get_adjoint_plan(qsim_state s, const qsim_circuit *c, int64_t nparams, const qsim_options *opts,
                                    AdjointPlan **out) {
    const int fwd_m = (opts && opts->tile_m > 0) ? opts->tile_m : (s->dtype == QSIM_C128 ? 11 : 12);
    // checkpoints: at most one per gap between gates
    const int nck = std::max(0, std::min(opts ? opts->checkpoints : 0, c->nops - 1));
    std::string key;
    auto put = [&key](const void *p, size_t n) { key.append(static_cast<const char *>(p), n); };
    put(&nparams, sizeof nparams);
    put(&fwd_m, sizeof fwd_m);
    put(&nck, sizeof nck);
    for (int i = 0; i < c->nops; ++i) {
        qsim_op op = c->ops[i];
        if (op.param >= 0) op.angles[0] = op.angles[1] = op.angles[2] = 0.0;
        put(&op, sizeof op);
    }
    if (c->mats && c->nmats > 0) put(c->mats, sizeof(double) * 2 * size_t(c->nmats));
    for (auto &ap : s->adj_plans)
        if (ap->key == key) {
            ap->last_use = ++s->use_clock;
            *out = ap.get();
            return QSIM_OK;
        }
    std::unique_ptr<AdjointPlan> ap(new (std::nothrow) AdjointPlan());
    if (!ap) return set_error(QSIM_ERR_OOM, "host allocation failed");
    // gates with placeholder angles; parametric rotations become device-formed ops
    std::vector<double> zeros(size_t(std::max<int64_t>(nparams, 1)), 0.0);
    std::vector<HostGate> gates(size_t(c->nops));
    for (int i = 0; i < c->nops; ++i) {
        qsim_status st = make_gate(c, i, zeros.data(), nparams, gates[size_t(i)]);
        if (st != QSIM_OK) return st;
        if (c->ops[i].param >= 0) {
            const int gen = rotation_kind_generator(c->ops[i].kind);
            if (!gen)
                return set_error(QSIM_ERR_UNSUPPORTED,
                                 "op " + std::to_string(i) + ": gradients need RX, RY or RZ for parametric ops");
            gates[size_t(i)].rot_gen = gen;
            gates[size_t(i)].rot_param = c->ops[i].param;
        }
    }
    // reverse sweep, last op first: its probe (if parametric), then its
    // inverse; first_item[i]: where op i's items start
    std::vector<HostGate> items;
    std::vector<int> slot_param, first_item(size_t(c->nops) + 1, 0);
    items.reserve(2 * gates.size());
    for (int i = c->nops - 1; i >= 0; --i) {
        first_item[size_t(i)] = int(items.size());
        const HostGate &g = gates[size_t(i)];
        if (g.rot_gen) {
            HostGate pr;
            pr.k = 1;
            pr.targets[0] = g.targets[0];
            pr.probe_gen = g.rot_gen;
            pr.probe_slot = int(slot_param.size());
            slot_param.push_back(g.rot_param);
            items.push_back(pr);
            HostGate inv = g;
            inv.rot_inv = 1;
            items.push_back(std::move(inv));
        } else {
            HostGate inv = g;
            const int d = 1 << g.k;
            for (int r = 0; r < d; ++r)
                for (int cc = 0; cc < d; ++cc) inv.M[size_t(r) * d + cc] = std::conj(g.M[size_t(cc) * d + r]);
            items.push_back(std::move(inv));
        }
    }
    ap->fwd.n = ap->rev.n = s->n;
    ap->fwd.dtype = ap->rev.dtype = s->dtype;
    // reverse tiles of 2^10 amplitudes per state (wider when a gate needs
    // it): measured on the 20-qubit ansatz, smaller tiles put more
    // workgroups on the chip
    if (nck == 0) {
        if (build_tile_plan(ap->fwd, gates, std::min(s->n, fwd_m)) < 0)
            return set_error(QSIM_ERR_UNSUPPORTED, "the planner could not place every op");
        ap->mtile = build_adjoint_plan(ap->rev, items, 10);
        if (ap->mtile < 0) return set_error(QSIM_ERR_UNSUPPORTED, "the planner could not place every op");
    } else {
        // runs of about equal gate counts, planned one by one so that every
        // cut is a pass boundary of both sweeps; one reverse tile width
        Plan trial;
        trial.n = s->n;
        trial.dtype = s->dtype;
        ap->mtile = build_adjoint_plan(trial, items, 10);
        if (ap->mtile < 0) return set_error(QSIM_ERR_UNSUPPORTED, "the planner could not place every op");
        std::vector<int> cut(size_t(nck) + 2, 0);
        for (int j = 0; j < nck; ++j) cut[size_t(j) + 1] = int((int64_t(j) + 1) * c->nops / (nck + 1));
        cut[size_t(nck) + 1] = c->nops;
        for (int j = 0; j <= nck; ++j) {
            const std::vector<HostGate> seg(gates.begin() + cut[size_t(j)], gates.begin() + cut[size_t(j) + 1]);
            if (build_tile_plan(ap->fwd, seg, std::min(s->n, fwd_m)) < 0)
                return set_error(QSIM_ERR_UNSUPPORTED, "the planner could not place every op");
            if (j < nck) ap->fwd_cut.push_back(int(ap->fwd.passes.size()));
        }
        for (int j = nck; j >= 0; --j) {
            // items of ops cut[j] .. cut[j+1]-1 (last op first)
            const int i0 = first_item[size_t(cut[size_t(j) + 1] - 1)];
            const int i1 = cut[size_t(j)] > 0 ? first_item[size_t(cut[size_t(j)] - 1)] : int(items.size());
            const std::vector<HostGate> seg(items.begin() + i0, items.begin() + i1);
            if (build_tile_plan(ap->rev, seg, ap->mtile, 2) != ap->mtile)
                return set_error(QSIM_ERR_UNSUPPORTED, "the planner could not place every op");
            if (j > 0) {
                ap->rev_cut.push_back(int(ap->rev.passes.size()));
                ap->rev_ck.push_back(j - 1);
            }
        }
        for (Pass &p : ap->rev.passes) p.bytes *= 2.0;   // two states per pass
        ap->fwd.items = int(gates.size());
        ap->rev.items = int(items.size());
        ap->nck = nck;
    }
    ap->nprobes = int(slot_param.size());
    ap->nparams = nparams;
    qsim_status st = upload_plan(s, ap->fwd);
    if (st != QSIM_OK) return st;
    st = upload_plan(s, ap->rev);
    if (st != QSIM_OK) return st;
    // probes of each parameter, in sweep order: row[j] .. row[j + 1] of idx
    std::vector<int32_t> row(size_t(nparams) + 1, 0), idx(size_t(std::max(1, ap->nprobes)), 0);
    for (int k = 0; k < ap->nprobes; ++k) ++row[size_t(slot_param[size_t(k)]) + 1];
    for (int64_t j = 0; j < nparams; ++j) row[size_t(j) + 1] += row[size_t(j)];
    {
        std::vector<int32_t> fill(row.begin(), row.end() - 1);
        for (int k = 0; k < ap->nprobes; ++k) idx[size_t(fill[size_t(slot_param[size_t(k)])]++)] = k;
    }
    ap->idx_off = (sizeof(int32_t) * row.size() + 255) & ~size_t(255);
    const size_t bytes = ap->idx_off + sizeof(int32_t) * idx.size();
    if (hipMallocAsync(&ap->dev, bytes, s->stream) != hipSuccess) {
        (void)hipGetLastError();
        ap->dev = nullptr;
        return set_error(QSIM_ERR_OOM, "cannot allocate device memory for the adjoint plan");
    }
    ap->dev_stream = s->stream;
    st = ensure_pinned(s, bytes);
    if (st != QSIM_OK) return st;
    char *h = static_cast<char *>(s->pinned);
    std::memcpy(h, row.data(), sizeof(int32_t) * row.size());
    std::memcpy(h + ap->idx_off, idx.data(), sizeof(int32_t) * idx.size());
    st = upload_staged(s, ap->dev, bytes);
    if (st != QSIM_OK) return st;
    if (s->adj_plans.size() >= kMaxAdjointPlans) {
        auto lru = std::min_element(s->adj_plans.begin(), s->adj_plans.end(),
                                    [](const std::unique_ptr<AdjointPlan> &a, const std::unique_ptr<AdjointPlan> &b) {
                                        return a->last_use < b->last_use;
                                    });
        s->adj_plans.erase(lru);   // released in stream order
    }
    ap->key = std::move(key);
    ap->last_use = ++s->use_clock;
    *out = ap.get();
    s->adj_plans.push_back(std::move(ap));
    return QSIM_OK;
}

// The layered adjoint plan of (circuit structure, parameter count,
// observable) on this state, planned and uploaded on first use; *out is
// null when the circuit cannot run layered.
static qsim_status get_layered_adjoint(qsim_state s, const qsim_circuit *c, int64_t nparams, const qsim_pauli_sum *H,
                                       LayeredAdjointPlan **out) {
    *out = nullptr;
    std::string key;
    auto put = [&key](const void *p, size_t n) { key.append(static_cast<const char *>(p), n); };
    put(&nparams, sizeof nparams);
    for (int i = 0; i < c->nops; ++i) {
        qsim_op op = c->ops[i];
        if (op.param >= 0) op.angles[0] = op.angles[1] = op.angles[2] = 0.0;
        put(&op, sizeof op);
    }
    if (c->mats && c->nmats > 0) put(c->mats, sizeof(double) * 2 * size_t(c->nmats));
    put(&H->nterms, sizeof H->nterms);
    if (H->nterms > 0) put(H->terms, sizeof(qsim_pauli_term) * size_t(H->nterms));
    for (auto &lp : s->adj_lplans)
        if (lp->key == key) {
            lp->last_use = ++s->use_clock;
            if (lp->ok) *out = lp.get();
            return QSIM_OK;
        }
    std::unique_ptr<LayeredAdjointPlan> lp(new (std::nothrow) LayeredAdjointPlan());
    if (!lp) return set_error(QSIM_ERR_OOM, "host allocation failed");
    qsim_status st = plan_layered_adjoint(c, nparams, H, s->dtype, lp->la, &lp->ok);
    if (st != QSIM_OK) return st;
    if (lp->ok) {
        const size_t bytes = lp->la.host.size();
        if (hipMallocAsync(&lp->dev, bytes, s->stream) != hipSuccess) {
            (void)hipGetLastError();
            lp->dev = nullptr;
            return set_error(QSIM_ERR_OOM, "cannot allocate device memory for the adjoint plan");
        }
        lp->dev_stream = s->stream;
        st = ensure_pinned(s, bytes);
        if (st != QSIM_OK) return st;
        std::memcpy(s->pinned, lp->la.host.data(), bytes);
        st = upload_staged(s, lp->dev, bytes);
        if (st != QSIM_OK) return st;
        QSIM_HIP(s, batch_layer_setup(s->dtype, lp->la.ld.R), "layered kernel set-up");
    }
    if (s->adj_lplans.size() >= kMaxAdjointPlans) {
        auto lru = std::min_element(
            s->adj_lplans.begin(), s->adj_lplans.end(),
            [](const std::unique_ptr<LayeredAdjointPlan> &a, const std::unique_ptr<LayeredAdjointPlan> &b) {
                return a->last_use < b->last_use;
            });
        s->adj_lplans.erase(lru);   // released in stream order
    }
    lp->key = std::move(key);
    lp->last_use = ++s->use_clock;
    if (lp->ok) *out = lp.get();
    s->adj_lplans.push_back(std::move(lp));
    return QSIM_OK;
}

static bool on_device(const void *p) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

qsim_status qsim_adjoint_grad(qsim_state s, const qsim_circuit *c, const double *params_dev, int64_t nparams,
                              const qsim_pauli_sum *H, const qsim_options *opts, double *energy_dev,
                              double *grad_dev) {
    qsim_status st = check_state(s);
    if (st != QSIM_OK) return st;
    if (!c || !H || !energy_dev) return set_error(QSIM_ERR_ARG, "NULL argument");
    if (c->n != s->n) return set_error(QSIM_ERR_ARG, "circuit width does not match the state");
    if (c->nops < 0 || (c->nops > 0 && !c->ops)) return set_error(QSIM_ERR_ARG, "bad op array");
    if (nparams < 0 || nparams > (int64_t(1) << 30) || (nparams > 0 && (!params_dev || !grad_dev)))
        return set_error(QSIM_ERR_ARG, "bad parameter arrays");
    if (H->nterms < 0 || (H->nterms > 0 && !H->terms)) return set_error(QSIM_ERR_ARG, "bad Pauli sum");
    st = check_options(opts);
    if (st != QSIM_OK) return st;
    const uint64_t lim = (1ull << s->n) - 1;
    for (int t = 0; t < H->nterms; ++t)
        if ((H->terms[t].xmask & ~lim) || (H->terms[t].zmask & ~lim))
            return set_error(QSIM_ERR_ARG, "Pauli mask has a bit at or above n");
    if (!on_device(energy_dev) || (nparams > 0 && (!on_device(params_dev) || !on_device(grad_dev))))
        return set_error(QSIM_ERR_ARG, "params, energy and grad must be device memory");
    const size_t sbytes = amp_bytes(s->dtype) << s->n;
    // states of 2^11 amplitudes and more without checkpoints: the
    // register-staged layered passes of the batch, one circuit
    if (!(opts && opts->checkpoints > 0) && !(opts && opts->tile_m > 0)) {
        LayeredAdjointPlan *lp = nullptr;
        st = get_layered_adjoint(s, c, nparams, H, &lp);
        if (st != QSIM_OK) return st;
        if (lp) {
            if (!s->adj_lam) {
                if (hipMalloc(&s->adj_lam, sbytes) != hipSuccess) {
                    (void)hipGetLastError();
                    s->adj_lam = nullptr;
                    return set_error(QSIM_ERR_OOM, "cannot allocate the adjoint state");
                }
            }
            st = ensure_scratch(s, lp->la.scratch_bytes);
            if (st != QSIM_OK) return st;
            bind_layered_adjoint(lp->la, lp->dev, s->data, s->adj_lam, s->scratch, params_dev, energy_dev, grad_dev);
            QSIM_HIP(s, injected_fault(), "injected fault (QSIM_FAULT)");
            prof_begin(s, QSIM_KCLASS_ADJOINT, lp->la.pass_bytes, 0.0);
            const hipError_t e = launch_batch_layered(s->stream, s->dtype, lp->la.ld);
            prof_end(s);
            if (e != hipSuccess) return device_error(s, e, "layered adjoint");
            return QSIM_OK;
        }
    }
    AdjointPlan *ap = nullptr;
    st = get_adjoint_plan(s, c, nparams, opts, &ap);
    if (st != QSIM_OK) return st;
    if (!s->adj_lam) {
        if (hipMalloc(&s->adj_lam, sbytes) != hipSuccess) {
            (void)hipGetLastError();
            s->adj_lam = nullptr;
            return set_error(QSIM_ERR_OOM, "cannot allocate the adjoint state");
        }
    }
    if (ap->nck > s->adj_ck_count) {
        if (s->adj_ck) {
            (void)hipStreamSynchronize(s->stream);
            (void)hipFree(s->adj_ck);
        }
        s->adj_ck = nullptr;
        s->adj_ck_count = 0;
        if (hipMalloc(&s->adj_ck, sbytes * size_t(ap->nck)) != hipSuccess) {
            (void)hipGetLastError();
            s->adj_ck = nullptr;
            return set_error(QSIM_ERR_OOM, "cannot allocate the adjoint checkpoints");
        }
        s->adj_ck_count = ap->nck;
    }
    char *ck = static_cast<char *>(s->adj_ck);
    // the Pauli sum on the device, grouped by X mask (kept while it is unchanged)
    struct DevGroup {
        uint64_t x;
        int32_t first, count;
    };
    struct DevTerm {
        double wr, wi;
        uint64_t z, pad;
    };
    std::map<uint64_t, std::vector<int>> bygroup;
    for (int t = 0; t < H->nterms; ++t) bygroup[H->terms[t].xmask].push_back(t);
    const int ng = int(bygroup.size());
    auto align = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t hterms_off = align(sizeof(DevGroup) * size_t(std::max(1, ng)));
    const size_t hbytes = hterms_off + sizeof(DevTerm) * size_t(std::max(1, H->nterms));
    const std::string hkey(reinterpret_cast<const char *>(H->terms), sizeof(qsim_pauli_term) * size_t(H->nterms));
    if (!s->adj_h || s->adj_h_key != hkey || s->adj_h_bytes < hbytes) {
        if (s->adj_h_bytes < hbytes) {
            if (s->adj_h) (void)hipFreeAsync(s->adj_h, s->stream);
            s->adj_h = nullptr;
            s->adj_h_bytes = 0;
            if (hipMallocAsync(&s->adj_h, hbytes, s->stream) != hipSuccess) {
                (void)hipGetLastError();
                s->adj_h = nullptr;
                return set_error(QSIM_ERR_OOM, "cannot allocate device memory for the Pauli sum");
            }
            s->adj_h_bytes = hbytes;
        }
        st = ensure_pinned(s, hbytes);
        if (st != QSIM_OK) return st;
        char *hp = static_cast<char *>(s->pinned);
        DevGroup *hg = reinterpret_cast<DevGroup *>(hp);
        DevTerm *ht = reinterpret_cast<DevTerm *>(hp + hterms_off);
        int gi = 0, slot = 0;
        for (auto &kv : bygroup) {
            hg[gi].x = kv.first;
            hg[gi].first = slot;
            hg[gi].count = int(kv.second.size());
            ++gi;
            for (int t : kv.second) {
                const qsim_pauli_term &pt = H->terms[t];
                const int ny = __builtin_popcountll(pt.xmask & pt.zmask) & 3;
                const double re[4] = {1, 0, -1, 0}, im[4] = {0, 1, 0, -1};
                ht[slot].wr = pt.coeff * re[ny];
                ht[slot].wi = pt.coeff * im[ny];
                ht[slot].z = pt.zmask;
                ht[slot].pad = 0;
                ++slot;
            }
        }
        st = upload_staged(s, s->adj_h, hbytes);
        if (st != QSIM_OK) return st;
        s->adj_h_key = hkey;
    }
    const int nprobes = ap->nprobes;
    const int ntiles = 1 << (s->n - ap->mtile);
    // scratch: [trig][energy partials][probe partials][probe sums + energy]
    const int egrid = pauli_apply_grid(1ull << s->n);
    const size_t off_epart = align(sizeof(double) * 2 * size_t(std::max<int64_t>(nparams, 1)));
    const size_t off_pp = align(off_epart + sizeof(double) * size_t(egrid));
    const size_t off_sums = align(off_pp + sizeof(double) * size_t(nprobes) * size_t(ntiles));
    const size_t total = off_sums + sizeof(double) * size_t(nprobes + 1);
    st = ensure_scratch(s, total);
    if (st != QSIM_OK) return st;
    char *scr = static_cast<char *>(s->scratch);
    double *trig = reinterpret_cast<double *>(scr);
    double *epart = reinterpret_cast<double *>(scr + off_epart);
    double *pp = reinterpret_cast<double *>(scr + off_pp);
    double *sums = reinterpret_cast<double *>(scr + off_sums);
    QSIM_HIP(s, injected_fault(), "injected fault (QSIM_FAULT)");
    QSIM_HIP(s, launch_half_angle_trig(s, params_dev, nparams, trig), "trig launch");
    // forward: psi <- C(theta) psi, with a copy of psi at every cut
    size_t next_cut = 0;
    for (size_t pi = 0; pi < ap->fwd.passes.size(); ++pi) {
        const Pass &p = ap->fwd.passes[pi];
        prof_begin(s, QSIM_KCLASS_TILE, p.bytes, p.flops);
        hipError_t e = launch_tile_pass(s, ap->fwd, p, trig);
        prof_end(s);
        if (e != hipSuccess) return device_error(s, e, "forward pass");
        if (next_cut < ap->fwd_cut.size() && int(pi) + 1 == ap->fwd_cut[next_cut]) {
            QSIM_HIP(s, hipMemcpyAsync(ck + sbytes * next_cut, s->data, sbytes, hipMemcpyDeviceToDevice, s->stream),
                     "checkpoint copy");
            ++next_cut;
        }
    }
    // lambda <- H psi, energy partials
    prof_begin(s, QSIM_KCLASS_EXPECT, 2.0 * double(sbytes) * double(std::max(1, ng)));
    QSIM_HIP(s, launch_pauli_apply(s, s->adj_lam, s->adj_h, ng, static_cast<char *>(s->adj_h) + hterms_off, epart),
             "pauli apply");
    prof_end(s);
    QSIM_HIP(s, launch_reduce(s, epart, egrid, sums + nprobes), "reduce");
    // reverse sweep over (psi, lambda); psi restored from its checkpoint at
    // every cut
    next_cut = 0;
    for (size_t pi = 0; pi < ap->rev.passes.size(); ++pi) {
        const Pass &p = ap->rev.passes[pi];
        prof_begin(s, QSIM_KCLASS_ADJOINT, p.bytes, 2.0 * p.flops);
        hipError_t e = launch_adjoint_pass(s, ap->rev, p, s->adj_lam, pp, trig);
        prof_end(s);
        if (e != hipSuccess) return device_error(s, e, "adjoint pass");
        if (next_cut < ap->rev_cut.size() && int(pi) + 1 == ap->rev_cut[next_cut]) {
            QSIM_HIP(s,
                     hipMemcpyAsync(s->data, ck + sbytes * size_t(ap->rev_ck[next_cut]), sbytes,
                                    hipMemcpyDeviceToDevice, s->stream),
                     "checkpoint restore");
            ++next_cut;
        }
    }
    QSIM_HIP(s, launch_reduce_rows(s, pp, nprobes, ntiles, sums), "reduce rows");
    const int32_t *row = static_cast<const int32_t *>(ap->dev);
    const int32_t *idx = reinterpret_cast<const int32_t *>(static_cast<const char *>(ap->dev) + ap->idx_off);
    QSIM_HIP(s, launch_gather_gradient(s, sums, row, idx, nparams, nprobes, grad_dev, energy_dev), "gradient gather");
    return QSIM_OK;
}

qsim_status qsim_autotune(qsim_state s, const qsim_circuit *c, const double *params, int64_t nparams, int reps,
                          qsim_options *best, double *best_ms) {
    qsim_status st = check_state(s);
    if (st != QSIM_OK) return st;
    if (!c || !best) return set_error(QSIM_ERR_ARG, "NULL argument");
    if (c->n != s->n) return set_error(QSIM_ERR_ARG, "circuit width does not match the state");
    if (c->nops < 1 || !c->ops) return set_error(QSIM_ERR_ARG, "empty circuit");
    if (reps < 1) return set_error(QSIM_ERR_ARG, "reps must be at least 1");
    // candidates: plain sweeps; LDS tiles of three sizes with fusion 1..3;
    // matrix-core blocks of 4..6 qubits
    std::vector<qsim_options> cands;
    cands.push_back({1, -1, -1, 0});
    const int mlo = s->dtype == QSIM_C128 ? 10 : 11;
    // (compiled register tiles: the split single-qubit form without fusion
    // has the least arithmetic; one compilation per tile size)
    const bool jit = jit_wanted(s->n);
    const int fmax = jit ? 1 : 3;
    for (int m = jit ? mlo + 1 : mlo; m <= mlo + 2; ++m) {
        if (m > s->n && m > mlo) break;
        for (int f = 1; f <= fmax; ++f) cands.push_back({f, m, -1, 0});
    }
    for (int f = 4; f <= 6; ++f)
        if (f <= s->n) cands.push_back({f, -1, 1, 0});
    hipEvent_t e0 = nullptr, e1 = nullptr;
    QSIM_HIP(s, hipEventCreate(&e0), "hipEventCreate");
    QSIM_HIP(s, hipEventCreate(&e1), "hipEventCreate");
    double best_t = 1e300;
    qsim_options chosen = cands[0];
    for (const qsim_options &o : cands) {
        Plan *plan = nullptr;
        st = get_plan(s, c, params, nparams, &o, &plan);
        if (st == QSIM_OK) st = run_plan(s, *plan);   // warm-up (and upload)
        if (st != QSIM_OK) break;
        QSIM_HIP(s, hipEventRecord(e0, s->stream), "hipEventRecord");
        for (int r = 0; r < reps && st == QSIM_OK; ++r) st = run_plan(s, *plan);
        if (st != QSIM_OK) break;
        QSIM_HIP(s, hipEventRecord(e1, s->stream), "hipEventRecord");
        QSIM_HIP(s, hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        QSIM_HIP(s, hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        const double t = double(ms) / reps;
        if (t < best_t) {
            best_t = t;
            chosen = o;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != QSIM_OK) return st;
    remember_tuning(c, s->n, s->dtype, chosen);
    *best = chosen;
    if (best_ms) *best_ms = best_t;
    return QSIM_OK;
}

qsim_status qsim_profile_enable(qsim_state s, int on) {
    qsim_status st = check_state(s);
    if (st != QSIM_OK) return st;
    if (on) {
        QSIM_HIP(s, hipStreamSynchronize(s->stream), "hipStreamSynchronize");
        prof_clear(s);
    }
    s->prof.on = on != 0;
    return QSIM_OK;
}

qsim_status qsim_profile_read(qsim_state s, int cls, int64_t *launches, double *ms, double *bytes,
                              double *flops) {
    qsim_status st = check_state(s);
    if (st != QSIM_OK) return st;
    if (cls < 0 || cls >= QSIM_KCLASS_COUNT_) return set_error(QSIM_ERR_ARG, "unknown kernel class");
    QSIM_HIP(s, hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    int64_t cnt = 0;
    double tot = 0.0, by = 0.0, fl = 0.0;
    for (auto &r : s->prof.recs) {
        if (r.cls != cls || !r.a || !r.b) continue;
        float t = 0.f;
        QSIM_HIP(s, hipEventElapsedTime(&t, r.a, r.b), "hipEventElapsedTime");
        ++cnt;
        tot += t;
        by += r.bytes;
        fl += r.flops;
    }
    if (launches) *launches = cnt;
    if (ms) *ms = tot;
    if (bytes) *bytes = by;
    if (flops) *flops = fl;
    return QSIM_OK;
}

}  // extern "C"
