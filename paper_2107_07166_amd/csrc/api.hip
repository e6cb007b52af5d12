// The C ABI (include/tfmm.h): argument checks, error capture and the order of
// the phases on the caller's stream.
#include <algorithm>
#include <cmath>
#include <new>

#include "common.h"

namespace tfmm {

DevBuf::~DevBuf() { release(); }

void DevBuf::release() {
    if (p && ctx) ctx->free(p, cap);
    p = nullptr;
    cap = 0;
}

void DevBuf::ensure(Ctx* c, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (p && cap >= bytes) return;
    release();
    ctx = c;
    const size_t want = (size_t)round_up((int64_t)bytes, 256);
    size_t got = 0;
    p = c->alloc(want, &got);
    cap = got;
}

void DevBuf::ensure_keep(Ctx* c, size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 16;
    if (p && cap >= bytes) return;
    const size_t want = (size_t)round_up((int64_t)bytes, 256);
    size_t got = 0;
    void* q = c->alloc(want, &got);
    if (p) {
        TFMM_HIP(hipMemcpyAsync(q, p, cap, hipMemcpyDeviceToDevice, s));
        TFMM_HIP(hipStreamSynchronize(s));
    }
    release();
    ctx = c;
    p = q;
    cap = got;
}

// A cached block of size in [bytes, 2 bytes] is reused as is; otherwise new
// memory, after giving the cache back if the budget or the device is short.
void* Ctx::alloc(size_t bytes, size_t* got) {
    auto it = cache.lower_bound(bytes);
    if (it != cache.end() && it->first <= 2 * bytes) {
        void* q = it->second;
        *got = it->first;
        cached -= it->first;
        cache.erase(it);
        return q;
    }
    if (budget && used + bytes > budget) trim_cache();
    if (budget && used + bytes > budget)
        fail(TFMM_ENOMEM, "device memory budget exceeded (" + std::to_string(used + bytes) + " > " +
                              std::to_string(budget) + " bytes)");
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if ((e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) && !cache.empty()) {
        (void)hipGetLastError();
        trim_cache();
        e = hipMalloc(&q, bytes);
    }
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        fail(TFMM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: out of device memory");
    }
    if (e != hipSuccess) fail(TFMM_EDEVICE, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    used += bytes;
    *got = bytes;
    return q;
}

// A buffer is only released when it grows or its owner goes away; kernels
// queued earlier may still read it, so the device must be idle before the
// block can serve a new owner.
void Ctx::free(void* q, size_t bytes) {
    if (!q) return;
    if (!idle_release) (void)hipDeviceSynchronize();
    cache.emplace(bytes, q);
    cached += bytes;
}

void Ctx::trim_cache() {
    if (cache.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto& kv : cache) {
        (void)hipFree(kv.second);
        used -= std::min(used, kv.first);
    }
    cache.clear();
    cached = 0;
}

namespace {

template <typename F>
int guarded(Ctx* ctx, F&& f) {
    if (ctx && ctx->broken) {
        ctx->err = "context is unusable after an earlier device error";
        return TFMM_EDEVICE;
    }
    try {
        if (ctx) ctx->err.clear();
        f();
        return TFMM_OK;
    } catch (const Error& e) {
        if (ctx) {
            ctx->err = e.msg;
            if (e.code == TFMM_EDEVICE) ctx->broken = true;
        }
        return e.code;
    } catch (const std::bad_alloc&) {
        if (ctx) ctx->err = "host allocation failed";
        return TFMM_ENOMEM;
    }
}

void set_device(Ctx* ctx) { TFMM_HIP(hipSetDevice(ctx->device)); }

void check_params(const tfmm_params* p) {
    if (!p) fail(TFMM_EINVAL, "params is NULL");
    if (p->p < 1 || p->p > kMaxP) fail(TFMM_EINVAL, "p must be in 1..8");
    if (!(p->theta >= 0.0) || !(p->theta < 1.0)) fail(TFMM_EINVAL, "theta must satisfy 0 <= theta < 1");
    if (!(p->softening >= 0.0) || !std::isfinite(p->softening)) fail(TFMM_EINVAL, "softening must be >= 0");
    if (!std::isfinite(p->G)) fail(TFMM_EINVAL, "G must be finite");
    if (p->variant != TFMM_STANDARD && p->variant != TFMM_CONSERVING && p->variant != TFMM_CONSERVING_R2)
        fail(TFMM_EINVAL, "unknown variant");
    if (p->variant == TFMM_CONSERVING_R2 && p->p != 1)
        fail(TFMM_EINVAL, "the conserving_r2 variant is zeroth order: p must be 1");
    if (p->precision != TFMM_FP64 && p->precision != TFMM_MIXED32) fail(TFMM_EINVAL, "unknown precision");
    if (p->scalar_degree != 0) {
        if (p->variant != TFMM_CONSERVING)
            fail(TFMM_EINVAL, "scalar_degree applies to the conserving variant only");
        if (p->scalar_degree < p->p - 1 || p->scalar_degree > std::min(p->p + 1, kKnobMaxK))
            fail(TFMM_EINVAL, "scalar_degree must satisfy p-1 <= K <= min(p+1, 6)");
    }
}

// Particle sets of a forest: offsets (host) ascending from 0, every set
// non-empty; returns the particle count.
int64_t check_sets(int n_sets, const int64_t* offsets) {
    if (n_sets < 1 || n_sets > kMaxSets) fail(TFMM_EINVAL, "n_sets must be in 1..4096");
    if (!offsets) fail(TFMM_EINVAL, "offsets is NULL");
    if (offsets[0] != 0) fail(TFMM_EINVAL, "offsets[0] must be 0");
    for (int k = 0; k < n_sets; ++k)
        if (offsets[k + 1] <= offsets[k]) fail(TFMM_EINVAL, "every set must hold at least one particle");
    const int64_t n = offsets[n_sets];
    if (n > (int64_t)INT32_MAX / 2) fail(TFMM_EINVAL, "n must be in 1..2^30");
    return n;
}

void set_sets(Tree& t, int n_sets, const int64_t* offsets, hipStream_t s) {
    t.n_sets = n_sets;
    if (n_sets > 1) upload(t, t.set_off, offsets, (size_t)(n_sets + 1) * sizeof(int64_t), 0, s);
}

// Degree of the conserving projection scalar (p - 1 unless raised).
int scalar_degree(const tfmm_params* p) {
    return p->scalar_degree == 0 ? p->p - 1 : p->scalar_degree;
}

// Two streams: s (the caller's) and the tree's second stream a.
//   a: moments (during the frontier passes) -> far-list chain -> M2L -> L2L
//      -> L2P's far part
//   s: sources -> frontier passes -> near-list chain -> P2P -> split-leaf
//      reduction -> [join a] -> forces (near + far)
// The latency-bound list chains hide behind each other, and P2P starts as
// soon as the near lists exist, beside M2L and L2L on the second stream.
// Adds the phase times of the last timed evaluation to the tree's sums.
// Events: moments [0,1], M2L [7,2], L2L [2,3] on the tree's second stream;
// P2P [6,4] (the near-field kernel; the partial-sum reduction follows it),
// the forces from near and far parts [8,5] on the caller's stream (8: after
// the streams join; L2P's far part runs before the join, after L2L);
// whole evaluation [0,5]; walk [11, later of 7 and 6], its frontier passes
// [11,12] (only in evaluations that walked).
double elapsed_ms(Tree& t, int i, int j) {
    float ms = 0.f;
    TFMM_HIP(hipEventElapsedTime(&ms, t.ev[i], t.ev[j]));
    return (double)ms;
}

void fold_times(Tree& t) {
    if (!t.ev_pending) return;
    TFMM_HIP(hipEventSynchronize(t.ev[5]));
    t.t_sum[0] += elapsed_ms(t, 7, 2);  // M2L
    t.t_sum[1] += elapsed_ms(t, 6, 4);  // P2P
    t.t_sum[2] += elapsed_ms(t, 2, 3);  // L2L
    t.t_sum[3] += elapsed_ms(t, 8, 5);  // forces after the join
    t.t_sum[4] += elapsed_ms(t, 0, 1);  // moments
    t.t_sum[5] += elapsed_ms(t, 0, 5);  // whole evaluation after the tree build
    {
        // the interaction pass: from the first of P2P and M2L to start (6, 7)
        // until the later of the two ends (4, 2)
        const int first = elapsed_ms(t, 7, 6) >= 0.0 ? 7 : 6;
        t.t_sum[9] += std::max(elapsed_ms(t, first, 4), elapsed_ms(t, first, 2));
    }
    if (t.ev_walked) {
        // the far-list chain ends where M2L starts (7), the near-list chain where P2P starts (6)
        t.t_sum[7] += std::max(elapsed_ms(t, 11, 7), elapsed_ms(t, 11, 6));
        t.t_sum[8] += elapsed_ms(t, 11, 12);
        t.t_walks += 1;
    }
    t.t_count += 1;
    t.ev_pending = false;
}

// Adds the time of the last timed rebuild to the tree's sums.
void fold_build(Tree& t) {
    if (!t.build_pending) return;
    TFMM_HIP(hipEventSynchronize(t.ev[10]));
    t.t_sum[6] += elapsed_ms(t, 9, 10);
    t.t_builds += 1;
    t.build_pending = false;
}

void timing_events(Tree& t) {
    if (t.timing && !t.ev_ready) {
        for (auto& e : t.ev) TFMM_HIP(hipEventCreate(&e));
        t.ev_ready = true;
    }
}

// theta_sets: one theta per set of a forest (host), or nullptr for
// params->theta everywhere.
void evaluate(Tree& t, const tfmm_params* prm, const double* theta_sets, double* force, double* potential,
              hipStream_t s) {
    const std::vector<double> theta =
        theta_sets ? std::vector<double>(theta_sets, theta_sets + t.n_sets) : std::vector<double>{prm->theta};
    const bool need_walk = !t.walk_valid || t.walk_theta != theta;
    // The zeroth-order magnitude realignment (Eq. aaB0) is quadratic in the
    // target offset and needs the node quadrupoles: it runs through the
    // conserving locals (P, Q') of order 2, with its own M2L.
    const bool r2 = prm->variant == TFMM_CONSERVING_R2;
    // A conserving projection scalar kept to degree K > p - 1 needs moments and
    // locals of order K + 1.
    const int kdeg = scalar_degree(prm);
    const bool knob = prm->variant == TFMM_CONSERVING && kdeg > prm->p - 1;
    const int pe = r2 ? 2 : (knob ? kdeg + 1 : prm->p);
    const int ve = r2 ? TFMM_CONSERVING : prm->variant;
    const double eps2 = prm->softening * prm->softening;
    timing_events(t);
    if (t.timing) fold_times(t);
    aux_fork(t, s);
    const hipStream_t a = t.aux;
    if (t.timing) TFMM_HIP(hipEventRecord(t.ev[0], a));
    compute_moments(t, pe, a);
    if (t.timing) TFMM_HIP(hipEventRecord(t.ev[1], a));
    prepare_sources(t, prm->precision, s);
    if (need_walk) {
        t.walk_valid = false;
        if (t.timing) TFMM_HIP(hipEventRecord(t.ev[11], s));
        walk_lists_begin(t, theta, s, t.timing ? t.ev[12] : nullptr);
    }
    if (t.timing) TFMM_HIP(hipEventRecord(t.ev[7], a));
    run_m2l(t, knob ? prm->p : pe, prm->variant, prm->precision, eps2, a, knob ? kdeg : -1);
    if (t.timing) TFMM_HIP(hipEventRecord(t.ev[2], a));
    run_l2l(t, pe, ve, a);
    if (t.timing) TFMM_HIP(hipEventRecord(t.ev[3], a));
    // the far-field part of L2P beside the near field; only the sum of the
    // two waits for both
    run_l2p_far(t, pe, ve, a);
    if (need_walk) walk_lists_end(t, s);
    if (t.timing) TFMM_HIP(hipEventRecord(t.ev[6], s));
    run_p2p(t, prm->precision, eps2, potential != nullptr, s);
    if (t.timing) TFMM_HIP(hipEventRecord(t.ev[4], s));
    run_p2p_reduce(t, potential != nullptr, s);
    aux_join(t, s);
    if (t.timing) TFMM_HIP(hipEventRecord(t.ev[8], s));
    run_force_combine(t, prm->G, force, s);
    if (potential) {
        // far-field potential from the standard expansion of order p (every
        // variant), after the forces on the same stream
        run_m2l_pot(t, prm->p, pe, prm->precision, eps2, s);
        run_potential_down(t, prm->p, prm->precision, eps2, prm->G, potential, s);
    }
    if (t.timing) {
        TFMM_HIP(hipEventRecord(t.ev[5], s));
        t.ev_pending = true;
        t.ev_walked = need_walk;
    }
}

}  // namespace
}  // namespace tfmm

using namespace tfmm;

extern "C" {

int tfmm_ctx_create(int device, size_t hbm_budget_bytes, tfmm_ctx** out) {
    if (!out) return TFMM_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return TFMM_EDEVICE;
    if (device < 0 || device >= ndev) return TFMM_EINVAL;
    tfmm_ctx* c = new (std::nothrow) tfmm_ctx();
    if (!c) return TFMM_ENOMEM;
    c->device = device;
    c->budget = hbm_budget_bytes;
    const int rc = guarded(c, [&] {
        set_device(c);
        diag_scratch_init(device);
        c->pinned_bytes = 1 << 16;
        TFMM_HIP(hipHostMalloc(&c->pinned, c->pinned_bytes, hipHostMallocDefault));
        void* mb = nullptr;
        TFMM_HIP(hipHostMalloc(&mb, kBoxBytes, hipHostMallocCoherent | hipHostMallocMapped));
        c->mbox = static_cast<uint32_t*>(mb);
        std::memset(mb, 0, kBoxBytes);
        void* mbd = nullptr;
        TFMM_HIP(hipHostGetDevicePointer(&mbd, mb, 0));
        c->mbox_dev = static_cast<uint32_t*>(mbd);
        TFMM_HIP(hipMalloc(reinterpret_cast<void**>(&c->dev_err), 256));
        TFMM_HIP(hipMemset(c->dev_err, 0, 256));
    });
    if (rc != TFMM_OK) {
        if (c->pinned) (void)hipHostFree(c->pinned);
        if (c->mbox) (void)hipHostFree(c->mbox);
        if (c->dev_err) (void)hipFree(c->dev_err);
        delete c;
        return rc;
    }
    *out = c;
    return TFMM_OK;
}

int tfmm_ctx_destroy(tfmm_ctx* ctx) {
    if (!ctx) return TFMM_OK;
    if (ctx->live_trees > 0) {
        ctx->err = "destroy every tree of the context first";
        return TFMM_ESTATE;
    }
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->trim_cache();
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->mbox) (void)hipHostFree(ctx->mbox);
    if (ctx->dev_err) (void)hipFree(ctx->dev_err);
    delete ctx;
    return TFMM_OK;
}

const char* tfmm_last_error(const tfmm_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

size_t tfmm_ctx_bytes_in_use(const tfmm_ctx* ctx) { return ctx ? ctx->used - ctx->cached : 0; }

size_t tfmm_ctx_bytes_held(const tfmm_ctx* ctx) { return ctx ? ctx->used : 0; }

int tfmm_ctx_set_budget(tfmm_ctx* ctx, size_t hbm_budget_bytes) {
    if (!ctx) return TFMM_EINVAL;
    return guarded(ctx, [&] {
        set_device(ctx);
        ctx->budget = hbm_budget_bytes;
        if (hbm_budget_bytes && ctx->used > hbm_budget_bytes) ctx->trim_cache();
    });
}

int tfmm_ctx_trim(tfmm_ctx* ctx) {
    if (!ctx) return TFMM_EINVAL;
    return guarded(ctx, [&] {
        set_device(ctx);
        ctx->trim_cache();
    });
}

int tfmm_build_tree(tfmm_ctx* ctx, int64_t n, const double* pos, const double* mass, int n_leaf, void* stream,
                    tfmm_tree** out) {
    if (!ctx) return TFMM_EINVAL;
    if (!out) {
        ctx->err = "out is NULL";
        return TFMM_EINVAL;
    }
    *out = nullptr;
    tfmm_tree* t = nullptr;
    const int rc = guarded(ctx, [&] {
        if (n < 1 || n > (int64_t)INT32_MAX / 2) fail(TFMM_EINVAL, "n must be in 1..2^30");
        if (!pos || !mass) fail(TFMM_EINVAL, "pos and mass must be device pointers");
        if (n_leaf < 1 || n_leaf > 4096) fail(TFMM_EINVAL, "n_leaf must be in 1..4096");
        set_device(ctx);
        t = new tfmm_tree();
        t->ctx = ctx;
        t->n = n;
        t->n_leaf = n_leaf;
        ctx->live_trees++;
        build_tree(*t, pos, mass, (hipStream_t)stream);
    });
    if (rc != TFMM_OK) {
        if (t) {
            ctx->live_trees--;
            delete t;
        }
        return rc;
    }
    *out = t;
    return TFMM_OK;
}

int tfmm_tree_rebuild(tfmm_tree* tree, int64_t n, const double* pos, const double* mass, void* stream) {
    if (!tree) return TFMM_EINVAL;
    return guarded(tree->ctx, [&] {
        if (n < 1 || n > (int64_t)INT32_MAX / 2) fail(TFMM_EINVAL, "n must be in 1..2^30");
        if (!pos || !mass) fail(TFMM_EINVAL, "pos and mass must be device pointers");
        set_device(tree->ctx);
        Tree& t = *tree;
        const hipStream_t s = (hipStream_t)stream;
        timing_events(t);
        if (t.timing) {
            fold_build(t);
            TFMM_HIP(hipEventRecord(t.ev[9], s));
        }
        t.n = n;
        t.n_sets = 1;
        build_tree(t, pos, mass, s);
        if (t.timing) {
            TFMM_HIP(hipEventRecord(t.ev[10], s));
            t.build_pending = true;
        }
    });
}

int tfmm_build_forest(tfmm_ctx* ctx, int n_sets, const int64_t* offsets, const double* pos, const double* mass,
                      int n_leaf, void* stream, tfmm_tree** out) {
    if (!ctx) return TFMM_EINVAL;
    if (!out) {
        ctx->err = "out is NULL";
        return TFMM_EINVAL;
    }
    *out = nullptr;
    tfmm_tree* t = nullptr;
    const int rc = guarded(ctx, [&] {
        const int64_t n = check_sets(n_sets, offsets);
        if (!pos || !mass) fail(TFMM_EINVAL, "pos and mass must be device pointers");
        if (n_leaf < 1 || n_leaf > 4096) fail(TFMM_EINVAL, "n_leaf must be in 1..4096");
        set_device(ctx);
        t = new tfmm_tree();
        t->ctx = ctx;
        t->n = n;
        t->n_leaf = n_leaf;
        ctx->live_trees++;
        set_sets(*t, n_sets, offsets, (hipStream_t)stream);
        build_tree(*t, pos, mass, (hipStream_t)stream);
    });
    if (rc != TFMM_OK) {
        if (t) {
            tfmm_tree_destroy(t);
        }
        return rc;
    }
    *out = t;
    return TFMM_OK;
}

int tfmm_forest_rebuild(tfmm_tree* tree, int n_sets, const int64_t* offsets, const double* pos,
                        const double* mass, void* stream) {
    if (!tree) return TFMM_EINVAL;
    return guarded(tree->ctx, [&] {
        const int64_t n = check_sets(n_sets, offsets);
        if (!pos || !mass) fail(TFMM_EINVAL, "pos and mass must be device pointers");
        set_device(tree->ctx);
        Tree& t = *tree;
        const hipStream_t s = (hipStream_t)stream;
        timing_events(t);
        if (t.timing) {
            fold_build(t);
            TFMM_HIP(hipEventRecord(t.ev[9], s));
        }
        t.n = n;
        set_sets(t, n_sets, offsets, s);
        build_tree(t, pos, mass, s);
        if (t.timing) {
            TFMM_HIP(hipEventRecord(t.ev[10], s));
            t.build_pending = true;
        }
    });
}

int tfmm_evaluate_forest(tfmm_tree* tree, const tfmm_params* params, const double* theta, double* force,
                         double* potential, void* stream) {
    if (!tree) return TFMM_EINVAL;
    return guarded(tree->ctx, [&] {
        check_params(params);
        if (!force) fail(TFMM_EINVAL, "force must be a device pointer");
        if (theta)
            for (int k = 0; k < tree->n_sets; ++k)
                if (!(theta[k] >= 0.0) || !(theta[k] < 1.0))
                    fail(TFMM_EINVAL, "theta must satisfy 0 <= theta < 1 for every set");
        set_device(tree->ctx);
        evaluate(*tree, params, theta, force, potential, (hipStream_t)stream);
    });
}

int tfmm_tree_walk(tfmm_tree* tree, double theta, void* stream) {
    if (!tree) return TFMM_EINVAL;
    return guarded(tree->ctx, [&] {
        if (!(theta >= 0.0) || !(theta < 1.0)) fail(TFMM_EINVAL, "theta must satisfy 0 <= theta < 1");
        set_device(tree->ctx);
        walk_tree(*tree, std::vector<double>{theta}, (hipStream_t)stream);
    });
}

int tfmm_evaluate_forces(tfmm_tree* tree, const tfmm_params* params, double* force, double* potential,
                         void* stream) {
    if (!tree) return TFMM_EINVAL;
    return guarded(tree->ctx, [&] {
        check_params(params);
        if (!force) fail(TFMM_EINVAL, "force must be a device pointer");
        set_device(tree->ctx);
        evaluate(*tree, params, nullptr, force, potential, (hipStream_t)stream);
    });
}

int tfmm_evaluate_forces_oneshot(tfmm_ctx* ctx, int64_t n, const double* pos, const double* mass, int n_leaf,
                                 const tfmm_params* params, double* force, void* stream) {
    if (!ctx) return TFMM_EINVAL;
    tfmm_tree* t = nullptr;
    int rc = guarded(ctx, [&] { check_params(params); });
    if (rc != TFMM_OK) return rc;
    rc = tfmm_build_tree(ctx, n, pos, mass, n_leaf, stream, &t);
    if (rc != TFMM_OK) return rc;
    rc = tfmm_evaluate_forces(t, params, force, nullptr, stream);
    if (rc == TFMM_OK) rc = guarded(ctx, [&] { TFMM_HIP(hipStreamSynchronize((hipStream_t)stream)); });
    const std::string keep = ctx->err;
    tfmm_tree_destroy(t);
    if (rc != TFMM_OK) ctx->err = keep;
    return rc;
}

int tfmm_leapfrog(tfmm_tree* tree, const tfmm_params* params, double* pos, double* vel, const double* mass,
                  double* force, double dt, int nsteps, int force_valid, void* stream) {
    if (!tree) return TFMM_EINVAL;
    return guarded(tree->ctx, [&] {
        check_params(params);
        if (!pos || !vel || !mass || !force) fail(TFMM_EINVAL, "pos, vel, mass and force must be device pointers");
        if (nsteps < 0 || !std::isfinite(dt)) fail(TFMM_EINVAL, "nsteps must be >= 0 and dt finite");
        if (tree->n_sets != 1) fail(TFMM_EINVAL, "leapfrog needs a tree of one particle set");
        set_device(tree->ctx);
        Tree& t = *tree;
        const hipStream_t s = (hipStream_t)stream;
        if (!force_valid) {
            build_tree(t, pos, mass, s);
            evaluate(t, params, nullptr, force, nullptr, s);
        }
        for (int k = 0; k < nsteps; ++k) {
            run_kick(t.n, vel, force, mass, 0.5 * dt, s);
            run_drift(t.n, pos, vel, dt, s);
            build_tree(t, pos, mass, s);
            evaluate(t, params, nullptr, force, nullptr, s);
            run_kick(t.n, vel, force, mass, 0.5 * dt, s);
        }
    });
}

int tfmm_momentum_diagnostics(tfmm_ctx* ctx, int64_t n, const double* pos, const double* vel, const double* mass,
                              const double* force, void* stream, double* out) {
    if (!ctx) return TFMM_EINVAL;
    return guarded(ctx, [&] {
        if (n < 1 || !pos || !mass || !force || !out) fail(TFMM_EINVAL, "bad diagnostics arguments");
        set_device(ctx);
        run_diagnostics(n, pos, vel, mass, force, out, ctx, (hipStream_t)stream);
    });
}

int tfmm_momentum_diagnostics_noalloc(tfmm_ctx* ctx, int64_t n, const double* pos, const double* vel,
                                      const double* mass, const double* force, double* out, void* stream) {
    if (!ctx) return TFMM_EINVAL;
    return guarded(ctx, [&] {
        if (n < 1 || n > kNoAllocMaxN)
            fail(TFMM_EINVAL, "n must be in 1..2^30 (the allocation-free diagnostics' limit)");
        if (!pos || !mass || !force || !out) fail(TFMM_EINVAL, "bad diagnostics arguments");
        set_device(ctx);
        run_diagnostics_noalloc(n, pos, vel, mass, force, out, ctx->device, (hipStream_t)stream);
    });
}

int tfmm_tree_info(const tfmm_tree* tree, int64_t* out) {
    if (!tree || !out) return TFMM_EINVAL;
    // the near-interaction count is computed on the first request after a walk
    Tree& t = const_cast<Tree&>(*static_cast<const Tree*>(tree));
    return guarded(t.ctx, [&] {
        set_device(t.ctx);
        out[0] = t.n;
        out[1] = t.n_nodes;
        out[2] = t.n_leaves;
        out[3] = t.max_level;
        out[4] = t.walk_valid ? t.n_m2l : -1;
        out[5] = t.walk_valid ? t.n_p2p : -1;
        out[6] = t.walk_valid ? near_interactions(t) : -1;
        out[7] = t.walk_valid ? 2 * t.n_m2l : -1;
    });
}

int tfmm_tree_export(tfmm_tree* tree, uint64_t* keys, int32_t* order, int32_t* level, uint64_t* prefix,
                     int32_t* first, int32_t* count, int32_t* child_first, int32_t* nchild, int32_t* parent,
                     double* com, double* mass, double* rmax) {
    if (!tree) return TFMM_EINVAL;
    return guarded(tree->ctx, [&] {
        Tree& t = *tree;
        set_device(t.ctx);
        TFMM_HIP(hipDeviceSynchronize());
        const size_t n = (size_t)t.n, nn = (size_t)t.n_nodes;
        if (keys || order) {
            std::vector<uint64_t> sk(n);
            std::vector<int32_t> pm(n);
            TFMM_HIP(hipMemcpy(sk.data(), t.keys.p, n * 8, hipMemcpyDeviceToHost));
            TFMM_HIP(hipMemcpy(pm.data(), t.perm.p, n * 4, hipMemcpyDeviceToHost));
            if (order) std::memcpy(order, pm.data(), n * 4);
            if (keys)
                for (size_t j = 0; j < n; ++j) keys[pm[j]] = sk[j];
        }
        if (level) TFMM_HIP(hipMemcpy(level, t.nd_level.p, nn * 4, hipMemcpyDeviceToHost));
        if (prefix) TFMM_HIP(hipMemcpy(prefix, t.nd_prefix.p, nn * 8, hipMemcpyDeviceToHost));
        if (first) TFMM_HIP(hipMemcpy(first, t.nd_first.p, nn * 4, hipMemcpyDeviceToHost));
        if (count) TFMM_HIP(hipMemcpy(count, t.nd_count.p, nn * 4, hipMemcpyDeviceToHost));
        if (child_first) TFMM_HIP(hipMemcpy(child_first, t.nd_child_first.p, nn * 4, hipMemcpyDeviceToHost));
        if (nchild) TFMM_HIP(hipMemcpy(nchild, t.nd_nchild.p, nn * 4, hipMemcpyDeviceToHost));
        if (parent) TFMM_HIP(hipMemcpy(parent, t.nd_parent.p, nn * 4, hipMemcpyDeviceToHost));
        if (rmax) TFMM_HIP(hipMemcpy(rmax, t.nd_rmax.p, nn * 8, hipMemcpyDeviceToHost));
        if (com || mass) {
            std::vector<double> z(nn * 4);
            TFMM_HIP(hipMemcpy(z.data(), t.nd_Z.p, nn * 32, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < nn; ++i) {
                if (com)
                    for (int d = 0; d < 3; ++d) com[3 * i + d] = z[4 * i + d];
                if (mass) mass[i] = z[4 * i + 3];
            }
        }
    });
}

int tfmm_lists_export(tfmm_tree* tree, int32_t* m2l_pairs, int32_t* p2p_pairs) {
    if (!tree) return TFMM_EINVAL;
    return guarded(tree->ctx, [&] {
        Tree& t = *tree;
        if (!t.walk_valid) fail(TFMM_ESTATE, "no walk has been run on this tree");
        set_device(t.ctx);
        TFMM_HIP(hipDeviceSynchronize());
        if (m2l_pairs && t.n_m2l > 0)
            TFMM_HIP(hipMemcpy(m2l_pairs, t.m2l_pairs.p, (size_t)t.n_m2l * 8, hipMemcpyDeviceToHost));
        if (p2p_pairs && t.n_p2p > 0)
            TFMM_HIP(hipMemcpy(p2p_pairs, t.p2p_pairs.p, (size_t)t.n_p2p * 8, hipMemcpyDeviceToHost));
    });
}

int tfmm_tree_destroy(tfmm_tree* tree) {
    if (!tree) return TFMM_OK;
    Ctx* ctx = tree->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (tree->ev_ready)
        for (auto& e : tree->ev) (void)hipEventDestroy(e);
    if (tree->aux) {
        (void)hipEventDestroy(tree->fork_ev);
        (void)hipEventDestroy(tree->join_ev);
        (void)hipStreamDestroy(tree->aux);
    }
    if (tree->stage) {
        (void)hipEventDestroy(tree->stage_ev);
        (void)hipHostFree(tree->stage);
    }
    // the device is idle: the tree's buffers go to the context's cache directly
    ctx->idle_release = true;
    delete tree;
    ctx->idle_release = false;
    ctx->live_trees--;
    return TFMM_OK;
}

size_t tfmm_footprint_bytes(int64_t n, int p, int n_leaf, int precision) {
    if (n < 1 || p < 1 || p > kMaxP || n_leaf < 1) return 0;
    const double nn = 4.0 * (double)n / (double)n_leaf + 1024.0;  // nodes (generous)
    const double nc = c_le(p), ncp = (double)round_up(c_le(p), 4), nloc = 4.0 * c_le(p - 1) + nc;
    double b = 0;
    b += (double)n * (8 + 8 + 4 + 4 + 1 + 4 + 8 + 32 + 4 + (precision == TFMM_MIXED32 ? 16 : 32) + 24 + 24);
    b += nn * (4 * 6 + 8 + 32 + 32 + 8 + 8 + 4);
    b += nn * (nc * 8 + ncp * 12 + 2 * nloc * 8);
    b += nn * (400.0 * 8 * 2 + 80.0 * 8 * 2);  // pair lists, directed lists, frontiers
    b += (double)n * 16;                       // scratch
    return (size_t)(b * 1.5) + (64u << 20);
}

int tfmm_tree_set_timing(tfmm_tree* tree, int enable) {
    if (!tree) return TFMM_EINVAL;
    return guarded(tree->ctx, [&] {
        Tree& t = *tree;
        if (t.ev_pending) TFMM_HIP(hipEventSynchronize(t.ev[5]));
        if (t.build_pending) TFMM_HIP(hipEventSynchronize(t.ev[10]));
        t.timing = enable != 0;
        t.ev_pending = false;
        t.build_pending = false;
        for (double& v : t.t_sum) v = 0.0;
        t.t_count = t.t_walks = t.t_builds = 0;
    });
}

int tfmm_tree_phase_times(tfmm_tree* tree, double* out) {
    if (!tree || !out) return TFMM_EINVAL;
    return guarded(tree->ctx, [&] {
        Tree& t = *tree;
        fold_times(t);
        fold_build(t);
        if (t.t_count == 0) fail(TFMM_ESTATE, "no timed evaluation on this tree");
        for (int k = 0; k < 6; ++k) out[k] = t.t_sum[k] / (double)t.t_count;
        out[6] = t.t_builds ? t.t_sum[6] / (double)t.t_builds : 0.0;
        out[7] = t.t_walks ? t.t_sum[7] / (double)t.t_walks : 0.0;
        out[8] = t.t_walks ? t.t_sum[8] / (double)t.t_walks : 0.0;
        out[9] = t.t_sum[9] / (double)t.t_count;
    });
}

}  // extern "C"
