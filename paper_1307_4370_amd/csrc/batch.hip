// Batched SDMM over many channels (observations or frequency channels) of
// uneven image and visibility sizes, and the gridding-tile autotuner.
//
// Each channel has its own plan.  The SDMM iterations of all channels are
// captured once into one HIP graph: a fork event on the caller's stream, one
// branch per channel on its own stream (default priority) running
// riop_sdmm_step, and a join back onto the caller's stream.  Replaying the
// graph runs every channel's iterations as one launch; the channels' kernels
// overlap on the GPU, so small channels no longer leave most of the 256
// compute units idle, and the per-kernel launch cost disappears.
//
// Autotuner: for each channel, every admissible gridding tile side is tried on
// a plan of that channel; Phi / Phi^dagger pairs (plan order) are timed with
// HIP events and the fastest tile's plan is kept.  Results are cached per
// (n, M, J, precision) for the life of the process.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "common.hpp"

struct riop_batch {
    std::vector<riop_plan *> plans;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
    hipStream_t cap = nullptr;          // stream the graph is captured on and launched from
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t exec = nullptr;
    int exec_iters = 0;
    std::vector<uint64_t> exec_epoch;  // each channel's SDMM workspace epoch at capture
    std::vector<int> tile;
    std::vector<std::vector<double>> tile_ms;  // per channel: ms per pair for tiles 8, 16, 32, 64
};

namespace riop {

static const int kTiles[4] = {8, 16, 32, 64};

static std::mutex g_tune_mu;
// Keyed by (n, M, J, precision, hash of the coverage): channels of one shape
// but different (u, v) get their own tile choice.
static std::map<std::tuple<int, int64_t, int, int, uint64_t>, std::pair<int, std::vector<double>>> g_tune_cache;

// 64-bit FNV-1a hash of the coverage's bytes (copied to the host once per
// tuned channel; the timing runs that follow cost far more).
static uint64_t coverage_hash(const riop_desc &d, const void *uv, hipStream_t s) {
    const size_t bytes = (size_t)d.M * 2 * (d.prec == RIOP_F64 ? 8 : 4);
    std::vector<unsigned char> h(bytes);
    if (bytes) {
        RIOP_HIP(hipMemcpyAsync(h.data(), uv, bytes, hipMemcpyDeviceToHost, s));
        RIOP_HIP(hipStreamSynchronize(s));
    }
    uint64_t x = 1469598103934665603ull;
    for (unsigned char c : h) x = (x ^ c) * 1099511628211ull;
    return x;
}

static double time_pairs(riop_plan *p, int reps, hipStream_t s) {
    DevBuf x, y;
    const size_t cb = cbytes(p);
    x.alloc(cb * (size_t)p->n * p->n);
    y.alloc(cb * (size_t)std::max<int64_t>(1, p->M));
    RIOP_HIP(hipMemsetAsync(x.ptr, 0, cb * (size_t)p->n * p->n, s));
    hipEvent_t a, b;
    RIOP_HIP(hipEventCreate(&a));
    RIOP_HIP(hipEventCreate(&b));
    auto pair = [&] {
        if (p->prec == RIOP_F64) {
            launch_phi_fft_forward<double>(p, x.ptr, s);
            launch_degrid<double>(p, y.ptr, 0, s);
            launch_grid<double>(p, y.ptr, 0, s);
            launch_phi_fft_adjoint<double>(p, x.ptr, s);
        } else {
            launch_phi_fft_forward<float>(p, x.ptr, s);
            launch_degrid<float>(p, y.ptr, 0, s);
            launch_grid<float>(p, y.ptr, 0, s);
            launch_phi_fft_adjoint<float>(p, x.ptr, s);
        }
    };
    pair();
    RIOP_HIP(hipEventRecord(a, s));
    for (int r = 0; r < reps; ++r) pair();
    RIOP_HIP(hipEventRecord(b, s));
    RIOP_HIP(hipEventSynchronize(b));
    float ms = 0;
    RIOP_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

// Returns the plan with the fastest tile; fills ms[4] (negative where not tried).
static riop_plan *tuned_plan(const riop_desc &d0, const void *uv, int reps, hipStream_t s, int *best_tile,
                             std::vector<double> &ms) {
    ms.assign(4, -1.0);
    const auto key = std::make_tuple(d0.n, d0.M, d0.J, (int)d0.prec, coverage_hash(d0, uv, s));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            riop_desc d = d0;
            d.tile = it->second.first;
            riop_plan *p = nullptr;
            riop_status st = riop_plan_create(&d, uv, s, &p);
            if (st != RIOP_OK) throw Error{st, riop_last_error()};
            *best_tile = d.tile;
            ms = it->second.second;
            return p;
        }
    }
    riop_plan *best = nullptr;
    double best_ms = 0;
    for (int i = 0; i < 4; ++i) {
        const int t = kTiles[i];
        const int K = 2 * d0.n;
        if (K % t || t < d0.J || (K / t) * (K / t) > 16384) continue;
        riop_desc d = d0;
        d.tile = t;
        riop_plan *p = nullptr;
        riop_status st = riop_plan_create(&d, uv, s, &p);
        if (st == RIOP_ENOTSUP) continue;  // e.g. the tile's gridding region does not fit in LDS
        if (st != RIOP_OK) throw Error{st, riop_last_error()};
        double m;
        try {
            m = time_pairs(p, reps, s);
        } catch (...) {
            riop_plan_destroy(p);
            if (best) riop_plan_destroy(best);
            throw;
        }
        ms[i] = m;
        if (!best || m < best_ms) {
            if (best) riop_plan_destroy(best);
            best = p;
            best_ms = m;
            *best_tile = t;
        } else {
            riop_plan_destroy(p);
        }
    }
    RIOP_REQUIRE(best, RIOP_ENOTSUP, "no admissible gridding tile");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {*best_tile, ms};
    return best;
}

template <typename F> static riop_status guarded3(F &&f) {
    try {
        clear_error();
        f();
        return RIOP_OK;
    } catch (const Error &e) {
        set_error("%s", e.msg.c_str());
        return e.status;
    } catch (...) {
        set_error("unexpected failure");
        return RIOP_EDEVICE;
    }
}

static void destroy_batch(riop_batch *b) {
    if (!b) return;
    // Wait for the batch's own streams (graph launches, channel branches).
    if (b->cap) (void)hipStreamSynchronize(b->cap);
    for (hipStream_t st : b->streams) (void)hipStreamSynchronize(st);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    for (hipEvent_t e : b->joins) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
    for (riop_plan *p : b->plans) riop_plan_destroy(p);
    delete b;
}

}  // namespace riop

using namespace riop;

extern "C" {

riop_status riop_autotune_tile(const riop_desc *desc, const void *uv, int32_t reps, void *stream, int32_t *best_tile,
                               double *pair_ms) {
    return guarded3([&] {
        RIOP_REQUIRE(desc && best_tile, RIOP_EINVAL, "NULL argument");
        RIOP_REQUIRE(reps >= 1, RIOP_EINVAL, "reps must be >= 1");
        std::vector<double> ms;
        int t = 0;
        riop_plan *p = tuned_plan(*desc, uv, reps, static_cast<hipStream_t>(stream), &t, ms);
        riop_plan_destroy(p);
        *best_tile = t;
        if (pair_ms) std::copy(ms.begin(), ms.end(), pair_ms);
    });
}

riop_status riop_batch_create(const riop_desc *descs, int32_t nchannels, const void *const *uv, int32_t autotune,
                              void *stream, riop_batch **out) {
    if (!out) {
        set_error("out is NULL");
        return RIOP_EINVAL;
    }
    *out = nullptr;
    riop_batch *b = nullptr;
    riop_status st = guarded3([&] {
        RIOP_REQUIRE(descs && uv && nchannels >= 1, RIOP_EINVAL, "need at least one channel");
        b = new riop_batch();
        const hipStream_t s = static_cast<hipStream_t>(stream);
        for (int c = 0; c < nchannels; ++c) {
            riop_plan *p = nullptr;
            std::vector<double> ms(4, -1.0);
            int t = 0;
            if (autotune) {
                p = tuned_plan(descs[c], uv[c], 3, s, &t, ms);
            } else {
                riop_status e = riop_plan_create(&descs[c], uv[c], stream, &p);
                if (e != RIOP_OK) throw Error{e, riop_last_error()};
                t = p->tile;
            }
            b->plans.push_back(p);
            b->tile.push_back(t);
            b->tile_ms.push_back(ms);
            hipStream_t cs;
            RIOP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            b->streams.push_back(cs);
            hipEvent_t e;
            RIOP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            b->joins.push_back(e);
        }
        RIOP_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        RIOP_HIP(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
        RIOP_HIP(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
        RIOP_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    });
    if (st != RIOP_OK) {
        destroy_batch(b);
        return st;
    }
    *out = b;
    return RIOP_OK;
}

riop_status riop_batch_plan(riop_batch *b, int32_t channel, riop_plan **plan) {
    return guarded3([&] {
        RIOP_REQUIRE(b && plan && channel >= 0 && channel < (int)b->plans.size(), RIOP_EINVAL, "bad channel");
        *plan = b->plans[channel];
    });
}

riop_status riop_batch_tile(const riop_batch *b, int32_t channel, int32_t *tile, double *pair_ms) {
    return guarded3([&] {
        RIOP_REQUIRE(b && channel >= 0 && channel < (int)b->plans.size(), RIOP_EINVAL, "bad channel");
        if (tile) *tile = b->tile[channel];
        if (pair_ms) std::copy(b->tile_ms[channel].begin(), b->tile_ms[channel].end(), pair_ms);
    });
}

riop_status riop_batch_sdmm(riop_batch *b, const void *const *y, const double *eps, const riop_sdmm_params *prm,
                            int32_t iters_per_graph, void *const *x_out, riop_sdmm_stats *stats, void *stream) {
    return guarded3([&] {
        RIOP_REQUIRE(b && y && eps && prm, RIOP_EINVAL, "NULL argument");
        RIOP_REQUIRE(iters_per_graph >= 1, RIOP_EINVAL, "iters_per_graph must be >= 1");
        RIOP_REQUIRE(!prm->resume && !prm->early_stop, RIOP_ENOTSUP, "batched SDMM starts fresh, no early stop");
        RIOP_REQUIRE(!prm->z1 && !prm->z2 && !prm->z3 && !prm->rhs && !prm->weights && !prm->history,
                     RIOP_ENOTSUP, "batched SDMM takes no per-channel state, weights or history pointers");
        const hipStream_t s = static_cast<hipStream_t>(stream);
        const int nc = (int)b->plans.size();
        for (int c = 0; c < nc; ++c) {
            riop_status e = riop_sdmm_init(b->plans[c], y[c], eps[c], prm, nullptr, stream);
            if (e != RIOP_OK) throw Error{e, riop_last_error()};
        }
        const int T = std::max(0, prm->T);
        const int ipg = std::min(iters_per_graph, std::max(1, T));
        // The caller's stream may be the null stream, which cannot be captured:
        // the graph lives on the batch's own stream, joined by events.
        const hipStream_t cs = b->cap;
        RIOP_HIP(hipEventRecord(b->ev_in, s));
        RIOP_HIP(hipStreamWaitEvent(cs, b->ev_in, 0));
        auto enqueue_all = [&](int iters) {
            RIOP_HIP(hipEventRecord(b->fork, cs));
            for (int c = 0; c < nc; ++c) {
                RIOP_HIP(hipStreamWaitEvent(b->streams[c], b->fork, 0));
                riop_status e = riop_sdmm_step(b->plans[c], iters, b->streams[c]);
                if (e != RIOP_OK) throw Error{e, riop_last_error()};
                RIOP_HIP(hipEventRecord(b->joins[c], b->streams[c]));
                RIOP_HIP(hipStreamWaitEvent(cs, b->joins[c], 0));
            }
        };
        // Capture again when the iteration count per graph changed or any
        // channel's captured workspace state did (history buffer address,
        // n_cg, cg_tol, weights: riop_sdmm_init moves the epoch then).
        bool stale = !b->exec || b->exec_iters != ipg || (int)b->exec_epoch.size() != nc;
        for (int c = 0; c < nc && !stale; ++c) stale = b->exec_epoch[c] != b->plans[c]->sd.epoch;
        if (T >= ipg && stale) {
            if (b->exec) {
                RIOP_HIP(hipGraphExecDestroy(b->exec));
                b->exec = nullptr;
            }
            hipGraph_t g = nullptr;
            RIOP_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            try {
                enqueue_all(ipg);
            } catch (...) {
                (void)hipStreamEndCapture(cs, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            RIOP_HIP(hipStreamEndCapture(cs, &g));
            const hipError_t ie = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            RIOP_HIP(ie);
            b->exec_iters = ipg;
            b->exec_epoch.resize(nc);
            for (int c = 0; c < nc; ++c) b->exec_epoch[c] = b->plans[c]->sd.epoch;
        }
        int done = 0;
        while (T - done >= ipg) {
            RIOP_HIP(hipGraphLaunch(b->exec, cs));
            done += ipg;
        }
        if (T > done) enqueue_all(T - done);
        RIOP_HIP(hipEventRecord(b->ev_out, cs));
        RIOP_HIP(hipStreamWaitEvent(s, b->ev_out, 0));
        for (int c = 0; c < nc; ++c) {
            riop_status e = riop_sdmm_finish(b->plans[c], nullptr, x_out ? x_out[c] : nullptr,
                                             stats ? &stats[c] : nullptr, stream);
            if (e != RIOP_OK) throw Error{e, riop_last_error()};
        }
    });
}

riop_status riop_batch_destroy(riop_batch *b) {
    return guarded3([&] { destroy_batch(b); });
}

}  // extern "C"
