// Batched factorisation: many polynomials of uneven degree in one call.
//
// Host roots/weights run on a thread pool (largest degree first) while the
// device thread queues each ready polynomial's search back-to-back on one
// stream: no host synchronisation between searches, one workspace reused in
// stream order, and per-search candidate regions copied back with one small
// asynchronous copy each.  After a wave of searches completes, candidates are
// confirmed on the thread pool.
#include <algorithm>
#include <atomic>
#include <numeric>
#include <thread>

#include "rfr_ctx.h"

namespace rfr {

constexpr int WAVE = 256;          // searches queued per synchronisation
constexpr uint64_t BCAP = 1024;    // candidate patterns per search in a wave
constexpr uint64_t HEAD = 64;      // candidate pairs copied back with the count
constexpr size_t REGION = 8 + 2 * BCAP * 8;

struct BatchState {
    char *dev = nullptr;   // WAVE regions: [count][2*BCAP candidates]
    char *host = nullptr;  // pinned mirror
};

void batch_release(rfr_ctx *ctx) {
    if (!ctx->batch) return;
    if (ctx->batch->dev) (void)hipFree(ctx->batch->dev);
    if (ctx->batch->host) (void)hipHostFree(ctx->batch->host);
    delete ctx->batch;
    ctx->batch = nullptr;
}

static rfr_status batch_init(rfr_ctx *ctx) {
    if (ctx->batch) return RFR_OK;
    BatchState *b = new BatchState();
    if (hipMalloc(&b->dev, WAVE * REGION) != hipSuccess ||
        hipHostMalloc(&b->host, WAVE * REGION, hipHostMallocDefault) != hipSuccess) {
        ctx->batch = b;
        batch_release(ctx);
        return fail(RFR_ENOMEM, "batch candidate buffers");
    }
    ctx->batch = b;
    return RFR_OK;
}

// Profiling: events of one search, and accumulation after it completed.
StageEvents *profile_events(rfr_ctx *ctx, int k) {
    if (!ctx->profiling) return nullptr;
    if ((int)ctx->prof_ev.size() < (k + 1) * 7) {
        size_t old = ctx->prof_ev.size();
        ctx->prof_ev.resize((k + 1) * 7, nullptr);
        for (size_t i = old; i < ctx->prof_ev.size(); ++i) (void)hipEventCreate(&ctx->prof_ev[i]);
        ctx->prof_se.resize(k + 1);
    }
    StageEvents &se = ctx->prof_se[k];
    for (int i = 0; i < 7; ++i) se.ev[i] = ctx->prof_ev[k * 7 + i];
    return &se;
}

void profile_collect(rfr_ctx *ctx, int k, int n) {
    if (!ctx->profiling || k >= (int)ctx->prof_se.size()) return;
    StageEvents &se = ctx->prof_se[k];
    for (int i = 0; i < 6; ++i) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, (hipEvent_t)se.ev[i], (hipEvent_t)se.ev[i + 1]) == hipSuccess)
            ctx->prof.stage_ms[i] += ms;
    }
    int na, nb;
    split_halves(n, na, nb);
    ctx->prof.searches += 1;
    ctx->prof.keys += (1ull << na) + (1ull << nb);
}

}  // namespace rfr

using namespace rfr;

extern "C" rfr_status rfr_factor_batch(rfr_ctx *ctx, int count, const int64_t *coeffs, const int32_t *degrees,
                                       rfr_result **out, rfr_status *status) {
    if (!ctx || count < 0 || (count > 0 && (!coeffs || !degrees || !out || !status)))
        return fail(RFR_EINVAL, "bad batch arguments");
    if (count == 0) return RFR_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(RFR_EDEVICE, "hipSetDevice failed");
    std::vector<size_t> off(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        if (degrees[i] < 1 || degrees[i] > RFR_MAX_DEGREE) return fail(RFR_EINVAL, "degree out of range");
        off[i + 1] = off[i] + (size_t)degrees[i] + 1;
    }
    rfr_status bst = batch_init(ctx);
    if (bst != RFR_OK) return bst;
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return degrees[a] > degrees[b]; });

    std::vector<Prepared> P(count);
    std::vector<rfr_status> st(count, RFR_OK);
    std::vector<std::string> err(count);
    std::vector<std::atomic<int>> ready(count);
    for (auto &r : ready) r.store(0);
    std::vector<std::vector<Pat>> cands(count);

    const int nthreads = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
    std::atomic<int> next{0};
    auto prep_work = [&]() {
        for (;;) {
            int k = next.fetch_add(1);
            if (k >= count) break;
            int i = order[k];
            st[i] = prepare(coeffs + off[i], degrees[i], P[i], err[i]);
            ready[i].store(1, std::memory_order_release);
        }
    };
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t) pool.emplace_back(prep_work);

    Slot &s = ctx->main;
    BatchState *B = ctx->batch;
    rfr_status dev_st = RFR_OK;
    std::vector<int> wave;
    for (int w0 = 0; w0 < count && dev_st == RFR_OK; w0 += WAVE) {
        wave.clear();
        const int w1 = std::min(count, w0 + WAVE);
        for (int k = w0; k < w1; ++k) {
            const int i = order[k];
            while (!ready[i].load(std::memory_order_acquire)) std::this_thread::yield();
            if (st[i] != RFR_OK || P[i].n <= 1) continue;
            if (P[i].n > 2 * dev::MAX_HALF + 1) {
                st[i] = RFR_EOVERFLOW;
                err[i] = "too many elements for the search tables";
                continue;
            }
            const size_t need = recombine_workspace(P[i].n);
            if (need > s.ws_bytes) {
                // growing the workspace: earlier searches of this wave still use it
                if (hipStreamSynchronize(s.stream) != hipSuccess) {
                    dev_st = fail(RFR_EDEVICE, "device search failed");
                    break;
                }
                rfr_status e = ensure_workspace(ctx, s, need);
                if (e != RFR_OK) {
                    st[i] = e;
                    err[i] = g_last_error;
                    continue;
                }
            }
            const int slot = (int)wave.size();
            char *dreg = B->dev + (size_t)slot * REGION;
            std::string e2;
            rfr_status e = enqueue_recombine(P[i].w.data(), P[i].n, P[i].t_lo, P[i].t_hi, s.ws, s.ws_bytes,
                                             s.stream, (uint64_t *)(dreg + 8), BCAP, (uint64_t *)dreg,
                                             profile_events(ctx, slot), e2);
            if (e != RFR_OK) {
                st[i] = e;
                err[i] = e2;
                continue;
            }
            if (hipMemcpyAsync(B->host + (size_t)slot * REGION, dreg, 8 + HEAD * 16, hipMemcpyDeviceToHost,
                               s.stream) != hipSuccess) {
                dev_st = fail(RFR_EDEVICE, "candidate copy failed");
                break;
            }
            wave.push_back(i);
        }
        if (dev_st != RFR_OK) break;
        if (hipStreamSynchronize(s.stream) != hipSuccess) {
            dev_st = fail(RFR_EDEVICE, "device search failed");
            break;
        }
        for (int slot = 0; slot < (int)wave.size(); ++slot) {
            const int i = wave[slot];
            profile_collect(ctx, slot, P[i].n);
            char *hreg = B->host + (size_t)slot * REGION;
            uint64_t cnt = *(uint64_t *)hreg;
            if (cnt == ~0ull) {
                // more than a wave region holds: redo with the full capacity
                rfr_status e = search_on_slot(ctx, s, P[i], cands[i]);
                if (e != RFR_OK) {
                    st[i] = e;
                    err[i] = g_last_error;
                }
                continue;
            }
            if (cnt > HEAD) {
                if (hipMemcpy(hreg + 8, B->dev + (size_t)slot * REGION + 8, cnt * 16, hipMemcpyDeviceToHost) !=
                    hipSuccess) {
                    dev_st = fail(RFR_EDEVICE, "candidate copy failed");
                    break;
                }
            }
            const uint64_t *hc = (const uint64_t *)(hreg + 8);
            int na, nb;
            split_halves(P[i].n, na, nb);
            cands[i].resize(cnt);
            for (uint64_t c = 0; c < cnt; ++c) {
                Pat p;
                for (int b = 0; b < na; ++b)
                    if ((hc[2 * c] >> b) & 1) p.set(b);
                for (int b = 0; b < nb; ++b)
                    if ((hc[2 * c + 1] >> b) & 1) p.set(na + b);
                cands[i][c] = p;
            }
        }
    }
    for (auto &t : pool) t.join();
    if (dev_st != RFR_OK) return dev_st;

    // confirmation and packing on the pool
    next.store(0);
    auto conf_work = [&]() {
        for (;;) {
            int k = next.fetch_add(1);
            if (k >= count) break;
            int i = order[k];
            out[i] = nullptr;
            if (st[i] == RFR_OK) {
                Factored F;
                if (P[i].n <= 1) trivial_factor(P[i], F);
                else st[i] = confirm_and_factor(P[i], cands[i], F, err[i]);
                if (st[i] == RFR_OK) {
                    out[i] = pack_result(P[i], F);
                    if (!out[i]) st[i] = RFR_ENOMEM;
                }
            }
            status[i] = st[i];
        }
    };
    pool.clear();
    for (int t = 0; t < nthreads; ++t) pool.emplace_back(conf_work);
    for (auto &t : pool) t.join();
    for (int i = 0; i < count; ++i)
        if (status[i] != RFR_OK && !err[i].empty()) g_last_error = err[i];
    return RFR_OK;
}

extern "C" rfr_status rfr_profile(rfr_ctx *ctx, int enable) {
    if (!ctx) return fail(RFR_EINVAL, "ctx is NULL");
    ctx->profiling = enable != 0;
    if (enable) ctx->prof = rfr_profile_t{};
    return RFR_OK;
}

extern "C" rfr_status rfr_profile_read(rfr_ctx *ctx, rfr_profile_t *out) {
    if (!ctx || !out) return fail(RFR_EINVAL, "NULL argument");
    *out = ctx->prof;
    return RFR_OK;
}
