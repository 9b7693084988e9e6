// Serving loop: continuous batching of factorisation requests.
//
// Host worker threads take requests as they arrive, compute roots and weights,
// and then ask for a device slot.  A request is admitted when a slot is free
// and the bytes of its search tables fit the memory budget together with the
// tables of the requests already on the device; otherwise it waits until a
// running request releases its slot.  Each slot owns its own HIP stream, so the
// searches of all admitted requests overlap on the GPU while newly arrived
// requests are admitted as soon as slots and memory free up.  Results are the
// same as rfr_factor's: every stage is deterministic per polynomial.
#include <algorithm>
#include <cstring>

#include "rfr_ctx.h"

namespace rfr {

// Pick a free slot with room for `need` workspace bytes (growing or trading
// workspaces of idle slots within the budget); blocks until possible.
// A search with a half of at least 2^BIG_HALF keys fills the GPU by itself:
// two of them side by side would each take about twice as long, so such
// searches are admitted one at a time (smaller ones still run beside them).
constexpr int BIG_HALF = 23;

static Slot *acquire_slot(rfr_ctx *ctx, size_t need, bool big, rfr_status &st) {
    std::unique_lock<std::mutex> lk(ctx->mu);
    if (need > ctx->budget) {
        st = fail(RFR_ENOMEM, "request tables exceed the memory budget");
        return nullptr;
    }
    for (;;) {
        if (big && ctx->big_running > 0) {
            ctx->cv_slot.wait(lk);
            continue;
        }
        Slot *best = nullptr;
        for (auto &s : ctx->slots) {
            if (s.busy) continue;
            if (s.ws_bytes >= need && (!best || s.ws_bytes < best->ws_bytes)) best = &s;
        }
        if (!best) {
            for (auto &s : ctx->slots)
                if (!s.busy && (!best || s.ws_bytes > best->ws_bytes)) best = &s;
            if (best) {
                size_t extra = need - best->ws_bytes;
                if (ctx->mem_used + extra > ctx->budget) {
                    // trade: release idle workspaces until it fits
                    for (auto &s : ctx->slots) {
                        if (ctx->mem_used + extra <= ctx->budget) break;
                        if (!s.busy && &s != best && s.ws) {
                            (void)hipFree(s.ws);
                            ctx->mem_used -= s.ws_bytes;
                            s.ws = nullptr;
                            s.ws_bytes = 0;
                        }
                    }
                }
                if (ctx->mem_used + extra <= ctx->budget) {
                    if (best->ws) {
                        (void)hipFree(best->ws);
                        ctx->mem_used -= best->ws_bytes;
                        best->ws = nullptr;
                        best->ws_bytes = 0;
                    }
                    if (hipMalloc(&best->ws, need) != hipSuccess) {
                        best->ws = nullptr;
                        st = fail(RFR_ENOMEM, "hipMalloc of a request workspace failed");
                        return nullptr;
                    }
                    best->ws_bytes = need;
                    ctx->mem_used += need;
                } else {
                    best = nullptr;
                }
            }
        }
        if (best) {
            best->busy = true;
            if (big) ++ctx->big_running;
            st = RFR_OK;
            return best;
        }
        bool any_busy = false;
        for (auto &s : ctx->slots) any_busy = any_busy || s.busy;
        if (!any_busy) {
            // nothing running will free memory: this request cannot be admitted
            st = fail(RFR_ENOMEM, "request tables do not fit the free memory budget");
            return nullptr;
        }
        ctx->cv_slot.wait(lk);
    }
}

static void release_slot(rfr_ctx *ctx, Slot *s, bool big) {
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        s->busy = false;
        if (big) --ctx->big_running;
    }
    ctx->cv_slot.notify_all();
}

// The square-free path for one polynomial: roots on this worker's stream,
// admission to a device slot, search, confirmation.
static rfr_status serve_poly(rfr_ctx *ctx, RootBuf &rb, const int64_t *coeffs, int degree, rfr_result **out) {
    double t0 = now_ms();
    Prepared P;
    std::string err;
    Factored F;
    std::vector<Pat> cands;
    rfr_result *res = nullptr;
    rfr_status st = prepare_dev(rb, coeffs, degree, P, err);
    if (st == RFR_OK) st = peel_singletons(P, err);
    if (st != RFR_OK) st = fail(st, err);
    double t1 = now_ms(), t2 = t1;
    if (st == RFR_OK && P.n <= 1) {
        trivial_factor(P, F);
    } else if (st == RFR_OK) {
        if (P.n > 2 * dev::MAX_HALF + 1) {
            st = fail(RFR_EOVERFLOW, "too many elements for the search tables");
        } else {
            // admission size: the full tables, or a chunked layout (half A
            // streamed) when the full tables would take over half the budget
            size_t need = recombine_workspace(P.n);
            if (need > ctx->budget / 2) need = choose_workspace(P.n, ctx->budget / 2);
            int na, nb;
            split_halves(P.n, na, nb);
            const bool big = na >= BIG_HALF;
            Slot *s = need ? acquire_slot(ctx, need, big, st) : nullptr;
            if (!need) st = fail(RFR_ENOMEM, "request tables do not fit the memory budget");
            if (s) {
                t1 = now_ms();
                st = search_on_slot(ctx, *s, P, cands);
                release_slot(ctx, s, big);
            }
        }
        t2 = now_ms();
        if (st == RFR_OK) {
            st = confirm_and_factor(P, cands, F, err);
            if (st != RFR_OK) st = fail(st, err);
        }
    }
    if (st == RFR_OK) {
        res = pack_result(P, F);
        if (!res) st = RFR_ENOMEM;
        else {
            res->ms_roots = t1 - t0;
            res->ms_search = t2 - t1;
            res->ms_confirm = now_ms() - t2;
        }
    }
    *out = res;
    return st;
}

static void serve_one(rfr_ctx *ctx, RootBuf &rb, Request *r) {
    const int degree = (int)r->coeffs.size() - 1;
    rfr_result *res = nullptr;
    rfr_status st = serve_poly(ctx, rb, r->coeffs.data(), degree, &res);
    if (st == RFR_ENOTSQFREE)
        st = factor_sqf_route(r->coeffs.data(), degree, [&](const int64_t *c, int d, rfr_result **o) {
            return serve_poly(ctx, rb, c, d, o);
        }, &res);
    std::lock_guard<std::mutex> lk(ctx->mu);
    r->status = st;
    r->result = res;
    r->t_done = now_ms();
}

static void worker_loop(rfr_ctx *ctx) {
    (void)hipSetDevice(ctx->device);
    // roots of this worker's requests are found on the device on a stream of
    // its own (the host finds them if these buffers cannot be had)
    RootBuf rb;
    if (rootbuf_init(rb, nullptr) != RFR_OK) rootbuf_free(rb);
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(ctx->mu);
            ctx->cv_work.wait(lk, [&] { return ctx->stopping || !ctx->queue.empty(); });
            if (ctx->queue.empty()) break;  // stopping and drained
            r = ctx->queue.front();
            ctx->queue.pop_front();
        }
        serve_one(ctx, rb, r);
    }
    rootbuf_free(rb);
}

}  // namespace rfr

using namespace rfr;

extern "C" {

rfr_status rfr_serve_start(rfr_ctx *ctx, int max_active, int host_threads) {
    if (!ctx || max_active < 1 || max_active > 64 || host_threads < 1 || host_threads > 256)
        return fail(RFR_EINVAL, "max_active in [1,64], host_threads in [1,256]");
    if (ctx->serving) return fail(RFR_EBUSY, "already serving");
    (void)hipSetDevice(ctx->device);
    // the serving slots trade workspaces among themselves: hand back the plain
    // path's workspace so its memory is available to admission
    if (ctx->main.ws) {
        (void)hipFree(ctx->main.ws);
        ctx->mem_used -= ctx->main.ws_bytes;
        ctx->main.ws = nullptr;
        ctx->main.ws_bytes = 0;
    }
    ctx->slots.assign(max_active, Slot());
    for (auto &s : ctx->slots) {
        rfr_status st = slot_init(ctx, s);
        if (st != RFR_OK) {
            for (auto &t : ctx->slots) slot_free(ctx, t);
            ctx->slots.clear();
            return st;
        }
    }
    ctx->stopping = false;
    ctx->serving = true;
    for (int i = 0; i < host_threads; ++i) ctx->workers.emplace_back(worker_loop, ctx);
    return RFR_OK;
}

rfr_status rfr_submit(rfr_ctx *ctx, const int64_t *coeffs, int degree, uint64_t *ticket) {
    if (!ctx || !coeffs || !ticket || degree < 1 || degree > RFR_MAX_DEGREE)
        return fail(RFR_EINVAL, "bad request");
    Request *r = new Request();
    r->coeffs.assign(coeffs, coeffs + degree + 1);
    r->t_submit = now_ms();
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!ctx->serving || ctx->stopping) {
            delete r;
            return fail(RFR_EINVAL, "serving loop not running");
        }
        r->ticket = ctx->next_ticket++;
        ctx->reqs[r->ticket] = r;
        ctx->queue.push_back(r);
        *ticket = r->ticket;
    }
    ctx->cv_work.notify_one();
    return RFR_OK;
}

rfr_status rfr_poll(rfr_ctx *ctx, uint64_t ticket, rfr_result **out, double *latency_ms) {
    if (!ctx || !out) return fail(RFR_EINVAL, "NULL argument");
    *out = nullptr;
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->reqs.find(ticket);
    if (it == ctx->reqs.end()) return fail(RFR_EINVAL, "unknown or already collected ticket");
    Request *r = it->second;
    if (r->status == RFR_EBUSY) return RFR_EBUSY;
    rfr_status st = r->status;
    *out = r->result;
    if (latency_ms) *latency_ms = r->t_done - r->t_submit;
    ctx->reqs.erase(it);
    delete r;
    return st;
}

rfr_status rfr_serve_stop(rfr_ctx *ctx) {
    if (!ctx) return fail(RFR_EINVAL, "ctx is NULL");
    if (!ctx->serving) return RFR_OK;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->stopping = true;
    }
    ctx->cv_work.notify_all();
    for (auto &t : ctx->workers) t.join();
    ctx->workers.clear();
    for (auto &s : ctx->slots) slot_free(ctx, s);
    ctx->slots.clear();
    for (auto &kv : ctx->reqs) {
        rfr_result_free(kv.second->result);
        delete kv.second;
    }
    ctx->reqs.clear();
    ctx->serving = false;
    return RFR_OK;
}

}  // extern "C"
