// Serving loop: continuous batching of factorisation requests.
//
// Host worker threads take requests as they arrive, compute roots and weights,
// and then ask for a device slot.  A request is admitted when a slot is free
// and the bytes of its search tables fit the memory budget together with the
// tables of the requests already on the device; otherwise it waits until a
// running request releases its slot.  Searches that fill the GPU run one at a
// time on one stream; all other device work runs on a second stream beside
// them, so newly arrived small requests are admitted and finished while a big
// search runs.  Results are the same as rfr_factor's: every stage is
// deterministic per polynomial.
#include <algorithm>
#include <cstring>

#include "rfr_ctx.h"

namespace rfr {

// A search with a half of at least 2^BIG_HALF keys fills the GPU by itself:
// two of them side by side would each take about twice as long, so such
// searches run one at a time, all on slot 0, whose workspace is theirs alone
// and only grows (the largest tables are allocated once, not traded back and
// forth).  Smaller searches take the other slots and run beside them and
// each other.
constexpr int BIG_HALF = 23;

// Workspace of every small slot, allocated when serving starts: the largest
// search below BIG_HALF fits it, so no small slot ever reallocates (hipFree
// waits for the whole device, big searches included).
static size_t small_workspace() { return recombine_workspace(2 * (BIG_HALF - 1) + 1); }

// Slot 0 for a big search, growing its workspace to `need` (within the
// budget, trading idle small workspaces if the budget requires); blocks while
// another big search runs.  The allocation itself runs outside the lock.
static Slot *acquire_big(rfr_ctx *ctx, size_t need, rfr_status &st) {
    std::unique_lock<std::mutex> lk(ctx->mu);
    Slot *s = &ctx->slots[0];
    while (s->busy) ctx->cv_slot.wait(lk);
    s->busy = true;
    ++ctx->big_running;
    if (s->ws_bytes >= need) {
        st = RFR_OK;
        return s;
    }
    // grow by at least a factor of two (within the budget), so that a run of
    // ever larger requests reallocates only a few times
    const size_t room = ctx->budget - (ctx->mem_used - s->ws_bytes);
    if (need < room) need = std::min(room, std::max(need, 2 * s->ws_bytes));
    const size_t extra = need - s->ws_bytes;
    for (size_t k = 1; k < ctx->slots.size() && ctx->mem_used + extra > ctx->budget; ++k) {
        Slot &t = ctx->slots[k];
        if (!t.busy && t.ws) {
            (void)hipFree(t.ws);
            ctx->mem_used -= t.ws_bytes;
            t.ws = nullptr;
            t.ws_bytes = 0;
        }
    }
    if (ctx->mem_used + extra > ctx->budget) {
        s->busy = false;
        --ctx->big_running;
        st = fail(RFR_ENOMEM, "request tables do not fit the free memory budget");
        return nullptr;
    }
    ctx->mem_used += extra;  // reserved; the old workspace is released below
    void *old = s->ws;
    s->ws = nullptr;
    s->ws_bytes = 0;
    lk.unlock();
    if (old) (void)hipFree(old);
    void *p = nullptr;
    const bool ok = hipMalloc(&p, need) == hipSuccess;
    lk.lock();
    if (!ok) {
        ctx->mem_used -= need;
        s->busy = false;
        --ctx->big_running;
        lk.unlock();
        ctx->cv_slot.notify_all();
        st = fail(RFR_ENOMEM, "hipMalloc of a request workspace failed");
        return nullptr;
    }
    s->ws = p;
    s->ws_bytes = need;
    st = RFR_OK;
    return s;
}

// A free small slot (1 .. max_active - 1) with room for `need` workspace
// bytes, growing or trading workspaces of idle small slots within the budget
// left beside slot 0; blocks until possible.
static Slot *acquire_small(rfr_ctx *ctx, size_t need, rfr_status &st) {
    std::unique_lock<std::mutex> lk(ctx->mu);
    if (need > ctx->budget) {
        st = fail(RFR_ENOMEM, "request tables exceed the memory budget");
        return nullptr;
    }
    const size_t n0 = ctx->slots.size() > 1 ? 1 : 0;
    for (;;) {
        Slot *best = nullptr;
        for (size_t k = n0; k < ctx->slots.size(); ++k) {
            Slot &s = ctx->slots[k];
            if (s.busy) continue;
            if (s.ws_bytes >= need && (!best || s.ws_bytes < best->ws_bytes)) best = &s;
        }
        if (!best) {
            for (size_t k = n0; k < ctx->slots.size(); ++k) {
                Slot &s = ctx->slots[k];
                if (!s.busy && (!best || s.ws_bytes > best->ws_bytes)) best = &s;
            }
            if (best) {
                size_t extra = need - best->ws_bytes;
                if (ctx->mem_used + extra > ctx->budget) {
                    // trade: release idle small workspaces until it fits
                    for (size_t k = n0; k < ctx->slots.size(); ++k) {
                        Slot &s = ctx->slots[k];
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

static Slot *acquire_slot(rfr_ctx *ctx, size_t need, bool big, rfr_status &st) {
    return big ? acquire_big(ctx, need, st) : acquire_small(ctx, need, st);
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
        if (P.n > dev::MAX_SEARCH_N) {
            st = fail(RFR_EOVERFLOW, "too many elements for the search tables");
        } else {
            // admission size: the full tables, or a chunked layout (half A
            // streamed) when the full tables would not fit the budget left
            // beside the small searches' slots
            int na, nb;
            split_halves(P.n, na, nb);
            const bool big = na >= BIG_HALF && ctx->slots.size() > 1;
            const size_t small_room = (ctx->slots.size() - 1) * recombine_workspace(2 * (BIG_HALF - 1) + 1);
            const size_t room = big && ctx->budget > 2 * small_room ? ctx->budget - small_room : ctx->budget / 2;
            size_t need = recombine_workspace(P.n);
            if (need > room) need = choose_workspace(P.n, room);
            Slot *s = need ? acquire_slot(ctx, need, big, st) : nullptr;
            if (!need) st = fail(RFR_ENOMEM, "request tables do not fit the memory budget");
            if (s) {
                t1 = now_ms();
                st = search_on_slot(ctx, *s, P, cands, &F.trace_folded);
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
    if (rootbuf_init(rb, ctx->lane_small) != RFR_OK) rootbuf_free(rb);
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
    // the plain path's workspace (as large as the largest search it ran)
    // becomes slot 0's, and goes back when serving stops: allocating tens of
    // GB takes long, so the largest tables are allocated once per context
    void *keep_ws = ctx->main.ws;
    const size_t keep_bytes = ctx->main.ws_bytes;
    ctx->main.ws = nullptr;
    ctx->main.ws_bytes = 0;
    // Two device lanes: the searches that fill the GPU (slot 0) on one stream,
    // everything else (roots, smaller searches) on the other, created one
    // after the other so that they sit on different hardware queues.  A
    // stream of its own per slot would let a small request's kernels queue
    // behind a big search's long kernels on a shared hardware queue.
    if (hipStreamCreateWithFlags(&ctx->lane_big, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->lane_small, hipStreamNonBlocking) != hipSuccess) {
        if (ctx->lane_big) (void)hipStreamDestroy(ctx->lane_big);
        ctx->lane_big = ctx->lane_small = nullptr;
        return fail(RFR_EDEVICE, "hipStreamCreate failed");
    }
    ctx->slots.assign(max_active, Slot());
    ctx->slots[0].ws = keep_ws;
    ctx->slots[0].ws_bytes = keep_bytes;
    for (size_t k = 0; k < ctx->slots.size(); ++k) {
        rfr_status st = slot_init(ctx, ctx->slots[k], k == 0 && max_active > 1 ? ctx->lane_big : ctx->lane_small);
        if (st != RFR_OK) {
            for (auto &t : ctx->slots) slot_free(ctx, t);
            ctx->slots.clear();
            (void)hipStreamDestroy(ctx->lane_big);
            (void)hipStreamDestroy(ctx->lane_small);
            ctx->lane_big = ctx->lane_small = nullptr;
            return st;
        }
    }
    if (max_active > 1) {
        const size_t w = small_workspace();
        for (size_t k = 1; k < ctx->slots.size(); ++k) {
            rfr_status st = ensure_workspace(ctx, ctx->slots[k], w);
            if (st != RFR_OK) {
                for (auto &t : ctx->slots) slot_free(ctx, t);
                ctx->slots.clear();
                (void)hipStreamDestroy(ctx->lane_big);
                (void)hipStreamDestroy(ctx->lane_small);
                ctx->lane_big = ctx->lane_small = nullptr;
                return st;
            }
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
    // slot 0's workspace (the largest) goes back to the plain path
    if (!ctx->slots.empty() && !ctx->main.ws) {
        ctx->main.ws = ctx->slots[0].ws;
        ctx->main.ws_bytes = ctx->slots[0].ws_bytes;
        ctx->slots[0].ws = nullptr;
        ctx->slots[0].ws_bytes = 0;
    }
    for (auto &s : ctx->slots) slot_free(ctx, s);
    ctx->slots.clear();
    if (ctx->lane_big) (void)hipStreamDestroy(ctx->lane_big);
    if (ctx->lane_small) (void)hipStreamDestroy(ctx->lane_small);
    ctx->lane_big = ctx->lane_small = nullptr;
    for (auto &kv : ctx->reqs) {
        rfr_result_free(kv.second->result);
        delete kv.second;
    }
    ctx->reqs.clear();
    ctx->serving = false;
    return RFR_OK;
}

}  // extern "C"
