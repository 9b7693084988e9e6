// Serving loop: continuous batching of factorisation requests.
//
// Host worker threads take requests as they arrive, compute roots and weights,
// and then ask for a device slot.  A request is admitted when a slot is free
// and the bytes of its search tables fit the memory budget together with the
// tables of the requests already on the device; otherwise it waits until a
// running request releases its slot.  Searches that fill the GPU run one at a
// time on slot 0 and its stream; all other device work runs on a second
// stream beside them, so newly arrived small requests are admitted and
// finished while a big search runs.  A worker never waits for slot 0: it
// hands such a prepared search to the big-search threads, in arrival order,
// and takes the next request (if workers waited, under overload every one of
// them would end up holding a big request and the small lane would stand
// idle).
// Results are the same as rfr_factor's: every stage is deterministic per
// polynomial.
#include <algorithm>
#include <cstring>

#include "rfr_ctx.h"

namespace rfr {

// A search with a half of at least 2^BIG_HALF keys fills the GPU by itself:
// such searches run one at a time, all on slot 0, whose workspace is theirs
// alone and only grows (the largest tables, tens of GB, are allocated once,
// not traded back and forth: hipMalloc of that much takes long and hipFree
// waits for the whole device).  Smaller searches take the other slots and run
// beside them and each other.
constexpr int BIG_HALF = 23;

// Workspace of every small slot, allocated when serving starts: the largest
// search below BIG_HALF fits it, so no small slot ever reallocates (hipFree
// waits for the whole device, big searches included).
static size_t small_workspace() { return recombine_workspace(2 * (BIG_HALF - 1) + 1); }

static void free_workspace(rfr_ctx *ctx, Slot &t) {
    (void)hipFree(t.ws);
    ctx->mem_used -= t.ws_bytes;
    t.ws = nullptr;
    t.ws_bytes = 0;
}

// Slot 0 for a big search of `need` workspace bytes, growing its workspace
// within the budget (idle small workspaces are released first); waits while
// another big search runs, and while busy small slots hold the memory it
// needs.  Growth is geometric, so that a run of ever larger requests
// reallocates only a few times.  The allocation itself runs outside the lock.
static Slot *acquire_big(rfr_ctx *ctx, size_t need, rfr_status &st) {
    std::unique_lock<std::mutex> lk(ctx->mu);
    Slot *s = &ctx->slots[0];
    auto fits = [&] { return need + (ctx->mem_used - s->ws_bytes) <= ctx->budget; };
    for (;;) {
        while (s->busy) ctx->cv_slot.wait(lk);
        if (s->ws_bytes >= need) break;
        for (size_t j = 1; j < ctx->slots.size() && !fits(); ++j)
            if (!ctx->slots[j].busy && ctx->slots[j].ws) free_workspace(ctx, ctx->slots[j]);
        if (fits()) break;
        bool other_busy = false;
        for (size_t j = 1; j < ctx->slots.size(); ++j) other_busy = other_busy || ctx->slots[j].busy;
        if (!other_busy) {
            st = fail(RFR_ENOMEM, "request tables do not fit the free memory budget");
            return nullptr;
        }
        ctx->cv_slot.wait(lk);  // a running request will release memory
    }
    s->busy = true;
    ++ctx->big_running;
    if (s->ws_bytes >= need) {
        st = RFR_OK;
        return s;
    }
    const size_t room = ctx->budget - (ctx->mem_used - s->ws_bytes);
    const size_t grow = std::min(room, std::max(need, 2 * s->ws_bytes));
    ctx->mem_used += grow - s->ws_bytes;  // reserved; the old workspace is released below
    void *old = s->ws;
    s->ws = nullptr;
    s->ws_bytes = 0;
    lk.unlock();
    if (old) (void)hipFree(old);
    void *p = nullptr;
    const bool ok = hipMalloc(&p, grow) == hipSuccess;
    lk.lock();
    if (!ok) {
        ctx->mem_used -= grow;
        s->busy = false;
        --ctx->big_running;
        lk.unlock();
        ctx->cv_slot.notify_all();
        st = fail(RFR_ENOMEM, "hipMalloc of a request workspace failed");
        return nullptr;
    }
    s->ws = p;
    s->ws_bytes = grow;
    st = RFR_OK;
    return s;
}

// A free small slot (n_big .. max_active - 1) with room for `need` workspace
// bytes, growing or trading workspaces of idle small slots within the budget
// left beside the big slots; blocks until possible.
static Slot *acquire_small(rfr_ctx *ctx, size_t need, rfr_status &st) {
    std::unique_lock<std::mutex> lk(ctx->mu);
    if (need > ctx->budget) {
        st = fail(RFR_ENOMEM, "request tables exceed the memory budget");
        return nullptr;
    }
    const size_t n0 = (size_t)ctx->n_big;
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

// A square-free request whose search fills the GPU, prepared by a worker and
// waiting for slot 0.
struct BigJob {
    Request *r = nullptr;
    Prepared P;
    size_t need = 0;  // workspace bytes of its search
    double t0 = 0;    // when its preparation started
};

// Internal status of serve_poly: the request went to the big-search threads,
// which complete it.
constexpr rfr_status HANDED_OFF = static_cast<rfr_status>(1);  // no public status is positive

// Search (on slot 0 when `big`), confirmation and packing of a prepared
// polynomial; t0 is when its preparation started.
static rfr_status finish_poly(rfr_ctx *ctx, Prepared &P, size_t need, bool big, double t0, rfr_result **out) {
    Factored F;
    std::vector<Pat> cands;
    std::string err;
    rfr_status st = RFR_OK;
    double t1 = now_ms();
    Slot *s = acquire_slot(ctx, need, big, st);
    if (s) {
        t1 = now_ms();
        st = search_on_slot(ctx, *s, P, cands, &F.trace_folded);
        release_slot(ctx, s, big);
    }
    const double t2 = now_ms();
    if (st == RFR_OK) {
        st = confirm_and_factor(P, cands, F, err);
        if (st != RFR_OK) st = fail(st, err);
    }
    rfr_result *res = nullptr;
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

static void complete(rfr_ctx *ctx, Request *r, rfr_status st, rfr_result *res) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    r->status = st;
    r->result = res;
    r->t_done = now_ms();
}

// The square-free path for one polynomial: roots on this worker's stream,
// admission to a device slot, search, confirmation.  With `handoff` (the
// request itself, on its top-level call) a search that fills the GPU is
// queued for the big-search threads instead, and HANDED_OFF is returned.
static rfr_status serve_poly(rfr_ctx *ctx, RootBuf &rb, const int64_t *coeffs, int degree, rfr_result **out,
                             Request *handoff = nullptr) {
    const double t0 = now_ms();
    Prepared P;
    std::string err;
    *out = nullptr;
    rfr_status st = prepare_dev(rb, coeffs, degree, P, err);
    if (st == RFR_OK) st = peel_singletons(P, err);
    if (st != RFR_OK) return fail(st, err);
    if (P.n <= 1) {
        Factored F;
        trivial_factor(P, F);
        rfr_result *res = pack_result(P, F);
        if (!res) return RFR_ENOMEM;
        res->ms_roots = now_ms() - t0;
        *out = res;
        return RFR_OK;
    }
    if (P.n > dev::MAX_SEARCH_N) return fail(RFR_EOVERFLOW, "too many elements for the search tables");
    // admission size: the full tables, or a chunked layout (half A streamed)
    // when the full tables would not fit the budget left beside the small
    // searches' slots
    int na, nb;
    split_halves(P.n, na, nb);
    const bool big = na >= BIG_HALF && ctx->n_big > 0;
    const size_t small_room = (ctx->slots.size() - ctx->n_big) * small_workspace();
    const size_t room = big && ctx->budget > 2 * small_room ? ctx->budget - small_room : ctx->budget / 2;
    size_t need = recombine_workspace(P.n);
    if (need > room) need = choose_workspace(P.n, room);
    if (!need) return fail(RFR_ENOMEM, "request tables do not fit the memory budget");
    if (big && handoff) {
        BigJob *j = new BigJob();
        j->r = handoff;
        j->P = std::move(P);
        j->need = need;
        j->t0 = t0;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->big_jobs.push_back(j);
        }
        ctx->cv_big.notify_one();
        return HANDED_OFF;
    }
    return finish_poly(ctx, P, need, big, t0, out);
}

static void serve_one(rfr_ctx *ctx, RootBuf &rb, Request *r) {
    const int degree = (int)r->coeffs.size() - 1;
    rfr_result *res = nullptr;
    rfr_status st = serve_poly(ctx, rb, r->coeffs.data(), degree, &res, r);
    if (st == HANDED_OFF) return;
    // the square-free parts of a request with repeated factors are served in
    // turn by this worker (a big one waits for slot 0 here)
    if (st == RFR_ENOTSQFREE)
        st = factor_sqf_route(r->coeffs.data(), degree, [&](const int64_t *c, int d, rfr_result **o) {
            return serve_poly(ctx, rb, c, d, o);
        }, &res);
    complete(ctx, r, st, res);
}

// Big-search thread: takes handed-off searches in arrival order and runs
// them on slot 0.  Two of them run, so that one confirms its candidates on
// the host while the other searches.
static void big_loop(rfr_ctx *ctx) {
    (void)hipSetDevice(ctx->device);
    for (;;) {
        BigJob *j = nullptr;
        {
            std::unique_lock<std::mutex> lk(ctx->mu);
            ctx->cv_big.wait(lk, [&] { return ctx->big_stopping || !ctx->big_jobs.empty(); });
            if (ctx->big_jobs.empty()) break;  // stopping and drained
            j = ctx->big_jobs.front();
            ctx->big_jobs.pop_front();
        }
        rfr_result *res = nullptr;
        const rfr_status st = finish_poly(ctx, j->P, j->need, true, j->t0, &res);
        complete(ctx, j->r, st, res);
        delete j;
    }
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
    // Two device lanes: the searches that fill the GPU (slot 0) on one
    // stream, everything else (roots, smaller searches) on the other, created
    // one after the other so that they sit on different hardware queues.  A
    // stream of its own per small slot would let a small request's kernels
    // queue behind a big search's long kernels on a shared hardware queue.
    const int n_big = max_active > 1 ? 1 : 0;
    auto drop_lanes = [&] {
        if (ctx->lane_big) (void)hipStreamDestroy(ctx->lane_big);
        if (ctx->lane_small) (void)hipStreamDestroy(ctx->lane_small);
        ctx->lane_big = ctx->lane_small = nullptr;
    };
    const bool lanes_ok = hipStreamCreateWithFlags(&ctx->lane_big, hipStreamNonBlocking) == hipSuccess &&
                          hipStreamCreateWithFlags(&ctx->lane_small, hipStreamNonBlocking) == hipSuccess;
    if (!lanes_ok) {
        drop_lanes();
        ctx->main.ws = keep_ws;
        ctx->main.ws_bytes = keep_bytes;
        return fail(RFR_EDEVICE, "hipStreamCreate failed");
    }
    ctx->n_big = n_big;
    ctx->slots.assign(max_active, Slot());
    ctx->slots[0].ws = keep_ws;
    ctx->slots[0].ws_bytes = keep_bytes;
    auto undo = [&] {
        for (auto &t : ctx->slots) slot_free(ctx, t);
        ctx->slots.clear();
        ctx->n_big = 0;
        drop_lanes();
    };
    for (size_t k = 0; k < ctx->slots.size(); ++k) {
        rfr_status st = slot_init(ctx, ctx->slots[k], (int)k < n_big ? ctx->lane_big : ctx->lane_small);
        if (st != RFR_OK) {
            undo();
            return st;
        }
    }
    const size_t w = small_workspace();
    for (size_t k = n_big; n_big > 0 && k < ctx->slots.size(); ++k) {
        rfr_status st = ensure_workspace(ctx, ctx->slots[k], w);
        if (st != RFR_OK) {
            undo();
            return st;
        }
    }
    ctx->stopping = false;
    ctx->serving = true;
    ctx->big_stopping = false;
    for (int i = 0; i < host_threads; ++i) ctx->workers.emplace_back(worker_loop, ctx);
    for (int i = 0; i < 2 * n_big; ++i) ctx->big_workers.emplace_back(big_loop, ctx);
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
    // the workers are done handing off: drain the big searches
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->big_stopping = true;
    }
    ctx->cv_big.notify_all();
    for (auto &t : ctx->big_workers) t.join();
    ctx->big_workers.clear();
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
    ctx->n_big = 0;
    for (auto &kv : ctx->reqs) {
        rfr_result_free(kv.second->result);
        delete kv.second;
    }
    ctx->reqs.clear();
    ctx->serving = false;
    return RFR_OK;
}

}  // extern "C"
