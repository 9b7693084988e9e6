// C ABI of the RFR library: contexts, plain factorisation, results, host-stage
// and kernel-level entry points.  Batched and served modes live in
// rfr_batch.cpp and rfr_serve.cpp.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdlib>
#include <cstring>
#include <new>

#include "rfr_ctx.h"
#include "rfr_roots.h"

namespace rfr {

thread_local std::string g_last_error;

rfr_status fail(rfr_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

rfr_result *pack_result(const Prepared &P, const Factored &F) {
    size_t nf = F.factors.size();
    size_t ncoef = 0;
    for (auto &f : F.factors) ncoef += f.size();
    size_t bytes = sizeof(rfr_result) + nf * sizeof(int32_t) + 8 + ncoef * sizeof(int64_t);
    char *mem = (char *)std::calloc(1, bytes);
    if (!mem) return nullptr;
    rfr_result *r = (rfr_result *)mem;
    int32_t *deg = (int32_t *)(mem + sizeof(rfr_result));
    int64_t *co = (int64_t *)(((uintptr_t)(deg + nf) + 7) & ~(uintptr_t)7);
    r->content = F.content;
    r->nfactors = (int32_t)nf;
    r->n_elements = P.n;
    r->n_real = P.r;
    r->degrees = deg;
    r->coeffs = co;
    r->n_candidates = F.n_candidates;
    r->trace_folded = F.trace_folded;
    r->n_confirmed = F.n_confirmed;
    r->t_lo = P.t_lo;
    r->t_hi = P.t_hi;
    size_t k = 0;
    for (size_t i = 0; i < nf; ++i) {
        deg[i] = (int32_t)F.factors[i].size() - 1;
        for (auto c : F.factors[i]) co[k++] = c;
    }
    return r;
}

rfr_status ensure_workspace(rfr_ctx *ctx, Slot &s, size_t need) {
    if (s.ws_bytes >= need) return RFR_OK;
    if (s.ws) {
        (void)hipFree(s.ws);
        ctx->mem_used -= s.ws_bytes;
        s.ws = nullptr;
        s.ws_bytes = 0;
    }
    if (ctx->mem_used + need > ctx->budget) return fail(RFR_ENOMEM, "search tables exceed the memory budget");
    if (hipMalloc(&s.ws, need) != hipSuccess) {
        s.ws = nullptr;
        return fail(RFR_ENOMEM, "hipMalloc of the search workspace failed");
    }
    s.ws_bytes = need;
    ctx->mem_used += need;
    return RFR_OK;
}

// RootBuf layout: coefficients [0, O_JOB) | job [O_JOB, O_OUT) | records.
constexpr size_t ROOT_O_JOB = ((RFR_MAX_DEGREE + 1) * 8 + 255) & ~(size_t)255;
constexpr size_t ROOT_O_OUT = ROOT_O_JOB + 256;
constexpr size_t ROOT_BYTES = ROOT_O_OUT + RFR_MAX_DEGREE * sizeof(RootOut);
static_assert(sizeof(RootJob) <= 256, "job descriptor fits its slot");

rfr_status rootbuf_init(RootBuf &b, hipStream_t stream) {
    b.own_stream = stream == nullptr;
    if (b.own_stream) {
        if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess)
            return fail(RFR_EDEVICE, "hipStreamCreate failed");
    }
    b.stream = stream;
    if (hipMalloc((void **)&b.dev, ROOT_BYTES) != hipSuccess) {
        b.dev = nullptr;
        return fail(RFR_ENOMEM, "hipMalloc of the root buffer failed");
    }
    if (hipHostMalloc((void **)&b.host, ROOT_BYTES, hipHostMallocDefault) != hipSuccess) {
        b.host = nullptr;
        return fail(RFR_ENOMEM, "hipHostMalloc of the root buffer failed");
    }
    return RFR_OK;
}

void rootbuf_free(RootBuf &b) {
    if (b.dev) (void)hipFree(b.dev);
    if (b.host) (void)hipHostFree(b.host);
    if (b.own_stream && b.stream) (void)hipStreamDestroy(b.stream);
    b = RootBuf();
}

rfr_status prepare_dev(RootBuf &b, const int64_t *coeffs, int degree, Prepared &P, std::string &err) {
    rfr_status st = normalise(coeffs, degree, P, err);
    if (st != RFR_OK) return st;
    const int d = (int)P.prim.size() - 1;
    if (d >= 2 && b.dev && b.host) {
        std::memcpy(b.host, P.prim.data(), (size_t)(d + 1) * 8);
        *(RootJob *)(b.host + ROOT_O_JOB) = RootJob{(const int64_t *)b.dev, d, (RootOut *)(b.dev + ROOT_O_OUT)};
        bool ok = hipMemcpyAsync(b.dev, b.host, ROOT_O_OUT, hipMemcpyHostToDevice, b.stream) == hipSuccess;
        ok = ok && launch_roots((const RootJob *)(b.dev + ROOT_O_JOB), 1, d, ROOT_LANES, b.stream) == hipSuccess;
        ok = ok && hipMemcpyAsync(b.host + ROOT_O_OUT, b.dev + ROOT_O_OUT, (size_t)d * sizeof(RootOut),
                                  hipMemcpyDeviceToHost, b.stream) == hipSuccess;
        ok = ok && hipStreamSynchronize(b.stream) == hipSuccess;
        if (ok && finish_elements(P, (const RootOut *)(b.host + ROOT_O_OUT), err) == RFR_OK) return RFR_OK;
        err.clear();
    }
    return prepare_elements(P, err);
}

rfr_status slot_init(rfr_ctx *ctx, Slot &s, hipStream_t lane) {
    if (lane) {
        s.stream = lane;
        s.own_stream = false;
    } else if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) {
        return fail(RFR_EDEVICE, "hipStreamCreate failed");
    }
    if (rootbuf_init(s.roots, s.stream) != RFR_OK) return RFR_ENOMEM;
    if (hipMalloc(&s.cand_dev, 2 * ctx->cap * sizeof(uint64_t) + 256) != hipSuccess)
        return fail(RFR_ENOMEM, "hipMalloc of the candidate buffer failed");
    s.count_dev = (uint64_t *)((char *)s.cand_dev + 2 * ctx->cap * sizeof(uint64_t));
    if (hipHostMalloc(&s.host, (2 * ctx->cap + 8) * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess)
        return fail(RFR_ENOMEM, "hipHostMalloc failed");
    s.cap = ctx->cap;
    return RFR_OK;
}

void slot_free(rfr_ctx *ctx, Slot &s) {
    if (s.ws) {
        (void)hipFree(s.ws);
        ctx->mem_used -= s.ws_bytes;
    }
    if (s.cand_dev) (void)hipFree(s.cand_dev);
    if (s.host) (void)hipHostFree(s.host);
    rootbuf_free(s.roots);
    if (s.stream && s.own_stream) (void)hipStreamDestroy(s.stream);
    s = Slot();
}

// Device search for a prepared polynomial on one slot; fills cands.
// Workspace for a search over n weights within `avail` bytes: the full tables
// if they fit, else the smallest chunked layout (half A streamed in chunks)
// that does; 0 if none fits.
size_t choose_workspace(int n, size_t avail) {
    size_t full = recombine_workspace(n);
    if (full <= avail) return full;
    int na, nb;
    split_halves(n, na, nb);
    for (int c = 1; c <= std::min(na, dev::MAX_CHUNK_BITS); ++c) {
        JobPlan P;
        size_t b = plan_job(na - c, nb, P, dev::KCAP_MAX);
        if (b <= avail) return b;
    }
    return 0;
}

rfr_status search_on_slot(rfr_ctx *ctx, Slot &s, const Prepared &P, std::vector<Pat> &cands, int *folded) {
    cands.clear();
    if (folded) *folded = 0;
    if (P.n <= 1) return RFR_OK;
    if (P.n > dev::MAX_SEARCH_N) return fail(RFR_EOVERFLOW, "too many elements for the search tables");
    rfr_status st = RFR_OK;
    if (s.ws_bytes < recombine_workspace(P.n) && chunk_bits(P.n, s.ws_bytes) < 0) {
        // grow within the budget; a search larger than the budget streams half A
        const size_t avail = ctx->budget - (ctx->mem_used - s.ws_bytes);
        const size_t need = choose_workspace(P.n, avail);
        if (!need) return fail(RFR_ENOMEM, "search tables exceed the memory budget even when chunked");
        st = ensure_workspace(ctx, s, need);
        if (st != RFR_OK) return st;
    }
    std::string err;
    const bool prof = ctx->profiling && !ctx->serving;
    uint64_t *hcount = s.host + 2 * s.cap;
    // the query design (Algorithm E variant) where the tuning table found it
    // faster for this size class (or the context asks for it), within its range
    int na, nb;
    split_halves(P.n, na, nb);
    const bool e_ok = nb >= 1 && na <= E_MAX_HALF;
    bool use_e = e_ok && (ctx->design == 2 || (ctx->design == 0 && get_tune(na).design == 1));
    if (use_e && s.ws_bytes < recombine_e_workspace(P.n)) {
        const size_t avail = ctx->budget - (ctx->mem_used - s.ws_bytes);
        if (recombine_e_workspace(P.n) > avail || ensure_workspace(ctx, s, recombine_e_workspace(P.n)) != RFR_OK)
            use_e = false;
    }
    auto run = [&](const uint64_t *w, uint64_t t_lo, uint64_t t_hi) -> rfr_status {
        if (use_e) {
            rfr_status r = enqueue_recombine_e(w, P.n, t_lo, t_hi, s.ws, s.ws_bytes, s.stream, s.cand_dev, s.cap,
                                               s.count_dev, err);
            if (r != RFR_OK) return fail(r, err);
            if (hipMemcpyAsync(hcount, s.count_dev, 8, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
                hipStreamSynchronize(s.stream) != hipSuccess)
                return fail(RFR_EDEVICE, "device search failed");
            if (*hcount != E_FALLBACK) return RFR_OK;
            // B' sums too clustered for the query design: Horowitz-Sahni
        }
        rfr_status r = enqueue_recombine(w, P.n, t_lo, t_hi, s.ws, s.ws_bytes, s.stream, s.cand_dev, s.cap,
                                         s.count_dev, prof ? profile_events(ctx, 0) : nullptr, err);
        if (r != RFR_OK) return fail(r, err);
        if (hipMemcpyAsync(hcount, s.count_dev, 8, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
            hipStreamSynchronize(s.stream) != hipSuccess)
            return fail(RFR_EDEVICE, "device search failed");
        if (prof) profile_collect(ctx, 0, P.n);
        return RFR_OK;
    };
    st = run(P.w.data(), P.t_lo, P.t_hi);
    if (st != RFR_OK) return st;
    uint64_t cnt = *hcount;
    if (cnt == ~0ull && P.tr2_ok && P.t_lo + P.t2_lo + P.t_hi + P.t2_hi < (1ull << 32)) {
        // A flood of patterns whose first trace is an integer (Swinnerton-Dyer
        // like inputs).  A true factor's second trace is an integer too, so
        // search again over w_i + v_i: a true factor's sum lands in the sum of
        // the two windows, while a pattern whose second trace is not an integer
        // lands anywhere (the pre-filter of the second trace, applied inside
        // the search at no extra table traffic).
        uint64_t u[dev::MAX_SEARCH_N];
        for (int i = 0; i < P.n; ++i) u[i] = P.w[i] + P.v2[i];
        st = run(u, P.t_lo + P.t2_lo, P.t_hi + P.t2_hi);
        if (st != RFR_OK) return st;
        cnt = *hcount;
        if (folded) *folded = 1;
    }
    if (cnt == ~0ull) return fail(RFR_ECANDIDATES, "candidate capacity exceeded");
    if (cnt) {
        if (hipMemcpyAsync(s.host, s.cand_dev, cnt * 16, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
            hipStreamSynchronize(s.stream) != hipSuccess)
            return fail(RFR_EDEVICE, "candidate copy failed");
    }
    cands.resize(cnt);
    for (uint64_t k = 0; k < cnt; ++k) {
        Pat p;
        uint64_t a = s.host[2 * k], b = s.host[2 * k + 1];
        for (int i = 0; i < na; ++i)
            if ((a >> i) & 1) p.set(i);
        for (int i = 0; i < nb; ++i)
            if ((b >> i) & 1) p.set(na + i);
        cands[k] = p;
    }
    return RFR_OK;
}

// Full plain factorisation of one polynomial on one slot.
rfr_status factor_on_slot(rfr_ctx *ctx, Slot &s, const int64_t *coeffs, int degree, rfr_result **out) {
    double t0 = now_ms();
    Prepared P;
    std::string err;
    rfr_status st = prepare_dev(s.roots, coeffs, degree, P, err);
    if (st == RFR_OK) st = peel_singletons(P, err);
    if (st != RFR_OK) return fail(st, err);
    double t1 = now_ms();
    Factored F;
    std::vector<Pat> cands;
    if (P.n <= 1) {
        trivial_factor(P, F);
    } else {
        st = search_on_slot(ctx, s, P, cands, &F.trace_folded);
        if (st != RFR_OK) return st;
    }
    double t2 = now_ms();
    if (P.n > 1) {
        st = confirm_and_factor(P, cands, F, err);
        if (st != RFR_OK) return fail(st, err);
    }
    double t3 = now_ms();
    rfr_result *r = pack_result(P, F);
    if (!r) return fail(RFR_ENOMEM, "result allocation failed");
    r->ms_roots = t1 - t0;
    r->ms_search = t2 - t1;
    r->ms_confirm = t3 - t2;
    *out = r;
    return RFR_OK;
}

}  // namespace rfr

using namespace rfr;

extern "C" {

rfr_status rfr_create(int device, size_t mem_budget_bytes, rfr_ctx **out) {
    if (!out) return fail(RFR_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(RFR_EDEVICE, "no such HIP device");
    if (hipSetDevice(device) != hipSuccess) return fail(RFR_EDEVICE, "hipSetDevice failed");
    tuning_autoload();
    rfr_ctx *ctx = new (std::nothrow) rfr_ctx();
    if (!ctx) return fail(RFR_ENOMEM, "context allocation failed");
    ctx->device = device;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        delete ctx;
        return fail(RFR_EDEVICE, "hipMemGetInfo failed");
    }
    ctx->budget = mem_budget_bytes ? mem_budget_bytes : (size_t)(0.9 * (double)fr);
    rfr_status st = slot_init(ctx, ctx->main);
    if (st != RFR_OK) {
        slot_free(ctx, ctx->main);
        delete ctx;
        return st;
    }
    *out = ctx;
    return RFR_OK;
}

void rfr_destroy(rfr_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    rfr_serve_stop(ctx);
    batch_release(ctx);
    for (auto e : ctx->prof_ev)
        if (e) (void)hipEventDestroy(e);
    slot_free(ctx, ctx->main);
    delete ctx;
}

rfr_status rfr_set_design(rfr_ctx *ctx, int design) {
    if (!ctx || design < 0 || design > 2) return fail(RFR_EINVAL, "design must be 0, 1 or 2");
    if (ctx->serving) return fail(RFR_EBUSY, "cannot change the design while serving");
    ctx->design = design;
    return RFR_OK;
}

rfr_status rfr_set_candidate_cap(rfr_ctx *ctx, uint64_t cap) {
    if (!ctx || cap < 1 || cap > (1ull << 26)) return fail(RFR_EINVAL, "cap must be in [1, 2^26]");
    if (ctx->serving) return fail(RFR_EBUSY, "cannot change the cap while serving");
    (void)hipSetDevice(ctx->device);
    size_t ws = ctx->main.ws_bytes;
    slot_free(ctx, ctx->main);
    ctx->cap = cap;
    rfr_status st = slot_init(ctx, ctx->main);
    (void)ws;
    return st;
}

rfr_status rfr_factor(rfr_ctx *ctx, const int64_t *coeffs, int degree, rfr_result **out) {
    if (!ctx || !out) return fail(RFR_EINVAL, "ctx/out is NULL");
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(RFR_EDEVICE, "hipSetDevice failed");
    rfr_status st = factor_on_slot(ctx, ctx->main, coeffs, degree, out);
    if (st != RFR_ENOTSQFREE) return st;
    return factor_sqf_route(coeffs, degree, [&](const int64_t *c, int d, rfr_result **o) {
        return factor_on_slot(ctx, ctx->main, c, d, o);
    }, out);
}

void rfr_result_free(rfr_result *res) { std::free(res); }

rfr_status rfr_results_pack(rfr_result *const *res, int count, int64_t *content, int32_t *nfactors,
                            int32_t *degrees, size_t deg_cap, int64_t *coeffs, size_t coef_cap, size_t *ndeg,
                            size_t *ncoef) {
    if (count < 0 || (count > 0 && !res) || !ndeg || !ncoef) return fail(RFR_EINVAL, "bad arguments");
    size_t nd = 0, nc = 0;
    for (int i = 0; i < count; ++i) {
        const rfr_result *r = res[i];
        if (!r) continue;
        nd += (size_t)r->nfactors;
        for (int k = 0; k < r->nfactors; ++k) nc += (size_t)r->degrees[k] + 1;
    }
    *ndeg = nd;
    *ncoef = nc;
    if (!degrees || !coeffs) return RFR_OK;
    if (!content || !nfactors || deg_cap < nd || coef_cap < nc) return fail(RFR_EINVAL, "buffers too small");
    size_t od = 0, oc = 0;
    for (int i = 0; i < count; ++i) {
        const rfr_result *r = res[i];
        content[i] = r ? r->content : 0;
        nfactors[i] = r ? r->nfactors : 0;
        if (!r) continue;
        size_t m = 0;
        for (int k = 0; k < r->nfactors; ++k) {
            degrees[od++] = r->degrees[k];
            m += (size_t)r->degrees[k] + 1;
        }
        std::memcpy(coeffs + oc, r->coeffs, m * sizeof(int64_t));
        oc += m;
    }
    return RFR_OK;
}

void rfr_results_free(rfr_result *const *res, int count) {
    for (int i = 0; res && i < count; ++i) std::free(res[i]);
}

const char *rfr_strerror(rfr_status st) {
    switch (st) {
        case RFR_OK: return "ok";
        case RFR_EINVAL: return "invalid argument";
        case RFR_ENOTSQFREE: return "polynomial is not square-free";
        case RFR_ENOMEM: return "out of memory or over budget";
        case RFR_EPRECISION: return "roots not separated / window too wide";
        case RFR_EOVERFLOW: return "value outside the supported range";
        case RFR_ECANDIDATES: return "candidate capacity exceeded";
        case RFR_EDEVICE: return "HIP runtime error";
        case RFR_EBUSY: return "not finished";
    }
    return "unknown status";
}

const char *rfr_last_error(void) { return g_last_error.c_str(); }

rfr_status rfr_weights(const int64_t *coeffs, int degree, uint64_t *w_out, int32_t *n_out,
                       int32_t *n_real_out, uint64_t *t_lo, uint64_t *t_hi) {
    if (!w_out || !n_out || !n_real_out || !t_lo || !t_hi) return fail(RFR_EINVAL, "NULL output");
    Prepared P;
    std::string err;
    rfr_status st = prepare(coeffs, degree, P, err);
    if (st != RFR_OK) return fail(st, err);
    for (int i = 0; i < P.n; ++i) w_out[i] = P.w[i];
    *n_out = P.n;
    *n_real_out = P.r;
    *t_lo = P.t_lo;
    *t_hi = P.t_hi;
    return RFR_OK;
}

size_t rfr_recombine_workspace_bytes(int n) { return recombine_workspace(n); }

size_t rfr_recombine_min_workspace_bytes(int n) {
    if (n < 2 || n > dev::MAX_SEARCH_N) return 0;
    int na, nb;
    split_halves(n, na, nb);
    JobPlan P;
    return plan_job(na - std::min(na, dev::MAX_CHUNK_BITS), nb, P, dev::KCAP_MAX);
}

rfr_status rfr_recombine_dev(const uint64_t *w_host, int n, uint64_t t_lo, uint64_t t_hi, void *workspace,
                             size_t ws_bytes, void *hip_stream, uint64_t *cand_dev, uint64_t cap,
                             uint64_t *count_dev) {
    std::string err;
    rfr_status st = enqueue_recombine(w_host, n, t_lo, t_hi, workspace, ws_bytes, (hipStream_t)hip_stream,
                                      cand_dev, cap, count_dev, nullptr, err);
    if (st != RFR_OK) return fail(st, err);
    return RFR_OK;
}

rfr_status rfr_recombine_dev_noalloc(const uint64_t *w_host, int n, uint64_t t_lo, uint64_t t_hi, void *hip_stream,
                                     uint64_t *cand_dev, uint64_t cap, uint64_t *count_dev) {
    std::string err;
    rfr_status st = enqueue_recombine_noalloc(w_host, n, t_lo, t_hi, (hipStream_t)hip_stream, cand_dev, cap,
                                              count_dev, err);
    if (st != RFR_OK) return fail(st, err);
    return RFR_OK;
}

size_t rfr_recombine_noalloc_scratch_bytes(void) { return rfr::NOALLOC_WS_BYTES; }

size_t rfr_recombine_e_workspace_bytes(int n) { return recombine_e_workspace(n); }

rfr_status rfr_recombine_e_dev(const uint64_t *w_host, int n, uint64_t t_lo, uint64_t t_hi, void *workspace,
                               size_t ws_bytes, void *hip_stream, uint64_t *cand_dev, uint64_t cap,
                               uint64_t *count_dev) {
    std::string err;
    rfr_status st = enqueue_recombine_e(w_host, n, t_lo, t_hi, workspace, ws_bytes, (hipStream_t)hip_stream,
                                        cand_dev, cap, count_dev, err);
    if (st != RFR_OK) return fail(st, err);
    return RFR_OK;
}

size_t rfr_expand_workspace_bytes(int m) { return expand_workspace(m); }

rfr_status rfr_expand_dev(const uint64_t *w_host, int m, int negate, void *workspace, size_t ws_bytes,
                          void *hip_stream, uint64_t *sorted_dev) {
    std::string err;
    rfr_status st = enqueue_expand(w_host, m, negate, workspace, ws_bytes, (hipStream_t)hip_stream, sorted_dev, err);
    if (st != RFR_OK) return fail(st, err);
    return RFR_OK;
}

}  // extern "C"
