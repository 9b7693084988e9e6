// Batched factorisation: many polynomials of uneven degree in one call.
#include <algorithm>
#include <atomic>
#include <numeric>
#include <thread>

#include "rfr_ctx.h"

namespace rfr {

struct BatchState {};

void batch_release(rfr_ctx *ctx) {
    delete ctx->batch;
    ctx->batch = nullptr;
}

}  // namespace rfr

using namespace rfr;

extern "C" rfr_status rfr_factor_batch(rfr_ctx *ctx, int count, const int64_t *coeffs, const int32_t *degrees,
                                       rfr_result **out, rfr_status *status) {
    if (!ctx || count < 0 || (count > 0 && (!coeffs || !degrees || !out || !status)))
        return fail(RFR_EINVAL, "bad batch arguments");
    if (count == 0) return RFR_OK;
    (void)hipSetDevice(ctx->device);
    std::vector<size_t> off(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        if (degrees[i] < 1 || degrees[i] > RFR_MAX_DEGREE) return fail(RFR_EINVAL, "degree out of range");
        off[i + 1] = off[i] + (size_t)degrees[i] + 1;
    }
    // largest first, so the long searches start early
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return degrees[a] > degrees[b]; });
    int nthreads = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
    nthreads = std::min(nthreads, count);
    std::vector<Slot> slots(nthreads);
    for (auto &s : slots) {
        rfr_status st = slot_init(ctx, s);
        if (st != RFR_OK) {
            for (auto &t : slots) slot_free(ctx, t);
            return st;
        }
    }
    std::mutex mem_mu;
    std::atomic<int> next{0};
    auto work = [&](int tid) {
        (void)hipSetDevice(ctx->device);
        Slot &s = slots[tid];
        for (;;) {
            int k = next.fetch_add(1);
            if (k >= count) break;
            int i = order[k];
            rfr_result *r = nullptr;
            Prepared P;
            std::string err;
            rfr_status st = prepare(coeffs + off[i], degrees[i], P, err);
            if (st == RFR_OK && P.n > 1) {
                size_t need = recombine_workspace(P.n);
                std::lock_guard<std::mutex> lk(mem_mu);
                st = ensure_workspace(ctx, s, need);
            }
            if (st == RFR_OK) {
                Factored F;
                std::vector<Pat> cands;
                if (P.n <= 1) trivial_factor(P, F);
                else {
                    st = search_on_slot(ctx, s, P, cands);
                    if (st == RFR_OK) {
                        st = confirm_and_factor(P, cands, F, err);
                        if (st != RFR_OK) st = fail(st, err);
                    }
                }
                if (st == RFR_OK) {
                    r = pack_result(P, F);
                    if (!r) st = RFR_ENOMEM;
                }
            } else {
                st = fail(st, err);
            }
            out[i] = r;
            status[i] = st;
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) th.emplace_back(work, t);
    for (auto &t : th) t.join();
    for (auto &s : slots) slot_free(ctx, s);
    return RFR_OK;
}
