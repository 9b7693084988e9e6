// Batched factorisation: many polynomials of uneven degree in one device pass.
//
//  1. normalisation on the host; the roots of every polynomial of degree >= 2
//     in one device launch (a workgroup per polynomial); disc checks,
//     elements, weights and window on a thread pool (a polynomial whose device
//     roots fail the checks has its roots found again on the host);
//  2. the searches are split by size: small ones (both halves <= 2^SMALL_HALF
//     keys) go to one persistent kernel (a workgroup per polynomial, largest
//     first from an atomic queue, everything in LDS); larger ones run through
//     the staged pipeline with ONE launch per stage for all of them (each
//     block finds its job from per-stage block offsets);
//  3. the whole device pass -- descriptor upload, both paths on two streams,
//     a summary gather and one copy back -- is captured once into a HIP graph
//     and replayed for every later batch with the same shape;
//  4. candidates are confirmed on the thread pool.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <numeric>
#include <sstream>
#include <thread>

#include "rfr_ctx.h"
#include "rfr_roots.h"

namespace rfr {

constexpr uint64_t BCAP = 1024;  // candidate patterns per search in a batch
constexpr uint64_t HEAD = 8;     // pairs returned with each count
constexpr int HUGE_HALF = 23;    // searches with a half of >= 2^23 keys are streamed one by one
constexpr size_t SUMMARY = 1 + 2 * HEAD;  // u64 per job in the summary

struct BatchState {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    char *ws = nullptr;        // device: workspaces of the large searches
    size_t ws_bytes = 0;
    char *dev = nullptr;       // device: descriptors + outputs
    size_t dev_bytes = 0;
    char *host = nullptr;      // pinned: descriptor staging
    size_t host_bytes = 0;
    char *outd = nullptr;      // device: counts, candidates, summary of every slot
    size_t outd_bytes = 0;
    char *hsum = nullptr;      // pinned: summary copy
    size_t hsum_bytes = 0;
    char *rdev = nullptr;      // device: root-finder coefficients, jobs and records
    size_t rdev_bytes = 0;
    char *rhost = nullptr;     // pinned: the same, staged
    size_t rhost_bytes = 0;
    std::string sig;           // shape of the captured graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t replays = 0, captures = 0;
};

static void drop_graph(BatchState *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->sig.clear();
}

void batch_release(rfr_ctx *ctx) {
    BatchState *b = ctx->batch;
    if (!b) return;
    drop_graph(b);
    if (b->ws) (void)hipFree(b->ws);
    if (b->dev) (void)hipFree(b->dev);
    if (b->host) (void)hipHostFree(b->host);
    if (b->outd) (void)hipFree(b->outd);
    if (b->hsum) (void)hipHostFree(b->hsum);
    if (b->rdev) (void)hipFree(b->rdev);
    if (b->rhost) (void)hipHostFree(b->rhost);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->side) (void)hipStreamDestroy(b->side);
    delete b;
    ctx->batch = nullptr;
}

static rfr_status grow(char **p, size_t *have, size_t need, bool pinned, BatchState *b) {
    if (*have >= need) return RFR_OK;
    drop_graph(b);  // the graph holds the old addresses
    if (*p) (void)(pinned ? hipHostFree(*p) : hipFree(*p));
    *p = nullptr;
    *have = 0;
    size_t sz = need + need / 4;
    hipError_t e = pinned ? hipHostMalloc((void **)p, sz, hipHostMallocDefault) : hipMalloc((void **)p, sz);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(RFR_ENOMEM, "batch buffer allocation failed");
    }
    *have = sz;
    return RFR_OK;
}

// Buffers outside the captured graph: reallocated without dropping it.
static rfr_status grow_buf(char **p, size_t *have, size_t need, bool pinned) {
    if (*have >= need) return RFR_OK;
    if (*p) (void)(pinned ? hipHostFree(*p) : hipFree(*p));
    *p = nullptr;
    *have = 0;
    size_t sz = need + need / 4;
    hipError_t e = pinned ? hipHostMalloc((void **)p, sz, hipHostMallocDefault) : hipMalloc((void **)p, sz);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(RFR_ENOMEM, "batch buffer allocation failed");
    }
    *have = sz;
    return RFR_OK;
}

// Roots of every normalised polynomial of degree >= 2 on the device; rec[i]
// points at polynomial i's records in host memory (nullptr: none).
static rfr_status device_roots(BatchState *B, hipStream_t st, std::vector<Prepared> &P,
                               const std::vector<rfr_status> &status, std::vector<const RootOut *> &rec) {
    const int count = (int)P.size();
    rec.assign(count, nullptr);
    std::vector<int> jobs;
    std::vector<size_t> co(count, 0), ro(count, 0);
    size_t nco = 0, nro = 0;
    for (int i = 0; i < count; ++i) {
        const int d = (int)P[i].prim.size() - 1;
        if (status[i] != RFR_OK || d < 2) continue;
        jobs.push_back(i);
        co[i] = nco;
        ro[i] = nro;
        nco += (size_t)d + 1;
        nro += (size_t)d;
    }
    if (jobs.empty()) return RFR_OK;
    // layout (same in both buffers): coefficients | jobs | records
    const size_t o_jobs = (nco * 8 + 255) & ~(size_t)255;
    const size_t o_out = (o_jobs + jobs.size() * sizeof(RootJob) + 255) & ~(size_t)255;
    const size_t bytes = o_out + nro * sizeof(RootOut);
    rfr_status e = grow_buf(&B->rdev, &B->rdev_bytes, bytes, false);
    if (e == RFR_OK) e = grow_buf(&B->rhost, &B->rhost_bytes, bytes, true);
    if (e != RFR_OK) return e;
    int64_t *hc = (int64_t *)B->rhost;
    RootJob *hj = (RootJob *)(B->rhost + o_jobs);
    for (size_t k = 0; k < jobs.size(); ++k) {
        const int i = jobs[k];
        std::memcpy(hc + co[i], P[i].prim.data(), P[i].prim.size() * 8);
        hj[k] = RootJob{(const int64_t *)(B->rdev) + co[i], (int)P[i].prim.size() - 1,
                        (RootOut *)(B->rdev + o_out) + ro[i]};
    }
    int dmax = 2;
    for (int i : jobs) dmax = std::max(dmax, (int)P[i].prim.size() - 1);
    bool ok = hipMemcpyAsync(B->rdev, B->rhost, o_out, hipMemcpyHostToDevice, st) == hipSuccess;
    // up to one polynomial per CU: ROOT_LANES lanes per root (shorter dependent
    // chains); beyond that one lane per root keeps more polynomials in flight
    const int lanes = jobs.size() <= 256 ? ROOT_LANES : 1;
    ok = ok && launch_roots((const RootJob *)(B->rdev + o_jobs), (int)jobs.size(), dmax, lanes, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(B->rhost + o_out, B->rdev + o_out, nro * sizeof(RootOut), hipMemcpyDeviceToHost,
                              st) == hipSuccess;
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) return fail(RFR_EDEVICE, "device root finding failed");
    for (int i : jobs) rec[i] = (const RootOut *)(B->rhost + o_out) + ro[i];
    return RFR_OK;
}

// Elements, weights and window of one normalised polynomial from its device
// root records, or from roots found on the host when there are none or they
// fail the disc checks.  Returns whether the device roots were used.
static bool finish_or_host(Prepared &P, const RootOut *rec, rfr_status &st, std::string &err) {
    if (rec && finish_elements(P, rec, err) == RFR_OK) {
        st = RFR_OK;
        return true;
    }
    err.clear();
    st = prepare_elements(P, err);
    return false;
}

// Copy each job's count and first HEAD pattern pairs into one compact summary.
__global__ void k_summary(const uint64_t *counts, const uint64_t *cand, uint64_t stride, int njobs,
                          uint64_t *summary) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= njobs) return;
    uint64_t *s = summary + (size_t)j * SUMMARY;
    const uint64_t c = counts[j];
    s[0] = c;
    const uint64_t *src = cand + (size_t)j * stride;
    const uint64_t k = c < HEAD ? c : HEAD;
    for (uint64_t i = 0; i < 2 * k; ++i) s[1 + i] = src[i];
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
    ctx->prof.launches += 1;
    ctx->prof.keys += (1ull << na) + (1ull << nb);
}

static void to_pat(const uint64_t *pair, int na, int nb, Pat &p) {
    for (int b = 0; b < na; ++b)
        if ((pair[0] >> b) & 1) p.set(b);
    for (int b = 0; b < nb; ++b)
        if ((pair[1] >> b) & 1) p.set(na + b);
}

}  // namespace rfr

using namespace rfr;

// One device pass of the mid-size and small searches (descriptors already
// staged): uploaded, both paths on two streams, summary of all slots, copy back.
static bool device_pass(BatchState *B, hipStream_t S0, size_t desc_bytes, size_t o_jobs, size_t o_bases,
                        size_t o_small, size_t o_queue, const MultiLaunch &ML, int nS, StageEvents *ev,
                        const uint64_t *counts_d, const uint64_t *cand_d, uint64_t *sum_d, uint64_t *sum_h,
                        int nslots) {
    bool ok = hipMemcpyAsync(B->dev, B->host, desc_bytes, hipMemcpyHostToDevice, S0) == hipSuccess;
    ok = ok && hipEventRecord(B->fork, S0) == hipSuccess;
    ok = ok && hipStreamWaitEvent(B->side, B->fork, 0) == hipSuccess;
    ok = ok && launch_small((const SmallJob *)(B->dev + o_small), nS, (uint32_t *)(B->dev + o_queue),
                            std::min(nS, 1024), B->side) == hipSuccess;
    ok = ok && ML.launch((const dev::JobArgs *)(B->dev + o_jobs), (const uint32_t *)(B->dev + o_bases), S0, ev) ==
                   hipSuccess;
    ok = ok && hipEventRecord(B->join, B->side) == hipSuccess;
    ok = ok && hipStreamWaitEvent(S0, B->join, 0) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_summary, dim3((nslots + 255) / 256), dim3(256), 0, S0, counts_d, cand_d,
                           (uint64_t)2 * BCAP, nslots, sum_d);
        ok = hipGetLastError() == hipSuccess;
    }
    ok = ok && hipMemcpyAsync(sum_h, sum_d, (size_t)nslots * SUMMARY * 8, hipMemcpyDeviceToHost, S0) == hipSuccess;
    return ok;
}

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
    if (!ctx->batch) {
        BatchState *b = new BatchState();
        if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess) {
            ctx->batch = b;
            batch_release(ctx);
            return fail(RFR_EDEVICE, "batch stream/event creation failed");
        }
        ctx->batch = b;
    }
    BatchState *B = ctx->batch;
    const int nthreads = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
    hipStream_t S0 = ctx->main.stream;

    // output slots: slot k belongs to the k-th polynomial in largest-first order
    //   counts[count] | cand[count][2*BCAP] | summary[count][SUMMARY]
    const size_t o_cand = ((size_t)8 * count + 255) & ~(size_t)255;
    const size_t o_sum = o_cand + (size_t)count * 2 * BCAP * 8;
    rfr_status e0 = grow(&B->outd, &B->outd_bytes, o_sum + (size_t)count * SUMMARY * 8, false, B);
    if (e0 == RFR_OK) e0 = grow(&B->hsum, &B->hsum_bytes, (size_t)count * SUMMARY * 8, true, B);
    if (e0 != RFR_OK) return e0;
    uint64_t *counts_d = (uint64_t *)B->outd;
    uint64_t *cand_d = (uint64_t *)(B->outd + o_cand);
    uint64_t *sum_d = (uint64_t *)(B->outd + o_sum);
    uint64_t *sum_h = (uint64_t *)B->hsum;

    // ---- 1. normalisation, device roots, then the host stage on the pool,
    //         largest first; the device thread below consumes the results as
    //         they become ready
    std::vector<Prepared> P(count);
    std::vector<rfr_status> st(count, RFR_OK);
    std::vector<std::string> err(count);
    for (int i = 0; i < count; ++i) {
        st[i] = normalise(coeffs + off[i], degrees[i], P[i], err[i]);
    }
    std::vector<const RootOut *> rec;
    rfr_status rst = device_roots(B, S0, P, st, rec);
    if (rst != RFR_OK) return rst;
    std::vector<int> order(count), slot(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return degrees[a] > degrees[b]; });
    for (int k = 0; k < count; ++k) slot[order[k]] = k;
    std::vector<std::atomic<int>> ready(count);
    for (auto &r : ready) r.store(0);
    std::atomic<int> next{0};
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t)
        pool.emplace_back([&] {
            for (int k; (k = next.fetch_add(1)) < count;) {
                const int i = order[k];
                if (st[i] == RFR_OK) (void)finish_or_host(P[i], rec[i], st[i], err[i]);
                if (st[i] == RFR_OK) st[i] = peel_singletons(P[i], err[i]);
                ready[i].store(1, std::memory_order_release);
            }
        });

    // ---- 2. huge searches are queued on the stream as soon as their roots are
    //         ready (each fills the GPU on its own); the rest is classified
    std::vector<int> huge, large, small;
    rfr_status dev_st = RFR_OK;
    for (int k = 0; k < count && dev_st == RFR_OK; ++k) {
        const int i = order[k];
        while (!ready[i].load(std::memory_order_acquire)) std::this_thread::yield();
        if (st[i] != RFR_OK || P[i].n <= 1) continue;
        if (P[i].n > dev::MAX_SEARCH_N) {
            st[i] = RFR_EOVERFLOW;
            err[i] = "too many elements for the search tables";
            continue;
        }
        int na, nb;
        split_halves(P[i].n, na, nb);
        if (na <= SMALL_HALF) {
            small.push_back(i);
            continue;
        }
        if (na < HUGE_HALF) {
            large.push_back(i);
            continue;
        }
        const size_t need = recombine_workspace(P[i].n);
        if (need > ctx->main.ws_bytes) {
            if (hipStreamSynchronize(S0) != hipSuccess) {
                dev_st = fail(RFR_EDEVICE, "device search failed");
                break;
            }
            rfr_status e = ensure_workspace(ctx, ctx->main, need);
            if (e != RFR_OK) {
                st[i] = e;
                err[i] = g_last_error;
                continue;
            }
        }
        std::string e2;
        rfr_status e = enqueue_recombine(P[i].w.data(), P[i].n, P[i].t_lo, P[i].t_hi, ctx->main.ws,
                                         ctx->main.ws_bytes, S0, cand_d + (size_t)k * 2 * BCAP, BCAP,
                                         counts_d + k, profile_events(ctx, 1 + (int)huge.size()), e2);
        if (e != RFR_OK) {
            st[i] = e;
            err[i] = e2;
            continue;
        }
        huge.push_back(i);
    }
    for (auto &t : pool) t.join();
    if (dev_st != RFR_OK) return dev_st;
    const int nL = (int)large.size(), nS = (int)small.size();

    // ---- 3. layout of the mid-size searches and the descriptors
    std::vector<JobPlan> plans(nL);
    std::vector<size_t> wsoff(nL + 1, 0);
    for (int k = 0; k < nL; ++k) {
        int na, nb;
        split_halves(P[large[k]].n, na, nb);
        size_t bts = plan_job(na, nb, plans[k], BCAP + 1, true);
        wsoff[k + 1] = wsoff[k] + ((bts + 255) & ~(size_t)255);
    }
    // descriptor block: JobArgs[nL] | bases and tables | SmallJob[nS] | queue counter
    const size_t o_jobs = 0;
    const size_t o_bases = (o_jobs + sizeof(dev::JobArgs) * nL + 255) & ~(size_t)255;
    size_t bases_bytes = 0;  // block offsets and block -> job tables of every stage
    {
        MultiLaunch T;
        for (int k = 0; k < nL; ++k) T.add(plans[k], dev::JobArgs{});
        bases_bytes = T.bases_bytes();
    }
    const size_t o_small = (o_bases + bases_bytes + 255) & ~(size_t)255;
    const size_t o_queue = (o_small + sizeof(SmallJob) * nS + 255) & ~(size_t)255;
    const size_t desc_bytes = o_queue + 256;
    rfr_status e = grow(&B->ws, &B->ws_bytes, std::max<size_t>(wsoff[nL], 256), false, B);
    if (e == RFR_OK) e = grow(&B->dev, &B->dev_bytes, desc_bytes, false, B);
    if (e == RFR_OK) e = grow(&B->host, &B->host_bytes, desc_bytes, true, B);
    if (e != RFR_OK) return e;
    MultiLaunch ML;
    for (int k = 0; k < nL; ++k) {
        const Prepared &Q = P[large[k]];
        const int sk = slot[large[k]];
        int na, nb;
        split_halves(Q.n, na, nb);
        std::vector<uint64_t> wneg(nb);
        for (int t = 0; t < nb; ++t) wneg[t] = 0 - Q.w[na + t];
        dev::JobArgs J;
        build_job(plans[k], B->ws + wsoff[k], Q.w.data(), wneg.data(), Q.t_lo, Q.t_hi,
                  cand_d + (size_t)sk * 2 * BCAP, counts_d + sk, BCAP, J);
        ML.add(plans[k], J);
    }
    if (nL) {
        std::memcpy(B->host + o_jobs, ML.jobs.data(), sizeof(dev::JobArgs) * nL);
        ML.pack_bases((uint32_t *)(B->host + o_bases));
    }
    SmallJob *sj = (SmallJob *)(B->host + o_small);
    for (int k = 0; k < nS; ++k) {
        const Prepared &Q = P[small[k]];
        const int sk = slot[small[k]];
        SmallJob S{};
        split_halves(Q.n, S.na, S.nb);
        for (int t = 0; t < Q.n - 1; ++t) S.w[t] = Q.w[t];
        S.t_lo = Q.t_lo;
        S.t_hi = Q.t_hi;
        S.out = cand_d + (size_t)sk * 2 * BCAP;
        S.out_count = counts_d + sk;
        S.cap = BCAP;
        sj[k] = S;
    }

    // ---- 4. the device pass: captured once per shape into a graph and
    //         replayed; when profiling, launched directly with stage events
    if (ctx->profiling) {
        StageEvents *ev = nL ? profile_events(ctx, 0) : nullptr;
        if (!device_pass(B, S0, desc_bytes, o_jobs, o_bases, o_small, o_queue, ML, nS, ev, counts_d, cand_d, sum_d,
                         sum_h, count) ||
            hipStreamSynchronize(S0) != hipSuccess)
            return fail(RFR_EDEVICE, "batch device pass failed");
        for (size_t h = 0; h < huge.size(); ++h) profile_collect(ctx, 1 + (int)h, P[huge[h]].n);
        if (nL) {
            for (int i = 0; i < 6; ++i) {
                float ms = 0;
                if (hipEventElapsedTime(&ms, (hipEvent_t)ev->ev[i], (hipEvent_t)ev->ev[i + 1]) == hipSuccess)
                    ctx->prof.stage_ms[i] += ms;
            }
            ctx->prof.searches += nL;
            ctx->prof.launches += 1;
            for (int k = 0; k < nL; ++k) {
                int na, nb;
                split_halves(P[large[k]].n, na, nb);
                ctx->prof.keys += (1ull << na) + (1ull << nb);
            }
        }
    } else {
        std::ostringstream sig;
        sig << count << ':' << nL << ':' << nS << ':' << (void *)B->ws << ':' << (void *)B->dev << ':'
            << (void *)B->host << ':' << (void *)B->outd << ':' << (void *)B->hsum << ':' << desc_bytes << ':'
            << ML.maxB1 << ':' << ML.maxB2;
        if (nL)
            for (int s = 0; s < dev::NSTAGES; ++s) sig << ':' << ML.bases[s].back();
        if (!B->exec || B->sig != sig.str()) {
            drop_graph(B);
            bool ok = hipStreamBeginCapture(S0, hipStreamCaptureModeThreadLocal) == hipSuccess;
            ok = ok && device_pass(B, S0, desc_bytes, o_jobs, o_bases, o_small, o_queue, ML, nS, nullptr, counts_d,
                                   cand_d, sum_d, sum_h, count);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(S0, &g);
            if (!ok || ec != hipSuccess || !g) {
                if (g) (void)hipGraphDestroy(g);
                return fail(RFR_EDEVICE, "batch graph capture failed");
            }
            B->graph = g;
            if (hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0) != hipSuccess) {
                B->exec = nullptr;
                drop_graph(B);
                return fail(RFR_EDEVICE, "batch graph instantiation failed");
            }
            B->sig = sig.str();
            ++B->captures;
        } else {
            ++B->replays;
        }
        if (hipGraphLaunch(B->exec, S0) != hipSuccess || hipStreamSynchronize(S0) != hipSuccess)
            return fail(RFR_EDEVICE, "batch device pass failed");
    }

    // ---- 5. candidates of every searched polynomial
    std::vector<std::vector<Pat>> cands(count);
    std::vector<int> folded(count, 0);
    auto take = [&](int i) -> rfr_status {
        const int k = slot[i];
        const uint64_t *s = sum_h + (size_t)k * SUMMARY;
        const uint64_t c = s[0];
        int na, nb;
        split_halves(P[i].n, na, nb);
        if (c == ~0ull) {
            // more candidates than a batch slot holds: redo with the full capacity
            rfr_status r = search_on_slot(ctx, ctx->main, P[i], cands[i], &folded[i]);
            if (r != RFR_OK) {
                st[i] = r;
                err[i] = g_last_error;
            }
            return RFR_OK;
        }
        cands[i].assign(c, Pat());
        if (c <= HEAD) {
            for (uint64_t q = 0; q < c; ++q) to_pat(s + 1 + 2 * q, na, nb, cands[i][q]);
        } else {
            std::vector<uint64_t> tmp(2 * c);
            if (hipMemcpy(tmp.data(), cand_d + (size_t)k * 2 * BCAP, 16 * c, hipMemcpyDeviceToHost) != hipSuccess)
                return fail(RFR_EDEVICE, "candidate copy failed");
            for (uint64_t q = 0; q < c; ++q) to_pat(tmp.data() + 2 * q, na, nb, cands[i][q]);
        }
        return RFR_OK;
    };
    for (auto *grp : {&huge, &large, &small})
        for (int i : *grp)
            if (take(i) != RFR_OK) return RFR_EDEVICE;

    // ---- 6. confirmation and packing on the pool
    next.store(0);
    pool.clear();
    for (int t = 0; t < nthreads; ++t)
        pool.emplace_back([&] {
            for (int k; (k = next.fetch_add(1)) < count;) {
                const int i = order[k];
                out[i] = nullptr;
                if (st[i] == RFR_OK) {
                    Factored F;
                    F.trace_folded = folded[i];
                    if (P[i].n <= 1) trivial_factor(P[i], F);
                    else st[i] = confirm_and_factor(P[i], cands[i], F, err[i]);
                    if (st[i] == RFR_OK) {
                        out[i] = pack_result(P[i], F);
                        if (!out[i]) st[i] = RFR_ENOMEM;
                    }
                }
                status[i] = st[i];
            }
        });
    for (auto &t : pool) t.join();
    // polynomials that are not square-free: their square-free parts through
    // the plain path, one after another (the batch's device work is done)
    for (int i = 0; i < count; ++i) {
        if (status[i] != RFR_ENOTSQFREE) continue;
        status[i] = factor_sqf_route(coeffs + off[i], degrees[i], [&](const int64_t *c, int d, rfr_result **o) {
            return factor_on_slot(ctx, ctx->main, c, d, o);
        }, &out[i]);
        err[i] = status[i] == RFR_OK ? std::string() : g_last_error;
    }
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
    out->graph_captures = ctx->batch ? ctx->batch->captures : 0;
    out->graph_replays = ctx->batch ? ctx->batch->replays : 0;
    return RFR_OK;
}

extern "C" rfr_status rfr_prepare_batch(rfr_ctx *ctx, int count, const int64_t *coeffs, const int32_t *degrees,
                                        uint64_t *w_out, int32_t *n_out, uint64_t *t_lo, uint64_t *t_hi,
                                        int32_t *device_roots_out, rfr_status *status) {
    if (!ctx || count < 0 ||
        (count > 0 && (!coeffs || !degrees || !w_out || !n_out || !t_lo || !t_hi || !device_roots_out || !status)))
        return fail(RFR_EINVAL, "bad batch arguments");
    if (count == 0) return RFR_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(RFR_EDEVICE, "hipSetDevice failed");
    std::vector<size_t> off(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        if (degrees[i] < 1 || degrees[i] > RFR_MAX_DEGREE) return fail(RFR_EINVAL, "degree out of range");
        off[i + 1] = off[i] + (size_t)degrees[i] + 1;
    }
    if (!ctx->batch) {
        BatchState *b = new BatchState();
        if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess) {
            ctx->batch = b;
            batch_release(ctx);
            return fail(RFR_EDEVICE, "batch stream/event creation failed");
        }
        ctx->batch = b;
    }
    std::vector<Prepared> P(count);
    std::vector<rfr_status> st(count, RFR_OK);
    std::vector<std::string> err(count);
    for (int i = 0; i < count; ++i) st[i] = normalise(coeffs + off[i], degrees[i], P[i], err[i]);
    std::vector<const RootOut *> rec;
    rfr_status e = device_roots(ctx->batch, ctx->main.stream, P, st, rec);
    if (e != RFR_OK) return e;
    for (int i = 0; i < count; ++i) {
        device_roots_out[i] = 0;
        n_out[i] = 0;
        t_lo[i] = t_hi[i] = 0;
        if (st[i] == RFR_OK) device_roots_out[i] = finish_or_host(P[i], rec[i], st[i], err[i]) ? 1 : 0;
        status[i] = st[i];
        if (st[i] != RFR_OK) continue;
        n_out[i] = P[i].n;
        t_lo[i] = P[i].t_lo;
        t_hi[i] = P[i].t_hi;
        std::memcpy(w_out + off[i] - i, P[i].w.data(), P[i].w.size() * 8);
    }
    return RFR_OK;
}
