// Context, device slots and the shared helpers of the ABI, batch and serving
// translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "rfr_device.h"
#include "rfr_internal.h"

namespace rfr {

// One device lane of work: a stream, a search workspace (grown on demand) and
// candidate buffers (device + pinned host).
// Buffers for finding one polynomial's roots on the device: coefficients,
// job descriptor and root records, pinned staging of the same layout.
struct RootBuf {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *dev = nullptr;
    char *host = nullptr;
};

struct Slot {
    hipStream_t stream = nullptr;
    bool own_stream = true;      // false: the stream is a serving lane shared with other slots
    RootBuf roots;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    uint64_t *cand_dev = nullptr;
    uint64_t *count_dev = nullptr;
    uint64_t *host = nullptr;  // pinned: [2*cap] candidates + count
    uint64_t cap = 0;
    bool busy = false;
};

struct Request {
    uint64_t ticket = 0;
    std::vector<int64_t> coeffs;
    double t_submit = 0, t_done = 0;
    rfr_status status = RFR_EBUSY;
    rfr_result *result = nullptr;
};

struct BatchState;  // persistent-kernel batch resources (rfr_batch.cpp)
struct BigJob;      // serving: a prepared search waiting for slot 0 (rfr_serve.cpp)

}  // namespace rfr

struct rfr_ctx {
    int device = 0;
    size_t budget = 0;
    size_t mem_used = 0;         // bytes of search workspaces held
    uint64_t cap = 65536;        // candidate patterns per polynomial
    int design = 0;              // search design: 0 per size class (tuning table), 1 Horowitz-Sahni, 2 query (E)
    rfr::Slot main;              // slot of the plain path
    // ---- serving
    bool serving = false;
    std::vector<rfr::Slot> slots;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_slot;
    std::deque<rfr::Request *> queue;
    std::map<uint64_t, rfr::Request *> reqs;
    int big_running = 0;         // admitted searches that fill the GPU on their own
    std::deque<rfr::BigJob *> big_jobs;  // serving: handed-off searches for slot 0, in arrival order
    std::vector<std::thread> big_workers;
    std::condition_variable cv_big;
    bool big_stopping = false;
    int n_big = 0;                     // serving: 1 when slot 0 takes the searches that fill the GPU
    hipStream_t lane_big = nullptr;    // serving: the stream of the searches that fill the GPU
    hipStream_t lane_small = nullptr;  // serving: the stream of every other request's device work
    uint64_t next_ticket = 1;
    bool stopping = false;
    // ---- batch
    rfr::BatchState *batch = nullptr;
    // ---- profiling (per-stage HIP events)
    bool profiling = false;
    rfr_profile_t prof{};
    std::vector<hipEvent_t> prof_ev;
    std::vector<rfr::StageEvents> prof_se;
    uint64_t prof_graph_replays = 0, prof_graph_captures = 0;
};

namespace rfr {
extern thread_local std::string g_last_error;
rfr_status fail(rfr_status st, const std::string &msg);
double now_ms();
rfr_result *pack_result(const Prepared &P, const Factored &F);
rfr_status ensure_workspace(rfr_ctx *ctx, Slot &s, size_t need);
// A slot with a stream of its own, or on `lane` (not owned) when given.
rfr_status slot_init(rfr_ctx *ctx, Slot &s, hipStream_t lane = nullptr);
void slot_free(rfr_ctx *ctx, Slot &s);
// *folded (if given) is set to 1 when the search had to fold the second trace
// into the weights (a first search overflowed the candidate capacity).
rfr_status search_on_slot(rfr_ctx *ctx, Slot &s, const Prepared &P, std::vector<Pat> &cands,
                          int *folded = nullptr);
size_t choose_workspace(int n, size_t avail);
void tuning_autoload();

// Root buffers on a given stream (nullptr: the buffers get a stream of their own).
rfr_status rootbuf_init(RootBuf &b, hipStream_t stream);
void rootbuf_free(RootBuf &b);
// normalise + elements, weights and window with the roots found on the device
// (one workgroup on b.stream); the host finds them itself for degree < 2 or
// when the device roots fail the disc checks.
rfr_status prepare_dev(RootBuf &b, const int64_t *coeffs, int degree, Prepared &P, std::string &err);
rfr_status factor_on_slot(rfr_ctx *ctx, Slot &s, const int64_t *coeffs, int degree, rfr_result **out);

// Square-free decomposition (Yun): p = content * prod parts[j].first ^ parts[j].second,
// parts primitive, square-free, lc > 0, pairwise coprime, sorted by (multiplicity,
// degree, coefficients); a factor x is its own part.
rfr_status squarefree_decompose(const int64_t *coeffs, int degree, int64_t &content,
                                std::vector<std::pair<std::vector<int64_t>, int>> &parts, std::string &err);
// Factorisation of a polynomial the square-free path rejected: every
// square-free part goes through `one` (the square-free path), its factors are
// listed by multiplicity.
using FactorOne = std::function<rfr_status(const int64_t *coeffs, int degree, rfr_result **out)>;
rfr_status factor_sqf_route(const int64_t *coeffs, int degree, const FactorOne &one, rfr_result **out);
void batch_release(rfr_ctx *ctx);
StageEvents *profile_events(rfr_ctx *ctx, int k);
void profile_collect(rfr_ctx *ctx, int k, int n);
}  // namespace rfr
