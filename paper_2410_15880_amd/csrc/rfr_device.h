// Device pipeline of the recombination search: tunables, argument structs and
// the host-side enqueue entry points (implemented in rfr_device.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rfr_internal.h"

namespace rfr {

namespace dev {
// ---- K0/K1/K4: Gray-code enumeration (256 lanes own the low 8 pattern bits)
constexpr int NT1 = 256;          // threads per workgroup
constexpr int KPT1 = 32;          // Gray steps per thread per tile of the count pass (with over 2^8 buckets)
constexpr int TILES1 = 8;         // KPT1-step tiles per K0/K1 workgroup of a half above 2^28 keys
constexpr int MAXB1_LOG = 12;     // level-1 digit bits (buckets) at most (12 only for halves of 2^34 keys)
constexpr int MAXB1 = 1 << MAXB1_LOG;
// ---- K2: per-bucket tile sort by the level-2 digit
constexpr int KPT2 = 8;           // keys per K2 thread
constexpr int T2_LOG = 12;        // level-2 tile of 2^12 keys (512-thread K2 workgroups)
constexpr int T2_BIG_LOG = 13;    // 2^13 keys (1024 threads) for one search with long level-1 buckets
                                  // (tiles <= 65535 keys: u16 digit offsets)
constexpr int MAXB2_LOG = 12;
constexpr int MAXB2 = 1 << MAXB2_LOG;
// ---- K3: sub-bucket gather, LDS radix sort of B', band join probing it with A
constexpr int NT3 = 256;
constexpr int SUB_LOG = 10;       // mean keys of the larger half per sub-bucket = 2^SUB_LOG (at most)
constexpr int SUB_LOG_MIN = 9;    // smallest sub-bucket mean the tuner may choose
constexpr int KP3 = 8;            // key slots per thread per half (registers)
constexpr int CAP3 = NT3 * KP3;   // keys per half a sub-bucket may hold on the fast path
constexpr int LB3 = 10;           // bits of the in-LDS counting sort of B'
constexpr int NB3 = 1 << LB3;
constexpr int CB3 = 15;           // bits of the semi-join's cell bitmaps
constexpr int LCAP3 = 512;        // entries of each semi-join list
constexpr int FB3 = 2048;         // B' keys staged per pass of the exact fallback
constexpr int NTS = 256;          // threads of the small-search kernel
constexpr int MAXT = 256;         // tile rows staged per gather chunk
// ---- K4/K5: candidate keys -> patterns
constexpr int KCAP_MAX = 4096;    // key pairs held per search
constexpr int RBITS_LOG = 18;     // LDS bitmap of candidate-key prefixes
constexpr int RBITS = 1 << RBITS_LOG;
constexpr int MAX_HALF = 34;      // elements per enumerated half (2^34 keys)
constexpr int MAX_SEARCH_N = 2 * MAX_HALF + 2;  // elements of a search (n - 1 = 69 leaves half A
                                  // 35 weights: it is then streamed in at least 2 chunks)
constexpr int MAX_CHUNK_BITS = 8; // half A streamed in at most 2^8 chunks
constexpr int RECOVER_FEW = 128;  // candidate key pairs handled by the meet-in-the-middle recovery
constexpr int RECOVER_WGS = 512;  // workgroups per half of a single search's many-candidate recovery
constexpr int SPT4 = 2;           // Gray steps per thread in that recovery (enough workgroups to fill the chip)

struct HalfArgs {
    uint64_t *keys;      // [N] partitioned keys
    uint64_t *hist1;     // [2^B1][nwg1] counts, then exclusive prefixes
    uint64_t *bstart;    // [2^B1 + 1] bucket starts
    uint32_t *tstart;    // [2^B1 + 1] first level-2 tile of each bucket
    uint16_t *digstart;  // [2^B2 + 1][ntile2_max] digit offsets inside each tile
    uint64_t N;          // 2^m
    uint64_t steps;      // 2^(m - L) Gray steps
    uint32_t spw;        // Gray steps per K0/K1/K4 workgroup
    uint32_t nwg1;       // K0/K1/K4 workgroups
    uint32_t ntile2_max; // level-2 tile capacity
    int m, L;            // weights in this half, lane bits
    int t2log;           // level-2 tile = 2^t2log keys
};

struct JobArgs {
    HalfArgs h[2];              // 0 = half A, 1 = half B' (negated)
    uint64_t wts[2][MAX_HALF];  // weights of each half (B' already negated)
    int B1, B2;                 // level-1 / level-2 digit bits
    uint64_t t_lo, t_hi;        // accept window
    uint64_t *kp;               // [2*kcap] candidate key pairs (a, b')
    uint64_t *kp_count;
    uint64_t kcap;
    uint64_t *rec;              // [2][kcap][2] (key, pattern) per half
    uint64_t *rec_count;        // [2]
    uint64_t *out;              // [2*cap] pattern pairs
    uint64_t *out_count;
    uint64_t cap;
    uint32_t *flags;            // bit 0: sort overflow, bit 1: join fallback used
    // chunked half A: every enumerated key of half h gets kbase[h] added and
    // every recovered pattern pbase[h] or-ed in (the chunk's fixed high bits)
    uint64_t kbase[2];
    uint64_t pbase[2];
    int first_chunk;            // 1: this launch starts the pattern count at 0
};

// Stages of the pipeline (kernel launches), in launch order.
enum Stage { ST_INIT, ST_COUNT, ST_COLS, ST_BUCKETS, ST_ENUM, ST_TILE2, ST_JOIN, ST_RFEW, ST_RMANY, ST_PAIRS, NSTAGES };

// Blocks per entry of a stage's block -> job table (see pick()).
constexpr uint32_t PICK_GRP = 64;

// Batch of jobs in device memory (see pick() in rfr_device.hip).
struct Multi {
    const JobArgs *jobs;
    const uint32_t *bases;      // [NSTAGES][njobs + 1]
    int njobs;
    const uint32_t *groups;     // per stage: job of block g * PICK_GRP, g = 0..ceil(grid / PICK_GRP), then njobs - 1
    uint32_t gofs[NSTAGES];     // start of each stage's table in groups
};
}  // namespace dev

// Optional events recorded between stages (any entry may be null):
// 0 start, 1 after count, 2 after scans, 3 after K1, 4 after K2, 5 after K3, 6 end.
struct StageEvents {
    void *ev[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
};

struct HalfPlan {
    int m = 0, L = 0;
    uint64_t N = 0, steps = 0;
    uint32_t spw = 0, nwg1 = 0, ntile2_max = 0;
    dev::HalfArgs a{};
};

struct JobPlan {
    int nhalves = 2;
    HalfPlan h[2];
    int B1 = 0, B2 = 0;
    int t2log = dev::T2_LOG;
    int sub = dev::SUB_LOG;  // log2 of the mean keys per sub-bucket of the larger half
    uint64_t kcap = dev::KCAP_MAX;
    uint64_t *kp = nullptr, *rec = nullptr, *counters = nullptr;
};

// Many searches launched stage by stage (one launch per stage for all jobs).
struct MultiLaunch {
    std::vector<dev::JobArgs> jobs;
    std::vector<std::vector<uint32_t>> bases;  // [stage][job + 1]
    int maxB1 = 0, maxB2 = 0, maxT2 = dev::T2_LOG;
    void add(const JobPlan &P, const dev::JobArgs &J);
    // bases, then the per-stage block -> job tables (bytes; see Multi)
    size_t bases_bytes() const;
    void pack_bases(uint32_t *dst) const;
    hipError_t launch(const dev::JobArgs *jobs_dev, const uint32_t *bases_dev, hipStream_t st,
                      StageEvents *ev = nullptr) const;
};

// A search small enough for one workgroup's LDS (both halves <= 2^SMALL_HALF).
constexpr int SMALL_HALF = 11;
struct SmallJob {
    uint64_t w[2 * SMALL_HALF];  // the n-1 searched weights
    int na, nb;
    uint64_t t_lo, t_hi;
    uint64_t *out;        // [2*cap] pattern pairs
    uint64_t *out_count;  // count, or ~0 on overflow
    uint64_t cap;
};


// Autotuned digit split for one size class (log2 of the larger half).
struct Tune {
    int b1;          // level-1 digit bits (-1: default)
    int sub_log;     // log2 of the mean keys per sub-bucket (SUB_LOG_MIN..SUB_LOG; -1: default)
    double ms;       // time measured by the autotuner
    int design = 0;  // 1: the query design (Algorithm E variant) was faster for this size class
};
void set_tune(int lg, Tune t);
Tune get_tune(int lg);

// Workspace bytes for a search of half sizes (na, nb); nb < 0 = one half only.
// `batch`: the search runs beside many others in one launch per stage.
uint64_t plan_job(int na, int nb, JobPlan &P, uint64_t kcap, bool batch = false);
// Lay the job out at ws and fill its kernel arguments (B' weights negated).
void build_job(JobPlan &P, char *ws, const uint64_t *wa, const uint64_t *wb, uint64_t t_lo, uint64_t t_hi,
               uint64_t *out, uint64_t *out_count, uint64_t cap, dev::JobArgs &J);
hipError_t launch_small(const SmallJob *jobs_dev, int njobs, uint32_t *queue_dev, int grid, hipStream_t st);
size_t recombine_workspace(int n);
// Chunk bits of half A so that a search over n weights fits ws_bytes (-1: none).
int chunk_bits(int n, size_t ws_bytes);
size_t expand_workspace(int m);

rfr_status enqueue_recombine(const uint64_t *w, int n, uint64_t t_lo, uint64_t t_hi, void *ws,
                             size_t ws_bytes, hipStream_t st, uint64_t *cand, uint64_t cap,
                             uint64_t *count, StageEvents *ev, std::string &err);
// Allocation-free search: the workspace is a fixed device array of
// NOALLOC_WS_BYTES per GPU (searches of up to NOALLOC_MAX_N elements fit it,
// the larger ones streaming half A in chunks).
constexpr size_t NOALLOC_WS_BYTES = 64ull << 20;
constexpr int NOALLOC_MAX_N = 46;
constexpr int NOALLOC_MAX_DEVICES = 64;
rfr_status enqueue_recombine_noalloc(const uint64_t *w, int n, uint64_t t_lo, uint64_t t_hi, hipStream_t st,
                                     uint64_t *cand, uint64_t cap, uint64_t *count, std::string &err);
// Algorithm E variant (Section 3.5): half B' expanded, sorted and laid out
// as a splat table; half A generated and queried, never stored.  Halves of at
// most 2^E_MAX_HALF keys.  A count of E_FALLBACK means the design could not
// run (B' sums too clustered for the expansion's sort): search with
// enqueue_recombine instead.
constexpr int E_MAX_HALF = 26;
constexpr uint64_t E_FALLBACK = ~0ull - 1;
size_t recombine_e_workspace(int n);
rfr_status enqueue_recombine_e(const uint64_t *w, int n, uint64_t t_lo, uint64_t t_hi, void *ws, size_t ws_bytes,
                               hipStream_t st, uint64_t *cand, uint64_t cap, uint64_t *count, std::string &err);
rfr_status enqueue_expand(const uint64_t *w, int m, int negate, void *ws, size_t ws_bytes,
                          hipStream_t st, uint64_t *sorted, std::string &err);

}  // namespace rfr
