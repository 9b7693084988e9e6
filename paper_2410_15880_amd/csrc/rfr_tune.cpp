// Autotuner of the search's radix split.
//
// For each size class (log2 of the larger half's key count) the tuner times
// the full device search on seeded random weights for every candidate split:
// the sub-bucket size (mean 2^9 or 2^10 keys of the larger half) and the
// number of level-1 bits (the rest go to the level-2 tile sort).  The fastest
// split of each class is installed for the process and written to a text
// table, which contexts load at creation (see tuning_autoload).
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "rfr_ctx.h"

namespace rfr {

static uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static bool load_table(const char *path) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    int loaded = 0;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        int lg, b1, sub, design = 0;
        double ms;
        const int got = std::sscanf(line, "%d %d %d %lf %d", &lg, &b1, &sub, &ms, &design);
        if (got < 4 || lg < 0 || lg > dev::MAX_HALF) continue;
        if (b1 >= 0 && b1 <= dev::MAXB1_LOG && sub >= dev::SUB_LOG_MIN && sub <= dev::SUB_LOG) {
            set_tune(lg, Tune{b1, sub, ms, design == 1 ? 1 : 0});
            ++loaded;
        } else if (b1 == -1 && sub == -1) {  // back to the fixed rule
            set_tune(lg, Tune{-1, -1, 0.0, 0});
            ++loaded;
        }
    }
    std::fclose(f);
    return loaded > 0;
}

// Load the table named by RFR_TUNING, else tuning/mi355x.txt beside the
// package that holds librfr.so; once per process.
void tuning_autoload() {
    static bool done = false;
    if (done) return;
    done = true;
    if (const char *p = std::getenv("RFR_TUNING")) {
        load_table(p);
        return;
    }
    Dl_info info;
    if (dladdr((void *)&tuning_autoload, &info) && info.dli_fname) {
        std::string so(info.dli_fname);
        size_t cut = so.rfind('/');
        if (cut != std::string::npos) {
            std::string dir = so.substr(0, cut);  // .../paper_2410_15880_amd/_lib
            size_t up = dir.rfind('/');
            if (up != std::string::npos) load_table((dir.substr(0, up) + "/tuning/mi355x.txt").c_str());
        }
    }
}

}  // namespace rfr

using namespace rfr;

extern "C" rfr_status rfr_load_tuning(const char *path) {
    if (!path) return fail(RFR_EINVAL, "path is NULL");
    if (!load_table(path)) return fail(RFR_EINVAL, "no tuning entries read from the file");
    return RFR_OK;
}

extern "C" rfr_status rfr_autotune(rfr_ctx *ctx, int lg_lo, int lg_hi, const char *path_out) {
    // lg = 32 times searches over n = 65 weights (both halves 2^32 keys, about
    // 80 GB of tables); larger classes would not fit twice in one GPU's memory
    if (!ctx || lg_lo < 8 || lg_hi > 32 || lg_lo > lg_hi) return fail(RFR_EINVAL, "need 8 <= lg_lo <= lg_hi <= 32");
    if (ctx->serving) return fail(RFR_EBUSY, "stop serving before tuning");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(RFR_EDEVICE, "hipSetDevice failed");
    Slot &s = ctx->main;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(RFR_EDEVICE, "hipEventCreate failed");
    std::string table =
        "# rfr autotune table: lg b1 sub_log ms design (larger half 2^lg keys; time of one search;\n"
        "# design 1: the query design, Algorithm E, was faster than the best split)\n";
    rfr_status st = RFR_OK;
    for (int lg = lg_lo; lg <= lg_hi && st == RFR_OK; ++lg) {
        const int n = 2 * lg + 1;  // halves of 2^lg keys each
        uint64_t seed = 0x5EED0000ull + (uint64_t)lg;
        std::vector<uint64_t> w(n);
        for (auto &x : w) x = splitmix64(seed);
        Tune best{-1, -1, 1e30, 0};
        for (int sub = dev::SUB_LOG_MIN; sub <= dev::SUB_LOG; ++sub) {
            const int LB = lg > sub ? lg - sub : 0;
            // level-1 buckets much larger than the level-2 digit range only
            // add tiles per sub-bucket, so the sweep starts near an even split
            const int lo = std::max({0, LB - dev::MAXB2_LOG, (LB + 1) / 2 - 2});
            const int hi = std::min(LB, dev::MAXB1_LOG);
            for (int b1 = lo; b1 <= hi; ++b1) {
                set_tune(lg, Tune{b1, sub, 0.0, 0});
                rfr_status e = ensure_workspace(ctx, s, recombine_workspace(n));
                if (e != RFR_OK) {
                    st = e;
                    break;
                }
                double t = 1e30;
                std::string err;
                for (int rep = 0; rep < 4 && st == RFR_OK; ++rep) {
                    (void)hipEventRecord(e0, s.stream);
                    rfr_status r = enqueue_recombine(w.data(), n, (uint64_t)n + 5, 5, s.ws, s.ws_bytes, s.stream,
                                                     s.cand_dev, s.cap, s.count_dev, nullptr, err);
                    (void)hipEventRecord(e1, s.stream);
                    if (r != RFR_OK || hipEventSynchronize(e1) != hipSuccess) {
                        st = fail(RFR_EDEVICE, "search failed while tuning: " + err);
                        break;
                    }
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (rep > 0) t = std::min(t, (double)ms);  // first run warms up
                }
                if (t < best.ms) best = Tune{b1, sub, t, 0};
            }
        }
        // the query design over the same weights (halves of at most 2^E_MAX_HALF keys)
        if (st == RFR_OK && lg <= E_MAX_HALF) {
            rfr_status e = ensure_workspace(ctx, s, recombine_e_workspace(n));
            double t = 1e30;
            std::string err;
            for (int rep = 0; rep < 4 && e == RFR_OK; ++rep) {
                (void)hipEventRecord(e0, s.stream);
                rfr_status r = enqueue_recombine_e(w.data(), n, (uint64_t)n + 5, 5, s.ws, s.ws_bytes, s.stream,
                                                   s.cand_dev, s.cap, s.count_dev, err);
                (void)hipEventRecord(e1, s.stream);
                if (r != RFR_OK || hipEventSynchronize(e1) != hipSuccess) {
                    st = fail(RFR_EDEVICE, "query design failed while tuning: " + err);
                    break;
                }
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) t = std::min(t, (double)ms);
            }
            if (t < best.ms) {
                best.design = 1;
                best.ms = t;
            }
        }
        set_tune(lg, best);
        char buf[96];
        std::snprintf(buf, sizeof buf, "%d %d %d %.4f %d\n", lg, best.b1, best.sub_log, best.ms, best.design);
        table += buf;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RFR_OK) return st;
    if (path_out) {
        FILE *f = std::fopen(path_out, "w");
        if (!f) return fail(RFR_EINVAL, "cannot write the tuning table");
        std::fputs(table.c_str(), f);
        std::fclose(f);
    }
    return RFR_OK;
}
