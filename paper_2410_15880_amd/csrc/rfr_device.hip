// Device side of the RFR recombination search for gfx950 (CDNA4, wave64).
//
// Paper: Iravanian, arXiv 2410.15880, Section 3.3 (Algorithm C = EXPAND both
// halves, sort, FIND).  The weights are the 64-bit integers of Eq 18; a pattern
// is accepted when its sum mod 2^64 lies in [2^64 - t_lo, 2^64) U [0, t_hi]
// (the integer form of Eq 19 widened by the quantisation and root error).
//
// Pipeline for one search over n-1 weights split into half A (n_a weights) and
// half B (n_b weights); half B is enumerated negated (B' = -B) so a match is
// A ~ B' within the window:
//   K0 k_enum<true>   Gray-code enumeration, level-1 digit histogram per WG
//   S1 k_scan_cols    per-bucket exclusive prefix over WGs
//   S2 k_scan_buckets bucket starts and level-2 tile table
//   K1 k_enum<false>  Gray-code enumeration, LDS counting sort of each tile by
//                     the level-1 digit (the tile held as a (step, lane)
//                     permutation), run-coalesced stores into buckets
//   K2 k_tile2        LDS counting sort of each bucket tile by the level-2
//                     digit, written back in place + per-digit tile offsets
//   K3 k_join         per sub-bucket (level-1 + level-2 prefix): gather both
//                     halves into registers, semi-join through LDS cell
//                     bitmaps (B' marks cells, A keys meeting a marked cell
//                     and the B' keys in their cells form two short lists),
//                     exact test of every list pair; every key pair in the
//                     window is emitted
//   K4 k_recover_few  candidate keys back to patterns: a meet in the middle
//      k_recover      inside each half (few keys), or a re-enumeration of
//                     the half against an LDS bitmap of the keys (many)
//   K5 k_pairs        one workgroup: de-duplicate key pairs, expand them into
//                     pattern pairs
// All arithmetic on keys is exact wrapping uint64.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "rfr_device.h"

namespace rfr {
namespace dev {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ uint32_t dig(uint64_t key, int shift, uint32_t mask) {
    return shift >= 64 ? 0u : (uint32_t)(key >> shift) & mask;
}

// Inclusive scan across one wavefront (64 lanes).
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread across the workgroup; returns the
// exclusive prefix and writes the block total to *total (all threads).
template <int NTH>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t *s_tmp, uint64_t *total) {
    constexpr int NW = NTH / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint64_t inc = wave_incl_scan(v);
    if (lane == 63) s_tmp[wv] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = 0;
        for (int i = 0; i < NW; ++i) {
            uint64_t t = s_tmp[i];
            s_tmp[i] = acc;
            acc += t;
        }
        s_tmp[NW] = acc;
    }
    __syncthreads();
    uint64_t r = inc - v + s_tmp[wv];
    *total = s_tmp[NW];
    __syncthreads();
    return r;
}

// Exclusive scan, in place, of an LDS array of n <= NTH*PER entries.
template <int NTH, int PER, typename T>
__device__ __forceinline__ uint64_t lds_excl_scan(T *a, int n, uint64_t *s_tmp) {
    uint64_t loc[PER];
    uint64_t sum = 0;
    const int base = threadIdx.x * PER;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        loc[k] = (base + k < n) ? (uint64_t)a[base + k] : 0;
        sum += loc[k];
    }
    uint64_t tot;
    uint64_t pre = block_excl_scan<NTH>(sum, s_tmp, &tot);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (base + k < n) a[base + k] = (T)pre;
        pre += loc[k];
    }
    __syncthreads();
    return tot;
}

// Cyclic window test on d = b' - a (mod 2^64): d in [2^64 - t_hi, 2^64) U [0, t_lo].
__device__ __forceinline__ bool in_win(uint64_t a, uint64_t b, uint64_t t_lo, uint64_t t_hi) {
    uint64_t dlt = b - a;
    return dlt <= t_lo || (0 - dlt) <= t_hi;
}

__device__ __forceinline__ void emit_pair(const JobArgs &J, uint64_t a, uint64_t b) {
    unsigned long long idx = atomicAdd((unsigned long long *)J.kp_count, 1ull);
    if (idx < J.kcap) {
        J.kp[2 * idx] = a;
        J.kp[2 * idx + 1] = b;
    }
}

// ------------------------------------------------------------------ job selection
// A launch serves one search (MULTI = false: the job is the kernel argument)
// or every search of a batch (MULTI = true: M.jobs in device memory and, per
// stage, M.bases[stage][0..njobs] the first block of each job, so block x
// belongs to the last job j with bases[j] <= x).  The stage's table in
// M.groups names the jobs of blocks g * PICK_GRP and (g + 1) * PICK_GRP, which
// bound x's job, so the search among bases takes a step or two instead of
// log2(njobs) dependent loads.  The job's arguments are read through the
// constant address space (no kernel writes them): scalar loads that stay
// valid across barriers, and the pointers in them are known to be global, as
// they are when the job is the kernel argument.
template <bool MULTI>
__device__ __forceinline__ bool pick(const JobArgs &arg, const Multi &M, int stage, const JobArgs *&J, uint32_t &bx) {
    if (!MULTI) {
        J = &arg;
        bx = blockIdx.x;
        return true;
    }
    const uint32_t *base = M.bases + (size_t)stage * (M.njobs + 1);
    const uint32_t *grp = M.groups + M.gofs[stage];
    const uint32_t x = blockIdx.x;
    if (x >= base[M.njobs]) return false;
    int lo = (int)grp[x / PICK_GRP], hi = (int)grp[x / PICK_GRP + 1];  // lo <= job(x) <= hi
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    J = (const JobArgs *)((const __attribute__((address_space(4))) JobArgs *)M.jobs + lo);
    bx = x - base[lo];
    return true;
}

// ------------------------------------------------------------------ init
template <bool MULTI>
__global__ void k_init(JobArgs Jarg, Multi M) {
    const JobArgs *Jp;
    uint32_t bx;
    if (!pick<MULTI>(Jarg, M, ST_INIT, Jp, bx)) return;
    const JobArgs &J = *Jp;
    if (threadIdx.x == 0) {
        *J.kp_count = 0;
        J.rec_count[0] = 0;
        J.rec_count[1] = 0;
        if (J.out_count && J.first_chunk) *J.out_count = 0;
        *J.flags = 0;
    }
}

// ------------------------------------------------------------------ K0 / K1
// Work of one workgroup: Gray-code steps [h0, h1) of its half.  Lane l owns the
// low L pattern bits (its partial sum is fixed); step h selects the high bits
// gray(h) = h ^ (h >> 1), so going from h to h+1 flips exactly bit ctz(h+1) and
// changes the high sum by one wavefront-uniform +-w.
template <bool COUNT, int NBMAX, bool MULTI>
__global__ __launch_bounds__(NT1) __attribute__((amdgpu_waves_per_eu(!COUNT ? 3 : 2))) void k_enum(JobArgs Jarg, Multi M) {
    const JobArgs *Jp;
    uint32_t wg;
    if (!pick<MULTI>(Jarg, M, COUNT ? ST_COUNT : ST_ENUM, Jp, wg)) return;
    const JobArgs &J = *Jp;
    const HalfArgs &H = J.h[blockIdx.y];
    if (wg >= H.nwg1) return;
    // Workgroup w's keys of bucket b fill the range between w - 1's and
    // w + 1's, so the cache lines at those seams are shared.  Neighbouring
    // workgroups run on the same XCD (hardware deals workgroups out to the 8
    // XCDs in turn), and odd workgroups fill their ranges from the top down, so
    // both halves of a seam line are written at about the same time (in both
    // workgroups' first tile, or both their last) into the same L2 instead of
    // reaching memory as two partial writes.
    if (!COUNT && !MULTI && (H.nwg1 & 7) == 0 && H.nwg1 >= 64) wg = (wg & 7) * (H.nwg1 >> 3) + (wg >> 3);
    const bool back = !COUNT && (wg & 1);
    const int B1 = J.B1;
    const int nb = 1 << B1;
    const int sh1 = 64 - B1;
    const uint32_t m1 = (uint32_t)nb - 1;
    const int tid = threadIdx.x;
    const int nl = 1 << H.L;
    const bool act = tid < nl;

    __shared__ uint64_t s_w[64];
    __shared__ uint32_t s_cnt[NBMAX];
    __shared__ uint32_t s_off[NBMAX];
    __shared__ uint64_t s_cur[COUNT ? 1 : NBMAX];
    __shared__ uint64_t s_tmp[NT1 / 64 + 1];
    // The partition pass keeps the tile in LDS as a permutation, not as
    // keys: a key is its lane's low sum plus its step's high sum (the same
    // for the whole workgroup), so sorted slot p holds (step << 8 | lane) and
    // the store phase rebuilds the key from two small tables.  Two bytes of
    // LDS per key instead of eight and no keys held in registers, so a tile
    // takes 64 steps (16,384 keys: runs per bucket twice as long) at more
    // workgroups per CU.  Per degree-100 search 0.268 ms against 0.306 with
    // 8192-key tiles of keys; with 2^10 and 2^11 buckets (halves of 2^30 to
    // 2^33 keys) 9.4 and 44 ms against 12.4 and 54.  With 2^11 buckets and
    // more a tile takes 128 steps (one workgroup per CU, runs of ~8 keys per
    // bucket instead of ~4): K1 at n = 65 52.2-53.6 -> 48.5-49 ms; with 2^10
    // buckets the 64-step tiles' two workgroups per CU are faster (halves of
    // 2^29 keys 11.3 against 13.0 ms per search).
    constexpr int KPTP = NBMAX >= 2048 ? 128 : 64;  // Gray steps per partition tile
    __shared__ uint16_t s_perm[COUNT ? 1 : NT1 * KPTP];
    __shared__ uint64_t s_slo[COUNT ? 1 : NT1];
    __shared__ uint64_t s_shi[COUNT ? 1 : KPTP];

    // A partition workgroup of a single tile (spw == KPTP) knows the tile's
    // bucket counts from the count pass (its range of bucket b holds hi - lo
    // keys, the same keys K0 counted for this workgroup), so it skips the
    // counting walk below and only needs the tile's step sums (0.199 -> 0.186
    // ms per degree-100 search).
    const bool one = !COUNT && H.spw == (uint32_t)KPTP;
    if (tid < H.m) s_w[tid] = J.wts[blockIdx.y][tid];
    for (int b = tid; b < nb; b += NT1) {
        uint32_t c = 0;
        if (!COUNT) {
            // range of (b, wg): [bstart + prefix(wg), bstart + prefix(wg + 1))
            const uint64_t lo = H.hist1[(size_t)b * H.nwg1 + wg];
            const uint64_t hi = wg + 1 < H.nwg1 ? H.hist1[(size_t)b * H.nwg1 + wg + 1] : H.bstart[b + 1] - H.bstart[b];
            s_cur[b] = H.bstart[b] + (back ? hi : lo);
            if (one) c = (uint32_t)(hi - lo);
        }
        s_cnt[b] = c;
    }
    uint64_t *const keys_out = H.keys;
    __syncthreads();

    uint64_t slo = J.kbase[blockIdx.y];
    for (int i = 0; i < H.L; ++i)
        if ((tid >> i) & 1) slo += s_w[i];
    if (!COUNT && act) s_slo[tid] = slo;
    const uint64_t h0 = (uint64_t)wg * H.spw;
    const uint64_t h1 = min(h0 + (uint64_t)H.spw, H.steps);
    uint64_t g = h0 ^ (h0 >> 1);
    uint64_t shi = 0;
    for (int i = 0; i < H.m - H.L; ++i)
        if ((g >> i) & 1) shi += s_w[H.L + i];
    // Tiles start at multiples of KPT steps, so inside a tile step k + 1 flips
    // bit ctz(k + 1) < log2 KPT: those weights sit in registers and only the
    // step into the next tile reads its weight by a computed index.  The count
    // pass, which keeps no tile in LDS, walks 16 steps at a time into at most
    // 256 buckets: half the registers of the keys, more waves in flight
    // (measured 0.064 against 0.076 ms per degree-100 search; with 2048
    // buckets, where its LDS counters are contended, 8.1 against 5.1 ms at
    // n = 65); the partition pass keeps KPT1-step tiles, whose longer runs per
    // bucket store faster than more waves would gain.
    constexpr int KPT = COUNT ? (NBMAX == NT1 ? 16 : KPT1) : KPTP;
    static_assert((KPT1 * TILES1) % KPTP == 0, "ranges of whole partition tiles");
    constexpr int LOGK = __builtin_ctz(KPT);
    static_assert((1 << LOGK) == KPT && (KPT1 * TILES1) % KPT == 0, "tiles of a power-of-two number of Gray steps");
    const int mh = H.m - H.L;
    uint64_t wlow[LOGK];
#pragma unroll
    for (int i = 0; i < LOGK; ++i) wlow[i] = mh > i ? s_w[H.L + i] : 0;

    for (uint64_t h = h0; h < h1; h += KPT) {
        const int ns = (int)min((uint64_t)KPT, h1 - h);
        // each key's level-1 digit is counted as the Gray walk produces it;
        // the partition pass ranks the keys in a second pass below, so no
        // rank is held in registers across the tile
        if (one) {
            // counts known: thread k only forms step k's high sum (a tile
            // starts the workgroup's range, so there is no next tile)
            if (tid < ns) {
                const uint64_t t = h + (uint64_t)tid;
                const uint64_t gk = t ^ (t >> 1);
                uint64_t sh = 0;
                for (int i = 0; i < mh; ++i)
                    if ((gk >> i) & 1) sh += s_w[H.L + i];
                s_shi[tid] = sh;
            }
        } else {
#pragma unroll
            for (int k = 0; k < KPT; ++k) {
                const uint64_t key = slo + shi;
                if (act && k < ns) atomicAdd(&s_cnt[dig(key, sh1, m1)], 1u);
                if (!COUNT && tid == 0 && k < ns) s_shi[k] = shi;  // the same for every lane
                const uint64_t t = h + k + 1;
                if (k < ns && t < h1) {
                    const int b = k < KPT - 1 ? __builtin_ctz(k + 1) : __builtin_ctzll(t);
                    const uint64_t wb = k < KPT - 1 ? wlow[__builtin_ctz(k + 1) % LOGK] : s_w[H.L + b];
                    g ^= 1ull << b;
                    shi += ((g >> b) & 1) ? wb : (0 - wb);
                }
            }
        }
        if constexpr (COUNT) continue;
        __syncthreads();
        if (NBMAX == NT1) {
            uint64_t tot;
            const uint32_t c = tid < nb ? s_cnt[tid] : 0;
            const uint64_t ex = block_excl_scan<NT1>(c, s_tmp, &tot);
            if (tid < nb) s_off[tid] = (uint32_t)ex;
            __syncthreads();
        } else {
            for (int b = tid; b < nb; b += NT1) s_off[b] = s_cnt[b];
            __syncthreads();
            lds_excl_scan<NT1, NBMAX / NT1>(s_off, nb, s_tmp);
        }
        // second pass over the tile: each key, rebuilt from its lane's and
        // step's sums, takes the next slot of its bucket (s_off as cursor).
        // Holding the 64 ranks of the first pass in registers instead took
        // 168 VGPRs (three workgroups per CU); with this pass K1 holds 84 and
        // LDS allows four: 0.243 -> 0.198 ms per degree-100 search.  The order
        // of keys inside a bucket is free: K2 sorts them and every later
        // result is a set.
        if (act) {
#pragma unroll 8
            for (int k = 0; k < ns; ++k) {
                const uint32_t slot = atomicAdd(&s_off[dig(slo + s_shi[k], sh1, m1)], 1u);
                s_perm[slot] = (uint16_t)((k << 8) | tid);
            }
        }
        __syncthreads();
        // s_off back to the bucket starts; destination of tile slot p of
        // bucket d: s_cur[d] - s_off[d] + p, the cursor first stepping down by
        // the run length when filling downwards
        for (int b = tid; b < nb; b += NT1) {
            const uint32_t st = s_off[b] - s_cnt[b];
            s_off[b] = st;
            s_cur[b] -= st + (back ? s_cnt[b] : 0u);
        }
        __syncthreads();
        const int tile = ns * nl;
        // in groups of 8 slots: LDS reads first (slots past the tile read stale
        // data and store nothing), then the stores; `keys_out` is a local so
        // that the stores do not make the compiler reload it from the argument
        // block between them
        auto store8 = [&](int i0) {
            uint64_t kv[8], dst[8];
            bool inner[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                // slots past the tile hold stale entries: masked into the tables
                const uint32_t e = s_perm[tid + (i0 + i) * NT1];
                kv[i] = s_slo[e & 255u] + s_shi[(e >> 8) & (KPTP - 1)];
            }
            // a key whose 128-byte line lies inside its run [g0, g1) (all 16
            // keys of the line come from this store phase) is streamed out;
            // the run's end lines, shared with other workgroups' runs, are
            // merged in L2 first
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t d = dig(kv[i], sh1, m1);
                const uint64_t c = s_cur[d];
                const uint64_t g0 = c + s_off[d];
                const uint64_t g1 = g0 + s_cnt[d];
                dst[i] = c + (uint64_t)(tid + (i0 + i) * NT1);
                const uint64_t l0 = dst[i] & ~(uint64_t)15;
                inner[i] = l0 >= g0 && l0 + 16 <= g1;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (tid + (i0 + i) * NT1 < tile) {
                    if (inner[i]) __builtin_nontemporal_store(kv[i], &keys_out[dst[i]]);
                    else keys_out[dst[i]] = kv[i];
                }
        };
        // the groups one after another: few registers, more workgroups
#pragma unroll 1
        for (int i0 = 0; i0 < KPT; i0 += 8) store8(i0);
        __syncthreads();
        for (int b = tid; b < nb; b += NT1) {
            s_cur[b] += s_off[b] + (back ? 0u : s_cnt[b]);
            s_cnt[b] = 0;
        }
        __syncthreads();
    }
    if (COUNT) {
        __syncthreads();
        for (int b = tid; b < nb; b += NT1) H.hist1[(size_t)b * H.nwg1 + wg] = s_cnt[b];
    }
}

// ------------------------------------------------------------------ S1 / S2
// Column prefix: hist1[b][w] becomes the exclusive prefix over w; the bucket
// total goes to bstart[b] (turned into bucket starts by S2).
template <bool MULTI>
__global__ __launch_bounds__(NT1) void k_scan_cols(JobArgs Jarg, Multi M) {
    const JobArgs *Jp;
    uint32_t bx;
    if (!pick<MULTI>(Jarg, M, ST_COLS, Jp, bx)) return;
    const JobArgs &J = *Jp;
    const HalfArgs &H = J.h[blockIdx.y];
    const int b = (int)bx;
    if (b >= (1 << J.B1)) return;
    __shared__ uint64_t s_tmp[NT1 / 64 + 1];
    uint64_t *col = H.hist1 + (size_t)b * H.nwg1;
    constexpr uint32_t SCAN_LDS = 4096;
    if (H.nwg1 <= SCAN_LDS) {
        // the column staged in LDS by coalesced loads; each thread scans a
        // contiguous chunk, one block scan joins the chunks (one block scan
        // instead of one per 256 entries).  One pad entry per 32 keeps the
        // threads' chunk strides off a single bank.
        __shared__ uint64_t s_col[SCAN_LDS + SCAN_LDS / 32];
        auto at = [](uint32_t i) { return i + (i >> 5); };
        const uint32_t n = H.nwg1, per = (n + NT1 - 1) / NT1;
        for (uint32_t i = threadIdx.x; i < n; i += NT1) s_col[at(i)] = col[i];
        __syncthreads();
        const uint32_t c0 = min(threadIdx.x * per, n), c1 = min(c0 + per, n);
        uint64_t sum = 0;
        for (uint32_t i = c0; i < c1; ++i) sum += s_col[at(i)];
        uint64_t tot;
        uint64_t run = block_excl_scan<NT1>(sum, s_tmp, &tot);
        for (uint32_t i = c0; i < c1; ++i) {
            const uint64_t v = s_col[at(i)];
            s_col[at(i)] = run;
            run += v;
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n; i += NT1) col[i] = s_col[at(i)];
        if (threadIdx.x == 0) H.bstart[b] = tot;
        return;
    }
    uint64_t carry = 0;
    for (uint32_t base = 0; base < H.nwg1; base += NT1) {
        const uint32_t i = base + threadIdx.x;
        const uint64_t v = i < H.nwg1 ? col[i] : 0;
        uint64_t tot;
        const uint64_t ex = block_excl_scan<NT1>(v, s_tmp, &tot);
        if (i < H.nwg1) col[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) H.bstart[b] = carry;
}

template <bool MULTI>
__global__ __launch_bounds__(NT1) void k_scan_buckets(JobArgs Jarg, Multi M) {
    const JobArgs *Jp;
    uint32_t bx;
    if (!pick<MULTI>(Jarg, M, ST_BUCKETS, Jp, bx)) return;
    const JobArgs &J = *Jp;
    const HalfArgs &H = J.h[blockIdx.y];
    const int nb = 1 << J.B1;
    __shared__ uint64_t s_tmp[NT1 / 64 + 1];
    uint64_t carry = 0, tcarry = 0;
    for (int base = 0; base < nb; base += NT1) {
        const int i = base + threadIdx.x;
        const uint64_t v = i < nb ? H.bstart[i] : 0;
        const uint64_t nt = (v + ((uint64_t)1 << H.t2log) - 1) >> H.t2log;
        uint64_t tot, ttot;
        const uint64_t ex = block_excl_scan<NT1>(v, s_tmp, &tot);
        const uint64_t tex = block_excl_scan<NT1>(nt, s_tmp, &ttot);
        if (i < nb) {
            H.bstart[i] = carry + ex;
            H.tstart[i] = (uint32_t)(tcarry + tex);
        }
        carry += tot;
        tcarry += ttot;
    }
    if (threadIdx.x == 0) {
        H.bstart[nb] = carry;
        H.tstart[nb] = (uint32_t)tcarry;
    }
}

// ------------------------------------------------------------------ K2
// One tile (<= NT*KPT2 = 2^t2log keys) of one level-1 bucket: counting sort by
// the level-2 digit in LDS, written back in place; digstart[d][tile] = offset
// of digit d inside the tile, digstart[nd][tile] = tile length.
template <int NBMAX, int NT, bool MULTI>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT >= 1024 ? 8 : 1))) void k_tile2(JobArgs Jarg, Multi M) {
    constexpr int TT = NT * KPT2;
    const JobArgs *Jp;
    uint32_t tile;
    if (!pick<MULTI>(Jarg, M, ST_TILE2, Jp, tile)) return;
    const JobArgs &J = *Jp;
    const HalfArgs &H = J.h[blockIdx.y];
    const int nb = 1 << J.B1;
    const uint32_t ntiles = H.tstart[nb];
    if (!MULTI) {
        // Consecutive tiles on one XCD (workgroups are dealt out to the 8 XCDs
        // in turn): tile t's digit offsets sit beside tile t+1's in every row
        // of digstart, so the rows' cache lines fill in one L2 instead of
        // reaching memory as many 2-byte partial writes.  The grid is a
        // multiple of 8 and at least 8 * ceil(ntiles / 8).
        const uint32_t chunk = (ntiles + 7) >> 3;
        if ((tile >> 3) >= chunk) return;
        tile = (tile & 7) * chunk + (tile >> 3);
    }
    if (tile >= ntiles) return;
    const int nd = 1 << J.B2;
    const int sh2 = 64 - J.B1 - J.B2;
    const uint32_t m2 = (uint32_t)nd - 1;
    const int tid = threadIdx.x;

    __shared__ uint64_t s_buf[TT];
    __shared__ uint32_t s_cnt[NBMAX];  // digit counts, then (scanned in place) digit offsets
    __shared__ uint64_t s_tmp[NT / 64 + 1];
    __shared__ int s_b;

    if (tid == 0) {
        int lo = 0, hi = nb - 1;  // largest b with tstart[b] <= tile
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (H.tstart[mid] <= tile) lo = mid;
            else hi = mid - 1;
        }
        s_b = lo;
    }
    for (int d = tid; d < nd; d += NT) s_cnt[d] = 0;
    __syncthreads();
    const int b = s_b;
    const uint64_t base = H.bstart[b] + ((uint64_t)(tile - H.tstart[b]) << H.t2log);
    const int len = (int)min((uint64_t)1 << H.t2log, H.bstart[b + 1] - base);  // <= TT by the launch
    uint64_t *const keys = H.keys + base;  // a local: stores must not force reloads of the argument block

    uint64_t key[KPT2];
    uint32_t rank[KPT2];
    // all loads first (independent, in flight together), then the ranks.  In
    // 1024-thread workgroups no branch: a slot past the tile's end re-reads
    // its last key (a tile holds at least one) and is not ranked.  Behind a
    // branch per slot the compiler moved the first slot's key between
    // registers before issuing the other loads, waiting for it: one more
    // memory round trip per workgroup.  (The 512-thread instantiations keep
    // the branches: without them their registers outgrow four workgroups per
    // CU.)
    if constexpr (NT >= 1024) {
#pragma unroll
        for (int k = 0; k < KPT2; ++k)
            key[k] = __builtin_nontemporal_load(&keys[min((uint32_t)(tid + k * NT), (uint32_t)len - 1u)]);
    } else {
#pragma unroll
        for (int k = 0; k < KPT2; ++k) {
            const int p = tid + k * NT;
            if (p < len) key[k] = __builtin_nontemporal_load(&keys[p]);
        }
    }
#pragma unroll
    for (int k = 0; k < KPT2; ++k) {
        const int p = tid + k * NT;
        if (p < len) rank[k] = atomicAdd(&s_cnt[dig(key[k], sh2, m2)], 1u);
    }
    __syncthreads();
    lds_excl_scan<NT, (NBMAX + NT - 1) / NT>(s_cnt, nd, s_tmp);
#pragma unroll
    for (int k = 0; k < KPT2; ++k) {
        const int p = tid + k * NT;
        if (p < len) s_buf[s_cnt[dig(key[k], sh2, m2)] + rank[k]] = key[k];
    }
    __syncthreads();
    uint64_t kv[KPT2];
#pragma unroll
    for (int k = 0; k < KPT2; ++k) kv[k] = s_buf[tid + k * NT];
    // streaming stores: the tile is written whole (K1's partial lines are
    // merged in L2 at its seams; K2 has none) and is next read by K3, long
    // after it would have left the caches
#pragma unroll
    for (int k = 0; k < KPT2; ++k)
        if (tid + k * NT < len) __builtin_nontemporal_store(kv[k], &keys[tid + k * NT]);
    for (int d = tid; d < nd; d += NT) H.digstart[(size_t)d * H.ntile2_max + tile] = (uint16_t)s_cnt[d];
    if (tid == 0) H.digstart[(size_t)nd * H.ntile2_max + tile] = (uint16_t)len;
}

// ------------------------------------------------------------------ K3
// Shared state of one sub-bucket of one half, gathered into LDS.
struct SubRef {
    uint32_t t0, t1;  // tile range of the level-1 bucket
    uint64_t pos0;    // bucket start
};

__device__ __forceinline__ SubRef sub_ref(const HalfArgs &H, int b) {
    SubRef r;
    r.t0 = H.tstart[b];
    r.t1 = H.tstart[b + 1];
    r.pos0 = H.bstart[b];
    return r;
}

// Visit every key of sub-bucket (b, d) of half H directly from global memory.
template <typename F>
__device__ __forceinline__ void for_each_global(const HalfArgs &H, int B2, int b, int d, F f) {
    const SubRef r = sub_ref(H, b);
    for (uint32_t t = r.t0; t < r.t1; ++t) {
        const uint32_t s = H.digstart[(size_t)d * H.ntile2_max + t];
        const uint32_t e = H.digstart[(size_t)(d + 1) * H.ntile2_max + t];
        const uint64_t tb = r.pos0 + ((uint64_t)(t - r.t0) << H.t2log);
        for (uint32_t q = s; q < e; ++q)
            if (!f(H.keys[tb + q])) return;
    }
}

// Partners of a in a neighbouring sub-bucket `ns` of half B' (slow path, rare):
// every key b there with b' - a in the window, except those the in-bucket
// merge already reported (b in [lo, hi] and inside sub-bucket s).
__device__ void edge_scan(const JobArgs &J, uint64_t a, uint32_t s, uint32_t ns, uint64_t lo, uint64_t hi) {
    const int LB = J.B1 + J.B2;
    const HalfArgs &HB = J.h[1];
    const int b = (int)(ns >> J.B2), d = (int)(ns & ((1u << J.B2) - 1));
    for_each_global(HB, J.B2, b, d, [&](uint64_t bk) {
        const bool in_s = LB == 0 || (uint32_t)(bk >> (64 - LB)) == s;
        if (in_win(a, bk, J.t_lo, J.t_hi) && !(in_s && bk >= lo && bk <= hi)) emit_pair(J, a, bk);
        return *J.kp_count <= J.kcap;
    });
}

// Exclusive prefix maximum across the workgroup of two 32-bit values packed in
// one 64-bit word (low and high halves taken separately); 0 is the identity.
__device__ __forceinline__ uint64_t max2(uint64_t x, uint64_t y) {
    const uint32_t lo = max((uint32_t)x, (uint32_t)y), hi = max((uint32_t)(x >> 32), (uint32_t)(y >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

template <int NTH>
__device__ __forceinline__ uint64_t block_excl_max2(uint64_t v, uint64_t *s_tmp) {
    constexpr int NW = NTH / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint64_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc = max2(inc, t);
    }
    uint64_t ex = __shfl_up(inc, 1, 64);
    if (lane == 0) ex = 0;
    if (lane == 63) s_tmp[wv] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = 0;
        for (int i = 0; i < NW; ++i) {
            const uint64_t t = s_tmp[i];
            s_tmp[i] = acc;
            acc = max2(acc, t);
        }
    }
    __syncthreads();
    ex = max2(ex, s_tmp[wv]);
    __syncthreads();
    return ex;
}

// Gather sub-bucket (b, d) of NH halves into register slots: key q of half h
// (q = tid + k*NT3) lands in kk[h][k].  The bucket's tiles are taken in chunks
// of MAXT.  Thread t holds tile t's digit-d segment bounds (per half; preloaded
// by the caller when the bucket has at most MAXT tiles); one packed block scan
// gives the segments' key offsets.  The tile map q -> tile is built in LDS
// without walking the segments: each non-empty segment puts its tile number at
// its first offset, and a prefix maximum over the map (tiles come in offset
// order) fills the rest; every thread owns CAP3 / NT3 consecutive map bytes per
// half.
// Each tile's key offset from the bucket start minus its first slot goes to
// LDS, so a slot's address is one LDS read and an add, and all slot loads of a
// chunk are in flight together.  Buckets below 2^29 keys keep byte offsets in
// 32 bits (larger ones are routed to the fallback by the caller).  Returns the
// key counts; counts beyond CAP3 are reported but not loaded.
template <int NH>
__device__ __forceinline__ void gather_regs(const JobArgs &J, int d, const SubRef (&r)[2], bool pre,
                                            const uint32_t (&pst)[2], const uint32_t (&pen)[2],
                                            uint64_t (&kk)[2][KP3], uint32_t (&n)[2], uint32_t (*s_src)[MAXT],
                                            uint32_t *s_mapw, uint64_t *s_tmp) {
    constexpr int MW = CAP3 / 4;     // map words per half
    constexpr int TW = MW / NT3;     // map words each thread owns per half
    static_assert(TW * NT3 * 4 == CAP3, "every thread owns whole map words");
    const int tid = threadIdx.x;
    uint8_t *s_map = (uint8_t *)s_mapw;
    uint32_t nt[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < NH; ++h) nt[h] = r[h].t1 - r[h].t0;
    const uint32_t ntmax = max(nt[0], NH > 1 ? nt[1] : 0u);
    uint32_t base[2] = {0, 0};
    for (uint32_t c0 = 0; c0 < ntmax; c0 += MAXT) {
        uint32_t len[2] = {0, 0}, st[2] = {0, 0};
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const HalfArgs &H = J.h[h];
            const uint32_t t = c0 + tid;
            if (t < nt[h]) {
                if (pre) {
                    st[h] = pst[h];
                    len[h] = pen[h] - pst[h];
                } else {
                    st[h] = H.digstart[(size_t)d * H.ntile2_max + r[h].t0 + t];
                    len[h] = H.digstart[(size_t)(d + 1) * H.ntile2_max + r[h].t0 + t] - st[h];
                }
            }
        }
        // cleared 16 bytes at a time (the map is 16-byte aligned in LDS)
        for (int i = tid; i < NH * MW / 4; i += NT3) reinterpret_cast<uint4 *>(s_mapw)[i] = make_uint4(0, 0, 0, 0);
        uint64_t tot;
        const uint64_t pre_off = block_excl_scan<NT3>((uint64_t)len[0] | ((uint64_t)len[1] << 32), s_tmp, &tot);
        const uint32_t cl[2] = {(uint32_t)tot, (uint32_t)(tot >> 32)};
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const uint32_t pos = base[h] + (h ? (uint32_t)(pre_off >> 32) : (uint32_t)pre_off);
            if (len[h] > 0) {
                if (pos < CAP3) s_map[h * CAP3 + pos] = (uint8_t)tid;
                s_src[h][tid] = ((c0 + tid) << J.h[h].t2log) + st[h] - pos;
            }
        }
        __syncthreads();
        // prefix maximum over the map
        uint32_t w[2][TW];
        uint64_t mx = 0;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            uint32_t m = 0;
#pragma unroll
            for (int j = 0; j < TW; ++j) {
                w[h][j] = s_mapw[h * MW + tid * TW + j];
#pragma unroll
                for (int k = 0; k < 4; ++k) m = max(m, (w[h][j] >> (8 * k)) & 0xFFu);
            }
            mx |= (uint64_t)m << (32 * h);
        }
        const uint64_t px = block_excl_max2<NT3>(mx, s_tmp);
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            uint32_t m = (uint32_t)(px >> (32 * h));
#pragma unroll
            for (int j = 0; j < TW; ++j) {
                uint32_t o = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    m = max(m, (w[h][j] >> (8 * k)) & 0xFFu);
                    o |= m << (8 * k);
                }
                s_mapw[h * MW + tid * TW + j] = o;
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const char *bk = (const char *)(J.h[h].keys + r[h].pos0);
#pragma unroll
            for (int k = 0; k < KP3; ++k) {
                const uint32_t q = tid + k * NT3;
                if (q >= base[h] && q < base[h] + cl[h] && q < CAP3) {
                    const uint32_t boff = (s_src[h][s_map[h * CAP3 + q]] + q) * 8u;
                    kk[h][k] = __builtin_nontemporal_load((const uint64_t *)(bk + boff));
                }
            }
            base[h] += cl[h];
        }
        __syncthreads();
    }
    n[0] = base[0];
    n[1] = base[1];
}

// Counting sort of the keys in kk[0..n) (register slots) into s_out by the
// LB3-bit digit at shift sh3; s_bin[0..NB3] receives the bin starts (and n).
// With `full`, each bin is then insertion-sorted, so s_out is fully sorted.
__device__ __forceinline__ void sort_slots(const uint64_t (&kk)[KP3], uint32_t n, int sh3, uint64_t *s_out,
                                           uint32_t *s_bin, uint64_t *s_tmp, bool full) {
    uint32_t rk[KP3];
#pragma unroll
    for (int k = 0; k < KP3; ++k) {
        const uint32_t q = threadIdx.x + k * NT3;
        if (q < n) rk[k] = atomicAdd(&s_bin[dig(kk[k], sh3, NB3 - 1)], 1u);
    }
    __syncthreads();
    lds_excl_scan<NT3, NB3 / NT3>(s_bin, NB3, s_tmp);
    if (threadIdx.x == 0) s_bin[NB3] = n;
#pragma unroll
    for (int k = 0; k < KP3; ++k) {
        const uint32_t q = threadIdx.x + k * NT3;
        if (q < n) s_out[s_bin[dig(kk[k], sh3, NB3 - 1)] + rk[k]] = kk[k];
    }
    __syncthreads();
    if (!full) return;
    for (int bn = threadIdx.x; bn < NB3; bn += NT3) {
        const uint32_t s = s_bin[bn], e = s_bin[bn + 1];
        for (uint32_t i = s + 1; i < e; ++i) {
            const uint64_t v = s_out[i];
            uint32_t j = i;
            while (j > s && s_out[j - 1] > v) {
                s_out[j] = s_out[j - 1];
                --j;
            }
            s_out[j] = v;
        }
    }
    __syncthreads();
}

// Over-capacity fallback: every a of A's sub-bucket s against every key of the
// distinct sub-buckets s-1, s, s+1 of B', straight from global memory.
__device__ void join_fallback(const JobArgs &J, uint32_t s, uint32_t NS, int b, int d) {
    if (threadIdx.x == 0) atomicOr(J.flags, 2u);
    uint32_t nbrs[3] = {(s + NS - 1) & (NS - 1), s, (s + 1) & (NS - 1)};
    int nn = 3;
    if (nbrs[0] == nbrs[2]) nn = (nbrs[0] == s) ? 1 : 2;
    if (nn == 1) nbrs[0] = s;
    if (nn == 2) nbrs[1] = s;
    const HalfArgs &HA = J.h[0];
    const SubRef ra = sub_ref(HA, b);
    for (uint32_t t = ra.t0; t < ra.t1; ++t) {
        const uint32_t st = HA.digstart[(size_t)d * HA.ntile2_max + t];
        const uint32_t en = HA.digstart[(size_t)(d + 1) * HA.ntile2_max + t];
        const uint64_t tb = ra.pos0 + ((uint64_t)(t - ra.t0) << HA.t2log);
        for (uint32_t q = st + threadIdx.x; q < en; q += NT3) {
            const uint64_t a = HA.keys[tb + q];
            for (int k = 0; k < nn; ++k) {
                const uint32_t ns = nbrs[k];
                for_each_global(J.h[1], J.B2, (int)(ns >> J.B2), (int)(ns & ((1u << J.B2) - 1)), [&](uint64_t bk) {
                    if (in_win(a, bk, J.t_lo, J.t_hi)) emit_pair(J, a, bk);
                    return *J.kp_count <= J.kcap;
                });
            }
            if (*J.kp_count > J.kcap) return;
        }
    }
}

// Exact band probe of B' bins (fallback when the semi-join's lists overflow):
// s_b holds the sub-bucket's B' keys counting-sorted by the LB3-bit digit.
__device__ __forceinline__ void probe_bins(const JobArgs &J, uint64_t a, uint64_t clo, uint64_t chi, uint64_t wlo,
                                           uint64_t whi, int sh3, const uint64_t *s_b, const uint32_t *s_bin) {
    const uint32_t b0 = dig(clo, sh3, NB3 - 1), b1 = dig(chi, sh3, NB3 - 1);
    const uint32_t e = s_bin[b1 + 1];
    for (uint32_t i = s_bin[b0]; i < e; ++i) {
        const uint64_t bk = s_b[i];
        if (bk >= wlo && bk <= whi) emit_pair(J, a, bk);
    }
}

// Append `cnt` items of this thread to an LDS list whose length is *counter:
// returns the index of the thread's first item.  One LDS atomic per
// wavefront; every lane of the wavefront must call it.
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, uint32_t cnt) {
    const int lane = threadIdx.x & 63;
    uint32_t inc = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    const uint32_t total = __shfl(inc, 63, 64);
    uint32_t base = 0;
    if (lane == 63 && total) base = atomicAdd(counter, total);
    return __shfl(base, 63, 64) + inc - cnt;
}

// Cell bitmaps of the semi-join.  A cell is at least as wide as the window,
// so the window [a - t_hi, a + t_lo] of a key in cell c meets cell c and, only
// when a lies within t_hi of the cell's low edge (t_lo of its high edge), cell
// c - 1 (c + 1) -- a case of probability about window / cell width.
__device__ __forceinline__ void mark1(uint32_t *bm, uint32_t c) { atomicOr(&bm[c >> 5], 1u << (c & 31)); }

__device__ __forceinline__ bool bit(const uint32_t *bm, uint32_t c) { return (bm[c >> 5] >> (c & 31)) & 1u; }

// Edge flags of key a in its cell (cell width 2^shc).
__device__ __forceinline__ void cell_edges(uint64_t a, int shc, uint64_t t_lo, uint64_t t_hi, bool &lo, bool &hi) {
    const uint64_t off = a & ((1ull << shc) - 1);
    lo = off < t_hi;
    hi = ((1ull << shc) - 1 - off) < t_lo;
}

// Does a's window meet a marked cell?  Marks those cells in `mk` if given.
template <uint32_t NC>
__device__ __forceinline__ bool window_hits(const uint32_t *bm, uint32_t c, bool lo, bool hi) {
    return bit(bm, c) || (lo && c > 0 && bit(bm, c - 1)) || (hi && c < NC - 1 && bit(bm, c + 1));
}

template <uint32_t NC>
__device__ __forceinline__ void mark_window(uint32_t *bm, uint32_t c, bool lo, bool hi) {
    mark1(bm, c);
    if (lo && c > 0) mark1(bm, c - 1);
    if (hi && c < NC - 1) mark1(bm, c + 1);
}

// LDS of a sorting (expansion) K3 workgroup: the sub-bucket's keys and bins.
struct alignas(16) SortLds {
    uint64_t b[CAP3];
    uint32_t bin[NB3 + 1];
    uint32_t src[2][MAXT];
    alignas(16) uint32_t mapw[2 * CAP3 / 4];
    uint64_t tmp[NT3 / 64 + 2];
    uint32_t nl[2];
};

// LDS of one joining K3 workgroup, sized so that six workgroups fit a CU.
// `u` holds either the semi-join's bitmap and two lists or, on the exact
// fallback, a chunk of B' keys.
struct alignas(16) JoinLds {
    static constexpr uint32_t NWD = (1u << CB3) / 32;  // bitmap words
    union {
        struct {
            uint32_t bm[2 * NWD];  // cells of B', then cells LA's windows meet
            uint64_t la[LCAP3];
            uint64_t lb[LCAP3];
        } sj;
        uint64_t keys[FB3];
    } u;
    uint32_t src[2][MAXT];
    alignas(16) uint32_t mapw[2 * CAP3 / 4];
    uint64_t tmp[NT3 / 64 + 2];
    uint32_t nl[2];
};

// Exact join of one sub-bucket without the semi-join (window wider than a
// cell, or clustered keys overflowing a list): B' is staged through LDS in
// chunks of FB3 keys and every a tests every staged b'.  Quadratic, only for
// such inputs.
__device__ __forceinline__ void join_exact(const JobArgs &J, const uint64_t (&kk)[2][KP3], uint32_t na, uint32_t nb,
                                        uint64_t *s_keys) {
    const int tid = threadIdx.x;
    const uint64_t t_lo = J.t_lo, t_hi = J.t_hi;
    for (uint32_t c0 = 0; c0 < nb; c0 += FB3) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KP3; ++k) {
            const uint32_t q = tid + k * NT3;
            if (q >= c0 && q < nb && q < c0 + FB3) s_keys[q - c0] = kk[1][k];
        }
        __syncthreads();
        const uint32_t cn = min((uint32_t)FB3, nb - c0);
#pragma unroll
        for (int k = 0; k < KP3; ++k) {
            if (tid + k * NT3 >= na) continue;
            const uint64_t a = kk[0][k];
            const uint64_t wlo = a >= t_hi ? a - t_hi : 0;
            const uint64_t whi = a <= ~0ull - t_lo ? a + t_lo : ~0ull;
            for (uint32_t i = 0; i < cn; ++i) {
                const uint64_t bk = s_keys[i];
                if (bk >= wlo && bk <= whi) emit_pair(J, a, bk);
            }
        }
    }
}

// Semi-join of one sub-bucket s = (b, d) whose keys are in register slots
// (see k_join, steps 2-4).
__device__ __forceinline__ void join_semi(const JobArgs &J, uint32_t s, int b, int d, const uint64_t (&kk)[2][KP3],
                                          uint32_t na, uint32_t nb, JoinLds &L) {
    constexpr uint32_t NC = 1u << CB3;  // cells
    constexpr uint32_t NWD = JoinLds::NWD;
    const int LB = J.B1 + J.B2;
    const uint32_t NS = 1u << LB;
    const int shc = 64 - LB - CB3;
    const int tid = threadIdx.x;
    uint32_t *bm = L.u.sj.bm;         // cells of B' keys
    uint32_t *bmA = L.u.sj.bm + NWD;  // cells LA's windows meet
    uint64_t *LA = L.u.sj.la;
    uint64_t *LBl = L.u.sj.lb;
    if (na > CAP3 || nb > CAP3) {
        join_fallback(J, s, NS, b, d);
        return;
    }
    __syncthreads();  // bitmap zeroing visible even when the gather had no chunk

    const uint64_t s_lo = LB == 0 ? 0 : ((uint64_t)s << (64 - LB));
    const uint64_t s_hi = LB == 0 ? ~0ull : (s_lo + ((1ull << (64 - LB)) - 1));
    const uint64_t t_lo = J.t_lo, t_hi = J.t_hi;
    const uint64_t cellw = 1ull << shc;
    const bool fast = t_lo <= cellw && t_hi <= cellw && LB <= 32;
    // 32-bit views of the keys: loc = key bits [63 - LB, 32 - LB] (the bits
    // below the sub-bucket's), so the cell is loc >> csh and loc & omask is the
    // key's offset in its cell without its low sh bits.  Near-edge flags taken
    // from that truncated offset are a superset of the exact ones: they only
    // send a few more keys to the neighbour-cell test, and every pair is
    // compared exactly in the end.
    const int sh = 32 - LB, csh = 32 - CB3;
    const uint32_t omask = (1u << csh) - 1;
    auto loc = [sh](uint64_t key) { return (uint32_t)(key >> sh); };
    bool lists = false;
    if (fast) {
        const uint64_t om = cellw - 1;
        const uint32_t lo_thr = (uint32_t)min(t_hi >> sh, (uint64_t)omask);        // near the low edge: off <= lo_thr
        const uint32_t hi_thr = t_lo > om ? 0u : (uint32_t)((om - t_lo) >> sh);  // near the high edge: off >= hi_thr
        // B' marks its cells
#pragma unroll
        for (int k = 0; k < KP3; ++k)
            if (tid + k * NT3 < nb) mark1(bm, loc(kk[1][k]) >> csh);
        __syncthreads();
        // A keys whose window meets a marked cell.  Every slot's own-cell word
        // is read first with no branch (the reads overlap; an unused slot reads
        // a stale but in-range cell), the bit tests follow; the rare keys near
        // their cell's edge take a second pass for the neighbour.
        uint32_t hits = 0, elo = 0, ehi = 0;
        {
            uint32_t cl[KP3], wd[KP3];
#pragma unroll
            for (int k = 0; k < KP3; ++k) cl[k] = loc(kk[0][k]) >> csh;
#pragma unroll
            for (int k = 0; k < KP3; ++k) wd[k] = bm[cl[k] >> 5];
#pragma unroll
            for (int k = 0; k < KP3; ++k) {
                const bool live = tid + k * NT3 < na;
                const uint32_t off = loc(kk[0][k]) & omask;
                hits |= (uint32_t)(live && ((wd[k] >> (cl[k] & 31)) & 1u)) << k;
                elo |= (uint32_t)(live && off <= lo_thr) << k;
                ehi |= (uint32_t)(live && off >= hi_thr) << k;
            }
        }
        if ((elo | ehi) & ~hits) {
#pragma unroll
            for (int k = 0; k < KP3; ++k) {  // static slot indices keep kk in registers
                if (!(((elo | ehi) & ~hits) >> k & 1u)) continue;
                if (window_hits<NC>(bm, loc(kk[0][k]) >> csh, (elo >> k) & 1u, (ehi >> k) & 1u))
                    hits |= 1u << k;
            }
        }
        // append the hits to LA and mark the cells their windows meet
        uint32_t o = wave_append(&L.nl[0], __popc(hits));
#pragma unroll
        for (int k = 0; k < KP3; ++k)
            if ((hits >> k) & 1u) {
                if (o < LCAP3) LA[o] = kk[0][k];
                ++o;
                mark_window<NC>(bmA, loc(kk[0][k]) >> csh, (elo >> k) & 1u, (ehi >> k) & 1u);
            }
        __syncthreads();
        const uint32_t nla = L.nl[0];
        if (nla <= LCAP3) {
            // B' keys in those cells
            uint32_t bh = 0, cl[KP3], wd[KP3];
#pragma unroll
            for (int k = 0; k < KP3; ++k) cl[k] = loc(kk[1][k]) >> csh;
#pragma unroll
            for (int k = 0; k < KP3; ++k) wd[k] = bmA[cl[k] >> 5];
#pragma unroll
            for (int k = 0; k < KP3; ++k)
                bh |= (uint32_t)(tid + k * NT3 < nb && ((wd[k] >> (cl[k] & 31)) & 1u)) << k;
            uint32_t ob = wave_append(&L.nl[1], __popc(bh));
#pragma unroll
            for (int k = 0; k < KP3; ++k)
                if ((bh >> k) & 1u) {
                    if (ob < LCAP3) LBl[ob] = kk[1][k];
                    ++ob;
                }
            __syncthreads();
        }
        const uint32_t nlb = L.nl[1];
        lists = nla <= LCAP3 && nlb <= LCAP3;
        if (lists) {
            // every pair of the lists: each wavefront takes LA entries, its
            // lanes hold LB entries
            const int lane = tid & 63, wv = tid >> 6;
            for (uint32_t j0 = 0; j0 < nlb; j0 += 64) {
                const uint32_t j = j0 + lane;
                const bool valid = j < nlb;
                const uint64_t bk = valid ? LBl[j] : 0;
#pragma unroll 4
                for (uint32_t i = wv; i < nla; i += NT3 / 64) {
                    const uint64_t a = LA[i];
                    const uint64_t wlo = a >= t_hi ? a - t_hi : 0;
                    const uint64_t whi = a <= ~0ull - t_lo ? a + t_lo : ~0ull;
                    if (valid && bk >= wlo && bk <= whi) emit_pair(J, a, bk);
                }
            }
        }
    }
    if (!lists) join_exact(J, kk, na, nb, L.u.keys);
    // windows reaching past this sub-bucket (or wrapping past 0); with
    // windows no wider than a cell only keys in the first or last cell can
#pragma unroll
    for (int k = 0; k < KP3; ++k) {
        if (tid + k * NT3 >= na) continue;
        const uint64_t a = kk[0][k];
        if (fast) {
            const uint32_t c = loc(a) >> csh;
            if (c != 0 && c != NC - 1) continue;
        }
        const bool low_edge = (a - s_lo) < t_hi;
        const bool high_edge = (s_hi - a) < t_lo;
        if (low_edge || high_edge) {
            const uint64_t wlo = a >= t_hi ? a - t_hi : 0;
            const uint64_t whi = a <= ~0ull - t_lo ? a + t_lo : ~0ull;
            const uint32_t nlo = (s + NS - 1) & (NS - 1), nhi = (s + 1) & (NS - 1);
            if (low_edge) edge_scan(J, a, s, nlo, wlo, whi);
            if (high_edge && !(low_edge && nhi == nlo)) edge_scan(J, a, s, nhi, wlo, whi);
        }
    }
}

// Join of one sub-bucket s = (b, d) (see k_join).
template <bool SORT_OUT, typename Lds>
__device__ __forceinline__ void join_sub(const JobArgs &J, uint32_t s, int b, int d, const SubRef (&r)[2], bool pre,
                                         const uint32_t (&pst)[2], const uint32_t (&pen)[2], uint64_t *sorted_out,
                                         Lds &L) {
    constexpr int NH = SORT_OUT ? 1 : 2;
    const int tid = threadIdx.x;

    if constexpr (SORT_OUT) {
        for (int i = tid; i < NB3; i += NT3) L.bin[i] = 0;
    } else {
        for (uint32_t i = tid; i < 2 * JoinLds::NWD / 4; i += NT3)
            reinterpret_cast<uint4 *>(L.u.sj.bm)[i] = make_uint4(0, 0, 0, 0);
        if (tid < 2) L.nl[tid] = 0;
    }
    uint32_t n[2];
    if constexpr (SORT_OUT) {
        uint64_t kk[2][KP3];
        gather_regs<NH>(J, d, r, pre, pst, pen, kk, n, L.src, L.mapw, L.tmp);
        const uint32_t na = n[0];
        if (na > CAP3) {
            if (tid == 0) atomicOr(J.flags, 1u);
            return;
        }
        sort_slots(kk[0], na, 64 - (J.B1 + J.B2) - LB3, L.b, L.bin, L.tmp, true);
        // output position: bucket start + keys of lower digits in every tile
        uint64_t part = 0;
        for (uint32_t t = r[0].t0 + tid; t < r[0].t1; t += NT3)
            part += J.h[0].digstart[(size_t)d * J.h[0].ntile2_max + t];
        uint64_t tot;
        block_excl_scan<NT3>(part, L.tmp, &tot);
        const uint64_t pos = r[0].pos0 + tot;
        for (uint32_t i = tid; i < na; i += NT3) sorted_out[pos + i] = L.b[i];
    } else {
        uint64_t kk[2][KP3];
        gather_regs<NH>(J, d, r, pre, pst, pen, kk, n, L.src, L.mapw, L.tmp);
        join_semi(J, s, b, d, kk, n[0], n[1], L);
    }
}

// K3: one sub-bucket s = (level-1 bucket b, level-2 digit d) per workgroup;
// consecutive sub-buckets go to the same XCD so the tile-segment cache lines
// they share meet in one L2.  Workgroups of NT3 threads with KP3 slots each
// and a small LDS footprint, so that several of them share a CU: the join is bound
// by the latency of its dependent loads (bucket extent, then segment bounds,
// then keys), which only more workgroups in flight hide.
//  1. gather both halves into register slots (gather_regs);
//  2. semi-join through an LDS bitmap over the sub-bucket's range cut into
//     2^CB3 cells, each at least as wide as the window, so a pair's keys lie
//     in the same or adjacent cells: every b' marks its cell and both
//     neighbours; every a whose own cell is marked joins list LA; the bitmap
//     is then rebuilt from LA's cells (dilated the same way) and every b'
//     whose cell is marked joins list LB.  Random keys leave a few hundred
//     entries in LA and a few dozen in LB, whose pairs are tested exactly;
//  3. if a list overflows (clustered keys) or the window is wider than a
//     cell, every a is tested against every b' instead (join_exact);
//  4. a window reaching past the sub-bucket (or wrapping past 0) also scans
//     the neighbour sub-bucket of B' from global memory (edge_scan).
// With SORT_OUT the single half is fully sorted in LDS and written instead.
template <bool SORT_OUT, bool MULTI>
__global__ __launch_bounds__(NT3) __attribute__((amdgpu_waves_per_eu(5))) void k_join(JobArgs Jarg, Multi M,
                                                                                        uint64_t *sorted_out) {
    constexpr int NH = SORT_OUT ? 1 : 2;
    const JobArgs *Jp;
    uint32_t s;
    if (!pick<MULTI>(Jarg, M, ST_JOIN, Jp, s)) return;
    if (!MULTI) s += blockIdx.y * gridDim.x;  // grids of more than 2^22 sub-buckets
    const JobArgs &J = *Jp;
    const int LB = J.B1 + J.B2;
    const uint32_t NS = 1u << LB;
    if (s >= NS) return;
    if (NS >= 64) s = (s & 7) * (NS >> 3) + (s >> 3);
    const int b = (int)(s >> J.B2), d = (int)(s & ((1u << J.B2) - 1));
    const int tid = threadIdx.x;
    __shared__ std::conditional_t<SORT_OUT, SortLds, JoinLds> L;

    SubRef r[2];
    uint32_t nt[2] = {0, 0};
    bool huge = false;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        r[h] = sub_ref(J.h[h], b);
        nt[h] = r[h].t1 - r[h].t0;
        huge = huge || (J.h[h].bstart[b + 1] - r[h].pos0) >= (1ull << 29);
    }
    if (huge) {
        // 32-bit slot offsets cannot address this bucket
        if (SORT_OUT) {
            if (tid == 0) atomicOr(J.flags, 1u);
        } else {
            join_fallback(J, s, NS, b, d);
        }
        return;
    }
    // tile `tid`'s segment bounds of each half, loaded up front when the
    // bucket's tiles fit one gather chunk
    const bool pre = max(nt[0], NH > 1 ? nt[1] : 0u) <= (uint32_t)MAXT;
    uint32_t pst[2] = {0, 0}, pen[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        const HalfArgs &H = J.h[h];
        if (pre && (uint32_t)tid < nt[h]) {
            pst[h] = H.digstart[(size_t)d * H.ntile2_max + r[h].t0 + tid];
            pen[h] = H.digstart[(size_t)(d + 1) * H.ntile2_max + r[h].t0 + tid];
        }
    }
    join_sub<SORT_OUT>(J, s, b, d, r, pre, pst, pen, sorted_out, L);
}

// ------------------------------------------------------------------ K4
// Pattern recovery when few candidate keys exist (the usual case): a key of
// this half is slo[l] + shi(g) with l the low L pattern bits and g = gray(h)
// the high ones.  The 2^L low sums are sorted once in LDS; then every Gray step
// h needs, per candidate key K, one binary search for K - shi(g) among them
// (a meet in the middle inside the half) instead of 2^L enumerated keys.
template <bool MULTI>
__global__ __launch_bounds__(NT1) void k_recover_few(JobArgs Jarg, Multi M) {
    const JobArgs *Jp;
    uint32_t bx;
    if (!pick<MULTI>(Jarg, M, ST_RFEW, Jp, bx)) return;
    const JobArgs &J = *Jp;
    const int half = blockIdx.y;
    const HalfArgs &H = J.h[half];
    const uint64_t cnt = *J.kp_count;
    if (cnt > RECOVER_FEW || cnt == 0) return;
    const int tid = threadIdx.x;
    const int nl = 1 << H.L;
    const uint64_t h0 = ((uint64_t)bx * NT1 + tid) * SPT4;
    if ((uint64_t)bx * NT1 * SPT4 >= H.steps) return;

    __shared__ uint64_t s_w[64];
    __shared__ uint64_t s_v[256], s_sorted[256];
    __shared__ uint32_t s_lane[256];
    __shared__ uint64_t s_list[RECOVER_FEW];
    __shared__ uint8_t s_dup[RECOVER_FEW];
    if (tid < H.m) s_w[tid] = J.wts[half][tid];
    for (uint32_t i = tid; i < cnt; i += NT1) s_list[i] = J.kp[2 * i + half];
    __syncthreads();
    // the same key listed twice (it pairs with several keys of the other
    // half) is recorded once: flag the repeats once, not at every step
    for (uint32_t i = tid; i < cnt; i += NT1) {
        bool dup = false;
        for (uint32_t c2 = 0; c2 < i && !dup; ++c2) dup = s_list[c2] == s_list[i];
        s_dup[i] = dup;
    }
    if (tid < nl) {
        uint64_t v = J.kbase[half];
        for (int i = 0; i < H.L; ++i)
            if ((tid >> i) & 1) v += s_w[i];
        s_v[tid] = v;
    }
    __syncthreads();
    if (tid < nl) {
        const uint64_t v = s_v[tid];
        int rk = 0;
        for (int l = 0; l < nl; ++l) {
            const uint64_t u = s_v[l];
            rk += (u < v) || (u == v && l < tid);
        }
        s_sorted[rk] = v;
        s_lane[rk] = (uint32_t)tid;
    }
    __syncthreads();
    if (h0 >= H.steps) return;
    const uint64_t h1 = min(h0 + (uint64_t)SPT4, H.steps);
    uint64_t g = h0 ^ (h0 >> 1);
    uint64_t shi = 0;
    for (int i = 0; i < H.m - H.L; ++i)
        if ((g >> i) & 1) shi += s_w[H.L + i];
    for (uint64_t h = h0; h < h1; ++h) {
        // the lower bounds of four candidates at a time, interleaved: four
        // independent chains of LDS reads in flight instead of one
        for (uint32_t c0 = 0; c0 < cnt; c0 += 4) {
            uint64_t x[4];
            int lo[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                x[j] = s_list[min(c0 + j, (uint32_t)cnt - 1)] - shi;  // past the list: a repeat, ignored
                lo[j] = 0;
            }
            if (nl == 256) {
#pragma unroll
                for (int step = 128; step > 0; step >>= 1)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (s_sorted[lo[j] + step - 1] < x[j]) lo[j] += step;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int l = 0, r = nl;
                    while (l < r) {
                        const int mid = (l + r) >> 1;
                        if (s_sorted[mid] < x[j]) l = mid + 1;
                        else r = mid;
                    }
                    lo[j] = l;
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t c = c0 + j;
                if (c >= cnt || s_dup[c]) continue;
                const uint64_t key = s_list[c];
                for (int q = lo[j]; q < nl && s_sorted[q] == x[j]; ++q) {
                    const uint64_t pat = ((uint64_t)s_lane[q] | (g << H.L)) | J.pbase[half];
                    const uint64_t r = atomicAdd((unsigned long long *)&J.rec_count[half], 1ull);
                    if (r < J.kcap) {
                        J.rec[((size_t)half * J.kcap + r) * 2] = key;
                        J.rec[((size_t)half * J.kcap + r) * 2 + 1] = pat;
                    }
                }
            }
        }
        const uint64_t t = h + 1;
        if (t < h1) {
            const int bb = __builtin_ctzll(t);
            g ^= 1ull << bb;
            const uint64_t wb = s_w[H.L + bb];
            shi += ((g >> bb) & 1) ? wb : (0 - wb);
        }
    }
}

// Pattern recovery for many candidate keys: re-enumerate the half (same Gray
// walk as K1, no stores) and look every key up in two LDS bitmaps of
// candidate key bit fields (2^(RBITS_LOG - 1) bits each), confirming a key
// that passes both by a binary search in the sorted candidate list.
template <bool MULTI>
__global__ __launch_bounds__(NT1) void k_recover(JobArgs Jarg, Multi M) {
    const JobArgs *Jp;
    uint32_t wg;
    if (!pick<MULTI>(Jarg, M, ST_RMANY, Jp, wg)) return;
    const JobArgs &J = *Jp;
    const int half = blockIdx.y;
    const HalfArgs &H = J.h[half];
    if (wg >= H.nwg1) return;
    const uint64_t cnt = *J.kp_count;
    if (cnt > J.kcap || cnt <= RECOVER_FEW) return;
    const int tid = threadIdx.x;
    const int nl = 1 << H.L;
    const bool act = tid < nl;

    __shared__ uint64_t s_w[64];
    // two prefix bitmaps of RBITS / 2 bits each, on independent key bits
    // (the top RB bits, the next RB bits): a key that is not a candidate
    // passes both with probability (cnt / 2^RB)^2, so the binary search
    // below runs for about one key in 37,000 at 683 candidates instead of one
    // in 380 with a single bitmap of RBITS bits (n = 65: 16.1 -> 8.3 ms)
    constexpr int RB = RBITS_LOG - 1;
    constexpr uint32_t RBW = (1u << RB) / 32;  // words per bitmap
    __shared__ uint32_t s_bits[RBITS / 32];
    __shared__ uint64_t s_list[KCAP_MAX];
    if (tid < H.m) s_w[tid] = J.wts[blockIdx.y][tid];
    for (int i = tid; i < RBITS / 32; i += NT1) s_bits[i] = 0;
    __syncthreads();
    // the candidate keys, padded with ~0 to a power of two and sorted (bitonic)
    // so that a key passing the prefix bitmap takes a binary search
    uint32_t np = 1;
    while (np < cnt) np <<= 1;
    for (uint32_t i = tid; i < np; i += NT1) {
        const uint64_t k = i < cnt ? J.kp[2 * i + half] : ~0ull;
        s_list[i] = k;
        if (i < cnt) {
            const uint32_t ha = (uint32_t)(k >> (64 - RB));
            const uint32_t hb = (uint32_t)(k >> (64 - 2 * RB)) & ((1u << RB) - 1);
            atomicOr(&s_bits[ha >> 5], 1u << (ha & 31));
            atomicOr(&s_bits[RBW + (hb >> 5)], 1u << (hb & 31));
        }
    }
    __syncthreads();
    for (uint32_t k = 2; k <= np; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = tid; i < np; i += NT1) {
                const uint32_t ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t a = s_list[i], b = s_list[ixj];
                    if ((a > b) == ((i & k) == 0)) {
                        s_list[i] = b;
                        s_list[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }

    uint64_t slo = J.kbase[half];
    for (int i = 0; i < H.L; ++i)
        if ((tid >> i) & 1) slo += s_w[i];
    constexpr int KPT = 16;
    constexpr int LOGK = 4;
    static_assert((1 << LOGK) == KPT && (KPT1 * TILES1) % KPT == 0, "ranges of whole tiles");
    const int mh = H.m - H.L;
    uint64_t wlow[LOGK];
#pragma unroll
    for (int i = 0; i < LOGK; ++i) wlow[i] = mh > i ? s_w[H.L + i] : 0;
    // A single search's grid is capped (RECOVER_WGS per half): the table
    // above is built once per workgroup, which then walks every gridDim.x-th
    // range of spw Gray steps.  A multi-job launch has one range per block.
    for (uint32_t w = wg; w < H.nwg1; w += MULTI ? H.nwg1 : gridDim.x) {
        const uint64_t h0 = (uint64_t)w * H.spw;
        const uint64_t h1 = min(h0 + (uint64_t)H.spw, H.steps);
        uint64_t g = h0 ^ (h0 >> 1);
        uint64_t shi = 0;
        for (int i = 0; i < H.m - H.L; ++i)
            if ((g >> i) & 1) shi += s_w[H.L + i];
        // tiles of KPT steps (the ranges start at multiples of spw, a multiple
        // of KPT): inside a tile step k + 1 flips bit ctz(k + 1) < log2 KPT,
        // whose weight sits in a register, so only the step into the next
        // tile reads its weight from LDS.  The tile only tests the prefix
        // bitmap; the rare keys that pass are rebuilt from their step's Gray
        // code and looked up afterwards.
        for (uint64_t h = h0; h < h1; h += KPT) {
            const int ns = (int)min((uint64_t)KPT, h1 - h);
            const uint64_t g0 = g, shi0 = shi;  // Gray code and high sum at the tile's first step
            uint32_t hitm = 0;
#pragma unroll
            for (int k = 0; k < KPT; ++k) {
                const uint64_t key = slo + shi;
                const uint32_t ha = (uint32_t)(key >> (64 - RB));
                hitm |= (uint32_t)(act && k < ns && ((s_bits[ha >> 5] >> (ha & 31)) & 1)) << k;
                const uint64_t t = h + k + 1;
                if (k < ns && t < h1) {
                    const int bb = k < KPT - 1 ? __builtin_ctz(k + 1) : __builtin_ctzll(t);
                    const uint64_t wb = k < KPT - 1 ? wlow[__builtin_ctz(k + 1) % LOGK] : s_w[H.L + bb];
                    g ^= 1ull << bb;
                    shi += ((g >> bb) & 1) ? wb : (0 - wb);
                }
            }
            while (hitm) {
                const int k = __builtin_ctz(hitm);
                hitm &= hitm - 1;
                // h is a multiple of KPT, so gray(h + k) = gray(h) ^ gray(k):
                // the key differs from the tile's first one only in the low
                // LOGK Gray bits, whose weights are in registers
                const uint32_t gd = (uint32_t)(k ^ (k >> 1));
                const uint64_t gk = g0 ^ gd;
                uint64_t key = slo + shi0;
#pragma unroll
                for (int i = 0; i < LOGK; ++i)
                    if ((gd >> i) & 1) key += ((g0 >> i) & 1) ? (0 - wlow[i]) : wlow[i];
                const uint32_t hb = (uint32_t)(key >> (64 - 2 * RB)) & ((1u << RB) - 1);
                if (!((s_bits[RBW + (hb >> 5)] >> (hb & 31)) & 1)) continue;
                uint32_t lo = 0, len = (uint32_t)cnt;  // first of s_list[0, cnt) not below key
                while (len > 0) {
                    const uint32_t half_len = len >> 1;
                    if (s_list[lo + half_len] < key) {
                        lo += half_len + 1;
                        len -= half_len + 1;
                    } else {
                        len = half_len;
                    }
                }
                if (lo < cnt && s_list[lo] == key) {
                    const uint64_t pat = ((uint64_t)tid | (gk << H.L)) | J.pbase[half];
                    const uint64_t r = atomicAdd((unsigned long long *)&J.rec_count[half], 1ull);
                    if (r < J.kcap) {
                        J.rec[((size_t)half * J.kcap + r) * 2] = key;
                        J.rec[((size_t)half * J.kcap + r) * 2 + 1] = pat;
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ K5
// One workgroup: distinct key pairs x (patterns of each key) -> pattern pairs.
template <bool MULTI>
__global__ __launch_bounds__(NT1) void k_pairs(JobArgs Jarg, Multi M) {
    const JobArgs *Jp;
    uint32_t bx;
    if (!pick<MULTI>(Jarg, M, ST_PAIRS, Jp, bx)) return;
    const JobArgs &J = *Jp;
    const uint64_t cnt = *J.kp_count;
    const uint64_t carry = *J.out_count;  // patterns of earlier chunks of half A
    __shared__ uint64_t s_total;
    if (threadIdx.x == 0) s_total = carry;
    __syncthreads();
    // key pairs past the capacity, or (key, pattern) records of either half
    // past it (many patterns sharing a candidate key), would lose pattern
    // pairs: report the overflow instead
    if (cnt > J.kcap || carry == ~0ull || J.rec_count[0] > J.kcap || J.rec_count[1] > J.kcap) {
        if (threadIdx.x == 0) *J.out_count = ~0ull;
        return;
    }
    if (*J.flags & 4u) {  // the query design could not run (its B' sort overflowed)
        if (threadIdx.x == 0) *J.out_count = E_FALLBACK;
        return;
    }
    const uint32_t ra = (uint32_t)min(J.rec_count[0], J.kcap), rb = (uint32_t)min(J.rec_count[1], J.kcap);
    // every distinct key pair (a, b') against the (key, pattern) records of
    // both halves; key(p, i) / rec_a(x) / rec_b(y) read the staged copies in
    // LDS for a single search (its one workgroup holds them all) and global
    // memory for a multi-job launch, whose many blocks keep a small footprint
    auto pairs = [&](auto key, auto rec_a, auto rec_b) {
        for (uint32_t p = threadIdx.x; p < cnt; p += NT1) {
            const uint64_t a = key(p, 0), bk = key(p, 1);
            bool first = true;
            for (uint32_t q = 0; q < p && first; ++q)
                if (key(q, 0) == a && key(q, 1) == bk) first = false;
            if (!first) continue;
            for (uint32_t x = 0; x < ra; ++x) {
                if (rec_a(x) != a) continue;
                const uint64_t pa = J.rec[2 * x + 1];
                for (uint32_t y = 0; y < rb; ++y) {
                    if (rec_b(y) != bk) continue;
                    const uint64_t pb = J.rec[((size_t)J.kcap + y) * 2 + 1];
                    if (pa == 0 && pb == 0) continue;  // the empty pattern s = 0
                    const unsigned long long o = atomicAdd((unsigned long long *)&s_total, 1ull);
                    if (o < J.cap) {
                        J.out[2 * o] = pa;
                        J.out[2 * o + 1] = pb;
                    }
                }
            }
        }
    };
    if constexpr (!MULTI) {
        __shared__ uint64_t s_kp[2 * KCAP_MAX], s_ra[KCAP_MAX], s_rb[KCAP_MAX];
        for (uint32_t i = threadIdx.x; i < 2 * cnt; i += NT1) s_kp[i] = J.kp[i];
        for (uint32_t i = threadIdx.x; i < ra; i += NT1) s_ra[i] = J.rec[2 * i];
        for (uint32_t i = threadIdx.x; i < rb; i += NT1) s_rb[i] = J.rec[((size_t)J.kcap + i) * 2];
        __syncthreads();
        pairs([&](uint32_t p, int h) { return s_kp[2 * p + h]; }, [&](uint32_t x) { return s_ra[x]; },
              [&](uint32_t y) { return s_rb[y]; });
    } else {
        pairs([&](uint32_t p, int h) { return J.kp[2 * p + h]; }, [&](uint32_t x) { return J.rec[2 * x]; },
              [&](uint32_t y) { return J.rec[((size_t)J.kcap + y) * 2]; });
    }
    __syncthreads();
    if (threadIdx.x == 0) *J.out_count = s_total > J.cap ? ~0ull : s_total;
}

}  // namespace dev

// ======================================================================
// host side: plans and enqueue
// ======================================================================
using namespace dev;

static inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

static void plan_half(int m, HalfPlan &h) {
    h.m = m;
    h.L = m < 8 ? m : 8;
    h.N = 1ull << m;
    h.steps = 1ull << (m - h.L);
    // Gray steps per K0/K1/K4 workgroup: one 64-step K1 tile for halves of at
    // most 2^28 keys (finer work units leave a smaller tail on the last round
    // of workgroups: K1 0.272 -> 0.241 ms per degree-100 search, the column
    // scan over the per-workgroup histograms 6 -> 14 us); four tiles above,
    // where the histograms (2^B1 buckets x workgroups) would grow to GBs.
    h.spw = (uint32_t)(m <= 28 ? 64 : KPT1 * TILES1);
    h.nwg1 = (uint32_t)((h.steps + h.spw - 1) / h.spw);
}

// Digit split of the 2^LB sub-buckets (mean 2^SUB_LOG keys of the larger half
// each): up to 16 bits as 8 + 8 (level-1 runs of ~16 keys per K1 tile, level-2
// runs of ~16 keys per K2 tile); beyond that both levels grow, level 1 first.
// Tuning table (size class log2 N -> level-1 bits and sub-bucket size), set
// by the autotuner or loaded from its file; -1 entries use the defaults below.
static Tune g_tune[MAX_HALF + 1] = {};
static bool g_tune_init = false;
static void tune_defaults() {
    if (g_tune_init) return;
    for (auto &t : g_tune) t = Tune{-1, -1, 0.0, 0};
    g_tune_init = true;
}
void set_tune(int lg, Tune t) {
    tune_defaults();
    if (lg >= 0 && lg <= MAX_HALF) g_tune[lg] = t;
}
Tune get_tune(int lg) {
    tune_defaults();
    return (lg >= 0 && lg <= MAX_HALF) ? g_tune[lg] : Tune{-1, -1, 0.0, 0};
}

static void plan_bits(uint64_t nmax, bool batch, bool expand, int &B1, int &B2, int &sub) {
    int lg = 0;
    while ((1ull << lg) < nmax) ++lg;
    const Tune tn = expand ? Tune{-1, -1, 0.0, 0} : get_tune(lg);
    // The join and EXPAND hold a sub-bucket in LDS (at most CAP3 keys per
    // half), so the mean is at most 2^SUB_LOG.  The search table is timed on
    // one search at a time, where smaller sub-buckets (more workgroups) fill
    // the chip; a batch fills it with its many searches, so it takes the
    // largest sub-buckets, as EXPAND does.
    if (expand || batch) sub = SUB_LOG;
    else sub = (tn.sub_log >= SUB_LOG_MIN && tn.sub_log <= SUB_LOG) ? tn.sub_log : SUB_LOG;
    int LB = lg > sub ? lg - sub : 0;
    if (LB > MAXB1_LOG + MAXB2_LOG) LB = MAXB1_LOG + MAXB2_LOG;
    if (tn.b1 >= 0) {
        B1 = std::min(std::min(tn.b1, LB), MAXB1_LOG);
        B2 = LB - B1;
        if (B2 > MAXB2_LOG) {
            B1 += B2 - MAXB2_LOG;
            B2 = MAXB2_LOG;
        }
        return;
    }
    if (LB <= 16) {
        B1 = LB < 8 ? LB : 8;
        B2 = LB - B1;
    } else {
        // level 1 at most 2^11 buckets (runs of 4 keys per K1 tile); the 12th
        // bit only when level 2 is full (halves of 2^34 keys)
        B1 = std::min(11, (LB + 1) / 2);
        B2 = LB - B1;
    }
    if (B2 > MAXB2_LOG) {
        B1 += B2 - MAXB2_LOG;
        B2 = MAXB2_LOG;
    }
}

// Carve the workspace; returns bytes needed.  With base == nullptr only sizes.
static uint64_t layout(JobPlan &P, char *base) {
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t o = off;
        off = align_up(off + bytes, 256);
        return base ? (void *)(base + o) : nullptr;
    };
    const int nb = 1 << P.B1, nd = 1 << P.B2;
    for (int k = 0; k < P.nhalves; ++k) {
        HalfPlan &h = P.h[k];
        h.ntile2_max = (uint32_t)((h.N >> P.t2log) + nb + 1);
        h.a.keys = (uint64_t *)take(h.N * 8);
        h.a.hist1 = (uint64_t *)take((uint64_t)nb * h.nwg1 * 8);
        h.a.bstart = (uint64_t *)take((uint64_t)(nb + 1) * 8);
        h.a.tstart = (uint32_t *)take((uint64_t)(nb + 1) * 4);
        h.a.digstart = (uint16_t *)take((uint64_t)(nd + 1) * h.ntile2_max * 2);
        h.a.N = h.N;
        h.a.steps = h.steps;
        h.a.spw = h.spw;
        h.a.nwg1 = h.nwg1;
        h.a.ntile2_max = h.ntile2_max;
        h.a.m = h.m;
        h.a.L = h.L;
        h.a.t2log = P.t2log;
    }
    P.kp = (uint64_t *)take(P.kcap * 16);
    P.rec = (uint64_t *)take(2ull * P.kcap * 16);
    P.counters = (uint64_t *)take(64);
    return off;
}

uint64_t plan_job(int na, int nb, JobPlan &P, uint64_t kcap, bool batch) {
    P = JobPlan();
    P.kcap = kcap;
    P.nhalves = nb >= 0 ? 2 : 1;
    plan_half(na, P.h[0]);
    uint64_t nmax = P.h[0].N;
    if (nb >= 0) {
        plan_half(nb, P.h[1]);
        nmax = std::max(nmax, P.h[1].N);
    }
    plan_bits(nmax, batch, nb < 0, P.B1, P.B2, P.sub);
    // One search whose level-1 buckets average four or more 2^13-key tiles
    // takes them: half as many tile segments per sub-bucket for K3 to gather.
    // A batch keeps the smaller tiles (its buckets hold a few partial ones).
    if (!batch && (nmax >> P.B1) >= (1ull << (T2_BIG_LOG + 2))) P.t2log = T2_BIG_LOG;
    return layout(P, nullptr);
}

void build_job(JobPlan &P, char *ws, const uint64_t *wa, const uint64_t *wb, uint64_t t_lo, uint64_t t_hi,
               uint64_t *out, uint64_t *out_count, uint64_t cap, JobArgs &J) {
    layout(P, ws);
    J = JobArgs();
    J.B1 = P.B1;
    J.B2 = P.B2;
    for (int k = 0; k < 2; ++k) J.h[k] = P.h[k < P.nhalves ? k : 0].a;
    for (int i = 0; i < P.h[0].m; ++i) J.wts[0][i] = wa[i];
    if (P.nhalves == 2)
        for (int i = 0; i < P.h[1].m; ++i) J.wts[1][i] = wb[i];
    else
        for (int i = 0; i < P.h[0].m; ++i) J.wts[1][i] = wa[i];
    J.kp = P.kp;
    J.kp_count = P.counters;
    J.rec = P.rec;
    J.rec_count = P.counters + 3;
    J.flags = (uint32_t *)(P.counters + 2);
    J.kcap = P.kcap;
    J.t_lo = t_lo;
    J.t_hi = t_hi;
    J.out = out;
    J.out_count = out_count;
    J.cap = cap;
    J.first_chunk = 1;
}

// Blocks (x) of every stage for one job; the y dimension is the half.
void stage_blocks(const JobPlan &P, uint32_t *x) {
    uint32_t mw = 0;
    uint64_t mt = 0, ms = 0;
    for (int k = 0; k < P.nhalves; ++k) {
        mw = std::max(mw, P.h[k].nwg1);
        mt = std::max<uint64_t>(mt, P.h[k].ntile2_max);
        ms = std::max(ms, P.h[k].steps);
    }
    x[ST_INIT] = 1;
    x[ST_COUNT] = mw;
    x[ST_COLS] = 1u << P.B1;
    x[ST_BUCKETS] = 1;
    x[ST_ENUM] = mw;
    x[ST_TILE2] = (uint32_t)mt;
    x[ST_JOIN] = 1u << (P.B1 + P.B2);
    x[ST_RFEW] = (uint32_t)((ms + (uint64_t)NT1 * SPT4 - 1) / ((uint64_t)NT1 * SPT4));
    x[ST_RMANY] = mw;
    x[ST_PAIRS] = 1;
}

// All stages of a single-job or multi-job launch; with MULTI the grid of each
// stage is grids[stage] and the per-job block offsets live in M.bases.
template <bool MULTI>
static hipError_t launch_all(const JobArgs &J, const Multi &M, const uint32_t *grids, int nh, int maxB1,
                             int maxB2, int maxT2, bool search, uint64_t *sorted, hipStream_t st,
                             StageEvents *ev) {
    auto rec = [&](int i) {
        if (ev && ev->ev[i]) (void)hipEventRecord((hipEvent_t)ev->ev[i], st);
    };
    rec(0);
    hipLaunchKernelGGL((k_init<MULTI>), dim3(grids[ST_INIT]), dim3(64), 0, st, J, M);
    if (maxB1 <= 8) hipLaunchKernelGGL((k_enum<true, 256, MULTI>), dim3(grids[ST_COUNT], nh), dim3(NT1), 0, st, J, M);
    else if (maxB1 <= 10) hipLaunchKernelGGL((k_enum<true, 1024, MULTI>), dim3(grids[ST_COUNT], nh), dim3(NT1), 0, st, J, M);
    else if (maxB1 <= 11) hipLaunchKernelGGL((k_enum<true, 2048, MULTI>), dim3(grids[ST_COUNT], nh), dim3(NT1), 0, st, J, M);
    else hipLaunchKernelGGL((k_enum<true, MAXB1, MULTI>), dim3(grids[ST_COUNT], nh), dim3(NT1), 0, st, J, M);
    rec(1);
    hipLaunchKernelGGL((k_scan_cols<MULTI>), dim3(grids[ST_COLS], nh), dim3(NT1), 0, st, J, M);
    hipLaunchKernelGGL((k_scan_buckets<MULTI>), dim3(grids[ST_BUCKETS], nh), dim3(NT1), 0, st, J, M);
    rec(2);
    if (maxB1 <= 8) hipLaunchKernelGGL((k_enum<false, 256, MULTI>), dim3(grids[ST_ENUM], nh), dim3(NT1), 0, st, J, M);
    else if (maxB1 <= 10) hipLaunchKernelGGL((k_enum<false, 1024, MULTI>), dim3(grids[ST_ENUM], nh), dim3(NT1), 0, st, J, M);
    else if (maxB1 <= 11) hipLaunchKernelGGL((k_enum<false, 2048, MULTI>), dim3(grids[ST_ENUM], nh), dim3(NT1), 0, st, J, M);
    else hipLaunchKernelGGL((k_enum<false, MAXB1, MULTI>), dim3(grids[ST_ENUM], nh), dim3(NT1), 0, st, J, M);
    rec(3);
    // the workgroup holds the launch's largest tile (a job's tiles may be
    // smaller); 2^11 digits get their own instantiation, whose LDS (81 KB with
    // 8192-key tiles) lets two workgroups share a CU where 4096 digits allow one
    if (maxT2 > T2_LOG) {
        constexpr int NT = (1 << T2_BIG_LOG) / KPT2;
        if (maxB2 <= 8) hipLaunchKernelGGL((k_tile2<256, NT, MULTI>), dim3(grids[ST_TILE2], nh), dim3(NT), 0, st, J, M);
        else if (maxB2 <= 10) hipLaunchKernelGGL((k_tile2<1024, NT, MULTI>), dim3(grids[ST_TILE2], nh), dim3(NT), 0, st, J, M);
        else if (maxB2 <= 11) hipLaunchKernelGGL((k_tile2<2048, NT, MULTI>), dim3(grids[ST_TILE2], nh), dim3(NT), 0, st, J, M);
        else hipLaunchKernelGGL((k_tile2<MAXB2, NT, MULTI>), dim3(grids[ST_TILE2], nh), dim3(NT), 0, st, J, M);
    } else {
        constexpr int NT = (1 << T2_LOG) / KPT2;
        if (maxB2 <= 8) hipLaunchKernelGGL((k_tile2<256, NT, MULTI>), dim3(grids[ST_TILE2], nh), dim3(NT), 0, st, J, M);
        else if (maxB2 <= 10) hipLaunchKernelGGL((k_tile2<1024, NT, MULTI>), dim3(grids[ST_TILE2], nh), dim3(NT), 0, st, J, M);
        else if (maxB2 <= 11) hipLaunchKernelGGL((k_tile2<2048, NT, MULTI>), dim3(grids[ST_TILE2], nh), dim3(NT), 0, st, J, M);
        else hipLaunchKernelGGL((k_tile2<MAXB2, NT, MULTI>), dim3(grids[ST_TILE2], nh), dim3(NT), 0, st, J, M);
    }
    rec(4);
    if (!search) {
        hipLaunchKernelGGL((k_join<true, MULTI>), dim3(grids[ST_JOIN]), dim3(NT3), 0, st, J, M, sorted);
        return hipGetLastError();
    }
    // a grid's work-items must number below 2^32: beyond 2^22 sub-buckets
    // (single searches only) the grid takes a second dimension
    const dim3 gj = (!MULTI && grids[ST_JOIN] > (1u << 22)) ? dim3(1u << 22, grids[ST_JOIN] >> 22) : dim3(grids[ST_JOIN]);
    hipLaunchKernelGGL((k_join<false, MULTI>), gj, dim3(NT3), 0, st, J, M, (uint64_t *)nullptr);
    rec(5);
    hipLaunchKernelGGL((k_recover_few<MULTI>), dim3(grids[ST_RFEW], 2), dim3(NT1), 0, st, J, M);
    hipLaunchKernelGGL((k_recover<MULTI>), dim3(MULTI ? grids[ST_RMANY] : std::min(grids[ST_RMANY], (uint32_t)RECOVER_WGS), 2),
                       dim3(NT1), 0, st, J, M);
    hipLaunchKernelGGL((k_pairs<MULTI>), dim3(grids[ST_PAIRS]), dim3(NT1), 0, st, J, M);
    rec(6);
    return hipGetLastError();
}

// Chunks of half A needed to fit ws_bytes: the smallest c such that a search
// over half A's low n_a - c weights (the top c fixed per chunk) plus all of
// half B' fits (c <= MAX_CHUNK_BITS).  Returns -1 if none fits.
int chunk_bits(int n, size_t ws_bytes) {
    int na, nb;
    split_halves(n, na, nb);
    for (int c = std::max(0, na - MAX_HALF); c <= std::min(na, MAX_CHUNK_BITS); ++c) {
        JobPlan P;
        if (plan_job(na - c, nb, P, KCAP_MAX) <= ws_bytes) return c;
    }
    return -1;
}

__global__ __launch_bounds__(NTS) void k_small_one(SmallJob S);  // below, with the batch's small searches

rfr_status enqueue_recombine(const uint64_t *w, int n, uint64_t t_lo, uint64_t t_hi, void *ws,
                             size_t ws_bytes, hipStream_t st, uint64_t *cand, uint64_t cap,
                             uint64_t *count, StageEvents *ev, std::string &err) {
    if (!w || n < 2 || n > MAX_SEARCH_N || !ws || !cand || !count) {
        err = "rfr_recombine_dev: bad argument (need 2 <= n <= 70 and non-NULL buffers)";
        return RFR_EINVAL;
    }
    if (t_lo >= (1ull << 32) || t_hi >= (1ull << 32) || t_lo + t_hi >= (1ull << 32)) {
        err = "rfr_recombine_dev: window must satisfy t_lo + t_hi < 2^32";
        return RFR_EINVAL;
    }
    if (cap < 1) {
        err = "rfr_recombine_dev: cap must be at least 1";
        return RFR_EINVAL;
    }
    int na, nb;
    split_halves(n, na, nb);
    if (na <= SMALL_HALF && nb <= SMALL_HALF) {
        // both halves fit one workgroup's LDS: the whole search is one launch
        SmallJob S{};
        S.na = na;
        S.nb = nb;
        for (int t = 0; t < n - 1; ++t) S.w[t] = w[t];
        S.t_lo = t_lo;
        S.t_hi = t_hi;
        S.out = cand;
        S.out_count = count;
        S.cap = cap;
        auto rec = [&](int i) {
            if (ev && ev->ev[i]) (void)hipEventRecord((hipEvent_t)ev->ev[i], st);
        };
        rec(0);
        hipLaunchKernelGGL(k_small_one, dim3(1), dim3(NTS), 0, st, S);
        for (int i = 1; i < 7; ++i) rec(i);
        if (hipGetLastError() != hipSuccess) {
            err = "kernel launch failed";
            return RFR_EDEVICE;
        }
        return RFR_OK;
    }
    const int c = chunk_bits(n, ws_bytes);
    if (c < 0) {
        err = "rfr_recombine_dev: workspace too small";
        return RFR_ENOMEM;
    }
    const int ma = na - c;  // weights of half A enumerated per chunk
    JobPlan P;
    plan_job(ma, nb, P, KCAP_MAX);
    uint64_t wneg[MAX_HALF];  // on the stack: the allocation-free entry point shares this path
    for (int i = 0; i < nb; ++i) wneg[i] = 0 - w[na + i];
    uint32_t grids[NSTAGES];
    stage_blocks(P, grids);
    grids[ST_TILE2] = (grids[ST_TILE2] + 7) & ~7u;  // single launch: K2 deals tiles to XCDs in 8 ranges
    Multi M{};
    const uint64_t nchunks = 1ull << c;
    for (uint64_t t = 0; t < nchunks; ++t) {
        JobArgs J;
        build_job(P, (char *)ws, w, wneg, t_lo, t_hi, cand, count, cap, J);
        J.kcap = std::min<uint64_t>(cap + 1, KCAP_MAX);
        uint64_t kb = 0;
        for (int i = 0; i < c; ++i)
            if ((t >> i) & 1) kb += w[ma + i];
        J.kbase[0] = kb;
        J.pbase[0] = t << ma;
        J.first_chunk = t == 0;
        // half B' is enumerated, partitioned and tile-sorted by the first chunk
        // only; later chunks redo half A and join against the resident B'
        if (launch_all<false>(J, M, grids, t == 0 ? 2 : 1, P.B1, P.B2, P.t2log, true, nullptr, st,
                              nchunks == 1 ? ev : nullptr) != hipSuccess) {
            err = "kernel launch failed";
            return RFR_EDEVICE;
        }
    }
    return RFR_OK;
}

// ---------------------------------------------------------------- allocation-free search
// Workspace of rfr_recombine_dev_noalloc: one fixed device array per GPU,
// allocated with the code object when the library is first used on that GPU
// and held until the process ends.  Host code never passes `scratch` itself to
// a kernel (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, once per device, with that device
// current, and is kept in g_scratch_dev.
static __device__ __align__(256) uint64_t scratch[NOALLOC_WS_BYTES / 8];

static std::mutex g_scratch_mu;
static void *g_scratch_dev[NOALLOC_MAX_DEVICES];

rfr_status enqueue_recombine_noalloc(const uint64_t *w, int n, uint64_t t_lo, uint64_t t_hi, hipStream_t st,
                                     uint64_t *cand, uint64_t cap, uint64_t *count, std::string &err) {
    if (n < 2 || n > NOALLOC_MAX_N) {
        err = "rfr_recombine_dev_noalloc: need 2 <= n <= " + std::to_string(NOALLOC_MAX_N) +
              " (the fixed device scratch holds " + std::to_string(NOALLOC_WS_BYTES >> 20) + " MiB)";
        return n < 2 ? RFR_EINVAL : RFR_ENOMEM;
    }
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= NOALLOC_MAX_DEVICES) {
        err = "rfr_recombine_dev_noalloc: no usable current device";
        return RFR_EDEVICE;
    }
    void *ws;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_dev[device]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                err = std::string("rfr_recombine_dev_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e);
                return RFR_EDEVICE;
            }
            g_scratch_dev[device] = p;
        }
        ws = g_scratch_dev[device];
    }
    // every counter the pipeline reads is cleared by its first kernel (k_init),
    // so the previous call's contents need no clearing here
    return enqueue_recombine(w, n, t_lo, t_hi, ws, NOALLOC_WS_BYTES, st, cand, cap, count, nullptr, err);
}

size_t recombine_workspace(int n) {
    if (n < 2 || n > MAX_SEARCH_N) return 0;
    int na, nb;
    split_halves(n, na, nb);
    JobPlan P;
    // a half A beyond MAX_HALF weights is always streamed: its largest chunk
    return plan_job(std::min(na, MAX_HALF), nb, P, KCAP_MAX);
}

size_t expand_workspace(int m) {
    if (m < 1 || m > 30) return 0;
    JobPlan P;
    return plan_job(m, -1, P, 1);
}

rfr_status enqueue_expand(const uint64_t *w, int m, int negate, void *ws, size_t ws_bytes,
                          hipStream_t st, uint64_t *sorted, std::string &err) {
    if (!w || m < 1 || m > 30 || !ws || !sorted) {
        err = "rfr_expand_dev: bad argument (need 1 <= m <= 30)";
        return RFR_EINVAL;
    }
    JobPlan P;
    uint64_t need = plan_job(m, -1, P, 1);
    if (ws_bytes < need) {
        err = "rfr_expand_dev: workspace too small";
        return RFR_ENOMEM;
    }
    std::vector<uint64_t> ww(w, w + m);
    if (negate)
        for (auto &v : ww) v = 0 - v;
    JobArgs J;
    build_job(P, (char *)ws, ww.data(), nullptr, 0, 0, nullptr, nullptr, 0, J);
    J.kcap = 1;
    uint32_t grids[NSTAGES];
    stage_blocks(P, grids);
    grids[ST_TILE2] = (grids[ST_TILE2] + 7) & ~7u;  // single launch: K2 deals tiles to XCDs in 8 ranges
    Multi M{};
    if (launch_all<false>(J, M, grids, 1, P.B1, P.B2, P.t2log, false, sorted, st, nullptr) != hipSuccess) {
        err = "kernel launch failed";
        return RFR_EDEVICE;
    }
    // A sub-bucket beyond the LDS sort's capacity (more than CAP3 keys share
    // their top B1 + B2 bits: many equal or clustered sums) is left unsorted
    // and flagged; report it rather than return a partly written output.
    uint32_t flags = 0;
    if (hipMemcpyAsync(&flags, J.flags, sizeof(flags), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        err = "rfr_expand_dev: device error";
        return RFR_EDEVICE;
    }
    if (flags & 1u) {
        err = "rfr_expand_dev: the sums are too clustered for the sort (a sub-bucket holds more than 2048 keys)";
        return RFR_EOVERFLOW;
    }
    return RFR_OK;
}

// ---------------------------------------------------------------- batches
void MultiLaunch::add(const JobPlan &P, const JobArgs &J) {
    uint32_t x[NSTAGES];
    stage_blocks(P, x);
    if (bases.empty()) bases.assign(NSTAGES, std::vector<uint32_t>(1, 0));
    for (int s = 0; s < NSTAGES; ++s) bases[s].push_back(bases[s].back() + x[s]);
    jobs.push_back(J);
    maxB1 = std::max(maxB1, P.B1);
    maxB2 = std::max(maxB2, P.B2);
    maxT2 = std::max(maxT2, P.t2log);
}

// Entries of each stage's block -> job table (see pick()).
static uint32_t group_entries(uint32_t grid) { return (grid + PICK_GRP - 1) / PICK_GRP + 1; }

size_t MultiLaunch::bases_bytes() const {
    size_t n = (size_t)NSTAGES * (jobs.size() + 1);
    for (int s = 0; s < NSTAGES; ++s) n += group_entries(bases.empty() ? 0 : bases[s].back());
    return n * 4;
}

void MultiLaunch::pack_bases(uint32_t *dst) const {
    const size_t nj = jobs.size();
    for (int s = 0; s < NSTAGES; ++s)
        for (size_t j = 0; j <= nj; ++j) dst[s * (nj + 1) + j] = bases.empty() ? 0 : bases[s][j];
    uint32_t *g = dst + (size_t)NSTAGES * (nj + 1);
    for (int s = 0; s < NSTAGES; ++s) {
        const uint32_t grid = bases.empty() ? 0 : bases[s].back();
        const uint32_t ne = group_entries(grid);
        size_t j = 0;  // last job whose first block is <= x
        for (uint32_t e = 0; e + 1 < ne; ++e) {
            const uint64_t x = (uint64_t)e * PICK_GRP;
            while (j + 1 < nj && bases[s][j + 1] <= x) ++j;
            g[e] = (uint32_t)j;
        }
        g[ne - 1] = nj ? (uint32_t)(nj - 1) : 0;
        g += ne;
    }
}

hipError_t MultiLaunch::launch(const JobArgs *jobs_dev, const uint32_t *bases_dev, hipStream_t st,
                               StageEvents *ev) const {
    if (jobs.empty()) return hipSuccess;
    Multi M{};
    M.jobs = jobs_dev;
    M.bases = bases_dev;
    M.njobs = (int)jobs.size();
    M.groups = bases_dev + (size_t)NSTAGES * (jobs.size() + 1);
    uint32_t off = 0;
    for (int s = 0; s < NSTAGES; ++s) {
        M.gofs[s] = off;
        off += group_entries(bases[s].back());
    }
    uint32_t grids[NSTAGES];
    for (int s = 0; s < NSTAGES; ++s) grids[s] = bases[s].back();
    JobArgs dummy{};
    return launch_all<true>(dummy, M, grids, 2, maxB1, maxB2, maxT2, true, nullptr, st, ev);
}

// ---------------------------------------------------------------- small searches
// One workgroup searches one polynomial with both halves <= 2^SMALL_HALF keys
// entirely in LDS: A's sums by pattern index, B' radix-sorted by its top LB3
// bits together with its pattern index, then every a probes the bins its
// cyclic window overlaps and emits pattern pairs directly.  Workgroups are
// persistent and take the next job (largest first) from an atomic counter.
// LDS of one small search.
struct SmallLds {
    uint64_t a[1 << SMALL_HALF];
    uint64_t b[1 << SMALL_HALF];
    uint16_t bi[1 << SMALL_HALF];
    uint32_t bin[NB3 + 1];
    uint64_t tmp[NTS / 64 + 2];
    unsigned long long cnt;
};

// One whole search in a workgroup's LDS: half A's sums in pattern order, half
// B' counting-sorted by its top LB3 bits, and every a's window looked up among
// the bins it covers.
__device__ void small_search(const SmallJob &S, SmallLds &L) {
    uint64_t *s_a = L.a, *s_b = L.b, *s_tmp = L.tmp;
    uint16_t *s_bi = L.bi;
    uint32_t *s_bin = L.bin;
    unsigned long long &s_cnt = L.cnt;
    const int tid = threadIdx.x;
    constexpr int KPS = (1 << SMALL_HALF) / NTS;
    const int na = S.na, nb = S.nb;
    const uint32_t NA = 1u << na, NBk = 1u << nb;
    for (int i = tid; i < NB3; i += NTS) s_bin[i] = 0;
    if (tid == 0) s_cnt = 0;
    for (uint32_t i = tid; i < NA; i += NTS) {
        uint64_t v = 0;
        for (int e = 0; e < na; ++e)
            if ((i >> e) & 1) v += S.w[e];
        s_a[i] = v;
    }
    __syncthreads();
    uint64_t kb[KPS];
    uint32_t rk[KPS];
#pragma unroll
    for (int k = 0; k < KPS; ++k) {
        const uint32_t i = tid + k * NTS;
        if (i < NBk) {
            uint64_t v = 0;
            for (int e = 0; e < nb; ++e)
                if ((i >> e) & 1) v -= S.w[na + e];
            kb[k] = v;
            rk[k] = atomicAdd(&s_bin[(uint32_t)(v >> (64 - LB3))], 1u);
        }
    }
    __syncthreads();
    lds_excl_scan<NTS, NB3 / NTS>(s_bin, NB3, s_tmp);
    if (tid == 0) s_bin[NB3] = NBk;
#pragma unroll
    for (int k = 0; k < KPS; ++k) {
        const uint32_t i = tid + k * NTS;
        if (i < NBk) {
            const uint32_t p = s_bin[(uint32_t)(kb[k] >> (64 - LB3))] + rk[k];
            s_b[p] = kb[k];
            s_bi[p] = (uint16_t)i;
        }
    }
    __syncthreads();
    const uint64_t t_lo = S.t_lo, t_hi = S.t_hi;
    for (uint32_t i = tid; i < NA; i += NTS) {
        const uint64_t a = s_a[i];
        // the cyclic window [a - t_hi, a + t_lo] as up to two plain ranges
        uint64_t lo[2], hi[2];
        int nr = 0;
        if (a >= t_hi) {
            lo[0] = a - t_hi;
        } else {
            lo[0] = 0;
            lo[1] = a - t_hi;  // wraps: [2^64 - (t_hi - a), 2^64)
            hi[1] = ~0ull;
            nr = 1;
        }
        if (a <= ~0ull - t_lo) {
            hi[0] = a + t_lo;
        } else {
            hi[0] = ~0ull;
            lo[1] = 0;
            hi[1] = a + t_lo;  // wraps: [0, a + t_lo - 2^64]
            nr = 1;
        }
        for (int r = 0; r <= nr; ++r) {
            const uint32_t b0 = (uint32_t)(lo[r] >> (64 - LB3)), b1 = (uint32_t)(hi[r] >> (64 - LB3));
            const uint32_t e = s_bin[b1 + 1];
            for (uint32_t q = s_bin[b0]; q < e; ++q) {
                const uint64_t bk = s_b[q];
                if (bk < lo[r] || bk > hi[r]) continue;
                const uint32_t pb = s_bi[q];
                if (i == 0 && pb == 0) continue;  // the empty pattern
                const unsigned long long o = atomicAdd(&s_cnt, 1ull);
                if (o < S.cap) {
                    S.out[2 * o] = i;
                    S.out[2 * o + 1] = pb;
                }
            }
        }
    }
    __syncthreads();
    if (tid == 0) *S.out_count = s_cnt > S.cap ? ~0ull : s_cnt;
    __syncthreads();
}

// Small searches of a batch: a persistent grid takes them from an atomic queue.
__global__ __launch_bounds__(NTS) void k_small(const SmallJob *jobs, int njobs, uint32_t *queue) {
    __shared__ SmallLds L;
    __shared__ int s_job;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_job = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int j = s_job;
        if (j >= njobs) return;
        small_search(jobs[j], L);
    }
}

// One small search passed by value (a plain or served request).
__global__ __launch_bounds__(NTS) void k_small_one(SmallJob S) {
    __shared__ SmallLds L;
    small_search(S, L);
}

__global__ void k_small_init(uint32_t *queue) {
    if (threadIdx.x == 0) *queue = 0;
}

hipError_t launch_small(const SmallJob *jobs_dev, int njobs, uint32_t *queue_dev, int grid, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_small_init, dim3(1), dim3(64), 0, st, queue_dev);
    hipLaunchKernelGGL(k_small, dim3(grid), dim3(NTS), 0, st, jobs_dev, njobs, queue_dev);
    return hipGetLastError();
}

// ================================================================= Algorithm E variant
// Section 3.5 (SPLAT, QUERY, RECOMBINE_E) and Section 4: half B' is expanded
// and sorted once (the EXPAND kernels above), then laid out as the paper's
// splat table -- k = 2 N_B cells, value x homed at cell floor(k x / 2^64),
// every value at or after its home, in ascending order, empty cells between
// runs -- and half A is never stored or sorted: every A key is generated by
// the Gray-code walk and looked up in the table (QUERY, reporting every
// partner in the window instead of the first).  Only candidate key pairs
// leave the query; the recovery and pair kernels of the search follow.
//
// The table is what inserting the sorted values one after another by the
// paper's INSERT gives: with values in ascending order no exchange happens,
// and value i lands at p_i = max(home_i, p_(i-1) + 1) = i + max_(j <= i)
// (home_j - j), a prefix maximum.  Cells are not wrapped around: the table
// has N_B extra cells at its end for the runs that pass cell k - 1.
namespace dev {

struct SplatArgs {
    const uint64_t *sorted;  // [nb] B' keys, ascending
    uint64_t *tbl;           // [tlen] cell values
    uint32_t *occ;           // [ceil(tlen / 32)] occupied cells
    int64_t *bmax;           // [nblk] per-block maxima of home_i - i, then their exclusive prefix maxima
    uint64_t nb, tlen;
    int hsh;                 // home(x) = x >> hsh (k = 2^(64 - hsh) cells)
    int nblk;
    const uint32_t *xflags;  // the expansion's flags (bit 0: a sub-bucket beyond its sort)
};
constexpr int SPT_E = 16;               // values per thread in the table build
constexpr int SPB_E = NT1 * SPT_E;      // values per block

__global__ __launch_bounds__(NT1) void k_splat_clear(SplatArgs S) {
    const uint64_t words = (S.tlen + 31) / 32;
    for (uint64_t i = (uint64_t)blockIdx.x * NT1 + threadIdx.x; i < words; i += (uint64_t)gridDim.x * NT1)
        S.occ[i] = 0;
}

__device__ __forceinline__ int64_t max_i64(int64_t a, int64_t b) { return a > b ? a : b; }

template <int NTH>
__device__ __forceinline__ int64_t block_max_i64(int64_t v, int64_t *s_tmp) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max_i64(v, __shfl_xor(v, o, 64));
    if (lane == 0) s_tmp[wv] = v;
    __syncthreads();
    int64_t r = s_tmp[0];
    for (int i = 1; i < NTH / 64; ++i) r = max_i64(r, s_tmp[i]);
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(NT1) void k_splat_max(SplatArgs S) {
    __shared__ int64_t s_tmp[NT1 / 64];
    const uint64_t i0 = (uint64_t)blockIdx.x * SPB_E;
    int64_t m = INT64_MIN;
    for (int k = 0; k < SPT_E; ++k) {
        const uint64_t i = i0 + (uint64_t)k * NT1 + threadIdx.x;
        if (i < S.nb) m = max_i64(m, (int64_t)(S.sorted[i] >> S.hsh) - (int64_t)i);
    }
    m = block_max_i64<NT1>(m, s_tmp);
    if (threadIdx.x == 0) S.bmax[blockIdx.x] = m;
}

// bmax[b] becomes the maximum over blocks before b (INT64_MIN for block 0)
__global__ __launch_bounds__(NT1) void k_splat_scan(SplatArgs S) {
    __shared__ int64_t s_tmp[NT1 / 64];
    int64_t carry = INT64_MIN;
    for (int base = 0; base < S.nblk; base += NT1) {
        const int i = base + (int)threadIdx.x;
        const int64_t v = i < S.nblk ? S.bmax[i] : INT64_MIN;
        // inclusive prefix maximum across the block
        int64_t inc = v;
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t t = __shfl_up(inc, o, 64);
            if (lane >= o) inc = max_i64(inc, t);
        }
        if (lane == 63) s_tmp[wv] = inc;
        __syncthreads();
        int64_t before = carry;
        for (int w = 0; w < wv; ++w) before = max_i64(before, s_tmp[w]);
        int64_t ex = __shfl_up(inc, 1, 64);
        if (lane == 0) ex = INT64_MIN;
        const int64_t excl = max_i64(before, ex);
        int64_t tot = carry;
        for (int w = 0; w < NT1 / 64; ++w) tot = max_i64(tot, s_tmp[w]);
        __syncthreads();
        if (i < S.nblk) S.bmax[i] = excl;
        carry = tot;
    }
}

__global__ __launch_bounds__(NT1) void k_splat_place(SplatArgs S) {
    __shared__ int64_t s_tmp[NT1 / 64 + 1];
    const uint64_t i0 = (uint64_t)blockIdx.x * SPB_E + (uint64_t)threadIdx.x * SPT_E;
    uint64_t x[SPT_E];
    int64_t run = INT64_MIN;
#pragma unroll
    for (int k = 0; k < SPT_E; ++k) {
        const uint64_t i = i0 + k;
        x[k] = i < S.nb ? S.sorted[i] : 0;
        if (i < S.nb) run = max_i64(run, (int64_t)(x[k] >> S.hsh) - (int64_t)i);
    }
    // exclusive prefix maximum of the threads' maxima, then the blocks before
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc = max_i64(inc, t);
    }
    if (lane == 63) s_tmp[wv] = inc;
    __syncthreads();
    int64_t m = S.bmax[blockIdx.x];
    for (int w = 0; w < wv; ++w) m = max_i64(m, s_tmp[w]);
    int64_t ex = __shfl_up(inc, 1, 64);
    if (lane != 0) m = max_i64(m, ex);
#pragma unroll
    for (int k = 0; k < SPT_E; ++k) {
        const uint64_t i = i0 + k;
        if (i >= S.nb) break;
        m = max_i64(m, (int64_t)(x[k] >> S.hsh) - (int64_t)i);
        const uint64_t p = i + (uint64_t)m;
        S.tbl[p] = x[k];
        atomicOr(&S.occ[p >> 5], 1u << (p & 31));
    }
}

// QUERY over [lo, hi] (lo <= hi): from lo's home cell, skip values below lo,
// report values up to hi, stop at a value above hi or at an empty cell past
// hi's home (every value <= hi sits in the run that starts at or before it).
__device__ __forceinline__ void splat_query(const JobArgs &J, const SplatArgs &S, uint64_t a, uint64_t lo,
                                            uint64_t hi) {
    const uint64_t e = hi >> S.hsh;
    for (uint64_t i = lo >> S.hsh; i < S.tlen; ++i) {
        if ((S.occ[i >> 5] >> (i & 31)) & 1u) {
            const uint64_t x = S.tbl[i];
            if (x > hi) break;
            if (x >= lo) emit_pair(J, a, x);
        } else if (i >= e) {
            break;
        }
    }
}

// RECOMBINE_E's loop: the A keys of Gray steps [h0, h1) of this workgroup
// (lane l owns the low L pattern bits, as in the enumeration kernels), each
// queried for B' keys b' with b' - a in [-t_hi, t_lo] (mod 2^64).
__global__ __launch_bounds__(NT1) void k_query(JobArgs J, SplatArgs S) {
    const HalfArgs &H = J.h[0];
    const uint32_t wg = blockIdx.x;
    if (wg >= H.nwg1) return;
    if (*S.xflags & 1u) {
        if (wg == 0 && threadIdx.x == 0) atomicOr(J.flags, 4u);
        return;
    }
    const int tid = threadIdx.x;
    const int nl = 1 << H.L;
    const bool act = tid < nl;
    __shared__ uint64_t s_w[64];
    if (tid < H.m) s_w[tid] = J.wts[0][tid];
    __syncthreads();
    uint64_t slo = J.kbase[0];
    for (int i = 0; i < H.L; ++i)
        if ((tid >> i) & 1) slo += s_w[i];
    const uint64_t h0 = (uint64_t)wg * H.spw;
    const uint64_t h1 = min(h0 + (uint64_t)H.spw, H.steps);
    uint64_t g = h0 ^ (h0 >> 1);
    uint64_t shi = 0;
    for (int i = 0; i < H.m - H.L; ++i)
        if ((g >> i) & 1) shi += s_w[H.L + i];
    const uint64_t t_lo = J.t_lo, t_hi = J.t_hi;
    for (uint64_t h = h0; h < h1; ++h) {
        if (act) {
            const uint64_t a = slo + shi;
            const uint64_t lo = a - t_hi, hi = a + t_lo;
            if (lo <= hi) {
                splat_query(J, S, a, lo, hi);
            } else {  // the window wraps past 0
                splat_query(J, S, a, lo, ~0ull);
                splat_query(J, S, a, 0, hi);
            }
        }
        const uint64_t t = h + 1;
        if (t < h1) {
            const int bb = __builtin_ctzll(t);
            g ^= 1ull << bb;
            const uint64_t wb = s_w[H.L + bb];
            shi += ((g >> bb) & 1) ? wb : (0 - wb);
        }
    }
}

}  // namespace dev

// Workspace of the query design: the expansion of half B' and its sorted
// output, the table and its occupancy bits, the per-block maxima, and the
// candidate buffers of the recovery.
struct EPlan {
    JobPlan X;  // expansion of half B'
    uint64_t off_sorted, off_tbl, off_occ, off_bmax, off_kp, off_rec, off_cnt, total;
    uint64_t nb, tlen;
    int hsh, nblk;
};

static uint64_t e_plan(int na, int nb, EPlan &E) {
    (void)na;
    uint64_t off = plan_job(nb, -1, E.X, 1);
    auto take = [&](uint64_t bytes) {
        off = align_up(off, 256);
        const uint64_t o = off;
        off += bytes;
        return o;
    };
    E.nb = 1ull << nb;
    E.hsh = 64 - (nb + 1);  // k = 2 N_B cells
    E.tlen = (2ull << nb) + E.nb;
    E.nblk = (int)((E.nb + SPB_E - 1) / SPB_E);
    E.off_sorted = take(E.nb * 8);
    E.off_tbl = take(E.tlen * 8);
    E.off_occ = take((E.tlen + 31) / 32 * 4);
    E.off_bmax = take((uint64_t)E.nblk * 8);
    E.off_kp = take((uint64_t)KCAP_MAX * 16);
    E.off_rec = take(2ull * KCAP_MAX * 16);
    E.off_cnt = take(64);
    E.total = align_up(off, 256);
    return E.total;
}

size_t recombine_e_workspace(int n) {
    if (n < 2 || n > 2 * E_MAX_HALF + 1) return 0;
    int na, nb;
    split_halves(n, na, nb);
    if (nb < 1) return 0;
    EPlan E;
    return e_plan(na, nb, E);
}

rfr_status enqueue_recombine_e(const uint64_t *w, int n, uint64_t t_lo, uint64_t t_hi, void *ws, size_t ws_bytes,
                               hipStream_t st, uint64_t *cand, uint64_t cap, uint64_t *count, std::string &err) {
    if (!w || n < 2 || n > 2 * E_MAX_HALF + 1 || !ws || !cand || !count || cap < 1) {
        err = "rfr_recombine_e_dev: bad argument (need 2 <= n <= 2 * 26 + 1 and non-NULL buffers)";
        return RFR_EINVAL;
    }
    int na, nb;
    split_halves(n, na, nb);
    if (nb < 1) {  // n = 2: no B' weights; the HS pipeline covers it
        err = "rfr_recombine_e_dev: needs n >= 3";
        return RFR_EINVAL;
    }
    EPlan E;
    if (e_plan(na, nb, E) > ws_bytes) {
        err = "rfr_recombine_e_dev: workspace too small";
        return RFR_ENOMEM;
    }
    char *base = (char *)ws;
    // 1. EXPAND of half B' (negated weights) into the sorted array
    uint64_t wneg[MAX_HALF];
    for (int i = 0; i < nb; ++i) wneg[i] = 0 - w[na + i];
    uint64_t *sorted = (uint64_t *)(base + E.off_sorted);
    JobArgs JX;
    build_job(E.X, base, wneg, nullptr, 0, 0, nullptr, nullptr, 0, JX);
    JX.kcap = 1;
    uint32_t gx[NSTAGES];
    stage_blocks(E.X, gx);
    gx[ST_TILE2] = (gx[ST_TILE2] + 7) & ~7u;
    Multi M{};
    if (launch_all<false>(JX, M, gx, 1, E.X.B1, E.X.B2, E.X.t2log, false, sorted, st, nullptr) != hipSuccess) {
        err = "kernel launch failed";
        return RFR_EDEVICE;
    }
    // 2. the search job: half A enumerated by the query, both halves recovered
    JobArgs J{};
    HalfPlan ha, hb;
    plan_half(na, ha);
    plan_half(nb, hb);
    J.h[0] = HalfArgs{};
    J.h[1] = HalfArgs{};
    for (int k = 0; k < 2; ++k) {
        const HalfPlan &h = k ? hb : ha;
        J.h[k].N = h.N;
        J.h[k].steps = h.steps;
        J.h[k].spw = h.spw;
        J.h[k].nwg1 = h.nwg1;
        J.h[k].m = h.m;
        J.h[k].L = h.L;
    }
    for (int i = 0; i < na; ++i) J.wts[0][i] = w[i];
    for (int i = 0; i < nb; ++i) J.wts[1][i] = wneg[i];
    J.t_lo = t_lo;
    J.t_hi = t_hi;
    J.kp = (uint64_t *)(base + E.off_kp);
    J.rec = (uint64_t *)(base + E.off_rec);
    uint64_t *ctr = (uint64_t *)(base + E.off_cnt);
    J.kp_count = ctr;
    J.flags = (uint32_t *)(ctr + 2);
    J.rec_count = ctr + 3;
    J.kcap = std::min<uint64_t>(cap + 1, KCAP_MAX);
    J.out = cand;
    J.out_count = count;
    J.cap = cap;
    J.first_chunk = 1;
    SplatArgs S{};
    S.sorted = sorted;
    S.tbl = (uint64_t *)(base + E.off_tbl);
    S.occ = (uint32_t *)(base + E.off_occ);
    S.bmax = (int64_t *)(base + E.off_bmax);
    S.nb = E.nb;
    S.tlen = E.tlen;
    S.hsh = E.hsh;
    S.nblk = E.nblk;
    S.xflags = JX.flags;
    const uint32_t clear_grid = (uint32_t)std::min<uint64_t>(((E.tlen + 31) / 32 + NT1 - 1) / NT1, 4096);
    hipLaunchKernelGGL((k_init<false>), dim3(1), dim3(64), 0, st, J, M);
    hipLaunchKernelGGL(k_splat_clear, dim3(clear_grid), dim3(NT1), 0, st, S);
    hipLaunchKernelGGL(k_splat_max, dim3(E.nblk), dim3(NT1), 0, st, S);
    hipLaunchKernelGGL(k_splat_scan, dim3(1), dim3(NT1), 0, st, S);
    hipLaunchKernelGGL(k_splat_place, dim3(E.nblk), dim3(NT1), 0, st, S);
    hipLaunchKernelGGL(k_query, dim3(ha.nwg1), dim3(NT1), 0, st, J, S);
    const uint32_t rfew = (uint32_t)((std::max(ha.steps, hb.steps) + (uint64_t)NT1 * SPT4 - 1) / ((uint64_t)NT1 * SPT4));
    hipLaunchKernelGGL((k_recover_few<false>), dim3(rfew, 2), dim3(NT1), 0, st, J, M);
    hipLaunchKernelGGL((k_recover<false>), dim3(std::min(std::max(ha.nwg1, hb.nwg1), (uint32_t)RECOVER_WGS), 2),
                       dim3(NT1), 0, st, J, M);
    hipLaunchKernelGGL((k_pairs<false>), dim3(1), dim3(NT1), 0, st, J, M);
    if (hipGetLastError() != hipSuccess) {
        err = "kernel launch failed";
        return RFR_EDEVICE;
    }
    return RFR_OK;
}

}  // namespace rfr
