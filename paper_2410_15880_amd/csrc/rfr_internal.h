// Internal declarations shared by the host core, the device pipeline and the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "rfr.h"

namespace rfr {

// ---------------------------------------------------------------- patterns
// A pattern s in {0,1}^n (Section 2: bit i selects element i), n <= 128.
struct Pat {
    uint64_t lo = 0, hi = 0;
    bool get(int i) const { return i < 64 ? (lo >> i) & 1 : (hi >> (i - 64)) & 1; }
    void set(int i) { if (i < 64) lo |= 1ull << i; else hi |= 1ull << (i - 64); }
    Pat operator&(const Pat &o) const { return {lo & o.lo, hi & o.hi}; }
    Pat operator~() const { return {~lo, ~hi}; }
    bool operator==(const Pat &o) const { return lo == o.lo && hi == o.hi; }
    bool operator<(const Pat &o) const { return hi != o.hi ? hi < o.hi : lo < o.lo; }
    bool empty() const { return lo == 0 && hi == 0; }
    static Pat full(int n) {
        Pat p;
        p.lo = n >= 64 ? ~0ull : ((1ull << n) - 1);
        p.hi = n <= 64 ? 0 : (n >= 128 ? ~0ull : ((1ull << (n - 64)) - 1));
        return p;
    }
};

// ---------------------------------------------------------------- double-double
struct dd {
    double hi = 0, lo = 0;
};
struct cdd {
    dd re, im;
};

// ---------------------------------------------------------------- host stages
// Everything the host knows about one polynomial before the search.
struct Prepared {
    int64_t content = 1;          // signed content
    int xpow = 0;                 // power of x split off (0 or 1)
    std::vector<int64_t> prim;    // primitive part, lc > 0, prim[0] != 0
    int n = 0, r = 0;             // elements, real roots
    std::vector<dd> reals;        // r real roots, ascending
    std::vector<cdd> pairs;       // c conjugate-pair representatives (Im > 0), by (Re, Im)
    std::vector<uint64_t> w;      // n weights, canonical element order
    uint64_t t_lo = 0, t_hi = 0;  // accept window
    // second trace (Section 2: sum of squares of the monic-transform roots, an
    // integer for every true factor): per-element weights floor(frac(e_i) 2^64)
    // with e_i = (a_d u)^2 or 2 Re((a_d z)^2), and their window, like w/t_lo/t_hi;
    // tr2_ok is false when the squares are too large for the weights' precision
    std::vector<uint64_t> v2;
    uint64_t t2_lo = 0, t2_hi = 0;
    bool tr2_ok = false;
    std::vector<double> rad;      // n inclusion radii (a pair: the larger of its two discs)
    std::vector<std::vector<int64_t>> peeled;  // factors of single elements split off before the search
};

// One irreducible factor list with content (the result before ABI packing).
struct Factored {
    int64_t content = 1;
    std::vector<std::vector<int64_t>> factors;  // canonical order
    uint64_t n_candidates = 0, n_confirmed = 0;
    int trace_folded = 0;  // 1: the search folded the second trace into the weights
};

// Split content, sign and x-power; validate.  Section 2 preconditions.
rfr_status normalise(const int64_t *coeffs, int degree, Prepared &P, std::string &err);

// One root of P.prim: complex double-double value and inclusion radius; for a
// disc meeting the real axis also the real polished value and its radius
// (rx = +inf otherwise).
struct RootOut {
    double re_hi, re_lo, im_hi, im_lo, r, x_hi, x_lo, rx;
};

// Roots (FP64 Aberth + double-double Newton polish, certified by disjoint
// inclusion discs), elements, weights and window (Sections 2 and 3.3).
rfr_status prepare_elements(Prepared &P, std::string &err);

// The part of prepare_elements after the roots: check the discs, classify,
// pair, order the elements, weights and window, from the d root records ro
// (found on the host or on the device).  P.prim must have degree >= 1.
rfr_status finish_elements(Prepared &P, const RootOut *ro, std::string &err);

// normalise + prepare_elements.
rfr_status prepare(const int64_t *coeffs, int degree, Prepared &P, std::string &err);

// Confirm candidate patterns (over elements [0, n-1)) by exact trial division
// and return the irreducible factors as atoms of the divisors found.
rfr_status confirm_and_factor(const Prepared &P, const std::vector<Pat> &cands, Factored &out,
                              std::string &err);

// Trivial factorisation when no search is needed (n <= 1).
void trivial_factor(const Prepared &P, Factored &out);
// Single-element factors (a real root whose a_d (x - u) rounds to an integer
// factor, a pair whose a_d (x^2 - t x + |z|^2) does) confirmed by exact
// division are split off before the search: prim becomes the quotient, the
// element leaves the set, and weights and window are recomputed for the
// quotient's leading coefficient.  Their factors go to P.peeled (and into the
// result).  This removes the flood of candidates from many rational roots.
rfr_status peel_singletons(Prepared &P, std::string &err);

// Search plan of the n-1 searched elements.
inline void split_halves(int n, int &na, int &nb) {
    int n1 = n - 1;
    na = (n1 + 1) / 2;
    nb = n1 - na;
}

}  // namespace rfr
