// Host core of the RFR library: normalisation, roots, elements, weights, window,
// confirmation and atoms.  Plain C++17, no device code; compiled without
// floating-point contraction so the error-free transformations stay exact.
//
// Paper: Iravanian, arXiv 2410.15880.
//   Section 2     preconditions (square-free, monic transform), Eq 1 real
//                 factorisation, the element set R, Algorithm FACTOR.
//   Section 3.3   integer weights rho_hat = floor(rho * M), Eq 18, accept Eq 19.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <numeric>

#include "rfr_internal.h"

namespace rfr {

// ======================================================================
// double-double arithmetic (error-free transformations, Dekker / Knuth)
// ======================================================================
static inline dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
static inline dd quick_two_sum(double a, double b) {
    double s = a + b;
    return {s, b - (s - a)};
}
static inline dd two_prod(double a, double b) {
    double p = a * b;
    return {p, std::fma(a, b, -p)};
}
static inline dd mkdd(double x) { return {x, 0.0}; }
static inline dd dd_from_i64(int64_t v) {
    // top has at most 52 significant bits (exact in a double), rest < 2^11
    int64_t top = v & ~(int64_t)0x7FF;
    int64_t rest = v - top;
    return two_sum((double)top, (double)rest);
}
static inline dd operator+(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
static inline dd operator-(dd a) { return {-a.hi, -a.lo}; }
static inline dd operator-(dd a, dd b) { return a + (-b); }
static inline dd operator*(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
static inline dd operator*(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
static inline dd operator/(dd a, dd b) {
    double q1 = a.hi / b.hi;
    dd r = a - b * q1;
    double q2 = r.hi / b.hi;
    r = r - b * q2;
    double q3 = r.hi / b.hi;
    dd q = quick_two_sum(q1, q2);
    return q + mkdd(q3);
}
static inline double to_d(dd a) { return a.hi + a.lo; }
static inline dd dd_abs(dd a) { return a.hi < 0 ? -a : a; }

static inline cdd operator+(cdd a, cdd b) { return {a.re + b.re, a.im + b.im}; }
static inline cdd operator-(cdd a, cdd b) { return {a.re - b.re, a.im - b.im}; }
static inline cdd operator*(cdd a, cdd b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
static inline cdd operator/(cdd a, cdd b) {
    dd den = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
static inline double cabs_d(cdd a) { return std::hypot(to_d(a.re), to_d(a.im)); }

// ======================================================================
// normalisation (Section 2 preconditions)
// ======================================================================
static int64_t gcd64(int64_t a, int64_t b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

rfr_status normalise(const int64_t *coeffs, int degree, Prepared &P, std::string &err) {
    if (!coeffs || degree < 1 || degree > RFR_MAX_DEGREE) {
        err = "degree must be in [1, RFR_MAX_DEGREE] and coeffs non-NULL";
        return RFR_EINVAL;
    }
    if (coeffs[degree] == 0) {
        err = "leading coefficient is zero";
        return RFR_EINVAL;
    }
    for (int i = 0; i <= degree; ++i) {
        if (coeffs[i] == INT64_MIN) {
            err = "coefficient INT64_MIN is not supported";
            return RFR_EOVERFLOW;
        }
    }
    int k = 0;
    while (coeffs[k] == 0) ++k;
    if (k > 1) {
        err = "x^2 divides p: not square-free";
        return RFR_ENOTSQFREE;
    }
    int64_t g = 0;
    for (int i = k; i <= degree; ++i) g = gcd64(g, coeffs[i]);
    if (coeffs[degree] < 0) g = -g;
    P.content = g;
    P.xpow = k;
    P.prim.assign(coeffs + k, coeffs + degree + 1);
    for (auto &c : P.prim) c /= g;
    return RFR_OK;
}

// ======================================================================
// modular square-free test (used only to classify a root-separation failure)
// ======================================================================
static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)((unsigned __int128)a * b % q);
}
static uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}
static int gcd_degree_mod(const std::vector<int64_t> &p, uint64_t q) {
    auto red = [&](int64_t v) { int64_t m = v % (int64_t)q; return (uint64_t)(m < 0 ? m + (int64_t)q : m); };
    std::vector<uint64_t> a(p.size()), b(p.size() - 1);
    for (size_t i = 0; i < p.size(); ++i) a[i] = red(p[i]);
    for (size_t i = 1; i < p.size(); ++i) b[i - 1] = mulmod(red(p[i]), (uint64_t)i % q, q);
    auto trim = [](std::vector<uint64_t> &v) { while (!v.empty() && v.back() == 0) v.pop_back(); };
    trim(a);
    trim(b);
    while (!b.empty()) {
        // a = a mod b
        uint64_t inv = powmod(b.back(), q - 2, q);
        while (a.size() >= b.size() && !a.empty()) {
            uint64_t f = mulmod(a.back(), inv, q);
            size_t sh = a.size() - b.size();
            for (size_t i = 0; i < b.size(); ++i)
                a[sh + i] = (a[sh + i] + q - mulmod(f, b[i], q)) % q;
            trim(a);
        }
        std::swap(a, b);
    }
    return a.empty() ? -1 : (int)a.size() - 1;
}
static bool probably_not_squarefree(const std::vector<int64_t> &p) {
    const uint64_t primes[3] = {2305843009213693951ull, 1152921504606846883ull, 576460752303423433ull};
    for (uint64_t q : primes) {
        if (gcd_degree_mod(p, q) <= 0) return false;  // certified square-free mod q
    }
    return true;
}

// ======================================================================
// roots: FP64 Aberth-Ehrlich, then double-double Newton polish
// ======================================================================
using cplx = std::complex<double>;

// p(z)/p'(z) in FP64; for |z| > 1 through the reversed polynomial.
static cplx newton_ratio(const std::vector<double> &a, cplx z) {
    int d = (int)a.size() - 1;
    if (std::abs(z) <= 1.0) {
        cplx p = a[d], dp = 0;
        for (int i = d - 1; i >= 0; --i) {
            dp = dp * z + p;
            p = p * z + a[i];
        }
        return p / dp;
    }
    cplx y = 1.0 / z;
    cplx q = a[0], dq = 0;
    for (int i = 1; i <= d; ++i) {
        dq = dq * y + q;
        q = q * y + a[i];
    }
    return z * q / ((double)d * q - y * dq);
}

// Initial approximations on circles from the upper convex hull of
// (i, log|a_i|) (the Newton polygon), one circle per hull edge.
static std::vector<cplx> initial_points(const std::vector<double> &a) {
    int d = (int)a.size() - 1;
    std::vector<int> idx;
    std::vector<double> lg;
    for (int i = 0; i <= d; ++i)
        if (a[i] != 0) {
            idx.push_back(i);
            lg.push_back(std::log(std::fabs(a[i])));
        }
    std::vector<int> hull;  // indices into idx
    for (int k = 0; k < (int)idx.size(); ++k) {
        while (hull.size() >= 2) {
            int i1 = hull[hull.size() - 2], i2 = hull.back();
            double x1 = idx[i1], y1 = lg[i1], x2 = idx[i2], y2 = lg[i2], x3 = idx[k], y3 = lg[k];
            if ((x2 - x1) * (y3 - y1) - (y2 - y1) * (x3 - x1) >= 0) hull.pop_back();
            else break;
        }
        hull.push_back(k);
    }
    std::vector<cplx> z;
    const double two_pi = 6.283185307179586;
    for (size_t h = 0; h + 1 < hull.size(); ++h) {
        int k = idx[hull[h]], l = idx[hull[h + 1]];
        double u = std::exp((lg[hull[h]] - lg[hull[h + 1]]) / (l - k));
        for (int j = 0; j < l - k; ++j) {
            double ang = two_pi * j / (l - k) + two_pi * k / d + 0.4;
            z.push_back(std::polar(u, ang));
        }
    }
    return z;
}

static void aberth(const std::vector<double> &a, std::vector<cplx> &z, int maxit) {
    int d = (int)a.size() - 1;
    std::vector<char> done(d, 0);
    for (int it = 0; it < maxit; ++it) {
        int active = 0;
        for (int i = 0; i < d; ++i) {
            if (done[i]) continue;
            cplx N = newton_ratio(a, z[i]);
            cplx S = 0;
            for (int j = 0; j < d; ++j)
                if (j != i) S += 1.0 / (z[i] - z[j]);
            cplx wc = N / (1.0 - N * S);
            if (!std::isfinite(wc.real()) || !std::isfinite(wc.imag())) {
                done[i] = 1;
                continue;
            }
            z[i] -= wc;
            if (std::abs(wc) <= 1e-15 * std::max(std::abs(z[i]), 1e-300)) done[i] = 1;
            else ++active;
        }
        if (!active) break;
    }
}

// Newton data at z in complex double-double: the step p(z)/p'(z) and the
// inclusion radius d |p(z)| / |p'(z)| (a root lies within it), bounded with
// the rounding error of the evaluation.  For |z| > 1 the polynomial is
// evaluated reversed at y = 1/z (p(z) = z^d q(y), p'(z) = z^(d-1) (d q - y q'))
// so no intermediate overflows for large roots.
struct Newton {
    cdd step;
    double radius;
};
static const double kHornerU = 16.0 * 5.0e-32;  // > 16 * 2^-104 (complex dd mul-add)

static Newton newton_c(const std::vector<dd> &a, const cdd &z) {
    const int d = (int)a.size() - 1;
    const double az = cabs_d(z);
    Newton out;
    if (az <= 1.0) {
        cdd p{a[d], mkdd(0)}, dp{mkdd(0), mkdd(0)};
        double s = std::fabs(to_d(a[d])), ds = 0;
        for (int i = d - 1; i >= 0; --i) {
            dp = dp * z + p;
            p = p * z + cdd{a[i], mkdd(0)};
            ds = ds * az + s;
            s = s * az + std::fabs(to_d(a[i]));
        }
        const double ep = 2.0 * d * kHornerU * s, edp = 2.0 * d * kHornerU * ds;
        const double adp = cabs_d(dp) - edp;
        out.step = cabs_d(dp) > 0 ? p / dp : cdd{mkdd(0), mkdd(0)};
        out.radius = adp > 0 ? d * (cabs_d(p) + ep) / adp * (1 + 1e-12) : INFINITY;
        return out;
    }
    const cdd one{mkdd(1), mkdd(0)};
    const cdd y = one / z;
    const double ay = cabs_d(y);
    cdd q{a[0], mkdd(0)}, dq{mkdd(0), mkdd(0)};
    double s = std::fabs(to_d(a[0])), ds = 0;
    for (int i = 1; i <= d; ++i) {
        dq = dq * y + q;
        q = q * y + cdd{a[i], mkdd(0)};
        ds = ds * ay + s;
        s = s * ay + std::fabs(to_d(a[i]));
    }
    const double eq = 2.0 * d * kHornerU * s, edq = 2.0 * d * kHornerU * ds;
    const cdd den = cdd{q.re * (double)d, q.im * (double)d} - y * dq;
    const double aden = cabs_d(den) - d * eq - ay * edq;
    out.step = cabs_d(den) > 0 ? (z * q) / den : cdd{mkdd(0), mkdd(0)};
    out.radius = aden > 0 ? d * az * (cabs_d(q) + eq) / aden * (1 + 1e-12) : INFINITY;
    return out;
}

// The same on the real axis (real double-double arithmetic).
struct NewtonR {
    dd step;
    double radius;
};
static NewtonR newton_r(const std::vector<dd> &a, const dd &x) {
    const int d = (int)a.size() - 1;
    const double ax = std::fabs(to_d(x));
    const double u = 8.0 * 5.0e-32;
    NewtonR out;
    if (ax <= 1.0) {
        dd p = a[d], dp = mkdd(0);
        double s = std::fabs(to_d(a[d])), ds = 0;
        for (int i = d - 1; i >= 0; --i) {
            dp = dp * x + p;
            p = p * x + a[i];
            ds = ds * ax + s;
            s = s * ax + std::fabs(to_d(a[i]));
        }
        const double ep = 2.0 * d * u * s, edp = 2.0 * d * u * ds;
        const double adp = std::fabs(to_d(dp)) - edp;
        out.step = to_d(dp) != 0 ? p / dp : mkdd(0);
        out.radius = adp > 0 ? d * (std::fabs(to_d(p)) + ep) / adp * (1 + 1e-12) : INFINITY;
        return out;
    }
    const dd y = mkdd(1) / x;
    const double ay = std::fabs(to_d(y));
    dd q = a[0], dq = mkdd(0);
    double s = std::fabs(to_d(a[0])), ds = 0;
    for (int i = 1; i <= d; ++i) {
        dq = dq * y + q;
        q = q * y + a[i];
        ds = ds * ay + s;
        s = s * ay + std::fabs(to_d(a[i]));
    }
    const double eq = 2.0 * d * u * s, edq = 2.0 * d * u * ds;
    const dd den = q * (double)d - y * dq;
    const double aden = std::fabs(to_d(den)) - d * eq - ay * edq;
    out.step = to_d(den) != 0 ? (x * q) / den : mkdd(0);
    out.radius = aden > 0 ? d * ax * (std::fabs(to_d(q)) + eq) / aden * (1 + 1e-12) : INFINITY;
    return out;
}

static cdd polish_c(const std::vector<dd> &a, cdd z, int iters) {
    for (int k = 0; k < iters; ++k) {
        const Newton nw = newton_c(a, z);
        z = z - nw.step;
        if (cabs_d(nw.step) <= 1e-31 * std::max(cabs_d(z), 1e-300)) break;
    }
    return z;
}
static dd polish_r(const std::vector<dd> &a, dd x, int iters) {
    for (int k = 0; k < iters; ++k) {
        const NewtonR nw = newton_r(a, x);
        x = x - nw.step;
        if (std::fabs(to_d(nw.step)) <= 1e-31 * std::max(std::fabs(to_d(x)), 1e-300)) break;
    }
    return x;
}

struct Disc {
    cplx c;
    double r;
};
static bool discs_disjoint(const std::vector<Disc> &D) {
    for (auto &x : D)
        if (!std::isfinite(x.c.real()) || !std::isfinite(x.c.imag()) || !std::isfinite(x.r)) return false;
    // sort by real part and sweep
    std::vector<int> o(D.size());
    std::iota(o.begin(), o.end(), 0);
    std::sort(o.begin(), o.end(), [&](int i, int j) { return D[i].c.real() - D[i].r < D[j].c.real() - D[j].r; });
    double rmax = 0;
    for (auto &x : D) rmax = std::max(rmax, x.r);
    for (size_t ii = 0; ii < o.size(); ++ii) {
        const Disc &A = D[o[ii]];
        for (size_t jj = ii + 1; jj < o.size(); ++jj) {
            const Disc &B = D[o[jj]];
            if (B.c.real() - B.r > A.c.real() + A.r + 2 * rmax) break;
            // compare with a small relative margin for the FP64 distance
            double dist = std::abs(A.c - B.c);
            if (dist * (1 - 1e-12) <= A.r + B.r) return false;
        }
    }
    return true;
}

static void fail_roots(const Prepared &P, rfr_status &st, std::string &err, const char *why) {
    if (probably_not_squarefree(P.prim)) {
        st = RFR_ENOTSQFREE;
        err = "p has a repeated factor (gcd(p, p') non-trivial)";
    } else {
        st = RFR_EPRECISION;
        err = why;
    }
}

// ======================================================================
// elements, weights, window (Section 2, Section 3.3 Eq 18-19)
// ======================================================================

// floor(frac(v) * 2^64) mod 2^64 for a double-double v, |v| < 2^60.
static uint64_t weight_of(dd v) {
    // v - floor(v.hi) as an exact double-double: v.hi - fl is not exactly
    // representable when v.hi lies in (-0.5, 0), so it goes through two_sum
    const double fl = std::floor(v.hi);
    dd f = two_sum(v.hi, -fl);
    f = f + mkdd(v.lo);
    while (f.hi < 0) f = f + mkdd(1.0);
    while (f.hi >= 1.0) f = f - mkdd(1.0);
    // f in [0,1) as hi + lo; scale by 2^64 exactly
    double H = std::ldexp(f.hi, 64), L = std::ldexp(f.lo, 64);
    double h0 = std::floor(H);
    double rem = (H - h0) + L;
    double fr = std::floor(rem);
    uint64_t hi_int = h0 >= 18446744073709551616.0 ? 0 : (uint64_t)h0;
    return hi_int + (uint64_t)(int64_t)fr;
}

// Roots of P.prim on the host: FP64 Aberth from Newton-polygon starting
// points, complex double-double polish and inclusion radius of every root, and
// for a disc meeting the real axis the real polish and its radius.  The same
// records as the device root finder produces.
static void host_roots(const Prepared &P, std::vector<RootOut> &ro) {
    const int d = (int)P.prim.size() - 1;
    std::vector<double> ad(d + 1);
    std::vector<dd> add(d + 1);
    for (int i = 0; i <= d; ++i) {
        ad[i] = (double)P.prim[i];
        add[i] = dd_from_i64(P.prim[i]);
    }
    std::vector<cplx> z;
    if (d == 1) {
        z = {cplx(-ad[0] / ad[1], 0)};
    } else {
        z = initial_points(ad);
        aberth(ad, z, 400);
    }
    ro.assign(d, RootOut());
    for (int i = 0; i < d; ++i) {
        cdd c{mkdd(z[i].real()), mkdd(z[i].imag())};
        c = polish_c(add, c, 6);
        const double r = newton_c(add, c).radius;
        RootOut &o = ro[i];
        o.re_hi = c.re.hi;
        o.re_lo = c.re.lo;
        o.im_hi = c.im.hi;
        o.im_lo = c.im.lo;
        o.r = r;
        o.x_hi = o.x_lo = 0;
        o.rx = INFINITY;
        if (std::fabs(to_d(c.im)) <= r) {
            const dd x = polish_r(add, c.re, 6);
            o.x_hi = x.hi;
            o.x_lo = x.lo;
            o.rx = newton_r(add, x).radius;
        }
    }
}

// Weights (Section 3.3, Eq 18: w = floor(frac(a_d t) 2^64) with the elements
// of the monic transform) and the accept window of the elements in P.
static rfr_status weights_window(Prepared &P, std::string &err) {
    const int d = (int)P.prim.size() - 1;
    const dd a_d = dd_from_i64(P.prim[d]);
    const double abs_ad = std::fabs((double)P.prim[d]);
    double sum_delta = 0, sum_tau = 0;
    P.w.clear();
    for (int i = 0; i < P.n; ++i) {
        const dd tau = i < P.r ? a_d * P.reals[i] : a_d * (P.pairs[i - P.r].re * 2.0);
        P.w.push_back(weight_of(tau));
        sum_delta += abs_ad * (i < P.r ? 1.0 : 2.0) * P.rad[i];
        sum_tau += std::fabs(to_d(tau));
    }
    // Window (reading of Eq 19): a true k-element subset lands in (-k - E, E]
    // mod 2^64 with E >= 2^64 * sum |a_d| delta_i; add the dd rounding of a_d t_i
    // and one unit per weight for the floor of a rounded value.
    double Ed = std::ldexp(2.0 * sum_delta + sum_tau * std::ldexp(1.0, -100), 64);
    if (!(Ed < std::ldexp(1.0, 31))) {
        err = "accept window too wide (roots not precise enough)";
        return RFR_EPRECISION;
    }
    uint64_t E = (uint64_t)std::ceil(Ed) + 2 * (uint64_t)P.n + 2;
    // the search takes windows with t_lo + t_hi < 2^32 (a cell of its join is
    // at least that wide); a wider one means the roots are not precise enough
    if ((uint64_t)P.n + 2 * E >= (1ull << 32)) {
        err = "accept window too wide (roots not precise enough)";
        return RFR_EPRECISION;
    }
    P.t_lo = (uint64_t)P.n + E;
    P.t_hi = E;
    // Second trace of every element (Section 2: the power sums of a factor's
    // monic-transform roots are integers).  A real root u gives e = tau^2 with
    // tau = a_d u; a conjugate pair z gives e = 2 Re(s^2) with s = a_d z.  With
    // |tau - tau_true| <= |a_d| delta: |e - e_true| <= |a_d| delta (2|tau| +
    // |a_d| delta), twice that for a pair.  Weights and window follow the
    // first trace's rules; the search folds them in only when its candidates
    // overflow (a flood of patterns whose first trace is an integer).
    P.v2.clear();
    P.tr2_ok = true;
    double sum_err2 = 0, sum_e = 0;
    for (int i = 0; i < P.n && P.tr2_ok; ++i) {
        const double dl = abs_ad * P.rad[i];
        dd e;
        double mag;  // |tau| or |s|
        if (i < P.r) {
            const dd tau = a_d * P.reals[i];
            e = tau * tau;
            mag = std::fabs(to_d(tau));
            sum_err2 += dl * (2.0 * mag + dl);
        } else {
            const cdd &z = P.pairs[i - P.r];
            const dd sr = a_d * z.re, si = a_d * z.im;
            e = (sr * sr - si * si) * 2.0;
            mag = std::hypot(to_d(sr), to_d(si));
            sum_err2 += 2.0 * dl * (2.0 * mag + dl);
        }
        // rounding of e in double-double is relative to the squares it sums
        // (|s|^2 for a pair, whose two squares may cancel)
        const double sq = 2.0 * mag * mag;
        if (!(sq < std::ldexp(1.0, 52))) P.tr2_ok = false;  // frac(e) would carry too few bits
        sum_e += sq;
        P.v2.push_back(weight_of(e));
    }
    if (P.tr2_ok) {
        const double E2d = std::ldexp(2.0 * sum_err2 + sum_e * std::ldexp(1.0, -100), 64);
        if (!(E2d < std::ldexp(1.0, 31))) {
            P.tr2_ok = false;
        } else {
            const uint64_t E2 = (uint64_t)std::ceil(E2d) + 2 * (uint64_t)P.n + 2;
            P.t2_lo = (uint64_t)P.n + E2;
            P.t2_hi = E2;
        }
    }
    return RFR_OK;
}

rfr_status finish_elements(Prepared &P, const RootOut *ro, std::string &err) {
    const int d = (int)P.prim.size() - 1;
    P.reals.clear();
    P.pairs.clear();
    P.w.clear();
    P.rad.clear();
    std::vector<cdd> zc(d);
    std::vector<Disc> D(d);
    for (int i = 0; i < d; ++i) {
        zc[i] = cdd{dd{ro[i].re_hi, ro[i].re_lo}, dd{ro[i].im_hi, ro[i].im_lo}};
        D[i] = {cplx(to_d(zc[i].re), to_d(zc[i].im)), ro[i].r};
    }
    rfr_status st = RFR_OK;
    if (!discs_disjoint(D)) {
        fail_roots(P, st, err, "root inclusion discs overlap (roots not separated)");
        return st;
    }
    // classify: a disc meeting the real axis is re-centred on it and polished in R
    std::vector<dd> reals;
    std::vector<double> rr;
    std::vector<cdd> up, down;
    std::vector<double> rup, rdown;
    std::vector<Disc> F;
    for (int i = 0; i < d; ++i) {
        if (std::fabs(D[i].c.imag()) <= D[i].r) {
            const dd x{ro[i].x_hi, ro[i].x_lo};
            const double rx = ro[i].rx;
            reals.push_back(x);
            rr.push_back(rx);
            F.push_back({cplx(to_d(x), 0), rx});
        } else {
            (D[i].c.imag() > 0 ? up : down).push_back(zc[i]);
            (D[i].c.imag() > 0 ? rup : rdown).push_back(D[i].r);
            F.push_back(D[i]);
        }
    }
    // the final discs must again be disjoint: one root each, and a disc centred
    // on the real axis then holds a real root
    if (!discs_disjoint(F)) {
        fail_roots(P, st, err, "root inclusion discs overlap after real classification");
        return st;
    }
    if (up.size() != down.size()) {
        err = "conjugate pairing failed";
        return RFR_EPRECISION;
    }
    std::vector<double> rpair(up.size());
    std::vector<char> used(down.size(), 0);
    for (size_t i = 0; i < up.size(); ++i) {
        cplx cz(to_d(up[i].re), -to_d(up[i].im));
        int best = -1;
        for (size_t j = 0; j < down.size(); ++j) {
            if (used[j]) continue;
            cplx w(to_d(down[j].re), to_d(down[j].im));
            if (std::abs(cz - w) <= rup[i] + rdown[j]) {
                if (best >= 0) {
                    err = "ambiguous conjugate pairing";
                    return RFR_EPRECISION;
                }
                best = (int)j;
            }
        }
        if (best < 0) {
            err = "conjugate pairing failed";
            return RFR_EPRECISION;
        }
        used[best] = 1;
        rpair[i] = std::max(rup[i], rdown[best]);
    }
    // canonical order: reals ascending, pairs by (Re, Im)
    std::vector<int> orr(reals.size()), op(up.size());
    std::iota(orr.begin(), orr.end(), 0);
    std::iota(op.begin(), op.end(), 0);
    std::sort(orr.begin(), orr.end(), [&](int i, int j) {
        return reals[i].hi != reals[j].hi ? reals[i].hi < reals[j].hi : reals[i].lo < reals[j].lo;
    });
    std::sort(op.begin(), op.end(), [&](int i, int j) {
        double ri = to_d(up[i].re), rj = to_d(up[j].re);
        if (ri != rj) return ri < rj;
        return to_d(up[i].im) < to_d(up[j].im);
    });
    P.r = (int)reals.size();
    P.n = P.r + (int)up.size();
    if (P.n > RFR_MAX_ELEMENTS) {
        err = "too many elements";
        return RFR_EOVERFLOW;
    }
    for (int k : orr) {
        P.reals.push_back(reals[k]);
        P.rad.push_back(rr[k]);
    }
    for (int k : op) {
        P.pairs.push_back(up[k]);
        P.rad.push_back(rpair[k]);
    }
    return weights_window(P, err);
}

rfr_status prepare_elements(Prepared &P, std::string &err) {
    const int d = (int)P.prim.size() - 1;
    P.reals.clear();
    P.pairs.clear();
    P.w.clear();
    if (d < 1) {
        P.n = P.r = 0;
        return RFR_OK;
    }
    std::vector<RootOut> ro;
    host_roots(P, ro);
    return finish_elements(P, ro.data(), err);
}

rfr_status prepare(const int64_t *coeffs, int degree, Prepared &P, std::string &err) {
    rfr_status st = normalise(coeffs, degree, P, err);
    if (st != RFR_OK) return st;
    return prepare_elements(P, err);
}

// ======================================================================
// confirmation (Algorithm FACTOR: keep candidates q in Z[x]) and atoms
// ======================================================================
using i128 = __int128;

static bool round_dd(dd v, int64_t &out) {
    if (!(std::fabs(v.hi) < 4.0e18)) return false;
    double r = std::nearbyint(v.hi);
    double fr = (v.hi - r) + v.lo;
    double adj = std::nearbyint(fr);
    fr -= adj;
    if (std::fabs(fr) > 0.25) return false;
    out = (int64_t)r + (int64_t)adj;
    return true;
}

// Exact division p / f in Z[x] (f primitive); false if f does not divide p.
// Sets overflow if an intermediate leaves the int128 range.
static bool exact_div(const std::vector<int64_t> &p, const std::vector<int64_t> &f,
                      std::vector<int64_t> &q, bool &overflow) {
    int dp = (int)p.size() - 1, df = (int)f.size() - 1;
    overflow = false;
    if (df > dp) return false;
    std::vector<i128> rem(p.begin(), p.end());
    q.assign(dp - df + 1, 0);
    const i128 lf = f[df];
    const i128 lim = (i128)1 << 120;
    for (int k = dp - df; k >= 0; --k) {
        i128 lead = rem[k + df];
        if (lead % lf != 0) return false;
        i128 qk = lead / lf;
        if (qk > (i128)INT64_MAX || qk < -(i128)INT64_MAX) {
            overflow = true;
            return false;
        }
        q[k] = (int64_t)qk;
        if (qk == 0) continue;
        for (int i = 0; i <= df; ++i) {
            rem[k + i] -= qk * (i128)f[i];
            if (rem[k + i] > lim || rem[k + i] < -lim) {
                overflow = true;
                return false;
            }
        }
    }
    for (int i = 0; i < df; ++i)
        if (rem[i] != 0) return false;
    return true;
}

static void make_primitive(std::vector<int64_t> &f) {
    int64_t g = 0;
    for (auto c : f) g = gcd64(g, c);
    if (g == 0) return;
    if (f.back() < 0) g = -g;
    for (auto &c : f) c /= g;
}

static bool canon_less(const std::vector<int64_t> &a, const std::vector<int64_t> &b) {
    if (a.size() != b.size()) return a.size() < b.size();
    return a < b;
}

void trivial_factor(const Prepared &P, Factored &out) {
    out.content = P.content;
    out.factors.clear();
    if (P.xpow == 1) out.factors.push_back({0, 1});
    if (P.prim.size() > 1) out.factors.push_back(P.prim);
    for (auto &f : P.peeled) out.factors.push_back(f);
    std::sort(out.factors.begin(), out.factors.end(), canon_less);
}

// Is sum over the side of tau^k (k = 2, 3) an integer within tolerance?  These
// are traces of the monic-transform factor, integers for every true factor
// (Section 2: q in Z[x] iff all its traces are integers).
static bool traces_integral(const Prepared &P, const Pat &side) {
    const int d = (int)P.prim.size() - 1;
    dd a_d = dd_from_i64(P.prim[d]);
    dd t2 = mkdd(0), t3 = mkdd(0);
    for (int i = 0; i < P.n; ++i) {
        if (!side.get(i)) continue;
        if (i < P.r) {
            dd u = a_d * P.reals[i];
            dd u2 = u * u;
            t2 = t2 + u2;
            t3 = t3 + u2 * u;
        } else {
            const cdd &z = P.pairs[i - P.r];
            cdd s{a_d * z.re, a_d * z.im};
            cdd s2 = s * s;
            cdd s3 = s2 * s;
            t2 = t2 + s2.re * 2.0;
            t3 = t3 + s3.re * 2.0;
        }
    }
    auto near_int = [](dd v, double lim) {
        if (!(std::fabs(v.hi) < lim)) return true;  // too large to decide: do not filter
        double r = std::nearbyint(v.hi);
        double fr = (v.hi - r) + v.lo;
        fr -= std::nearbyint(fr);
        return std::fabs(fr) <= 1e-3;
    };
    return near_int(t2, 1e24) && near_int(t3, 1e21);
}

rfr_status confirm_and_factor(const Prepared &P, const std::vector<Pat> &cands, Factored &out,
                              std::string &err) {
    const int n = P.n;
    const int d = (int)P.prim.size() - 1;
    const Pat full = Pat::full(n);
    std::map<Pat, std::vector<int64_t>> found;
    out.n_candidates = cands.size();
    out.n_confirmed = 0;
    auto deg_of = [&](const Pat &s) {
        int e = 0;
        for (int i = 0; i < n; ++i)
            if (s.get(i)) e += i < P.r ? 1 : 2;
        return e;
    };
    const dd a_d = dd_from_i64(P.prim[d]);
    // a_d * prod over the side's roots (x - u) or (x^2 - 2 Re z x + |z|^2), in double-double
    auto side_poly = [&](const Pat &side) {
        std::vector<dd> q{a_d};
        for (int i = 0; i < n; ++i) {
            if (!side.get(i)) continue;
            std::vector<dd> nq(q.size() + (i < P.r ? 1 : 2), mkdd(0));
            if (i < P.r) {
                dd u = P.reals[i];
                for (size_t k = 0; k < q.size(); ++k) {
                    nq[k + 1] = nq[k + 1] + q[k];
                    nq[k] = nq[k] - q[k] * u;
                }
            } else {
                const cdd &z = P.pairs[i - P.r];
                dd t = z.re * 2.0;
                dd s2 = z.re * z.re + z.im * z.im;
                for (size_t k = 0; k < q.size(); ++k) {
                    nq[k + 2] = nq[k + 2] + q[k];
                    nq[k + 1] = nq[k + 1] - q[k] * t;
                    nq[k] = nq[k] + q[k] * s2;
                }
            }
            q.swap(nq);
        }
        return q;
    };
    for (const Pat &s0 : cands) {
        if (s0.empty()) continue;
        Pat comp = full & ~s0;
        if (found.count(s0)) continue;
        bool small_is_s = deg_of(s0) <= deg_of(comp);
        const Pat &side = small_is_s ? s0 : comp;
        if (!traces_integral(P, side)) continue;
        const std::vector<dd> q = side_poly(side);
        std::vector<int64_t> f(q.size());
        bool ok = true;
        for (size_t k = 0; k < q.size() && ok; ++k) ok = round_dd(q[k], f[k]);
        if (!ok) continue;
        make_primitive(f);
        if (f.back() <= 0) continue;
        std::vector<int64_t> g;
        bool ovf = false;
        if (!exact_div(P.prim, f, g, ovf)) {
            if (ovf) {
                // For a true factor f the quotient is the cofactor a_d/lc(f) *
                // prod over the other side, whose size the roots give.  If that
                // cofactor fits int64 with room to spare (and f times it cannot
                // reach the int128 limit of the division), a true division could
                // not have overflowed: the candidate is not a factor.  Otherwise
                // the factorisation may not be representable.
                const Pat &other = small_is_s ? comp : s0;
                const std::vector<dd> gq = side_poly(other);
                double gmax = 0, fmax = 0;
                const double scale = 1.0 / std::fabs((double)f.back());
                for (const dd &c : gq) gmax = std::max(gmax, std::fabs(to_d(c)) * scale);
                for (int64_t c : f) fmax = std::max(fmax, std::fabs((double)c));
                if (gmax < std::ldexp(1.0, 62) && fmax * gmax * (double)f.size() < std::ldexp(1.0, 118)) continue;
                err = "trial division overflowed int128";
                return RFR_EOVERFLOW;
            }
            continue;
        }
        if (g.back() <= 0) continue;
        ++out.n_confirmed;
        if (small_is_s) {
            found[s0] = f;
            found[comp] = g;
        } else {
            found[s0] = g;
            found[comp] = f;
        }
    }
    // atoms: the intersection of every divisor set that holds element i
    std::vector<Pat> sets;
    for (auto &kv : found) sets.push_back(kv.first);
    sets.push_back(full);
    std::vector<Pat> atoms;
    for (int i = 0; i < n; ++i) {
        Pat a = full;
        for (auto &t : sets)
            if (t.get(i)) a = a & t;
        if (std::find(atoms.begin(), atoms.end(), a) == atoms.end()) atoms.push_back(a);
    }
    out.content = P.content;
    out.factors.clear();
    if (P.xpow == 1) out.factors.push_back({0, 1});
    for (auto &a : atoms) {
        if (a == full) {
            out.factors.push_back(P.prim);
            continue;
        }
        auto it = found.find(a);
        if (it == found.end()) {
            err = "an atom of the divisors found has no confirmed factor";
            return RFR_EPRECISION;
        }
        out.factors.push_back(it->second);
    }
    for (auto &f : P.peeled) out.factors.push_back(f);
    std::sort(out.factors.begin(), out.factors.end(), canon_less);
    return RFR_OK;
}

// Does the root of the integer factor f (degree 1, or degree 2 with complex
// roots) lie in element i's inclusion disc?  Only then is f that element's
// factor (the discs are disjoint and hold one root each).
static bool root_in_disc(const Prepared &P, int i, const std::vector<int64_t> &f) {
    const double r = P.rad[i];
    if (i < P.r) {
        const dd g = dd_from_i64(f[1]), h = dd_from_i64(f[0]);
        const dd res = g * P.reals[i] + h;  // g (u - root)
        const double tol = std::fabs(to_d(g)) * r * (1 + 1e-9) +
                           std::ldexp(std::fabs(to_d(g * P.reals[i])) + std::fabs(to_d(h)), -96);
        return std::fabs(to_d(res)) <= tol;
    }
    if (f.size() != 3) return false;
    for (int64_t c : f)
        if (c > ((int64_t)1 << 60) || c < -((int64_t)1 << 60)) return false;  // keeps the discriminant in range
    const i128 disc = (i128)4 * f[2] * f[0] - (i128)f[1] * f[1];
    if (disc <= 0) return false;
    const dd two_g = dd_from_i64(f[2]) * 2.0;
    const dd re = -dd_from_i64(f[1]) / two_g;
    // sqrt of disc in double-double: one Newton step from the double root
    const double dd_hi = (double)disc;
    const dd dv = dd_from_i64((int64_t)(disc >> 62)) * std::ldexp(1.0, 62) + dd_from_i64((int64_t)(disc & (((i128)1 << 62) - 1)));
    double x0 = std::sqrt(dd_hi);
    dd x = mkdd(x0);
    x = x + (dv - x * x) / (x * 2.0);
    const dd im = x / two_g;
    const cdd &z = P.pairs[i - P.r];
    const double dre = to_d(re - z.re), dim = to_d(im - z.im);
    const double tol = r * (1 + 1e-9) + std::ldexp(std::fabs(to_d(z.re)) + std::fabs(to_d(z.im)), -96);
    return std::hypot(dre, dim) <= tol;
}

rfr_status peel_singletons(Prepared &P, std::string &err) {
    if (P.n < 2) return RFR_OK;
    std::vector<char> gone(P.n, 0);
    int npeeled = 0;
    for (int i = 0; i < P.n; ++i) {
        const int d = (int)P.prim.size() - 1;
        if (d < 2) break;  // what is left is irreducible
        const dd a_d = dd_from_i64(P.prim[d]);
        std::vector<dd> q;
        if (i < P.r) {
            q = {a_d * P.reals[i] * -1.0, a_d};
        } else {
            const cdd &z = P.pairs[i - P.r];
            const dd t = z.re * 2.0, s2 = z.re * z.re + z.im * z.im;
            q = {a_d * s2, a_d * t * -1.0, a_d};
        }
        std::vector<int64_t> f(q.size());
        bool ok = true;
        for (size_t k = 0; k < q.size() && ok; ++k) ok = round_dd(q[k], f[k]);
        if (!ok) continue;
        make_primitive(f);
        if (f.back() <= 0) continue;
        // f's root must lie in this element's disc (else the rounding hit an
        // integer by chance, or the root belongs to another element); only
        // then is the exact division tried (an overflow there means no factor)
        if (!root_in_disc(P, i, f)) continue;
        std::vector<int64_t> g;
        bool ovf = false;
        if (!exact_div(P.prim, f, g, ovf) || g.back() <= 0) continue;
        P.peeled.push_back(f);
        P.prim = g;
        gone[i] = 1;
        ++npeeled;
    }
    if (!npeeled) return RFR_OK;
    std::vector<dd> reals;
    std::vector<cdd> pairs;
    std::vector<double> rad;
    for (int i = 0; i < P.n; ++i) {
        if (gone[i]) continue;
        if (i < P.r) reals.push_back(P.reals[i]);
        else pairs.push_back(P.pairs[i - P.r]);
        rad.push_back(P.rad[i]);
    }
    P.reals.swap(reals);
    P.pairs.swap(pairs);
    P.rad.swap(rad);
    P.r = (int)P.reals.size();
    P.n = P.r + (int)P.pairs.size();
    if ((int)P.prim.size() - 1 != P.r + 2 * (int)P.pairs.size()) {
        err = "degree mismatch after splitting off single-element factors";
        return RFR_EPRECISION;
    }
    return weights_window(P, err);
}

}  // namespace rfr
