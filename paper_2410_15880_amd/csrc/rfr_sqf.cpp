// Square-free decomposition ahead of the search.  The method takes a
// square-free polynomial (Section 2); one that is not is split by Yun's
// algorithm into pairwise coprime square-free parts p = c * prod_m a_m^m, each
// part is factored by the square-free path, and every factor is listed m times.
//
// Integer polynomials are ascending int64 vectors.  The gcds are modular: the
// monic gcd modulo primes near 2^61 (primes dividing a leading coefficient are
// skipped, and only those giving the smallest degree are kept), lifted to Z by
// the Chinese remainder theorem over two primes after scaling by the gcd of
// the leading coefficients, and accepted only when the primitive candidate
// divides both inputs exactly.  Every step checks its range and reports
// RFR_EOVERFLOW rather than wrap.

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "rfr_ctx.h"

namespace rfr {
namespace {

using Poly = std::vector<int64_t>;
using i128 = __int128;
using u128 = unsigned __int128;

bool fits64(i128 v) { return v > (i128)INT64_MIN && v <= (i128)INT64_MAX; }

void trim(Poly &p) {
    while (p.size() > 1 && p.back() == 0) p.pop_back();
}

bool is_zero(const Poly &p) {
    for (int64_t c : p)
        if (c) return false;
    return true;
}

int deg(const Poly &p) { return is_zero(p) ? -1 : (int)p.size() - 1; }  // p trimmed

int64_t gcd_i64(int64_t a, int64_t b) {
    uint64_t x = a < 0 ? 0 - (uint64_t)a : (uint64_t)a, y = b < 0 ? 0 - (uint64_t)b : (uint64_t)b;
    while (y) {
        const uint64_t t = x % y;
        x = y;
        y = t;
    }
    return (int64_t)x;
}

// Primitive part with positive leading coefficient (p nonzero, trimmed).
void make_primitive(Poly &p) {
    int64_t g = 0;
    for (int64_t c : p) g = gcd_i64(g, c);
    if (p.back() < 0) g = -g;
    for (auto &c : p) c /= g;
}

bool derivative(const Poly &p, Poly &d) {
    d.assign(p.size() > 1 ? p.size() - 1 : 1, 0);
    for (size_t i = 1; i < p.size(); ++i) {
        const i128 v = (i128)p[i] * (i128)i;
        if (!fits64(v)) return false;
        d[i - 1] = (int64_t)v;
    }
    trim(d);
    return true;
}

bool subtract(const Poly &a, const Poly &b, Poly &r) {
    const size_t n = std::max(a.size(), b.size());
    r.assign(n, 0);
    for (size_t i = 0; i < n; ++i) {
        const i128 v = (i128)(i < a.size() ? a[i] : 0) - (i128)(i < b.size() ? b[i] : 0);
        if (!fits64(v)) return false;
        r[i] = (int64_t)v;
    }
    trim(r);
    return true;
}

// q = a / b if b (nonzero) divides a in Z[x]; false if it does not, or if a
// quotient coefficient or remainder leaves the checked range.
bool divexact(const Poly &a, const Poly &b, Poly &q) {
    const int da = deg(a), db = deg(b);
    if (db < 0) return false;
    if (da < 0) {
        q.assign(1, 0);
        return true;
    }
    if (da < db) return false;
    constexpr i128 LIM = (i128)1 << 125;
    std::vector<i128> rem(a.begin(), a.begin() + da + 1);
    q.assign(da - db + 1, 0);
    const i128 lb = b[db];
    for (int k = da - db; k >= 0; --k) {
        const i128 lead = rem[k + db];
        if (lead % lb) return false;
        const i128 qk = lead / lb;
        if (!fits64(qk)) return false;
        q[k] = (int64_t)qk;
        if (!qk) continue;
        for (int i = 0; i <= db; ++i) {
            const i128 v = rem[k + i] - qk * (i128)b[i];
            if (v > LIM || v < -LIM) return false;
            rem[k + i] = v;
        }
    }
    for (int i = 0; i < db; ++i)
        if (rem[i]) return false;
    trim(q);
    return true;
}

// ---------------------------------------------------------------- modular gcd
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod(r, a, m);
        a = mulmod(a, a, m);
        e >>= 1;
    }
    return r;
}

// Deterministic Miller-Rabin for 64-bit n (these bases suffice below 3.3e24).
bool is_prime(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t p : bases)
        if (n % p == 0) return n == p;
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) {
        d >>= 1;
        ++s;
    }
    for (uint64_t a : bases) {
        uint64_t x = powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s && comp; ++r) {
            x = mulmod(x, x, n);
            if (x == n - 1) comp = false;
        }
        if (comp) return false;
    }
    return true;
}

// The 16 largest primes below 2^61, found once.
const std::vector<uint64_t> &primes() {
    static const std::vector<uint64_t> P = [] {
        std::vector<uint64_t> v;
        for (uint64_t n = (1ull << 61) - 1; v.size() < 16; n -= 2)
            if (is_prime(n)) v.push_back(n);
        return v;
    }();
    return P;
}

uint64_t reduce(int64_t v, uint64_t m) {
    const int64_t r = v % (int64_t)m;
    return (uint64_t)(r < 0 ? r + (int64_t)m : r);
}

void trim_mod(std::vector<uint64_t> &v) {
    while (!v.empty() && v.back() == 0) v.pop_back();
}

// Monic gcd of f and g modulo the prime m (Euclid); both nonzero mod m.
std::vector<uint64_t> gcd_mod(const Poly &f, const Poly &g, uint64_t m) {
    std::vector<uint64_t> a(f.size()), b(g.size());
    for (size_t i = 0; i < f.size(); ++i) a[i] = reduce(f[i], m);
    for (size_t i = 0; i < g.size(); ++i) b[i] = reduce(g[i], m);
    trim_mod(a);
    trim_mod(b);
    while (!b.empty()) {
        const uint64_t inv = powmod(b.back(), m - 2, m);
        while (a.size() >= b.size()) {
            const uint64_t c = mulmod(a.back(), inv, m);
            const size_t sh = a.size() - b.size();
            for (size_t i = 0; i < b.size(); ++i) a[sh + i] = (a[sh + i] + m - mulmod(c, b[i], m)) % m;
            trim_mod(a);
            if (a.empty()) break;
        }
        std::swap(a, b);
    }
    const uint64_t inv = powmod(a.back(), m - 2, m);
    for (auto &c : a) c = mulmod(c, inv, m);
    return a;
}

i128 gcd_i128(i128 a, i128 b) {
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) {
        const i128 t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Lift from two primes: the residues of gamma * h (coefficients below
// m1 * m2 / 2 in absolute value) by the Chinese remainder theorem, then the
// primitive part.  False when the primitive part leaves int64.
bool lift2(const std::vector<uint64_t> &h1, uint64_t m1, const std::vector<uint64_t> &h2, uint64_t m2,
           Poly &out) {
    const uint64_t inv = powmod(m1 % m2, m2 - 2, m2);
    const u128 M = (u128)m1 * m2;
    std::vector<i128> v(h1.size());
    for (size_t i = 0; i < h1.size(); ++i) {
        const uint64_t t = mulmod((h2[i] + m2 - h1[i] % m2) % m2, inv, m2);
        const u128 x = (u128)h1[i] + (u128)m1 * t;
        v[i] = x > M / 2 ? (i128)x - (i128)M : (i128)x;
    }
    i128 g = 0;
    for (auto c : v) g = gcd_i128(g, c);
    if (g == 0) return false;
    if (v.back() < 0) g = -g;
    out.assign(v.size(), 0);
    for (size_t i = 0; i < v.size(); ++i) {
        const i128 c = v[i] / g;
        if (!fits64(c)) return false;
        out[i] = (int64_t)c;
    }
    return true;
}

// Primitive gcd (lc > 0) of two integer polynomials, not both zero.
bool gcd_z(const Poly &f, const Poly &g, Poly &out) {
    if (is_zero(g) || is_zero(f)) {
        out = is_zero(g) ? f : g;
        trim(out);
        make_primitive(out);
        return true;
    }
    const int64_t gam = gcd_i64(f.back(), g.back());
    int best = INT_MAX;
    std::vector<std::pair<uint64_t, std::vector<uint64_t>>> got;  // (prime, gamma * monic gcd)
    for (uint64_t m : primes()) {
        if (reduce(f.back(), m) == 0 || reduce(g.back(), m) == 0) continue;
        std::vector<uint64_t> h = gcd_mod(f, g, m);
        const int dh = (int)h.size() - 1;
        if (dh == 0) {  // coprime mod m with both degrees kept: coprime over Q
            out.assign(1, 1);
            return true;
        }
        if (dh > best) continue;  // an unlucky prime
        if (dh < best) {
            best = dh;
            got.clear();
        }
        const uint64_t gm = reduce(gam, m);
        for (auto &c : h) c = mulmod(c, gm, m);
        got.emplace_back(m, std::move(h));
        if (got.size() < 2) continue;
        const auto &A = got[got.size() - 2];
        const auto &B = got.back();
        Poly cand, q1, q2;
        if (lift2(A.second, A.first, B.second, B.first, cand) && divexact(f, cand, q1) && divexact(g, cand, q2)) {
            out = cand;
            return true;
        }
    }
    return false;
}

// Yun's algorithm on f (primitive, lc > 0, f(0) != 0, degree >= 1):
// a0 = gcd(f, f'), b = f / a0, c = f' / a0, d = c - b'; then a = gcd(b, d) is
// the part of the next multiplicity, b <- b / a, c <- d / a, d <- c - b',
// until b is constant.  With primitive associates every quotient is exact in
// Z[x] (Gauss's lemma) and b, c, d keep a common scale, so the parts are those
// of the rational algorithm.  parts[m - 1] is the part of multiplicity m
// (constant 1 when there is none).
bool yun(const Poly &f, std::vector<Poly> &parts) {
    Poly fd, a0, b, c, d, bd;
    if (!derivative(f, fd) || !gcd_z(f, fd, a0)) return false;
    if (!divexact(f, a0, b) || !divexact(fd, a0, c) || !derivative(b, bd) || !subtract(c, bd, d)) return false;
    while (deg(b) > 0) {
        Poly a;
        if (is_zero(d)) {
            a = b;
            make_primitive(a);
        } else if (!gcd_z(b, d, a)) {
            return false;
        }
        parts.push_back(a);
        Poly b2, c2;
        if (!divexact(b, a, b2)) return false;
        if (is_zero(d)) c2.assign(1, 0);
        else if (!divexact(d, a, c2)) return false;
        b = b2;
        if (!derivative(b, bd) || !subtract(c2, bd, d)) return false;
    }
    return true;
}

}  // namespace

rfr_status squarefree_decompose(const int64_t *coeffs, int degree, int64_t &content,
                                std::vector<std::pair<std::vector<int64_t>, int>> &parts, std::string &err) {
    parts.clear();
    if (!coeffs || degree < 1 || degree > RFR_MAX_DEGREE || coeffs[degree] == 0) {
        err = "degree must be in [1, RFR_MAX_DEGREE] with a nonzero leading coefficient";
        return RFR_EINVAL;
    }
    for (int i = 0; i <= degree; ++i)
        if (coeffs[i] == INT64_MIN) {
            err = "coefficient INT64_MIN is not supported";
            return RFR_EOVERFLOW;
        }
    int k = 0;
    while (coeffs[k] == 0) ++k;
    Poly f(coeffs + k, coeffs + degree + 1);
    int64_t g = 0;
    for (int64_t c : f) g = gcd_i64(g, c);
    if (f.back() < 0) g = -g;
    for (auto &c : f) c /= g;
    content = g;
    std::vector<Poly> bym;
    if (f.size() > 1 && !yun(f, bym)) {
        err = "square-free decomposition leaves the int64 range";
        return RFR_EOVERFLOW;
    }
    for (size_t m = 0; m < bym.size(); ++m)
        if (bym[m].size() > 1) parts.emplace_back(bym[m], (int)m + 1);
    if (k) parts.emplace_back(Poly{0, 1}, k);
    std::sort(parts.begin(), parts.end(), [](const auto &x, const auto &y) {
        if (x.second != y.second) return x.second < y.second;
        if (x.first.size() != y.first.size()) return x.first.size() < y.first.size();
        return x.first < y.first;
    });
    return RFR_OK;
}

rfr_status factor_sqf_route(const int64_t *coeffs, int degree, const FactorOne &one, rfr_result **out) {
    *out = nullptr;
    const double t0 = now_ms();
    int64_t content = 0;
    std::vector<std::pair<Poly, int>> parts;
    std::string err;
    rfr_status st = squarefree_decompose(coeffs, degree, content, parts, err);
    if (st != RFR_OK) return fail(st, err);
    if (parts.size() == 1 && parts[0].second == 1)  // square-free after all: the roots were not separable
        return fail(RFR_EPRECISION, "roots not separated although p is square-free");
    Prepared P;
    Factored F;
    F.content = content;
    double ms_roots = now_ms() - t0, ms_search = 0, ms_confirm = 0;
    int nmax = -1;
    for (const auto &pm : parts) {
        const Poly &a = pm.first;
        if (a.size() == 2 && a[0] == 0 && a[1] == 1) {
            for (int m = 0; m < pm.second; ++m) F.factors.push_back(a);
            continue;
        }
        rfr_result *r = nullptr;
        st = one(a.data(), (int)a.size() - 1, &r);
        if (st != RFR_OK) return st == RFR_ENOTSQFREE ? fail(RFR_EPRECISION, "square-free part rejected") : st;
        if (r->content != 1) {
            rfr_result_free(r);
            return fail(RFR_EPRECISION, "square-free part is not primitive");
        }
        size_t off = 0;
        for (int j = 0; j < r->nfactors; ++j) {
            Poly q(r->coeffs + off, r->coeffs + off + r->degrees[j] + 1);
            off += (size_t)r->degrees[j] + 1;
            for (int m = 0; m < pm.second; ++m) F.factors.push_back(q);
        }
        P.n += r->n_elements;
        P.r += r->n_real;
        F.n_candidates += r->n_candidates;
        F.n_confirmed += r->n_confirmed;
        F.trace_folded |= r->trace_folded;
        if (r->n_elements > nmax) {
            nmax = r->n_elements;
            P.t_lo = r->t_lo;
            P.t_hi = r->t_hi;
        }
        ms_roots += r->ms_roots;
        ms_search += r->ms_search;
        ms_confirm += r->ms_confirm;
        rfr_result_free(r);
    }
    std::sort(F.factors.begin(), F.factors.end(), [](const Poly &x, const Poly &y) {
        if (x.size() != y.size()) return x.size() < y.size();
        return x < y;
    });
    rfr_result *r = pack_result(P, F);
    if (!r) return fail(RFR_ENOMEM, "result allocation failed");
    r->ms_roots = ms_roots;
    r->ms_search = ms_search;
    r->ms_confirm = ms_confirm;
    *out = r;
    return RFR_OK;
}

}  // namespace rfr

using namespace rfr;

extern "C" rfr_status rfr_squarefree(const int64_t *coeffs, int degree, int64_t *content, int64_t *parts_out,
                                     int32_t *degrees_out, int32_t *mult_out, int *nparts) {
    if (!content || !parts_out || !degrees_out || !mult_out || !nparts) return fail(RFR_EINVAL, "NULL output");
    int64_t c = 0;
    std::vector<std::pair<Poly, int>> parts;
    std::string err;
    rfr_status st = squarefree_decompose(coeffs, degree, c, parts, err);
    if (st != RFR_OK) return fail(st, err);
    *content = c;
    *nparts = (int)parts.size();
    size_t off = 0;
    for (size_t j = 0; j < parts.size(); ++j) {
        degrees_out[j] = (int32_t)parts[j].first.size() - 1;
        mult_out[j] = parts[j].second;
        std::memcpy(parts_out + off, parts[j].first.data(), parts[j].first.size() * sizeof(int64_t));
        off += parts[j].first.size();
    }
    return RFR_OK;
}
