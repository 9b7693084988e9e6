"""Reference (oracle) implementation of Real-Factors-Recombination factorisation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this module; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It is deliberately plain and slow: exact Python integers,
numpy for bulk subset sums and sorting, mpmath for high-precision roots.

What it computes (paper sections in brackets):

* ``normalise``      content, sign and powers of x split off [Section 2: the
                     method assumes a square-free input; a non-monic input is
                     handled through its monic transform].
* ``elements``       real roots u_i and conjugate-pair representatives z_j
                     (Eq 1), giving the element values t = u_i or z_j + conj(z_j)
                     (the set R of Section 2).
* ``weights``        rho_i = frac(a_d * t_i) quantised to M = 2**64 as
                     floor(rho_i * M) (Section 3.3, Eq 18); a_d * t_i are the
                     element values of the monic transform a_d**(d-1) p(x/a_d).
* ``window``         integer accept window replacing Eq 19 (see the readings
                     below).
* ``search_brute``   Algorithm A (Section 3.1): every pattern s < 2**(n-1).
* ``search_hs``      Algorithm C (Section 3.3): EXPAND both halves, sort, and
                     find every pair whose sum lies in the window (FIND that
                     reports all pairs).
* ``second_trace``   the second power sum of a candidate's monic-transform
                     roots (Section 2: every power sum of a true factor is an
                     integer), as weights and a window like the first; the
                     candidates failing it are dropped before confirmation.
* ``confirm``        FACTOR's test that the candidate q lies in Z[x]
                     (Section 2, Algorithm FACTOR), done by rounding
                     a_d * q and exact trial division.
* ``factor``         FACTOR end to end, returning the irreducible
                     factorisation (the atoms of all divisors found).
* ``squarefree``     Yun's square-free decomposition [Section 2: a
                     polynomial that is not square-free is split into
                     square-free parts first], and ``factor_general``: FACTOR
                     on each part, factors repeated by multiplicity.

Readings of the paper taken here (each also stated where it is used):

* M = 2**64 and wrapping uint64 sums (Section 3.3 leaves M free, M > 1/eps).
* Eq 19 accepts only {0, M-1}; flooring each weight biases a k-element sum
  into (-k, 0], and root error adds +-E, so the window is [-(n+E), +E].
* Non-monic inputs use the roots of the monic transform, a_d * root.
* The last element is left out of the search (complement symmetry, Section
  3.1), also for Algorithm C.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, List, Optional, Sequence, Tuple

import mpmath
import numpy as np

MOD = 1 << 64
MASK = MOD - 1
PREC_BITS = 400          # working precision of roots and reconstruction


class OracleError(RuntimeError):
    pass


# --------------------------------------------------------------------------
# exact polynomial helpers (ascending coefficient lists of Python ints)
# --------------------------------------------------------------------------

def _trim(p: List[int]) -> List[int]:
    p = list(p)
    while len(p) > 1 and p[-1] == 0:
        p.pop()
    return p


def content(p: Sequence[int]) -> int:
    g = 0
    for c in p:
        g = math.gcd(g, int(c))
    return g


def primitive(p: Sequence[int]) -> List[int]:
    """Primitive part with positive leading coefficient."""
    p = _trim([int(c) for c in p])
    g = content(p)
    if g == 0:
        raise OracleError("zero polynomial")
    if p[-1] < 0:
        g = -g
    return [c // g for c in p]


def exact_divide(p: Sequence[int], f: Sequence[int]) -> Optional[List[int]]:
    """Quotient p / f if f divides p in Z[x], else None (f primitive)."""
    p = [int(c) for c in p]
    f = [int(c) for c in f]
    df, dp = len(f) - 1, len(p) - 1
    if df > dp:
        return None
    rem = list(p)
    q = [0] * (dp - df + 1)
    lf = f[-1]
    for k in range(dp - df, -1, -1):
        lead = rem[k + df]
        if lead % lf:
            return None
        qk = lead // lf
        q[k] = qk
        if qk:
            for i in range(df + 1):
                rem[k + i] -= qk * f[i]
    if any(rem[:df]):
        return None
    return q


def poly_mul_exact(f: Sequence[int], g: Sequence[int]) -> List[int]:
    out = [0] * (len(f) + len(g) - 1)
    for i, a in enumerate(f):
        for j, b in enumerate(g):
            out[i + j] += int(a) * int(b)
    return out


def normalise(coeffs: Sequence[int]) -> Tuple[int, int, List[int]]:
    """Split p = cont * x**k * prim with prim primitive, lc(prim) > 0, prim(0) != 0.

    Section 2 takes a square-free, monic input; this removes the integer
    content, the sign and the powers of x before the roots are taken.
    """
    p = _trim([int(c) for c in coeffs])
    if len(p) < 2:
        raise OracleError("degree must be at least 1")
    k = 0
    while p[k] == 0:
        k += 1
    core = p[k:]
    g = content(core)
    if core[-1] < 0:
        g = -g
    prim = [c // g for c in core]
    return g, k, prim


def is_squarefree(prim: Sequence[int]) -> bool:
    """gcd(p, p') == 1 over Q (sympy's polynomial gcd used as a library step)."""
    import sympy
    x = sympy.Symbol("x")
    P = sympy.Poly(list(reversed([int(c) for c in prim])), x)
    return sympy.degree(sympy.gcd(P, P.diff(x)), x) == 0


# --------------------------------------------------------------------------
# roots and elements (Eq 1, the set R of Section 2)
# --------------------------------------------------------------------------

def _horner(cs_mp, x):
    """p(x) and p'(x) for ascending mp coefficients."""
    pv = cs_mp[-1]
    dv = mpmath.mpf(0)
    for c in reversed(cs_mp[:-1]):
        dv = dv * x + pv
        pv = pv * x + c
    return pv, dv


def _abs_bound(cs_mp, ax):
    s = mpmath.mpf(0)
    for c in reversed(cs_mp):
        s = s * ax + abs(c)
    return s


def _newton_polish(cs_mp, x, real: bool, prec: int, maxit: int = 200):
    tol = mpmath.mpf(2) ** (-prec + 24)
    for _ in range(maxit):
        pv, dv = _horner(cs_mp, x)
        if dv == 0:
            break
        step = pv / dv
        if real:
            step = mpmath.re(step)
        x = x - step
        if abs(step) <= tol * max(1, abs(x)):
            break
    return x


def _radius(cs_mp, x, prec: int):
    """Inclusion radius d*|p(x)|/|p'(x)| (a root lies within it), with a
    margin for the rounding of the evaluation at ``prec`` bits."""
    d = len(cs_mp) - 1
    pv, dv = _horner(cs_mp, x)
    err = _abs_bound(cs_mp, abs(x)) * mpmath.mpf(2) ** (-prec + 16)
    if abs(dv) <= err:
        return mpmath.inf
    return d * (abs(pv) + err) / (abs(dv) - err)


def roots_hp(prim: Sequence[int], prec: int = PREC_BITS):
    """All roots of prim at high precision, classified real / conjugate pairs.

    Starting values come from numpy.roots (companion-matrix eigenvalues); each
    is polished by Newton's method at ``prec`` bits.  The polished set is
    accepted only if the inclusion discs are pairwise disjoint (so each holds
    exactly one root); otherwise mpmath.polyroots is used instead.

    Returns (reals, pairs, radii_real, radii_pair) with reals ascending and
    pairs (Im > 0) sorted by (Re, Im).
    """
    d = len(prim) - 1
    with mpmath.workprec(prec):
        cs = [mpmath.mpf(int(c)) for c in prim]
        start = np.roots(np.array([float(c) for c in reversed(prim)], dtype=np.float64))
        approx = [_newton_polish(cs, mpmath.mpc(complex(z)), False, prec) for z in start]
        res = _classify(cs, approx, prec)
        if res is None:
            approx = mpmath.polyroots([mpmath.mpf(int(c)) for c in reversed(prim)],
                                      maxsteps=400, extraprec=2 * prec)
            approx = [_newton_polish(cs, mpmath.mpc(z), False, prec) for z in approx]
            res = _classify(cs, approx, prec)
        if res is None:
            raise OracleError("could not separate the roots")
        return res


def _classify(cs, approx, prec):
    d = len(cs) - 1
    if len(approx) != d:
        return None
    rad = [_radius(cs, z, prec) for z in approx]
    # disjointness: d discs, each holding at least one root
    for i in range(d):
        for j in range(i + 1, d):
            if abs(approx[i] - approx[j]) <= rad[i] + rad[j]:
                return None
    reals, rr, cplx, rc = [], [], [], []
    centers, radii = [], []
    for z, r in zip(approx, rad):
        if abs(mpmath.im(z)) <= r:
            # the disc meets the real axis: re-centre on it and polish in R
            x = _newton_polish(cs, mpmath.mpf(mpmath.re(z)), True, prec)
            rx = _radius(cs, x, prec)
            reals.append(mpmath.mpf(x))
            rr.append(rx)
            centers.append(mpmath.mpc(x))
            radii.append(rx)
        else:
            cplx.append(z)
            rc.append(r)
            centers.append(z)
            radii.append(r)
    # the final discs must again be pairwise disjoint: then each holds exactly
    # one root, a disc centred on the real axis holds a real root (its
    # conjugate lies in the same disc) and a disc missing the axis a non-real one
    for i in range(d):
        for j in range(i + 1, d):
            if abs(centers[i] - centers[j]) <= radii[i] + radii[j]:
                return None
    # pair each Im>0 root with its conjugate
    ups = [(z, r) for z, r in zip(cplx, rc) if mpmath.im(z) > 0]
    downs = [(z, r) for z, r in zip(cplx, rc) if mpmath.im(z) < 0]
    if len(ups) != len(downs):
        return None
    used = [False] * len(downs)
    pairs, rp = [], []
    for z, r in ups:
        best = None
        for k, (w, rw) in enumerate(downs):
            if not used[k] and abs(mpmath.conj(z) - w) <= r + rw:
                if best is not None:
                    return None
                best = k
        if best is None:
            return None
        used[best] = True
        pairs.append(z)
        rp.append(max(r, downs[best][1]))
    order_r = sorted(range(len(reals)), key=lambda i: reals[i])
    order_p = sorted(range(len(pairs)), key=lambda i: (mpmath.re(pairs[i]), mpmath.im(pairs[i])))
    return ([reals[i] for i in order_r], [pairs[i] for i in order_p],
            [rr[i] for i in order_r], [rp[i] for i in order_p])


def elements(prim: Sequence[int], prec: int = PREC_BITS):
    """Element values t_i (reals first, then z_j + conj z_j) and their root groups.

    Returns (ts, groups, deltas) where groups[i] is ('r', u) or ('c', z) and
    deltas[i] bounds |t_i(computed) - t_i(true)|.
    """
    reals, pairs, rr, rp = roots_hp(prim, prec)
    ts, groups, deltas = [], [], []
    with mpmath.workprec(prec):
        for u, r in zip(reals, rr):
            ts.append(mpmath.mpf(u))
            groups.append(("r", u))
            deltas.append(r)
        for z, r in zip(pairs, rp):
            ts.append(2 * mpmath.re(z))
            groups.append(("c", z))
            deltas.append(2 * r)
    return ts, groups, deltas


# --------------------------------------------------------------------------
# weights and window (Section 3.3, Eq 18-19)
# --------------------------------------------------------------------------

def _ratio(x):
    """Exact (numerator, denominator) of a binary mpf."""
    s, m, e, _bc = x._mpf_
    v = int(m)
    if s:
        v = -v
    if e >= 0:
        return v << e, 1
    return v, 1 << (-e)


def weight_of(a_d: int, t) -> int:
    """w = floor(frac(a_d * t) * 2**64), computed exactly from the binary value t."""
    num, den = _ratio(mpmath.mpf(t))
    # a_d * t * 2^64 = a_d * num * 2^64 / den ; floor then reduce mod 2^64
    return ((a_d * num) << 64) // den & MASK


def weights(prim: Sequence[int], ts) -> List[int]:
    a_d = int(prim[-1])
    with mpmath.workprec(PREC_BITS):
        return [weight_of(a_d, t) for t in ts]


def window(prim: Sequence[int], deltas, safety: int = 4) -> Tuple[int, int]:
    """(T_lo, T_hi) with accept(y) = y in [2**64 - T_lo, 2**64) U [0, T_hi].

    Reading of Eq 19: with floor quantisation a true k-element subset lands in
    (-k - E, E] mod 2**64, where E bounds 2**64 * |a_d| * sum(delta_i).
    """
    n = len(deltas)
    a_d = abs(int(prim[-1]))
    with mpmath.workprec(PREC_BITS):
        tot = mpmath.fsum(deltas) * a_d * safety * mpmath.mpf(MOD)
        E = int(mpmath.ceil(tot)) + 1
    return n + E, E


# --------------------------------------------------------------------------
# searches: Algorithm A (brute force) and Algorithm C (Horowitz-Sahni)
# --------------------------------------------------------------------------

def in_window(y: int, t_lo: int, t_hi: int) -> bool:
    y &= MASK
    return y <= t_hi or y >= MOD - t_lo


def subset_sums(ws: Sequence[int], negate: bool = False) -> np.ndarray:
    """All 2**m subset sums mod 2**64; entry j is the sum over the set bits of j."""
    out = np.zeros(1, dtype=np.uint64)
    for w in ws:
        w = int(w) & MASK
        if negate:
            w = (-w) & MASK
        out = np.concatenate([out, out + np.uint64(w)])
    return out


def _accept_mask(sums: np.ndarray, t_lo: int, t_hi: int) -> np.ndarray:
    m = sums <= np.uint64(t_hi)
    if t_lo > 0:
        m |= sums >= np.uint64(MOD - t_lo)
    return m


def search_brute(w: Sequence[int], t_lo: int, t_hi: int) -> List[int]:
    """Algorithm A over the first n-1 elements: every s in [1, 2**(n-1))."""
    n1 = len(w) - 1
    if n1 <= 0:
        return []
    sums = subset_sums(w[:n1])
    idx = np.nonzero(_accept_mask(sums, t_lo, t_hi))[0]
    return [int(s) for s in idx if s != 0]


def expand(ws: Sequence[int], negate: bool = False) -> np.ndarray:
    """EXPAND (Section 3.3): all subset sums of one half, sorted ascending."""
    return np.sort(subset_sums(ws, negate))


def search_hs(w: Sequence[int], t_lo: int, t_hi: int, chunk: int = 1 << 24) -> List[int]:
    """Algorithm C over the first n-1 elements, reporting every pair in the window.

    Split n' = n-1 into n_a = ceil(n'/2) and n_b = floor(n'/2).  alpha holds the
    sums of half A sorted (the pattern kept alongside), and beta' = -beta the
    negated sums of half B, also sorted.  A pair (i, j) is accepted when
    alpha_i + beta_j lies in the window, i.e. alpha_i lies in
    [beta'_j - T_lo, beta'_j + T_hi] mod 2**64: one contiguous range of sorted
    alpha, or two when the range wraps past 0.  Every pair is reported.
    """
    n1 = len(w) - 1
    if n1 <= 0:
        return []
    na = (n1 + 1) // 2
    alpha = subset_sums(w[:na])
    perm = np.argsort(alpha, kind="stable")
    a_sorted = alpha[perm]
    del alpha
    negb = subset_sums(w[na:n1], negate=True)
    permb = np.argsort(negb, kind="stable")
    b_sorted = negb[permb]
    del negb
    NA = a_sorted.shape[0]
    out = []
    for j0 in range(0, b_sorted.shape[0], chunk):
        nb_ = b_sorted[j0:j0 + chunk]
        lo = nb_ - np.uint64(t_lo)
        hi = nb_ + np.uint64(t_hi)
        wrap = lo > hi
        left = np.searchsorted(a_sorted, lo, side="left").astype(np.int64)
        right = np.searchsorted(a_sorted, hi, side="right").astype(np.int64)
        cnt = np.where(wrap, 0, right - left)
        cnt_w1 = np.where(wrap, NA - left, 0)
        cnt_w2 = np.where(wrap, right, 0)
        js = permb[j0:j0 + nb_.shape[0]].astype(np.int64)
        for starts, counts in ((left, cnt), (left, cnt_w1), (np.zeros_like(right), cnt_w2)):
            tot = int(counts.sum())
            if tot == 0:
                continue
            rep_j = np.repeat(js, counts)
            rep_s = np.repeat(starts, counts)
            offs = np.arange(tot, dtype=np.int64) - np.repeat(np.cumsum(counts) - counts, counts)
            pa = perm[rep_s + offs]
            for a, bj in zip(pa.tolist(), rep_j.tolist()):
                s = int(a) | (int(bj) << na)
                if s != 0:
                    out.append(s)
    return sorted(out)


def search(w: Sequence[int], t_lo: int, t_hi: int, brute_max: int = 22) -> List[int]:
    if len(w) - 1 <= brute_max:
        return search_brute(w, t_lo, t_hi)
    return search_hs(w, t_lo, t_hi)


# --------------------------------------------------------------------------
# second trace (Section 2: a factor q of the monic transform has integer power
# sums of its roots; the search tests the first, here the second)
# --------------------------------------------------------------------------

def second_trace(prim: Sequence[int], groups, deltas, safety: int = 4):
    """Per-element weights of the second trace and their window.

    Element i contributes e_i = (a_d u)**2 for a real root u and
    (a_d z)**2 + (a_d conj z)**2 = 2 Re((a_d z)**2) for a pair z; its weight is
    floor(frac(e_i) * 2**64), computed exactly from the binary value of e_i.
    The window has the first trace's form [-(n + E2), +E2] with E2 bounding
    2**64 times the sum of |e_i - e_i(true)| <= |a_d| r (2 |a_d root| + |a_d| r)
    (twice that for a pair), r the root's inclusion radius.
    """
    a_d = int(prim[-1])
    n = len(groups)
    vs = []
    with mpmath.workprec(PREC_BITS):
        err = mpmath.mpf(0)
        for (kind, z), dl in zip(groups, deltas):
            if kind == "r":
                x = a_d * z
                e = x * x
                r = abs(a_d) * dl
                err += r * (2 * abs(x) + r)
            else:
                x = a_d * z
                e = 2 * mpmath.re(x * x)
                r = abs(a_d) * dl / 2          # deltas hold 2r for a pair (the bound on 2 Re z)
                err += 2 * r * (2 * abs(x) + r)
            vs.append(weight_of(1, e))
        E2 = int(mpmath.ceil(err * safety * MOD)) + 1
    return vs, (n + E2, E2)


def second_trace_filter(cands: Sequence[int], v: Sequence[int], t2: Tuple[int, int]) -> List[int]:
    """The candidates whose second trace lies in its window (sums mod 2**64)."""
    if not cands:
        return []
    nbits = max(int(c).bit_length() for c in cands)
    if nbits <= 64:
        cs = np.array([int(c) for c in cands], dtype=np.uint64)
        tot = np.zeros(len(cs), dtype=np.uint64)
        for i in range(nbits):
            m = ((cs >> np.uint64(i)) & np.uint64(1)).astype(bool)
            tot[m] += np.uint64(v[i])
        keep = _accept_mask(tot, t2[0], t2[1])
        return [int(c) for c, k in zip(cands, keep) if k]
    return [c for c in cands if in_window(sum(v[i] for i in range(nbits) if (c >> i) & 1), t2[0], t2[1])]


# --------------------------------------------------------------------------
# confirmation (Algorithm FACTOR, the test q in Z[x]) and atoms
# --------------------------------------------------------------------------

def _side_poly(a_d: int, groups, members: Sequence[int]):
    """a_d * prod over members of (x - u) or (x^2 - 2Re(z) x + |z|^2), at PREC_BITS."""
    with mpmath.workprec(PREC_BITS):
        q = [mpmath.mpf(a_d)]
        for i in members:
            kind, r = groups[i]
            if kind == "r":
                fac = [-r, mpmath.mpf(1)]
            else:
                fac = [mpmath.re(r) ** 2 + mpmath.im(r) ** 2, -2 * mpmath.re(r), mpmath.mpf(1)]
            nq = [mpmath.mpf(0)] * (len(q) + len(fac) - 1)
            for a, ca in enumerate(q):
                for b, cb in enumerate(fac):
                    nq[a + b] += ca * cb
            q = nq
        ints = []
        for c in q:
            k = int(mpmath.nint(c))
            if abs(c - k) > mpmath.mpf(1) / 4:
                return None
            ints.append(k)
        return ints


def confirm(prim: Sequence[int], groups, s: int, n: int):
    """Return (f, g) with prim = f * g, f the integer factor for pattern s, or None.

    The side (s or its complement) with fewer roots is rebuilt as a_d * q(x),
    rounded, made primitive, and tried by exact division.
    """
    full = (1 << n) - 1
    comp = full & ~s
    deg = lambda m: sum(1 if groups[i][0] == "r" else 2 for i in range(n) if (m >> i) & 1)
    side, other = (s, comp) if deg(s) <= deg(comp) else (comp, s)
    a_d = int(prim[-1])
    ints = _side_poly(a_d, groups, [i for i in range(n) if (side >> i) & 1])
    if ints is None or content(ints) == 0:
        return None
    f = primitive(ints)
    q = exact_divide(prim, f)
    if q is None:
        return None
    g = primitive(q)
    if q[-1] < 0:
        return None
    return (f, g) if side == s else (g, f)


def atoms(n: int, confirmed: Dict[int, List[int]]) -> List[int]:
    """Atoms of the divisor sets found: the AND of every found set holding element i."""
    full = (1 << n) - 1
    sets = list(confirmed.keys()) + [full]
    out = set()
    for i in range(n):
        a = full
        for t in sets:
            if (t >> i) & 1:
                a &= t
        out.add(a)
    return sorted(out)


# --------------------------------------------------------------------------
# square-free decomposition (Section 2: Yun's algorithm ahead of FACTOR)
# --------------------------------------------------------------------------

def _derivative(p: Sequence[int]) -> List[int]:
    return [i * int(p[i]) for i in range(1, len(p))] or [0]


def _is_zero(p: Sequence[int]) -> bool:
    return all(int(c) == 0 for c in p)


def _gcd_z(f: Sequence[int], g: Sequence[int]) -> List[int]:
    """Primitive gcd (lc > 0) of two integer polynomials; sympy's polynomial
    gcd serves as the library step."""
    import sympy
    x = sympy.Symbol("x")
    if _is_zero(g):
        return primitive(f)
    if _is_zero(f):
        return primitive(g)
    F = sympy.Poly(list(reversed([int(c) for c in f])), x)
    G = sympy.Poly(list(reversed([int(c) for c in g])), x)
    h = sympy.gcd(F, G)
    return primitive([int(c) for c in reversed(h.all_coeffs())])


def _sub(a: Sequence[int], b: Sequence[int]) -> List[int]:
    n = max(len(a), len(b))
    a = list(a) + [0] * (n - len(a))
    b = list(b) + [0] * (n - len(b))
    return _trim([int(x) - int(y) for x, y in zip(a, b)])


def squarefree(coeffs: Sequence[int]) -> Tuple[int, List[Tuple[Tuple[int, ...], int]]]:
    """Square-free decomposition p = content * prod part**mult.

    Yun's algorithm over Z with primitive associates (every quotient below is
    exact): with f the primitive part of p without its powers of x,
    a0 = gcd(f, f'), b = f / a0, c = f' / a0, d = c - b'; then repeatedly
    a = gcd(b, d) is the part of the next multiplicity, b <- b / a,
    c <- d / a, d <- c - b', until b is constant.  A power x**k is the part x
    with multiplicity k.  Parts are primitive with lc > 0, sorted by
    (multiplicity, degree, coefficients).
    """
    cont, k, f = normalise(coeffs)
    parts: List[Tuple[Tuple[int, ...], int]] = []
    if k:
        parts.append(((0, 1), k))
    if len(f) > 1:
        fd = _derivative(f)
        a0 = _gcd_z(f, fd)
        b = exact_divide(f, a0)
        c = exact_divide(fd, a0)
        if b is None or c is None:
            raise OracleError("inexact division in the square-free decomposition")
        d = _sub(c, _derivative(b))
        mult = 1
        while len(b) > 1:
            a = primitive(b) if _is_zero(d) else _gcd_z(b, d)
            if len(a) > 1:
                parts.append((tuple(a), mult))
            b2 = exact_divide(b, a)
            c2 = [0] if _is_zero(d) else exact_divide(d, a)
            if b2 is None or c2 is None:
                raise OracleError("inexact division in the square-free decomposition")
            b = _trim(b2)
            d = _sub(c2, _derivative(b))
            mult += 1
    parts.sort(key=lambda pm: (pm[1], len(pm[0]), pm[0]))
    return cont, parts


def factor_general(coeffs: Sequence[int]) -> Tuple[int, List[Tuple[int, ...]]]:
    """Irreducible factorisation of any nonzero p of degree >= 1: FACTOR on
    every square-free part (Section 2), each factor listed as often as its
    multiplicity, in the canonical order."""
    cont, parts = squarefree(coeffs)
    facs: List[List[int]] = []
    for part, mult in parts:
        c1, fs = factor(list(part))
        if c1 != 1:
            raise OracleError("square-free part is not primitive")
        for f in fs:
            facs.extend([list(f)] * mult)
    return cont, canonical(facs)


def canonical(factors: List[List[int]]) -> List[Tuple[int, ...]]:
    return sorted((tuple(int(c) for c in f) for f in factors), key=lambda f: (len(f), f))


# --------------------------------------------------------------------------
# FACTOR end to end
# --------------------------------------------------------------------------

class Trace:
    """Intermediates of one oracle run (exposed for the tests)."""
    def __init__(self):
        self.n = 0
        self.w: List[int] = []
        self.t_lo = 0
        self.t_hi = 0
        self.candidates: List[int] = []
        self.confirmed: Dict[int, List[int]] = {}
        self.groups = []
        self.tr2_kept: List[int] = []    # candidates whose second trace is an integer
        self.v2: List[int] = []
        self.t2 = (0, 0)


def factor(coeffs: Sequence[int], trace: Optional[Trace] = None,
           brute_max: int = 22) -> Tuple[int, List[Tuple[int, ...]]]:
    """Irreducible factorisation over Z: p = content * prod(factors).

    Factors are primitive with positive leading coefficient, sorted by
    (degree, ascending coefficient tuple).  Raises OracleError for a
    non-square-free input.
    """
    cont, k, prim = normalise(coeffs)
    if k > 1:
        raise OracleError("not square-free (x^2 divides p)")
    extra = [(0, 1)] if k == 1 else []
    if len(prim) == 1:
        return cont, canonical([list(f) for f in extra])
    if len(prim) > 2 and not is_squarefree(prim):
        raise OracleError("not square-free")
    ts, groups, deltas = elements(prim)
    n = len(ts)
    w = weights(prim, ts)
    t_lo, t_hi = window(prim, deltas)
    cands = search(w, t_lo, t_hi, brute_max=brute_max)
    # a true factor's second trace is an integer as well: only those
    # candidates go on to the (expensive) reconstruction and division
    v2, t2 = second_trace(prim, groups, deltas)
    kept = second_trace_filter(cands, v2, t2)
    confirmed: Dict[int, List[int]] = {}
    full = (1 << n) - 1
    for s in kept:
        r = confirm(prim, groups, s, n)
        if r is not None:
            f, g = r
            confirmed[s] = f
            confirmed[full & ~s] = g
    facs = []
    for a in atoms(n, confirmed):
        if a == full:
            facs.append(list(prim))
        elif a in confirmed:
            facs.append(confirmed[a])
        else:
            raise OracleError("atom without a confirmed factor")
    if trace is not None:
        trace.n, trace.w, trace.t_lo, trace.t_hi = n, w, t_lo, t_hi
        trace.candidates, trace.confirmed, trace.groups = cands, confirmed, groups
        trace.tr2_kept, trace.v2, trace.t2 = kept, v2, t2
    return cont, canonical(facs + [list(f) for f in extra])
