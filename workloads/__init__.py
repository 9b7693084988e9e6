"""Seeded synthetic inputs for the recombination benchmarks and tests.

This module only draws integer polynomials; it holds none of the factorisation
arithmetic, so both the product path and the CPU oracle may import it.

Polynomials are lists of Python ints in ascending order: ``c[i]`` is the
coefficient of ``x**i``.  Every draw uses ``numpy.random.Generator(PCG64(seed))``
and ``integers(lo, hi + 1)``.

Workload families (sizes follow the paper's benchmark, Section 5: products of
two random integer polynomials, coefficients drawn uniformly):

* ``config_small``   degree 20: product of two random degree-10 polynomials,
  coefficients in [-10, 10] (seed 1001).
* ``config_mid``     degree 60, 16 polynomials: 8 random in [-100, 100] and
  8 planted products of degree 20 x 40 (seeds 2000..2015).
* ``config_large``   degree 100, 16 polynomials: 8 random in [-1000, 1000] and
  8 planted products of degree 30 x 70 (seeds 3000..3015).
* ``config_batch``   4096 polynomials, degree uniform in [16, 80], even index
  random, odd index a planted two-factor product (seeds 4000..8095).
* ``config_stream``  Poisson request stream, degree log-uniform in [24, 128],
  coefficients in [-1000, 1000], 30 % planted (stream seed 5000).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Workload", "rand_poly", "poly_mul", "planted_split",
    "config_small", "config_mid", "config_large", "config_batch", "config_stream",
    "config_repeated", "swinnerton_dyer", "config_flood",
]


@dataclass
class Workload:
    """One input polynomial plus how it was drawn."""
    coeffs: List[int]
    seed: int
    kind: str                      # "random" or "planted"
    planted: List[List[int]] = field(default_factory=list)  # the drawn factors

    @property
    def degree(self) -> int:
        return len(self.coeffs) - 1


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def rand_poly(rng: np.random.Generator, degree: int, lo: int, hi: int) -> List[int]:
    """Random integer polynomial of exact degree ``degree``.

    Coefficients are iid uniform in [lo, hi]; the leading and constant
    coefficients are re-drawn until nonzero.
    """
    c = [int(v) for v in rng.integers(lo, hi + 1, size=degree + 1)]
    while c[0] == 0:
        c[0] = int(rng.integers(lo, hi + 1))
    while c[-1] == 0:
        c[-1] = int(rng.integers(lo, hi + 1))
    return c


def poly_mul(f: List[int], g: List[int]) -> List[int]:
    """Exact product of two integer polynomials (input construction only)."""
    out = [0] * (len(f) + len(g) - 1)
    for i, a in enumerate(f):
        if a:
            for j, b in enumerate(g):
                out[i + j] += a * b
    return out


def planted_split(rng: np.random.Generator, d: int) -> int:
    """Degree of the smaller planted factor: uniform in [ceil(0.3 d), floor(d/2)]."""
    lo = max(1, math.ceil(0.3 * d))
    hi = max(lo, d // 2)
    return int(rng.integers(lo, hi + 1))


def _planted(rng, d1: int, d2: int, lo: int, hi: int, seed: int) -> Workload:
    f = rand_poly(rng, d1, lo, hi)
    g = rand_poly(rng, d2, lo, hi)
    return Workload(poly_mul(f, g), seed, "planted", [f, g])


def config_small(seed: int = 1001) -> Workload:
    """Degree-20 product of two degree-10 polynomials, coefficients in [-10, 10]."""
    rng = _rng(seed)
    return _planted(rng, 10, 10, -10, 10, seed)


def config_mid(count: int = 16, base_seed: int = 2000) -> List[Workload]:
    """Degree 60: indices < 8 random in [-100,100]; the rest 20 x 40 products."""
    out = []
    for i in range(count):
        seed = base_seed + i
        rng = _rng(seed)
        if i < 8:
            out.append(Workload(rand_poly(rng, 60, -100, 100), seed, "random"))
        else:
            out.append(_planted(rng, 20, 40, -100, 100, seed))
    return out


def config_large(count: int = 16, base_seed: int = 3000) -> List[Workload]:
    """Degree 100: indices < 8 random in [-1000,1000]; the rest 30 x 70 products."""
    out = []
    for i in range(count):
        seed = base_seed + i
        rng = _rng(seed)
        if i < 8:
            out.append(Workload(rand_poly(rng, 100, -1000, 1000), seed, "random"))
        else:
            out.append(_planted(rng, 30, 70, -1000, 1000, seed))
    return out


def config_batch(count: int = 4096, base_seed: int = 4000,
                 dmin: int = 16, dmax: int = 80) -> List[Workload]:
    """Uneven batch: degree uniform in [dmin, dmax], coefficients in [-100, 100].

    Even indices are random (almost surely irreducible); odd indices are
    planted two-factor products with the smaller degree drawn by
    :func:`planted_split`.
    """
    out = []
    for i in range(count):
        seed = base_seed + i
        rng = _rng(seed)
        d = int(rng.integers(dmin, dmax + 1))
        if i % 2 == 0:
            out.append(Workload(rand_poly(rng, d, -100, 100), seed, "random"))
        else:
            d1 = planted_split(rng, d)
            out.append(_planted(rng, d1, d - d1, -100, 100, seed))
    return out


@dataclass
class Request:
    """One served request: arrival time (seconds from stream start) + input."""
    t_arrive: float
    work: Workload


def config_stream(count: int, rate_per_s: float, seed: int = 5000,
                  dmin: int = 24, dmax: int = 128, p_planted: float = 0.3,
                  lo: int = -1000, hi: int = 1000,
                  dcap: Optional[int] = None) -> List[Request]:
    """Poisson request stream with log-uniform degrees.

    Inter-arrival gaps are exponential with mean ``1/rate_per_s``; the degree is
    ``round(exp(U(ln dmin, ln dmax)))`` (optionally clipped to ``dcap``); each
    request is a planted product with probability ``p_planted``.
    """
    rng = _rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        d = int(round(math.exp(rng.uniform(math.log(dmin), math.log(dmax)))))
        if dcap is not None:
            d = min(d, dcap)
        sub = _rng(seed * 100003 + k)
        if float(rng.uniform()) < p_planted and d >= 2:
            d1 = planted_split(sub, d)
            w = _planted(sub, d1, d - d1, lo, hi, seed * 100003 + k)
        else:
            w = Workload(rand_poly(sub, d, lo, hi), seed * 100003 + k, "random")
        out.append(Request(t, w))
    return out


def config_repeated(count: int = 24, base_seed: int = 6000, lo: int = -20, hi: int = 20) -> List[Workload]:
    """Polynomials that are not square-free: p = c * x**k * prod_m f_m**m.

    For each seed: 1-3 random factors (degree 1-8 each, coefficients in
    [lo, hi]) with multiplicities drawn from 1..3 (at least one above 1),
    a power x**k with k in 0..2, and a content c in [1, 3] with a random
    sign.  ``planted`` lists every drawn factor once per multiplicity (x as
    [0, 1]); the content is the product's, not part of ``planted``.
    """
    out = []
    for i in range(count):
        seed = base_seed + i
        rng = _rng(seed)
        nf = int(rng.integers(1, 4))
        mults = [int(rng.integers(1, 4)) for _ in range(nf)]
        if max(mults) == 1:
            mults[int(rng.integers(0, nf))] = int(rng.integers(2, 4))
        k = int(rng.integers(0, 3))
        c = int(rng.integers(1, 4)) * (1 if rng.uniform() < 0.5 else -1)
        p = [c]
        planted = []
        for m in mults:
            f = rand_poly(rng, int(rng.integers(1, 9)), lo, hi)
            for _ in range(m):
                p = poly_mul(p, f)
                planted.append(f)
        for _ in range(k):
            p = poly_mul(p, [0, 1])
            planted.append([0, 1])
        out.append(Workload(p, seed, "repeated", planted))
    return out


def swinnerton_dyer(k: int) -> List[int]:
    """Swinnerton-Dyer f_k (Section 2, Eq 5): the minimal polynomial of
    sqrt(2) + sqrt(3) + ... + sqrt(p_k) (degree 2**k, all roots real), built
    exactly with sympy."""
    import sympy
    x = sympy.Symbol("x")
    s = sum(sympy.sqrt(sympy.prime(i)) for i in range(1, k + 1))
    mp = sympy.Poly(sympy.minimal_polynomial(s, x), x)
    return [int(v) for v in reversed(mp.all_coeffs())]


def config_flood() -> List[Workload]:
    """Inputs that flood the first-trace search with candidates (Section 2,
    Eq 5-7: subsets of a Swinnerton-Dyer polynomial's roots with an integer
    sum that are not factors):

    * f_5 (degree 32, 32 real roots), irreducible;
    * f_5(x) * (x**32 - x - 1) (degree 64), two irreducible factors (the
      second by Selmer's theorem on x**n - x - 1), coefficients within int64.
    """
    f5 = swinnerton_dyer(5)
    selmer = [-1, -1] + [0] * 30 + [1]
    return [Workload(f5, 9201, "swinnerton-dyer", [f5]),
            Workload(poly_mul(f5, selmer), 9202, "planted", [f5, selmer])]
