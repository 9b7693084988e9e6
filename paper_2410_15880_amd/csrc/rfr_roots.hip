// Device root finding for batches of polynomials (the roots -> elements step
// ahead of the search): one workgroup per polynomial, one thread per root.
//
//   1. starting points on circles from the Newton polygon of (i, log|a_i|);
//   2. simultaneous Aberth-Ehrlich iteration in FP64 (every root updated from
//      the previous iterate of all the others);
//   3. Newton polish of every root in complex double-double, then its
//      inclusion radius d |p(z)| / |p'(z)| bounded with the evaluation error
//      (a root of p lies within it); for |z| > 1 the polynomial is evaluated
//      reversed at 1/z so nothing overflows;
//   4. a root whose disc meets the real axis is re-centred there and polished
//      in real double-double, with its own radius.
// The host checks the discs (disjoint, conjugate pairing), orders the
// elements and forms the weights and window, exactly as for roots it found
// itself; a polynomial whose device roots fail those checks is redone there.
//
// Compiled without floating-point contraction: the double-double arithmetic
// relies on exactly rounded adds, with fused multiply-adds written out.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rfr_roots.h"

namespace rfr {
namespace droots {

// ---------------------------------------------------------------- FP64 complex
struct Z {
    double re, im;
};
__device__ inline Z zadd(Z a, Z b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline Z zsub(Z a, Z b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline Z zmul(Z a, Z b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Z zscale(Z a, double s) { return {a.re * s, a.im * s}; }
__device__ inline double zabs(Z a) { return hypot(a.re, a.im); }
// Smith's division (no overflow of |b|^2)
__device__ inline Z zdiv(Z a, Z b) {
    if (fabs(b.re) >= fabs(b.im)) {
        const double r = b.im / b.re, den = b.re + b.im * r;
        return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
    }
    const double r = b.re / b.im, den = b.re * r + b.im;
    return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}

// ---------------------------------------------------------------- double-double
struct D2 {
    double hi, lo;
};
__device__ inline D2 two_sum(double a, double b) {
    const double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ inline D2 quick_two_sum(double a, double b) {
    const double s = a + b;
    return {s, b - (s - a)};
}
__device__ inline D2 two_prod(double a, double b) {
    const double p = a * b;
    return {p, fma(a, b, -p)};
}
__device__ inline D2 mk(double x) { return {x, 0.0}; }
__device__ inline D2 from_i64(int64_t v) {
    const int64_t top = v & ~(int64_t)0x7FF;  // at most 52 significant bits
    return two_sum((double)top, (double)(v - top));
}
__device__ inline D2 add(D2 a, D2 b) {
    D2 s = two_sum(a.hi, b.hi);
    const D2 t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
__device__ inline D2 neg(D2 a) { return {-a.hi, -a.lo}; }
__device__ inline D2 sub(D2 a, D2 b) { return add(a, neg(b)); }
__device__ inline D2 mul(D2 a, D2 b) {
    D2 p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
__device__ inline D2 muld(D2 a, double b) {
    D2 p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
__device__ inline D2 div(D2 a, D2 b) {
    const double q1 = a.hi / b.hi;
    D2 r = sub(a, muld(b, q1));
    const double q2 = r.hi / b.hi;
    r = sub(r, muld(b, q2));
    const double q3 = r.hi / b.hi;
    return add(quick_two_sum(q1, q2), mk(q3));
}
__device__ inline double to_d(D2 a) { return a.hi + a.lo; }

struct C2 {
    D2 re, im;
};
__device__ inline C2 cadd(C2 a, C2 b) { return {add(a.re, b.re), add(a.im, b.im)}; }
__device__ inline C2 csub(C2 a, C2 b) { return {sub(a.re, b.re), sub(a.im, b.im)}; }
__device__ inline C2 cmul(C2 a, C2 b) {
    return {sub(mul(a.re, b.re), mul(a.im, b.im)), add(mul(a.re, b.im), mul(a.im, b.re))};
}
__device__ inline C2 cdiv(C2 a, C2 b) {
    const D2 den = add(mul(b.re, b.re), mul(b.im, b.im));
    return {div(add(mul(a.re, b.re), mul(a.im, b.im)), den), div(sub(mul(a.im, b.re), mul(a.re, b.im)), den)};
}
__device__ inline double cabs_d(C2 a) { return hypot(to_d(a.re), to_d(a.im)); }

constexpr double kHornerU = 16.0 * 5.0e-32;  // > 16 * 2^-104 (complex double-double mul-add)
constexpr double kHornerUR = 8.0 * 5.0e-32;  // real double-double mul-add

// Newton step p(z)/p'(z) and inclusion radius at z (complex double-double).
__device__ void newton_c(const D2 *a, const double *aa, int d, C2 z, C2 &step, double &radius) {
    const double az = cabs_d(z);
    if (az <= 1.0) {
        C2 p{a[d], mk(0)}, dp{mk(0), mk(0)};
        double s = aa[d], ds = 0;
        for (int i = d - 1; i >= 0; --i) {
            dp = cadd(cmul(dp, z), p);
            p = cadd(cmul(p, z), C2{a[i], mk(0)});
            ds = ds * az + s;
            s = s * az + aa[i];
        }
        const double ep = 2.0 * d * kHornerU * s, edp = 2.0 * d * kHornerU * ds;
        const double adp = cabs_d(dp) - edp;
        step = cabs_d(dp) > 0 ? cdiv(p, dp) : C2{mk(0), mk(0)};
        radius = adp > 0 ? d * (cabs_d(p) + ep) / adp * (1 + 1e-12) : INFINITY;
        return;
    }
    const C2 y = cdiv(C2{mk(1), mk(0)}, z);
    const double ay = cabs_d(y);
    C2 q{a[0], mk(0)}, dq{mk(0), mk(0)};
    double s = aa[0], ds = 0;
    for (int i = 1; i <= d; ++i) {
        dq = cadd(cmul(dq, y), q);
        q = cadd(cmul(q, y), C2{a[i], mk(0)});
        ds = ds * ay + s;
        s = s * ay + aa[i];
    }
    const double eq = 2.0 * d * kHornerU * s, edq = 2.0 * d * kHornerU * ds;
    const C2 den = csub(C2{muld(q.re, (double)d), muld(q.im, (double)d)}, cmul(y, dq));
    const double aden = cabs_d(den) - d * eq - ay * edq;
    step = cabs_d(den) > 0 ? cdiv(cmul(z, q), den) : C2{mk(0), mk(0)};
    radius = aden > 0 ? d * az * (cabs_d(q) + eq) / aden * (1 + 1e-12) : INFINITY;
}

// The same on the real axis (real double-double).
__device__ void newton_r(const D2 *a, const double *aa, int d, D2 x, D2 &step, double &radius) {
    const double ax = fabs(to_d(x));
    if (ax <= 1.0) {
        D2 p = a[d], dp = mk(0);
        double s = aa[d], ds = 0;
        for (int i = d - 1; i >= 0; --i) {
            dp = add(mul(dp, x), p);
            p = add(mul(p, x), a[i]);
            ds = ds * ax + s;
            s = s * ax + aa[i];
        }
        const double ep = 2.0 * d * kHornerUR * s, edp = 2.0 * d * kHornerUR * ds;
        const double adp = fabs(to_d(dp)) - edp;
        step = to_d(dp) != 0 ? div(p, dp) : mk(0);
        radius = adp > 0 ? d * (fabs(to_d(p)) + ep) / adp * (1 + 1e-12) : INFINITY;
        return;
    }
    const D2 y = div(mk(1), x);
    const double ay = fabs(to_d(y));
    D2 q = a[0], dq = mk(0);
    double s = aa[0], ds = 0;
    for (int i = 1; i <= d; ++i) {
        dq = add(mul(dq, y), q);
        q = add(mul(q, y), a[i]);
        ds = ds * ay + s;
        s = s * ay + aa[i];
    }
    const double eq = 2.0 * d * kHornerUR * s, edq = 2.0 * d * kHornerUR * ds;
    const D2 den = sub(muld(q, (double)d), mul(y, dq));
    const double aden = fabs(to_d(den)) - d * eq - ay * edq;
    step = to_d(den) != 0 ? div(mul(x, q), den) : mk(0);
    radius = aden > 0 ? d * ax * (fabs(to_d(q)) + eq) / aden * (1 + 1e-12) : INFINITY;
}

// p(z)/p'(z) in FP64; for |z| > 1 through the reversed polynomial.
__device__ Z newton_ratio(const double *a, int d, Z z) {
    if (zabs(z) <= 1.0) {
        Z p{a[d], 0}, dp{0, 0};
        for (int i = d - 1; i >= 0; --i) {
            dp = zadd(zmul(dp, z), p);
            p = zadd(zmul(p, z), Z{a[i], 0});
        }
        return zdiv(p, dp);
    }
    const Z y = zdiv(Z{1, 0}, z);
    Z q{a[0], 0}, dq{0, 0};
    for (int i = 1; i <= d; ++i) {
        dq = zadd(zmul(dq, y), q);
        q = zadd(zmul(q, y), Z{a[i], 0});
    }
    return zdiv(zmul(z, q), zsub(zscale(q, (double)d), zmul(y, dq)));
}

__device__ inline bool finite(Z z) { return isfinite(z.re) && isfinite(z.im); }

__global__ __launch_bounds__(ROOT_THREADS) void k_roots(const RootJob *jobs, int njobs) {
    const int j = blockIdx.x;
    if (j >= njobs) return;
    const RootJob J = jobs[j];
    const int d = J.degree;
    const int tid = threadIdx.x;
    __shared__ double s_a[RFR_MAX_DEGREE + 1];   // coefficients (FP64)
    __shared__ double s_aa[RFR_MAX_DEGREE + 1];  // |coefficients| (FP64)
    __shared__ D2 s_add[RFR_MAX_DEGREE + 1];     // coefficients (double-double, exact)
    __shared__ Z s_z[RFR_MAX_DEGREE];            // current iterate
    __shared__ double s_lg[RFR_MAX_DEGREE + 1];   // log|a_i| (a_i != 0)
    __shared__ int s_hull[RFR_MAX_DEGREE + 1];    // hull vertices (coefficient indices)
    __shared__ int s_nh;
    if (d < 2 || d > RFR_MAX_DEGREE) return;  // the host handles linear inputs

    for (int i = tid; i <= d; i += ROOT_THREADS) {
        const int64_t c = J.coeffs[i];
        s_a[i] = (double)c;
        s_add[i] = from_i64(c);
        s_aa[i] = fabs(to_d(s_add[i]));
        s_lg[i] = c != 0 ? log(fabs((double)c)) : 0.0;
    }
    __syncthreads();
    // 1. starting points: one circle per edge of the upper convex hull of
    //    (i, log|a_i|) over the nonzero coefficients, radius from the edge's
    //    slope; the hull walk is serial, the points are set in parallel
    if (tid == 0) {
        int h = 0;
        for (int k = 0; k <= d; ++k) {
            if (s_a[k] == 0) continue;
            while (h >= 2) {
                const int i1 = s_hull[h - 2], i2 = s_hull[h - 1];
                if ((double)(i2 - i1) * (s_lg[k] - s_lg[i1]) - (s_lg[i2] - s_lg[i1]) * (double)(k - i1) >= 0) --h;
                else break;
            }
            s_hull[h++] = k;
        }
        s_nh = h;
    }
    __syncthreads();
    if (tid < d) {
        // root slot tid lies on the edge [k, l) with k <= tid < l (a_0, a_d != 0,
        // so the hull spans 0..d and its edges cover every slot once)
        int e = 0;
        while (e + 2 < s_nh && s_hull[e + 1] <= tid) ++e;
        const int k = s_hull[e], l = s_hull[e + 1], q = tid - k;
        const double two_pi = 6.283185307179586;
        const double u = exp((s_lg[k] - s_lg[l]) / (l - k));
        const double ang = two_pi * q / (l - k) + two_pi * k / d + 0.4;
        double sn, cs;
        sincos(ang, &sn, &cs);
        s_z[tid] = Z{u * cs, u * sn};
    }
    __syncthreads();
    // 2. simultaneous Aberth-Ehrlich iteration.  A root stops when its step is
    //    below 1e-13 of its modulus, or small and no longer shrinking (the
    //    FP64 evaluation noise floor); the double-double polish takes it from
    //    there.  The workgroup iterates until every root has stopped.
    Z z = tid < d ? s_z[tid] : Z{0, 0};
    bool done = tid >= d;
    double prev = INFINITY;
    for (int it = 0; it < ROOT_MAXIT; ++it) {
        Z wc{0, 0};
        bool upd = false;
        if (!done) {
            const Z N = newton_ratio(s_a, d, z);
            // S = sum over the other roots of 1 / (z - z_q) = conj(w) / |w|^2,
            // four independent partial sums so the divisions overlap; the own
            // term is replaced by w = 1 and taken out at the end
            double sr[4] = {0, 0, 0, 0}, si[4] = {0, 0, 0, 0};
            int q = 0;
            for (; q + 4 <= d; q += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    Z w = zsub(z, s_z[q + u]);
                    if (q + u == tid) w = Z{1, 0};
                    const double inv = 1.0 / (w.re * w.re + w.im * w.im);
                    sr[u] += w.re * inv;
                    si[u] -= w.im * inv;
                }
            }
            for (; q < d; ++q) {
                Z w = zsub(z, s_z[q]);
                if (q == tid) w = Z{1, 0};
                const double inv = 1.0 / (w.re * w.re + w.im * w.im);
                sr[0] += w.re * inv;
                si[0] -= w.im * inv;
            }
            const Z S{(sr[0] + sr[1]) + (sr[2] + sr[3]) - 1.0, (si[0] + si[1]) + (si[2] + si[3])};
            wc = zdiv(N, zsub(Z{1, 0}, zmul(N, S)));
            if (!finite(wc)) done = true;
            else upd = true;
        }
        __syncthreads();
        if (upd) {
            z = zsub(z, wc);
            s_z[tid] = z;
            const double step = zabs(wc), scale = fmax(zabs(z), 1e-300);
            if (step <= 1e-13 * scale || (step <= 1e-9 * scale && step >= 0.5 * prev)) done = true;
            prev = step;
        }
        if (!__syncthreads_or(!done)) break;
    }
    if (tid >= d) return;
    // 3. complex double-double polish and inclusion radius
    C2 c{mk(z.re), mk(z.im)};
    C2 step;
    double radius;
    // Newton converges quadratically from the FP64 root.  Once a step is below
    // 1e-20 of the root, the point it was computed at is kept: its disc
    // (radius from that same evaluation) is already far below what the
    // weights need, so no further evaluation is spent on the last few digits.
    bool conv = false;
    for (int k = 0; k < ROOT_POLISH && !conv; ++k) {
        newton_c(s_add, s_aa, d, c, step, radius);
        conv = cabs_d(step) <= 1e-20 * fmax(cabs_d(c), 1e-300);
        if (!conv) c = csub(c, step);
    }
    if (!conv) newton_c(s_add, s_aa, d, c, step, radius);
    RootOut out;
    out.re_hi = c.re.hi;
    out.re_lo = c.re.lo;
    out.im_hi = c.im.hi;
    out.im_lo = c.im.lo;
    out.r = radius;
    out.x_hi = out.x_lo = 0;
    out.rx = INFINITY;
    // 4. a disc meeting the real axis: real polish and radius
    if (fabs(to_d(c.im)) <= radius) {
        D2 x = c.re, sx;
        double rx;
        bool convr = false;
        for (int k = 0; k < ROOT_POLISH && !convr; ++k) {
            newton_r(s_add, s_aa, d, x, sx, rx);
            convr = fabs(to_d(sx)) <= 1e-20 * fmax(fabs(to_d(x)), 1e-300);
            if (!convr) x = sub(x, sx);
        }
        if (!convr) newton_r(s_add, s_aa, d, x, sx, rx);
        out.x_hi = x.hi;
        out.x_lo = x.lo;
        out.rx = rx;
    }
    J.out[tid] = out;
}

}  // namespace droots

hipError_t launch_roots(const RootJob *jobs_dev, int njobs, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(droots::k_roots, dim3(njobs), dim3(ROOT_THREADS), 0, st, jobs_dev, njobs);
    return hipGetLastError();
}

}  // namespace rfr
