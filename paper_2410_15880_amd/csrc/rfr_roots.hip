// Device root finding for batches of polynomials (the roots -> elements step
// ahead of the search): one workgroup per polynomial, one thread per root in a
// batch, a group of ROOT_LANES threads per root for a single polynomial.
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

// ---------------------------------------------------------------- lane groups
// A root may be served by L lanes (L = 1 or ROOT_LANES, consecutive lanes of a
// wavefront): lane l evaluates the l-th run of m = ceil((d+1)/L) coefficients
// by Horner, and the runs are combined with the powers x^(l m).  The group
// sums are butterflies; each step adds the same two operands in either order,
// which FP64 and double-double addition do bit for bit alike, so every lane of
// a group ends with identical values and takes identical steps.
__device__ inline double gsum(double v, int L) {
    for (int o = 1; o < L; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline D2 gsum(D2 v, int L) {
    for (int o = 1; o < L; o <<= 1) v = add(v, D2{__shfl_xor(v.hi, o, 64), __shfl_xor(v.lo, o, 64)});
    return v;
}
__device__ inline C2 gsum(C2 v, int L) { return {gsum(v.re, L), gsum(v.im, L)}; }

// newton_ratio over a lane group.
__device__ Z newton_ratio_group(const double *a, int d, Z z, int lane, int L) {
    const int m = (d + L) / L;
    const bool inside = zabs(z) <= 1.0;
    const Z x = inside ? z : zdiv(Z{1, 0}, z);  // |z| > 1: y^d p(1/y) in y = 1/z
    const int j0 = lane * m, j1 = min(j0 + m, d + 1);
    Z P{0, 0}, dP{0, 0};
    for (int j = j1 - 1; j >= j0; --j) {
        dP = zadd(zmul(dP, x), P);
        P = zadd(zmul(P, x), Z{a[inside ? j : d - j], 0});
    }
    Z pw{1, 0}, b = x;  // x^j0
    for (int e = j0; e; e >>= 1) {
        if (e & 1) pw = zmul(pw, b);
        b = zmul(b, b);
    }
    const Z v = zmul(pw, P), dv = zmul(pw, dP);
    const double sc = (double)j0;  // d/dx x^j0 P = x^j0 P' + j0 x^(j0 - 1) P
    const Z val{gsum(v.re, L), gsum(v.im, L)};
    Z der{gsum(dv.re, L), gsum(dv.im, L)};
    if (L > 1) der = zadd(der, zdiv(Z{gsum(v.re * sc, L), gsum(v.im * sc, L)}, x));
    if (inside) return zdiv(val, der);
    return zdiv(zmul(z, val), zsub(zscale(val, (double)d), zmul(x, der)));
}

// newton_c over a lane group.  The evaluation error is bounded as for one
// Horner run of length d (each lane's run is shorter) plus a margin of 64
// units for the powers of x and the combination, which is far above their
// few roundings.
__device__ void newton_c_group(const D2 *a, const double *aa, int d, C2 z, int lane, int L, C2 &step,
                               double &radius) {
    const double az = cabs_d(z);
    const bool inside = az <= 1.0;
    const C2 x = inside ? z : cdiv(C2{mk(1), mk(0)}, z);
    const double ax = inside ? az : cabs_d(x);
    const int m = (d + L) / L;
    const int j0 = lane * m, j1 = min(j0 + m, d + 1);
    C2 P{mk(0), mk(0)}, dP{mk(0), mk(0)};
    double sp = 0, sd = 0;
    for (int j = j1 - 1; j >= j0; --j) {
        const int i = inside ? j : d - j;
        dP = cadd(cmul(dP, x), P);
        P = cadd(cmul(P, x), C2{a[i], mk(0)});
        sd = sd * ax + sp;
        sp = sp * ax + aa[i];
    }
    C2 pw{mk(1), mk(0)}, b = x;  // x^j0 and |x|^j0
    double apw = 1, ab = ax;
    for (int e = j0; e; e >>= 1) {
        if (e & 1) {
            pw = cmul(pw, b);
            apw *= ab;
        }
        b = cmul(b, b);
        ab *= ab;
    }
    const C2 val = gsum(cmul(pw, P), L);
    C2 der = gsum(cmul(pw, dP), L);
    const double S = gsum(apw * sp, L);
    const double DS = gsum(apw * sd + (j0 > 0 ? (double)j0 * (apw / ax) * sp : 0.0), L);
    if (L > 1) {
        const C2 v = cmul(pw, P);
        der = cadd(der, cdiv(gsum(C2{muld(v.re, (double)j0), muld(v.im, (double)j0)}, L), x));
    }
    const double kk = (2.0 * d + (L > 1 ? 64.0 : 0.0)) * kHornerU;
    if (inside) {
        const double ep = kk * S, edp = kk * DS;
        const double adp = cabs_d(der) - edp;
        step = cabs_d(der) > 0 ? cdiv(val, der) : C2{mk(0), mk(0)};
        radius = adp > 0 ? d * (cabs_d(val) + ep) / adp * (1 + 1e-12) : INFINITY;
        return;
    }
    const double eq = kk * S, edq = kk * DS;
    const C2 den = csub(C2{muld(val.re, (double)d), muld(val.im, (double)d)}, cmul(x, der));
    const double aden = cabs_d(den) - d * eq - ax * edq;
    step = cabs_d(den) > 0 ? cdiv(cmul(z, val), den) : C2{mk(0), mk(0)};
    radius = aden > 0 ? d * az * (cabs_d(val) + eq) / aden * (1 + 1e-12) : INFINITY;
}

// newton_r over a lane group (real double-double), same bound.
__device__ void newton_r_group(const D2 *a, const double *aa, int d, D2 xr, int lane, int L, D2 &step,
                               double &radius) {
    const double axr = fabs(to_d(xr));
    const bool inside = axr <= 1.0;
    const D2 x = inside ? xr : div(mk(1), xr);
    const double ax = inside ? axr : fabs(to_d(x));
    const int m = (d + L) / L;
    const int j0 = lane * m, j1 = min(j0 + m, d + 1);
    D2 P = mk(0), dP = mk(0);
    double sp = 0, sd = 0;
    for (int j = j1 - 1; j >= j0; --j) {
        const int i = inside ? j : d - j;
        dP = add(mul(dP, x), P);
        P = add(mul(P, x), a[i]);
        sd = sd * ax + sp;
        sp = sp * ax + aa[i];
    }
    D2 pw = mk(1), b = x;
    double apw = 1, ab = ax;
    for (int e = j0; e; e >>= 1) {
        if (e & 1) {
            pw = mul(pw, b);
            apw *= ab;
        }
        b = mul(b, b);
        ab *= ab;
    }
    const D2 val = gsum(mul(pw, P), L);
    D2 der = gsum(mul(pw, dP), L);
    const double S = gsum(apw * sp, L);
    const double DS = gsum(apw * sd + (j0 > 0 ? (double)j0 * (apw / ax) * sp : 0.0), L);
    if (L > 1) der = add(der, div(gsum(muld(mul(pw, P), (double)j0), L), x));
    const double kk = (2.0 * d + (L > 1 ? 64.0 : 0.0)) * kHornerUR;
    if (inside) {
        const double ep = kk * S, edp = kk * DS;
        const double adp = fabs(to_d(der)) - edp;
        step = to_d(der) != 0 ? div(val, der) : mk(0);
        radius = adp > 0 ? d * (fabs(to_d(val)) + ep) / adp * (1 + 1e-12) : INFINITY;
        return;
    }
    const double eq = kk * S, edq = kk * DS;
    const D2 den = sub(muld(val, (double)d), mul(x, der));
    const double aden = fabs(to_d(den)) - d * eq - ax * edq;
    step = to_d(den) != 0 ? div(mul(xr, val), den) : mk(0);
    radius = aden > 0 ? d * axr * (fabs(to_d(val)) + eq) / aden * (1 + 1e-12) : INFINITY;
}

__device__ inline bool finite(Z z) { return isfinite(z.re) && isfinite(z.im); }

__global__ __launch_bounds__(ROOT_THREADS) void k_roots(const RootJob *jobs, int njobs, int L) {
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

    for (int i = tid; i <= d; i += (int)blockDim.x) {
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
    // 2. simultaneous Aberth-Ehrlich iteration, L lanes per root (root
    //    r = tid / L): the lanes share its Horner evaluation and the sum over
    //    the other roots.  A root stops when its step is below 1e-13 of its
    //    modulus, or small and no longer shrinking (the FP64 evaluation noise
    //    floor); the double-double polish takes it from there.  The workgroup
    //    iterates until every root has stopped.
    const int r = tid / L, lane = tid % L;
    Z z = r < d ? s_z[r] : Z{0, 0};
    bool done = r >= d;
    double prev = INFINITY;
    for (int it = 0; it < ROOT_MAXIT; ++it) {
        Z wc{0, 0};
        bool upd = false;
        if (!done) {
            const Z N = newton_ratio_group(s_a, d, z, lane, L);
            // S = sum over the other roots of 1 / (z - z_q) = conj(w) / |w|^2,
            // lane l taking q = l mod L, two partial sums so the divisions
            // overlap; the own term is replaced by w = 1 and taken out at the end
            double sr[2] = {0, 0}, si[2] = {0, 0};
            int q = lane;
            for (; q + L < d; q += 2 * L) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int qq = q + u * L;
                    Z w = zsub(z, s_z[qq]);
                    if (qq == r) w = Z{1, 0};
                    const double inv = 1.0 / (w.re * w.re + w.im * w.im);
                    sr[u] += w.re * inv;
                    si[u] -= w.im * inv;
                }
            }
            for (; q < d; q += L) {
                Z w = zsub(z, s_z[q]);
                if (q == r) w = Z{1, 0};
                const double inv = 1.0 / (w.re * w.re + w.im * w.im);
                sr[0] += w.re * inv;
                si[0] -= w.im * inv;
            }
            const Z S{gsum(sr[0] + sr[1], L) - 1.0, gsum(si[0] + si[1], L)};
            wc = zdiv(N, zsub(Z{1, 0}, zmul(N, S)));
            if (!finite(wc)) done = true;
            else upd = true;
        }
        __syncthreads();
        if (upd) {
            z = zsub(z, wc);
            if (lane == 0) s_z[r] = z;
            const double step = zabs(wc), scale = fmax(zabs(z), 1e-300);
            if (step <= 1e-13 * scale || (step <= 1e-9 * scale && step >= 0.5 * prev)) done = true;
            prev = step;
        }
        if (!__syncthreads_or(!done)) break;
    }
    if (r >= d) return;
    // 3. complex double-double polish and inclusion radius (the group's lanes
    //    in step).  Newton converges quadratically from the FP64 root.  Once a
    //    step is below 1e-20 of the root, the point it was computed at is kept:
    //    its disc (radius from that same evaluation) is already far below what
    //    the weights need, so no further evaluation is spent on the last digits.
    C2 c{mk(z.re), mk(z.im)};
    C2 step;
    double radius;
    bool conv = false;
    for (int k = 0; k < ROOT_POLISH && !conv; ++k) {
        newton_c_group(s_add, s_aa, d, c, lane, L, step, radius);
        conv = cabs_d(step) <= 1e-20 * fmax(cabs_d(c), 1e-300);
        if (!conv) c = csub(c, step);
    }
    if (!conv) newton_c_group(s_add, s_aa, d, c, lane, L, step, radius);
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
            newton_r_group(s_add, s_aa, d, x, lane, L, sx, rx);
            convr = fabs(to_d(sx)) <= 1e-20 * fmax(fabs(to_d(x)), 1e-300);
            if (!convr) x = sub(x, sx);
        }
        if (!convr) newton_r_group(s_add, s_aa, d, x, lane, L, sx, rx);
        out.x_hi = x.hi;
        out.x_lo = x.lo;
        out.rx = rx;
    }
    if (lane == 0) J.out[r] = out;
}

}  // namespace droots

hipError_t launch_roots(const RootJob *jobs_dev, int njobs, int max_degree, int lanes, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    if (max_degree < 2 || max_degree > RFR_MAX_DEGREE || (lanes != 1 && lanes != ROOT_LANES))
        return hipErrorInvalidValue;
    const int threads = (lanes * max_degree + 63) / 64 * 64;
    hipLaunchKernelGGL(droots::k_roots, dim3(njobs), dim3(threads), 0, st, jobs_dev, njobs, lanes);
    return hipGetLastError();
}

}  // namespace rfr
