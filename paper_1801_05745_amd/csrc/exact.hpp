// Exact decisions for instances that the FP64 fast path leaves inside a guard band.
//
// Two tools, both built from error-free transformations of IEEE binary64
// (the library is compiled with -ffp-contract=off, so a + b and a * b are
// single rounded operations and fma is explicit):
//   * expansion arithmetic (Shewchuk 1997, "Adaptive precision floating-point
//     arithmetic and fast robust geometric predicates"): exact sign of a sum
//     of products of doubles — used for every comparison that involves only the
//     coordinates and square roots of rational expressions in them;
//   * double-double arithmetic (Dekker 1971; Hida, Li & Bailey 2001) — used for
//     the azimuth tt = 2 phi / pi, which is transcendental for every direction
//     except the axes and diagonals, so its floors are never exact ties and a
//     ~2^-100 accurate value decides them (certified against an error margin).
//
// Pixel conventions (the paper names HEALPix; the formulas are Gorski et al. 2005):
// floor() at every boundary, |z| = 2/3 in the equatorial belt, phi = 0 on the
// z axis, the zero vector in pixel 0.
#pragma once

#include "common.hpp"

namespace ufx {

// ---------------------------------------------------------------- error-free transforms
struct dd {
    double hi, lo;
};

UFX_FN dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
UFX_FN dd fast_two_sum(double a, double b) {  // |a| >= |b|
    double s = a + b;
    return {s, b - (s - a)};
}
UFX_FN dd two_prod(double a, double b) {
    double p = a * b;
    return {p, fma(a, b, -p)};
}

// ---------------------------------------------------------------- double-double
UFX_FN dd dd_from(double a) { return {a, 0.0}; }
UFX_FN dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
UFX_FN dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}
UFX_FN dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
UFX_FN dd dd_mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return fast_two_sum(p.hi, p.lo);
}
UFX_FN dd dd_mul_d(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return fast_two_sum(p.hi, p.lo);
}
UFX_FN dd dd_div(dd a, dd b) {
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    dd q = fast_two_sum(q1, q2);
    return dd_add(q, dd_from(q3));
}
UFX_FN dd dd_sqrt(dd a) {
    if (a.hi <= 0.0) return {0.0, 0.0};
    double x = sqrt(a.hi);
    dd xx = two_prod(x, x);
    dd r = dd_sub(a, xx);
    double c = r.hi / (2.0 * x);
    dd y = fast_two_sum(x, c);
    // one more Newton correction in double-double
    dd r2 = dd_sub(a, dd_mul(y, y));
    return dd_add(y, dd_from(r2.hi / (2.0 * y.hi)));
}

// pi/2 as a double-double (hi = fl(pi/2), lo = pi/2 - hi)
UFX_FN dd dd_half_pi() { return {1.5707963267948966, 6.123233995736766e-17}; }

// tt = 2 phi / pi in [0, 4) for a direction that is not an axis or a diagonal.
// Octant reduction to t = min/max in (0, 1), three half-angle steps
// atan(t) = 2 atan(t / (1 + sqrt(1 + t^2))) to |t| < tan(pi/32), then the
// alternating Taylor series (|t|^2 < 0.0097; 17 terms reach 2^-110).
UFX_NOINLINE dd tt_dd(double dx, double dy) {
    double ax = fabs(dx), ay = fabs(dy);
    bool swap = ay > ax;
    dd t = dd_div(dd_from(swap ? ax : ay), dd_from(swap ? ay : ax));
    for (int k = 0; k < 3; ++k) {
        dd s = dd_sqrt(dd_add(dd_from(1.0), dd_mul(t, t)));
        t = dd_div(t, dd_add(dd_from(1.0), s));
    }
    dd t2 = dd_mul(t, t);
    dd term = t, sum = t;
    for (int k = 1; k <= 17; ++k) {
        term = dd_mul(term, t2);
        dd c = dd_div(term, dd_from((double)(2 * k + 1)));
        sum = (k & 1) ? dd_sub(sum, c) : dd_add(sum, c);
    }
    dd a = dd_mul_d(sum, 8.0);                 // atan(min/max) in [0, pi/4]
    dd th = dd_div(a, dd_half_pi());           // in quarter turns, [0, 1/2]
    if (swap) th = dd_sub(dd_from(1.0), th);   // angle measured from the x axis, [0, 1]
    if (dx > 0.0 && dy > 0.0) return th;
    if (dx < 0.0 && dy > 0.0) return dd_sub(dd_from(2.0), th);
    if (dx < 0.0 && dy < 0.0) return dd_add(dd_from(2.0), th);
    return dd_sub(dd_from(4.0), th);          // dx > 0, dy < 0
}

// ---------------------------------------------------------------- expansions
// A nonoverlapping expansion of at most CAP components, least significant
// first; the sign of the represented sum is the sign of the last nonzero one.
template <int CAP>
struct expansion {
    double c[CAP];
    int n = 0;
    UFX_FN void add(double b) {  // Grow-Expansion with zero elimination
        double q = b;
        int m = 0;
        for (int i = 0; i < n; ++i) {
            dd s = two_sum(q, c[i]);
            q = s.hi;
            if (s.lo != 0.0) c[m++] = s.lo;
        }
        if (q != 0.0 || m == 0) c[m++] = q;
        n = m;
    }
    // add coef * v * v exactly, coef given as an exact double-double (hi + lo)
    UFX_FN void add_scaled_square(dd coef, double v) {
        dd sq = two_prod(v, v);
        dd p;
        p = two_prod(coef.hi, sq.hi); add(p.hi); add(p.lo);
        p = two_prod(coef.hi, sq.lo); add(p.hi); add(p.lo);
        p = two_prod(coef.lo, sq.hi); add(p.hi); add(p.lo);
        p = two_prod(coef.lo, sq.lo); add(p.hi); add(p.lo);
    }
    UFX_FN int sign() const {
        for (int i = n - 1; i >= 0; --i)
            if (c[i] != 0.0) return c[i] > 0.0 ? 1 : -1;
        return 0;
    }
};

// exact coefficient k (|k| < 2^63 as an integer) as a double-double
UFX_FN dd exact_int(int64_t k) {
    double hi = (double)k;
    int64_t rest = k - (int64_t)hi;  // exact: hi is within 2^10 of k for |k| < 2^63
    return {hi, (double)rest};
}

// sign(A dz^2 - B (dx^2 + dy^2 + dz^2)) for integer coefficients A, B
UFX_NOINLINE int sign_quadratic(int64_t A, int64_t B, double dx, double dy, double dz) {
    expansion<72> e;
    dd a = exact_int(A), b = exact_int(-B);
    e.add_scaled_square(a, dz);
    e.add_scaled_square(b, dx);
    e.add_scaled_square(b, dy);
    e.add_scaled_square(b, dz);
    return e.sign();
}

// sign(dx^2 + dy^2 + dz^2 - e^2), exactly
UFX_NOINLINE int sign_r2_minus_e2(double dx, double dy, double dz, double edge) {
    expansion<40> e;
    dd one = {1.0, 0.0};
    e.add_scaled_square(one, dx);
    e.add_scaled_square(one, dy);
    e.add_scaled_square(one, dz);
    e.add_scaled_square({-1.0, 0.0}, edge);
    return e.sign();
}

// ---------------------------------------------------------------- exact shell
// b in [0, nb) with e[b] <= |d| < e[b+1] (edges e[0..nb], ascending, >= 0), or -1.
UFX_FN int exact_shell(double dx, double dy, double dz, const double *e, int nb) {
    if (sign_r2_minus_e2(dx, dy, dz, e[0]) < 0) return -1;
    if (sign_r2_minus_e2(dx, dy, dz, e[nb]) >= 0) return -1;
    int lo = 0, hi = nb;  // invariant: e[lo]^2 <= r^2 < e[hi]^2
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (sign_r2_minus_e2(dx, dy, dz, e[mid]) >= 0) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------- certified floors
// floor of a double-double value; *ok = 0 when it lies within `margin` of an integer.
// The distances to both neighbouring integers are formed in double-double, so a
// value like 1 - 4e-17 (hi = 1, lo < 0) is floored to 0 and is not mistaken for a tie.
UFX_FN int64_t dd_floor(dd v, double margin, int *ok) {
    double f = floor(v.hi);
    if (v.hi == f && v.lo < 0.0) f -= 1.0;
    const dd below = dd_sub(v, dd_from(f));
    const dd above = dd_sub(dd_from(f + 1.0), v);
    if (below.hi <= margin || above.hi <= margin) *ok = 0;
    return (int64_t)f;
}

// Special directions: floor(c0 + sgn * (3/4) N dz / r) with c0 = C2 / 2 exactly (C2 integer).
// The candidate m comes from a double-double estimate and is checked exactly
// (compare signs, then squares).
UFX_FN bool belt_ge(int64_t N, int sgn, int64_t C2, int64_t m, double dx, double dy, double dz) {
    // value >= m  <=>  sgn (3/4) N dz / r >= m - C2/2  <=>  sgn 3 N dz >= 2 V r,  V = 2m - C2
    int64_t V = 2 * m - C2;
    double lhs_sign = (double)sgn * dz;  // sign of the left side
    if (V == 0) return lhs_sign >= 0.0;
    if (V < 0 && lhs_sign >= 0.0) return true;
    if (V > 0 && lhs_sign <= 0.0) return false;
    // same sign: compare 9 N^2 dz^2 with 4 V^2 r^2
    int s = sign_quadratic(9 * N * N, 4 * V * V, dx, dy, dz);  // sign(9N^2 dz^2 - 4V^2 r^2)
    if (V > 0) return s >= 0;        // both positive: |lhs| >= |rhs|
    return s <= 0;                   // both negative: |lhs| <= |rhs|
}

UFX_FN int64_t belt_floor_exact(int64_t N, int sgn, int64_t C2, double approx,
                                                    double dx, double dy, double dz) {
    int64_t m = (int64_t)floor(approx);
    for (int it = 0; it < 4 && !belt_ge(N, sgn, C2, m, dx, dy, dz); ++it) --m;
    for (int it = 0; it < 4 && belt_ge(N, sgn, C2, m + 1, dx, dy, dz); ++it) ++m;
    return m;
}

// Special directions in the caps: floor(sigma / H), H in {1, 2}, sigma = N sqrt(3 (1 - |z|)).
// With Hp = 2/H:  sigma/H >= m  <=>  sigma^2 >= H^2 m^2  <=>  |z| <= 1 - H^2 m^2/(3N^2)
// <=>  K |dz| <= (K - 4 m^2) r  with K = 3 Hp^2 N^2.
UFX_FN bool cap_ge(int64_t N, int Hp, int64_t m, double dx, double dy, double dz) {
    if (m <= 0) return true;
    int64_t K = 3 * (int64_t)Hp * Hp * N * N;   // Hp = 2/H in {2, 1}
    int64_t M = K - 4 * m * m;
    if (M < 0) return false;
    // K |dz| <= M r  <=>  K^2 dz^2 <= M^2 r^2 (both sides >= 0)
    expansion<72> e;
    dd K2 = two_prod((double)K, (double)K);
    dd M2 = two_prod((double)M, (double)M);
    e.add_scaled_square(K2, dz);
    dd nM2 = {-M2.hi, -M2.lo};
    e.add_scaled_square(nM2, dx);
    e.add_scaled_square(nM2, dy);
    e.add_scaled_square(nM2, dz);
    return e.sign() <= 0;
}

UFX_FN int64_t cap_floor_exact(int64_t N, int Hp, double approx, double dx, double dy, double dz) {
    int64_t m = (int64_t)floor(approx);
    if (m < 0) m = 0;
    for (int it = 0; it < 4 && m > 0 && !cap_ge(N, Hp, m, dx, dy, dz); ++it) --m;
    for (int it = 0; it < 4 && cap_ge(N, Hp, m + 1, dx, dy, dz); ++it) ++m;
    return m;
}

// ---------------------------------------------------------------- exact RING pixel
// Returns the pixel; *unresolved is set when a transcendental floor could not be
// certified at double-double precision (not expected to happen in practice).
UFX_NOINLINE int64_t exact_ring_pixel(int64_t N, double dx, double dy, double dz, int *unresolved) {
    if (dx == 0.0 && dy == 0.0 && dz == 0.0) return 0;
    // exact azimuth for the axes and diagonals, as twice tt (integer)
    int tt2 = -1;
    if (dy == 0.0) tt2 = dx < 0.0 ? 4 : 0;
    else if (dx == 0.0) tt2 = dy > 0.0 ? 2 : 6;
    else if (dx == dy) tt2 = dx > 0.0 ? 1 : 5;
    else if (dx == -dy) tt2 = dx < 0.0 ? 3 : 7;

    const double Nd = (double)N;
    // |z| <= 2/3  <=>  5 dz^2 <= 4 (dx^2 + dy^2)  <=>  sign(9 dz^2 - 4 r^2) <= 0
    bool belt = sign_quadratic(9, 4, dx, dy, dz) <= 0;

    // double-double geometry
    dd sx = two_prod(dx, dx), sy = two_prod(dy, dy), sz = two_prod(dz, dz);
    dd rho2 = dd_add(sx, sy);
    dd r2 = dd_add(rho2, sz);
    dd r = dd_sqrt(r2);
    dd z = dd_div(dd_from(dz), r);
    int ok = 1;

    if (belt) {
        int64_t jp, jm;
        if (tt2 >= 0) {
            // c0 = N (1/2 + tt) = N (1 + tt2) / 2
            int64_t C2 = N * (1 + tt2);
            double w = 0.75 * Nd * (z.hi + z.lo);
            double c0 = 0.5 * (double)C2;
            jp = belt_floor_exact(N, -1, C2, c0 - w, dx, dy, dz);
            jm = belt_floor_exact(N, +1, C2, c0 + w, dx, dy, dz);
        } else {
            dd tt = tt_dd(dx, dy);
            dd t1 = dd_mul_d(dd_add(dd_from(0.5), tt), Nd);
            dd t2 = dd_mul_d(z, 0.75 * Nd);
            double margin = 0x1p-88 * (Nd * 5.0 + 1.0);
            jp = dd_floor(dd_sub(t1, t2), margin, &ok);
            jm = dd_floor(dd_add(t1, t2), margin, &ok);
        }
        int64_t k = N + 1 + jp - jm;
        int64_t s = (k & 1) ? 0 : 1;
        int64_t q = (jp + jm - N + s + 1) >> 1;
        q %= 4 * N;
        if (q < 0) q += 4 * N;
        if (!ok) *unresolved = 1;
        return 2 * N * (N - 1) + 4 * N * (k - 1) + q;
    }

    int64_t k, q;
    if (tt2 >= 0) {
        // u = tt - floor(tt) is 0 (tt2 even) or 1/2 (tt2 odd)
        dd one_minus = dd_div(rho2, dd_mul(r, dd_add(r, dd_from(fabs(dz)))));
        double sig = Nd * sqrt(3.0 * one_minus.hi);
        int64_t jp, jm;
        if ((tt2 & 1) == 0) {
            jp = 0;
            jm = cap_floor_exact(N, 2, sig, dx, dy, dz);          // floor(sigma)
        } else {
            jp = cap_floor_exact(N, 1, 0.5 * sig, dx, dy, dz);    // floor(sigma/2)
            jm = jp;
        }
        k = jp + jm + 1;
        q = (tt2 * k) >> 1;   // floor(tt k) = floor(tt2 k / 2), tt2 k >= 0
    } else {
        dd tt = tt_dd(dx, dy);
        double margin = 0x1p-88 * (Nd * 5.0 + 1.0);
        int64_t ftt = dd_floor(tt, 0x1p-90, &ok);
        dd u = dd_sub(tt, dd_from((double)ftt));
        dd one_minus = dd_div(rho2, dd_mul(r, dd_add(r, dd_from(fabs(dz)))));
        dd sig = dd_mul_d(dd_sqrt(dd_mul_d(one_minus, 3.0)), Nd);
        int64_t jp = dd_floor(dd_mul(u, sig), margin, &ok);
        int64_t jm = dd_floor(dd_mul(dd_sub(dd_from(1.0), u), sig), margin, &ok);
        k = jp + jm + 1;
        q = dd_floor(dd_mul_d(tt, (double)k), margin, &ok);
    }
    q %= 4 * k;
    if (q < 0) q += 4 * k;
    if (!ok) *unresolved = 1;
    if (dz > 0.0) return 2 * k * (k - 1) + q;
    return 12 * N * N - 2 * k * (k + 1) + q;
}

}  // namespace ufx
