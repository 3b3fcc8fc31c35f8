// FP64 fast path: shell index and HEALPix RING pixel of one particle image,
// with guard bands.  A decision is accepted only when its FP64 argument lies
// farther from the decision boundary than a margin that exceeds the FP64 error
// of this code by orders of magnitude; otherwise the caller re-takes it with
// the exact path (exact.hpp).
//
// RING pixel of direction d (HEALPix, Gorski et al. 2005; the paper uses 12*Nside^2
// pixels, section 2.4), with z = dz/|d| and tt = 2 phi/pi in [0, 4):
//   belt |z| <= 2/3:  jp = floor(N(1/2+tt) - 3Nz/4), jm = floor(N(1/2+tt) + 3Nz/4),
//                     k = N + 1 + jp - jm (ring counted from z = 2/3),
//                     q = ((jp + jm - N + [k even] + 1) / 2) mod 4N,
//                     pix = 2N(N-1) + 4N(k-1) + q
//   caps |z| > 2/3:   u = tt - floor(tt), sigma = N sqrt(3(1-|z|)),
//                     k = floor(u sigma) + floor((1-u) sigma) + 1, q = floor(tt k) mod 4k,
//                     pix = 2k(k-1) + q (north), 12N^2 - 2k(k+1) + q (south)
#pragma once

#include "common.hpp"

namespace ufx {

// Relative guard for r^2 against squared shell edges and for 5dz^2 against 4rho^2.
constexpr double kRelGuard = 0x1p-38;

// margin on floor arguments: N * 2^-38 (the FP64 error of the arguments is
// below ~6 N ulp(1) ~ N * 2^-50 for tt < 4, |z| <= 1)
UFX_HD double floor_margin(double Nd) { return Nd * 0x1p-38; }

UFX_FN bool clear_of_integer(double v, double eps, double &fl) {
    fl = floor(v);
    return (v - fl) > eps && (fl + 1.0 - v) > eps;
}

// tt = 2 phi / pi in [0, 4] for phi = atan2(dy, dx) taken in [0, 2 pi).
// One division reduces the azimuth to an octant: with mn = min(|dx|,|dy|),
// mx = max(|dx|,|dy|), u = mn/mx, or u = (mn - mx)/(mn + mx) plus a quarter of a
// quadrant when mn/mx > tan(pi/8), so |u| <= tan(pi/8); then
// (2/pi) atan(u) = u P(u^2) with P of degree 9 (gen_tt_poly.py: relative error
// < 1e-15 before rounding).  The absolute error of tt stays below ~2e-15, far
// inside the floor margin N 2^-38.  tt may round to 4.0 just below the +x axis;
// the guard band catches it.
UFX_FN double fast_tt(double dx, double dy) {
    const double ax = fabs(dx), ay = fabs(dy);
    const double mn = ax < ay ? ax : ay;
    const double mx = ax < ay ? ay : ax;
    const bool upper = mn > 0.4142 * mx;
    const double num = upper ? mn - mx : mn;
    const double den = upper ? mn + mx : mx;
    const double u = den > 0.0 ? num / den : 0.0;
    const double s = u * u;
    double p = -0.016116971463406102;
    p = fma(p, s, 0.0319886291636091);
    p = fma(p, s, -0.041418373955876615);
    p = fma(p, s, 0.04885124377544614);
    p = fma(p, s, -0.05786574491875008);
    p = fma(p, s, 0.07073513392040226);
    p = fma(p, s, -0.09094567142790448);
    p = fma(p, s, 0.1273239543359597);
    p = fma(p, s, -0.21220659078848142);
    p = fma(p, s, 0.6366197723675807);
    double th = fma(u, p, upper ? 0.5 : 0.0);  // quarter turns of atan(mn/mx), in [0, 1/2]
    th = ay > ax ? 1.0 - th : th;              // quarter turns of the angle of (|dx|, |dy|)
    if (dx >= 0.0) return dy >= 0.0 ? th : 4.0 - th;
    return dy >= 0.0 ? 2.0 - th : 2.0 + th;
}

// Returns true and the pixel when every decision is clear of its boundary.
// Pixel arithmetic is 32-bit: 12 N^2 < 2^31 for N <= 8192.
//
// Written without data-dependent branches: a wave holds belt and cap directions
// together, so both formulas are evaluated and selected per lane.  Every lane
// computes exactly the FP64 expressions of its own region (one division serves
// both: z = dz / r in the belt, 1 - |z| = rho2 / (r (r + |dz|)) in the caps), so
// the values are those of a branching evaluation.
UFX_FN bool fast_ring_pixel(int32_t N, double Nd, double eps, double dx, double dy, double dz, int32_t &pix) {
    const double rho2 = dx * dx + dy * dy;
    const double dz2 = dz * dz;
    const double a5 = 5.0 * dz2, a4 = 4.0 * rho2;
    bool ok = fabs(a5 - a4) > kRelGuard * (a5 + a4);  // false near |z| = 2/3 (or d = 0)
    const bool belt = a5 < a4;
    const double r = sqrt(rho2 + dz2);
    const double tt = fast_tt(dx, dy);
    const double num = belt ? dz : rho2;
    const double den0 = belt ? r : r * (r + fabs(dz));
    const double den = ok ? den0 : 1.0;              // keeps rejected lanes finite
    const double qd = num / den;                     // z (belt) or 1 - |z| (caps)
    // belt arguments
    const double t1 = Nd * (0.5 + tt);
    const double t2 = 0.75 * Nd * qd;
    // cap arguments
    const double ftt = floor(tt);
    const double u = tt - ftt;
    const double sig = Nd * sqrt(3.0 * (belt ? 0.0 : qd));
    const double va = belt ? t1 - t2 : u * sig;
    const double vb = belt ? t1 + t2 : (1.0 - u) * sig;
    double fa, fb;
    ok = ok & clear_of_integer(va, eps, fa);
    ok = ok & clear_of_integer(vb, eps, fb);
    ok = ok & (belt | ((tt - ftt) > eps && (ftt + 1.0 - tt) > eps));
    const int32_t ia = (int32_t)(ok ? fa : 0.0), ib = (int32_t)(ok ? fb : 0.0);
    // belt: jp = ia, jm = ib, ring k below z = 2/3 in 1 .. 2N+1
    const int32_t kb = N + 1 + ia - ib;
    int32_t qb = (ia + ib - N + ((kb & 1) ^ 1) + 1) >> 1;            // 0 .. 4N+1
    qb = qb >= 4 * N ? qb - 4 * N : qb;
    const int32_t pix_b = 2 * N * (N - 1) + 4 * N * (kb - 1) + qb;
    // caps: ring k from the pole in 1 .. N, q = floor(tt k) mod 4k
    const int32_t kc = belt ? 1 : ia + ib + 1;                       // (belt lanes: a harmless 1)
    double fq;
    ok = ok & (belt | clear_of_integer(tt * (double)kc, eps, fq));
    int32_t qc = (int32_t)(ok && !belt ? fq : 0.0);                  // 0 .. 4k-1 when clear
    qc = qc >= 4 * kc ? qc - 4 * kc : qc;
    const int32_t pix_c = dz > 0.0 ? 2 * kc * (kc - 1) + qc : 12 * N * N - 2 * kc * (kc + 1) + qc;
    pix = belt ? pix_b : pix_c;
    return ok;
}

// Largest j in [-1, nb] with e2[j] <= r2 (e2 ascending, j = -1 below e2[0]);
// *clear is false when r2 is within the relative guard of e2[j] or e2[j+1].
UFX_FN int fast_shell(const double *e2, int nb, int steps, double r2, bool &clear) {
    // branch-free binary search for the count of edges <= r2 over nb + 1 edges
    int lo = 0;
    for (int s = steps; s >= 0; --s) {
        int probe = lo + (1 << s);
        if (probe <= nb + 1 && e2[probe - 1] <= r2) lo = probe;
    }
    const int j = lo - 1;
    clear = true;
    if (j >= 0) clear = fabs(r2 - e2[j]) > kRelGuard * e2[j];
    if (j + 1 <= nb) clear = clear && fabs(r2 - e2[j + 1]) > kRelGuard * e2[j + 1];
    return j;
}

}  // namespace ufx
