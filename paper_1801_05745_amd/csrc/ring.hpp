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
UFX_FN bool fast_ring_pixel(int32_t N, double Nd, double eps, double dx, double dy, double dz, int32_t &pix) {
    const double rho2 = dx * dx + dy * dy;
    const double dz2 = dz * dz;
    const double a5 = 5.0 * dz2, a4 = 4.0 * rho2;
    if (fabs(a5 - a4) <= kRelGuard * (a5 + a4)) return false;   // near |z| = 2/3 (or d = 0)
    const double r = sqrt(rho2 + dz2);
    const double tt = fast_tt(dx, dy);
    if (a5 < a4) {
        const double z = dz / r;
        const double t1 = Nd * (0.5 + tt);
        const double t2 = 0.75 * Nd * z;
        double fa, fb;
        if (!clear_of_integer(t1 - t2, eps, fa) || !clear_of_integer(t1 + t2, eps, fb)) return false;
        const int32_t jp = (int32_t)fa, jm = (int32_t)fb;
        const int32_t k = N + 1 + jp - jm;                              // ring below z = 2/3, 1 .. 2N+1
        int32_t q = (jp + jm - N + ((k & 1) ^ 1) + 1) >> 1;             // 0 .. 4N+1
        q = q >= 4 * N ? q - 4 * N : q;
        pix = 2 * N * (N - 1) + 4 * N * (k - 1) + q;
        return true;
    }
    double ftt;
    if (!clear_of_integer(tt, eps, ftt)) return false;
    const double u = tt - ftt;
    const double one_minus = rho2 / (r * (r + fabs(dz)));
    const double sig = Nd * sqrt(3.0 * one_minus);
    double fp, fm;
    if (!clear_of_integer(u * sig, eps, fp) || !clear_of_integer((1.0 - u) * sig, eps, fm)) return false;
    const int32_t k = (int32_t)fp + (int32_t)fm + 1;                    // ring from the pole, 1 .. N
    double fq;
    if (!clear_of_integer(tt * (double)k, eps, fq)) return false;
    int32_t q = (int32_t)fq;                                            // 0 .. 4k-1 when clear
    q = q >= 4 * k ? q - 4 * k : q;
    pix = dz > 0.0 ? 2 * k * (k - 1) + q : 12 * N * N - 2 * k * (k + 1) + q;
    return true;
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
