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

// Returns true and the pixel when every decision is clear of its boundary.
UFX_FN bool fast_ring_pixel(int64_t N, double Nd, double eps, double dx, double dy, double dz, int64_t &pix) {
    const double rho2 = dx * dx + dy * dy;
    const double dz2 = dz * dz;
    const double a5 = 5.0 * dz2, a4 = 4.0 * rho2;
    if (fabs(a5 - a4) <= kRelGuard * (a5 + a4)) return false;   // near |z| = 2/3 (or d = 0)
    const double r = sqrt(rho2 + dz2);
    double tt = atan2(dy, dx) * 0.63661977236758134308;         // 2/pi
    tt = tt < 0.0 ? tt + 4.0 : tt;
    if (a5 < a4) {
        const double z = dz / r;
        const double t1 = Nd * (0.5 + tt);
        const double t2 = 0.75 * Nd * z;
        double fa, fb;
        if (!clear_of_integer(t1 - t2, eps, fa) || !clear_of_integer(t1 + t2, eps, fb)) return false;
        const int64_t jp = (int64_t)fa, jm = (int64_t)fb;
        const int64_t k = N + 1 + jp - jm;
        const int64_t q = ((jp + jm - N + ((k & 1) ^ 1) + 1) >> 1) % (4 * N);
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
    const int64_t k = (int64_t)fp + (int64_t)fm + 1;
    double fq;
    if (!clear_of_integer(tt * (double)k, eps, fq)) return false;
    const int64_t q = ((int64_t)fq) % (4 * k);
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
