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
// below ~16 N 2^-46 for tt < 4, |z| <= 1: a few roundings, the refined
// reciprocals below and the azimuth polynomial)
UFX_HD double floor_margin(double Nd) { return Nd * 0x1p-38; }

// 1/sqrt(x) and 1/x for positive normal x: the hardware estimate refined by one
// Newton step, which squares its relative error.  The estimates are good to
// 2^-23.2 (rsq) and 2^-24.4 (rcp), measured over 2^24 seeded inputs spanning
// 121 binades on gfx950, so the refined values are good to ~2^-46; even an
// estimate of only 2^-20 would leave ~2^-40, inside the floor margin.  A host
// build uses the IEEE values as the estimates, or, in a test build that defines
// UFX_HOST_ESTIMATE_MODEL, estimates with a relative error the test sets, so
// that the refinement and the margin are checked on the CPU too.
#if !defined(__HIP_DEVICE_COMPILE__) && defined(UFX_HOST_ESTIMATE_MODEL)
double host_rsq_estimate(double x);
double host_rcp_estimate(double x);
#endif

UFX_FN double rsq_estimate(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsq(x);
#elif defined(UFX_HOST_ESTIMATE_MODEL)
    return host_rsq_estimate(x);
#else
    return 1.0 / sqrt(x);
#endif
}

UFX_FN double rcp_estimate(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcp(d);
#elif defined(UFX_HOST_ESTIMATE_MODEL)
    return host_rcp_estimate(d);
#else
    return 1.0 / d;
#endif
}

UFX_FN double rsqrt_nr(double x) {
    const double y = rsq_estimate(x);
    const double e = fma(-(x * y), y, 1.0);  // 1 - x y^2
    return fma(0.5 * e, y, y);
}

UFX_FN double rcp_nr(double d) {
    const double r = rcp_estimate(d);
    const double e = fma(-d, r, 1.0);  // 1 - d r
    return fma(r, e, r);
}

// Product of two operands in [0, 2^24) whose product fits 32 bits (the pixel
// index terms, N <= 8192): one full-rate 24-bit multiply on the device.
UFX_FN int32_t mul24(int32_t a, int32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return (int32_t)__umul24((unsigned)a, (unsigned)b);
#else
    return a * b;
#endif
}

// floor(v), and whether v lies more than eps from both integers around it.  The
// callers' arguments are >= 0 (a negative rounding residue fails the test), so
// v - floor(v) is exact.
UFX_FN bool clear_of_integer(double v, double eps, double &fl) {
    fl = floor(v);
    const double frac = v - fl;
    return frac > eps && frac < 1.0 - eps;
}

// tt = 2 phi / pi in [0, 4] for phi = atan2(dy, dx) taken in [0, 2 pi).
// One reciprocal reduces the azimuth to an octant: with mn = min(|dx|,|dy|),
// mx = max(|dx|,|dy|), u = mn/mx, or u = (mn - mx)/(mn + mx) plus a quarter of a
// quadrant when mn/mx > tan(pi/8), so |u| <= tan(pi/8); then
// (2/pi) atan(u) = u P(u^2) with P of degree 9 (gen_tt_poly.py: relative error
// < 1e-15 before rounding).  The absolute error of tt stays below ~2e-15, far
// inside the floor margin N 2^-38.  tt may round to 4.0 just below the +x axis;
// the guard band catches it.
// Coefficients of P, constant term first (gen_tt_poly.py).
constexpr int kTtTerms = 10;
constexpr double kTtCoef[kTtTerms] = {
    0.6366197723675807,   -0.21220659078848142, 0.1273239543359597,   -0.09094567142790448, 0.07073513392040226,
    -0.05786574491875008, 0.04885124377544614,  -0.041418373955876615, 0.0319886291636091,  -0.016116971463406102};

// `c` holds kTtCoef (the device code passes a copy in LDS, read through a
// volatile pointer: every use is a fresh load the FMA may overwrite, so no
// registers stay pinned to constants).
template <typename CoefPtr>
UFX_FN double fast_tt_c(double dx, double dy, CoefPtr c) {
    const double ax = fabs(dx), ay = fabs(dy);
    const double mn = ax < ay ? ax : ay;
    const double mx = ax < ay ? ay : ax;
    const bool upper = mn > 0.4142 * mx;
    const double num = upper ? mn - mx : mn;
    const double den = upper ? mn + mx : mx;
    const double u = num * rcp_nr(den);  // den is normal whenever the caller accepts (else NaN, rejected)
    const double s = u * u;
    double p = c[kTtTerms - 1];
    for (int k = kTtTerms - 2; k >= 0; --k) p = fma(p, s, c[k]);
    const double th = fma(u, p, upper ? 0.5 : 0.0);  // quarter turns of atan(mn/mx), in [0, 1/2]
    // The angle of (|dx|, |dy|) is th, or 1 - th when |dy| > |dx|; the quadrant
    // maps it to a, 2 - a, 2 + a or 4 - a.  Together: tt = o + s th with an
    // integer o in 0..4 and s = +-1, one rounding.
    const bool nx = dx < 0.0, ny = dy < 0.0, swap = ay > ax;
    const int o = (nx ? 2 : (ny ? 4 : 0)) + (swap ? (nx == ny ? 1 : -1) : 0);
    const bool neg = (nx != ny) != swap;
    return (double)o + (neg ? -th : th);
}

UFX_FN double fast_tt(double dx, double dy) { return fast_tt_c(dx, dy, kTtCoef); }

// Returns true and the pixel when every decision is clear of its boundary, for
// a direction already known to lie in the belt (kBelt: 5 dz^2 < 4 rho^2, i.e.
// |z| < 2/3) or in a cap; a direction of the other region, or near |z| = 2/3,
// is deferred.  Pixel arithmetic is 32-bit: 12 N^2 < 2^31 for N <= 8192.
//
// With y = 1/|d| (refined reciprocal square root): z = dz y in the belt, and in
// the caps 1 - |z| = rho^2 / (r (r + |dz|)) = rho^2 y^2 / (1 + |z|), which has no
// cancellation near the poles.  Vectors so short that a reciprocal would leave
// the normal range (|d|^2 <= 2^-600 or dx^2 + dy^2 <= 2^-1000) are deferred.
// No data-dependent branches: rejected lanes may carry NaN or infinities, which
// every integer conversion masks with the acceptance flag.
template <bool kBelt, typename CoefPtr>
UFX_FN bool fast_ring_pixel_region(int32_t N, double Nd, double eps, double dx, double dy, double dz, int32_t &pix,
                                   CoefPtr tt_coef) {
    const double rho2 = dx * dx + dy * dy;
    const double dz2 = dz * dz;
    const double r2 = rho2 + dz2;
    const double a5 = 5.0 * dz2, a4 = 4.0 * rho2;
    const bool region = (a5 < a4) == kBelt;
    const bool away = fabs(a5 - a4) > kRelGuard * (a5 + a4);  // not near |z| = 2/3 (nor d = 0)
    // rho^2 > 2^-1000 keeps max(|dx|, |dy|) > 2^-500.5, the azimuth's divisor in range
    bool ok = region && away && r2 > 0x1p-600 && rho2 > 0x1p-1000;
    const double y = rsqrt_nr(r2);                              // 1 / |d| (rejected lanes may carry NaN)
    const double tt = fast_tt_c(dx, dy, tt_coef);
    const double z = dz * y;
    if (kBelt) {
        const double t1 = Nd * (0.5 + tt);
        const double t2 = 0.75 * Nd * z;
        double fa, fb;
        ok = ok & clear_of_integer(t1 - t2, eps, fa);
        ok = ok & clear_of_integer(t1 + t2, eps, fb);
        const int32_t jp = (int32_t)(ok ? fa : 0.0), jm = (int32_t)(ok ? fb : 0.0);
        const int32_t k = N + 1 + jp - jm;                              // ring below z = 2/3, 1 .. 2N+1
        int32_t q = (jp + jm - N + ((k & 1) ^ 1) + 1) >> 1;             // 0 .. 4N+1
        q = q >= 4 * N ? q - 4 * N : q;
        pix = 2 * N * (N - 1) + mul24(4 * N, k - 1) + q;
    } else {
        const double om = rho2 * y * y * rcp_nr(1.0 + fabs(z));       // 1 - |z|
        double ftt;
        ok = ok & clear_of_integer(tt, eps, ftt);
        const double u = tt - ftt;
        const double om3 = 3.0 * om;                                  // sqrt(om3) = om3 / sqrt(om3)
        const double sig = Nd * (om3 * rsqrt_nr(om3));              // om3 > 0 when rho^2 > 0
        double fa, fb;
        ok = ok & clear_of_integer(u * sig, eps, fa);
        ok = ok & clear_of_integer((1.0 - u) * sig, eps, fb);
        const int32_t k = (int32_t)(ok ? fa : 0.0) + (int32_t)(ok ? fb : 0.0) + 1;  // ring from the pole, 1 .. N
        double fq;
        ok = ok & clear_of_integer(tt * (double)k, eps, fq);
        int32_t q = (int32_t)(ok ? fq : 0.0);                          // 0 .. 4k-1 when clear
        q = q >= 4 * k ? q - 4 * k : q;
        // north 2k(k-1) + q, south 12N^2 - 2k(k+1) + q: one product, no branch
        const bool north = dz > 0.0;
        const int32_t p2 = mul24(2 * k, north ? k - 1 : k + 1);
        pix = (north ? p2 : 12 * N * N - p2) + q;
    }
    return ok;
}

// The same for any direction: the region is read off the vector.
UFX_FN bool fast_ring_pixel(int32_t N, double Nd, double eps, double dx, double dy, double dz, int32_t &pix) {
    const double rho2 = dx * dx + dy * dy;
    const double dz2 = dz * dz;
    return 5.0 * dz2 < 4.0 * rho2 ? fast_ring_pixel_region<true>(N, Nd, eps, dx, dy, dz, pix, kTtCoef)
                                  : fast_ring_pixel_region<false>(N, Nd, eps, dx, dy, dz, pix, kTtCoef);
}

// Squared-edge sentinels: e2[-2], e2[-1] = -kEdgeSentinel and e2[nb+1], e2[nb+2] =
// +kEdgeSentinel make the guard tests at the ends of the range vacuous.
constexpr double kEdgeSentinel = 1e300;
constexpr int kShellTabMax = 1024;  // cells of the shell lookup table, at most

// The shell holding r^2 = x: (number of e2[0..nb] that are <= x) - 1, by binary search.
UFX_HD int shell_of_r2(const double *e2, int nb, int steps, double x) {
    int lo = 0;
    for (int s = steps; s >= 0; --s) {
        const int probe = lo + (1 << s);
        if (probe <= nb + 1 && e2[probe - 1] <= x) lo = probe;
    }
    return lo - 1;
}

// Cells of the lookup table over r^2 in [lo2, hi2): the fewest (a power of two
// <= kShellTabMax) for which consecutive squared edges lie at least two cells
// apart; 0 when there are none (then the binary search is used).
UFX_HD int shell_table_cells(const double *e2, int nb, double lo2, double hi2) {
    double gap = kEdgeSentinel;
    for (int j = 0; j < nb; ++j) gap = e2[j + 1] - e2[j] < gap ? e2[j + 1] - e2[j] : gap;
    const double span = hi2 - lo2;
    if (!(span > 0.0)) return 0;
    for (int g = 64; g <= kShellTabMax; g *= 2)
        if (2.0 * span / g <= gap) return g;
    return 0;
}

// Entry of the shell lookup table for the cell [a, b) of r^2: the shell holding
// r^2 = a (plus one, so that -1 is stored as 0) in the low 12 bits, and in bits
// 12-13 which edge lies within delta of the cell, if any: 1 for e2[base + 1]
// (inside the cell or just past its end), 2 for e2[base] (just below its
// start), 0 for none.  delta = 2^-24 cells + 2^-30 |b| covers the rounding of
// the cell index of r^2 and every guard band (2^-38 relative); consecutive
// edges being two cells apart, at most one edge is within delta of a cell.
UFX_HD int16_t shell_table_entry(const double *e2, int nb, int steps, double a, double b) {
    const int base = shell_of_r2(e2, nb, steps, a);
    const double delta = 0x1p-24 * (b - a) + 0x1p-30 * fabs(b);
    int which = 0;
    if (base + 1 <= nb && e2[base + 1] <= b + delta) which = 1;
    else if (base >= 0 && e2[base] >= a - delta) which = 2;
    return (int16_t)((base + 1) | (which << 12));
}

// Largest j in [-1, nb] with e2[j] <= r2 (e2 ascending, indexable from -2 to
// nb + 2 with the sentinels above); *clear is false when r2 is within the
// relative guard of e2[j] or e2[j+1].  With a table (tab_n > 0) of tab_n equal
// cells of r^2 from tab_lo (cell width 1/tab_scale; entries from
// shell_table_entry), the cell's entry gives the shell of its start and the one
// edge that can be near r^2: one comparison with that edge decides the shell and
// the guard (every other edge is farther than any guard band from the cell).
UFX_FN int fast_shell(const double *e2, int nb, int steps, const int16_t *tab, int tab_n, double tab_lo,
                      double tab_scale, double r2, bool &clear) {
    if (tab_n > 0) {
        const double cf = fmin(fmax((r2 - tab_lo) * tab_scale, 0.0), (double)(tab_n - 1));
        const int t = tab[(int)cf];
        const int base1 = t & 0xFFF, which = t >> 12;
        const int k = which == 2 ? base1 - 1 : base1;  // the near edge (any valid index when none)
        const double ek = e2[k];
        const bool up = r2 >= ek;
        clear = which == 0 || fabs(r2 - ek) > kRelGuard * ek;
        return which == 0 ? base1 - 1 : (up ? k : k - 1);
    }
    const int j = shell_of_r2(e2, nb, steps, r2);
    const double elo = e2[j], ehi = e2[j + 1];
    const bool clear_lo = fabs(r2 - elo) > kRelGuard * elo;
    const bool clear_hi = fabs(r2 - ehi) > kRelGuard * ehi;
    clear = clear_lo && clear_hi;
    return j;
}

}  // namespace ufx
