/*
 * Oracle (test infrastructure only): plain single-threaded FP64 particle loop
 * for shell binning onto HEALPix RING pixels.  Not part of the library; only
 * the tests and the bench's CPU-baseline leg load it.
 *
 * What it computes (section 2.3 eq. (5): n_p(pix, Delta chi_b) is the number of
 * particles of shell b that fall in pixel pix; section 2.4 eq. (8): shell
 * membership by comoving radius; section 2.4: HEALPix pixelisation with
 * 12*Nside^2 pixels, observer at the box centre, subvolume maps summed):
 *
 *   for every particle i and every periodic image s in {-R..R}^3
 *       d   = fl64(fl64(x_i - o) + fl64(s * L))          (per axis)
 *       b   : e_b <= |d| < e_{b+1},  b in [b0, b1)        (half-open shells)
 *       pix : HEALPix RING pixel of the direction d       (Gorski et al. 2005)
 *       counts[b - b0][pix] += 1
 *
 * Every decision is taken in FP64 only when the FP64 value lies clearly away
 * from the decision boundary (a guard band far wider than the FP64 error of
 * this code: glibc atan2 < 1 ulp, correctly rounded sqrt/division, no FMA
 * contraction).  Instances inside a guard band are not counted here; they are
 * returned in `flagged` and the Python side decides them exactly (rational
 * arithmetic, or certified high-precision evaluation).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (see build.py).
 */
#include <math.h>
#include <stdint.h>

#define HALF_PI_INV 0.63661977236758134308  /* 2/pi */

/* Relative guard on r^2 against e^2 and on 5 dz^2 against 4 rho^2. */
static const double REL_GUARD = 0x1p-40;

static int near_integer(double v, double eps)
{
    double f = floor(v);
    return (v - f) <= eps || (f + 1.0 - v) <= eps;
}

static int64_t imod(int64_t a, int64_t m)
{
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

/*
 * RING pixel of direction (dx, dy, dz), FP64 with guard bands.
 * Returns 1 and sets *pix when every decision is clear, 0 when the instance
 * must be decided exactly.
 *
 * Equatorial belt |z| <= 2/3 (z = dz/r):
 *   A = N(1/2 + tt) - (3/4) N z,  B = N(1/2 + tt) + (3/4) N z,  tt = 2 phi / pi in [0,4)
 *   jp = floor(A), jm = floor(B), ring-from-belt-top k = N + 1 + jp - jm,
 *   s = 1 if k even else 0, q = floor((jp + jm - N + s + 1)/2) mod 4N,
 *   pix = 2N(N-1) + 4N(k-1) + q.
 * Polar caps |z| > 2/3:
 *   u = tt - floor(tt), sigma = N sqrt(3(1-|z|)),
 *   k = floor(u sigma) + floor((1-u) sigma) + 1, q = floor(tt k) mod 4k,
 *   pix = 2k(k-1) + q (north) or 12N^2 - 2k(k+1) + q (south).
 */
static int fast_ring_pixel(int64_t N, double dx, double dy, double dz, int64_t *pix)
{
    const double Nd = (double)N;
    const double eps = Nd * 0x1p-40;
    double rho2 = dx * dx + dy * dy;
    double dz2 = dz * dz;
    double lhs = 5.0 * dz2, rhs = 4.0 * rho2;   /* |z| <= 2/3  <=>  5 dz^2 <= 4 rho^2 */
    if (fabs(lhs - rhs) <= REL_GUARD * (lhs + rhs))
        return 0;                               /* also catches d == 0 */
    double r = sqrt(rho2 + dz2);
    double phi = atan2(dy, dx);
    double tt = phi * HALF_PI_INV;
    if (tt < 0.0)
        tt += 4.0;

    if (lhs < rhs) {                            /* equatorial belt */
        double z = dz / r;
        double t1 = Nd * (0.5 + tt);
        double t2 = 0.75 * Nd * z;
        double A = t1 - t2, B = t1 + t2;
        if (near_integer(A, eps) || near_integer(B, eps))
            return 0;
        int64_t jp = (int64_t)floor(A);
        int64_t jm = (int64_t)floor(B);
        int64_t k = N + 1 + jp - jm;
        int64_t s = (k % 2 == 0) ? 1 : 0;
        int64_t num = jp + jm - N + s + 1;
        int64_t q = imod(num >= 0 ? num / 2 : -((-num + 1) / 2), 4 * N);
        *pix = 2 * N * (N - 1) + 4 * N * (k - 1) + q;
        return 1;
    }

    /* polar caps */
    if (near_integer(tt, eps))
        return 0;
    double u = tt - floor(tt);
    double one_minus_az = rho2 / (r * (r + fabs(dz)));
    double sigma = Nd * sqrt(3.0 * one_minus_az);
    double P = u * sigma, Q = (1.0 - u) * sigma;
    if (near_integer(P, eps) || near_integer(Q, eps))
        return 0;
    int64_t k = (int64_t)floor(P) + (int64_t)floor(Q) + 1;
    double T = tt * (double)k;
    if (near_integer(T, eps))
        return 0;
    int64_t q = imod((int64_t)floor(T), 4 * k);
    if (dz > 0.0)
        *pix = 2 * k * (k - 1) + q;
    else
        *pix = 12 * N * N - 2 * k * (k + 1) + q;
    return 1;
}

/* Exposed for the pixel-level pins. */
int oracle_fast_ring_pixel(int64_t nside, double dx, double dy, double dz, int64_t *pix)
{
    return fast_ring_pixel(nside, dx, dy, dz, pix);
}

static double load(const void *p, int is_f64, int64_t i)
{
    return is_f64 ? ((const double *)p)[i] : (double)((const float *)p)[i];
}

/*
 * Bin particles [i0, i1).  counts has (b1 - b0) rows of 12*nside^2 int64.
 * flagged receives (particle index, image code) pairs, image code =
 * ((sx+R)*(2R+1) + (sy+R))*(2R+1) + (sz+R); at most flag_cap pairs are stored,
 * the return value is the total number flagged.
 * stats[0] += instances counted here, stats[1] += particles with a non-finite
 * coordinate (skipped).  With atomic != 0 the count increments are atomic so
 * several threads may share one map.
 */
int64_t oracle_bin_fast(const void *xs, const void *ys, const void *zs, int is_f64,
                        int64_t i0, int64_t i1,
                        double ox, double oy, double oz, double L, int R,
                        const double *edges, int b0, int b1, int64_t nside,
                        int64_t *counts, int64_t *flagged, int64_t flag_cap,
                        int64_t *stats, int atomic)
{
    const int64_t npix = 12 * nside * nside;
    const int W = 2 * R + 1;
    double e2[1025];
    int64_t nflag = 0, ninst = 0, ninvalid = 0;
    for (int j = b0; j <= b1; ++j)
        e2[j - b0] = edges[j] * edges[j];
    const int nb = b1 - b0;

    for (int64_t i = i0; i < i1; ++i) {
        double x = load(xs, is_f64, i), y = load(ys, is_f64, i), z = load(zs, is_f64, i);
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
            ++ninvalid;
            continue;
        }
        double bx = x - ox, by = y - oy, bz = z - oz;
        for (int sx = -R; sx <= R; ++sx)
            for (int sy = -R; sy <= R; ++sy)
                for (int sz = -R; sz <= R; ++sz) {
                    double dx = bx + (double)sx * L;
                    double dy = by + (double)sy * L;
                    double dz = bz + (double)sz * L;
                    double r2 = dx * dx + dy * dy + dz * dz;
                    /* outside the range by more than the guard: no shell, no flag */
                    if (r2 < e2[0] * (1.0 - 2.0 * REL_GUARD) || r2 > e2[nb] * (1.0 + 2.0 * REL_GUARD))
                        continue;
                    int flag = 0, b = -1;
                    /* plain linear scan over the edges of [b0, b1] */
                    for (int j = 0; j <= nb; ++j) {
                        if (fabs(r2 - e2[j]) <= REL_GUARD * e2[j]) {
                            flag = 1;
                            break;
                        }
                        if (e2[j] <= r2)
                            b = j;
                    }
                    if (!flag && (b < 0 || b >= nb))
                        continue;                       /* outside [e_b0, e_b1) */
                    int64_t pix = 0;
                    if (!flag && !fast_ring_pixel(nside, dx, dy, dz, &pix))
                        flag = 1;
                    if (flag) {
                        if (nflag < flag_cap) {
                            flagged[2 * nflag] = i;
                            flagged[2 * nflag + 1] = ((int64_t)(sx + R) * W + (sy + R)) * W + (sz + R);
                        }
                        ++nflag;
                        continue;
                    }
                    int64_t *cell = counts + (int64_t)b * npix + pix;
                    if (atomic)
                        __atomic_fetch_add(cell, 1, __ATOMIC_RELAXED);
                    else
                        ++*cell;
                    ++ninst;
                }
    }
    if (atomic) {
        __atomic_fetch_add(&stats[0], ninst, __ATOMIC_RELAXED);
        __atomic_fetch_add(&stats[1], ninvalid, __ATOMIC_RELAXED);
    } else {
        stats[0] += ninst;
        stats[1] += ninvalid;
    }
    return nflag;
}

/*
 * Per-shell instance totals (section 2.4 eq. (8) alone, no pixelisation):
 * totals[b - b0] += number of instances of particles [i0, i1) with
 * e_b <= |d| < e_{b+1}.  Instances whose r^2 lies within the relative guard of
 * an edge are not counted; they are returned in `flagged` (as in
 * oracle_bin_fast) for an exact decision.  Returns the number flagged;
 * stats[1] += particles with a non-finite coordinate.
 */
int64_t oracle_shell_totals(const void *xs, const void *ys, const void *zs, int is_f64,
                            int64_t i0, int64_t i1,
                            double ox, double oy, double oz, double L, int R,
                            const double *edges, int b0, int b1,
                            int64_t *totals, int64_t *flagged, int64_t flag_cap,
                            int64_t *stats, int atomic)
{
    const int W = 2 * R + 1;
    double e2[1025];
    int64_t nflag = 0, ninvalid = 0;
    for (int j = b0; j <= b1; ++j)
        e2[j - b0] = edges[j] * edges[j];
    const int nb = b1 - b0;
    int64_t local[1024];
    for (int j = 0; j < nb; ++j)
        local[j] = 0;

    for (int64_t i = i0; i < i1; ++i) {
        double x = load(xs, is_f64, i), y = load(ys, is_f64, i), z = load(zs, is_f64, i);
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
            ++ninvalid;
            continue;
        }
        double bx = x - ox, by = y - oy, bz = z - oz;
        for (int sx = -R; sx <= R; ++sx)
            for (int sy = -R; sy <= R; ++sy)
                for (int sz = -R; sz <= R; ++sz) {
                    double dx = bx + (double)sx * L;
                    double dy = by + (double)sy * L;
                    double dz = bz + (double)sz * L;
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < e2[0] * (1.0 - 2.0 * REL_GUARD) || r2 > e2[nb] * (1.0 + 2.0 * REL_GUARD))
                        continue;
                    int flag = 0, b = -1;
                    for (int j = 0; j <= nb; ++j) {
                        if (fabs(r2 - e2[j]) <= REL_GUARD * e2[j]) {
                            flag = 1;
                            break;
                        }
                        if (e2[j] <= r2)
                            b = j;
                    }
                    if (flag) {
                        if (nflag < flag_cap) {
                            flagged[2 * nflag] = i;
                            flagged[2 * nflag + 1] = ((int64_t)(sx + R) * W + (sy + R)) * W + (sz + R);
                        }
                        ++nflag;
                    } else if (b >= 0 && b < nb) {
                        ++local[b];
                    }
                }
    }
    for (int j = 0; j < nb; ++j) {
        if (atomic)
            __atomic_fetch_add(&totals[j], local[j], __ATOMIC_RELAXED);
        else
            totals[j] += local[j];
    }
    if (atomic)
        __atomic_fetch_add(&stats[1], ninvalid, __ATOMIC_RELAXED);
    else
        stats[1] += ninvalid;
    return nflag;
}
