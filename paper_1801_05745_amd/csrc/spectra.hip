// Spherical-harmonic analysis of HEALPix RING maps, angular power spectra and
// their covariance over realisations (section 3.1 eq. (9); section 3.2
// eqs. (10) and (11)); synthesis with a Gaussian beam and the one-point
// moments of the smoothed maps (section 3.3 eqs. (12) and (13)).
//
// a_lm = (4 pi / N_pix) sum_p map_p lambda_lm(z_p) e^{-i m phi_p}: the pixel
// quadrature that ANAFAST evaluates without iterative refinement.  Pixels of
// one ring share z, so the sum factors into
//   1. ring sums   F_r(m) = sum_j map_j e^{-i m phi_j},  phi_j = pi (2j + s_r)/n_r,
//   2. a Legendre contraction over rings at each m, using lambda_lm(-z) =
//      (-1)^{l+m} lambda_lm(z) to fold ring i and its mirror 4N - i into
//      E = F_i + F_mirror (l+m even) and O = F_i - F_mirror (l+m odd).
// Everything is FP64.  Reductions run in a fixed order, so results are
// bitwise reproducible.
//
// Kernels:
//   ring_dft_kernel     ring DFTs by one radix-4 decimation (every ring holds
//                       4 n4 pixels): one lane per k' < n4/K (K output classes),
//                       RG rings of equal length per workgroup, the map chunk
//                       staged in LDS (FP32 or FP64 in, FP64 out) and read as
//                       broadcasts;
//   lambda_seed_kernel  lambda_mm(z) of every ring pair for m = 0..lmax, carried
//                       as value * 2^{-600 k} so sin^m(theta) cannot underflow,
//                       one wave per segment of m;
//   legendre_kernel     one workgroup per (m, block of kLegThreads R ring pairs):
//                       the three-term recurrence in l, R pairs per lane, partial
//                       sums over C consecutive l reduced through LDS;
//   alm2cl              fixed-order reductions;
//   cov_kernel          the covariance of spectra over realisations on the FP64
//                       matrix cores;
//   legendre_synth_kernel, ring_idft_kernel   the synthesis: per m and ring pair
//                       E and O of the beam-weighted a_lm, then the aliasing folds
//                       and the inverse ring transforms;
//   moments_*           mean, then the central moments, in fixed-size blocks.
#include "../../include/ufalcon.h"
#include "internal.hpp"

#include <type_traits>

namespace ufx {
namespace {

constexpr int kDftThreads = 256;
constexpr int kDftJ = 64;      // pixels per staged chunk (and twiddle re-seed period)
constexpr int kDftShort = 64;  // polar rings up to this n4 write their aliased outputs with the whole workgroup
constexpr int kFoldBatch = 4;  // loads in flight per step of the inverse transform's folds
constexpr int kEqRings = 4;    // equatorial rings (all 4N long) per workgroup
constexpr int kEqRingsSplit = 2;  // the same with the even/odd split of the outputs
constexpr int kLegThreads = 128;
constexpr int kLegR = 4;       // ring pairs per lane
constexpr int kLegC = 8;       // l values per reduction chunk
constexpr int kLegStage = kLegThreads < 128 ? kLegThreads : 128;  // l values per coefficient stage in LDS
constexpr int kLegBufs = 2;    // reduction buffers: a chunk's sums are read while the next chunk fills the other
constexpr int kLegLanes = kLegThreads / (2 * kLegC);  // lanes summing one output
static_assert(kLegLanes * 2 * kLegC == kLegThreads && (kLegLanes & (kLegLanes - 1)) == 0, "reduction layout");
static_assert(kLegStage % kLegC == 0 && kLegStage / kLegC >= 2, "coefficient stages");
constexpr double kScaleUp = 0x1p600;
constexpr double kScaleDown = 0x1p-600;
constexpr double kTiny = 0x1p-300;
constexpr double kBig = 0x1p300;

// Ring i = 1 .. 4N-1 (RING scheme, Gorski et al. 2005).
__host__ __device__ __forceinline__ int64_t ring_first(int64_t N, int64_t i) {
    if (i < N) return 2 * i * (i - 1);
    if (i <= 3 * N) return 2 * N * (N - 1) + 4 * N * (i - N);
    const int64_t ii = 4 * N - i;
    return 12 * N * N - 2 * ii * (ii + 1);
}
// phi_j = pi (2j + s)/n
__host__ __device__ __forceinline__ int ring_shift(int64_t N, int64_t i) {
    if (i < N || i > 3 * N) return 1;
    return ((i - N) & 1) == 0 ? 1 : 0;
}
// z and sin(theta) of a northern ring i <= 2N from integer numerators: each
// z is one correctly rounded division.
__device__ __forceinline__ void ring_z_sin(int64_t N, int64_t i, double &z, double &st) {
    if (i < N) {
        const double d = (double)(3 * N * N);
        z = (double)(3 * N * N - i * i) / d;
        st = (double)i * sqrt((double)(6 * N * N - i * i)) / d;
    } else {
        const double d = (double)(3 * N);
        z = (double)(4 * N - 2 * i) / d;
        st = sqrt((double)((2 * i - N) * (7 * N - 2 * i))) / d;
    }
}

// ------------------------------------------------------------------ ring sums
// Every ring has n = 4 n4 pixels, so its DFT splits by decimation into four
// DFTs of length n4 over the pixels j = 4j' + q:
//   D_q[k'] = sum_{j'} x[4j' + q] e^{-2 pi i k' j' / n4},          k' < n4
//   DFT[k' + t n4] = sum_q (-i)^{t q} e^{-2 pi i k' q / n} D_q[k'],   t = 0..3
// and F(m) = e^{-i pi m s / n} DFT[m mod n] (aliasing for m >= n).  Lane k'
// accumulates D_0..D_3 of RG rings of equal length (the twiddle advancing by
// one complex multiply per j', re-seeded exactly every kDftJ steps), then
// writes F(m) for every m = k' + t n4 + u n <= lmax.  With K output classes
// (K = 2 when n4 is even, 4 when 4 | n4; equatorial rings), lane k' < n4/K
// also yields D_q[k' + s n4/K]: the sums over the classes of j' mod K are kept
// apart (for K = 2, D_q[k'] = E + O and D_q[k' + n4/2] = E - O), so every
// product x w serves K outputs and each LDS read K times as many.

// F(m) of one ring from its four D_q[kp].
// With gs (short rings), G(k) goes to gs[k] instead, and the workgroup writes
// the aliased F(m) afterwards (ring_dft_spread).
__device__ __forceinline__ void ring_dft_outputs(const double (&ar)[4], const double (&ai)[4], int64_t kp, int64_t n4,
                                                 bool shift, int64_t col, int64_t nring, int32_t lmax,
                                                 double2 *__restrict__ F, double2 *gs = nullptr) {
    const int64_t n = 4 * n4;
    // e^{-2 pi i k' q / n}, q = 1, 2, 3
    double s1, c1;
    sincospi(-2.0 * (double)kp / (double)n, &s1, &c1);
    const double c2 = c1 * c1 - s1 * s1, s2 = 2.0 * c1 * s1;
    const double c3 = c2 * c1 - s2 * s1, s3 = c2 * s1 + s2 * c1;
    const double a0r = ar[0], a0i = ai[0];
    const double a1r = ar[1] * c1 - ai[1] * s1, a1i = ar[1] * s1 + ai[1] * c1;
    const double a2r = ar[2] * c2 - ai[2] * s2, a2i = ar[2] * s2 + ai[2] * c2;
    const double a3r = ar[3] * c3 - ai[3] * s3, a3i = ar[3] * s3 + ai[3] * c3;
    // radix-4 butterfly, (-i)(x + iy) = y - ix
    double dr[4], di[4];
    dr[0] = (a0r + a2r) + (a1r + a3r);
    di[0] = (a0i + a2i) + (a1i + a3i);
    dr[2] = (a0r + a2r) - (a1r + a3r);
    di[2] = (a0i + a2i) - (a1i + a3i);
    dr[1] = (a0r - a2r) + (a1i - a3i);
    di[1] = (a0i - a2i) - (a1r - a3r);
    dr[3] = (a0r - a2r) - (a1i - a3i);
    di[3] = (a0i - a2i) + (a1r - a3r);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t k = kp + t * n4;  // k < n
        if (k > lmax) break;
        double gr = dr[t], gi = di[t];
        if (shift) {  // e^{-i pi k / n}
            double s, c;
            sincospi(-(double)k / (double)n, &s, &c);
            gr = dr[t] * c - di[t] * s;
            gi = dr[t] * s + di[t] * c;
        }
        if (gs) {
            gs[k] = make_double2(gr, gi);
            continue;
        }
        // F(k + u n) = (-1)^{u s} G(k)
        for (int64_t m = k, u = 0; m <= lmax; m += n, ++u) {
            const double sg = (shift && (u & 1)) ? -1.0 : 1.0;
            F[m * nring + col] = make_double2(sg * gr, sg * gi);
        }
    }
}

// F(m) = (-1)^{u s} G(m - u n), u = m / n, for every m <= lmax, one m per thread:
// a short ring has few lanes and lmax / n aliases per k, too many for one lane.
__device__ __forceinline__ void ring_dft_spread(const double2 *gs, int64_t n, bool shift, int64_t col, int64_t nring,
                                                int32_t lmax, double2 *__restrict__ F) {
    for (int64_t m = threadIdx.x; m <= lmax; m += kDftThreads) {
        const int64_t u = m / n;
        const double2 g = gs[m - u * n];
        const double sg = (shift && (u & 1)) ? -1.0 : 1.0;
        F[m * nring + col] = make_double2(sg * g.x, sg * g.y);
    }
}

// K output classes: lane k' < n4/K yields D_q[k' + s n4/K], s < K, from the
// sums over j' = h mod K kept apart (E_h): D_q[k' + s n4/K] =
// sum_h e^{-2 pi i s h / K} E_h, the factors +-1 for K = 2 and also +-i for K = 4.
template <typename T, bool kPolar, int K>
__global__ __launch_bounds__(kDftThreads) void ring_dft_kernel(const T *__restrict__ map, int64_t N, int32_t lmax,
                                                               double2 *__restrict__ F) {
    static_assert(K == 1 || K == 2 || (K == 4 && !kPolar), "output classes");
    constexpr bool kSplit = K > 1;
    constexpr int RG = kPolar ? 2 : (K == 4 ? 1 : (K == 2 ? kEqRingsSplit : kEqRings));
    constexpr int H = K;  // accumulators per output: one per class of j'
    __shared__ double xs[RG][4][kDftJ];
    __shared__ double2 gsm[kPolar ? RG : 1][kPolar ? 4 * kDftShort : 1];  // G(k) of short polar rings
    const int64_t nring = 4 * N - 1;
    int64_t ring[RG];
    bool valid[RG];
    int64_t n4;
    if (kPolar) {
        // the even (K = 2) or odd (K = 1) polar rings i < N, the longest first so
        // that the short ones fill the tail of the launch
        const int64_t imax = ((N - 1) % 2 == (kSplit ? 0 : 1)) ? N - 1 : N - 2;
        const int64_t i = imax - 2 * (int64_t)blockIdx.y;
        ring[0] = i;
        ring[RG - 1] = 4 * N - i;
        valid[0] = valid[RG - 1] = true;
        n4 = i;
    } else {
        const int64_t i0 = N + (int64_t)blockIdx.y * RG;
#pragma unroll
        for (int g = 0; g < RG; ++g) {
            valid[g] = i0 + g <= 3 * N;
            ring[g] = valid[g] ? i0 + g : 3 * N;
        }
        n4 = N;
    }
    const int64_t nk = n4 / K;                                // lanes needed
    if ((int64_t)blockIdx.x * kDftThreads >= nk) return;  // whole workgroup past this ring length
    const int64_t kp = (int64_t)blockIdx.x * kDftThreads + threadIdx.x;  // k'
    int64_t first[RG];
#pragma unroll
    for (int g = 0; g < RG; ++g) first[g] = ring_first(N, ring[g]);

    double ar[H][RG][4], ai[H][RG][4];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int q = 0; q < 4; ++q) ar[h][g][q] = ai[h][g][q] = 0.0;
    double ws, wc;  // step e^{-2 pi i k' / n4}
    sincospi(-2.0 * (double)(kp % n4) / (double)n4, &ws, &wc);

    for (int64_t jb = 0; jb < n4; jb += kDftJ) {
        const int cnt = (int)(n4 - jb < kDftJ ? n4 - jb : kDftJ);  // a multiple of K
        for (int e = threadIdx.x; e < RG * 4 * kDftJ; e += kDftThreads) {
            const int g = e / (4 * kDftJ), r = e % (4 * kDftJ);  // r = 4 jj + q: pixels in order
            const int jj = r / 4, q = r % 4;
            xs[g][q][jj] = jj < cnt ? (double)map[first[g] + 4 * jb + r] : 0.0;
        }
        __syncthreads();
        double wr, wi;
        sincospi(-2.0 * (double)((kp * jb) % n4) / (double)n4, &wi, &wr);
        for (int jj = 0; jj < cnt; jj += H) {
#pragma unroll
            for (int h = 0; h < H; ++h) {  // jb is a multiple of K, so j' = h mod K
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double x = xs[g][q][jj + h];
                        ar[h][g][q] = fma(x, wr, ar[h][g][q]);
                        ai[h][g][q] = fma(x, wi, ai[h][g][q]);
                    }
                const double nr = fma(wr, wc, -(wi * ws));
                const double ni = fma(wr, ws, wi * wc);
                wr = nr;
                wi = ni;
            }
        }
        __syncthreads();
    }
    // polar rings of at most kDftShort pixels per quarter: G(k) through LDS, then
    // the aliased outputs with the whole workgroup (uniform over the workgroup)
    const bool short_ring = kPolar && n4 <= kDftShort;
#pragma unroll
    for (int g = 0; g < RG; ++g) {
        if (!valid[g] || kp >= nk) continue;
        const bool shift = ring_shift(N, ring[g]) != 0;
        const int64_t col = ring[g] - 1;
        if constexpr (K == 4) {
            // D_q[k' + s n4/4] = sum_h (-i)^{s h} E_h, in h order; (-i)(x + iy) = y - ix
#pragma unroll
            for (int sc = 0; sc < 4; ++sc) {
                double dr[4], di[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    double vr = 0.0, vi = 0.0;
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        const int e = (sc * h) & 3;
                        const double xr = ar[h][g][q], xi = ai[h][g][q];
                        vr += e == 0 ? xr : (e == 1 ? xi : (e == 2 ? -xr : -xi));
                        vi += e == 0 ? xi : (e == 1 ? -xr : (e == 2 ? -xi : xr));
                    }
                    dr[q] = vr;
                    di[q] = vi;
                }
                ring_dft_outputs(dr, di, kp + sc * (n4 / 4), n4, shift, col, nring, lmax, F);
            }
        } else if (kSplit) {
            double lo_r[4], lo_i[4], hi_r[4], hi_i[4];  // D_q[k'] = E + O, D_q[k' + n4/2] = E - O
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                lo_r[q] = ar[0][g][q] + ar[H - 1][g][q];
                lo_i[q] = ai[0][g][q] + ai[H - 1][g][q];
                hi_r[q] = ar[0][g][q] - ar[H - 1][g][q];
                hi_i[q] = ai[0][g][q] - ai[H - 1][g][q];
            }
            double2 *gs = short_ring ? gsm[kPolar ? g : 0] : nullptr;
            ring_dft_outputs(lo_r, lo_i, kp, n4, shift, col, nring, lmax, F, gs);
            ring_dft_outputs(hi_r, hi_i, kp + n4 / 2, n4, shift, col, nring, lmax, F, gs);
        } else {
            ring_dft_outputs(ar[0][g], ai[0][g], kp, n4, shift, col, nring, lmax, F,
                             short_ring ? gsm[kPolar ? g : 0] : nullptr);
        }
    }
    if (kPolar && short_ring) {
        __syncthreads();
#pragma unroll
        for (int g = 0; g < RG; ++g)
            ring_dft_spread(gsm[kPolar ? g : 0], 4 * n4, ring_shift(N, ring[g]) != 0, ring[g] - 1, nring, lmax, F);
    }
}

// ------------------------------------------------------------------ lambda_mm seeds
// lambda_mm = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1}, kept as v 2^{-600 k}
// with v >= 2^-300.  A workgroup holds 64 ring pairs (one per lane) and
// kSeedSegs waves; wave w owns the values of m in its segment.  Each wave first
// forms the product of its segment's factors (rescaled the same way), the
// products of the earlier segments then give its start value, and it runs the
// segment again writing (v, k) for every m.
constexpr int kSeedSegs = 16;
__device__ __forceinline__ double seed_factor(int m, double st) {
    return -sqrt((double)(2 * m + 3) / (double)(2 * m + 2)) * st;  // lambda_mm -> lambda_{m+1,m+1}
}
// Bring v back into [2^-300, 2^300) (the window the step-by-step product keeps):
// up while it is below, down while it is at or above and k > 0 (the product of
// two values of the window can reach 2^600).
__device__ __forceinline__ void seed_rescale(double &v, int32_t &k) {
    while (v != 0.0 && fabs(v) < kTiny) {
        v *= kScaleUp;
        ++k;
    }
    while (k > 0 && fabs(v) >= kBig) {
        v *= kScaleDown;
        --k;
    }
}
__global__ __launch_bounds__(64 * kSeedSegs) void lambda_seed_kernel(int64_t N, int32_t lmax, double *__restrict__ seed,
                                                                    int32_t *__restrict__ seed_k) {
    __shared__ double prod[kSeedSegs][64];
    __shared__ int32_t pexp[kSeedSegs][64];
    __shared__ double fac[kSeedSegs][64];  // the next 64 factors of each segment, shared by the 64 rings
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t npair = 2 * N;
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    double z = 0.0, st = 0.0;
    if (p < npair) ring_z_sin(N, p + 1, z, st);
    const int len = (lmax + 1 + kSeedSegs - 1) / kSeedSegs;
    const int m0 = w * len, m1 = min(m0 + len, lmax + 1);
    // f(i0 .. i0 + 63) of this wave's segment into fac[w]; the same trip count in every wave
    auto stage = [&](int i0) {
        __syncthreads();
        const int m = m0 + i0 + lane;
        fac[w][lane] = m < m1 ? seed_factor(m, 1.0) : 1.0;
        __syncthreads();
        return max(0, min(64, m1 - (m0 + i0)));
    };
    // the factors taking lambda_{m0,m0} to lambda_{m1,m1}
    double pv = 1.0;
    int32_t pk = 0;
    for (int i0 = 0; i0 < len; i0 += 64) {
        const int cnt = stage(i0);
        for (int c = 0; c < cnt; ++c) {
            pv *= fac[w][c] * st;
            seed_rescale(pv, pk);
        }
    }
    prod[w][lane] = pv;
    pexp[w][lane] = pk;
    __syncthreads();
    double v = 0.28209479177387814;  // lambda_00 = 1/sqrt(4 pi)
    int32_t k = 0;
    for (int j = 0; j < w; ++j) {
        v *= prod[j][lane];
        k += pexp[j][lane];
        seed_rescale(v, k);
    }
    for (int i0 = 0; i0 < len; i0 += 64) {
        const int cnt = stage(i0);
        if (p >= npair) continue;
        for (int c = 0; c < cnt; ++c) {
            const int64_t idx = (int64_t)(m0 + i0 + c) * npair + p;
            seed[idx] = v;
            seed_k[idx] = k;
            v *= fac[w][c] * st;
            seed_rescale(v, k);
        }
    }
}

// Recurrence coefficients per (m, l), packed like a_lm.  With
// c_l = sqrt((4l^2 - 1)/(l^2 - m^2)) (c_{m+1} = sqrt(2m+3)), the recurrence
// lambda_l = c_l z lambda_{l-1} - (c_l / c_{l-1}) lambda_{l-2} is run on
// mu_l = lambda_l / sigma_l, sigma_l = prod of c_j from the start l0 of the
// l-chunk (chunks of kLegC from m) to l:
//   mu_l = z mu_{l-1} - g_l mu_{l-2},   g_l = 1 / c_{l-1}^2,
// and the state (mu_{l-2}, mu_{l-1}) passes to the next chunk multiplied by
// sigma at the chunk's last l.  Entry (g_l, sigma_l); at l = m the entry is
// (-1, 1) with the state primed as (lambda_mm, 0), at l = m+1 it is (0, c_{m+1}).
__global__ void legendre_coef_kernel(int32_t lmax, double2 *__restrict__ coef) {
    const int m = blockIdx.y;
    const int l0 = m + (blockIdx.x * blockDim.x + threadIdx.x) * kLegC;
    if (l0 > lmax) return;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double mm = m;
    double sig = 1.0;
    for (int l = l0; l < l0 + kLegC && l <= lmax; ++l) {
        double g, c;
        if (l == m) {
            g = -1.0;
            c = 1.0;
        } else {
            const double ll = l;
            c = sqrt((4.0 * ll * ll - 1.0) / (ll * ll - mm * mm));
            if (l == m + 1) {
                g = 0.0;
            } else {
                const double l1 = l - 1;
                g = (l1 * l1 - mm * mm) / (4.0 * l1 * l1 - 1.0);  // 1 / c_{l-1}^2
            }
        }
        sig *= c;
        coef[base + l] = make_double2(g, sig);
    }
}

// ------------------------------------------------------------------ Legendre contraction
// DPP lane sums: exchanges within quads (lane ^ 1, ^ 2), then half-row and row
// mirrors.  Every lane of a group ends with the same value (the additions are
// pairwise and commutative), so the order is fixed.
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// Sum over aligned groups of kL = 4, 8 or 16 lanes.
template <int kL>
__device__ __forceinline__ double lane_group_sum(double v) {
    static_assert(kL == 4 || kL == 8 || kL == 16, "a quad, half-row or row");
    v += dpp_f64<0xB1>(v);                    // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);                    // quad_perm [2, 3, 0, 1]
    if (kL >= 8) v += dpp_f64<0x141>(v);      // row_half_mirror
    if (kL >= 16) v += dpp_f64<0x140>(v);     // row_mirror
    return v;
}

// State of the ring pairs one lane owns: z, the scaled recurrence pair
// (mu_{l-2}, mu_{l-1}) times 2^{600 k}, and the folded ring sums E, O (zero
// while k > 0, i.e. while the pair's lambda is below 2^-300).
template <int R>
struct PairState {
    double z[R], prev[R], cur[R], er[R], ei[R], orr[R], oi[R];
    int32_t k[R];
};

struct Folded {
    double er, ei, orr, oi;
};

__device__ __forceinline__ Folded load_folded(const double2 *__restrict__ F, int64_t N, int64_t nring, int m,
                                              int64_t p) {
    const double2 fn = F[(int64_t)m * nring + p];
    if (p + 1 == 2 * N) return {fn.x, fn.y, 0.0, 0.0};  // the equator is its own mirror
    const double2 fs = F[(int64_t)m * nring + (nring - 1 - p)];
    return {fn.x + fs.x, fn.y + fs.y, fn.x - fs.x, fn.y - fs.y};
}

template <int R>
__global__ __launch_bounds__(kLegThreads) void legendre_kernel(const double2 *__restrict__ F,
                                                               const double *__restrict__ seed,
                                                               const int32_t *__restrict__ seed_k,
                                                               const double2 *__restrict__ coef, int64_t N,
                                                               int32_t lmax, double w, double2 *__restrict__ out,
                                                               int64_t out_stride) {
    __shared__ double red[kLegBufs][2 * kLegC][kLegThreads];
    out += (int64_t)blockIdx.y * out_stride;
    const int m = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t npair = 2 * N, nring = 4 * N - 1;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;

    PairState<R> S;
    bool dead = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t p = ((int64_t)blockIdx.y * R + r) * kLegThreads + tid;
        S.er[r] = S.ei[r] = S.orr[r] = S.oi[r] = 0.0;
        S.z[r] = S.prev[r] = S.cur[r] = 0.0;
        S.k[r] = 0;
        if (p < npair) {
            double st;
            ring_z_sin(N, p + 1, S.z[r], st);
            S.prev[r] = seed[(int64_t)m * npair + p];
            S.k[r] = seed_k[(int64_t)m * npair + p];
            if (S.k[r] == 0) {
                const Folded f = load_folded(F, N, nring, m, p);
                S.er[r] = f.er;
                S.ei[r] = f.ei;
                S.orr[r] = f.orr;
                S.oi[r] = f.oi;
            }
        }
        dead |= S.k[r] > 0;
    }

    const int o = tid / kLegLanes, part = tid % kLegLanes;
    // Coefficients pass through LDS in stages of kLegStage values of l (double
    // buffered): the global load for the next stage is issued at the start of
    // a stage and written to LDS half a stage later, hiding its latency.
    __shared__ double2 cst[2][kLegStage];
    // entry of l, with g = 0 past lmax (the recurrence then stays bounded there)
    auto coef_at = [&](int l) {
        double2 c = coef[base + min(l, lmax)];
        c.x = l <= lmax ? c.x : 0.0;
        return c;
    };
    if (tid < kLegStage) cst[0][tid] = coef_at(m + tid);
    __syncthreads();
    double2 pre = make_double2(0.0, 0.0);

    // Reduction of a chunk: this lane's values summed as a tree, then the
    // kLegLanes lanes of the group; the reads are issued at the end of the
    // chunk and the sums taken after the next chunk's recurrence.
    double vp[kLegThreads / kLegLanes];
    double sigp = 0.0;
    int l0p = 0;
    bool pending = false;
    auto finish = [&]() {
#pragma unroll
        for (int w2 = kLegThreads / kLegLanes / 2; w2 > 0; w2 /= 2)
#pragma unroll
            for (int t = 0; t < w2; ++t) vp[t] += vp[t + w2];
        const double s = lane_group_sum<kLegLanes>(vp[0]);
        const int l = l0p + o / 2;
        if (part == 0 && l <= lmax) {
            double *dst = reinterpret_cast<double *>(out + base + l);
            dst[o & 1] = (w * sigp) * s;
        }
    };

    // One chunk of kLegC values of l.  kRevive: some lane of the wave still has
    // a pair below 2^-300; once none has, none will again, and the rest of the
    // loop runs without that bookkeeping (the folded sums then stay in place).
    auto chunk = [&](int l0, int buf, auto revive_tag) {
        constexpr bool kRevive = decltype(revive_tag)::value;
        const int ci = (l0 - m) / kLegC;
        const int stage = ci / (kLegStage / kLegC), within = ci % (kLegStage / kLegC);
        const double2 *cs = cst[stage & 1] + within * kLegC;
        if (within == 0 && tid < kLegStage) pre = coef_at(l0 + kLegStage + tid);
        if (within == kLegStage / kLegC / 2 && tid < kLegStage) cst[(stage + 1) & 1][tid] = pre;
        double2 cf[kLegC];
#pragma unroll
        for (int c = 0; c < kLegC; ++c) cf[c] = cs[c];
        double acc[2 * kLegC];
#pragma unroll
        for (int c = 0; c < kLegC; ++c) {
            acc[2 * c] = acc[2 * c + 1] = 0.0;
            const double g = cf[c].x;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double v = fma(-g, S.prev[r], S.z[r] * S.cur[r]);
                S.prev[r] = S.cur[r];
                S.cur[r] = v;
                // (l - m) even <=> c even, since l0 - m is a multiple of kLegC
                acc[2 * c] = fma(v, c % 2 == 0 ? S.er[r] : S.orr[r], acc[2 * c]);
                acc[2 * c + 1] = fma(v, c % 2 == 0 ? S.ei[r] : S.oi[r], acc[2 * c + 1]);
            }
        }
        // hand the state to the next chunk: multiply by sigma at its last l
        const double sg = cf[kLegC - 1].y;
        if (kRevive) {
            // pairs still below 2^-300 (times their scale) become live once they grow
            uint32_t revive = 0;
            dead = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double t = S.cur[r] * sg;
                const bool grow = S.k[r] > 0 && fabs(t) > kBig;
                const double f = grow ? kScaleDown : 1.0;
                S.cur[r] = t * f;
                S.prev[r] = S.prev[r] * sg * f;
                S.k[r] -= grow ? 1 : 0;
                revive |= (grow && S.k[r] == 0) ? 1u << r : 0u;
                dead |= S.k[r] > 0;
            }
            if (revive) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (revive & (1u << r)) {
                        const Folded f =
                            load_folded(F, N, nring, m, ((int64_t)blockIdx.y * R + r) * kLegThreads + tid);
                        S.er[r] = f.er;
                        S.ei[r] = f.ei;
                        S.orr[r] = f.orr;
                        S.oi[r] = f.oi;
                    }
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                S.cur[r] *= sg;
                S.prev[r] *= sg;
            }
        }
        // the previous chunk's sums, whose LDS reads were issued a chunk ago
        if (pending) finish();
#pragma unroll
        for (int q = 0; q < 2 * kLegC; ++q) red[buf][q][tid] = acc[q];
        __syncthreads();
        // issue this chunk's reads now; they are summed after the next chunk's
        // recurrence (red is double buffered: the next writes go to the other half)
#pragma unroll
        for (int t = 0; t < kLegThreads / kLegLanes; ++t) vp[t] = red[buf][o][part + kLegLanes * t];
        sigp = cs[o / 2].y;
        l0p = l0;
        pending = true;
    };
    // Every chunk has the same barriers in both loops, so the waves of a
    // workgroup may leave the first loop at different chunks.
    int l0 = m, buf = 0;
    for (; l0 <= lmax && __builtin_amdgcn_ballot_w64(dead) != 0; l0 += kLegC, buf ^= 1)
        chunk(l0, buf, std::true_type{});
    for (; l0 <= lmax; l0 += kLegC, buf ^= 1) chunk(l0, buf, std::false_type{});
    if (pending) finish();
}

// out[i] = sum_b part[b][i], b in order
__global__ void sum_partials_kernel(const double2 *__restrict__ part, int32_t nb, int64_t n, double2 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 s = part[i];
    for (int b = 1; b < nb; ++b) {
        const double2 v = part[(int64_t)b * n + i];
        s.x += v.x;
        s.y += v.y;
    }
    out[i] = s;
}

// C_l = (|a_l0|^2 + 2 sum_{m>=1} |a_lm|^2) / (2l+1).  One workgroup per (64
// consecutive l, map): lane = l (coalesced rows of the m-major layout), wave w
// sums m = w, w + kClWaves, ...; the waves' partial sums are added in order.
constexpr int kClWaves = 16;
__global__ __launch_bounds__(64 * kClWaves) void alm2cl_kernel(const double2 *__restrict__ alm, int32_t lmax,
                                                               int64_t n_alm, double *__restrict__ cl) {
    __shared__ double part[kClWaves][64];
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    const int l = blockIdx.x * 64 + lane;
    const double2 *a = alm + (int64_t)blockIdx.y * n_alm;
    const int mtop = min(blockIdx.x * 64 + 63, lmax);
    double s = 0.0;
    if (l <= lmax) {
#pragma unroll 4
        for (int m = wv; m <= mtop; m += kClWaves) {
            if (m > l) break;
            const double2 v = a[(int64_t)m * (2 * lmax + 1 - m) / 2 + l];
            const double q = v.x * v.x + v.y * v.y;
            s += m == 0 ? q : 2.0 * q;
        }
    }
    part[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && l <= lmax) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kClWaves; ++w) t += part[w][lane];
        cl[(int64_t)blockIdx.y * (lmax + 1) + l] = t / (double)(2 * l + 1);
    }
}

// ------------------------------------------------------------------ covariance over realisations
// X[r][b] = mean of cl[r][l] over the band
__global__ void band_kernel(const double *__restrict__ cl, int32_t R, int32_t n_ell, int32_t l0, int32_t dl,
                            int32_t nb, double *__restrict__ X) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)R * nb) return;
    const int64_t r = i / nb;
    const int b = (int)(i % nb);
    const double *row = cl + r * n_ell + l0 + (int64_t)b * dl;
    double s = 0.0;
    for (int j = 0; j < dl; ++j) s += row[j];
    X[i] = s / (double)dl;
}

__global__ void band_mean_kernel(const double *__restrict__ X, int32_t R, int32_t nb, double *__restrict__ mean) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double s = 0.0;
    int r = 0;
    for (; r + 8 <= R; r += 8) {  // eight loads in flight, the sum still in order
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = X[(int64_t)(r + u) * nb + b];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; r < R; ++r) s += X[(int64_t)r * nb + b];
    mean[b] = s / (double)R;
}

// cov[b][c] = sum_r Y[r][b] Y[r][c] / (R - ddof), Y[r][b] = X[r][b] - mean[b]: the
// product Y^T Y on the FP64 matrix cores.  One wave owns TB x TC tiles of 16 x 16
// and adds four rows of Y per step (rows past R and columns past nb are zero).
// Small per-wave blocks keep several waves on each SIMD, which hides the operand
// loads (Y stays in L2); 2 x 2 tiles measured faster than 4 x 4, 4 x 2 and 2 x 4.
// v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and holds D[l / 16 + 4 i][l % 16], i = 0..3.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kCovTB = 2, kCovTC = 2;  // 16 x 16 tiles per wave along b and along c (5 waves per SIMD)
template <int TB, int TC>
__global__ __launch_bounds__(64) void cov_kernel(const double *__restrict__ X, const double *__restrict__ mean,
                                                 int32_t R, int32_t nb, double denom, double *__restrict__ cov) {
    const int lane = threadIdx.x, li = lane % 16, lk = lane / 16;
    const int b0 = blockIdx.y * 16 * TB, c0 = blockIdx.x * 16 * TC;
    // Every load reads a valid address (row and column clamped); the centring and
    // the zeroing of rows past R and columns past nb are selects on the values.
    double mb[TB], mc[TC];
    bool vb[TB], vc[TC];
    int colb[TB], colc[TC];
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const int b = b0 + 16 * t + li;
        vb[t] = b < nb;
        colb[t] = min(b, nb - 1);
        mb[t] = mean[colb[t]];
    }
#pragma unroll
    for (int u = 0; u < TC; ++u) {
        const int c = c0 + 16 * u + li;
        vc[u] = c < nb;
        colc[u] = min(c, nb - 1);
        mc[u] = mean[colc[u]];
    }
    v4d acc[TB][TC];
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int u = 0; u < TC; ++u) acc[t][u] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int r0 = 0; r0 < R; r0 += 4) {
        const bool vr = r0 + lk < R;
        const double *row = X + (int64_t)min(r0 + lk, R - 1) * nb;
        double a[TB], bv[TC];
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            const double x = row[colb[t]];
            a[t] = (vr && vb[t]) ? x - mb[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < TC; ++u) {
            const double x = row[colc[u]];
            bv[u] = (vr && vc[u]) ? x - mc[u] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < TB; ++t)
#pragma unroll
            for (int u = 0; u < TC; ++u) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], bv[u], acc[t][u], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = b0 + 16 * t + lk + 4 * i;
            if (b >= nb) continue;
#pragma unroll
            for (int u = 0; u < TC; ++u) {
                const int c = c0 + 16 * u + li;
                if (c < nb) cov[(int64_t)b * nb + c] = acc[t][u][i] / denom;
            }
        }
}

// sd[b] = sqrt(cov[b][b]), then corr[b][c] = cov[b][c] / (sd[b] sd[c])
__global__ void sd_kernel(const double *__restrict__ cov, int32_t nb, double *__restrict__ sd) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) sd[b] = sqrt(cov[(int64_t)b * nb + b]);
}

__global__ void corr_kernel(const double *__restrict__ cov, const double *__restrict__ sd, int32_t nb,
                            double *__restrict__ corr) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (c >= nb) return;
    corr[(int64_t)b * nb + c] = cov[(int64_t)b * nb + c] / (sd[b] * sd[c]);
}

// ------------------------------------------------------------------ synthesis (alm2map)
// map_p = sum_l b_l [a_l0 lambda_l0 + 2 Re sum_{m>=1} a_lm lambda_lm e^{i m phi_p}]
// (the real field with coefficients a_lm).  Per m, every ring pair gets
//   E = sum_{l-m even} b_l a_lm lambda_lm(z),  O = sum_{l-m odd} ...,
// F_north(m) = E + O and F_south(m) = E - O (lambda_lm(-z) = (-1)^{l+m}
// lambda_lm(z)); no cross-lane reduction is needed.  Then each ring folds
// F(m) over m mod n and runs the inverse of the radix-4 ring transform.

__global__ void gaussian_beam_kernel(double sigma, int32_t lmax, double *__restrict__ beam) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax) return;
    beam[l] = exp(-0.5 * (double)l * (double)(l + 1) * sigma * sigma);
}

template <int R>
__global__ __launch_bounds__(kLegThreads) void legendre_synth_kernel(const double2 *__restrict__ alm,
                                                                     const double *__restrict__ beam,
                                                                     const double *__restrict__ seed,
                                                                     const int32_t *__restrict__ seed_k,
                                                                     const double2 *__restrict__ coef, int64_t N,
                                                                     int32_t lmax, double2 *__restrict__ F) {
    // per l of the current stage: (g_l, sigma_l) and sigma_l b_l a_lm
    __shared__ double2 cst[2][kLegStage];
    __shared__ double2 ast[2][kLegStage];
    const int m = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t npair = 2 * N, nring = 4 * N - 1;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;

    double z[R], prev[R], cur[R], er[R], ei[R], orr[R], oi[R];
    int32_t k[R];
    bool dead = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t p = ((int64_t)blockIdx.y * R + r) * kLegThreads + tid;
        z[r] = prev[r] = cur[r] = 0.0;
        er[r] = ei[r] = orr[r] = oi[r] = 0.0;
        k[r] = 0;
        if (p < npair) {
            double st;
            ring_z_sin(N, p + 1, z[r], st);
            prev[r] = seed[(int64_t)m * npair + p];
            k[r] = seed_k[(int64_t)m * npair + p];
        }
        dead |= k[r] > 0;
    }
    // entries of l: (g_l, sigma_l) with g = 0 past lmax (the recurrence then
    // stays bounded there), and sigma_l b_l a_lm, zero past lmax
    auto stage_entry = [&](int l, double2 &c, double2 &a) {
        const int lc = min(l, lmax);
        c = coef[base + lc];
        c.x = l <= lmax ? c.x : 0.0;
        const double2 v = alm[base + lc];
        const double f = l <= lmax ? c.y * (beam ? beam[lc] : 1.0) : 0.0;
        a = make_double2(f * v.x, m == 0 ? 0.0 : f * v.y);
    };
    if (tid < kLegStage) stage_entry(m + tid, cst[0][tid], ast[0][tid]);
    __syncthreads();
    double2 pc = make_double2(0.0, 0.0), pa = make_double2(0.0, 0.0);
    for (int l0 = m; l0 <= lmax; l0 += kLegC) {
        const int ci = (l0 - m) / kLegC;
        const int stage = ci / (kLegStage / kLegC), within = ci % (kLegStage / kLegC);
        const double2 *cs = cst[stage & 1] + within * kLegC;
        const double2 *as = ast[stage & 1] + within * kLegC;
        if (within == 0 && tid < kLegStage) stage_entry(l0 + kLegStage + tid, pc, pa);
        if (within == kLegStage / kLegC / 2 && tid < kLegStage) {
            cst[(stage + 1) & 1][tid] = pc;
            ast[(stage + 1) & 1][tid] = pa;
        }
#pragma unroll
        for (int c = 0; c < kLegC; ++c) {
            const double g = cs[c].x;
            const double2 a = as[c];  // zero past lmax
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double v = fma(-g, prev[r], z[r] * cur[r]);
                prev[r] = cur[r];
                cur[r] = v;
                if (c % 2 == 0) {
                    er[r] = fma(v, a.x, er[r]);
                    ei[r] = fma(v, a.y, ei[r]);
                } else {
                    orr[r] = fma(v, a.x, orr[r]);
                    oi[r] = fma(v, a.y, oi[r]);
                }
            }
        }
        const double sg = cs[kLegC - 1].y;
        if (__builtin_amdgcn_ballot_w64(dead)) {
            // a pair below 2^-300 has accumulated scaled values only: they are
            // dropped when it revives (their true size is below 2^-240 |a|)
            dead = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double t = cur[r] * sg;
                const bool grow = k[r] > 0 && fabs(t) > kBig;
                const double f = grow ? kScaleDown : 1.0;
                cur[r] = t * f;
                prev[r] = prev[r] * sg * f;
                k[r] -= grow ? 1 : 0;
                const bool drop = grow && k[r] == 0;
                er[r] = drop ? 0.0 : er[r];
                ei[r] = drop ? 0.0 : ei[r];
                orr[r] = drop ? 0.0 : orr[r];
                oi[r] = drop ? 0.0 : oi[r];
                dead |= k[r] > 0;
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cur[r] *= sg;
                prev[r] *= sg;
            }
        }
        __syncthreads();  // stage buffers: the next chunk may switch stages
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t p = ((int64_t)blockIdx.y * R + r) * kLegThreads + tid;
        if (p >= npair) continue;
        const bool live = k[r] == 0;
        const double2 fn = live ? make_double2(er[r] + orr[r], ei[r] + oi[r]) : make_double2(0.0, 0.0);
        F[(int64_t)m * nring + p] = fn;
        if (p + 1 != 2 * N)
            F[(int64_t)m * nring + (nring - 1 - p)] =
                live ? make_double2(er[r] - orr[r], ei[r] - oi[r]) : make_double2(0.0, 0.0);
    }
}

// Inverse ring transform.  With H[k] = sum_{m = k mod n, m <= lmax} c_m F(m) e^{i pi m s/n}
// (c_0 = 1, c_m = 2), map_j = Re sum_{k<n} H[k] e^{2 pi i k j/n}; by decimation,
//   map[4j' + q] = Re sum_{k'<n4} P_q[k'] e^{2 pi i k' j'/n4},
//   P_q[k'] = e^{2 pi i k' q/n} sum_t i^{t q} H[k' + t n4].
// Lane j' accumulates the four outputs of RG rings of equal length.
// K output classes: lane j' < n4/K writes pixels j' + s n4/K, s < K, from the
// sums over k' = h mod K kept apart: e^{2 pi i (j' + s n4/K) k' / n4} =
// e^{2 pi i j' k' / n4} e^{2 pi i s h / K}.  K = 2 needs only the real parts
// Re P cos and Im P sin (the factors are +-1); K = 4 and 8 keep the complex
// sums, as the factors include +-i and (+-1 +-i)/sqrt(2).  TH threads per
// workgroup (128 for K = 8, whose n4/8 lanes would leave half of 256 idle).
// J = 2 (with K = 1, any n4): each lane also takes pixel j' + ceil(n4/2), with a
// second twiddle chain, so that every LDS read serves two outputs.
template <typename T, bool kPolar, int K, int TH = kDftThreads, int J = 1>
__global__ __launch_bounds__(TH, kPolar ? (J > 1 ? 2 : (K > 1 ? 3 : 4)) : (K == 8 ? 2 : (K > 1 ? 3 : 1))) void ring_idft_kernel(
    const double2 *__restrict__ F, int64_t N, int32_t lmax, T *__restrict__ map) {
    static_assert(K == 1 || K == 2 || ((K == 4 || K == 8) && !kPolar), "output classes");
    static_assert(J == 1 || (J == 2 && K == 1), "two pixels per lane without output classes");
    constexpr bool kSplit = K > 1;
    constexpr int RG = kPolar ? 2 : (K >= 4 ? 1 : (K == 2 ? kEqRingsSplit : kEqRings));
    constexpr int H = K;
    __shared__ double2 ps[RG][4][kDftJ];
    const int64_t nring = 4 * N - 1;
    int64_t ring[RG];
    bool valid[RG];
    int64_t n4;
    if (kPolar) {
        // the even (K = 2) or odd (K = 1) polar rings i < N, the longest first so
        // that the short ones fill the tail of the launch
        const int64_t imax = ((N - 1) % 2 == (kSplit ? 0 : 1)) ? N - 1 : N - 2;
        const int64_t i = imax - 2 * (int64_t)blockIdx.y;
        ring[0] = i;
        ring[RG - 1] = 4 * N - i;
        valid[0] = valid[RG - 1] = true;
        n4 = i;
    } else {
        const int64_t i0 = N + (int64_t)blockIdx.y * RG;
#pragma unroll
        for (int g = 0; g < RG; ++g) {
            valid[g] = i0 + g <= 3 * N;
            ring[g] = valid[g] ? i0 + g : 3 * N;
        }
        n4 = N;
    }
    const int64_t nj = J == 2 ? (n4 + 1) / 2 : n4 / K;  // lanes needed
    if ((int64_t)blockIdx.x * TH >= nj) return;
    const int64_t jp = (int64_t)blockIdx.x * TH + threadIdx.x;  // j'
    const int64_t jb = jp + nj;                                  // the second pixel (J = 2)
    const int64_t n = 4 * n4;

    // per class h of k': K <= 2, the sums of Re P cos and Im P sin (the output is
    // their difference); K >= 4, the real and imaginary parts of sum P w
    double acc[H][RG][4], acn[H][RG][4];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[h][g][q] = acn[h][g][q] = 0.0;
    double acc2[RG][4], acn2[RG][4];  // J = 2: the sums of pixel jb
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc2[g][q] = acn2[g][q] = 0.0;
    double ws2 = 0.0, wc2 = 1.0;  // J = 2: step e^{2 pi i jb / n4}
    if (J == 2) sincospi(2.0 * (double)(jb % n4) / (double)n4, &ws2, &wc2);
    double ws, wc;  // step e^{2 pi i j' / n4}
    sincospi(2.0 * (double)(jp % n4) / (double)n4, &ws, &wc);

    for (int64_t kb = 0; kb < n4; kb += kDftJ) {
        const int cnt = (int)(n4 - kb < kDftJ ? n4 - kb : kDftJ);
        // First the folded sums H_t[k'] = e^{i pi kf/n} sum_u c_m F_m over m = kf + u n,
        // kf = k' + t n4 (c_0 = 1, otherwise 2, with the sign (-1)^u on shifted rings),
        // one (ring, t, k') per work item, so that the long folds of the short polar
        // rings spread over the workgroup, with kFoldBatch loads in flight per step.
        for (int e = threadIdx.x; e < RG * 4 * kDftJ; e += TH) {
            const int g = e / (4 * kDftJ), t = (e / kDftJ) % 4, kk = e % kDftJ;
            double hr = 0.0, hi = 0.0;
            if (kk < cnt) {
                const int64_t kf = kb + kk + t * n4;  // < n
                const bool shift = ring_shift(N, ring[g]) != 0;
                const double2 *col = F + (ring[g] - 1);
                if (kf == 0 && lmax >= 0) {  // c_0 = 1: start from -F_0, the first term adds 2 F_0
                    hr = -col[0].x;
                    hi = -col[0].y;
                }
                int64_t mm = kf;
                for (; mm + (kFoldBatch - 1) * n <= lmax; mm += kFoldBatch * n) {  // u even at each start
                    double2 f[kFoldBatch];
#pragma unroll
                    for (int v = 0; v < kFoldBatch; ++v) f[v] = col[(mm + v * n) * nring];
#pragma unroll
                    for (int v = 0; v < kFoldBatch; ++v) {
                        const double cm = (shift && (v & 1)) ? -2.0 : 2.0;
                        hr = fma(cm, f[v].x, hr);
                        hi = fma(cm, f[v].y, hi);
                    }
                }
                for (int v = 0; mm <= lmax; mm += n, ++v) {
                    const double2 f = col[mm * nring];
                    const double cm = (shift && (v & 1)) ? -2.0 : 2.0;
                    hr = fma(cm, f.x, hr);
                    hi = fma(cm, f.y, hi);
                }
                if (shift) {
                    double sn, cs;
                    sincospi((double)kf / (double)n, &sn, &cs);
                    const double r0 = hr * cs - hi * sn;
                    hi = hr * sn + hi * cs;
                    hr = r0;
                }
            }
            ps[g][t][kk] = make_double2(hr, hi);
        }
        __syncthreads();
        // then P_q[k'] = e^{2 pi i k' q / n} sum_t i^{tq} H_t[k'], in place: each work
        // item reads and writes only its own (ring, k') column
        for (int e = threadIdx.x; e < RG * kDftJ; e += TH) {
            const int g = e / kDftJ, kk = e % kDftJ;
            double2 P[4] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0),
                            make_double2(0.0, 0.0)};
            if (kk < cnt) {
                double2 Hh[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) Hh[t] = ps[g][t][kk];
                double s0, c0;
                sincospi((double)(kb + kk) / (double)n, &s0, &c0);  // h0 = e^{i pi k'/n}
                // sum_t i^{tq} H_t, i (x + iy) = -y + ix
                const double ar = Hh[0].x + Hh[2].x, ai = Hh[0].y + Hh[2].y;
                const double br = Hh[0].x - Hh[2].x, bi = Hh[0].y - Hh[2].y;
                const double cr = Hh[1].x + Hh[3].x, ci = Hh[1].y + Hh[3].y;
                const double dr = Hh[1].x - Hh[3].x, di = Hh[1].y - Hh[3].y;
                const double qr[4] = {ar + cr, br - di, ar - cr, br + di};
                const double qi[4] = {ai + ci, bi + dr, ai - ci, bi - dr};
                // e^{2 pi i k' q / n} from h0^2
                const double c1 = c0 * c0 - s0 * s0, s1 = 2.0 * c0 * s0;
                const double c2 = c1 * c1 - s1 * s1, s2 = 2.0 * c1 * s1;
                const double c3 = c2 * c1 - s2 * s1, s3 = c2 * s1 + s2 * c1;
                const double tc[4] = {1.0, c1, c2, c3}, ts[4] = {0.0, s1, s2, s3};
#pragma unroll
                for (int q = 0; q < 4; ++q) P[q] = make_double2(qr[q] * tc[q] - qi[q] * ts[q], qr[q] * ts[q] + qi[q] * tc[q]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) ps[g][q][kk] = P[q];
        }
        __syncthreads();
        double wr, wi, wr2 = 1.0, wi2 = 0.0;
        sincospi(2.0 * (double)((jp * kb) % n4) / (double)n4, &wi, &wr);
        if (J == 2) sincospi(2.0 * (double)((jb * kb) % n4) / (double)n4, &wi2, &wr2);
        for (int kk = 0; kk < cnt; kk += H) {
#pragma unroll
            for (int h = 0; h < H; ++h) {  // kb is a multiple of K, so k' = h mod K
                // all of this step's LDS reads first, so that they are in flight together
                double2 P[RG][4];
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q) P[g][q] = ps[g][q][kk + h];
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if constexpr (K >= 4) {
                            acc[h][g][q] = fma(-P[g][q].y, wi, fma(P[g][q].x, wr, acc[h][g][q]));
                            acn[h][g][q] = fma(P[g][q].y, wr, fma(P[g][q].x, wi, acn[h][g][q]));
                        } else {
                            acc[h][g][q] = fma(P[g][q].x, wr, acc[h][g][q]);
                            acn[h][g][q] = fma(P[g][q].y, wi, acn[h][g][q]);
                            if (J == 2) {
                                acc2[g][q] = fma(P[g][q].x, wr2, acc2[g][q]);
                                acn2[g][q] = fma(P[g][q].y, wi2, acn2[g][q]);
                            }
                        }
                    }
                const double nr = fma(wr, wc, -(wi * ws));
                const double ni = fma(wr, ws, wi * wc);
                wr = nr;
                wi = ni;
                if (J == 2) {
                    const double nr2 = fma(wr2, wc2, -(wi2 * ws2));
                    const double ni2 = fma(wr2, ws2, wi2 * wc2);
                    wr2 = nr2;
                    wi2 = ni2;
                }
            }
        }
        __syncthreads();
    }
    if (jp >= nj) return;
#pragma unroll
    for (int g = 0; g < RG; ++g) {
        if (!valid[g]) continue;
        T *dst = map + ring_first(N, ring[g]) + 4 * jp;
        if constexpr (K >= 4) {
            // pixel j' + s n4/K: sum_h Re(w^{s h} E_h), w = e^{2 pi i / K}, in h order;
            // w^e = e^{i pi e' / 4} with e' = e 8/K: Re(w^e E) = cos Re E - sin Im E
            constexpr double kR = 0.70710678118654752440;  // cos(pi/4)
            constexpr double c8[8] = {1.0, kR, 0.0, -kR, -1.0, -kR, 0.0, kR};
            constexpr double s8[8] = {0.0, kR, 1.0, kR, 0.0, -kR, -1.0, -kR};
#pragma unroll
            for (int sc = 0; sc < K; ++sc) {
                T *d = dst + sc * (4 * n4 / K);  // 4 (j' + sc n4/K)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    double v = 0.0;
#pragma unroll
                    for (int h = 0; h < K; ++h) {
                        const int e = ((sc * h) % K) * (8 / K);
                        if (s8[e] == 0.0)
                            v += c8[e] * acc[h][g][q];
                        else if (c8[e] == 0.0)
                            v -= s8[e] * acn[h][g][q];
                        else
                            v += c8[e] * acc[h][g][q] - s8[e] * acn[h][g][q];
                    }
                    d[q] = (T)v;
                }
            }
        } else if (kSplit) {
            // map[4 j' + q] = E + O, map[4 (j' + n4/2) + q] = E - O
            T *dst2 = dst + 2 * n4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double e = acc[0][g][q] - acn[0][g][q], o = acc[H - 1][g][q] - acn[H - 1][g][q];
                dst[q] = (T)(e + o);
                dst2[q] = (T)(e - o);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = (T)(acc[0][g][q] - acn[0][g][q]);
            if (J == 2 && jb < n4) {
                T *dstb = map + ring_first(N, ring[g]) + 4 * jb;
#pragma unroll
                for (int q = 0; q < 4; ++q) dstb[q] = (T)(acc2[g][q] - acn2[g][q]);
            }
        }
    }
}

// ------------------------------------------------------------------ map moments (eqs. (12), (13))
constexpr int kMomBlocks = 1024;  // fixed, so the reduction order does not depend on the device
constexpr int kMomThreads = 256;

__device__ __forceinline__ double block_sum_fixed(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kMomThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// pass 0: sum q; pass 1: sum (q - mean)^2 and sum (q - mean)^4 (mean from the
// previous pass's total).  Block b covers a fixed contiguous range.
template <typename T>
__global__ __launch_bounds__(kMomThreads) void moments_partial_kernel(const T *__restrict__ q, int64_t npix, int pass,
                                                                      const double *__restrict__ mean,
                                                                      double *__restrict__ part) {
    __shared__ double sh[kMomThreads];
    const T *x = q + (int64_t)blockIdx.y * npix;
    const int64_t per = (npix + kMomBlocks - 1) / kMomBlocks;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < npix ? lo + per : npix;
    const double mu = pass ? mean[blockIdx.y] : 0.0;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kMomThreads) {
        const double d = (double)x[i] - mu;
        if (pass) {
            const double d2 = d * d;
            s1 += d2;
            s2 = fma(d2, d2, s2);
        } else {
            s1 += d;
        }
    }
    s1 = block_sum_fixed(s1, sh);
    s2 = block_sum_fixed(s2, sh);
    if (threadIdx.x == 0) {
        double *o = part + ((int64_t)blockIdx.y * kMomBlocks + blockIdx.x) * 2;
        o[0] = s1;
        o[1] = s2;
    }
}

// one block per map: totals of the partials; pass 0 writes the mean, pass 1 the moments
__global__ __launch_bounds__(kMomThreads) void moments_final_kernel(const double *__restrict__ part, int64_t npix,
                                                                    int pass, double *__restrict__ mean,
                                                                    double *__restrict__ out) {
    __shared__ double sh[kMomThreads];
    const double *p = part + (int64_t)blockIdx.x * kMomBlocks * 2;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < kMomBlocks; i += kMomThreads) {
        a += p[2 * i];
        b += p[2 * i + 1];
    }
    a = block_sum_fixed(a, sh);
    b = block_sum_fixed(b, sh);
    if (threadIdx.x != 0) return;
    const double Nn = (double)npix;
    if (pass == 0) {
        mean[blockIdx.x] = a / Nn;
        return;
    }
    const double m2 = a / Nn, m4 = b / Nn;
    double *o = out + (int64_t)blockIdx.x * UFALCON_NMOMENTS;
    o[0] = mean[blockIdx.x];
    o[1] = m2;
    o[2] = m4;
    o[3] = m2;  // s^2
    o[4] = (Nn - 1.0) * (Nn - 1.0) / (Nn * Nn * Nn) * m4 - (Nn - 1.0) * (Nn - 3.0) / (Nn * Nn * Nn) * m2 * m2;
}

// ------------------------------------------------------------------ host side
// Inverse ring transforms of one map, in the same arrangement as launch_ring_dft.
template <typename T>
void launch_ring_idft(const double2 *F, int64_t N, int32_t lmax, T *mp, hipStream_t s) {
    const unsigned dx = (unsigned)((N + kDftThreads - 1) / kDftThreads);
    // polar rings i < N: odd i directly, even i with the even/odd split (polar
    // 0.71 -> 0.39 + 0.24 ms at Nside 1024)
    if (N > 1)
        hipLaunchKernelGGL((ring_idft_kernel<T, true, 1, kDftThreads, 2>),
                           dim3((unsigned)((N / 2 + kDftThreads - 1) / kDftThreads), (unsigned)(N / 2)),
                           dim3(kDftThreads), 0, s, F, N, lmax, mp);
    if ((N - 1) / 2 > 0)
        hipLaunchKernelGGL((ring_idft_kernel<T, true, 2>),
                           dim3((unsigned)((N / 2 + kDftThreads - 1) / kDftThreads), (unsigned)((N - 1) / 2)),
                           dim3(kDftThreads), 0, s, F, N, lmax, mp);
    // equatorial rings (n4 = N): eight output classes when 8 | N, four when 4 | N,
    // two when 2 | N
    if (N % 8 == 0)
        hipLaunchKernelGGL((ring_idft_kernel<T, false, 8, 128>),
                           dim3((unsigned)((N / 8 + 127) / 128), (unsigned)(2 * N + 1)), dim3(128), 0, s, F, N, lmax,
                           mp);
    else if (N % 4 == 0)
        hipLaunchKernelGGL((ring_idft_kernel<T, false, 4>),
                           dim3((unsigned)((N / 4 + kDftThreads - 1) / kDftThreads), (unsigned)(2 * N + 1)),
                           dim3(kDftThreads), 0, s, F, N, lmax, mp);
    else if (N % 2 == 0)
        hipLaunchKernelGGL((ring_idft_kernel<T, false, 2>),
                           dim3((unsigned)((N / 2 + kDftThreads - 1) / kDftThreads),
                                (unsigned)((2 * N + 1 + kEqRingsSplit - 1) / kEqRingsSplit)),
                           dim3(kDftThreads), 0, s, F, N, lmax, mp);
    else
        hipLaunchKernelGGL((ring_idft_kernel<T, false, 1>),
                           dim3(dx, (unsigned)((2 * N + 1 + kEqRings - 1) / kEqRings)), dim3(kDftThreads), 0, s, F,
                           N, lmax, mp);
}

// Ring DFTs of one map: polar ring pairs, then the equatorial rings (split when n4 = N is even).
template <typename T>
void launch_ring_dft(const T *mp, int64_t N, int32_t lmax, double2 *F, hipStream_t s) {
    const unsigned dx = (unsigned)((N + kDftThreads - 1) / kDftThreads);
    // all polar rings in one launch (split into odd rings and even rings with the
    // even/odd split of the outputs, as the inverse does, the two launches took
    // 0.30 + 0.28 ms against 0.47 ms at Nside 1024)
    if (N > 1)
        hipLaunchKernelGGL((ring_dft_kernel<T, true, 1>), dim3(dx, (unsigned)(N / 2)), dim3(kDftThreads), 0, s, mp, N,
                           lmax, F);
    if ((N - 1) / 2 > 0)
        hipLaunchKernelGGL((ring_dft_kernel<T, true, 2>),
                           dim3((unsigned)((N / 2 + kDftThreads - 1) / kDftThreads), (unsigned)((N - 1) / 2)),
                           dim3(kDftThreads), 0, s, mp, N, lmax, F);
    // equatorial rings (n4 = N): four output classes when 4 | N, two when 2 | N
    if (N % 4 == 0)
        hipLaunchKernelGGL((ring_dft_kernel<T, false, 4>),
                           dim3((unsigned)((N / 4 + kDftThreads - 1) / kDftThreads), (unsigned)(2 * N + 1)),
                           dim3(kDftThreads), 0, s, mp, N, lmax, F);
    else if (N % 2 == 0)
        hipLaunchKernelGGL((ring_dft_kernel<T, false, 2>),
                           dim3((unsigned)((N / 2 + kDftThreads - 1) / kDftThreads),
                                (unsigned)((2 * N + 1 + kEqRingsSplit - 1) / kEqRingsSplit)),
                           dim3(kDftThreads), 0, s, mp, N, lmax, F);
    else
        hipLaunchKernelGGL((ring_dft_kernel<T, false, 1>),
                           dim3(dx, (unsigned)((2 * N + 1 + kEqRings - 1) / kEqRings)), dim3(kDftThreads), 0, s, mp,
                           N, lmax, F);
}

struct ShtLayout {
    int64_t N, nring, npair, nalm;
    int32_t lmax, n_rb;
    size_t off_F, off_seed, off_k, off_coef, off_part, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

ShtLayout sht_layout(int64_t nside, int32_t lmax) {
    ShtLayout L{};
    L.N = nside;
    L.lmax = lmax;
    L.nring = 4 * nside - 1;
    L.npair = 2 * nside;
    L.nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    L.n_rb = (int32_t)((L.npair + (int64_t)kLegThreads * kLegR - 1) / ((int64_t)kLegThreads * kLegR));
    const int64_t M = (int64_t)lmax + 1;
    size_t off = 0;
    L.off_F = off;
    off = align256(off + (size_t)(M * L.nring) * sizeof(double2));
    L.off_seed = off;
    off = align256(off + (size_t)(M * L.npair) * sizeof(double));
    L.off_k = off;
    off = align256(off + (size_t)(M * L.npair) * sizeof(int32_t));
    L.off_coef = off;
    off = align256(off + (size_t)L.nalm * sizeof(double2));
    L.off_part = off;
    if (L.n_rb > 1) off = align256(off + (size_t)L.n_rb * L.nalm * sizeof(double2));
    L.total = off;
    return L;
}

constexpr int32_t kMaxLmax = 4 * UFALCON_MAX_NSIDE;

}  // namespace
}  // namespace ufx

using namespace ufx;

extern "C" size_t ufalcon_map2alm_workspace_size(int64_t nside, int32_t lmax) {
    if (check_nside(nside) || lmax < 0 || lmax > kMaxLmax) return 0;
    return sht_layout(nside, lmax).total;
}

extern "C" int ufalcon_map2alm(const void *maps, int dtype, int32_t n_maps, int64_t nside, int32_t lmax, double *alm,
                               void *workspace, size_t workspace_bytes, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_map2alm");
    int rc = check_nside(nside);
    if (rc) return rc;
    if (n_maps < 0 || lmax < 0 || lmax > kMaxLmax) return UFALCON_EINVAL;
    if (dtype != UFALCON_F32 && dtype != UFALCON_F64) return UFALCON_EINVAL;
    if (n_maps == 0) return UFALCON_OK;
    if (!maps || !alm || !workspace) return UFALCON_EINVAL;
    const ShtLayout L = sht_layout(nside, lmax);
    if (workspace_bytes < L.total) return UFALCON_EWORKSPACE;
    hipStream_t s = as_stream(stream);
    char *ws = static_cast<char *>(workspace);
    double2 *F = reinterpret_cast<double2 *>(ws + L.off_F);
    double *seed = reinterpret_cast<double *>(ws + L.off_seed);
    int32_t *seed_k = reinterpret_cast<int32_t *>(ws + L.off_k);
    double2 *coef = reinterpret_cast<double2 *>(ws + L.off_coef);
    double2 *part = reinterpret_cast<double2 *>(ws + L.off_part);
    const int64_t N = nside, npix = npix_of(nside);
    const int64_t M = (int64_t)lmax + 1;

    hipLaunchKernelGGL(lambda_seed_kernel, dim3(blocks_for(L.npair, 64)), dim3(64 * kSeedSegs), 0, s, N, lmax,
                       seed, seed_k);
    hipLaunchKernelGGL(legendre_coef_kernel, dim3(blocks_for((M + kLegC - 1) / kLegC, 256), (unsigned)M), dim3(256), 0, s,
                       lmax, coef);
    UFX_HIP_CHECK(hipGetLastError());
    const double w = 4.0 * M_PI / (double)npix;
    for (int32_t t = 0; t < n_maps; ++t) {
        double2 *a = reinterpret_cast<double2 *>(alm) + (int64_t)t * L.nalm;
        if (dtype == UFALCON_F32)
            launch_ring_dft(static_cast<const float *>(maps) + t * npix, N, lmax, F, s);
        else
            launch_ring_dft(static_cast<const double *>(maps) + t * npix, N, lmax, F, s);
        double2 *dst = L.n_rb > 1 ? part : a;
        hipLaunchKernelGGL(legendre_kernel<kLegR>, dim3((unsigned)M, (unsigned)L.n_rb), dim3(kLegThreads), 0, s, F, seed,
                           seed_k, coef, N, lmax, w, dst, L.n_rb > 1 ? L.nalm : (int64_t)0);
        if (L.n_rb > 1)
            hipLaunchKernelGGL(sum_partials_kernel, dim3(blocks_for(L.nalm, 256)), dim3(256), 0, s, part, L.n_rb,
                               L.nalm, a);
        UFX_HIP_CHECK(hipGetLastError());
    }
    return UFALCON_OK;
}

extern "C" int ufalcon_alm2cl(const double *alm, int32_t n_maps, int32_t lmax, double *cl, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_alm2cl");
    if (n_maps < 0 || lmax < 0 || lmax > kMaxLmax) return UFALCON_EINVAL;
    if (n_maps == 0) return UFALCON_OK;
    if (!alm || !cl) return UFALCON_EINVAL;
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    hipLaunchKernelGGL(alm2cl_kernel, dim3(blocks_for((int64_t)lmax + 1, 64), (unsigned)n_maps), dim3(64 * kClWaves), 0,
                       as_stream(stream), reinterpret_cast<const double2 *>(alm), lmax, nalm, cl);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

extern "C" size_t ufalcon_cl_covariance_workspace_size(int32_t n_real, int32_t n_bands) {
    if (n_real < 1 || n_bands < 1) return 0;
    return ((size_t)n_real + 1) * (size_t)n_bands * sizeof(double);  // band powers, then the deviations
}

extern "C" int ufalcon_cl_covariance(const double *cl, int32_t n_real, int32_t n_ell, int32_t ell_min,
                                     int32_t delta_ell, int32_t n_bands, int32_t ddof, double *band_mean, double *cov,
                                     double *corr, void *workspace, size_t workspace_bytes, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_cl_covariance");
    if (!cl || !band_mean || !cov || !workspace) return UFALCON_EINVAL;
    if (n_real < 1 || n_ell < 1 || ell_min < 0 || delta_ell < 1 || n_bands < 1) return UFALCON_EINVAL;
    if (ddof != 0 && ddof != 1) return UFALCON_EINVAL;
    if (n_real <= ddof) return UFALCON_EINVAL;
    if ((int64_t)ell_min + (int64_t)n_bands * delta_ell > n_ell) return UFALCON_EINVAL;
    if (n_bands > 65535) return UFALCON_EINVAL;
    if (workspace_bytes < ufalcon_cl_covariance_workspace_size(n_real, n_bands)) return UFALCON_EWORKSPACE;
    hipStream_t s = as_stream(stream);
    double *X = static_cast<double *>(workspace);
    hipLaunchKernelGGL(band_kernel, dim3(blocks_for((int64_t)n_real * n_bands, 256)), dim3(256), 0, s, cl, n_real,
                       n_ell, ell_min, delta_ell, n_bands, X);
    hipLaunchKernelGGL(band_mean_kernel, dim3(blocks_for(n_bands, 64)), dim3(64), 0, s, X, n_real, n_bands,
                       band_mean);
    hipLaunchKernelGGL((cov_kernel<kCovTB, kCovTC>),
                       dim3((unsigned)((n_bands + 16 * kCovTC - 1) / (16 * kCovTC)),
                            (unsigned)((n_bands + 16 * kCovTB - 1) / (16 * kCovTB))),
                       dim3(64), 0, s, X, band_mean, n_real, n_bands, (double)(n_real - ddof), cov);
    if (corr) {
        double *sd = X + (int64_t)n_real * n_bands;
        hipLaunchKernelGGL(sd_kernel, dim3(blocks_for(n_bands, 256)), dim3(256), 0, s, cov, n_bands, sd);
        hipLaunchKernelGGL(corr_kernel, dim3(blocks_for(n_bands, 256), (unsigned)n_bands), dim3(256), 0, s, cov, sd,
                           n_bands, corr);
    }
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

extern "C" int ufalcon_gaussian_beam(double sigma, int32_t lmax, double *beam, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_gaussian_beam");
    if (!beam || lmax < 0 || lmax > kMaxLmax || !std::isfinite(sigma) || sigma < 0.0) return UFALCON_EINVAL;
    hipLaunchKernelGGL(gaussian_beam_kernel, dim3(blocks_for((int64_t)lmax + 1, 256)), dim3(256), 0,
                       as_stream(stream), sigma, lmax, beam);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

extern "C" size_t ufalcon_alm2map_workspace_size(int64_t nside, int32_t lmax) {
    if (check_nside(nside) || lmax < 0 || lmax > kMaxLmax) return 0;
    return sht_layout(nside, lmax).off_part;  // ring sums, seeds and coefficients
}

extern "C" int ufalcon_alm2map(const double *alm, int32_t n_maps, int64_t nside, int32_t lmax, const double *beam,
                               void *maps, int dtype, void *workspace, size_t workspace_bytes,
                               ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_alm2map");
    int rc = check_nside(nside);
    if (rc) return rc;
    if (n_maps < 0 || lmax < 0 || lmax > kMaxLmax) return UFALCON_EINVAL;
    if (dtype != UFALCON_F32 && dtype != UFALCON_F64) return UFALCON_EINVAL;
    if (n_maps == 0) return UFALCON_OK;
    if (!alm || !maps || !workspace) return UFALCON_EINVAL;
    const ShtLayout L = sht_layout(nside, lmax);
    if (workspace_bytes < L.off_part) return UFALCON_EWORKSPACE;
    hipStream_t s = as_stream(stream);
    char *ws = static_cast<char *>(workspace);
    double2 *F = reinterpret_cast<double2 *>(ws + L.off_F);
    double *seed = reinterpret_cast<double *>(ws + L.off_seed);
    int32_t *seed_k = reinterpret_cast<int32_t *>(ws + L.off_k);
    double2 *coef = reinterpret_cast<double2 *>(ws + L.off_coef);
    const int64_t N = nside, npix = npix_of(nside);
    const int64_t M = (int64_t)lmax + 1;
    hipLaunchKernelGGL(lambda_seed_kernel, dim3(blocks_for(L.npair, 64)), dim3(64 * kSeedSegs), 0, s, N, lmax,
                       seed, seed_k);
    hipLaunchKernelGGL(legendre_coef_kernel, dim3(blocks_for((M + kLegC - 1) / kLegC, 256), (unsigned)M), dim3(256), 0, s,
                       lmax, coef);
    UFX_HIP_CHECK(hipGetLastError());
    for (int32_t t = 0; t < n_maps; ++t) {
        const double2 *a = reinterpret_cast<const double2 *>(alm) + (int64_t)t * L.nalm;
        hipLaunchKernelGGL(legendre_synth_kernel<kLegR>, dim3((unsigned)M, (unsigned)L.n_rb), dim3(kLegThreads), 0, s,
                           a, beam, seed, seed_k, coef, N, lmax, F);
        if (dtype == UFALCON_F32)
            launch_ring_idft(F, N, lmax, static_cast<float *>(maps) + t * npix, s);
        else
            launch_ring_idft(F, N, lmax, static_cast<double *>(maps) + t * npix, s);
        UFX_HIP_CHECK(hipGetLastError());
    }
    return UFALCON_OK;
}

extern "C" size_t ufalcon_map_moments_workspace_size(int32_t n_maps) {
    if (n_maps < 1) return 0;
    return (size_t)n_maps * (2 * kMomBlocks + 1) * sizeof(double);
}

extern "C" int ufalcon_map_moments(const void *maps, int dtype, int32_t n_maps, int64_t npix, double *moments,
                                   void *workspace, size_t workspace_bytes, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_map_moments");
    if (n_maps < 0 || npix < 1) return UFALCON_EINVAL;
    if (dtype != UFALCON_F32 && dtype != UFALCON_F64) return UFALCON_EINVAL;
    if (n_maps == 0) return UFALCON_OK;
    if (!maps || !moments || !workspace) return UFALCON_EINVAL;
    if (n_maps > 65535) return UFALCON_EINVAL;
    if (workspace_bytes < ufalcon_map_moments_workspace_size(n_maps)) return UFALCON_EWORKSPACE;
    hipStream_t s = as_stream(stream);
    double *part = static_cast<double *>(workspace);
    double *mean = part + (int64_t)n_maps * 2 * kMomBlocks;
    for (int pass = 0; pass < 2; ++pass) {
        if (dtype == UFALCON_F32)
            hipLaunchKernelGGL(moments_partial_kernel<float>, dim3(kMomBlocks, (unsigned)n_maps), dim3(kMomThreads), 0,
                               s, static_cast<const float *>(maps), npix, pass, mean, part);
        else
            hipLaunchKernelGGL(moments_partial_kernel<double>, dim3(kMomBlocks, (unsigned)n_maps), dim3(kMomThreads), 0,
                               s, static_cast<const double *>(maps), npix, pass, mean, part);
        hipLaunchKernelGGL(moments_final_kernel, dim3((unsigned)n_maps), dim3(kMomThreads), 0, s, part, npix, pass, mean,
                           moments);
    }
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}
