// Spherical-harmonic analysis of HEALPix RING maps, angular power spectra and
// their covariance over realisations (section 3.1 eq. (9); section 3.2
// eqs. (10) and (11)).
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
//   ring_dft_kernel     one lane per m, RG rings of equal length per workgroup:
//                       the map chunk is staged in LDS (FP32 or FP64 in, FP64
//                       out) and read as broadcasts; the twiddle e^{-2 pi i m j/n}
//                       advances by one complex multiply per pixel and is
//                       re-seeded exactly from (m j mod n) every kDftJ pixels;
//   lambda_seed_kernel  lambda_mm(z) of every ring pair for m = 0..lmax, carried
//                       as value * 2^{-600 k} so sin^m(theta) cannot underflow;
//   legendre_kernel     one workgroup per (m, block of 256 R ring pairs): the
//                       three-term recurrence in l, R pairs per lane, partial
//                       sums over C consecutive l reduced through LDS;
//   alm2cl / covariance small fixed-order reductions.
#include "../../include/ufalcon.h"
#include "internal.hpp"

namespace ufx {
namespace {

constexpr int kDftThreads = 256;
constexpr int kDftJ = 64;      // pixels per staged chunk (and twiddle re-seed period)
constexpr int kEqRings = 16;   // equatorial rings (all 4N long) per workgroup
constexpr int kLegThreads = 256;
constexpr int kLegR = 8;       // ring pairs per lane
constexpr int kLegC = 8;       // l values per reduction chunk
static_assert(2 * kLegC * 16 == kLegThreads, "reduction layout: 16 lanes per output");
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
template <typename T, bool kPolar>
__global__ __launch_bounds__(kDftThreads) void ring_dft_kernel(const T *__restrict__ map, int64_t N, int32_t lmax,
                                                               double2 *__restrict__ F) {
    constexpr int RG = kPolar ? 2 : kEqRings;
    __shared__ double xs[RG][kDftJ];
    const int m = blockIdx.x * kDftThreads + threadIdx.x;
    const int64_t nring = 4 * N - 1;
    int64_t ring[RG];
    bool valid[RG];
    int64_t n;
    if (kPolar) {
        const int64_t i = (int64_t)blockIdx.y + 1;
        ring[0] = i;
        ring[RG - 1] = 4 * N - i;
        valid[0] = valid[RG - 1] = true;
        n = 4 * i;
    } else {
        const int64_t i0 = N + (int64_t)blockIdx.y * RG;
#pragma unroll
        for (int g = 0; g < RG; ++g) {
            valid[g] = i0 + g <= 3 * N;
            ring[g] = valid[g] ? i0 + g : 3 * N;
        }
        n = 4 * N;
    }
    int64_t first[RG];
#pragma unroll
    for (int g = 0; g < RG; ++g) first[g] = ring_first(N, ring[g]);

    double ar[RG], ai[RG];
#pragma unroll
    for (int g = 0; g < RG; ++g) ar[g] = ai[g] = 0.0;
    // step e^{-2 pi i m / n}
    double ws, wc;
    sincospi(-2.0 * (double)((int64_t)m % n) / (double)n, &ws, &wc);

    for (int64_t jb = 0; jb < n; jb += kDftJ) {
        const int cnt = (int)(n - jb < kDftJ ? n - jb : kDftJ);
        for (int e = threadIdx.x; e < RG * kDftJ; e += kDftThreads) {
            const int g = e / kDftJ, jj = e % kDftJ;
            xs[g][jj] = jj < cnt ? (double)map[first[g] + jb + jj] : 0.0;
        }
        __syncthreads();
        double wr, wi;
        sincospi(-2.0 * (double)(((int64_t)m * jb) % n) / (double)n, &wi, &wr);
        for (int jj = 0; jj < cnt; ++jj) {
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const double x = xs[g][jj];
                ar[g] = fma(x, wr, ar[g]);
                ai[g] = fma(x, wi, ai[g]);
            }
            const double nr = fma(wr, wc, -(wi * ws));
            const double ni = fma(wr, ws, wi * wc);
            wr = nr;
            wi = ni;
        }
        __syncthreads();
    }
    if (m > lmax) return;
#pragma unroll
    for (int g = 0; g < RG; ++g) {
        if (!valid[g]) continue;
        double re = ar[g], im = ai[g];
        if (ring_shift(N, ring[g])) {  // e^{-i m pi / n}
            double s, c;
            sincospi(-(double)((int64_t)m % (2 * n)) / (double)n, &s, &c);
            re = ar[g] * c - ai[g] * s;
            im = ar[g] * s + ai[g] * c;
        }
        F[(int64_t)m * nring + (ring[g] - 1)] = make_double2(re, im);
    }
}

// ------------------------------------------------------------------ lambda_mm seeds
__global__ void lambda_seed_kernel(int64_t N, int32_t lmax, double *__restrict__ seed, int32_t *__restrict__ seed_k) {
    const int64_t npair = 2 * N;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npair) return;
    double z, st;
    ring_z_sin(N, p + 1, z, st);
    double v = 0.28209479177387814;  // 1/sqrt(4 pi)
    int32_t k = 0;
    for (int m = 0; m <= lmax; ++m) {
        seed[(int64_t)m * npair + p] = v;
        seed_k[(int64_t)m * npair + p] = k;
        v = v * (-sqrt((double)(2 * m + 3) / (double)(2 * m + 2))) * st;
        if (v != 0.0 && fabs(v) < kTiny) {
            v *= kScaleUp;
            ++k;
        }
    }
}

// Recurrence coefficients per (m, l), packed like the coefficients:
//   lambda_l = a_l z lambda_{l-1} - b_l lambda_{l-2}
// l = m:   (0, -1)  with the state primed as (lambda_{l-2}, lambda_{l-1}) = (seed, 0)
// l = m+1: (sqrt(2m+3), 0)
// l > m+1: (c_l, c_l / c_{l-1}),  c_l = sqrt((4l^2-1)/(l^2-m^2)).
__global__ void legendre_coef_kernel(int32_t lmax, double2 *__restrict__ coef) {
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax) return;
    const int64_t idx = (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
    double a, b;
    if (l == m) {
        a = 0.0;
        b = -1.0;
    } else if (l == m + 1) {
        a = sqrt((double)(2 * m + 3));
        b = 0.0;
    } else {
        const double ll = l, mm = m, l1 = l - 1;
        a = sqrt((4.0 * ll * ll - 1.0) / (ll * ll - mm * mm));
        const double c1 = sqrt((4.0 * l1 * l1 - 1.0) / (l1 * l1 - mm * mm));
        b = a / c1;
    }
    coef[idx] = make_double2(a, b);
}

// ------------------------------------------------------------------ Legendre contraction
__global__ __launch_bounds__(kLegThreads) void legendre_kernel(const double2 *__restrict__ F,
                                                               const double *__restrict__ seed,
                                                               const int32_t *__restrict__ seed_k,
                                                               const double2 *__restrict__ coef, int64_t N,
                                                               int32_t lmax, double w, double2 *__restrict__ out,
                                                               int64_t out_stride) {
    __shared__ double red[2 * kLegC][kLegThreads];
    out += (int64_t)blockIdx.y * out_stride;
    const int m = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t npair = 2 * N, nring = 4 * N - 1;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;

    double z[kLegR], prev[kLegR], cur[kLegR], er[kLegR], ei[kLegR], orr[kLegR], oi[kLegR];
    int32_t k[kLegR];
#pragma unroll
    for (int r = 0; r < kLegR; ++r) {
        const int64_t p = ((int64_t)blockIdx.y * kLegR + r) * kLegThreads + tid;
        er[r] = ei[r] = orr[r] = oi[r] = 0.0;
        z[r] = 0.0;
        prev[r] = cur[r] = 0.0;
        k[r] = 0;
        if (p < npair) {
            double st;
            ring_z_sin(N, p + 1, z[r], st);
            prev[r] = seed[(int64_t)m * npair + p];
            k[r] = seed_k[(int64_t)m * npair + p];
            if (k[r] == 0) {
                const double2 fn = F[(int64_t)m * nring + p];
                const double2 fs = p + 1 == 2 * N ? make_double2(0.0, 0.0) : F[(int64_t)m * nring + (nring - 1 - p)];
                if (p + 1 == 2 * N) {  // the equator is its own mirror
                    er[r] = fn.x;
                    ei[r] = fn.y;
                } else {
                    er[r] = fn.x + fs.x;
                    ei[r] = fn.y + fs.y;
                    orr[r] = fn.x - fs.x;
                    oi[r] = fn.y - fs.y;
                }
            }
        }
    }

    const int o = tid / 16, part = tid % 16;
    for (int l0 = m; l0 <= lmax; l0 += kLegC) {
        double acc[2 * kLegC];
#pragma unroll
        for (int c = 0; c < kLegC; ++c) {
            acc[2 * c] = acc[2 * c + 1] = 0.0;
            const int l = l0 + c;
            if (l <= lmax) {
                const double2 ab = coef[base + l];
#pragma unroll
                for (int r = 0; r < kLegR; ++r) {
                    const double v = fma(-ab.y, prev[r], ab.x * (z[r] * cur[r]));
                    prev[r] = cur[r];
                    cur[r] = v;
                    // (l - m) even <=> c even, since l0 - m is a multiple of kLegC
                    if (c % 2 == 0) {
                        acc[2 * c] = fma(v, er[r], acc[2 * c]);
                        acc[2 * c + 1] = fma(v, ei[r], acc[2 * c + 1]);
                    } else {
                        acc[2 * c] = fma(v, orr[r], acc[2 * c]);
                        acc[2 * c + 1] = fma(v, oi[r], acc[2 * c + 1]);
                    }
                }
            }
        }
        // pairs still below 2^-300 (times their scale) become live once they grow
#pragma unroll
        for (int r = 0; r < kLegR; ++r) {
            if (k[r] > 0 && fabs(cur[r]) > kBig) {
                cur[r] *= kScaleDown;
                prev[r] *= kScaleDown;
                if (--k[r] == 0) {
                    const int64_t p = ((int64_t)blockIdx.y * kLegR + r) * kLegThreads + tid;
                    const double2 fn = F[(int64_t)m * nring + p];
                    if (p + 1 == 2 * N) {
                        er[r] = fn.x;
                        ei[r] = fn.y;
                    } else {
                        const double2 fs = F[(int64_t)m * nring + (nring - 1 - p)];
                        er[r] = fn.x + fs.x;
                        ei[r] = fn.y + fs.y;
                        orr[r] = fn.x - fs.x;
                        oi[r] = fn.y - fs.y;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 2 * kLegC; ++q) red[q][tid] = acc[q];
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < kLegThreads / 16; ++t) s += red[o][part + 16 * t];
        s += __shfl_xor(s, 8, 16);
        s += __shfl_xor(s, 4, 16);
        s += __shfl_xor(s, 2, 16);
        s += __shfl_xor(s, 1, 16);
        const int l = l0 + o / 2;
        if (part == 0 && l <= lmax) {
            double *dst = reinterpret_cast<double *>(out + base + l);
            dst[o & 1] = w * s;
        }
        __syncthreads();
    }
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

// C_l = (|a_l0|^2 + 2 sum_{m>=1} |a_lm|^2) / (2l+1); one lane per (map, l)
__global__ void alm2cl_kernel(const double2 *__restrict__ alm, int32_t lmax, int64_t n_alm, double *__restrict__ cl) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax) return;
    const double2 *a = alm + (int64_t)blockIdx.y * n_alm;
    double s = 0.0;
    for (int m = 0; m <= l; ++m) {
        const double2 v = a[(int64_t)m * (2 * lmax + 1 - m) / 2 + l];
        const double p = v.x * v.x + v.y * v.y;
        s += m == 0 ? p : 2.0 * p;
    }
    cl[(int64_t)blockIdx.y * (lmax + 1) + l] = s / (double)(2 * l + 1);
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
    for (int r = 0; r < R; ++r) s += X[(int64_t)r * nb + b];
    mean[b] = s / (double)R;
}

// cov[b][c] = sum_r (X[r][b] - mean[b]) (X[r][c] - mean[c]) / (R - ddof), r in order
__global__ void cov_kernel(const double *__restrict__ X, const double *__restrict__ mean, int32_t R, int32_t nb,
                           double denom, double *__restrict__ cov) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (c >= nb) return;
    const double mb = mean[b], mc = mean[c];
    double s = 0.0;
    for (int r = 0; r < R; ++r) {
        const double *row = X + (int64_t)r * nb;
        s = fma(row[b] - mb, row[c] - mc, s);
    }
    cov[(int64_t)b * nb + c] = s / denom;
}

__global__ void corr_kernel(const double *__restrict__ cov, int32_t nb, double *__restrict__ corr) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (c >= nb) return;
    const double sb = sqrt(cov[(int64_t)b * nb + b]), sc = sqrt(cov[(int64_t)c * nb + c]);
    corr[(int64_t)b * nb + c] = cov[(int64_t)b * nb + c] / (sb * sc);
}

// ------------------------------------------------------------------ host side
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

    hipLaunchKernelGGL(lambda_seed_kernel, dim3(blocks_for(L.npair, 256)), dim3(256), 0, s, N, lmax, seed, seed_k);
    hipLaunchKernelGGL(legendre_coef_kernel, dim3(blocks_for(M, 256), (unsigned)M), dim3(256), 0, s, lmax, coef);
    UFX_HIP_CHECK(hipGetLastError());
    const double w = 4.0 * M_PI / (double)npix;
    const dim3 dft_x((unsigned)((M + kDftThreads - 1) / kDftThreads));
    for (int32_t t = 0; t < n_maps; ++t) {
        double2 *a = reinterpret_cast<double2 *>(alm) + (int64_t)t * L.nalm;
        if (dtype == UFALCON_F32) {
            const float *mp = static_cast<const float *>(maps) + t * npix;
            if (N > 1)
                hipLaunchKernelGGL((ring_dft_kernel<float, true>), dim3(dft_x.x, (unsigned)(N - 1)), dim3(kDftThreads),
                                   0, s, mp, N, lmax, F);
            hipLaunchKernelGGL((ring_dft_kernel<float, false>),
                               dim3(dft_x.x, (unsigned)((2 * N + 1 + kEqRings - 1) / kEqRings)), dim3(kDftThreads), 0,
                               s, mp, N, lmax, F);
        } else {
            const double *mp = static_cast<const double *>(maps) + t * npix;
            if (N > 1)
                hipLaunchKernelGGL((ring_dft_kernel<double, true>), dim3(dft_x.x, (unsigned)(N - 1)),
                                   dim3(kDftThreads), 0, s, mp, N, lmax, F);
            hipLaunchKernelGGL((ring_dft_kernel<double, false>),
                               dim3(dft_x.x, (unsigned)((2 * N + 1 + kEqRings - 1) / kEqRings)), dim3(kDftThreads), 0,
                               s, mp, N, lmax, F);
        }
        double2 *dst = L.n_rb > 1 ? part : a;
        hipLaunchKernelGGL(legendre_kernel, dim3((unsigned)M, (unsigned)L.n_rb), dim3(kLegThreads), 0, s, F, seed,
                           seed_k, coef, N, lmax, w, dst, L.n_rb > 1 ? L.nalm : (int64_t)0);
        if (L.n_rb > 1)
            hipLaunchKernelGGL(sum_partials_kernel, dim3(blocks_for(L.nalm, 256)), dim3(256), 0, s, part, L.n_rb,
                               L.nalm, a);
        UFX_HIP_CHECK(hipGetLastError());
    }
    return UFALCON_OK;
}

extern "C" int ufalcon_alm2cl(const double *alm, int32_t n_maps, int32_t lmax, double *cl, ufalcon_stream_t stream) {
    if (n_maps < 0 || lmax < 0 || lmax > kMaxLmax) return UFALCON_EINVAL;
    if (n_maps == 0) return UFALCON_OK;
    if (!alm || !cl) return UFALCON_EINVAL;
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    hipLaunchKernelGGL(alm2cl_kernel, dim3(blocks_for((int64_t)lmax + 1, 256), (unsigned)n_maps), dim3(256), 0,
                       as_stream(stream), reinterpret_cast<const double2 *>(alm), lmax, nalm, cl);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

extern "C" size_t ufalcon_cl_covariance_workspace_size(int32_t n_real, int32_t n_bands) {
    if (n_real < 1 || n_bands < 1) return 0;
    return (size_t)n_real * (size_t)n_bands * sizeof(double);
}

extern "C" int ufalcon_cl_covariance(const double *cl, int32_t n_real, int32_t n_ell, int32_t ell_min,
                                     int32_t delta_ell, int32_t n_bands, int32_t ddof, double *band_mean, double *cov,
                                     double *corr, void *workspace, size_t workspace_bytes, ufalcon_stream_t stream) {
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
    hipLaunchKernelGGL(band_mean_kernel, dim3(blocks_for(n_bands, 256)), dim3(256), 0, s, X, n_real, n_bands,
                       band_mean);
    hipLaunchKernelGGL(cov_kernel, dim3(blocks_for(n_bands, 256), (unsigned)n_bands), dim3(256), 0, s, X, band_mean,
                       n_real, n_bands, (double)(n_real - ddof), cov);
    if (corr)
        hipLaunchKernelGGL(corr_kernel, dim3(blocks_for(n_bands, 256), (unsigned)n_bands), dim3(256), 0, s, cov,
                           n_bands, corr);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}
