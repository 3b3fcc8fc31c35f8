// Per-shell scalars of the Born sum: comoving distance, lensing weights with
// forward-mode derivatives, and 1/nbar (section 2.3 eqs. (1)-(6)).
//
// Cosmology: flat LambdaCDM, E(z) = sqrt(Om (1+z)^3 + 1 - Om), dimensionless
// comoving distance D(z) = int_0^z dz'/E(z') = (H0/c) chi(z).
//
// Weight of shell b for source bin t, written in D (dD = dz/E, so the shell
// limits D_b = chi_b / (c/H0) do not move when Om changes):
//   W_tb = (3/2) Om int_{D_b}^{D_b+1} (1 + z(D)) D q_t(D) dD
//   delta source at z_s:  q = 1 - D/D_s, integral clipped at D_s
//   n(z) on [0, z_max]:   q = int_{z(D)}^{z_max} nhat(z') (1 - D/D(z')) dz',
//                          nhat = n / int_0^{z_max} n,  n = z^alpha exp(-(z/z0)^beta)
// All integrals are fixed Gauss-Legendre rules; z(D) is Newton's inversion of D(z).
// Every quantity is a dual number carrying d/dOm and d/d(source parameters),
// so dW comes out exactly for the discretised integrals (forward mode).
#include "../../include/ufalcon.h"
#include "internal.hpp"
#include "gl_rules.hpp"

namespace ufx {

constexpr double kCoverH0 = 2997.92458;  // c/H0 in Mpc/h
constexpr int NP = UFALCON_NPARAM;

struct dual {
    double v;
    double d[NP];
};

__device__ __forceinline__ dual dconst(double v) {
    dual r;
    r.v = v;
#pragma unroll
    for (int k = 0; k < NP; ++k) r.d[k] = 0.0;
    return r;
}
__device__ __forceinline__ dual dvar(double v, int slot) {
    dual r = dconst(v);
    r.d[slot] = 1.0;
    return r;
}
__device__ __forceinline__ dual operator+(dual a, dual b) {
    a.v += b.v;
#pragma unroll
    for (int k = 0; k < NP; ++k) a.d[k] += b.d[k];
    return a;
}
__device__ __forceinline__ dual operator-(dual a, dual b) {
    a.v -= b.v;
#pragma unroll
    for (int k = 0; k < NP; ++k) a.d[k] -= b.d[k];
    return a;
}
__device__ __forceinline__ dual operator*(dual a, dual b) {
    dual r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < NP; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
__device__ __forceinline__ dual operator*(double s, dual a) {
    a.v *= s;
#pragma unroll
    for (int k = 0; k < NP; ++k) a.d[k] *= s;
    return a;
}
__device__ __forceinline__ dual operator+(double s, dual a) {
    a.v += s;
    return a;
}
__device__ __forceinline__ dual operator/(dual a, dual b) {
    dual r;
    const double inv = 1.0 / b.v;
    r.v = a.v * inv;
#pragma unroll
    for (int k = 0; k < NP; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * inv;
    return r;
}
__device__ __forceinline__ dual dsqrt(dual a) {
    dual r;
    r.v = sqrt(a.v);
    const double h = 0.5 / r.v;
#pragma unroll
    for (int k = 0; k < NP; ++k) r.d[k] = a.d[k] * h;
    return r;
}
__device__ __forceinline__ dual dexp(dual a) {
    dual r;
    r.v = exp(a.v);
#pragma unroll
    for (int k = 0; k < NP; ++k) r.d[k] = a.d[k] * r.v;
    return r;
}
__device__ __forceinline__ dual dlog(dual a) {
    dual r;
    r.v = log(a.v);
    const double inv = 1.0 / a.v;
#pragma unroll
    for (int k = 0; k < NP; ++k) r.d[k] = a.d[k] * inv;
    return r;
}

// ------------------------------------------------------------------ Gauss-Legendre
// Nodes and weights on [-1, 1], tabulated once from 60-digit roots of P_n.
constexpr int kGL_D = 32;   // D(z) on [0, z]
constexpr int kGL_O = 16;   // outer integral over a shell
constexpr int kGL_I = 48;   // inner n(z) integral over [z, z_max]
constexpr int kGL_N = 16;   // per panel of the n(z) normalisation
constexpr int kNormPanels = 14;
static_assert(sizeof(kGLDx) == kGL_D * sizeof(double) && sizeof(kGLOx) == kGL_O * sizeof(double) &&
                  sizeof(kGLIx) == kGL_I * sizeof(double) && sizeof(kGLNx) == kGL_N * sizeof(double),
              "rule sizes");

// ------------------------------------------------------------------ cosmology in duals
__device__ __forceinline__ dual inv_E(dual z, dual om) {
    const dual a = 1.0 + z;
    return dconst(1.0) / dsqrt(om * (a * a * a) + (1.0 + (-1.0) * om));
}

__device__ dual D_of_z(dual z, dual om) {
    dual s = dconst(0.0);
#pragma unroll 4
    for (int i = 0; i < kGL_D; ++i) {
        const dual zi = (0.5 * (1.0 + kGLDx[i])) * z;
        s = s + kGLDw[i] * inv_E(zi, om);
    }
    return 0.5 * (z * s);
}

__device__ double D_of_z_plain(double z, double om) {
    double s = 0.0;
#pragma unroll 8
    for (int i = 0; i < kGL_D; ++i) {
        const double zi = 0.5 * (1.0 + kGLDx[i]) * z;
        const double a = 1.0 + zi;
        s += kGLDw[i] / sqrt(om * a * a * a + 1.0 - om);
    }
    return 0.5 * z * s;
}

// z with D(z) = Dt: Newton in plain FP64, then two dual Newton steps that carry
// the tangents (dz = -(dD/dtheta - dDt) E at the root).
__device__ dual z_of_D(dual Dt, dual om) {
    // start from the second-order expansion D = z - (3/4) Om z^2 inverted, then Newton;
    // stop once the step is at the rounding level (quadratic convergence takes ~4 steps)
    double z = Dt.v * (1.0 + 0.75 * om.v * Dt.v);
    for (int it = 0; it < 40; ++it) {
        const double a = 1.0 + z;
        const double E = sqrt(om.v * a * a * a + 1.0 - om.v);
        const double dz = (D_of_z_plain(z, om.v) - Dt.v) * E;
        z -= dz;
        if (fabs(dz) <= 1e-15 * (1.0 + z)) break;
    }
    dual zd = dconst(z);
    for (int it = 0; it < 2; ++it) {
        const dual f = D_of_z(zd, om) - Dt;
        const dual invE = inv_E(zd, om);
        zd = zd - f / invE;
    }
    return zd;
}

// ------------------------------------------------------------------ source model
struct SrcParams {
    int kind;
    double zs, alpha, beta, z0, zmax;
};

__device__ __forceinline__ dual smail_n(dual z, dual alpha, dual beta, dual z0) {
    // z^alpha exp(-(z/z0)^beta) = exp(alpha ln z - exp(beta ln(z/z0)))
    const dual lz = dlog(z);
    const dual t = dexp(beta * (lz - dlog(z0)));
    return dexp(alpha * lz - t);
}

// ------------------------------------------------------------------ weights kernel
struct WeightParams {
    double om;
    int32_t T, B;
    double *W;      // [T][B]
    double *dW;     // [T][B][NP] or null
    SrcParams src[UFALCON_MAX_BINS];
    double D[UFALCON_MAX_SHELLS + 1];  // edges in units of c/H0
};

// Sum of one dual per thread over a kWThreads block, in a fixed tree order (the
// result does not depend on scheduling).  `red` holds kWThreads duals.
constexpr int kWThreads = kGL_O * kGL_I;  // one thread per (outer, inner) node pair
static_assert(kWThreads == 768 && kNormPanels * kGL_N <= kWThreads, "block shape");

__device__ dual block_sum(dual v, dual *red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    if (tid < 256) red[tid] = red[tid] + red[tid + 256] + red[tid + 512];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = red[tid] + red[tid + s];
        __syncthreads();
    }
    const dual r = red[0];
    __syncthreads();
    return r;
}

// One block per (t, b).  Thread (o, i) = (tid / kGL_I, tid % kGL_I) evaluates
// outer node o of the shell and inner node i of the n(z) integral at z(D_o).
__global__ __launch_bounds__(kWThreads) void lensing_weights_kernel(WeightParams p) {
    __shared__ dual red[kWThreads];
    __shared__ dual zmax_D_s;
    const int t = blockIdx.x / p.B, b = blockIdx.x % p.B;

    const SrcParams sp = p.src[t];
    const dual om = dvar(p.om, 0);
    const int tid = threadIdx.x;
    const bool delta = sp.kind == UFALCON_SOURCE_DELTA;
    dual alpha = dvar(sp.alpha, 1), beta = dvar(sp.beta, 2), z0 = dvar(sp.z0, 3);

    // normalisation of n(z) on graded panels [0, zmax 2^-13], ..., [zmax/2, zmax]
    dual norm = dconst(1.0);
    if (!delta) {
        dual s = dconst(0.0);
        if (tid < kNormPanels * kGL_N) {
            const int pnl = tid / kGL_N, i = tid % kGL_N;
            const double hi = sp.zmax * ldexp(1.0, -(kNormPanels - 1 - pnl));
            const double lo = pnl == 0 ? 0.0 : 0.5 * hi;
            const double zi = lo + 0.5 * (hi - lo) * (1.0 + kGLNx[i]);
            s = (0.5 * (hi - lo) * kGLNw[i]) * smail_n(dconst(zi), alpha, beta, z0);
        }
        norm = block_sum(s, red);
        if (tid == 0) zmax_D_s = D_of_z(dconst(sp.zmax), om);
    } else if (tid == 0) {
        zmax_D_s = D_of_z(dvar(sp.zs, 1), om);  // D_s, depends on Om and z_s
    }
    __syncthreads();

    // outer limits in D: [D_b, min(D_{b+1}, D_cut)]
    const dual Dcut = zmax_D_s;
    const double Dlo = p.D[b];
    dual Dhi = dconst(p.D[b + 1]);
    bool empty = false;
    if (Dcut.v <= Dlo) empty = true;
    else if (Dcut.v < Dhi.v) Dhi = Dcut;

    dual contrib = dconst(0.0);
    const int o = tid / kGL_I, i = tid % kGL_I;
    if (!empty) {
        const dual half = 0.5 * (Dhi + (-1.0) * dconst(Dlo));
        const dual Dk = dconst(Dlo) + (1.0 + kGLOx[o]) * half;
        if (delta) {
            if (i == 0) {
                const dual zk = z_of_D(Dk, om);
                const dual q = 1.0 + (-1.0) * (Dk / Dcut);
                contrib = (kGLOw[o] * half) * ((1.0 + zk) * (Dk * q));
            }
        } else {
            // inner node i of the integral over [zk, zmax]
            const dual zk = z_of_D(Dk, om);
            const dual span = 0.5 * (dconst(sp.zmax) - zk);
            const dual zi = zk + (1.0 + kGLIx[i]) * span;
            const dual Di = D_of_z(zi, om);
            const dual nz = smail_n(zi, alpha, beta, z0);
            const dual inner = (kGLIw[i] * span) * (nz * (1.0 + (-1.0) * (Dk / Di)));
            contrib = (kGLOw[o] * half) * ((1.0 + zk) * (Dk * inner));
        }
    }
    dual acc = block_sum(contrib, red);
    if (tid == 0) {
        if (!delta) acc = acc / norm;
        const dual Wd = (1.5 * om) * acc;
        p.W[t * p.B + b] = empty ? 0.0 : Wd.v;
        if (p.dW)
            for (int k = 0; k < NP; ++k) p.dW[((int64_t)t * p.B + b) * NP + k] = empty ? 0.0 : Wd.d[k];
    }
}

__global__ void comoving_distance_kernel(const double *z, int64_t n, double om, double *chi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) chi[i] = kCoverH0 * D_of_z_plain(z[i], om);
}

__global__ void weights_vjp_kernel(const double *dW, const double *gW, int32_t T, int32_t B, double *out) {
    const int k = threadIdx.x;
    if (k >= T * NP) return;
    const int t = k / NP, j = k % NP;
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += gW[t * B + b] * dW[((int64_t)t * B + b) * NP + j];
    out[k] = s;
}

struct NbarParams {
    double dens_over_npix;
    int32_t b0, b1, mode;
    double *inv_nbar;
    double e[UFALCON_MAX_SHELLS + 1];
};

__global__ void inv_nbar_kernel(NbarParams p) {
    const int b = p.b0 + threadIdx.x;
    if (b >= p.b1) return;
    const double e0 = p.e[b], e1 = p.e[b + 1];
    double vol;
    if (p.mode == UFALCON_NBAR_EXACT_VOLUME)
        vol = (4.0 * M_PI / 3.0) * (e1 - e0) * (e1 * e1 + e1 * e0 + e0 * e0);
    else
        vol = 4.0 * M_PI * e0 * e0 * (e1 - e0);
    p.inv_nbar[b] = 1.0 / (p.dens_over_npix * vol);
}

}  // namespace ufx

using namespace ufx;

extern "C" int ufalcon_comoving_distance(const double *z, int64_t n, double omega_m, double *chi,
                                         ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_comoving_distance");
    if (n < 0 || (n > 0 && (!z || !chi)) || !std::isfinite(omega_m) || omega_m < 0.0 || omega_m > 1.0)
        return UFALCON_EINVAL;
    if (n == 0) return UFALCON_OK;
    hipLaunchKernelGGL(comoving_distance_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, as_stream(stream), z, n,
                       omega_m, chi);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

extern "C" int ufalcon_lensing_weights(double omega_m, const ufalcon_source *sources, int32_t T,
                                       const double *chi_edges, int32_t n_shells, double *W, double *dW,
                                       ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_lensing_weights");
    if (!sources || !W || T < 1) return UFALCON_EINVAL;
    if (T > UFALCON_MAX_BINS) return UFALCON_ETOO_MANY_SHELLS;
    if (!std::isfinite(omega_m) || !(omega_m > 0.0) || omega_m > 1.0) return UFALCON_EINVAL;
    int rc = check_edges(chi_edges, n_shells);
    if (rc) return rc;
    WeightParams p{};
    p.om = omega_m;
    p.T = T;
    p.B = n_shells;
    p.W = W;
    p.dW = dW;
    for (int t = 0; t < T; ++t) {
        const ufalcon_source &s = sources[t];
        SrcParams &d = p.src[t];
        d.kind = s.kind;
        if (s.kind == UFALCON_SOURCE_DELTA) {
            if (!std::isfinite(s.z_s) || !(s.z_s > 0.0)) return UFALCON_EINVAL;
            d.zs = s.z_s;
            d.alpha = d.beta = d.z0 = d.zmax = 0.0;
        } else if (s.kind == UFALCON_SOURCE_SMAIL) {
            if (!(s.alpha >= 0.0) || !(s.beta > 0.0) || !(s.z0 > 0.0) || !(s.z_max > 0.0) ||
                !std::isfinite(s.alpha) || !std::isfinite(s.beta) || !std::isfinite(s.z0) || !std::isfinite(s.z_max))
                return UFALCON_EINVAL;
            d.zs = 0.0;
            d.alpha = s.alpha;
            d.beta = s.beta;
            d.z0 = s.z0;
            d.zmax = s.z_max;
        } else {
            return UFALCON_EINVAL;
        }
    }
    for (int j = 0; j <= n_shells; ++j) p.D[j] = chi_edges[j] / kCoverH0;
    hipLaunchKernelGGL(lensing_weights_kernel, dim3(T * n_shells), dim3(kWThreads), 0, as_stream(stream), p);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

extern "C" int ufalcon_lensing_weights_vjp(const double *dW, const double *grad_W, int32_t T, int32_t n_shells,
                                           double *grad_theta, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_lensing_weights_vjp");
    if (!dW || !grad_W || !grad_theta || T < 1 || n_shells < 1) return UFALCON_EINVAL;
    if (T > UFALCON_MAX_BINS || n_shells > UFALCON_MAX_SHELLS) return UFALCON_ETOO_MANY_SHELLS;
    hipLaunchKernelGGL(weights_vjp_kernel, dim3(1), dim3(64), 0, as_stream(stream), dW, grad_W, T, n_shells,
                       grad_theta);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

extern "C" int ufalcon_inv_nbar(int64_t n_src, double box_L, const double *chi_edges, int32_t n_shells,
                                int32_t shell_begin, int32_t shell_end, int64_t nside, int32_t mode,
                                double *inv_nbar, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_inv_nbar");
    if (n_src <= 0 || !std::isfinite(box_L) || !(box_L > 0.0) || !inv_nbar) return UFALCON_EINVAL;
    if (mode != UFALCON_NBAR_EXACT_VOLUME && mode != UFALCON_NBAR_LOWER_EDGE) return UFALCON_EINVAL;
    int rc = check_edges(chi_edges, n_shells);
    if (rc) return rc;
    if ((rc = check_nside(nside))) return rc;
    if (shell_begin < 0 || shell_begin > shell_end || shell_end > n_shells) return UFALCON_EINVAL;
    if (mode == UFALCON_NBAR_LOWER_EDGE && shell_begin < shell_end && chi_edges[shell_begin] == 0.0)
        return UFALCON_EINVAL;  // lower-edge volume vanishes at chi = 0
    if (shell_begin == shell_end) return UFALCON_OK;
    NbarParams p{};
    p.dens_over_npix = ((double)n_src / (box_L * box_L * box_L)) / (double)npix_of(nside);
    p.b0 = shell_begin;
    p.b1 = shell_end;
    p.mode = mode;
    p.inv_nbar = inv_nbar;
    for (int j = 0; j <= n_shells; ++j) p.e[j] = chi_edges[j];
    hipLaunchKernelGGL(inv_nbar_kernel, dim3(1), dim3(UFALCON_MAX_SHELLS), 0, as_stream(stream), p);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}
