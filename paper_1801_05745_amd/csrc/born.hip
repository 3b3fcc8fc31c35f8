// Born convergence sum and its adjoint (section 2.3 eqs. (2), (6), (7)).
//
//   kappa[t][p]  = sum_b W[t][b] (n_b[p] / nbar_b - 1)
//   grad_W[t][b] = sum_p g[t][p] (n_b[p] / nbar_b - 1)
//
// Both are streaming passes over the uint32 count maps: about 2 FLOP per
// 4-byte count, far below the FP64 ridge, so they are bound by HBM and MFMA
// has no role.  Each lane owns one or two quads of consecutive pixels and reads
// 16 bytes per quad and shell row (a wavefront reads 1 KiB contiguous per quad
// and row), accumulates in FP64 in shell order and rounds once.  The adjoint reduces over pixels in two
// stages with a fixed partition of the pixels, so its result is bitwise
// reproducible run to run.
#include "../../include/ufalcon.h"
#include "internal.hpp"

namespace ufx {

constexpr int kBornBlock = 256;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// streaming 16-byte loads that should not displace reused data in the caches
__device__ __forceinline__ u32x4 ld_stream_u4(const uint32_t *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
}

struct BornParams {
    const uint32_t *counts;
    int64_t npix;
    int32_t B, T;
    const double *W;         // [T][B] device, or null: use w_inline (T = 1)
    const double *inv_nbar;  // [B]
    void *out;               // [T][npix]
    double w_inline[UFALCON_MAX_SHELLS];
};

// Quads of pixels per lane: two for one or two source bins (more 16-byte loads in
// flight per shell row), one for more bins (their accumulators fill the registers).
template <int TT>
constexpr int born_quads() { return TT <= 2 ? 2 : 1; }
template <int TT>
constexpr int64_t born_pix_per_block() { return (int64_t)kBornBlock * 4 * born_quads<TT>(); }

// One block: pixels [blk * P, blk * P + P) of one map, P = born_pix_per_block;
// thread i owns the quads at blk * P + 4 i + 1024 h, h < born_quads.
template <int TT, typename OutT>
__device__ __forceinline__ void born_block(const uint32_t *counts, int64_t npix, int B, const double *W,
                                           const double *w_inline, const double *inv_nbar, void *out, int64_t blk,
                                           double *a_s, double *c_s) {
    constexpr int Q = born_quads<TT>();
    for (int k = threadIdx.x; k < TT * B; k += kBornBlock) {
        const int b = k % B;
        const double w = W ? W[k] : w_inline[b];
        a_s[k] = w * inv_nbar[b];
    }
    if (threadIdx.x < TT) {
        double c = 0.0;
        for (int b = 0; b < B; ++b) c += W ? W[threadIdx.x * B + b] : w_inline[b];
        c_s[threadIdx.x] = c;
    }
    __syncthreads();

    // npix = 12 Nside^2 is a multiple of 4: quads are whole.  A quad past the end
    // repeats the load of the first one and is not written.
    const int64_t first = blk * born_pix_per_block<TT>() + (int64_t)threadIdx.x * 4;
    if (first >= npix) return;
    int64_t pq[Q];
    bool in[Q];
#pragma unroll
    for (int h = 0; h < Q; ++h) {
        const int64_t p = first + (int64_t)h * kBornBlock * 4;
        in[h] = p < npix;
        pq[h] = in[h] ? p : first;
    }
    double acc[TT][4 * Q];
#pragma unroll
    for (int t = 0; t < TT; ++t)
#pragma unroll
        for (int j = 0; j < 4 * Q; ++j) acc[t][j] = 0.0;

    int b = 0;
    for (; b + 4 <= B; b += 4) {
        u32x4 v[4][Q];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int h = 0; h < Q; ++h) v[u][h] = ld_stream_u4(counts + (int64_t)(b + u) * npix + pq[h]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int t = 0; t < TT; ++t) {
                const double a = a_s[t * B + b + u];
#pragma unroll
                for (int h = 0; h < Q; ++h) {
                    acc[t][4 * h + 0] += a * (double)v[u][h].x;
                    acc[t][4 * h + 1] += a * (double)v[u][h].y;
                    acc[t][4 * h + 2] += a * (double)v[u][h].z;
                    acc[t][4 * h + 3] += a * (double)v[u][h].w;
                }
            }
        }
    }
    for (; b < B; ++b) {
        u32x4 v[Q];
#pragma unroll
        for (int h = 0; h < Q; ++h) v[h] = ld_stream_u4(counts + (int64_t)b * npix + pq[h]);
#pragma unroll
        for (int t = 0; t < TT; ++t) {
            const double a = a_s[t * B + b];
#pragma unroll
            for (int h = 0; h < Q; ++h) {
                acc[t][4 * h + 0] += a * (double)v[h].x;
                acc[t][4 * h + 1] += a * (double)v[h].y;
                acc[t][4 * h + 2] += a * (double)v[h].z;
                acc[t][4 * h + 3] += a * (double)v[h].w;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < TT; ++t) {
        const double c = c_s[t];
#pragma unroll
        for (int h = 0; h < Q; ++h) {
            if (!in[h]) continue;
            OutT *o = static_cast<OutT *>(out) + (int64_t)t * npix + pq[h];
            const double *r = acc[t] + 4 * h;
            if constexpr (sizeof(OutT) == 4) {
                float4 f = {(float)(r[0] - c), (float)(r[1] - c), (float)(r[2] - c), (float)(r[3] - c)};
                *reinterpret_cast<float4 *>(o) = f;
            } else {
                double2 r0 = {r[0] - c, r[1] - c};
                double2 r1 = {r[2] - c, r[3] - c};
                reinterpret_cast<double2 *>(o)[0] = r0;
                reinterpret_cast<double2 *>(o)[1] = r1;
            }
        }
    }
}

template <int TT, typename OutT>
__global__ __launch_bounds__(kBornBlock) void born_kernel(BornParams p) {
    __shared__ double a_s[UFALCON_MAX_BINS * UFALCON_MAX_SHELLS];
    __shared__ double c_s[UFALCON_MAX_BINS];
    born_block<TT, OutT>(p.counts, p.npix, p.B, p.W, p.w_inline, p.inv_nbar, p.out, blockIdx.x, a_s, c_s);
}

struct BornItemDev {
    const uint32_t *counts;  // [B][npix]
    const double *W;         // [T][B]
    const double *inv_nbar;  // [B]
    void *kappa;             // [T][npix]
    int32_t B;
    int32_t pad;
};

// One launch for a batch of maps: block = (map, pixel block), map-major.
template <int TT, typename OutT>
__global__ __launch_bounds__(kBornBlock) void born_batched_kernel(const BornItemDev *items, int64_t npix,
                                                                  int64_t blocks_per_map) {
    __shared__ double a_s[UFALCON_MAX_BINS * UFALCON_MAX_SHELLS];
    __shared__ double c_s[UFALCON_MAX_BINS];
    const int64_t m = blockIdx.x / blocks_per_map;
    const int64_t blk = blockIdx.x % blocks_per_map;
    const BornItemDev it = items[m];
    born_block<TT, OutT>(it.counts, npix, it.B, it.W, nullptr, it.inv_nbar, it.kappa, blk, a_s, c_s);
}

template <typename OutT>
int launch_born_t(const BornParams &p, hipStream_t s) {
    switch (p.T) {
#define UFX_BORN_CASE(k)                                                                            \
        case k:                                                                                     \
            hipLaunchKernelGGL((born_kernel<k, OutT>), dim3(blocks_for(p.npix, born_pix_per_block<k>(), 1u << 30)), \
                               dim3(kBornBlock), 0, s, p);                                          \
            break;
        UFX_BORN_CASE(1) UFX_BORN_CASE(2) UFX_BORN_CASE(3) UFX_BORN_CASE(4)
        UFX_BORN_CASE(5) UFX_BORN_CASE(6) UFX_BORN_CASE(7) UFX_BORN_CASE(8)
#undef UFX_BORN_CASE
        default: return UFALCON_ETOO_MANY_SHELLS;
    }
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

int launch_born(const BornParams &p, int out_dtype, hipStream_t s) {
    return out_dtype == UFALCON_F32 ? launch_born_t<float>(p, s) : launch_born_t<double>(p, s);
}

template <typename OutT>
int launch_born_batched_t(const BornItemDev *items, int32_t n_items, int64_t npix, int32_t T, hipStream_t s) {
    switch (T) {
#define UFX_BORNB_CASE(k)                                                                               \
        case k: {                                                                                      \
            const int64_t bpm = (npix + born_pix_per_block<k>() - 1) / born_pix_per_block<k>();       \
            hipLaunchKernelGGL((born_batched_kernel<k, OutT>), dim3((unsigned)(bpm * n_items)), dim3(kBornBlock), 0, \
                               s, items, npix, bpm);                                                   \
            break;                                                                                     \
        }
        UFX_BORNB_CASE(1) UFX_BORNB_CASE(2) UFX_BORNB_CASE(3) UFX_BORNB_CASE(4)
        UFX_BORNB_CASE(5) UFX_BORNB_CASE(6) UFX_BORNB_CASE(7) UFX_BORNB_CASE(8)
#undef UFX_BORNB_CASE
        default: return UFALCON_ETOO_MANY_SHELLS;
    }
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

int launch_born_batched(const BornItemDev *items, int32_t n_items, int64_t npix, int32_t T, int out_dtype,
                        hipStream_t s) {
    return out_dtype == UFALCON_F32 ? launch_born_batched_t<float>(items, n_items, npix, T, s)
                                    : launch_born_batched_t<double>(items, n_items, npix, T, s);
}

// ------------------------------------------------------------------ adjoint
constexpr int kAdjBlock = 256;
constexpr int64_t kAdjPixPerBlock = 2048;  // fixed pixel partition of stage 1 (4096: 5 % slower, 16384: 15 %)

struct AdjParams {
    const uint32_t *counts;
    int64_t npix;
    int32_t B, T, SB, nchunk;
    const void *g;            // [T][npix]
    double *partial;          // [G][T][B]
    double *partial0;         // [G][T]
    int64_t G;
};

template <typename GT>
__device__ __forceinline__ void load4(const GT *g, double out[4]) {
    if constexpr (sizeof(GT) == 4) {
        const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(g));
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
        const double2 v0 = reinterpret_cast<const double2 *>(g)[0];
        const double2 v1 = reinterpret_cast<const double2 *>(g)[1];
        out[0] = v0.x; out[1] = v0.y; out[2] = v1.x; out[3] = v1.y;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }
constexpr int pow2_at_least(int v) { return v <= 1 ? 1 : 2 * pow2_at_least((v + 1) / 2); }

// Sum of each of P (a power of two <= 64) per-lane values over the wave, spread
// over the lanes: every step exchanges half of the remaining values with the
// lane `off` away and keeps the half its lane bit selects (P/2 + P/4 + ... + 1
// shuffles instead of 6 per value), then xor steps over the lane bits left
// complete the sums.  Lane L returns the sum of value L >> (6 - log2 P).  The
// tree is fixed, so the result is the same on every run.
template <int P, int kOff = 32>
__device__ __forceinline__ double wave_reduce_scatter(double *v) {
    if constexpr (P > 1) {
        constexpr int n = P / 2;
        const bool upper = (threadIdx.x & kOff) != 0;
#pragma unroll
        for (int k = 0; k < n; ++k) {
            const double send = upper ? v[k] : v[k + n];
            const double keep = upper ? v[k + n] : v[k];
            v[k] = keep + __shfl_xor(send, kOff, 64);
        }
        return wave_reduce_scatter<n, kOff / 2>(v);
    } else {
        double r = v[0];
#pragma unroll
        for (int off = kOff; off >= 1; off >>= 1) r += __shfl_xor(r, off, 64);
        return r;
    }
}

// Stage 1: block (chunk c, pixel range gblk) accumulates S1[t][b] for the shells of
// chunk c and, for chunk 0, S0[t] = sum_p g[t][p].
template <int TT, int SB, typename GT>
__global__ __launch_bounds__(kAdjBlock) void adjoint_stage1(AdjParams p) {
    __shared__ double red[kAdjBlock / 64][TT * SB + TT];
    const int64_t gblk = blockIdx.x / p.nchunk;
    const int chunk = blockIdx.x % p.nchunk;
    const int b0 = chunk * SB;
    const int nb = (p.B - b0) < SB ? (p.B - b0) : SB;
    const int64_t pbeg = gblk * kAdjPixPerBlock;
    const int64_t pend = (pbeg + kAdjPixPerBlock) < p.npix ? (pbeg + kAdjPixPerBlock) : p.npix;
    double acc[TT][SB];
    double acc0[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
        acc0[t] = 0.0;
#pragma unroll
        for (int k = 0; k < SB; ++k) acc[t][k] = 0.0;
    }
    const GT *g = static_cast<const GT *>(p.g);
    for (int64_t q = pbeg + (int64_t)threadIdx.x * 4; q < pend; q += kAdjBlock * 4) {
        double gv[TT][4];
#pragma unroll
        for (int t = 0; t < TT; ++t) {
            load4<GT>(g + (int64_t)t * p.npix + q, gv[t]);
            acc0[t] += (gv[t][0] + gv[t][1]) + (gv[t][2] + gv[t][3]);
        }
#pragma unroll
        for (int k = 0; k < SB; ++k) {
            if (k < nb) {
                const u32x4 v = ld_stream_u4(p.counts + (int64_t)(b0 + k) * p.npix + q);
#pragma unroll
                for (int t = 0; t < TT; ++t)
                    acc[t][k] += (gv[t][0] * (double)v.x + gv[t][1] * (double)v.y) +
                                 (gv[t][2] * (double)v.z + gv[t][3] * (double)v.w);
            }
        }
    }
    // Every sum over the wave first (one fixed reduce-scatter tree), then over
    // the waves in order, all behind one barrier.
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    constexpr int P = pow2_at_least(TT * SB);
    constexpr int kSh = 6 - ilog2(P);
    static_assert(P <= 64, "one value per lane at most");
    double vals[P];
#pragma unroll
    for (int i = 0; i < P; ++i) vals[i] = i < TT * SB ? acc[i / SB][i % SB] : 0.0;
    const double r = wave_reduce_scatter<P>(vals);
    if ((lane & ((1 << kSh) - 1)) == 0 && (lane >> kSh) < TT * SB) red[w][lane >> kSh] = r;
#pragma unroll
    for (int t = 0; t < TT; ++t) {
        const double v0 = wave_sum(acc0[t]);
        if (lane == 0) red[w][TT * SB + t] = v0;
    }
    __syncthreads();
    double *out = p.partial + gblk * (int64_t)p.T * p.B;
    for (int i = threadIdx.x; i < TT * SB + TT; i += kAdjBlock) {
        double s = 0.0;
        for (int k = 0; k < kAdjBlock / 64; ++k) s += red[k][i];  // fixed order
        if (i < TT * SB) {
            const int t = i / SB, k = i % SB;
            if (k < nb) out[t * p.B + b0 + k] = s;
        } else if (chunk == 0) {
            p.partial0[gblk * p.T + (i - TT * SB)] = s;
        }
    }
}

// Stage 2: grad_W[t][b] = inv_nbar[b] * sum_blocks S1 - sum_blocks S0.  One workgroup
// per (t, b); thread j sums blocks j, j + 1024, ... in that order (four loads in
// flight), then a fixed-shape tree over the 1024 partial sums: the same order on
// every run.
constexpr int kS2Threads = 1024;
__global__ __launch_bounds__(kS2Threads) void adjoint_stage2(const double *partial, const double *partial0, int64_t G,
                                                             int32_t T, int32_t B, const double *inv_nbar,
                                                             double *grad_W) {
    __shared__ double r1[kS2Threads], r0[kS2Threads];
    const int k = blockIdx.x;
    const int t = k / B, b = k % B;
    const int64_t TB = (int64_t)T * B;
    double s1 = 0.0, s0 = 0.0;
    int64_t i = threadIdx.x;
    for (; i + 3 * kS2Threads < G; i += 4 * kS2Threads) {
        double a[4], c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = partial[(i + u * kS2Threads) * TB + k];
            c[u] = partial0[(i + u * kS2Threads) * T + t];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            s1 += a[u];
            s0 += c[u];
        }
    }
    for (; i < G; i += kS2Threads) {
        s1 += partial[i * TB + k];
        s0 += partial0[i * T + t];
    }
    r1[threadIdx.x] = s1;
    r0[threadIdx.x] = s0;
    __syncthreads();
    for (int off = kS2Threads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            r1[threadIdx.x] += r1[threadIdx.x + off];
            r0[threadIdx.x] += r0[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) grad_W[k] = inv_nbar[b] * r1[0] - r0[0];
}

int64_t adjoint_blocks(int64_t npix) { return (npix + kAdjPixPerBlock - 1) / kAdjPixPerBlock; }

template <int TT, typename GT>
int launch_adj_t(AdjParams p, hipStream_t s) {
    constexpr int SB = TT == 1 ? 32 : (TT == 2 ? 16 : 8);
    p.SB = SB;
    p.nchunk = (p.B + SB - 1) / SB;
    const int64_t grid = p.G * p.nchunk;
    hipLaunchKernelGGL((adjoint_stage1<TT, SB, GT>), dim3((unsigned)grid), dim3(kAdjBlock), 0, s, p);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

template <typename GT>
int launch_adj(AdjParams p, hipStream_t s) {
    switch (p.T) {
        case 1: return launch_adj_t<1, GT>(p, s);
        case 2: return launch_adj_t<2, GT>(p, s);
        case 3: return launch_adj_t<3, GT>(p, s);
        case 4: return launch_adj_t<4, GT>(p, s);
        case 5: return launch_adj_t<5, GT>(p, s);
        case 6: return launch_adj_t<6, GT>(p, s);
        case 7: return launch_adj_t<7, GT>(p, s);
        case 8: return launch_adj_t<8, GT>(p, s);
        default: return UFALCON_ETOO_MANY_SHELLS;
    }
}

}  // namespace ufx

using namespace ufx;

static int check_born_common(const uint32_t *counts, int32_t n_shells, int64_t nside, int32_t T) {
    if (!counts) return UFALCON_EINVAL;
    if (n_shells < 1) return UFALCON_EINVAL;
    if (n_shells > UFALCON_MAX_SHELLS) return UFALCON_ETOO_MANY_SHELLS;
    if (T < 1 || T > UFALCON_MAX_BINS) return T < 1 ? UFALCON_EINVAL : UFALCON_ETOO_MANY_SHELLS;
    if (((uintptr_t)counts & 15u)) return UFALCON_EINVAL;
    return check_nside(nside);
}

extern "C" int ufalcon_born_kappa(const uint32_t *counts, int32_t n_shells, int64_t nside, const double *W,
                                  const double *inv_nbar, int32_t T, void *kappa, int out_dtype,
                                  ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_born_kappa");
    int rc = check_born_common(counts, n_shells, nside, T);
    if (rc) return rc;
    if (!W || !inv_nbar || !kappa || (out_dtype != UFALCON_F32 && out_dtype != UFALCON_F64)) return UFALCON_EINVAL;
    if ((uintptr_t)kappa & 15u) return UFALCON_EINVAL;
    BornParams p{};
    p.counts = counts;
    p.npix = npix_of(nside);
    p.B = n_shells;
    p.T = T;
    p.W = W;
    p.inv_nbar = inv_nbar;
    p.out = kappa;
    return launch_born(p, out_dtype, as_stream(stream));
}

extern "C" int ufalcon_overdensity(const uint32_t *counts, int32_t n_shells, int64_t nside, const double *chi_edges,
                                   const double *inv_nbar, void *delta, int out_dtype, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_overdensity");
    int rc = check_born_common(counts, n_shells, nside, 1);
    if (rc) return rc;
    if ((rc = check_edges(chi_edges, n_shells))) return rc;
    if (!inv_nbar || !delta || (out_dtype != UFALCON_F32 && out_dtype != UFALCON_F64)) return UFALCON_EINVAL;
    if ((uintptr_t)delta & 15u) return UFALCON_EINVAL;
    BornParams p{};
    p.counts = counts;
    p.npix = npix_of(nside);
    p.B = n_shells;
    p.T = 1;
    p.W = nullptr;
    p.inv_nbar = inv_nbar;
    p.out = delta;
    const double total = chi_edges[n_shells] - chi_edges[0];
    for (int b = 0; b < n_shells; ++b) p.w_inline[b] = (chi_edges[b + 1] - chi_edges[b]) / total;
    return launch_born(p, out_dtype, as_stream(stream));
}

extern "C" size_t ufalcon_born_kappa_adjoint_workspace_size(int32_t n_shells, int64_t nside, int32_t T) {
    if (n_shells < 1 || T < 1 || nside < 1) return 0;
    const int64_t G = adjoint_blocks(npix_of(nside));
    return (size_t)G * (size_t)T * ((size_t)n_shells + 1) * sizeof(double) + 256;
}

extern "C" int ufalcon_born_kappa_adjoint(const uint32_t *counts, int32_t n_shells, int64_t nside,
                                          const double *inv_nbar, const void *grad_kappa, int grad_dtype, int32_t T,
                                          double *grad_W, void *workspace, size_t workspace_bytes,
                                          ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_born_kappa_adjoint");
    int rc = check_born_common(counts, n_shells, nside, T);
    if (rc) return rc;
    if (!inv_nbar || !grad_kappa || !grad_W || (grad_dtype != UFALCON_F32 && grad_dtype != UFALCON_F64))
        return UFALCON_EINVAL;
    if ((uintptr_t)grad_kappa & 15u) return UFALCON_EINVAL;
    if (!workspace || workspace_bytes < ufalcon_born_kappa_adjoint_workspace_size(n_shells, nside, T) ||
        ((uintptr_t)workspace & 255u))
        return UFALCON_EWORKSPACE;
    AdjParams p{};
    p.counts = counts;
    p.npix = npix_of(nside);
    p.B = n_shells;
    p.T = T;
    p.g = grad_kappa;
    p.G = adjoint_blocks(p.npix);
    p.partial = static_cast<double *>(workspace);
    p.partial0 = p.partial + p.G * (int64_t)T * n_shells;
    hipStream_t s = as_stream(stream);
    rc = grad_dtype == UFALCON_F32 ? launch_adj<float>(p, s) : launch_adj<double>(p, s);
    if (rc) return rc;
    hipLaunchKernelGGL(adjoint_stage2, dim3(T * n_shells), dim3(kS2Threads), 0, s, p.partial, p.partial0, p.G, T,
                       n_shells, inv_nbar, grad_W);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}
