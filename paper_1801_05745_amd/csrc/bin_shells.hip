// Shell binning: particles -> (radial shell, HEALPix RING pixel) count maps,
// plain and batched.
//
// Section 2.3 eq. (5) counts n_p(pix, Delta chi_b), the particles of shell b in
// pixel pix; section 2.4 eq. (8) assigns shells by comoving radius around an
// observer at the box centre, and builds the map from independent subvolumes
// whose maps are summed.  On one GPU the subvolumes are particle tiles: every
// wavefront streams its particles (coalesced SoA loads), generates their
// periodic images, and adds one to the count cell of every image in range.
//
// Per wavefront the work is split in two phases to keep the 64 lanes busy:
//   A. each lane walks the images of its particle and tests the squared radius
//      against the (guard-widened) shell range: cheap FP64 adds and multiplies;
//      images in range are appended to a per-wave queue in LDS (ballot prefix);
//   B. whenever 64 queued images are ready, every lane takes one and runs the
//      FP64 shell search and RING pixelisation, then one global atomic add.
// Without the queue, phase B would run for every image slot with only the
// in-range lanes active (about a third for the configurations of interest).
//
// Instances whose FP64 decisions fall inside a guard band (a few per 10^8) are
// not decided here: their vectors go to a list in the caller's workspace and a
// second kernel decides them exactly (exact.hpp).  Keeping the exact code out of
// the streaming kernel keeps its register count, and so its occupancy, low.  If
// the list overflows, a third kernel (which otherwise exits at once) re-walks
// all images and decides every guarded one exactly, and the list is ignored.
//
// The batched form (many realisations, section 3.2's 150 maps) runs the same
// per-wave core in a persistent kernel whose workgroups pull (realisation,
// tile) items from an atomic work counter until the queue is empty.
#include "binning_core.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

namespace ufx {


template <typename T, int kMode>
__global__ __launch_bounds__(kBinBlock) void bin_shells_kernel(BinParams p) {
    if (kMode == kRescue && p.guard->overflow == 0u) return;  // uniform: nothing to rescue
    __shared__ EdgeLds E;
    __shared__ double qbuf[kBinWaves][3 * kQueue];
    __shared__ double radii[kMode == kRescue ? UFALCON_MAX_SHELLS + 1 : 1];
    load_edges(E, p.c, p.e, kMode == kRescue ? radii : nullptr);
    const int w = threadIdx.x >> 6;
    const Shared sh = shared_of(p);
    LaneStats st;
    Emitter em{};
    WaveQueue q{qbuf[w], 0, 0};
    const int64_t base = (int64_t)blockIdx.x * kBinBlock + w * 64;
    const int64_t stride = (int64_t)gridDim.x * kBinBlock;
    bin_wave_range<T, kMode>(p.c, sh, E, base, p.c.n, stride, q, st, em);
    drain_queue<kMode>(p.c, sh, E, q, st, em);
    flush_stats(p.status, st);
}

// Exact decisions for the listed guarded instances (skipped after an overflow).
__global__ __launch_bounds__(256) void bin_guarded_kernel(BinParams p) {
    __shared__ double e_s[UFALCON_MAX_SHELLS + 1];
    for (int j = threadIdx.x; j <= p.c.nb; j += 256) e_s[j] = p.e[j];
    __syncthreads();
    if (p.guard->overflow != 0u) return;
    const unsigned int seen = p.guard->count;
    const int64_t m = (int64_t)seen < p.guard_cap ? (int64_t)seen : p.guard_cap;
    const GuardEntry *ent = reinterpret_cast<const GuardEntry *>(reinterpret_cast<const char *>(p.guard) + kGuardHeader);
    LaneStats st;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < m; k += (int64_t)gridDim.x * 256) {
        const int r = bin_instance_exact(p.c.counts, p.npix, p.nside, e_s, p.c.nb, ent[k].dx, ent[k].dy, ent[k].dz);
        st.inst += r & 1;
        st.unresolved += (r >> 1) & 1;
    }
    flush_stats(p.status, st);
}

__global__ void guard_reset_kernel(GuardList *g) {
    if (threadIdx.x == 0) {
        g->count = 0u;
        g->overflow = 0u;
        g->next = 0u;
        g->next_rescue = 0u;
    }
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // 16-byte stores over the aligned bulk, scalar stores for the ends
    const int64_t head = (int64_t)(((16u - ((uintptr_t)p & 15u)) & 15u) / 4u);
    const int64_t h = head < n ? head : n;
    if (i < h) p[i] = v;
    uint4 *q = reinterpret_cast<uint4 *>(p + h);
    const int64_t nv = (n - h) / 4;
    const uint4 vv = {v, v, v, v};
    for (int64_t k = i; k < nv; k += stride) q[k] = vv;
    const int64_t tail0 = h + nv * 4;
    if (i < n - tail0) p[tail0 + i] = v;
}

// out[i] (+)= counts[i] widened to int64
__global__ void widen_counts_kernel(const uint32_t *c, int64_t n, int64_t *out, int accumulate) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (accumulate ? out[i] : 0) + (int64_t)c[i];
}

// ------------------------------------------------------------------ batched
struct BatchItemDev {
    BinCore c;
    int32_t edge_off;      // first edge of the range in the plan's edge array
    int32_t pad;
    int64_t tile_begin;    // prefix sum of tiles over items
};

struct BatchParams {
    const BatchItemDev *items;
    const double *edges;
    int32_t n_items;
    int32_t pad;
    int64_t total_tiles;
    int64_t tile;          // particles per work item
    Shared sh;
    ufalcon_status *status;
};

__device__ __forceinline__ int find_item(const BatchItemDev *items, int n_items, int64_t t) {
    int lo = 0, hi = n_items;  // largest k with tile_begin <= t
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (items[mid].tile_begin <= t) lo = mid; else hi = mid;
    }
    return lo;
}

template <typename T, int kMode>
__global__ __launch_bounds__(kBinBlock) void bin_batched_kernel(BatchParams p) {
    if (kMode == kRescue && p.sh.guard->overflow == 0u) return;
    __shared__ EdgeLds E;
    __shared__ double qbuf[kBinWaves][3 * kQueue];
    __shared__ double radii[kMode == kRescue ? UFALCON_MAX_SHELLS + 1 : 1];
    __shared__ int64_t work;
    __shared__ int cur_item;
    const int w = threadIdx.x >> 6;
    if (threadIdx.x == 0) cur_item = -1;
    LaneStats st;
    Emitter em{};
    WaveQueue q{qbuf[w], 0, 0};
    unsigned int *ctr = kMode == kRescue ? &p.sh.guard->next_rescue : &p.sh.guard->next;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) work = (int64_t)atomicAdd(ctr, 1u);
        __syncthreads();
        const int64_t t = work;
        if (t >= p.total_tiles) break;  // uniform over the block: every wave exits here
        const int k = find_item(p.items, p.n_items, t);
        const BinCore c = p.items[k].c;
        if (k != cur_item) {  // uniform: `work` is shared
            __syncthreads();
            load_edges(E, c, p.edges + p.items[k].edge_off, kMode == kRescue ? radii : nullptr);
            if (threadIdx.x == 0) cur_item = k;
        }
        const int64_t first = (t - p.items[k].tile_begin) * p.tile;
        const int64_t last = first + p.tile < c.n ? first + p.tile : c.n;
        bin_wave_range<T, kMode>(c, p.sh, E, first + w * 64, last, kBinBlock, q, st, em);
        drain_queue<kMode>(c, p.sh, E, q, st, em);
    }
    flush_stats(p.status, st);
}

__global__ __launch_bounds__(256) void bin_batched_guarded_kernel(BatchParams p) {
    if (p.sh.guard->overflow != 0u) return;
    const unsigned int seen = p.sh.guard->count;
    const int64_t m = (int64_t)seen < p.sh.guard_cap ? (int64_t)seen : p.sh.guard_cap;
    const GuardEntry *ent =
        reinterpret_cast<const GuardEntry *>(reinterpret_cast<const char *>(p.sh.guard) + kGuardHeader);
    LaneStats st;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < m; k += (int64_t)gridDim.x * 256) {
        const GuardEntry g = ent[k];
        const BatchItemDev &it = p.items[g.item];
        const int r = bin_instance_exact(it.c.counts, p.sh.npix, p.sh.nside, p.edges + it.edge_off, it.c.nb, g.dx,
                                         g.dy, g.dz);
        st.inst += r & 1;
        st.unresolved += (r >> 1) & 1;
    }
    flush_stats(p.status, st);
}

double cell_instance_bound(int64_t n, double L, int32_t R, const double *e, int32_t b0, int32_t b1, int64_t nside) {
    const double psi = pixel_diameter_bound(nside);
    double per = 1.0;
    const double side = 2.0 * R + 1.0;
    for (int32_t b = b0; b < b1; ++b) {
        const double D = (e[b + 1] - e[b]) + e[b + 1] * psi;
        double k = (R == 0) ? 1.0 : std::floor(D / L) + 1.0;
        if (k > side) k = side;
        const double cube = k * k * k;
        if (cube > per) per = cube;
    }
    return (double)n * per;
}

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

// Validate one particle set and fill its core description.
int fill_core(BinCore &c, double *e_out, const void *x, const void *y, const void *z, int64_t n,
              const double *observer, double box_L, int32_t n_rep, const double *chi_edges, int32_t n_shells,
              int32_t shell_begin, int32_t shell_end, int64_t nside, uint32_t *counts) {
    if (n < 0 || !observer || !counts) return UFALCON_EINVAL;
    if (n > 0 && (!x || !y || !z)) return UFALCON_EINVAL;
    int rc = check_edges(chi_edges, n_shells);
    if (rc) return rc;
    if ((rc = check_nside(nside))) return rc;
    if (shell_begin < 0 || shell_begin > shell_end || shell_end > n_shells) return UFALCON_EINVAL;
    if (n_rep < 0 || n_rep > 64) return UFALCON_EINVAL;
    if (!std::isfinite(box_L) || (n_rep > 0 && !(box_L > 0.0))) return UFALCON_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(observer[k])) return UFALCON_EINVAL;
    if (shell_end > shell_begin &&
        cell_instance_bound(n, box_L, n_rep, chi_edges, shell_begin, shell_end, nside) > 4294967295.0)
        return UFALCON_EOVERFLOW;
    c.x = x;
    c.y = y;
    c.z = z;
    c.n = n;
    c.ox = observer[0];
    c.oy = observer[1];
    c.oz = observer[2];
    c.L = box_L;
    c.R = n_rep;
    c.nb = shell_end - shell_begin;
    int steps = 0;
    while ((2 << steps) <= c.nb + 1) ++steps;
    c.steps = steps;
    c.item = 0;
    c.counts = counts + (int64_t)shell_begin * npix_of(nside);
    for (int j = 0; j <= c.nb; ++j) e_out[j] = chi_edges[shell_begin + j];
    const double elo = e_out[0], ehi = e_out[c.nb];
    c.lo2 = elo * elo * (1.0 - 0x1p-36);
    c.hi2 = ehi * ehi * (1.0 + 0x1p-36);
    // shell lookup table over the prefilter range [lo2, hi2)
    double e2[UFALCON_MAX_SHELLS + 1];
    for (int j = 0; j <= c.nb; ++j) e2[j] = e_out[j] * e_out[j];
    c.tab_n = shell_table_cells(e2, c.nb, c.lo2, c.hi2);
    c.key32 = (int64_t)c.nb * npix_of(nside) < (int64_t)0xFFFFFFFF ? 1 : 0;
    c.tab_lo = c.lo2;
    c.tab_h = c.tab_n ? (c.hi2 - c.lo2) / c.tab_n : 0.0;
    c.tab_scale = c.tab_n ? c.tab_n / (c.hi2 - c.lo2) : 0.0;
    return UFALCON_OK;
}

int check_workspace(void *workspace, size_t bytes) {
    if (!workspace || bytes < kGuardHeader || ((uintptr_t)workspace & 255u)) return UFALCON_EWORKSPACE;
    return UFALCON_OK;
}

int64_t guard_capacity(size_t bytes) {
    int64_t cap = (int64_t)((bytes - kGuardHeader) / sizeof(GuardEntry));
    return cap > 0x7fffffffLL ? 0x7fffffffLL : cap;
}

template <typename T>
int launch_bin_t(const BinParams &p, hipStream_t s, ufalcon_phase_timer *timer) {
    const unsigned grid =
        blocks_for(p.c.n, kBinBlock, resident_grid(bin_shells_kernel<T, kAtomic>, kBinBlock, (unsigned)device_cus()));
    timer_start(timer, s);
    hipLaunchKernelGGL(guard_reset_kernel, dim3(1), dim3(64), 0, s, p.guard);
    timer_mark(timer, UFALCON_PHASE_SETUP, s);
    hipLaunchKernelGGL((bin_shells_kernel<T, kAtomic>), dim3(grid), dim3(kBinBlock), 0, s, p);
    timer_mark(timer, UFALCON_PHASE_DECIDE, s);
    hipLaunchKernelGGL(bin_guarded_kernel, dim3(64), dim3(256), 0, s, p);
    hipLaunchKernelGGL((bin_shells_kernel<T, kRescue>), dim3(grid), dim3(kBinBlock), 0, s, p);
    timer_mark(timer, UFALCON_PHASE_EXACT, s);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

}  // namespace ufx

namespace ufx {
int try_partitioned(BinParams &p, int dtype, void *workspace, size_t bytes, hipStream_t s, int *rc,
                    ufalcon_phase_timer *timer, const PartHooks *hooks = nullptr);
size_t partitioned_size_for(const BinParams &p);
}

using namespace ufx;

extern "C" const char *ufalcon_strerror(int code) {
    switch (code) {
        case UFALCON_OK: return "ok";
        case UFALCON_EINVAL: return "invalid argument";
        case UFALCON_EUNSORTED_EDGES: return "shell edges must be finite, >= 0 and strictly ascending";
        case UFALCON_ENSIDE: return "nside outside [1, 8192]";
        case UFALCON_EOVERFLOW: return "a uint32 count cell could overflow";
        case UFALCON_EWORKSPACE: return "workspace missing, misaligned or too small";
        case UFALCON_EHIP: return "HIP runtime error";
        case UFALCON_ETOO_MANY_SHELLS: return "too many shells or source bins";
        case UFALCON_EINJECTED: return "failure injected by UFALCON_FAULT_INJECT";
        default: return "unknown error";
    }
}

namespace ufx {
bool fault_injected(const char *point) {
    const char *v = std::getenv("UFALCON_FAULT_INJECT");
    if (!v || !*v) return false;
    const size_t n = std::strlen(point);
    for (const char *s = v;;) {
        const char *e = std::strchr(s, ',');
        const size_t len = e ? (size_t)(e - s) : std::strlen(s);
        if ((len == 1 && *s == '*') || (len == n && std::strncmp(s, point, n) == 0)) return true;
        if (!e) return false;
        s = e + 1;
    }
}
}  // namespace ufx

extern "C" int ufalcon_version(void) { return 100; }

extern "C" size_t ufalcon_bin_shells_workspace_size(int64_t max_listed) {
    if (max_listed < 0) max_listed = 0;
    return kGuardHeader + (size_t)max_listed * sizeof(GuardEntry);
}

extern "C" int ufalcon_fill_u32(uint32_t *p, int64_t n, uint32_t value, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_fill_u32");
    if (n < 0 || (n > 0 && !p)) return UFALCON_EINVAL;
    if (n == 0) return UFALCON_OK;
    const unsigned blocks = blocks_for(n / 4 + 1, 256 * 4, 8192);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, as_stream(stream), p, n, value);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

extern "C" int ufalcon_counts_to_i64(const uint32_t *counts, int64_t n, int64_t *out, int accumulate,
                                     ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_counts_to_i64");
    if (n < 0 || (n > 0 && (!counts || !out)) || (accumulate != 0 && accumulate != 1)) return UFALCON_EINVAL;
    if (n == 0) return UFALCON_OK;
    hipLaunchKernelGGL(widen_counts_kernel, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, as_stream(stream), counts,
                       n, out, accumulate);
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

static int bin_shells_entry(const void *x, const void *y, const void *z, int64_t n, int dtype,
                            const double *observer, double box_L, int32_t n_rep, const double *chi_edges,
                            int32_t n_shells, int32_t shell_begin, int32_t shell_end, int64_t nside, uint32_t *counts,
                            ufalcon_status *status, void *workspace, size_t workspace_bytes, ufalcon_stream_t stream,
                            ufalcon_phase_timer *timer) {
    if (dtype != UFALCON_F32 && dtype != UFALCON_F64) return UFALCON_EINVAL;
    BinParams p;
    int rc = fill_core(p.c, p.e, x, y, z, n, observer, box_L, n_rep, chi_edges, n_shells, shell_begin, shell_end,
                       nside, counts);
    if (rc) return rc;
    if ((rc = check_workspace(workspace, workspace_bytes))) return rc;
    p.nside = nside;
    p.npix = npix_of(nside);
    p.eps = floor_margin((double)nside);
    p.status = status;
    p.guard = static_cast<GuardList *>(workspace);
    p.guard_cap = guard_capacity(workspace_bytes);
    hipStream_t s = as_stream(stream);
    if (p.c.n == 0 || p.c.nb == 0) {
        timer_start(timer, s);  // an empty record: every phase reads 0 ms
        return UFALCON_OK;
    }
    int prc = UFALCON_OK;
    if (try_partitioned(p, dtype, workspace, workspace_bytes, s, &prc, timer)) return prc;
    return dtype == UFALCON_F32 ? launch_bin_t<float>(p, s, timer) : launch_bin_t<double>(p, s, timer);
}

extern "C" int ufalcon_bin_shells(const void *x, const void *y, const void *z, int64_t n, int dtype,
                                  const double *observer, double box_L, int32_t n_rep, const double *chi_edges,
                                  int32_t n_shells, int32_t shell_begin, int32_t shell_end, int64_t nside,
                                  uint32_t *counts, ufalcon_status *status, void *workspace, size_t workspace_bytes,
                                  ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_bin_shells");
    return bin_shells_entry(x, y, z, n, dtype, observer, box_L, n_rep, chi_edges, n_shells, shell_begin, shell_end,
                            nside, counts, status, workspace, workspace_bytes, stream, nullptr);
}

extern "C" int ufalcon_bin_shells_timed(const void *x, const void *y, const void *z, int64_t n, int dtype,
                                        const double *observer, double box_L, int32_t n_rep, const double *chi_edges,
                                        int32_t n_shells, int32_t shell_begin, int32_t shell_end, int64_t nside,
                                        uint32_t *counts, ufalcon_status *status, void *workspace,
                                        size_t workspace_bytes, ufalcon_stream_t stream, ufalcon_phase_timer *timer) {
    UFX_API_ENTRY("ufalcon_bin_shells_timed");
    if (!timer) return UFALCON_EINVAL;
    return bin_shells_entry(x, y, z, n, dtype, observer, box_L, n_rep, chi_edges, n_shells, shell_begin, shell_end,
                            nside, counts, status, workspace, workspace_bytes, stream, timer);
}

// ------------------------------------------------------------------ allocation-free binning
// The workspace of the atomic accumulation path (guard-list header + listed
// guarded instances) kept in a file-scope device array instead of a caller
// buffer.  Each GPU holds its own copy for the life of the process; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name is not a device address on the host).
constexpr size_t kScratchBytes = kGuardHeader + (size_t)UFALCON_NOALLOC_GUARD_ENTRIES * sizeof(GuardEntry);
static_assert(kScratchBytes % 256 == 0, "scratch keeps the workspace's 256-byte granularity");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchMaxDevices] = {};

// Device address of this device's scratch array, looked up on the first call
// with the device current and kept per device.
int scratch_for_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchMaxDevices) return UFALCON_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return UFALCON_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return UFALCON_OK;
}
}  // namespace

extern "C" int ufalcon_bin_shells_noalloc(const void *x, const void *y, const void *z, int64_t n, int dtype,
                                          const double *observer, double box_L, int32_t n_rep,
                                          const double *chi_edges, int32_t n_shells, int32_t shell_begin,
                                          int32_t shell_end, int64_t nside, uint32_t *counts,
                                          ufalcon_status *status, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_bin_shells_noalloc");
    if (dtype != UFALCON_F32 && dtype != UFALCON_F64) return UFALCON_EINVAL;
    BinParams p;
    int rc = fill_core(p.c, p.e, x, y, z, n, observer, box_L, n_rep, chi_edges, n_shells, shell_begin, shell_end,
                       nside, counts);
    if (rc) return rc;
    void *ws = nullptr;
    if ((rc = scratch_for_current_device(&ws))) return rc;
    p.nside = nside;
    p.npix = npix_of(nside);
    p.eps = floor_margin((double)nside);
    p.status = status;
    p.guard = static_cast<GuardList *>(ws);
    p.guard_cap = UFALCON_NOALLOC_GUARD_ENTRIES;
    if (p.c.n == 0 || p.c.nb == 0) return UFALCON_OK;
    // the guard list is reset by a kernel at the start of the call; more guarded
    // instances than it holds are decided by the rescue pass, so no input size
    // needs more scratch than this
    hipStream_t s = as_stream(stream);
    return dtype == UFALCON_F32 ? launch_bin_t<float>(p, s, nullptr) : launch_bin_t<double>(p, s, nullptr);
}

// ------------------------------------------------------------------ batch plan
namespace ufx {
struct BornItemDev {
    const uint32_t *counts;  // [B][npix]
    const double *W;         // [T][B]
    const double *inv_nbar;  // [B]
    void *kappa;             // [T][npix]
    int32_t B;
    int32_t pad;
};
int launch_born_batched(const BornItemDev *items, int32_t n_items, int64_t npix, int32_t T, int out_dtype,
                        hipStream_t s);
}  // namespace ufx

struct ufalcon_batch_plan {
    int dtype, out_dtype;
    int32_t n_items, T;
    int64_t nside, npix, tile, total_tiles;
    int32_t wgs;
    std::vector<BatchItemDev> host_items;
    std::vector<uint32_t *> count_ptrs;
    std::vector<int64_t> count_words;
    BatchItemDev *d_items = nullptr;
    double *d_edges = nullptr;
    BornItemDev *d_born = nullptr;
    void *d_work = nullptr;  // guard list + work counters
    size_t work_bytes = 0;
    int accumulation = UFALCON_ACCUMULATE_PARTITIONED;
    // partitioned accumulation: two lanes (the caller's stream and aux_stream),
    // each with its own workspace; realisations alternate between them, and the
    // first key pass of realisation k waits for the first one of k-1
    // (keys_done[k-1]), so one realisation's partitions and later chunks overlap
    // the next one's key passes
    void *d_part = nullptr;  // workspace of lane 0
    void *d_part2 = nullptr; // workspace of lane 1
    size_t part_bytes = 0;
    hipStream_t aux_stream = nullptr;
    hipEvent_t fork_event = nullptr, join_event = nullptr;
    std::vector<hipEvent_t> keys_done;
    bool shared_rows = false;  // two realisations write overlapping count rows: one lane, in order
    std::vector<BinParams> item_params;  // per-item parameters for the partitioned path
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    ufalcon_status *graph_status = nullptr;
};

static void free_plan(ufalcon_batch_plan *p) {
    if (!p) return;
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->d_items) (void)hipFree(p->d_items);
    if (p->d_edges) (void)hipFree(p->d_edges);
    if (p->d_born) (void)hipFree(p->d_born);
    if (p->d_work) (void)hipFree(p->d_work);
    if (p->d_part) (void)hipFree(p->d_part);
    if (p->d_part2) (void)hipFree(p->d_part2);
    for (hipEvent_t e : p->keys_done)
        if (e) (void)hipEventDestroy(e);
    if (p->fork_event) (void)hipEventDestroy(p->fork_event);
    if (p->join_event) (void)hipEventDestroy(p->join_event);
    if (p->aux_stream) (void)hipStreamDestroy(p->aux_stream);
    delete p;
}

// ------------------------------------------------------------------ autotune cache
namespace {
struct TuneKey {
    std::string arch;
    int cus, dtype;
    int64_t nside;
    int32_t T, n_items, log2n, max_rep;
    bool operator<(const TuneKey &o) const {
        return std::tie(arch, cus, dtype, nside, T, n_items, log2n, max_rep) <
               std::tie(o.arch, o.cus, o.dtype, o.nside, o.T, o.n_items, o.log2n, o.max_rep);
    }
};
struct TuneChoice {
    int32_t accumulation, wgs;
    int64_t tile;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune;  // the library's only global state

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a(prop.gcnArchName);
    const size_t colon = a.find(':');  // drop feature suffixes (":sramecc+:xnack-")
    return colon == std::string::npos ? a : a.substr(0, colon);
}

TuneKey tune_key(const ufalcon_batch_item *items, int32_t n_items, int dtype, int64_t nside, int32_t T) {
    TuneKey k{};
    k.arch = device_arch();
    k.cus = device_cus();
    k.dtype = dtype;
    k.nside = nside;
    k.T = T;
    k.n_items = n_items;
    int64_t total = 0;
    int32_t max_rep = 0;
    for (int32_t i = 0; i < n_items; ++i) {
        total += items[i].n > 0 ? items[i].n : 0;
        max_rep = std::max(max_rep, items[i].n_rep);
    }
    int l = 0;
    while (l < 62 && ((int64_t)1 << (l + 1)) <= total) ++l;
    k.log2n = l;
    k.max_rep = max_rep;
    return k;
}

bool valid_accumulation(int32_t a) {
    return a == UFALCON_ACCUMULATE_PARTITIONED || a == UFALCON_ACCUMULATE_ATOMIC ||
           a == UFALCON_ACCUMULATE_PARTITIONED_ONE_STREAM;
}

// The number after "\"name\":" in a line of the tuning file.
bool json_number(const std::string &line, const char *name, double &v) {
    const std::string key = std::string("\"") + name + "\":";
    const size_t at = line.find(key);
    if (at == std::string::npos) return false;
    const char *p = line.c_str() + at + key.size();
    char *end = nullptr;
    v = std::strtod(p, &end);
    return end != p;
}

bool json_string(const std::string &line, const char *name, std::string &v) {
    const std::string key = std::string("\"") + name + "\":\"";
    const size_t at = line.find(key);
    if (at == std::string::npos) return false;
    const size_t b = at + key.size(), e = line.find('"', b);
    if (e == std::string::npos) return false;
    v = line.substr(b, e - b);
    return true;
}
}  // namespace

extern "C" int ufalcon_batch_plan_create(const ufalcon_batch_item *items, int32_t n_items, int dtype, int64_t nside,
                                         int32_t T, int out_dtype, int64_t tile, int32_t persistent_wgs,
                                         int32_t accumulation, ufalcon_batch_plan **plan) {
    UFX_API_ENTRY("ufalcon_batch_plan_create");
    if (!items || n_items < 1 || !plan) return UFALCON_EINVAL;
    if (accumulation == UFALCON_ACCUMULATE_AUTO) {
        accumulation = UFALCON_ACCUMULATE_PARTITIONED;
        const TuneKey key = tune_key(items, n_items, dtype, nside, T);
        std::lock_guard<std::mutex> lock(g_tune_mu);
        const auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            accumulation = it->second.accumulation;
            if (tile == 0) tile = it->second.tile;
            if (persistent_wgs == 0) persistent_wgs = it->second.wgs;
        }
    }
    if (!valid_accumulation(accumulation)) return UFALCON_EINVAL;
    const bool one_stream = accumulation == UFALCON_ACCUMULATE_PARTITIONED_ONE_STREAM;
    if (one_stream) accumulation = UFALCON_ACCUMULATE_PARTITIONED;
    if (dtype != UFALCON_F32 && dtype != UFALCON_F64) return UFALCON_EINVAL;
    if (out_dtype != UFALCON_F32 && out_dtype != UFALCON_F64) return UFALCON_EINVAL;
    if (T < 0 || T > UFALCON_MAX_BINS) return UFALCON_EINVAL;
    if (tile < 0 || persistent_wgs < 0) return UFALCON_EINVAL;
    int rc = check_nside(nside);
    if (rc) return rc;
    *plan = nullptr;
    ufalcon_batch_plan *p = new ufalcon_batch_plan();
    p->dtype = dtype;
    p->out_dtype = out_dtype;
    p->n_items = n_items;
    p->T = T;
    p->nside = nside;
    p->npix = npix_of(nside);
    p->tile = tile > 0 ? tile : (int64_t)1 << 18;
    p->tile = (p->tile + 63) / 64 * 64;
    p->wgs = persistent_wgs > 0 ? persistent_wgs : device_cus() * 8;
    p->accumulation = accumulation;
    size_t part_need = 0;
    std::vector<double> edges;
    std::vector<BornItemDev> born(n_items);
    int64_t tiles = 0;
    for (int32_t k = 0; k < n_items; ++k) {
        const ufalcon_batch_item &it = items[k];
        BatchItemDev d{};
        double e[UFALCON_MAX_SHELLS + 1];
        rc = fill_core(d.c, e, it.x, it.y, it.z, it.n, it.observer, it.box_L, it.n_rep, it.chi_edges, it.n_shells,
                       it.shell_begin, it.shell_end, nside, it.counts);
        if (rc) {
            free_plan(p);
            return rc;
        }
        d.c.item = k;
        if (accumulation == UFALCON_ACCUMULATE_PARTITIONED && d.c.nb > 0 && it.n > 0) {
            BinParams bp;
            bp.c = d.c;
            bp.c.item = 0;
            for (int j = 0; j <= d.c.nb; ++j) bp.e[j] = e[j];
            bp.nside = nside;
            bp.npix = p->npix;
            bp.eps = floor_margin((double)nside);
            bp.status = nullptr;
            bp.guard = nullptr;
            bp.guard_cap = 0;
            p->item_params.push_back(bp);
            const size_t need = partitioned_size_for(bp);
            if (need == 0) {
                free_plan(p);
                return UFALCON_EINVAL;
            }
            part_need = std::max(part_need, need);
        }
        d.edge_off = (int32_t)edges.size();
        for (int j = 0; j <= d.c.nb; ++j) edges.push_back(e[j]);
        d.tile_begin = tiles;
        const int64_t nt = d.c.nb > 0 ? (it.n + p->tile - 1) / p->tile : 0;
        tiles += nt;
        p->host_items.push_back(d);
        p->count_ptrs.push_back(it.counts);
        p->count_words.push_back((int64_t)it.n_shells * p->npix);
        born[k].counts = it.counts;
        born[k].W = it.W;
        born[k].inv_nbar = it.inv_nbar;
        born[k].kappa = it.kappa;
        born[k].B = it.n_shells;
        if (T > 0 && (!it.W || !it.inv_nbar || !it.kappa)) {
            free_plan(p);
            return UFALCON_EINVAL;
        }
    }
    p->total_tiles = tiles;
    // count rows written by each realisation (its shell range of its map); the
    // partitioned block updates are not atomic, so realisations whose rows
    // overlap (subvolumes of one map) must not run on different lanes
    for (int32_t a = 0; a < n_items && !p->shared_rows; ++a)
        for (int32_t b = a + 1; b < n_items; ++b) {
            const uintptr_t a0 = (uintptr_t)(items[a].counts + (int64_t)items[a].shell_begin * p->npix);
            const uintptr_t a1 = (uintptr_t)(items[a].counts + (int64_t)items[a].shell_end * p->npix);
            const uintptr_t b0 = (uintptr_t)(items[b].counts + (int64_t)items[b].shell_begin * p->npix);
            const uintptr_t b1 = (uintptr_t)(items[b].counts + (int64_t)items[b].shell_end * p->npix);
            if (a0 < a1 && b0 < b1 && a0 < b1 && b0 < a1) {
                p->shared_rows = true;
                break;
            }
        }
    p->work_bytes = kGuardHeader + (size_t)65536 * sizeof(GuardEntry);
    if (part_need > 0) {
        p->part_bytes = part_need;
        bool ok = hipMalloc(&p->d_part, part_need) == hipSuccess;
        if (ok && p->item_params.size() > 1 && !p->shared_rows && !one_stream) {  // the second lane
            ok = hipMalloc(&p->d_part2, part_need) == hipSuccess &&
                 hipStreamCreateWithFlags(&p->aux_stream, hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&p->fork_event, hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&p->join_event, hipEventDisableTiming) == hipSuccess;
            p->keys_done.assign(p->item_params.size(), nullptr);
            for (size_t i = 0; ok && i < p->keys_done.size(); ++i)
                ok = hipEventCreateWithFlags(&p->keys_done[i], hipEventDisableTiming) == hipSuccess;
        }
        if (!ok) {
            free_plan(p);
            return UFALCON_EHIP;
        }
    }
    if (hipMalloc(&p->d_items, sizeof(BatchItemDev) * n_items) != hipSuccess ||
        hipMalloc(&p->d_edges, sizeof(double) * edges.size()) != hipSuccess ||
        hipMalloc(&p->d_born, sizeof(BornItemDev) * n_items) != hipSuccess ||
        hipMalloc(&p->d_work, p->work_bytes) != hipSuccess ||
        hipMemcpy(p->d_items, p->host_items.data(), sizeof(BatchItemDev) * n_items, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_edges, edges.data(), sizeof(double) * edges.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_born, born.data(), sizeof(BornItemDev) * n_items, hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(p);
        return UFALCON_EHIP;
    }
    *plan = p;
    return UFALCON_OK;
}

extern "C" int ufalcon_batch_plan_destroy(ufalcon_batch_plan *plan) {
    UFX_API_RANGE("ufalcon_batch_plan_destroy");
    if (!plan) return UFALCON_EINVAL;
    free_plan(plan);
    return UFALCON_OK;
}

extern "C" int ufalcon_batch_clear(ufalcon_batch_plan *plan, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_batch_clear");
    if (!plan) return UFALCON_EINVAL;
    for (int32_t k = 0; k < plan->n_items; ++k) {
        const int rc = ufalcon_fill_u32(plan->count_ptrs[k], plan->count_words[k], 0u, stream);
        if (rc) return rc;
    }
    return UFALCON_OK;
}

static BatchParams batch_params(ufalcon_batch_plan *plan, ufalcon_status *status) {
    BatchParams bp{};
    bp.items = plan->d_items;
    bp.edges = plan->d_edges;
    bp.n_items = plan->n_items;
    bp.total_tiles = plan->total_tiles;
    bp.tile = plan->tile;
    bp.sh.guard = static_cast<GuardList *>(plan->d_work);
    bp.sh.guard_cap = guard_capacity(plan->work_bytes);
    bp.sh.nside = plan->nside;
    bp.sh.npix = plan->npix;
    bp.sh.eps = floor_margin((double)plan->nside);
    bp.sh.status = status;
    bp.status = status;
    return bp;
}

extern "C" int ufalcon_bin_shells_batched(ufalcon_batch_plan *plan, ufalcon_status *status, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_bin_shells_batched");
    if (!plan) return UFALCON_EINVAL;
    if (plan->total_tiles == 0) return UFALCON_OK;
    if (plan->accumulation == UFALCON_ACCUMULATE_PARTITIONED) {
        hipStream_t s0 = as_stream(stream);
        const size_t m = plan->item_params.size();
        if (m == 1 || !plan->aux_stream) {  // one lane, realisations in order
            for (BinParams bp : plan->item_params) {
                bp.status = status;
                int rc = UFALCON_OK;
                if (!try_partitioned(bp, plan->dtype, plan->d_part, plan->part_bytes, s0, &rc, nullptr))
                    return UFALCON_EWORKSPACE;
                if (rc) return rc;
            }
            return UFALCON_OK;
        }
        // two lanes: fork the aux stream from the caller's, alternate realisations,
        // chain the key passes, join at the end (also valid under stream capture)
        UFX_HIP_CHECK(hipEventRecord(plan->fork_event, s0));
        UFX_HIP_CHECK(hipStreamWaitEvent(plan->aux_stream, plan->fork_event, 0));
        for (size_t k = 0; k < m; ++k) {
            BinParams bp = plan->item_params[k];
            bp.status = status;
            PartHooks hooks;
            hooks.wait_keys = k > 0 ? plan->keys_done[k - 1] : nullptr;
            hooks.done_keys = plan->keys_done[k];
            hipStream_t sk = (k & 1) ? plan->aux_stream : s0;
            void *ws = (k & 1) ? plan->d_part2 : plan->d_part;
            int rc = UFALCON_OK;
            if (!try_partitioned(bp, plan->dtype, ws, plan->part_bytes, sk, &rc, nullptr, &hooks))
                return UFALCON_EWORKSPACE;
            if (rc) return rc;
        }
        UFX_HIP_CHECK(hipEventRecord(plan->join_event, plan->aux_stream));
        UFX_HIP_CHECK(hipStreamWaitEvent(s0, plan->join_event, 0));
        return UFALCON_OK;
    }
    const BatchParams bp = batch_params(plan, status);
    hipStream_t s = as_stream(stream);
    const unsigned wgs = (unsigned)std::min<int64_t>(plan->wgs, plan->total_tiles);
    hipLaunchKernelGGL(guard_reset_kernel, dim3(1), dim3(64), 0, s, bp.sh.guard);
    if (plan->dtype == UFALCON_F32) {
        hipLaunchKernelGGL((bin_batched_kernel<float, kAtomic>), dim3(wgs), dim3(kBinBlock), 0, s, bp);
        hipLaunchKernelGGL(bin_batched_guarded_kernel, dim3(64), dim3(256), 0, s, bp);
        hipLaunchKernelGGL((bin_batched_kernel<float, kRescue>), dim3(wgs), dim3(kBinBlock), 0, s, bp);
    } else {
        hipLaunchKernelGGL((bin_batched_kernel<double, kAtomic>), dim3(wgs), dim3(kBinBlock), 0, s, bp);
        hipLaunchKernelGGL(bin_batched_guarded_kernel, dim3(64), dim3(256), 0, s, bp);
        hipLaunchKernelGGL((bin_batched_kernel<double, kRescue>), dim3(wgs), dim3(kBinBlock), 0, s, bp);
    }
    UFX_HIP_CHECK(hipGetLastError());
    return UFALCON_OK;
}

extern "C" int ufalcon_born_kappa_batched(ufalcon_batch_plan *plan, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_born_kappa_batched");
    if (!plan || plan->T < 1) return UFALCON_EINVAL;
    return launch_born_batched(plan->d_born, plan->n_items, plan->npix, plan->T, plan->out_dtype, as_stream(stream));
}

extern "C" int ufalcon_batch_run_graph(ufalcon_batch_plan *plan, ufalcon_status *status, ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_batch_run_graph");
    if (!plan) return UFALCON_EINVAL;
    if (!plan->graph_exec || plan->graph_status != status) {
        if (plan->graph_exec) {
            UFX_HIP_CHECK(hipGraphExecDestroy(plan->graph_exec));
            plan->graph_exec = nullptr;
        }
        if (!plan->capture_stream) UFX_HIP_CHECK(hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking));
        hipStream_t cs = plan->capture_stream;
        UFX_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        int rc = ufalcon_batch_clear(plan, cs);
        if (!rc) rc = ufalcon_bin_shells_batched(plan, status, cs);
        if (!rc && plan->T > 0) rc = ufalcon_born_kappa_batched(plan, cs);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (rc || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc ? rc : UFALCON_EHIP;
        }
        const hipError_t ie = hipGraphInstantiate(&plan->graph_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return UFALCON_EHIP;
        plan->graph_status = status;
    }
    UFX_HIP_CHECK(hipGraphLaunch(plan->graph_exec, as_stream(stream)));
    return UFALCON_OK;
}

extern "C" int ufalcon_batch_autotune(const ufalcon_batch_item *items, int32_t n_items, int dtype, int64_t nside,
                                      int32_t T, int out_dtype, int32_t sample_items, ufalcon_batch_tuning *tuning,
                                      ufalcon_stream_t stream) {
    UFX_API_ENTRY("ufalcon_batch_autotune");
    if (!items || n_items < 1 || !tuning) return UFALCON_EINVAL;
    const int32_t m = sample_items > 0 ? std::min(sample_items, n_items) : n_items;
    *tuning = ufalcon_batch_tuning{};
    struct Cand {
        int32_t acc, wgs;
        int64_t tile;
    };
    const int cus = device_cus();
    const std::vector<Cand> cands = {{UFALCON_ACCUMULATE_PARTITIONED, 0, 0},
                                     {UFALCON_ACCUMULATE_PARTITIONED_ONE_STREAM, 0, 0},
                                     {UFALCON_ACCUMULATE_ATOMIC, cus * 8, (int64_t)1 << 18},
                                     {UFALCON_ACCUMULATE_ATOMIC, cus * 16, (int64_t)1 << 16}};
    constexpr int kReps = 3;
    hipStream_t s = as_stream(stream);
    hipEvent_t ev[kReps + 1] = {};
    for (int r = 0; r <= kReps; ++r)
        if (hipEventCreate(&ev[r]) != hipSuccess) {
            for (int q = 0; q < r; ++q) (void)hipEventDestroy(ev[q]);
            return UFALCON_EHIP;
        }
    int rc = UFALCON_OK;
    double best = 0.0;
    int bi = -1;
    for (size_t i = 0; i < cands.size() && !rc; ++i) {
        const Cand &c = cands[i];
        ufalcon_batch_plan *plan = nullptr;
        rc = ufalcon_batch_plan_create(items, m, dtype, nside, T, out_dtype, c.tile, c.wgs, c.acc, &plan);
        if (rc) break;
        auto run = [&]() {
            int r = ufalcon_batch_clear(plan, stream);
            if (!r) r = ufalcon_bin_shells_batched(plan, nullptr, stream);
            if (!r && T > 0) r = ufalcon_born_kappa_batched(plan, stream);
            return r;
        };
        rc = run();  // warm-up
        for (int r = 0; r < kReps && !rc; ++r) {
            if (hipEventRecord(ev[r], s) != hipSuccess) rc = UFALCON_EHIP;
            if (!rc) rc = run();
        }
        if (!rc && (hipEventRecord(ev[kReps], s) != hipSuccess || hipEventSynchronize(ev[kReps]) != hipSuccess))
            rc = UFALCON_EHIP;
        double t[kReps] = {};
        for (int r = 0; r < kReps && !rc; ++r) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev[r], ev[r + 1]) != hipSuccess) rc = UFALCON_EHIP;
            t[r] = ms;
        }
        if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = UFALCON_EHIP;
        ufalcon_batch_plan_destroy(plan);
        if (rc) break;
        std::sort(t, t + kReps);
        const double med = t[kReps / 2];
        tuning->ms[i] = med;
        tuning->cand_accumulation[i] = c.acc;
        tuning->cand_wgs[i] = c.wgs;
        tuning->cand_tile[i] = c.tile;
        tuning->n_tried = (int32_t)i + 1;
        if (bi < 0 || med < best) {
            best = med;
            bi = (int)i;
        }
    }
    for (int r = 0; r <= kReps; ++r) (void)hipEventDestroy(ev[r]);
    if (rc) return rc;
    tuning->best = bi;
    tuning->accumulation = cands[bi].acc;
    tuning->persistent_wgs = cands[bi].wgs;
    tuning->tile = cands[bi].tile;
    const TuneKey key = tune_key(items, n_items, dtype, nside, T);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = TuneChoice{cands[bi].acc, cands[bi].wgs, cands[bi].tile};
    return UFALCON_OK;
}

extern "C" int ufalcon_batch_tuning_save(const char *path) {
    UFX_API_ENTRY("ufalcon_batch_tuning_save");
    if (!path) return UFALCON_EINVAL;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return UFALCON_EHIP;
    bool ok = true;
    for (const auto &kv : g_tune) {
        const TuneKey &k = kv.first;
        const TuneChoice &c = kv.second;
        ok = ok && std::fprintf(f,
                                "{\"arch\":\"%s\",\"cus\":%d,\"dtype\":%d,\"nside\":%lld,\"T\":%d,\"items\":%d,"
                                "\"log2n\":%d,\"max_rep\":%d,\"accumulation\":%d,\"wgs\":%d,\"tile\":%lld}\n",
                                k.arch.c_str(), k.cus, k.dtype, (long long)k.nside, k.T, k.n_items, k.log2n, k.max_rep,
                                c.accumulation, c.wgs, (long long)c.tile) > 0;
    }
    ok = (std::fclose(f) == 0) && ok;
    return ok ? UFALCON_OK : UFALCON_EHIP;
}

extern "C" int ufalcon_batch_tuning_load(const char *path, int32_t *n_loaded) {
    UFX_API_ENTRY("ufalcon_batch_tuning_load");
    if (!path) return UFALCON_EINVAL;
    std::ifstream in(path);
    if (!in) return UFALCON_EHIP;
    std::vector<std::pair<TuneKey, TuneChoice>> got;
    std::string line;
    while (std::getline(in, line)) {
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        TuneKey k{};
        TuneChoice c{};
        double v[10];
        const char *names[10] = {"cus", "dtype", "nside", "T", "items", "log2n", "max_rep", "accumulation", "wgs",
                                 "tile"};
        if (!json_string(line, "arch", k.arch)) return UFALCON_EINVAL;
        for (int i = 0; i < 10; ++i)
            if (!json_number(line, names[i], v[i])) return UFALCON_EINVAL;
        k.cus = (int)v[0];
        k.dtype = (int)v[1];
        k.nside = (int64_t)v[2];
        k.T = (int32_t)v[3];
        k.n_items = (int32_t)v[4];
        k.log2n = (int32_t)v[5];
        k.max_rep = (int32_t)v[6];
        c.accumulation = (int32_t)v[7];
        c.wgs = (int32_t)v[8];
        c.tile = (int64_t)v[9];
        if (!valid_accumulation(c.accumulation) || c.wgs < 0 || c.tile < 0) return UFALCON_EINVAL;
        got.emplace_back(k, c);
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const auto &kv : got) g_tune[kv.first] = kv.second;
    if (n_loaded) *n_loaded = (int32_t)got.size();
    return UFALCON_OK;
}
