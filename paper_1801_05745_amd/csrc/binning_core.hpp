// Per-wavefront binning core shared by the plain, batched and partitioned kernels.
//
// A wave walks the periodic images of 64 particles at a time, queues the images
// whose squared radius falls in the (guard-widened) shell range in LDS, and
// whenever 64 are queued every lane takes one and decides its shell and RING
// pixel in FP64 (ring.hpp).  What happens to a decided instance depends on the mode:
//   kAtomic  add 1 to its count cell with a global atomic;
//   kEmit    emit its key b * npix + pix into a key buffer (partitioned
//            accumulation: the keys are grouped by cell block later and counted
//            in LDS, see partition.hip);
//   kRescue  skip it (it was counted by an earlier pass) — only guarded
//            instances are decided, exactly.
// Instances inside a guard band are listed in the workspace for the exact
// kernel (kAtomic, kEmit) or decided exactly at once (kRescue).
#pragma once

#include "../../include/ufalcon.h"
#include "exact.hpp"
#include "internal.hpp"
#include "ring.hpp"

namespace ufx {

constexpr int kBinBlock = 256;
constexpr int kBinWaves = kBinBlock / 64;
constexpr int kQueue = 128;  // < 64 pending + up to 64 new entries

enum BinMode { kAtomic = 0, kRescue = 1, kEmit = 2 };

constexpr uint32_t kNoKey = 0xFFFFFFFFu;   // sentinel in key buffers
constexpr int kKeyChunk = 1024;            // key slots a wave reserves at a time

// Workspace layout: this header, then guard_cap entries.
struct GuardList {
    unsigned int count;     // guarded instances seen (may exceed the capacity)
    unsigned int overflow;  // nonzero when some guarded instance was not stored
    unsigned int next;      // work counter of the persistent kernel
    unsigned int next_rescue;
    unsigned int pad[60];
};
struct GuardEntry {
    double dx, dy, dz;
    int32_t item;
    int32_t pad;
};
constexpr size_t kGuardHeader = sizeof(GuardList);
static_assert(kGuardHeader == 256, "workspace header is 256 bytes");

// Everything the per-wave core needs about one particle set.
struct BinCore {
    const void *x, *y, *z;
    int64_t n;
    double ox, oy, oz, L;
    double lo2, hi2;      // guard-widened [e_b0^2, e_b1^2)
    int32_t R;            // images {-R..R}^3
    int32_t nb;           // shells in range
    int32_t steps;        // binary-search steps over nb + 1 edges
    int32_t item;         // realisation index (batched) or 0
    uint32_t *counts;     // row of the first shell in range
};

struct BinParams {
    BinCore c;
    int64_t nside, npix;
    double eps;           // floor-argument margin
    ufalcon_status *status;
    GuardList *guard;     // workspace header
    int64_t guard_cap;    // entries the workspace holds
    double e[UFALCON_MAX_SHELLS + 1];  // edges of the range, e_b0 .. e_b1
};

struct LaneStats {
    unsigned long long inst = 0, guarded = 0, unresolved = 0, invalid = 0;
};

struct Shared {
    GuardList *guard;
    int64_t guard_cap;
    int64_t nside, npix;
    double eps;
};

// Key emission state of one wave (kEmit).  All lanes hold the same values.
struct Emitter {
    uint32_t *keys;                    // key buffer (slots)
    unsigned long long *reserved;      // global count of reserved slots
    unsigned long long cap;            // usable slots (a multiple of kKeyChunk)
    uint32_t *hist;                    // LDS histogram of key >> shift (per workgroup)
    int shift;
    unsigned long long base;           // current chunk [base, base + kKeyChunk)
    int fill;                          // slots used in the current chunk
    bool full;                         // the key buffer is exhausted: fall back to atomics
};

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Exact decision for one guarded instance.  Returns bit 0: counted, bit 1: unresolved.
__device__ __noinline__ int bin_instance_exact(uint32_t *counts, int64_t npix, int64_t nside, const double *e, int nb,
                                               double dx, double dy, double dz) {
    const int b = exact_shell(dx, dy, dz, e, nb);
    if (b < 0 || b >= nb) return 0;
    int unresolved = 0;
    const int64_t pix = exact_ring_pixel(nside, dx, dy, dz, &unresolved);
    if (pix < 0 || pix >= npix) return 2;  // never expected; reported as unresolved, not written
    atomicAdd(counts + (int64_t)b * npix + pix, 1u);
    return 1 | (unresolved << 1);
}

// Decide one queued instance.  Returns its key (kEmit) or kNoKey.
template <int kMode>
__device__ __forceinline__ uint32_t bin_instance(const BinCore &c, const Shared &sh, const double *e_s,
                                                 const double *e2_s, double Nd, double dx, double dy, double dz,
                                                 LaneStats &st) {
    const double r2 = dx * dx + dy * dy + dz * dz;
    bool clear;
    const int j = fast_shell(e2_s, c.nb, c.steps, r2, clear);
    if (clear) {
        if (j < 0 || j >= c.nb) return kNoKey;
        int32_t pix;
        // the range test costs two compares and keeps any logic slip from writing out of bounds
        if (fast_ring_pixel((int32_t)sh.nside, Nd, sh.eps, dx, dy, dz, pix) && pix >= 0 && pix < sh.npix) {
            if (kMode == kRescue) return kNoKey;
            ++st.inst;
            if (kMode == kAtomic) {
                atomicAdd(c.counts + (int64_t)j * sh.npix + pix, 1u);
                return kNoKey;
            }
            return (uint32_t)((int64_t)j * sh.npix + pix);
        }
    }
    if (kMode == kRescue) {
        const int r = bin_instance_exact(c.counts, sh.npix, sh.nside, e_s, c.nb, dx, dy, dz);
        st.inst += r & 1;
        st.unresolved += (r >> 1) & 1;
    } else {
        ++st.guarded;
        const unsigned int slot = atomicAdd(&sh.guard->count, 1u);
        if ((int64_t)slot < sh.guard_cap) {
            GuardEntry *ent = reinterpret_cast<GuardEntry *>(reinterpret_cast<char *>(sh.guard) + kGuardHeader) + slot;
            ent->dx = dx;
            ent->dy = dy;
            ent->dz = dz;
            ent->item = c.item;
        } else {
            atomicOr(&sh.guard->overflow, 1u);
        }
    }
    return kNoKey;
}

// Wave-cooperative append of the lanes' keys (kNoKey lanes skip).  Must be
// reached by all 64 lanes of the wave.
__device__ __forceinline__ void emit_keys(Emitter &em, const BinCore &c, uint32_t key) {
    const int lane = threadIdx.x & 63;
    const bool has = key != kNoKey;
    const unsigned long long m = __ballot(has);
    if (m == 0ull) return;
    if (em.full) {  // buffer exhausted earlier: count directly
        if (has) atomicAdd(c.counts + key, 1u);
        return;
    }
    const int n = __popcll(m);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    const int room = kKeyChunk - em.fill;
    if (has && rank < room) {
        em.keys[em.base + em.fill + rank] = key;
        if (em.hist) atomicAdd(&em.hist[key >> em.shift], 1u);
    }
    if (n <= room) {
        em.fill += n;
        return;
    }
    // the current chunk is full: reserve the next one
    unsigned long long b = 0;
    if (lane == 0) b = atomicAdd(em.reserved, (unsigned long long)kKeyChunk);
    b = __shfl(b, 0, 64);
    if (b + kKeyChunk > em.cap) {
        // chunk-aligned capacity: this reservation lies wholly outside the buffer
        em.full = true;
        em.fill = kKeyChunk;
        if (has && rank >= room) atomicAdd(c.counts + key, 1u);
        return;
    }
    em.base = b;
    if (has && rank >= room) {
        em.keys[b + (rank - room)] = key;
        if (em.hist) atomicAdd(&em.hist[key >> em.shift], 1u);
    }
    em.fill = n - room;
}

// Pad the unused tail of the wave's current chunk with sentinels.
__device__ __forceinline__ void close_emitter(Emitter &em) {
    if (em.full || em.fill >= kKeyChunk) return;
    const int lane = threadIdx.x & 63;
    for (int k = em.fill + lane; k < kKeyChunk; k += 64) em.keys[em.base + k] = kNoKey;
}

// Per-wave core: this wave handles particles base, base + stride, ... (64 at a
// time) below `end`; queued images persist in (Qx, Qy, Qz, count) across calls
// and are drained by drain_queue().
template <typename T, int kMode>
__device__ __forceinline__ void bin_wave_range(const BinCore &c, const Shared &sh, const double *e_s,
                                               const double *e2_s, int64_t base, int64_t end, int64_t stride,
                                               double *Qx, double *Qy, double *Qz, int &count, LaneStats &st,
                                               Emitter &em) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const T *X = static_cast<const T *>(c.x);
    const T *Y = static_cast<const T *>(c.y);
    const T *Z = static_cast<const T *>(c.z);
    const double Nd = (double)sh.nside;
    for (; base < end; base += stride) {
        const int64_t i = base + lane;
        bool valid = false;
        double bx = 0.0, by = 0.0, bz = 0.0;
        if (i < end) {
            const double x = (double)X[i], y = (double)Y[i], z = (double)Z[i];
            if (isfinite(x) && isfinite(y) && isfinite(z)) {
                valid = true;
                bx = x - c.ox;
                by = y - c.oy;
                bz = z - c.oz;
            } else if (kMode != kRescue) {
                ++st.invalid;
            }
        }
        for (int sx = -c.R; sx <= c.R; ++sx) {
            const double dx = bx + (double)sx * c.L;
            for (int sy = -c.R; sy <= c.R; ++sy) {
                const double dy = by + (double)sy * c.L;
                for (int sz = -c.R; sz <= c.R; ++sz) {
                    const double dz = bz + (double)sz * c.L;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const bool in = valid && r2 >= c.lo2 && r2 < c.hi2;
                    const unsigned long long m = __ballot(in);
                    if (m == 0ull) continue;
                    const int pos = count + __popcll(m & below);
                    if (in) {
                        Qx[pos] = dx;
                        Qy[pos] = dy;
                        Qz[pos] = dz;
                    }
                    count += __popcll(m);
                    if (count >= 64) {
                        wave_lds_sync();
                        const double ax = Qx[lane], ay = Qy[lane], az = Qz[lane];
                        const int rest = count - 64;
                        double rx = 0.0, ry = 0.0, rz = 0.0;
                        if (lane < rest) {
                            rx = Qx[64 + lane];
                            ry = Qy[64 + lane];
                            rz = Qz[64 + lane];
                        }
                        wave_lds_sync();
                        if (lane < rest) {
                            Qx[lane] = rx;
                            Qy[lane] = ry;
                            Qz[lane] = rz;
                        }
                        count = rest;
                        const uint32_t key = bin_instance<kMode>(c, sh, e_s, e2_s, Nd, ax, ay, az, st);
                        if (kMode == kEmit) emit_keys(em, c, key);
                    }
                }
            }
        }
    }
}

template <int kMode>
__device__ __forceinline__ void drain_queue(const BinCore &c, const Shared &sh, const double *e_s, const double *e2_s,
                                            double *Qx, double *Qy, double *Qz, int &count, LaneStats &st,
                                            Emitter &em) {
    const int lane = threadIdx.x & 63;
    wave_lds_sync();
    uint32_t key = kNoKey;
    if (lane < count) key = bin_instance<kMode>(c, sh, e_s, e2_s, (double)sh.nside, Qx[lane], Qy[lane], Qz[lane], st);
    if (kMode == kEmit) emit_keys(em, c, key);
    wave_lds_sync();
    count = 0;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void flush_stats(ufalcon_status *status, LaneStats &st) {
    const unsigned long long a = wave_sum(st.inst), b = wave_sum(st.guarded), c = wave_sum(st.unresolved),
                             d = wave_sum(st.invalid);
    if (status && (threadIdx.x & 63) == 0) {
        if (a) atomicAdd(&status->n_instances, a);
        if (b) atomicAdd(&status->n_guarded, b);
        if (c) atomicAdd(&status->n_unresolved, c);
        if (d) atomicAdd(&status->n_invalid, d);
    }
}

__device__ __forceinline__ Shared shared_of(const BinParams &p) {
    return Shared{p.guard, p.guard_cap, p.nside, p.npix, p.eps};
}

// Host helpers (bin_shells.hip)
int fill_core(BinCore &c, double *e_out, const void *x, const void *y, const void *z, int64_t n,
              const double *observer, double box_L, int32_t n_rep, const double *chi_edges, int32_t n_shells,
              int32_t shell_begin, int32_t shell_end, int64_t nside, uint32_t *counts);
int device_cus();
int64_t guard_capacity(size_t bytes);

// Workgroups of `kernel` that are resident on the whole device at once: a
// grid-stride kernel launched with more leaves a second, partly empty round.
template <typename K>
unsigned resident_grid(K kernel, int threads, unsigned cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * (unsigned)per_cu;
}

}  // namespace ufx
