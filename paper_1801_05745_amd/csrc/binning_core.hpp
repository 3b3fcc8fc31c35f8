// Per-wavefront binning core shared by the plain, batched and partitioned kernels.
//
// A wave walks the periodic images of 64 particles at a time, queues the images
// whose squared radius falls in the (guard-widened) shell range in LDS, and
// whenever 64 are queued every lane takes one and decides its shell and RING
// pixel in FP64 (ring.hpp).  What happens to a decided instance depends on the mode:
//   kAtomic  add 1 to its count cell with a global atomic (equal keys of the
//            wave's batch aggregated into one atomic when the keys fit 32 bits);
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
// Per-wave LDS queue of in-range images, two-ended: belt directions fill it from
// the bottom, cap directions from the top, and each end is taken 64 at a time,
// so that every lane of a batch runs the same pixel formula.  Before an image
// step each end holds < 64 entries and the step adds at most 64: 63 + 63 + 64
// entries fit in 192 slots without the ends meeting.
constexpr int kQueue = 192;
constexpr int kMaxRep = 64;  // largest n_rep the entry points accept

enum BinMode { kAtomic = 0, kRescue = 1, kEmit = 2 };

constexpr uint32_t kNoKey = 0xFFFFFFFFu;   // sentinel in key buffers
constexpr int kKeyChunk = 4096;            // key slots a wave reserves at a time (larger: fewer contended reservations)

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
    int32_t tab_n;        // cells of the shell lookup table (0: binary search)
    int32_t key32;        // the range's cells fit 32-bit keys (atomic accumulation aggregates equal keys)
    double tab_lo, tab_h, tab_scale;  // table over r^2 from tab_lo, cell width tab_h = 1 / tab_scale
};

// Edges of one shell range in LDS: the squared radii with two sentinels on each
// side (e2() is indexable from -2 to nb + 2), the shell lookup table, and a
// pointer to the radii, which only the exact path reads (kRescue kernels keep
// them in an LDS array of their own; elsewhere the pointer is null).
struct EdgeLds {
    const double *e;
    double e2p[UFALCON_MAX_SHELLS + 5];
    double sL[2 * kMaxRep + 1];  // fl(s L) for s = -R .. R (index s + R)
    double ttc[kTtTerms];         // azimuth polynomial
    int16_t tab[kShellTabMax];
    __device__ const double *e2() const { return e2p + 2; }
};

// Fill `E` for the range of `c` with radii `e`, copying the radii to `radii`
// (UFALCON_MAX_SHELLS + 1 LDS doubles) when the kernel decides exactly.  Every
// thread of the block calls it (it synchronises twice).
__device__ inline void load_edges(EdgeLds &E, const BinCore &c, const double *e, double *radii = nullptr) {
    for (int j = threadIdx.x; j <= c.nb; j += blockDim.x) {
        if (radii) radii[j] = e[j];
        E.e2p[j + 2] = e[j] * e[j];
    }
    if (threadIdx.x == 0) E.e = radii;
    if (threadIdx.x < 2) {
        E.e2p[threadIdx.x] = -kEdgeSentinel;
        E.e2p[c.nb + 3 + threadIdx.x] = kEdgeSentinel;
    }
    for (int k = threadIdx.x; k <= 2 * c.R; k += blockDim.x) E.sL[k] = (double)(k - c.R) * c.L;
    if (threadIdx.x < kTtTerms) E.ttc[threadIdx.x] = kTtCoef[threadIdx.x];
    __syncthreads();
    for (int t = threadIdx.x; t < c.tab_n; t += blockDim.x)
        E.tab[t] = shell_table_entry(E.e2(), c.nb, c.steps, c.tab_lo + (double)t * c.tab_h,
                                     t + 1 < c.tab_n ? c.tab_lo + (double)(t + 1) * c.tab_h : c.hi2);
    __syncthreads();
}

struct BinParams {
    BinCore c;
    int64_t nside, npix;
    double eps;           // floor-argument margin
    ufalcon_status *status;
    GuardList *guard;     // workspace header
    int64_t guard_cap;    // entries the workspace holds
    double e[UFALCON_MAX_SHELLS + 1];  // edges of the range, e_b0 .. e_b1
};

// Per-lane event counts, flushed into the status by flush_stats (also whenever a
// lane's instance count passes 2^30, see bin_wave_range).
struct LaneStats {
    uint32_t inst = 0, guarded = 0, unresolved = 0, invalid = 0, fallback = 0;
};

struct Shared {
    GuardList *guard;
    int64_t guard_cap;
    int64_t nside, npix;
    double eps;
    ufalcon_status *status;  // event counts (may be null)
};

// Level-1 buckets (key >> shift) that the key pass can count per reservation.
constexpr int kHistBins = 256;

// Key emission state of one wave (kEmit).  All lanes hold the same values.
// With `hist`, the wave also counts its keys per level-1 bucket in LDS (two
// 16-bit counters per word: a reservation holds at most 4096 keys) and, when a
// reservation is closed, writes the counts to that reservation's row of
// `hist_rows` (kHistBins 16-bit counts), so that the partition needs no pass
// over the keys to histogram them.
struct Emitter {
    uint32_t *keys;                    // key buffer (slots)
    unsigned long long *reserved;      // global count of reserved slots
    unsigned long long cap;            // usable slots (a multiple of kKeyChunk)
    uint32_t *hist;                    // the wave's kHistBins / 2 LDS words, or null
    uint16_t *hist_rows;               // [cap / kKeyChunk][kHistBins] counts per reservation
    int shift;
    unsigned long long base;           // current chunk [base, base + kKeyChunk)
    int fill;                          // slots used in the current chunk; kKeyChunk + 1: no chunk held
    bool full;                         // the key buffer is exhausted: fall back to atomics
};


__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Add the wave's counts to the status and reset them.  Reached by all 64 lanes.
__device__ __forceinline__ void flush_stats(ufalcon_status *status, LaneStats &st) {
    const unsigned long long a = wave_sum(st.inst), b = wave_sum(st.guarded), c = wave_sum(st.unresolved),
                             d = wave_sum(st.invalid), f = wave_sum(st.fallback);
    if (status && (threadIdx.x & 63) == 0) {
        if (a) atomicAdd(&status->n_instances, a);
        if (b) atomicAdd(&status->n_guarded, b);
        if (c) atomicAdd(&status->n_unresolved, c);
        if (d) atomicAdd(&status->n_invalid, d);
        if (f) atomicAdd(&status->n_fallback, f);
    }
    st = LaneStats{};
}

// 0, but opaque to the compiler: an LDS index offset by it is reloaded where it
// is used instead of being hoisted out of loops into registers kept for the
// whole kernel (the azimuth coefficients).  Emits no instruction.
__device__ __forceinline__ int opaque_zero() {
    int z = 0;
    asm volatile("" : "+v"(z));
    return z;
}

// An LDS array's address, opaque to the compiler in the same way: every element
// read through it is a fresh load, and all of them share the one address
// register (constant offsets in the load instructions).
typedef __attribute__((address_space(3))) const double LdsDouble;
__device__ __forceinline__ LdsDouble *opaque_lds(const double *p) {
    LdsDouble *q = (LdsDouble *)p;
    asm volatile("" : "+v"(q));
    return q;
}

// Ballot of a lane predicate (the compare's lane mask, without a round trip
// through a VGPR) and the number of lanes below this one set in a mask.
__device__ __forceinline__ unsigned long long wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ int lanes_below(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// The first active lane's 64-bit value in every lane (scalar registers).  The
// halves go through readfirstlane, whose int result is zero-extended back:
// sign-extending it would corrupt values with bit 31 or bit 63 set.
__device__ __forceinline__ unsigned long long wave_first_u64(unsigned long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | (unsigned long long)lo;
}

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
template <int kMode, bool kBelt>
__device__ __forceinline__ uint32_t bin_instance(const BinCore &c, const Shared &sh, const EdgeLds &E, double Nd,
                                                 double dx, double dy, double dz, LaneStats &st) {
    const double r2 = dx * dx + dy * dy + dz * dz;
    bool clear;
    const int j = fast_shell(E.e2(), c.nb, c.steps, E.tab, c.tab_n, c.tab_lo, c.tab_scale, r2, clear);
    if (clear) {
        if (j < 0 || j >= c.nb) return kNoKey;
        int32_t pix;
        // the range test costs two compares and keeps any logic slip from writing out of bounds
        if (fast_ring_pixel_region<kBelt>((int32_t)sh.nside, Nd, sh.eps, dx, dy, dz, pix, opaque_lds(E.ttc)) &&
            (uint32_t)pix < (uint32_t)sh.npix) {  // npix < 2^31 for nside <= 8192
            if (kMode == kRescue) return kNoKey;
            ++st.inst;
            if (kMode == kAtomic && !c.key32) {
                atomicAdd(c.counts + (int64_t)j * sh.npix + pix, 1u);
                return kNoKey;
            }
            return (uint32_t)j * (uint32_t)sh.npix + (uint32_t)pix;  // < 2^32: key32, or the host checks B * npix
        }
    }
    if (kMode == kRescue) {
        const int r = bin_instance_exact(c.counts, sh.npix, sh.nside, E.e, c.nb, dx, dy, dz);
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

__device__ __forceinline__ void hist_add(const Emitter &em, uint32_t key) {
    const uint32_t b = key >> em.shift;
    atomicAdd(&em.hist[key >> (em.shift + 1)], (b & 1u) ? 0x10000u : 1u);  // word b / 2, half b % 2
}

// Write the counts of the wave's current reservation to its row and clear them.
// All 64 lanes call it.  Lane l holds bins 4l .. 4l+3 in words 2l and 2l + 1,
// which are the row's 16-bit entries 4l .. 4l+3 in order.
__device__ __forceinline__ void flush_hist(Emitter &em) {
    const int lane = threadIdx.x & 63;
    wave_lds_sync();
    const uint2 v = reinterpret_cast<const uint2 *>(em.hist)[lane];
    reinterpret_cast<uint2 *>(em.hist_rows + (em.base / kKeyChunk) * (unsigned long long)kHistBins)[lane] = v;
    reinterpret_cast<uint2 *>(em.hist)[lane] = make_uint2(0u, 0u);
    wave_lds_sync();
}

// Wave-cooperative append of the lanes' keys (kNoKey lanes skip).  Must be
// reached by all 64 lanes of the wave.
__device__ __forceinline__ void emit_keys(Emitter &em, const BinCore &c, uint32_t key, LaneStats &st) {
    const int lane = threadIdx.x & 63;
    const bool has = key != kNoKey;
    const unsigned long long m = wave_ballot(has);
    if (m == 0ull) return;
    if (em.full) {  // buffer exhausted earlier: count directly
        if (has) {
            atomicAdd(c.counts + key, 1u);
            ++st.fallback;
        }
        return;
    }
    const int n = __popcll(m);
    const unsigned rank = (unsigned)lanes_below(m);  // unsigned: a 32-bit offset from a scalar base
    const int room = em.fill < kKeyChunk ? kKeyChunk - em.fill : 0;  // fill is kKeyChunk + 1 when no chunk is held
    if (has && rank < (unsigned)room) {
        uint32_t *dst = em.keys + (em.base + (unsigned long long)em.fill);  // uniform: one scalar base per wave
        dst[rank] = key;
        if (em.hist) hist_add(em, key);
    }
    if (n <= room) {
        em.fill += n;
        return;
    }
    // the current chunk is full (or none is held): close it and reserve the next one
    if (em.hist && em.fill <= kKeyChunk) flush_hist(em);
    unsigned long long b = 0;
    if (lane == 0) b = atomicAdd(em.reserved, (unsigned long long)kKeyChunk);
    b = wave_first_u64(b);  // lane 0's reservation (every lane is active here)
    if (b + kKeyChunk > em.cap) {
        // chunk-aligned capacity: this reservation lies wholly outside the buffer
        em.full = true;
        em.fill = kKeyChunk + 1;
        if (has && rank >= (unsigned)room) {
            atomicAdd(c.counts + key, 1u);
            ++st.fallback;
        }
        return;
    }
    em.base = b;
    if (has && rank >= (unsigned)room) {
        em.keys[b + (rank - room)] = key;
        if (em.hist) hist_add(em, key);
    }
    em.fill = n - room;
}

// Atomic accumulation with equal keys aggregated over the wave: the 64 keys
// (kNoKey for lanes without an instance) are sorted across the lanes (bitonic
// network over lane-index bits), and the first lane of every run of equal keys
// adds the run's length with one atomic.  Must be reached by all 64 lanes.
__device__ __forceinline__ void aggregate_add(uint32_t *counts, uint32_t key) {
    const int lane = threadIdx.x & 63;
    if (wave_ballot(key != kNoKey) == 0ull) return;  // uniform
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t other = __shfl_xor(key, j, 64);
            const bool ascending = (lane & k) == 0;
            const bool lower = (lane & j) == 0;
            key = (lower == ascending) ? min(key, other) : max(key, other);
        }
    }
    const uint32_t prev = __shfl_up(key, 1, 64);
    const bool valid = key != kNoKey;
    const bool head = valid && (lane == 0 || prev != key);
    // a run ends at the next head or at the first lane without a key (kNoKey sorts last)
    const unsigned long long stops = wave_ballot(head) | ~wave_ballot(valid);
    if (head) {
        const unsigned long long above = lane == 63 ? 0ull : (stops >> (lane + 1)) << (lane + 1);
        const int next = above ? __builtin_ctzll(above) : 64;
        atomicAdd(counts + key, (uint32_t)(next - lane));
    }
}

// Pad the unused tail of the wave's current chunk with sentinels and write its
// counts.  All 64 lanes call it.
__device__ __forceinline__ void close_emitter(Emitter &em) {
    if (em.fill > kKeyChunk) return;  // no chunk held
    const int lane = threadIdx.x & 63;
    for (int k = em.fill + lane; k < kKeyChunk; k += 64) em.keys[em.base + k] = kNoKey;
    if (em.hist) flush_hist(em);
    em.fill = kKeyChunk + 1;
}

// The wave's queue (LDS arrays of kQueue slots) and its fill at each end.
struct WaveQueue {
    double *q;  // x at q[s], y at q[kQueue + s], z at q[2 kQueue + s] for slot s
    int nb;     // belt entries in slots [0, nb)
    int nc;     // cap entries in slots [kQueue - nc, kQueue)
};

// Take the 64 most recently queued entries at one end of the queue (the top 64 of
// the belt end, the bottom 64 of the cap end; no entry moves) and decide them,
// one per lane.  All 64 lanes call it.
template <int kMode, bool kBelt>
__device__ __forceinline__ void take_batch(const BinCore &c, const Shared &sh, const EdgeLds &E, double Nd,
                                           WaveQueue &q, LaneStats &st, Emitter &em) {
    const int lane = threadIdx.x & 63;
    const int take = kBelt ? q.nb - 64 + lane : kQueue - q.nc + lane;
    wave_lds_sync();
    const double ax = q.q[take], ay = q.q[kQueue + take], az = q.q[2 * kQueue + take];
    if (kBelt)
        q.nb -= 64;
    else
        q.nc -= 64;
    const uint32_t key = bin_instance<kMode, kBelt>(c, sh, E, Nd, ax, ay, az, st);
    if (kMode == kEmit) emit_keys(em, c, key, st);
    if (kMode == kAtomic) aggregate_add(c.counts, key);
}

// Never stop early (the plain passes).
struct NoStop {
    __device__ bool operator()() const { return false; }
};

// Per-wave core: this wave handles particles base, base + stride, ... (64 at a
// time) below `end`; queued images persist in `q` across calls and are drained
// by drain_queue().  `stop` is asked before every batch of 64 particles after
// the first; the return value is the base of the first batch not processed
// (>= end when the range is done).
template <typename T, int kMode, typename Stop = NoStop>
__device__ __forceinline__ int64_t bin_wave_range(const BinCore &c, const Shared &sh, const EdgeLds &E,
                                                  int64_t base, int64_t end, int64_t stride, WaveQueue &q,
                                                  LaneStats &st, Emitter &em, Stop stop = Stop{}) {
    const int lane = threadIdx.x & 63;
    const T *X = static_cast<const T *>(c.x);
    const T *Y = static_cast<const T *>(c.y);
    const T *Z = static_cast<const T *>(c.z);
    const double Nd = (double)sh.nside;
    // positions are loaded one iteration ahead, so that their memory latency
    // overlaps the images of the current 64 particles
    T px = T(0), py = T(0), pz = T(0);
    if (base + lane < end) {
        px = X[base + lane];
        py = Y[base + lane];
        pz = Z[base + lane];
    }
    for (bool first = true; base < end; base += stride, first = false) {
        if (!first && stop()) break;  // uniform
        const int64_t i = base + lane;
        const double x = (double)px, y = (double)py, z = (double)pz;
        const int64_t inext = base + stride + lane;
        if (base + stride < end && inext < end) {
            px = X[inext];
            py = Y[inext];
            pz = Z[inext];
        }
        bool valid = false;
        double bx = 0.0, by = 0.0, bz = 0.0;
        if (i < end) {
            if (isfinite(x) && isfinite(y) && isfinite(z)) {
                valid = true;
                bx = x - c.ox;
                by = y - c.oy;
                bz = z - c.oz;
            } else if (kMode != kRescue) {
                ++st.invalid;
            }
        }
        const unsigned long long mvalid = wave_ballot(valid);
        const int side = 2 * c.R + 1;
        for (int ix = 0; ix < side; ++ix) {
            const double dx = bx + E.sL[ix];  // d = (x - o) + fl(s L), per axis
            for (int iy = 0; iy < side; ++iy) {
                const double dy = by + E.sL[iy];
                const double rho2 = dx * dx + dy * dy;
                // belt when 5 dz^2 < 4 rho^2, tested as dz^2 < 0.8 rho^2: a direction this
                // puts in the other queue lies within rounding of |z| = 2/3, where the
                // decision code defers it
                const double a08 = 0.8 * rho2;
                for (int iz = 0; iz < side; ++iz) {
                    const double dz = bz + E.sL[iz];
                    const double dz2 = dz * dz;
                    const double r2 = rho2 + dz2;  // the same roundings as the decision code
                    // lane masks straight from the compares; the per-lane flags read back
                    // from them
                    const unsigned long long mi = wave_ballot(r2 >= c.lo2) & wave_ballot(r2 < c.hi2) & mvalid;
                    if (mi == 0ull) continue;
                    const unsigned long long mbelt = wave_ballot(dz2 < a08);
                    const unsigned long long mb = mi & mbelt, mc = mi & ~mbelt;
                    if (__builtin_amdgcn_inverse_ballot_w64(mi)) {
                        const bool belt = __builtin_amdgcn_inverse_ballot_w64(mbelt);
                        const int pos = belt ? q.nb + lanes_below(mb) : kQueue - 1 - q.nc - lanes_below(mc);
                        q.q[pos] = dx;
                        q.q[kQueue + pos] = dy;
                        q.q[2 * kQueue + pos] = dz;
                    }
                    q.nb += __popcll(mb);
                    q.nc += __popcll(mc);
                    if (q.nb >= 64) take_batch<kMode, true>(c, sh, E, Nd, q, st, em);
                    if (q.nc >= 64) take_batch<kMode, false>(c, sh, E, Nd, q, st, em);
                }
            }
        }
        // one iteration adds at most (2R+1)^3 <= 129^3 instances per lane: flushing
        // past 2^30 keeps the 32-bit counts exact
        if (__ballot(st.inst >= (1u << 30)) != 0ull) flush_stats(sh.status, st);
    }
    return base;
}

// Decide what is left in the queue (fewer than 64 at each end).
template <int kMode>
__device__ __forceinline__ void drain_queue(const BinCore &c, const Shared &sh, const EdgeLds &E, WaveQueue &q,
                                            LaneStats &st, Emitter &em) {
    const int lane = threadIdx.x & 63;
    const double Nd = (double)sh.nside;
    wave_lds_sync();
    uint32_t key = kNoKey;
    if (lane < q.nb)
        key = bin_instance<kMode, true>(c, sh, E, Nd, q.q[lane], q.q[kQueue + lane], q.q[2 * kQueue + lane], st);
    if (kMode == kEmit) emit_keys(em, c, key, st);
    if (kMode == kAtomic) aggregate_add(c.counts, key);
    key = kNoKey;
    const int t = kQueue - 1 - lane;
    if (lane < q.nc) key = bin_instance<kMode, false>(c, sh, E, Nd, q.q[t], q.q[kQueue + t], q.q[2 * kQueue + t], st);
    if (kMode == kEmit) emit_keys(em, c, key, st);
    if (kMode == kAtomic) aggregate_add(c.counts, key);
    wave_lds_sync();
    q.nb = 0;
    q.nc = 0;
}

__device__ __forceinline__ Shared shared_of(const BinParams &p) {
    return Shared{p.guard, p.guard_cap, p.nside, p.npix, p.eps, p.status};
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
